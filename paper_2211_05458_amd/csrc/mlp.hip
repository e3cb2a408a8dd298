// Learned Newton initial guess: features, training pairs from Newton, a
// 84-64-64-64-3 tanh MLP (forward, backward, Adam) in FP32, and the flags of
// strongly curved elements on which the guess is used.
#include <mutex>

#include "fp_device.h"
#include "fp_launch.h"

namespace fp {

constexpr int H = 64, NI = kMlpIn, NO = 3;
constexpr int NW = H * NI + H + 2 * (H * H + H) + NO * H + NO;
constexpr int ROW = kMlpRow;   // per-row activations and deltas

template <int NG>
__global__ void k_mlp_features(MeshView m, int64_t n, const int32_t* __restrict__ elem, const double* __restrict__ x,
                               float* feat) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double xx[3] = {x[r * 3], x[r * 3 + 1], x[r * 3 + 2]};
  float f[NI];
  mlp_features<NG>(m, elem[r], xx, f);
  for (int i = 0; i < NI; ++i) feat[r * NI + i] = f[i];
}

template <int NN, int NG>
__global__ void k_newton_pairs(MeshView m, Particles P, int64_t n, float* feat, float* xo, int32_t* ids,
                               int32_t* count) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || P.status[p] != ACTIVE) return;
  const int64_t cap = P.cap;
  int e = P.elem[p];
  double x[3] = {P.x[p], P.x[cap + p], P.x[2 * cap + p]};
  double xi[3];
  int it = 0, calls = 0, fb = 0;
  if (!locate_xi<NN, NG>(m, e, x, xi, 50, false, it, calls, fb) || !inside_ref(xi)) return;
  int q = atomicAdd(count, 1);
  float f[NI];
  mlp_features<NG>(m, e, x, f);
  for (int i = 0; i < NI; ++i) feat[(int64_t)q * NI + i] = f[i];
  for (int k = 0; k < 3; ++k) xo[(int64_t)q * 3 + k] = (float)xi[k];
  if (ids) ids[q] = P.id[p];
}

// max deviation of the geometry nodes from the trilinear map of the corners
template <int NG>
__global__ void k_curved_flags(MeshView m, double thresh, uint8_t* flag, int32_t* count) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.E) return;
  const double* P = m.X + (size_t)e * NG * NG * NG * 3;
  constexpr int G = NG - 1;
  double cor[8][3];
  for (int c = 0; c < 8; ++c) {
    const double* Q = P + ((((c >> 2) & 1) * G * NG + ((c >> 1) & 1) * G) * NG + (c & 1) * G) * 3;
    for (int r = 0; r < 3; ++r) cor[c][r] = Q[r];
  }
  double dev = 0.0;
  for (int k = 0; k < NG; ++k)
    for (int j = 0; j < NG; ++j)
      for (int i = 0; i < NG; ++i) {
        double s = (double)i / G, t = (double)j / G, u = (double)k / G;
        double tri[3] = {0, 0, 0};
        for (int c = 0; c < 8; ++c) {
          double w = ((c & 1) ? s : 1 - s) * (((c >> 1) & 1) ? t : 1 - t) * (((c >> 2) & 1) ? u : 1 - u);
          for (int r = 0; r < 3; ++r) tri[r] += w * cor[c][r];
        }
        const double* Q = P + ((k * NG + j) * NG + i) * 3;
        double dx = Q[0] - tri[0], dy = Q[1] - tri[1], dz = Q[2] - tri[2];
        dev = fmax(dev, sqrt(dx * dx + dy * dy + dz * dz));
      }
  uint8_t fl = dev > thresh * m.hE[e];
  flag[e] = fl;
  if (fl) atomicAdd(count, 1);
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ w, int64_t n,
                                                     const float* __restrict__ in, float* out) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  float x[NI], o[3];
  for (int i = 0; i < NI; ++i) x[i] = in[r * NI + i];
  mlp_forward_row(w, x, o);
  for (int k = 0; k < 3; ++k) out[r * 3 + k] = o[k];
}

// ---------------------------------------------------------------------------
// Training on the matrix cores (FP32, v_mfma_f32_16x16x4f32).  The network
// runs transposed, units as rows and batch rows as columns: a layer's 16x16
// output tile holds, in lane (row l % 16, group q = l / 16), units
// 16 t + 4 q + i in register i.  Taking the k-steps of the next product as the
// unit sets {16 t + 4 k + i : k = 0..3} (k = lane group), register i of that
// tile is already the B operand, forward (W H^T) and backward (W^T dZ^T)
// alike; the weights are the A operands, read from LDS.
// Lane layout: A[m][k], B[k][n] in lane (m or n) + 16 k; D[m][n] in lane
// n + 16 (m / 4), register m % 4.
// ---------------------------------------------------------------------------
typedef float v4f32 __attribute__((ext_vector_type(4)));

constexpr int FBT = 2;   // 16-row tiles per wavefront of the training pass

// forward and backward of 16 FBT batch rows per wavefront (one per workgroup);
// activations and deltas to buf[row][ROW] (x, h1, h2, h3, d1, d2, d3, dy), the
// mean squared error to *loss
__global__ __launch_bounds__(64) void k_mlp_fb(const float* __restrict__ w, int64_t n, const float* __restrict__ in,
                                               const float* __restrict__ target, const int32_t* __restrict__ rows,
                                               float* buf, float* loss) {
  __shared__ float W[NW];
  for (int i = threadIdx.x; i < NW; i += 64) W[i] = w[i];
  __syncthreads();
  const float* W1 = W;
  const float* b1 = W1 + H * NI;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + H * H;
  const float* W4 = b3 + H;
  const float* b4 = W4 + NO * H;
  const int lane = threadIdx.x, kq = lane >> 4, col = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * (16 * FBT);
  const float scale = 1.0f / (float)(n * NO);
  int64_t src[FBT];
  bool ok[FBT];
#pragma unroll
  for (int nt = 0; nt < FBT; ++nt) {
    const int64_t r = r0 + 16 * nt + col;
    ok[nt] = r < n;
    src[nt] = ok[nt] ? (rows ? rows[r] : r) : 0;
  }
  // layer 1: k-steps of four consecutive inputs 4 s + k
  v4f32 h1[4][FBT], h2[4][FBT], h3[4][FBT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < FBT; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) h1[mt][nt][i] = b1[16 * mt + 4 * kq + i];
#pragma unroll 3
  for (int st = 0; st < NI / 4; ++st) {
    float xb[FBT];
#pragma unroll
    for (int nt = 0; nt < FBT; ++nt) {
      xb[nt] = ok[nt] ? in[src[nt] * NI + 4 * st + kq] : 0.f;
      if (ok[nt]) buf[(r0 + 16 * nt + col) * ROW + 4 * st + kq] = xb[nt];
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const float a = W1[(16 * mt + col) * NI + 4 * st + kq];
#pragma unroll
      for (int nt = 0; nt < FBT; ++nt) h1[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xb[nt], h1[mt][nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < FBT; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) h1[mt][nt][i] = tanhf(h1[mt][nt][i]);
  // hidden layers: k-step (t, i) = units 16 t + 4 k + i
  auto forward = [&](const float* Wl, const float* bl, v4f32 (*hin)[FBT], v4f32 (*hout)[FBT]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
      for (int nt = 0; nt < FBT; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) hout[mt][nt][i] = bl[16 * mt + 4 * kq + i];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float a = Wl[(16 * mt + col) * H + 16 * t + 4 * kq + i];
#pragma unroll
          for (int nt = 0; nt < FBT; ++nt)
            hout[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, hin[t][nt][i], hout[mt][nt], 0, 0, 0);
        }
#pragma unroll
      for (int nt = 0; nt < FBT; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) hout[mt][nt][i] = tanhf(hout[mt][nt][i]);
    }
  };
  forward(W2, b2, h1, h2);
  forward(W3, b3, h2, h3);
  // output rows 0..2 (lanes of group 0, register j), error and its gradient
  float lsum = 0.f;
  float dyv[FBT][NO];
#pragma unroll
  for (int nt = 0; nt < FBT; ++nt) {
    v4f32 y;
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = (kq == 0 && i < NO) ? b4[i] : 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float a = col < NO ? W4[col * H + 16 * t + 4 * kq + i] : 0.f;
        y = __builtin_amdgcn_mfma_f32_16x16x4f32(a, h3[t][nt][i], y, 0, 0, 0);
      }
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      float g = 0.f;
      if (kq == 0 && ok[nt]) {
        const float diff = y[j] - target[src[nt] * NO + j];
        lsum += diff * diff * scale;
        g = 2.0f * diff * scale;
      }
      dyv[nt][j] = g;
    }
  }
  // d3 = W4^T dy (k = output j, one k-step) * (1 - h3^2)
  v4f32 d3[4][FBT], d2[4][FBT], d1[4][FBT];
#pragma unroll
  for (int nt = 0; nt < FBT; ++nt) {
    const float s0 = __shfl(dyv[nt][0], col, 64), s1 = __shfl(dyv[nt][1], col, 64), s2 = __shfl(dyv[nt][2], col, 64);
    const float bdy = kq == 0 ? s0 : kq == 1 ? s1 : kq == 2 ? s2 : 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const float a = kq < NO ? W4[kq * H + 16 * mt + col] : 0.f;
      v4f32 z = {0.f, 0.f, 0.f, 0.f};
      z = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bdy, z, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) d3[mt][nt][i] = z[i] * (1.f - h3[mt][nt][i] * h3[mt][nt][i]);
    }
    if (kq == 0 && ok[nt]) {
#pragma unroll
      for (int j = 0; j < NO; ++j) buf[(r0 + 16 * nt + col) * ROW + NI + 6 * H + j] = dyv[nt][j];
    }
  }
  // d_prev = W^T d (A[m = input unit][k = output unit]) * (1 - h_prev^2)
  auto backward = [&](const float* Wl, v4f32 (*din)[FBT], v4f32 (*hprev)[FBT], v4f32 (*dout)[FBT]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      v4f32 z[FBT];
#pragma unroll
      for (int nt = 0; nt < FBT; ++nt) z[nt] = (v4f32){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float a = Wl[(16 * t + 4 * kq + i) * H + 16 * mt + col];
#pragma unroll
          for (int nt = 0; nt < FBT; ++nt) z[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, din[t][nt][i], z[nt], 0, 0, 0);
        }
#pragma unroll
      for (int nt = 0; nt < FBT; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) dout[mt][nt][i] = z[nt][i] * (1.f - hprev[mt][nt][i] * hprev[mt][nt][i]);
    }
  };
  backward(W3, d3, h2, d2);
  backward(W2, d2, h1, d1);
  // rows to the buffer: four consecutive units per lane and tile
#pragma unroll
  for (int nt = 0; nt < FBT; ++nt) {
    if (!ok[nt]) continue;
    float* B = buf + (r0 + 16 * nt + col) * ROW + NI;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int u = 16 * mt + 4 * kq;
      *(float4*)(B + 0 * H + u) = make_float4(h1[mt][nt][0], h1[mt][nt][1], h1[mt][nt][2], h1[mt][nt][3]);
      *(float4*)(B + 1 * H + u) = make_float4(h2[mt][nt][0], h2[mt][nt][1], h2[mt][nt][2], h2[mt][nt][3]);
      *(float4*)(B + 2 * H + u) = make_float4(h3[mt][nt][0], h3[mt][nt][1], h3[mt][nt][2], h3[mt][nt][3]);
      *(float4*)(B + 3 * H + u) = make_float4(d1[mt][nt][0], d1[mt][nt][1], d1[mt][nt][2], d1[mt][nt][3]);
      *(float4*)(B + 4 * H + u) = make_float4(d2[mt][nt][0], d2[mt][nt][1], d2[mt][nt][2], d2[mt][nt][3]);
      *(float4*)(B + 5 * H + u) = make_float4(d3[mt][nt][0], d3[mt][nt][1], d3[mt][nt][2], d3[mt][nt][3]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
  if (lane == 0) atomicAdd(loss, lsum);
}

// Weight and bias gradients on the matrix cores: one wavefront per 16x16
// tile of a layer's gradient, summing over the batch rows (k-steps of four
// rows): dW[o][i] = sum_r d[r][o] h_in[r][i]; the bias column is the tile whose
// input is 1 in column 0.
struct GradTile { int layer, mt, it; };   // it == -1: the bias tile
__device__ inline GradTile grad_tile(int b) {
  // layer 1: 4 x 6 tiles (84 inputs) + 4 bias tiles; layers 2, 3: 4 x 4 + 4;
  // output layer: 1 x 4 + 1
  if (b < 28) return {0, b / 7, b % 7 == 6 ? -1 : b % 7};
  b -= 28;
  if (b < 20) return {1, b / 5, b % 5 == 4 ? -1 : b % 5};
  b -= 20;
  if (b < 20) return {2, b / 5, b % 5 == 4 ? -1 : b % 5};
  b -= 20;
  return {3, 0, b == 4 ? -1 : b};
}
constexpr int kGradTiles = 28 + 20 + 20 + 5;

// four wavefronts per tile, each summing every fourth group of four rows,
// then the four partial tiles added in a fixed order
__global__ __launch_bounds__(256) void k_mlp_wgrad_mfma(int64_t n, const float* __restrict__ buf, float* grad) {
  __shared__ v4f32 part[3][64];
  const GradTile T = grad_tile(blockIdx.x);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, kq = lane >> 4, col = lane & 15;
  const int nin = T.layer == 0 ? NI : H, nout = T.layer == 3 ? NO : H;
  const int in_off = T.layer == 0 ? 0 : NI + (T.layer - 1) * H;
  const int d_off = T.layer == 3 ? NI + 6 * H : NI + (3 + T.layer) * H;
  const size_t wofs = T.layer == 0 ? 0 : (size_t)H * NI + H + (size_t)(T.layer - 1) * (H * H + H);
  const int o = 16 * T.mt + col, i = 16 * T.it + col;
  const bool ao = o < nout, bi = T.it >= 0 && i < nin;
  v4f32 acc = {0.f, 0.f, 0.f, 0.f};
  constexpr int U = 4;   // k-steps in flight
  for (int64_t r0 = 4 * (int64_t)wv; r0 < n; r0 += 16 * U) {
    float a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + 16 * u + kq;
      const bool live = r < n;
      const float* B = buf + (live ? r : 0) * ROW;
      a[u] = (ao && live) ? B[d_off + o] : 0.f;
      b[u] = T.it >= 0 ? ((bi && live) ? B[in_off + i] : 0.f) : ((col == 0 && live) ? 1.f : 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
  }
  if (wv > 0) part[wv - 1][lane] = acc;
  __syncthreads();
  if (wv != 0) return;
  acc += part[0][lane];
  acc += part[1][lane];
  acc += part[2][lane];
  // D[m = output 16 mt + 4 kq + j][n = input col]
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int oo = 16 * T.mt + 4 * kq + j;
    if (oo >= nout) continue;
    if (T.it >= 0) {
      if (bi) grad[wofs + (size_t)oo * nin + i] = acc[j];
    } else if (col == 0) {
      grad[wofs + (size_t)nout * nin + oo] = acc[j];
    }
  }
}

__global__ void k_zero_f32(float* a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

__global__ void k_adam(float* w, float* m, float* v, const float* __restrict__ g, int64_t nw, float lr, float c1,
                       float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw) return;
  float gi = g[i];
  float mi = 0.9f * m[i] + 0.1f * gi;
  float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

hipError_t launch_mlp_features(const MeshView& m, int64_t n, const int32_t* elem, const double* x, float* feat,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 g((unsigned)((n + 255) / 256));
  switch (m.ng) {
    case 2: k_mlp_features<2><<<g, 256, 0, s>>>(m, n, elem, x, feat); break;
    case 3: k_mlp_features<3><<<g, 256, 0, s>>>(m, n, elem, x, feat); break;
    case 5: k_mlp_features<5><<<g, 256, 0, s>>>(m, n, elem, x, feat); break;
    case 7: k_mlp_features<7><<<g, 256, 0, s>>>(m, n, elem, x, feat); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#include "fp_shapes.h"

hipError_t launch_newton_pairs(const MeshView& m, const Particles& P, int64_t n, float* feat, float* xi,
                               int32_t* ids, int32_t* count, hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 g((unsigned)((n + 255) / 256));
#define FP_L(A, B) \
  if (m.n == A && m.ng == B) { k_newton_pairs<A, B><<<g, 256, 0, s>>>(m, P, n, feat, xi, ids, count); return hipGetLastError(); }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

// Per element (one 64-thread workgroup, one hidden unit per thread): the first
// layer's pre-activation from the 81 inputs that depend on the element only,
// bias included, summed in the order of the full forward pass, and the corner
// mean and length scale that turn a point into the last three inputs.
template <int NG>
__global__ __launch_bounds__(64) void k_mlp_elem_table(MeshView m, const float* __restrict__ w, float* h1,
                                                      double* ctr) {
  const int e = blockIdx.x, o = threadIdx.x;
  float feat[kMlpIn];
  double ci[4];
  const double x0[3] = {0.0, 0.0, 0.0};
  mlp_features<NG>(m, e, x0, feat, ci);
  float s = w[64 * kMlpIn + o];
  for (int i = 0; i < kMlpIn - 3; ++i) s += w[o * kMlpIn + i] * feat[i];
  h1[(size_t)e * 64 + o] = s;
  if (o < 4) ctr[(size_t)e * 4 + o] = ci[o];
}

hipError_t launch_mlp_elem_table(const MeshView& m, const float* w, float* h1, double* ctr, hipStream_t s) {
  switch (m.ng) {
    case 2: k_mlp_elem_table<2><<<m.E, 64, 0, s>>>(m, w, h1, ctr); break;
    case 3: k_mlp_elem_table<3><<<m.E, 64, 0, s>>>(m, w, h1, ctr); break;
    case 5: k_mlp_elem_table<5><<<m.E, 64, 0, s>>>(m, w, h1, ctr); break;
    case 7: k_mlp_elem_table<7><<<m.E, 64, 0, s>>>(m, w, h1, ctr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_curved_flags(const MeshView& m, double thresh, uint8_t* flag, int32_t* count, hipStream_t s) {
  dim3 g((unsigned)((m.E + 255) / 256));
  switch (m.ng) {
    case 2: k_curved_flags<2><<<g, 256, 0, s>>>(m, thresh, flag, count); break;
    case 3: k_curved_flags<3><<<g, 256, 0, s>>>(m, thresh, flag, count); break;
    case 5: k_curved_flags<5><<<g, 256, 0, s>>>(m, thresh, flag, count); break;
    case 7: k_curved_flags<7><<<g, 256, 0, s>>>(m, thresh, flag, count); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Learned guesses of a stage on the matrix cores.  Each wavefront takes 64
// particles at a time (persistent grid) and runs the network transposed, units
// as rows and particles as columns: Z^T = W H^T on v_mfma_f32_16x16x16bf16_1k
// (bf16 weights and activations, FP32 sums).  With that orientation the
// 16x16 output tile of a layer (lane: particle lane % 16, four consecutive
// units 4 (lane / 16) + i) is, after tanh and rounding to bf16, already the B
// operand of the next layer, so no activation leaves the registers.  The first
// layer takes the element's part from the table (W1 g_e + b1) and adds the
// point's three inputs on the VALU.  The guess only starts Newton, which
// converges to the same root from any guess in its basin; bf16 rounding of
// the network moves the guess by about 1e-2 of the reference cell at most.
// Lane layout (gfx950): A[m][k] in lane m + 16 (k / 4), element k % 4; B[k][n]
// in lane n + 16 (k / 4), element k % 4; D[m][n] in lane n + 16 (m / 4),
// register m % 4.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

// four floats -> four bf16 (round to nearest even, v_cvt_pk_bf16_f32)
__device__ __forceinline__ v4s to_bf16(v4f x) { return __builtin_bit_cast(v4s, __builtin_convertvector(x, v4bf)); }

// tanh(x) = 1 - 2 / (exp(2x) + 1), exact at both saturations; relative error
// of a few float ulps, far below the bf16 rounding that follows
__device__ __forceinline__ float tanh_guess(float x) {
  const float e = __expf(2.f * x);
  return 1.f - __fdividef(2.f, e + 1.f);
}

// the weights as the A operands of each lane (lane-major, so that a
// wavefront reads one fragment with one 8-byte LDS load per lane), and the
// first layer's point weights and the biases of the units a lane holds in
// the output layout (unit 16 mt + 4 (lane / 16) + i)
struct GuessLds {
  v4s a2[4][4][64], a3[4][4][64], a4[4][64];
  float w1p[4][4][4][3];   // [lane / 16][mt][i][input 81 + k]
  float b2[64], b3[64];
};

// the particles that take a learned guess this stage: active, in a flagged
// element, and without continued reference coordinates (warm != 0: the first
// guess of the others is their continued xi, and only a learned guess computed
// here is ever read)
// (one atomic per workgroup of 1024 particles: a counter that every wavefront
// hits serialises 1e5 atomics, about 1.4 ms for 1e7 particles)
constexpr int kSelectWaves = 16;
__global__ __launch_bounds__(64 * kSelectWaves) void k_mlp_select(MeshView m, Particles P, int64_t n, int warm,
                                                                  int32_t* __restrict__ list,
                                                                  int32_t* __restrict__ count) {
  __shared__ int sh[kSelectWaves + 1];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool use = false;
  if (p < n && P.status[p] == ACTIVE && m.mlp_flag[P.elem[p]] != 0) {
    double gw[3];
    use = !(warm && warm_guess(P, p, gw));
  }
  const int slot = block_push<kSelectWaves>(count, use, sh);
  if (use) list[slot] = (int32_t)p;
}

__global__ void k_set_i32(int32_t* a, int32_t v) { *a = v; }

// guesses of the listed particles (*count entries)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_mlp_guess(
    MeshView m, Particles P, const int32_t* __restrict__ list, const int32_t* __restrict__ count,
    float* __restrict__ guess) {
  __shared__ GuessLds S;
  const int lane = threadIdx.x & 63, kq = lane >> 4, col = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t cap = P.cap;
  const float* W1 = m.mlp_w;
  const float* W2 = W1 + H * NI + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + H * H;
  const float* W4 = b3 + H;
  const float* b4 = W4 + NO * H;
  // A[m][k] = W[16 mt + m][16 st + k] in lane m + 16 (k / 4), element k % 4
  for (int idx = threadIdx.x; idx < 16 * 64; idx += blockDim.x) {
    const int l = idx & 63, mt = (idx >> 6) & 3, st = idx >> 8;
    const int o = 16 * mt + (l & 15), i0 = 16 * st + 4 * (l >> 4);
    v4f w2, w3;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      w2[j] = W2[o * H + i0 + j];
      w3[j] = W3[o * H + i0 + j];
    }
    S.a2[mt][st][l] = to_bf16(w2);
    S.a3[mt][st][l] = to_bf16(w3);
    if (mt == 0) {
      v4f w4;
#pragma unroll
      for (int j = 0; j < 4; ++j) w4[j] = (l & 15) < NO ? W4[(l & 15) * H + i0 + j] : 0.f;
      S.a4[st][l] = to_bf16(w4);
    }
  }
  for (int idx = threadIdx.x; idx < 64; idx += blockDim.x) {
    S.b2[idx] = b2[idx];
    S.b3[idx] = b3[idx];
    const int q = idx >> 4, mt = (idx >> 2) & 3, i = idx & 3, o = 16 * mt + 4 * q + i;
#pragma unroll
    for (int k = 0; k < 3; ++k) S.w1p[q][mt][i][k] = W1[o * NI + 81 + k];
  }
  __syncthreads();
  const int64_t n = *count;
  for (int64_t base = wave * 64; base < n; base += nwave * 64) {
    int e[4];
    int64_t pp[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int64_t i = base + 16 * nt + col;
      pp[nt] = i < n ? (int64_t)list[i] : -1;
      e[nt] = pp[nt] >= 0 ? P.elem[pp[nt]] : 0;
    }
    // layer 1 on the VALU: listed particles base + 16 nt + lane % 16
    v4s hb[4][4];   // B operands [input tile][particle tile]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int64_t p = pp[nt];
      const double* c = m.mlp_ctr + (size_t)e[nt] * 4;
      float xh[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) xh[k] = p >= 0 ? (float)((P.x[k * cap + p] - c[k]) * c[3]) : 0.f;
      const float* h1e = m.mlp_h1 + (size_t)e[nt] * H;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const float4 t = *(const float4*)(h1e + 16 * mt + 4 * kq);
        const float tv[4] = {t.x, t.y, t.z, t.w};
        v4f z;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float* w = S.w1p[kq][mt][i];
          z[i] = tanh_guess(tv[i] + w[0] * xh[0] + w[1] * xh[1] + w[2] * xh[2]);
        }
        hb[mt][nt] = to_bf16(z);
      }
    }
    // layers 2 and 3 on the matrix cores
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
      v4s nb[4][4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        v4f acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[nt][i] = layer == 0 ? S.b2[16 * mt + 4 * kq + i] : S.b3[16 * mt + 4 * kq + i];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const v4s a = layer == 0 ? S.a2[mt][st][lane] : S.a3[mt][st][lane];
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, hb[st][nt], acc[nt], 0, 0, 0);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          v4f z;
#pragma unroll
          for (int i = 0; i < 4; ++i) z[i] = tanh_guess(acc[nt][i]);
          nb[mt][nt] = to_bf16(z);
        }
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) hb[mt][nt] = nb[mt][nt];
    }
    // output layer: rows 0..2 of the tile (lanes 0..15) are the guess
    v4f acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[nt][i] = (kq == 0 && i < NO) ? b4[i] : 0.f;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const v4s a = S.a4[st][lane];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, hb[st][nt], acc[nt], 0, 0, 0);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int64_t p = pp[nt];
      if (kq == 0 && p >= 0) {
#pragma unroll
        for (int k = 0; k < NO; ++k) guess[k * cap + p] = acc[nt][k];
      }
    }
  }
}

hipError_t launch_mlp_guess(const MeshView& m, const Particles& P, int64_t n, int warm, int32_t* list,
                            int32_t* count, float* guess, hipStream_t s) {
  if (n == 0 || !m.mlp_w) return hipSuccess;
  k_set_i32<<<1, 1, 0, s>>>(count, 0);
  k_mlp_select<<<dim3((unsigned)((n + 64 * kSelectWaves - 1) / (64 * kSelectWaves))), 64 * kSelectWaves, 0, s>>>(
      m, P, n, warm, list, count);
  // persistent: each wavefront converts the weights once
  const int64_t waves = std::min<int64_t>((n + 63) / 64, 4096);
  k_mlp_guess<<<dim3((unsigned)((waves + 3) / 4)), 256, 0, s>>>(m, P, list, count, guess);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* w, int64_t n, const float* in, float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_mlp_forward<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(w, n, in, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row buffer of fp_mlp_loss_grad_static (callers that cannot allocate): a
// fixed device array, one copy per GPU, held until the process ends.  In host
// code `scratch` names a host-side stand-in, never the device memory: the
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address reaches kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) float scratch[(size_t)kMlpStaticRows * ROW];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
float* scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t mlp_static_rows(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = (float*)p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_mlp_loss_grad(const float* w, int64_t n, const float* in, const float* target,
                                const int32_t* rows, float* grad, float* loss, float* rowbuf, hipStream_t s) {
  if (n <= 0 || n > kMlpMaxBatch) return hipErrorInvalidValue;
  k_zero_f32<<<1, 64, 0, s>>>(loss, 1);
  k_mlp_fb<<<dim3((unsigned)((n + 16 * FBT - 1) / (16 * FBT))), 64, 0, s>>>(w, n, in, target, rows, rowbuf, loss);
  k_mlp_wgrad_mfma<<<dim3(kGradTiles), 256, 0, s>>>(n, rowbuf, grad);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, float* m, float* v, const float* g, int64_t nw, int64_t t, float lr, hipStream_t s) {
  float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
  k_adam<<<dim3((unsigned)((nw + 255) / 256)), 256, 0, s>>>(w, m, v, g, nw, lr, c1, c2);
  return hipGetLastError();
}

}  // namespace fp

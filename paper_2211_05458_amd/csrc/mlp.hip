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

// per-row forward and backward; activations and deltas to buf[row][ROW]
__global__ __launch_bounds__(128) void k_mlp_rows(const float* __restrict__ w, int64_t n, const float* __restrict__ in,
                                                  const float* __restrict__ target, const int32_t* __restrict__ rows,
                                                  float* buf, float* loss) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float lsum = 0.0f;
  if (r < n) {
    int64_t src = rows ? rows[r] : r;
    const float* W1 = w;
    const float* b1 = W1 + H * NI;
    const float* W2 = b1 + H;
    const float* b2 = W2 + H * H;
    const float* W3 = b2 + H;
    const float* b3 = W3 + H * H;
    const float* W4 = b3 + H;
    const float* b4 = W4 + NO * H;
    float* B = buf + r * ROW;
    float* x = B;
    float* h1 = x + NI;
    float* h2 = h1 + H;
    float* h3 = h2 + H;
    float* d1 = h3 + H;
    float* d2 = d1 + H;
    float* d3 = d2 + H;
    float* dy = d3 + H;
    float xr[NI];
    for (int i = 0; i < NI; ++i) { xr[i] = in[src * NI + i]; x[i] = xr[i]; }
    float a[H], b[H];
    for (int o = 0; o < H; ++o) {
      float s = b1[o];
      for (int i = 0; i < NI; ++i) s += W1[o * NI + i] * xr[i];
      a[o] = tanhf(s);
      h1[o] = a[o];
    }
    for (int o = 0; o < H; ++o) {
      float s = b2[o];
      for (int i = 0; i < H; ++i) s += W2[o * H + i] * a[i];
      b[o] = tanhf(s);
      h2[o] = b[o];
    }
    for (int o = 0; o < H; ++o) {
      float s = b3[o];
      for (int i = 0; i < H; ++i) s += W3[o * H + i] * b[i];
      a[o] = tanhf(s);
      h3[o] = a[o];
    }
    const float scale = 1.0f / (float)(n * NO);
    float g[NO];
    for (int o = 0; o < NO; ++o) {
      float s = b4[o];
      for (int i = 0; i < H; ++i) s += W4[o * H + i] * a[i];
      float diff = s - target[src * NO + o];
      lsum += diff * diff * scale;
      g[o] = 2.0f * diff * scale;
      dy[o] = g[o];
    }
    // deltas (pre-activation gradients)
    for (int i = 0; i < H; ++i) {
      float s = 0.0f;
      for (int o = 0; o < NO; ++o) s += W4[o * H + i] * g[o];
      b[i] = s * (1.0f - a[i] * a[i]);
      d3[i] = b[i];
    }
    for (int i = 0; i < H; ++i) {
      float s = 0.0f;
      for (int o = 0; o < H; ++o) s += W3[o * H + i] * b[o];
      float hv = h2[i];
      a[i] = s * (1.0f - hv * hv);
      d2[i] = a[i];
    }
    for (int i = 0; i < H; ++i) {
      float s = 0.0f;
      for (int o = 0; o < H; ++o) s += W2[o * H + i] * a[o];
      float hv = h1[i];
      d1[i] = s * (1.0f - hv * hv);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, lsum);
}

// weight gradients: block (o, layer), threads stride over the layer's inputs,
// each summing over the rows
__global__ __launch_bounds__(128) void k_mlp_wgrad(int64_t n, const float* __restrict__ buf, float* grad) {
  int o = blockIdx.x, layer = blockIdx.y;
  int nin = layer == 0 ? NI : H;
  int nout = layer == 3 ? NO : H;
  if (o >= nout) return;
  int in_off = layer == 0 ? 0 : (layer == 1 ? NI : (layer == 2 ? NI + H : NI + 2 * H));
  int d_off = layer == 0 ? NI + 3 * H : (layer == 1 ? NI + 4 * H : (layer == 2 ? NI + 5 * H : NI + 6 * H));
  size_t wofs = layer == 0 ? 0 : (layer == 1 ? H * NI + H : (layer == 2 ? H * NI + H + H * H + H : H * NI + H + 2 * (H * H + H)));
  for (int i = threadIdx.x; i < nin; i += blockDim.x) {
    float g = 0.0f;
    for (int64_t r = 0; r < n; ++r) {
      const float* B = buf + r * ROW;
      g += B[d_off + o] * B[in_off + i];
    }
    grad[wofs + (size_t)o * nin + i] = g;
  }
  if (threadIdx.x == 0) {
    float gb = 0.0f;
    for (int64_t r = 0; r < n; ++r) gb += buf[r * ROW + d_off + o];
    grad[wofs + (size_t)nout * nin + o] = gb;
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

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_mlp_guess(MeshView m, Particles P, int64_t n, float* __restrict__ guess) {
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
  for (int64_t base = wave * 64; base < n; base += nwave * 64) {
    int e[4];
    bool use[4];
    bool any = false;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int64_t p = base + 16 * nt + col;
      e[nt] = 0;
      use[nt] = false;
      if (p < n && P.status[p] == ACTIVE) {
        e[nt] = P.elem[p];
        use[nt] = m.mlp_flag[e[nt]] != 0;
      }
      any = any || use[nt];
    }
    if (!__ballot(any)) continue;   // no particle of these 64 is in a flagged element
    // layer 1 on the VALU: particles base + 16 nt + lane % 16
    v4s hb[4][4];   // B operands [input tile][particle tile]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int64_t p = base + 16 * nt + col;
      const double* c = m.mlp_ctr + (size_t)e[nt] * 4;
      float xh[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) xh[k] = p < n ? (float)((P.x[k * cap + p] - c[k]) * c[3]) : 0.f;
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
      const int64_t p = base + 16 * nt + col;
      if (kq == 0 && use[nt]) {
#pragma unroll
        for (int k = 0; k < NO; ++k) guess[k * cap + p] = acc[nt][k];
      }
    }
  }
}

hipError_t launch_mlp_guess(const MeshView& m, const Particles& P, int64_t n, float* guess, hipStream_t s) {
  if (n == 0 || !m.mlp_w) return hipSuccess;
  // persistent: each wavefront converts the weights once
  const int64_t waves = std::min<int64_t>((n + 63) / 64, 4096);
  k_mlp_guess<<<dim3((unsigned)((waves + 3) / 4)), 256, 0, s>>>(m, P, n, guess);
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
  k_mlp_rows<<<dim3((unsigned)((n + 127) / 128)), 128, 0, s>>>(w, n, in, target, rows, rowbuf, loss);
  k_mlp_wgrad<<<dim3(H, 4), 128, 0, s>>>(n, rowbuf, grad);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, float* m, float* v, const float* g, int64_t nw, int64_t t, float lr, hipStream_t s) {
  float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
  k_adam<<<dim3((unsigned)((nw + 255) / 256)), 256, 0, s>>>(w, m, v, g, nw, lr, c1, c2);
  return hipGetLastError();
}

}  // namespace fp

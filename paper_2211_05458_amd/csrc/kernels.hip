// Kernels of the per-particle step for gfx950: setup (faces, nodes), particle
// location, the fused RK stage, final reference coordinates and the
// nearest-DOF source.  One thread per particle; particles are kept sorted by
// element so that a wavefront reads the same element data.
#include "fp_device.h"
#include "fp_launch.h"

namespace fp {

struct MinvArg { double v[kMaxNodes * kMaxNodes]; };

// ---------------------------------------------------------------------------
// setup: Bezier control points, slab boxes, classification (Sec. 3.2.4)
// ---------------------------------------------------------------------------
template <int NG>
__global__ void k_face_setup(int E, const double* __restrict__ X, const int32_t* __restrict__ nbr_elem,
                             const int32_t* __restrict__ nbr_face, const int8_t* __restrict__ bc,
                             const double* __restrict__ shift, MinvArg Mi, FaceRec* faces, double* cpo) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= E * 6) return;
  int e = gid / 6, f = gid % 6;
  FaceRec F;
  face_setup<NG>(X + (size_t)e * NG * NG * NG * 3, f, Mi.v, cpo + (size_t)gid * NG * NG * 3, F);
  F.nbr_elem = nbr_elem[gid];
  F.nbr_face = nbr_face[gid];
  F.bc = bc[gid];
  for (int q = 0; q < 3; ++q) F.shift[q] = shift[gid * 3 + q];
  faces[gid] = F;
}

// DG node positions x(xi_ijk), volumes w_i w_j w_k J(xi_ijk), element length scale
template <int NN, int NG>
__global__ void k_nodes(MeshView m, double* xnode, double* vol, double* hE, int32_t* bad) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int N3 = NN * NN * NN;
  if (gid >= (int64_t)m.E * N3) return;
  int e = (int)(gid / N3), q = (int)(gid % N3);
  int i = q % NN, j = (q / NN) % NN, k = q / (NN * NN);
  double xi[3] = {m.xdg[i], m.xdg[j], m.xdg[k]}, x[3], J[3][3];
  map_jac<NG>(m, m.X + (size_t)e * NG * NG * NG * 3, xi, x, J);
  xnode[gid * 3 + 0] = x[0]; xnode[gid * 3 + 1] = x[1]; xnode[gid * 3 + 2] = x[2];
  double dj = det3(J);
  vol[gid] = m.wdg[i] * m.wdg[j] * m.wdg[k] * dj;
  if (!(dj > 0.0)) atomicAdd(bad, 1);
  if (q == 0) {
    const double* P = m.X + (size_t)e * NG * NG * NG * 3;
    constexpr int G = NG - 1;
    double hm = 0.0;
    for (int a = 0; a < 8; ++a)
      for (int bit = 0; bit < 3; ++bit) {
        int b = a ^ (1 << bit);
        if (b < a) continue;
        int ia = ((((a >> 2) & 1) * G) * NG + ((a >> 1) & 1) * G) * NG + (a & 1) * G;
        int ib = ((((b >> 2) & 1) * G) * NG + ((b >> 1) & 1) * G) * NG + (b & 1) * G;
        double r[3] = {P[ia * 3] - P[ib * 3], P[ia * 3 + 1] - P[ib * 3 + 1], P[ia * 3 + 2] - P[ib * 3 + 2]};
        hm = fmax(hm, sqrt(dot3(r, r)));
      }
    hE[e] = hm;
  }
}

// box of each element's DG nodes (one wave per element) and the largest
// distance by which a node lies outside the padded element box
template <int NN>
__global__ __launch_bounds__(64) void k_node_box(MeshView m, const double* xnode, double* nbox,
                                                 unsigned long long* node_pad) {
  constexpr int N3 = NN * NN * NN;
  const int e = blockIdx.x, lane = threadIdx.x;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int q = lane; q < N3; q += 64)
    for (int k = 0; k < 3; ++k) {
      double x = xnode[((size_t)e * N3 + q) * 3 + k];
      lo[k] = fmin(lo[k], x);
      hi[k] = fmax(hi[k], x);
    }
  for (int k = 0; k < 3; ++k)
    for (int off = 32; off > 0; off >>= 1) {
      lo[k] = fmin(lo[k], __shfl_xor(lo[k], off, 64));
      hi[k] = fmax(hi[k], __shfl_xor(hi[k], off, 64));
    }
  if (lane == 0) {
    double ov = 0.0;
    for (int k = 0; k < 3; ++k) {
      nbox[(size_t)e * 6 + k] = lo[k];
      nbox[(size_t)e * 6 + 3 + k] = hi[k];
      ov = fmax(ov, fmax(m.elo[e * 3 + k] - lo[k], hi[k] - m.ehi[e * 3 + k]));
    }
    if (ov > 0.0) atomicMax(node_pad, (unsigned long long)__double_as_longlong(ov));
  }
}

// Upper bounds over each element (one wave per element) of G_i = |grad xi_i|
// = |row i of J^-1| and of H_i = |Hessian of xi_i| (Frobenius norm): the
// largest values on reference lattices that include the element's faces,
// edges and corners ((2 n_g + 2)^3 points), times
// kGxiMargin and kHxiMargin; +inf where the sampled Jacobian is not positive.
// Along a path inside the element xi_i changes by at most G_i per unit
// length, so a segment of length L from xi with L G_i < 1 - |xi_i| for every i
// stays inside and crosses no face; H_i bounds the second-order term of the
// same change (Hessian of xi_i = -J^-T (sum_k (J^-1)_ik d2 chi_k) J^-1).
constexpr double kGxiMargin = 1.2;
constexpr double kHxiMargin = 2.0;

__device__ inline bool inv3(const double J[3][3], double K[3][3]) {
  const double dj = det3(J);
  if (!(dj > 0.0)) return false;
  const double id = 1.0 / dj;
  K[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
  K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  K[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
  K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  K[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
  K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  return true;
}

template <int NG>
__global__ __launch_bounds__(64) void k_gxi_bound(MeshView m, double* gxi) {
  const int e = blockIdx.x, lane = threadIdx.x;
  const double* X = m.X + (size_t)e * NG * NG * NG * 3;
  double g[3] = {0.0, 0.0, 0.0}, h[3] = {0.0, 0.0, 0.0};
  bool bad = false;
  constexpr int S = 2 * NG + 2;
  for (int q = lane; q < S * S * S; q += 64) {
    const double xi[3] = {-1.0 + 2.0 * (q % S) / (S - 1), -1.0 + 2.0 * ((q / S) % S) / (S - 1),
                          -1.0 + 2.0 * (q / (S * S)) / (S - 1)};
    double x[3], J[3][3], K[3][3];
    map_jac<NG>(m, X, xi, x, J);
    if (!inv3(J, K)) {
      bad = true;
      continue;
    }
    for (int i = 0; i < 3; ++i) g[i] = fmax(g[i], sqrt(dot3(K[i], K[i])));
  }
  constexpr int SH = 2 * NG + 2;
  for (int q = lane; q < SH * SH * SH; q += 64) {
    const double xi[3] = {-1.0 + 2.0 * (q % SH) / (SH - 1), -1.0 + 2.0 * ((q / SH) % SH) / (SH - 1),
                          -1.0 + 2.0 * (q / (SH * SH)) / (SH - 1)};
    double l[3][NG], dl[3][NG], d2l[3][NG];
    for (int a = 0; a < 3; ++a) lagrange_d2<NG>(m.xgeo, m.cgeo, xi[a], l[a], dl[a], d2l[a]);
    // first and second derivatives of the map: J[k][p], M[k][pq] (pq: 00 11 22 01 02 12)
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, M[3][6] = {{0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0},
                                                                   {0, 0, 0, 0, 0, 0}};
    for (int kk = 0; kk < NG; ++kk)
      for (int jj = 0; jj < NG; ++jj)
        for (int ii = 0; ii < NG; ++ii) {
          const double* P = X + ((kk * NG + jj) * NG + ii) * 3;
          const double b1[3] = {dl[0][ii] * l[1][jj] * l[2][kk], l[0][ii] * dl[1][jj] * l[2][kk],
                                l[0][ii] * l[1][jj] * dl[2][kk]};
          const double b2[6] = {d2l[0][ii] * l[1][jj] * l[2][kk], l[0][ii] * d2l[1][jj] * l[2][kk],
                                l[0][ii] * l[1][jj] * d2l[2][kk], dl[0][ii] * dl[1][jj] * l[2][kk],
                                dl[0][ii] * l[1][jj] * dl[2][kk], l[0][ii] * dl[1][jj] * dl[2][kk]};
          for (int k = 0; k < 3; ++k) {
            for (int p = 0; p < 3; ++p) J[k][p] += P[k] * b1[p];
            for (int r = 0; r < 6; ++r) M[k][r] += P[k] * b2[r];
          }
        }
    double K[3][3];
    if (!inv3(J, K)) {
      bad = true;
      continue;
    }
    for (int i = 0; i < 3; ++i) {
      // T = sum_k K[i][k] M_k (symmetric), H = K^T T K
      double T[3][3];
      const int idx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
      for (int p = 0; p < 3; ++p)
        for (int r = 0; r < 3; ++r)
          T[p][r] = K[i][0] * M[0][idx[p][r]] + K[i][1] * M[1][idx[p][r]] + K[i][2] * M[2][idx[p][r]];
      double f2 = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double v = 0.0;
          for (int p = 0; p < 3; ++p)
            for (int r = 0; r < 3; ++r) v += K[p][a] * T[p][r] * K[r][b];
          f2 += v * v;
        }
      h[i] = fmax(h[i], sqrt(f2));
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int off = 32; off > 0; off >>= 1) {
      g[i] = fmax(g[i], __shfl_xor(g[i], off, 64));
      h[i] = fmax(h[i], __shfl_xor(h[i], off, 64));
    }
  bad = __any(bad);
  if (lane == 0)
    for (int i = 0; i < 3; ++i) {
      gxi[(size_t)e * 6 + i] = bad ? 1e300 : kGxiMargin * g[i];
      gxi[(size_t)e * 6 + 3 + i] = bad ? 1e300 : kHxiMargin * h[i];
    }
}

// ---------------------------------------------------------------------------
// particle location (push): hint element, else background-mesh candidates
// ---------------------------------------------------------------------------
template <int NN, int NG>
__global__ __launch_bounds__(256) void k_locate(MeshView m, Particles P, const int32_t* __restrict__ hint, int64_t n) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t cap = P.cap;
  double x[3] = {P.x[p], P.x[cap + p], P.x[2 * cap + p]};
  double xi[3] = {0, 0, 0};
  int found = -1, it = 0, calls = 0, fb = 0;
  if (hint) {
    int h = hint[p];
    if (h >= 0 && h < m.E && locate_xi<NN, NG>(m, h, x, xi, 50, false, it, calls, fb) && inside_ref(xi)) found = h;
  }
  if (found < 0) {
    int c[3];
    bool in = true;
    for (int k = 0; k < 3; ++k) {
      c[k] = (int)floor((x[k] - m.blo[k]) / m.bdx[k]);
      if (c[k] < 0 || c[k] >= m.bn[k]) in = false;
    }
    if (in) {
      int64_t cell = ((int64_t)c[2] * m.bn[1] + c[1]) * m.bn[0] + c[0];
      for (int q = m.bstart[cell]; q < m.bstart[cell + 1]; ++q) {
        int e = m.blist[q];
        if (x[0] < m.elo[e * 3] || x[0] > m.ehi[e * 3] || x[1] < m.elo[e * 3 + 1] || x[1] > m.ehi[e * 3 + 1] ||
            x[2] < m.elo[e * 3 + 2] || x[2] > m.ehi[e * 3 + 2])
          continue;
        if (locate_xi<NN, NG>(m, e, x, xi, 50, false, it, calls, fb) && inside_ref(xi)) { found = e; break; }
      }
    }
  }
  P.elem[p] = found < 0 ? 0 : found;
  P.status[p] = found < 0 ? REJECTED : ACTIVE;
  P.hits[p] = 0;
  P.id[p] = (int32_t)p;
  for (int k = 0; k < 3; ++k) {
    P.xi[k * cap + p] = xi[k];
    P.kx[k * cap + p] = 0.0;
    P.kv[k * cap + p] = 0.0;
  }
}

// positive doubles order like their bit patterns, so the largest complement
// of the bits is the complement of the smallest value's bits
__global__ __launch_bounds__(256) void k_min_positive(const double* __restrict__ d, int64_t n,
                                                      unsigned long long* inv_bits, int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long m = 0;
  int b = 0;
  if (i < n) {
    const double v = d[i];
    if (v > 0.0 && v < INFINITY) m = ~(unsigned long long)__double_as_longlong(v);
    else b = 1;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
    b += __shfl_xor(b, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (m) atomicMax(inv_bits, m);
    if (b) atomicAdd(bad, b);
  }
}

hipError_t launch_min_positive(const double* d, int64_t n, unsigned long long* inv_bits, int32_t* bad,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_min_positive<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(d, n, inv_bits, bad);
  return hipGetLastError();
}

// reference coordinates of the current positions, with the inside check:
// all n particles, or the list[0 .. *count) the element pass left over
template <int NN, int NG>
__global__ __launch_bounds__(256) void k_finalize(MeshView m, Particles P, int64_t n, const int32_t* __restrict__ list,
                                                  const int32_t* __restrict__ count, int warm,
                                                  unsigned long long* stats) {
  const int64_t cnt = list ? (int64_t)*count : n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int nlost = 0, nrec = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
  const int64_t p = list ? (int64_t)list[i] : i;
  if (P.status[p] == ACTIVE) {
    const int64_t cap = P.cap;
    double x[3] = {P.x[p], P.x[cap + p], P.x[2 * cap + p]};
    double xi[3];
    int it = 0, calls = 0, fb = 0, e = P.elem[p];
    double gw[3];
    const bool wv = warm && warm_guess(P, p, gw);
    bool ok = locate_xi<NN, NG>(m, e, x, xi, 50, false, it, calls, fb, wv, gw);
    bool inside = ok && inside_ref(xi);
    if (!ok) {
      // as in the stage: the background-mesh candidates of the point
      const int f = bgm_locate<NN, NG>(m, x, xi, it, calls, fb);
      if (f >= 0) {
        ok = inside = true;
        nrec++;
        P.elem[p] = f;
      }
    } else if (!inside && recover_elem<NN, NG>(m, e, x, xi, 50, it, calls, fb)) {
      inside = true;
      nrec++;
      P.elem[p] = e;
      for (int k = 0; k < 3; ++k) P.x[k * cap + p] = x[k];
    }
    if (!ok) { P.status[p] = LOST_NEWTON; nlost++; }
    else if (!inside) { P.status[p] = LOST_TRACK; nlost++; }
    for (int k = 0; k < 3; ++k) P.xi[k * cap + p] = xi[k];
  }
  }
  wave_add(stats + ST_LOST * kStatSlots, nlost);
  wave_add(stats + ST_RECOVER * kStatSlots, nrec);
}

// ---------------------------------------------------------------------------
// two-way source at the nearest DOF (Sec. 2.3): S = -F / V_ijk, S_e = -F.v / V,
// F the fluid force of the particle's equation of motion
// ---------------------------------------------------------------------------
template <int NN, int NG, typename UT, typename ST>
__global__ __launch_bounds__(256) void k_deposit_nearest(MeshView m, Particles P, Fluid fl, int64_t n, ST* S,
                                                         ForceModel fm) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || P.status[p] != ACTIVE) return;
  constexpr int N3 = NN * NN * NN;
  const int64_t cap = P.cap;
  int e = P.elem[p];
  // the source is taken in the element that contains the particle: the
  // caller locates every particle before the deposit (reference coordinates
  // in P.xi)
  const double xi[3] = {P.xi[p], P.xi[cap + p], P.xi[2 * cap + p]};
  if (!inside_ref(xi)) return;
  double v[3] = {P.v[p], P.v[cap + p], P.v[2 * cap + p]};
  double F[3];
  source_force<NN, NG, UT>(m, fl, fm, e, xi, v, P.d[p], F);
  double Fv = F[0] * v[0] + F[1] * v[1] + F[2] * v[2];
  int idx[3];
  for (int k = 0; k < 3; ++k) {
    int best = 0;
    double bd = 1e300;
    for (int i = 0; i < NN; ++i) {
      double dd = fabs(xi[k] - m.xdg[i]);
      if (dd < bd) { bd = dd; best = i; }
    }
    idx[k] = best;
  }
  int node = (idx[2] * NN + idx[1]) * NN + idx[0];
  double iV = 1.0 / m.vol[(size_t)e * N3 + node];
  ST* Se = S + (size_t)e * 4 * N3 + node;
  atomicAdd(Se + 0 * N3, (ST)(-F[0] * iV));
  atomicAdd(Se + 1 * N3, (ST)(-F[1] * iV));
  atomicAdd(Se + 2 * N3, (ST)(-F[2] * iV));
  atomicAdd(Se + 3 * N3, (ST)(-Fv * iV));
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#include "fp_shapes.h"

bool supported(int n, int ng) {
#define FP_SUP(A, B) if (n == A && ng == B) return true;
  FP_FOR_EACH_SHAPE(FP_SUP)
#undef FP_SUP
  return false;
}

static inline dim3 grid_for(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

hipError_t launch_face_setup(const MeshView& m, const double* X, const int32_t* nbr_elem, const int32_t* nbr_face,
                             const int8_t* bc, const double* shift, const double* Minv, FaceRec* faces, double* cp,
                             hipStream_t s) {
  MinvArg Mi;
  for (int i = 0; i < kMaxNodes * kMaxNodes; ++i) Mi.v[i] = (i < m.ng * m.ng) ? Minv[i] : 0.0;
  dim3 g = grid_for((int64_t)m.E * 6, 128);
  switch (m.ng) {
    case 2: k_face_setup<2><<<g, 128, 0, s>>>(m.E, X, nbr_elem, nbr_face, bc, shift, Mi, faces, cp); break;
    case 3: k_face_setup<3><<<g, 128, 0, s>>>(m.E, X, nbr_elem, nbr_face, bc, shift, Mi, faces, cp); break;
    case 5: k_face_setup<5><<<g, 128, 0, s>>>(m.E, X, nbr_elem, nbr_face, bc, shift, Mi, faces, cp); break;
    case 7: k_face_setup<7><<<g, 128, 0, s>>>(m.E, X, nbr_elem, nbr_face, bc, shift, Mi, faces, cp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_nodes(const MeshView& m, double* xnode, double* vol, double* hE, double* nbox, double* gxi,
                        int32_t* bad, unsigned long long* node_pad, hipStream_t s) {
  int64_t tot = (int64_t)m.E * m.n * m.n * m.n;
#define FP_L(A, B)                                                                           \
  if (m.n == A && m.ng == B) {                                                               \
    k_nodes<A, B><<<grid_for(tot), 256, 0, s>>>(m, xnode, vol, hE, bad);                     \
    k_node_box<A><<<m.E, 64, 0, s>>>(m, xnode, nbox, node_pad);                              \
    k_gxi_bound<B><<<m.E, 64, 0, s>>>(m, gxi);                                               \
    return hipGetLastError();                                                                \
  }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

hipError_t launch_locate(const MeshView& m, const Particles& P, const int32_t* hint, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
#define FP_L(A, B) \
  if (m.n == A && m.ng == B) { k_locate<A, B><<<grid_for(n), 256, 0, s>>>(m, P, hint, n); return hipGetLastError(); }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const MeshView& m, const Particles& P, int64_t n, const int32_t* list,
                           const int32_t* count, int warm, unsigned long long* stats, hipStream_t s) {
  if (n == 0) return hipSuccess;
  // a list's length is on the device: a grid that strides over it
  const dim3 g = list ? dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)) : grid_for(n);
#define FP_L(A, B)                                                                    \
  if (m.n == A && m.ng == B) {                                                        \
    k_finalize<A, B><<<g, 256, 0, s>>>(m, P, n, list, count, warm, stats);            \
    return hipGetLastError();                                                         \
  }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

hipError_t launch_deposit_nearest(const MeshView& m, const Particles& P, const Fluid& fl, int64_t n, void* S,
                                  int s_f32, const ForceModel& fm, hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 g = grid_for(n);
#define FP_L(A, B)                                                                                              \
  if (m.n == A && m.ng == B) {                                                                                  \
    if (fl.f32 && s_f32) k_deposit_nearest<A, B, float, float><<<g, 256, 0, s>>>(m, P, fl, n, (float*)S, fm);      \
    else if (fl.f32) k_deposit_nearest<A, B, float, double><<<g, 256, 0, s>>>(m, P, fl, n, (double*)S, fm);        \
    else if (s_f32) k_deposit_nearest<A, B, double, float><<<g, 256, 0, s>>>(m, P, fl, n, (float*)S, fm);          \
    else k_deposit_nearest<A, B, double, double><<<g, 256, 0, s>>>(m, P, fl, n, (double*)S, fm);                   \
    return hipGetLastError();                                                                                   \
  }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

}  // namespace fp

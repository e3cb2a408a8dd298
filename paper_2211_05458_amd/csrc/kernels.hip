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
  constexpr int D = NG - 1;
  int d = f / 2, a = (d == 0) ? 1 : 0, b = (d == 2) ? 1 : 2;
  int fix = (f & 1) ? D : 0;
  const double* Xe = X + (size_t)e * NG * NG * NG * 3;
  double T[NG * NG][3];
  // Lagrange nodes -> Bernstein control points: P = M^-1 F M^-T
  for (int n = 0; n < NG; ++n)
    for (int mm = 0; mm < NG; ++mm) {
      double s[3] = {0, 0, 0};
      for (int r = 0; r < NG; ++r) {
        int idx[3];
        idx[d] = fix; idx[a] = r; idx[b] = n;
        const double* P = Xe + ((idx[2] * NG + idx[1]) * NG + idx[0]) * 3;
        double w = Mi.v[mm * NG + r];
        s[0] += w * P[0]; s[1] += w * P[1]; s[2] += w * P[2];
      }
      T[n * NG + mm][0] = s[0]; T[n * NG + mm][1] = s[1]; T[n * NG + mm][2] = s[2];
    }
  double* cp = cpo + (size_t)gid * NG * NG * 3;
  for (int n = 0; n < NG; ++n)
    for (int mm = 0; mm < NG; ++mm) {
      double s[3] = {0, 0, 0};
      for (int r = 0; r < NG; ++r) {
        double w = Mi.v[n * NG + r];
        s[0] += w * T[r * NG + mm][0]; s[1] += w * T[r * NG + mm][1]; s[2] += w * T[r * NG + mm][2];
      }
      cp[(n * NG + mm) * 3 + 0] = s[0]; cp[(n * NG + mm) * 3 + 1] = s[1]; cp[(n * NG + mm) * 3 + 2] = s[2];
    }
  FaceRec F;
  const double* C00 = cp;
  const double* CN0 = cp + D * 3;
  const double* C0N = cp + D * NG * 3;
  const double* CNN = cp + (D * NG + D) * 3;
  double diam = 0.0;
  for (int i = 0; i < NG * NG; ++i)
    for (int j = i + 1; j < NG * NG; ++j) {
      double r[3] = {cp[i * 3] - cp[j * 3], cp[i * 3 + 1] - cp[j * 3 + 1], cp[i * 3 + 2] - cp[j * 3 + 2]};
      diam = fmax(diam, sqrt(dot3(r, r)));
    }
  double g1[3], g2[3], eu[3];
  for (int q = 0; q < 3; ++q) {
    g1[q] = CNN[q] - C00[q];
    g2[q] = C0N[q] - CN0[q];
    eu[q] = (CN0[q] - C00[q]) + (CNN[q] - C0N[q]);
  }
  cross3(g1, g2, F.nrm);
  double il = 1.0 / sqrt(dot3(F.nrm, F.nrm));
  for (int q = 0; q < 3; ++q) F.nrm[q] *= il;
  double pr = dot3(eu, F.nrm);
  for (int q = 0; q < 3; ++q) eu[q] -= pr * F.nrm[q];
  il = 1.0 / sqrt(dot3(eu, eu));
  for (int q = 0; q < 3; ++q) F.e1[q] = eu[q] * il;
  cross3(F.nrm, F.e1, F.e2);
  for (int q = 0; q < 3; ++q) {
    F.org[q] = C00[q];
    F.lo[q] = 1e300;
    F.hi[q] = -1e300;
  }
  for (int i = 0; i < NG * NG; ++i) {
    double r[3] = {cp[i * 3] - F.org[0], cp[i * 3 + 1] - F.org[1], cp[i * 3 + 2] - F.org[2]};
    double p0 = dot3(r, F.nrm), p1 = dot3(r, F.e1), p2 = dot3(r, F.e2);
    F.lo[0] = fmin(F.lo[0], p0); F.hi[0] = fmax(F.hi[0], p0);
    F.lo[1] = fmin(F.lo[1], p1); F.hi[1] = fmax(F.hi[1], p1);
    F.lo[2] = fmin(F.lo[2], p2); F.hi[2] = fmax(F.hi[2], p2);
  }
  F.diam = diam;
  for (int q = 0; q < 3; ++q) {
    F.A[q] = 0.25 * (C00[q] - CN0[q] - C0N[q] + CNN[q]);
    F.B[q] = 0.25 * (-C00[q] + CN0[q] - C0N[q] + CNN[q]);
    F.C[q] = 0.25 * (-C00[q] - CN0[q] + C0N[q] + CNN[q]);
    F.D[q] = 0.25 * (C00[q] + CN0[q] + C0N[q] + CNN[q]);
  }
  double tol = 1e-12 * diam;
  bool planar = (F.hi[0] - F.lo[0]) <= tol;
  bool bilin = true;
  for (int n = 0; n < NG && bilin; ++n)
    for (int mm = 0; mm < NG && bilin; ++mm) {
      double s = (double)mm / D, t = (double)n / D;
      for (int q = 0; q < 3; ++q) {
        double p = (1 - s) * (1 - t) * C00[q] + s * (1 - t) * CN0[q] + (1 - s) * t * C0N[q] + s * t * CNN[q];
        if (fabs(p - cp[(n * NG + mm) * 3 + q]) > tol) { bilin = false; break; }
      }
    }
  double tw = sqrt(dot3(F.A, F.A));
  F.type = (planar && bilin && tw <= tol) ? FACE_PLANAR : (bilin ? FACE_BILINEAR : FACE_CURVED);
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

// reference coordinates of the current positions, with the inside check
template <int NN, int NG>
__global__ __launch_bounds__(256) void k_finalize(MeshView m, Particles P, int64_t n, unsigned long long* stats) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int nlost = 0;
  if (p < n && P.status[p] == ACTIVE) {
    const int64_t cap = P.cap;
    double x[3] = {P.x[p], P.x[cap + p], P.x[2 * cap + p]};
    double xi[3];
    int it = 0, calls = 0, fb = 0;
    bool ok = locate_xi<NN, NG>(m, P.elem[p], x, xi, 50, false, it, calls, fb);
    if (!ok) { P.status[p] = LOST_NEWTON; nlost++; }
    else if (!inside_ref(xi)) { P.status[p] = LOST_TRACK; nlost++; }
    for (int k = 0; k < 3; ++k) P.xi[k * cap + p] = xi[k];
  }
  wave_add(stats + ST_LOST * kStatSlots, nlost);
}

// ---------------------------------------------------------------------------
// two-way source at the nearest DOF (Sec. 2.3): S = -F / V_ijk, S_e = -F.v / V
// ---------------------------------------------------------------------------
template <int NN, int NG, typename UT, typename ST>
__global__ __launch_bounds__(256) void k_deposit_nearest(MeshView m, Particles P, Fluid fl, int64_t n, ST* S,
                                                         int drag) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || P.status[p] != ACTIVE) return;
  constexpr int N3 = NN * NN * NN;
  const int64_t cap = P.cap;
  int e = P.elem[p];
  double x[3] = {P.x[p], P.x[cap + p], P.x[2 * cap + p]};
  double xi[3];
  int it = 0, calls = 0, fb = 0;
  if (!locate_xi<NN, NG>(m, e, x, xi, 50, false, it, calls, fb)) return;
  double Uc[5];
  interp<NN, UT>(m, (const UT*)fl.U + (size_t)e * 5 * N3, xi, Uc);
  double ir = 1.0 / Uc[0];
  double u[3] = {Uc[1] * ir, Uc[2] * ir, Uc[3] * ir};
  double v[3] = {P.v[p], P.v[cap + p], P.v[2 * cap + p]};
  double d = P.d[p], a[3], fD;
  drag_accel<double>(drag, Uc[0], u, v, d, fl.mu, fl.rho_p, a, fD);
  double c = 3.0 * M_PI * fl.mu * d * fD;
  double F[3] = {c * (u[0] - v[0]), c * (u[1] - v[1]), c * (u[2] - v[2])};
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

hipError_t launch_nodes(const MeshView& m, double* xnode, double* vol, double* hE, int32_t* bad, hipStream_t s) {
  int64_t tot = (int64_t)m.E * m.n * m.n * m.n;
#define FP_L(A, B) \
  if (m.n == A && m.ng == B) { k_nodes<A, B><<<grid_for(tot), 256, 0, s>>>(m, xnode, vol, hE, bad); return hipGetLastError(); }
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

hipError_t launch_finalize(const MeshView& m, const Particles& P, int64_t n, unsigned long long* stats,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
#define FP_L(A, B) \
  if (m.n == A && m.ng == B) { k_finalize<A, B><<<grid_for(n), 256, 0, s>>>(m, P, n, stats); return hipGetLastError(); }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

hipError_t launch_deposit_nearest(const MeshView& m, const Particles& P, const Fluid& fl, int64_t n, void* S,
                                  int s_f32, int drag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 g = grid_for(n);
#define FP_L(A, B)                                                                                              \
  if (m.n == A && m.ng == B) {                                                                                  \
    if (fl.f32 && s_f32) k_deposit_nearest<A, B, float, float><<<g, 256, 0, s>>>(m, P, fl, n, (float*)S, drag);    \
    else if (fl.f32) k_deposit_nearest<A, B, float, double><<<g, 256, 0, s>>>(m, P, fl, n, (double*)S, drag);      \
    else if (s_f32) k_deposit_nearest<A, B, double, float><<<g, 256, 0, s>>>(m, P, fl, n, (float*)S, drag);        \
    else k_deposit_nearest<A, B, double, double><<<g, 256, 0, s>>>(m, P, fl, n, (double*)S, drag);                 \
    return hipGetLastError();                                                                                   \
  }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

}  // namespace fp

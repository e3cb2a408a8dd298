// Two-way coupling source with a polynomial shape kernel K(r) = (1-(r/R)^2)^2
// over all DG nodes within R of a particle, normalised per particle so that
// sum_k S_k V_k = -F (the projection keeps the conservation property of the
// nearest-DOF operator of Sec. 2.3 while spreading the source).
//
// Two kernels, no atomics:
//  1. per particle: drag force F and the normalisation sum_j K(r_j) V_j,
//     stored as G = F / norm;
//  2. per target element (one workgroup): every node gathers K(r) G over the
//     particles of the candidate source elements (particles sorted by element).
#include "fp_device.h"
#include "fp_launch.h"

namespace fp {

struct DepGeo {
  double R, R2, iR2;
  double period[3];
};

// element candidates of the box [lo, hi] through the background mesh; each
// element is visited once (in the first background cell of the overlap)
template <typename F>
__device__ inline void for_each_candidate(const MeshView& m, const double* lo, const double* hi, F&& fn) {
  int c0[3], c1[3];
  for (int k = 0; k < 3; ++k) {
    c0[k] = (int)floor((lo[k] - m.blo[k]) / m.bdx[k]);
    c1[k] = (int)floor((hi[k] - m.blo[k]) / m.bdx[k]);
    c0[k] = max(c0[k], 0);
    c1[k] = min(c1[k], m.bn[k] - 1);
    if (c0[k] > c1[k]) return;
  }
  for (int z = c0[2]; z <= c1[2]; ++z)
    for (int y = c0[1]; y <= c1[1]; ++y)
      for (int x = c0[0]; x <= c1[0]; ++x) {
        int64_t cell = ((int64_t)z * m.bn[1] + y) * m.bn[0] + x;
        for (int q = m.bstart[cell]; q < m.bstart[cell + 1]; ++q) {
          int e = m.blist[q];
          int own[3] = {x, y, z};
          bool first = true;
          for (int k = 0; k < 3; ++k) {
            int ec = (int)floor((m.elo[e * 3 + k] - m.blo[k]) / m.bdx[k]);
            ec = max(ec, 0);
            if (own[k] != max(c0[k], ec)) first = false;
          }
          if (!first) continue;
          // box distance test
          bool near = true;
          for (int k = 0; k < 3; ++k)
            if (m.elo[e * 3 + k] > hi[k] || m.ehi[e * 3 + k] < lo[k]) near = false;
          if (near) fn(e);
        }
      }
}

__device__ __forceinline__ void min_image(double* r, const double* period) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (period[k] > 0.0) r[k] -= period[k] * rint(r[k] / period[k]);
}

template <int NN, int NG, typename UT>
__global__ __launch_bounds__(256) void k_dep_force(MeshView m, Particles P, Fluid fl, int64_t n, int drag, DepGeo g,
                                                   double* G) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  constexpr int N3 = NN * NN * NN;
  double* Gp = G + p * 4;
  Gp[0] = Gp[1] = Gp[2] = Gp[3] = 0.0;
  if (P.status[p] != ACTIVE) return;
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
  double F[4] = {c * (u[0] - v[0]), c * (u[1] - v[1]), c * (u[2] - v[2]), 0.0};
  F[3] = F[0] * v[0] + F[1] * v[1] + F[2] * v[2];
  // normalisation over all nodes within R (periodic images by shifted boxes)
  double norm = 0.0;
  int nimg[3];
  for (int k = 0; k < 3; ++k) nimg[k] = g.period[k] > 0.0 ? 3 : 1;
  for (int iz = 0; iz < nimg[2]; ++iz)
    for (int iy = 0; iy < nimg[1]; ++iy)
      for (int ix = 0; ix < nimg[0]; ++ix) {
        int img[3] = {ix == 2 ? -1 : ix, iy == 2 ? -1 : iy, iz == 2 ? -1 : iz};
        double lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
          double cc = x[k] + img[k] * g.period[k];
          lo[k] = cc - g.R;
          hi[k] = cc + g.R;
        }
        for_each_candidate(m, lo, hi, [&](int es) {
          const double* xn = m.xnode + (size_t)es * N3 * 3;
          const double* vol = m.vol + (size_t)es * N3;
          for (int q = 0; q < N3; ++q) {
            double r[3] = {xn[q * 3] - x[0], xn[q * 3 + 1] - x[1], xn[q * 3 + 2] - x[2]};
            min_image(r, g.period);
            double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (r2 < g.R2) {
              double s = 1.0 - r2 * g.iR2;
              norm += s * s * vol[q];
            }
          }
        });
      }
  if (norm > 0.0) {
    double in = 1.0 / norm;
    for (int k = 0; k < 4; ++k) Gp[k] = -F[k] * in;
  }
}

template <int NN, typename ST>
__global__ __launch_bounds__(256) void k_dep_gather(MeshView m, Particles P, const int32_t* __restrict__ elem_start,
                                                    DepGeo g, const double* __restrict__ G, ST* S) {
  int t = blockIdx.x;
  constexpr int N3 = NN * NN * NN;
  constexpr int PER = (N3 + 255) / 256;
  double xn[PER][3], acc[PER][4];
  for (int s = 0; s < PER; ++s) {
    int q = threadIdx.x + s * 256;
    for (int k = 0; k < 4; ++k) acc[s][k] = 0.0;
    for (int k = 0; k < 3; ++k) xn[s][k] = (q < N3) ? m.xnode[((size_t)t * N3 + q) * 3 + k] : 1e300;
  }
  const int64_t cap = P.cap;
  int nimg[3];
  for (int k = 0; k < 3; ++k) nimg[k] = g.period[k] > 0.0 ? 3 : 1;
  for (int iz = 0; iz < nimg[2]; ++iz)
    for (int iy = 0; iy < nimg[1]; ++iy)
      for (int ix = 0; ix < nimg[0]; ++ix) {
        int img[3] = {ix == 2 ? -1 : ix, iy == 2 ? -1 : iy, iz == 2 ? -1 : iz};
        double lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
          lo[k] = m.elo[t * 3 + k] + img[k] * g.period[k] - g.R;
          hi[k] = m.ehi[t * 3 + k] + img[k] * g.period[k] + g.R;
        }
        for_each_candidate(m, lo, hi, [&](int es) {
          for (int p = elem_start[es]; p < elem_start[es + 1]; ++p) {
            double xp[3] = {P.x[p], P.x[cap + p], P.x[2 * cap + p]};
            double G0 = G[(int64_t)p * 4], G1 = G[(int64_t)p * 4 + 1], G2 = G[(int64_t)p * 4 + 2],
                   G3 = G[(int64_t)p * 4 + 3];
            for (int s = 0; s < PER; ++s) {
              double r[3] = {xn[s][0] - xp[0], xn[s][1] - xp[1], xn[s][2] - xp[2]};
              min_image(r, g.period);
              double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
              if (r2 < g.R2) {
                double w = 1.0 - r2 * g.iR2;
                w *= w;
                acc[s][0] += w * G0;
                acc[s][1] += w * G1;
                acc[s][2] += w * G2;
                acc[s][3] += w * G3;
              }
            }
          }
        });
      }
  for (int s = 0; s < PER; ++s) {
    int q = threadIdx.x + s * 256;
    if (q < N3)
      for (int k = 0; k < 4; ++k) {
        ST* dst = S + ((size_t)t * 4 + k) * N3 + q;
        *dst = (ST)((double)*dst + acc[s][k]);
      }
  }
}

#include "fp_shapes.h"

hipError_t launch_deposit_shape(const MeshView& m, const Particles& P, const Fluid& fl, int64_t n, void* S,
                                int s_f32, int drag, double R, const double* period, double* norm_buf,
                                double* force_buf, const int32_t* elem_start, hipStream_t s) {
  (void)norm_buf;
  DepGeo g;
  g.R = R;
  g.R2 = R * R;
  g.iR2 = 1.0 / (R * R);
  for (int k = 0; k < 3; ++k) g.period[k] = period[k];
  dim3 gp((unsigned)((std::max<int64_t>(n, 1) + 255) / 256));
#define FP_L(A, B)                                                                                     \
  if (m.n == A && m.ng == B) {                                                                         \
    if (n > 0) {                                                                                       \
      if (fl.f32) k_dep_force<A, B, float><<<gp, 256, 0, s>>>(m, P, fl, n, drag, g, force_buf);      \
      else k_dep_force<A, B, double><<<gp, 256, 0, s>>>(m, P, fl, n, drag, g, force_buf);            \
    }                                                                                                  \
    if (s_f32) k_dep_gather<A, float><<<m.E, 256, 0, s>>>(m, P, elem_start, g, force_buf, (float*)S);  \
    else k_dep_gather<A, double><<<m.E, 256, 0, s>>>(m, P, elem_start, g, force_buf, (double*)S);     \
    return hipGetLastError();                                                                          \
  }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

}  // namespace fp

/*
 * FP64 CPU oracle for the per-particle Lagrangian step (Kopper et al.,
 * arXiv 2211.05458).  TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the product path.
 * Plain, slow, obviously correct: every sum is written out as the paper defines
 * it, in FP64, without blocking, fusion or reordering.  Built with
 * -O2 -ffp-contract=off, OpenMP over independent particles only.
 *
 * Paper sections followed:
 *   Sec. 3.1  eq. (dgsem_curvedfaces), (dgsem_interpolation): tensor-product
 *             Lagrange geometry of degree Ng and DG state of degree N.
 *   Sec. 3.2.1 eq. (part_interpolation) + Newton for chi(xi) - x = 0 with the
 *             three initial-guess approaches.
 *   Sec. 2.2  drag law eq. (dragforce), (dragfactor), relaxation time in
 *             eq. (stokesnumber).
 *   Sec. 3.1/3.2.2 low-storage Runge-Kutta stage update and the straight stage
 *             trajectory eq. (parttrajectory).
 *   Sec. 3.2.3/3.2.4 physical-space tracking: Bezier faces, bounding boxes,
 *             planar / bilinear / curved (Bezier clipping) intersection, BCs.
 *   Sec. 2.4  hard-sphere specular reflection.
 *   Sec. 2.3  eq. (theory:source): source projected to the nearest DOF, a/V_ijk.
 *   Sec. 4.1.2 Cartesian background mesh for locating points.
 * Readings where the paper is silent are noted at each function.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXG 12           /* max nodes per direction (degree 11) */
#define NEWTON_TOL 1e-10  /* stop once an applied update has max-norm <= tol */
#define INSIDE_EPS 1e-10  /* xi in [-1-eps, 1+eps]^3 counts as inside */
#define UV_EPS 1e-12      /* face parameter tolerance */
#define ENTRY_REL 1e-9    /* entry-face root threshold, relative to the face diameter */
/* sign that turns dp/du x dp/dv of local face f into its outward normal (face
 * parameters are the two other reference axes in increasing order) */
static const double FACE_SIGN[6] = {-1.0, 1.0, 1.0, -1.0, -1.0, 1.0};
#define RECOVER_HOPS 3    /* neighbour hops for a located particle outside its element */
#define CLIP_TOL 1e-12    /* Bezier clipping interval width (parameter space [0,1]) */
#define CLIP_PAD 1e-10    /* relative padding of each clipped interval */
#define CLIP_STACK 16
#define CLIP_STEPS 64

struct or_ctx {
  int E, ng, n_geo, n, N;
  double *X;
  int32_t *nbr_elem, *nbr_face;
  int8_t *bc;
  double *shift;
  double xgeo[MAXG];
  double xdg[MAXG], wdg[MAXG];
  double *xnode;          /* physical DG node positions [E][n^3][3] */
  double *vol;            /* V_ijk [E][n^3] */
  double *hE;             /* element length scale (max corner edge) */
  /* faces: E*6 */
  double *cp;             /* control points [E*6][ng*ng][3] */
  int *ftype;
  double *fframe;         /* [E*6][9]: n, e1, e2 */
  double *forig;          /* [E*6][3] */
  double *flo, *fhi;      /* [E*6][3] extents along (n, e1, e2) */
  double *fdiam;
  /* background mesh */
  double blo[3], bdx[3];
  int bn[3];
  int *bstart, *blist;
  double *elo, *ehi;      /* padded element AABB [E][3] */
  double *dsafe;          /* [E] lower bound of the distance to a boundary face */
  /* non-conforming faces: per big mortar face, (small element, face) x 4 */
  int n_mortar;
  int32_t *mortar;
  /* fluid */
  const double *U;
  double mu, kappa, rho_p;
  /* particles */
  int64_t np;
  double *x, *v, *kx, *kv, *d, *xi;
  int32_t *elem, *hits;
  int8_t *status;
  /* stats */
  int64_t st_newton_it, st_newton_calls, st_cross, st_hits, st_lost, st_fallback, st_recover;
  /* learned guess */
  double *mlp_w;
  uint8_t *mlp_flag;
};

/* ======================================================================== */
/* 1-D bases                                                                 */
/* ======================================================================== */
static void legendre(int n, double x, double* P, double* dP) {
  /* P_n and P_n' by the three-term recurrence */
  double p0 = 1.0, p1 = x, dp0 = 0.0, dp1 = 1.0;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    double dp2 = dp0 + (2.0 * k - 1.0) * p1;
    p0 = p1; p1 = p2; dp0 = dp1; dp1 = dp2;
  }
  *P = p1; *dP = dp1;
}

/* Legendre-Gauss nodes: roots of P_n by Newton, weights 2/((1-x^2) P_n'(x)^2). */
void or_gauss_nodes(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = -cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, z, &P, &dP);
      double dz = P / dP;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double P, dP;
    legendre(n, z, &P, &dP);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
}

/* Legendre-Gauss-Lobatto nodes: +-1 and the roots of P_{n-1}'. */
void or_lobatto_nodes(int n, double* x, double* w) {
  int N = n - 1;
  x[0] = -1.0; x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double z = -cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(N, z, &P, &dP);
      /* (1-z^2) P'' = 2 z P' - N(N+1) P */
      double d2P = (2.0 * z * dP - N * (N + 1.0) * P) / (1.0 - z * z);
      double dz = dP / d2P;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
  for (int i = 0; i <= N; ++i) {
    double P, dP;
    legendre(N, x[i], &P, &dP);
    w[i] = 2.0 / (N * (N + 1.0) * P * P);
  }
}

/* Lagrange basis in product form: l_i(x) = prod_{j!=i} (x - x_j)/(x_i - x_j),
 * and its derivative as the sum over the dropped factor. */
void or_lagrange(int n, const double* nodes, double xi, double* l, double* dl) {
  for (int i = 0; i < n; ++i) {
    double p = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != i) p *= (xi - nodes[j]) / (nodes[i] - nodes[j]);
    l[i] = p;
    if (dl) {
      double s = 0.0;
      for (int m = 0; m < n; ++m) {
        if (m == i) continue;
        double q = 1.0 / (nodes[i] - nodes[m]);
        for (int j = 0; j < n; ++j)
          if (j != i && j != m) q *= (xi - nodes[j]) / (nodes[i] - nodes[j]);
        s += q;
      }
      dl[i] = s;
    }
  }
}

/* Low-storage RK coefficients (Sec. 3.1: the 2N-storage scheme of Carpenter &
 * Kennedy, five stages, fourth order; also the three-stage third-order
 * Williamson scheme used by the curved workloads).  Stage i:
 * k <- A_i k + dt f(y); y <- y + B_i k.  c_i are the stage times. */
void or_rk_coeffs(int scheme, int* stages, double* A, double* B, double* c) {
  if (scheme == 0) {
    static const double a[5] = {0.0, -567301805773.0 / 1357537059087.0,
                                -2404267990393.0 / 2016746695238.0,
                                -3550918686646.0 / 2091501179385.0,
                                -1275806237668.0 / 842570457699.0};
    static const double b[5] = {1432997174477.0 / 9575080441755.0,
                                5161836677717.0 / 13612068292357.0,
                                1720146321549.0 / 2090206949498.0,
                                3134564353537.0 / 4481467310338.0,
                                2277821191437.0 / 14882151754819.0};
    static const double cc[5] = {0.0, 1432997174477.0 / 9575080441755.0,
                                 2526269341429.0 / 6820363962896.0,
                                 2006345519317.0 / 3224310063776.0,
                                 2802321613138.0 / 2924317926251.0};
    *stages = 5;
    for (int i = 0; i < 5; ++i) { A[i] = a[i]; B[i] = b[i]; c[i] = cc[i]; }
  } else {
    *stages = 3;
    A[0] = 0.0; A[1] = -5.0 / 9.0; A[2] = -153.0 / 128.0;
    B[0] = 1.0 / 3.0; B[1] = 15.0 / 16.0; B[2] = 8.0 / 15.0;
    c[0] = 0.0; c[1] = 1.0 / 3.0; c[2] = 3.0 / 4.0;
  }
}

/* ======================================================================== */
/* small vector helpers                                                      */
/* ======================================================================== */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }
static double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}
static double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}
/* Bernstein polynomials of degree deg on t in [0,1] */
static void bernstein(int deg, double t, double* B) {
  for (int m = 0; m <= deg; ++m) B[m] = binom(deg, m) * pow(t, m) * pow(1.0 - t, deg - m);
}
static void bernstein_d(int deg, double t, double* dB) {
  /* d/dt B_m^deg = deg (B_{m-1}^{deg-1} - B_m^{deg-1}) */
  double b[MAXG];
  if (deg == 0) { dB[0] = 0.0; return; }
  bernstein(deg - 1, t, b);
  for (int m = 0; m <= deg; ++m) {
    double lo = (m >= 1) ? b[m - 1] : 0.0;
    double hi = (m <= deg - 1) ? b[m] : 0.0;
    dB[m] = deg * (lo - hi);
  }
}

/* ======================================================================== */
/* mapping chi_e(xi) and its Jacobian (Sec. 3.1, eq. dgsem_curvedfaces in 3-D) */
/* ======================================================================== */
void or_map(const or_ctx* c, int e, const double* xi, double* x, double* Jout) {
  int ng = c->ng;
  double l1[MAXG], l2[MAXG], l3[MAXG], d1[MAXG], d2[MAXG], d3[MAXG];
  or_lagrange(ng, c->xgeo, xi[0], l1, d1);
  or_lagrange(ng, c->xgeo, xi[1], l2, d2);
  or_lagrange(ng, c->xgeo, xi[2], l3, d3);
  double J[3][3] = {{0}};
  double xx[3] = {0, 0, 0};
  const double* X = c->X + (size_t)e * ng * ng * ng * 3;
  for (int k = 0; k < ng; ++k)
    for (int j = 0; j < ng; ++j)
      for (int i = 0; i < ng; ++i) {
        const double* P = X + ((k * ng + j) * ng + i) * 3;
        for (int q = 0; q < 3; ++q) {
          xx[q] += P[q] * l1[i] * l2[j] * l3[k];
          J[q][0] += P[q] * d1[i] * l2[j] * l3[k];
          J[q][1] += P[q] * l1[i] * d2[j] * l3[k];
          J[q][2] += P[q] * l1[i] * l2[j] * d3[k];
        }
      }
  for (int q = 0; q < 3; ++q) x[q] = xx[q];
  if (Jout)
    for (int q = 0; q < 3; ++q)
      for (int d = 0; d < 3; ++d) Jout[q * 3 + d] = J[q][d];
}

static int inside_ref(const double* xi) {
  return fabs(xi[0]) <= 1.0 + INSIDE_EPS && fabs(xi[1]) <= 1.0 + INSIDE_EPS &&
         fabs(xi[2]) <= 1.0 + INSIDE_EPS;
}

/* Newton for chi(xi) - x = 0 (Sec. 3.2.1).  Reading (paper silent): the linear
 * system J dxi = -F is solved by Cramer's rule; stop after an applied update
 * with max-norm <= 1e-10; at most 50 iterations; declare divergence when
 * |xi|_inf > 2 after the third iteration.  Returns 1 on convergence. */
static int newton_core(const or_ctx* c, int e, const double* x, const double* xi0, double* xi,
                       int* iters, int max_it) {
  double z[3] = {xi0[0], xi0[1], xi0[2]};
  for (int it = 1; it <= max_it; ++it) {
    double F[3], Jf[9], J[3][3];
    or_map(c, e, z, F, Jf);
    for (int q = 0; q < 3; ++q) {
      F[q] -= x[q];
      for (int d = 0; d < 3; ++d) J[q][d] = Jf[q * 3 + d];
    }
    double det = det3(J);
    if (det == 0.0 || !isfinite(det)) { *iters = it; return 0; }
    double dz[3];
    for (int d = 0; d < 3; ++d) {
      double M[3][3];
      memcpy(M, J, sizeof(M));
      for (int q = 0; q < 3; ++q) M[q][d] = -F[q];
      dz[d] = det3(M) / det;
    }
    double dmax = 0.0;
    for (int d = 0; d < 3; ++d) {
      z[d] += dz[d];
      if (fabs(dz[d]) > dmax) dmax = fabs(dz[d]);
    }
    if (!isfinite(z[0]) || !isfinite(z[1]) || !isfinite(z[2])) { *iters = it; return 0; }
    if (dmax <= NEWTON_TOL) {
      xi[0] = z[0]; xi[1] = z[1]; xi[2] = z[2];
      *iters = it;
      return 1;
    }
    if (it >= 3 && (fabs(z[0]) > 2.0 || fabs(z[1]) > 2.0 || fabs(z[2]) > 2.0)) { *iters = it; return 0; }
  }
  *iters = max_it;
  return 0;
}

/* Initial guess (Sec. 3.2.1).  Straight-sided elements (Ng = 1): the nearest
 * DG interpolation point in physical space (approach 1); curved elements: the
 * nearest geometry (mesh) node (approach 2).  Ties go to the lowest node index. */
void or_guess(const or_ctx* c, int e, const double* x, double* xi0) {
  if (c->n_geo == 1) {
    int n = c->n, best = 0;
    double bd = INFINITY;
    const double* P = c->xnode + (size_t)e * n * n * n * 3;
    for (int q = 0; q < n * n * n; ++q) {
      double dx = P[q * 3] - x[0], dy = P[q * 3 + 1] - x[1], dz = P[q * 3 + 2] - x[2];
      double dd = dx * dx + dy * dy + dz * dz;
      if (dd < bd) { bd = dd; best = q; }
    }
    xi0[0] = c->xdg[best % n];
    xi0[1] = c->xdg[(best / n) % n];
    xi0[2] = c->xdg[best / (n * n)];
  } else {
    int ng = c->ng, best = 0;
    double bd = INFINITY;
    const double* P = c->X + (size_t)e * ng * ng * ng * 3;
    for (int q = 0; q < ng * ng * ng; ++q) {
      double dx = P[q * 3] - x[0], dy = P[q * 3 + 1] - x[1], dz = P[q * 3 + 2] - x[2];
      double dd = dx * dx + dy * dy + dz * dz;
      if (dd < bd) { bd = dd; best = q; }
    }
    xi0[0] = c->xgeo[best % ng];
    xi0[1] = c->xgeo[(best / ng) % ng];
    xi0[2] = c->xgeo[best / (ng * ng)];
  }
}

/* Third approach (Sec. 3.2.1): project x - x_E onto the directions to the
 * barycentres of opposite faces.  Reading: x_E is the mean of all geometry
 * nodes, a face barycentre the mean of that face's nodes, and
 * xi_d = 0.5 (<r, s+>/|s+|^2 - <r, s->/|s-|^2), clamped to [-1, 1]. */
void or_guess_faces(const or_ctx* c, int e, const double* x, double* xi0) {
  int ng = c->ng;
  const double* P = c->X + (size_t)e * ng * ng * ng * 3;
  double xe[3] = {0, 0, 0};
  for (int q = 0; q < ng * ng * ng; ++q)
    for (int k = 0; k < 3; ++k) xe[k] += P[q * 3 + k];
  for (int k = 0; k < 3; ++k) xe[k] /= (double)(ng * ng * ng);
  double r[3] = {x[0] - xe[0], x[1] - xe[1], x[2] - xe[2]};
  for (int d = 0; d < 3; ++d) {
    double s[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int side = 0; side < 2; ++side) {
      int fix = side ? ng - 1 : 0;
      for (int b = 0; b < ng; ++b)
        for (int a = 0; a < ng; ++a) {
          int idx[3];
          idx[d] = fix;
          idx[d == 0 ? 1 : 0] = a;
          idx[d == 2 ? 1 : 2] = b;
          const double* Q = P + ((idx[2] * ng + idx[1]) * ng + idx[0]) * 3;
          for (int k = 0; k < 3; ++k) s[side][k] += Q[k];
        }
      for (int k = 0; k < 3; ++k) s[side][k] = s[side][k] / (double)(ng * ng) - xe[k];
    }
    double v = 0.5 * (dot3(r, s[1]) / dot3(s[1], s[1]) - dot3(r, s[0]) / dot3(s[0], s[0]));
    if (v > 1.0) v = 1.0;
    if (v < -1.0) v = -1.0;
    xi0[d] = v;
  }
}

static double* mlp_forward1(const double* w, const double* in, double* out);

/* Newton with the guess chain: learned guess (if enabled for this element),
 * then the paper's guess, then the face-barycentre guess. */
static int newton_chain(const or_ctx* c, int e, const double* x, double* xi, int max_it,
                        int use_mlp, int64_t* it_sum, int64_t* calls, int64_t* fallbacks) {
  double g[3];
  int it = 0;
  if (use_mlp && c->mlp_w && c->mlp_flag && c->mlp_flag[e]) {
    double feat[OR_MLP_NIN];
    or_mlp_features(c, e, x, feat);
    mlp_forward1(c->mlp_w, feat, g);
    int ok = newton_core(c, e, x, g, xi, &it, max_it);
    *it_sum += it; *calls += 1;
    if (ok) return 1;
    *fallbacks += 1;
  }
  or_guess(c, e, x, g);
  int ok = newton_core(c, e, x, g, xi, &it, max_it);
  *it_sum += it; *calls += 1;
  if (ok) return 1;
  *fallbacks += 1;
  or_guess_faces(c, e, x, g);
  ok = newton_core(c, e, x, g, xi, &it, max_it);
  *it_sum += it; *calls += 1;
  return ok;
}

int or_newton(or_ctx* c, int e, const double* x, const double* xi0, double* xi, int* iters) {
  return newton_core(c, e, x, xi0, xi, iters, 50);
}

/* ======================================================================== */
/* interpolation (eq. part_interpolation) and primitives                     */
/* ======================================================================== */
void or_interp(const or_ctx* c, int e, const double* xi, double* Uout) {
  int n = c->n, n3 = n * n * n;
  double l1[MAXG], l2[MAXG], l3[MAXG];
  or_lagrange(n, c->xdg, xi[0], l1, NULL);
  or_lagrange(n, c->xdg, xi[1], l2, NULL);
  or_lagrange(n, c->xdg, xi[2], l3, NULL);
  const double* U = c->U + (size_t)e * 5 * n3;
  for (int var = 0; var < 5; ++var) {
    double s = 0.0;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) s += U[var * n3 + (k * n + j) * n + i] * l1[i] * l2[j] * l3[k];
    Uout[var] = s;
  }
}

/* primitive state (rho, u1, u2, u3, p) from the conservative one (Sec. 2.1/3.2.1) */
static void cons2prim(double kappa, const double* U, double* prim) {
  prim[0] = U[0];
  prim[1] = U[1] / U[0];
  prim[2] = U[2] / U[0];
  prim[3] = U[3] / U[0];
  prim[4] = (kappa - 1.0) * (U[4] - 0.5 * U[0] * (prim[1] * prim[1] + prim[2] * prim[2] + prim[3] * prim[3]));
}

/* Drag acceleration (Sec. 2.2.1): F_D = 3 pi mu d f_D (u - v), with
 * m_p = rho_p pi d^3/6 this is a = f_D (u - v)/tau_p, tau_p = rho_p d^2/(18 mu).
 * f_D: 1 (Stokes) or 1 + 0.15 Re^0.687 (Schiller-Naumann, Re < 800); the paper
 * gives no value at Re >= 800, read here as the Newton regime 0.44 Re/24.
 * drag == 2 switches drag off (ballistic tests). */
void or_drag_accel(const or_ctx* c, int drag, const double* prim, const double* v, double d,
                   const double* g, double* a, double* fD_out) {
  double w[3] = {prim[1] - v[0], prim[2] - v[1], prim[3] - v[2]};
  double fD = 1.0;
  if (drag == 1) {
    double Re = prim[0] * norm3(w) * d / c->mu;
    fD = (Re < 800.0) ? 1.0 + 0.15 * pow(Re, 0.687) : 0.44 * Re / 24.0;
  }
  double tau = c->rho_p * d * d / (18.0 * c->mu);
  for (int q = 0; q < 3; ++q) a[q] = (drag == 2 ? 0.0 : fD * w[q] / tau) + (g ? g[q] : 0.0);
  if (fD_out) *fD_out = (drag == 2) ? 0.0 : fD;
}

/* Primitive state and physical velocity gradient G[i][j] = du_i/dx_j at xi
 * (needed by the undisturbed-flow stress, added mass and lift, Sec. 2.2):
 * derivatives of the interpolant (eq. part_interpolation) with respect to
 * xi_d, then the chain rule df/dx_j = sum_d df/dxi_d (J^-1)_dj with J the
 * element map's Jacobian at xi, and u = m / rho:
 * du_i/dx_j = (dm_i/dx_j - u_i drho/dx_j) / rho. */
void or_fluid_grad(const or_ctx* c, int e, const double* xi, double* prim, double* G) {
  int n = c->n, n3 = n * n * n;
  double l[3][MAXG], dl[3][MAXG];
  for (int d = 0; d < 3; ++d) or_lagrange(n, c->xdg, xi[d], l[d], dl[d]);
  const double* U = c->U + (size_t)e * 5 * n3;
  double Uc[5], dU[4][3];
  for (int var = 0; var < 5; ++var) {
    double s = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double u = U[var * n3 + (k * n + j) * n + i];
          s += u * l[0][i] * l[1][j] * l[2][k];
          s0 += u * dl[0][i] * l[1][j] * l[2][k];
          s1 += u * l[0][i] * dl[1][j] * l[2][k];
          s2 += u * l[0][i] * l[1][j] * dl[2][k];
        }
    Uc[var] = s;
    if (var < 4) { dU[var][0] = s0; dU[var][1] = s1; dU[var][2] = s2; }
  }
  cons2prim(c->kappa, Uc, prim);
  double x[3], Jf[9];
  or_map(c, e, xi, x, Jf);
  /* inverse of J by cofactors */
  double Ji[9];
  Ji[0] = Jf[4] * Jf[8] - Jf[5] * Jf[7];
  Ji[1] = Jf[2] * Jf[7] - Jf[1] * Jf[8];
  Ji[2] = Jf[1] * Jf[5] - Jf[2] * Jf[4];
  Ji[3] = Jf[5] * Jf[6] - Jf[3] * Jf[8];
  Ji[4] = Jf[0] * Jf[8] - Jf[2] * Jf[6];
  Ji[5] = Jf[2] * Jf[3] - Jf[0] * Jf[5];
  Ji[6] = Jf[3] * Jf[7] - Jf[4] * Jf[6];
  Ji[7] = Jf[1] * Jf[6] - Jf[0] * Jf[7];
  Ji[8] = Jf[0] * Jf[4] - Jf[1] * Jf[3];
  double det = Jf[0] * Ji[0] + Jf[1] * Ji[3] + Jf[2] * Ji[6];
  for (int q = 0; q < 9; ++q) Ji[q] /= det;
  double gx[4][3];   /* physical gradients of rho, m1, m2, m3 */
  for (int var = 0; var < 4; ++var)
    for (int jx = 0; jx < 3; ++jx)
      gx[var][jx] = dU[var][0] * Ji[0 * 3 + jx] + dU[var][1] * Ji[1 * 3 + jx] + dU[var][2] * Ji[2 * 3 + jx];
  for (int i = 0; i < 3; ++i)
    for (int jx = 0; jx < 3; ++jx) G[i * 3 + jx] = (gx[1 + i][jx] - prim[1 + i] * gx[0][jx]) / prim[0];
}

/* Particle acceleration and fluid force from the generalised equation of
 * motion (eq. theory:maxey) with the terms selected in `forces`:
 *   m_p dv/dt = F_D + m_f Du/Dt + m_f/2 (Du/Dt - dv/dt) + F_L + g (m_p - m_f),
 * m_p = rho_p pi d^3/6, m_f = rho pi d^3/6 (r = rho/rho_p).  The fluid state
 * is frozen over a step, so Du/Dt = (u . grad) u.  Basset history and Magnus
 * lift are not included.  Without OR_F_BUOYANCY the body force is g m_p (the
 * model of the other configurations); with OR_F_ADDED_MASS the dv/dt term is
 * moved to the left: (1 + r/2) dv/dt = ...  Saffman lift (Sec. 2.2.2) with
 * Mei's correction, read as C_S = (1 - 0.3314 sqrt(th)) exp(-Re/10)
 * + 0.3314 sqrt(th) for Re <= 40 (the bracketing that meets the Re > 40 branch
 * 0.0524 sqrt(th Re) at Re = 40), th = d |w| / (2 |u - v|) limited to
 * [0.005, 0.4], and with the direction (u - v) x w (w the vorticity): the
 * relative velocity of the paper's cross product is read as particle minus
 * fluid, which turns a particle that lags the fluid in a shear flow towards
 * the faster fluid (Saffman's result).
 * a[3]: dv/dt; F[3] (may be NULL): the fluid force of the two-way source
 * (eq. theory:source): F_D + m_f Du/Dt + m_f/2 (Du/Dt - dv/dt) + F_L. */
void or_particle_accel(const or_ctx* c, int drag, int forces, const double* prim, const double* G,
                       const double* v, double d, const double* g, double* a, double* F) {
  double w[3] = {prim[1] - v[0], prim[2] - v[1], prim[3] - v[2]};
  double aD[3], fD;
  or_drag_accel(c, drag, prim, v, d, NULL, aD, &fD);
  double r = prim[0] / c->rho_p;
  double DuDt[3] = {0, 0, 0}, aL[3] = {0, 0, 0};
  if (forces & (OR_F_STRESS | OR_F_ADDED_MASS))
    for (int i = 0; i < 3; ++i) DuDt[i] = G[i * 3 + 0] * prim[1] + G[i * 3 + 1] * prim[2] + G[i * 3 + 2] * prim[3];
  if (forces & OR_F_SAFFMAN) {
    double om[3] = {G[2 * 3 + 1] - G[1 * 3 + 2], G[0 * 3 + 2] - G[2 * 3 + 0], G[1 * 3 + 0] - G[0 * 3 + 1]};
    double wo = norm3(om), ww = norm3(w);
    if (wo > 0.0 && ww > 0.0) {
      double Re = prim[0] * ww * d / c->mu;
      double th = d * wo / (2.0 * ww);
      if (th < 0.005) th = 0.005;
      if (th > 0.4) th = 0.4;
      double CS = (Re <= 40.0) ? (1.0 - 0.3314 * sqrt(th)) * exp(-0.1 * Re) + 0.3314 * sqrt(th)
                               : 0.0524 * sqrt(th * Re);
      double mp = c->rho_p * M_PI * d * d * d / 6.0;
      double coef = 6.46 / 4.0 * CS * d * d * sqrt(prim[0] * c->mu / wo) / mp;
      double cr[3];
      cross3(w, om, cr);
      for (int q = 0; q < 3; ++q) aL[q] = coef * cr[q];
    }
  }
  double cs = ((forces & OR_F_STRESS) ? 1.0 : 0.0) + ((forces & OR_F_ADDED_MASS) ? 0.5 : 0.0);
  double den = (forces & OR_F_ADDED_MASS) ? 1.0 + 0.5 * r : 1.0;
  double gb = (forces & OR_F_BUOYANCY) ? 1.0 - r : 1.0;
  for (int q = 0; q < 3; ++q) a[q] = (aD[q] + cs * r * DuDt[q] + aL[q] + gb * (g ? g[q] : 0.0)) / den;
  if (F) {
    /* drag as in eq. dragforce, the other terms per unit particle mass times m_p */
    double mp = c->rho_p * M_PI * d * d * d / 6.0;
    for (int q = 0; q < 3; ++q) {
      double f = aL[q];
      if (forces & OR_F_STRESS) f += r * DuDt[q];
      if (forces & OR_F_ADDED_MASS) f += 0.5 * r * (DuDt[q] - a[q]);
      F[q] = 3.0 * M_PI * c->mu * d * fD * w[q] + mp * f;
    }
  }
}

/* ======================================================================== */
/* faces: Lagrange -> Bernstein control points, type, slab bounding box      */
/* ======================================================================== */
static void invert(int n, double* M) {
  /* Gauss-Jordan with partial pivoting, in place, n <= MAXG */
  double A[MAXG][2 * MAXG];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) A[i][j] = (j < n) ? M[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (piv != col)
      for (int j = 0; j < 2 * n; ++j) { double t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
    double p = A[col][col];
    for (int j = 0; j < 2 * n; ++j) A[col][j] /= p;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = A[r][col];
      for (int j = 0; j < 2 * n; ++j) A[r][j] -= f * A[col][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) M[i * n + j] = A[i][j + n];
}

/* face f of an element: fixed axis d = f/2 at side f%2; free axes in
 * increasing order give the face parameters (u, v) */
static void face_axes(int f, int* d, int* a, int* b) {
  *d = f / 2;
  *a = (*d == 0) ? 1 : 0;
  *b = (*d == 2) ? 1 : 2;
}

/* Control points of the Bezier form of face f (Sec. 3.2.4): P = M^-1 F M^-T
 * with M_ab = B_b(t_a) the Bernstein-Vandermonde matrix on the geometry nodes. */
static void build_face(or_ctx* c, int e, int f) {
  int ng = c->ng, deg = ng - 1;
  int d, a, b;
  face_axes(f, &d, &a, &b);
  int fix = (f % 2) ? ng - 1 : 0;
  const double* X = c->X + (size_t)e * ng * ng * ng * 3;
  double F[MAXG * MAXG][3];
  for (int nn = 0; nn < ng; ++nn)
    for (int m = 0; m < ng; ++m) {
      int idx[3];
      idx[d] = fix; idx[a] = m; idx[b] = nn;
      const double* P = X + ((idx[2] * ng + idx[1]) * ng + idx[0]) * 3;
      for (int q = 0; q < 3; ++q) F[nn * ng + m][q] = P[q];
    }
  double M[MAXG * MAXG];
  for (int i = 0; i < ng; ++i) {
    double Bv[MAXG];
    bernstein(deg, 0.5 * (c->xgeo[i] + 1.0), Bv);
    for (int j = 0; j < ng; ++j) M[i * ng + j] = Bv[j];
  }
  invert(ng, M);
  double T[MAXG * MAXG][3];
  /* along m (u) */
  for (int nn = 0; nn < ng; ++nn)
    for (int m = 0; m < ng; ++m)
      for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (int r = 0; r < ng; ++r) s += M[m * ng + r] * F[nn * ng + r][q];
        T[nn * ng + m][q] = s;
      }
  double* cp = c->cp + ((size_t)e * 6 + f) * ng * ng * 3;
  for (int nn = 0; nn < ng; ++nn)
    for (int m = 0; m < ng; ++m)
      for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (int r = 0; r < ng; ++r) s += M[nn * ng + r] * T[r * ng + m][q];
        cp[(nn * ng + m) * 3 + q] = s;
      }
  /* corners */
  const double* C00 = cp;
  const double* CN0 = cp + deg * 3;
  const double* C0N = cp + deg * ng * 3;
  const double* CNN = cp + (deg * ng + deg) * 3;
  double diam = 0.0;
  for (int i = 0; i < ng * ng; ++i)
    for (int j = i + 1; j < ng * ng; ++j) {
      double r[3] = {cp[i * 3] - cp[j * 3], cp[i * 3 + 1] - cp[j * 3 + 1], cp[i * 3 + 2] - cp[j * 3 + 2]};
      double l = norm3(r);
      if (l > diam) diam = l;
    }
  /* frame: normal from the diagonals, e1 along the mean u edge */
  double g1[3], g2[3], nrm[3], e1[3], e2[3];
  for (int q = 0; q < 3; ++q) { g1[q] = CNN[q] - C00[q]; g2[q] = C0N[q] - CN0[q]; }
  cross3(g1, g2, nrm);
  double ln = norm3(nrm);
  for (int q = 0; q < 3; ++q) nrm[q] /= ln;
  double eu[3];
  for (int q = 0; q < 3; ++q) eu[q] = (CN0[q] - C00[q]) + (CNN[q] - C0N[q]);
  double pr = dot3(eu, nrm);
  for (int q = 0; q < 3; ++q) eu[q] -= pr * nrm[q];
  double le = norm3(eu);
  for (int q = 0; q < 3; ++q) e1[q] = eu[q] / le;
  cross3(nrm, e1, e2);
  double* fr = c->fframe + ((size_t)e * 6 + f) * 9;
  double* org = c->forig + ((size_t)e * 6 + f) * 3;
  double* lo = c->flo + ((size_t)e * 6 + f) * 3;
  double* hi = c->fhi + ((size_t)e * 6 + f) * 3;
  for (int q = 0; q < 3; ++q) { fr[q] = nrm[q]; fr[3 + q] = e1[q]; fr[6 + q] = e2[q]; org[q] = C00[q]; }
  for (int ax = 0; ax < 3; ++ax) { lo[ax] = INFINITY; hi[ax] = -INFINITY; }
  for (int i = 0; i < ng * ng; ++i) {
    double r[3] = {cp[i * 3] - org[0], cp[i * 3 + 1] - org[1], cp[i * 3 + 2] - org[2]};
    for (int ax = 0; ax < 3; ++ax) {
      double p = dot3(r, fr + 3 * ax);
      if (p < lo[ax]) lo[ax] = p;
      if (p > hi[ax]) hi[ax] = p;
    }
  }
  c->fdiam[e * 6 + f] = diam;
  /* classification (Sec. 3.2.4): zero-thickness box -> planar; a planar face
   * that is a parallelogram uses the planar formula, every face equal to the
   * degree-elevated bilinear patch of its corners uses the bilinear method,
   * everything else is curved. */
  double tol = 1e-12 * diam;
  int planar = (hi[0] - lo[0]) <= tol;
  double twist[3];
  for (int q = 0; q < 3; ++q) twist[q] = 0.25 * (C00[q] - CN0[q] - C0N[q] + CNN[q]);
  int bilin = 1;
  for (int nn = 0; nn < ng && bilin; ++nn)
    for (int m = 0; m < ng; ++m) {
      double s = (double)m / deg, t = (double)nn / deg;
      for (int q = 0; q < 3; ++q) {
        double p = (1 - s) * (1 - t) * C00[q] + s * (1 - t) * CN0[q] + (1 - s) * t * C0N[q] + s * t * CNN[q];
        if (fabs(p - cp[(nn * ng + m) * 3 + q]) > tol) { bilin = 0; break; }
      }
      if (!bilin) break;
    }
  int type;
  if (planar && bilin && norm3(twist) <= tol) type = OR_FACE_PLANAR;
  else if (bilin) type = OR_FACE_BILINEAR;
  else type = OR_FACE_CURVED;
  c->ftype[e * 6 + f] = type;
}

int or_face_info(const or_ctx* c, int e, int f, double* cp, int* type) {
  int ng = c->ng;
  if (cp) memcpy(cp, c->cp + ((size_t)e * 6 + f) * ng * ng * 3, sizeof(double) * ng * ng * 3);
  if (type) *type = c->ftype[e * 6 + f];
  return ng;
}

/* conservative segment / slab-box overlap test (Sec. 3.2.4: boxes reject faces) */
static int bbox_hit(const or_ctx* c, int fid, const double* xs, const double* xe) {
  const double* fr = c->fframe + (size_t)fid * 9;
  const double* org = c->forig + (size_t)fid * 3;
  double pad = 1e-9 * c->fdiam[fid];
  double r0[3] = {xs[0] - org[0], xs[1] - org[1], xs[2] - org[2]};
  double r1[3] = {xe[0] - org[0], xe[1] - org[1], xe[2] - org[2]};
  for (int ax = 0; ax < 3; ++ax) {
    double p0 = dot3(r0, fr + 3 * ax), p1 = dot3(r1, fr + 3 * ax);
    double mn = p0 < p1 ? p0 : p1, mx = p0 < p1 ? p1 : p0;
    if (mx < c->flo[fid * 3 + ax] - pad || mn > c->fhi[fid * 3 + ax] + pad) return 0;
  }
  return 1;
}

/* projection planes (Sec. 3.2.4, curved faces): n1 orthogonal to the ray,
 * n2 = n1 x t.  Reading: n1 = normalize(t x e_k) with e_k the axis of the
 * smallest |t_k| (lowest k on ties). */
static void ray_planes(const double* t, double* n1, double* n2) {
  int k = 0;
  if (fabs(t[1]) < fabs(t[k])) k = 1;
  if (fabs(t[2]) < fabs(t[k])) k = 2;
  double ek[3] = {0, 0, 0};
  ek[k] = 1.0;
  cross3(t, ek, n1);
  double l = norm3(n1);
  for (int q = 0; q < 3; ++q) n1[q] /= l;
  cross3(n1, t, n2);
}

/* corner coefficients of the bilinear form p = A uv + B u + C v + D */
static void bilinear_coeffs(const double* C00, const double* CN0, const double* C0N, const double* CNN,
                            double* A, double* B, double* C, double* D) {
  for (int q = 0; q < 3; ++q) {
    A[q] = 0.25 * (C00[q] - CN0[q] - C0N[q] + CNN[q]);
    B[q] = 0.25 * (-C00[q] + CN0[q] - C0N[q] + CNN[q]);
    C[q] = 0.25 * (-C00[q] - CN0[q] + C0N[q] + CNN[q]);
    D[q] = 0.25 * (C00[q] + CN0[q] + C0N[q] + CNN[q]);
  }
}

/* Planar (parallelogram) face, Sec. 3.2.4: alpha = ((x_m - x0).n)/(t.n) with
 * the face mid point x_m; (u, v) from p = a u + b v + c solved analytically
 * (normal equations of the 2 x 3 system). */
static int planar_intersect(const double* A, const double* B, const double* C, const double* D,
                            const double* x0, const double* t, double* alpha, double* uv) {
  (void)A;
  double nrm[3];
  cross3(B, C, nrm);
  double tn = dot3(t, nrm);
  if (tn == 0.0) return 0;
  double r[3] = {D[0] - x0[0], D[1] - x0[1], D[2] - x0[2]};
  double al = dot3(r, nrm) / tn;
  double xh[3] = {x0[0] + al * t[0] - D[0], x0[1] + al * t[1] - D[1], x0[2] + al * t[2] - D[2]};
  double bb = dot3(B, B), bc = dot3(B, C), cc = dot3(C, C);
  double rb = dot3(xh, B), rc = dot3(xh, C);
  double det = bb * cc - bc * bc;
  alpha[0] = al;
  uv[0] = (rb * cc - rc * bc) / det;
  uv[1] = (bb * rc - bc * rb) / det;
  return 1;
}

/* Bilinear patch (Sec. 3.2.4, after Ramsey et al.): project onto the two ray
 * planes, giving A_k uv + B_k u + C_k v + D_k = 0 (k = 1, 2); eliminating u
 * leaves a quadratic in v, solved by the cancellation-free formula. */
static int bilinear_intersect(const double* A, const double* B, const double* C, const double* D,
                              const double* x0, const double* t, double* alpha, double* uv) {
  double n1[3], n2[3];
  ray_planes(t, n1, n2);
  double Dr[3] = {D[0] - x0[0], D[1] - x0[1], D[2] - x0[2]};
  double a1 = dot3(A, n1), b1 = dot3(B, n1), c1 = dot3(C, n1), d1 = dot3(Dr, n1);
  double a2 = dot3(A, n2), b2 = dot3(B, n2), c2 = dot3(C, n2), d2 = dot3(Dr, n2);
  double qa = a1 * c2 - a2 * c1;
  double qb = a1 * d2 + b1 * c2 - a2 * d1 - b2 * c1;
  double qc = b1 * d2 - b2 * d1;
  double vs[2];
  int nv = 0;
  double scale = fabs(qa) > fabs(qb) ? fabs(qa) : fabs(qb);
  if (fabs(qc) > scale) scale = fabs(qc);
  if (scale == 0.0) return 0;
  if (fabs(qa) <= 1e-14 * scale) {
    if (qb != 0.0) vs[nv++] = -qc / qb;
  } else {
    double disc = qb * qb - 4.0 * qa * qc;
    if (disc < 0.0) return 0;
    double sq = sqrt(disc);
    double q = -0.5 * (qb + (qb >= 0.0 ? sq : -sq));
    vs[nv++] = q / qa;
    if (q != 0.0) vs[nv++] = qc / q;
  }
  int nr = 0;
  for (int i = 0; i < nv; ++i) {
    double v = vs[i];
    double den1 = a1 * v + b1, den2 = a2 * v + b2;
    double u;
    if (fabs(den1) >= fabs(den2)) {
      if (den1 == 0.0) continue;
      u = -(c1 * v + d1) / den1;
    } else {
      u = -(c2 * v + d2) / den2;
    }
    double p[3];
    for (int q = 0; q < 3; ++q) p[q] = A[q] * u * v + B[q] * u + C[q] * v + D[q] - x0[q];
    alpha[nr] = dot3(p, t);
    uv[2 * nr] = u;
    uv[2 * nr + 1] = v;
    nr++;
  }
  return nr;
}

/* ---- Bezier clipping (Sec. 3.2.4; Nishita et al. 1990) --------------------- */
typedef struct {
  /* [m along u][n along v]: signed distances of the control points to the two
   * planes that contain the line (0, 1) and their displacement along it (2) */
  double q[MAXG][MAXG][3];
  double u0, u1, v0, v1;     /* parameter interval in [0,1] */
} clip_patch;

/* Reading (the paper leaves the clipping loop to the literature): a
 * sub-patch whose control points all have displacement outside [amin, amax]
 * holds no root in that band (convex hull) and is dropped.  At grazing
 * incidence the zero set of the two plane distances is a long thin band in
 * (u, v) of which only the part within the stage segment matters; without
 * this test the clipping budget can run out before the root is isolated. */
static int patch_outside_band(const clip_patch* P, int ng, double amin, double amax) {
  double lo = INFINITY, hi = -INFINITY;
  for (int m = 0; m < ng; ++m)
    for (int n = 0; n < ng; ++n) {
      if (P->q[m][n][2] < lo) lo = P->q[m][n][2];
      if (P->q[m][n][2] > hi) hi = P->q[m][n][2];
    }
  return hi < amin || lo > amax;
}

/* interval of t where the convex hull of (t_m, dmin_m), (t_m, dmax_m) meets 0 */
static int hull_zero(int ng, const double* dmin, const double* dmax, double* ta, double* tb) {
  double tt[2 * MAXG], dd[2 * MAXG];
  int np = 0;
  for (int m = 0; m < ng; ++m) {
    double t = (double)m / (ng - 1);
    tt[np] = t; dd[np++] = dmin[m];
    tt[np] = t; dd[np++] = dmax[m];
  }
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < np; ++i) {
    if (dd[i] == 0.0) {
      if (tt[i] < lo) lo = tt[i];
      if (tt[i] > hi) hi = tt[i];
    }
    for (int j = i + 1; j < np; ++j) {
      if ((dd[i] < 0.0 && dd[j] > 0.0) || (dd[i] > 0.0 && dd[j] < 0.0)) {
        double t = tt[i] + (tt[j] - tt[i]) * (dd[i] / (dd[i] - dd[j]));
        if (t < lo) lo = t;
        if (t > hi) hi = t;
      }
    }
  }
  if (lo > hi) return 0;
  *ta = lo;
  *tb = hi;
  return 1;
}

/* restrict a 1-D Bezier coefficient list to [a, b] by two de Casteljau splits */
static void restrict_1d(double* c, int n, double a, double b) {
  double tmp[MAXG], left[MAXG];
  /* left part [0, b] */
  memcpy(tmp, c, sizeof(double) * n);
  left[0] = tmp[0];
  for (int r = 1; r < n; ++r) {
    for (int i = 0; i < n - r; ++i) tmp[i] = (1.0 - b) * tmp[i] + b * tmp[i + 1];
    left[r] = tmp[0];
  }
  if (b <= 0.0) { for (int i = 0; i < n; ++i) c[i] = left[0]; return; }
  double s = a / b;
  /* right part [s, 1] of the left piece */
  memcpy(tmp, left, sizeof(double) * n);
  c[n - 1] = tmp[n - 1];
  for (int r = 1; r < n; ++r) {
    for (int i = 0; i < n - r; ++i) tmp[i] = (1.0 - s) * tmp[i] + s * tmp[i + 1];
    c[n - 1 - r] = tmp[n - 1 - r];
  }
}

static void patch_restrict(clip_patch* P, int ng, int dir, double a, double b) {
  double col[MAXG];
  for (int k = 0; k < ng; ++k)
    for (int co = 0; co < 3; ++co) {
      for (int i = 0; i < ng; ++i) col[i] = (dir == 0) ? P->q[i][k][co] : P->q[k][i][co];
      restrict_1d(col, ng, a, b);
      for (int i = 0; i < ng; ++i) {
        if (dir == 0) P->q[i][k][co] = col[i];
        else P->q[k][i][co] = col[i];
      }
    }
  if (dir == 0) {
    double w = P->u1 - P->u0;
    double n0 = P->u0 + a * w, n1 = P->u0 + b * w;
    P->u0 = n0; P->u1 = n1;
  } else {
    double w = P->v1 - P->v0;
    double n0 = P->v0 + a * w, n1 = P->v0 + b * w;
    P->v0 = n0; P->v1 = n1;
  }
}

/* clip direction dir (0: u, 1: v) against the line through the origin that
 * runs along the other parameter direction */
/* t-extent of the part of the convex hull of (t_m, lo_m), (t_m, hi_m) with
 * y >= c (ge) or y <= c: its vertices are hull points on that side and the
 * crossings of y = c by hull edges; every segment between two points on
 * opposite sides crosses inside the hull, so all such pairs are taken */
static int hull_side(int ng, const double* lo, const double* hi, double c, int ge, double* ta, double* tb) {
  double tt[2 * MAXG], yy[2 * MAXG];
  int np = 0;
  for (int m = 0; m < ng; ++m) {
    double t = (double)m / (ng - 1);
    tt[np] = t; yy[np++] = lo[m];
    tt[np] = t; yy[np++] = hi[m];
  }
  double a = INFINITY, b = -INFINITY;
  for (int i = 0; i < np; ++i) {
    int in_i = ge ? yy[i] >= c : yy[i] <= c;
    if (in_i) { if (tt[i] < a) a = tt[i]; if (tt[i] > b) b = tt[i]; }
    for (int j = i + 1; j < np; ++j) {
      int in_j = ge ? yy[j] >= c : yy[j] <= c;
      if (in_i == in_j || yy[i] == yy[j]) continue;
      double t = tt[i] + (tt[j] - tt[i]) * ((c - yy[i]) / (yy[j] - yy[i]));
      if (t < a) a = t;
      if (t > b) b = t;
    }
  }
  if (a > b) return 0;
  *ta = a; *tb = b;
  return 1;
}

/* Reading (the paper leaves the clipping loop to the literature): besides the
 * two plane distances, each direction is also clipped to the part of the
 * patch whose displacement lies in [amin, amax] (same convex-hull argument),
 * so the search starts on the stage segment's strip of the face. */
static int clip_dir(const clip_patch* P, int ng, int dir, double amin, double amax, double* a, double* b) {
  int N = ng - 1;
  double L[2];
  if (dir == 0)
    for (int co = 0; co < 2; ++co) L[co] = (P->q[0][N][co] - P->q[0][0][co]) + (P->q[N][N][co] - P->q[N][0][co]);
  else
    for (int co = 0; co < 2; ++co) L[co] = (P->q[N][0][co] - P->q[0][0][co]) + (P->q[N][N][co] - P->q[0][N][co]);
  double ll = sqrt(L[0] * L[0] + L[1] * L[1]);
  if (ll == 0.0) {
    /* degenerate direction: take the perpendicular of the other one */
    double K[2];
    if (dir == 0)
      for (int co = 0; co < 2; ++co) K[co] = (P->q[N][0][co] - P->q[0][0][co]) + (P->q[N][N][co] - P->q[0][N][co]);
    else
      for (int co = 0; co < 2; ++co) K[co] = (P->q[0][N][co] - P->q[0][0][co]) + (P->q[N][N][co] - P->q[N][0][co]);
    L[0] = -K[1]; L[1] = K[0];
    ll = sqrt(L[0] * L[0] + L[1] * L[1]);
    if (ll == 0.0) { L[0] = 1.0; L[1] = 0.0; ll = 1.0; }
  }
  double nx = -L[1] / ll, ny = L[0] / ll;
  double dmin[MAXG], dmax[MAXG];
  for (int i = 0; i < ng; ++i) {
    dmin[i] = INFINITY; dmax[i] = -INFINITY;
    for (int k = 0; k < ng; ++k) {
      const double* q = (dir == 0) ? P->q[i][k] : P->q[k][i];
      double dist = nx * q[0] + ny * q[1];
      if (dist < dmin[i]) dmin[i] = dist;
      if (dist > dmax[i]) dmax[i] = dist;
    }
  }
  if (!hull_zero(ng, dmin, dmax, a, b)) return 0;
  for (int i = 0; i < ng; ++i) {
    dmin[i] = INFINITY; dmax[i] = -INFINITY;
    for (int k = 0; k < ng; ++k) {
      double al = (dir == 0) ? P->q[i][k][2] : P->q[k][i][2];
      if (al < dmin[i]) dmin[i] = al;
      if (al > dmax[i]) dmax[i] = al;
    }
  }
  double a1, b1, a2, b2;
  if (!hull_side(ng, dmin, dmax, amin, 1, &a1, &b1)) return 0;
  if (!hull_side(ng, dmin, dmax, amax, 0, &a2, &b2)) return 0;
  if (a1 > *a) *a = a1;
  if (a2 > *a) *a = a2;
  if (b1 < *b) *b = b1;
  if (b2 < *b) *b = b2;
  if (*a > *b) return 0;
  *a -= CLIP_PAD; *b += CLIP_PAD;
  if (*a < 0.0) *a = 0.0;
  if (*b > 1.0) *b = 1.0;
  return 1;
}

/* 2-D Newton polish on the projected patch G(s, t) = sum q_mn B_m(s) B_n(t) = 0 */
static void clip_polish(int ng, double q0[MAXG][MAXG][2], double* s, double* t) {
  int deg = ng - 1;
  for (int it = 0; it < 3; ++it) {
    double Bs[MAXG], Bt[MAXG], dBs[MAXG], dBt[MAXG];
    bernstein(deg, *s, Bs); bernstein(deg, *t, Bt);
    bernstein_d(deg, *s, dBs); bernstein_d(deg, *t, dBt);
    double G[2] = {0, 0}, Gs[2] = {0, 0}, Gt[2] = {0, 0};
    for (int m = 0; m < ng; ++m)
      for (int k = 0; k < ng; ++k)
        for (int co = 0; co < 2; ++co) {
          G[co] += q0[m][k][co] * Bs[m] * Bt[k];
          Gs[co] += q0[m][k][co] * dBs[m] * Bt[k];
          Gt[co] += q0[m][k][co] * Bs[m] * dBt[k];
        }
    double det = Gs[0] * Gt[1] - Gs[1] * Gt[0];
    if (det == 0.0 || !isfinite(det)) return;
    double ds = -(G[0] * Gt[1] - G[1] * Gt[0]) / det;
    double dt = -(Gs[0] * G[1] - Gs[1] * G[0]) / det;
    *s += ds; *t += dt;
  }
}

/* evaluate the 3-D Bezier face at (u, v) in [-1,1]^2 and its tangents */
static void bezier_eval(int ng, const double* cp, double u, double v, double* p, double* pu, double* pv) {
  int deg = ng - 1;
  double Bu[MAXG], Bv[MAXG], dBu[MAXG], dBv[MAXG];
  double s = 0.5 * (u + 1.0), t = 0.5 * (v + 1.0);
  bernstein(deg, s, Bu); bernstein(deg, t, Bv);
  bernstein_d(deg, s, dBu); bernstein_d(deg, t, dBv);
  for (int q = 0; q < 3; ++q) { p[q] = 0.0; if (pu) pu[q] = 0.0; if (pv) pv[q] = 0.0; }
  for (int k = 0; k < ng; ++k)
    for (int m = 0; m < ng; ++m) {
      const double* P = cp + (k * ng + m) * 3;
      for (int q = 0; q < 3; ++q) {
        p[q] += P[q] * Bu[m] * Bv[k];
        if (pu) pu[q] += P[q] * 0.5 * dBu[m] * Bv[k];
        if (pv) pv[q] += P[q] * 0.5 * Bu[m] * dBv[k];
      }
    }
}

/* all intersections of the line x0 + alpha t (|t| = 1) with a Bezier face */
/* roots with displacement in [amin, amax] (all roots: +-INFINITY) */
static int bezier_band(int ng, const double* cp, const double* x0, const double* t, double amin,
                       double amax, double* alpha, double* uv, int max_roots) {
  double n1[3], n2[3];
  ray_planes(t, n1, n2);
  static __thread clip_patch stack[CLIP_STACK];
  double q0[MAXG][MAXG][2];
  for (int k = 0; k < ng; ++k)
    for (int m = 0; m < ng; ++m) {
      const double* P = cp + (k * ng + m) * 3;
      double r[3] = {P[0] - x0[0], P[1] - x0[1], P[2] - x0[2]};
      q0[m][k][0] = dot3(r, n1);
      q0[m][k][1] = dot3(r, n2);
      stack[0].q[m][k][0] = q0[m][k][0];
      stack[0].q[m][k][1] = q0[m][k][1];
      stack[0].q[m][k][2] = dot3(r, t);
    }
  int sp = 0, nroots = 0, budget = CLIP_STEPS;
  stack[0].u0 = 0.0; stack[0].u1 = 1.0; stack[0].v0 = 0.0; stack[0].v1 = 1.0;
  sp = 1;
  while (sp > 0 && budget > 0) {
    clip_patch P = stack[--sp];
    for (;;) {
      if (--budget < 0) break;
      if (patch_outside_band(&P, ng, amin, amax)) break;
      double a, b, ru, rv;
      if (!clip_dir(&P, ng, 0, amin, amax, &a, &b)) break;
      patch_restrict(&P, ng, 0, a, b);
      ru = b - a;
      if (!clip_dir(&P, ng, 1, amin, amax, &a, &b)) break;
      patch_restrict(&P, ng, 1, a, b);
      rv = b - a;
      double wu = P.u1 - P.u0, wv = P.v1 - P.v0;
      int conv = (wu <= CLIP_TOL && wv <= CLIP_TOL);
      int split_u = (ru > 0.8 && wu > CLIP_TOL), split_v = (rv > 0.8 && wv > CLIP_TOL);
      if (!conv && (split_u || split_v) && sp + 2 > CLIP_STACK) conv = 1; /* stack full: take it */
      if (conv) {
        double s = 0.5 * (P.u0 + P.u1), tt = 0.5 * (P.v0 + P.v1);
        clip_polish(ng, q0, &s, &tt);
        double u = 2.0 * s - 1.0, v = 2.0 * tt - 1.0;
        int dup = 0;
        for (int r = 0; r < nroots; ++r)
          if (fabs(uv[2 * r] - u) < 1e-9 && fabs(uv[2 * r + 1] - v) < 1e-9) dup = 1;
        if (!dup && nroots < max_roots) {
          double p[3];
          bezier_eval(ng, cp, u, v, p, NULL, NULL);
          double r3[3] = {p[0] - x0[0], p[1] - x0[1], p[2] - x0[2]};
          alpha[nroots] = dot3(r3, t);
          uv[2 * nroots] = u;
          uv[2 * nroots + 1] = v;
          nroots++;
        }
        break;
      }
      if (split_u || split_v) {
        int dir = (split_u && split_v) ? (wu >= wv ? 0 : 1) : (split_u ? 0 : 1);
        clip_patch L = P, R = P;
        patch_restrict(&L, ng, dir, 0.0, 0.5);
        patch_restrict(&R, ng, dir, 0.5, 1.0);
        stack[sp++] = R;
        stack[sp++] = L;
        break;
      }
    }
  }
  return nroots;
}

int or_bezier_intersect(int ng, const double* cp, const double* x0, const double* t,
                        double* alpha, double* uv, int max_roots) {
  return bezier_band(ng, cp, x0, t, -INFINITY, INFINITY, alpha, uv, max_roots);
}

/* all roots of the face equation along the line (any alpha) */
int or_face_intersect(const or_ctx* c, int e, int f, const double* x0, const double* t,
                      double* alpha, double* uv, int max_roots) {
  int ng = c->ng, deg = ng - 1;
  const double* cp = c->cp + ((size_t)e * 6 + f) * ng * ng * 3;
  int type = c->ftype[e * 6 + f];
  if (type == OR_FACE_CURVED) return or_bezier_intersect(ng, cp, x0, t, alpha, uv, max_roots);
  double A[3], B[3], C[3], D[3];
  bilinear_coeffs(cp, cp + deg * 3, cp + deg * ng * 3, cp + (deg * ng + deg) * 3, A, B, C, D);
  if (type == OR_FACE_PLANAR) return planar_intersect(A, B, C, D, x0, t, alpha, uv);
  return bilinear_intersect(A, B, C, D, x0, t, alpha, uv);
}

/* unit normal of face fid at (u, v) */
static void face_normal(const or_ctx* c, int fid, double u, double v, double* nrm) {
  int ng = c->ng;
  const double* cp = c->cp + (size_t)fid * ng * ng * 3;
  double p[3], pu[3], pv[3];
  bezier_eval(ng, cp, u, v, p, pu, pv);
  cross3(pu, pv, nrm);
  double l = norm3(nrm);
  for (int q = 0; q < 3; ++q) nrm[q] /= l;
}

/* ======================================================================== */
/* context                                                                   */
/* ======================================================================== */
int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* threads of the parallel particle loops from now on (timing on one core) */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static void build_bgm(or_ctx* c) {
  int E = c->E, ng = c->ng;
  double glo[3] = {INFINITY, INFINITY, INFINITY}, ghi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double hsum = 0.0;
  for (int e = 0; e < E; ++e) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const double* X = c->X + (size_t)e * ng * ng * ng * 3;
    for (int q = 0; q < ng * ng * ng; ++q)
      for (int k = 0; k < 3; ++k) {
        if (X[q * 3 + k] < lo[k]) lo[k] = X[q * 3 + k];
        if (X[q * 3 + k] > hi[k]) hi[k] = X[q * 3 + k];
      }
    /* reading: pad the node box by 5 % of its extent so that curved elements,
     * which may bulge beyond their nodes, stay inside their box */
    for (int k = 0; k < 3; ++k) {
      double p = 0.05 * (hi[k] - lo[k]);
      c->elo[e * 3 + k] = lo[k] - p;
      c->ehi[e * 3 + k] = hi[k] + p;
      if (c->elo[e * 3 + k] < glo[k]) glo[k] = c->elo[e * 3 + k];
      if (c->ehi[e * 3 + k] > ghi[k]) ghi[k] = c->ehi[e * 3 + k];
    }
    hsum += c->hE[e];
  }
  double h = hsum / E;
  for (int k = 0; k < 3; ++k) {
    int nb = (int)ceil((ghi[k] - glo[k]) / h);
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    c->bn[k] = nb;
    c->blo[k] = glo[k];
    c->bdx[k] = (ghi[k] - glo[k]) / nb;
    if (c->bdx[k] <= 0.0) c->bdx[k] = 1.0;
  }
  size_t ncell = (size_t)c->bn[0] * c->bn[1] * c->bn[2];
  c->bstart = (int*)calloc(ncell + 1, sizeof(int));
  for (int pass = 0; pass < 2; ++pass) {
    int* fill = NULL;
    if (pass == 1) {
      for (size_t i = 0; i < ncell; ++i) c->bstart[i + 1] += c->bstart[i];
      c->blist = (int*)malloc(sizeof(int) * (c->bstart[ncell] + 1));
      fill = (int*)calloc(ncell, sizeof(int));
    }
    for (int e = 0; e < E; ++e) {
      int i0[3], i1[3];
      for (int k = 0; k < 3; ++k) {
        i0[k] = (int)floor((c->elo[e * 3 + k] - c->blo[k]) / c->bdx[k]);
        i1[k] = (int)floor((c->ehi[e * 3 + k] - c->blo[k]) / c->bdx[k]);
        if (i0[k] < 0) i0[k] = 0;
        if (i1[k] >= c->bn[k]) i1[k] = c->bn[k] - 1;
      }
      for (int z = i0[2]; z <= i1[2]; ++z)
        for (int y = i0[1]; y <= i1[1]; ++y)
          for (int x = i0[0]; x <= i1[0]; ++x) {
            size_t cell = ((size_t)z * c->bn[1] + y) * c->bn[0] + x;
            if (pass == 0) c->bstart[cell + 1]++;
            else c->blist[c->bstart[cell] + fill[cell]++] = e;
          }
    }
    free(fill);
  }
}

/* Reading (the paper traces particles near boundaries in physical space and
 * localises the others in reference space, but gives no distance rule): a
 * lower bound of the distance from element e to any face that is not
 * internal (wall, open, periodic): the distance between e's padded node box
 * and the face's control-point box (which contains the face, convex hull),
 * over the boundary faces within h_e, less 0.1 h_e; capped at 0.9 h_e. */
static double box_gap(const double* alo, const double* ahi, const double* blo, const double* bhi) {
  double s = 0.0;
  for (int k = 0; k < 3; ++k) {
    double d = 0.0;
    if (blo[k] > ahi[k]) d = blo[k] - ahi[k];
    else if (alo[k] > bhi[k]) d = alo[k] - bhi[k];
    s += d * d;
  }
  return sqrt(s);
}

static void build_boundary_distance(or_ctx* c) {
  int E = c->E, ng = c->ng;
  size_t ncell = (size_t)c->bn[0] * c->bn[1] * c->bn[2];
  /* boundary-face boxes bucketed in the background-mesh cells */
  int nbf = 0;
  for (int i = 0; i < E * 6; ++i) nbf += c->bc[i] != 0;
  double* fb = (double*)malloc(sizeof(double) * 6 * (nbf + 1));
  int* fstart = (int*)calloc(ncell + 1, sizeof(int));
  int nf = 0;
  for (int i = 0; i < E * 6; ++i) {
    if (c->bc[i] == 0) continue;
    double* b = fb + 6 * nf++;
    for (int k = 0; k < 3; ++k) { b[k] = INFINITY; b[3 + k] = -INFINITY; }
    const double* P = c->cp + (size_t)i * ng * ng * 3;
    for (int q = 0; q < ng * ng; ++q)
      for (int k = 0; k < 3; ++k) {
        if (P[q * 3 + k] < b[k]) b[k] = P[q * 3 + k];
        if (P[q * 3 + k] > b[3 + k]) b[3 + k] = P[q * 3 + k];
      }
  }
  int* flist = NULL;
  for (int pass = 0; pass < 2; ++pass) {
    int* fill = NULL;
    if (pass == 1) {
      for (size_t q = 0; q < ncell; ++q) fstart[q + 1] += fstart[q];
      flist = (int*)malloc(sizeof(int) * (fstart[ncell] + 1));
      fill = (int*)calloc(ncell, sizeof(int));
    }
    for (int j = 0; j < nf; ++j) {
      int lo[3], hi[3];
      for (int k = 0; k < 3; ++k) {
        lo[k] = (int)floor((fb[6 * j + k] - c->blo[k]) / c->bdx[k]);
        hi[k] = (int)floor((fb[6 * j + 3 + k] - c->blo[k]) / c->bdx[k]);
        if (lo[k] < 0) lo[k] = 0;
        if (hi[k] >= c->bn[k]) hi[k] = c->bn[k] - 1;
      }
      for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
          for (int x = lo[0]; x <= hi[0]; ++x) {
            size_t id = ((size_t)z * c->bn[1] + y) * c->bn[0] + x;
            if (pass == 0) fstart[id + 1]++;
            else flist[fstart[id] + fill[id]++] = j;
          }
    }
    free(fill);
  }
#pragma omp parallel for schedule(static)
  for (int e = 0; e < E; ++e) {
    double h = c->hE[e], best = h;
    const double* alo = c->elo + e * 3;
    const double* ahi = c->ehi + e * 3;
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = (int)floor((alo[k] - h - c->blo[k]) / c->bdx[k]);
      hi[k] = (int)floor((ahi[k] + h - c->blo[k]) / c->bdx[k]);
      if (lo[k] < 0) lo[k] = 0;
      if (hi[k] >= c->bn[k]) hi[k] = c->bn[k] - 1;
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) {
          size_t id = ((size_t)z * c->bn[1] + y) * c->bn[0] + x;
          for (int q = fstart[id]; q < fstart[id + 1]; ++q) {
            const double* b = fb + 6 * flist[q];
            double g = box_gap(alo, ahi, b, b + 3);
            if (g < best) best = g;
          }
        }
    best -= 0.1 * h;
    c->dsafe[e] = best > 0.0 ? best : 0.0;
  }
  free(fb); free(fstart); free(flist);
}

or_ctx* or_create(int n_elem, int n_geo, const double* X, const int32_t* nbr_elem,
                  const int32_t* nbr_face, const int8_t* bc, const double* shift, int N,
                  int dg_nodes) {
  if (n_elem <= 0 || n_geo < 1 || n_geo + 1 > MAXG || N < 0 || N + 1 > MAXG) return NULL;
  or_ctx* c = (or_ctx*)calloc(1, sizeof(or_ctx));
  c->E = n_elem; c->n_geo = n_geo; c->ng = n_geo + 1; c->N = N; c->n = N + 1;
  int ng = c->ng, n = c->n, E = n_elem;
  size_t nX = (size_t)E * ng * ng * ng * 3;
  c->X = (double*)malloc(sizeof(double) * nX);
  memcpy(c->X, X, sizeof(double) * nX);
  c->nbr_elem = (int32_t*)malloc(sizeof(int32_t) * E * 6);
  c->nbr_face = (int32_t*)malloc(sizeof(int32_t) * E * 6);
  c->bc = (int8_t*)malloc(E * 6);
  c->shift = (double*)malloc(sizeof(double) * E * 18);
  memcpy(c->nbr_elem, nbr_elem, sizeof(int32_t) * E * 6);
  memcpy(c->nbr_face, nbr_face, sizeof(int32_t) * E * 6);
  memcpy(c->bc, bc, E * 6);
  memcpy(c->shift, shift, sizeof(double) * E * 18);
  /* geometry nodes: equidistant on [-1, 1] including the end points (reading) */
  for (int i = 0; i < ng; ++i) c->xgeo[i] = -1.0 + 2.0 * i / n_geo;
  if (dg_nodes == 0) or_gauss_nodes(n, c->xdg, c->wdg);
  else or_lobatto_nodes(n, c->xdg, c->wdg);
  /* element length scale: longest edge between corners */
  c->hE = (double*)malloc(sizeof(double) * E);
  for (int e = 0; e < E; ++e) {
    const double* P = c->X + (size_t)e * ng * ng * ng * 3;
    int cor[8];
    for (int k = 0; k < 2; ++k)
      for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i)
          cor[(k * 2 + j) * 2 + i] = ((k * n_geo) * ng + j * n_geo) * ng + i * n_geo;
    double hm = 0.0;
    for (int a = 0; a < 8; ++a)
      for (int bit = 0; bit < 3; ++bit) {
        int b = a ^ (1 << bit);
        if (b < a) continue;
        double r[3] = {P[cor[a] * 3] - P[cor[b] * 3], P[cor[a] * 3 + 1] - P[cor[b] * 3 + 1],
                       P[cor[a] * 3 + 2] - P[cor[b] * 3 + 2]};
        double l = norm3(r);
        if (l > hm) hm = l;
      }
    c->hE[e] = hm;
  }
  /* DG node positions and volumes V_ijk = w_i w_j w_k J(xi_ijk) */
  c->xnode = (double*)malloc(sizeof(double) * (size_t)E * n * n * n * 3);
  c->vol = (double*)malloc(sizeof(double) * (size_t)E * n * n * n);
#pragma omp parallel for schedule(static)
  for (int e = 0; e < E; ++e)
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double xi[3] = {c->xdg[i], c->xdg[j], c->xdg[k]}, xx[3], J[9];
          or_map(c, e, xi, xx, J);
          size_t q = ((size_t)e * n * n * n) + (k * n + j) * n + i;
          for (int r = 0; r < 3; ++r) c->xnode[q * 3 + r] = xx[r];
          double JJ[3][3];
          for (int r = 0; r < 9; ++r) JJ[r / 3][r % 3] = J[r];
          c->vol[q] = c->wdg[i] * c->wdg[j] * c->wdg[k] * det3(JJ);
        }
  /* faces */
  c->cp = (double*)malloc(sizeof(double) * (size_t)E * 6 * ng * ng * 3);
  c->ftype = (int*)malloc(sizeof(int) * E * 6);
  c->fframe = (double*)malloc(sizeof(double) * (size_t)E * 6 * 9);
  c->forig = (double*)malloc(sizeof(double) * (size_t)E * 6 * 3);
  c->flo = (double*)malloc(sizeof(double) * (size_t)E * 6 * 3);
  c->fhi = (double*)malloc(sizeof(double) * (size_t)E * 6 * 3);
  c->fdiam = (double*)malloc(sizeof(double) * (size_t)E * 6);
#pragma omp parallel for schedule(static)
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) build_face(c, e, f);
  c->elo = (double*)malloc(sizeof(double) * E * 3);
  c->ehi = (double*)malloc(sizeof(double) * E * 3);
  build_bgm(c);
  c->dsafe = (double*)malloc(sizeof(double) * E);
  build_boundary_distance(c);
  c->mu = 1.8e-5; c->kappa = 1.4; c->rho_p = 2500.0;
  return c;
}

void or_destroy(or_ctx* c) {
  if (!c) return;
  free(c->X); free(c->nbr_elem); free(c->nbr_face); free(c->bc); free(c->shift);
  free(c->xnode); free(c->vol); free(c->hE); free(c->cp); free(c->ftype); free(c->fframe);
  free(c->forig); free(c->flo); free(c->fhi); free(c->fdiam); free(c->bstart); free(c->blist);
  free(c->elo); free(c->ehi); free(c->dsafe); free(c->mortar);
  free(c->x); free(c->v); free(c->kx); free(c->kv); free(c->d); free(c->xi); free(c->elem);
  free(c->hits); free(c->status); free(c->mlp_w); free(c->mlp_flag);
  free(c);
}

void or_set_fluid(or_ctx* c, const double* U, double mu, double kappa, double rho_p) {
  c->U = U; c->mu = mu; c->kappa = kappa; c->rho_p = rho_p;
}

double or_volume(const or_ctx* c, int e, int node) { return c->vol[(size_t)e * c->n * c->n * c->n + node]; }
void or_dg_node_pos(const or_ctx* c, int e, int node, double* x) {
  size_t q = (size_t)e * c->n * c->n * c->n + node;
  for (int r = 0; r < 3; ++r) x[r] = c->xnode[q * 3 + r];
}

/* ======================================================================== */
/* locating a point (Sec. 4.1.2 background mesh + Sec. 3.2.3 inside test)     */
/* ======================================================================== */
int or_locate(or_ctx* c, const double* x, int hint, double* xi) {
  int64_t it = 0, calls = 0, fb = 0;
  if (hint >= 0 && hint < c->E) {
    if (newton_chain(c, hint, x, xi, 50, 0, &it, &calls, &fb) && inside_ref(xi)) return hint;
  }
  int cell[3];
  for (int k = 0; k < 3; ++k) {
    cell[k] = (int)floor((x[k] - c->blo[k]) / c->bdx[k]);
    if (cell[k] < 0 || cell[k] >= c->bn[k]) return -1;
  }
  size_t id = ((size_t)cell[2] * c->bn[1] + cell[1]) * c->bn[0] + cell[0];
  for (int q = c->bstart[id]; q < c->bstart[id + 1]; ++q) {
    int e = c->blist[q];
    if (x[0] < c->elo[e * 3] || x[0] > c->ehi[e * 3] || x[1] < c->elo[e * 3 + 1] ||
        x[1] > c->ehi[e * 3 + 1] || x[2] < c->elo[e * 3 + 2] || x[2] > c->ehi[e * 3 + 2])
      continue;
    if (newton_chain(c, e, x, xi, 50, 0, &it, &calls, &fb) && inside_ref(xi)) return e;
  }
  return -1;
}

int or_push(or_ctx* c, int64_t n, const double* x, const double* v, const double* d,
            const int32_t* hint, int32_t* status_out) {
  free(c->x); free(c->v); free(c->kx); free(c->kv); free(c->d); free(c->xi); free(c->elem);
  free(c->hits); free(c->status);
  c->np = n;
  c->x = (double*)malloc(sizeof(double) * n * 3);
  c->v = (double*)malloc(sizeof(double) * n * 3);
  c->kx = (double*)calloc(n * 3, sizeof(double));
  c->kv = (double*)calloc(n * 3, sizeof(double));
  c->d = (double*)malloc(sizeof(double) * n);
  c->xi = (double*)calloc(n * 3, sizeof(double));
  c->elem = (int32_t*)malloc(sizeof(int32_t) * n);
  c->hits = (int32_t*)calloc(n, sizeof(int32_t));
  c->status = (int8_t*)malloc(n);
  memcpy(c->x, x, sizeof(double) * n * 3);
  memcpy(c->v, v, sizeof(double) * n * 3);
  memcpy(c->d, d, sizeof(double) * n);
  int nbad = 0;
#pragma omp parallel for schedule(static) reduction(+ : nbad)
  for (int64_t p = 0; p < n; ++p) {
    double xi[3] = {0, 0, 0};
    int e = or_locate(c, x + p * 3, hint ? hint[p] : -1, xi);
    c->elem[p] = e < 0 ? 0 : e;
    c->status[p] = e < 0 ? OR_REJECTED : OR_ACTIVE;
    for (int k = 0; k < 3; ++k) c->xi[p * 3 + k] = xi[k];
    if (status_out) status_out[p] = c->status[p];
    if (e < 0) nbad++;
  }
  return nbad;
}

/* ======================================================================== */
/* tracking in physical space (Sec. 3.2.3, 3.2.4, 2.4)                       */
/* ======================================================================== */
/* Reading of the paper's loop: along the straight stage segment xs -> xe the
 * hit with the smallest displacement alpha in (eps, remaining length] whose
 * (u, v) lies in [-1,1]^2 is taken (ties: lowest local face); eps = 1e-12 h_e.
 * A planar entry face is excluded after a hand-off or reflection.  Internal:
 * move to the neighbour; periodic: also translate the hit and end points;
 * reflective: mirror the remaining displacement, v, and the stage registers
 * with I - 2 n n^T (specular, Delta p = 0) and count the hit; open: the
 * particle leaves the domain. */
static void track(or_ctx* c, int64_t p, double* xs_in, double* xe, double* v, double* kx, double* kv,
                  int max_cross, int64_t* ncross, int64_t* nhits) {
  int e = c->elem[p];
  double xs[3] = {xs_in[0], xs_in[1], xs_in[2]};
  int excl = -1;   /* planar face just entered through: no further root possible */
  int entry = -1;  /* non-planar face just entered through (see below) */
  int count = 0;
  for (;;) {
    double t[3] = {xe[0] - xs[0], xe[1] - xs[1], xe[2] - xs[2]};
    double L = norm3(t);
    if (L == 0.0) break;
    for (int q = 0; q < 3; ++q) t[q] /= L;
    double eps = 1e-12 * c->hE[e];
    double best = INFINITY, bu = 0.0, bv = 0.0;
    int bf = -1;
    for (int f = 0; f < 6; ++f) {
      if (f == excl) continue;
      int fid = e * 6 + f;
      if (!bbox_hit(c, fid, xs, xe)) continue;
      /* Reading (the paper accepts 0 < alpha <= remaining length and says
       * nothing about the entry point): a non-planar face the particle has
       * just entered through (hand-off or reflection) returns the entry point
       * itself as a root at alpha ~ 0, whose rounding error grows like
       * 1 / sin(incidence) at grazing incidence and can exceed eps.  On that
       * face only roots beyond ENTRY_REL * face diameter count; a genuine
       * second crossing closer than that requires near-tangency, and its
       * excursion outside the element stays far below INSIDE_EPS. */
      double amin = (f == entry) ? fmax(eps, ENTRY_REL * c->fdiam[fid]) : eps;
      double al[8], uv[16];
      int nr;
      if (c->ftype[fid] == OR_FACE_CURVED) {
        /* only roots in (amin, L] matter: clip to that band, padded */
        double pad = 1e-9 * c->fdiam[fid];
        nr = bezier_band(c->ng, c->cp + (size_t)fid * c->ng * c->ng * 3, xs, t, amin - pad, L + pad, al, uv, 8);
      } else {
        nr = or_face_intersect(c, e, f, xs, t, al, uv, 8);
      }
      for (int r = 0; r < nr; ++r) {
        if (!(al[r] > amin && al[r] <= L)) continue;
        if (fabs(uv[2 * r]) > 1.0 + UV_EPS || fabs(uv[2 * r + 1]) > 1.0 + UV_EPS) continue;
        /* Reading (the paper counts every root in (0, remaining length]): only a
         * root where the path leaves the element is a crossing.  A root where
         * it enters (the other half of a tangential touch of a curved face, or
         * the entry point) is not; without this a touch whose leaving root the
         * clipping does not separate hands the particle over at the entering
         * one.  Outward normal: FACE_SIGN[f] * (dp/du x dp/dv) for J > 0. */
        double nrm[3];
        face_normal(c, fid, uv[2 * r], uv[2 * r + 1], nrm);
        if (!(FACE_SIGN[f] * dot3(nrm, t) > 0.0)) continue;
        if (al[r] < best) { best = al[r]; bf = f; bu = uv[2 * r]; bv = uv[2 * r + 1]; }
      }
    }
    if (bf < 0) break;
    if (count >= max_cross) { c->status[p] = OR_MAX_CROSS; break; }
    count++;
    (*ncross)++;
    double xh[3] = {xs[0] + best * t[0], xs[1] + best * t[1], xs[2] + best * t[2]};
    int fid = e * 6 + bf;
    int bc = c->bc[fid];
    if (bc == 0 || bc == 3) {
      int ne = c->nbr_elem[fid], nf = c->nbr_face[fid];
      if (bc == 3)
        for (int q = 0; q < 3; ++q) { xh[q] += c->shift[fid * 3 + q]; xe[q] += c->shift[fid * 3 + q]; }
      e = ne;
      excl = (c->ftype[ne * 6 + nf] == OR_FACE_PLANAR) ? nf : -1;
      entry = (c->ftype[ne * 6 + nf] == OR_FACE_PLANAR) ? -1 : nf;
      for (int q = 0; q < 3; ++q) xs[q] = xh[q];
    } else if (bc == OR_BC_MORTAR) {
      /* Non-conforming side (Sec. 3.2.3): the big face is matched by two or
       * four small faces of neighbouring elements.  As in the paper, the
       * trajectory is inverted (from the leg end back towards its start) and
       * intersected with the small faces: a root where the inverted path
       * leaves a small element is where the forward path enters it.  Of those
       * roots the one nearest the big-face crossing (alpha = best) is the
       * crossing; the particle continues from it in that small element.  If
       * none is found (rounding at the seam of two small faces) the leg ends
       * in the big element and the next location step finds the element. */
      int m = c->nbr_elem[fid];
      double tb[3] = {-t[0], -t[1], -t[2]};
      double bd = INFINITY, sa = 0.0;
      int se = -1, sf = -1;
      for (int j = 0; j < 4; ++j) {
        int s = c->mortar[m * 8 + 2 * j], fs = c->mortar[m * 8 + 2 * j + 1];
        if (s < 0) continue;
        int sfid = s * 6 + fs;
        double al[8], uv[16];
        int nr = (c->ftype[sfid] == OR_FACE_CURVED)
                     ? bezier_band(c->ng, c->cp + (size_t)sfid * c->ng * c->ng * 3, xe, tb, -1e-9 * c->fdiam[sfid],
                                   L + 1e-9 * c->fdiam[sfid], al, uv, 8)
                     : or_face_intersect(c, s, fs, xe, tb, al, uv, 8);
        for (int r = 0; r < nr; ++r) {
          double pad = 1e-9 * c->fdiam[sfid];
          if (!(al[r] >= -pad && al[r] <= L + pad)) continue;
          if (fabs(uv[2 * r]) > 1.0 + UV_EPS || fabs(uv[2 * r + 1]) > 1.0 + UV_EPS) continue;
          double nrm[3];
          face_normal(c, sfid, uv[2 * r], uv[2 * r + 1], nrm);
          if (!(FACE_SIGN[fs] * dot3(nrm, tb) > 0.0)) continue;
          double a = L - al[r];
          if (fabs(a - best) < bd) { bd = fabs(a - best); sa = a; se = s; sf = fs; }
        }
      }
      if (se < 0) { for (int q = 0; q < 3; ++q) xs[q] = xh[q]; excl = -1; entry = bf; continue; }
      e = se;
      excl = (c->ftype[se * 6 + sf] == OR_FACE_PLANAR) ? sf : -1;
      entry = (c->ftype[se * 6 + sf] == OR_FACE_PLANAR) ? -1 : sf;
      for (int q = 0; q < 3; ++q) xs[q] = xs[q] + sa * t[q];
    } else if (bc == 2) {
      double nrm[3];
      face_normal(c, fid, bu, bv, nrm);
      double r[3] = {xe[0] - xh[0], xe[1] - xh[1], xe[2] - xh[2]};
      double dr = dot3(r, nrm), dv = dot3(v, nrm), dkx = dot3(kx, nrm), dkv = dot3(kv, nrm);
      for (int q = 0; q < 3; ++q) {
        xe[q] = xh[q] + (r[q] - 2.0 * dr * nrm[q]);
        v[q] -= 2.0 * dv * nrm[q];
        kx[q] -= 2.0 * dkx * nrm[q];
        kv[q] -= 2.0 * dkv * nrm[q];
      }
      c->hits[p]++;
      (*nhits)++;
      excl = (c->ftype[fid] == OR_FACE_PLANAR) ? bf : -1;
      entry = (c->ftype[fid] == OR_FACE_PLANAR) ? -1 : bf;
      for (int q = 0; q < 3; ++q) xs[q] = xh[q];
    } else {
      c->status[p] = OR_OPEN_EXIT;
      for (int q = 0; q < 3; ++q) xe[q] = xh[q];
      break;
    }
  }
  c->elem[p] = e;
}

/* Reading (the paper verifies a located particle by xi in [-1,1]^3 and does
 * not say what follows a failed check): a particle that the location step
 * finds outside its element crossed a face that was not traced (reference-
 * space localisation) or that the intersection search missed (the clipping
 * budget can run out at grazing incidence).  Internal faces do not change the
 * path, so the particle is followed across the face through which its
 * reference coordinate left (largest |xi_d|, lowest axis on ties), with the
 * periodic shift where the face is periodic, and located again, at most
 * RECOVER_HOPS times; then, as in the paper's localisation, the
 * background-mesh candidates of the point are tried.  A wall or open face
 * ends the hops.  Returns 1 with e, x, xi updated when inside. */
static int recover_elem(or_ctx* c, int* e, double* x, double* xi, int max_it, int64_t* it_sum,
                        int64_t* calls, int64_t* nfb) {
  int eh = *e;
  double xh[3] = {x[0], x[1], x[2]};
  for (int hop = 0; hop < RECOVER_HOPS; ++hop) {
    int d = 0;
    double ex = fabs(xi[0]);
    if (fabs(xi[1]) > ex) { d = 1; ex = fabs(xi[1]); }
    if (fabs(xi[2]) > ex) { d = 2; ex = fabs(xi[2]); }
    int fid = eh * 6 + 2 * d + (xi[d] > 0.0 ? 1 : 0);
    int bc = c->bc[fid];
    if (bc != 0 && bc != 3) break;
    if (bc == 3)
      for (int q = 0; q < 3; ++q) xh[q] += c->shift[fid * 3 + q];
    eh = c->nbr_elem[fid];
    if (!newton_chain(c, eh, xh, xi, max_it, 0, it_sum, calls, nfb)) break;
    if (inside_ref(xi)) {
      *e = eh;
      for (int q = 0; q < 3; ++q) x[q] = xh[q];
      return 1;
    }
  }
  /* the paper's localisation: the background-mesh candidates of the point,
   * in element order, the first that contains it */
  int f = or_locate(c, x, -1, xi);
  if (f < 0) return 0;
  *e = f;
  return 1;
}

double or_boundary_distance(const or_ctx* c, int e) { return c->dsafe[e]; }

/* Non-conforming (mortar) faces: table[m][4][2] lists the (element, local
 * face) of the small faces that tile big face m, (-1, -1) where unused; a big
 * face has bc OR_BC_MORTAR and nbr_elem = m, each small face bc internal with
 * the big element and face as neighbour.  Returns 0, or -1 on an inconsistent
 * table (then nothing is stored). */
int or_set_mortar(or_ctx* c, int n, const int32_t* table) {
  for (int m = 0; m < n; ++m) {
    int big = -1, nsmall = 0;
    for (int e = 0; e < c->E && big < 0; ++e)
      for (int f = 0; f < 6; ++f)
        if (c->bc[e * 6 + f] == OR_BC_MORTAR && c->nbr_elem[e * 6 + f] == m) { big = e * 6 + f; break; }
    if (big < 0) return -1;
    for (int j = 0; j < 4; ++j) {
      int s = table[m * 8 + 2 * j], fs = table[m * 8 + 2 * j + 1];
      if (s < 0) continue;
      if (s >= c->E || fs < 0 || fs > 5) return -1;
      if (c->bc[s * 6 + fs] != 0 || c->nbr_elem[s * 6 + fs] * 6 + c->nbr_face[s * 6 + fs] != big) return -1;
      nsmall++;
    }
    if (nsmall != 2 && nsmall != 4) return -1;
  }
  free(c->mortar);
  c->mortar = (int32_t*)malloc(sizeof(int32_t) * 8 * (n > 0 ? n : 1));
  memcpy(c->mortar, table, sizeof(int32_t) * 8 * n);
  c->n_mortar = n;
  return 0;
}

void or_default_opts(or_step_opts* o) {
  memset(o, 0, sizeof(*o));
  o->rk = 0; o->drag = 1; o->max_newton_it = 50; o->max_crossings = 64;
  o->drag_mask[0] = o->drag_mask[1] = o->drag_mask[2] = 1.0;
}

/* One or more time steps.  Per stage (Sec. 3.2): locate xi in the current
 * element (guess + Newton, with the inside check that verifies the tracking),
 * interpolate U, primitives, drag, low-storage update, then track the stage
 * segment. */
int or_step(or_ctx* c, double dt, int n_steps, const or_step_opts* o) {
  int S;
  double A[5], B[5], cc[5];
  or_rk_coeffs(o->rk, &S, A, B, cc);
  int64_t it_sum = 0, calls = 0, ncross = 0, nhits = 0, nlost = 0, nfb = 0, nrec = 0;
  for (int step = 0; step < n_steps; ++step)
    for (int s = 0; s < S; ++s) {
#pragma omp parallel for schedule(static) reduction(+ : it_sum, calls, ncross, nhits, nlost, nfb, nrec)
      for (int64_t p = 0; p < c->np; ++p) {
        if (c->status[p] != OR_ACTIVE) continue;
        int e = c->elem[p];
        double* x = c->x + p * 3;
        double* v = c->v + p * 3;
        double* kx = c->kx + p * 3;
        double* kv = c->kv + p * 3;
        double xi[3];
        if (!newton_chain(c, e, x, xi, o->max_newton_it, o->use_mlp, &it_sum, &calls, &nfb)) {
          /* Newton diverges in the recorded element: the point left it along
           * a segment that was not traced (reference-space localisation), and
           * the map continued beyond a strongly curved element need not be
           * invertible there.  The paper's localisation: the background-mesh
           * candidates of the point. */
          int f = or_locate(c, x, -1, xi);
          if (f < 0) { c->status[p] = OR_LOST_NEWTON; nlost++; continue; }
          e = f;
          c->elem[p] = e;
          nrec++;
        } else if (!inside_ref(xi)) {
          if (!recover_elem(c, &e, x, xi, o->max_newton_it, &it_sum, &calls, &nfb)) {
            c->status[p] = OR_LOST_TRACK; nlost++; continue;
          }
          c->elem[p] = e;
          nrec++;
        }
        for (int k = 0; k < 3; ++k) c->xi[p * 3 + k] = xi[k];
        double Uc[5], prim[5], a[3];
        if (o->forces) {
          double G[9];
          or_fluid_grad(c, e, xi, prim, G);
          or_particle_accel(c, o->drag, o->forces, prim, G, v, c->d[p], o->gravity, a, NULL);
        } else {
          or_interp(c, e, xi, Uc);
          cons2prim(c->kappa, Uc, prim);
          or_drag_accel(c, o->drag, prim, v, c->d[p], NULL, a, NULL);
          for (int k = 0; k < 3; ++k) a[k] = a[k] * o->drag_mask[k] + o->gravity[k];
        }
        double xe[3];
        for (int k = 0; k < 3; ++k) {
          kx[k] = A[s] * kx[k] + dt * v[k];
          kv[k] = A[s] * kv[k] + dt * a[k];
          xe[k] = x[k] + B[s] * kx[k];
          v[k] = v[k] + B[s] * kv[k];
        }
        /* reference-space localisation (Sec. 3.2.3): a segment that cannot
         * reach a boundary face is not traced; the next location step finds
         * the element (recover_elem) */
        double L = sqrt((xe[0] - x[0]) * (xe[0] - x[0]) + (xe[1] - x[1]) * (xe[1] - x[1]) +
                        (xe[2] - x[2]) * (xe[2] - x[2]));
        if (!(o->tracking == 1 && L < c->dsafe[e]))
          track(c, p, x, xe, v, kx, kv, o->max_crossings, &ncross, &nhits);
        for (int k = 0; k < 3; ++k) x[k] = xe[k];
      }
    }
  /* reference coordinates of the final positions (and the inside verification) */
#pragma omp parallel for schedule(static) reduction(+ : nlost, nrec)
  for (int64_t p = 0; p < c->np; ++p) {
    if (c->status[p] != OR_ACTIVE) continue;
    double xi[3];
    int64_t a0 = 0, a1 = 0, a2 = 0;
    int e = c->elem[p];
    if (!newton_chain(c, e, c->x + p * 3, xi, o->max_newton_it, 0, &a0, &a1, &a2)) {
      /* as in the stage loop: the background-mesh candidates */
      int f = or_locate(c, c->x + p * 3, -1, xi);
      if (f < 0) { c->status[p] = OR_LOST_NEWTON; nlost++; continue; }
      c->elem[p] = f;
      nrec++;
    } else if (!inside_ref(xi)) {
      if (recover_elem(c, &e, c->x + p * 3, xi, o->max_newton_it, &a0, &a1, &a2)) {
        c->elem[p] = e;
        nrec++;
      } else {
        c->status[p] = OR_LOST_TRACK; nlost++;
      }
    }
    for (int k = 0; k < 3; ++k) c->xi[p * 3 + k] = xi[k];
  }
  c->st_newton_it += it_sum; c->st_newton_calls += calls; c->st_cross += ncross;
  c->st_hits += nhits; c->st_lost += nlost; c->st_fallback += nfb; c->st_recover += nrec;
  return 0;
}

void or_read(or_ctx* c, double* x, double* v, int32_t* elem, double* xi, int32_t* hits, int8_t* status) {
  int64_t n = c->np;
  if (x) memcpy(x, c->x, sizeof(double) * n * 3);
  if (v) memcpy(v, c->v, sizeof(double) * n * 3);
  if (elem) memcpy(elem, c->elem, sizeof(int32_t) * n);
  if (xi) memcpy(xi, c->xi, sizeof(double) * n * 3);
  if (hits) memcpy(hits, c->hits, sizeof(int32_t) * n);
  if (status) memcpy(status, c->status, n);
}

void or_stats(const or_ctx* c, int64_t* out) {
  out[0] = c->st_newton_it; out[1] = c->st_newton_calls; out[2] = c->st_cross;
  out[3] = c->st_hits; out[4] = c->st_lost; out[5] = c->st_fallback; out[6] = c->st_recover;
}
void or_reset_stats(or_ctx* c) {
  c->st_newton_it = c->st_newton_calls = c->st_cross = c->st_hits = c->st_lost = c->st_fallback = 0;
  c->st_recover = 0;
}

/* ======================================================================== */
/* two-way coupling source (Sec. 2.3, eq. theory:source)                     */
/* ======================================================================== */
/* kind 0: nearest DOF, P{a} = a / V_ijk with V_ijk = w_i w_j w_k J(xi_ijk) and
 * the nearest DOF taken per axis in reference space (lower index on ties).
 * kind 1: polynomial shape kernel K(r) = (1 - (r/R)^2)^2 over all DG nodes
 * within R, discretely normalised so that sum_k S_k V_k = a (not in the
 * paper; a smoother projection operator of the same conservation property).
 * Momentum source S_m = -F (F_D, plus the undisturbed-flow stress, added
 * mass and lift terms selected in `forces`, as in eq. theory:source; the
 * added-mass term uses dv/dt, hence the gravity argument), energy source
 * S_e = -F . v_p.  Output layout
 * [E][4][(N+1)^3]; S is accumulated into. */
int or_deposit(or_ctx* c, double* S, int kind, double R, const double* period, int drag, int forces,
               const double* gravity) {
  int n = c->n, n3 = n * n * n;
  int64_t np = c->np;
  double* F = (double*)malloc(sizeof(double) * np * 4);
  int* ok = (int*)calloc(np, sizeof(int));
  double* xi_all = (double*)malloc(sizeof(double) * np * 3);
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    if (c->status[p] != OR_ACTIVE) continue;
    int e = c->elem[p];
    double xi[3];
    int64_t a0 = 0, a1 = 0, a2 = 0;
    if (!newton_chain(c, e, c->x + p * 3, xi, 50, 0, &a0, &a1, &a2)) continue;
    double Uc[5], prim[5], a[3], fD;
    double dd = c->d[p];
    double Fv[3], fdot = 0.0;
    if (forces) {
      double G[9];
      or_fluid_grad(c, e, xi, prim, G);
      or_particle_accel(c, drag, forces, prim, G, c->v + p * 3, dd, gravity, a, Fv);
    } else {
      or_interp(c, e, xi, Uc);
      cons2prim(c->kappa, Uc, prim);
      or_drag_accel(c, drag, prim, c->v + p * 3, dd, NULL, a, &fD);
      for (int k = 0; k < 3; ++k) Fv[k] = 3.0 * M_PI * c->mu * dd * fD * (prim[1 + k] - c->v[p * 3 + k]);
    }
    for (int k = 0; k < 3; ++k) fdot += Fv[k] * c->v[p * 3 + k];
    for (int k = 0; k < 3; ++k) F[p * 4 + k] = Fv[k];
    F[p * 4 + 3] = fdot;
    for (int k = 0; k < 3; ++k) xi_all[p * 3 + k] = xi[k];
    ok[p] = 1;
  }
  if (kind == 0) {
    for (int64_t p = 0; p < np; ++p) {
      if (!ok[p]) continue;
      int e = c->elem[p];
      int idx[3];
      for (int k = 0; k < 3; ++k) {
        int best = 0;
        double bd = INFINITY;
        for (int i = 0; i < n; ++i) {
          double dd = fabs(xi_all[p * 3 + k] - c->xdg[i]);
          if (dd < bd) { bd = dd; best = i; }
        }
        idx[k] = best;
      }
      int node = (idx[2] * n + idx[1]) * n + idx[0];
      double V = c->vol[(size_t)e * n3 + node];
      for (int comp = 0; comp < 4; ++comp) S[((size_t)e * 4 + comp) * n3 + node] += -F[p * 4 + comp] / V;
    }
  } else {
    int* mark = (int*)calloc(c->E, sizeof(int));
    int* cand = (int*)malloc(sizeof(int) * c->E);
    int stamp = 0;
    for (int64_t p = 0; p < np; ++p) {
      if (!ok[p]) continue;
      const double* xp = c->x + p * 3;
      stamp++;
      int nc = 0;
      /* candidate elements: background cells overlapping the support box,
       * including periodic images */
      int img[3][3], nimg[3];
      for (int k = 0; k < 3; ++k) {
        nimg[k] = 1; img[k][0] = 0;
        if (period && period[k] > 0.0) { nimg[k] = 3; img[k][1] = 1; img[k][2] = -1; }
      }
      for (int iz = 0; iz < nimg[2]; ++iz)
        for (int iy = 0; iy < nimg[1]; ++iy)
          for (int ix = 0; ix < nimg[0]; ++ix) {
            double ctr[3] = {xp[0] + (period ? img[0][ix] * period[0] : 0.0),
                             xp[1] + (period ? img[1][iy] * period[1] : 0.0),
                             xp[2] + (period ? img[2][iz] * period[2] : 0.0)};
            int lo[3], hi[3], skip = 0;
            for (int k = 0; k < 3; ++k) {
              lo[k] = (int)floor((ctr[k] - R - c->blo[k]) / c->bdx[k]);
              hi[k] = (int)floor((ctr[k] + R - c->blo[k]) / c->bdx[k]);
              if (lo[k] < 0) lo[k] = 0;
              if (hi[k] >= c->bn[k]) hi[k] = c->bn[k] - 1;
              if (lo[k] > hi[k]) skip = 1;
            }
            if (skip) continue;
            for (int z = lo[2]; z <= hi[2]; ++z)
              for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                  size_t id = ((size_t)z * c->bn[1] + y) * c->bn[0] + x;
                  for (int q = c->bstart[id]; q < c->bstart[id + 1]; ++q) {
                    int e = c->blist[q];
                    if (mark[e] != stamp) { mark[e] = stamp; cand[nc++] = e; }
                  }
                }
          }
      /* element order for a deterministic sum */
      for (int i = 1; i < nc; ++i) {
        int v = cand[i], j = i - 1;
        while (j >= 0 && cand[j] > v) { cand[j + 1] = cand[j]; j--; }
        cand[j + 1] = v;
      }
      double norm = 0.0;
      for (int pass = 0; pass < 2; ++pass) {
        for (int ci = 0; ci < nc; ++ci) {
          int e = cand[ci];
          for (int q = 0; q < n3; ++q) {
            const double* xn = c->xnode + ((size_t)e * n3 + q) * 3;
            double r[3];
            for (int k = 0; k < 3; ++k) {
              r[k] = xn[k] - xp[k];
              if (period && period[k] > 0.0) r[k] -= period[k] * nearbyint(r[k] / period[k]);
            }
            double rr = sqrt(dot3(r, r));
            if (rr >= R) continue;
            double s = 1.0 - (rr / R) * (rr / R);
            double K = s * s;
            double V = c->vol[(size_t)e * n3 + q];
            if (pass == 0) norm += K * V;
            else
              for (int comp = 0; comp < 4; ++comp) S[((size_t)e * 4 + comp) * n3 + q] += -F[p * 4 + comp] * K / norm;
          }
        }
        if (pass == 0 && norm <= 0.0) break;
      }
    }
    free(mark); free(cand);
  }
  free(F); free(ok); free(xi_all);
  return 0;
}

/* ======================================================================== */
/* learned initial guess: 84 -> 64 -> 64 -> 64 -> 3 tanh MLP                  */
/* ======================================================================== */
/* weight layout: W1[64][84] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3] */
int64_t or_mlp_n_weights(void) {
  return (int64_t)OR_MLP_H * OR_MLP_NIN + OR_MLP_H + 2 * (OR_MLP_H * OR_MLP_H + OR_MLP_H) +
         OR_MLP_NOUT * OR_MLP_H + OR_MLP_NOUT;
}

/* Inputs (84): the 8 element corners relative to the corner mean (24); the
 * deviation of the element map from the trilinear map of its corners at the 19
 * other points of the {-1,0,1}^3 lattice (57), which carries the curvature; the
 * point relative to the corner mean (3).  All lengths are divided by the mean
 * corner-edge length. */
void or_mlp_features(const or_ctx* c, int e, const double* x, double* feat) {
  int ng = c->ng, G = c->n_geo;
  const double* P = c->X + (size_t)e * ng * ng * ng * 3;
  double cor[8][3], ctr[3] = {0, 0, 0};
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) {
        int q = ((k * G) * ng + j * G) * ng + i * G;
        for (int r = 0; r < 3; ++r) { cor[(k * 2 + j) * 2 + i][r] = P[q * 3 + r]; ctr[r] += P[q * 3 + r]; }
      }
  for (int r = 0; r < 3; ++r) ctr[r] /= 8.0;
  double hs = 0.0;
  for (int a = 0; a < 8; ++a)
    for (int bit = 0; bit < 3; ++bit) {
      int b = a ^ (1 << bit);
      if (b < a) continue;
      double d[3] = {cor[a][0] - cor[b][0], cor[a][1] - cor[b][1], cor[a][2] - cor[b][2]};
      hs += norm3(d);
    }
  double h = hs / 12.0;
  for (int a = 0; a < 8; ++a)
    for (int r = 0; r < 3; ++r) feat[a * 3 + r] = (cor[a][r] - ctr[r]) / h;
  int f = 24;
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) {
        if (i != 1 && j != 1 && k != 1) continue;     /* corners */
        double xi[3] = {(double)(i - 1), (double)(j - 1), (double)(k - 1)};
        double pm[3];
        or_map(c, e, xi, pm, NULL);
        double tri[3] = {0, 0, 0};
        for (int kk = 0; kk < 2; ++kk)
          for (int jj = 0; jj < 2; ++jj)
            for (int ii = 0; ii < 2; ++ii) {
              double wgt = 0.125 * (1.0 + (ii ? 1 : -1) * xi[0]) * (1.0 + (jj ? 1 : -1) * xi[1]) *
                           (1.0 + (kk ? 1 : -1) * xi[2]);
              for (int r = 0; r < 3; ++r) tri[r] += wgt * cor[(kk * 2 + jj) * 2 + ii][r];
            }
        for (int r = 0; r < 3; ++r) feat[f + r] = (pm[r] - tri[r]) / h;
        f += 3;
      }
  for (int r = 0; r < 3; ++r) feat[81 + r] = (x[r] - ctr[r]) / h;
}

static double* mlp_forward1(const double* w, const double* in, double* out) {
  const int H = OR_MLP_H;
  const double* W1 = w;
  const double* b1 = W1 + H * OR_MLP_NIN;
  const double* W2 = b1 + H;
  const double* b2 = W2 + H * H;
  const double* W3 = b2 + H;
  const double* b3 = W3 + H * H;
  const double* W4 = b3 + H;
  const double* b4 = W4 + OR_MLP_NOUT * H;
  double h1[OR_MLP_H], h2[OR_MLP_H], h3[OR_MLP_H];
  for (int o = 0; o < H; ++o) {
    double s = b1[o];
    for (int i = 0; i < OR_MLP_NIN; ++i) s += W1[o * OR_MLP_NIN + i] * in[i];
    h1[o] = tanh(s);
  }
  for (int o = 0; o < H; ++o) {
    double s = b2[o];
    for (int i = 0; i < H; ++i) s += W2[o * H + i] * h1[i];
    h2[o] = tanh(s);
  }
  for (int o = 0; o < H; ++o) {
    double s = b3[o];
    for (int i = 0; i < H; ++i) s += W3[o * H + i] * h2[i];
    h3[o] = tanh(s);
  }
  for (int o = 0; o < OR_MLP_NOUT; ++o) {
    double s = b4[o];
    for (int i = 0; i < H; ++i) s += W4[o * H + i] * h3[i];
    out[o] = s;
  }
  return out;
}

void or_mlp_forward(const double* w, int64_t n, const double* in, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) mlp_forward1(w, in + r * OR_MLP_NIN, out + r * OR_MLP_NOUT);
}

/* mean squared error over n rows and 3 outputs, and its gradient (backprop) */
double or_mlp_loss_grad(const double* w, int64_t n, const double* in, const double* target, double* grad) {
  const int H = OR_MLP_H, NI = OR_MLP_NIN, NO = OR_MLP_NOUT;
  int64_t nw = or_mlp_n_weights();
  memset(grad, 0, sizeof(double) * nw);
  const double* W1 = w;
  const double* b1 = W1 + H * NI;
  const double* W2 = b1 + H;
  const double* b2 = W2 + H * H;
  const double* W3 = b2 + H;
  const double* b3 = W3 + H * H;
  const double* W4 = b3 + H;
  const double* b4 = W4 + NO * H;
  double* gW1 = grad;
  double* gb1 = gW1 + H * NI;
  double* gW2 = gb1 + H;
  double* gb2 = gW2 + H * H;
  double* gW3 = gb2 + H;
  double* gb3 = gW3 + H * H;
  double* gW4 = gb3 + H;
  double* gb4 = gW4 + NO * H;
  double loss = 0.0;
  double scale = 1.0 / ((double)n * NO);
  for (int64_t r = 0; r < n; ++r) {
    const double* x = in + r * NI;
    double h1[OR_MLP_H], h2[OR_MLP_H], h3[OR_MLP_H], y[OR_MLP_NOUT];
    for (int o = 0; o < H; ++o) { double s = b1[o]; for (int i = 0; i < NI; ++i) s += W1[o * NI + i] * x[i]; h1[o] = tanh(s); }
    for (int o = 0; o < H; ++o) { double s = b2[o]; for (int i = 0; i < H; ++i) s += W2[o * H + i] * h1[i]; h2[o] = tanh(s); }
    for (int o = 0; o < H; ++o) { double s = b3[o]; for (int i = 0; i < H; ++i) s += W3[o * H + i] * h2[i]; h3[o] = tanh(s); }
    for (int o = 0; o < NO; ++o) { double s = b4[o]; for (int i = 0; i < H; ++i) s += W4[o * H + i] * h3[i]; y[o] = s; }
    double dy[OR_MLP_NOUT];
    for (int o = 0; o < NO; ++o) {
      double diff = y[o] - target[r * NO + o];
      loss += diff * diff * scale;
      dy[o] = 2.0 * diff * scale;
    }
    double d3[OR_MLP_H], d2[OR_MLP_H], d1[OR_MLP_H];
    for (int i = 0; i < H; ++i) {
      double s = 0.0;
      for (int o = 0; o < NO; ++o) s += W4[o * H + i] * dy[o];
      d3[i] = s * (1.0 - h3[i] * h3[i]);
    }
    for (int o = 0; o < NO; ++o) {
      gb4[o] += dy[o];
      for (int i = 0; i < H; ++i) gW4[o * H + i] += dy[o] * h3[i];
    }
    for (int i = 0; i < H; ++i) {
      double s = 0.0;
      for (int o = 0; o < H; ++o) s += W3[o * H + i] * d3[o];
      d2[i] = s * (1.0 - h2[i] * h2[i]);
    }
    for (int o = 0; o < H; ++o) {
      gb3[o] += d3[o];
      for (int i = 0; i < H; ++i) gW3[o * H + i] += d3[o] * h2[i];
    }
    for (int i = 0; i < H; ++i) {
      double s = 0.0;
      for (int o = 0; o < H; ++o) s += W2[o * H + i] * d2[o];
      d1[i] = s * (1.0 - h1[i] * h1[i]);
    }
    for (int o = 0; o < H; ++o) {
      gb2[o] += d2[o];
      for (int i = 0; i < H; ++i) gW2[o * H + i] += d2[o] * h1[i];
    }
    for (int o = 0; o < H; ++o) {
      gb1[o] += d1[o];
      for (int i = 0; i < NI; ++i) gW1[o * NI + i] += d1[o] * x[i];
    }
  }
  return loss;
}

/* Adam (Kingma & Ba 2015) with bias correction; t is the 1-based step */
void or_adam(double* w, double* m, double* v, const double* g, int64_t nw, int64_t t, double lr,
             double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < nw; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    w[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* one epoch of minibatch Adam over rows in the given order */
double or_mlp_train(double* w, double* m, double* v, int64_t* t, const double* in, const double* target,
                    const int32_t* order, int64_t n, int batch, double lr, double* loss_hist) {
  int64_t nw = or_mlp_n_weights();
  double* g = (double*)malloc(sizeof(double) * nw);
  double* bi = (double*)malloc(sizeof(double) * (size_t)batch * OR_MLP_NIN);
  double* bt = (double*)malloc(sizeof(double) * (size_t)batch * OR_MLP_NOUT);
  double tot = 0.0;
  int64_t nb = 0;
  for (int64_t s = 0; s + batch <= n; s += batch) {
    for (int r = 0; r < batch; ++r) {
      int64_t src = order[s + r];
      memcpy(bi + r * OR_MLP_NIN, in + src * OR_MLP_NIN, sizeof(double) * OR_MLP_NIN);
      memcpy(bt + r * OR_MLP_NOUT, target + src * OR_MLP_NOUT, sizeof(double) * OR_MLP_NOUT);
    }
    double l = or_mlp_loss_grad(w, batch, bi, bt, g);
    (*t)++;
    or_adam(w, m, v, g, nw, *t, lr, 0.9, 0.999, 1e-8);
    if (loss_hist) loss_hist[nb] = l;
    tot += l;
    nb++;
  }
  free(g); free(bi); free(bt);
  return nb ? tot / nb : 0.0;
}

/* The draws of a seeded training run.  Generator: SplitMix64 (Steele, Lea and
 * Flood, OOPSLA 2014), the i-th output of stream `seed` being the finaliser
 * applied to seed + i * 0x9E3779B97F4A7C15 (i = 1, 2, ...).  Uniform in [0, 1):
 * the top 53 bits times 2^-53.  Order of the draws: one uniform per weight in
 * layout order (Xavier-uniform matrices, a * (2u - 1) with
 * a = sqrt(6 / (fan_in + fan_out)); biases zero, no draw), then for each
 * epoch a Fisher-Yates shuffle of 0..n-1: for i = n-1 down to 1 swap a[i]
 * with a[j], j = floor(z (i + 1) / 2^64) for the next output z.
 * orders: [epochs][n]. */
static uint64_t sm64_next(uint64_t* st) {
  uint64_t z;
  *st += 0x9E3779B97F4A7C15ull;
  z = *st;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void or_mlp_draws(uint64_t seed, int64_t n, int epochs, double* w0, int32_t* orders) {
  const int rows[4] = {OR_MLP_H, OR_MLP_H, OR_MLP_H, OR_MLP_NOUT};
  const int cols[4] = {OR_MLP_NIN, OR_MLP_H, OR_MLP_H, OR_MLP_H};
  uint64_t st = seed;
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    double a = sqrt(6.0 / (double)(rows[l] + cols[l]));
    for (int i = 0; i < rows[l] * cols[l]; ++i) {
      double u = (double)(sm64_next(&st) >> 11) * (1.0 / 9007199254740992.0);
      w0[o++] = a * (2.0 * u - 1.0);
    }
    for (int i = 0; i < rows[l]; ++i) w0[o++] = 0.0;
  }
  for (int ep = 0; ep < epochs; ++ep) {
    int32_t* a = orders + (int64_t)ep * n;
    for (int64_t i = 0; i < n; ++i) a[i] = (int32_t)i;
    for (int64_t i = n - 1; i >= 1; --i) {
      uint64_t z = sm64_next(&st);
      int64_t j = (int64_t)(((unsigned __int128)z * (unsigned __int128)(i + 1)) >> 64);
      int32_t t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
}

void or_set_mlp(or_ctx* c, const double* w, const uint8_t* flag) {
  free(c->mlp_w); free(c->mlp_flag);
  c->mlp_w = NULL; c->mlp_flag = NULL;
  if (!w) return;
  int64_t nw = or_mlp_n_weights();
  c->mlp_w = (double*)malloc(sizeof(double) * nw);
  memcpy(c->mlp_w, w, sizeof(double) * nw);
  c->mlp_flag = (uint8_t*)malloc(c->E);
  memcpy(c->mlp_flag, flag, c->E);
}

/* strongly curved elements: some geometry node deviates from the trilinear
 * interpolant of the 8 corners by more than thresh * h_e */
void or_curved_flags(const or_ctx* c, double thresh, uint8_t* flag) {
  int ng = c->ng, G = c->n_geo;
  for (int e = 0; e < c->E; ++e) {
    const double* P = c->X + (size_t)e * ng * ng * ng * 3;
    double dev = 0.0;
    for (int k = 0; k < ng; ++k)
      for (int j = 0; j < ng; ++j)
        for (int i = 0; i < ng; ++i) {
          double s = (double)i / G, t = (double)j / G, u = (double)k / G;
          double tri[3] = {0, 0, 0};
          for (int kk = 0; kk < 2; ++kk)
            for (int jj = 0; jj < 2; ++jj)
              for (int ii = 0; ii < 2; ++ii) {
                double wgt = (ii ? s : 1 - s) * (jj ? t : 1 - t) * (kk ? u : 1 - u);
                int q = ((kk * G) * ng + jj * G) * ng + ii * G;
                for (int r = 0; r < 3; ++r) tri[r] += wgt * P[q * 3 + r];
              }
          const double* Q = P + ((k * ng + j) * ng + i) * 3;
          double d[3] = {Q[0] - tri[0], Q[1] - tri[1], Q[2] - tri[2]};
          double l = norm3(d);
          if (l > dev) dev = l;
        }
    flag[e] = dev > thresh * c->hE[e];
  }
}

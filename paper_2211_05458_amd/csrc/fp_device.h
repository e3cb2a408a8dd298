// Device building blocks of the per-particle step (gfx950).  Loop bounds are
// compile-time node counts so that the tensor-product sums unroll into
// straight FMA chains.
#pragma once
#include "fp_internal.h"

namespace fp {

__device__ __forceinline__ double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// ---------------------------------------------------------------------------
// Lagrange basis l_i(x) = c_i prod_{j != i}(x - x_j), c_i = 1/prod_{j != i}(x_i - x_j)
// ---------------------------------------------------------------------------
template <int N, typename T>
__device__ __forceinline__ void lagrange(const T* nodes, const T* cden, T x, T* l) {
  T dx[N];
#pragma unroll
  for (int j = 0; j < N; ++j) dx[j] = x - nodes[j];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T p = cden[i];
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j != i) p *= dx[j];
    l[i] = p;
  }
}

template <int N>
__device__ __forceinline__ void lagrange_d(const double* nodes, const double* cden, double x, double* l,
                                           double* dl) {
  double dx[N];
#pragma unroll
  for (int j = 0; j < N; ++j) dx[j] = x - nodes[j];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double p = 1.0, dp = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j != i) {
        dp = dp * dx[j] + p;
        p *= dx[j];
      }
    l[i] = cden[i] * p;
    dl[i] = cden[i] * dp;
  }
}

// l_i, l_i' and l_i'' at x (product rule over the factors (x - x_j))
template <int N>
__device__ __forceinline__ void lagrange_d2(const double* nodes, const double* cden, double x, double* l,
                                            double* dl, double* d2l) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double p = 1.0, dp = 0.0, d2p = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j != i) {
        const double dx = x - nodes[j];
        d2p = d2p * dx + 2.0 * dp;
        dp = dp * dx + p;
        p *= dx;
      }
    l[i] = cden[i] * p;
    dl[i] = cden[i] * dp;
    d2l[i] = cden[i] * d2p;
  }
}

// ---------------------------------------------------------------------------
// chi_e(xi) and J = d chi / d xi by sum factorisation over i, then j, then k
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void lagrange1_d(const double* nodes, const double* cden, double x, int i, double& l,
                                            double& dl) {
  double p = 1.0, dp = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j)
    if (j != i) {
      double dx = x - nodes[j];
      dp = dp * dx + p;
      p *= dx;
    }
  l = cden[i] * p;
  dl = cden[i] * dp;
}

template <int N, typename T>
__device__ __forceinline__ T lagrange1(const T* nodes, const T* cden, T x, int i) {
  T p = cden[i];
#pragma unroll
  for (int j = 0; j < N; ++j)
    if (j != i) p *= (x - nodes[j]);
  return p;
}

template <int NG>
__device__ __forceinline__ void map_jac(const MeshView& m, const double* __restrict__ X, const double* xi,
                                        double* x, double J[3][3]) {
  double l1[NG], d1[NG], l2[NG], d2[NG];
  lagrange_d<NG>(m.xgeo, m.cgeo, xi[0], l1, d1);
  lagrange_d<NG>(m.xgeo, m.cgeo, xi[1], l2, d2);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    x[q] = 0.0;
    J[q][0] = J[q][1] = J[q][2] = 0.0;
  }
  // one xi3-slab of NG*NG nodes per iteration; l_k(xi3) computed in the slab
#pragma unroll 1
  for (int k = 0; k < NG; ++k) {
    double l3, d3;
    lagrange1_d<NG>(m.xgeo, m.cgeo, xi[2], k, l3, d3);
    const double* Xk = X + k * NG * NG * 3;
    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0}, c[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      double s0[3] = {0, 0, 0}, s1[3] = {0, 0, 0};
#pragma unroll
      for (int i = 0; i < NG; ++i) {
        const double* P = Xk + (j * NG + i) * 3;
        double p0 = P[0], p1 = P[1], p2 = P[2];
        s0[0] += p0 * l1[i]; s0[1] += p1 * l1[i]; s0[2] += p2 * l1[i];
        s1[0] += p0 * d1[i]; s1[1] += p1 * d1[i]; s1[2] += p2 * d1[i];
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        a[q] += s0[q] * l2[j];
        b[q] += s1[q] * l2[j];
        c[q] += s0[q] * d2[j];
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      x[q] += a[q] * l3;
      J[q][0] += b[q] * l3;
      J[q][1] += c[q] * l3;
      J[q][2] += a[q] * d3;
    }
  }
}

// Newton for chi(xi) = x (Sec. 3.2.1): Cramer's rule, stop after an update with
// max-norm <= 1e-10, divergence when |xi| > 2 after the third iteration.
// Ji (may be null): on success, the inverse of the last Jacobian (row-major),
// the Jacobian at the iterate before the final update, for continuing xi
// along a short displacement
template <int NG>
__device__ bool newton_e(const MeshView& m, const double* __restrict__ X, const double* x, double* z, int max_it,
                         int& iters, double* Ji = nullptr, double tol = kNewtonTol) {
  for (int it = 1; it <= max_it; ++it) {
    double F[3], J[3][3];
    map_jac<NG>(m, X, z, F, J);
    F[0] -= x[0]; F[1] -= x[1]; F[2] -= x[2];
    double det = det3(J);
    if (!(det != 0.0) || !isfinite(det)) { iters += it; return false; }
    double inv = 1.0 / det;
    // Cramer: dz_d = det(J with column d replaced by -F) / det
    double dz0 = -(F[0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (F[1] * J[2][2] - J[1][2] * F[2]) +
                   J[0][2] * (F[1] * J[2][1] - J[1][1] * F[2])) * inv;
    double dz1 = -(J[0][0] * (F[1] * J[2][2] - J[1][2] * F[2]) - F[0] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                   J[0][2] * (J[1][0] * F[2] - F[1] * J[2][0])) * inv;
    double dz2 = -(J[0][0] * (J[1][1] * F[2] - F[1] * J[2][1]) - J[0][1] * (J[1][0] * F[2] - F[1] * J[2][0]) +
                   F[0] * (J[1][0] * J[2][1] - J[1][1] * J[2][0])) * inv;
    z[0] += dz0; z[1] += dz1; z[2] += dz2;
    double dmax = fmax(fabs(dz0), fmax(fabs(dz1), fabs(dz2)));
    if (!isfinite(z[0]) || !isfinite(z[1]) || !isfinite(z[2])) { iters += it; return false; }
    if (dmax <= tol) {
      iters += it;
      if (Ji) {
        Ji[0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * inv;
        Ji[1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * inv;
        Ji[2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * inv;
        Ji[3] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * inv;
        Ji[4] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * inv;
        Ji[5] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * inv;
        Ji[6] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * inv;
        Ji[7] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * inv;
        Ji[8] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * inv;
      }
      return true;
    }
    if (it >= 3 && fmax(fabs(z[0]), fmax(fabs(z[1]), fabs(z[2]))) > 2.0) { iters += it; return false; }
  }
  iters += max_it;
  return false;
}

template <int NG>
__device__ __forceinline__ bool newton(const MeshView& m, int e, const double* x, double* z, int max_it, int& iters) {
  return newton_e<NG>(m, m.X + (size_t)e * (NG * NG * NG * 3), x, z, max_it, iters);
}

// nearest of n3 nodes P[q][3] (lowest index on ties)
template <int N3>
__device__ __forceinline__ int nearest_node(const double* __restrict__ P, const double* x) {
  int best = 0;
  double bd = 1e300;
#pragma unroll 5
  for (int q = 0; q < N3; ++q) {
    double dx = P[q * 3] - x[0], dy = P[q * 3 + 1] - x[1], dz = P[q * 3 + 2] - x[2];
    double dd = dx * dx + dy * dy + dz * dz;
    if (dd < bd) { bd = dd; best = q; }
  }
  return best;
}

// Paper's initial guess (Sec. 3.2.1): nearest DG node (straight elements) or
// nearest geometry node (curved), lowest index on ties.  Xe / XNe are the
// element's geometry nodes and physical DG node positions.
template <int NN, int NG>
__device__ __forceinline__ void guess_paper_e(const MeshView& m, const double* __restrict__ Xe,
                                              const double* __restrict__ XNe, const double* x, double* g) {
  if (NG == 2) {
    int best = nearest_node<NN * NN * NN>(XNe, x);
    g[0] = m.xdg[best % NN];
    g[1] = m.xdg[(best / NN) % NN];
    g[2] = m.xdg[best / (NN * NN)];
  } else {
    int best = nearest_node<NG * NG * NG>(Xe, x);
    g[0] = m.xgeo[best % NG];
    g[1] = m.xgeo[(best / NG) % NG];
    g[2] = m.xgeo[best / (NG * NG)];
  }
}

template <int NN, int NG>
__device__ __forceinline__ void guess_paper(const MeshView& m, int e, const double* x, double* g) {
  guess_paper_e<NN, NG>(m, m.X + (size_t)e * (NG * NG * NG * 3), m.xnode + (size_t)e * (NN * NN * NN * 3), x, g);
}

// Third approach of Sec. 3.2.1: projection onto the directions from the node
// mean to the node means of opposite faces.
template <int NG>
__device__ void guess_faces_e(const double* __restrict__ P, const double* x, double* g) {
  double c[3] = {0, 0, 0};
  double f[6][3] = {{0}};
  for (int k = 0; k < NG; ++k)
    for (int j = 0; j < NG; ++j)
      for (int i = 0; i < NG; ++i) {
        const double* Q = P + ((k * NG + j) * NG + i) * 3;
        for (int r = 0; r < 3; ++r) {
          c[r] += Q[r];
          if (i == 0) f[0][r] += Q[r];
          if (i == NG - 1) f[1][r] += Q[r];
          if (j == 0) f[2][r] += Q[r];
          if (j == NG - 1) f[3][r] += Q[r];
          if (k == 0) f[4][r] += Q[r];
          if (k == NG - 1) f[5][r] += Q[r];
        }
      }
  const double inv3 = 1.0 / (NG * NG * NG), inv2 = 1.0 / (NG * NG);
  for (int r = 0; r < 3; ++r) c[r] *= inv3;
  double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  for (int a = 0; a < 3; ++a) {
    double sm[3], sp[3];
    for (int r = 0; r < 3; ++r) {
      sm[r] = f[2 * a][r] * inv2 - c[r];
      sp[r] = f[2 * a + 1][r] * inv2 - c[r];
    }
    double val = 0.5 * (dot3(d, sp) / dot3(sp, sp) - dot3(d, sm) / dot3(sm, sm));
    g[a] = fmin(1.0, fmax(-1.0, val));
  }
}

template <int NG>
__device__ __forceinline__ void guess_faces(const MeshView& m, int e, const double* x, double* g) {
  guess_faces_e<NG>(m.X + (size_t)e * (NG * NG * NG * 3), x, g);
}

__device__ __forceinline__ bool inside_ref(const double* xi) {
  return fabs(xi[0]) <= 1.0 + kInsideEps && fabs(xi[1]) <= 1.0 + kInsideEps && fabs(xi[2]) <= 1.0 + kInsideEps;
}

// ---------------------------------------------------------------------------
// learned guess: features and forward pass (FP32)
// ---------------------------------------------------------------------------
// Learned-guess inputs (84): corners relative to their mean (24), deviation of
// the element map from the trilinear map of the corners at the 19 non-corner
// points of the {-1,0,1}^3 lattice (57; zero for straight elements), and the
// point (3); lengths divided by the mean corner-edge length.
template <int NG>
__device__ void mlp_features(const MeshView& m, int e, const double* x, float* feat, double* ctr_ih = nullptr) {
  const double* P = m.X + (size_t)e * (NG * NG * NG * 3);
  constexpr int G = NG - 1;
  double cor[8][3], ctr[3] = {0, 0, 0};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    int i = c & 1, j = (c >> 1) & 1, k = c >> 2;
    const double* Q = P + (((k * G) * NG + j * G) * NG + i * G) * 3;
    for (int r = 0; r < 3; ++r) { cor[c][r] = Q[r]; ctr[r] += Q[r]; }
  }
  for (int r = 0; r < 3; ++r) ctr[r] *= 0.125;
  double hs = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int bit = 0; bit < 3; ++bit) {
      int b = a ^ (1 << bit);
      if (b < a) continue;
      double dx = cor[a][0] - cor[b][0], dy = cor[a][1] - cor[b][1], dz = cor[a][2] - cor[b][2];
      hs += sqrt(dx * dx + dy * dy + dz * dz);
    }
  double ih = 12.0 / hs;
  if (ctr_ih) {
    ctr_ih[0] = ctr[0]; ctr_ih[1] = ctr[1]; ctr_ih[2] = ctr[2]; ctr_ih[3] = ih;
  }
#pragma unroll
  for (int a = 0; a < 8; ++a)
    for (int r = 0; r < 3; ++r) feat[a * 3 + r] = (float)((cor[a][r] - ctr[r]) * ih);
  int f = 24;
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) {
        if (i != 1 && j != 1 && k != 1) continue;
        if (G % 2 != 0) {
          feat[f] = feat[f + 1] = feat[f + 2] = 0.0f;   // degree-1 geometry is trilinear
        } else {
          const double* Q = P + (((k * G / 2) * NG + j * G / 2) * NG + i * G / 2) * 3;
          double s0 = i - 1.0, s1 = j - 1.0, s2 = k - 1.0;
          for (int r = 0; r < 3; ++r) {
            double tri = 0.0;
            for (int c = 0; c < 8; ++c)
              tri += 0.125 * (1.0 + ((c & 1) ? 1 : -1) * s0) * (1.0 + (((c >> 1) & 1) ? 1 : -1) * s1) *
                     (1.0 + ((c >> 2) ? 1 : -1) * s2) * cor[c][r];
            feat[f + r] = (float)((Q[r] - tri) * ih);
          }
        }
        f += 3;
      }
  for (int r = 0; r < 3; ++r) feat[81 + r] = (float)((x[r] - ctr[r]) * ih);
}

__device__ __forceinline__ float fast_tanh(float s) { return tanhf(s); }

// 84-64-64-64-3 forward for one row; weights read through the scalar path
// (uniform addresses).
__device__ inline void mlp_forward_row(const float* __restrict__ w, const float* in, float* out) {
  constexpr int H = 64, NI = kMlpIn;
  const float* W1 = w;
  const float* b1 = W1 + H * NI;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + H * H;
  const float* W4 = b3 + H;
  const float* b4 = W4 + 3 * H;
  float h1[H], h2[H];
#pragma unroll 4
  for (int o = 0; o < H; ++o) {
    float s = b1[o];
#pragma unroll
    for (int i = 0; i < NI; ++i) s += W1[o * NI + i] * in[i];
    h1[o] = fast_tanh(s);
  }
#pragma unroll 2
  for (int o = 0; o < H; ++o) {
    float s = b2[o];
#pragma unroll
    for (int i = 0; i < H; ++i) s += W2[o * H + i] * h1[i];
    h2[o] = fast_tanh(s);
  }
#pragma unroll 2
  for (int o = 0; o < H; ++o) {
    float s = b3[o];
#pragma unroll
    for (int i = 0; i < H; ++i) s += W3[o * H + i] * h2[i];
    h1[o] = fast_tanh(s);
  }
  for (int o = 0; o < 3; ++o) {
    float s = b4[o];
#pragma unroll
    for (int i = 0; i < H; ++i) s += W4[o * H + i] * h1[i];
    out[o] = s;
  }
}

// Reference coordinates of x in element e: the continued coordinates of the
// particle's previous position (gw, may be null), then the learned guess
// (flagged elements; gin, the stage's precomputed guess of this particle),
// then the paper's guess, then the face-barycentre guess.  Ji (may be null):
// see newton_e.
// (The guesses come as arrays with flags, not as pointers that may be null:
// a pointer chosen at run time between an array and null keeps the array out
// of registers.)
template <int NN, int NG, bool MLP = false>
__device__ bool locate_xi_e(const MeshView& m, int e, const double* __restrict__ Xe, const double* __restrict__ XNe,
                            const double* x, double* xi, int max_it, int& it_sum, int& calls, int& fallbacks,
                            bool use_gin = false, const float* gin = nullptr, bool use_gw = false,
                            const double* gw = nullptr, double* Ji = nullptr, double tol = kNewtonTol) {
  double g[3];
  // the first guess of each lane (continued coordinates, else the learned
  // guess on a flagged element, else the paper's), then one Newton for all
  // lanes of the wavefront together; the other guesses only on failure
  const bool learned = MLP && use_gin && m.mlp_flag[e];
  int first;
  if (use_gw) {
    first = 0;
    g[0] = gw[0]; g[1] = gw[1]; g[2] = gw[2];
  } else if (learned) {
    first = 1;
    g[0] = gin[0]; g[1] = gin[1]; g[2] = gin[2];
  } else {
    first = 2;
    guess_paper_e<NN, NG>(m, Xe, XNe, x, g);
  }
  calls++;
  if (newton_e<NG>(m, Xe, x, g, max_it, it_sum, Ji, tol)) { xi[0] = g[0]; xi[1] = g[1]; xi[2] = g[2]; return true; }
  fallbacks++;
  if (first < 1 && learned) {
    g[0] = gin[0]; g[1] = gin[1]; g[2] = gin[2];
    calls++;
    if (newton_e<NG>(m, Xe, x, g, max_it, it_sum, Ji, tol)) { xi[0] = g[0]; xi[1] = g[1]; xi[2] = g[2]; return true; }
    fallbacks++;
  }
  if (first < 2) {
    guess_paper_e<NN, NG>(m, Xe, XNe, x, g);
    calls++;
    if (newton_e<NG>(m, Xe, x, g, max_it, it_sum, Ji, tol)) { xi[0] = g[0]; xi[1] = g[1]; xi[2] = g[2]; return true; }
    fallbacks++;
  }
  guess_faces_e<NG>(Xe, x, g);
  calls++;
  bool ok = newton_e<NG>(m, Xe, x, g, max_it, it_sum, Ji, tol);
  xi[0] = g[0]; xi[1] = g[1]; xi[2] = g[2];
  return ok;
}

// the continued reference coordinates of a particle, if stored and plausible
__device__ __forceinline__ bool warm_guess(const Particles& P, int64_t p, double* gw) {
  const int64_t cap = P.cap;
  gw[0] = P.xi[p];
  gw[1] = P.xi[cap + p];
  gw[2] = P.xi[2 * cap + p];
  return fabs(gw[0]) <= 1.5 && fabs(gw[1]) <= 1.5 && fabs(gw[2]) <= 1.5;   // false for the NaN mark
}

// xi + Ji (xe - x): the reference coordinates of the end of a short step
// from x, to first order, stored as the next location's guess
__device__ __forceinline__ void store_warm(const Particles& P, int64_t p, const double* xi, const double* Ji,
                                           const double* x, const double* xe) {
  const int64_t cap = P.cap;
  const double d[3] = {xe[0] - x[0], xe[1] - x[1], xe[2] - x[2]};
#pragma unroll
  for (int k = 0; k < 3; ++k) P.xi[k * cap + p] = xi[k] + Ji[3 * k] * d[0] + Ji[3 * k + 1] * d[1] + Ji[3 * k + 2] * d[2];
}

template <int NN, int NG>
__device__ __forceinline__ bool locate_xi(const MeshView& m, int e, const double* x, double* xi, int max_it,
                                          bool use_mlp, int& it_sum, int& calls, int& fallbacks,
                                          bool use_gw = false, const double* gw = nullptr) {
  (void)use_mlp;
  return locate_xi_e<NN, NG, false>(m, e, m.X + (size_t)e * (NG * NG * NG * 3),
                                    m.xnode + (size_t)e * (NN * NN * NN * 3), x, xi, max_it, it_sum, calls, fallbacks,
                                    false, nullptr, use_gw, gw);
}

// A located particle lies outside its element: a crossing that was not traced
// (reference-space localisation) or that the clipping budget missed at
// grazing incidence.  Follow the reference coordinate with the largest excess
// to the neighbour across that face (lowest axis on ties), applying the
// periodic shift, and locate again, at most kRecoverHops times; then try the
// background-mesh candidates of the point (the paper's localisation).  Walls
// and open faces end the hops.  On success e, x and xi describe the particle
// in its element.
template <int NN, int NG>
__device__ inline int bgm_locate(const MeshView& m, const double* x, double* xi, int& it_sum, int& calls,
                                 int& fallbacks);

template <int NN, int NG>
__device__ inline bool recover_elem(const MeshView& m, int& e, double* x, double* xi, int max_it, int& it_sum,
                                    int& calls, int& fallbacks) {
  int eh = e;
  double xh[3] = {x[0], x[1], x[2]};
#pragma unroll 1
  for (int hop = 0; hop < kRecoverHops; ++hop) {
    int d = 0;
    double ex = fabs(xi[0]);
    if (fabs(xi[1]) > ex) { d = 1; ex = fabs(xi[1]); }
    if (fabs(xi[2]) > ex) { d = 2; ex = fabs(xi[2]); }
    const FaceRec& F = m.faces[eh * 6 + 2 * d + (xi[d] > 0.0 ? 1 : 0)];
    if (F.bc != BC_INTERNAL && F.bc != BC_PERIODIC) break;
    if (F.bc == BC_PERIODIC)
      for (int k = 0; k < 3; ++k) xh[k] += F.shift[k];
    eh = F.nbr_elem;
    if (!locate_xi<NN, NG>(m, eh, xh, xi, max_it, false, it_sum, calls, fallbacks)) break;
    if (inside_ref(xi)) {
      e = eh;
      x[0] = xh[0]; x[1] = xh[1]; x[2] = xh[2];
      return true;
    }
  }
  // the paper's localisation: the background-mesh candidates of the point
  const int f = bgm_locate<NN, NG>(m, x, xi, it_sum, calls, fallbacks);
  if (f < 0) return false;
  e = f;
  return true;
}

// first background-mesh candidate of x (element order) whose padded box holds
// x and whose Newton solution lies inside; -1 if none
template <int NN, int NG>
__device__ inline int bgm_locate(const MeshView& m, const double* x, double* xi, int& it_sum, int& calls,
                                 int& fallbacks) {
  int c[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = (int)floor((x[k] - m.blo[k]) / m.bdx[k]);
    if (!(c[k] >= 0 && c[k] < m.bn[k])) return -1;
  }
  const int64_t cell = ((int64_t)c[2] * m.bn[1] + c[1]) * m.bn[0] + c[0];
#pragma unroll 1
  for (int q = m.bstart[cell]; q < m.bstart[cell + 1]; ++q) {
    const int e = m.blist[q];
    if (x[0] < m.elo[e * 3] || x[0] > m.ehi[e * 3] || x[1] < m.elo[e * 3 + 1] || x[1] > m.ehi[e * 3 + 1] ||
        x[2] < m.elo[e * 3 + 2] || x[2] > m.ehi[e * 3 + 2])
      continue;
    if (locate_xi<NN, NG>(m, e, x, xi, 50, false, it_sum, calls, fallbacks) && inside_ref(xi)) return e;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// interpolation of the conservative variables (eq. part_interpolation).  The
// drag law reads density and momentum only (constant viscosity), so the
// energy, the fifth variable of each element's block, is not interpolated
// (kInterpVars).
// ---------------------------------------------------------------------------

template <int NN, typename UT>
__device__ __forceinline__ void interp(const MeshView& m, const UT* __restrict__ U, const double* xi, double* out) {
  double l1[NN], l2[NN];
  lagrange<NN, double>(m.xdg, m.cdg, xi[0], l1);
  lagrange<NN, double>(m.xdg, m.cdg, xi[1], l2);
  constexpr int N3 = NN * NN * NN;
  double acc[kInterpVars] = {};
  // one xi3-slab per iteration: the NN*NN nodes of every variable read
#pragma unroll 1
  for (int k = 0; k < NN; ++k) {
    double l3 = lagrange1<NN, double>(m.xdg, m.cdg, xi[2], k);
#pragma unroll
    for (int var = 0; var < kInterpVars; ++var) {
      const UT* Uk = U + var * N3 + k * NN * NN;
      double sk = 0.0;
#pragma unroll
      for (int j = 0; j < NN; ++j) {
        double sj = 0.0;
#pragma unroll
        for (int i = 0; i < NN; ++i) sj += (double)Uk[j * NN + i] * l1[i];
        sk += sj * l2[j];
      }
      acc[var] += sk * l3;
    }
  }
#pragma unroll
  for (int var = 0; var < kInterpVars; ++var) out[var] = acc[var];
}

// FP32 interpolation (mixed precision): FP32 basis and accumulation.
template <int NN, typename UT>
__device__ __forceinline__ void interp_f32(const MeshView& m, const UT* __restrict__ U, const double* xi, float* out) {
  float l1[NN], l2[NN];
  lagrange<NN, float>(m.xdgf, m.cdgf, (float)xi[0], l1);
  lagrange<NN, float>(m.xdgf, m.cdgf, (float)xi[1], l2);
  constexpr int N3 = NN * NN * NN;
  float acc[kInterpVars] = {};
#pragma unroll 1
  for (int k = 0; k < NN; ++k) {
    float l3 = lagrange1<NN, float>(m.xdgf, m.cdgf, (float)xi[2], k);
#pragma unroll
    for (int var = 0; var < kInterpVars; ++var) {
      const UT* Uk = U + var * N3 + k * NN * NN;
      float sk = 0.0f;
#pragma unroll
      for (int j = 0; j < NN; ++j) {
        float sj = 0.0f;
#pragma unroll
        for (int i = 0; i < NN; ++i) sj += (float)Uk[j * NN + i] * l1[i];
        sk += sj * l2[j];
      }
      acc[var] += sk * l3;
    }
  }
#pragma unroll
  for (int var = 0; var < kInterpVars; ++var) out[var] = acc[var];
}

// drag acceleration f_D (u - v)/tau_p (Sec. 2.2.1); fD returned for the source
template <typename T>
__device__ __forceinline__ void drag_accel(int drag, T rho, const T* u, const T* v, T d, T mu, T rho_p, T* a, T& fD) {
  T w0 = u[0] - v[0], w1 = u[1] - v[1], w2 = u[2] - v[2];
  fD = T(1);
  if (drag == 1) {
    T Re = rho * sqrt(w0 * w0 + w1 * w1 + w2 * w2) * d / mu;
    fD = (Re < T(800)) ? T(1) + T(0.15) * pow(Re, T(0.687)) : T(0.44) * Re / T(24);
  }
  if (drag == 2) {
    fD = T(0);
    a[0] = a[1] = a[2] = T(0);
    return;
  }
  T itau = T(18) * mu / (rho_p * d * d);
  a[0] = fD * w0 * itau;
  a[1] = fD * w1 * itau;
  a[2] = fD * w2 * itau;
}

// ---------------------------------------------------------------------------
// extra terms of the equation of motion (eq. theory:maxey): buoyancy, the
// undisturbed-flow stress m_f Du/Dt, added mass and Saffman lift
// ---------------------------------------------------------------------------
template <int N, typename T>
__device__ __forceinline__ void lagrange_dt(const T* nodes, const T* cden, T x, T* l, T* dl) {
  T dx[N];
#pragma unroll
  for (int j = 0; j < N; ++j) dx[j] = x - nodes[j];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T p = T(1), dp = T(0);
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j != i) {
        dp = dp * dx[j] + p;
        p *= dx[j];
      }
    l[i] = cden[i] * p;
    dl[i] = cden[i] * dp;
  }
}

// density and momentum (eq. part_interpolation) and their derivatives along
// xi_1, xi_2, xi_3, by sum factorisation in precision T
template <int NN, typename T, typename UT>
__device__ void interp_grad(const T* xdg, const T* cdg, const UT* __restrict__ U, const double* xi, T* val,
                            T (*dval)[3]) {
  T l1[NN], d1[NN], l2[NN], d2[NN], l3[NN], d3[NN];
  lagrange_dt<NN, T>(xdg, cdg, (T)xi[0], l1, d1);
  lagrange_dt<NN, T>(xdg, cdg, (T)xi[1], l2, d2);
  lagrange_dt<NN, T>(xdg, cdg, (T)xi[2], l3, d3);
  constexpr int N3 = NN * NN * NN;
#pragma unroll 1
  for (int var = 0; var < kInterpVars; ++var) {
    T s = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 1
    for (int k = 0; k < NN; ++k) {
      const UT* Uk = U + var * N3 + k * NN * NN;
      T a = 0, b = 0, c = 0;
#pragma unroll
      for (int j = 0; j < NN; ++j) {
        T p = 0, q = 0;
#pragma unroll
        for (int i = 0; i < NN; ++i) {
          const T u = (T)Uk[j * NN + i];
          p += u * l1[i];
          q += u * d1[i];
        }
        a += p * l2[j];
        b += q * l2[j];
        c += p * d2[j];
      }
      s += a * l3[k];
      s1 += b * l3[k];
      s2 += c * l3[k];
      s3 += a * d3[k];
    }
    val[var] = s;
    dval[var][0] = s1;
    dval[var][1] = s2;
    dval[var][2] = s3;
  }
}

// velocity u = m / rho and its physical gradient G[i][j] = du_i/dx_j:
// df/dx_j = sum_d df/dxi_d (J^-1)_dj, du_i = (dm_i - u_i drho) / rho
template <typename T>
__device__ void velocity_gradient(const double J[3][3], const T* val, const T (*dval)[3], T* u, T (*G)[3]) {
  double Ji[3][3];
  Ji[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  Ji[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  Ji[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  Ji[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  Ji[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  Ji[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  Ji[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  Ji[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  Ji[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double idet = 1.0 / (J[0][0] * Ji[0][0] + J[0][1] * Ji[1][0] + J[0][2] * Ji[2][0]);
  T gx[kInterpVars][3];
#pragma unroll
  for (int var = 0; var < kInterpVars; ++var)
#pragma unroll
    for (int jx = 0; jx < 3; ++jx)
      gx[var][jx] = dval[var][0] * (T)(Ji[0][jx] * idet) + dval[var][1] * (T)(Ji[1][jx] * idet) +
                    dval[var][2] * (T)(Ji[2][jx] * idet);
  const T ir = T(1) / val[0];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u[i] = val[1 + i] * ir;
#pragma unroll
    for (int jx = 0; jx < 3; ++jx) G[i][jx] = (gx[1 + i][jx] - u[i] * gx[0][jx]) * ir;
  }
}

// dv/dt from m_p dv/dt = F_D + m_f Du/Dt + m_f/2 (Du/Dt - dv/dt) + F_L
// + g (m_p - m_f) with the terms selected in `forces` (m_f = rho pi d^3/6,
// r = rho / rho_p).  The fluid state is frozen over a step, so
// Du/Dt = (u . grad) u.  Without kForceBuoyancy the body force is g m_p; with
// kForceAddedMass the dv/dt term moves to the left, (1 + r/2) dv/dt = ....
// Saffman lift (Sec. 2.2.2): 6.46/4 C_S d^2 sqrt(rho mu / |w|) (u - v) x w
// (w the vorticity; the direction that lifts a particle lagging a shear flow
// towards the faster fluid), Mei's C_S = (1 - 0.3314 sqrt(th)) exp(-Re/10)
// + 0.3314 sqrt(th) for Re <= 40 and 0.0524 sqrt(th Re) above, with
// th = d |w| / (2 |u - v|) limited to [0.005, 0.4].  F (may be null): the fluid
// force of the two-way source (eq. theory:source), F_D + m_f Du/Dt
// + m_f/2 (Du/Dt - dv/dt) + F_L.
template <typename T>
__device__ void particle_accel(int drag, int forces, T rho, const T* u, const T (*G)[3], const T* v, T d, T mu,
                               T rho_p, const double* g, T* a, T* F) {
  T aD[3], fD;
  drag_accel<T>(drag, rho, u, v, d, mu, rho_p, aD, fD);
  const T w[3] = {u[0] - v[0], u[1] - v[1], u[2] - v[2]};
  const T r = rho / rho_p;
  const T mp = rho_p * T(M_PI) * d * d * d / T(6);
  T DuDt[3] = {0, 0, 0}, aL[3] = {0, 0, 0};
  if (forces & (kForceStress | kForceAddedMass))
#pragma unroll
    for (int i = 0; i < 3; ++i) DuDt[i] = G[i][0] * u[0] + G[i][1] * u[1] + G[i][2] * u[2];
  if (forces & kForceSaffman) {
    const T om[3] = {G[2][1] - G[1][2], G[0][2] - G[2][0], G[1][0] - G[0][1]};
    const T wo = sqrt(om[0] * om[0] + om[1] * om[1] + om[2] * om[2]);
    const T ww = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (wo > T(0) && ww > T(0)) {
      const T Re = rho * ww * d / mu;
      const T th = fmin(fmax(d * wo / (T(2) * ww), T(0.005)), T(0.4));
      const T CS = (Re <= T(40)) ? (T(1) - T(0.3314) * sqrt(th)) * exp(T(-0.1) * Re) + T(0.3314) * sqrt(th)
                                 : T(0.0524) * sqrt(th * Re);
      const T coef = T(6.46) / T(4) * CS * d * d * sqrt(rho * mu / wo) / mp;
      aL[0] = coef * (w[1] * om[2] - w[2] * om[1]);
      aL[1] = coef * (w[2] * om[0] - w[0] * om[2]);
      aL[2] = coef * (w[0] * om[1] - w[1] * om[0]);
    }
  }
  const T cs = ((forces & kForceStress) ? T(1) : T(0)) + ((forces & kForceAddedMass) ? T(0.5) : T(0));
  const T den = (forces & kForceAddedMass) ? T(1) + T(0.5) * r : T(1);
  const T gb = (forces & kForceBuoyancy) ? T(1) - r : T(1);
#pragma unroll
  for (int q = 0; q < 3; ++q) a[q] = (aD[q] + cs * r * DuDt[q] + aL[q] + gb * (T)g[q]) / den;
  if (F) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      T f = aL[q];
      if (forces & kForceStress) f += r * DuDt[q];
      if (forces & kForceAddedMass) f += T(0.5) * r * (DuDt[q] - a[q]);
      F[q] = T(3) * T(M_PI) * mu * d * fD * w[q] + mp * f;
    }
  }
}

// fluid force on a particle at xi in element e for the two-way source
// (eq. theory:source): drag F_D = 3 pi mu d f_D (u - v) (eq. dragforce), plus
// the extra terms of fm.forces (FP64 throughout)
template <int NN, int NG, typename UT>
__device__ void source_force(const MeshView& m, const Fluid& fl, const ForceModel& fm, int e, const double* xi,
                             const double* v, double d, double* F) {
  constexpr int N3 = NN * NN * NN;
  const UT* Ue = (const UT*)fl.U + (size_t)e * 5 * N3;
  if (fm.forces) {
    double val[kInterpVars], dval[kInterpVars][3], u[3], G[3][3], J[3][3], xm[3], a[3];
    interp_grad<NN, double, UT>(m.xdg, m.cdg, Ue, xi, val, dval);
    map_jac<NG>(m, m.X + (size_t)e * NG * NG * NG * 3, xi, xm, J);
    velocity_gradient<double>(J, val, dval, u, G);
    particle_accel<double>(fm.drag, fm.forces, val[0], u, G, v, d, fl.mu, fl.rho_p, fm.gravity, a, F);
  } else {
    double Uc[kInterpVars];
    interp<NN, UT>(m, Ue, xi, Uc);
    double ir = 1.0 / Uc[0];
    double u[3] = {Uc[1] * ir, Uc[2] * ir, Uc[3] * ir};
    double a[3], fD;
    drag_accel<double>(fm.drag, Uc[0], u, v, d, fl.mu, fl.rho_p, a, fD);
    double c = 3.0 * M_PI * fl.mu * d * fD;
    F[0] = c * (u[0] - v[0]);
    F[1] = c * (u[1] - v[1]);
    F[2] = c * (u[2] - v[2]);
  }
}

// ---------------------------------------------------------------------------
// face intersection (Sec. 3.2.4)
// ---------------------------------------------------------------------------
// Bezier control points of local face f of an element (Lagrange geometry
// nodes Xe -> Bernstein form, P = M^-1 F M^-T with Mi = M^-1 row-major), its
// oriented bounding box, corner bilinear coefficients and type (Sec. 3.2.4).
// Neighbour, boundary and shift fields are left to the caller.
template <int NG>
__device__ inline void face_setup(const double* __restrict__ Xe, int f, const double* __restrict__ Mi, double* cp,
                                  FaceRec& F) {
  constexpr int D = NG - 1;
  int d = f / 2, a = (d == 0) ? 1 : 0, b = (d == 2) ? 1 : 2;
  int fix = (f & 1) ? D : 0;
  double T[NG * NG][3];
  for (int n = 0; n < NG; ++n)
    for (int mm = 0; mm < NG; ++mm) {
      double s[3] = {0, 0, 0};
      for (int r = 0; r < NG; ++r) {
        int idx[3];
        idx[d] = fix; idx[a] = r; idx[b] = n;
        const double* P = Xe + ((idx[2] * NG + idx[1]) * NG + idx[0]) * 3;
        double w = Mi[mm * NG + r];
        s[0] += w * P[0]; s[1] += w * P[1]; s[2] += w * P[2];
      }
      T[n * NG + mm][0] = s[0]; T[n * NG + mm][1] = s[1]; T[n * NG + mm][2] = s[2];
    }
  for (int n = 0; n < NG; ++n)
    for (int mm = 0; mm < NG; ++mm) {
      double s[3] = {0, 0, 0};
      for (int r = 0; r < NG; ++r) {
        double w = Mi[n * NG + r];
        s[0] += w * T[r * NG + mm][0]; s[1] += w * T[r * NG + mm][1]; s[2] += w * T[r * NG + mm][2];
      }
      cp[(n * NG + mm) * 3 + 0] = s[0]; cp[(n * NG + mm) * 3 + 1] = s[1]; cp[(n * NG + mm) * 3 + 2] = s[2];
    }
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
}

// Local faces that a segment of squared length L2 starting at reference
// point xi of element e could reach (bit f; face f lies at xi_{f/2} = -1 for
// even f, +1 for odd f): along a path inside the element xi_i changes by at
// most gxi[e][i] per unit length, so face f is out of reach when that times
// L stays below its reference distance.  A segment that reaches no face stays
// inside and crosses nothing.
__device__ __forceinline__ unsigned reachable_faces(const MeshView& m, int e, const double* xi, double L2) {
  const double* g = m.gxi + (size_t)e * 6;
  unsigned mask = 0u;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double gl2 = L2 * g[i] * g[i];
    const double rm = 1.0 + xi[i], rp = 1.0 - xi[i];
    if (!(rm > 0.0 && gl2 < rm * rm)) mask |= 1u << (2 * i);
    if (!(rp > 0.0 && gl2 < rp * rp)) mask |= 1u << (2 * i + 1);
  }
  return mask;
}

// Refinement of reachable_faces for a segment x -> xe from reference point xi
// (x = chi_e(xi)): along the segment, while inside the element, xi_i moves by
// at most s (grad xi_i(x) . t) + s^2 H_i / 2 after a length s, where H_i
// bounds the Hessian of xi_i over the element (gxi[e][3 + i]); the bound is
// convex in s, so face (i, +1) is out of reach when it stays below 1 - xi_i at
// s = L (face (i, -1) likewise with the sign of the first term reversed).
// grad xi_i(x) is row i of J^-1 at xi.  The 1e-9 slack covers xi being
// Newton's solution (to 1e-10) rather than the exact preimage of x.
template <int NG>
__device__ __forceinline__ unsigned reachable_faces_taylor(const MeshView& m, int e, const double* __restrict__ Xe,
                                                           const double* xi, const double* x, const double* xe,
                                                           double L2, unsigned reach) {
  double xm[3], J[3][3];
  map_jac<NG>(m, Xe, xi, xm, J);
  const double dj = det3(J);
  if (!(dj > 0.0)) return reach;
  const double d[3] = {xe[0] - x[0], xe[1] - x[1], xe[2] - x[2]};
  // rows of the adjugate dotted with d, over det: first-order change of xi_i
  double a[3];
  a[0] = ((J[1][1] * J[2][2] - J[1][2] * J[2][1]) * d[0] + (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * d[1] +
          (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * d[2]) / dj;
  a[1] = ((J[1][2] * J[2][0] - J[1][0] * J[2][2]) * d[0] + (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * d[1] +
          (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * d[2]) / dj;
  a[2] = ((J[1][0] * J[2][1] - J[1][1] * J[2][0]) * d[0] + (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * d[1] +
          (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * d[2]) / dj;
  const double* h = m.gxi + (size_t)e * 6 + 3;
  unsigned out = 0u;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double q = 0.5 * L2 * h[i] + 1e-9;
    if (-a[i] + q >= 1.0 + xi[i]) out |= 1u << (2 * i);
    if (a[i] + q >= 1.0 - xi[i]) out |= 1u << (2 * i + 1);
  }
  return reach & out;
}

__device__ inline bool bbox_hit(const FaceRec& F, const double* xs, const double* xe) {
  double pad = 1e-9 * F.diam;
  double r0[3] = {xs[0] - F.org[0], xs[1] - F.org[1], xs[2] - F.org[2]};
  double r1[3] = {xe[0] - F.org[0], xe[1] - F.org[1], xe[2] - F.org[2]};
  const double* ax[3] = {F.nrm, F.e1, F.e2};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double p0 = dot3(r0, ax[a]), p1 = dot3(r1, ax[a]);
    if (fmax(p0, p1) < F.lo[a] - pad || fmin(p0, p1) > F.hi[a] + pad) return false;
  }
  return true;
}

__device__ inline void ray_planes(const double* t, double* n1, double* n2) {
  int k = 0;
  if (fabs(t[1]) < fabs(t[k])) k = 1;
  if (fabs(t[2]) < fabs(t[k])) k = 2;
  double ek[3] = {0, 0, 0};
  ek[k] = 1.0;
  cross3(t, ek, n1);
  double il = 1.0 / sqrt(dot3(n1, n1));
  n1[0] *= il; n1[1] *= il; n1[2] *= il;
  cross3(n1, t, n2);
}

__device__ inline int planar_hit(const FaceRec& F, const double* x0, const double* t, double* al, double* uv) {
  double nrm[3];
  cross3(F.B, F.C, nrm);
  double tn = dot3(t, nrm);
  if (tn == 0.0) return 0;
  double r[3] = {F.D[0] - x0[0], F.D[1] - x0[1], F.D[2] - x0[2]};
  double a = dot3(r, nrm) / tn;
  double h[3] = {x0[0] + a * t[0] - F.D[0], x0[1] + a * t[1] - F.D[1], x0[2] + a * t[2] - F.D[2]};
  double bb = dot3(F.B, F.B), bc = dot3(F.B, F.C), cc = dot3(F.C, F.C);
  double rb = dot3(h, F.B), rc = dot3(h, F.C);
  double det = bb * cc - bc * bc;
  al[0] = a;
  uv[0] = (rb * cc - rc * bc) / det;
  uv[1] = (bb * rc - bc * rb) / det;
  return 1;
}

__device__ inline int bilinear_hit(const FaceRec& F, const double* x0, const double* t, double* al, double* uv) {
  double n1[3], n2[3];
  ray_planes(t, n1, n2);
  double Dr[3] = {F.D[0] - x0[0], F.D[1] - x0[1], F.D[2] - x0[2]};
  double a1 = dot3(F.A, n1), b1 = dot3(F.B, n1), c1 = dot3(F.C, n1), d1 = dot3(Dr, n1);
  double a2 = dot3(F.A, n2), b2 = dot3(F.B, n2), c2 = dot3(F.C, n2), d2 = dot3(Dr, n2);
  double qa = a1 * c2 - a2 * c1;
  double qb = a1 * d2 + b1 * c2 - a2 * d1 - b2 * c1;
  double qc = b1 * d2 - b2 * d1;
  double scale = fmax(fabs(qa), fmax(fabs(qb), fabs(qc)));
  if (scale == 0.0) return 0;
  double vs[2];
  int nv = 0;
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
    double den1 = a1 * v + b1, den2 = a2 * v + b2, u;
    if (fabs(den1) >= fabs(den2)) {
      if (den1 == 0.0) continue;
      u = -(c1 * v + d1) / den1;
    } else {
      u = -(c2 * v + d2) / den2;
    }
    double p[3];
    for (int q = 0; q < 3; ++q) p[q] = F.A[q] * u * v + F.B[q] * u + F.C[q] * v + F.D[q] - x0[q];
    al[nr] = dot3(p, t);
    uv[2 * nr] = u;
    uv[2 * nr + 1] = v;
    nr++;
  }
  return nr;
}

// Bernstein basis of degree D at t in [0,1] and its t-derivative
template <int D>
__device__ __forceinline__ void bern(double t, double* B, double* dB) {
  double tp[D + 1], sp[D + 1];
  tp[0] = 1.0; sp[0] = 1.0;
  double s = 1.0 - t;
#pragma unroll
  for (int m = 1; m <= D; ++m) { tp[m] = tp[m - 1] * t; sp[m] = sp[m - 1] * s; }
  double c = 1.0;
#pragma unroll
  for (int m = 0; m <= D; ++m) {
    B[m] = c * tp[m] * sp[D - m];
    c = c * (D - m) / (m + 1);
  }
  if (dB) {
    // d/dt B_m^D = D (B_{m-1}^{D-1} - B_m^{D-1})
    double cb = 1.0, lower[D + 1];
#pragma unroll
    for (int m = 0; m < D; ++m) {
      lower[m] = cb * tp[m] * sp[D - 1 - m];
      cb = cb * (D - 1 - m) / (m + 1);
    }
#pragma unroll
    for (int m = 0; m <= D; ++m) {
      double lo = (m >= 1) ? lower[m - 1] : 0.0;
      double hi = (m <= D - 1) ? lower[m] : 0.0;
      dB[m] = D * (lo - hi);
    }
  }
}

template <int NG>
__device__ inline void bezier_eval(const double* __restrict__ cp, double u, double v, double* p, double* pu,
                                   double* pv) {
  constexpr int D = NG - 1;
  double Bu[NG], Bv[NG], dBu[NG], dBv[NG];
  bern<D>(0.5 * (u + 1.0), Bu, dBu);
  bern<D>(0.5 * (v + 1.0), Bv, dBv);
  for (int q = 0; q < 3; ++q) { p[q] = 0.0; if (pu) { pu[q] = 0.0; pv[q] = 0.0; } }
#pragma unroll 1
  for (int k = 0; k < NG; ++k)
#pragma unroll 1
    for (int mm = 0; mm < NG; ++mm) {
      const double* P = cp + (k * NG + mm) * 3;
      double w = Bu[mm] * Bv[k];
      for (int q = 0; q < 3; ++q) {
        p[q] += P[q] * w;
        if (pu) {
          pu[q] += P[q] * 0.5 * dBu[mm] * Bv[k];
          pv[q] += P[q] * 0.5 * Bu[mm] * dBv[k];
        }
      }
    }
}

// restrict a stride-s list of NG Bezier coefficients to [a, b]
template <int NG>
__device__ inline void restrict1(double* c, int s, double a, double b) {
  double tmp[NG], left[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) tmp[i] = c[i * s];
  left[0] = tmp[0];
#pragma unroll
  for (int r = 1; r < NG; ++r) {
#pragma unroll
    for (int i = 0; i < NG - r; ++i) tmp[i] = (1.0 - b) * tmp[i] + b * tmp[i + 1];
    left[r] = tmp[0];
  }
  if (b <= 0.0) {
#pragma unroll
    for (int i = 0; i < NG; ++i) c[i * s] = left[0];
    return;
  }
  double t = a / b;
#pragma unroll
  for (int i = 0; i < NG; ++i) tmp[i] = left[i];
  c[(NG - 1) * s] = tmp[NG - 1];
#pragma unroll
  for (int r = 1; r < NG; ++r) {
#pragma unroll
    for (int i = 0; i < NG - r; ++i) tmp[i] = (1.0 - t) * tmp[i] + t * tmp[i + 1];
    c[(NG - 1 - r) * s] = tmp[NG - 1 - r];
  }
}

// q[m][k][C] with m along u, k along v; restrict direction dir to [a, b]
template <int NG, int C>
__device__ inline void patch_restrict(double* q, int dir, double a, double b) {
#pragma unroll
  for (int k = 0; k < NG; ++k)
#pragma unroll
    for (int co = 0; co < C; ++co) {
      if (dir == 0) restrict1<NG>(q + k * C + co, NG * C, a, b);   // along m
      else restrict1<NG>(q + k * NG * C + co, C, a, b);            // along k
    }
}

// t-extent of H intersected with {y >= c} (ge) or {y <= c}, where H is the
// convex hull of the columns t_i = i/(NP-1), y in [lo_i, hi_i].  Only the
// column maxima (ge) or minima bound that intersection; its extent is spanned
// by the columns inside the half-plane and by the crossings of y = c on the
// segments between a column inside and a column outside (every such crossing
// lies in H, and the hull edge that leaves the half-plane is one of them).
template <int NP>
__device__ __forceinline__ bool half_extent(const double* lo, const double* hi, double c, bool ge, double& a,
                                            double& b) {
  const double* y = ge ? hi : lo;
  const double step = 1.0 / (NP - 1);
  double tmin = 1e300, tmax = -1e300;
  bool in[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    in[i] = ge ? (y[i] >= c) : (y[i] <= c);
    if (in[i]) { tmin = fmin(tmin, i * step); tmax = fmax(tmax, i * step); }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int j = i + 1; j < NP; ++j)
      if (in[i] != in[j]) {
        double t = (i + (j - i) * ((c - y[i]) / (y[j] - y[i]))) * step;
        tmin = fmin(tmin, t);
        tmax = fmax(tmax, t);
      }
  a = tmin;
  b = tmax;
  return tmin <= tmax;
}

// Clip direction dir (0: u, 1: v) of the projected patch q[m][k][3] (signed
// distances to the two planes that contain the ray in components 0 and 1):
// Bezier clipping against the line through the origin that runs along the
// other parameter direction.  The convex-hull property of the Bernstein form
// keeps every root.
template <int NG>
__device__ inline bool clip_dir(const double* q, int dir, double amin, double amax, double& a, double& b) {
  constexpr int N = NG - 1;
#define QQ(m, k, c) q[((m) * NG + (k)) * 3 + (c)]
  double L0, L1;
  if (dir == 0) {
    L0 = (QQ(0, N, 0) - QQ(0, 0, 0)) + (QQ(N, N, 0) - QQ(N, 0, 0));
    L1 = (QQ(0, N, 1) - QQ(0, 0, 1)) + (QQ(N, N, 1) - QQ(N, 0, 1));
  } else {
    L0 = (QQ(N, 0, 0) - QQ(0, 0, 0)) + (QQ(N, N, 0) - QQ(0, N, 0));
    L1 = (QQ(N, 0, 1) - QQ(0, 0, 1)) + (QQ(N, N, 1) - QQ(0, N, 1));
  }
  double ll = sqrt(L0 * L0 + L1 * L1);
  if (ll == 0.0) {
    double K0, K1;
    if (dir == 0) {
      K0 = (QQ(N, 0, 0) - QQ(0, 0, 0)) + (QQ(N, N, 0) - QQ(0, N, 0));
      K1 = (QQ(N, 0, 1) - QQ(0, 0, 1)) + (QQ(N, N, 1) - QQ(0, N, 1));
    } else {
      K0 = (QQ(0, N, 0) - QQ(0, 0, 0)) + (QQ(N, N, 0) - QQ(N, 0, 0));
      K1 = (QQ(0, N, 1) - QQ(0, 0, 1)) + (QQ(N, N, 1) - QQ(N, 0, 1));
    }
    L0 = -K1; L1 = K0;
    ll = sqrt(L0 * L0 + L1 * L1);
    if (ll == 0.0) { L0 = 1.0; L1 = 0.0; ll = 1.0; }
  }
  double nx = -L1 / ll, ny = L0 / ll;
  double dlo[NG], dhi[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    double mn = 1e300, mx = -1e300;
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      double dist = (dir == 0) ? nx * QQ(i, k, 0) + ny * QQ(i, k, 1) : nx * QQ(k, i, 0) + ny * QQ(k, i, 1);
      mn = fmin(mn, dist);
      mx = fmax(mx, dist);
    }
    dlo[i] = mn;
    dhi[i] = mx;
  }
#undef QQ
  double a1, b1, a2, b2;
  if (!half_extent<NG>(dlo, dhi, 0.0, true, a1, b1)) return false;
  if (!half_extent<NG>(dlo, dhi, 0.0, false, a2, b2)) return false;
  double lo = fmax(a1, a2), hi = fmin(b1, b2);
  if (lo > hi) return false;
  // the displacement band amin <= alpha <= amax (component 2), on the same
  // convex hull of the rows' ranges
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    double mn = 1e300, mx = -1e300;
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      double al = (dir == 0) ? q[(i * NG + k) * 3 + 2] : q[(k * NG + i) * 3 + 2];
      mn = fmin(mn, al);
      mx = fmax(mx, al);
    }
    dlo[i] = mn;
    dhi[i] = mx;
  }
  if (!half_extent<NG>(dlo, dhi, amin, true, a1, b1)) return false;
  if (!half_extent<NG>(dlo, dhi, amax, false, a2, b2)) return false;
  lo = fmax(lo, fmax(a1, a2));
  hi = fmin(hi, fmin(b1, b2));
  if (lo > hi) return false;
  a = fmax(0.0, lo - kClipPad);
  b = fmin(1.0, hi + kClipPad);
  return true;
}

// projected control points of the whole face: distances to the planes n1, n2
// (components 0, 1) and displacement along t (component 2), [m along u][k along v]
template <int NG>
__device__ __forceinline__ void project_face(const double* __restrict__ cp, const double* x0, const double* t,
                                             const double* n1, const double* n2, double* q) {
#pragma unroll
  for (int k = 0; k < NG; ++k)
#pragma unroll
    for (int mm = 0; mm < NG; ++mm) {
      const double* P = cp + (k * NG + mm) * 3;
      double r[3] = {P[0] - x0[0], P[1] - x0[1], P[2] - x0[2]};
      q[(mm * NG + k) * 3 + 0] = dot3(r, n1);
      q[(mm * NG + k) * 3 + 1] = dot3(r, n2);
      q[(mm * NG + k) * 3 + 2] = dot3(r, t);
    }
}

// the displacement of every point of the (sub-)patch lies outside [amin, amax]
template <int NG>
__device__ __forceinline__ bool outside_band(const double* q, double amin, double amax) {
  double lo = 1e300, hi = -1e300;
#pragma unroll
  for (int i = 0; i < NG * NG; ++i) {
    lo = fmin(lo, q[i * 3 + 2]);
    hi = fmax(hi, q[i * 3 + 2]);
  }
  return hi < amin || lo > amax;
}

// Physical-space tracking of the queued straight stage segments xs -> xe
// (Sec. 3.2.3): smallest alpha in (1e-12 h_e, remaining length] with (u, v) in
// [-1,1]^2, ties to the lowest local face; hand-off, periodic shift, specular
// reflection (Sec. 2.4) of the remaining displacement, v and the stage
// registers; open boundaries end the particle.
//
// Written as a per-lane state machine: one loop iteration advances a lane by
// one step of its own work (next candidate face, pop of a clipping box, one
// Bezier-clipping iteration, end of a leg), so the lanes of a wavefront that
// test different faces, need different iteration counts or cross different
// numbers of faces all share the clipping iteration that dominates the cost.
// A lane whose segment is done takes the next one from the queue (one atomic
// per wavefront and iteration for all its idle lanes), so the lanes stay busy
// until the queue is drained instead of each wavefront waiting for its
// slowest segment.  The results do not depend on the order.
__device__ __forceinline__ int lane_rank64(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

template <int NG, bool MORT>
__device__ void track_queue(const MeshView& m, const Particles& P, const int32_t* __restrict__ trk_p,
                            const double* __restrict__ trk_x, const uint8_t* __restrict__ trk_m, int32_t* head,
                            int64_t nq, int max_cross, int& ncross, int& nhits) {
  constexpr double kBoxTol = 1e-7;
  // Bezier clipping contracts a box around a simple root quadratically; once
  // both sides are below kNewtonBox and the last iteration cut each of them to
  // at most kQuadRatio, the box holds one transversal root and the 2-D Newton
  // below reaches it in three steps (a double root, where the clipping only
  // contracts linearly, keeps clipping down to kBoxTol)
  constexpr double kNewtonBox = 1e-3, kQuadRatio = 0.25;
  enum { NEW_LEG, NEXT_FACE, POP, CLIP, LEG_END, MORT_FACE, MORT_END, DONE };
  // idle lanes take new segments once at least kRefill of them wait (one
  // atomic on the queue head and one pass of the refill code per batch):
  // measured per-stage tracking, degree 4 with 1.1e6 segments 6.6 -> 5.2 ms
  // at 32 (8: 6.3, 16: 5.6), degree 6 with 1.3e6 segments 23.7 -> 22.7 ms at
  // 8 (16: 22.9, 32: 23.8); a queue of 4e4 segments loses 0.01 ms at either
  constexpr int kRefill = NG >= 7 ? 8 : 32;
  const int64_t cap = P.cap;
  // the lane's segment: particle, element at the start, wall hits, crossings
  int64_t p = -1;
  int e = 0, e0 = 0, hits = 0, nseg = 0;
  int8_t status = ACTIVE;
  unsigned reach = 0x3Fu;
  double xe[3] = {0, 0, 0}, v[3] = {0, 0, 0}, kx[3] = {0, 0, 0}, kv[3] = {0, 0, 0};
  double xs[3] = {0, 0, 0};
  // excl: planar face just entered through (no further root possible);
  // entry: non-planar face just entered through, whose root at the entry point
  // (alpha ~ 0, error growing like 1/sin(incidence)) is ignored below
  // kEntryRel * face diameter
  int excl = -1, entry = -1, count = 0;
  double t[3] = {0, 0, 0}, n1[3] = {0, 0, 0}, n2[3] = {0, 0, 0}, L = 0.0, eps = 0.0;
  double best = 1e300, bu = 0.0, bv = 0.0, amin = 0.0, bmin = 0.0, bmax = 0.0;
  int bf = -1, f = 0;
  int fl = 0;   // local index of the face under test (its outward-normal sign)
  // non-conforming side: mortar index, cursor over its small faces, the
  // big-face crossing and the small-face root nearest it
  int mort = -1, mj = 0, mbig = -1, ms = -1, mf = -1, mse = -1, msf = -1;
  double astar = 0.0, mbd = 1e300, msa = 0.0;
  const double* cpf = m.cp;
  double stk[kClipStack][4];
  int sp = 0, budget = 0;
  double u0 = 0.0, u1 = 1.0, v0 = 0.0, v1 = 1.0;
  double q[NG * NG * 3];
  // a root counts if it lies in (amin, L], on the face, and the path leaves
  // the element there: tn = t . outward normal > 0 (a root where the path
  // enters, at a tangential touch or the entry point, is not a crossing)
  auto consider = [&](double a, double uu, double vv, double tn) {
    if (fabs(uu) > 1.0 + kUVEps || fabs(vv) > 1.0 + kUVEps) return;
    if (MORT && mort >= 0) {
      // small face of a mortar: a root where the path enters the small element
      // (where the inverted path leaves it), the one nearest the big-face crossing
      if (!(a >= bmin && a <= bmax) || !(tn < 0.0)) return;
      const double dd = fabs(a - astar);
      if (dd < mbd) { mbd = dd; msa = a; mse = ms; msf = mf; }
      return;
    }
    if (!(a > amin && a <= L)) return;
    if (!(tn > 0.0)) return;
    if (a < best) { best = a; bf = f; bu = uu; bv = vv; }
  };
  int mode = DONE;
  bool drained = false;   // wave-uniform: the queue has no segment left
  const int lane = threadIdx.x & 63;
#pragma unroll 1
  while (true) {
    if (!drained) {
      const unsigned long long idle = __ballot(mode == DONE);
      if (idle && (__popcll(idle) >= kRefill || __popcll(idle) == 64)) {
        const int nidle = __popcll(idle);
        const int leader = __ffsll((long long)idle) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(head, nidle);
        base = __shfl(base, leader, 64);
        if ((int64_t)base + nidle >= nq) drained = true;
        if (mode == DONE) {
          const int64_t i = (int64_t)base + lane_rank64(idle);
          if (i < nq) {
            p = trk_p[i];
            xs[0] = trk_x[i]; xs[1] = trk_x[cap + i]; xs[2] = trk_x[2 * cap + i];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              xe[k] = P.x[k * cap + p];
              v[k] = P.v[k * cap + p];
              kx[k] = P.kx[k * cap + p];
              kv[k] = P.kv[k * cap + p];
            }
            e = e0 = P.elem[p];
            hits = nseg = 0;
            status = ACTIVE;
            reach = trk_m[i];
            excl = entry = -1;
            count = 0;
            mort = -1;
            mode = NEW_LEG;
          }
        }
      }
    }
    if (__ballot(mode != DONE) == 0ull) break;
    if (mode == NEW_LEG) {
      t[0] = xe[0] - xs[0]; t[1] = xe[1] - xs[1]; t[2] = xe[2] - xs[2];
      L = sqrt(dot3(t, t));
      if (L == 0.0) {
        mode = DONE;
      } else {
        double iL = 1.0 / L;
        t[0] *= iL; t[1] *= iL; t[2] *= iL;
        ray_planes(t, n1, n2);
        eps = 1e-12 * m.hE[e];
        best = 1e300;
        bf = -1;
        f = 0;
        mode = NEXT_FACE;
      }
    }
    if (mode == NEXT_FACE) {
      // reach: the faces the first leg can reach (all of them on later legs)
      while (f < 6 && (f == excl || !((reach >> f) & 1u) || !bbox_hit(m.faces[e * 6 + f], xs, xe))) f++;
      if (f == 6) {
        mode = LEG_END;
      } else {
        const FaceRec& F = m.faces[e * 6 + f];
        fl = f;
        amin = (f == entry) ? fmax(eps, kEntryRel * F.diam) : eps;
        if (F.type != FACE_CURVED) {
          double al[2], uv[4];
          int nr = (F.type == FACE_PLANAR) ? planar_hit(F, xs, t, al, uv) : bilinear_hit(F, xs, t, al, uv);
          for (int r = 0; r < nr; ++r) {
            double pu[3], pv[3], nrm[3];
            for (int k = 0; k < 3; ++k) {
              pu[k] = F.A[k] * uv[2 * r + 1] + F.B[k];
              pv[k] = F.A[k] * uv[2 * r] + F.C[k];
            }
            cross3(pu, pv, nrm);
            consider(al[r], uv[2 * r], uv[2 * r + 1], kFaceSign[f] * dot3(nrm, t));
          }
          f++;
        } else {
          // only roots with displacement in (amin, L] matter: clip to a padded band
          const double pad = 1e-9 * F.diam;
          bmin = amin - pad;
          bmax = L + pad;
          cpf = m.cp + (size_t)(e * 6 + f) * (NG * NG * 3);
          stk[0][0] = 0.0; stk[0][1] = 1.0; stk[0][2] = 0.0; stk[0][3] = 1.0;
          sp = 1;
          budget = kClipSteps;
          mode = POP;
        }
      }
    }
    if (MORT && mode == MORT_FACE) {
      // the small faces of the big mortar face just crossed (Sec. 3.2.3)
      while (mj < 4 && (m.mortar[mort * 8 + 2 * mj] < 0 ||
                        !bbox_hit(m.faces[m.mortar[mort * 8 + 2 * mj] * 6 + m.mortar[mort * 8 + 2 * mj + 1]], xs, xe)))
        mj++;
      if (mj == 4) {
        mode = MORT_END;
      } else {
        ms = m.mortar[mort * 8 + 2 * mj];
        mf = m.mortar[mort * 8 + 2 * mj + 1];
        fl = mf;
        const FaceRec& F = m.faces[ms * 6 + mf];
        const double pad = 1e-9 * F.diam;
        bmin = -pad;
        bmax = L + pad;
        if (F.type != FACE_CURVED) {
          double al[2], uv[4];
          int nr = (F.type == FACE_PLANAR) ? planar_hit(F, xs, t, al, uv) : bilinear_hit(F, xs, t, al, uv);
          for (int r = 0; r < nr; ++r) {
            double pu[3], pv[3], nrm[3];
            for (int k = 0; k < 3; ++k) {
              pu[k] = F.A[k] * uv[2 * r + 1] + F.B[k];
              pv[k] = F.A[k] * uv[2 * r] + F.C[k];
            }
            cross3(pu, pv, nrm);
            consider(al[r], uv[2 * r], uv[2 * r + 1], kFaceSign[mf] * dot3(nrm, t));
          }
          mj++;
        } else {
          cpf = m.cp + (size_t)(ms * 6 + mf) * (NG * NG * 3);
          stk[0][0] = 0.0; stk[0][1] = 1.0; stk[0][2] = 0.0; stk[0][3] = 1.0;
          sp = 1;
          budget = kClipSteps;
          mode = POP;
        }
      }
    }
    if (mode == POP) {
      if (sp == 0 || budget <= 0) {
        if (MORT && mort >= 0) {
          mj++;
          mode = MORT_FACE;
        } else {
          f++;
          mode = NEXT_FACE;
        }
      } else {
        --sp;
        u0 = stk[sp][0]; u1 = stk[sp][1]; v0 = stk[sp][2]; v1 = stk[sp][3];
        project_face<NG>(cpf, xs, t, n1, n2, q);
        if (u0 != 0.0 || u1 != 1.0) patch_restrict<NG, 3>(q, 0, u0, u1);
        if (v0 != 0.0 || v1 != 1.0) patch_restrict<NG, 3>(q, 1, v0, v1);
        mode = CLIP;
      }
    }
    if (mode == CLIP) {
      // one Bezier-clipping iteration (Sec. 3.2.4) on the live box
      double a, b;
      mode = POP;
      if (--budget >= 0 && !outside_band<NG>(q, bmin, bmax) && clip_dir<NG>(q, 0, bmin, bmax, a, b)) {
        patch_restrict<NG, 3>(q, 0, a, b);
        double w = u1 - u0;
        double nu0 = u0 + a * w, nu1 = u0 + b * w;
        u0 = nu0; u1 = nu1;
        const double ru = b - a;
        if (clip_dir<NG>(q, 1, bmin, bmax, a, b)) {
          patch_restrict<NG, 3>(q, 1, a, b);
          w = v1 - v0;
          double nv0 = v0 + a * w, nv1 = v0 + b * w;
          v0 = nv0; v1 = nv1;
          const double rv = b - a;
          const double wu = u1 - u0, wv = v1 - v0;
          bool conv = (wu <= kBoxTol && wv <= kBoxTol) ||
                      (wu <= kNewtonBox && wv <= kNewtonBox && ru <= kQuadRatio && rv <= kQuadRatio);
          const bool su = (ru > 0.8 && wu > kBoxTol), sv = (rv > 0.8 && wv > kBoxTol);
          if (!conv && (su || sv) && sp + 2 > kClipStack) conv = true;
          if (conv) {
            // 2-D Newton on the plane distances from the box centre
            double u = (u0 + u1) - 1.0, vv = (v0 + v1) - 1.0;
            double pp[3], pu[3], pv[3];
#pragma unroll 1
            for (int it = 0; it < 3; ++it) {
              bezier_eval<NG>(cpf, u, vv, pp, pu, pv);
              double r[3] = {pp[0] - xs[0], pp[1] - xs[1], pp[2] - xs[2]};
              double G0 = dot3(r, n1), G1 = dot3(r, n2);
              double Gu0 = dot3(pu, n1), Gu1 = dot3(pu, n2), Gv0 = dot3(pv, n1), Gv1 = dot3(pv, n2);
              double det = Gu0 * Gv1 - Gu1 * Gv0;
              if (det == 0.0 || !isfinite(det)) break;
              u += -(G0 * Gv1 - G1 * Gv0) / det;
              vv += -(Gu0 * G1 - Gu1 * G0) / det;
            }
            bezier_eval<NG>(cpf, u, vv, pp, pu, pv);
            double r3[3] = {pp[0] - xs[0], pp[1] - xs[1], pp[2] - xs[2]}, nrm[3];
            cross3(pu, pv, nrm);
            consider(dot3(r3, t), u, vv, kFaceSign[fl] * dot3(nrm, t));
          } else if (su || sv) {
            const int dir = (su && sv) ? (wu >= wv ? 0 : 1) : (su ? 0 : 1);
            if (dir == 0) {
              const double um = 0.5 * (u0 + u1);
              stk[sp][0] = um; stk[sp][1] = u1; stk[sp][2] = v0; stk[sp][3] = v1; sp++;
              stk[sp][0] = u0; stk[sp][1] = um; stk[sp][2] = v0; stk[sp][3] = v1; sp++;
            } else {
              const double vm = 0.5 * (v0 + v1);
              stk[sp][0] = u0; stk[sp][1] = u1; stk[sp][2] = vm; stk[sp][3] = v1; sp++;
              stk[sp][0] = u0; stk[sp][1] = u1; stk[sp][2] = v0; stk[sp][3] = vm; sp++;
            }
          } else {
            mode = CLIP;   // the box shrank: clip it again
          }
        }
      }
    }
    if (mode == LEG_END) {
      if (bf < 0) {
        mode = DONE;
      } else if (count >= max_cross) {
        status = MAX_CROSS;
        mode = DONE;
      } else {
        count++;
        nseg++;
        double xh[3] = {xs[0] + best * t[0], xs[1] + best * t[1], xs[2] + best * t[2]};
        const int fid = e * 6 + bf;
        const FaceRec& F = m.faces[fid];
        const int bc = F.bc;
        mode = NEW_LEG;
        reach = 0x3Fu;
        if (bc == BC_INTERNAL || bc == BC_PERIODIC) {
          const int ne = F.nbr_elem, nf = F.nbr_face;
          if (bc == BC_PERIODIC)
            for (int k = 0; k < 3; ++k) { xh[k] += F.shift[k]; xe[k] += F.shift[k]; }
          e = ne;
          const bool planar = m.faces[ne * 6 + nf].type == FACE_PLANAR;
          excl = planar ? nf : -1;
          entry = planar ? -1 : nf;
          xs[0] = xh[0]; xs[1] = xh[1]; xs[2] = xh[2];
        } else if (MORT && bc == BC_MORTAR) {
          // non-conforming side: find the small face the path enters through
          mort = F.nbr_elem;
          mj = 0;
          mse = -1;
          mbd = 1e300;
          astar = best;
          mbig = bf;
          mode = MORT_FACE;
        } else if (bc == BC_REFLECT) {
          double nrm[3];
          if (F.type == FACE_CURVED) {
            double pp[3], pu[3], pv[3];
            bezier_eval<NG>(m.cp + (size_t)fid * (NG * NG * 3), bu, bv, pp, pu, pv);
            cross3(pu, pv, nrm);
          } else {
            double pu[3], pv[3];
            for (int k = 0; k < 3; ++k) { pu[k] = F.A[k] * bv + F.B[k]; pv[k] = F.A[k] * bu + F.C[k]; }
            cross3(pu, pv, nrm);
          }
          const double il = 1.0 / sqrt(dot3(nrm, nrm));
          nrm[0] *= il; nrm[1] *= il; nrm[2] *= il;
          const double r[3] = {xe[0] - xh[0], xe[1] - xh[1], xe[2] - xh[2]};
          const double dr = dot3(r, nrm), dv = dot3(v, nrm), dkx = dot3(kx, nrm), dkv = dot3(kv, nrm);
          for (int k = 0; k < 3; ++k) {
            xe[k] = xh[k] + (r[k] - 2.0 * dr * nrm[k]);
            v[k] -= 2.0 * dv * nrm[k];
            kx[k] -= 2.0 * dkx * nrm[k];
            kv[k] -= 2.0 * dkv * nrm[k];
          }
          hits++;
          excl = (F.type == FACE_PLANAR) ? bf : -1;
          entry = (F.type == FACE_PLANAR) ? -1 : bf;
          xs[0] = xh[0]; xs[1] = xh[1]; xs[2] = xh[2];
        } else {
          status = OPEN_EXIT;
          xe[0] = xh[0]; xe[1] = xh[1]; xe[2] = xh[2];
          mode = DONE;
        }
      }
    }
    if (MORT && mode == MORT_END) {
      if (mse >= 0) {
        // continue from the small-face crossing in the small element
        e = mse;
        const bool planar = m.faces[mse * 6 + msf].type == FACE_PLANAR;
        excl = planar ? msf : -1;
        entry = planar ? -1 : msf;
        xs[0] += msa * t[0]; xs[1] += msa * t[1]; xs[2] += msa * t[2];
      } else {
        // no small face found (rounding at a seam): the leg ends in the big
        // element and the next location step finds the particle
        xs[0] += astar * t[0]; xs[1] += astar * t[1]; xs[2] += astar * t[2];
        excl = -1;
        entry = mbig;
      }
      mort = -1;
      mode = NEW_LEG;
      reach = 0x3Fu;
    }
    if (mode == DONE && p >= 0) {
      // segment done: write back what changed
      ncross += nseg;
      nhits += hits;
      if (nseg || status != ACTIVE) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          P.x[k * cap + p] = xe[k];
          P.v[k * cap + p] = v[k];
          P.kx[k * cap + p] = kx[k];
          P.kv[k * cap + p] = kv[k];
        }
        if (e != e0) P.elem[p] = e;
        if (hits) P.hits[p] += hits;
        if (status != ACTIVE) P.status[p] = status;
        P.xi[p] = NAN;   // the continued reference coordinates no longer hold
      }
      p = -1;
    }
  }
}

// wave-aggregated queue append: returns the slot of each predicated lane (-1
// otherwise); must be reached by every lane of the wave
__device__ __forceinline__ int wave_push(int32_t* counter, bool pred) {
  unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return -1;
  int lane = threadIdx.x & 63;
  int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, (int)__popcll(mask));
  base = __shfl(base, leader, 64);
  return pred ? base + (int)__popcll(mask & ((1ull << lane) - 1ull)) : -1;
}

// wave-level sum then one atomic per wave into counter slot blockIdx % 64
// (stats + counter * kStatSlots is the base of a counter's slots)
__device__ __forceinline__ void wave_add(unsigned long long* dst, long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v != 0) atomicAdd(dst + (blockIdx.x & (kStatSlots - 1)), (unsigned long long)v);
}

// workgroup-aggregated queue append (blockDim.x == 64 * NW): one atomic per
// workgroup; returns each predicated thread's slot (-1 otherwise).  Must be
// reached by every thread of the workgroup.
template <int NW = 4>
__device__ __forceinline__ int block_push(int32_t* counter, bool pred, int* sh /* [NW + 1] shared */) {
  unsigned long long mask = __ballot(pred);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[wid] = (int)__popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += sh[w];
    sh[NW] = tot ? atomicAdd(counter, tot) : 0;
  }
  __syncthreads();
  int base = sh[NW];
  for (int w = 0; w < wid; ++w) base += sh[w];
  int r = pred ? base + (int)__popcll(mask & ((1ull << lane) - 1ull)) : -1;
  __syncthreads();
  return r;
}

// block_push for two queues whose counters are adjacent (counters[0] and
// counters[1], 8-byte aligned): one 64-bit atomic per workgroup returns both
// bases (each count stays below 2^31, so the low word never carries).  The
// per-workgroup atomics of the element stage kernel are serialised on one
// address and cost it measurably (four times as many: +23 % kernel time).
template <int NW = 4>
__device__ __forceinline__ void block_push2(int32_t* counters, bool p0, bool p1, int* sh /* [2 NW + 2] shared */,
                                            int& s0, int& s1) {
  const unsigned long long m0 = __ballot(p0), m1 = __ballot(p1);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    sh[wid] = (int)__popcll(m0);
    sh[NW + wid] = (int)__popcll(m1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t0 = 0, t1 = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      t0 += (unsigned long long)sh[w];
      t1 += (unsigned long long)sh[NW + w];
    }
    unsigned long long old = 0;
    if (t0 | t1) old = atomicAdd((unsigned long long*)counters, t0 | (t1 << 32));
    sh[2 * NW] = (int)(old & 0xffffffffull);
    sh[2 * NW + 1] = (int)(old >> 32);
  }
  __syncthreads();
  int b0 = sh[2 * NW], b1 = sh[2 * NW + 1];
  for (int w = 0; w < wid; ++w) {
    b0 += sh[w];
    b1 += sh[NW + w];
  }
  const unsigned long long below = (1ull << lane) - 1ull;
  s0 = p0 ? b0 + (int)__popcll(m0 & below) : -1;
  s1 = p1 ? b1 + (int)__popcll(m1 & below) : -1;
  __syncthreads();
}

}  // namespace fp

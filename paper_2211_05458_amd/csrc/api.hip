// C ABI of the flexipart library (see include/flexipart.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/flexipart.h"
#include "fp_launch.h"

using namespace fp;

struct fp_ctx {
  hipStream_t stream = nullptr;
  std::string err;
  // mesh (host staging)
  bool mesh_ok = false;
  int E = 0, n_geo = 0, ng = 0, N = 0, n = 0, dg_nodes = 0;
  std::vector<double> X, shift, elo, ehi, dsafe;
  std::vector<int32_t> nbr_elem, nbr_face, bstart, blist, mortar;
  int task_tp = 64;          // particles per element task of the last sort
  int n_mortar = 0;
  std::vector<int8_t> bc;
  std::vector<double> Minv;
  double blo[3], bdx[3];
  int bn[3];
  double max_extent = 0.0;   // largest element box edge
  double node_pad = 0.0;     // largest distance of a DG node outside its padded element box
  double xgeo[kMaxNodes], cgeo[kMaxNodes], xdg[kMaxNodes], cdg[kMaxNodes], wdg[kMaxNodes];
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t cap = 0;
  MeshView mv{};
  Particles P[2]{};
  int cur = 0;
  unsigned long long* stats = nullptr;
  int32_t *sort_count = nullptr, *sort_start = nullptr, *sort_rank = nullptr, *sort_sums = nullptr;
  int32_t* scratch_i32 = nullptr;
  uint8_t* mlp_flag = nullptr;
  double* dep_buf = nullptr;   // per-particle force (4 doubles), then a validity flag (int32)
  // candidate lists of the FP32 shape-kernel source, valid for (dl_R, dl_per)
  int32_t *dl_count = nullptr, *dl_start = nullptr, *dl_list = nullptr;
  // caller memory for the FP32 source's per-target staged particles (optional)
  void* rl_buf = nullptr;
  int32_t rl_cap = 0;
  bool dl_valid = false, dl_tried = false;
  double dl_R = 0.0, dl_per[3] = {0, 0, 0}, dl_pad = 0.0;
  unsigned long long* dep_pad = nullptr;   // largest distance of a particle outside its element box
  float* mlp_rows = nullptr;   // per-row activations for MLP gradients
  float* mlp_grad = nullptr;   // gradient + loss scratch
  int32_t *tcount = nullptr, *tstart = nullptr, *qcnt = nullptr, *strag = nullptr, *trk_p = nullptr;
  void* tasks = nullptr;
  double* trk_x = nullptr;
  uint8_t* trk_m = nullptr;
  bool tasks_valid = false;
  // fluid
  Fluid fl{};
  bool fluid_ok = false;
  // particles
  int64_t np = 0;
  double d_min = 0.0;
  bool xi_dirty = false;
  bool xi_warm = false;   // P.xi holds each particle's continued reference coordinates (or NaN)
  bool sorted_fresh = false;   // sorted by element, and no particle moved since
  int64_t steps_done = 0, sorts = 0;
  // caller-owned particle block (fp_bind_particles): P[0] then lives there and
  // holds the current state after every call that moves particles
  bool bound = false;
  char* part0 = nullptr;          // the workspace's first particle buffer
  // learned guess: the weights in use are the workspace copy mlp_wbuf
  const float* mlp_w = nullptr;
  float* mlp_wbuf = nullptr;
  float* mlp_adam = nullptr;      // Adam moments m, v of fp_mlp_train [2][nw]
  int32_t* mlp_order = nullptr;   // row order of one epoch [cap]
  float* mlp_bloss = nullptr;     // batch losses of one epoch [cap]
  float* mlp_guess = nullptr;     // learned guesses of a stage [3][cap]
  int64_t n_flagged = 0;
  // timing
  bool timing = false;
  bool count_pairs = false;   // count the shape-kernel pairs within R (timing bit 1)
  std::vector<hipEvent_t> ev_pool;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  size_t ev_used = 0;
};

namespace {

int fail(fp_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(fp_ctx* c, hipError_t e, const char* where) {
  return fail(c, FP_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr)                                   \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return hip_fail(c, _e, #expr);  \
  } while (0)

// Legendre polynomial and derivative by the three-term recurrence
void legendre_pd(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // (x^2 - 1) P_n' = n (x P_n - P_{n-1})
  dP = (std::fabs(x) == 1.0) ? 0.5 * n * (n + 1) * std::pow(x, n + 1) : n * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (n - i - 0.25) / (n + 0.5));
    for (int it = 0; it < 60; ++it) {
      double P, dP;
      legendre_pd(n, z, P, dP);
      double dz = P / dP;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double P, dP;
    legendre_pd(n, z, P, dP);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
}

void gauss_lobatto(int n, double* x, double* w) {
  int N = n - 1;
  for (int i = 0; i <= N; ++i) {
    double z = -std::cos(M_PI * i / N);
    if (i > 0 && i < N)
      for (int it = 0; it < 60; ++it) {
        // roots of (1 - z^2) P_N'(z): Newton on q = P_{N+1} - P_{N-1}
        double Pa, dPa, Pb, dPb;
        legendre_pd(N + 1, z, Pa, dPa);
        legendre_pd(N - 1, z, Pb, dPb);
        double dz = (Pa - Pb) / (dPa - dPb);
        z -= dz;
        if (std::fabs(dz) < 1e-17) break;
      }
    x[i] = z;
    double P, dP;
    legendre_pd(N, z, P, dP);
    w[i] = 2.0 / (N * (N + 1.0) * P * P);
  }
}

void lagrange_weights(int n, const double* x, double* c) {
  for (int i = 0; i < n; ++i) {
    double p = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != i) p *= (x[i] - x[j]);
    c[i] = 1.0 / p;
  }
}

// inverse of the Bernstein-Vandermonde matrix M_ab = B_b((s_a + 1)/2)
std::vector<double> bernstein_vandermonde_inverse(int ng, const double* s) {
  int D = ng - 1;
  std::vector<double> A(ng * 2 * ng, 0.0);
  for (int a = 0; a < ng; ++a) {
    double t = 0.5 * (s[a] + 1.0);
    double binom = 1.0;
    for (int b = 0; b <= D; ++b) {
      A[a * 2 * ng + b] = binom * std::pow(t, b) * std::pow(1.0 - t, D - b);
      binom = binom * (D - b) / (b + 1);
    }
    A[a * 2 * ng + ng + a] = 1.0;
  }
  for (int col = 0; col < ng; ++col) {
    int piv = col;
    for (int r = col + 1; r < ng; ++r)
      if (std::fabs(A[r * 2 * ng + col]) > std::fabs(A[piv * 2 * ng + col])) piv = r;
    for (int j = 0; j < 2 * ng; ++j) std::swap(A[col * 2 * ng + j], A[piv * 2 * ng + j]);
    double p = A[col * 2 * ng + col];
    for (int j = 0; j < 2 * ng; ++j) A[col * 2 * ng + j] /= p;
    for (int r = 0; r < ng; ++r) {
      if (r == col) continue;
      double f = A[r * 2 * ng + col];
      for (int j = 0; j < 2 * ng; ++j) A[r * 2 * ng + j] -= f * A[col * 2 * ng + j];
    }
  }
  std::vector<double> M(ng * ng);
  for (int i = 0; i < ng; ++i)
    for (int j = 0; j < ng; ++j) M[i * ng + j] = A[i * 2 * ng + ng + j];
  return M;
}

// record an event pair around a launch when timing is enabled
// event pool for the optional kernel timing
hipEvent_t take_event(fp_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// record an event pair around the launches in its scope when timing is enabled
struct Timed {
  fp_ctx* c;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(fp_ctx* c_, int cls_) : c(c_), cls(cls_) {
    if (!c->timing) return;
    a = take_event(c);
    b = take_event(c);
    if (a) hipEventRecord(a, c->stream);
  }
  ~Timed() {
    if (!c->timing || !a || !b) return;
    hipEventRecord(b, c->stream);
    c->recs.push_back({cls, a, b});
  }
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Byte offsets of the particle arrays in one block of capacity cap (the
// layout fp_particle_block_layout documents): x, v, kx, kv, xi [3][cap] f64,
// d [cap] f64, elem, hits, id [cap] i32, status [cap] i8, each array starting
// on a 256-byte boundary.
void particle_offsets(int64_t cap, int64_t* off, size_t* total) {
  size_t pc = (size_t)std::max<int64_t>(cap, 1), o = 0;
  for (int a = 0; a < 5; ++a) { off[a] = (int64_t)o; o += align256(pc * 3 * 8); }
  off[5] = (int64_t)o; o += align256(pc * 8);
  for (int a = 6; a < 9; ++a) { off[a] = (int64_t)o; o += align256(pc * 4); }
  off[9] = (int64_t)o; o += align256(pc);
  *total = o;
}


struct Layout {
  size_t X, faces, cp, hE, xnode, vol, elo, ehi, nbox, dsafe, gxi, mortar, nbr_elem, nbr_face, bc, shift, bstart, blist,
      mlp_flag, mlp_h1, mlp_ctr, mlp_w, mlp_adam, mlp_order, mlp_bloss, dl_count, dl_start, dl_list, stats,
      sort_count, sort_start, sort_rank, sort_sums, scratch, dep, mlp_rows, mlp_grad, tcount, tstart, tasks, qcnt,
      strag, trk_p, trk_x, trk_m, mlp_guess, part[2], total;
  size_t part_bytes;
};

Layout layout(const fp_ctx* c, int64_t cap) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  size_t E = c->E, ng3 = (size_t)c->ng * c->ng * c->ng, n3 = (size_t)c->n * c->n * c->n;
  L.X = take(E * ng3 * 3 * 8);
  L.faces = take(E * 6 * sizeof(FaceRec));
  L.cp = take(E * 6 * c->ng * c->ng * 3 * 8);
  L.hE = take(E * 8);
  L.xnode = take(E * n3 * 3 * 8);
  L.vol = take(E * n3 * 8);
  L.elo = take(E * 3 * 8);
  L.ehi = take(E * 3 * 8);
  L.nbox = take(E * 6 * 8);
  L.dsafe = take(E * 8);
  L.gxi = take(E * 6 * 8);
  L.mortar = take(std::max<size_t>(1, c->mortar.size()) * 4);
  L.nbr_elem = take(E * 6 * 4);
  L.nbr_face = take(E * 6 * 4);
  L.bc = take(E * 6);
  L.shift = take(E * 18 * 8);
  L.bstart = take(c->bstart.size() * 4);
  L.blist = take(std::max<size_t>(1, c->blist.size()) * 4);
  L.mlp_flag = take(E);
  L.mlp_h1 = take(E * 64 * 4);
  L.mlp_ctr = take(E * 4 * 8);
  L.mlp_w = take((size_t)kMlpWeights * 4);
  L.mlp_adam = take((size_t)kMlpWeights * 2 * 4);
  L.mlp_order = take((size_t)std::max<int64_t>(cap, 1) * 4);
  L.mlp_bloss = take((size_t)std::max<int64_t>(cap, 1) * 4);
  L.dl_count = take((E + 1) * 4);
  L.dl_start = take((E + 1) * 4);
  L.dl_list = take(E * (size_t)kDepListPerElem * 4);
  L.stats = take(16 * kStatSlots * 8);
  L.sort_count = take((E + 1) * 4);
  L.sort_start = take((E + 1) * 4);
  L.sort_rank = take((size_t)std::max<int64_t>(cap, 1) * 4);
  L.sort_sums = take(((std::max<size_t>(E + 1, cap) + 1023) / 1024 + 2) * 4);
  L.scratch = take(64);
  // F (4 doubles), validity flag, FP32 normalisation sum, FP32 local position (float4)
  L.dep = take((size_t)std::max<int64_t>(cap, 1) * 7 * 8 + 16);
  L.mlp_rows = take((size_t)kMlpMaxBatch * kMlpRow * 4);
  L.mlp_grad = take((size_t)(kMlpWeights + 64) * 4);
  size_t pc1 = (size_t)std::max<int64_t>(cap, 1);
  L.tcount = take((E + 1) * 4);
  L.tstart = take((E + 1) * 4);
  L.tasks = take((E + pc1 / kMinTaskParticles + 2) * task_bytes());
  L.qcnt = take(64);
  L.strag = take(pc1 * 4);
  L.trk_p = take(pc1 * 4);
  L.trk_x = take(pc1 * 3 * 8);
  L.trk_m = take(pc1);
  L.mlp_guess = take(pc1 * 3 * 4);
  {
    int64_t off[10];
    particle_offsets(cap, off, &L.part_bytes);
  }
  L.part[0] = take(L.part_bytes);
  L.part[1] = take(L.part_bytes);
  L.total = o;
  return L;
}

Particles carve(char* base, int64_t cap) {
  Particles P{};
  int64_t off[10];
  size_t total;
  particle_offsets(cap, off, &total);
  P.cap = cap;
  P.x = (double*)(base + off[0]); P.v = (double*)(base + off[1]); P.kx = (double*)(base + off[2]);
  P.kv = (double*)(base + off[3]); P.xi = (double*)(base + off[4]); P.d = (double*)(base + off[5]);
  P.elem = (int32_t*)(base + off[6]); P.hits = (int32_t*)(base + off[7]); P.id = (int32_t*)(base + off[8]);
  P.status = (int8_t*)(base + off[9]);
  return P;
}

// A caller-owned block holds the current state: after a sort left it in the
// workspace buffer, copy it back (same indices, so element tasks stay valid).
int sync_bound(fp_ctx* c);

}  // namespace

namespace {
// counting sort of the current particle buffer into the other one, then the
// element tasks of the fast stage kernel
// Lower bound of the distance from each element to any face that is not
// internal (wall, open, periodic), for the reference-space localisation: the
// gap between the element's padded node box and the face's Bernstein
// control-point box (which contains the face), over the faces within h_e of
// the element, less 0.1 h_e, in [0, 0.9 h_e].  Host, at mesh set-up.
void boundary_distance(fp_ctx* c) {
  const int E = c->E, ng = c->ng, D = ng - 1;
  const size_t ng3 = (size_t)ng * ng * ng;
  const size_t ncell = (size_t)c->bn[0] * c->bn[1] * c->bn[2];
  std::vector<double> fbox;   // [6] per boundary face
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      if (c->bc[e * 6 + f] == 0) continue;
      // Lagrange nodes of the face -> Bernstein control points, P = M^-1 F M^-T
      int d = f / 2, a = (d == 0) ? 1 : 0, b = (d == 2) ? 1 : 2, fix = (f & 1) ? D : 0;
      const double* Xe = c->X.data() + (size_t)e * ng3 * 3;
      std::vector<double> T((size_t)ng * ng * 3), P((size_t)ng * ng * 3);
      for (int n = 0; n < ng; ++n)
        for (int mm = 0; mm < ng; ++mm)
          for (int q = 0; q < 3; ++q) {
            double acc = 0.0;
            for (int r = 0; r < ng; ++r) {
              int idx[3];
              idx[d] = fix; idx[a] = r; idx[b] = n;
              acc += c->Minv[mm * ng + r] * Xe[((idx[2] * ng + idx[1]) * ng + idx[0]) * 3 + q];
            }
            T[(n * ng + mm) * 3 + q] = acc;
          }
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int n = 0; n < ng; ++n)
        for (int mm = 0; mm < ng; ++mm)
          for (int q = 0; q < 3; ++q) {
            double acc = 0.0;
            for (int r = 0; r < ng; ++r) acc += c->Minv[n * ng + r] * T[(r * ng + mm) * 3 + q];
            lo[q] = std::min(lo[q], acc);
            hi[q] = std::max(hi[q], acc);
          }
      for (int q = 0; q < 3; ++q) fbox.push_back(lo[q]);
      for (int q = 0; q < 3; ++q) fbox.push_back(hi[q]);
    }
  const int nbf = (int)(fbox.size() / 6);
  auto cell_range = [&](const double* lo, const double* hi, double pad, int* c0, int* c1) {
    for (int k = 0; k < 3; ++k) {
      c0[k] = std::max(0, (int)std::floor((lo[k] - pad - c->blo[k]) / c->bdx[k]));
      c1[k] = std::min(c->bn[k] - 1, (int)std::floor((hi[k] + pad - c->blo[k]) / c->bdx[k]));
    }
  };
  std::vector<int> fstart(ncell + 1, 0), flist;
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int> fill;
    if (pass == 1) {
      for (size_t q = 0; q < ncell; ++q) fstart[q + 1] += fstart[q];
      flist.assign(std::max(1, fstart[ncell]), 0);
      fill.assign(ncell, 0);
    }
    for (int j = 0; j < nbf; ++j) {
      int c0[3], c1[3];
      cell_range(&fbox[6 * j], &fbox[6 * j + 3], 0.0, c0, c1);
      for (int z = c0[2]; z <= c1[2]; ++z)
        for (int y = c0[1]; y <= c1[1]; ++y)
          for (int x = c0[0]; x <= c1[0]; ++x) {
            size_t id = ((size_t)z * c->bn[1] + y) * c->bn[0] + x;
            if (pass == 0) fstart[id + 1]++;
            else flist[fstart[id] + fill[id]++] = j;
          }
    }
  }
  c->dsafe.assign(E, 0.0);
  for (int e = 0; e < E; ++e) {
    // element length scale: longest corner-to-corner edge
    const double* Pn = c->X.data() + (size_t)e * ng3 * 3;
    double h = 0.0;
    for (int v = 0; v < 8; ++v)
      for (int bit = 0; bit < 3; ++bit) {
        int w = v ^ (1 << bit);
        if (w < v) continue;
        int iv = ((((v >> 2) & 1) * D) * ng + ((v >> 1) & 1) * D) * ng + (v & 1) * D;
        int iw = ((((w >> 2) & 1) * D) * ng + ((w >> 1) & 1) * D) * ng + (w & 1) * D;
        double r2 = 0.0;
        for (int q = 0; q < 3; ++q) r2 += (Pn[iv * 3 + q] - Pn[iw * 3 + q]) * (Pn[iv * 3 + q] - Pn[iw * 3 + q]);
        h = std::max(h, std::sqrt(r2));
      }
    const double* lo = &c->elo[e * 3];
    const double* hi = &c->ehi[e * 3];
    double best = h;
    int c0[3], c1[3];
    cell_range(lo, hi, h, c0, c1);
    for (int z = c0[2]; z <= c1[2]; ++z)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x) {
          size_t id = ((size_t)z * c->bn[1] + y) * c->bn[0] + x;
          for (int q = fstart[id]; q < fstart[id + 1]; ++q) {
            const double* fb = &fbox[6 * flist[q]];
            double g2 = 0.0;
            for (int k = 0; k < 3; ++k) {
              double gap = std::max(0.0, std::max(fb[k] - hi[k], lo[k] - fb[3 + k]));
              g2 += gap * gap;
            }
            best = std::min(best, std::sqrt(g2));
          }
        }
    c->dsafe[e] = std::max(0.0, best - 0.1 * h);
  }
}

// counting sort by element, then the element tasks of tp particles each
int sort_particles(fp_ctx* c, int tp) {
  hipStream_t s = c->stream;
  if (c->np == 0) {   // nothing to bucket: no histogram is computed, so no tasks either
    c->tasks_valid = false;
    return FP_OK;
  }
  HIPCHK(c, launch_sort(c->P[c->cur], c->P[1 - c->cur], c->np, c->E, c->sort_count, c->sort_start, c->sort_rank,
                        c->sort_sums, s));
  c->cur = 1 - c->cur;
  c->sorts++;
  c->sorted_fresh = true;
  HIPCHK(c, launch_tasks(c->sort_count, c->sort_start, c->E, tp, c->tcount, c->tstart, c->sort_sums, c->tasks,
                         c->qcnt + 4, (int64_t)c->E + c->cap / tp + 2, s));
  c->tasks_valid = true;
  c->task_tp = tp;
  return FP_OK;
}

int sync_bound(fp_ctx* c) {
  if (!c->bound || c->cur == 0 || c->np == 0) return FP_OK;
  const Particles& S = c->P[1];
  const Particles& D = c->P[0];
  const size_t n = (size_t)c->np;
  hipStream_t s = c->stream;
  for (int k = 0; k < 3; ++k) {
    HIPCHK(c, hipMemcpyAsync(D.x + k * D.cap, S.x + k * S.cap, n * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(D.v + k * D.cap, S.v + k * S.cap, n * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(D.kx + k * D.cap, S.kx + k * S.cap, n * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(D.kv + k * D.cap, S.kv + k * S.cap, n * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(D.xi + k * D.cap, S.xi + k * S.cap, n * 8, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(c, hipMemcpyAsync(D.d, S.d, n * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(D.elem, S.elem, n * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(D.hits, S.hits, n * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(D.id, S.id, n * 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(D.status, S.status, n, hipMemcpyDeviceToDevice, s));
  c->cur = 0;
  return FP_OK;
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): output i of stream `seed` is the mix of
// seed + (i + 1) * 0x9E3779B97F4A7C15.  Draws of fp_mlp_train: the initial
// weights first (one per weight, in layout order), then one Fisher-Yates
// shuffle per epoch (draws for i = n-1 down to 1).
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }                       // [0, 1)
  uint32_t below(uint32_t k) { return (uint32_t)(((unsigned __int128)next() * k) >> 64); }  // [0, k)
};

// Xavier-uniform weights (limit sqrt(6 / (fan_in + fan_out))), zero biases
void mlp_xavier(SplitMix64& g, std::vector<float>& w) {
  const int shapes[4][2] = {{64, kMlpIn}, {64, 64}, {64, 64}, {3, 64}};
  size_t o = 0;
  for (auto& sh : shapes) {
    const double a = std::sqrt(6.0 / (sh[0] + sh[1]));
    for (int i = 0; i < sh[0] * sh[1]; ++i) w[o++] = (float)(a * (2.0 * g.uniform() - 1.0));
    for (int i = 0; i < sh[0]; ++i) w[o++] = 0.0f;
  }
}

void shuffle(SplitMix64& g, std::vector<int32_t>& a) {
  for (int64_t i = (int64_t)a.size() - 1; i >= 1; --i) std::swap(a[i], a[g.below((uint32_t)(i + 1))]);
}
}  // namespace

extern "C" {

static_assert(FP_MLP_STATIC_ROWS == kMlpStaticRows, "row limit of fp_mlp_loss_grad_static");

int fp_create(fp_ctx** out, void* hip_stream) {
  if (!out) return FP_EINVAL;
  fp_ctx* c = new fp_ctx();
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return FP_OK;
}

void fp_destroy(fp_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  delete c;
}

const char* fp_last_error(fp_ctx* c) { return c ? c->err.c_str() : "null context"; }

int fp_init_mesh(fp_ctx* c, const fp_mesh_desc* d) {
  if (!c || !d) return FP_EINVAL;
  if (d->n_elem <= 0 || d->n_geo < 1 || d->n_geo > 6 || d->n_dg < 1 || d->n_dg > 7 || !d->X || !d->nbr_elem ||
      !d->nbr_face || !d->bc || !d->periodic_shift)
    return fail(c, FP_EINVAL, "fp_init_mesh: bad sizes or null arrays");
  if (!supported(d->n_dg + 1, d->n_geo + 1))
    return fail(c, FP_EINVAL, "fp_init_mesh: no compiled kernels for this (N, Ngeo)");
  int E = d->n_elem;
  const int NM = d->n_mortar;
  if (NM < 0 || (NM > 0 && !d->mortar)) return fail(c, FP_EINVAL, "fp_init_mesh: bad mortar table");
  // small face (e, f) listed under big mortar face m
  auto listed = [&](int m, int e, int f) {
    for (int j = 0; j < 4; ++j)
      if (d->mortar[m * 8 + 2 * j] == e && d->mortar[m * 8 + 2 * j + 1] == f) return true;
    return false;
  };
  // neighbour reciprocity (a small face points to its big face, which lists it)
  std::vector<int> mortar_owner(NM, -1);
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      int nb = d->nbr_elem[e * 6 + f], nf = d->nbr_face[e * 6 + f], b = d->bc[e * 6 + f];
      if (b < 0 || b > 4) return fail(c, FP_EMESH, "fp_init_mesh: bad boundary code");
      if (b == FP_BC_MORTAR) {
        if (nb < 0 || nb >= NM || mortar_owner[nb] >= 0) return fail(c, FP_EMESH, "fp_init_mesh: bad mortar index");
        mortar_owner[nb] = e * 6 + f;
      } else if (b == FP_BC_INTERNAL || b == FP_BC_PERIODIC) {
        if (nb < 0 || nb >= E || nf < 0 || nf > 5) return fail(c, FP_EMESH, "fp_init_mesh: bad neighbour");
        if (d->bc[nb * 6 + nf] == FP_BC_MORTAR) {
          const int m = d->nbr_elem[nb * 6 + nf];
          if (b != FP_BC_INTERNAL || m < 0 || m >= NM || !listed(m, e, f))
            return fail(c, FP_EMESH, "fp_init_mesh: small face not listed by its mortar");
        } else if (d->nbr_elem[nb * 6 + nf] != e || d->nbr_face[nb * 6 + nf] != f) {
          return fail(c, FP_EMESH, "fp_init_mesh: non-reciprocal neighbour table");
        }
      }
    }
  for (int m = 0; m < NM; ++m) {
    if (mortar_owner[m] < 0) return fail(c, FP_EMESH, "fp_init_mesh: mortar without a big face");
    int nsmall = 0;
    for (int j = 0; j < 4; ++j) {
      const int s = d->mortar[m * 8 + 2 * j], fs = d->mortar[m * 8 + 2 * j + 1];
      if (s < 0) continue;
      if (s >= E || fs < 0 || fs > 5 || d->bc[s * 6 + fs] != FP_BC_INTERNAL ||
          d->nbr_elem[s * 6 + fs] * 6 + d->nbr_face[s * 6 + fs] != mortar_owner[m])
        return fail(c, FP_EMESH, "fp_init_mesh: mortar lists a face that does not point back");
      nsmall++;
    }
    if (nsmall != 2 && nsmall != 4) return fail(c, FP_EMESH, "fp_init_mesh: a mortar needs 2 or 4 small faces");
  }
  c->n_mortar = NM;
  c->mortar.assign(NM ? d->mortar : nullptr, NM ? d->mortar + (size_t)NM * 8 : nullptr);
  c->E = E; c->n_geo = d->n_geo; c->ng = d->n_geo + 1; c->N = d->n_dg; c->n = d->n_dg + 1;
  c->dg_nodes = d->dg_nodes;
  size_t ng3 = (size_t)c->ng * c->ng * c->ng;
  c->X.assign(d->X, d->X + (size_t)E * ng3 * 3);
  c->nbr_elem.assign(d->nbr_elem, d->nbr_elem + E * 6);
  c->nbr_face.assign(d->nbr_face, d->nbr_face + E * 6);
  c->bc.assign(d->bc, d->bc + E * 6);
  c->shift.assign(d->periodic_shift, d->periodic_shift + (size_t)E * 18);
  for (int i = 0; i < c->ng; ++i) c->xgeo[i] = -1.0 + 2.0 * i / c->n_geo;
  lagrange_weights(c->ng, c->xgeo, c->cgeo);
  if (c->dg_nodes == 0) gauss_legendre(c->n, c->xdg, c->wdg);
  else gauss_lobatto(c->n, c->xdg, c->wdg);
  lagrange_weights(c->n, c->xdg, c->cdg);
  c->Minv = bernstein_vandermonde_inverse(c->ng, c->xgeo);
  // element boxes (node box padded by 5 % per axis) and the background mesh
  c->elo.resize((size_t)E * 3);
  c->ehi.resize((size_t)E * 3);
  double glo[3] = {1e300, 1e300, 1e300}, ghi[3] = {-1e300, -1e300, -1e300}, ext = 0.0;
  for (int e = 0; e < E; ++e) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    const double* P = c->X.data() + (size_t)e * ng3 * 3;
    for (size_t q = 0; q < ng3; ++q)
      for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], P[q * 3 + k]); hi[k] = std::max(hi[k], P[q * 3 + k]); }
    double em = 0.0;
    for (int k = 0; k < 3; ++k) {
      double pad = 0.05 * (hi[k] - lo[k]);
      c->elo[e * 3 + k] = lo[k] - pad;
      c->ehi[e * 3 + k] = hi[k] + pad;
      glo[k] = std::min(glo[k], c->elo[e * 3 + k]);
      ghi[k] = std::max(ghi[k], c->ehi[e * 3 + k]);
      em = std::max(em, hi[k] - lo[k]);
    }
    ext += em;
    c->max_extent = std::max(c->max_extent, 1.1 * em);
  }
  double h = ext / E;
  for (int k = 0; k < 3; ++k) {
    int nb = (int)std::ceil((ghi[k] - glo[k]) / h);
    nb = std::max(1, std::min(nb, 1024));
    c->bn[k] = nb;
    c->blo[k] = glo[k];
    c->bdx[k] = (ghi[k] - glo[k]) / nb;
    if (!(c->bdx[k] > 0.0)) c->bdx[k] = 1.0;
  }
  size_t ncell = (size_t)c->bn[0] * c->bn[1] * c->bn[2];
  c->bstart.assign(ncell + 1, 0);
  std::vector<int> lo3((size_t)E * 3), hi3((size_t)E * 3);
  for (int e = 0; e < E; ++e)
    for (int k = 0; k < 3; ++k) {
      lo3[e * 3 + k] = std::max(0, (int)std::floor((c->elo[e * 3 + k] - c->blo[k]) / c->bdx[k]));
      hi3[e * 3 + k] = std::min(c->bn[k] - 1, (int)std::floor((c->ehi[e * 3 + k] - c->blo[k]) / c->bdx[k]));
    }
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int32_t> fill;
    if (pass == 1) {
      for (size_t i = 0; i < ncell; ++i) c->bstart[i + 1] += c->bstart[i];
      c->blist.assign(c->bstart[ncell], 0);
      fill.assign(ncell, 0);
    }
    for (int e = 0; e < E; ++e)
      for (int z = lo3[e * 3 + 2]; z <= hi3[e * 3 + 2]; ++z)
        for (int y = lo3[e * 3 + 1]; y <= hi3[e * 3 + 1]; ++y)
          for (int x = lo3[e * 3]; x <= hi3[e * 3]; ++x) {
            size_t cell = ((size_t)z * c->bn[1] + y) * c->bn[0] + x;
            if (pass == 0) c->bstart[cell + 1]++;
            else c->blist[c->bstart[cell] + fill[cell]++] = e;
          }
  }
  boundary_distance(c);
  c->mesh_ok = true;
  c->rl_buf = nullptr;   // sized for the previous mesh's elements
  c->rl_cap = 0;
  c->ws = nullptr;
  c->np = 0;
  c->fluid_ok = false;
  return FP_OK;
}

int fp_workspace_size(fp_ctx* c, int64_t max_particles, size_t* bytes) {
  if (!c || !bytes || max_particles < 0) return FP_EINVAL;
  if (!c->mesh_ok) return fail(c, FP_ESTATE, "fp_workspace_size: no mesh");
  if (max_particles > (int64_t)INT32_MAX) return fail(c, FP_EINVAL, "fp_workspace_size: too many particles");
  *bytes = layout(c, max_particles).total + 256;
  return FP_OK;
}

int fp_bind_workspace(fp_ctx* c, void* dev, size_t bytes) {
  if (!c || !dev) return FP_EINVAL;
  if (!c->mesh_ok) return fail(c, FP_ESTATE, "fp_bind_workspace: no mesh");
  if (((uintptr_t)dev) & 255) return fail(c, FP_EINVAL, "fp_bind_workspace: pointer not 256-byte aligned");
  // largest particle capacity that fits
  int64_t lo = 0, hi = 1;
  while (layout(c, hi).total + 256 <= bytes && hi < ((int64_t)1 << 31)) hi *= 2;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) / 2;
    if (layout(c, mid).total + 256 <= bytes) lo = mid; else hi = mid;
  }
  if (layout(c, lo).total + 256 > bytes) return fail(c, FP_EINVAL, "fp_bind_workspace: too small for the mesh");
  Layout L = layout(c, lo);
  char* b = (char*)dev;
  c->ws = b;
  c->ws_bytes = bytes;
  c->cap = lo;
  hipStream_t s = c->stream;
  size_t E = c->E, ng3 = (size_t)c->ng * c->ng * c->ng;
  HIPCHK(c, hipMemcpyAsync(b + L.X, c->X.data(), E * ng3 * 3 * 8, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(b + L.elo, c->elo.data(), E * 3 * 8, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(b + L.dsafe, c->dsafe.data(), E * 8, hipMemcpyHostToDevice, s));
  if (!c->mortar.empty())
    HIPCHK(c, hipMemcpyAsync(b + L.mortar, c->mortar.data(), c->mortar.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(b + L.ehi, c->ehi.data(), E * 3 * 8, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(b + L.nbr_elem, c->nbr_elem.data(), E * 6 * 4, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(b + L.nbr_face, c->nbr_face.data(), E * 6 * 4, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(b + L.bc, c->bc.data(), E * 6, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(b + L.shift, c->shift.data(), E * 18 * 8, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(b + L.bstart, c->bstart.data(), c->bstart.size() * 4, hipMemcpyHostToDevice, s));
  if (!c->blist.empty())
    HIPCHK(c, hipMemcpyAsync(b + L.blist, c->blist.data(), c->blist.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemsetAsync(b + L.stats, 0, 16 * kStatSlots * 8, s));
  HIPCHK(c, hipMemsetAsync(b + L.mlp_flag, 0, E, s));
  MeshView& m = c->mv;
  m = MeshView{};
  m.E = c->E; m.ng = c->ng; m.n = c->n; m.n_geo = c->n_geo;
  m.X = (const double*)(b + L.X);
  m.faces = (const FaceRec*)(b + L.faces);
  m.cp = (const double*)(b + L.cp);
  m.hE = (const double*)(b + L.hE);
  m.xnode = (const double*)(b + L.xnode);
  m.vol = (const double*)(b + L.vol);
  m.elo = (const double*)(b + L.elo);
  m.ehi = (const double*)(b + L.ehi);
  m.nbox = (const double*)(b + L.nbox);
  m.dsafe = (const double*)(b + L.dsafe);
  m.gxi = (const double*)(b + L.gxi);
  m.mortar = (const int32_t*)(b + L.mortar);
  m.n_mortar = c->n_mortar;
  for (int i = 0; i < kMaxNodes; ++i) {
    m.xgeo[i] = i < c->ng ? c->xgeo[i] : 0.0;
    m.cgeo[i] = i < c->ng ? c->cgeo[i] : 0.0;
    m.xdg[i] = i < c->n ? c->xdg[i] : 0.0;
    m.cdg[i] = i < c->n ? c->cdg[i] : 0.0;
    m.wdg[i] = i < c->n ? c->wdg[i] : 0.0;
    m.xdgf[i] = (float)m.xdg[i];
    m.cdgf[i] = (float)m.cdg[i];
  }
  for (int k = 0; k < 3; ++k) { m.blo[k] = c->blo[k]; m.bdx[k] = c->bdx[k]; m.bn[k] = c->bn[k]; }
  m.bstart = (const int32_t*)(b + L.bstart);
  m.blist = (const int32_t*)(b + L.blist);
  m.mlp_flag = (const uint8_t*)(b + L.mlp_flag);
  m.mlp_w = nullptr;
  m.mlp_h1 = (const float*)(b + L.mlp_h1);
  m.mlp_ctr = (const double*)(b + L.mlp_ctr);
  c->mlp_flag = (uint8_t*)(b + L.mlp_flag);
  c->stats = (unsigned long long*)(b + L.stats);
  c->sort_count = (int32_t*)(b + L.sort_count);
  c->sort_start = (int32_t*)(b + L.sort_start);
  c->sort_rank = (int32_t*)(b + L.sort_rank);
  c->sort_sums = (int32_t*)(b + L.sort_sums);
  c->scratch_i32 = (int32_t*)(b + L.scratch);
  c->dep_buf = (double*)(b + L.dep);
  c->mlp_rows = (float*)(b + L.mlp_rows);
  c->mlp_grad = (float*)(b + L.mlp_grad);
  c->tcount = (int32_t*)(b + L.tcount);
  c->tstart = (int32_t*)(b + L.tstart);
  c->tasks = (void*)(b + L.tasks);
  c->qcnt = (int32_t*)(b + L.qcnt);
  c->strag = (int32_t*)(b + L.strag);
  c->trk_p = (int32_t*)(b + L.trk_p);
  c->trk_x = (double*)(b + L.trk_x);
  c->trk_m = (uint8_t*)(b + L.trk_m);
  c->tasks_valid = false;
  c->part0 = b + L.part[0];
  c->P[0] = carve(b + L.part[0], c->cap);
  c->P[1] = carve(b + L.part[1], c->cap);
  c->cur = 0;
  c->bound = false;
  c->mlp_wbuf = (float*)(b + L.mlp_w);
  c->mlp_adam = (float*)(b + L.mlp_adam);
  c->mlp_order = (int32_t*)(b + L.mlp_order);
  c->mlp_bloss = (float*)(b + L.mlp_bloss);
  c->mlp_guess = (float*)(b + L.mlp_guess);
  c->mlp_w = nullptr;
  c->dl_count = (int32_t*)(b + L.dl_count);
  c->dl_start = (int32_t*)(b + L.dl_start);
  c->dl_list = (int32_t*)(b + L.dl_list);
  c->dl_valid = c->dl_tried = false;
  HIPCHK(c, hipMemsetAsync(c->scratch_i32, 0, 64, s));
  HIPCHK(c, launch_face_setup(m, m.X, (const int32_t*)(b + L.nbr_elem), (const int32_t*)(b + L.nbr_face),
                              (const int8_t*)(b + L.bc), (const double*)(b + L.shift), c->Minv.data(),
                              (FaceRec*)(b + L.faces), (double*)(b + L.cp), s));
  HIPCHK(c, launch_nodes(m, (double*)(b + L.xnode), (double*)(b + L.vol), (double*)(b + L.hE), (double*)(b + L.nbox),
                         (double*)(b + L.gxi), c->scratch_i32, (unsigned long long*)(b + L.scratch + 8), s));
  int32_t bad = 0;
  unsigned long long pad_bits = 0;
  HIPCHK(c, hipMemcpyAsync(&bad, c->scratch_i32, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(&pad_bits, b + L.scratch + 8, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (bad) return fail(c, FP_EMESH, "fp_bind_workspace: non-positive Jacobian at " + std::to_string(bad) + " nodes");
  std::memcpy(&c->node_pad, &pad_bits, 8);
  c->dep_pad = (unsigned long long*)(b + L.scratch + 16);
  c->np = 0;
  return FP_OK;
}

int fp_set_fluid_state(fp_ctx* c, const void* U, fp_dtype dt, const fp_fluid_params* prm) {
  if (!c || !U || !prm) return FP_EINVAL;
  if (!(prm->mu > 0.0) || !(prm->rho_p > 0.0)) return fail(c, FP_EINVAL, "fp_set_fluid_state: bad parameters");
  c->fl.U = U;
  c->fl.f32 = (dt == FP_F32);
  c->fl.mu = prm->mu;
  c->fl.kappa = prm->kappa;
  c->fl.rho_p = prm->rho_p;
  c->fluid_ok = true;
  return FP_OK;
}

int fp_push_particles(fp_ctx* c, int64_t n, const double* x, const double* v, const double* d,
                      const int32_t* hint, int32_t* status_out) {
  if (!c || n < 0) return FP_EINVAL;
  const bool in_place = !x && !v && !d;
  if (n > 0 && !in_place && (!x || !v || !d)) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_push_particles: no workspace");
  if (in_place && n > 0 && !c->bound)
    return fail(c, FP_EINVAL, "fp_push_particles: x, v, d may be NULL only with a bound particle block");
  hipStream_t s = c->stream;
  c->cur = 0;
  Particles& P = c->P[0];
  int64_t cap = P.cap;
  if (n > cap) return fail(c, FP_EINVAL, "fp_push_particles: more particles than capacity");
  double dmin = 1e300;
  if (in_place) {
    // x, v and d are already in the bound block: smallest diameter (and a
    // check that every one is positive) on the device
    if (n > 0) {
      HIPCHK(c, hipMemsetAsync(c->scratch_i32 + 8, 0, 24, s));
      HIPCHK(c, launch_min_positive(P.d, n, (unsigned long long*)(c->scratch_i32 + 8), c->scratch_i32 + 12, s));
      unsigned long long bits = 0;
      int32_t bad = 0;
      HIPCHK(c, hipMemcpyAsync(&bits, c->scratch_i32 + 8, 8, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipMemcpyAsync(&bad, c->scratch_i32 + 12, 4, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      if (bad) return fail(c, FP_EINVAL, "fp_push_particles: non-positive diameter");
      bits = ~bits;
      std::memcpy(&dmin, &bits, 8);
    }
  } else {
    std::vector<double> tx((size_t)n * 3), tv((size_t)n * 3);
    for (int64_t p = 0; p < n; ++p) {
      for (int k = 0; k < 3; ++k) {
        tx[k * n + p] = x[p * 3 + k];
        tv[k * n + p] = v[p * 3 + k];
      }
      dmin = std::min(dmin, d[p]);
      if (!(d[p] > 0.0)) return fail(c, FP_EINVAL, "fp_push_particles: non-positive diameter");
    }
    for (int k = 0; k < 3 && n > 0; ++k) {
      HIPCHK(c, hipMemcpyAsync(P.x + k * cap, tx.data() + k * n, n * 8, hipMemcpyHostToDevice, s));
      HIPCHK(c, hipMemcpyAsync(P.v + k * cap, tv.data() + k * n, n * 8, hipMemcpyHostToDevice, s));
    }
    if (n > 0) HIPCHK(c, hipMemcpyAsync(P.d, d, n * 8, hipMemcpyHostToDevice, s));
    // the copies read pageable host memory: finish them before tx, tv go
    HIPCHK(c, hipStreamSynchronize(s));
  }
  const int32_t* dh = nullptr;
  if (hint && n > 0) {
    HIPCHK(c, hipMemcpyAsync(c->sort_rank, hint, n * 4, hipMemcpyHostToDevice, s));
    dh = c->sort_rank;
  }
  HIPCHK(c, launch_locate(c->mv, P, dh, n, s));
  std::vector<int8_t> st((size_t)std::max<int64_t>(n, 1));
  if (n > 0) HIPCHK(c, hipMemcpyAsync(st.data(), P.status, n, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  int nrej = 0;
  for (int64_t p = 0; p < n; ++p) {
    if (st[p] != FP_ACTIVE) nrej++;
    if (status_out) status_out[p] = st[p];
  }
  c->np = n;
  c->d_min = dmin;
  c->xi_dirty = false;
  c->tasks_valid = false;
  c->sorted_fresh = false;
  c->steps_done = 0;
  return nrej;
}

int fp_step(fp_ctx* c, double dt, int32_t n_steps, const fp_step_opts* o) {
  if (!c || !o || n_steps < 0 || !(dt > 0.0)) return FP_EINVAL;
  if (!c->ws || !c->fluid_ok) return fail(c, FP_ESTATE, "fp_step: workspace or fluid state missing");
  if (o->rk < 0 || o->rk > 1 || o->drag < 0 || o->drag > 2 || o->precision < 0 || o->precision > 1 ||
      o->tracking < 0 || o->tracking > 1 || (o->forces & ~kForceAll) != 0)
    return fail(c, FP_EINVAL, "fp_step: bad options");
  if (o->precision == 0 && c->fl.f32)
    ;  // FP64 arithmetic on an FP32 state is allowed (values widened on load)
  // low-storage coefficients (Carpenter-Kennedy 5-stage 4th order; Williamson 3-stage 3rd order)
  static const double A4[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
  static const double B4[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};
  static const double A3[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
  static const double B3[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
  const double* A = o->rk == 0 ? A4 : A3;
  const double* B = o->rk == 0 ? B4 : B3;
  int S = o->rk == 0 ? 5 : 3;
  StepParams sp{};
  sp.dt = dt;
  for (int k = 0; k < 3; ++k) sp.gravity[k] = o->gravity[k];
  sp.drag = o->drag;
  sp.max_it = o->max_newton_it > 0 ? o->max_newton_it : 50;
  sp.max_cross = o->max_crossings > 0 ? o->max_crossings : 64;
  sp.use_mlp = ((o->guess & 1) && c->mlp_w) ? 1 : 0;
  sp.warm = (o->guess & 2) ? 1 : 0;
  sp.refspace = o->tracking;
  sp.forces = o->forces;
  sp.mlp_guess = (sp.use_mlp && c->n_flagged > 0) ? c->mlp_guess : nullptr;
  hipStream_t s = c->stream;
  const int tp = task_particles(c->n, c->ng, o->precision == 1);
  for (int st = 0; st < n_steps; ++st) {
    if (o->sort_every < 0 || (o->sort_every > 0 && (c->steps_done % o->sort_every) == 0)) {
      // a sort since the particles last moved (the shape-kernel source sorts
      // after locating them) already holds the tasks of this step
      if (!(c->sorted_fresh && c->tasks_valid && c->task_tp == tp)) {
        Timed tm(c, 0);
        int rc = sort_particles(c, tp);
        if (rc) return rc;
      }
    }
    c->sorted_fresh = false;
    for (int i = 0; i < S; ++i) {
      if (o->sort_every < 0 && i > 0) {
        // every stage: the particles that crossed a face in the last stage
        // join their new element's task instead of the per-lane kernel
        Timed tm(c, 0);
        int rc = sort_particles(c, tp);
        if (rc) return rc;
      }
      sp.A = A[i];
      sp.B = B[i];
      StageLaunch Lc{};
      Lc.m = c->mv;
      Lc.P = c->P[c->cur];
      Lc.fl = c->fl;
      Lc.sp = sp;
      Lc.n = c->np;
      Lc.mixed = o->precision;
      Lc.mlp = sp.use_mlp;
      Lc.tasks = c->tasks_valid ? c->tasks : nullptr;
      Lc.task_tp = c->task_tp;
      Lc.ntask = c->qcnt + 4;
      Lc.counters = c->qcnt;
      Lc.strag = c->strag;
      Lc.trk_p = c->trk_p;
      Lc.trk_x = c->trk_x;
      Lc.trk_m = c->trk_m;
      Lc.stats = c->stats;
      if (c->timing)
        for (int k = 0; k < (sp.mlp_guess ? 8 : 6); ++k) Lc.ev[k] = take_event(c);
      HIPCHK(c, launch_stage(Lc, s));
      if (c->timing) {
        if (stage_uses_tasks(Lc) && Lc.ev[0] && Lc.ev[1]) c->recs.push_back({1, Lc.ev[0], Lc.ev[1]});
        if (Lc.ev[2] && Lc.ev[3]) c->recs.push_back({5, Lc.ev[2], Lc.ev[3]});
        if (Lc.ev[4] && Lc.ev[5]) c->recs.push_back({6, Lc.ev[4], Lc.ev[5]});
        if (Lc.ev[6] && Lc.ev[7]) c->recs.push_back({9, Lc.ev[6], Lc.ev[7]});
      }
    }
    c->steps_done++;
  }
  c->xi_dirty = true;
  c->xi_warm = sp.warm != 0;
  {
    int rc = sync_bound(c);
    if (rc) return rc;
  }
  // stability of the drag term: dt * f_D / tau_p within the real-axis bound of the scheme
  double tau_min = c->fl.rho_p * c->d_min * c->d_min / (18.0 * c->fl.mu);
  double bound = o->rk == 0 ? 4.65 : 2.51;
  if (o->drag != 2 && c->np > 0 && dt > bound * tau_min) {
    c->err = "fp_step: dt exceeds the drag stability bound";
    return FP_WDT;
  }
  return FP_OK;
}

// reference coordinates of every active particle's position: along the
// element tasks of the step's sort when they still describe the particle
// order (the stages do not reorder), the rest per lane
static hipError_t finalize(fp_ctx* c, hipStream_t s) {
  const int warm = c->xi_warm ? 1 : 0;
  const Particles& P = c->P[c->cur];
  if (c->tasks_valid)
    return launch_finalize_elem(c->mv, P, c->tasks, c->qcnt + 4, c->task_tp, c->np, warm, c->qcnt, c->strag,
                                c->stats, s);
  return launch_finalize(c->mv, P, c->np, nullptr, nullptr, warm, c->stats, s);
}

int fp_deposit_source(fp_ctx* c, void* S, fp_dtype dt, int32_t kind, double radius, const double* period,
                      int32_t drag, int32_t forces, const double* gravity) {
  if (!c || !S || kind < 0 || kind > 1 || drag < 0 || drag > 2 || (forces & ~kForceAll) != 0) return FP_EINVAL;
  if (!c->ws || !c->fluid_ok) return fail(c, FP_ESTATE, "fp_deposit_source: workspace or fluid state missing");
  ForceModel fm{};
  fm.drag = drag;
  fm.forces = forces;
  for (int k = 0; k < 3; ++k) fm.gravity[k] = gravity ? gravity[k] : 0.0;
  if (kind == 1) {
    if (!(radius > 0.0)) return fail(c, FP_EINVAL, "fp_deposit_source: radius must be positive");
    for (int k = 0; k < 3; ++k)
      if (period && period[k] > 0.0 && period[k] <= 2.0 * radius)
        return fail(c, FP_EINVAL, "fp_deposit_source: a period must exceed twice the kernel radius");
  }
  // the source belongs to the element that contains each particle at the end
  // of the last step: locate them first (a segment that was not traced, or a
  // crossing the face intersection missed, leaves the old element recorded)
  if (c->xi_dirty && c->np > 0) {
    Timed tm(c, 2);
    HIPCHK(c, finalize(c, c->stream));
    c->xi_dirty = false;
    c->sorted_fresh = false;
  }
  if (kind == 0) {
    Timed tm(c, 3);
    HIPCHK(c, launch_deposit_nearest(c->mv, c->P[c->cur], c->fl, c->np, S, dt == FP_F32, fm, c->stream));
    return FP_OK;
  }
  double per[3] = {0, 0, 0};
  if (period)
    for (int k = 0; k < 3; ++k) per[k] = period[k];
  if (c->np == 0) return FP_OK;
  // FP32 source: candidate lists for this radius and these periods, built
  // once (they depend on the mesh only); over budget, the kernels search
  if (dt == FP_F32 && (!c->dl_tried || c->dl_R != radius || c->dl_per[0] != per[0] || c->dl_per[1] != per[1] ||
                       c->dl_per[2] != per[2])) {
    Timed tm(c, 4);
    c->dl_tried = true;
    c->dl_valid = false;
    c->dl_R = radius;
    for (int k = 0; k < 3; ++k) c->dl_per[k] = per[k];
    c->dl_pad = 0.05 * c->max_extent;
    HIPCHK(c, launch_dep_lists(c->mv, radius, per, c->dl_pad, 0, c->dl_count, nullptr, nullptr, c->stream));
    HIPCHK(c, scan_i32(c->dl_count, c->dl_start, (int64_t)c->E + 1, c->sort_sums, c->stream));
    int32_t total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, c->dl_start + c->E, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // entries pack the element in 27 bits
    if (total >= 0 && (size_t)total <= (size_t)c->E * kDepListPerElem && c->E < (1 << 27)) {
      HIPCHK(c, launch_dep_lists(c->mv, radius, per, c->dl_pad, 1, nullptr, c->dl_start, c->dl_list, c->stream));
      c->dl_valid = true;
    }
  }
  // gather needs the particles bucketed by their current element (tasks for
  // the stage that ran last)
  int rc = sort_particles(c, c->task_tp);
  if (rc) return rc;
  {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (c->timing)
      for (int k = 0; k < 4; ++k) ev[k] = take_event(c);
    {
      Timed tm(c, 4);
      HIPCHK(c, launch_deposit_shape(c->mv, c->P[c->cur], c->fl, c->np, S, dt == FP_F32, fm, radius, per,
                                     c->node_pad, c->dep_buf, c->sort_start, c->dep_pad,
                                     c->count_pairs ? c->stats + ST_DEP_PAIRS * kStatSlots : nullptr, c->dl_valid ? c->dl_start : nullptr,
                                     c->dl_list, c->dl_pad, c->rl_buf, c->rl_cap,
                                     c->tasks_valid ? c->tasks : nullptr, c->qcnt + 4, c->task_tp, ev, c->stream));
    }
    if (c->timing && ev[0] && ev[1] && ev[2] && ev[3]) {
      c->recs.push_back({7, ev[0], ev[1]});
      c->recs.push_back({8, ev[2], ev[3]});
    }
  }
  return sync_bound(c);
}

int fp_node_volumes(fp_ctx* c, double* V) {
  if (!c || !V) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_node_volumes: no workspace");
  size_t bytes = (size_t)c->E * c->n * c->n * c->n * sizeof(double);
  HIPCHK(c, hipMemcpyAsync(V, c->mv.vol, bytes, hipMemcpyDeviceToDevice, c->stream));
  return FP_OK;
}

int fp_read_particles(fp_ctx* c, int64_t* n_out, double* x, double* v, int32_t* elem, double* xi,
                      int32_t* hits, int8_t* status) {
  if (!c) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_read_particles: no workspace");
  hipStream_t s = c->stream;
  int64_t n = c->np;
  if (n_out) *n_out = n;
  if (n == 0) return FP_OK;
  Particles& P = c->P[c->cur];
  const int64_t cap = P.cap;
  if (c->xi_dirty) {
    Timed tm(c, 2);
    HIPCHK(c, finalize(c, s));
    c->xi_dirty = false;
    c->sorted_fresh = false;
  }
  std::vector<double> hx((size_t)n * 3), hv((size_t)n * 3), hxi((size_t)n * 3);
  std::vector<int32_t> he(n), hh(n), hid(n);
  std::vector<int8_t> hs(n);
  for (int k = 0; k < 3; ++k) {
    HIPCHK(c, hipMemcpyAsync(hx.data() + k * n, P.x + k * cap, n * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(hv.data() + k * n, P.v + k * cap, n * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(hxi.data() + k * n, P.xi + k * cap, n * 8, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(c, hipMemcpyAsync(he.data(), P.elem, n * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(hh.data(), P.hits, n * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(hid.data(), P.id, n * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(hs.data(), P.status, n, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (int64_t q = 0; q < n; ++q) {
    int64_t p = hid[q];
    if (p < 0 || p >= n) return fail(c, FP_EDEVICE, "fp_read_particles: corrupt particle ids");
    for (int k = 0; k < 3; ++k) {
      if (x) x[p * 3 + k] = hx[k * n + q];
      if (v) v[p * 3 + k] = hv[k * n + q];
      if (xi) xi[p * 3 + k] = hxi[k * n + q];
    }
    if (elem) elem[p] = he[q];
    if (hits) hits[p] = hh[q];
    if (status) status[p] = hs[q];
  }
  return FP_OK;
}

int fp_get_stats(fp_ctx* c, int64_t* out) {
  static_assert(ST_N <= 16, "the stats area holds 16 counters");
  if (!c || !out) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_get_stats: no workspace");
  std::vector<unsigned long long> slots((size_t)ST_N * kStatSlots);
  HIPCHK(c, hipMemcpyAsync(slots.data(), c->stats, slots.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  unsigned long long h[ST_N] = {0};
  for (int k = 0; k < ST_N; ++k)
    for (int j = 0; j < kStatSlots; ++j) h[k] += slots[(size_t)k * kStatSlots + j];
  for (int i = 0; i < 6; ++i) out[i] = (int64_t)h[i];
  out[6] = c->sorts;
  out[7] = (int64_t)h[ST_STRAG];
  out[8] = (int64_t)h[ST_TRACKQ];
  out[9] = (int64_t)h[ST_RECOVER];
  out[10] = (int64_t)h[ST_DEP_PAIRS];
  return FP_OK;
}

int fp_reset_stats(fp_ctx* c) {
  if (!c) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_reset_stats: no workspace");
  HIPCHK(c, hipMemsetAsync(c->stats, 0, 16 * kStatSlots * 8, c->stream));
  c->sorts = 0;
  return FP_OK;
}

int fp_set_timing(fp_ctx* c, int32_t enable) {
  if (!c) return FP_EINVAL;
  c->timing = (enable & 1) != 0;
  c->count_pairs = (enable & 2) != 0;
  return FP_OK;
}

int fp_get_timing(fp_ctx* c, double* out) {
  if (!c || !out) return FP_EINVAL;
  for (int k = 0; k < 2 * FP_TIMING_CLASSES; ++k) out[k] = 0.0;
  for (auto& r : c->recs) {
    HIPCHK(c, hipEventSynchronize(r.b));
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, r.a, r.b));
    out[2 * r.cls] += 1.0;
    out[2 * r.cls + 1] += ms;
  }
  c->recs.clear();
  c->ev_used = 0;
  return FP_OK;
}

// ---- learned guess --------------------------------------------------------
int64_t fp_mlp_n_weights(void) { return kMlpWeights; }

int fp_mlp_features(fp_ctx* c, int64_t n, const int32_t* elem, const double* x, float* feat) {
  if (!c || n < 0 || (n > 0 && (!elem || !x || !feat))) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_mlp_features: no workspace");
  HIPCHK(c, launch_mlp_features(c->mv, n, elem, x, feat, c->stream));
  return FP_OK;
}

int fp_newton_pairs(fp_ctx* c, int64_t* n_out, float* feat, float* xi, int32_t* ids, int64_t capacity) {
  if (!c || !n_out || !feat || !xi) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_newton_pairs: no workspace");
  if (capacity < c->np) return fail(c, FP_EINVAL, "fp_newton_pairs: capacity below particle count");
  HIPCHK(c, hipMemsetAsync(c->scratch_i32, 0, 4, c->stream));
  HIPCHK(c, launch_newton_pairs(c->mv, c->P[c->cur], c->np, feat, xi, ids, c->scratch_i32, c->stream));
  int32_t cnt = 0;
  HIPCHK(c, hipMemcpyAsync(&cnt, c->scratch_i32, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *n_out = cnt;
  return FP_OK;
}

int fp_mlp_forward(fp_ctx* c, const float* w, int64_t n, const float* in, float* out) {
  if (!c || !w || n < 0 || (n > 0 && (!in || !out))) return FP_EINVAL;
  HIPCHK(c, launch_mlp_forward(w, n, in, out, c->stream));
  return FP_OK;
}

int fp_mlp_loss_grad(fp_ctx* c, const float* w, int64_t n, const float* in, const float* target, float* grad,
                     float* loss) {
  if (!c || !w || n <= 0 || !in || !target || !grad || !loss) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_mlp_loss_grad: no workspace");
  if (n > kMlpMaxBatch) return fail(c, FP_EINVAL, "fp_mlp_loss_grad: at most 8192 rows per call");
  HIPCHK(c, launch_mlp_loss_grad(w, n, in, target, nullptr, grad, loss, c->mlp_rows, c->stream));
  return FP_OK;
}

int fp_mlp_loss_grad_static(fp_ctx* c, const float* w, int64_t n, const float* in, const float* target,
                            float* grad, float* loss) {
  if (!c || !w || !in || !target || !grad || !loss) return FP_EINVAL;
  if (n <= 0 || n > FP_MLP_STATIC_ROWS)
    return fail(c, FP_EINVAL, "fp_mlp_loss_grad_static: n must be in [1, FP_MLP_STATIC_ROWS]");
  float* rows = nullptr;
  HIPCHK(c, mlp_static_rows(&rows));
  HIPCHK(c, launch_mlp_loss_grad(w, n, in, target, nullptr, grad, loss, rows, c->stream));
  return FP_OK;
}

int fp_mlp_train_epoch(fp_ctx* c, float* w, float* m, float* v, int64_t* t, const float* in, const float* target,
                       const int32_t* order, int64_t n, int32_t batch, float lr, float* loss) {
  if (!c || !w || !m || !v || !t || !in || !target || !order || n <= 0 || batch <= 0) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_mlp_train_epoch: no workspace");
  if (batch > kMlpMaxBatch) return fail(c, FP_EINVAL, "fp_mlp_train_epoch: batch above 8192");
  int64_t nw = fp_mlp_n_weights();
  float* grad = c->mlp_grad;
  float* lbuf = grad + nw;
  int64_t nb = n / batch;
  for (int64_t bi = 0; bi < nb; ++bi) {
    HIPCHK(c, launch_mlp_loss_grad(w, batch, in, target, order + bi * batch, grad,
                                   loss ? loss + bi : lbuf, c->mlp_rows, c->stream));
    (*t)++;
    HIPCHK(c, launch_adam(w, m, v, grad, nw, *t, lr, c->stream));
  }
  return FP_OK;
}

int fp_mlp_set_weights(fp_ctx* c, const float* w, double thresh) {
  if (!c) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_mlp_set_weights: no workspace");
  if (!w) {
    c->mlp_w = nullptr;
    c->mv.mlp_w = nullptr;
    c->n_flagged = 0;
    return FP_OK;
  }
  // the guess uses a copy: later changes of w (training in place) do not
  // reach the stage kernels or the per-element first-layer table
  if (w != c->mlp_wbuf)
    HIPCHK(c, hipMemcpyAsync(c->mlp_wbuf, w, (size_t)kMlpWeights * 4, hipMemcpyDeviceToDevice, c->stream));
  c->mlp_w = c->mlp_wbuf;
  c->mv.mlp_w = c->mlp_wbuf;
  HIPCHK(c, hipMemsetAsync(c->scratch_i32, 0, 4, c->stream));
  HIPCHK(c, launch_curved_flags(c->mv, thresh, c->mlp_flag, c->scratch_i32, c->stream));
  HIPCHK(c, launch_mlp_elem_table(c->mv, c->mlp_wbuf, (float*)c->mv.mlp_h1, (double*)c->mv.mlp_ctr, c->stream));
  int32_t cnt = 0;
  HIPCHK(c, hipMemcpyAsync(&cnt, c->scratch_i32, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->n_flagged = cnt;
  return FP_OK;
}

int fp_mlp_train(fp_ctx* c, const float* in, const float* target, int64_t n, int32_t epochs, int32_t batch,
                 float lr, uint64_t seed, float* w_out, float* loss_hist) {
  if (!c || !in || !target || !w_out || n <= 0 || epochs < 0 || batch <= 0) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_mlp_train: no workspace");
  if (batch > kMlpMaxBatch) return fail(c, FP_EINVAL, "fp_mlp_train: batch above 8192");
  if (n > c->cap) return fail(c, FP_EINVAL, "fp_mlp_train: more rows than the workspace's particle capacity");
  if (n < batch) return fail(c, FP_EINVAL, "fp_mlp_train: fewer rows than one batch");
  hipStream_t s = c->stream;
  const int64_t nw = kMlpWeights, nb = n / batch;
  SplitMix64 g{seed};
  std::vector<float> w0((size_t)nw);
  mlp_xavier(g, w0);
  HIPCHK(c, hipMemcpyAsync(w_out, w0.data(), nw * 4, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemsetAsync(c->mlp_adam, 0, (size_t)nw * 2 * 4, s));
  std::vector<int32_t> order((size_t)n);
  std::vector<float> bl((size_t)nb);
  int64_t t = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
    shuffle(g, order);
    // the previous epoch's copy of `order` must be done before it is reused
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipMemcpyAsync(c->mlp_order, order.data(), n * 4, hipMemcpyHostToDevice, s));
    for (int64_t bi = 0; bi < nb; ++bi) {
      HIPCHK(c, launch_mlp_loss_grad(w_out, batch, in, target, c->mlp_order + bi * batch, c->mlp_grad,
                                     c->mlp_bloss + bi, c->mlp_rows, s));
      ++t;
      HIPCHK(c, launch_adam(w_out, c->mlp_adam, c->mlp_adam + nw, c->mlp_grad, nw, t, lr, s));
    }
    if (loss_hist) {
      HIPCHK(c, hipMemcpyAsync(bl.data(), c->mlp_bloss, nb * 4, hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      double sum = 0.0;
      for (int64_t bi = 0; bi < nb; ++bi) sum += bl[bi];
      loss_hist[ep] = (float)(sum / nb);
    }
  }
  HIPCHK(c, hipStreamSynchronize(s));
  return FP_OK;
}

int fp_particle_block_layout(int64_t capacity, fp_dtype dtype, int64_t* offsets, size_t* bytes) {
  if (capacity <= 0 || !bytes || dtype != FP_F64) return FP_EINVAL;
  int64_t off[10];
  size_t total;
  particle_offsets(capacity, off, &total);
  if (offsets)
    for (int a = 0; a < 10; ++a) offsets[a] = off[a];
  *bytes = total;
  return FP_OK;
}

int fp_bind_particles(fp_ctx* c, int64_t capacity, fp_dtype dtype, void* soa) {
  if (!c) return FP_EINVAL;
  if (!c->ws) return fail(c, FP_ESTATE, "fp_bind_particles: no workspace");
  if (!soa) {   // back to the workspace's own particle buffer
    c->P[0] = carve(c->part0, c->cap);
    c->bound = false;
    c->np = 0;
    c->cur = 0;
    c->tasks_valid = false;
    return FP_OK;
  }
  if (dtype != FP_F64)
    return fail(c, FP_EINVAL, "fp_bind_particles: the particle block is FP64 in both precisions");
  if (capacity <= 0 || capacity > c->cap)
    return fail(c, FP_EINVAL, "fp_bind_particles: capacity must be in (0, workspace particle capacity]");
  if (((uintptr_t)soa) & 255) return fail(c, FP_EINVAL, "fp_bind_particles: block not 256-byte aligned");
  c->P[0] = carve((char*)soa, capacity);
  c->bound = true;
  c->np = 0;
  c->cur = 0;
  c->tasks_valid = false;
  return FP_OK;
}

int fp_deposit_list_bytes(fp_ctx* c, int32_t cap, size_t* bytes) {
  if (!c || !bytes || cap <= 0) return FP_EINVAL;
  if (!c->mesh_ok) return fail(c, FP_ESTATE, "fp_deposit_list_bytes: no mesh");
  *bytes = deposit_reuse_bytes(c->E, cap);
  return FP_OK;
}

int fp_bind_deposit_list(fp_ctx* c, void* dev, size_t bytes) {
  if (!c) return FP_EINVAL;
  if (!c->mesh_ok) return fail(c, FP_ESTATE, "fp_bind_deposit_list: no mesh");
  if (!dev) {
    c->rl_buf = nullptr;
    c->rl_cap = 0;
    return FP_OK;
  }
  if (((uintptr_t)dev) & 255) return fail(c, FP_EINVAL, "fp_bind_deposit_list: memory not 256-byte aligned");
  const size_t head = deposit_reuse_bytes(c->E, 0);
  const size_t cap = bytes > head ? (bytes - head) / ((size_t)c->E * 16) : 0;
  if (cap < 16) return fail(c, FP_EINVAL, "fp_bind_deposit_list: fewer than 16 rows per element");
  c->rl_buf = dev;
  c->rl_cap = (int32_t)std::min<size_t>(cap, (size_t)INT32_MAX / 2);
  return FP_OK;
}

int fp_mlp_num_flagged(fp_ctx* c, int64_t* n) {
  if (!c || !n) return FP_EINVAL;
  *n = c->n_flagged;
  return FP_OK;
}

}  // extern "C"

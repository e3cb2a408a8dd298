// Two-way coupling source with a polynomial shape kernel K(r) = (1-(r/R)^2)^2
// over all DG nodes within R of a particle, normalised per particle so that
// sum_k S_k V_k = -F (the projection keeps the conservation property of the
// nearest-DOF operator of Sec. 2.3 while spreading the source).
//
// Three kernels, no atomics on the source itself:
//  1. per particle: drag force F and a validity flag;
//  2. per source element (one workgroup): the normalisation sum_j K(r_j) V_j
//     of each of its particles.  Lanes hold the DG nodes of one candidate
//     target element; the test "particle within R of the target's node box"
//     is uniform over the wave, so far pairs cost one branch.  F is replaced
//     in place by G = -F / norm;
//  3. per target element (one workgroup, one thread per DG node): candidate
//     source particles are staged through LDS in chunks, culled against the
//     target's node box, and every node accumulates K(r) G.
// Candidate elements come from the background mesh and are streamed through
// LDS in windows, so no element count is limited by LDS capacity.
// Workgroups are mapped to elements XCD by XCD (contiguous element ranges per
// XCD), so neighbouring elements share an L2.
#include "fp_device.h"
#include "fp_launch.h"

namespace fp {

namespace {

constexpr int kNormThreads = 128;    // k_dep_norm: two wavefronts per source element
constexpr int kGatherThreads = 128;  // k_dep_gather: each thread holds several target nodes
constexpr int kDepCand = 256;        // candidate elements per LDS window
constexpr int kNormChunk = 32;       // particles per normalisation pass
constexpr int kXcd = 8;

struct DepGeo {
  double R, R2, iR;   // radius, its square and its inverse
  double node_pad;     // largest distance of a DG node outside its element box
  double period[3];
};

template <int TH>
struct CandLds {
  int32_t e[kDepCand];
  int8_t img[kDepCand];        // ((iz+1)*3 + (iy+1))*3 + (ix+1)
  int32_t wsum[TH / 64];
};

__device__ __forceinline__ int xcd_element(int b, int E) {
  int per = (E + kXcd - 1) / kXcd;
  return (b % kXcd) * per + b / kXcd;
}

__device__ __forceinline__ void image_shift(int code, const double* period, double* s) {
  s[0] = (code % 3 - 1) * period[0];
  s[1] = ((code / 3) % 3 - 1) * period[1];
  s[2] = (code / 9 - 1) * period[2];
}

// squared distance from x to the box [lo, hi]
__device__ __forceinline__ double box_dist2(const double* x, const double* lo, const double* hi) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double d = fmax(fmax(lo[k] - x[k], x[k] - hi[k]), 0.0);
    s += d * d;
  }
  return s;
}

__device__ __forceinline__ int lane_rank(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// exclusive prefix sum over the workgroup of TH threads; every thread must call it
template <int TH>
__device__ inline int block_excl_scan(int v, int32_t* wsum, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < TH / 64; ++k) {
    int t = wsum[k];
    base += (k < w) ? t : 0;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + x - v;
}

// Every element whose (padded) box overlaps [lo - pad, hi + pad], or a periodic
// image of that box shifted by +img * period, is passed exactly once (in the
// first background cell of the overlap) to body(count), in windows of at most
// kDepCand entries held in L.e / L.img.  Order is deterministic.  All threads
// of the workgroup must call it with the same arguments.
template <int TH, class Body>
__device__ __forceinline__ void stream_candidates(const MeshView& m, const double* period, const double* lo,
                                                  const double* hi, double pad, CandLds<TH>& L, Body&& body) {
  for (int code = 0; code < 27; ++code) {
    const int im[3] = {code % 3 - 1, (code / 3) % 3 - 1, code / 9 - 1};
    bool skip = false;
    double qlo[3], qhi[3];
    int c0[3], c1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (im[k] != 0 && !(period[k] > 0.0)) skip = true;
      qlo[k] = lo[k] + im[k] * period[k] - pad;
      qhi[k] = hi[k] + im[k] * period[k] + pad;
      c0[k] = max((int)floor((qlo[k] - m.blo[k]) / m.bdx[k]), 0);
      c1[k] = min((int)floor((qhi[k] - m.blo[k]) / m.bdx[k]), m.bn[k] - 1);
      if (c0[k] > c1[k]) skip = true;
    }
    if (skip) continue;
    const int nx = c1[0] - c0[0] + 1, ny = c1[1] - c0[1] + 1, nz = c1[2] - c0[2] + 1;
    const int ncell = nx * ny * nz;
    for (int cb = 0; cb < ncell; cb += TH) {
      const int ci = cb + threadIdx.x;
      int own[3] = {0, 0, 0}, beg = 0, end = 0;
      if (ci < ncell) {
        own[0] = c0[0] + ci % nx;
        own[1] = c0[1] + (ci / nx) % ny;
        own[2] = c0[2] + ci / (nx * ny);
        int64_t cell = ((int64_t)own[2] * m.bn[1] + own[1]) * m.bn[0] + own[0];
        beg = m.bstart[cell];
        end = m.bstart[cell + 1];
      }
      auto accept = [&](int e) {
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double el = m.elo[e * 3 + k];
          int ec = max((int)floor((el - m.blo[k]) / m.bdx[k]), 0);
          if (own[k] != max(c0[k], ec)) ok = false;
          if (el > qhi[k] || m.ehi[e * 3 + k] < qlo[k]) ok = false;
        }
        return ok;
      };
      int cnt = 0;
      for (int q = beg; q < end; ++q) cnt += accept(m.blist[q]) ? 1 : 0;
      int tot = 0;
      const int off = block_excl_scan<TH>(cnt, L.wsum, tot);
      for (int w0 = 0; w0 < tot; w0 += kDepCand) {
        if (cnt > 0 && off < w0 + kDepCand && off + cnt > w0) {
          int r = off;
          for (int q = beg; q < end; ++q) {
            int e = m.blist[q];
            if (!accept(e)) continue;
            if (r >= w0 && r < w0 + kDepCand) {
              L.e[r - w0] = e;
              L.img[r - w0] = (int8_t)code;
            }
            ++r;
          }
        }
        __syncthreads();
        body(min(tot - w0, kDepCand));
        __syncthreads();
      }
    }
  }
}

// 1. force and validity ------------------------------------------------------
template <int NN, int NG, typename UT>
__global__ __launch_bounds__(256) void k_dep_force(MeshView m, Particles P, Fluid fl, int64_t n, ForceModel fm,
                                                   double* F, int32_t* ok, unsigned long long* povh) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double* Fp = F + p * 4;
  Fp[0] = Fp[1] = Fp[2] = Fp[3] = 0.0;
  ok[p] = 0;
  if (P.status[p] != ACTIVE) return;
  const int64_t cap = P.cap;
  int e = P.elem[p];
  double x[3] = {P.x[p], P.x[cap + p], P.x[2 * cap + p]};
  {
    // largest distance of a particle outside its element's box: the candidate
    // searches pad the element boxes by it
    double ov = 0.0;
    for (int k = 0; k < 3; ++k) ov = fmax(ov, fmax(m.elo[e * 3 + k] - x[k], x[k] - m.ehi[e * 3 + k]));
    if (ov > 0.0) atomicMax(povh, (unsigned long long)__double_as_longlong(ov));
  }
  // the caller has located every particle (reference coordinates in P.xi)
  const double xi[3] = {P.xi[p], P.xi[cap + p], P.xi[2 * cap + p]};
  if (!inside_ref(xi)) return;
  double v[3] = {P.v[p], P.v[cap + p], P.v[2 * cap + p]};
  double Fq[3];
  source_force<NN, NG, UT>(m, fl, fm, e, xi, v, P.d[p], Fq);
  Fp[0] = Fq[0];
  Fp[1] = Fq[1];
  Fp[2] = Fq[2];
  Fp[3] = Fq[0] * v[0] + Fq[1] * v[1] + Fq[2] * v[2];
  ok[p] = 1;
}

// 2. normalisation per source element ---------------------------------------
// For each window of candidate targets the chunk's particles are first tested
// against every target's node box (two targets per wave instruction, one
// particle per lane); targets with no particle within R go no further, and
// the others form a list that the wavefronts share, so node data is fetched
// only for targets that contribute.  Each lane keeps its partial sums in its
// own LDS column (s_acc[wave][i][lane]), and the next listed target's nodes
// are loaded while the current one is evaluated.  Distances are taken in
// units of R, so K = max(1 - |d|^2, 0)^2 needs no cut-off test.
template <int NN>
__global__ __launch_bounds__(kNormThreads) void k_dep_norm(MeshView m, Particles P,
                                                           const int32_t* __restrict__ elem_start, DepGeo g,
                                                           double* F, const int32_t* __restrict__ ok,
                                                           unsigned long long* povh) {
  constexpr int TH = kNormThreads, NW = TH / 64, CH = kNormChunk;
  static_assert(CH <= 32, "a ballot holds the masks of two targets");
  const int es = xcd_element(blockIdx.x, m.E);
  if (es >= m.E) return;
  const int p0 = elem_start[es], p1 = elem_start[es + 1];
  if (p0 == p1) return;
  constexpr int N3 = NN * NN * NN;
  constexpr int NPL = (N3 + 63) / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t cap = P.cap;
  __shared__ CandLds<TH> L;
  __shared__ double s_x[CH][3];     // positions
  __shared__ double s_xs[CH][3];    // positions / R
  __shared__ double s_acc[NW][CH][64];
  __shared__ uint32_t s_mask[kDepCand];
  __shared__ int32_t s_list[kDepCand];
  __shared__ double s_q[6];
  __shared__ int s_any;
  for (int c0 = p0; c0 < p1; c0 += CH) {
    const int cnt = min(CH, p1 - c0);
    if (threadIdx.x < CH) {
      const int i = threadIdx.x;
      double x[3] = {1e300, 1e300, 1e300};
      if (i < cnt && ok[c0 + i]) {
        const int64_t p = c0 + i;
        x[0] = P.x[p]; x[1] = P.x[cap + p]; x[2] = P.x[2 * cap + p];
        double ov = 0.0;
        for (int k = 0; k < 3; ++k)
          ov = fmax(ov, fmax(m.elo[es * 3 + k] - x[k], x[k] - m.ehi[es * 3 + k]));
        if (ov > 0.0) atomicMax(povh, (unsigned long long)__double_as_longlong(ov));
      }
      for (int k = 0; k < 3; ++k) {
        s_x[i][k] = x[k];
        s_xs[i][k] = x[k] * g.iR;
      }
    }
    for (int i = 0; i < CH; ++i) s_acc[wave][i][lane] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      int any = 0;
      for (int i = 0; i < cnt; ++i)
        if (s_x[i][0] < 1e299) {
          any = 1;
          for (int k = 0; k < 3; ++k) { lo[k] = fmin(lo[k], s_x[i][k]); hi[k] = fmax(hi[k], s_x[i][k]); }
        }
      for (int k = 0; k < 3; ++k) { s_q[k] = lo[k]; s_q[3 + k] = hi[k]; }
      s_any = any;
    }
    __syncthreads();
    if (!s_any) continue;   // uniform
    double qlo[3] = {s_q[0], s_q[1], s_q[2]}, qhi[3] = {s_q[3], s_q[4], s_q[5]};
    stream_candidates<TH>(m, g.period, qlo, qhi, g.R + g.node_pad, L, [&](int nc) {
      // particle masks: lanes 0..31 test target t0, lanes 32..63 target t0 + 1
      for (int t0 = 2 * wave; t0 < nc; t0 += 2 * NW) {
        const int t = t0 + (lane >> 5), i = lane & 31;
        bool near = false;
        if (t < nc && i < CH) {
          double sh[3];
          image_shift(L.img[t], g.period, sh);
          const double* nb = m.nbox + (size_t)L.e[t] * 6;
          const double blo[3] = {nb[0] - sh[0], nb[1] - sh[1], nb[2] - sh[2]};
          const double bhi[3] = {nb[3] - sh[0], nb[4] - sh[1], nb[5] - sh[2]};
          const double px[3] = {s_x[i][0], s_x[i][1], s_x[i][2]};
          near = box_dist2(px, blo, bhi) < g.R2;
        }
        const unsigned long long bal = __ballot(near);
        if (lane == 0) s_mask[t0] = (uint32_t)bal;
        if (lane == 32 && t < nc) s_mask[t] = (uint32_t)(bal >> 32);
      }
      __syncthreads();
      int nl = 0;
      for (int cb = 0; cb < nc; cb += TH) {
        const int c = cb + threadIdx.x;
        const int f = (c < nc && s_mask[c] != 0u) ? 1 : 0;
        int tot = 0;
        const int off = block_excl_scan<TH>(f, L.wsum, tot);
        if (f) s_list[nl + off] = c;
        nl += tot;
      }
      __syncthreads();
      // two register sets in turn: one target is evaluated while the next
      // one's nodes are in flight
      // Lanes past the last node load the last node again (every lane issues
      // the same loads, so the wait for one set never waits for the other)
      // and contribute with zero volume.
      double xa[NPL][3], va[NPL], xb[NPL][3], vb[NPL];
      auto load = [&](int t, double (&X)[NPL][3], double (&V)[NPL]) {
        const size_t e = (size_t)L.e[t];
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
          const int q = min(lane + 64 * j, N3 - 1);
          const double* src = m.xnode + (e * N3 + q) * 3;
          X[j][0] = src[0]; X[j][1] = src[1]; X[j][2] = src[2];
          V[j] = m.vol[e * N3 + q];
        }
      };
      auto eval = [&](int t, const double (&X)[NPL][3], const double (&V)[NPL]) {
        // nodes in units of R, shifted into the particles' periodic image
        double sh[3], xs[NPL][3], vv[NPL];
        image_shift(L.img[t], g.period, sh);
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
#pragma unroll
          for (int k = 0; k < 3; ++k) xs[j][k] = (X[j][k] - sh[k]) * g.iR;
          vv[j] = (lane + 64 * j < N3) ? V[j] : 0.0;
        }
        uint32_t mask = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_mask[t]);
        for (; mask; mask &= mask - 1u) {
          const int i = __builtin_ctz(mask);
          const double ps0 = s_xs[i][0], ps1 = s_xs[i][1], ps2 = s_xs[i][2];
          double a = 0.0;
#pragma unroll
          for (int j = 0; j < NPL; ++j) {
            const double d0 = xs[j][0] - ps0, d1 = xs[j][1] - ps1, d2 = xs[j][2] - ps2;
            double w = fma(-d0, d0, fma(-d1, d1, fma(-d2, d2, 1.0)));
            w = fmax(w, 0.0);
            a = fma(w * vv[j], w, a);
          }
          // each lane owns its column, so the no-return LDS add keeps the
          // summation order fixed while hiding the read-modify-write latency
          __hip_atomic_fetch_add(&s_acc[wave][i][lane], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      };
      // the prefetch is issued on every path (past the list's end it loads
      // the last target again), so its loads are always the newest in flight
      if (wave < nl) load(s_list[wave], xa, va);
      for (int jl = wave; jl < nl; jl += 2 * NW) {
        load(s_list[min(jl + NW, nl - 1)], xb, vb);
        eval(s_list[jl], xa, va);
        if (jl + NW >= nl) break;
        load(s_list[min(jl + 2 * NW, nl - 1)], xa, va);
        eval(s_list[jl + NW], xb, vb);
      }
    });
    // sum over waves and lanes: TH / CH threads per particle, fixed order
    {
      constexpr int TPP = TH / CH;
      const int i = threadIdx.x / TPP, sub = threadIdx.x % TPP;
      double v = 0.0;
      for (int w = 0; w < NW; ++w)
        for (int l = sub; l < 64; l += TPP) v += s_acc[w][i][l];
#pragma unroll
      for (int off = TPP / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (sub == 0 && i < cnt) {
        const int64_t p = c0 + i;
        double* Fp = F + p * 4;
        const bool use = ok[p] && v > 0.0;
        const double in = use ? -1.0 / v : 0.0;
        for (int k = 0; k < 4; ++k) Fp[k] = use ? Fp[k] * in : 0.0;
      }
    }
    __syncthreads();
  }
}

// 3. gather per target element ----------------------------------------------
// Each thread holds PER target nodes, so every staged particle read from LDS
// serves PER kernel evaluations.  Nodes and particles are held in units of R.
template <int NN, typename ST>
__global__ __launch_bounds__(kGatherThreads) void k_dep_gather(MeshView m, Particles P,
                                                               const int32_t* __restrict__ elem_start, DepGeo g,
                                                               const double* __restrict__ G,
                                                               const unsigned long long* __restrict__ povh, ST* S) {
  constexpr int TH = kGatherThreads, NW = TH / 64;
  const int t = xcd_element(blockIdx.x, m.E);
  if (t >= m.E) return;
  constexpr int N3 = NN * NN * NN;
  constexpr int PER = (N3 + TH - 1) / TH;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t cap = P.cap;
  __shared__ CandLds<TH> L;
  __shared__ int32_t s_pre[kDepCand + 1];
  __shared__ double s_px[TH][3];
  __shared__ double s_pg[TH][4];
  __shared__ int32_t s_wcnt[NW];
  double xn[PER][3], acc[PER][4];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int q = threadIdx.x + s * TH;
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[s][k] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) xn[s][k] = (q < N3) ? m.xnode[((size_t)t * N3 + q) * 3 + k] * g.iR : 1e300;
  }
  const double* nb = m.nbox + (size_t)t * 6;
  const double blo[3] = {nb[0], nb[1], nb[2]}, bhi[3] = {nb[3], nb[4], nb[5]};
  const double part_pad = __longlong_as_double((long long)*povh);
  stream_candidates<TH>(m, g.period, blo, bhi, g.R + part_pad, L, [&](int nc) {
    // prefix over the candidates' particle counts (windows hold <= kDepCand)
    int T = 0;
    for (int cb = 0; cb < nc; cb += TH) {
      const int c = cb + threadIdx.x;
      const int cntc = (c < nc) ? elem_start[L.e[c] + 1] - elem_start[L.e[c]] : 0;
      int tot = 0;
      const int off = block_excl_scan<TH>(cntc, L.wsum, tot);
      if (c < nc) s_pre[c] = T + off;
      T += tot;
    }
    __syncthreads();
    for (int jb = 0; jb < T; jb += TH) {
      const int j = jb + threadIdx.x;
      bool keep = false;
      double px[3] = {0, 0, 0}, pg[4] = {0, 0, 0, 0};
      if (j < T) {
        int lo = 0, hi = nc - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[mid] <= j) lo = mid;
          else hi = mid - 1;
        }
        const int e = L.e[lo];
        const int64_t p = elem_start[e] + (j - s_pre[lo]);
        double sh[3];
        image_shift(L.img[lo], g.period, sh);
        px[0] = P.x[p] - sh[0];
        px[1] = P.x[cap + p] - sh[1];
        px[2] = P.x[2 * cap + p] - sh[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) pg[k] = G[p * 4 + k];
        keep = (pg[0] != 0.0 || pg[1] != 0.0 || pg[2] != 0.0 || pg[3] != 0.0) && box_dist2(px, blo, bhi) < g.R2;
      }
      const unsigned long long bal = __ballot(keep);
      if (lane == 0) s_wcnt[wave] = (int)__popcll(bal);
      __syncthreads();
      int base = 0, nk = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        base += (w < wave) ? s_wcnt[w] : 0;
        nk += s_wcnt[w];
      }
      if (keep) {
        const int slot = base + lane_rank(bal);
#pragma unroll
        for (int k = 0; k < 3; ++k) s_px[slot][k] = px[k] * g.iR;
#pragma unroll
        for (int k = 0; k < 4; ++k) s_pg[slot][k] = pg[k];
      }
      __syncthreads();
#pragma unroll 4
      for (int k = 0; k < nk; ++k) {
        const double x0 = s_px[k][0], x1 = s_px[k][1], x2 = s_px[k][2];
        const double g0 = s_pg[k][0], g1 = s_pg[k][1], g2 = s_pg[k][2], g3 = s_pg[k][3];
#pragma unroll
        for (int s = 0; s < PER; ++s) {
          const double d0 = xn[s][0] - x0, d1 = xn[s][1] - x1, d2 = xn[s][2] - x2;
          double w = fmax(fma(-d0, d0, fma(-d1, d1, fma(-d2, d2, 1.0))), 0.0);
          w = w * w;
          acc[s][0] += w * g0;
          acc[s][1] += w * g1;
          acc[s][2] += w * g2;
          acc[s][3] += w * g3;
        }
      }
      __syncthreads();
    }
  });
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int q = threadIdx.x + s * TH;
    if (q < N3)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ST* dst = S + ((size_t)t * 4 + k) * N3 + q;
        *dst = (ST)((double)*dst + acc[s][k]);
      }
  }
}


// ---------------------------------------------------------------------------
// Candidate lists of the FP32 source: for every target element, the elements
// (with the periodic image, entry = element | image << 27, unsigned) whose box, shifted
// by the image, lies within R + pad of the target's node box (Euclidean
// box-to-box distance).  Built once per radius and periods by two passes of
// the background-mesh search (count, then fill at the scanned offsets), so
// the source kernels read their candidates instead of searching.  Particles
// lie within pad of their element's box as long as the largest overhang
// measured at the deposit does not exceed pad; otherwise the kernels search.
// ---------------------------------------------------------------------------
struct DepLists {
  const int32_t* start;   // [E + 1]
  const int32_t* list;
  double pad;
  int32_t valid;
};

// the normalisation pass's staged particles of each target, kept for the
// node-sum pass (caller memory, optional): per target up to cap entries of
// 2 p and the particle index (its bits in the fourth float), and the number
// of particles it staged (more than cap: the node-sum pass stages again)
struct DepRec {
  float4* f;       // [E][cap], null: nothing recorded
  int32_t* cnt;    // [E]
  int32_t cap;
};

// a staged row (2 p, alpha_p = 1 - |p|^2) from the FP32 position p relative
// to the target centre in units of R; the operations are spelled out so that
// both passes round alpha_p alike from the same p
__device__ __forceinline__ float4 staged_row(float p0, float p1, float p2) {
  const float pp = __fmaf_rn(p2, p2, __fmaf_rn(p1, p1, __fmul_rn(p0, p0)));
  return make_float4(2.f * p0, 2.f * p1, 2.f * p2, __fsub_rn(1.f, pp));
}

__device__ __forceinline__ double box_box_dist2(const double* alo, const double* ahi, const double* blo,
                                                const double* bhi) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double d = fmax(fmax(alo[k] - bhi[k], blo[k] - ahi[k]), 0.0);
    s += d * d;
  }
  return s;
}

__global__ __launch_bounds__(256) void k_dep_lists(MeshView m, DepGeo g, double pad, int pass, int32_t* count,
                                                   const int32_t* __restrict__ start, int32_t* list) {
  const int t = blockIdx.x;
  if (t >= m.E) return;
  __shared__ CandLds<256> L;
  const double* nb = m.nbox + (size_t)t * 6;
  const double blo[3] = {nb[0], nb[1], nb[2]}, bhi[3] = {nb[3], nb[4], nb[5]};
  const double reach2 = (g.R + pad) * (g.R + pad);
  int written = 0;
  stream_candidates<256>(m, g.period, blo, bhi, g.R + pad, L, [&](int nc) {
    for (int cb = 0; cb < nc; cb += 256) {
      const int c = cb + threadIdx.x;
      bool keep = false;
      int e = 0, code = 0;
      if (c < nc) {
        e = L.e[c];
        code = L.img[c];
        double sh[3];
        image_shift(code, g.period, sh);
        double elo[3], ehi[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          elo[k] = m.elo[e * 3 + k] - sh[k];
          ehi[k] = m.ehi[e * 3 + k] - sh[k];
        }
        keep = box_box_dist2(elo, ehi, blo, bhi) < reach2;
      }
      int tot = 0;
      const int off = block_excl_scan<256>(keep ? 1 : 0, L.wsum, tot);
      if (pass == 1 && keep) list[start[t] + written + off] = (int32_t)((uint32_t)e | ((uint32_t)code << 27));
      written += tot;
    }
  });
  if (pass == 0 && threadIdx.x == 0) count[t] = written;
  if (pass == 0 && t == m.E - 1 && threadIdx.x == 0) count[m.E] = 0;
}

// body(nc) over the target's candidates in windows of kDepCand (L.e, L.img):
// from the list when it is valid for the particles' overhang, else by search
template <int TH, class Body>
__device__ __forceinline__ void for_candidates(const MeshView& m, const DepGeo& g, const DepLists& dl, int t,
                                               const double* blo, const double* bhi, double part_pad,
                                               CandLds<TH>& L, Body&& body) {
  if (dl.valid && part_pad <= dl.pad) {
    const int b = dl.start[t], e = dl.start[t + 1];
    for (int w0 = b; w0 < e; w0 += kDepCand) {
      const int nc = min(kDepCand, e - w0);
      for (int c = threadIdx.x; c < nc; c += TH) {
        const uint32_t v = (uint32_t)dl.list[w0 + c];
        L.e[c] = (int32_t)(v & ((1u << 27) - 1u));
        L.img[c] = (int8_t)(v >> 27);
      }
      __syncthreads();
      body(nc);
      __syncthreads();
    }
  } else {
    stream_candidates<TH>(m, g.period, blo, bhi, g.R + part_pad, L, body);
  }
}

// ---------------------------------------------------------------------------
// FP32 source on the matrix cores.  With node and particle positions n, p
// relative to the target element's centre in units of R,
//   q = 1 - |n - p|^2 = 2 p . n + alpha_p - |n|^2,   alpha_p = 1 - |p|^2,
// so the kernel argument of 16 particles x 16 nodes is one rank-4 product plus
// a term that depends on one side only, which enters as the accumulator input:
// one v_mfma_f32_16x16x4f32 per tile.  Both passes are node-major: a workgroup
// owns one target element, each of its waves a group of at most TPW 16-node
// tiles whose features stay in registers; the candidate particles (from the
// per-target candidate lists) are culled once per workgroup against the
// target's node box, staged in LDS and processed 16 at a time by every wave.
//  * Pass 1 (rows = nodes): the node features carry sqrt(V_n), so that
//    max(q', 0)^2 = K V_n and the per-particle sum takes two VALU operations
//    per pair; one float atomic per particle and wave adds it to the norm.
//  * Pass 2 (rows = particles): K = max(q, 0)^2 (two VALU operations per
//    pair), then sum_p K G_p per node on v_mfma_f32_4x4x1f32 (16 blocks of a
//    4-node x 1-particle by 1-particle x 4-component product), the K tile
//    being already in that instruction's A layout; S += once per node.
//    With caller memory bound for it, pass 1 records each target's staged
//    rows and pass 2 reads them back instead of staging again.
// Lane layouts (gfx950): 16x16x4: A[row][k], B[k][col] in lane (row or col)
// + 16 k, D[row][col] in lane col + 16 (row / 4), register row % 4.
// 4x4x1 (16 blocks): A[b][row], B[b][col] in lane (row or col) + 4 b,
// D[b][row][col] in lane col + 4 b, register row.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

template <int NN>
struct NodeTiling {
  static constexpr int N3 = NN * NN * NN;
  static constexpr int NT = (N3 + 15) / 16;                          // 16-node tiles per element
  static constexpr int W = NN >= 8 ? 4 : 2;                          // waves per workgroup
  static constexpr int TH = 64 * W;
  static constexpr int TPW = (NT + W - 1) / W;                       // tiles per wave
  static constexpr int CAP = TH + 16;                                // staged particles
};

// staged particles (structure of arrays in LDS)
template <int CAP>
struct PStage {
  float4 f[CAP];    // 2 p, alpha_p = 1 - |p|^2 (padding rows: 0, 0, 0, -1)
  float4 g[CAP];    // G_p (pass 2)
  float acc[CAP];   // normalisation sums of both wavefronts (pass 1), zero outside the processed tiles
  int32_t id[CAP];  // particle index, -1 for a padding row
};

// One wave's node group.  Pass 1: feature (lane / 16) of sqrt(V) (n, 1) of
// node tile*16 + lane % 16, and the accumulator input -sqrt(V) |n|^2 of the
// node rows 4 (lane / 16) + i.  Pass 2: feature (lane / 16) of (n, -|n|^2).
template <int NN>
struct NodeGroup {
  static constexpr int TPW = NodeTiling<NN>::TPW;
  float b[TPW];
  v4f c[TPW];
};

template <int NN, bool NORM>
__device__ inline void load_node_group(const MeshView& m, int t, const double* ctr, double iR, int wave, int lane,
                                       NodeGroup<NN>& G) {
  using T = NodeTiling<NN>;
  const int t0 = wave * T::TPW;   // tiles past the element's nodes keep zero features (q = 0)
  const int kq = lane >> 4;
#pragma unroll
  for (int tt = 0; tt < T::TPW; ++tt) {
    const int q = (t0 + tt) * 16 + (lane & 15);
    float f[4] = {0.f, 0.f, 0.f, 0.f};
    if (q < T::N3) {
      double r[3], rr = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        r[k] = (m.xnode[((size_t)t * T::N3 + q) * 3 + k] - ctr[k]) * iR;
        rr += r[k] * r[k];
      }
      const double s = NORM ? sqrt(m.vol[(size_t)t * T::N3 + q]) : 1.0;
      f[0] = (float)(s * r[0]);
      f[1] = (float)(s * r[1]);
      f[2] = (float)(s * r[2]);
      f[3] = NORM ? (float)s : (float)(-rr);
    }
    // feature kq without indexing a private array (scratch)
    G.b[tt] = kq == 0 ? f[0] : kq == 1 ? f[1] : kq == 2 ? f[2] : f[3];
    v4f c = {0.f, 0.f, 0.f, 0.f};
    if (NORM) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int qr = (t0 + tt) * 16 + 4 * kq + i;
        if (qr < T::N3) {
          double rr = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double d = (m.xnode[((size_t)t * T::N3 + qr) * 3 + k] - ctr[k]) * iR;
            rr += d * d;
          }
          c[i] = (float)(-sqrt(m.vol[(size_t)t * T::N3 + qr]) * rr);
        }
      }
    }
    G.c[tt] = c;
  }
}

// exclusive prefix count of pred over the workgroup of TH threads; every
// thread must call it
template <int TH>
__device__ inline int block_scan_bool(bool pred, int32_t* wsum, int& total) {
  const unsigned long long b = __ballot(pred);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) wsum[w] = __popcll(b);
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < TH / 64; ++k) {
    const int t = wsum[k];
    base += (k < w) ? t : 0;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + lane_rank(b);
}

// FP32 position of every particle relative to the centre of its element's
// node box, in units of R; w = 0 if the particle deposits (valid force), 1
// if not.  The staging of the matrix-core passes reads it instead of the FP64
// positions: a candidate element's offset to the target is added once per
// element, in FP32.
__global__ __launch_bounds__(256) void k_dep_local(MeshView m, Particles P, int64_t n, const int32_t* __restrict__ ok,
                                                   double iR, float4* __restrict__ xl) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (!ok[p]) {
    xl[p] = make_float4(0.f, 0.f, 0.f, 1.f);
    return;
  }
  const int64_t cap = P.cap;
  const double* nb = m.nbox + (size_t)P.elem[p] * 6;
  xl[p] = make_float4((float)((P.x[p] - 0.5 * (nb[0] + nb[3])) * iR),
                      (float)((P.x[cap + p] - 0.5 * (nb[1] + nb[4])) * iR),
                      (float)((P.x[2 * cap + p] - 0.5 * (nb[2] + nb[5])) * iR), 0.f);
}

constexpr int kSlotCap = 5120;   // particle slots of one candidate window mapped to their element

// per-window staging tables in LDS
struct WinLds {
  float4 off[kDepCand];        // candidate element's node-box centre (image shifted) - target centre, units of R
  int32_t base[kDepCand];      // first particle of the candidate minus its first slot
  int32_t pre[kDepCand + 1];   // first slot of each candidate, pre[nc] = slots of the window
  uint8_t slot[kSlotCap];      // candidate of each slot (windows of at most kSlotCap slots)
};

// Stream the target's candidate particles through the workgroup: for every
// window of candidate elements the particles of the window are numbered
// (slots) and each thread takes one slot at a time, keeps the particle if it
// deposits and lies within R of the target's node box, and the kept ones are
// appended (features in FP32, relative to the target's centre, units of R) to
// the shared staging list; then every wave runs tile(first) on each full
// 16-particle tile of the list with its own node tiles.  The last partial
// tile is padded (q <= -1, so K = 0) and flushed.  All threads of the
// workgroup must call it.
template <int NN, class Tile, class Flush>
__device__ inline void stream_particles(const MeshView& m, const int32_t* __restrict__ elem_start, const DepGeo& g,
                                        const DepLists& dl, const float4* __restrict__ xl,
                                        const float* __restrict__ Gp, int t, const double* ctr, double part_pad,
                                        CandLds<NodeTiling<NN>::TH>& L, WinLds& Wl,
                                        PStage<NodeTiling<NN>::CAP>& s_c, const DepRec& rec, Tile&& tile,
                                        Flush&& flush) {
  constexpr int TH = NodeTiling<NN>::TH;
  const double* nb = m.nbox + (size_t)t * 6;
  const double blo[3] = {nb[0], nb[1], nb[2]}, bhi[3] = {nb[3], nb[4], nb[5]};
  float flo[3], fhi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    flo[k] = (float)((blo[k] - ctr[k]) * g.iR);
    fhi[k] = (float)((bhi[k] - ctr[k]) * g.iR);
  }
  int n = 0;    // entries in s_c (uniform)
  int nr = 0;   // particles staged so far (uniform), the recorded list's length
  float4* rf = rec.f ? rec.f + (size_t)t * rec.cap : nullptr;
  for_candidates<TH>(m, g, dl, t, blo, bhi, part_pad, L, [&](int nc) {
    // candidate tables: slot numbering, particle base and FP32 offset
    int T = 0;
    for (int cb = 0; cb < nc; cb += TH) {
      const int c = cb + threadIdx.x;
      int beg = 0, cntc = 0;
      if (c < nc) {
        const int e = L.e[c];
        beg = elem_start[e];
        cntc = elem_start[e + 1] - beg;
      }
      int tot = 0;
      const int off = block_excl_scan<TH>(cntc, L.wsum, tot);
      if (c < nc) {
        const int e = L.e[c];
        double sh[3];
        image_shift(L.img[c], g.period, sh);
        const double* eb = m.nbox + (size_t)e * 6;
        Wl.off[c] = make_float4((float)((0.5 * (eb[0] + eb[3]) - sh[0] - ctr[0]) * g.iR),
                                (float)((0.5 * (eb[1] + eb[4]) - sh[1] - ctr[1]) * g.iR),
                                (float)((0.5 * (eb[2] + eb[5]) - sh[2] - ctr[2]) * g.iR), 0.f);
        Wl.pre[c] = T + off;
        Wl.base[c] = beg - (T + off);
      }
      T += tot;
    }
    if (threadIdx.x == 0) Wl.pre[nc] = T;
    __syncthreads();
    const bool mapped = T <= kSlotCap;
    if (mapped) {
      for (int c = threadIdx.x; c < nc; c += TH)
        for (int k = Wl.pre[c]; k < Wl.pre[c + 1]; ++k) Wl.slot[k] = (uint8_t)c;
      __syncthreads();
    }
    for (int jb = 0; jb < T; jb += TH) {
      const int j = jb + threadIdx.x;
      bool keep = false;
      float r[3] = {0.f, 0.f, 0.f};
      float4 gg = make_float4(0.f, 0.f, 0.f, 0.f);
      int32_t pi = -1;
      if (j < T) {
        int c;
        if (mapped) {
          c = Wl.slot[j];
        } else {
          int lo = 0, hi = nc - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (Wl.pre[mid] <= j) lo = mid;
            else hi = mid - 1;
          }
          c = lo;
        }
        pi = Wl.base[c] + j;
        const float4 v = xl[pi];
        const float4 o = Wl.off[c];
        r[0] = v.x + o.x;
        r[1] = v.y + o.y;
        r[2] = v.z + o.z;
        float d2 = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float dd = fmaxf(fmaxf(flo[k] - r[k], r[k] - fhi[k]), 0.f);
          d2 = fmaf(dd, dd, d2);
        }
        keep = v.w == 0.f && d2 < 1.f;
        if (Gp && keep) gg = *(const float4*)(Gp + (int64_t)pi * 8);
      }
      int tot = 0;
      const int off = block_scan_bool<TH>(keep, L.wsum, tot);
      if (keep) {
        const float4 f4 = staged_row(r[0], r[1], r[2]);
        s_c.f[n + off] = f4;
        s_c.g[n + off] = gg;
        s_c.id[n + off] = pi;
        if (rf && nr + off < rec.cap) {
          rf[nr + off] = make_float4(f4.x, f4.y, f4.z, __int_as_float(pi));
        }
      }
      n += tot;
      nr += tot;
      __syncthreads();
      int first = 0;
      for (; n - first >= 16; first += 16) tile(first);
      if (first > 0) {
        // the processed entries' sums out, the remainder (< 16 entries) to the front
        const int rem = n - first;
        float4 f0 = make_float4(0.f, 0.f, 0.f, 0.f), g0 = f0;
        int32_t i0 = -1;
        __syncthreads();
        flush(first);
        if ((int)threadIdx.x < rem) {
          f0 = s_c.f[first + threadIdx.x];
          g0 = s_c.g[first + threadIdx.x];
          i0 = s_c.id[first + threadIdx.x];
        }
        __syncthreads();
        if ((int)threadIdx.x < rem) {
          s_c.f[threadIdx.x] = f0;
          s_c.g[threadIdx.x] = g0;
          s_c.id[threadIdx.x] = i0;
        }
        n = rem;
      }
      __syncthreads();
    }
  });
  if (n > 0) {
    if ((int)threadIdx.x >= n && threadIdx.x < 16) {
      s_c.f[threadIdx.x] = make_float4(0.f, 0.f, 0.f, -1.f);
      s_c.g[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
      s_c.id[threadIdx.x] = -1;
    }
    __syncthreads();
    tile(0);
    __syncthreads();
    flush(16);
  }
  if (rf && threadIdx.x == 0) rec.cnt[t] = nr;
}

// the node-sum pass from the recorded list of the target's staged particles:
// the same rows in the same order, so the same 16-particle tiles (the last
// one padded) as staging them again
template <int NN, class Tile>
__device__ inline void stream_list(const DepRec& rec, int t, int cnt, const float* __restrict__ Gp,
                                   PStage<NodeTiling<NN>::CAP>& s_c, Tile&& tile) {
  constexpr int TH = NodeTiling<NN>::TH;
  const float4* lf = rec.f + (size_t)t * rec.cap;
  // each thread's row of the next chunk is loaded while the tiles of the
  // current one run
  float4 f = make_float4(0.f, 0.f, 0.f, -1.f), g = make_float4(0.f, 0.f, 0.f, 0.f);
  int32_t pi = -1;
  auto fetch = [&](int j) {
    f = make_float4(0.f, 0.f, 0.f, -1.f);   // padding row: alpha = -1, no kernel weight
    g = make_float4(0.f, 0.f, 0.f, 0.f);
    pi = -1;
    if (j < cnt) {
      const float4 e = lf[j];
      pi = __float_as_int(e.w);
      f = staged_row(0.5f * e.x, 0.5f * e.y, 0.5f * e.z);   // 2 p halved is p exactly
      g = *(const float4*)(Gp + (int64_t)pi * 8);
    }
  };
  fetch(threadIdx.x);
  for (int j0 = 0; j0 < cnt; j0 += TH) {
    const int mlen = min(TH, cnt - j0);
    s_c.f[threadIdx.x] = f;
    s_c.g[threadIdx.x] = g;
    s_c.id[threadIdx.x] = pi;
    __syncthreads();
    fetch(j0 + TH + threadIdx.x);
    for (int first = 0; first < mlen; first += 16) tile(first);
    __syncthreads();
  }
}

// max(x, 0) as one integer max: a float with the sign bit set is a negative
// int (fmaxf would first quieten a signalling NaN, a second instruction)
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// pass 1: norm[p] += sum over the wave's nodes of K V (rows = nodes); with
// COUNT, the (particle, node) pairs within R are counted as well
template <int NN, bool COUNT>
__global__ __launch_bounds__(NodeTiling<NN>::TH) __attribute__((amdgpu_waves_per_eu(4))) void k_dep_norm_mfma(
    MeshView m, const int32_t* __restrict__ elem_start, DepGeo g, DepLists dl, const float4* __restrict__ xl,
    const unsigned long long* __restrict__ povh, float* norm, unsigned long long* pairs, DepRec rec) {
  using T = NodeTiling<NN>;
  const int t = xcd_element(blockIdx.x, m.E);
  if (t >= m.E) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ CandLds<T::TH> L;
  __shared__ WinLds Wl;
  __shared__ PStage<T::CAP> s_c;
  const double* nb = m.nbox + (size_t)t * 6;
  const double ctr[3] = {0.5 * (nb[0] + nb[3]), 0.5 * (nb[1] + nb[4]), 0.5 * (nb[2] + nb[5])};
  NodeGroup<NN> NG;
  load_node_group<NN, true>(m, t, ctr, g.iR, wave, lane, NG);
  const double part_pad = __longlong_as_double((long long)*povh);
  unsigned long long npairs = 0;   // wave-uniform
  auto tile = [&](int first) {
    // B operand: feature (lane / 16) of particle first + lane % 16
    const int pc = first + (lane & 15);
    const float pb = ((const float*)&s_c.f[pc])[lane >> 4];
    float acc = 0.f;
    v4f q[T::TPW];
#pragma unroll
    for (int u = 0; u < T::TPW; ++u) q[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(NG.b[u], pb, NG.c[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < T::TPW; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float w = relu(q[u][i]);
        if (COUNT) npairs += __popcll(__ballot(w > 0.f));
        acc = fmaf(w, w, acc);
      }
    if (!COUNT) {
      // software pipeline: each tile's MFMA is issued two tiles ahead of the
      // VALU work that reads it
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
#pragma unroll
      for (int u = 0; u + 2 < T::TPW; ++u) {
        __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x002, 16, 0);
    }
    // sum over the node rows held by the four lane groups, then both
    // wavefronts' sums in LDS (one global atomic per particle and target)
    acc += __shfl_xor(acc, 16, 64);
    acc += __shfl_xor(acc, 32, 64);
    if (lane < 16 && acc != 0.f) atomicAdd(&s_c.acc[pc], acc);
  };
  // entries [0, cnt) are processed: their sums to the particles, LDS cleared
  auto flush = [&](int cnt) {
    for (int k = threadIdx.x; k < cnt; k += T::TH) {
      const float a = s_c.acc[k];
      const int32_t id = s_c.id[k];
      if (id >= 0 && a != 0.f) atomicAdd(norm + id, a);
      s_c.acc[k] = 0.f;
    }
  };
  for (int k = threadIdx.x; k < T::CAP; k += T::TH) s_c.acc[k] = 0.f;
  __syncthreads();
  stream_particles<NN>(m, elem_start, g, dl, xl, nullptr, t, ctr, part_pad, L, Wl, s_c, rec, tile, flush);
  if (COUNT && pairs && lane == 0 && npairs) atomicAdd(pairs + (blockIdx.x & (kStatSlots - 1)), npairs);
}

// G_p = -F_p / norm_p (FP32, written over F_p), zero for particles that
// deposit nothing
__global__ __launch_bounds__(256) void k_dep_scale(int64_t n, double* F, const int32_t* __restrict__ ok,
                                                   const float* __restrict__ norm) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double nv = norm[p];
  const bool use = ok[p] && nv > 0.0;
  const double in = use ? -1.0 / nv : 0.0;
  double f[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) f[k] = F[p * 4 + k];
  float* G = (float*)(F + p * 4);
#pragma unroll
  for (int k = 0; k < 4; ++k) G[k] = use ? (float)(f[k] * in) : 0.f;
}

// pass 2: S[node] += sum_p K G_p (rows = particles)
template <int NN>
__global__ __launch_bounds__(NodeTiling<NN>::TH) __attribute__((amdgpu_waves_per_eu(4))) void k_dep_gather_mfma(
    MeshView m, const int32_t* __restrict__ elem_start, DepGeo g, DepLists dl, const float4* __restrict__ xl,
    const float* __restrict__ Gp, const unsigned long long* __restrict__ povh, float* S, DepRec rec) {
  using T = NodeTiling<NN>;
  const int t = xcd_element(blockIdx.x, m.E);
  if (t >= m.E) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ CandLds<T::TH> L;
  __shared__ WinLds Wl;
  __shared__ PStage<T::CAP> s_c;
  const double* nb = m.nbox + (size_t)t * 6;
  const double ctr[3] = {0.5 * (nb[0] + nb[3]), 0.5 * (nb[1] + nb[4]), 0.5 * (nb[2] + nb[5])};
  NodeGroup<NN> NG;
  load_node_group<NN, false>(m, t, ctr, g.iR, wave, lane, NG);
  const double part_pad = __longlong_as_double((long long)*povh);
  // acc[tt]: block (node group 4 g, particle quarter kq) of node tile tt,
  // register r = node 4 g + r, lane c + 4 g + 16 kq = component c
  v4f acc[T::TPW];
#pragma unroll
  for (int tt = 0; tt < T::TPW; ++tt) acc[tt] = (v4f){0.f, 0.f, 0.f, 0.f};
  const int kq = lane >> 4;
  auto tile = [&](int first) {
    // A operand: feature kq of (2 p, 1) of particle first + lane % 16; the
    // accumulator input alpha of the particle rows 4 kq + i
    const float fk = ((const float*)&s_c.f[first + (lane & 15)])[kq];
    const float pa = kq == 3 ? 1.f : fk;
    v4f cin;
    float gb[4];   // B of the 4x4x1 products: G_c of particle 4 kq + i, c = lane % 4
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      cin[i] = s_c.f[first + 4 * kq + i].w;
      gb[i] = ((const float*)&s_c.g[first + 4 * kq + i])[lane & 3];
    }
    v4f q[T::TPW];
#pragma unroll
    for (int u = 0; u < T::TPW; ++u) q[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa, NG.b[u], cin, 0, 0, 0);
    float kk[T::TPW][4];
#pragma unroll
    for (int u = 0; u < T::TPW; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float w = relu(q[u][i]);
        kk[u][i] = w * w;
      }
#pragma unroll
    for (int u = 0; u < T::TPW; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[u] = __builtin_amdgcn_mfma_f32_4x4x1f32(kk[u][i], gb[i], acc[u], 0, 0, 0);
    // software pipeline: tile u's kernel-argument MFMA two tiles ahead of its
    // VALU work, its four 4x4x1 products one tile behind
    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);
#pragma unroll
    for (int u = 1; u < T::TPW; ++u) {
      if (u + 1 < T::TPW) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // kernel argument of tile u + 1
      __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);                        // products of tile u - 1
      __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);                        // K of tile u
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
  };
  const int rc = rec.f ? rec.cnt[t] : -1;
  if (rc >= 0 && rc <= rec.cap) {
    stream_list<NN>(rec, t, rc, Gp, s_c, tile);
  } else {
    const DepRec none{nullptr, nullptr, 0};
    stream_particles<NN>(m, elem_start, g, dl, xl, Gp, t, ctr, part_pad, L, Wl, s_c, none, tile, [](int) {});
  }
  // sum over the particle quarters, then one read-modify-write of each
  // (node, component)
  const int t0 = wave * T::TPW;
#pragma unroll
  for (int tt = 0; tt < T::TPW; ++tt) {
    v4f v = acc[tt];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v[r] += __shfl_xor(v[r], 16, 64);
      v[r] += __shfl_xor(v[r], 32, 64);
    }
    if (lane < 16) {
      const int c = lane & 3, g4 = lane >> 2;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = (t0 + tt) * 16 + 4 * g4 + r;
        if (q < T::N3) {
          float* dst = S + ((size_t)t * 4 + c) * T::N3 + q;
          *dst += v[r];
        }
      }
    }
  }
}

__global__ void k_dep_reset(unsigned long long* povh, float* norm, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *povh = 0ull;
  if (i < n) norm[i] = 0.f;
}

}  // namespace

#include "fp_shapes.h"

hipError_t launch_dep_lists(const MeshView& m, double R, const double* period, double pad, int pass,
                            int32_t* count, const int32_t* start, int32_t* list, hipStream_t s) {
  DepGeo g{};
  g.R = R;
  g.R2 = R * R;
  g.iR = 1.0 / R;
  for (int k = 0; k < 3; ++k) g.period[k] = period[k];
  k_dep_lists<<<dim3((unsigned)m.E), 256, 0, s>>>(m, g, pad, pass, count, start, list);
  return hipGetLastError();
}

hipError_t launch_deposit_shape(const MeshView& m, const Particles& P, const Fluid& fl, int64_t n, void* S,
                                int s_f32, const ForceModel& fm, double R, const double* period, double node_pad,
                                double* dep, const int32_t* elem_start, unsigned long long* povh,
                                unsigned long long* pairs, const int32_t* list_start, const int32_t* list,
                                double list_pad, void* reuse, int32_t reuse_cap, const void* tasks,
                                const int32_t* ntask, int task_tp, hipEvent_t* ev, hipStream_t s) {
  DepLists dl{list_start, list, list_pad, list_start != nullptr ? 1 : 0};
  // the reuse list: counts [E], then rows float4 [E][cap] (256-byte aligned)
  DepRec rc{nullptr, nullptr, 0};
  if (reuse && reuse_cap > 0) {
    rc.cnt = (int32_t*)reuse;
    rc.f = (float4*)(((uintptr_t)(rc.cnt + m.E) + 255) & ~(uintptr_t)255);
    rc.cap = reuse_cap;
  }
  auto rec = [&](int i) { if (ev && ev[i]) hipEventRecord(ev[i], s); };
  DepGeo g;
  g.R = R;
  g.R2 = R * R;
  g.iR = 1.0 / R;
  g.node_pad = node_pad;
  for (int k = 0; k < 3; ++k) g.period[k] = period[k];
  double* F = dep;
  int32_t* ok = (int32_t*)(dep + 4 * P.cap);
  dim3 gp((unsigned)((std::max<int64_t>(n, 1) + 255) / 256));
  dim3 ge((unsigned)(((m.E + kXcd - 1) / kXcd) * kXcd));
  // FP32 source: the normalisation sums of the matrix-core pass (float[cap],
  // after the validity flags)
  float* norm = (float*)(ok + P.cap);
  // FP32 local positions (float4[cap], 16-byte aligned after the sums)
  float4* xl = (float4*)(((uintptr_t)(norm + P.cap) + 15) & ~(uintptr_t)15);
  k_dep_reset<<<gp, 256, 0, s>>>(povh, norm, s_f32 ? n : 0);
#define FP_L(A, B)                                                                                           \
  if (m.n == A && m.ng == B) {                                                                               \
    if (s_f32 && fl.f32 && fm.forces == 0 && tasks) {                                                       \
      const hipError_t fe = launch_dep_force_elem(m, P, fl, fm.drag, tasks, ntask, task_tp, n, F, ok, povh, s); \
      if (fe != hipSuccess) return fe;                                                                       \
    } else if (fl.f32) {                                                                                     \
      k_dep_force<A, B, float><<<gp, 256, 0, s>>>(m, P, fl, n, fm, F, ok, povh);                             \
    } else {                                                                                                 \
      k_dep_force<A, B, double><<<gp, 256, 0, s>>>(m, P, fl, n, fm, F, ok, povh);                            \
    }                                                                                                        \
    if (s_f32) {                                                                                             \
      rec(0);                                                                                                \
      k_dep_local<<<gp, 256, 0, s>>>(m, P, n, ok, g.iR, xl);                                                 \
      if (pairs)                                                                                             \
        k_dep_norm_mfma<A, true><<<ge, NodeTiling<A>::TH, 0, s>>>(m, elem_start, g, dl, xl, povh, norm, pairs,     \
                                                                  rc);                                       \
      else                                                                                                   \
        k_dep_norm_mfma<A, false><<<ge, NodeTiling<A>::TH, 0, s>>>(m, elem_start, g, dl, xl, povh, norm, pairs,    \
                                                                   rc);                                      \
      rec(1);                                                                                                \
      k_dep_scale<<<gp, 256, 0, s>>>(n, F, ok, norm);                                                        \
      rec(2);                                                                                                \
      k_dep_gather_mfma<A><<<ge, NodeTiling<A>::TH, 0, s>>>(m, elem_start, g, dl, xl, (const float*)F,      \
                                                            povh, (float*)S, rc);                            \
      rec(3);                                                                                                \
    } else {                                                                                                 \
      rec(0);                                                                                                \
      k_dep_norm<A><<<ge, kNormThreads, 0, s>>>(m, P, elem_start, g, F, ok, povh);                           \
      rec(1);                                                                                                \
      rec(2);                                                                                                \
      k_dep_gather<A, double><<<ge, kGatherThreads, 0, s>>>(m, P, elem_start, g, F, povh, (double*)S);       \
      rec(3);                                                                                                \
    }                                                                                                        \
    return hipGetLastError();                                                                                \
  }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

}  // namespace fp

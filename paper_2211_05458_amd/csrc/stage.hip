// One low-storage RK stage (Sec. 3.2), split by the data each part touches:
//
//  k_stage_elem  one wavefront per (element, <= 64 particles) task built after
//                the counting sort (or one per half for tasks of <= 32).  The
//                element's geometry nodes and fluid state are staged in LDS
//                once per task and read as broadcasts.  Per particle: guess,
//                Newton, inside check, interpolation, drag, stage update, and
//                the bounding-box test of the element's faces (Sec. 3.2.4);
//                the mixed stage interpolates for the whole wavefront at once
//                on the matrix cores.  Particles whose segment touches a face box go
//                to the tracking queue; particles that left the task element
//                in an earlier stage, or that Newton does not locate inside
//                it, go to the straggler queue.
//  k_stage_lane  the same stage for the straggler queue (or for all particles
//                when no sort has been done), with per-lane element data.
//  k_track       physical-space tracking (Sec. 3.2.3/3.2.4) of the queued
//                segments: face intersection, hand-off, periodic shift, wall
//                reflection.
#include "fp_device.h"
#include "fp_launch.h"

namespace fp {

// The second-order reach test (reachable_faces_taylor) costs the stage
// kernels a map evaluation per wavefront and registers; it pays where the
// tracking queue keeps the tracker throughput-bound, measured on the
// strongly curved geometry of degree 6 (N_geo = 6: tracking queue -63 %, step
// time -40 % on the annular passage), not on degree 4 (32^3 sine box: the
// shorter queue left the latency-bound tracker as slow and the stage kernel
// 5 % slower).
template <int NG>
constexpr bool kReach2 = NG >= 7;

// the low-storage update of the mixed stage (FP32) from the acceleration a
__device__ __forceinline__ void mixed_lsrk(const float* a, const double* x, double* v, double* kx, double* kv,
                                           const StepParams& sp, double* xe) {
  const float A = (float)sp.A, B = (float)sp.B, dt = (float)sp.dt;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float vf = (float)v[k];
    float kxf = A * (float)kx[k] + dt * vf;
    float kvf = A * (float)kv[k] + dt * a[k];
    kx[k] = kxf;
    kv[k] = kvf;
    xe[k] = x[k] + (double)(B * kxf);
    v[k] = (double)(vf + B * kvf);
  }
}

// drag (plus gravity) and the low-storage update of the mixed stage from the
// interpolated density and momentum Uc (FP32)
__device__ __forceinline__ void mixed_update(const float* Uc, const double* x, double* v, double* kx, double* kv,
                                             double d, const Fluid& fl, const StepParams& sp, double* xe) {
  float vf[3] = {(float)v[0], (float)v[1], (float)v[2]};
  float ir = 1.0f / Uc[0];
  float u[3] = {Uc[1] * ir, Uc[2] * ir, Uc[3] * ir};
  float a[3], fD;
  drag_accel<float>(sp.drag, Uc[0], u, vf, (float)d, (float)fl.mu, (float)fl.rho_p, a, fD);
#pragma unroll
  for (int k = 0; k < 3; ++k) a[k] += (float)sp.gravity[k];
  mixed_lsrk(a, x, v, kx, kv, sp, xe);
}

// interpolation, drag and the low-storage update for one particle.  FORCES:
// the extra terms of the equation of motion selected in sp.forces (they need
// the velocity gradient, hence the element's geometry nodes Xe).
template <int NN, int NG, typename UT, bool MIXED, bool FORCES>
__device__ __forceinline__ void stage_update(const MeshView& m, const UT* __restrict__ Ue,
                                             const double* __restrict__ Xe, const double* xi, const double* x,
                                             double* v, double* kx, double* kv, double d, const Fluid& fl,
                                             const StepParams& sp, double* xe) {
  double Jg[3][3];
  if (FORCES) {
    double xm[3];
    map_jac<NG>(m, Xe, xi, xm, Jg);
  }
  if (!MIXED) {
    double a[3];
    if (FORCES) {
      double val[kInterpVars], dval[kInterpVars][3], u[3], G[3][3];
      interp_grad<NN, double, UT>(m.xdg, m.cdg, Ue, xi, val, dval);
      velocity_gradient<double>(Jg, val, dval, u, G);
      particle_accel<double>(sp.drag, sp.forces, val[0], u, G, v, d, fl.mu, fl.rho_p, sp.gravity, a, nullptr);
    } else {
      double Uc[kInterpVars];
      interp<NN, UT>(m, Ue, xi, Uc);
      double rho = Uc[0], ir = 1.0 / rho;
      double u[3] = {Uc[1] * ir, Uc[2] * ir, Uc[3] * ir};
      double fD;
      drag_accel<double>(sp.drag, rho, u, v, d, fl.mu, fl.rho_p, a, fD);
#pragma unroll
      for (int k = 0; k < 3; ++k) a[k] += sp.gravity[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      kx[k] = sp.A * kx[k] + sp.dt * v[k];
      kv[k] = sp.A * kv[k] + sp.dt * a[k];
      xe[k] = x[k] + sp.B * kx[k];
      v[k] = v[k] + sp.B * kv[k];
    }
  } else {
    float vf[3] = {(float)v[0], (float)v[1], (float)v[2]};
    float a[3];
    if (FORCES) {
      float val[kInterpVars], dval[kInterpVars][3], u[3], G[3][3];
      interp_grad<NN, float, UT>(m.xdgf, m.cdgf, Ue, xi, val, dval);
      velocity_gradient<float>(Jg, val, dval, u, G);
      particle_accel<float>(sp.drag, sp.forces, val[0], u, G, vf, (float)d, (float)fl.mu, (float)fl.rho_p,
                            sp.gravity, a, nullptr);
      mixed_lsrk(a, x, v, kx, kv, sp, xe);
    } else {
      float Uc[kInterpVars];
      interp_f32<NN, UT>(m, Ue, xi, Uc);
      mixed_update(Uc, x, v, kx, kv, d, fl, sp, xe);
    }
  }
}

typedef float v4f __attribute__((ext_vector_type(4)));

// Interpolation of the drag law's variables (FP32) for the particles of a
// whole wavefront at once, with the contraction over xi_1 on 4x4x1 FP32
// matrix products.  Block b of the product's 16 takes the particles of lanes
// 4b .. 4b+3 as its four columns (operand B: l_i(xi_1) of the lane's own
// particle) and four consecutive rows R = (var, k, j) of the element's state
// as its rows (operand A: lane 4b + r reads row R0 + r), so after the sum
// over i register r of every lane holds sum_i U[var][k][j][i] l_i(xi_1) of
// row R0 + r for its own particle; the weights l_j(xi_2) and l_k(xi_3) are
// applied in the lane.  The four lanes of a block read the same element (U is
// the lane's element's state, [var][k][j][i], in LDS or global memory).
// Every lane of the wavefront calls it, a lane without a particle with any
// finite xi.
template <int NN>
__device__ __forceinline__ void interp_f32_mfma(const MeshView& m, const float* __restrict__ U, const double* xi,
                                                float* out) {
  float l1[NN], l2[NN], l3[NN];
  lagrange<NN, float>(m.xdgf, m.cdgf, (float)xi[0], l1);
  lagrange<NN, float>(m.xdgf, m.cdgf, (float)xi[1], l2);
  lagrange<NN, float>(m.xdgf, m.cdgf, (float)xi[2], l3);
  const float* Ur = U + (threadIdx.x & 3) * NN;
  constexpr int kRows = kInterpVars * NN * NN;
#pragma unroll
  for (int v = 0; v < kInterpVars; ++v) out[v] = 0.0f;
  float s = 0.0f;
#pragma unroll
  for (int g = 0; g < kRows / 4; ++g) {
    v4f d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < NN; ++i) d = __builtin_amdgcn_mfma_f32_4x4x1f32(Ur[4 * g * NN + i], l1[i], d, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int R = 4 * g + r, j = R % NN, k = (R / NN) % NN, v = R / (NN * NN);
      s += d[r] * l2[j];
      if (j == NN - 1) {
        out[v] += s * l3[k];
        s = 0.0f;
      }
    }
  }
}

// local faces of an element that are not internal (wall, open, periodic,
// mortar): their crossings cannot be repaired by following xi to a neighbour
__device__ __forceinline__ unsigned boundary_faces(const FaceRec* __restrict__ Fe) {
  unsigned b = 0;
#pragma unroll
  for (int f = 0; f < 6; ++f) b |= (Fe[f].bc != BC_INTERNAL ? 1u : 0u) << f;
  return b;
}

struct Task { int32_t e, p0, cnt, pad; };

struct Queues {
  int32_t* counters;  // [0] stragglers, [1] tracking (one 8-byte aligned word), [2] next tracking entry
  int32_t* strag;     // [cap]
  int32_t* trk_p;     // [cap]
  double* trk_x;      // [3][cap] segment start
  uint8_t* trk_m;     // [cap] local faces the segment can reach (bit f)
};

// Tasks of up to 64 particles: one per wavefront, four wavefronts per
// workgroup, four per SIMD (at most 128 VGPRs: the Newton and interpolation
// loops wait on LDS reads, and the fourth wavefront hides more of that
// latency than the few spilled registers cost).  Tasks of up to 32 particles
// (mixed stage, small elements): two per wavefront, one per half, each with
// its own element in LDS, two wavefronts per workgroup, three per SIMD:
// elements hold about 30 particles, so one element per wavefront leaves half
// of every LDS broadcast and VALU instruction idle.  (Two FP64 elements per
// wavefront leave room for only two wavefronts per SIMD, which measured
// slower, and so do FP32 elements of N = 7 or N_geo = 6.)
constexpr int elem_waves(int tp) { return tp == 64 ? 4 : 2; }

// the element kernel's wavefronts per SIMD: four for tasks of 64 particles
// (three for two tasks of 32 per wavefront), fewer where the staged element
// data of a workgroup leave room for fewer workgroups in a CU's 160 KB of LDS.
// Geometry degree 6 takes three: the degree-6 map and its reach test spill
// about 250 registers at the 128 of four wavefronts per SIMD, and three with
// fewer spills measured faster on the annular passage (FP64 10.9 -> 9.8 ms,
// mixed 8.8 -> 7.4 ms per stage; two: 12.4 and 8.7 ms)
template <int NN, int NG, typename UT, bool MIXED>
constexpr int elem_occupancy() {
  constexpr int tp = task_particles(NN, NG, MIXED), slots = elem_waves(tp) * (64 / tp);
  constexpr int ng3 = NG * NG * NG, nn3 = NN * NN * NN;
  constexpr bool stage_u = ng3 * 3 * 8 + kInterpVars * nn3 * (int)sizeof(UT) <= 12 * 1024 && ng3 * 3 * 8 <= 4096;
  constexpr int lds = slots * (ng3 * 3 * 8 + (stage_u ? kInterpVars * nn3 * (int)sizeof(UT) : 0)) + 64;
  constexpr int by_lds = (160 * 1024 / lds) * elem_waves(tp) / 4;
  constexpr int want = (tp == 64 && NG < 7) ? 4 : 3;
  return by_lds < want ? (by_lds < 1 ? 1 : by_lds) : want;
}

template <int NN, int NG, typename UT, bool MIXED, bool MLP, bool FORCES>
__global__ __launch_bounds__(64 * elem_waves(task_particles(NN, NG, MIXED)))
__attribute__((amdgpu_waves_per_eu(elem_occupancy<NN, NG, UT, MIXED>())))
void k_stage_elem(MeshView m, const double* __restrict__ X, const double* __restrict__ XN, const UT* __restrict__ U,
                  const FaceRec* __restrict__ faces, const Task* __restrict__ tasks, const int32_t* __restrict__ ntask,
                  Particles P, Fluid fl, StepParams sp, Queues q, unsigned long long* stats) {
  constexpr int NG3 = NG * NG * NG, NN3 = NN * NN * NN;
  constexpr int TP = task_particles(NN, NG, MIXED), kElemWaves = elem_waves(TP), PER = 64 / TP;
  constexpr int SLOTS = kElemWaves * PER;
  // the task element's geometry nodes and fluid state, staged once per task
  // with coalesced vector loads and read as LDS broadcasts by every Newton
  // iteration and the interpolation; U stays in global memory when both would
  // not fit four elements per workgroup in 48 KB, or when the geometry nodes
  // alone take more than 4 KB (N_geo = 6: with U as well, three workgroups per
  // CU and one wavefront per SIMD)
  constexpr bool kStageU =
      NG3 * 3 * 8 + kInterpVars * NN3 * (int)sizeof(UT) <= 12 * 1024 && NG3 * 3 * 8 <= 4096;
  __shared__ double sX[SLOTS][NG3 * 3];
  __shared__ UT sU[SLOTS][kStageU ? kInterpVars * NN3 : 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int half = (TP == 64) ? 0 : lane / TP, tl = lane % TP, slot = w * PER + half;
  const int wid = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kElemWaves + w));
  const int ti = wid * PER + half;
  const int nt = __builtin_amdgcn_readfirstlane(*ntask);
  int it_sum = 0, calls = 0, fb = 0;
  bool strag = false, trk = false;
  int64_t p = 0;
  double xs0 = 0, xs1 = 0, xs2 = 0;
  unsigned reach = 0x3Fu;
  const int64_t cap = P.cap;
  Task t{0, 0, 0, 0};
  if (ti < nt) {
    t = tasks[ti];
    const int e = (TP == 64) ? __builtin_amdgcn_readfirstlane(t.e) : t.e;
    const double* Xg = X + (size_t)e * NG3 * 3;
    for (int i = tl; i < NG3 * 3; i += TP) sX[slot][i] = Xg[i];
    if (kStageU) {
      const UT* Ug = U + (size_t)e * 5 * NN3;
      for (int i = tl; i < kInterpVars * NN3; i += TP) sU[slot][i] = Ug[i];
    }
  }
  __syncthreads();
  // the mixed stage interpolates on the matrix cores, all lanes together,
  // between the location of the lanes' particles and their update (the
  // element's state from LDS, or from global memory where it is not staged)
  constexpr bool kMfmaInterp = MIXED && !FORCES;
  bool ok = false;
  int e = 0;
  double x[3] = {0.0, 0.0, 0.0}, xi[3] = {0.0, 0.0, 0.0};
  if (ti < nt) {
    e = (TP == 64) ? __builtin_amdgcn_readfirstlane(t.e) : t.e;
    const int p0 = (TP == 64) ? __builtin_amdgcn_readfirstlane(t.p0) : t.p0;
    const int cnt = (TP == 64) ? __builtin_amdgcn_readfirstlane(t.cnt) : t.cnt;
    p = (int64_t)p0 + tl;
    bool act = tl < cnt && P.status[p] == ACTIVE;
    if (act && P.elem[p] != e) {
      strag = true;
      act = false;
    }
    if (act) {
      const double* XNe = XN + (size_t)e * NN3 * 3;
      x[0] = P.x[p]; x[1] = P.x[cap + p]; x[2] = P.x[2 * cap + p];
      double gw[3], Ji[9];
      const bool wv = sp.warm && warm_guess(P, p, gw);
      // the guess pass computed learned guesses only for particles without
      // continued coordinates
      const bool lg = MLP && sp.mlp_guess && !wv;
      float gl[3] = {0.f, 0.f, 0.f};
      if (lg) {
        gl[0] = sp.mlp_guess[p]; gl[1] = sp.mlp_guess[cap + p]; gl[2] = sp.mlp_guess[2 * cap + p];
      }
      if (!locate_xi_e<NN, NG, MLP>(m, e, sX[slot], XNe, x, xi, sp.max_it, it_sum, calls, fb,
                                    lg, gl, wv, gw, Ji, MIXED ? kNewtonTolMixed : kNewtonTol) ||
          !inside_ref(xi)) {
        strag = true;   // not located in its element: the per-lane kernel recovers it
        xi[0] = xi[1] = xi[2] = 0.0;
      } else {
        ok = true;
        if (sp.warm) {
          // the stage moves x by B (A kx + dt v): continue xi along it
          double xe1[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) xe1[k] = x[k] + sp.B * (sp.A * P.kx[k * cap + p] + sp.dt * P.v[k * cap + p]);
          store_warm(P, p, xi, Ji, x, xe1);
        }
      }
    }
  }
  float Uc[kInterpVars];
  if constexpr (kMfmaInterp) {
    if (wid * PER < nt)
      interp_f32_mfma<NN>(m, kStageU ? (const float*)sU[slot] : (const float*)U + (size_t)e * 5 * NN3, xi, Uc);
  }
  if (ok) {
    const double* Xe = sX[slot];
    const UT* Ue = kStageU ? sU[slot] : U + (size_t)e * 5 * NN3;
    double v[3] = {P.v[p], P.v[cap + p], P.v[2 * cap + p]};
    double kx[3] = {P.kx[p], P.kx[cap + p], P.kx[2 * cap + p]};
    double kv[3] = {P.kv[p], P.kv[cap + p], P.kv[2 * cap + p]};
    double xe[3];
    if constexpr (kMfmaInterp) mixed_update(Uc, x, v, kx, kv, P.d[p], fl, sp, xe);
    else stage_update<NN, NG, UT, MIXED, FORCES>(m, Ue, Xe, xi, x, v, kx, kv, P.d[p], fl, sp, xe);
    const FaceRec* Fe = faces + (size_t)e * 6;
    bool any = false;
    // reference-space localisation: a segment that cannot reach a
    // boundary face is not traced (the next location step finds it); in
    // either mode only the boxes of the faces the segment can reach count
    const double L2 = (xe[0] - x[0]) * (xe[0] - x[0]) + (xe[1] - x[1]) * (xe[1] - x[1]) +
                      (xe[2] - x[2]) * (xe[2] - x[2]);
    const double ds = m.dsafe[e];
    if (!(sp.refspace && L2 < ds * ds)) {
      // the sampled reach bounds drop internal faces only: the faces that
      // are not internal (wall, open, periodic) keep their bit and meet the
      // box test, and a crossing of an internal face the bound misses is
      // repaired exactly by the location step (xi followed to the neighbour)
      const unsigned keep = boundary_faces(Fe);
      reach = reachable_faces(m, e, xi, L2) | keep;
#pragma unroll 1
      for (int f = 0; f < 6; ++f) any = any || (((reach >> f) & 1u) && bbox_hit(Fe[f], x, xe));
      if (kReach2<NG> && any) {
        reach = reachable_faces_taylor<NG>(m, e, Xe, xi, x, xe, L2, reach) | keep;
        any = false;
#pragma unroll 1
        for (int f = 0; f < 6; ++f) any = any || (((reach >> f) & 1u) && bbox_hit(Fe[f], x, xe));
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      P.x[k * cap + p] = xe[k];
      P.v[k * cap + p] = v[k];
      P.kx[k * cap + p] = kx[k];
      P.kv[k * cap + p] = kv[k];
    }
    if (any) {
      trk = true;
      xs0 = x[0]; xs1 = x[1]; xs2 = x[2];
    }
  }
  __shared__ int sh[2 * kElemWaves + 2];
  int s1, s2;
  block_push2<kElemWaves>(q.counters, strag, trk, sh, s1, s2);
  if (strag) q.strag[s1] = (int32_t)p;
  wave_add(stats + ST_STRAG * kStatSlots, strag ? 1 : 0);
  wave_add(stats + ST_TRACKQ * kStatSlots, trk ? 1 : 0);
  if (trk) {
    q.trk_p[s2] = (int32_t)p;
    q.trk_m[s2] = (uint8_t)reach;
    q.trk_x[s2] = xs0;
    q.trk_x[cap + s2] = xs1;
    q.trk_x[2 * cap + s2] = xs2;
  }
  wave_add(stats + ST_NEWTON_IT * kStatSlots, it_sum);
  wave_add(stats + ST_NEWTON_CALLS * kStatSlots, calls);
  wave_add(stats + ST_FALLBACK * kStatSlots, fb);
}

// per-lane stage for the straggler queue (list != null) or all n particles;
// updated particles whose segment touches a face box go to the tracking queue
template <int NN, int NG, typename UT, bool MIXED, bool MLP>
__global__ __launch_bounds__(256) void k_stage_lane(MeshView m, const int32_t* __restrict__ list, int64_t n_all,
                                                    Particles P, Fluid fl, StepParams sp, Queues q,
                                                    unsigned long long* stats) {
  constexpr int NG3 = NG * NG * NG, NN3 = NN * NN * NN;
  const int64_t count = list ? (int64_t)q.counters[0] : n_all;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t cap = P.cap;
  int it_sum = 0, calls = 0, fb = 0, nlost = 0, nrec = 0;
  // the workgroup's 256 queue entries of an iteration sorted by element in
  // LDS (bitonic), so that the lanes of a wavefront that share an element
  // read its geometry and fluid state at the same addresses
  __shared__ int32_t skey[256], sval[256];
  __shared__ int shq[5];
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < count; base += stride) {
    const int64_t i = base + threadIdx.x;
    bool trk = false;
    int64_t p = 0;
    double xs0 = 0, xs1 = 0, xs2 = 0;
    unsigned reach = 0x3Fu;
    bool have = i < count;
    if (list) {
      const int32_t pl = have ? list[i] : -1;
      skey[threadIdx.x] = have ? P.elem[pl] : 0x7fffffff;
      sval[threadIdx.x] = pl;
      __syncthreads();
      for (int k = 2; k <= 256; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
          const int t = threadIdx.x, o = t ^ j;
          if (o > t) {
            const bool up = (t & k) == 0;
            const int32_t a = skey[t], b = skey[o];
            if ((a > b) == up) {
              skey[t] = b; skey[o] = a;
              const int32_t va = sval[t];
              sval[t] = sval[o]; sval[o] = va;
            }
          }
          __syncthreads();
        }
      const int32_t ps = sval[threadIdx.x];
      have = ps >= 0;
      p = have ? ps : 0;
      __syncthreads();   // skey / sval are rewritten in the next iteration
    } else {
      p = i;
    }
    if (have) {
      if (P.status[p] == ACTIVE) {
        int e = P.elem[p];
        double x[3] = {P.x[p], P.x[cap + p], P.x[2 * cap + p]};
        double xi[3];
        double gw[3], Ji[9];
        const bool wv = sp.warm && warm_guess(P, p, gw);
        const bool lg = MLP && sp.mlp_guess && !wv;   // computed only without continued coordinates
        float gl[3] = {0.f, 0.f, 0.f};
        if (lg) {
          gl[0] = sp.mlp_guess[p]; gl[1] = sp.mlp_guess[cap + p]; gl[2] = sp.mlp_guess[2 * cap + p];
        }
        bool ok = locate_xi_e<NN, NG, MLP>(m, e, m.X + (size_t)e * NG3 * 3, m.xnode + (size_t)e * NN3 * 3, x, xi,
                                           sp.max_it, it_sum, calls, fb, lg, gl, wv, gw, Ji,
                                           MIXED ? kNewtonTolMixed : kNewtonTol);
        bool inside = ok && inside_ref(xi);
        const bool direct = inside;   // located in the recorded element (Ji belongs to this xi)
        if (!ok) {
          // Newton diverges in the recorded element: the point left it along a
          // segment that was not traced (reference-space localisation), and the
          // map continued beyond a strongly curved element need not be
          // invertible there; the paper's localisation takes the
          // background-mesh candidates of the point
          const int f = bgm_locate<NN, NG>(m, x, xi, it_sum, calls, fb);
          if (f >= 0) {
            ok = inside = true;
            e = f;
            nrec++;
            P.elem[p] = e;
          }
        } else if (!inside) {
          inside = recover_elem<NN, NG>(m, e, x, xi, sp.max_it, it_sum, calls, fb);
          if (inside) {
            nrec++;
            P.elem[p] = e;
          }
        }
        if (!ok) {
          P.status[p] = LOST_NEWTON;
          nlost++;
        } else if (!inside) {
          P.status[p] = LOST_TRACK;
          nlost++;
        } else {
          double v[3] = {P.v[p], P.v[cap + p], P.v[2 * cap + p]};
          double kx[3] = {P.kx[p], P.kx[cap + p], P.kx[2 * cap + p]};
          double kv[3] = {P.kv[p], P.kv[cap + p], P.kv[2 * cap + p]};
          if (sp.warm) {
            if (direct) {
              double xe1[3];
#pragma unroll
              for (int k = 0; k < 3; ++k) xe1[k] = x[k] + sp.B * (sp.A * kx[k] + sp.dt * v[k]);
              store_warm(P, p, xi, Ji, x, xe1);
            } else {
              P.xi[p] = NAN;   // located by a recovery: no Jacobian of this xi at hand
            }
          }
          double xe[3];
          const UT* Ue = (const UT*)fl.U + (size_t)e * 5 * NN3;
          const double* Xe = m.X + (size_t)e * NG3 * 3;
          if (sp.forces) stage_update<NN, NG, UT, MIXED, true>(m, Ue, Xe, xi, x, v, kx, kv, P.d[p], fl, sp, xe);
          else stage_update<NN, NG, UT, MIXED, false>(m, Ue, Xe, xi, x, v, kx, kv, P.d[p], fl, sp, xe);
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            P.x[k * cap + p] = xe[k];
            P.v[k * cap + p] = v[k];
            P.kx[k * cap + p] = kx[k];
            P.kv[k * cap + p] = kv[k];
          }
          // the same prefilter as the element kernel: reference-space skip,
          // then the bounding boxes of the faces the segment can reach
          const double L2 = (xe[0] - x[0]) * (xe[0] - x[0]) + (xe[1] - x[1]) * (xe[1] - x[1]) +
                            (xe[2] - x[2]) * (xe[2] - x[2]);
          const double ds = m.dsafe[e];
          if (!(sp.refspace && L2 < ds * ds)) {
            const FaceRec* Fe = m.faces + (size_t)e * 6;
            const unsigned keep = boundary_faces(Fe);
            reach = reachable_faces(m, e, xi, L2) | keep;
#pragma unroll 1
            for (int f = 0; f < 6 && !trk; ++f) trk = ((reach >> f) & 1u) && bbox_hit(Fe[f], x, xe);
            if (kReach2<NG> && trk) {
              reach = reachable_faces_taylor<NG>(m, e, Xe, xi, x, xe, L2, reach) | keep;
              trk = false;
#pragma unroll 1
              for (int f = 0; f < 6 && !trk; ++f) trk = ((reach >> f) & 1u) && bbox_hit(Fe[f], x, xe);
            }
          }
          xs0 = x[0]; xs1 = x[1]; xs2 = x[2];
        }
      }
    }
    const int s = block_push<4>(q.counters + 1, trk, shq);   // the loop is uniform over the workgroup
    if (trk) {
      q.trk_p[s] = (int32_t)p;
      q.trk_m[s] = (uint8_t)reach;
      q.trk_x[s] = xs0;
      q.trk_x[cap + s] = xs1;
      q.trk_x[2 * cap + s] = xs2;
    }
  }
  wave_add(stats + ST_NEWTON_IT * kStatSlots, it_sum);
  wave_add(stats + ST_NEWTON_CALLS * kStatSlots, calls);
  wave_add(stats + ST_FALLBACK * kStatSlots, fb);
  wave_add(stats + ST_RECOVER * kStatSlots, nrec);
  wave_add(stats + ST_LOST * kStatSlots, nlost);
}

// MORT: the mesh has non-conforming (mortar) faces; conforming meshes run the
// variant without that part of the state machine (fewer registers)
template <int NG, bool MORT>
__global__ __launch_bounds__(256) void k_track(MeshView m, Particles P, Queues q, StepParams sp,
                                               unsigned long long* stats) {
  int ncross = 0, nhits = 0;
  track_queue<NG, MORT>(m, P, q.trk_p, q.trk_x, q.trk_m, q.counters + 2, q.counters[1], sp.max_cross, ncross, nhits);
  wave_add(stats + ST_CROSS * kStatSlots, ncross);
  wave_add(stats + ST_HITS * kStatSlots, nhits);
}

__global__ void k_reset_counters(int32_t* c) {
  if (threadIdx.x < 3) c[threadIdx.x] = 0;   // stragglers, tracking queue, its head
}

// Reference coordinates of the final positions along the element tasks of
// the step's sort: the task element's geometry nodes staged in LDS as in the
// stage kernel, one Newton per particle (from its continued coordinates when
// the step kept them); particles that left the task's element, or are not
// located inside it, go to the list that the per-lane pass finishes.
template <int NN, int NG, int TP>
__global__ __launch_bounds__(64 * elem_waves(TP)) void k_finalize_elem(MeshView m, const Task* __restrict__ tasks,
                                                                        const int32_t* __restrict__ ntask,
                                                                        Particles P, int warm, Queues q,
                                                                        unsigned long long* stats) {
  constexpr int NG3 = NG * NG * NG, NN3 = NN * NN * NN;
  constexpr int kW = elem_waves(TP), PER = 64 / TP, SLOTS = kW * PER;
  __shared__ double sX[SLOTS][NG3 * 3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int half = (TP == 64) ? 0 : lane / TP, tl = lane % TP, slot = w * PER + half;
  const int wid = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kW + w));
  const int ti = wid * PER + half;
  const int nt = __builtin_amdgcn_readfirstlane(*ntask);
  const int64_t cap = P.cap;
  int it_sum = 0, calls = 0, fb = 0;
  bool strag = false;
  int64_t p = 0;
  Task t{0, 0, 0, 0};
  if (ti < nt) {
    t = tasks[ti];
    const int e = (TP == 64) ? __builtin_amdgcn_readfirstlane(t.e) : t.e;
    const double* Xg = m.X + (size_t)e * NG3 * 3;
    for (int i = tl; i < NG3 * 3; i += TP) sX[slot][i] = Xg[i];
  }
  __syncthreads();
  if (ti < nt && tl < t.cnt) {
    const int e = t.e;
    p = (int64_t)t.p0 + tl;
    if (P.status[p] == ACTIVE) {
      if (P.elem[p] != e) {
        strag = true;
      } else {
        const double x[3] = {P.x[p], P.x[cap + p], P.x[2 * cap + p]};
        double xi[3], gw[3];
        const bool wv = warm && warm_guess(P, p, gw);
        if (locate_xi_e<NN, NG, false>(m, e, sX[slot], m.xnode + (size_t)e * NN3 * 3, x, xi, 50, it_sum, calls, fb,
                                       false, nullptr, wv, gw) &&
            inside_ref(xi)) {
#pragma unroll
          for (int k = 0; k < 3; ++k) P.xi[k * cap + p] = xi[k];
        } else {
          strag = true;
        }
      }
    }
  }
  __shared__ int sh[kW + 1];
  const int s1 = block_push<kW>(q.counters + 0, strag, sh);
  if (strag) q.strag[s1] = (int32_t)p;
}



// Fluid force of the FP32 shape-kernel source (drag only, FP32 state) along
// the element tasks of the source's sort: the element's state staged in LDS,
// the interpolation for the whole wavefront on the matrix cores, drag in FP32.
// F and ok are cleared beforehand; particles outside their element's
// reference cube (not located) deposit nothing, as in the per-lane kernel.
template <int NN, int TP>
__global__ __launch_bounds__(64 * elem_waves(TP)) void k_dep_force_elem(MeshView m, const Task* __restrict__ tasks,
                                                                         const int32_t* __restrict__ ntask,
                                                                         Particles P, Fluid fl, int drag,
                                                                         double* __restrict__ F,
                                                                         int32_t* __restrict__ ok,
                                                                         unsigned long long* povh) {
  constexpr int NN3 = NN * NN * NN;
  constexpr int kW = elem_waves(TP), PER = 64 / TP, SLOTS = kW * PER;
  __shared__ float sU[SLOTS][kInterpVars * NN3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int half = (TP == 64) ? 0 : lane / TP, tl = lane % TP, slot = w * PER + half;
  const int wid = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kW + w));
  const int ti = wid * PER + half;
  const int nt = __builtin_amdgcn_readfirstlane(*ntask);
  const int64_t cap = P.cap;
  Task t{0, 0, 0, 0};
  if (ti < nt) {
    t = tasks[ti];
    const float* Ug = (const float*)fl.U + (size_t)t.e * 5 * NN3;
    for (int i = tl; i < kInterpVars * NN3; i += TP) sU[slot][i] = Ug[i];
  }
  __syncthreads();
  bool act = false;
  int64_t p = 0;
  double xi[3] = {0.0, 0.0, 0.0};
  if (ti < nt && tl < t.cnt) {
    p = (int64_t)t.p0 + tl;
    if (P.status[p] == ACTIVE) {
      const int e = t.e;
      double ov = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double xk = P.x[k * cap + p];
        ov = fmax(ov, fmax(m.elo[e * 3 + k] - xk, xk - m.ehi[e * 3 + k]));
      }
      if (ov > 0.0) atomicMax(povh, (unsigned long long)__double_as_longlong(ov));
      const double xq[3] = {P.xi[p], P.xi[cap + p], P.xi[2 * cap + p]};
      act = inside_ref(xq);
      if (act) {
        xi[0] = xq[0]; xi[1] = xq[1]; xi[2] = xq[2];
      }
    }
  }
  float Uc[kInterpVars];
  if (wid * PER < nt) interp_f32_mfma<NN>(m, sU[slot], xi, Uc);
  if (act) {
    const double v[3] = {P.v[p], P.v[cap + p], P.v[2 * cap + p]};
    const float vf[3] = {(float)v[0], (float)v[1], (float)v[2]};
    const float ir = 1.0f / Uc[0];
    const float u[3] = {Uc[1] * ir, Uc[2] * ir, Uc[3] * ir};
    const float d = (float)P.d[p], mu = (float)fl.mu;
    float a[3], fD;
    drag_accel<float>(drag, Uc[0], u, vf, d, mu, (float)fl.rho_p, a, fD);
    const float c = 3.0f * (float)M_PI * mu * d * fD;
    double* Fp = F + p * 4;
    double Fq[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) Fq[k] = (double)(c * (u[k] - vf[k]));
    Fp[0] = Fq[0];
    Fp[1] = Fq[1];
    Fp[2] = Fq[2];
    Fp[3] = Fq[0] * v[0] + Fq[1] * v[1] + Fq[2] * v[2];
    ok[p] = 1;
  }
}

__global__ void k_dep_clear(double* F, int32_t* ok, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) F[p * 4 + k] = 0.0;
  ok[p] = 0;
}

// tasks of <= tp particles per element after the counting sort
__global__ void k_task_count(const int32_t* __restrict__ count, int E, int tp, int32_t* tcount) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) tcount[e] = (count[e] + tp - 1) / tp;
  else if (e == E) tcount[E] = 0;
}

__global__ void k_task_fill(const int32_t* __restrict__ count, const int32_t* __restrict__ start,
                            const int32_t* __restrict__ tstart, int E, int tp, Task* tasks, int32_t* ntask,
                            int64_t max_tasks) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int c = count[e], t0 = tstart[e], s0 = start[e];
  for (int j = 0; tp * j < c && (int64_t)t0 + j < max_tasks; ++j) {
    Task t;
    t.e = e;
    t.p0 = s0 + tp * j;
    t.cnt = min(tp, c - tp * j);
    t.pad = 0;
    tasks[t0 + j] = t;
  }
  if (e == E - 1) *ntask = (int32_t)min((int64_t)tstart[E], max_tasks);
}

hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* sums, hipStream_t s);

hipError_t launch_tasks(const int32_t* count, const int32_t* start, int E, int tp, int32_t* tcount, int32_t* tstart,
                        int32_t* sums, void* tasks, int32_t* ntask, int64_t max_tasks, hipStream_t s) {
  dim3 g((unsigned)((E + 1 + 255) / 256));
  k_task_count<<<g, 256, 0, s>>>(count, E, tp, tcount);
  hipError_t err = scan_i32(tcount, tstart, E + 1, sums, s);
  if (err != hipSuccess) return err;
  k_task_fill<<<g, 256, 0, s>>>(count, start, tstart, E, tp, (Task*)tasks, ntask, max_tasks);
  return hipGetLastError();
}

size_t task_bytes() { return sizeof(Task); }

#include "fp_shapes.h"

hipError_t launch_finalize_elem(const MeshView& m, const Particles& P, const void* tasks, const int32_t* ntask, int tp,
                                int64_t n, int warm, int32_t* counters, int32_t* list, unsigned long long* stats,
                                hipStream_t s) {
  Queues q{counters, list, nullptr, nullptr, nullptr};
  k_reset_counters<<<1, 64, 0, s>>>(counters);
  const int64_t max_tasks = (int64_t)m.E + P.cap / tp + 1;
#define FP_L(A, B)                                                                                         \
  if (m.n == A && m.ng == B) {                                                                             \
    if (tp == 64) {                                                                                        \
      const int64_t waves = max_tasks;                                                                     \
      k_finalize_elem<A, B, 64><<<dim3((unsigned)((waves + elem_waves(64) - 1) / elem_waves(64))),         \
                                  64 * elem_waves(64), 0, s>>>(m, (const Task*)tasks, ntask, P, warm, q, stats); \
    } else if (tp == 32) {                                                                                 \
      const int64_t waves = (max_tasks + 1) / 2;                                                           \
      k_finalize_elem<A, B, 32><<<dim3((unsigned)((waves + elem_waves(32) - 1) / elem_waves(32))),         \
                                  64 * elem_waves(32), 0, s>>>(m, (const Task*)tasks, ntask, P, warm, q, stats); \
    } else {                                                                                               \
      return hipErrorInvalidValue;                                                                         \
    }                                                                                                      \
    return launch_finalize(m, P, n, list, counters, warm, stats, s);                                       \
  }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

hipError_t launch_dep_force_elem(const MeshView& m, const Particles& P, const Fluid& fl, int drag,
                                 const void* tasks, const int32_t* ntask, int tp, int64_t n, double* F,
                                 int32_t* ok, unsigned long long* povh, hipStream_t s) {
  if (!fl.f32 || (tp != 32 && tp != 64)) return hipErrorInvalidValue;
  k_dep_clear<<<dim3((unsigned)((std::max<int64_t>(n, 1) + 255) / 256)), 256, 0, s>>>(F, ok, n);
  const int64_t max_tasks = (int64_t)m.E + P.cap / tp + 1;
  const int64_t waves = tp == 64 ? max_tasks : (max_tasks + 1) / 2;
  const int nw = elem_waves(tp);
  const dim3 g((unsigned)((waves + nw - 1) / nw));
#define FP_L(A, B)                                                                                             \
  if (m.n == A && m.ng == B) {                                                                                 \
    if (tp == 64)                                                                                              \
      k_dep_force_elem<A, 64><<<g, 64 * nw, 0, s>>>(m, (const Task*)tasks, ntask, P, fl, drag, F, ok, povh);   \
    else                                                                                                       \
      k_dep_force_elem<A, 32><<<g, 64 * nw, 0, s>>>(m, (const Task*)tasks, ntask, P, fl, drag, F, ok, povh);   \
    return hipGetLastError();                                                                                  \
  }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

// the element kernel runs when tasks of its size exist (with the extra forces
// it has an instantiation of its own, except together with the learned guess)
bool stage_uses_tasks(const StageLaunch& L) {
  return L.tasks != nullptr && L.task_tp == task_particles(L.m.n, L.m.ng, L.mixed != 0) &&
         (L.sp.forces == 0 || !L.mlp);
}

template <int NN, int NG, typename UT, bool MIXED, bool MLP>
static void run_stage(const StageLaunch& L, hipStream_t s) {
  const MeshView& m = L.m;
  Queues q{L.counters, L.strag, L.trk_p, L.trk_x, L.trk_m};
  int64_t lane_blocks;
  auto rec = [&](int i) { if (L.ev[i]) hipEventRecord(L.ev[i], s); };
  if (MLP && L.sp.mlp_guess) {
    // the straggler list and its counter hold the guess list until the reset
    rec(6);
    (void)launch_mlp_guess(m, L.P, L.n, L.sp.warm, L.strag, L.counters, const_cast<float*>(L.sp.mlp_guess), s);
    rec(7);
  }
  k_reset_counters<<<1, 64, 0, s>>>(L.counters);
  if (stage_uses_tasks(L)) {
    // at most E + cap / tp + 1 tasks, 64 / tp per wavefront
    constexpr int tp = task_particles(NN, NG, MIXED), nw = elem_waves(tp);
    const int64_t max_tasks = (int64_t)m.E + L.P.cap / tp + 1;
    const int64_t waves = (max_tasks * tp + 63) / 64;
    rec(0);
    const dim3 grid((unsigned)((waves + nw - 1) / nw));
    if (!MLP && L.sp.forces)
      k_stage_elem<NN, NG, UT, MIXED, false, true><<<grid, 64 * nw, 0, s>>>(
          m, m.X, m.xnode, (const UT*)L.fl.U, m.faces, (const Task*)L.tasks, L.ntask, L.P, L.fl, L.sp, q, L.stats);
    else
      k_stage_elem<NN, NG, UT, MIXED, MLP, false><<<grid, 64 * nw, 0, s>>>(
          m, m.X, m.xnode, (const UT*)L.fl.U, m.faces, (const Task*)L.tasks, L.ntask, L.P, L.fl, L.sp, q, L.stats);
    rec(1);
    lane_blocks = std::min<int64_t>((L.n + 255) / 256, 256);
    rec(2);
    k_stage_lane<NN, NG, UT, MIXED, MLP><<<dim3((unsigned)std::max<int64_t>(lane_blocks, 1)), 256, 0, s>>>(
        m, L.strag, L.n, L.P, L.fl, L.sp, q, L.stats);
    rec(3);
  } else {
    lane_blocks = (L.n + 255) / 256;
    rec(2);
    k_stage_lane<NN, NG, UT, MIXED, MLP><<<dim3((unsigned)std::max<int64_t>(lane_blocks, 1)), 256, 0, s>>>(
        m, nullptr, L.n, L.P, L.fl, L.sp, q, L.stats);
    rec(3);
  }
  int64_t trk_blocks = std::max<int64_t>(1, std::min<int64_t>((L.n + 255) / 256, 1024));
  rec(4);
  if (m.n_mortar > 0) k_track<NG, true><<<dim3((unsigned)trk_blocks), 256, 0, s>>>(m, L.P, q, L.sp, L.stats);
  else k_track<NG, false><<<dim3((unsigned)trk_blocks), 256, 0, s>>>(m, L.P, q, L.sp, L.stats);
  rec(5);
}

hipError_t launch_stage(const StageLaunch& L, hipStream_t s) {
  if (L.n == 0) return hipSuccess;
  const MeshView& m = L.m;
  const bool f32 = L.fl.f32 != 0, mixed = L.mixed != 0, mlp = L.mlp != 0;
#define FP_L(A, B)                                                                            \
  if (m.n == A && m.ng == B) {                                                                \
    if (mixed != f32) return hipErrorInvalidValue;                                            \
    if (mlp) {                                                                                \
      if (f32) run_stage<A, B, float, true, true>(L, s);                                      \
      else run_stage<A, B, double, false, true>(L, s);                                        \
    } else if (f32) run_stage<A, B, float, true, false>(L, s);                                \
    else run_stage<A, B, double, false, false>(L, s);                                         \
    return hipGetLastError();                                                                 \
  }
  FP_FOR_EACH_SHAPE(FP_L)
#undef FP_L
  return hipErrorInvalidValue;
}

}  // namespace fp

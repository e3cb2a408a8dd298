// Internal structures of the flexipart HIP library (gfx950).  Shared by the
// host API and the kernels of this library only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fp {

constexpr int kMaxNodes = 8;        // n = N+1 <= 8, ng = Ngeo+1 <= 7
constexpr int kClipStack = 16;      // Bezier-clipping interval stack
constexpr int kClipSteps = 64;      // clipping iterations per face test
constexpr int kMaxRoots = 8;
constexpr int kMlpMaxBatch = 8192;   // rows per MLP gradient evaluation
constexpr int kMlpStaticRows = 4096; // rows of fp_mlp_loss_grad_static (fixed device array)
constexpr int kMlpIn = 84;           // learned-guess inputs: corners, curvature, point
constexpr int kMlpRow = kMlpIn + 6 * 64 + 3;  // activations and deltas kept per row
constexpr int kMlpWeights = 64 * kMlpIn + 64 + 2 * (64 * 64 + 64) + 3 * 64 + 3;
constexpr double kNewtonTol = 1e-10;
// Newton's acceptance in the mixed stage, whose interpolation is FP32: a step
// of at most 1e-5 in the quadratic regime leaves an error of about
// (M / 2) 1e-10, M = |J^-1| |second derivatives of the map| (below 1 on the
// workloads' elements), far below the FP32 interpolation's resolution
constexpr double kNewtonTolMixed = 1e-5;
constexpr double kInsideEps = 1e-10;
constexpr double kUVEps = 1e-12;
constexpr double kClipTol = 1e-12;
constexpr double kClipPad = 1e-10;
constexpr double kEntryRel = 1e-9;   // entry-face root threshold, relative to the face diameter
// sign that turns dp/du x dp/dv of local face f into its outward normal (face
// parameters are the two other reference axes in increasing order, J > 0)
__device__ constexpr double kFaceSign[6] = {-1.0, 1.0, 1.0, -1.0, -1.0, 1.0};
constexpr int kRecoverHops = 3;      // neighbour hops when a located particle lies outside its element

enum { ACTIVE = 0, OPEN_EXIT = 1, LOST_NEWTON = 2, LOST_TRACK = 3, MAX_CROSS = 4, REJECTED = 5 };
enum { FACE_PLANAR = 0, FACE_BILINEAR = 1, FACE_CURVED = 2 };
enum { BC_INTERNAL = 0, BC_OPEN = 1, BC_REFLECT = 2, BC_PERIODIC = 3, BC_MORTAR = 4 };
enum { ST_NEWTON_IT = 0, ST_NEWTON_CALLS, ST_CROSS, ST_HITS, ST_LOST, ST_FALLBACK, ST_STRAG, ST_TRACKQ, ST_RECOVER,
       ST_DEP_PAIRS, ST_N };
constexpr int kStatSlots = 64;   // each counter is spread over slots (blockIdx % 64) to avoid atomic contention

// One element face: slab bounding box (Sec. 3.2.4), corner bilinear form,
// connectivity.  Bezier control points live in a separate array.
struct FaceRec {
  double nrm[3], e1[3], e2[3], org[3];
  double lo[3], hi[3];          // extents along (nrm, e1, e2) relative to org
  double A[3], B[3], C[3], D[3];// p(u,v) = A uv + B u + C v + D from the corners
  double shift[3];
  double diam;
  int32_t type, nbr_elem, nbr_face, bc;
};

// Everything a kernel needs to know about the mesh (passed by value).
struct MeshView {
  int32_t E, ng, n, n_geo;
  const double* X;        // [E][ng^3][3]
  const FaceRec* faces;   // [E*6]
  const double* cp;       // [E*6][ng*ng][3]
  const double* hE;       // [E]
  const double* xnode;    // [E][n^3][3] physical DG node positions
  const double* vol;      // [E][n^3]
  const double* elo;      // [E][3] padded element box
  const double* ehi;
  const double* nbox;     // [E][6] box of the DG nodes (lo xyz, hi xyz)
  const double* dsafe;    // [E] lower bound of the distance to a face that is not internal
  const double* gxi;      // [E][6] upper bounds over the element of |grad xi_i| (0..2) and of the norm of
                          // the Hessian of xi_i (3..5) (sampled, with margins)
  const int32_t* mortar;  // [n_mortar][4][2] (small element, local face) per big mortar face, -1 unused
  int32_t n_mortar;
  double xgeo[kMaxNodes], cgeo[kMaxNodes];  // geometry nodes, 1/prod(x_i - x_j)
  double xdg[kMaxNodes], cdg[kMaxNodes], wdg[kMaxNodes];
  float xdgf[kMaxNodes], cdgf[kMaxNodes];
  double blo[3], bdx[3];
  int32_t bn[3];
  const int32_t* bstart;  // background-mesh cell -> element CSR
  const int32_t* blist;
  const uint8_t* mlp_flag;// [E] learned guess enabled
  const float* mlp_w;     // weights (device), or null
  const float* mlp_h1;    // [E][64] first layer's pre-activation from the element inputs (bias included)
  const double* mlp_ctr;  // [E][4] corner mean (xyz) and length scale of the inputs (1 / mean corner edge)
};

// Particle state, structure of arrays, capacity cap.
struct Particles {
  int64_t cap;
  double* x;      // [3][cap]
  double* v;      // [3][cap]
  double* kx;     // [3][cap]
  double* kv;     // [3][cap]
  double* d;      // [cap]
  double* xi;     // [3][cap]
  int32_t* elem;
  int32_t* hits;
  int32_t* id;    // index in push order
  int8_t* status;
};

struct Fluid {
  const void* U;
  int32_t f32;    // U stored as float
  double mu, kappa, rho_p;
};

// conservative variables the drag law reads (density, momentum): with
// constant viscosity the energy is never used
constexpr int kInterpVars = 4;

// particles per element task after the counting sort: two tasks per
// wavefront, one per half (32), when the stage is mixed and four elements'
// geometry nodes and FP32 state fit in 27 KB of LDS (three two-wavefront
// workgroups per SIMD); one task per wavefront (64) otherwise
__host__ __device__ constexpr int task_particles(int nn, int ng, bool mixed) {
  return (mixed && 4 * (ng * ng * ng * 3 * 8 + kInterpVars * nn * nn * nn * 4) <= 27 * 1024) ? 32 : 64;
}
constexpr int kMinTaskParticles = 32;

// extra terms of the equation of motion (eq. theory:maxey), bit flags
constexpr int kForceBuoyancy = 1, kForceStress = 2, kForceAddedMass = 4, kForceSaffman = 8;
constexpr int kForceAll = 15;

struct StepParams {
  double dt;
  double A, B;          // low-storage coefficients of this stage
  double gravity[3];
  int32_t drag, max_it, max_cross, use_mlp;
  int32_t refspace;     // reference-space localisation of segments that cannot reach a boundary face
  int32_t forces;       // kForce* terms beyond drag and gravity
  const float* mlp_guess;   // [3][cap] learned guesses of the stage (flagged elements), or null
  int32_t warm;             // locate from the particle's continued reference coordinates (P.xi) first
};

// force model of the two-way source (the fluid force of the equation of motion)
struct ForceModel {
  double gravity[3];
  int32_t drag, forces;
};

}  // namespace fp

/*
 * flexipart: MI355X (gfx950) library for the per-particle Lagrangian step of a
 * DGSEM particle framework (Kopper et al., "A framework for high-fidelity
 * particle tracking on massively parallel systems", arXiv 2211.05458).
 *
 * One call of fp_step advances every active particle through all stages of a
 * low-storage Runge-Kutta step: reference coordinates by Newton on the curved
 * element map (Sec. 3.2.1), tensor-product Lagrange interpolation of the DG
 * state (eq. part_interpolation), drag (eq. dragforce, dragfactor), the stage
 * update (Sec. 3.1/3.2.2) and physical-space tracking with face intersection,
 * element hand-off and wall reflection (Sec. 3.2.3, 3.2.4, 2.4).
 * fp_deposit_source projects the particle force back onto the DG nodes
 * (Sec. 2.3, eq. theory:source).
 *
 * Conventions common to every entry point
 *  - Every function returns 0 (FP_OK) on success or a negative fp_err code; a
 *    positive return is a warning.  fp_last_error(ctx) describes the last
 *    failure.  No C++ exception crosses this boundary.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory of the current device.  Every pointer is borrowed: the library
 *    never frees caller memory and never keeps a host pointer past the call.
 *    Device pointers given to fp_bind_workspace, fp_set_fluid_state and
 *    fp_mlp_set_weights must stay valid and unmodified until they are
 *    replaced or the context is destroyed.
 *  - The library never allocates device memory: all device state lives in the
 *    caller-allocated workspace (fp_workspace_size / fp_bind_workspace), or in
 *    a caller-allocated particle block (fp_bind_particles).
 *  - All device work is enqueued on the stream given to fp_create, in order.
 *    Only fp_push_particles, fp_read_particles, fp_get_stats,
 *    fp_bind_workspace, fp_newton_pairs, fp_mlp_set_weights and fp_mlp_train
 *    synchronise that stream.
 *  - Element local faces: 0: xi1=-1, 1: xi1=+1, 2: xi2=-1, 3: xi2=+1,
 *    4: xi3=-1, 5: xi3=+1.  Volume node index i + n*(j + n*k), i along xi1.
 */
#ifndef FLEXIPART_H
#define FLEXIPART_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fp_ctx fp_ctx;

enum fp_err {
  FP_OK = 0,
  FP_EINVAL = -1,   /* bad argument, size or unsupported degree */
  FP_EMESH = -2,    /* inconsistent mesh (non-reciprocal neighbours, J <= 0) */
  FP_EDEVICE = -3,  /* HIP runtime error */
  FP_ESTATE = -4,   /* call out of order (e.g. step before push) */
  FP_WDT = 1        /* warning: dt exceeds the stability bound of the drag term */
};
typedef enum { FP_F32 = 0, FP_F64 = 1 } fp_dtype;
/* FP_BC_MORTAR: the big side of a non-conforming face (Sec. 3.2.3), matched
 * by two or four small faces of neighbouring elements (fp_mesh_desc.mortar) */
typedef enum { FP_BC_INTERNAL = 0, FP_BC_OPEN = 1, FP_BC_REFLECT = 2, FP_BC_PERIODIC = 3, FP_BC_MORTAR = 4 } fp_bc;
/* per-particle status (not errors) */
enum { FP_ACTIVE = 0, FP_OPEN_EXIT = 1, FP_LOST_NEWTON = 2, FP_LOST_TRACK = 3,
       FP_MAX_CROSS = 4, FP_REJECTED = 5 };

/* Mesh of curved hexahedra (Sec. 3.1, eq. dgsem_curvedfaces): element e is the
 * tensor-product Lagrange map of degree n_geo through X[e], and the fluid state
 * is a tensor-product Lagrange polynomial of degree n_dg.  All pointers host. */
typedef struct {
  int32_t n_elem;
  int32_t n_geo;               /* geometry degree, 1..6 (nodes equidistant on [-1,1]) */
  const double* X;             /* [n_elem][(n_geo+1)^3][3] */
  const int32_t* nbr_elem;     /* [n_elem][6], neighbour across each local face (-1: none) */
  const int32_t* nbr_face;     /* [n_elem][6], the neighbour's local face */
  const int8_t* bc;            /* [n_elem][6], fp_bc */
  const double* periodic_shift;/* [n_elem][6][3], added to a particle crossing a periodic face */
  int32_t n_dg;                /* DG degree N, 1..7 */
  int32_t dg_nodes;            /* 0: Legendre-Gauss, 1: Legendre-Gauss-Lobatto */
  int32_t n_mortar;            /* number of big mortar faces (0: conforming mesh) */
  const int32_t* mortar;       /* [n_mortar][4][2]: (element, local face) of the small faces that tile
                                  big face m, (-1, -1) where unused (2:1); may be NULL if n_mortar = 0.
                                  A big face has bc FP_BC_MORTAR and nbr_elem = m (nbr_face unused);
                                  each small face is FP_BC_INTERNAL with the big element and face as its
                                  neighbour.  The small faces must tile the big one geometrically. */
} fp_mesh_desc;

/* Fluid and particle-material constants (Sec. 2.1, 2.2). */
typedef struct {
  double mu;      /* dynamic viscosity */
  double kappa;   /* ratio of specific heats (pressure from rho e) */
  double rho_p;   /* particle density */
} fp_fluid_params;

typedef struct {
  int32_t rk;            /* 0: 5-stage 4th-order low-storage RK (Carpenter-Kennedy), 1: 3-stage 3rd-order (Williamson) */
  int32_t drag;          /* 0: Stokes (f_D = 1), 1: Schiller-Naumann, 2: no drag */
  int32_t precision;     /* 0: FP64 throughout; 1: mixed (FP32 interpolation/drag/RK, FP64 Newton tail and tracking) */
  int32_t guess;         /* bit 0: learned guess on flagged elements (the paper's guess as fallback);
                            bit 1: first try each particle's reference coordinates of the previous
                            stage continued along its displacement (xi + J^-1 dx, kept from the
                            last Newton of that stage; not after a crossing or reflection);
                            with both bits, the learned guess is computed and used only for
                            the particles without such coordinates (their failures fall back
                            to the paper's guess);
                            0: the paper's initial guess (Sec. 3.2.1).  The converged xi is the
                            same from any guess in Newton's basin. */
  int32_t sort_every;    /* counting-sort particles by element every k steps (0: never;
                            negative: before every stage, so that the particles that
                            crossed a face run in their new element's task) */
  int32_t max_newton_it; /* Newton iteration cap (50) */
  int32_t max_crossings; /* face crossings per stage before FP_MAX_CROSS (64) */
  int32_t tracking;      /* 0: physical-space tracking of every segment (Sec. 3.2.3);
                            1: reference-space localisation: a segment that cannot reach a
                            face that is not internal (wall, open, periodic) is not traced,
                            the next location step finds its element */
  int32_t forces;        /* extra terms of the equation of motion (eq. theory:maxey), FP_F_* bits;
                            0: drag and gravity only (see below) */
  double gravity[3];     /* body acceleration g */
} fp_step_opts;

/* Extra terms of the particle equation of motion (Sec. 2.2, eq. theory:maxey)
 *   m_p dv/dt = F_D + m_f Du/Dt + m_f/2 (Du/Dt - dv/dt) + F_L + g (m_p - m_f)
 * with m_p = rho_p pi d^3/6 and m_f = rho pi d^3/6 (rho the interpolated fluid
 * density).  FP_F_BUOYANCY: body force g (m_p - m_f) instead of g m_p.
 * FP_F_STRESS: undisturbed-flow stress m_f Du/Dt.  FP_F_ADDED_MASS: the added
 * mass, solved implicitly ((m_p + m_f/2) dv/dt on the left).  FP_F_SAFFMAN:
 * Saffman lift with Mei's correction (Sec. 2.2.2), directed along (u - v) x w
 * (w the vorticity).  The fluid state is frozen over a step, so
 * Du/Dt = (u . grad) u from the interpolant's gradient.  Basset history and
 * Magnus lift are not provided.  Together with the learned guess (guess = 1)
 * these terms run through the per-lane stage kernel (slower). */
enum { FP_F_BUOYANCY = 1, FP_F_STRESS = 2, FP_F_ADDED_MASS = 4, FP_F_SAFFMAN = 8 };

/* Create a context bound to a HIP stream (hipStream_t, may be NULL for the
 * null stream) on the current device. */
int fp_create(fp_ctx** out, void* hip_stream);
void fp_destroy(fp_ctx* ctx);
const char* fp_last_error(fp_ctx* ctx);

/* Validate and stage a mesh (host).  Checks neighbour reciprocity; the
 * Jacobian sign is checked at fp_bind_workspace.  FP_EINVAL / FP_EMESH. */
int fp_init_mesh(fp_ctx* ctx, const fp_mesh_desc* desc);

/* Device bytes needed for the mesh plus up to max_particles particles. */
int fp_workspace_size(fp_ctx* ctx, int64_t max_particles, size_t* bytes);

/* Bind caller-allocated device memory (>= fp_workspace_size, 256-byte
 * aligned).  Uploads the mesh, builds the Bezier faces and their bounding
 * boxes (Sec. 3.2.4), DG node positions and volumes, and the background mesh
 * (Sec. 4.1.2).  Synchronises the stream. */
int fp_bind_workspace(fp_ctx* ctx, void* dev_ptr, size_t bytes);

/* Borrow the DG state U (device) [n_elem][5][(n_dg+1)^3]: the nodal values
 * U_ijk of the conservative variables (rho, rho u, rho e) of Sec. 2.1 that
 * the tensor-product Lagrange polynomial of Sec. 3.1 (eq.
 * dgsem_interpolation) interpolates, in FP64 or FP32; node index
 * i + n (j + n k).  params: viscosity, ratio of specific heats and particle
 * density (Sec. 2.1, 2.2).  The pointer must stay valid and unmodified until
 * it is replaced.  FP_EINVAL for a null pointer or a non-positive viscosity
 * or density. */
int fp_set_fluid_state(fp_ctx* ctx, const void* U_dev, fp_dtype dtype, const fp_fluid_params* params);

/* ---- particle block owned by the caller ----------------------------------
 * The particle state of Sec. 2.2 (position, velocity, diameter) together with
 * the low-storage Runge-Kutta registers of Sec. 3.2.2 and the reference
 * position of Sec. 3.2.1, as one structure-of-arrays block of capacity `cap`:
 *   offsets[0] x [3][cap] f64     offsets[1] v [3][cap] f64
 *   offsets[2] kx [3][cap] f64    offsets[3] kv [3][cap] f64 (RK registers)
 *   offsets[4] xi [3][cap] f64    offsets[5] d [cap] f64
 *   offsets[6] elem [cap] i32     offsets[7] wall hits [cap] i32
 *   offsets[8] id [cap] i32 (index in push order)
 *   offsets[9] status [cap] i8 (FP_ACTIVE, ...)
 * fp_particle_block_layout writes the ten byte offsets (host, may be NULL)
 * and the block size; the block is FP64 in both precisions (FP_EINVAL for
 * FP_F32: mixed precision rounds on load). */
int fp_particle_block_layout(int64_t capacity, fp_dtype dtype, int64_t* offsets, size_t* bytes);
/* Bind a caller-allocated device block of that layout (256-byte aligned,
 * 0 < capacity <= the workspace's particle capacity) as the context's
 * particle state, replacing the workspace's own buffer; soa_dev = NULL returns
 * to it.  Any particle set is dropped (push again).  After fp_push_particles,
 * fp_step and fp_deposit_source the block holds the current state, rows in
 * element order (id gives the push order); the sort's second buffer stays in
 * the workspace.  The block is borrowed: it must stay valid until it is
 * replaced or the context is destroyed. */
int fp_bind_particles(fp_ctx* ctx, int64_t capacity, fp_dtype dtype, void* soa_dev);

/* Insert n particles replacing any previous set: positions, velocities and
 * diameters (Sec. 2.2) as host arrays x[n][3], v[n][3], d[n]; or, with a
 * bound particle block, x = v = d = NULL to take the block's first n entries
 * of x, v and d as they are.  elem_hint[n] (host) or NULL.  Each particle is
 * located by Newton for its reference position (Sec. 3.2.1) in its hint
 * element, else in the candidates of the Cartesian background mesh (Sec.
 * 4.1.2) in element order; status_out (host, may be NULL) receives
 * FP_ACTIVE or FP_REJECTED (outside every element).  Returns the number of
 * rejected particles (>= 0), FP_EINVAL for n above the capacity or a
 * non-positive diameter.  Synchronises the stream. */
int fp_push_particles(fp_ctx* ctx, int64_t n, const double* x, const double* v, const double* d,
                      const int32_t* elem_hint, int32_t* status_out);

/* Advance all active particles by n_steps steps of size dt.  Each stage
 * locates the particle in its element by Newton (Sec. 3.2.1); one that lies
 * outside it (a crossing missed by the face intersection, at grazing incidence)
 * is followed across the face its reference coordinate left through, up to
 * three internal or periodic faces, before it is counted lost.  Asynchronous. */
int fp_step(fp_ctx* ctx, double dt, int32_t n_steps, const fp_step_opts* opts);

/* Add the two-way coupling source of the current particle state to S (device)
 * [n_elem][4][(n_dg+1)^3] (3 momentum components, energy), FP64 or FP32.
 * kind 0: nearest DOF, S = -F/V_ijk (Sec. 2.3).  kind 1: polynomial shape
 * kernel (1-(r/R)^2)^2 of radius `radius` over all DG nodes, normalised so that
 * sum_k S_k V_k = -F; period[3] (host, may be NULL) are the domain periods for
 * the minimum-image distance (0: not periodic).  Each positive period must
 * exceed 2 * radius (FP_EINVAL otherwise), so that at most one image of a node
 * lies within reach of a particle.  Particles with no node within reach deposit
 * nothing.  F is the fluid force of the equation of motion (eq. theory:source):
 * the drag law `drag` (as in fp_step_opts) plus the terms of `forces` (FP_F_*;
 * the added mass needs dv/dt, hence gravity[3], host, may be NULL for zero);
 * gravity and buoyancy themselves are not part of it.  Sorts the particles by
 * element.  Asynchronous. */
int fp_deposit_source(fp_ctx* ctx, void* S_dev, fp_dtype dtype, int32_t kind, double radius,
                      const double* period, int32_t drag, int32_t forces, const double* gravity);

/* Optional caller-allocated device memory (256-byte aligned) in which the FP32
 * shape-kernel source of fp_deposit_source (Sec. 2.3, kind 1, FP_F32) keeps,
 * per target element, the
 * particles its normalisation pass staged, so that the node-sum pass reads
 * them instead of staging them again (the same rows in the same order: the
 * same result).  Each element gets cap = (bytes - align256(4 n_elem)) /
 * (16 n_elem) rows (fp_deposit_list_bytes gives the bytes for a cap); a target
 * with more staged particles than cap stages again.  About
 * ppe (1 + 6 r + 3 pi r^2 + 4 pi r^3 / 3) particles are staged per target,
 * ppe = particles per element, r = radius / element width.  dev = NULL
 * unbinds.  FP_EINVAL if the memory holds fewer than 16 rows per element.
 * Borrowed until replaced or the context is destroyed. */
int fp_bind_deposit_list(fp_ctx* ctx, void* dev, size_t bytes);
int fp_deposit_list_bytes(fp_ctx* ctx, int32_t cap, size_t* bytes);

/* Copy the quadrature volumes V_ijk = w_i w_j w_k J(xi_ijk) of all DG nodes
 * (device output V[n_elem][(n_dg+1)^3], f64) -- the measure in which the
 * deposited source is conservative: sum_k S_k V_k = -sum_p F_p.  Async. */
int fp_node_volumes(fp_ctx* ctx, double* V_dev);

/* Copy the particle state to host buffers (any may be NULL) in the order of
 * fp_push_particles: position and velocity (Sec. 2.2), element, reference
 * position xi with chi_elem(xi) = x (Sec. 3.2.1; every active particle is
 * located first), wall-hit count (reflections, Sec. 2.4) and status.
 * Synchronises. */
int fp_read_particles(fp_ctx* ctx, int64_t* n, double* x, double* v, int32_t* elem, double* xi,
                      int32_t* wall_hits, int8_t* status);

/* Counters since the last reset (host out[11]): out[0] Newton iterations,
 * out[1] Newton solves, out[2] face crossings, out[3] wall hits, out[4] lost
 * particles, out[5] learned-guess fallbacks, out[6] sorts, out[7]
 * particle-stages taken by the per-lane kernel (they left their sorted element
 * or lie outside it), out[8] particle-stages queued for face intersection,
 * out[9] particles recovered in a neighbour element after a crossing the face
 * intersection missed (see fp_step), out[10] (particle, DG node) pairs within
 * the shape-kernel radius evaluated by FP32 sources (the kernel's unit of
 * work), counted only while fp_set_timing's bit 1 is set.  Synchronises. */
int fp_get_stats(fp_ctx* ctx, int64_t* out11);
int fp_reset_stats(fp_ctx* ctx);

/* ---- kernel timing (tracing) ---------------------------------------------
 * When enabled, HIP events on the context stream bracket every launch of the
 * step and source kernels.  fp_get_timing synchronises and writes, for each
 * class (0 sort, 1 element-wise stage kernel, 2 final reference coordinates,
 * 3 nearest-DOF source, 4 shape-kernel source (all of its kernels), 5 per-lane
 * stage kernel, 6 tracking kernel, 7 the shape-kernel source's normalisation
 * pass, 8 its node-sum pass, 9 the learned guesses of a stage), out[2*k] =
 * launches and out[2*k+1] = total
 * milliseconds since the last call; the counters are then cleared.
 * enable: bit 0 the events, bit 1 the count of shape-kernel pairs within the
 * radius (fp_get_stats out[10]), which costs the FP32 source's normalisation
 * pass one more VALU operation per pair. */
#define FP_TIMING_CLASSES 10
int fp_set_timing(fp_ctx* ctx, int32_t enable);
int fp_get_timing(fp_ctx* ctx, double* out /* [2*FP_TIMING_CLASSES] */);

/* ---- learned Newton initial guess (84-64-64-64-3 tanh MLP, FP32) --------- */
/* Extension of the initial-guess approaches of Sec. 3.2.1 (not in the paper).
 * Weight layout: W1[64][84] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3]. */
int64_t fp_mlp_n_weights(void);
/* Features of n (element, point) pairs: the 8 corners relative to their mean
 * (24), the deviation of the element map from the trilinear corner map at the
 * 19 non-corner points of the {-1,0,1}^3 lattice (57), and the point (3); all
 * divided by the mean corner-edge length (device in/out: elem[n] i32,
 * x[n][3] f64 -> feat[n][84] f32). */
int fp_mlp_features(fp_ctx* ctx, int64_t n, const int32_t* elem_dev, const double* x_dev, float* feat_dev);
/* Training pairs from the current particles: features and the converged
 * Newton xi (device outputs feat[n][84], xi[n][3]; ids[n], may be NULL,
 * receives each row's particle index in push order).  Rows are in no
 * particular order; *n = number of particles whose Newton solve converged
 * inside their element.  capacity (rows) must be >= the particle count. */
int fp_newton_pairs(fp_ctx* ctx, int64_t* n, float* feat_dev, float* xi_dev, int32_t* ids_dev, int64_t capacity);
/* Forward pass (device): out[n][3]. */
int fp_mlp_forward(fp_ctx* ctx, const float* w_dev, int64_t n, const float* in_dev, float* out_dev);
/* Mean squared error loss and its gradient over n rows (device; grad[nw]). */
int fp_mlp_loss_grad(fp_ctx* ctx, const float* w_dev, int64_t n, const float* in_dev,
                     const float* target_dev, float* grad_dev, float* loss_dev);
/* fp_mlp_loss_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * needs only fp_create (for the stream), no workspace.  The per-row
 * activations and deltas live in a fixed device array of the library
 * (FP_MLP_STATIC_ROWS rows of 471 floats, 7.7 MB on each GPU the library runs
 * on, held until the process ends); every row is written before it is read,
 * so nothing in it needs clearing.  All calls on one GPU share that array:
 * calls that overlap on one GPU (two streams, two threads) race.  Same
 * arguments and results as fp_mlp_loss_grad; n in [1, FP_MLP_STATIC_ROWS]
 * (FP_EINVAL otherwise).  Allocates nothing.  Asynchronous. */
#define FP_MLP_STATIC_ROWS 4096
int fp_mlp_loss_grad_static(fp_ctx* ctx, const float* w_dev, int64_t n, const float* in_dev,
                            const float* target_dev, float* grad_dev, float* loss_dev);
/* One epoch of minibatch Adam (beta1 0.9, beta2 0.999, eps 1e-8) in the row
 * order given by order_dev[n]; w, m, v (device, nw each) updated in place;
 * *t is the Adam step counter; loss_dev[n/batch] receives batch losses. */
int fp_mlp_train_epoch(fp_ctx* ctx, float* w_dev, float* m_dev, float* v_dev, int64_t* t,
                       const float* in_dev, const float* target_dev, const int32_t* order_dev,
                       int64_t n, int32_t batch, float lr, float* loss_dev);
/* Train the network from scratch on n (features, xi) rows (device
 * in[n][84], target[n][3], e.g. from fp_newton_pairs): Xavier-uniform initial
 * weights and zero biases, then `epochs` epochs of minibatch Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, step lr) on the mean squared error in batches of
 * `batch` rows (the last n mod batch rows of each epoch's order are left
 * out).  Every random draw comes from SplitMix64 seeded with `seed`: one
 * uniform per weight in layout order, then one Fisher-Yates shuffle of the
 * rows per epoch (a draw for i = n-1 down to 1, j = floor(u64 * (i+1) / 2^64)).
 * w_out (device, fp_mlp_n_weights floats) receives the trained weights;
 * loss_hist (host [epochs], may be NULL) the mean batch loss of each epoch.
 * FP_EINVAL for batch > 8192, n < batch or n above the workspace's particle
 * capacity.  Synchronises. */
int fp_mlp_train(fp_ctx* ctx, const float* in_dev, const float* target_dev, int64_t n, int32_t epochs,
                 int32_t batch, float lr, uint64_t seed, float* w_out_dev, float* loss_hist);
/* Enable the learned guess with weights w_dev (device; copied into the
 * workspace, so later changes of w_dev have no effect until the next call;
 * NULL disables the guess) on elements whose geometry deviates from the
 * trilinear corner map by > thresh * h_e. */
int fp_mlp_set_weights(fp_ctx* ctx, const float* w_dev, double thresh);
int fp_mlp_num_flagged(fp_ctx* ctx, int64_t* n);

#ifdef __cplusplus
}
#endif
#endif

// Kernel launchers of the flexipart library (host side declarations).
#pragma once
#include "fp_internal.h"

namespace fp {

// true if (n, ng) has compiled kernels
bool supported(int n, int ng);

hipError_t launch_face_setup(const MeshView& m, const double* X, const int32_t* nbr_elem, const int32_t* nbr_face,
                             const int8_t* bc, const double* shift, const double* Minv, FaceRec* faces, double* cp,
                             hipStream_t s);
hipError_t launch_nodes(const MeshView& m, double* xnode, double* vol, double* hE, double* nbox, double* gxi,
                        int32_t* bad, unsigned long long* node_pad, hipStream_t s);
hipError_t launch_locate(const MeshView& m, const Particles& P, const int32_t* hint, int64_t n, hipStream_t s);
// smallest of n doubles that are all positive, as the complement of its bit
// pattern (*inv_bits, zeroed by the caller, receives the largest complement),
// and the count of entries that are not positive and finite (*bad, zeroed)
hipError_t launch_min_positive(const double* d, int64_t n, unsigned long long* inv_bits, int32_t* bad,
                               hipStream_t s);
struct StageLaunch {
  MeshView m;
  Particles P;
  Fluid fl;
  StepParams sp;
  int64_t n;
  int mixed, mlp;
  const void* tasks;        // element tasks from the last sort, or null
  int task_tp;              // particles per task of those tasks
  const int32_t* ntask;
  int32_t* counters;        // queue counters [2]
  int32_t* strag;           // [cap]
  int32_t* trk_p;           // [cap]
  double* trk_x;            // [3][cap]
  uint8_t* trk_m;           // [cap] faces the first leg can reach
  unsigned long long* stats;
  hipEvent_t ev[8];         // optional (start, end) pairs around the elem, lane, track and learned-guess kernels
};
hipError_t launch_stage(const StageLaunch& L, hipStream_t s);
bool stage_uses_tasks(const StageLaunch& L);   // k_stage_elem runs (else all particles go per lane)
hipError_t launch_tasks(const int32_t* count, const int32_t* start, int E, int tp, int32_t* tcount, int32_t* tstart,
                        int32_t* sums, void* tasks, int32_t* ntask, int64_t max_tasks, hipStream_t s);
size_t task_bytes();
hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* sums, hipStream_t s);
hipError_t launch_finalize_elem(const MeshView& m, const Particles& P, const void* tasks, const int32_t* ntask, int tp,
                                int64_t n, int warm, int32_t* counters, int32_t* list, unsigned long long* stats,
                                hipStream_t s);
hipError_t launch_finalize(const MeshView& m, const Particles& P, int64_t n, const int32_t* list,
                           const int32_t* count, int warm, unsigned long long* stats,
                           hipStream_t s);
hipError_t launch_deposit_nearest(const MeshView& m, const Particles& P, const Fluid& fl, int64_t n, void* S,
                                  int s_f32, const ForceModel& fm, hipStream_t s);
hipError_t launch_deposit_shape(const MeshView& m, const Particles& P, const Fluid& fl, int64_t n, void* S,
                                int s_f32, const ForceModel& fm, double R, const double* period, double node_pad,
                                double* dep, const int32_t* elem_start, unsigned long long* povh,
                                unsigned long long* pairs, const int32_t* list_start, const int32_t* list,
                                double list_pad, void* reuse /* or null */, int32_t reuse_cap,
                                const void* tasks /* element tasks of the particles' order, or null */,
                                const int32_t* ntask, int task_tp,
                                hipEvent_t* ev /* [4] or null: around the two node passes */, hipStream_t s);
// fluid force (drag only) and validity of the FP32 shape-kernel source along
// the element tasks of the sort that precedes it (FP32 state)
hipError_t launch_dep_force_elem(const MeshView& m, const Particles& P, const Fluid& fl, int drag,
                                 const void* tasks, const int32_t* ntask, int tp, int64_t n, double* F,
                                 int32_t* ok, unsigned long long* povh, hipStream_t s);
// bytes of a source reuse list with cap rows per target element
inline size_t deposit_reuse_bytes(int E, int32_t cap) {
  return (((size_t)E * 4 + 255) & ~(size_t)255) + (size_t)E * cap * 16;
}
// candidate lists of the FP32 shape-kernel source: pass 0 counts per target
// (count[E + 1], last entry 0), pass 1 fills list at the scanned start[]
hipError_t launch_dep_lists(const MeshView& m, double R, const double* period, double pad, int pass,
                            int32_t* count, const int32_t* start, int32_t* list, hipStream_t s);
constexpr int kDepListPerElem = 256;   // workspace budget of candidate-list entries per element
hipError_t launch_sort(const Particles& src, const Particles& dst, int64_t n, int E, int32_t* count,
                       int32_t* start, int32_t* rank, int32_t* block_sums, hipStream_t s);
hipError_t launch_elem_start(const Particles& P, int64_t n, int E, int32_t* elem_start, hipStream_t s);

// learned guess
hipError_t launch_mlp_features(const MeshView& m, int64_t n, const int32_t* elem, const double* x, float* feat,
                               hipStream_t s);
hipError_t launch_newton_pairs(const MeshView& m, const Particles& P, int64_t n, float* feat, float* xi,
                               int32_t* ids, int32_t* count, hipStream_t s);
hipError_t launch_mlp_forward(const float* w, int64_t n, const float* in, float* out, hipStream_t s);
// learned guesses of the active particles in flagged elements that have no
// continued reference coordinates (all of them with warm == 0); list and
// count (device, cap and one entries) are scratch that this call overwrites
hipError_t launch_mlp_guess(const MeshView& m, const Particles& P, int64_t n, int warm, int32_t* list,
                            int32_t* count, float* guess, hipStream_t s);
hipError_t launch_mlp_loss_grad(const float* w, int64_t n, const float* in, const float* target,
                                const int32_t* rows, float* grad, float* loss, float* rowbuf, hipStream_t s);
// device address of the fixed row buffer of fp_mlp_loss_grad_static on the
// current device (kMlpStaticRows rows)
hipError_t mlp_static_rows(float** out);
hipError_t launch_adam(float* w, float* m, float* v, const float* g, int64_t nw, int64_t t, float lr,
                       hipStream_t s);
hipError_t launch_curved_flags(const MeshView& m, double thresh, uint8_t* flag, int32_t* count, hipStream_t s);
hipError_t launch_mlp_elem_table(const MeshView& m, const float* w, float* h1, double* ctr, hipStream_t s);

}  // namespace fp

// Host-side launchers of the libppp kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppp_internal.hpp"

namespace ppp {

bool chain_shape_supported(int G, int B);
int sim_blocks_per_cu(int precision, int G, int B, int lds_cap);  // resident workgroups of the persistent kernel
// workgroup-private xi histograms: up to this many bins live in LDS (else counts go straight to memory)
constexpr int kLdsHistCap = 16384;

hipError_t launch_sim(const DevProblem *d_probs, const WorkItem *d_items, int n_items, char *ws, int64_t step_begin,
                      int64_t step_end, int model, int precision, int G, int B, double *traj, int64_t traj_rep,
                      int lds_cap, hipStream_t stream);
hipError_t launch_sim_persistent(const DevProblem *d_probs, const WorkItem *d_items, int n_items, int *d_ticket,
                                 char *ws, int precision, int G, int B, int n_groups, int lds_cap, hipStream_t stream);
hipError_t launch_eval(const DevProblem *d_probs, const double *coords, int n_rep, double centre, double *forces,
                       double *energy, int model, int precision, int G, int B, hipStream_t stream);
hipError_t launch_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int n, uint32_t *words,
                         double *z64, float *z32, double *y64, float *y32, hipStream_t stream);

// Zero the accumulators, histograms and work distributions of problems [0, n_probs);
// clear n_tickets queue counters.
hipError_t launch_init(const DevProblem *d_probs, int n_probs, char *ws, int max_windows, int max_k, int max_m,
                       int *d_tickets, int n_tickets, hipStream_t stream);
// replica records -> (window, block) records -> window totals, estimators, diagnostics
hipError_t launch_reduce(const DevProblem *d_probs, int n_probs, char *ws, int max_windows, int max_blocks,
                         hipStream_t stream);
hipError_t launch_estimators(const DevProblem *d_probs, int n_probs, char *ws, int max_windows, hipStream_t stream);
// App. C: shift/probability pairs, the j-th folding step, statistics of Omega
hipError_t launch_appc(const DevProblem *d_probs, int n_probs, char *ws, int max_windows, int max_m,
                       hipStream_t stream);

// MLP surrogate
hipError_t launch_mlp_forward(const float *params, const float *t, int n, float *y, float *dy, hipStream_t stream);
hipError_t launch_mlp_grad(const float *params, const float *t, const float *yv, const float *wv, const float *ys,
                           const float *wsl, int n, float *grad, float *loss, hipStream_t stream);
hipError_t launch_mlp_adam(float *params, const float *grad, float *m, float *v, float lr, int step,
                           hipStream_t stream);

}  // namespace ppp

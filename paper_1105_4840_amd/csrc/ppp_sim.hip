// Dispatch of the simulation kernels: the 1-D kernel and the Philox probe
// live here; every chain shape (G lanes x B beads per lane, fp32 and fp64) is
// compiled in its own translation unit generated from ppp_shapes.hpp.
#include <hip/hip_runtime.h>

#include "ppp_shapes.hpp"
#include "ppp_sim_impl.hpp"

namespace ppp {

__global__ void philox_blocks(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int n,
                              uint32_t *__restrict__ words, double *__restrict__ z64, float *__restrict__ z32,
                              double *__restrict__ y64, float *__restrict__ y32) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U4 r = philox(seed, c0 + (uint32_t)i, c1, c2, c3);
    if (words) { words[4 * i] = r.x; words[4 * i + 1] = r.y; words[4 * i + 2] = r.z; words[4 * i + 3] = r.w; }
    if (z64) { double z[4]; Normal4<double>::get(seed, c0 + (uint32_t)i, c1, c2, c3, z); for (int q = 0; q < 4; ++q) z64[4 * i + q] = z[q]; }
    if (z32) { float z[4]; Normal4<float>::get(seed, c0 + (uint32_t)i, c1, c2, c3, z); for (int q = 0; q < 4; ++q) z32[4 * i + q] = z[q]; }
    if (y64) { double y[6]; Normal6<double>::get(seed, c0 + (uint32_t)i, c1, c2, c3, y); for (int q = 0; q < 6; ++q) y64[6 * i + q] = y[q]; }
    if (y32) { float y[6]; Normal6<float>::get(seed, c0 + (uint32_t)i, c1, c2, c3, y); for (int q = 0; q < 6; ++q) y32[6 * i + q] = y[q]; }
}

#define PPP_DECLARE(GG, BB)                                                                                         \
    extern template hipError_t launch_chain_direct<float, GG, BB>(const DevProblem *, const WorkItem *, int, char *, \
                                                                  int64_t, int64_t, double *, int64_t, int, hipStream_t); \
    extern template hipError_t launch_chain_direct<double, GG, BB>(const DevProblem *, const WorkItem *, int, char *, \
                                                                   int64_t, int64_t, double *, int64_t, int, hipStream_t); \
    extern template hipError_t launch_chain_persistent<float, GG, BB>(const DevProblem *, const WorkItem *, int, int *, \
                                                                      char *, int, int, hipStream_t);              \
    extern template hipError_t launch_chain_persistent<double, GG, BB>(const DevProblem *, const WorkItem *, int, int *, \
                                                                       char *, int, int, hipStream_t);             \
    extern template hipError_t launch_chain_eval<float, GG, BB>(const DevProblem *, const double *, int, double, double *, \
                                                                double *, hipStream_t);                            \
    extern template hipError_t launch_chain_eval<double, GG, BB>(const DevProblem *, const double *, int, double, double *, \
                                                                 double *, hipStream_t);                           \
    extern template int chain_blocks_per_cu<float, GG, BB>(int);                                                   \
    extern template int chain_blocks_per_cu<double, GG, BB>(int);
PPP_FOR_EACH_SHAPE(PPP_DECLARE)
#undef PPP_DECLARE

bool chain_shape_supported(int G, int B) {
#define PPP_CHECK(GG, BB) if (G == GG && B == BB) return true;
    PPP_FOR_EACH_SHAPE(PPP_CHECK)
#undef PPP_CHECK
    return false;
}

int sim_blocks_per_cu(int precision, int G, int B, int lds_cap) {
#define PPP_OCC(GG, BB) \
    if (G == GG && B == BB) return precision == 1 ? chain_blocks_per_cu<double, GG, BB>(lds_cap) : chain_blocks_per_cu<float, GG, BB>(lds_cap);
    PPP_FOR_EACH_SHAPE(PPP_OCC)
#undef PPP_OCC
    return 1;
}

hipError_t launch_sim(const DevProblem *d_probs, const WorkItem *d_items, int n_items, char *ws, int64_t step_begin,
                      int64_t step_end, int model, int precision, int G, int B, double *traj, int64_t traj_rep,
                      int lds_cap, hipStream_t stream) {
    if (n_items <= 0) return hipSuccess;
    if (model == 0) {
        const size_t sh = (size_t)lds_cap * 4;
        if (precision == 1) hipLaunchKernelGGL(sim_1d<double>, dim3(n_items), dim3(WG), sh, stream, d_probs, d_items, n_items, ws, step_begin, step_end, traj, (int)traj_rep, lds_cap);
        else hipLaunchKernelGGL(sim_1d<float>, dim3(n_items), dim3(WG), sh, stream, d_probs, d_items, n_items, ws, step_begin, step_end, traj, (int)traj_rep, lds_cap);
        return hipGetLastError();
    }
#define PPP_LAUNCH(GG, BB)                                                                                              \
    if (G == GG && B == BB)                                                                                            \
        return precision == 1 ? launch_chain_direct<double, GG, BB>(d_probs, d_items, n_items, ws, step_begin, step_end, traj, traj_rep, lds_cap, stream) \
                              : launch_chain_direct<float, GG, BB>(d_probs, d_items, n_items, ws, step_begin, step_end, traj, traj_rep, lds_cap, stream);
    PPP_FOR_EACH_SHAPE(PPP_LAUNCH)
#undef PPP_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_sim_persistent(const DevProblem *d_probs, const WorkItem *d_items, int n_items, int *d_ticket,
                                 char *ws, int precision, int G, int B, int n_groups, int lds_cap, hipStream_t stream) {
    if (n_items <= 0) return hipSuccess;
#define PPP_LAUNCH(GG, BB)                                                                                              \
    if (G == GG && B == BB)                                                                                            \
        return precision == 1 ? launch_chain_persistent<double, GG, BB>(d_probs, d_items, n_items, d_ticket, ws, n_groups, lds_cap, stream) \
                              : launch_chain_persistent<float, GG, BB>(d_probs, d_items, n_items, d_ticket, ws, n_groups, lds_cap, stream);
    PPP_FOR_EACH_SHAPE(PPP_LAUNCH)
#undef PPP_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_eval(const DevProblem *d_probs, const double *coords, int n_rep, double centre, double *forces,
                       double *energy, int model, int precision, int G, int B, hipStream_t stream) {
    if (n_rep <= 0) return hipSuccess;
    if (model == 0) {
        const int nb = (n_rep + 255) / 256;
        if (precision == 1) hipLaunchKernelGGL(pot1d_eval<double>, dim3(nb), dim3(256), 0, stream, d_probs, coords, n_rep, centre, forces, energy);
        else hipLaunchKernelGGL(pot1d_eval<float>, dim3(nb), dim3(256), 0, stream, d_probs, coords, n_rep, centre, forces, energy);
        return hipGetLastError();
    }
#define PPP_LAUNCH(GG, BB)                                                                                              \
    if (G == GG && B == BB)                                                                                            \
        return precision == 1 ? launch_chain_eval<double, GG, BB>(d_probs, coords, n_rep, centre, forces, energy, stream) \
                              : launch_chain_eval<float, GG, BB>(d_probs, coords, n_rep, centre, forces, energy, stream);
    PPP_FOR_EACH_SHAPE(PPP_LAUNCH)
#undef PPP_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int n, uint32_t *words,
                         double *z64, float *z32, double *y64, float *y32, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_blocks, dim3((n + 255) / 256), dim3(256), 0, stream, seed, c0, c1, c2, c3, n, words, z64, z32,
                       y64, y32);
    return hipGetLastError();
}

}  // namespace ppp

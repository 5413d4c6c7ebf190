// Issue-rate probe of the vector ALU, outside the protocol: it measures the
// fp32 FMA rate the simulation kernels are held against.
#pragma once
#include <hip/hip_runtime.h>

namespace ppp {
// n_blocks workgroups of 256 threads; each thread runs kProbeChains independent
// FMA chains of `iters` steps and writes their sum to out[thread]; b and c in
// scalar registers, or in vector registers with `vgprs`.
constexpr int kProbeChains = 8;
hipError_t launch_valu_probe(int n_blocks, int iters, float b, float c, bool vgprs, float *out, hipStream_t stream);
}  // namespace ppp

// fp32 FMA issue-rate probe.  Eight independent chains per thread hide the FMA
// latency, so with enough wavefronts per SIMD the loop runs at the VALU issue
// rate; the chains' sums are written out so that none of them is removed.
// The multiplier and addend come either as kernel arguments, which the loop
// reads from scalar registers (VGPRS = false), or as per-lane copies held in
// vector registers (VGPRS = true): an empty asm statement with a "+v" operand
// places each copy in a VGPR and makes it opaque, so it is not folded back.
#include "ppp_probe.hpp"

namespace ppp {

template <bool VGPRS>
__global__ __launch_bounds__(256) void valu_fma_probe(int iters, float b, float c, float *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (VGPRS) asm volatile("" : "+v"(b), "+v"(c));
    float a[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = (float)((i + k) & 1023) * 1e-6f;
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kProbeChains; ++k) a[k] = __builtin_fmaf(a[k], b, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += a[k];
    out[i] = s;
}

hipError_t launch_valu_probe(int n_blocks, int iters, float b, float c, bool vgprs, float *out, hipStream_t stream) {
    if (n_blocks <= 0 || iters <= 0) return hipSuccess;
    if (vgprs) hipLaunchKernelGGL(valu_fma_probe<true>, dim3(n_blocks), dim3(256), 0, stream, iters, b, c, out);
    else hipLaunchKernelGGL(valu_fma_probe<false>, dim3(n_blocks), dim3(256), 0, stream, iters, b, c, out);
    return hipGetLastError();
}

}  // namespace ppp

/*
 * ppp_probe.h -- measurement aid shipped in libppp beside the protocol's C ABI
 * (include/ppp.h); not part of the protocol.
 *
 * The simulation kernels are bound by fp32 vector-ALU issue; their roofline
 * fractions are read against the published MI355X peak, and this probe measures
 * the rate the same instruction form (non-packed v_fma_f32) reaches on the
 * device, as context for that peak: with its multiplier and addend in scalar
 * registers (one operand of each FMA an SGPR) or in vector registers (every
 * operand a VGPR), two forms that issue at different rates on gfx950.
 */
#ifndef PPP_PROBE_H
#define PPP_PROBE_H

#include <stdint.h>

#include "ppp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PPP_PROBE_SGPR_OPERANDS 0 /* b and c read from scalar registers */
#define PPP_PROBE_VGPR_OPERANDS 1 /* b and c copied into vector registers first */

/* Vector-ALU issue-rate probe: the fp32 FMA rate the simulation kernels'
 * roofline is read against.  n_blocks workgroups of
 * 256 threads each run 8 independent chains a <- fma(a, b, c) for iters steps
 * (16 iters flops per thread), chain k of thread i starting at
 * ((i + k) mod 1024) 1e-6, and write the sum of the 8 chains to d_out[i]
 * (device fp32 [n_blocks * 256], caller-owned).  `operands` is one of the
 * PPP_PROBE_* values above; both give the same results.  Asynchronous on
 * hip_stream, to be timed with events there.  PPP_E_INVALID_ARG for
 * n_blocks < 1, iters < 1, another `operands` value or a NULL d_out. */
ppp_status ppp_probe_valu(int32_t n_blocks, int32_t iters, float b, float c, int32_t operands, float *d_out,
                          void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PPP_PROBE_H */

// Host stand-in for <hip/hip_runtime.h> used by the lane model (tests only):
// the simulation kernels' per-lane device code compiles for the CPU, where one
// wavefront is 64 threads that meet at a barrier for every cross-lane move.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline

namespace lane_model {
int lane();                         // this thread's lane, 0..63
int bpermute(int byte_addr, int v); // ds_bpermute_b32: v of lane byte_addr / 4
int permute(int byte_addr, int v);  // ds_permute_b32: v goes to lane byte_addr / 4
}  // namespace lane_model

#define __lane_id() (lane_model::lane())
#define __builtin_amdgcn_ds_bpermute(a, v) (lane_model::bpermute((a), (v)))
#define __builtin_amdgcn_ds_permute(a, v) (lane_model::permute((a), (v)))
// the kernels use truth table 0x96 only: three-input exclusive or
#define __builtin_amdgcn_bitop3_b32(a, b, c, t) \
    ((t) == 0x96 ? ((uint32_t)(a) ^ (uint32_t)(b) ^ (uint32_t)(c)) : lane_model_bad_bitop3())
// v_alignbit_b32: low 32 bits of ({hi, lo} >> s)
#define __builtin_amdgcn_alignbit(hi, lo, s) \
    ((uint32_t)(((((uint64_t)(uint32_t)(hi)) << 32) | (uint32_t)(lo)) >> ((s) & 31)))
// fp32 hardware approximations stand in as the library functions (the model
// compares fp32 forces at the fp32 tolerance only)
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
#define __builtin_amdgcn_rsqf(x) (1.0f / std::sqrt(x))
#define __builtin_amdgcn_sqrtf(x) (std::sqrt(x))
#define __builtin_amdgcn_logf(x) (std::log2(x))
#define __builtin_amdgcn_sinf(x) (std::sin(6.283185307179586f * (x)))
#define __builtin_amdgcn_cosf(x) (std::cos(6.283185307179586f * (x)))

inline uint32_t lane_model_bad_bitop3() { __builtin_trap(); }
inline float __int_as_float(int i) { float f; std::memcpy(&f, &i, 4); return f; }
inline int __float_as_int(float f) { int i; std::memcpy(&i, &f, 4); return i; }
inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }

// Device building blocks for gfx950: counter-based noise, log-sum-exp
// accumulation and cross-lane data movement within a replica's lane group.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppp_internal.hpp"

namespace ppp {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// 4x32 Philox S-box; the key advances by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply each (v_mad_u64_u32) instead of separate hi/lo products
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        // three-input xor in one v_bitop3_b32 (truth table 0x96)
        uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
        uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// (r >> 9 + 1/2) 2^-23 in two instructions: the bits 0x3f800000 | (r >> 9)
// (v_alignbit_b32 of 0x7f and r by 9) are the float 1 + (r >> 9) 2^-23, and
// subtracting 1 - 2^-24 is exact.
__device__ __forceinline__ float unit_f32(uint32_t r) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, r, 9u)) - 0.99999994039535522f;
}

// Four standard normals per Philox block by Box-Muller, in the requested
// precision.  fp64: u = (r + 1/2) 2^-32 (exact); fp32: u = (r>>9 + 1/2) 2^-23
// (exact in fp32, hardware log2/sqrt/sin/cos; sin and cos take turns).
template <typename T> struct Normal4;

template <> struct Normal4<double> {
    __device__ __forceinline__ static void get(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, double z[4]) {
        U4 r = philox(seed, c0, c1, c2, c3);
        const double scale = 1.0 / 4294967296.0;
        const double two_pi = 6.283185307179586476925286766559;
        double ua = ((double)r.x + 0.5) * scale, ub = ((double)r.y + 0.5) * scale;
        double uc = ((double)r.z + 0.5) * scale, ud = ((double)r.w + 0.5) * scale;
        double ra = sqrt(-2.0 * log(ua)), rc = sqrt(-2.0 * log(uc));
        z[0] = ra * cos(two_pi * ub); z[1] = ra * sin(two_pi * ub);
        z[2] = rc * cos(two_pi * ud); z[3] = rc * sin(two_pi * ud);
    }
};

template <> struct Normal4<float> {
    __device__ __forceinline__ static void get(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, float z[4]) {
        U4 r = philox(seed, c0, c1, c2, c3);
        const float m2ln2 = -2.0f * 0.69314718055994531f;
        const float ua = unit_f32(r.x), ub = unit_f32(r.y), uc = unit_f32(r.z), ud = unit_f32(r.w);
        float ra = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(ua));
        float rc = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(uc));
        z[0] = ra * __builtin_amdgcn_cosf(ub); z[1] = ra * __builtin_amdgcn_sinf(ub);
        z[2] = rc * __builtin_amdgcn_cosf(ud); z[3] = rc * __builtin_amdgcn_sinf(ud);
    }
};

// Six standard normals per Philox block, the noise of the chain (two beads
// per block).  The 128 bits give six 21-bit integers: a_k = r_k >> 11 for
// k = 0..3, a_4 = (r_0 mod 2^11) 2^10 + (r_1 mod 2^10) and a_5 likewise from
// r_2 and r_3; u_k = (a_k + 1/2) 2^-21, exact in both precisions; Box-Muller on
// (u_0, u_1), (u_2, u_3), (u_4, u_5).  Half a block per bead instead of one
// block halves the Philox rounds of the chain kernels; |z| stays below
// sqrt(44 ln 2) = 5.52 (the smallest u is 2^-22).
template <typename T> struct Normal6;

template <> struct Normal6<double> {
    __device__ __forceinline__ static void get(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, double z[6]) {
        const U4 r = philox(seed, c0, c1, c2, c3);
        const uint32_t a[6] = {r.x >> 11, r.y >> 11, r.z >> 11, r.w >> 11, ((r.x & 0x7ffu) << 10) | (r.y & 0x3ffu),
                               ((r.z & 0x7ffu) << 10) | (r.w & 0x3ffu)};
        const double two_pi = 6.283185307179586476925286766559;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const double ua = ((double)a[2 * p] + 0.5) * 0x1p-21, ub = ((double)a[2 * p + 1] + 0.5) * 0x1p-21;
            const double rad = sqrt(-2.0 * log(ua));
            z[2 * p] = rad * cos(two_pi * ub);
            z[2 * p + 1] = rad * sin(two_pi * ub);
        }
    }
};

template <> struct Normal6<float> {
    // 1 + a 2^-21 is the float with bits 0x3f800000 | (a << 2); subtracting
    // 1 - 2^-22 leaves (a + 1/2) 2^-21 exactly
    __device__ __forceinline__ static float top21(uint32_t r) {
        return __uint_as_float(((r >> 9) & 0x7ffffcu) | 0x3f800000u) - (1.0f - 0x1p-22f);
    }
    __device__ __forceinline__ static float low21(uint32_t hi, uint32_t lo) {
        return __uint_as_float(((hi & 0x7ffu) << 12) | ((lo & 0x3ffu) << 2) | 0x3f800000u) - (1.0f - 0x1p-22f);
    }
    __device__ __forceinline__ static void get(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, float z[6]) {
        const U4 r = philox(seed, c0, c1, c2, c3);
        const float m2ln2 = -2.0f * 0.69314718055994531f;
        const float u[6] = {top21(r.x), top21(r.y), top21(r.z), top21(r.w), low21(r.x, r.y), low21(r.z, r.w)};
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            // hardware log2, sqrt, and sin/cos of 2 pi times the argument
            const float rad = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u[2 * p]));
            z[2 * p] = rad * __builtin_amdgcn_cosf(u[2 * p + 1]);
            z[2 * p + 1] = rad * __builtin_amdgcn_sinf(u[2 * p + 1]);
        }
    }
};

// ---------------------------------------------------------------------------
// Reciprocal and length in the working precision: the hardware instructions
// (about 1 ulp) in fp32, IEEE division and square root in fp64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }
// |v| and 1/|v| from |v|^2
__device__ __forceinline__ void len_inv(float r2, float &len, float &inv) {
    inv = __builtin_amdgcn_rsqf(r2);
    len = r2 * inv;
}
__device__ __forceinline__ void len_inv(double r2, double &len, double &inv) {
    len = sqrt(r2);
    inv = 1.0 / len;
}

// ---------------------------------------------------------------------------
// Running log-sum-exp (m, S): ln sum_k exp(a_k) = m + ln S.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lse_merge(double &m, double &S, double m2, double S2) {
    if (S2 == 0.0) return;
    if (S == 0.0) { m = m2; S = S2; return; }
    double M = fmax(m, m2);
    S = S * exp(m - M) + S2 * exp(m2 - M);
    m = M;
}
// Adds a to the running log-sum-exp (m, S) of a, and 2a to (m2, S2), with one
// exponential: the running maximum of 2a is twice that of a, so its rescaling
// factor is the square of a's.  t = exp(-|a - m|) serves both branches, so
// lanes that disagree on a > m still evaluate one exponential.
__device__ __forceinline__ void lse_push_pair(double &m, double &S, double &m2, double &S2, double a) {
    const double d = a - m;
    const bool up = d > 0.0;
    const double t = exp(up ? -d : d);
    const double t2 = t * t;
    S = up ? S * t + 1.0 : S + t;
    S2 = up ? S2 * t2 + 1.0 : S2 + t2;
    m = up ? a : m;
    m2 = 2.0 * m;
}
__device__ __forceinline__ double lse_value(double m, double S) {
    return S > 0.0 ? m + log(S) : -INFINITY;
}

// Merge record b into record a (fixed field semantics, see AccField).
__device__ __forceinline__ void acc_merge(double *a, const double *b) {
    a[A_N] += b[A_N]; a[A_S1] += b[A_S1]; a[A_S2] += b[A_S2];
    a[A_XMIN] = fmin(a[A_XMIN], b[A_XMIN]); a[A_XMAX] = fmax(a[A_XMAX], b[A_XMAX]);
    lse_merge(a[A_MF], a[A_SF], b[A_MF], b[A_SF]);
    lse_merge(a[A_MF2], a[A_SF2], b[A_MF2], b[A_SF2]);
    lse_merge(a[A_MR], a[A_SR], b[A_MR], b[A_SR]);
    lse_merge(a[A_MR2], a[A_SR2], b[A_MR2], b[A_SR2]);
    a[A_UNDER] += b[A_UNDER]; a[A_OVER] += b[A_OVER]; a[A_BLOWN] += b[A_BLOWN];
}
__device__ __forceinline__ void acc_empty(double *a) {
    for (int f = 0; f < A_NFIELDS; ++f) a[f] = 0.0;
    a[A_XMIN] = INFINITY; a[A_XMAX] = -INFINITY;
    a[A_MF] = a[A_MF2] = a[A_MR] = a[A_MR2] = -INFINITY;
}

// ---------------------------------------------------------------------------
// Cross-lane moves inside a group of G consecutive lanes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ float pull_f(int src_lane, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}
// fp64 values travel as two 32-bit halves; the split and the join are bit
// casts (no pointer type punning, which would break strict aliasing)
struct I2 { int lo, hi; };
__device__ __forceinline__ double pull_f(int src_lane, double v) {
    I2 w = __builtin_bit_cast(I2, v);
    w.lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, w.lo);
    w.hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, w.hi);
    return __builtin_bit_cast(double, w);
}
__device__ __forceinline__ int pull_i(int src_lane, int v) {
    return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}
// push: lane dst_lane receives v (every destination must be written by exactly one lane)
__device__ __forceinline__ float push_f(int dst_lane, float v) {
    return __int_as_float(__builtin_amdgcn_ds_permute(dst_lane << 2, __float_as_int(v)));
}
__device__ __forceinline__ double push_f(int dst_lane, double v) {
    I2 w = __builtin_bit_cast(I2, v);
    w.lo = __builtin_amdgcn_ds_permute(dst_lane << 2, w.lo);
    w.hi = __builtin_amdgcn_ds_permute(dst_lane << 2, w.hi);
    return __builtin_bit_cast(double, w);
}

}  // namespace ppp

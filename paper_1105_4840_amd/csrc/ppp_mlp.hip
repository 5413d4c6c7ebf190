// Surrogate F(lambda) for learned window placement: a 1 -> 64 -> 64 -> 1 tanh
// network y(t) with its input derivative dy/dt (the slope the protocol
// measures as k (lambda_i - <x_i>), Eq. 14), trained on value and slope
// targets.  Parameters are used through their bf16 values; the activations
// entering a product (h1, u1, h2, u2 and the layer-2 error signals) are bf16;
// all arithmetic and accumulation is fp32.  The three dense contractions per
// tile of 16 points,
//   [a2 | v2]         = W2   [h1 | u1]          (forward, value and slope path)
//   [g_h1 | g_u1]     = W2^T [g_a2 | g_v2]      (backward)
//   dW2              += [g_a2 | g_v2] [h1 | u1]^T
// run on the matrix cores (v_mfma_f32_16x16x32_bf16, wave64).
#include <hip/hip_runtime.h>

#include "ppp_launch.hpp"

namespace ppp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MH = 64;        // hidden width
constexpr int MT = 16;        // batch points per tile
constexpr int MC = 2 * MT;    // GEMM columns per tile: value path then slope path
constexpr int NP = MH + MH + MH * MH + MH + MH + 1;
constexpr int OFF_W1 = 0, OFF_B1 = MH, OFF_W2 = 2 * MH, OFF_B2 = 2 * MH + MH * MH, OFF_W3 = OFF_B2 + MH,
              OFF_B3 = OFF_W3 + MH;

// bf16 by round-to-nearest-even of the fp32 bit pattern
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(float x) { return __uint_as_float((uint32_t)bf16_bits(x) << 16); }

struct MlpShared {
    alignas(16) uint16_t w2[MH * MH];    // [out][in]
    alignas(16) uint16_t w2t[MH * MH];   // [in][out]
    alignas(16) uint16_t xc[MC * MH];    // [column][unit]   (h1 | u1), point-major
    alignas(16) uint16_t xm[MH * MC];    // [unit][column]
    alignas(16) uint16_t gc[MC * MH];    // (g_a2 | g_v2), point-major
    alignas(16) uint16_t gm[MH * MC];
    float y2[MH * MC];       // W2 [h1 | u1]
    float b2g[MH * MC];      // W2^T [g_a2 | g_v2]
    float red_y[MT * MH], red_dy[MT * MH];
    float w1[MH], b1[MH], b2[MH], w3[MH];
    float pt[MT][4];         // t, ey, ed, valid
    float b3;
};

// One 16x16 output tile: acc += A[16 rows][K] * B[K][16 cols], A row-major with
// row stride lda, B given transposed (column-major, stride ldb), K a multiple of 32.
__device__ __forceinline__ f32x4 mfma_tile(const uint16_t *A, int lda, const uint16_t *Bt, int ldb, int K, f32x4 acc) {
    const int l = __lane_id();
    const int r = l & 15, kq = (l >> 4) * 8;
    for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(A + r * lda + k0 + kq);
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Bt + r * ldb + k0 + kq);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    return acc;
}
// D layout of the 16x16 tile: lane l holds column l & 15, rows 4 (l >> 4) + i.
__device__ __forceinline__ void store_tile(float *D, int ldd, int r0, int c0, f32x4 acc) {
    const int l = __lane_id();
    for (int i = 0; i < 4; ++i) D[(r0 + 4 * (l >> 4) + i) * ldd + c0 + (l & 15)] = acc[i];
}

__device__ void load_params(MlpShared &S, const float *__restrict__ P) {
    for (int i = threadIdx.x; i < MH * MH; i += blockDim.x) {
        const uint16_t b = bf16_bits(P[OFF_W2 + i]);
        S.w2[i] = b;
        S.w2t[(i % MH) * MH + i / MH] = b;
    }
    for (int i = threadIdx.x; i < MH; i += blockDim.x) {
        S.w1[i] = bf16_val(P[OFF_W1 + i]); S.b1[i] = bf16_val(P[OFF_B1 + i]);
        S.b2[i] = bf16_val(P[OFF_B2 + i]); S.w3[i] = bf16_val(P[OFF_W3 + i]);
    }
    if (threadIdx.x == 0) S.b3 = bf16_val(P[OFF_B3]);
}

// layer 1 for the tile: h1 and u1 = (1 - h1^2) W1 into the bf16 GEMM inputs
__device__ void layer1(MlpShared &S, const float *__restrict__ t, int n, int base) {
    for (int idx = threadIdx.x; idx < MH * MT; idx += blockDim.x) {
        const int j = idx % MH, p = idx / MH;
        const int P = base + p;
        const bool valid = P < n;
        const float tp = valid ? t[P] : 0.f;
        const float h1 = tanhf(S.w1[j] * tp + S.b1[j]);
        const float u1 = (1.f - h1 * h1) * S.w1[j];
        const uint16_t bh = valid ? bf16_bits(h1) : 0, bu = valid ? bf16_bits(u1) : 0;
        S.xc[p * MH + j] = bh; S.xc[(MT + p) * MH + j] = bu;
        S.xm[j * MC + p] = bh; S.xm[j * MC + MT + p] = bu;
        if (j == 0) { S.pt[p][0] = tp; S.pt[p][3] = valid ? 1.f : 0.f; }
    }
}

// [a2 - b2 | v2] = W2 [h1 | u1]: 4 x 2 output tiles, wave w takes row tile w
__device__ void gemm_forward(MlpShared &S) {
    const int w = threadIdx.x >> 6;
    for (int nt = 0; nt < 2; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma_tile(S.w2 + 16 * w * MH, MH, S.xc + 16 * nt * MH, MH, MH, acc);
        store_tile(S.y2, MC, 16 * w, 16 * nt, acc);
    }
}

template <bool GRAD>
__global__ __launch_bounds__(256) void mlp_kernel(const float *__restrict__ params, const float *__restrict__ t,
                                                  const float *__restrict__ yv, const float *__restrict__ wv,
                                                  const float *__restrict__ ys, const float *__restrict__ wsl, int n,
                                                  float *__restrict__ y_out, float *__restrict__ dy_out,
                                                  float *__restrict__ grad, float *__restrict__ loss) {
    __shared__ MlpShared S;
    load_params(S, params);
    // per-thread accumulators for the unit j = tid % 64 (GRAD)
    float aW1 = 0.f, aB1 = 0.f, aB2 = 0.f, aW3 = 0.f, aB3 = 0.f, aL = 0.f;
    f32x4 dW2[4];
    for (int q = 0; q < 4; ++q) dW2[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int tiles = (n + MT - 1) / MT;
    const int t_begin = GRAD ? 0 : blockIdx.x;
    const int t_step = GRAD ? 1 : gridDim.x;
    __syncthreads();
    for (int tile = t_begin; tile < tiles; tile += t_step) {
        const int base = tile * MT;
        layer1(S, t, n, base);
        __syncthreads();
        gemm_forward(S);
        __syncthreads();
        // layer 2 and the output
        for (int idx = threadIdx.x; idx < MH * MT; idx += blockDim.x) {
            const int j = idx % MH, p = idx / MH;
            const float h2 = tanhf(S.y2[j * MC + p] + S.b2[j]);
            const float u2 = (1.f - h2 * h2) * S.y2[j * MC + MT + p];
            S.red_y[p * MH + j] = S.w3[j] * bf16_val(h2);
            S.red_dy[p * MH + j] = S.w3[j] * bf16_val(u2);
        }
        __syncthreads();
        if ((int)threadIdx.x < MT) {
            const int p = threadIdx.x, P = base + p;
            float y = 0.f, dy = 0.f;
            for (int j = 0; j < MH; ++j) { y += S.red_y[p * MH + j]; dy += S.red_dy[p * MH + j]; }
            y += S.b3;
            float ey = 0.f, ed = 0.f;
            if (P < n) {
                if (!GRAD) { y_out[P] = y; if (dy_out) dy_out[P] = dy; }
                else {
                    const float ry = y - yv[P], rd = dy - ys[P];
                    ey = 2.f * wv[P] * ry; ed = 2.f * wsl[P] * rd;
                    aL += wv[P] * ry * ry + wsl[P] * rd * rd;
                    aB3 += ey;
                }
            }
            S.pt[p][1] = ey; S.pt[p][2] = ed;
        }
        __syncthreads();
        if (!GRAD) continue;
        // backward through layer 2 (both paths)
        for (int idx = threadIdx.x; idx < MH * MT; idx += blockDim.x) {
            const int j = idx % MH, p = idx / MH;
            const float v2 = S.y2[j * MC + MT + p];
            const float h2 = tanhf(S.y2[j * MC + p] + S.b2[j]);
            const float s2 = 1.f - h2 * h2;
            const float u2 = s2 * v2;
            const float ey = S.pt[p][1], ed = S.pt[p][2];
            aW3 += ey * bf16_val(h2) + ed * bf16_val(u2);
            const float g_u2 = ed * S.w3[j];
            const float g_h2 = ey * S.w3[j] + g_u2 * (-2.f * h2 * v2);
            const float g_v2 = g_u2 * s2;
            const float g_a2 = g_h2 * s2;
            aB2 += g_a2;
            const uint16_t ba = bf16_bits(g_a2), bv = bf16_bits(g_v2);
            S.gc[p * MH + j] = ba; S.gc[(MT + p) * MH + j] = bv;
            S.gm[j * MC + p] = ba; S.gm[j * MC + MT + p] = bv;
        }
        __syncthreads();
        {
            const int w = threadIdx.x >> 6;
            // [g_h1 | g_u1] = W2^T [g_a2 | g_v2]
            for (int nt = 0; nt < 2; ++nt) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = mfma_tile(S.w2t + 16 * w * MH, MH, S.gc + 16 * nt * MH, MH, MH, acc);
                store_tile(S.b2g, MC, 16 * w, 16 * nt, acc);
            }
            // dW2[m][k] += sum_c G[m][c] X[k][c]
            for (int nt = 0; nt < 4; ++nt)
                dW2[nt] = mfma_tile(S.gm + 16 * w * MC, MC, S.xm + 16 * nt * MC, MC, MC, dW2[nt]);
        }
        __syncthreads();
        // backward through layer 1
        for (int idx = threadIdx.x; idx < MH * MT; idx += blockDim.x) {
            const int j = idx % MH, p = idx / MH;
            if (S.pt[p][3] == 0.f) continue;
            const float tp = S.pt[p][0];
            const float h1 = tanhf(S.w1[j] * tp + S.b1[j]);
            const float s1 = 1.f - h1 * h1;
            const float g_u1 = S.b2g[j * MC + MT + p];
            const float g_h1 = S.b2g[j * MC + p] + g_u1 * (-2.f * h1 * S.w1[j]);
            const float g_a1 = g_h1 * s1;
            aW1 += g_u1 * s1 + g_a1 * tp;
            aB1 += g_a1;
        }
        __syncthreads();
    }
    if (!GRAD) return;
    // fixed-order reductions of the per-thread accumulators
    {
        const int w = threadIdx.x >> 6;
        for (int nt = 0; nt < 4; ++nt) store_tile(grad + OFF_W2, MH, 16 * w, 16 * nt, dW2[nt]);
    }
    __syncthreads();
    float *acc = S.b2g;   // reused: [4 partials][256 threads]
    acc[0 * 256 + threadIdx.x] = aW1; acc[1 * 256 + threadIdx.x] = aB1;
    acc[2 * 256 + threadIdx.x] = aB2; acc[3 * 256 + threadIdx.x] = aW3;
    __syncthreads();
    if ((int)threadIdx.x < MH) {
        const int j = threadIdx.x;
        float s[4] = {0.f, 0.f, 0.f, 0.f};
        for (int q = 0; q < 4; ++q)
            for (int g = 0; g < 4; ++g) s[q] += acc[q * 256 + g * MH + j];
        grad[OFF_W1 + j] = s[0]; grad[OFF_B1 + j] = s[1]; grad[OFF_B2 + j] = s[2]; grad[OFF_W3 + j] = s[3];
    }
    __syncthreads();
    acc[threadIdx.x] = aB3; acc[256 + threadIdx.x] = aL;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b3 = 0.f, L = 0.f;
        for (int i = 0; i < MT; ++i) { b3 += acc[i]; L += acc[256 + i]; }
        grad[OFF_B3] = b3;
        if (loss) loss[0] = L;
    }
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi; v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

hipError_t launch_mlp_forward(const float *params, const float *t, int n, float *y, float *dy, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int tiles = (n + MT - 1) / MT;
    hipLaunchKernelGGL(mlp_kernel<false>, dim3(tiles < 1024 ? tiles : 1024), dim3(256), 0, stream, params, t, nullptr,
                       nullptr, nullptr, nullptr, n, y, dy, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *params, const float *t, const float *yv, const float *wv, const float *ys,
                           const float *wsl, int n, float *grad, float *loss, hipStream_t stream) {
    hipLaunchKernelGGL(mlp_kernel<true>, dim3(1), dim3(256), 0, stream, params, t, yv, wv, ys, wsl, n, nullptr,
                       nullptr, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *params, const float *grad, float *m, float *v, float lr, int step,
                           hipStream_t stream) {
    const float c1 = 1.f - powf(0.9f, (float)step), c2 = 1.f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, stream, params, grad, m, v, lr, c1, c2);
    return hipGetLastError();
}

}  // namespace ppp

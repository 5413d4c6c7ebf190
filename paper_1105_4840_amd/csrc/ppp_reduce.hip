// Reductions, estimators and work distributions of libppp (all fp64, fixed
// merge order, so results do not depend on scheduling).
//
//   replica records --(per window, jackknife block)--> block records
//   block records   --(per window)--> window totals
//   window totals   --> Eq. 12 (JE, factorised over the independent windows),
//                       Eq. 14 and Eq. 13 with the actual increments
//                       lambda_{i+1} - lambda_i, combined estimate and its
//                       uncertainty (Sec. IV B, IV D), reverse JE, gamma_i^2,
//                       jackknife standard errors, Kish effective size,
//                       overlap of adjacent histograms, the Sec. IV B criterion
//   histograms      --> App. C work distributions Omega_j, dF^JE from them and
//                       the variance formula of Sec. IV A.
#include <hip/hip_runtime.h>

#include "ppp.h"
#include "ppp_device.hpp"
#include "ppp_launch.hpp"

namespace ppp {

__device__ __forceinline__ double *dptr(char *ws, int64_t off) { return reinterpret_cast<double *>(ws + off); }

// ---------------------------------------------------------------------------
__global__ void k_init(const DevProblem *__restrict__ probs, char *__restrict__ ws, int *tickets, int n_tickets) {
    const DevProblem &P = probs[blockIdx.y];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(ws + P.off_hist);
    const int64_t nh = (int64_t)P.n_sim_windows * P.xi_nbins;
    for (int64_t i = tid; i < nh; i += stride) hist[i] = 0ull;
    if (P.w_half_bins > 0) {
        double *om = dptr(ws, P.off_omega);
        const int64_t nb = 2 * (int64_t)P.w_half_bins + 1;
        const int64_t no = (int64_t)P.n_windows * nb;
        for (int64_t i = tid; i < kAppcChains * no; i += stride)     // every chain; Omega_1: W = 0
            om[i] = (i % no == P.w_half_bins) ? 1.0 : 0.0;
    }
    if (blockIdx.y == 0 && tid < n_tickets) tickets[tid] = 0;
}

hipError_t launch_init(const DevProblem *d_probs, int n_probs, char *ws, int max_windows, int max_k, int max_m,
                       int *d_tickets, int n_tickets, hipStream_t stream) {
    int64_t work = (int64_t)max_windows * max_k;
    const int64_t wo = kAppcChains * (int64_t)max_windows * (2 * (int64_t)max_m + 1);
    if (wo > work) work = wo;
    int nb = (int)((work + 255) / 256);
    if (nb < 1) nb = 1;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_init, dim3(nb, n_probs), dim3(256), 0, stream, d_probs, ws, d_tickets, n_tickets);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One wave per (window, block): lanes merge strided replicas in order, then a
// fixed butterfly-free tree (lane l takes lane l + off) down to lane 0.
__global__ __launch_bounds__(64) void k_reduce_blocks(const DevProblem *__restrict__ probs, char *__restrict__ ws) {
    const DevProblem &P = probs[blockIdx.y];
    const int B = P.n_blocks, R = P.n_replicas;
    const int wb = blockIdx.x;
    if (wb >= P.n_sim_windows * B) return;
    const int w = wb / B, b = wb % B;
    const int lo = (int)(((int64_t)b * R + B - 1) / B);
    const int hi = (int)(((int64_t)(b + 1) * R + B - 1) / B);
    const double *rec = dptr(ws, P.off_acc) + ((int64_t)w * R) * A_NFIELDS;
    double a[A_NFIELDS];
    acc_empty(a);
    const int l = threadIdx.x;
    for (int r = lo + l; r < hi; r += 64) acc_merge(a, rec + (int64_t)r * A_NFIELDS);
    for (int off = 32; off >= 1; off >>= 1) {
        double o[A_NFIELDS];
        for (int f = 0; f < A_NFIELDS; ++f) o[f] = pull_f(l + off < 64 ? l + off : l, a[f]);
        if (l < off) acc_merge(a, o);
    }
    if (l == 0) {
        double *dst = dptr(ws, P.off_blk) + (int64_t)wb * A_NFIELDS;
        for (int f = 0; f < A_NFIELDS; ++f) dst[f] = a[f];
    }
}

hipError_t launch_reduce(const DevProblem *d_probs, int n_probs, char *ws, int max_windows, int max_blocks,
                         hipStream_t stream) {
    hipLaunchKernelGGL(k_reduce_blocks, dim3(max_windows * max_blocks, n_probs), dim3(64), 0, stream, d_probs, ws);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
struct WinStat {
    double n, mean, var, lse_f, lse_r;
};
__device__ __forceinline__ WinStat win_stat(const double *a, double lam) {
    WinStat s;
    s.n = a[A_N];
    const double m1 = a[A_S1] / a[A_N];
    s.mean = lam + m1;
    s.var = (a[A_S2] - a[A_N] * m1 * m1) / (a[A_N] - 1.0);
    s.lse_f = lse_value(a[A_MF], a[A_SF]);
    s.lse_r = lse_value(a[A_MR], a[A_SR]);
    return s;
}

// contributions of the step i -> i+1 to JE, fluct, gauss
__device__ __forceinline__ void step_terms(const DevProblem &P, const WinStat &st, double li, double lj, double &je,
                                           double &fl, double &ga) {
    const double dl = lj - li;
    je = -P.kT * (st.lse_f - log(st.n));
    fl = P.k * dl * (li - st.mean);
    const double gamma2 = P.k * st.var / P.kT;
    ga = fl + 0.5 * P.k * dl * dl * (1.0 - gamma2);
}

// Turn-on free energies from the records of window 1 (a1), window s (as) and
// the unrestrained ensemble (a0); je_s = dF^JE(lambda_s) from the same records.
struct TurnOn {
    double eq5_first, eq6_first, eq5_last, eq6_last, eq10;
};
__device__ __forceinline__ TurnOn turn_on(const DevProblem &P, const double *a1, const double *as, const double *a0,
                                          double je_s) {
    TurnOn r;
    // Eq. 5: DF = kT ln <exp(+beta k/2 (x - lambda)^2)> over the restrained window
    r.eq5_first = P.kT * (lse_value(a1[A_MR], a1[A_SR]) - log(a1[A_N]));
    r.eq5_last = P.kT * (lse_value(as[A_MF], as[A_SF]) - log(as[A_N]));
    // Eq. 6: DF = -kT ln <exp(-beta k/2 (x_0 - lambda)^2)> over the free ensemble
    r.eq6_first = -P.kT * (lse_value(a0[A_MF], a0[A_SF]) - log(a0[A_N]));
    r.eq6_last = -P.kT * (lse_value(a0[A_MR], a0[A_SR]) - log(a0[A_N]));
    // Eq. 10 factorised over x_0, x_1 .. x_s: the turn-on at lambda_1 from x_0, the
    // steps, and the turn-off at lambda_s from x_s
    r.eq10 = -P.beta * (r.eq6_first + je_s - r.eq5_last);
    return r;
}

__device__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off >= 1; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_estimators(const DevProblem *__restrict__ probs, char *__restrict__ ws) {
    const DevProblem &P = probs[blockIdx.x];
    __shared__ double sh[256];
    const int s = P.n_windows, B = P.n_blocks, K = P.xi_nbins;
    const int t = threadIdx.x;
    const double *lam = dptr(ws, P.off_lambda);
    const double *blk = dptr(ws, P.off_blk);
    double *tot = dptr(ws, P.off_tot);
    double *out = dptr(ws, P.off_out);
    double *jack = dptr(ws, P.off_jack);
    const unsigned long long *hist = reinterpret_cast<const unsigned long long *>(ws + P.off_hist);
#define OUT(f, i) out[(int64_t)(f) * s + (i)]

    const int S = P.n_sim_windows;
    // (a) window totals: blocks merged in block order
    for (int w = t; w < S; w += blockDim.x) {
        double a[A_NFIELDS];
        acc_empty(a);
        for (int b = 0; b < B; ++b) acc_merge(a, blk + ((int64_t)w * B + b) * A_NFIELDS);
        for (int f = 0; f < A_NFIELDS; ++f) tot[(int64_t)w * A_NFIELDS + f] = a[f];
    }
    __syncthreads();
    // (b) per-window statistics
    for (int w = t; w < s; w += blockDim.x) {
        const double *a = tot + (int64_t)w * A_NFIELDS;
        const WinStat st = win_stat(a, lam[w]);
        OUT(O_XI_MEAN, w) = st.mean;
        OUT(O_XI_STD, w) = sqrt(st.var);
        OUT(O_GAMMA2, w) = P.k * st.var / P.kT;
        OUT(O_XI_MINS, w) = a[A_XMIN];
        OUT(O_XI_MAXS, w) = a[A_XMAX];
        OUT(O_LSE_FWD, w) = w + 1 < s ? st.lse_f : NAN;
        OUT(O_LSE_REV, w) = w > 0 ? st.lse_r : NAN;
        OUT(O_N_SAMPLES, w) = a[A_N];
        OUT(O_N_BLOWN, w) = a[A_BLOWN];
        OUT(O_UNDER, w) = a[A_UNDER];
        OUT(O_OVER, w) = a[A_OVER];
        if (w + 1 < s) {
            const double dl = lam[w + 1] - lam[w];
            OUT(O_KISH, w) = exp(2.0 * st.lse_f - lse_value(a[A_MF2], a[A_SF2])) / st.n;
            OUT(O_DL_SIGMA, w) = fabs(dl) / sqrt(st.var);
            const double reach = dl > 0 ? a[A_XMAX] - st.mean : st.mean - a[A_XMIN];
            OUT(O_DL_REACH, w) = fabs(dl) / reach;
            OUT(O_CRIT, w) = fabs(dl) <= reach ? 1.0 : 0.0;
        } else {
            OUT(O_KISH, w) = NAN; OUT(O_DL_SIGMA, w) = NAN; OUT(O_DL_REACH, w) = NAN; OUT(O_CRIT, w) = NAN;
        }
    }
    __syncthreads();
    // (c) profiles: prefix sums over the steps
    if (t == 0) {
        double je = 0, fl = 0, ga = 0, rev = 0;
        double s1 = 0, s2 = 0;   // sums over i < j of (lambda_i - <x_i>) and (1 - gamma_i^2)
        OUT(O_DF_JE, 0) = 0; OUT(O_DF_FLUCT, 0) = 0; OUT(O_DF_GAUSS, 0) = 0; OUT(O_DF_REV, 0) = 0;
        OUT(O_DF_FLUCT_LIT, 0) = 0; OUT(O_DF_GAUSS_LIT, 0) = 0;
        for (int j = 1; j < s; ++j) {
            const WinStat st = win_stat(tot + (int64_t)(j - 1) * A_NFIELDS, lam[j - 1]);
            double dje, dfl, dga;
            step_terms(P, st, lam[j - 1], lam[j], dje, dfl, dga);
            je += dje; fl += dfl; ga += dga;
            // Eqs. 14 and 13 as printed, lambda_j taken as the end point of j + 1 windows
            s1 += lam[j - 1] - st.mean;
            s2 += 1.0 - P.k * st.var / P.kT;
            const double span = lam[j] - lam[0], npts = (double)(j + 1);
            const double fl_lit = P.k * span * s1 / npts;
            OUT(O_DF_FLUCT_LIT, j) = fl_lit;
            OUT(O_DF_GAUSS_LIT, j) = P.k * span * span / (2.0 * npts) * s2 / npts + fl_lit;
            const WinStat sj = win_stat(tot + (int64_t)j * A_NFIELDS, lam[j]);
            rev += P.kT * (sj.lse_r - log(sj.n));
            OUT(O_DF_JE, j) = je; OUT(O_DF_FLUCT, j) = fl; OUT(O_DF_GAUSS, j) = ga; OUT(O_DF_REV, j) = rev;
        }
        for (int j = 0; j < s; ++j) {
            OUT(O_DF_COM, j) = 0.5 * (OUT(O_DF_JE, j) + OUT(O_DF_FLUCT, j));
            OUT(O_DF_UNC, j) = 0.5 * (OUT(O_DF_JE, j) - OUT(O_DF_FLUCT, j));
        }
        double *turn = dptr(ws, P.off_turn);
        if (P.free_ens) {
            const double *a1 = tot, *as = tot + (int64_t)(s - 1) * A_NFIELDS, *a0 = tot + (int64_t)s * A_NFIELDS;
            const TurnOn on = turn_on(P, a1, as, a0, OUT(O_DF_JE, s - 1));
            turn[PPP_ON_EQ5_FIRST] = on.eq5_first;
            turn[PPP_ON_EQ6_FIRST] = on.eq6_first;
            turn[PPP_ON_EQ5_LAST] = on.eq5_last;
            turn[PPP_ON_EQ6_LAST] = on.eq6_last;
            turn[PPP_ON_EQ10_LOG] = on.eq10;
            // Eq. 7: <k/2 (x - lambda)^2> over the restrained window and over x_0
            const double dls = lam[s - 1] - lam[0];
            turn[PPP_ON_LOWER_FIRST] = 0.5 * P.k * a1[A_S2] / a1[A_N];
            turn[PPP_ON_UPPER_FIRST] = 0.5 * P.k * a0[A_S2] / a0[A_N];
            turn[PPP_ON_LOWER_LAST] = 0.5 * P.k * as[A_S2] / as[A_N];
            turn[PPP_ON_UPPER_LAST] = 0.5 * P.k * (a0[A_S2] - 2.0 * dls * a0[A_S1] + a0[A_N] * dls * dls) / a0[A_N];
            const WinStat f0 = win_stat(a0, lam[0]);
            turn[PPP_ON_FREE_N] = a0[A_N];
            turn[PPP_ON_FREE_BLOWN] = a0[A_BLOWN];
            turn[PPP_ON_FREE_MEAN] = f0.mean;
            turn[PPP_ON_FREE_STD] = sqrt(f0.var);
            turn[PPP_ON_FREE_UNDER] = a0[A_UNDER];
            turn[PPP_ON_FREE_OVER] = a0[A_OVER];
            for (int j = 0; j < s; ++j) OUT(O_G, j) = OUT(O_DF_JE, j) - on.eq5_first;   // Eq. 15
        } else {
            for (int f = 0; f < PPP_ON_NFIELDS; ++f) turn[f] = NAN;
            for (int j = 0; j < s; ++j) OUT(O_G, j) = NAN;
        }
    }
    // (d) jackknife: block b removed from every window.  First every (block,
    // step) term from its window without that block, in parallel; then the
    // prefix sums per block.  Blocks are merged in block order as before.
    auto loo = [&](int b, int w, double *a) {
        acc_empty(a);
        for (int c = 0; c < B; ++c)
            if (c != b) acc_merge(a, blk + ((int64_t)w * B + c) * A_NFIELDS);
    };
    if (B > 1) {
        for (int q = t; q < B * (s - 1); q += blockDim.x) {
            const int b = q / (s - 1), j = q % (s - 1) + 1;
            double a[A_NFIELDS];
            loo(b, j - 1, a);
            const WinStat st = win_stat(a, lam[j - 1]);
            double dje, dfl, dga;
            step_terms(P, st, lam[j - 1], lam[j], dje, dfl, dga);
            double *jb = jack + (int64_t)b * JK_FIELDS * s;
            jb[0 * s + j] = dje; jb[1 * s + j] = dfl; jb[2 * s + j] = dga;
        }
        __syncthreads();
        for (int b = t; b < B; b += blockDim.x) {
            double je = 0, fl = 0, ga = 0;
            double *jb = jack + (int64_t)b * JK_FIELDS * s;
            jb[0 * s] = 0; jb[1 * s] = 0; jb[2 * s] = 0; jb[3 * s] = 0;
            for (int j = 1; j < s; ++j) {
                je += jb[0 * s + j]; fl += jb[1 * s + j]; ga += jb[2 * s + j];
                jb[0 * s + j] = je; jb[1 * s + j] = fl; jb[2 * s + j] = ga; jb[3 * s + j] = 0.5 * (je + fl);
            }
            if (P.free_ens) {
                double a1[A_NFIELDS], as[A_NFIELDS], a0[A_NFIELDS];
                loo(b, 0, a1);
                loo(b, s - 1, as);
                loo(b, s, a0);
                const TurnOn on = turn_on(P, a1, as, a0, je);
                double *jt = dptr(ws, P.off_jack_turn) + (int64_t)b * JK_TURN;
                jt[0] = on.eq5_first; jt[1] = on.eq6_first; jt[2] = on.eq5_last; jt[3] = on.eq6_last; jt[4] = on.eq10;
                for (int j = 0; j < s; ++j) jb[4 * s + j] = jb[0 * s + j] - on.eq5_first;
            } else {
                for (int j = 0; j < s; ++j) jb[4 * s + j] = NAN;
            }
        }
    }
    __syncthreads();
    if (t == 0 && P.free_ens) {
        const int fields[JK_TURN] = {PPP_ON_EQ5_FIRST_SE, PPP_ON_EQ6_FIRST_SE, PPP_ON_EQ5_LAST_SE,
                                     PPP_ON_EQ6_LAST_SE, PPP_ON_EQ10_LOG_SE};
        const double *jt = dptr(ws, P.off_jack_turn);
        double *turn = dptr(ws, P.off_turn);
        for (int q = 0; q < JK_TURN; ++q) {
            double se = NAN;
            if (B > 1) {
                double m = 0;
                for (int b = 0; b < B; ++b) m += jt[b * JK_TURN + q];
                m /= B;
                double ss = 0;
                for (int b = 0; b < B; ++b) {
                    const double d = jt[b * JK_TURN + q] - m;
                    ss += d * d;
                }
                se = sqrt((B - 1.0) / B * ss);
            }
            turn[fields[q]] = se;
        }
    }
    for (int j = t; j < s; j += blockDim.x) {
        const int fields[JK_FIELDS] = {O_DF_JE_SE, O_DF_FLUCT_SE, O_DF_GAUSS_SE, O_DF_COM_SE, O_G_SE};
        for (int q = 0; q < JK_FIELDS; ++q) {
            double se = NAN;
            if (B > 1) {
                double m = 0;
                for (int b = 0; b < B; ++b) m += jack[((int64_t)b * JK_FIELDS + q) * s + j];
                m /= B;
                double ss = 0;
                for (int b = 0; b < B; ++b) {
                    const double d = jack[((int64_t)b * JK_FIELDS + q) * s + j] - m;
                    ss += d * d;
                }
                se = sqrt((B - 1.0) / B * ss);
            }
            OUT(fields[q], j) = se;
        }
    }
    // (e) overlap of adjacent histograms: sum_b min(rho_i(b), rho_{i+1}(b)), one
    // wavefront per adjacent pair (lanes stride the bins, then a fixed tree)
    {
        const int wave = t >> 6, lane = t & 63, n_waves = blockDim.x >> 6;
        for (int i = wave; i + 1 < s; i += n_waves) {
            const double ni = tot[(int64_t)i * A_NFIELDS + A_N], nj = tot[(int64_t)(i + 1) * A_NFIELDS + A_N];
            double part = 0;
            for (int b = lane; b < K; b += 64)
                part += fmin((double)hist[(int64_t)i * K + b] / ni, (double)hist[(int64_t)(i + 1) * K + b] / nj);
            for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off);
            if (lane == 0) OUT(O_OVL, i) = part;
        }
        if (t == 0) OUT(O_OVL, s - 1) = NAN;
    }
#undef OUT
}

// ---------------------------------------------------------------------------
// The paper's sigma_i (Sec. IV A: gamma_i^2 = k sigma_i^2 / kT with sigma_i by
// least-squares fitting of the x_i distribution): the Gaussian A exp(-(x -
// mu)^2 / (2 sigma^2)) closest in least squares to the histogram density
// count_b / (n dxi) at the bin centres, by Levenberg-Marquardt from the sample
// moments.  One workgroup per window; each iteration sums J^T J, J^T r and the
// squared residual over the bins in one block reduction.
template <int NV>
__device__ __forceinline__ void block_sum_vec(double (&v)[NV], double *sh) {
    for (int q = 0; q < NV; ++q)
        for (int off = 32; off >= 1; off >>= 1) v[q] += __shfl_xor(v[q], off);
    const int wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < NV; ++q) sh[q * 4 + wave] = v[q];
    __syncthreads();
    for (int q = 0; q < NV; ++q) {
        double t = 0;
        for (int u = 0; u < n_waves; ++u) t += sh[q * 4 + u];
        v[q] = t;
    }
}

__global__ __launch_bounds__(256) void k_gauss_fit(const DevProblem *__restrict__ probs, char *__restrict__ ws) {
    const DevProblem &P = probs[blockIdx.y];
    const int w = blockIdx.x, s = P.n_windows, K = P.xi_nbins;
    if (w >= s) return;
    double *out = dptr(ws, P.off_out);
    const double *a = dptr(ws, P.off_tot) + (int64_t)w * A_NFIELDS;
    const unsigned long long *hist = reinterpret_cast<const unsigned long long *>(ws + P.off_hist) + (int64_t)w * K;
    const double *lam = dptr(ws, P.off_lambda);
    __shared__ double sh[10 * 4];
    __shared__ double s_p[3];
    __shared__ int s_done;
    const double n = a[A_N];
    const double m1 = a[A_S1] / n;
    const double var = (a[A_S2] - n * m1 * m1) / (n - 1.0);
    double nz[1] = {0.0};                             // non-empty bins
    for (int b = threadIdx.x; b < K; b += blockDim.x) nz[0] += hist[b] ? 1.0 : 0.0;
    block_sum_vec<1>(nz, sh);
    if (!(n > 2.0) || !(var > 0.0) || nz[0] < 3.0) {   // three parameters need three points
        if (threadIdx.x == 0) { out[(int64_t)O_SIGMA_LSQ * s + w] = NAN; out[(int64_t)O_GAMMA2_LSQ * s + w] = NAN; }
        return;
    }
    const double norm = 1.0 / (n * P.xi_bin);
    double A = 1.0 / (sqrt(var) * 2.5066282746310002), mu = lam[w] + m1, sg = sqrt(var);
    double lm = 1e-3;
    // squared residual of (A, mu, sg)
    auto cost = [&](double pA, double pm, double ps) {
        double c[1] = {0.0};
        const double i2 = 1.0 / (2.0 * ps * ps);
        for (int b = threadIdx.x; b < K; b += blockDim.x) {
            const double x = P.xi_min + ((double)b + 0.5) * P.xi_bin, d = x - pm;
            const double r = (double)hist[b] * norm - pA * exp(-d * d * i2);
            c[0] += r * r;
        }
        block_sum_vec<1>(c, sh);
        return c[0];
    };
    double c0 = cost(A, mu, sg);
    for (int it = 0; it < 200; ++it) {
        double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // JtJ (6), Jtr (3), unused
        const double i2 = 1.0 / (2.0 * sg * sg), is2 = 1.0 / (sg * sg);
        for (int b = threadIdx.x; b < K; b += blockDim.x) {
            const double x = P.xi_min + ((double)b + 0.5) * P.xi_bin, d = x - mu;
            const double e = exp(-d * d * i2);
            const double f = A * e;
            const double r = (double)hist[b] * norm - f;
            const double jA = e, jm = f * d * is2, js = f * d * d * is2 / sg;
            v[0] += jA * jA; v[1] += jA * jm; v[2] += jA * js;
            v[3] += jm * jm; v[4] += jm * js; v[5] += js * js;
            v[6] += jA * r; v[7] += jm * r; v[8] += js * r;
        }
        block_sum_vec<10>(v, sh);
        if (threadIdx.x == 0) {
            // (J^T J + lm diag) delta = J^T r, by Cramer's rule on the 3x3 system
            const double a00 = v[0] * (1 + lm), a11 = v[3] * (1 + lm), a22 = v[5] * (1 + lm);
            const double a01 = v[1], a02 = v[2], a12 = v[4];
            const double det = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) + a02 * (a01 * a12 - a11 * a02);
            const double b0 = v[6], b1 = v[7], b2 = v[8];
            const double d0 = (b0 * (a11 * a22 - a12 * a12) - a01 * (b1 * a22 - a12 * b2) + a02 * (b1 * a12 - a11 * b2)) / det;
            const double d1 = (a00 * (b1 * a22 - a12 * b2) - b0 * (a01 * a22 - a12 * a02) + a02 * (a01 * b2 - b1 * a02)) / det;
            const double d2 = (a00 * (a11 * b2 - b1 * a12) - a01 * (a01 * b2 - b1 * a02) + b0 * (a01 * a12 - a11 * a02)) / det;
            s_p[0] = A + d0; s_p[1] = mu + d1; s_p[2] = sg + d2;
            s_done = (fabs(d0) <= 1e-14 * fabs(A) && fabs(d1) <= 1e-14 * (fabs(mu) + sg) && fabs(d2) <= 1e-14 * sg) ? 1 : 0;
        }
        __syncthreads();
        const double nA = s_p[0], nm = s_p[1], ns = fabs(s_p[2]);
        const int done = s_done;
        const double c1 = cost(nA, nm, ns);
        if (c1 <= c0) { A = nA; mu = nm; sg = ns; c0 = c1; lm = fmax(lm * 0.1, 1e-15); }
        else lm *= 10.0;
        if (done || lm > 1e12) break;
    }
    if (threadIdx.x == 0) {
        out[(int64_t)O_SIGMA_LSQ * s + w] = sg;
        out[(int64_t)O_GAMMA2_LSQ * s + w] = P.k * sg * sg / P.kT;
    }
}

// Eq. 13 with gamma_i^2 from the fitted sigma_i, <x_i> the sample mean.
__global__ void k_gauss_fit_profile(const DevProblem *__restrict__ probs, char *__restrict__ ws) {
    const DevProblem &P = probs[blockIdx.x];
    if (threadIdx.x != 0) return;
    const int s = P.n_windows;
    double *out = dptr(ws, P.off_out);
    const double *lam = dptr(ws, P.off_lambda);
    double g = 0.0;
    out[(int64_t)O_DF_GAUSS_LSQ * s] = 0.0;
    for (int j = 1; j < s; ++j) {
        const double dl = lam[j] - lam[j - 1];
        const double mean = out[(int64_t)O_XI_MEAN * s + j - 1];
        const double g2 = out[(int64_t)O_GAMMA2_LSQ * s + j - 1];
        g += P.k * dl * (lam[j - 1] - mean) + 0.5 * P.k * dl * dl * (1.0 - g2);
        out[(int64_t)O_DF_GAUSS_LSQ * s + j] = g;
    }
}

hipError_t launch_estimators(const DevProblem *d_probs, int n_probs, char *ws, int max_windows, hipStream_t stream) {
    hipLaunchKernelGGL(k_estimators, dim3(n_probs), dim3(256), 0, stream, d_probs, ws);
    hipLaunchKernelGGL(k_gauss_fit, dim3(max_windows, n_probs), dim3(256), 0, stream, d_probs, ws);
    hipLaunchKernelGGL(k_gauss_fit_profile, dim3(n_probs), dim3(64), 0, stream, d_probs, ws);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// App. C.  For the step i -> i+1, every non-empty x bin b of rho_i moves the work
// by a whole number of bins and carries probability rho_i(b); consecutive
// non-empty bins with the same move are merged into one (shift, probability)
// pair (the move is monotone in b).  Chain 0: x at the bin centre, move
// floor(dW_i(x) / dW).  Chain 1, the listing as printed: x at the bin's upper
// edge and truncation toward zero of W = w dW + dW_i(x), i.e. the move is
// floor(f) for w + f >= 0 and ceil(f) below, f = dW_i(x) / dW; its pairs keep
// both and merge only where both agree.  Chain 2, the reverse path: the bins of
// rho_{i+1} with the work of moving the centre back, dW^rev_i(x) = k/2
// [(x - lambda_i)^2 - (x - lambda_{i+1})^2], x at the bin centre, move floor.
//
// One 256-thread block per (window step, problem, chain).  The bins are taken 256
// at a time: the non-empty ones are compacted in order, run heads are marked, and
// each head sums its run left to right, the first run of a chunk continuing the
// last one of the previous chunk where the shifts agree, so every probability is
// the same left-to-right sum as in a sequential pass.
__device__ __forceinline__ int block_excl_scan(int v, int *sh, int &total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int a = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[255];
    const int r = sh[t] - v;
    __syncthreads();
    return r;
}

__device__ __forceinline__ int clamp_shift(double f) {
    return f > 2.0e9 ? 2000000000 : (f < -2.0e9 ? -2000000000 : (int)f);
}

__global__ __launch_bounds__(256) void k_appc_pairs(const DevProblem *__restrict__ probs, char *__restrict__ ws) {
#pragma clang fp contract(off)
    const DevProblem &P = probs[blockIdx.y];
    const int i = blockIdx.x, chain = blockIdx.z, t = threadIdx.x;
    if (P.w_half_bins <= 0 || i + 1 >= P.n_windows) return;
    const int K = P.xi_nbins;
    const int64_t sK = (int64_t)P.n_windows * K;
    const double *lam = dptr(ws, P.off_lambda);
    const double *tot = dptr(ws, P.off_tot);
    const int src = chain == 2 ? i + 1 : i;         // window whose x distribution is folded in
    const unsigned long long *hist = reinterpret_cast<const unsigned long long *>(ws + P.off_hist) + (int64_t)src * K;
    int *key0 = reinterpret_cast<int *>(ws + P.off_pairs_shift) + chain * sK + (int64_t)i * K;
    int *key1 = reinterpret_cast<int *>(ws + P.off_pairs_ceil) + (int64_t)i * K;   // chain 1 only
    double *prob = dptr(ws, P.off_pairs_prob) + chain * sK + (int64_t)i * K;
    const double n = tot[(int64_t)src * A_NFIELDS + A_N];
    const double li = lam[i], lj = lam[i + 1];
    __shared__ int s_scan[256];
    __shared__ int s_k0[256], s_k1[256], s_head[256];
    __shared__ double s_pb[256];
    int np = 0, last0 = 0, last1 = 0;
    for (int c0 = 0; c0 < K; c0 += 256) {
        const int b = c0 + t;
        const unsigned long long c = b < K ? hist[b] : 0ull;
        int k0 = 0, k1 = 0;
        double pb = 0.0;
        if (c != 0ull) {
            pb = (double)c / n;
            if (chain != 1) {
                const double xb = P.xi_min + ((double)b + 0.5) * P.xi_bin;
                const double la = chain == 0 ? li : lj, lb = chain == 0 ? lj : li;   // from la to lb
                const double dW = 0.5 * P.k * ((xb - lb) * (xb - lb) - (xb - la) * (xb - la));
                k0 = k1 = clamp_shift(floor(dW / P.w_bin));
            } else {
                const double xb = P.xi_min + ((double)b + 1.0) * P.xi_bin;
                const double f = 0.5 * P.k * ((xb - lj) * (xb - lj) - (xb - li) * (xb - li)) / P.w_bin;
                k0 = clamp_shift(floor(f));
                k1 = clamp_shift(ceil(f));
            }
        }
        int nnz;
        const int pos = block_excl_scan(c != 0ull ? 1 : 0, s_scan, nnz);
        if (c != 0ull) { s_k0[pos] = k0; s_k1[pos] = k1; s_pb[pos] = pb; }
        __syncthreads();
        int head = 0;
        if (t < nnz) {
            const int p0 = t ? s_k0[t - 1] : last0, p1 = t ? s_k1[t - 1] : last1;
            head = (t == 0 && np == 0) || s_k0[t] != p0 || s_k1[t] != p1;
            s_head[t] = head;
        }
        int nheads;
        const int rid = block_excl_scan(head, s_scan, nheads);
        if (head) {
            double p = s_pb[t];
            for (int m = t + 1; m < nnz && !s_head[m]; ++m) p += s_pb[m];
            key0[np + rid] = s_k0[t];
            if (chain == 1) key1[np + rid] = s_k1[t];
            prob[np + rid] = p;
        } else if (t == 0 && nnz > 0) {
            // the chunk opens inside the previous chunk's last run
            double p = prob[np - 1];
            for (int m = 0; m < nnz && !s_head[m]; ++m) p += s_pb[m];
            prob[np - 1] = p;
        }
        if (nnz > 0) { last0 = s_k0[nnz - 1]; last1 = s_k1[nnz - 1]; }
        np += nheads;
        __syncthreads();
    }
    if (t == 0) reinterpret_cast<int *>(ws + P.off_npairs)[chain * P.n_windows + i] = np;
}

// Omega_j(w) = sum_t prob_t Omega_{j-1}(w - shift_t), the folding step of App. C,
// for the three chains (blockIdx.z; chain 2, the reverse path, folds like chain 0).
// Chain 1 folds as printed: target w > 0 takes source w - floor(f),
// w < 0 takes w - ceil(f); at w = 0 the printed step keeps the mean of the
// results at w = -1 and w = +1 instead, which are exactly what the targets -1 and
// +1 compute, so the bin is left unsmoothed here and every reader of Omega_j
// (j >= 1) of chain 1 takes the mean of its neighbours there (omega_at).
//
// A block owns 256 consecutive target bins.  Pairs are taken 256 at a time; for
// each, the sources that the block's targets read lie in 259 consecutive bins
// (one spare on either side), which are staged in LDS together with those of
// the other pairs of the chunk, so the inner loop is one LDS read and one FMA per
// pair.  Pairs whose sources cannot all share one staging window of kAppcStage
// bins are taken in further windows; pairs whose sources lie wholly outside the
// histogram get weight 0.  With one window the sums run in pair order.
constexpr int kAppcStage = 4096;
constexpr int kAppcSpan = 259;                  // sources of one pair for one block

__device__ __forceinline__ double omega_at(const double *om, int64_t b, int M, bool smooth) {
    return (smooth && b == M) ? 0.5 * (om[M - 1] + om[M + 1]) : om[b];
}

__device__ __forceinline__ int64_t block_min_max(int64_t v, bool is_min, int64_t *sh) {
    for (int off = 32; off >= 1; off >>= 1) {
        const int64_t o = __shfl_xor(v, off);
        v = is_min ? (o < v ? o : v) : (o > v ? o : v);
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t r = sh[0];
    for (int q = 1; q < 4; ++q) r = is_min ? (sh[q] < r ? sh[q] : r) : (sh[q] > r ? sh[q] : r);
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_appc_step(const DevProblem *__restrict__ probs, char *__restrict__ ws, int j) {
    const DevProblem &P = probs[blockIdx.y];
    if (P.w_half_bins <= 0 || j >= P.n_windows) return;
    const int chain = blockIdx.z;
    const int M = P.w_half_bins;
    const int64_t nb = 2 * (int64_t)M + 1;
    const int64_t w0 = (int64_t)blockIdx.x * 256;
    if (w0 >= nb) return;
    const int64_t sK = (int64_t)P.n_windows * P.xi_nbins;
    const int64_t w = w0 + threadIdx.x;
    const int np = reinterpret_cast<const int *>(ws + P.off_npairs)[chain * P.n_windows + j - 1];
    const int *shift = reinterpret_cast<const int *>(ws + P.off_pairs_shift) + chain * sK + (int64_t)(j - 1) * P.xi_nbins;
    const int *ceil_s = reinterpret_cast<const int *>(ws + P.off_pairs_ceil) + (int64_t)(j - 1) * P.xi_nbins;
    const double *prob = dptr(ws, P.off_pairs_prob) + chain * sK + (int64_t)(j - 1) * P.xi_nbins;
    const double *prev = dptr(ws, P.off_omega) + chain * (int64_t)P.n_windows * nb + (int64_t)(j - 1) * nb;
    double *cur = dptr(ws, P.off_omega) + chain * (int64_t)P.n_windows * nb + (int64_t)j * nb;
    const bool smooth_prev = chain == 1 && j >= 2;
    __shared__ int s_sf[256], s_sc[256], s_win[256];
    __shared__ double s_prob[256];
    __shared__ int64_t s_red[4];
    __shared__ double s_src[kAppcStage];
    // chain 1 below W = 0 reads through ceil(f), everything else through floor(f)
    const int *sel = (chain == 1 && w < M) ? s_sc : s_sf;
    constexpr int64_t kNone = INT64_MAX;
    constexpr int64_t step = kAppcStage - kAppcSpan;
    double acc = 0.0;
    for (int t0 = 0; t0 < np; t0 += 256) {
        const int cnt = np - t0 < 256 ? np - t0 : 256;
        const int t = threadIdx.x;
        int sf = 0, sc = 0;
        double pt = 0.0;
        int64_t first = kNone;
        if (t < cnt) {
            sf = shift[t0 + t];
            sc = chain == 1 ? ceil_s[t0 + t] : sf;
            pt = prob[t0 + t];
            first = w0 - 1 - (int64_t)(sc > sf ? sc : sf);
            if (first + kAppcSpan <= 0 || first >= nb) first = kNone;    // reads nothing in range
        }
        const int64_t base = block_min_max(first, true, s_red);
        if (base == kNone) continue;                                      // uniform
        const int64_t top = block_min_max(first == kNone ? INT64_MIN : first, false, s_red);
        if (t < cnt) {
            if (first == kNone) {          // weight 0, reading a staged bin of the first window
                sf = sc = (int)(w0 - 1 - base);
                pt = 0.0;
                first = base;
            }
            s_sf[t] = sf;
            s_sc[t] = sc;
            s_prob[t] = pt;
            s_win[t] = (int)((first - base) / step);
        }
        const int n_win = (int)((top - base) / step) + 1;
        for (int win = 0; win < n_win; ++win) {
            const int64_t start = base + (int64_t)win * step;
            const int64_t len = top - start + kAppcSpan < kAppcStage ? top - start + kAppcSpan : kAppcStage;
            for (int q = threadIdx.x; q < len; q += 256) {
                const int64_t src = start + q;
                s_src[q] = (src >= 0 && src < nb) ? omega_at(prev, src, M, smooth_prev) : 0.0;
            }
            __syncthreads();
            if (w < nb) {
                const int off = (int)(w - start);   // s_src[off - s] = Omega_{j-1}(w - s)
                if (n_win == 1) {
#pragma unroll 8
                    for (int u = 0; u < cnt; ++u) acc += s_prob[u] * s_src[off - sel[u]];
                } else {
                    for (int u = 0; u < cnt; ++u)
                        if (s_win[u] == win) acc += s_prob[u] * s_src[off - sel[u]];
                }
            }
            __syncthreads();
        }
    }
    if (w < nb) cur[w] = acc;
}

// Statistics of Omega_j: normalised exponential average (App. B.5), spread and
// the number of non-empty bins, the JE variance formula of Sec. IV A.
__global__ __launch_bounds__(256) void k_appc_stats(const DevProblem *__restrict__ probs, char *__restrict__ ws) {
    const DevProblem &P = probs[blockIdx.y];
    const int j = blockIdx.x;
    const int chain = blockIdx.z;
    __shared__ double sh[256];
    const int s = P.n_windows;
    if (P.w_half_bins <= 0 || j >= s) return;
    const int M = P.w_half_bins;
    const int64_t nb = 2 * (int64_t)M + 1;
    const double *om = dptr(ws, P.off_omega) + chain * (int64_t)s * nb + (int64_t)j * nb;
    double *out = dptr(ws, P.off_out);
    const double beta = P.beta, dWb = P.w_bin;
    const double shift_mid = 0.5 * (double)j * dWb;
    double tot = 0, q = 0, mw = 0, emax = -INFINITY;
    const bool smooth = chain == 1 && j >= 1;   // chain 1 keeps W = 0 unsmoothed in memory
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
        const double o = omega_at(om, b, M, smooth);
        if (o != 0.0) {
            const double W = (double)(b - M) * dWb;
            tot += o; q += 1.0; mw += o * W;
            emax = fmax(emax, -beta * W);
        }
    }
    tot = block_sum(tot, sh);
    q = block_sum(q, sh);
    mw = block_sum(mw, sh);
    // block max
    sh[threadIdx.x] = emax;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    emax = sh[0];
    __syncthreads();
    const double mean = mw / tot;
    double sl = 0, sm = 0, vv = 0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
        const double o = omega_at(om, b, M, smooth);
        if (o != 0.0) {
            const double W = (double)(b - M) * dWb;
            sl += o * exp(-beta * W - emax);
            sm += o * exp(-beta * (W + shift_mid) - emax);
            vv += o * (W - mean) * (W - mean);
        }
    }
    sl = block_sum(sl, sh);
    sm = block_sum(sm, sh);
    vv = block_sum(vv, sh);
    if (chain == 2) {
        // reverse JE over the path lambda_j -> lambda_1: <exp(-beta W_rev)> = exp(+beta dF_j)
        if (threadIdx.x == 0) out[(int64_t)O_DF_REV_HIST * s + j] = tot > 0 ? P.kT * (emax + log(sl / tot)) : NAN;
        // Crooks and Kofke: the forward distribution against the mirrored reverse one.
        // After j folds a forward bin w holds work in [w, w + j) dW and a reverse bin v
        // in [v, v + j) dW, so -W_rev matches forward bin w at v = -w - j.
        const double *of = dptr(ws, P.off_omega) + (int64_t)j * nb;      // chain 0
        double ovl = 0, wm = 0, wf = 0;
        for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
            const int64_t v = 2 * (int64_t)M - b - j;                     // index of bin -w - j
            if (v < 0 || v >= nb) continue;
            const double f = of[b], r = om[v];
            const double m = fmin(f, r);
            ovl += m;
            if (f > 0.0 && r > 0.0) {
                // P_f(W) / P_r(-W) = exp(beta (W - dF)): each common bin gives W - kT ln(P_f / P_r)
                wm += m;
                wf += m * (((double)(b - M) + 0.5 * j) * dWb - P.kT * log(f / r));
            }
        }
        ovl = block_sum(ovl, sh);
        wm = block_sum(wm, sh);
        wf = block_sum(wf, sh);
        if (threadIdx.x == 0) {
            out[(int64_t)O_CROOKS_OVL * s + j] = ovl;
            out[(int64_t)O_DF_CROOKS * s + j] = wm > 0 ? wf / wm : NAN;
        }
    } else if (threadIdx.x == 0 && chain == 1) {
        out[(int64_t)O_DF_JE_HIST_LIT * s + j] = tot > 0 ? -P.kT * (emax + log(sl / tot)) : NAN;
    } else if (threadIdx.x == 0) {
        const double kT = P.kT;
        const double sig = sqrt(fmax(vv / tot, 0.0));
        out[(int64_t)O_DF_JE_HIST * s + j] = tot > 0 ? -kT * (emax + log(sl / tot)) : NAN;
        out[(int64_t)O_DF_JE_HIST_MID * s + j] = tot > 0 ? -kT * (emax + log(sm / tot)) : NAN;
        out[(int64_t)O_SIGMA_W * s + j] = sig;
        out[(int64_t)O_Q_BINS * s + j] = q;
        out[(int64_t)O_WORK_LOST * s + j] = 1.0 - tot;
        double var = 0.0;
        if (j > 0 && q > 1.0) var = sig * sig / q + beta * beta * sig * sig * sig * sig / (2.0 * (q - 1.0));
        out[(int64_t)O_VAR_PAPER * s + j] = var;
    }
}

hipError_t launch_appc(const DevProblem *d_probs, int n_probs, char *ws, int max_windows, int max_m,
                       hipStream_t stream) {
    if (max_m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_appc_pairs, dim3(max_windows, n_probs, kAppcChains), dim3(256), 0, stream, d_probs, ws);
    const int64_t nb = 2 * (int64_t)max_m + 1;
    const int grid = (int)((nb + 255) / 256);
    for (int j = 1; j < max_windows; ++j)
        hipLaunchKernelGGL(k_appc_step, dim3(grid, n_probs, kAppcChains), dim3(256), 0, stream, d_probs, ws, j);
    hipLaunchKernelGGL(k_appc_stats, dim3(max_windows, n_probs, kAppcChains), dim3(256), 0, stream, d_probs, ws);
    return hipGetLastError();
}

}  // namespace ppp

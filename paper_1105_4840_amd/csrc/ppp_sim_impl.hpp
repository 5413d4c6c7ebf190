// Simulation kernels (device code, included by the shape translation units) of the parallel pulling protocol (Sec. III(ii)): many
// independent restrained Langevin replicas per window lambda_i, all started
// from the shared state x_o, each recording xi every sample_every steps after
// n_equil and folding it straight into fp64 accumulators:
//   n, sum(xi - lambda_i), sum(xi - lambda_i)^2, min, max, the histogram rho_i,
//   and running log-sum-exp pairs of a = -beta dW_i (Eq. 9 summand) for the
//   forward step and of the reverse step, each also for 2a (Kish size).
//
// Two kernels:
//   * sim_1d: one lane per replica, overdamped dynamics of one coordinate.
//   * sim_chain<T, G, B>: G consecutive lanes of a wavefront per replica (any G
//     up to 64; 64 / G groups per wavefront, the remaining lanes idle), B beads
//     per lane in registers (lane g owns beads gB .. gB+B-1).  The
//     Lennard-Jones sum uses each unique pair once (Newton's third law): the
//     j-beads rotate one lane per round through the group together with an
//     accumulator of their reaction forces, which finally is pushed back to
//     the owning lane (for even G the last round, which meets the opposite
//     lane, is done from both sides instead).  Each bond and angle is
//     computed once, by the lane owning its first or central bead, from a
//     one-bead halo read from the neighbouring lanes, which read back the
//     forces on their halo beads.  Inside the step loop nothing leaves
//     registers except each sample's accumulator update and histogram count
//     (LDS).
#pragma once
#include <hip/hip_runtime.h>

#include "ppp_device.hpp"
#include "ppp_launch.hpp"
#include "ppp_chain_force.hpp"

namespace ppp {

__device__ __forceinline__ double centre_at(const DevProblem &P, double lam, int64_t n) {
    if (P.n_pull <= 0 || n >= P.n_pull) return lam;
    return P.xi_start + (lam - P.xi_start) * ((double)n / (double)P.n_pull);
}

// Sequential protocol: every replica runs the windows one after another,
// n_steps each, with steps counted from the start of window 1.  A launch never
// crosses a window boundary, so its window is that of its first step.  The
// parallel protocol is the case of window 0 for every launch.
__device__ __forceinline__ int64_t seq_window(const DevProblem &P, int64_t step_begin) {
    return P.sequential ? step_begin / P.n_steps : 0;
}

// First step after `after` at which xi is sampled (steps n > n_equil with
// n - n_equil a multiple of sample_every); the loops then count up to it
// instead of taking a 64-bit remainder every step.
__device__ __forceinline__ int64_t next_sample_after(const DevProblem &P, int64_t after) {
    if (after < P.n_equil) return P.n_equil + P.sample_every;
    return P.n_equil + ((after - P.n_equil) / P.sample_every + 1) * P.sample_every;
}

// Per-replica constants of the sampling step: the forward and reverse exponents
// a = -beta dW of one sample, evaluated exactly as written below but with the
// window's lambda values read once per replica instead of once per sample.
// kind 1: a step to the neighbouring window, a = cf (d - h) with cf = beta k dl,
// h = dl/2, dl the centre's move, d = xi - lambda_w; kind 2: switching the
// restraint on or off, a = q e e with e = xi - ref.
struct SampleCoef {
    double lam_w;
    int kind_f, kind_r;
    double cf, hf, cr, hr;
    double qf, qr, ref_f, ref_r;
};

__device__ __forceinline__ SampleCoef sample_coef(const DevProblem &P, const double *lam, int w) {
    const int s = P.n_windows;
    SampleCoef c;
    c.lam_w = lam[w];
    c.kind_f = c.kind_r = 0;
    c.cf = c.hf = c.cr = c.hr = c.qf = c.qr = c.ref_f = c.ref_r = 0.0;
    const double bk = P.beta * P.k;
    if (w == s) {
        // the unrestrained ensemble (d = xi - lambda_1): switching the restraint on
        // at lambda_1 or at lambda_s costs W_H = k/2 (x_0 - lambda)^2 (Eqs. 4, 6)
        c.kind_f = c.kind_r = 2;
        c.qf = c.qr = -0.5 * P.beta * P.k;
        c.ref_f = lam[s];                 // lambda_1
        c.ref_r = lam[s - 1];
    } else {
        if (w + 1 < s) {
            // a = -beta k/2 [(xi - lambda_{i+1})^2 - (xi - lambda_i)^2] = beta k dl (d - dl/2)
            const double dl = lam[w + 1] - lam[w];
            c.kind_f = 1; c.cf = bk * dl; c.hf = 0.5 * dl;
        } else if (P.free_ens) {
            // switching the restraint at lambda_s off: a = +beta k/2 d^2 (Eq. 5)
            c.kind_f = 2; c.qf = 0.5 * P.beta * P.k; c.ref_f = lam[w];
        }
        if (w > 0) {
            const double dl = lam[w - 1] - lam[w];
            c.kind_r = 1; c.cr = bk * dl; c.hr = 0.5 * dl;
        } else if (P.free_ens) {
            c.kind_r = 2; c.qr = 0.5 * P.beta * P.k; c.ref_r = lam[w];   // the same at lambda_1 (Eq. 5)
        }
    }
    return c;
}

// Folds one sample xi of window w into the replica's accumulator.  The
// histogram count goes to the workgroup's LDS copy of window w's histogram
// (lhist) when there is one, else straight to memory.
__device__ __forceinline__ void accumulate(const DevProblem &P, const SampleCoef &C, int w, double xi,
                                           double *acc, unsigned long long *hist, unsigned int *lhist) {
    const double d = xi - C.lam_w;
    acc[A_N] += 1.0;
    acc[A_S1] += d;
    acc[A_S2] += d * d;
    acc[A_XMIN] = fmin(acc[A_XMIN], xi);
    acc[A_XMAX] = fmax(acc[A_XMAX], xi);
    if (C.kind_f == 1) {
        lse_push_pair(acc[A_MF], acc[A_SF], acc[A_MF2], acc[A_SF2], C.cf * (d - C.hf));
    } else if (C.kind_f == 2) {
        const double e = xi - C.ref_f;
        lse_push_pair(acc[A_MF], acc[A_SF], acc[A_MF2], acc[A_SF2], C.qf * e * e);
    }
    if (C.kind_r == 1) {
        lse_push_pair(acc[A_MR], acc[A_SR], acc[A_MR2], acc[A_SR2], C.cr * (d - C.hr));
    } else if (C.kind_r == 2) {
        const double e = xi - C.ref_r;
        lse_push_pair(acc[A_MR], acc[A_SR], acc[A_MR2], acc[A_SR2], C.qr * e * e);
    }
    const double fb = floor((xi - P.xi_min) / P.xi_bin);
    if (fb < 0.0) acc[A_UNDER] += 1.0;
    else if (fb >= (double)P.xi_nbins) acc[A_OVER] += 1.0;
    else if (lhist) atomicAdd(lhist + (int)fb, 1u);
    else atomicAdd(hist + (int64_t)w * P.xi_nbins + (int64_t)fb, 1ull);
}

// Workgroup-private histogram: cleared before an item, added to the window's
// histogram in memory after it (one atomic per non-empty bin).
__device__ __forceinline__ void lhist_clear(unsigned int *lhist, int K) {
    for (int b = threadIdx.x; b < K; b += blockDim.x) lhist[b] = 0u;
    __syncthreads();
}
__device__ __forceinline__ void lhist_flush(unsigned int *lhist, int K, unsigned long long *dst) {
    __syncthreads();
    for (int b = threadIdx.x; b < K; b += blockDim.x) {
        const unsigned int c = lhist[b];
        if (c) atomicAdd(dst + b, (unsigned long long)c);
    }
    __syncthreads();
}

// Bins of the workgroup histogram of an item: K for every window its replicas
// fall in (INT32_MAX when that would not fit an int).
__device__ __forceinline__ int item_hist_bins(const DevProblem &P, const WorkItem &item) {
    const int64_t last = (int64_t)item.window * P.n_replicas + item.rep_begin + item.n_reps - 1;
    const int64_t nw = last / P.n_replicas - item.window + 1;
    const int64_t nk = nw * (int64_t)P.xi_nbins;
    return nk < (int64_t)INT32_MAX ? (int)nk : INT32_MAX;
}

template <typename T> __device__ __forceinline__ T *state_ptr(char *ws, const DevProblem &P) {
    return reinterpret_cast<T *>(ws + P.off_state);
}

// ===========================================================================
// 1-D overdamped model: x_{n+1} = x_n + mu dt F(x_n) + sqrt(mu kT dt/2) (eta_n + eta_{n+1})
// (Leimkuhler-Matthews) or + sqrt(2 mu kT dt) eta_{n+1} (Euler-Maruyama).
// eta_n is component n mod 4 of the Philox block with counter (gid, n div 4, 0, 0).
// ===========================================================================
template <typename T>
__device__ __forceinline__ T force_1d(const DevProblem &P, T x, T centre, T kr) {
    T f;
    if (P.pot_kind == 0) f = (T)(-4.0 * P.pot_a) * x * (x * x - (T)P.pot_b);
    else f = (T)(-P.pot_kappa) * x;
    return f - kr * (x - centre);
}

// Restraint stiffness of window w: k, or 0 for the unrestrained ensemble (w = s).
__device__ __forceinline__ double window_k(const DevProblem &P, int w) { return w < P.n_windows ? P.k : 0.0; }

template <typename T>
__device__ __forceinline__ void sim_1d_replica(const DevProblem &P, const WorkItem &item, int w, int rep, char *ws,
                                               int64_t step_begin, int64_t step_end, double *traj, int traj_rep,
                                               unsigned int *lhist) {
    if ((int)threadIdx.x >= item.n_reps) return;
    // record (window, replica); the sequential protocol keeps one state per replica
    // and draws replica `rep`'s window-1 noise all the way
    const int64_t g = (int64_t)w * P.n_replicas + rep;
    const int64_t gs = P.sequential ? rep : g;
    const uint32_t gid = (uint32_t)gs;
    const int64_t s0 = P.sequential ? (int64_t)w * P.n_steps : 0;   // first step of this window
    const double *lam = reinterpret_cast<const double *>(ws + P.off_lambda);
    double *acc_g = reinterpret_cast<double *>(ws + P.off_acc) + g * A_NFIELDS;
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(ws + P.off_hist);
    T *st = state_ptr<T>(ws, P) + gs * 2;
    const double lam_w = lam[w];
    const SampleCoef coef = sample_coef(P, lam, w);
    const double x_start = reinterpret_cast<const double *>(ws + P.off_init)[0];
    const int64_t n_end = step_end < s0 + P.n_steps ? step_end : s0 + P.n_steps;

    double acc[A_NFIELDS];
    T x, eta_prev;
    if (step_begin == 0) {
        acc_empty(acc);
        x = (T)x_start;
        T z[4];
        Normal4<T>::get(P.seed, gid, 0u, 0u, 0u, z);
        eta_prev = z[0];
    } else if (step_begin == s0) {
        // sequential protocol entering window w: the state goes on, the record starts
        // empty, and a replica frozen in the previous window stays frozen
        acc_empty(acc);
        acc[A_BLOWN] = acc_g[-(int64_t)P.n_replicas * A_NFIELDS + A_BLOWN];
        x = st[0]; eta_prev = st[1];
    } else {
        for (int f = 0; f < A_NFIELDS; ++f) acc[f] = acc_g[f];
        x = st[0]; eta_prev = st[1];
    }
    const bool record = traj != nullptr && g == traj_rep;
    if (record && step_begin == 0) traj[0] = (double)x;
    const T kr = (T)window_k(P, w);
    const T mu_dt = (T)(P.mobility * P.dt);
    const T amp = P.integrator_1d == 0 ? (T)sqrt(0.5 * P.mobility * P.kT * P.dt)
                                       : (T)sqrt(2.0 * P.mobility * P.kT * P.dt);
    bool alive = acc[A_BLOWN] == 0.0;
    T z[4];
    uint32_t zblock = 0xFFFFFFFFu;
    int64_t n_sample = s0 + next_sample_after(P, step_begin - s0);
    for (int64_t n = step_begin + 1; n <= n_end && alive; ++n) {
        const T F = force_1d<T>(P, x, (T)(w == 0 || !P.sequential ? centre_at(P, lam_w, n - 1) : lam_w), kr);
        const uint32_t blk = (uint32_t)(n >> 2);
        if (blk != zblock) { Normal4<T>::get(P.seed, gid, blk, 0u, 0u, z); zblock = blk; }
        const T eta = z[n & 3];
        if (P.integrator_1d == 0) x = x + mu_dt * F + amp * (eta_prev + eta);
        else x = x + mu_dt * F + amp * eta;
        eta_prev = eta;
        if (record && n <= 100000) traj[n] = (double)x;
        if (n == n_sample) {
            n_sample += P.sample_every;
            const double xi = (double)x;
            if (!isfinite(xi) || fabs(xi) > P.xi_bound) { acc[A_BLOWN] = 1.0; alive = false; break; }
            accumulate(P, coef, w, xi, acc, hist, lhist);
        }
    }
    for (int f = 0; f < A_NFIELDS; ++f) acc_g[f] = acc[f];
    st[0] = x; st[1] = eta_prev;
}

template <typename T>
__global__ __launch_bounds__(WG) void sim_1d(const DevProblem *__restrict__ probs, const WorkItem *__restrict__ items,
                                             int n_items, char *__restrict__ ws, int64_t step_begin,
                                             int64_t step_end, double *__restrict__ traj, int traj_rep, int lds_cap) {
    extern __shared__ unsigned int s_hist[];
    const int it = blockIdx.x;
    if (it >= n_items) return;
    const WorkItem item = items[it];
    const DevProblem &P = probs[item.prob];
    const int w = P.sequential ? (int)seq_window(P, step_begin) : item.window;
    const int rep = item.rep_begin + (int)threadIdx.x;
    unsigned int *lhist = P.xi_nbins <= lds_cap ? s_hist : nullptr;
    if (lhist) lhist_clear(lhist, P.xi_nbins);
    sim_1d_replica<T>(P, item, w, rep, ws, step_begin, step_end, traj, traj_rep, lhist);
    if (lhist) lhist_flush(lhist, P.xi_nbins, reinterpret_cast<unsigned long long *>(ws + P.off_hist) + (int64_t)w * P.xi_nbins);
}


template <typename T, int G, int B>
__device__ __forceinline__ void run_chain_item(const DevProblem &P, const WorkItem &item, char *ws, int64_t step_begin,
                                               int64_t step_end, double *traj, int64_t traj_rep, double *s_acc,
                                               unsigned int *lhist) {
    constexpr int NPAD = G * B;
    constexpr int GPW = groups_per_wave(G);
    const int lane = lane_id();
    const bool lane_used = lane < GPW * G;
    const int grp = (int)(threadIdx.x >> 6) * GPW + (lane_used ? lane / G : 0);
    const int g = lane_used ? lane % G : 0;
    const int gbase = lane_used ? lane - g : lane;
    const bool active = lane_used && grp < item.n_reps;
    const int N = P.n_beads;
    const int64_t gfirst = (int64_t)item.window * P.n_replicas + item.rep_begin;
    // gi: replica number (window * R + replica); the sequential protocol's items are
    // window-1 replicas that run window `stage` in this launch
    const int64_t gi = gfirst + (active ? grp : 0);
    const int64_t stage = seq_window(P, step_begin);
    const int64_t s0 = stage * P.n_steps;         // first step of this window (0: parallel protocol)
    const int w = P.sequential ? (int)stage : (int)(gi / P.n_replicas);   // this replica's window now
    const int64_t grec = P.sequential ? stage * P.n_replicas + gi : gi;   // its record
    const uint32_t gid = (uint32_t)gi;
    // the workgroup's histogram holds the windows item.window, item.window + 1, ...
    // (the one window `stage` in the sequential protocol)
    unsigned int *lhist_w = lhist ? lhist + (P.sequential ? 0 : (int64_t)(w - item.window) * P.xi_nbins) : nullptr;
    const double *lam = reinterpret_cast<const double *>(ws + P.off_lambda);
    const double *x0 = reinterpret_cast<const double *>(ws + P.off_init);
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(ws + P.off_hist);
    double *acc_g = reinterpret_cast<double *>(ws + P.off_acc) + grec * A_NFIELDS;
    T *st = state_ptr<T>(ws, P) + gi * 6 * NPAD;
    const double lam_w = lam[w];
    const SampleCoef coef = sample_coef(P, lam, w);
    const int64_t n_end = step_end < s0 + P.n_steps ? step_end : s0 + P.n_steps;
    auto centre = [&](int64_t n) { return stage == 0 ? centre_at(P, lam_w, n) : lam_w; };
    const T kr = (T)window_k(P, w);
    const int i0 = g * B;
    const int last = N - 1;
    const int owner = last / B;       // lane (within group) owning the pulled end
    double *acc = s_acc + grp * A_NFIELDS;

    T px[B], py[B], pz[B], vx[B], vy[B], vz[B], fx[B], fy[B], fz[B];
    if (step_begin == 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            if (i < N) { px[b] = (T)x0[3 * i]; py[b] = (T)x0[3 * i + 1]; pz[b] = (T)x0[3 * i + 2]; }
            else { px[b] = 0; py[b] = 0; pz[b] = (T)(P.pad_z0 + P.pad_dz * (i - N)); }
        }
        lane_noise<T, B>(P, gid, 0u, i0, [&](int b, const T *z) {
            const int i = i0 + b;
            const bool mobile = i > 0 && i < N;
            vx[b] = mobile ? (T)P.sd_v * z[0] : (T)0;
            vy[b] = mobile ? (T)P.sd_v * z[1] : (T)0;
            vz[b] = mobile ? (T)P.sd_v * z[2] : (T)0;
        });
        if (lane_used && g == owner) acc_empty(acc);
    } else {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            px[b] = st[0 * NPAD + i0 + b]; py[b] = st[1 * NPAD + i0 + b]; pz[b] = st[2 * NPAD + i0 + b];
            vx[b] = st[3 * NPAD + i0 + b]; vy[b] = st[4 * NPAD + i0 + b]; vz[b] = st[5 * NPAD + i0 + b];
        }
        if (lane_used && g == owner) {
            if (step_begin == s0) {
                // sequential protocol entering window `stage`: the record starts empty,
                // and a replica frozen in the previous window stays frozen
                acc_empty(acc);
                acc[A_BLOWN] = acc_g[-(int64_t)P.n_replicas * A_NFIELDS + A_BLOWN];
            } else {
                for (int f = 0; f < A_NFIELDS; ++f) acc[f] = acc_g[f];
            }
        }
    }
    const bool record = traj != nullptr && gi == traj_rep && active;
    if (record && step_begin == 0) {
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (i0 + b < N) { traj[3 * (i0 + b)] = (double)px[b]; traj[3 * (i0 + b) + 1] = (double)py[b]; traj[3 * (i0 + b) + 2] = (double)pz[b]; }
    }
    // group-uniform liveness (owner's accumulator holds the flag)
    const int blown0 = (g == owner) ? (int)acc[A_BLOWN] : 0;
    const uint64_t bal0 = __ballot(blown0 != 0);
    bool alive = active && ((bal0 >> gbase) & ((G == 64) ? ~0ull : ((1ull << G) - 1))) == 0ull;

    ChainForce<T, G, B, false>::compute(P, g, gbase, (T)centre(step_begin), kr, px, py, pz, fx, fy, fz, nullptr);

    const T h = (T)(0.5 * P.dt);
    const T c1 = (T)P.c1;
    const T hm = (T)(0.5 * P.dt * P.inv_mass);
    const T c2sd = (T)P.c2sd;
    int64_t n_sample = s0 + next_sample_after(P, step_begin - s0);
    for (int64_t n = step_begin + 1; n <= n_end; ++n) {
        if (!alive) break;
        baoab_step<T, G, B>(P, g, gbase, gid, (uint32_t)n, (T)centre(n), kr, h, hm, c1, c2sd, px, py, pz, vx, vy, vz,
                            fx, fy, fz);
        if (record && n <= 100000) {
#pragma unroll
            for (int b = 0; b < B; ++b)
                if (i0 + b < N) {
                    double *o = traj + (int64_t)n * 3 * N + 3 * (i0 + b);
                    o[0] = (double)px[b]; o[1] = (double)py[b]; o[2] = (double)pz[b];
                }
        }
        if (n == n_sample) {
            n_sample += P.sample_every;
            bool ok = true;
#pragma unroll
            for (int b = 0; b < B; ++b)
                if (i0 + b < N) ok = ok && isfinite((double)px[b]) && isfinite((double)py[b]) && isfinite((double)pz[b]);
            double xi = 0.0;
            if (g == owner) {
#pragma unroll
                for (int b = 0; b < B; ++b)
                    if (i0 + b == last) {
                        const double dx = (double)px[b] - P.fix_x, dy = (double)py[b] - P.fix_y, dz = (double)pz[b] - P.fix_z;
                        xi = P.rc_mode == 1 ? dz : sqrt(dx * dx + dy * dy + dz * dz);
                    }
                ok = ok && isfinite(xi) && fabs(xi) <= P.xi_bound;
            }
            const uint64_t bad = __ballot(!ok);
            const bool grp_bad = ((bad >> gbase) & ((G == 64) ? ~0ull : ((1ull << G) - 1))) != 0ull;
            if (grp_bad) {
                if (g == owner) acc[A_BLOWN] = 1.0;
                alive = false;
            } else if (g == owner) {
                accumulate(P, coef, w, xi, acc, hist, lhist_w);
            }
        }
    }
    if (active) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            st[0 * NPAD + i0 + b] = px[b]; st[1 * NPAD + i0 + b] = py[b]; st[2 * NPAD + i0 + b] = pz[b];
            st[3 * NPAD + i0 + b] = vx[b]; st[4 * NPAD + i0 + b] = vy[b]; st[5 * NPAD + i0 + b] = vz[b];
        }
        if (g == owner) for (int f = 0; f < A_NFIELDS; ++f) acc_g[f] = acc[f];
    }
}

// Waves per SIMD the compiler schedules the chain kernels for.  The 64x4
// kernel keeps a replica's 16 pair distances and all its lane exchanges of a
// round in flight (about 250 registers): it runs two waves per SIMD whatever
// the schedule, and asked for more the scheduler trades that overlap away and
// the kernel slows by a sixth.  Every other shape keeps the default (8).
template <int G, int B> constexpr int chain_max_waves() { return (G == 64 && B == 4) ? 2 : 8; }

// Least waves per SIMD a direct launch is compiled for.  Left to itself the
// compiler lands the fp32 kernels of chains longer than ten beads a few
// registers above a wave boundary (16x2: 147 VGPRs, three waves; 3x4, 4x4 and
// 8x4..32x4: 171-173, two waves).  Asked for one wave more they fit under it
// (128, 168) without spilling and run 5-11% faster on 12- to 128-bead chains,
// with the same machine arithmetic.  The 5x2 kernel keeps the default: the
// 10-bead workload gives each SIMD fewer than two waves, and the tighter
// budget costs it 4%.  The persistent kernel keeps one: its item loop holds
// the fp64 exponential's constants in registers for the whole launch, and at
// these floors it spills.
template <typename T, int G, int B> constexpr int chain_min_waves() {
    return sizeof(T) != 4 ? 1 : (B == 2 && G >= 8) ? 4 : (B == 4 && G >= 3 && G <= 32) ? 3 : 1;
}

// Direct launch: one work item per workgroup.
template <typename T, int G, int B>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(chain_min_waves<T, G, B>(), chain_max_waves<G, B>()))) void sim_chain(const DevProblem *__restrict__ probs, const WorkItem *__restrict__ items,
                                                int n_items, char *__restrict__ ws, int64_t step_begin,
                                                int64_t step_end, double *__restrict__ traj, int64_t traj_rep,
                                                int lds_cap) {
    __shared__ double s_acc[chain_reps_per_wg(G) * A_NFIELDS];
    extern __shared__ unsigned int s_hist[];
    if ((int)blockIdx.x >= n_items) return;
    const WorkItem item = items[blockIdx.x];
    const DevProblem &P = probs[item.prob];
    const int nk = item_hist_bins(P, item);
    unsigned int *lhist = nk <= lds_cap ? s_hist : nullptr;
    if (lhist) lhist_clear(lhist, nk);
    run_chain_item<T, G, B>(P, item, ws, step_begin, step_end, traj, traj_rep, s_acc, lhist);
    const int64_t w0 = P.sequential ? seq_window(P, step_begin) : item.window;
    if (lhist) lhist_flush(lhist, nk, reinterpret_cast<unsigned long long *>(ws + P.off_hist) + w0 * P.xi_nbins);
}

// Persistent launch: workgroups take items from a queue (atomic ticket) until
// it is empty; items are ordered longest first by the host.
template <typename T, int G, int B>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(1, chain_max_waves<G, B>()))) void sim_chain_persistent(const DevProblem *__restrict__ probs,
                                                           const WorkItem *__restrict__ items, int n_items,
                                                           int *__restrict__ ticket, char *__restrict__ ws,
                                                           int lds_cap) {
    __shared__ double s_acc[chain_reps_per_wg(G) * A_NFIELDS];
    __shared__ int s_item;
    extern __shared__ unsigned int s_hist[];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(ticket, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= n_items) break;
        const WorkItem item = items[it];
        const DevProblem &P = probs[item.prob];
        const int nk = item_hist_bins(P, item);
        unsigned int *lhist = nk <= lds_cap ? s_hist : nullptr;
        if (lhist) lhist_clear(lhist, nk);
        run_chain_item<T, G, B>(P, item, ws, 0, INT64_MAX, nullptr, -1, s_acc, lhist);
        if (lhist) lhist_flush(lhist, nk, reinterpret_cast<unsigned long long *>(ws + P.off_hist) + (int64_t)item.window * P.xi_nbins);
    }
}

// Energies and forces of configurations (parity hook): one group per configuration.
template <typename T, int G, int B>
__global__ __launch_bounds__(WG) void chain_eval(const DevProblem *__restrict__ probs, const double *__restrict__ coords,
                                                 int n_rep, double centre, double *__restrict__ forces,
                                                 double *__restrict__ energy) {
    const DevProblem &P = probs[0];
    constexpr int GPW = groups_per_wave(G);
    const int lane = lane_id();
    const bool lane_used = lane < GPW * G;
    const int grp = (int)(threadIdx.x >> 6) * GPW + (lane_used ? lane / G : 0);
    const int g = lane_used ? lane % G : 0;
    const int gbase = lane_used ? lane - g : lane;
    const int c = blockIdx.x * chain_reps_per_wg(G) + grp;
    const bool active = lane_used && c < n_rep;
    const int cc = active ? c : 0;
    const int N = P.n_beads;
    const int i0 = g * B;
    T px[B], py[B], pz[B], fx[B], fy[B], fz[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int i = i0 + b;
        if (i < N) { px[b] = (T)coords[(int64_t)cc * 3 * N + 3 * i]; py[b] = (T)coords[(int64_t)cc * 3 * N + 3 * i + 1]; pz[b] = (T)coords[(int64_t)cc * 3 * N + 3 * i + 2]; }
        else { px[b] = 0; py[b] = 0; pz[b] = (T)(P.pad_z0 + P.pad_dz * (i - N)); }
    }
    double e[4];
    ChainForce<T, G, B, true>::compute(P, g, gbase, (T)centre, (T)P.k, px, py, pz, fx, fy, fz, e);
    // group sums of the energy parts (fixed order over lanes)
    double tot[4];
    for (int q = 0; q < 4; ++q) {
        double s = 0.0;
        for (int l = 0; l < G; ++l) s += pull_f(lane_used ? gbase + l : lane, e[q]);
        tot[q] = s;
    }
    if (!active) return;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int i = i0 + b;
        if (i < N) {
            forces[(int64_t)c * 3 * N + 3 * i] = (double)fx[b];
            forces[(int64_t)c * 3 * N + 3 * i + 1] = (double)fy[b];
            forces[(int64_t)c * 3 * N + 3 * i + 2] = (double)fz[b];
        }
    }
    if (g == 0) {
        energy[c * 5 + 0] = tot[0] + tot[1] + tot[2] + tot[3];
        for (int q = 0; q < 4; ++q) energy[c * 5 + 1 + q] = tot[q];
    }
}

template <typename T>
__global__ void pot1d_eval(const DevProblem *__restrict__ probs, const double *__restrict__ coords, int n_rep,
                           double centre, double *__restrict__ forces, double *__restrict__ energy) {
    const DevProblem &P = probs[0];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_rep) return;
    const T x = (T)coords[c];
    forces[c] = (double)force_1d<T>(P, x, (T)centre, (T)P.k);
    double ho;
    if (P.pot_kind == 0) { const double q = (double)x * (double)x - P.pot_b; ho = P.pot_a * q * q; }
    else ho = 0.5 * P.pot_kappa * (double)x * (double)x;
    const double res = 0.5 * P.k * ((double)x - centre) * ((double)x - centre);
    energy[c * 5 + 0] = ho + res; energy[c * 5 + 1] = ho; energy[c * 5 + 2] = 0; energy[c * 5 + 3] = 0; energy[c * 5 + 4] = res;
}

// Per-shape launchers; each shape is instantiated in its own translation unit.
template <typename T, int G, int B>
hipError_t launch_chain_direct(const DevProblem *d_probs, const WorkItem *d_items, int n_items, char *ws,
                               int64_t step_begin, int64_t step_end, double *traj, int64_t traj_rep, int lds_cap,
                               hipStream_t stream) {
    hipLaunchKernelGGL((sim_chain<T, G, B>), dim3(n_items), dim3(WG), (size_t)lds_cap * 4, stream, d_probs, d_items,
                       n_items, ws, step_begin, step_end, traj, traj_rep, lds_cap);
    return hipGetLastError();
}
template <typename T, int G, int B>
hipError_t launch_chain_persistent(const DevProblem *d_probs, const WorkItem *d_items, int n_items, int *d_ticket,
                                   char *ws, int n_groups, int lds_cap, hipStream_t stream) {
    hipLaunchKernelGGL((sim_chain_persistent<T, G, B>), dim3(n_groups), dim3(WG), (size_t)lds_cap * 4, stream, d_probs,
                       d_items, n_items, d_ticket, ws, lds_cap);
    return hipGetLastError();
}
template <typename T, int G, int B>
hipError_t launch_chain_eval(const DevProblem *d_probs, const double *coords, int n_rep, double centre,
                             double *forces, double *energy, hipStream_t stream) {
    const int per = chain_reps_per_wg(G);
    const int nb = (n_rep + per - 1) / per;
    hipLaunchKernelGGL((chain_eval<T, G, B>), dim3(nb), dim3(WG), 0, stream, d_probs, coords, n_rep, centre, forces,
                       energy);
    return hipGetLastError();
}
template <typename T, int G, int B>
int chain_blocks_per_cu(int lds_cap) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sim_chain_persistent<T, G, B>, WG, (size_t)lds_cap * 4) != hipSuccess) n = 1;
    return n;
}

#define PPP_INSTANTIATE_SHAPE(T, G, B)                                                                              \
    template hipError_t launch_chain_direct<T, G, B>(const DevProblem *, const WorkItem *, int, char *, int64_t,   \
                                                     int64_t, double *, int64_t, int, hipStream_t);                \
    template hipError_t launch_chain_persistent<T, G, B>(const DevProblem *, const WorkItem *, int, int *, char *, \
                                                         int, int, hipStream_t);                                   \
    template hipError_t launch_chain_eval<T, G, B>(const DevProblem *, const double *, int, double, double *,      \
                                                   double *, hipStream_t);                                         \
    template int chain_blocks_per_cu<T, G, B>(int);

}  // namespace ppp

// Internal layout shared by the HIP kernels and the host runtime of libppp.
// Nothing here is part of the C ABI (include/ppp.h).
#pragma once
#include <stdint.h>

namespace ppp {

// Per-replica accumulator record (fp64), also the per-(window, block) and
// per-window record after reduction.
enum AccField : int {
    A_N = 0,      // number of samples
    A_S1,         // sum (xi - lambda_i)
    A_S2,         // sum (xi - lambda_i)^2
    A_XMIN,       // smallest sample
    A_XMAX,       // largest sample
    A_MF, A_SF,   // running log-sum-exp of a = -beta dW_i (forward): max and scaled sum
    A_MF2, A_SF2, // same for 2a
    A_MR, A_SR,   // reverse perturbation lambda_i -> lambda_{i-1}
    A_MR2, A_SR2,
    // With the free ensemble (index s) the ends are perturbed toward it as well:
    // window 1's reverse and window s's forward entries hold a = +beta k/2 d^2
    // (Eq. 5); the free ensemble's forward and reverse entries hold
    // a = -beta k/2 (xi - lambda_1)^2 and -beta k/2 (xi - lambda_s)^2 (Eq. 6).
    A_UNDER, A_OVER,
    A_BLOWN,      // 1 if the replica was frozen
    A_NFIELDS
};

// Output arrays of one problem (each [s] doubles), in this order.
enum OutField : int {
    O_DF_JE = 0, O_DF_JE_SE, O_DF_FLUCT, O_DF_FLUCT_SE, O_DF_GAUSS, O_DF_GAUSS_SE,
    O_DF_COM, O_DF_COM_SE, O_DF_UNC, O_DF_REV,
    O_DF_JE_HIST, O_DF_JE_HIST_MID, O_VAR_PAPER, O_SIGMA_W, O_Q_BINS, O_WORK_LOST,
    O_XI_MEAN, O_XI_STD, O_GAMMA2, O_XI_MINS, O_XI_MAXS, O_LSE_FWD, O_LSE_REV,
    O_N_SAMPLES, O_N_BLOWN, O_UNDER, O_OVER,
    O_KISH, O_OVL, O_DL_SIGMA, O_DL_REACH, O_CRIT,
    O_DF_FLUCT_LIT, O_DF_GAUSS_LIT, O_DF_JE_HIST_LIT,
    O_G, O_G_SE,            // Eq. 15, with the free ensemble only
    O_DF_REV_HIST, O_CROOKS_OVL, O_DF_CROOKS,   // reverse-path work distribution checks
    O_SIGMA_LSQ, O_GAMMA2_LSQ, O_DF_GAUSS_LSQ,   // sigma_i by least-squares Gaussian fit, Eq. 13 with it
    O_NFIELDS
};

// App. C work-distribution chains: 0 the primary reading, 1 the listing as
// printed, 2 the reverse path (lambda_j back to lambda_1).
constexpr int kAppcChains = 3;

// Jackknife leave-one-out profiles stored per block: JE, fluct, gauss, com, G.
constexpr int JK_FIELDS = 5;
// Leave-one-out turn-on values per block: Eq. 5 and Eq. 6 at lambda_1 and
// lambda_s, and the Eq. 10 log-average.
constexpr int JK_TURN = 5;

struct DevProblem {
    // model
    int32_t model;          // 0: 1-D, 1: chain
    int32_t precision;      // 0: fp32 forces, 1: fp64
    int32_t pot_kind, integrator_1d;
    int32_t n_beads, n_pad, rc_mode;
    int32_t n_windows, n_replicas, n_blocks;
    int32_t xi_nbins, w_half_bins;
    int32_t sample_every;
    int32_t variant_lanes, variant_beads;   // chain kernel shape (G lanes x B beads per lane)
    int32_t sequential;     // 1: sequential pulling protocol (windows one after another per replica)
    int32_t free_ens;       // 1: the unrestrained ensemble runs as window index s (k = 0)
    int32_t n_sim_windows;  // s + free_ens: windows with replicas, records and histograms
    int64_t n_steps, n_equil, n_pull;
    uint64_t seed;
    double k, kT, beta, dt;
    double pot_a, pot_b, pot_kappa, mobility;
    double k_bond, r0, k_angle;
    double lj_A, lj_B;      // force: f = inv_r2^4 (A inv_r2^3 - B) with A = 48 eps sig^12, B = 24 eps sig^6
    double lj_eA, lj_eB;    // energy: inv_r2^3 (eA inv_r2^3 - eB) - ucut
    double lj_ucut, rc2;
    double mass, inv_mass, c1, c2sd, sd_v;   // BAOAB constants
    double xi_min, xi_bin, w_bin, xi_bound, xi_start;
    double fix_x, fix_y, fix_z;              // fixed bead 0
    double pad_z0, pad_dz;                   // where padding beads are parked
    // byte offsets of this problem's arrays inside the workspace
    // S = n_sim_windows; the free ensemble's lambda entry is lambda_1
    int64_t off_lambda;     // double [S]
    int64_t off_init;       // double [3 N] (chain) or [1]
    int64_t off_state;      // T [S R][6][n_pad] (chain) or T [S R][2] (1-D: x, eta)
    int64_t off_acc;        // double [S R][A_NFIELDS]
    int64_t off_hist;       // u64 [S][K]
    int64_t off_blk;        // double [S][B][A_NFIELDS]
    int64_t off_tot;        // double [S][A_NFIELDS]
    int64_t off_jack;       // double [B][JK_FIELDS][s]
    int64_t off_jack_turn;  // double [B][JK_TURN]
    int64_t off_out;        // double [O_NFIELDS][s]
    int64_t off_turn;       // double [PPP_ON_NFIELDS]
    // App. C, kAppcChains chains
    int64_t off_pairs_shift;// int32 [3][s][K] (chain 1: floor of the work in bins)
    int64_t off_pairs_ceil; // int32 [s][K] (chain 1: its ceiling)
    int64_t off_pairs_prob; // double [3][s][K]
    int64_t off_npairs;     // int32 [3][s]
    int64_t off_omega;      // double [3][s][2M+1]
};

// n_reps consecutive replicas of one problem, starting at replica rep_begin of
// window `window`.  Replicas are numbered gid = window * R + replica, so an item
// of a chain problem may run on into the following windows (the kernels take
// each replica's window from its own gid).
struct WorkItem {
    int32_t prob, window, rep_begin, n_reps;
};

constexpr int WG = 256;  // threads per workgroup of the simulation kernels

// Chain kernels give each replica G consecutive lanes of one wavefront; a
// wavefront holds 64 / G whole groups and its last 64 mod G lanes stay idle.
constexpr int groups_per_wave(int G) { return 64 / G; }
constexpr int chain_reps_per_wg(int G) { return (WG / 64) * groups_per_wave(G); }

}  // namespace ppp

/*
 * ppp.h -- C ABI of libppp, the MI355X (gfx950) implementation of the
 * parallel pulling protocol of V. A. Ngo, "A Parallel-pulling Protocol for
 * Free Energy Evaluation" (arXiv:1105.4840).
 *
 * The protocol (Sec. III(ii), Fig. 1b): s independent simulations, one per
 * window lambda_i, all started from the same state x_o, each relaxing under the
 * restraint k/2 (xi - lambda_i)^2 (Eq. 3) and recording the reaction
 * coordinate xi.  From the recorded xi the library computes:
 *   - the step-wise work dW_i(xi) = k/2[(xi - lambda_{i+1})^2 - (xi - lambda_i)^2]
 *     (the summand of Eq. 9) and the Jarzynski estimate of Eq. 12, which for
 *     independent windows factorises into per-window exponential averages;
 *   - the alternative estimate from window averages, Eq. 14, the Gaussian
 *     estimate Eq. 13, and the combined estimate (dF^JE + dF_fluct)/2 with
 *     uncertainty (dF^JE - dF_fluct)/2 (Sec. IV B, IV D);
 *   - the xi histograms rho_i and the work distributions Omega_j (App. C) with
 *     the JE variance formula of Sec. IV A;
 *   - adjacent-window overlap diagnostics (Sec. III, Sec. IV B, Sec. V).
 *
 * Conventions for every function:
 *   - returns ppp_status; never aborts, never prints;
 *   - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *     pointers are GPU memory owned by the caller (e.g. a torch tensor's
 *     data_ptr()); hip_stream is a hipStream_t (NULL = the null stream);
 *   - device work is enqueued asynchronously on hip_stream; ppp_get_result and
 *     ppp_checkpoint synchronise that stream;
 *   - the library allocates no device memory on the run path: every device
 *     byte it touches lies in the caller's workspace or buffers;
 *   - one handle must not be used from two threads at once; handles share no
 *     mutable state.
 */
#ifndef PPP_H
#define PPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PPP_OK = 0,
    PPP_E_INVALID_ARG = 1,   /* rejected before any device work */
    PPP_E_OUT_OF_MEMORY = 2, /* host allocation failed or workspace too small */
    PPP_E_DEVICE = 3,        /* a HIP call failed; ppp_last_error has the HIP message */
    PPP_E_NUMERICAL = 4,     /* more than 1% of the replicas of some window were frozen */
    PPP_E_STATE = 5,         /* call out of order (e.g. result before run) */
    PPP_E_UNSUPPORTED = 6    /* valid request this library does not implement */
} ppp_status;

typedef enum { PPP_MODEL_1D = 0, PPP_MODEL_CHAIN = 1 } ppp_model;
/* PPP_FP32_FORCES: forces, noise and integration in fp32; the step-wise work,
 * its log-sum-exp, the moments and every estimator in fp64.
 * PPP_FP64: everything in fp64 (for parity with an fp64 reference). */
typedef enum { PPP_FP32_FORCES = 0, PPP_FP64 = 1 } ppp_precision;
/* overdamped 1-D schemes: Leimkuhler-Matthews (default) or Euler-Maruyama */
typedef enum { PPP_INT_LM = 0, PPP_INT_EM = 1 } ppp_integrator_1d;

/* H_o of the 1-D model: kind 0: a (x^2 - b)^2; kind 1: kappa/2 x^2.
 * Overdamped dynamics with the given mobility (diffusion mobility * kT). */
typedef struct {
    int32_t kind;
    double a, b, kappa;
    double mobility;
} ppp_pot1d;

/* H_o of the bead-spring chain (stand-in for the pulled molecule of Sec. IV):
 * bonds k_bond/2 (|r_{i+1} - r_i| - r0)^2; angles k_angle (1 - cos phi) with phi
 * the angle between successive bond vectors; Lennard-Jones
 * 4 eps [(sigma/r)^12 - (sigma/r)^6] shifted to 0 at lj_rc * sigma, pairs |i-j| > 2.
 * Bead 0 is held fixed (Sec. IV A: one end fixed).  xi = |r_{N-1} - r_0|
 * (rc_mode 0) or z_{N-1} - z_0 (rc_mode 1).  BAOAB Langevin with friction gamma. */
typedef struct {
    int32_t n_beads;         /* 2 .. PPP_MAX_BEADS */
    double k_bond, r0, k_angle;
    double lj_eps, lj_sigma, lj_rc;
    int32_t rc_mode;
    double mass, gamma;
} ppp_chain;

#define PPP_MAX_BEADS 256

typedef struct {
    ppp_model model;
    ppp_pot1d pot1d;             /* used when model == PPP_MODEL_1D */
    ppp_chain chain;             /* used when model == PPP_MODEL_CHAIN */
    int32_t n_windows;           /* s >= 2 */
    const double *lambda;        /* host [n_windows], strictly monotone; copied at create */
    double k, kT, dt;            /* restraint stiffness, temperature, time step (all > 0) */
    int64_t n_steps;             /* relaxation steps per replica (tau_i / dt) */
    int64_t n_equil;             /* steps before the first sample, 0 <= n_equil < n_steps */
    int64_t n_pull;              /* 0: restraint switched on at lambda_i (Eq. 3); > 0: centre
                                    moves linearly from xi(x_o) to lambda_i over n_pull steps */
    int32_t sample_every;        /* record xi every sample_every steps after n_equil (>= 1) */
    int32_t n_replicas;          /* independent replicas per window (>= 1) */
    uint64_t seed;               /* Philox4x32-10 key */
    ppp_precision precision;
    ppp_integrator_1d integrator_1d;
    const double *init_coords;   /* host, optional: 1-D [1] or chain [3 n_beads]; NULL: x_o =
                                    lambda_1 (1-D) or an ideal helix (chain); copied at create */
    double xi_min, xi_bin;       /* histogram of xi: bin b = floor((xi - xi_min)/xi_bin) */
    int32_t xi_nbins;            /* K in [1, 2^26] */
    double w_bin;                /* work-distribution bin width dW > 0 */
    int32_t w_half_bins;         /* M in [0, 5e7]: 2M+1 work bins; 0 disables App. C */
    int32_t n_jack_blocks;       /* jackknife blocks B in [0, 4096] (0: 32); above n_replicas: n_replicas */
    double xi_bound;             /* |xi| above this freezes a replica (<= 0: 1e4) */
    uint32_t flags;              /* 0, or PPP_FLAG_SEQUENTIAL or PPP_FLAG_FREE_ENSEMBLE */
} ppp_problem;

/* Sequential pulling protocol (Sec. III(i), Fig. 1b) instead of the parallel
 * one: each of the n_replicas replicas starts from x_o in window 1, relaxes
 * n_steps there, and continues from its last state in window 2, and so on to
 * window s (s * n_steps steps per replica, the same replica-steps as the
 * parallel protocol).  n_equil and sample_every apply inside every window; a
 * linear pull (n_pull) applies to window 1 only.  The per-window records and
 * every estimator are those of the parallel protocol.  A replica frozen in one
 * window stays frozen in the later ones.  Noise: replica r uses the counters
 * of replica r of window 1 in the parallel protocol, with the step counted
 * from the start of window 1, so window 1 gives the same samples in both
 * protocols.  Not available for batched or adaptive runs, nor for
 * ppp_trajectory. */
#define PPP_FLAG_SEQUENTIAL 1u

/* Turn-on free energy (Sec. II, Eqs. 4-7 and 10; App. A; the state function
 * G of Eq. 15).  Besides the s restrained windows the run simulates the
 * unrestrained system H_o (k = 0): n_replicas more replicas from the same
 * start state with the same step schedule, numbered after those of window s
 * (replica r has noise counters of replica number s R + r).  Their samples
 * x_0 and those of windows 1 and s give ppp_result.turn_on:
 *   DF(lambda_1, k) = F(lambda_1, k) - F_0 by Eq. 5 (an average over window
 *   1 of exp(+beta k/2 (x_1 - lambda_1)^2)) and by Eq. 6 (an average over x_0
 *   of exp(-beta k/2 (x_0 - lambda_1)^2)), each with its jackknife error, and
 *   the two bounds of Eq. 7; the same at lambda_s from window s and x_0;
 *   ln <exp(-beta W_total)> of Eq. 10 with the average factorised over the
 *   independent ensembles x_0, x_1 .. x_s (0 in expectation);
 *   the free ensemble's sample count, frozen replicas, mean and spread of xi;
 * and ppp_result.G[j] = dF_je[j] - DF(lambda_1, k) with DF by Eq. 5, the state
 * function of Eq. 15.  The per-window profiles do not change.  Not available
 * with PPP_FLAG_SEQUENTIAL or for adaptive runs (PPP_E_UNSUPPORTED);
 * ppp_trajectory serves the restrained windows only. */
#define PPP_FLAG_FREE_ENSEMBLE 2u

/* Entries of ppp_result.turn_on ("first": lambda_1, "last": lambda_s). */
enum {
    PPP_ON_EQ5_FIRST = 0, PPP_ON_EQ5_FIRST_SE, PPP_ON_EQ6_FIRST, PPP_ON_EQ6_FIRST_SE,
    PPP_ON_LOWER_FIRST, PPP_ON_UPPER_FIRST,          /* Eq. 7: <k/2 (x_1 - l)^2>_l and <k/2 (x_0 - l)^2>_0 */
    PPP_ON_EQ5_LAST, PPP_ON_EQ5_LAST_SE, PPP_ON_EQ6_LAST, PPP_ON_EQ6_LAST_SE,
    PPP_ON_LOWER_LAST, PPP_ON_UPPER_LAST,
    PPP_ON_EQ10_LOG, PPP_ON_EQ10_LOG_SE,
    PPP_ON_FREE_N, PPP_ON_FREE_BLOWN, PPP_ON_FREE_MEAN, PPP_ON_FREE_STD, PPP_ON_FREE_UNDER, PPP_ON_FREE_OVER,
    PPP_ON_NFIELDS
};

/* Caller-owned host output buffers; any pointer may be NULL (not wanted).
 * s = n_windows, K = xi_nbins, M = w_half_bins.  Profiles are relative to
 * lambda_1 (entry 0 is 0), the reference point of Sec. IV A. */
typedef struct {
    /* [s] free-energy profiles and their jackknife standard errors */
    double *dF_je, *dF_je_se;          /* Eq. 12 from per-window exponential averages */
    double *dF_fluct, *dF_fluct_se;    /* Eq. 14 with dlambda_i = lambda_{i+1} - lambda_i */
    double *dF_gauss, *dF_gauss_se;    /* Eq. 13 with the same increments */
    double *dF_com, *dF_com_se;        /* (dF_je + dF_fluct)/2 */
    double *dF_unc;                    /* (dF_je - dF_fluct)/2 */
    double *dF_rev;                    /* JE from the reverse perturbation lambda_{i+1} -> lambda_i */
    /* [s] work-distribution (App. C) results */
    double *dF_je_hist;                /* Eq. 12 from Omega_j, work at the left bin edge w dW */
    double *dF_je_hist_mid;            /* same, work at w dW + (j-1) dW/2 */
    double *dF_je_var_paper;           /* sigma_W^2/Q + beta^2 sigma_W^4/(2(Q-1)) */
    double *sigma_w;                   /* standard deviation of Omega_j */
    int64_t *q_bins;                   /* non-zero bins of Omega_j */
    double *work_lost;                 /* probability mass of Omega_j outside the 2M+1 bins */
    /* [s] window statistics */
    double *xi_mean, *xi_std, *gamma2; /* <x_i>, sigma_i, gamma_i^2 = k sigma_i^2 / kT */
    double *xi_min_sample, *xi_max_sample;
    double *lse_fwd, *lse_rev;         /* ln sum exp(-beta dW) forward / reverse */
    int64_t *n_samples, *n_blown_up;
    /* [s-1] adjacent-pair diagnostics */
    double *kish_frac;                 /* effective-sample fraction of exp(-beta dW_i) */
    double *overlap_ovl;               /* sum_b min(rho_i(b), rho_{i+1}(b)) */
    double *dlambda_over_sigma;        /* |dlambda_i| / sigma_i */
    double *dlambda_over_reach;        /* |dlambda_i| / (end of rho_i in the pulling direction - <x_i>) */
    int32_t *criterion_ok;             /* |dlambda_i| <= that reach (Sec. IV B) */
    /* [s] the paper's formulas as printed, beside the readings above */
    double *dF_fluct_literal;          /* Eq. 14 with (lambda_j - lambda_1)/j in place of every
                                          increment up to lambda_j (j counted from 1) */
    double *dF_gauss_literal;          /* Eq. 13 likewise */
    double *dF_je_hist_literal;        /* App. C as printed: x at the bin's upper edge, work bin
                                          [W/dW] by truncation toward zero, Omega_j(0) replaced by
                                          the mean of its neighbours (j >= 2) */
    /* histograms */
    uint64_t *xi_hist;                 /* [s*K] */
    uint64_t *xi_under_over;           /* [s*2] */
    double *work_hist;                 /* [s*(2M+1)], Omega_j, bin w at index w + M */
    /* with PPP_FLAG_FREE_ENSEMBLE (else filled with NaN, and zero counts) */
    double *turn_on;                   /* [PPP_ON_NFIELDS] */
    double *G, *G_se;                  /* [s] Eq. 15 */
    uint64_t *xi_hist_free;            /* [K] histogram of x_0 */
    /* [s] the reverse path lambda_j -> lambda_1 by App. C from rho_2 .. rho_j with
     * the work of moving the centre back, dW^rev_i(x) = k/2 [(x - lambda_i)^2 -
     * (x - lambda_{i+1})^2] (x at the bin centre, floor to bins), checked against the
     * forward distribution (Crooks fluctuation theorem; Kofke's overlap, Sec. V):
     * a forward bin w, work in [w, w + j-1) dW after j-1 steps, meets reverse bin
     * -w - (j-1).  NaN without App. C (M = 0). */
    double *dF_rev_hist;               /* +kT ln sum_v Omega^rev_j(v) exp(-beta v dW) */
    double *crooks_ovl;                /* sum_w min(Omega_j(w), Omega^rev_j(-w - (j-1))) */
    double *dF_crooks;                 /* over the bins both hold, weighted by that minimum:
                                          W_w - kT ln(Omega_j(w) / Omega^rev_j(-w - (j-1))),
                                          W_w = (w + (j-1)/2) dW */
    double *work_hist_rev;             /* [s*(2M+1)], Omega^rev_j, bin v at index v + M */
    /* [s] sigma_i as the paper obtains it (Sec. IV A: least-squares fitting of the
     * x_i distribution): the Gaussian A exp(-(x - mu)^2 / (2 sigma^2)) closest in
     * least squares to the histogram density count_b / (n xi_bin) at the bin
     * centres (Levenberg-Marquardt from the sample moments; NaN for windows with
     * fewer than 3 samples or fewer than 3 non-empty bins); gamma_i^2 =
     * k sigma_i^2 / kT from it; and Eq. 13 with that gamma_i^2 and the sample
     * means */
    double *sigma_lsq, *gamma2_lsq, *dF_gauss_lsq;
} ppp_result;

typedef struct {
    double sim_ms;       /* simulation kernel(s) of the last run, HIP-event time */
    double reduce_ms;    /* replica -> block -> window reductions and estimators */
    double appc_ms;      /* App. C work distributions */
    double total_ms;     /* whole last ppp_run, first to last event */
    int64_t replica_steps;
    int32_t sim_launches;
    int32_t variant_lanes, variant_beads_per_lane;  /* kernel shape chosen for the chain */
    double last_advance_ms;  /* simulation kernel(s) of the latest ppp_advance (or of the whole
                                relaxation in ppp_run), HIP-event time; NaN for batched handles */
} ppp_timings;

typedef struct ppp_handle ppp_handle;

/* The parallel pulling protocol of Sec. III(ii) and Fig. 1b: s independent
 * relaxations, one per window lambda_i, from the shared start state x_o, each
 * under the restraint of Eq. 3, recording xi for the estimators of Eqs. 9 and
 * 12-14 and the work distributions of App. C (the run settings and records of
 * Sec. IV A).
 *
 * Validates and copies the problem, chooses the kernel shape (from the table
 * file named by the environment variable PPP_TUNE_TABLE if set, see
 * ppp_autotune, else a built-in heuristic) and the workspace layout.  PPP_E_INVALID_ARG for: s < 2, lambda not strictly
 * monotone or non-finite, k, kT, dt <= 0, n_replicas < 1, sample_every < 1,
 * n_equil < 0 or >= n_steps, K < 1, xi_bin <= 0, w_bin <= 0 with M > 0,
 * chain with n_beads < 2 or > PPP_MAX_BEADS, non-positive mass or bond
 * length, unknown flags, or a sequential run of more than 2^32 - 1 steps per
 * replica; PPP_E_UNSUPPORTED for PPP_FLAG_SEQUENTIAL with
 * PPP_FLAG_FREE_ENSEMBLE.  *out is NULL on failure. */
ppp_status ppp_create(const ppp_problem *p, ppp_handle **out);

/* Batched form (uneven chains, windows, replicas, steps): all problems run in
 * one persistent, HIP-graph-captured launch.  The paper runs one protocol at a
 * time; batching several is this library's extension, sound because every
 * window of every problem is an independent relaxation (Sec. III(ii)), so each
 * problem gives what its own ppp_run gives, bit for bit.  tune_table_path (optional, may
 * be NULL) is a text file written by ppp_autotune; without it a built-in
 * shape heuristic is used.  Results are read per problem with
 * ppp_batch_get_result. */
ppp_status ppp_batch_create(const ppp_problem *ps, int32_t n, const char *tune_table_path,
                            ppp_handle **out);

/* Device bytes the caller must supply to ppp_run (256-byte aligned). */
ppp_status ppp_workspace_size(const ppp_handle *h, size_t *bytes);

/* Enqueues the whole protocol of Sec. III(ii) (Fig. 1b) on hip_stream: the
 * shared initial state x_o, all relaxation steps of every window, the
 * reductions, the estimators of Eqs. 12-14 and the work distributions of
 * App. C.  d_workspace must
 * stay valid until ppp_get_result returns.  PPP_E_OUT_OF_MEMORY if bytes is
 * below ppp_workspace_size. */
ppp_status ppp_run(ppp_handle *h, void *d_workspace, size_t bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ppp_run with
 * the workspace taken from a device array the library holds, one per GPU, for
 * the life of the process (PPP_STATIC_WORKSPACE_BYTES; each GPU the library runs
 * on keeps it until the process ends), instead of a caller buffer.  The caller
 * passes the handle and a stream; results come back through ppp_get_result as
 * after ppp_run.  Makes no device or host allocation: no hipMalloc or hipFree,
 * and no timing events (ppp_get_timings then reports NaN times unless an earlier
 * ppp_run on the handle created them).  Every call on one GPU shares that GPU's
 * array and leaves its contents there (the run clears what it accumulates into
 * before it starts), so calls that overlap on one GPU -- two handles, or two
 * streams, before the first one's ppp_get_result -- race and give wrong results.
 * Single-problem handles only (PPP_E_UNSUPPORTED for batched ones);
 * PPP_E_OUT_OF_MEMORY, before any device work and with the sizes in
 * ppp_last_error, for a problem whose ppp_workspace_size exceeds
 * PPP_STATIC_WORKSPACE_BYTES. */
#define PPP_STATIC_WORKSPACE_BYTES (64u << 20)
ppp_status ppp_run_static(ppp_handle *h, void *hip_stream);

/* Incremental form of ppp_run (same protocol, Sec. III(ii)): begin (initial
 * state), advance by n steps (clamped to the steps left), finalize (reductions,
 * estimators and App. C on what has been sampled so far; an advance may follow
 * and a later finalize includes it).  */
ppp_status ppp_begin(ppp_handle *h, void *d_workspace, size_t bytes, void *hip_stream);
ppp_status ppp_advance(ppp_handle *h, int64_t n_steps, void *hip_stream);
ppp_status ppp_finalize(ppp_handle *h, void *hip_stream);
ppp_status ppp_steps_done(const ppp_handle *h, int64_t *steps);

/* Results of the run (ppp_result above): the profiles of Eq. 12 (JE over the
 * step-wise work, factorised over independent windows), Eq. 14 and Eq. 13, the
 * combined estimate and uncertainty of Sec. IV B and IV D, the window
 * statistics and histograms of Sec. IV A, the work distributions and variance
 * formula of App. C, and the overlap diagnostics of Sec. IV B.
 * Synchronises the stream of the last run and copies the outputs into the
 * caller's host buffers.  Returns PPP_E_NUMERICAL (buffers still filled) when
 * more than 1% of some window's replicas were frozen. */
ppp_status ppp_get_result(ppp_handle *h, ppp_result *out);
ppp_status ppp_batch_get_result(ppp_handle *h, int32_t index, ppp_result *out);
ppp_status ppp_get_timings(const ppp_handle *h, ppp_timings *out);

/* Replica state, accumulators and step counter after the last begin/advance.
 * host_buf == NULL: *bytes receives the size.  ppp_restore puts a checkpoint
 * of an identical problem back into d_workspace; advancing from it gives the
 * same results as an uninterrupted run (the noise is a function of the step).
 * Layout: 8 bytes of magic, the steps done (int64), then per problem its
 * replica states first: for replica gid = window * n_replicas + replica, a
 * chain holds 6 * n_pad values of the working precision (fp32 or fp64): x of
 * the n_pad bead slots, then y, z, v_x, v_y, v_z, with n_pad = lanes x beads
 * per lane of the kernel shape (ppp_timings.variant_*; slots from n_beads on
 * are padding); a 1-D replica holds x and the normal deviate of the last
 * step (the Leimkuhler-Matthews scheme uses it again).  Accumulators and histograms
 * follow, in the library's own layout. */
ppp_status ppp_checkpoint(ppp_handle *h, void *host_buf, size_t *bytes);
ppp_status ppp_restore(ppp_handle *h, void *d_workspace, size_t ws_bytes, const void *host_buf,
                       size_t bytes, void *hip_stream);

ppp_status ppp_destroy(ppp_handle *h);
const char *ppp_status_string(ppp_status s);
/* Message of the last failed ppp_create / ppp_batch_create on this thread. */
const char *ppp_create_error(void);
const char *ppp_last_error(const ppp_handle *h); /* NULL-safe; "" when no error */

/* ---- parity hooks (same kernels as the run path) ------------------------ */

/* Energy and forces of n_rep configurations of h's system at restraint
 * centre lambda, computed by the simulation kernel's force routine in the
 * problem's precision.  Uses (and clobbers) d_workspace of h (a later ppp_run
 * starts afresh).  d_coords: device fp64 [n_rep][dof]; d_forces: device fp64
 * [n_rep][dof]; d_energy: device fp64 [n_rep][5] = {total, bond, angle, lj,
 * restraint} (1-D: {total, H_o, 0, 0, restraint}); dof = 3 n_beads or 1.
 * Bead 0 is held fixed, so its force omits the restraint's reaction. */
ppp_status ppp_eval_forces(ppp_handle *h, void *d_workspace, size_t bytes, const double *d_coords,
                           int32_t n_rep, double lambda, double *d_forces, double *d_energy,
                           void *hip_stream);

/* Coordinates of replica `replica` of window `window` of h after each of the
 * first n_steps (1 <= n_steps <= min(100000, problem n_steps)) steps, step 0
 * being the start state, recorded by the simulation kernel itself (it runs the
 * workgroup holding that replica).  Uses and clobbers d_workspace of h.
 * d_out: device fp64 [n_steps+1][dof]. */
ppp_status ppp_trajectory(ppp_handle *h, void *d_workspace, size_t bytes, int32_t window,
                          int32_t replica, int32_t n_steps, double *d_out, void *hip_stream);

/* Raw Philox4x32-10 blocks and the kernels' normal deviates: for i < n,
 * counter (c0 + i, c1, c2, c3) under key seed.  d_words: device u32 [n][4];
 * d_normals, d_normals32: device fp64 / fp32 [n][4], the four Box-Muller
 * normals of a block (the 1-D model's noise: 32-bit uniforms in fp64, 23-bit
 * in fp32); d_normals6, d_normals6_32: device fp64 / fp32 [n][6], the six
 * normals of a block from 21-bit uniforms (the chain's noise, beads 2m and
 * 2m + 1 of replica gid at step n sharing counter (gid, n, m, 0)).  Every
 * output but d_words may be NULL.  Errors: PPP_E_INVALID_ARG for n < 0,
 * PPP_E_DEVICE if the launch fails. */
ppp_status ppp_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int32_t n,
                      uint32_t *d_words, double *d_normals, float *d_normals32, double *d_normals6,
                      float *d_normals6_32, void *hip_stream);

/* ---- learned window placement ------------------------------------------ */

/* Surrogate F(lambda): 1 -> 64 -> 64 -> 1 tanh MLP with bf16 weights and
 * activations and fp32 accumulation on the matrix cores.  Parameters are one
 * fp32 master vector of PPP_MLP_PARAMS floats laid out as
 * W1[64], b1[64], W2[64][64] (row = output), b2[64], W3[64], b3[1];
 * inputs are scaled as t = (lambda - shift) / scale by the caller. */
#define PPP_MLP_HIDDEN 64
#define PPP_MLP_PARAMS (64 + 64 + 64 * 64 + 64 + 64 + 1)

/* Forward: y[i] = F(t[i]) and dy[i] = dF/dt at t[i].  Device fp32 arrays. */
ppp_status ppp_mlp_forward(const float *d_params, const float *d_t, int32_t n, float *d_y,
                           float *d_dy, void *hip_stream);

/* Gradient of L = sum_i wv[i] (y_i - yv[i])^2 + ws[i] (dy_i - ys[i])^2 over the
 * batch with respect to the parameters (value and slope targets; a weight of
 * 0 drops a term).  d_grad: device fp32 [PPP_MLP_PARAMS] (overwritten);
 * d_loss: device fp32 [1] (may be NULL).  n <= 4096. */
ppp_status ppp_mlp_grad(const float *d_params, const float *d_t, const float *d_yv, const float *d_wv,
                        const float *d_ys, const float *d_ws, int32_t n, float *d_grad, float *d_loss,
                        void *hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the fp32 master
 * parameters; d_m, d_v: device fp32 [PPP_MLP_PARAMS] moments; step >= 1. */
ppp_status ppp_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, float lr,
                        int32_t step, void *hip_stream);

/* Adaptive protocol with learned window placement.  Exploration rounds run
 * short protocols (explore_replicas replicas, explore_steps steps) on new
 * windows; the surrogate is trained on the GPU on every explored window's
 * slope F'(lambda_i) = k (lambda_i - <x_i>) (Eq. 14 read as thermodynamic
 * integration, Sec. V) and on the JE increments of Eq. 12 between adjacent
 * explored windows (weighted by their Kish effective-sample fraction); its
 * curvature gives sigma(lambda)^2 = (k - F''(lambda)) / (beta k^2), the width
 * of the xi distribution at lambda, and windows are placed so that
 * |dlambda| / sigma(lambda) = target_dl_over_sigma, the adjacent-overlap
 * criterion of Sec. IV B and Sec. V.  Windows the surrogate predicts but no
 * round has explored are explored next.  Then one production run of the
 * protocol on the placed windows uses the rest of the budget: base's
 * n_replicas and steps = remaining budget / (windows x replicas), unless that
 * is below min_production_steps, in which case the replicas per window are
 * reduced (not below 16) so every window relaxes at least that long (the
 * relaxation time decides the accuracy, Sec. IV D).  The answer is that run's
 * plain profiles; uniform windows are the fallback when the surrogate fails
 * to train.  Exploration uses at most half of the budget.  */
typedef struct {
    int64_t budget_replica_steps;   /* exploration + production */
    int32_t initial_windows;        /* round-0 uniform windows (>= 2) */
    int32_t max_rounds, max_windows;
    double target_dl_over_sigma;    /* wanted |dlambda_i| / sigma between neighbours (> 0) */
    int32_t train_iters;            /* Adam steps per round */
    double lr;
    uint64_t init_seed;             /* surrogate initialisation */
    int32_t explore_replicas;       /* replicas per exploration window (0: n_replicas / 8) */
    int64_t explore_steps;          /* steps per exploration window (0: n_steps / 4) */
    int64_t min_production_steps;   /* relaxation steps every production window gets (see above);
                                       PPP_E_INVALID_ARG if the budget cannot afford them */
    int32_t placement;              /* where sigma(lambda) comes from: PPP_PLACE_LEARNED (the
                                       surrogate's curvature, above) or PPP_PLACE_EXPLORED (no
                                       network: the sample sigma_i of the explored windows,
                                       interpolated linearly in lambda; same rounds, placement
                                       rule and budget, to isolate what the surrogate adds) */
} ppp_adaptive;

#define PPP_PLACE_LEARNED 0
#define PPP_PLACE_EXPLORED 1

/* base describes the system, the lambda range [lambda[0], lambda[n_windows-1]],
 * replicas and the other run settings; lambda_out (host, capacity
 * max_windows) and *n_windows_out receive the production windows, out the
 * production run's results (buffers sized for max_windows), and
 * *replica_steps_used the total spent.  d_workspace: at least
 * ppp_adaptive_workspace_size bytes. */
ppp_status ppp_adaptive_workspace_size(const ppp_problem *base, const ppp_adaptive *a, size_t *bytes);
ppp_status ppp_adaptive_run(const ppp_problem *base, const ppp_adaptive *a, void *d_workspace,
                            size_t bytes, void *hip_stream, double *lambda_out,
                            int32_t *n_windows_out, int64_t *replica_steps_used, ppp_result *out);

/* Times every candidate kernel shape on representative chain lengths and
 * writes the fastest per length bucket to path (text).  Runs on hip_stream
 * inside d_workspace (>= 256 MiB). */
ppp_status ppp_autotune(const char *path, void *d_workspace, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PPP_H */

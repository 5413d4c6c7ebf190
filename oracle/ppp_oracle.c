/*
 * ppp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, double-precision CPU reference for the parallel pulling
 * protocol (PPP) of V. A. Ngo, "A Parallel-pulling Protocol for Free Energy
 * Evaluation" (arXiv:1105.4840).  It produces, for every window lambda_i and
 * every replica, the stream of sampled reaction-coordinate values xi that the
 * protocol collects (Sec. III(ii): s independent simulations, each started
 * from the same state x_o with the restraint centre fixed at lambda_i; the
 * estimators of Eqs. 12-14 and the work distributions of App. C are computed
 * from these streams by oracle/estimators.py and oracle/appc.py).
 *
 * Only tests/, the package's smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header or constant
 * table with the GPU library; nothing here is ever called on the product path.
 *
 * Everything is fp64 and written for readability: one replica at a time, all
 * pairs by a double loop, no blocking or fusion.  OpenMP only distributes
 * independent replicas over host threads (each replica is a serial loop, so
 * the result does not depend on the thread count).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Problem description (the oracle's own layout; independent of include/).   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t model;          /* 0: one particle in 1-D, 1: bead-spring chain in 3-D */
    /* 1-D potential H_o(x) */
    int32_t pot_kind;       /* 0: a (x^2 - b)^2, 1: kappa/2 x^2 */
    double pot_a, pot_b, pot_kappa;
    double mobility;        /* overdamped mobility (diffusion D = mobility * kT) */
    int32_t integrator_1d;  /* 0: Leimkuhler-Matthews, 1: Euler-Maruyama */
    /* chain H_o */
    int32_t n_beads;
    double k_bond, r0, k_angle, lj_eps, lj_sigma, lj_rc;
    int32_t rc_mode;        /* 0: xi = |r_{N-1} - r_0|, 1: xi = z_{N-1} - z_0 */
    double mass, gamma;
    /* protocol */
    int32_t n_windows;
    const double *lambda;   /* [n_windows] restraint centres */
    double k, kT, dt;
    int64_t n_steps, n_equil;
    int32_t sample_every;
    int32_t n_replicas;     /* per window */
    uint64_t seed;
    const double *init_coords; /* chain: [3 N]; 1-D: [1]; NULL: default x_o */
    double xi_bound;        /* |xi| above this (or non-finite state) freezes a replica */
    int64_t n_pull;         /* steps over which the centre moves from xi(x_o) to lambda_i (0: switched on at once) */
    int32_t sequential;     /* 1: sequential pulling protocol (Sec. III(i)) instead of the parallel one */
    int32_t free_ensemble;  /* 1: also sample the unrestrained system H_o (Sec. II, Eq. 6) as an extra
                               window numbered n_windows, restraint k = 0 */
} oracle_problem;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of the 4x32 Philox S-box with the    */
/* published multipliers and Weyl key increments.                            */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t key_in[2], const uint32_t ctr_in[4], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t k0 = key_in[0], k1 = key_in[1];
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Uniform on the open interval (0,1): (r + 1/2) 2^-32, exact in fp64. */
static double u32_to_open_unit(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

/* Four standard normals from one Philox block by the Box-Muller transform:
 * (z0, z1) from (u0, u1) and (z2, z3) from (u2, u3), each pair being
 * sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b). */
void oracle_normals4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, double z[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t r[4];
    oracle_philox4x32_10(key, ctr, r);
    const double two_pi = 6.283185307179586476925286766559;
    for (int p = 0; p < 2; ++p) {
        double ua = u32_to_open_unit(r[2 * p]);
        double ub = u32_to_open_unit(r[2 * p + 1]);
        double rad = sqrt(-2.0 * log(ua));
        z[2 * p] = rad * cos(two_pi * ub);
        z[2 * p + 1] = rad * sin(two_pi * ub);
    }
}

/* Six standard normals from one Philox block.  The 128 bits give six 21-bit
 * integers: a_k = r_k >> 11 (k = 0..3), a_4 = (r_0 mod 2^11) 2^10 + (r_1 mod
 * 2^10), a_5 = (r_2 mod 2^11) 2^10 + (r_3 mod 2^10); u_k = (a_k + 1/2) 2^-21,
 * exact in fp64 and in fp32.  (z_{2p}, z_{2p+1}) = sqrt(-2 ln u_{2p})
 * (cos 2 pi u_{2p+1}, sin 2 pi u_{2p+1}) for p = 0, 1, 2.  The smallest u is
 * 2^-22, so |z| <= sqrt(44 ln 2) = 5.52; a normal lies beyond that with
 * probability 3.4e-8. */
void oracle_normals6(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, double z[6])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t r[4];
    oracle_philox4x32_10(key, ctr, r);
    const uint32_t a[6] = {r[0] >> 11, r[1] >> 11, r[2] >> 11, r[3] >> 11,
                           ((r[0] & 0x7ffu) << 10) | (r[1] & 0x3ffu), ((r[2] & 0x7ffu) << 10) | (r[3] & 0x3ffu)};
    const double two_pi = 6.283185307179586476925286766559;
    for (int p = 0; p < 3; ++p) {
        double ua = ((double)a[2 * p] + 0.5) * (1.0 / 2097152.0);
        double ub = ((double)a[2 * p + 1] + 0.5) * (1.0 / 2097152.0);
        double rad = sqrt(-2.0 * log(ua));
        z[2 * p] = rad * cos(two_pi * ub);
        z[2 * p + 1] = rad * sin(two_pi * ub);
    }
}

/* The three normals of chain bead i of replica gid at step n (n = 0: the
 * initial velocities): beads 2m and 2m + 1 share the block with counter
 * (gid, n, m, 0), the even bead taking z_0..z_2 and the odd one z_3..z_5. */
static void bead_normals(uint64_t seed, uint32_t gid, uint32_t n, int i, double z[3])
{
    double z6[6];
    oracle_normals6(seed, gid, n, (uint32_t)(i >> 1), 0u, z6);
    for (int c = 0; c < 3; ++c) z[c] = z6[3 * (i & 1) + c];
}

/* The normal deviate eta_n of the 1-D model for replica gid at step n:
 * component n mod 4 of the block with counter (gid, n div 4, 0, 0). */
static double eta_1d(uint64_t seed, uint32_t gid, int64_t n)
{
    double z[4];
    oracle_normals4(seed, gid, (uint32_t)(n / 4), 0u, 0u, z);
    return z[n % 4];
}

/* ------------------------------------------------------------------------ */
/* Potentials.  Energies and forces F = -dU/dr written out term by term.     */
/* ------------------------------------------------------------------------ */
static double pot1d_energy(const oracle_problem *p, double x)
{
    if (p->pot_kind == 0) { double q = x * x - p->pot_b; return p->pot_a * q * q; }
    return 0.5 * p->pot_kappa * x * x;
}
static double pot1d_force(const oracle_problem *p, double x)
{
    if (p->pot_kind == 0) return -4.0 * p->pot_a * x * (x * x - p->pot_b);
    return -p->pot_kappa * x;
}

/* Reaction coordinate of the chain (end-to-end distance or z-projection of
 * the pulled end relative to the fixed end). */
static double chain_xi(const oracle_problem *p, const double *r)
{
    int last = p->n_beads - 1;
    double dx = r[3 * last] - r[0], dy = r[3 * last + 1] - r[1], dz = r[3 * last + 2] - r[2];
    if (p->rc_mode == 1) return dz;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Chain energy and forces with the restraint k/2 (xi - lam)^2.
 * e_parts (may be NULL) receives {bond, angle, lj, restraint}. */
double oracle_chain_forces(const oracle_problem *p, const double *r, double lam, double *f, double *e_parts)
{
    const int N = p->n_beads;
    double e_bond = 0, e_angle = 0, e_lj = 0, e_res = 0;
    for (int i = 0; i < 3 * N; ++i) f[i] = 0.0;

    /* harmonic bonds k_b/2 (|b| - r0)^2, b = r_{i+1} - r_i */
    for (int i = 0; i + 1 < N; ++i) {
        double b[3], d = 0;
        for (int c = 0; c < 3; ++c) { b[c] = r[3 * (i + 1) + c] - r[3 * i + c]; d += b[c] * b[c]; }
        d = sqrt(d);
        e_bond += 0.5 * p->k_bond * (d - p->r0) * (d - p->r0);
        double g = p->k_bond * (d - p->r0) / d;   /* dU/db = g b */
        for (int c = 0; c < 3; ++c) { f[3 * i + c] += g * b[c]; f[3 * (i + 1) + c] -= g * b[c]; }
    }
    /* cosine angle k_theta (1 - cos phi), phi between successive bond vectors */
    for (int i = 0; i + 2 < N; ++i) {
        double a[3], b[3], la = 0, lb = 0, ab = 0;
        for (int c = 0; c < 3; ++c) {
            a[c] = r[3 * (i + 1) + c] - r[3 * i + c];
            b[c] = r[3 * (i + 2) + c] - r[3 * (i + 1) + c];
            la += a[c] * a[c]; lb += b[c] * b[c]; ab += a[c] * b[c];
        }
        la = sqrt(la); lb = sqrt(lb);
        double cs = ab / (la * lb);
        e_angle += p->k_angle * (1.0 - cs);
        for (int c = 0; c < 3; ++c) {
            double dcs_da = b[c] / (la * lb) - cs * a[c] / (la * la);
            double dcs_db = a[c] / (la * lb) - cs * b[c] / (lb * lb);
            double dU_da = -p->k_angle * dcs_da, dU_db = -p->k_angle * dcs_db;
            /* a = r_{i+1} - r_i, b = r_{i+2} - r_{i+1} */
            f[3 * i + c] += dU_da;
            f[3 * (i + 1) + c] += -dU_da + dU_db;
            f[3 * (i + 2) + c] += -dU_db;
        }
    }
    /* Lennard-Jones, energy shifted to zero at the cutoff, pairs |i-j| > 2 */
    const double rc = p->lj_rc * p->lj_sigma;
    const double src6 = pow(p->lj_sigma / rc, 6.0);
    const double u_cut = 4.0 * p->lj_eps * (src6 * src6 - src6);
    for (int i = 0; i < N; ++i) {
        for (int j = i + 3; j < N; ++j) {
            double d[3], r2 = 0;
            for (int c = 0; c < 3; ++c) { d[c] = r[3 * i + c] - r[3 * j + c]; r2 += d[c] * d[c]; }
            if (r2 >= rc * rc) continue;
            double sr2 = p->lj_sigma * p->lj_sigma / r2;
            double sr6 = sr2 * sr2 * sr2;
            e_lj += 4.0 * p->lj_eps * (sr6 * sr6 - sr6) - u_cut;
            double fscal = 24.0 * p->lj_eps * (2.0 * sr6 * sr6 - sr6) / r2; /* F_i = fscal d */
            for (int c = 0; c < 3; ++c) { f[3 * i + c] += fscal * d[c]; f[3 * j + c] -= fscal * d[c]; }
        }
    }
    /* restraint on the reaction coordinate */
    {
        int last = N - 1;
        double xi = chain_xi(p, r);
        e_res = 0.5 * p->k * (xi - lam) * (xi - lam);
        double dxi[3];
        if (p->rc_mode == 1) { dxi[0] = 0; dxi[1] = 0; dxi[2] = 1.0; }
        else for (int c = 0; c < 3; ++c) dxi[c] = (r[3 * last + c] - r[c]) / xi;
        for (int c = 0; c < 3; ++c) {
            f[3 * last + c] -= p->k * (xi - lam) * dxi[c];
            f[c] += p->k * (xi - lam) * dxi[c];
        }
    }
    if (e_parts) { e_parts[0] = e_bond; e_parts[1] = e_angle; e_parts[2] = e_lj; e_parts[3] = e_res; }
    return e_bond + e_angle + e_lj + e_res;
}

/* 1-D energy and force including the restraint. */
double oracle_pot1d(const oracle_problem *p, double x, double lam, double *force)
{
    if (force) *force = pot1d_force(p, x) - p->k * (x - lam);
    return pot1d_energy(p, x) + 0.5 * p->k * (x - lam) * (x - lam);
}

/* Default shared start state x_o of the chain: an ideal helix with unit
 * bonds, 100 degrees of turn per bead and rise 0.395 per bead along z, with
 * bead 0 at the origin. */
void oracle_default_helix(int N, double r0, double *r)
{
    const double theta = 100.0 * 3.14159265358979323846 / 180.0;
    const double rise = 0.395 * r0;
    const double rho = sqrt((r0 * r0 - rise * rise) / (2.0 * (1.0 - cos(theta))));
    for (int j = 0; j < N; ++j) {
        r[3 * j] = rho * (cos(j * theta) - 1.0);
        r[3 * j + 1] = rho * sin(j * theta);
        r[3 * j + 2] = j * rise;
    }
}

/* Restraint centre during step n of a window whose target is lam, starting
 * from the reaction coordinate xi_start of the shared start state: the centre
 * moves linearly from xi_start to lam over the first n_pull steps (the pull
 * from x_o to the targeted configuration of Sec. III(ii)) and then stays at
 * lam.  With n_pull = 0 the restraint sits at lam from the first step. */
static double centre_at(const oracle_problem *p, double xi_start, double lam, int64_t n)
{
    if (p->n_pull <= 0 || n >= p->n_pull) return lam;
    return xi_start + (lam - xi_start) * ((double)n / (double)p->n_pull);
}

static int sample_now(const oracle_problem *p, int64_t n)
{
    return n > p->n_equil && ((n - p->n_equil) % p->sample_every) == 0;
}

int64_t oracle_samples_per_replica(const oracle_problem *p)
{
    if (p->n_steps <= p->n_equil) return 0;
    return (p->n_steps - p->n_equil) / p->sample_every;
}

/* ------------------------------------------------------------------------ */
/* One replica of one window.  Writes its sampled xi values to xi_out and    */
/* returns how many were kept.  If traj is non-NULL, the coordinates after   */
/* each of the first traj_steps steps are recorded (step 0 = start state).   */
/* A replica whose state becomes non-finite, or whose |xi| exceeds xi_bound, */
/* at a sampling step is frozen: that sample and all later ones are dropped.*/
/* ------------------------------------------------------------------------ */
static int64_t run_replica_1d(const oracle_problem *p, int window, int replica,
                              double *xi_out, double *traj, int64_t traj_steps)
{
    const double lam = window < p->n_windows ? p->lambda[window] : p->lambda[0];
    const uint32_t gid = (uint32_t)((int64_t)window * p->n_replicas + replica);
    double x = p->init_coords ? p->init_coords[0] : p->lambda[0];
    const double x_start = x;
    const double mu = p->mobility;
    int64_t kept = 0;
    double eta_prev = eta_1d(p->seed, gid, 0);
    if (traj) traj[0] = x;
    for (int64_t n = 1; n <= p->n_steps; ++n) {
        double F;
        oracle_pot1d(p, x, centre_at(p, x_start, lam, n - 1), &F);
        double eta = eta_1d(p->seed, gid, n);
        if (p->integrator_1d == 0) /* x_{n+1} = x_n + mu dt F + sqrt(mu kT dt / 2)(eta_n + eta_{n+1}) */
            x = x + mu * p->dt * F + sqrt(0.5 * mu * p->kT * p->dt) * (eta_prev + eta);
        else                       /* x_{n+1} = x_n + mu dt F + sqrt(2 mu kT dt) eta_{n+1} */
            x = x + mu * p->dt * F + sqrt(2.0 * mu * p->kT * p->dt) * eta;
        eta_prev = eta;
        if (traj && n <= traj_steps) traj[n] = x;
        if (sample_now(p, n)) {
            if (!isfinite(x) || fabs(x) > p->xi_bound) break;
            xi_out[kept++] = x;
        }
    }
    return kept;
}

static int64_t run_replica_chain(const oracle_problem *p, int window, int replica,
                                 double *xi_out, double *traj, int64_t traj_steps)
{
    const int N = p->n_beads;
    const double lam = window < p->n_windows ? p->lambda[window] : p->lambda[0];
    const uint32_t gid = (uint32_t)((int64_t)window * p->n_replicas + replica);
    double *r = (double *)malloc(sizeof(double) * 3 * N);
    double *v = (double *)calloc(3 * N, sizeof(double));
    double *f = (double *)malloc(sizeof(double) * 3 * N);
    if (p->init_coords) memcpy(r, p->init_coords, sizeof(double) * 3 * N);
    else oracle_default_helix(N, p->r0, r);
    const double sd_v = sqrt(p->kT / p->mass);
    /* Maxwell velocities of the mobile beads from counter step 0 */
    for (int i = 1; i < N; ++i) {
        double z[3];
        bead_normals(p->seed, gid, 0u, i, z);
        for (int c = 0; c < 3; ++c) v[3 * i + c] = sd_v * z[c];
    }
    const double xi_start = chain_xi(p, r);
    oracle_chain_forces(p, r, centre_at(p, xi_start, lam, 0), f, NULL);
    if (traj) memcpy(traj, r, sizeof(double) * 3 * N);
    /* BAOAB with friction gamma: c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2) */
    const double h = 0.5 * p->dt;
    const double c1 = exp(-p->gamma * p->dt);
    const double c2 = sqrt(1.0 - c1 * c1);
    int64_t kept = 0;
    for (int64_t n = 1; n <= p->n_steps; ++n) {
        for (int i = 1; i < N; ++i) {              /* bead 0 stays fixed */
            double z[3];
            bead_normals(p->seed, gid, (uint32_t)n, i, z);
            for (int c = 0; c < 3; ++c) {
                int q = 3 * i + c;
                v[q] += h * f[q] / p->mass;        /* B */
                r[q] += h * v[q];                  /* A */
                v[q] = c1 * v[q] + c2 * sd_v * z[c]; /* O */
                r[q] += h * v[q];                  /* A */
            }
        }
        oracle_chain_forces(p, r, centre_at(p, xi_start, lam, n), f, NULL);
        for (int q = 3; q < 3 * N; ++q) v[q] += h * f[q] / p->mass; /* B */
        if (traj && n <= traj_steps) memcpy(traj + 3 * N * n, r, sizeof(double) * 3 * N);
        if (sample_now(p, n)) {
            int finite = 1;
            for (int q = 0; q < 3 * N; ++q) if (!isfinite(r[q])) finite = 0;
            double xi = chain_xi(p, r);
            if (!finite || !isfinite(xi) || fabs(xi) > p->xi_bound) break;
            xi_out[kept++] = xi;
        }
    }
    free(r); free(v); free(f);
    return kept;
}

/* ------------------------------------------------------------------------ */
/* Sequential pulling protocol (Sec. III(i)): one simulation per replica     */
/* that sets the restraint centre to lambda_1, lambda_2, ... lambda_s in      */
/* turn, relaxing n_steps at each and recording xi there (burn-in n_equil and */
/* the record interval restart in every window).  Steps are counted from the  */
/* start of window 1 and the noise is that of replica `replica` of window 1   */
/* of the parallel protocol, so window 1 repeats the parallel protocol's.     */
/* The linear pull (n_pull) applies to window 1.  A replica that blows up     */
/* keeps no sample from that window on.  Its records go to rows               */
/* w * n_replicas + replica of xi_out / n_kept, as in the parallel protocol.  */
/* ------------------------------------------------------------------------ */
static void run_sequential_1d(const oracle_problem *p, int replica, double *xi_out, int64_t *n_kept, int64_t S)
{
    const uint32_t gid = (uint32_t)replica;
    double x = p->init_coords ? p->init_coords[0] : p->lambda[0];
    const double x_start = x;
    const double mu = p->mobility;
    double eta_prev = eta_1d(p->seed, gid, 0);
    int frozen = 0;
    for (int w = 0; w < p->n_windows; ++w) {
        const int64_t row = (int64_t)w * p->n_replicas + replica;
        int64_t kept = 0;
        for (int64_t t = 1; t <= p->n_steps && !frozen; ++t) {
            const int64_t n = (int64_t)w * p->n_steps + t;
            const double centre = (w == 0) ? centre_at(p, x_start, p->lambda[0], t - 1) : p->lambda[w];
            double F;
            oracle_pot1d(p, x, centre, &F);
            double eta = eta_1d(p->seed, gid, n);
            if (p->integrator_1d == 0)
                x = x + mu * p->dt * F + sqrt(0.5 * mu * p->kT * p->dt) * (eta_prev + eta);
            else
                x = x + mu * p->dt * F + sqrt(2.0 * mu * p->kT * p->dt) * eta;
            eta_prev = eta;
            if (sample_now(p, t)) {
                if (!isfinite(x) || fabs(x) > p->xi_bound) { frozen = 1; break; }
                xi_out[row * S + kept++] = x;
            }
        }
        n_kept[row] = kept;
    }
}

static void run_sequential_chain(const oracle_problem *p, int replica, double *xi_out, int64_t *n_kept, int64_t S)
{
    const int N = p->n_beads;
    const uint32_t gid = (uint32_t)replica;
    double *r = (double *)malloc(sizeof(double) * 3 * N);
    double *v = (double *)calloc(3 * N, sizeof(double));
    double *f = (double *)malloc(sizeof(double) * 3 * N);
    if (p->init_coords) memcpy(r, p->init_coords, sizeof(double) * 3 * N);
    else oracle_default_helix(N, p->r0, r);
    const double sd_v = sqrt(p->kT / p->mass);
    for (int i = 1; i < N; ++i) {
        double z[3];
        bead_normals(p->seed, gid, 0u, i, z);
        for (int c = 0; c < 3; ++c) v[3 * i + c] = sd_v * z[c];
    }
    const double xi_start = chain_xi(p, r);
    const double h = 0.5 * p->dt;
    const double c1 = exp(-p->gamma * p->dt);
    const double c2 = sqrt(1.0 - c1 * c1);
    int frozen = 0;
    for (int w = 0; w < p->n_windows; ++w) {
        const int64_t row = (int64_t)w * p->n_replicas + replica;
        const double lam = p->lambda[w];
        int64_t kept = 0;
        /* the restraint moves to lambda_w: forces of the new Hamiltonian */
        oracle_chain_forces(p, r, (w == 0) ? centre_at(p, xi_start, lam, 0) : lam, f, NULL);
        for (int64_t t = 1; t <= p->n_steps && !frozen; ++t) {
            const int64_t n = (int64_t)w * p->n_steps + t;
            for (int i = 1; i < N; ++i) {
                double z[3];
                bead_normals(p->seed, gid, (uint32_t)n, i, z);
                for (int c = 0; c < 3; ++c) {
                    int q = 3 * i + c;
                    v[q] += h * f[q] / p->mass;
                    r[q] += h * v[q];
                    v[q] = c1 * v[q] + c2 * sd_v * z[c];
                    r[q] += h * v[q];
                }
            }
            oracle_chain_forces(p, r, (w == 0) ? centre_at(p, xi_start, lam, t) : lam, f, NULL);
            for (int q = 3; q < 3 * N; ++q) v[q] += h * f[q] / p->mass;
            if (sample_now(p, t)) {
                int finite = 1;
                for (int q = 0; q < 3 * N; ++q) if (!isfinite(r[q])) finite = 0;
                double xi = chain_xi(p, r);
                if (!finite || !isfinite(xi) || fabs(xi) > p->xi_bound) { frozen = 1; break; }
                xi_out[row * S + kept++] = xi;
            }
        }
        n_kept[row] = kept;
    }
    free(r); free(v); free(f);
}

/* Runs every replica of every window.  xi_out is [W*n_replicas][S] with
 * W = n_windows (+1 with the free ensemble) and S = oracle_samples_per_replica(p);
 * n_kept is [W*n_replicas].
 * Returns the number of host threads used. */
int oracle_run(const oracle_problem *p, double *xi_out, int64_t *n_kept, int n_threads)
{
    const int64_t S = oracle_samples_per_replica(p);
    /* the unrestrained ensemble is window n_windows: the same system with k = 0 */
    const int64_t total = ((int64_t)p->n_windows + (p->free_ensemble ? 1 : 0)) * p->n_replicas;
    oracle_problem free_sys = *p;
    free_sys.k = 0.0;
    int used = 1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        used = omp_get_num_threads();
#endif
        if (p->sequential) {
#pragma omp for schedule(dynamic, 1)
            for (int r = 0; r < p->n_replicas; ++r) {
                if (p->model == 0) run_sequential_1d(p, r, xi_out, n_kept, S);
                else run_sequential_chain(p, r, xi_out, n_kept, S);
            }
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t g = 0; g < total; ++g) {
                int window = (int)(g / p->n_replicas), replica = (int)(g % p->n_replicas);
                const oracle_problem *q = window < p->n_windows ? p : &free_sys;
                double *dst = xi_out + g * S;
                n_kept[g] = (p->model == 0) ? run_replica_1d(q, window, replica, dst, NULL, 0)
                                            : run_replica_chain(q, window, replica, dst, NULL, 0);
            }
        }
    }
    return used;
}

/* Coordinates of one replica over its first n_steps steps (parity hook).
 * out is [n_steps + 1][dof], dof = 1 (1-D) or 3 N (chain). */
void oracle_trajectory(const oracle_problem *p, int window, int replica, int64_t n_steps, double *out)
{
    oracle_problem q = *p;
    q.n_steps = n_steps;
    q.n_equil = n_steps;           /* no sampling needed */
    double dummy;
    if (p->model == 0) run_replica_1d(&q, window, replica, &dummy, out, n_steps);
    else run_replica_chain(&q, window, replica, &dummy, out, n_steps);
}

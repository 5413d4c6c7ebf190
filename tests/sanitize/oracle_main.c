/* Drives every entry of the CPU oracle once on small problems, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure only).
 * The oracle source is compiled into this translation unit. */
#include "../../oracle/ppp_oracle.c"

#include <stdio.h>

static oracle_problem base(int model, int n_beads)
{
    static const double lam1d[6] = {-1.5, -0.9, -0.3, 0.3, 0.9, 1.5};
    static const double lamc[4] = {3.2, 3.8, 4.4, 5.0};
    oracle_problem p;
    memset(&p, 0, sizeof(p));
    p.model = model;
    p.pot_kind = 0; p.pot_a = 5.0; p.pot_b = 1.0; p.pot_kappa = 4.0; p.mobility = 1.0; p.integrator_1d = 0;
    p.n_beads = n_beads; p.k_bond = 100.0; p.r0 = 1.0; p.k_angle = 5.0;
    p.lj_eps = 1.0; p.lj_sigma = 1.0; p.lj_rc = 2.5; p.rc_mode = 0; p.mass = 1.0; p.gamma = 1.0;
    p.n_windows = model == 0 ? 6 : 4;
    p.lambda = model == 0 ? lam1d : lamc;
    p.k = 20.0; p.kT = 1.0; p.dt = model == 0 ? 1e-3 : 0.005;
    p.n_steps = 300; p.n_equil = 30; p.sample_every = 7; p.n_replicas = 5; p.seed = 11;
    p.xi_bound = 1e4;
    return p;
}

static int run_case(const char *name, const oracle_problem *p)
{
    const int64_t S = oracle_samples_per_replica(p);
    const int64_t rows = ((int64_t)p->n_windows + (p->free_ensemble ? 1 : 0)) * p->n_replicas;
    double *xi = (double *)calloc((size_t)(rows * (S > 0 ? S : 1)), sizeof(double));
    int64_t *kept = (int64_t *)calloc((size_t)rows, sizeof(int64_t));
    oracle_run(p, xi, kept, 2);
    int64_t tot = 0;
    for (int64_t r = 0; r < rows; ++r) tot += kept[r];
    printf("%s: %lld samples\n", name, (long long)tot);
    free(xi); free(kept);
    return tot > 0 ? 0 : 1;
}

int main(void)
{
    int bad = 0;
    oracle_problem p = base(0, 1);
    bad |= run_case("1d", &p);
    p.integrator_1d = 1; p.n_pull = 100;
    bad |= run_case("1d-em-pull", &p);
    p = base(0, 1); p.sequential = 1;
    bad |= run_case("1d-sequential", &p);
    p = base(0, 1); p.free_ensemble = 1;
    bad |= run_case("1d-free", &p);
    for (int N = 2; N <= 13; N += 11) {
        p = base(1, N);
        bad |= run_case("chain", &p);
        p.sequential = 1;
        bad |= run_case("chain-sequential", &p);
        p.sequential = 0; p.free_ensemble = 1; p.n_pull = 50;
        bad |= run_case("chain-free-pull", &p);
    }
    /* forces, energies and a trajectory of a 13-bead chain; a NaN start freezes */
    p = base(1, 13);
    double r[39], f[39], e[4];
    oracle_default_helix(13, 1.0, r);
    oracle_chain_forces(&p, r, 4.0, f, e);
    double *traj = (double *)malloc(sizeof(double) * 39 * 21);
    oracle_trajectory(&p, 1, 2, 20, traj);
    free(traj);
    double x = 0.2, fx;
    oracle_pot1d(&p, x, 0.1, &fx);
    double init[39];
    memcpy(init, r, sizeof(init));
    init[3 * 12] = NAN;
    p.init_coords = init;
    const int64_t S = oracle_samples_per_replica(&p);
    double *xi = (double *)calloc((size_t)(4 * 5 * S), sizeof(double));
    int64_t kept[20];
    oracle_run(&p, xi, kept, 1);
    free(xi);
    for (int q = 0; q < 20; ++q) bad |= kept[q] != 0;
    printf("done %d\n", bad);
    return bad;
}

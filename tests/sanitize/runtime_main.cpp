// Drives the host side of the C ABI (validation, planning, workspace layout,
// batches, error strings, checkpoint size queries) on small problems, for a
// build of the host runtime with AddressSanitizer (test infrastructure only).
// Nothing here touches a GPU.
#include <cstdio>
#include <cstring>
#include <vector>

#include "ppp.h"

static ppp_problem chain_problem(const std::vector<double> &lam, int n_beads) {
    ppp_problem p;
    std::memset(&p, 0, sizeof(p));
    p.model = PPP_MODEL_CHAIN;
    p.chain = ppp_chain{n_beads, 100.0, 1.0, 5.0, 1.0, 1.0, 2.5, 0, 1.0, 1.0};
    p.n_windows = (int32_t)lam.size();
    p.lambda = lam.data();
    p.k = 20.0; p.kT = 1.0; p.dt = 0.005;
    p.n_steps = 1000; p.n_equil = 100; p.sample_every = 10; p.n_replicas = 37; p.seed = 3;
    p.precision = PPP_FP32_FORCES;
    p.xi_min = 0.0; p.xi_bin = 0.01; p.xi_nbins = 1024; p.w_bin = 0.05; p.w_half_bins = 500;
    p.n_jack_blocks = 8;
    return p;
}

static int expect(const char *what, ppp_status got, ppp_status want) {
    if (got != want) { std::printf("FAIL %s: %d (want %d) %s\n", what, (int)got, (int)want, ppp_create_error()); return 1; }
    return 0;
}

int main() {
    int bad = 0;
    std::vector<double> lam = {3.2, 3.8, 4.4, 5.0, 5.6};
    for (int n_beads : {2, 10, 37, 256}) {
        for (uint32_t flags : {0u, (uint32_t)PPP_FLAG_SEQUENTIAL, (uint32_t)PPP_FLAG_FREE_ENSEMBLE}) {
            ppp_problem p = chain_problem(lam, n_beads);
            p.flags = flags;
            ppp_handle *h = nullptr;
            bad |= expect("create", ppp_create(&p, &h), PPP_OK);
            size_t bytes = 0, ck = 0;
            bad |= expect("workspace", ppp_workspace_size(h, &bytes), PPP_OK);
            bad |= expect("checkpoint size", ppp_checkpoint(h, nullptr, &ck), PPP_OK);
            if (bytes == 0 || ck == 0) { std::printf("FAIL sizes\n"); bad = 1; }
            std::printf("N=%d flags=%u workspace %zu checkpoint %zu\n", n_beads, flags, bytes, ck);
            bad |= expect("destroy", ppp_destroy(h), PPP_OK);
        }
    }
    // rejected problems: each before any device work, with a message
    {
        ppp_problem p = chain_problem(lam, 10);
        ppp_handle *h = nullptr;
        p.k = 0.0;
        bad |= expect("k = 0", ppp_create(&p, &h), PPP_E_INVALID_ARG);
        p = chain_problem(lam, 10);
        std::vector<double> bad_lam = {1.0, 2.0, 2.0};
        p.lambda = bad_lam.data(); p.n_windows = 3;
        bad |= expect("non-monotone", ppp_create(&p, &h), PPP_E_INVALID_ARG);
        p = chain_problem(lam, 10);
        p.flags = PPP_FLAG_SEQUENTIAL | PPP_FLAG_FREE_ENSEMBLE;
        bad |= expect("sequential + free", ppp_create(&p, &h), PPP_E_UNSUPPORTED);
        p = chain_problem(lam, 10);
        p.flags = 8u;
        bad |= expect("unknown flag", ppp_create(&p, &h), PPP_E_INVALID_ARG);
        if (std::strlen(ppp_create_error()) == 0) { std::printf("FAIL no message\n"); bad = 1; }
        bad |= expect("null", ppp_create(nullptr, &h), PPP_E_INVALID_ARG);
    }
    // a batch of uneven chains
    {
        std::vector<std::vector<double>> lams;
        std::vector<ppp_problem> ps;
        for (int c = 0; c < 9; ++c) {
            std::vector<double> l;
            for (int w = 0; w < 3 + c; ++w) l.push_back(2.0 + 0.3 * w);
            lams.push_back(l);
        }
        for (int c = 0; c < 9; ++c) {
            ppp_problem p = chain_problem(lams[c], 8 + 13 * c);
            p.n_replicas = 16 + 7 * c;
            p.n_steps = 500 + 100 * c;
            if (c % 3 == 0) p.flags = PPP_FLAG_FREE_ENSEMBLE;
            ps.push_back(p);
        }
        ppp_handle *h = nullptr;
        bad |= expect("batch", ppp_batch_create(ps.data(), (int32_t)ps.size(), nullptr, &h), PPP_OK);
        size_t bytes = 0;
        bad |= expect("batch workspace", ppp_workspace_size(h, &bytes), PPP_OK);
        std::printf("batch workspace %zu\n", bytes);
        bad |= expect("batch destroy", ppp_destroy(h), PPP_OK);
    }
    // the 1-D model and the window-placement sizing
    {
        std::vector<double> l1 = {-1.5, -0.5, 0.5, 1.5};
        ppp_problem p;
        std::memset(&p, 0, sizeof(p));
        p.model = PPP_MODEL_1D;
        p.pot1d = ppp_pot1d{0, 5.0, 1.0, 0.0, 1.0};
        p.n_windows = 4; p.lambda = l1.data();
        p.k = 50.0; p.kT = 1.0; p.dt = 1e-3; p.n_steps = 2000; p.n_equil = 200; p.sample_every = 10;
        p.n_replicas = 64; p.seed = 1; p.precision = PPP_FP64;
        p.xi_min = -2.5; p.xi_bin = 0.001; p.xi_nbins = 5000; p.w_bin = 0.01; p.w_half_bins = 1000;
        ppp_handle *h = nullptr;
        bad |= expect("1d", ppp_create(&p, &h), PPP_OK);
        bad |= expect("1d destroy", ppp_destroy(h), PPP_OK);
        ppp_adaptive a;
        std::memset(&a, 0, sizeof(a));
        a.budget_replica_steps = 100000000; a.initial_windows = 5; a.max_rounds = 2; a.max_windows = 32;
        a.target_dl_over_sigma = 1.0; a.train_iters = 10; a.lr = 1e-3; a.init_seed = 1;
        size_t bytes = 0;
        bad |= expect("adaptive size", ppp_adaptive_workspace_size(&p, &a, &bytes), PPP_OK);
        a.max_windows = 1;
        bad |= expect("adaptive invalid", ppp_adaptive_workspace_size(&p, &a, &bytes), PPP_E_INVALID_ARG);
    }
    for (int s = 0; s < 7; ++s)
        if (!ppp_status_string((ppp_status)s) || !*ppp_status_string((ppp_status)s)) bad = 1;
    if (std::strcmp(ppp_last_error(nullptr), "") != 0) bad = 1;
    std::printf("done %d\n", bad);
    return bad;
}

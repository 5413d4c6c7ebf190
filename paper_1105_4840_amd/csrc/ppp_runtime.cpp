// Host runtime of libppp: the C ABI of include/ppp.h.
//
// A handle holds one or more validated problems, the kernel shape chosen for
// each, the work items (window x replica range handled by one workgroup) and
// the byte layout of the caller's device workspace.  Runs enqueue kernels on
// the caller's stream; nothing is allocated on the device by the library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "ppp.h"
#include "ppp_internal.hpp"
#include "ppp_internal_api.hpp"
#include "ppp_launch.hpp"
#include "ppp_probe.h"
#include "ppp_probe.hpp"
#include "ppp_shapes.hpp"

using namespace ppp;

namespace {

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct ProblemHost {
    ppp_problem p{};
    std::vector<double> lambda;
    std::vector<double> init;   // resolved shared start state x_o
    DevProblem dev{};
    int G = 1, B = 1;
    int first_item = 0, n_items = 0;
    int item_windows = 1;        // most windows one work item's replicas fall in
    int64_t region_begin = 0, region_end = 0;   // byte range of this problem in the workspace
};

struct VariantGroup {
    int precision, G, B;
    int first_item, n_items;   // items of this group are contiguous, longest first
};

}  // namespace

struct ppp_handle {
    std::vector<ProblemHost> probs;
    std::vector<DevProblem> dev;     // the problems' device records, built with the layout
    std::vector<WorkItem> items;
    std::vector<VariantGroup> groups;
    bool batch = false;
    int64_t off_probs = 0, off_items = 0, off_tickets = 0;
    int64_t ws_bytes = 0;
    int max_windows = 0, max_blocks = 0, max_k = 0, max_m = 0;
    // run state
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    bool begun = false, finalized = false, ran = false, restored = false;
    int64_t steps_done = 0;
    std::string err;
    hipEvent_t ev[8] = {};       // 0-4: begin, sim start, reduce, App. C, end; 5-6: last advance
    bool advanced = false;       // ev[5], ev[6] hold an advance
    bool events_ok = false;
    int sim_launches = 0;
    // batch graph
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    char *graph_ws = nullptr;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_ev;
};

namespace {

ppp_status fail(ppp_handle *h, ppp_status st, const std::string &msg) {
    if (h) h->err = msg;
    return st;
}
ppp_status hip_fail(ppp_handle *h, hipError_t e, const char *where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(h, PPP_E_DEVICE, m);
}
#define HIPCHK(h, call)                                       \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail((h), e_, #call); \
    } while (0)

// Ideal helix through the origin: unit-bond geometry scaled by r0, 100 degrees
// of turn and a rise of 0.395 r0 per bead along z.
void helix(int N, double r0, std::vector<double> &r) {
    const double theta = 100.0 * M_PI / 180.0;
    const double rise = 0.395 * r0;
    const double rho = std::sqrt((r0 * r0 - rise * rise) / (2.0 * (1.0 - std::cos(theta))));
    r.assign(3 * (size_t)N, 0.0);
    for (int j = 0; j < N; ++j) {
        r[3 * j] = rho * (std::cos(j * theta) - 1.0);
        r[3 * j + 1] = rho * std::sin(j * theta);
        r[3 * j + 2] = j * rise;
    }
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

ppp_status validate(const ppp_problem *p, std::string &msg) {
    if (!p) { msg = "problem is NULL"; return PPP_E_INVALID_ARG; }
    if (p->model != PPP_MODEL_1D && p->model != PPP_MODEL_CHAIN) { msg = "unknown model"; return PPP_E_INVALID_ARG; }
    if (p->n_windows < 2) { msg = "n_windows must be >= 2"; return PPP_E_INVALID_ARG; }
    if (!p->lambda) { msg = "lambda is NULL"; return PPP_E_INVALID_ARG; }
    int dir = 0;
    for (int i = 0; i < p->n_windows; ++i) {
        if (!std::isfinite(p->lambda[i])) { msg = "lambda must be finite"; return PPP_E_INVALID_ARG; }
        if (i > 0) {
            const double d = p->lambda[i] - p->lambda[i - 1];
            const int sd = d > 0 ? 1 : (d < 0 ? -1 : 0);
            if (sd == 0 || (dir != 0 && sd != dir)) { msg = "lambda must be strictly monotone"; return PPP_E_INVALID_ARG; }
            dir = sd;
        }
    }
    if (!finite_pos(p->k)) { msg = "k must be > 0"; return PPP_E_INVALID_ARG; }
    if (!finite_pos(p->kT)) { msg = "kT must be > 0"; return PPP_E_INVALID_ARG; }
    if (!finite_pos(p->dt)) { msg = "dt must be > 0"; return PPP_E_INVALID_ARG; }
    if (p->n_replicas < 1) { msg = "n_replicas must be >= 1"; return PPP_E_INVALID_ARG; }
    const int64_t sim_windows = (int64_t)p->n_windows + ((p->flags & PPP_FLAG_FREE_ENSEMBLE) ? 1 : 0);
    if (sim_windows * p->n_replicas > 0x7fffffffLL) { msg = "too many replicas"; return PPP_E_INVALID_ARG; }
    if (p->sample_every < 1) { msg = "sample_every must be >= 1"; return PPP_E_INVALID_ARG; }
    if (p->n_steps < 1 || p->n_steps > 0xffffffffLL) { msg = "n_steps must be in [1, 2^32)"; return PPP_E_INVALID_ARG; }
    if (p->n_equil < 0 || p->n_equil >= p->n_steps) { msg = "need 0 <= n_equil < n_steps"; return PPP_E_INVALID_ARG; }
    if (p->n_pull < 0) { msg = "n_pull must be >= 0"; return PPP_E_INVALID_ARG; }
    // samples taken while the centre still moves would be charged the work and the
    // window mean of the fixed lambda_i (Eqs. 9, 14): the pull must end before sampling
    if (p->n_pull > p->n_equil) { msg = "need n_pull <= n_equil (no samples while the centre moves)"; return PPP_E_INVALID_ARG; }
    // the bin loops step in int by up to 256 at a time, so K stays far from 2^31
    if (p->xi_nbins < 1 || p->xi_nbins > (1 << 26)) { msg = "xi_nbins must be in [1, 2^26]"; return PPP_E_INVALID_ARG; }
    if (!finite_pos(p->xi_bin) || !std::isfinite(p->xi_min)) { msg = "xi_bin must be > 0, xi_min finite"; return PPP_E_INVALID_ARG; }
    if (p->w_half_bins < 0 || p->w_half_bins > 50000000) { msg = "w_half_bins out of range"; return PPP_E_INVALID_ARG; }
    if (p->w_half_bins > 0 && !finite_pos(p->w_bin)) { msg = "w_bin must be > 0"; return PPP_E_INVALID_ARG; }
    if (p->n_jack_blocks < 0 || p->n_jack_blocks > 4096) { msg = "n_jack_blocks must be in [0, 4096]"; return PPP_E_INVALID_ARG; }
    if ((p->flags & ~(PPP_FLAG_SEQUENTIAL | PPP_FLAG_FREE_ENSEMBLE)) != 0) { msg = "unknown flags"; return PPP_E_INVALID_ARG; }
    if ((p->flags & PPP_FLAG_SEQUENTIAL) && (int64_t)p->n_windows * p->n_steps > 0xffffffffLL) {
        msg = "a sequential run must have fewer than 2^32 steps per replica"; return PPP_E_INVALID_ARG;
    }
    if ((p->flags & PPP_FLAG_SEQUENTIAL) && (p->flags & PPP_FLAG_FREE_ENSEMBLE)) {
        msg = "the free ensemble runs with the parallel protocol only"; return PPP_E_UNSUPPORTED;
    }
    if (p->precision != PPP_FP32_FORCES && p->precision != PPP_FP64) { msg = "unknown precision"; return PPP_E_INVALID_ARG; }
    if (p->model == PPP_MODEL_1D) {
        const ppp_pot1d &q = p->pot1d;
        if (q.kind != 0 && q.kind != 1) { msg = "pot1d.kind must be 0 or 1"; return PPP_E_INVALID_ARG; }
        if (!finite_pos(q.mobility)) { msg = "mobility must be > 0"; return PPP_E_INVALID_ARG; }
        if (!std::isfinite(q.a) || !std::isfinite(q.b) || !std::isfinite(q.kappa)) { msg = "pot1d parameters must be finite"; return PPP_E_INVALID_ARG; }
        if (p->integrator_1d != PPP_INT_LM && p->integrator_1d != PPP_INT_EM) { msg = "unknown integrator"; return PPP_E_INVALID_ARG; }
    } else {
        const ppp_chain &c = p->chain;
        if (c.n_beads < 2 || c.n_beads > PPP_MAX_BEADS) { msg = "n_beads must be in [2, PPP_MAX_BEADS]"; return PPP_E_INVALID_ARG; }
        if (!finite_pos(c.r0) || !finite_pos(c.mass) || !finite_pos(c.lj_sigma) || !finite_pos(c.lj_rc)) { msg = "r0, mass, lj_sigma, lj_rc must be > 0"; return PPP_E_INVALID_ARG; }
        if (!(c.k_bond >= 0) || !(c.k_angle >= 0) || !(c.lj_eps >= 0) || !(c.gamma >= 0)) { msg = "k_bond, k_angle, lj_eps, gamma must be >= 0"; return PPP_E_INVALID_ARG; }
        if (c.rc_mode != 0 && c.rc_mode != 1) { msg = "rc_mode must be 0 or 1"; return PPP_E_INVALID_ARG; }
    }
    if (p->init_coords) {
        const int n = p->model == PPP_MODEL_1D ? 1 : 3 * p->chain.n_beads;
        for (int i = 0; i < n; ++i)
            if (std::isnan(p->init_coords[i]) && p->model == PPP_MODEL_CHAIN && i < 3) { msg = "bead 0 must be finite"; return PPP_E_INVALID_ARG; }
    }
    return PPP_OK;
}

// Kernel shape (lanes per replica G, beads per lane B) for a chain length.
void default_shape(int N, int precision, int &G, int &B) {
    // measured on MI355X: short chains want a few lanes per replica to fill the
    // chip (21504 ten-bead replicas: 5 lanes each give 1792 wavefronts for the
    // 1024 SIMDs, 2 lanes only 672), long chains more beads per lane for fewer
    // rotation rounds; fp64 (twice the registers) keeps two beads per lane so
    // that nothing spills
    if (precision == PPP_FP64) {
        if (N <= 4) { G = 1; B = 4; }
        else if (N <= 10) { G = 5; B = 2; }
        else if (N <= 12) { G = 3; B = 4; }
        else if (N <= 16) { G = 8; B = 2; }
        else if (N <= 32) { G = 16; B = 2; }
        else if (N <= 64) { G = 32; B = 2; }
        else if (N <= 128) { G = 64; B = 2; }
        else { G = 64; B = 4; }
        return;
    }
    if (N <= 4) { G = 1; B = 4; }
    else if (N <= 8) { G = 1; B = 8; }
    else if (N <= 10) { G = 5; B = 2; }
    else if (N <= 12) { G = 3; B = 4; }
    else if (N <= 16) { G = 4; B = 4; }
    else if (N <= 32) { G = 16; B = 2; }
    else if (N <= 64) { G = 16; B = 4; }
    else if (N <= 128) { G = 32; B = 4; }
    else { G = 64; B = 4; }
}

struct TuneEntry { int nmax, precision, G, B; };

std::vector<TuneEntry> read_tune_table(const char *path) {
    std::vector<TuneEntry> t;
    if (!path) return t;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        TuneEntry e{};
        if (is >> e.nmax >> e.precision >> e.G >> e.B) t.push_back(e);
    }
    std::sort(t.begin(), t.end(), [](const TuneEntry &a, const TuneEntry &b) { return a.nmax < b.nmax; });
    return t;
}

void choose_shape(int N, int precision, const std::vector<TuneEntry> &tune, int &G, int &B) {
    default_shape(N, precision, G, B);
    for (const auto &e : tune)
        if (e.precision == precision && N <= e.nmax && e.G * e.B >= N && chain_shape_supported(e.G, e.B) &&
            (e.G == 1 || e.B >= 2)) {
            G = e.G; B = e.B;
            return;
        }
}

ppp_status build_problem(const ppp_problem *p, ProblemHost &ph, const std::vector<TuneEntry> &tune, std::string &msg) {
    ppp_status st = validate(p, msg);
    if (st != PPP_OK) return st;
    ph.p = *p;
    ph.lambda.assign(p->lambda, p->lambda + p->n_windows);
    // the unrestrained ensemble's entry: its xi is recorded relative to lambda_1
    if (p->flags & PPP_FLAG_FREE_ENSEMBLE) ph.lambda.push_back(p->lambda[0]);
    ph.p.lambda = ph.lambda.data();
    const bool chain = p->model == PPP_MODEL_CHAIN;
    if (chain) {
        const int N = p->chain.n_beads;
        if (p->init_coords) ph.init.assign(p->init_coords, p->init_coords + 3 * N);
        else helix(N, p->chain.r0, ph.init);
        choose_shape(N, p->precision, tune, ph.G, ph.B);
    } else {
        ph.init.assign(1, p->init_coords ? p->init_coords[0] : p->lambda[0]);
        ph.G = 1; ph.B = 1;
    }
    ph.p.init_coords = ph.init.data();
    DevProblem &d = ph.dev;
    std::memset(&d, 0, sizeof(d));
    d.model = p->model;
    d.precision = p->precision;
    d.pot_kind = p->pot1d.kind;
    d.integrator_1d = p->integrator_1d;
    d.n_beads = chain ? p->chain.n_beads : 1;
    d.n_pad = chain ? ph.G * ph.B : 1;
    d.rc_mode = p->chain.rc_mode;
    d.n_windows = p->n_windows;
    d.n_replicas = p->n_replicas;
    int B = p->n_jack_blocks == 0 ? 32 : p->n_jack_blocks;
    B = std::min(B, p->n_replicas);
    d.n_blocks = B;
    d.xi_nbins = p->xi_nbins;
    d.w_half_bins = p->w_half_bins;
    d.sample_every = p->sample_every;
    d.variant_lanes = ph.G;
    d.variant_beads = ph.B;
    d.n_steps = p->n_steps;
    d.sequential = (p->flags & PPP_FLAG_SEQUENTIAL) ? 1 : 0;
    d.free_ens = (p->flags & PPP_FLAG_FREE_ENSEMBLE) ? 1 : 0;
    d.n_sim_windows = d.n_windows + d.free_ens;
    d.n_equil = p->n_equil;
    d.n_pull = p->n_pull;
    d.seed = p->seed;
    d.k = p->k; d.kT = p->kT; d.beta = 1.0 / p->kT; d.dt = p->dt;
    d.pot_a = p->pot1d.a; d.pot_b = p->pot1d.b; d.pot_kappa = p->pot1d.kappa; d.mobility = p->pot1d.mobility;
    if (chain) {
        const ppp_chain &c = p->chain;
        d.k_bond = c.k_bond; d.r0 = c.r0; d.k_angle = c.k_angle;
        const double s2 = c.lj_sigma * c.lj_sigma, s6 = s2 * s2 * s2, s12 = s6 * s6;
        d.lj_A = 48.0 * c.lj_eps * s12; d.lj_B = 24.0 * c.lj_eps * s6;
        d.lj_eA = 4.0 * c.lj_eps * s12; d.lj_eB = 4.0 * c.lj_eps * s6;
        const double rc = c.lj_rc * c.lj_sigma;
        const double q = std::pow(c.lj_sigma / rc, 6.0);
        d.lj_ucut = 4.0 * c.lj_eps * (q * q - q);
        d.rc2 = rc * rc;
        d.mass = c.mass; d.inv_mass = 1.0 / c.mass;
        d.c1 = std::exp(-c.gamma * p->dt);
        d.sd_v = std::sqrt(p->kT / c.mass);
        d.c2sd = std::sqrt(1.0 - d.c1 * d.c1) * d.sd_v;
        d.fix_x = ph.init[0]; d.fix_y = ph.init[1]; d.fix_z = ph.init[2];
        const int last = c.n_beads - 1;
        const double dx = ph.init[3 * last] - d.fix_x, dy = ph.init[3 * last + 1] - d.fix_y, dz = ph.init[3 * last + 2] - d.fix_z;
        d.xi_start = c.rc_mode == 1 ? dz : std::sqrt(dx * dx + dy * dy + dz * dz);
        d.pad_z0 = 1.0e5 * c.lj_sigma;
        d.pad_dz = 4.0 * rc;
    } else {
        d.xi_start = ph.init[0];
    }
    d.xi_min = p->xi_min; d.xi_bin = p->xi_bin; d.w_bin = p->w_bin;
    d.xi_bound = p->xi_bound > 0 ? p->xi_bound : 1.0e4;
    return PPP_OK;
}

// Byte layout of the problem's arrays from offset `at`; returns the end.
int64_t layout_problem(ProblemHost &ph, int64_t at) {
    DevProblem &d = ph.dev;
    const int64_t s = d.n_windows, S = d.n_sim_windows, R = d.n_replicas, K = d.xi_nbins, Bk = d.n_blocks;
    const int64_t tsize = d.precision == PPP_FP64 ? 8 : 4;
    ph.region_begin = at;
    auto take = [&](int64_t bytes) { const int64_t o = at; at = align_up(at + std::max<int64_t>(bytes, 1)); return o; };
    d.off_lambda = take(S * 8);
    d.off_init = take((int64_t)ph.init.size() * 8);
    d.off_state = take(d.model == PPP_MODEL_CHAIN ? S * R * 6 * d.n_pad * tsize : S * R * 2 * tsize);
    d.off_acc = take(S * R * A_NFIELDS * 8);
    d.off_hist = take(S * K * 8);
    d.off_blk = take(S * Bk * A_NFIELDS * 8);
    d.off_tot = take(S * A_NFIELDS * 8);
    d.off_jack = take(Bk * JK_FIELDS * s * 8);
    d.off_jack_turn = take(Bk * JK_TURN * 8);
    d.off_out = take((int64_t)O_NFIELDS * s * 8);
    d.off_turn = take(PPP_ON_NFIELDS * 8);
    if (d.w_half_bins > 0) {
        d.off_pairs_shift = take(kAppcChains * s * K * 4);
        d.off_pairs_ceil = take(s * K * 4);
        d.off_pairs_prob = take(kAppcChains * s * K * 8);
        d.off_npairs = take(kAppcChains * s * 4);
        d.off_omega = take(kAppcChains * s * (2 * (int64_t)d.w_half_bins + 1) * 8);
    }
    ph.region_end = at;
    return at;
}

// Steps each replica takes: n_steps, or n_steps in every window one after
// another for the sequential protocol.
int64_t total_steps(const ProblemHost &ph) {
    return ph.dev.sequential ? (int64_t)ph.dev.n_windows * ph.dev.n_steps : ph.dev.n_steps;
}

int reps_per_item(const ProblemHost &ph) { return ph.dev.model == PPP_MODEL_CHAIN ? chain_reps_per_wg(ph.G) : WG; }

// Work items of one problem.  Per window (every item inside one window), or,
// for chain problems whose windows do not split into whole items, as runs of
// consecutive replicas that may cross into the next window (no workgroup is
// left part empty at a window's end), provided the workgroup histogram of all
// windows one item touches still fits in LDS.
void make_items(ProblemHost &ph, int prob_index, std::vector<WorkItem> &items, bool allow_span) {
    const int per = reps_per_item(ph);
    const int64_t R = ph.dev.n_replicas, total = (int64_t)ph.dev.n_sim_windows * R;
    ph.first_item = (int)items.size();
    ph.item_windows = 1;
    const int64_t span_windows = (per - 1) / R + 2;   // a run of `per` replicas touches at most this many
    const bool span = allow_span && ph.dev.model == PPP_MODEL_CHAIN && R % per != 0 &&
                      span_windows * ph.dev.xi_nbins <= kLdsHistCap;
    if (ph.dev.sequential) {
        // the replicas of window 1; every window is run by the same items in turn
        for (int r = 0; r < ph.dev.n_replicas; r += per)
            items.push_back(WorkItem{prob_index, 0, r, std::min(per, ph.dev.n_replicas - r)});
    } else if (span) {
        for (int64_t g = 0; g < total; g += per) {
            const int n = (int)std::min<int64_t>(per, total - g);
            items.push_back(WorkItem{prob_index, (int)(g / R), (int)(g % R), n});
            ph.item_windows = std::max(ph.item_windows, (int)((g + n - 1) / R - g / R + 1));
        }
    } else {
        for (int w = 0; w < ph.dev.n_sim_windows; ++w)
            for (int r = 0; r < ph.dev.n_replicas; r += per)
                items.push_back(WorkItem{prob_index, w, r, std::min(per, ph.dev.n_replicas - r)});
    }
    ph.n_items = (int)items.size() - ph.first_item;
}

void finish_layout(ppp_handle *h) {
    int64_t at = 0;
    h->off_probs = at; at = align_up(at + (int64_t)h->probs.size() * sizeof(DevProblem));
    h->off_items = at; at = align_up(at + (int64_t)std::max<size_t>(h->items.size(), 1) * sizeof(WorkItem));
    h->off_tickets = at; at = align_up(at + 64 * sizeof(int));
    h->max_windows = h->max_blocks = h->max_k = h->max_m = 0;
    for (auto &ph : h->probs) {
        at = layout_problem(ph, at);
        h->max_windows = std::max(h->max_windows, ph.dev.n_sim_windows);
        h->max_blocks = std::max(h->max_blocks, ph.dev.n_blocks);
        h->max_k = std::max(h->max_k, ph.dev.xi_nbins);
        h->max_m = std::max(h->max_m, ph.dev.w_half_bins);
    }
    h->ws_bytes = at;
    h->dev.clear();
    for (auto &ph : h->probs) h->dev.push_back(ph.dev);
}

ppp_status check_ws(ppp_handle *h, void *ws, size_t bytes) {
    if (!ws) return fail(h, PPP_E_INVALID_ARG, "workspace is NULL");
    if ((uintptr_t)ws % kAlign != 0) return fail(h, PPP_E_INVALID_ARG, "workspace must be 256-byte aligned");
    if ((int64_t)bytes < h->ws_bytes) return fail(h, PPP_E_OUT_OF_MEMORY, "workspace smaller than ppp_workspace_size");
    return PPP_OK;
}

const DevProblem *d_probs(ppp_handle *h) { return reinterpret_cast<const DevProblem *>(h->ws + h->off_probs); }
const WorkItem *d_items(ppp_handle *h) { return reinterpret_cast<const WorkItem *>(h->ws + h->off_items); }

ppp_status upload(ppp_handle *h, hipStream_t st) {
    HIPCHK(h, hipMemcpyAsync(h->ws + h->off_probs, h->dev.data(), h->dev.size() * sizeof(DevProblem), hipMemcpyHostToDevice, st));
    if (!h->items.empty())
        HIPCHK(h, hipMemcpyAsync(h->ws + h->off_items, h->items.data(), h->items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, st));
    for (auto &ph : h->probs) {
        HIPCHK(h, hipMemcpyAsync(h->ws + ph.dev.off_lambda, ph.lambda.data(), ph.lambda.size() * 8, hipMemcpyHostToDevice, st));
        HIPCHK(h, hipMemcpyAsync(h->ws + ph.dev.off_init, ph.init.data(), ph.init.size() * 8, hipMemcpyHostToDevice, st));
    }
    // the descriptors live in pageable memory: make sure the copies are done before they change
    HIPCHK(h, hipStreamSynchronize(st));
    return PPP_OK;
}

ppp_status ensure_events(ppp_handle *h) {
    if (h->events_ok) return PPP_OK;
    for (auto &e : h->ev) HIPCHK(h, hipEventCreate(&e));
    h->events_ok = true;
    return PPP_OK;
}

// Records event i on st when the handle has its events (a run without them, the
// allocation-free entry point's on a fresh handle, takes no timings).
ppp_status mark(ppp_handle *h, int i, hipStream_t st) {
    if (h->events_ok) HIPCHK(h, hipEventRecord(h->ev[i], st));
    return PPP_OK;
}
#define MARK(h, i, st)                                   \
    do {                                                 \
        ppp_status m_ = mark((h), (i), (st));            \
        if (m_ != PPP_OK) return m_;                     \
    } while (0)

ppp_status launch_items(ppp_handle *h, const ProblemHost &ph, int64_t b, int64_t e, hipStream_t st, double *traj,
                        int64_t traj_rep, int first, int count) {
    const int64_t nk = (int64_t)ph.item_windows * ph.dev.xi_nbins;
    const int cap = nk <= kLdsHistCap ? (int)nk : 0;
    if (!ph.dev.sequential) {
        HIPCHK(h, launch_sim(d_probs(h), d_items(h) + first, count, h->ws, b, e, ph.dev.model, ph.dev.precision, ph.G,
                             ph.B, traj, traj_rep, cap, st));
        return PPP_OK;
    }
    // sequential protocol: one launch per window touched, so a launch never
    // crosses a window boundary (the kernel takes the window from its first step)
    const int64_t T = ph.dev.n_steps;
    int64_t at = b;
    do {
        const int64_t stop = std::min(e, (at / T + 1) * T);
        HIPCHK(h, launch_sim(d_probs(h), d_items(h) + first, count, h->ws, at, stop, ph.dev.model, ph.dev.precision,
                             ph.G, ph.B, traj, traj_rep, cap, st));
        at = stop;
    } while (at < e);
    return PPP_OK;
}

double ev_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return NAN;
    return (double)ms;
}

void put(double *dst, const std::vector<double> &src, int64_t at, int64_t n) {
    if (dst) std::memcpy(dst, src.data() + at, n * sizeof(double));
}
void put_i64(int64_t *dst, const std::vector<double> &src, int64_t at, int64_t n) {
    if (dst) for (int64_t i = 0; i < n; ++i) dst[i] = (int64_t)std::llround(src[at + i]);
}

ppp_status copy_result(ppp_handle *h, const ProblemHost &ph, ppp_result *out) {
    const DevProblem &d = ph.dev;
    const int64_t s = d.n_windows, K = d.xi_nbins;
    std::vector<double> o((size_t)O_NFIELDS * s);
    HIPCHK(h, hipMemcpy(o.data(), h->ws + d.off_out, o.size() * 8, hipMemcpyDeviceToHost));
    auto F = [&](int f) { return (int64_t)f * s; };
    put(out->dF_je, o, F(O_DF_JE), s);
    put(out->dF_je_se, o, F(O_DF_JE_SE), s);
    put(out->dF_fluct, o, F(O_DF_FLUCT), s);
    put(out->dF_fluct_se, o, F(O_DF_FLUCT_SE), s);
    put(out->dF_gauss, o, F(O_DF_GAUSS), s);
    put(out->dF_gauss_se, o, F(O_DF_GAUSS_SE), s);
    put(out->dF_com, o, F(O_DF_COM), s);
    put(out->dF_com_se, o, F(O_DF_COM_SE), s);
    put(out->dF_unc, o, F(O_DF_UNC), s);
    put(out->dF_rev, o, F(O_DF_REV), s);
    put(out->dF_fluct_literal, o, F(O_DF_FLUCT_LIT), s);
    put(out->sigma_lsq, o, F(O_SIGMA_LSQ), s);
    put(out->gamma2_lsq, o, F(O_GAMMA2_LSQ), s);
    put(out->dF_gauss_lsq, o, F(O_DF_GAUSS_LSQ), s);
    put(out->dF_gauss_literal, o, F(O_DF_GAUSS_LIT), s);
    const bool appc = d.w_half_bins > 0;
    if (appc) {
        put(out->dF_je_hist, o, F(O_DF_JE_HIST), s);
        put(out->dF_je_hist_mid, o, F(O_DF_JE_HIST_MID), s);
        put(out->dF_je_var_paper, o, F(O_VAR_PAPER), s);
        put(out->sigma_w, o, F(O_SIGMA_W), s);
        put_i64(out->q_bins, o, F(O_Q_BINS), s);
        put(out->work_lost, o, F(O_WORK_LOST), s);
        put(out->dF_je_hist_literal, o, F(O_DF_JE_HIST_LIT), s);
        put(out->dF_rev_hist, o, F(O_DF_REV_HIST), s);
        put(out->crooks_ovl, o, F(O_CROOKS_OVL), s);
        put(out->dF_crooks, o, F(O_DF_CROOKS), s);
    } else {
        for (double *p : {out->dF_je_hist, out->dF_je_hist_mid, out->dF_je_var_paper, out->sigma_w, out->work_lost,
                          out->dF_je_hist_literal, out->dF_rev_hist, out->crooks_ovl, out->dF_crooks})
            if (p) for (int64_t i = 0; i < s; ++i) p[i] = NAN;
        if (out->q_bins) for (int64_t i = 0; i < s; ++i) out->q_bins[i] = 0;
    }
    put(out->xi_mean, o, F(O_XI_MEAN), s);
    put(out->xi_std, o, F(O_XI_STD), s);
    put(out->gamma2, o, F(O_GAMMA2), s);
    put(out->xi_min_sample, o, F(O_XI_MINS), s);
    put(out->xi_max_sample, o, F(O_XI_MAXS), s);
    put(out->lse_fwd, o, F(O_LSE_FWD), s);
    put(out->lse_rev, o, F(O_LSE_REV), s);
    put_i64(out->n_samples, o, F(O_N_SAMPLES), s);
    put_i64(out->n_blown_up, o, F(O_N_BLOWN), s);
    put(out->kish_frac, o, F(O_KISH), s - 1);
    put(out->overlap_ovl, o, F(O_OVL), s - 1);
    put(out->dlambda_over_sigma, o, F(O_DL_SIGMA), s - 1);
    put(out->dlambda_over_reach, o, F(O_DL_REACH), s - 1);
    if (out->criterion_ok) for (int64_t i = 0; i + 1 < s; ++i) out->criterion_ok[i] = o[F(O_CRIT) + i] > 0.5 ? 1 : 0;
    if (out->xi_hist) HIPCHK(h, hipMemcpy(out->xi_hist, h->ws + d.off_hist, s * K * 8, hipMemcpyDeviceToHost));
    if (out->xi_under_over)
        for (int64_t i = 0; i < s; ++i) {
            out->xi_under_over[2 * i] = (uint64_t)std::llround(o[F(O_UNDER) + i]);
            out->xi_under_over[2 * i + 1] = (uint64_t)std::llround(o[F(O_OVER) + i]);
        }
    const int64_t nbw = s * (2 * (int64_t)d.w_half_bins + 1);
    if (out->work_hist && appc) HIPCHK(h, hipMemcpy(out->work_hist, h->ws + d.off_omega, nbw * 8, hipMemcpyDeviceToHost));
    if (out->work_hist_rev && appc)
        HIPCHK(h, hipMemcpy(out->work_hist_rev, h->ws + d.off_omega + 2 * nbw * 8, nbw * 8, hipMemcpyDeviceToHost));
    // the turn-on outputs (Eqs. 5-7, 10, 15)
    std::vector<double> turn(PPP_ON_NFIELDS, NAN);
    if (d.free_ens) HIPCHK(h, hipMemcpy(turn.data(), h->ws + d.off_turn, PPP_ON_NFIELDS * 8, hipMemcpyDeviceToHost));
    put(out->turn_on, turn, 0, PPP_ON_NFIELDS);
    put(out->G, o, F(O_G), s);
    put(out->G_se, o, F(O_G_SE), s);
    if (out->xi_hist_free) {
        if (d.free_ens) HIPCHK(h, hipMemcpy(out->xi_hist_free, h->ws + d.off_hist + s * K * 8, K * 8, hipMemcpyDeviceToHost));
        else std::memset(out->xi_hist_free, 0, K * 8);
    }
    // more than 1% of some window's replicas (the free ensemble's included) frozen?
    for (int64_t i = 0; i < s; ++i)
        if (o[F(O_N_BLOWN) + i] > 0.01 * d.n_replicas) return fail(h, PPP_E_NUMERICAL, "more than 1% of the replicas of a window were frozen");
    if (d.free_ens && turn[PPP_ON_FREE_BLOWN] > 0.01 * d.n_replicas)
        return fail(h, PPP_E_NUMERICAL, "more than 1% of the replicas of the free ensemble were frozen");
    return PPP_OK;
}

ppp_status do_begin(ppp_handle *h, void *ws, size_t bytes, hipStream_t st, bool timing = true) {
    ppp_status s = check_ws(h, ws, bytes);
    if (s != PPP_OK) return s;
    if (timing && (s = ensure_events(h)) != PPP_OK) return s;
    h->ws = static_cast<char *>(ws);
    h->stream = st;
    if ((s = upload(h, st)) != PPP_OK) return s;
    MARK(h, 0, st);
    HIPCHK(h, launch_init(d_probs(h), (int)h->probs.size(), h->ws, h->max_windows, h->max_k, h->max_m,
                          reinterpret_cast<int *>(h->ws + h->off_tickets), 64, st));
    // the first advance starts at step 0, where the kernel builds the initial state
    MARK(h, 1, st);
    h->begun = true; h->finalized = false; h->restored = false; h->steps_done = 0; h->sim_launches = 0;
    h->advanced = false;
    return PPP_OK;
}

ppp_status do_advance(ppp_handle *h, int64_t n, hipStream_t st) {
    if (!h->begun) return fail(h, PPP_E_STATE, "advance before begin");
    if (n < 0) return fail(h, PPP_E_INVALID_ARG, "n_steps must be >= 0");
    int64_t maxsteps = 0;
    for (auto &ph : h->probs) maxsteps = std::max(maxsteps, total_steps(ph));
    const int64_t e = std::min(maxsteps, h->steps_done + n);
    if (e <= h->steps_done) return PPP_OK;
    MARK(h, 5, st);
    for (auto &ph : h->probs) {
        const int64_t pe = std::min(e, total_steps(ph));
        if (pe <= h->steps_done) continue;
        ppp_status s = launch_items(h, ph, h->steps_done, pe, st, nullptr, -1, ph.first_item, ph.n_items);
        if (s != PPP_OK) return s;
    }
    MARK(h, 6, st);
    h->advanced = true;
    h->steps_done = e;
    h->sim_launches++;
    h->stream = st;
    return PPP_OK;
}

ppp_status do_finalize(ppp_handle *h, hipStream_t st) {
    if (!h->begun) return fail(h, PPP_E_STATE, "finalize before begin");
    for (auto &ph : h->probs) {
        if (h->steps_done == 0 && !h->restored) {
            // no step was taken: still build the initial state and empty accumulators
            ppp_status s = launch_items(h, ph, 0, 0, st, nullptr, -1, ph.first_item, ph.n_items);
            if (s != PPP_OK) return s;
        }
        if (ph.dev.sequential) {
            // windows the run has not entered yet get their (empty) accumulators
            for (int64_t w = 1; w < ph.dev.n_windows; ++w) {
                const int64_t at = w * ph.dev.n_steps;
                if (at < h->steps_done) continue;
                ppp_status s = launch_items(h, ph, at, at, st, nullptr, -1, ph.first_item, ph.n_items);
                if (s != PPP_OK) return s;
            }
        }
    }
    MARK(h, 2, st);
    HIPCHK(h, launch_reduce(d_probs(h), (int)h->probs.size(), h->ws, h->max_windows, h->max_blocks, st));
    HIPCHK(h, launch_estimators(d_probs(h), (int)h->probs.size(), h->ws, h->max_windows, st));
    MARK(h, 3, st);
    HIPCHK(h, launch_appc(d_probs(h), (int)h->probs.size(), h->ws, h->max_windows, h->max_m, st));
    MARK(h, 4, st);
    h->finalized = true;
    h->ran = true;
    h->stream = st;
    return PPP_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *ppp_status_string(ppp_status s) {
    switch (s) {
        case PPP_OK: return "ok";
        case PPP_E_INVALID_ARG: return "invalid argument";
        case PPP_E_OUT_OF_MEMORY: return "out of memory";
        case PPP_E_DEVICE: return "device error";
        case PPP_E_NUMERICAL: return "too many frozen replicas";
        case PPP_E_STATE: return "call out of order";
        case PPP_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *ppp_last_error(const ppp_handle *h) { return h ? h->err.c_str() : ""; }

static thread_local std::string g_create_err;
const char *ppp_create_error(void) { return g_create_err.c_str(); }


ppp_status ppp_create(const ppp_problem *p, ppp_handle **out) {
    if (!out) return PPP_E_INVALID_ARG;
    *out = nullptr;
    ppp_handle *h = new (std::nothrow) ppp_handle();
    if (!h) return PPP_E_OUT_OF_MEMORY;
    h->probs.resize(1);
    std::string msg;
    // an optional shape table (written by ppp_autotune) named by PPP_TUNE_TABLE
    ppp_status s = build_problem(p, h->probs[0], read_tune_table(std::getenv("PPP_TUNE_TABLE")), msg);
    if (s != PPP_OK) { g_create_err = msg; delete h; return s; }
    make_items(h->probs[0], 0, h->items, true);
    finish_layout(h);
    *out = h;
    return PPP_OK;
}

ppp_status ppp_batch_create(const ppp_problem *ps, int32_t n, const char *tune_table_path, ppp_handle **out) {
    if (!out) return PPP_E_INVALID_ARG;
    *out = nullptr;
    if (!ps || n < 1) { g_create_err = "need at least one problem"; return PPP_E_INVALID_ARG; }
    ppp_handle *h = new (std::nothrow) ppp_handle();
    if (!h) return PPP_E_OUT_OF_MEMORY;
    h->batch = true;
    const std::vector<TuneEntry> tune = read_tune_table(tune_table_path ? tune_table_path : std::getenv("PPP_TUNE_TABLE"));
    h->probs.resize(n);
    for (int i = 0; i < n; ++i) {
        std::string msg;
        ppp_status s = build_problem(&ps[i], h->probs[i], tune, msg);
        if (s == PPP_OK && ps[i].model != PPP_MODEL_CHAIN) { s = PPP_E_UNSUPPORTED; msg = "batched runs take chain problems"; }
        if (s == PPP_OK && (ps[i].flags & PPP_FLAG_SEQUENTIAL)) { s = PPP_E_UNSUPPORTED; msg = "batched runs use the parallel protocol"; }
        if (s != PPP_OK) { g_create_err = "problem " + std::to_string(i) + ": " + msg; delete h; return s; }
    }
    // group problems by kernel shape; inside a group order items longest first
    struct Key { int prec, G, B; };
    std::vector<Key> keys;
    for (auto &ph : h->probs) {
        bool found = false;
        for (auto &k : keys) if (k.prec == ph.dev.precision && k.G == ph.G && k.B == ph.B) found = true;
        if (!found) keys.push_back(Key{ph.dev.precision, ph.G, ph.B});
    }
    for (auto &k : keys) {
        VariantGroup g{k.prec, k.G, k.B, (int)h->items.size(), 0};
        std::vector<std::pair<double, WorkItem>> its;
        for (int i = 0; i < n; ++i) {
            ProblemHost &ph = h->probs[i];
            if (ph.dev.precision != k.prec || ph.G != k.G || ph.B != k.B) continue;
            std::vector<WorkItem> tmp;
            make_items(ph, i, tmp, false);
            const double npair = 0.5 * (double)ph.dev.n_beads * ph.dev.n_beads + 20.0 * ph.dev.n_beads;
            for (auto &it : tmp) its.push_back({npair * it.n_reps * (double)ph.dev.n_steps, it});
        }
        std::stable_sort(its.begin(), its.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
        for (auto &x : its) h->items.push_back(x.second);
        g.n_items = (int)h->items.size() - g.first_item;
        h->groups.push_back(g);
    }
    // per-problem item ranges are not contiguous in a batch; step-0 init uses the direct kernel per group
    for (auto &ph : h->probs) { ph.first_item = 0; ph.n_items = 0; }
    finish_layout(h);
    *out = h;
    return PPP_OK;
}

ppp_status ppp_workspace_size(const ppp_handle *h, size_t *bytes) {
    if (!h || !bytes) return PPP_E_INVALID_ARG;
    *bytes = (size_t)h->ws_bytes;
    return PPP_OK;
}

ppp_status ppp_begin(ppp_handle *h, void *ws, size_t bytes, void *stream) {
    if (!h) return PPP_E_INVALID_ARG;
    if (h->batch) return fail(h, PPP_E_UNSUPPORTED, "batched handles run with ppp_run");
    return do_begin(h, ws, bytes, (hipStream_t)stream);
}
ppp_status ppp_advance(ppp_handle *h, int64_t n, void *stream) {
    if (!h) return PPP_E_INVALID_ARG;
    if (h->batch) return fail(h, PPP_E_UNSUPPORTED, "batched handles run with ppp_run");
    return do_advance(h, n, (hipStream_t)stream);
}
ppp_status ppp_finalize(ppp_handle *h, void *stream) {
    if (!h) return PPP_E_INVALID_ARG;
    if (h->batch) return fail(h, PPP_E_UNSUPPORTED, "batched handles run with ppp_run");
    return do_finalize(h, (hipStream_t)stream);
}
ppp_status ppp_steps_done(const ppp_handle *h, int64_t *steps) {
    if (!h || !steps) return PPP_E_INVALID_ARG;
    *steps = h->steps_done;
    return PPP_OK;
}

static ppp_status batch_capture(ppp_handle *h) {
    // one graph: init -> (fork) one persistent kernel per shape group -> (join) -> reductions, estimators, App. C
    if (!h->cap) HIPCHK(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    while (h->side.size() < h->groups.size()) {
        hipStream_t s;
        HIPCHK(h, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        h->side.push_back(s);
    }
    while (h->side_ev.size() < h->groups.size() + 1) {
        hipEvent_t e;
        HIPCHK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->side_ev.push_back(e);
    }
    int cus = 0, dev = 0;
    HIPCHK(h, hipGetDevice(&dev));
    HIPCHK(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    int *tickets = reinterpret_cast<int *>(h->ws + h->off_tickets);
    hipError_t e = launch_init(d_probs(h), (int)h->probs.size(), h->ws, h->max_windows, h->max_k, h->max_m, tickets, 64, h->cap);
    // the persistent kernels start every item at step 0, where its initial state is built
    if (e == hipSuccess) e = hipEventRecord(h->side_ev[0], h->cap);
    for (size_t gi = 0; gi < h->groups.size() && e == hipSuccess; ++gi) {
        const VariantGroup &g = h->groups[gi];
        e = hipStreamWaitEvent(h->side[gi], h->side_ev[0], 0);
        int kmax = 0;
        for (auto &ph : h->probs)
            if (ph.dev.precision == g.precision && ph.G == g.G && ph.B == g.B) kmax = std::max(kmax, ph.dev.xi_nbins);
        const int cap = kmax <= kLdsHistCap ? kmax : 0;
        const int per_cu = std::max(1, sim_blocks_per_cu(g.precision, g.G, g.B, cap));
        const int groups = std::min(g.n_items, std::max(1, per_cu * cus));
        if (e == hipSuccess) e = launch_sim_persistent(d_probs(h), d_items(h) + g.first_item, g.n_items, tickets + gi, h->ws, g.precision, g.G, g.B, groups, cap, h->side[gi]);
        if (e == hipSuccess) e = hipEventRecord(h->side_ev[gi + 1], h->side[gi]);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->cap, h->side_ev[gi + 1], 0);
    }
    if (e == hipSuccess) e = launch_reduce(d_probs(h), (int)h->probs.size(), h->ws, h->max_windows, h->max_blocks, h->cap);
    if (e == hipSuccess) e = launch_estimators(d_probs(h), (int)h->probs.size(), h->ws, h->max_windows, h->cap);
    if (e == hipSuccess) e = launch_appc(d_probs(h), (int)h->probs.size(), h->ws, h->max_windows, h->max_m, h->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(h->cap, &g);
    if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_fail(h, e, "batch capture"); }
    if (e2 != hipSuccess) return hip_fail(h, e2, "hipStreamEndCapture");
    if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
    if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
    h->graph = g;
    HIPCHK(h, hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
    h->graph_ws = h->ws;
    return PPP_OK;
}

ppp_status ppp_run(ppp_handle *h, void *ws, size_t bytes, void *stream) {
    if (!h) return PPP_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    ppp_status s;
    if (!h->batch) {
        if ((s = do_begin(h, ws, bytes, st)) != PPP_OK) return s;
        if ((s = do_advance(h, INT64_MAX / 4, st)) != PPP_OK) return s;
        return do_finalize(h, st);
    }
    if ((s = check_ws(h, ws, bytes)) != PPP_OK) return s;
    if ((s = ensure_events(h)) != PPP_OK) return s;
    h->ws = static_cast<char *>(ws);
    h->stream = st;
    if (h->graph_ws != h->ws || !h->gexec) {
        if ((s = upload(h, st)) != PPP_OK) return s;
        if ((s = batch_capture(h)) != PPP_OK) return s;
    }
    HIPCHK(h, hipEventRecord(h->ev[0], st));
    HIPCHK(h, hipEventRecord(h->ev[1], st));
    HIPCHK(h, hipGraphLaunch(h->gexec, st));
    HIPCHK(h, hipEventRecord(h->ev[2], st));
    HIPCHK(h, hipEventRecord(h->ev[3], st));
    HIPCHK(h, hipEventRecord(h->ev[4], st));
    int64_t mx = 0;
    for (auto &ph : h->probs) mx = std::max(mx, ph.dev.n_steps);
    h->steps_done = mx;
    h->sim_launches = 1;
    h->begun = true; h->finalized = true; h->ran = true;
    return PPP_OK;
}

ppp_status ppp_get_result(ppp_handle *h, ppp_result *out) {
    if (!h || !out) return PPP_E_INVALID_ARG;
    if (h->batch) return fail(h, PPP_E_INVALID_ARG, "use ppp_batch_get_result for batched handles");
    return ppp_batch_get_result(h, 0, out);
}

ppp_status ppp_batch_get_result(ppp_handle *h, int32_t index, ppp_result *out) {
    if (!h || !out) return PPP_E_INVALID_ARG;
    if (index < 0 || index >= (int)h->probs.size()) return fail(h, PPP_E_INVALID_ARG, "problem index out of range");
    if (!h->finalized) return fail(h, PPP_E_STATE, "no finished run");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return copy_result(h, h->probs[index], out);
}

ppp_status ppp_get_timings(const ppp_handle *hc, ppp_timings *out) {
    ppp_handle *h = const_cast<ppp_handle *>(hc);
    if (!h || !out) return PPP_E_INVALID_ARG;
    if (!h->ran) return fail(h, PPP_E_STATE, "no finished run");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    std::memset(out, 0, sizeof(*out));
    if (h->batch) {
        out->sim_ms = ev_ms(h->ev[1], h->ev[2]);
        out->reduce_ms = 0; out->appc_ms = 0;
    } else {
        out->sim_ms = ev_ms(h->ev[1], h->ev[2]);
        out->reduce_ms = ev_ms(h->ev[2], h->ev[3]);
        out->appc_ms = ev_ms(h->ev[3], h->ev[4]);
    }
    out->total_ms = ev_ms(h->ev[0], h->ev[4]);
    out->last_advance_ms = h->advanced && !h->batch ? ev_ms(h->ev[5], h->ev[6]) : NAN;
    int64_t rs = 0;
    for (auto &ph : h->probs)
        rs += ph.dev.sequential ? (int64_t)ph.dev.n_replicas * std::min(total_steps(ph), h->steps_done)
                                : (int64_t)ph.dev.n_sim_windows * ph.dev.n_replicas * std::min(ph.dev.n_steps, h->steps_done);
    out->replica_steps = rs;
    out->sim_launches = h->sim_launches;
    out->variant_lanes = h->probs[0].G;
    out->variant_beads_per_lane = h->probs[0].B;
    return PPP_OK;
}

// checkpoint format: magic, steps_done, then for each problem its state, accumulator and histogram bytes
static const uint64_t kMagic = 0x3150504350504350ull;

ppp_status ppp_checkpoint(ppp_handle *h, void *host_buf, size_t *bytes) {
    if (!h || !bytes) return PPP_E_INVALID_ARG;
    if (h->batch) return fail(h, PPP_E_UNSUPPORTED, "checkpoint of batched handles");
    size_t need = 16;
    for (auto &ph : h->probs) need += (size_t)(ph.dev.off_hist + (int64_t)ph.dev.n_sim_windows * ph.dev.xi_nbins * 8 - ph.dev.off_state);
    if (!host_buf) { *bytes = need; return PPP_OK; }
    if (*bytes < need) return fail(h, PPP_E_INVALID_ARG, "checkpoint buffer too small");
    if (!h->begun) return fail(h, PPP_E_STATE, "nothing to checkpoint");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    char *p = static_cast<char *>(host_buf);
    std::memcpy(p, &kMagic, 8);
    std::memcpy(p + 8, &h->steps_done, 8);
    size_t at = 16;
    for (auto &ph : h->probs) {
        const size_t n = (size_t)(ph.dev.off_hist + (int64_t)ph.dev.n_sim_windows * ph.dev.xi_nbins * 8 - ph.dev.off_state);
        HIPCHK(h, hipMemcpy(p + at, h->ws + ph.dev.off_state, n, hipMemcpyDeviceToHost));
        at += n;
    }
    *bytes = need;
    return PPP_OK;
}

ppp_status ppp_restore(ppp_handle *h, void *ws, size_t ws_bytes, const void *host_buf, size_t bytes, void *stream) {
    if (!h || !host_buf) return PPP_E_INVALID_ARG;
    if (h->batch) return fail(h, PPP_E_UNSUPPORTED, "restore of batched handles");
    size_t need = 16;
    for (auto &ph : h->probs) need += (size_t)(ph.dev.off_hist + (int64_t)ph.dev.n_sim_windows * ph.dev.xi_nbins * 8 - ph.dev.off_state);
    if (bytes != need) return fail(h, PPP_E_INVALID_ARG, "checkpoint size does not match this problem");
    const char *p = static_cast<const char *>(host_buf);
    uint64_t magic;
    std::memcpy(&magic, p, 8);
    if (magic != kMagic) return fail(h, PPP_E_INVALID_ARG, "not a checkpoint");
    ppp_status s = check_ws(h, ws, ws_bytes);
    if (s != PPP_OK) return s;
    if ((s = ensure_events(h)) != PPP_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    h->ws = static_cast<char *>(ws);
    h->stream = st;
    if ((s = upload(h, st)) != PPP_OK) return s;
    HIPCHK(h, hipEventRecord(h->ev[0], st));
    HIPCHK(h, launch_init(d_probs(h), (int)h->probs.size(), h->ws, h->max_windows, h->max_k, h->max_m,
                          reinterpret_cast<int *>(h->ws + h->off_tickets), 64, st));
    size_t at = 16;
    for (auto &ph : h->probs) {
        const size_t n = (size_t)(ph.dev.off_hist + (int64_t)ph.dev.n_sim_windows * ph.dev.xi_nbins * 8 - ph.dev.off_state);
        HIPCHK(h, hipMemcpyAsync(h->ws + ph.dev.off_state, p + at, n, hipMemcpyHostToDevice, st));
        at += n;
    }
    HIPCHK(h, hipStreamSynchronize(st));
    HIPCHK(h, hipEventRecord(h->ev[1], st));
    std::memcpy(&h->steps_done, p + 8, 8);
    h->begun = true; h->finalized = false; h->restored = true; h->sim_launches = 0;
    return PPP_OK;
}

ppp_status ppp_destroy(ppp_handle *h) {
    if (!h) return PPP_OK;
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    for (auto s : h->side) (void)hipStreamDestroy(s);
    for (auto e : h->side_ev) (void)hipEventDestroy(e);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->events_ok) for (auto e : h->ev) (void)hipEventDestroy(e);
    delete h;
    return PPP_OK;
}

ppp_status ppp_eval_forces(ppp_handle *h, void *ws, size_t bytes, const double *d_coords, int32_t n_rep, double lambda,
                           double *d_forces, double *d_energy, void *stream) {
    if (!h) return PPP_E_INVALID_ARG;
    if (h->batch) return fail(h, PPP_E_UNSUPPORTED, "use a single-problem handle");
    if (!d_coords || !d_forces || !d_energy || n_rep < 0 || !std::isfinite(lambda)) return fail(h, PPP_E_INVALID_ARG, "bad arguments");
    ppp_status s = check_ws(h, ws, bytes);
    if (s != PPP_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    h->ws = static_cast<char *>(ws);
    if ((s = upload(h, st)) != PPP_OK) return s;
    const ProblemHost &ph = h->probs[0];
    HIPCHK(h, launch_eval(d_probs(h), d_coords, n_rep, lambda, d_forces, d_energy, ph.dev.model, ph.dev.precision, ph.G, ph.B, st));
    h->begun = false; h->finalized = false;
    return PPP_OK;
}

ppp_status ppp_trajectory(ppp_handle *h, void *ws, size_t bytes, int32_t window, int32_t replica, int32_t n_steps,
                          double *d_out, void *stream) {
    if (!h) return PPP_E_INVALID_ARG;
    if (h->batch) return fail(h, PPP_E_UNSUPPORTED, "use a single-problem handle");
    const ProblemHost &ph = h->probs[0];
    if (ph.dev.sequential) return fail(h, PPP_E_UNSUPPORTED, "trajectories are recorded for the parallel protocol");
    if (window < 0 || window >= ph.dev.n_windows || replica < 0 || replica >= ph.dev.n_replicas || !d_out)
        return fail(h, PPP_E_INVALID_ARG, "window/replica out of range");
    if (n_steps < 1 || n_steps > 100000 || n_steps > ph.dev.n_steps) return fail(h, PPP_E_INVALID_ARG, "n_steps out of range");
    ppp_status s = check_ws(h, ws, bytes);
    if (s != PPP_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    h->ws = static_cast<char *>(ws);
    if ((s = upload(h, st)) != PPP_OK) return s;
    HIPCHK(h, launch_init(d_probs(h), 1, h->ws, h->max_windows, h->max_k, h->max_m, reinterpret_cast<int *>(h->ws + h->off_tickets), 64, st));
    const int64_t gid = (int64_t)window * ph.dev.n_replicas + replica;
    int item = -1;
    for (int i = ph.first_item; i < ph.first_item + ph.n_items && item < 0; ++i) {
        const WorkItem &it = h->items[i];
        const int64_t g0 = (int64_t)it.window * ph.dev.n_replicas + it.rep_begin;
        if (gid >= g0 && gid < g0 + it.n_reps) item = i;
    }
    if (item < 0) return fail(h, PPP_E_INVALID_ARG, "replica not in any work item");
    if ((s = launch_items(h, ph, 0, n_steps, st, d_out, gid, item, 1)) != PPP_OK) return s;
    h->begun = false; h->finalized = false;
    return PPP_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: for each chain-length bucket, time every compiled shape that holds
// the chain on a synthetic problem sized to fill the GPU, keep the fastest.
// ---------------------------------------------------------------------------
ppp_status ppp_autotune(const char *path, void *ws, size_t bytes, void *stream) {
    if (!path || !ws) return PPP_E_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    static const int kBuckets[] = {4, 8, 10, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
    static const int kShapes[][2] = {
#define PPP_LIST(GG, BB) {GG, BB},
        PPP_FOR_EACH_SHAPE_RT(PPP_LIST)
#undef PPP_LIST
    };
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PPP_E_DEVICE;
    std::ostringstream table;
    table << "# nmax precision lanes beads_per_lane   (ppp_autotune: fastest measured shape per chain length)\n";
    ppp_status result = PPP_OK;
    for (int prec = 0; prec <= 1 && result == PPP_OK; ++prec) {
        for (int N : kBuckets) {
            double best = 1e300; int bG = 0, bB = 0;
            for (const auto &sh : kShapes) {
                const int G = sh[0], B = sh[1];
                if (G * B < N || G * B > 4 * N + 8) continue;
                std::vector<double> lam(8);
                for (int i = 0; i < 8; ++i) lam[i] = 0.35 * (N - 1) + 0.05 * i;
                ppp_problem p{};
                p.model = PPP_MODEL_CHAIN;
                p.chain = ppp_chain{N, 100.0, 1.0, 5.0, 1.0, 1.0, 2.5, 0, 1.0, 1.0};
                p.n_windows = 8; p.lambda = lam.data();
                p.k = 20.0; p.kT = 1.0; p.dt = 0.005;
                p.n_steps = N >= 256 ? 60 : (N >= 64 ? 200 : 600);
                p.n_equil = p.n_steps / 2; p.sample_every = 10;
                // enough replicas for about eight waves per SIMD of the whole chip
                const int64_t lanes = (int64_t)cus * 4 * 64 * 8;
                p.n_replicas = (int)std::max<int64_t>(64, std::min<int64_t>(16384, lanes / G / 8));
                if (N >= 256) p.n_replicas = std::min(p.n_replicas, 2048);
                p.seed = 7; p.precision = (ppp_precision)prec;
                p.xi_min = 0.0; p.xi_bin = 0.01 * N; p.xi_nbins = 128; p.w_half_bins = 0; p.n_jack_blocks = 8;
                ppp_handle *h = new ppp_handle();
                h->probs.resize(1);
                std::string msg;
                std::vector<TuneEntry> force{TuneEntry{N, prec, G, B}};
                if (build_problem(&p, h->probs[0], force, msg) != PPP_OK || h->probs[0].G != G || h->probs[0].B != B) { delete h; continue; }
                make_items(h->probs[0], 0, h->items, true);
                finish_layout(h);
                if (h->ws_bytes > (int64_t)bytes) { delete h; continue; }
                ppp_status s2 = do_begin(h, ws, bytes, st);
                if (s2 == PPP_OK && hipEventRecord(e0, st) != hipSuccess) s2 = PPP_E_DEVICE;
                if (s2 == PPP_OK) s2 = do_advance(h, p.n_steps, st);
                if (s2 == PPP_OK && hipEventRecord(e1, st) != hipSuccess) s2 = PPP_E_DEVICE;
                if (s2 == PPP_OK && hipEventSynchronize(e1) != hipSuccess) s2 = PPP_E_DEVICE;
                if (s2 != PPP_OK) { ppp_destroy(h); result = s2; break; }
                const double t = ev_ms(e0, e1) / ((double)p.n_windows * p.n_replicas * p.n_steps);
                ppp_destroy(h);
                if (t < best) { best = t; bG = G; bB = B; }
            }
            if (result != PPP_OK) break;
            if (bG > 0) table << N << " " << prec << " " << bG << " " << bB << "   # " << best * 1e6 << " ns per replica-step\n";
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != PPP_OK) return result;
    std::ofstream f(path);
    if (!f) return PPP_E_INVALID_ARG;
    f << table.str();
    return f ? PPP_OK : PPP_E_INVALID_ARG;
}

ppp_status ppp_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int32_t n, uint32_t *d_words,
                      double *d_normals, float *d_normals32, double *d_normals6, float *d_normals6_32, void *stream) {
    if (n < 0) return PPP_E_INVALID_ARG;
    hipError_t e = launch_philox(seed, c0, c1, c2, c3, n, d_words, d_normals, d_normals32, d_normals6, d_normals6_32,
                                 (hipStream_t)stream);
    return e == hipSuccess ? PPP_OK : PPP_E_DEVICE;
}

ppp_status ppp_probe_valu(int32_t n_blocks, int32_t iters, float b, float c, int32_t operands, float *d_out,
                          void *stream) {
    if (n_blocks < 1 || iters < 1 || !d_out) return PPP_E_INVALID_ARG;
    if (operands != PPP_PROBE_SGPR_OPERANDS && operands != PPP_PROBE_VGPR_OPERANDS) return PPP_E_INVALID_ARG;
    hipError_t e = launch_valu_probe(n_blocks, iters, b, c, operands == PPP_PROBE_VGPR_OPERANDS, d_out,
                                     (hipStream_t)stream);
    return e == hipSuccess ? PPP_OK : PPP_E_DEVICE;
}

}  // extern "C"

// ===========================================================================
// Internal entry points for the adaptive protocol (ppp_adaptive.cpp).
// ===========================================================================
namespace ppp {

void set_error(ppp_handle *h, const std::string &msg) {
    if (h) h->err = msg;
}

ppp_status run_without_allocation(ppp_handle *h, void *ws, size_t bytes, void *stream) {
    if (!h) return PPP_E_INVALID_ARG;
    if (h->batch) return fail(h, PPP_E_UNSUPPORTED, "the allocation-free run takes single-problem handles");
    if ((int64_t)bytes < h->ws_bytes)
        return fail(h, PPP_E_OUT_OF_MEMORY, "problem needs " + std::to_string(h->ws_bytes) +
                                                " workspace bytes, above the static workspace of " +
                                                std::to_string(bytes));
    hipStream_t st = (hipStream_t)stream;
    ppp_status s;
    if ((s = do_begin(h, ws, bytes, st, false)) != PPP_OK) return s;
    if ((s = do_advance(h, INT64_MAX / 4, st)) != PPP_OK) return s;
    return do_finalize(h, st);
}

size_t workspace_bytes_for(const ppp_problem *p) {
    ppp_handle *h = nullptr;
    if (ppp_create(p, &h) != PPP_OK) return 0;
    const size_t n = (size_t)h->ws_bytes;
    ppp_destroy(h);
    return n;
}

}  // namespace ppp

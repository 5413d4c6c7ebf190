// Learned window placement: the surrogate's C entry points and the adaptive
// protocol (exploration rounds, surrogate training on the GPU, placement by
// the adjacent-overlap criterion, one production run).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "ppp.h"
#include "ppp_internal_api.hpp"
#include "ppp_launch.hpp"

using namespace ppp;

namespace {

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr int kGrid = 1025;          // surrogate evaluation grid over the lambda range
constexpr int kMaxTrain = 4096;      // points per gradient launch

struct MlpBuffers {
    float *params, *grad, *m, *v, *loss;
    float *t, *yv, *wv, *ys, *ws;    // training data [kMaxTrain]
    float *gt, *gy, *gdy;            // grid evaluation [kGrid]
};

int64_t mlp_bytes() {
    int64_t b = 0;
    b += 4 * align_up(PPP_MLP_PARAMS * 4) + align_up(4);
    b += 5 * align_up(kMaxTrain * 4);
    b += 3 * align_up(kGrid * 4);
    return b;
}

MlpBuffers carve(char *p) {
    MlpBuffers m{};
    auto take = [&](int64_t bytes) { float *r = reinterpret_cast<float *>(p); p += align_up(bytes); return r; };
    m.params = take(PPP_MLP_PARAMS * 4); m.grad = take(PPP_MLP_PARAMS * 4);
    m.m = take(PPP_MLP_PARAMS * 4); m.v = take(PPP_MLP_PARAMS * 4); m.loss = take(4);
    m.t = take(kMaxTrain * 4); m.yv = take(kMaxTrain * 4); m.wv = take(kMaxTrain * 4);
    m.ys = take(kMaxTrain * 4); m.ws = take(kMaxTrain * 4);
    m.gt = take(kGrid * 4); m.gy = take(kGrid * 4); m.gdy = take(kGrid * 4);
    return m;
}

bool valid_adaptive(const ppp_problem *b, const ppp_adaptive *a) {
    if (!b || !a) return false;
    if (a->budget_replica_steps <= 0 || a->initial_windows < 2 || a->max_rounds < 1) return false;
    if (a->max_windows < a->initial_windows || a->max_windows > 2048) return false;
    if (!(a->target_dl_over_sigma > 0) || a->train_iters < 0 || !(a->lr > 0)) return false;
    if (a->explore_replicas < 0 || a->explore_steps < 0 || a->min_production_steps < 0) return false;
    if (a->placement != PPP_PLACE_LEARNED && a->placement != PPP_PLACE_EXPLORED) return false;
    return b->n_windows >= 2 && b->lambda && std::isfinite(b->lambda[0]) && std::isfinite(b->lambda[b->n_windows - 1]) &&
           b->lambda[0] != b->lambda[b->n_windows - 1];
}

// One protocol run on windows `lam` with the given replicas and steps; fills res arrays.
struct RunOut {
    std::vector<double> mean, sd, dF_je, kish;
};

ppp_status run_windows(const ppp_problem *base, const std::vector<double> &lam, int32_t reps, int64_t steps,
                       void *ws, size_t bytes, hipStream_t st, ppp_result *full, RunOut *ro) {
    ppp_problem p = *base;
    p.n_windows = (int32_t)lam.size();
    p.lambda = lam.data();
    p.n_replicas = reps;
    const double ef = base->n_steps > 0 ? (double)base->n_equil / (double)base->n_steps : 0.1;
    const double pf = base->n_steps > 0 ? (double)base->n_pull / (double)base->n_steps : 0.0;
    p.n_steps = steps;
    p.n_equil = std::min<int64_t>(steps - 1, (int64_t)(ef * steps));
    p.n_pull = (int64_t)(pf * steps);
    ppp_handle *h = nullptr;
    ppp_status s = ppp_create(&p, &h);
    if (s != PPP_OK) return s;
    s = ppp_run(h, ws, bytes, st);
    if (s == PPP_OK && full) s = ppp_get_result(h, full);
    if ((s == PPP_OK || s == PPP_E_NUMERICAL) && ro) {
        const size_t n = lam.size();
        ro->mean.assign(n, NAN); ro->sd.assign(n, NAN); ro->dF_je.assign(n, NAN); ro->kish.assign(n, NAN);
        ppp_result r{};
        r.xi_mean = ro->mean.data(); r.xi_std = ro->sd.data(); r.dF_je = ro->dF_je.data(); r.kish_frac = ro->kish.data();
        s = ppp_get_result(h, &r);
    }
    ppp_destroy(h);
    return s;
}

// Glorot-style uniform initial weights, zero biases (host, then copied to the device).
std::vector<float> init_params(uint64_t seed) {
    std::mt19937_64 g(seed);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    std::vector<float> p(PPP_MLP_PARAMS, 0.f);
    const int H = PPP_MLP_HIDDEN;
    for (int i = 0; i < H; ++i) p[i] = (float)(u(g) * std::sqrt(6.0 / (1 + H)));
    for (int i = 0; i < H * H; ++i) p[2 * H + i] = (float)(u(g) * std::sqrt(6.0 / (2 * H)));
    for (int i = 0; i < H; ++i) p[3 * H + H * H + i] = (float)(u(g) * std::sqrt(6.0 / (H + 1)));
    return p;
}

}  // namespace

extern "C" {

ppp_status ppp_mlp_forward(const float *d_params, const float *d_t, int32_t n, float *d_y, float *d_dy, void *stream) {
    if (n < 0 || (n > 0 && (!d_params || !d_t || !d_y))) return PPP_E_INVALID_ARG;
    return launch_mlp_forward(d_params, d_t, n, d_y, d_dy, (hipStream_t)stream) == hipSuccess ? PPP_OK : PPP_E_DEVICE;
}

ppp_status ppp_mlp_grad(const float *d_params, const float *d_t, const float *d_yv, const float *d_wv, const float *d_ys,
                        const float *d_ws, int32_t n, float *d_grad, float *d_loss, void *stream) {
    if (n < 1 || n > kMaxTrain || !d_params || !d_t || !d_yv || !d_wv || !d_ys || !d_ws || !d_grad) return PPP_E_INVALID_ARG;
    return launch_mlp_grad(d_params, d_t, d_yv, d_wv, d_ys, d_ws, n, d_grad, d_loss, (hipStream_t)stream) == hipSuccess
               ? PPP_OK : PPP_E_DEVICE;
}

ppp_status ppp_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, float lr, int32_t step,
                        void *stream) {
    if (!d_params || !d_grad || !d_m || !d_v || step < 1 || !(lr > 0.f)) return PPP_E_INVALID_ARG;
    return launch_mlp_adam(d_params, d_grad, d_m, d_v, lr, step, (hipStream_t)stream) == hipSuccess ? PPP_OK
                                                                                                    : PPP_E_DEVICE;
}

ppp_status ppp_adaptive_workspace_size(const ppp_problem *base, const ppp_adaptive *a, size_t *bytes) {
    if (!bytes || !valid_adaptive(base, a)) return PPP_E_INVALID_ARG;
    // placement runs the parallel protocol on restrained windows only
    if (base->flags & (PPP_FLAG_SEQUENTIAL | PPP_FLAG_FREE_ENSEMBLE)) return PPP_E_UNSUPPORTED;
    // the largest run: max_windows windows with the production replica count
    std::vector<double> lam(a->max_windows);
    const double lo = base->lambda[0], hi = base->lambda[base->n_windows - 1];
    for (int i = 0; i < a->max_windows; ++i) lam[i] = lo + (hi - lo) * i / (a->max_windows - 1);
    ppp_problem p = *base;
    p.n_windows = a->max_windows;
    p.lambda = lam.data();
    const size_t run = workspace_bytes_for(&p);
    if (run == 0) return PPP_E_INVALID_ARG;
    *bytes = (size_t)align_up((int64_t)run) + (size_t)mlp_bytes();
    return PPP_OK;
}

ppp_status ppp_adaptive_run(const ppp_problem *base, const ppp_adaptive *a, void *d_ws, size_t bytes, void *stream,
                            double *lambda_out, int32_t *n_windows_out, int64_t *used_out, ppp_result *out) {
    if (!valid_adaptive(base, a) || !d_ws || !lambda_out || !n_windows_out || !out) return PPP_E_INVALID_ARG;
    size_t need = 0;
    ppp_status s = ppp_adaptive_workspace_size(base, a, &need);
    if (s != PPP_OK) return s;
    if (bytes < need) return PPP_E_OUT_OF_MEMORY;
    hipStream_t st = (hipStream_t)stream;
    const size_t run_bytes = need - (size_t)mlp_bytes();
    char *ws = static_cast<char *>(d_ws);
    MlpBuffers mb = carve(ws + run_bytes);

    const double lo = base->lambda[0], hi = base->lambda[base->n_windows - 1];
    const double centre = 0.5 * (lo + hi), half = 0.5 * (hi - lo);       // t = (lambda - centre) / half
    const double span = std::fabs(hi - lo);
    const double k = base->k, kT = base->kT, beta = 1.0 / kT;
    const int32_t Re = a->explore_replicas > 0 ? a->explore_replicas : std::max(1, base->n_replicas / 8);
    const int64_t ne = a->explore_steps > 0 ? a->explore_steps : std::max<int64_t>(100, base->n_steps / 4);
    const int64_t cost_e = (int64_t)Re * ne;
    int64_t used = 0;

    std::vector<double> xl, xs, xsd;   // explored windows: lambda, slope k (lambda - <x>), sigma_i
    std::vector<double> vl, vF, vw;    // value targets from the first round's JE chain
    std::vector<double> placed;        // latest placement
    std::vector<double> fresh(a->initial_windows);
    for (int i = 0; i < a->initial_windows; ++i) fresh[i] = lo + (hi - lo) * i / (a->initial_windows - 1);

    std::vector<float> p0 = init_params(a->init_seed);
    std::vector<float> zeros(PPP_MLP_PARAMS, 0.f);
    if (hipMemcpy(mb.params, p0.data(), p0.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mb.m, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mb.v, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return PPP_E_DEVICE;
    int adam_step = 0;
    double Fs = 1.0;
    bool trained = false;

    for (int round = 0; round < a->max_rounds && !fresh.empty(); ++round) {
        // exploration budget: at most half of the total
        const int64_t room = (a->budget_replica_steps / 2 - used) / cost_e;
        if (room < 2) break;
        if ((int64_t)fresh.size() > room) fresh.resize(room);
        if (fresh.size() < 2) break;          // a single unexplored window: the placement has settled
        std::sort(fresh.begin(), fresh.end());
        if (hi < lo) std::reverse(fresh.begin(), fresh.end());
        RunOut ro;
        s = run_windows(base, fresh, Re, ne, ws, run_bytes, st, nullptr, &ro);
        if (s != PPP_OK && s != PPP_E_NUMERICAL) return s;
        used += (int64_t)fresh.size() * cost_e;
        for (size_t i = 0; i < fresh.size(); ++i) {
            if (!std::isfinite(ro.mean[i])) continue;
            xl.push_back(fresh[i]);
            xs.push_back(k * (fresh[i] - ro.mean[i]));      // dF/dlambda, Eq. 14 in the small-step limit
            xsd.push_back(ro.sd[i]);
        }
        if (round == 0) {
            double wmin = 1.0;
            for (size_t i = 0; i < fresh.size(); ++i) {
                if (i > 0 && std::isfinite(ro.kish[i - 1])) wmin = std::min(wmin, std::max(ro.kish[i - 1], 0.0));
                if (!std::isfinite(ro.dF_je[i])) break;
                vl.push_back(fresh[i]); vF.push_back(ro.dF_je[i]); vw.push_back(i == 0 ? 1.0 : wmin);
            }
        }
        const double dl = (hi - lo) / (kGrid - 1);
        const double s2_free = kT / k;
        std::vector<double> sig(kGrid);
        if (a->placement == PPP_PLACE_EXPLORED) {
            // ---- no network: sigma(lambda) through the explored windows' sample sigma_i ----
            std::vector<std::pair<double, double>> pts;
            for (size_t i = 0; i < xl.size(); ++i)
                if (std::isfinite(xsd[i]) && xsd[i] > 0) pts.push_back({(xl[i] - lo) / dl, xsd[i]});
            if (pts.size() < 2) break;            // uniform fallback below
            std::sort(pts.begin(), pts.end());
            size_t j = 0;
            for (int i = 0; i < kGrid; ++i) {
                while (j + 2 < pts.size() && pts[j + 1].first <= i) ++j;
                const double x0 = pts[j].first, x1 = pts[j + 1].first;
                const double f = x1 > x0 ? std::min(1.0, std::max(0.0, (i - x0) / (x1 - x0))) : 0.0;
                const double sd = pts[j].second * (1 - f) + pts[j + 1].second * f;
                sig[i] = std::sqrt(std::min(std::max(sd * sd, 0.05 * s2_free), 100.0 * s2_free));
            }
            trained = true;
        } else {
        // ---- train the surrogate on all window data ----
        double smax = 0.0, fmax = 1.0;
        for (double v : xs) smax = std::max(smax, std::fabs(v) * std::fabs(half));
        for (double v : vF) fmax = std::max(fmax, std::fabs(v));
        Fs = std::max(fmax, smax);
        const int nd = (int)std::min<size_t>(kMaxTrain, xl.size() + vl.size());
        std::vector<float> t(nd), yv(nd, 0.f), wv(nd, 0.f), ys(nd, 0.f), wsl(nd, 0.f);
        int q = 0;
        for (size_t i = 0; i < xl.size() && q < nd; ++i, ++q) {
            t[q] = (float)((xl[i] - centre) / half); ys[q] = (float)(xs[i] * half / Fs); wsl[q] = 1.f;
        }
        for (size_t i = 0; i < vl.size() && q < nd; ++i, ++q) {
            t[q] = (float)((vl[i] - centre) / half); yv[q] = (float)(vF[i] / Fs); wv[q] = (float)vw[i];
        }
        if (hipMemcpy(mb.t, t.data(), nd * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(mb.yv, yv.data(), nd * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(mb.wv, wv.data(), nd * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(mb.ys, ys.data(), nd * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(mb.ws, wsl.data(), nd * 4, hipMemcpyHostToDevice) != hipSuccess)
            return PPP_E_DEVICE;
        for (int it = 0; it < a->train_iters; ++it) {
            if (launch_mlp_grad(mb.params, mb.t, mb.yv, mb.wv, mb.ys, mb.ws, nd, mb.grad, mb.loss, st) != hipSuccess ||
                launch_mlp_adam(mb.params, mb.grad, mb.m, mb.v, (float)a->lr, ++adam_step, st) != hipSuccess)
                return PPP_E_DEVICE;
        }
        // ---- sigma(lambda) from the surrogate's curvature ----
        std::vector<float> gt(kGrid), gdy(kGrid);
        for (int i = 0; i < kGrid; ++i) gt[i] = (float)(-1.0 + 2.0 * i / (kGrid - 1));
        float loss = NAN;
        if (hipMemcpy(mb.gt, gt.data(), kGrid * 4, hipMemcpyHostToDevice) != hipSuccess ||
            launch_mlp_forward(mb.params, mb.gt, kGrid, mb.gy, mb.gdy, st) != hipSuccess ||
            hipMemcpyAsync(gdy.data(), mb.gdy, kGrid * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&loss, mb.loss, 4, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
            return PPP_E_DEVICE;
        bool ok = std::isfinite(loss);
        std::vector<double> slope(kGrid);
        for (int i = 0; i < kGrid; ++i) { slope[i] = (double)gdy[i] * Fs / half; ok = ok && std::isfinite(slope[i]); }
        if (!ok) break;                       // uniform fallback below
        trained = true;
        for (int i = 0; i < kGrid; ++i) {
            const int a0 = std::max(0, i - 1), a1 = std::min(kGrid - 1, i + 1);
            const double curv = (slope[a1] - slope[a0]) / ((a1 - a0) * dl);          // F''(lambda)
            const double s2 = (k - curv) / (beta * k * k);
            sig[i] = std::sqrt(std::min(std::max(s2, 0.05 * s2_free), 100.0 * s2_free));
        }
        }
        auto sigma_at = [&](double l) {
            double x = (l - lo) / dl;
            int i = std::min(kGrid - 2, std::max(0, (int)std::floor(x)));
            double f = std::min(1.0, std::max(0.0, x - i));
            return sig[i] * (1 - f) + sig[i + 1] * f;
        };
        // ---- place windows with |dlambda| / sigma = target ----
        double target = a->target_dl_over_sigma;
        std::vector<double> grid;
        for (int attempt = 0; attempt < 60; ++attempt) {
            grid.clear();
            double l = lo, dir = hi > lo ? 1.0 : -1.0;
            grid.push_back(l);
            while (dir * (hi - l) > 1e-12 * span) {
                l += dir * target * sigma_at(l);
                if (dir * (hi - l) < 0.25 * target * sigma_at(hi)) l = hi;
                grid.push_back(l);
                if ((int)grid.size() > a->max_windows) break;
            }
            if ((int)grid.size() <= a->max_windows && grid.back() == hi) break;
            target *= 1.1;                    // too many windows for the cap: widen uniformly
        }
        placed = grid;
        // windows the placement asks for that no round has explored yet
        fresh.clear();
        for (double g : placed) {
            double dmin = 1e300;
            for (double x : xl) dmin = std::min(dmin, std::fabs(g - x));
            if (dmin > 0.5 * target * sigma_at(g)) fresh.push_back(g);
        }
    }
    if (!trained || placed.size() < 2) {
        placed.resize(a->initial_windows);
        for (int i = 0; i < a->initial_windows; ++i) placed[i] = lo + (hi - lo) * i / (a->initial_windows - 1);
    }
    // ---- production run on the placed windows with the remaining budget ----
    // every window keeps at least min_production_steps of relaxation (Sec. IV D: the
    // relaxation time decides the accuracy); replicas give way first, down to 16
    const int64_t left = a->budget_replica_steps - used;
    const int64_t W = (int64_t)placed.size();
    int32_t R = base->n_replicas;
    int64_t steps = left / (W * R);
    if (steps < a->min_production_steps) {
        R = (int32_t)std::max<int64_t>(16, left / (W * std::max<int64_t>(1, a->min_production_steps)));
        R = std::min(R, base->n_replicas);
        steps = left / (W * R);
    }
    if (steps < std::max<int64_t>(2, a->min_production_steps)) return PPP_E_INVALID_ARG;
    const int64_t per_step = W * R;
    s = run_windows(base, placed, R, steps, ws, run_bytes, st, out, nullptr);
    if (s != PPP_OK && s != PPP_E_NUMERICAL) return s;
    used += per_step * steps;
    for (size_t i = 0; i < placed.size(); ++i) lambda_out[i] = placed[i];
    *n_windows_out = (int32_t)placed.size();
    if (used_out) *used_out = used;
    return s;
}

}  // extern "C"

// Lane model of the chain kernels (tests only, CPU): the device routines that
// spread one replica over G lanes of a wavefront (ChainForce, baoab_step in
// paper_1105_4840_amd/csrc/ppp_chain_force.hpp, with the lane moves and noise
// of ppp_device.hpp) compiled for the host through the stand-in
// <hip/hip_runtime.h> of this directory.  A wavefront is 64 threads; every
// ds_bpermute / ds_permute is an exchange through a shared slot array between
// two barriers, and a permute checks that each destination lane is written by
// at most one lane.  Built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_lane_model.py, one binary per kernel shape, which compares its
// forces and trajectories with the oracle for every shape, including shapes the
// GPU build leaves out because they spill registers there.
//
// Input (stdin, whitespace separated):
//   mode G B precision N n_conf n_steps gid
//   k_bond r0 k_angle lj_eps lj_sigma lj_rc rc_mode mass gamma kT dt k centre seed
//   then n_conf configurations of 3 N coordinates (bead 0 first; for mode 1 one
//   start configuration)
// mode 0: forces and energies of each configuration at restraint centre
//         `centre` (the parity hook's evaluation): per configuration 3 N forces,
//         then total, bond, angle, Lennard-Jones and restraint energies.
// mode 1: n_steps BAOAB steps of replica number `gid` from the configuration,
//         velocities drawn at step 0 as the kernel does; (n_steps + 1) x 3 N
//         positions.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "ppp_internal.hpp"
#include "ppp_device.hpp"
#include "ppp_chain_force.hpp"

namespace lane_model {

// Sense-reversing barrier of the 64 lane threads; waiting threads yield the CPU
// (there are more lanes than cores), which is far cheaper here than sleeping.
struct Barrier {
    std::atomic<int> count{0};
    std::atomic<int> phase{0};
    void arrive_and_wait() {
        const int ph = phase.load(std::memory_order_acquire);
        if (count.fetch_add(1, std::memory_order_acq_rel) == 63) {
            count.store(0, std::memory_order_relaxed);
            phase.store(ph + 1, std::memory_order_release);
        } else {
            while (phase.load(std::memory_order_acquire) == ph) std::this_thread::yield();
        }
    }
};

struct Wave {
    Barrier bar;
    int slot[64] = {};
    std::atomic<int> writes[64];
};
thread_local int t_lane = 0;
thread_local Wave *t_wave = nullptr;
std::atomic<int> g_permute_conflicts{0};

int lane() { return t_lane; }

int bpermute(int byte_addr, int v) {
    Wave &w = *t_wave;
    w.slot[t_lane] = v;
    w.bar.arrive_and_wait();
    const int r = w.slot[(byte_addr >> 2) & 63];
    w.bar.arrive_and_wait();
    return r;
}

int permute(int byte_addr, int v) {
    Wave &w = *t_wave;
    w.writes[t_lane].store(0);
    w.slot[t_lane] = 0;
    w.bar.arrive_and_wait();
    const int dst = (byte_addr >> 2) & 63;
    if (w.writes[dst].fetch_add(1) != 0) g_permute_conflicts.fetch_add(1);
    w.slot[dst] = v;
    w.bar.arrive_and_wait();
    const int r = w.slot[t_lane];
    w.bar.arrive_and_wait();
    return r;
}

}  // namespace lane_model

using namespace ppp;

struct Input {
    int mode, G, B, prec, N, n_conf, n_steps;
    long gid;
    double k_bond, r0, k_angle, eps, sig, rc_f, mass, gamma, kT, dt, k, centre;
    int rc_mode;
    unsigned long long seed;
    std::vector<double> coords;
};

DevProblem make_problem(const Input &in) {
    DevProblem d;
    std::memset(&d, 0, sizeof(d));
    d.model = 1;
    d.precision = in.prec == 64 ? 1 : 0;
    d.n_beads = in.N;
    d.n_pad = in.G * in.B;
    d.rc_mode = in.rc_mode;
    d.seed = in.seed;
    d.k = in.k; d.kT = in.kT; d.beta = 1.0 / in.kT; d.dt = in.dt;
    d.k_bond = in.k_bond; d.r0 = in.r0; d.k_angle = in.k_angle;
    const double s2 = in.sig * in.sig, s6 = s2 * s2 * s2, s12 = s6 * s6;
    d.lj_A = 48.0 * in.eps * s12; d.lj_B = 24.0 * in.eps * s6;
    d.lj_eA = 4.0 * in.eps * s12; d.lj_eB = 4.0 * in.eps * s6;
    const double rc = in.rc_f * in.sig;
    const double q = std::pow(in.sig / rc, 6.0);
    d.lj_ucut = 4.0 * in.eps * (q * q - q);
    d.rc2 = rc * rc;
    d.mass = in.mass; d.inv_mass = 1.0 / in.mass;
    d.c1 = std::exp(-in.gamma * in.dt);
    d.sd_v = std::sqrt(in.kT / in.mass);
    d.c2sd = std::sqrt(1.0 - d.c1 * d.c1) * d.sd_v;
    d.fix_x = in.coords[0]; d.fix_y = in.coords[1]; d.fix_z = in.coords[2];
    d.pad_z0 = 1.0e5 * in.sig;
    d.pad_dz = 4.0 * rc;
    return d;
}

// One lane's part of the parity hook's evaluation (as chain_eval): lane l of a
// wavefront holds bead block g of configuration c = wave * (64 / G) + l / G.
template <typename T, int G, int B>
void lane_forces(const DevProblem &P, const Input &in, std::vector<double> &forces, std::vector<double> &energy) {
    constexpr int GPW = groups_per_wave(G);
    const int lane = lane_model::t_lane;
    const bool lane_used = lane < GPW * G;
    const int grp = lane_used ? lane / G : 0;
    const int g = lane_used ? lane % G : 0;
    const int gbase = lane_used ? lane - g : lane;
    const int N = P.n_beads, i0 = g * B;
    const int waves = (in.n_conf + GPW - 1) / GPW;
    for (int wv = 0; wv < waves; ++wv) {
        const int c = wv * GPW + grp;
        const bool active = lane_used && c < in.n_conf;
        const int cc = active ? c : 0;
        T px[B], py[B], pz[B], fx[B], fy[B], fz[B];
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            if (i < N) {
                px[b] = (T)in.coords[(size_t)cc * 3 * N + 3 * i];
                py[b] = (T)in.coords[(size_t)cc * 3 * N + 3 * i + 1];
                pz[b] = (T)in.coords[(size_t)cc * 3 * N + 3 * i + 2];
            } else {
                px[b] = 0; py[b] = 0; pz[b] = (T)(P.pad_z0 + P.pad_dz * (i - N));
            }
        }
        double e[4];
        ChainForce<T, G, B, true>::compute(P, g, gbase, (T)in.centre, (T)P.k, px, py, pz, fx, fy, fz, e);
        double tot[4];
        for (int q = 0; q < 4; ++q) {
            double s = 0.0;
            for (int l = 0; l < G; ++l) s += pull_f(lane_used ? gbase + l : lane, e[q]);
            tot[q] = s;
        }
        if (!active) continue;
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            if (i < N) {
                forces[(size_t)c * 3 * N + 3 * i] = (double)fx[b];
                forces[(size_t)c * 3 * N + 3 * i + 1] = (double)fy[b];
                forces[(size_t)c * 3 * N + 3 * i + 2] = (double)fz[b];
            }
        }
        if (g == 0) {
            energy[(size_t)c * 5] = tot[0] + tot[1] + tot[2] + tot[3];
            for (int q = 0; q < 4; ++q) energy[(size_t)c * 5 + 1 + q] = tot[q];
        }
    }
}

// One lane's part of a replica's trajectory (the step loop of the simulation
// kernel without sampling): every group of the wavefront runs the same replica,
// group 0 records.
template <typename T, int G, int B>
void lane_traj(const DevProblem &P, const Input &in, std::vector<double> &traj) {
    constexpr int GPW = groups_per_wave(G);
    const int lane = lane_model::t_lane;
    const bool lane_used = lane < GPW * G;
    const int grp = lane_used ? lane / G : 0;
    const int g = lane_used ? lane % G : 0;
    const int gbase = lane_used ? lane - g : lane;
    const int N = P.n_beads, i0 = g * B;
    const uint32_t gid = (uint32_t)in.gid;
    T px[B], py[B], pz[B], vx[B], vy[B], vz[B], fx[B], fy[B], fz[B];
    for (int b = 0; b < B; ++b) {
        const int i = i0 + b;
        if (i < N) { px[b] = (T)in.coords[3 * i]; py[b] = (T)in.coords[3 * i + 1]; pz[b] = (T)in.coords[3 * i + 2]; }
        else { px[b] = 0; py[b] = 0; pz[b] = (T)(P.pad_z0 + P.pad_dz * (i - N)); }
    }
    lane_noise<T, B>(P, gid, 0u, i0, [&](int b, const T *z) {
        const int i = i0 + b;
        const bool mobile = i > 0 && i < N;
        vx[b] = mobile ? (T)P.sd_v * z[0] : (T)0;
        vy[b] = mobile ? (T)P.sd_v * z[1] : (T)0;
        vz[b] = mobile ? (T)P.sd_v * z[2] : (T)0;
    });
    const bool rec = lane_used && grp == 0;
    auto record = [&](int n) {
        if (!rec) return;
        for (int b = 0; b < B; ++b)
            if (i0 + b < N) {
                double *o = traj.data() + (size_t)n * 3 * N + 3 * (i0 + b);
                o[0] = (double)px[b]; o[1] = (double)py[b]; o[2] = (double)pz[b];
            }
    };
    record(0);
    const T kr = (T)P.k, centre = (T)in.centre;
    ChainForce<T, G, B, false>::compute(P, g, gbase, centre, kr, px, py, pz, fx, fy, fz, nullptr);
    const T h = (T)(0.5 * P.dt), c1 = (T)P.c1, hm = (T)(0.5 * P.dt * P.inv_mass), c2sd = (T)P.c2sd;
    for (int n = 1; n <= in.n_steps; ++n) {
        baoab_step<T, G, B>(P, g, gbase, gid, (uint32_t)n, centre, kr, h, hm, c1, c2sd, px, py, pz, vx, vy, vz, fx, fy,
                            fz);
        record(n);
    }
}

template <typename T, int G, int B>
int run_shape(const Input &in) {
    const DevProblem P = make_problem(in);
    const int N = in.N;
    std::vector<double> forces((size_t)in.n_conf * 3 * N, NAN), energy((size_t)in.n_conf * 5, NAN);
    std::vector<double> traj((size_t)(in.n_steps + 1) * 3 * N, NAN);
    lane_model::Wave wave;
    std::vector<std::thread> th;
    for (int l = 0; l < 64; ++l)
        th.emplace_back([&, l] {
            lane_model::t_lane = l;
            lane_model::t_wave = &wave;
            if (in.mode == 0) lane_forces<T, G, B>(P, in, forces, energy);
            else lane_traj<T, G, B>(P, in, traj);
        });
    for (auto &t : th) t.join();
    if (in.mode == 0) {
        for (int c = 0; c < in.n_conf; ++c) {
            for (int q = 0; q < 3 * N; ++q) std::printf("%.17g\n", forces[(size_t)c * 3 * N + q]);
            for (int q = 0; q < 5; ++q) std::printf("%.17g\n", energy[(size_t)c * 5 + q]);
        }
    } else {
        for (double v : traj) std::printf("%.17g\n", v);
    }
    std::fprintf(stderr, "permute conflicts %d\n", lane_model::g_permute_conflicts.load());
    return lane_model::g_permute_conflicts.load() == 0 ? 0 : 3;
}

// One kernel shape per build: -DLM_G=<lanes> -DLM_B=<beads per lane>.
#if !defined(LM_G) || !defined(LM_B)
#error "build with -DLM_G=<lanes per replica> -DLM_B=<beads per lane>"
#endif

int main() {
    Input in{};
    if (std::scanf("%d %d %d %d %d %d %d %ld", &in.mode, &in.G, &in.B, &in.prec, &in.N, &in.n_conf, &in.n_steps,
                   &in.gid) != 8)
        return 2;
    if (std::scanf("%lf %lf %lf %lf %lf %lf %d %lf %lf %lf %lf %lf %lf %llu", &in.k_bond, &in.r0, &in.k_angle, &in.eps,
                   &in.sig, &in.rc_f, &in.rc_mode, &in.mass, &in.gamma, &in.kT, &in.dt, &in.k, &in.centre,
                   &in.seed) != 14)
        return 2;
    const int n = (in.mode == 0 ? in.n_conf : 1) * 3 * in.N;
    in.coords.resize(n);
    for (int i = 0; i < n; ++i)
        if (std::scanf("%lf", &in.coords[i]) != 1) return 2;
    if (in.N < 2 || in.N > in.G * in.B) return 2;
    if (in.G != LM_G || in.B != LM_B) return 2;
    return in.prec == 64 ? run_shape<double, LM_G, LM_B>(in) : run_shape<float, LM_G, LM_B>(in);
}

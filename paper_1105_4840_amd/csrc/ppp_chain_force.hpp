// One replica's chain forces and BAOAB step across the G lanes of its group
// (device code of the simulation kernels; the parity hook for forces uses the
// same routine).  Included after ppp_device.hpp, which supplies the lane
// moves (pull_f, push_f), the working-precision reciprocal and length
// (rcp_t, len_inv) and the noise (Normal6).
#pragma once

namespace ppp {

// ===========================================================================
// Chain model.
// ===========================================================================
template <typename T, int G, int B, bool ENERGY>
struct ChainForce {
    // groups of at most 6 lanes run no Newton-3 rounds beyond round 2
    static constexpr bool kHaloFromRound1 = G > 1 && (G - 1) / 2 <= 2;
    // Small groups of two-bead lanes (5x2, 6x2), where the bonded terms are a
    // sixth of the step, mask the bonds beyond the chain's ends, the halo
    // forces of the group's edge lanes and the closing half-kick of the fixed
    // bead with 0/1 factors instead of selects: a select reads a lane mask
    // from scalar registers and issues at about half the rate of a
    // vector-register multiply or FMA, and an add followed by a select becomes
    // one FMA.  Multiplying by 1 is exact, so the results are the same.  The
    // factors stay in vector registers for the whole loop, which the kernels
    // compiled for more waves per SIMD cannot spare.
    static constexpr bool kMaskFactors = G > 1 && G <= 6 && B == 2;

    // Lennard-Jones between bead sets a (owned) and b; N3: also accumulate reaction on b.
    template <bool N3, bool MASK>
    __device__ __forceinline__ static void lj_block(const DevProblem &P, const T (&ax)[B], const T (&ay)[B],
                                                    const T (&az)[B], const T (&bx)[B], const T (&by)[B],
                                                    const T (&bz)[B], T (&fx)[B], T (&fy)[B], T (&fz)[B],
                                                    T (&gx)[B], T (&gy)[B], T (&gz)[B], int ia0, int ib0,
                                                    T lA, T lB, T rc2, double &e_lj) {
#pragma clang fp contract(on)
#pragma unroll
        for (int b1 = 0; b1 < B; ++b1) {
#pragma unroll
            for (int b2 = 0; b2 < B; ++b2) {
                const T dx = ax[b1] - bx[b2], dy = ay[b1] - by[b2], dz = az[b1] - bz[b2];
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T ir2 = rcp_t(r2);
                const T ir6 = ir2 * ir2 * ir2;
                T f = ir6 * ir2 * (lA * ir6 - lB);
                bool ok = r2 < rc2;
                if (MASK) {
                    const int dij = (ia0 + b1) - (ib0 + b2);
                    ok = ok && (dij > 2 || dij < -2);
                }
                f = ok ? f : (T)0;
                if (ENERGY && ok) e_lj += (double)(ir6 * ((T)P.lj_eA * ir6 - (T)P.lj_eB)) - P.lj_ucut;
                fx[b1] += f * dx; fy[b1] += f * dy; fz[b1] += f * dz;
                if (N3) { gx[b2] -= f * dx; gy[b2] -= f * dy; gz[b2] -= f * dz; }
            }
        }
    }

    // Forces on the owned beads with the restraint kr/2 (xi - centre)^2.  lane g of
    // group base `gbase`; an idle lane (beyond the wavefront's last whole group:
    // gbase + G > 64) only exchanges data with itself.
    // e[0..3] = bond, angle, lj, restraint energy contributions of this lane (ENERGY only).
    __device__ __forceinline__ static void compute(const DevProblem &P, int g, int gbase, T centre, T kr,
                                                   const T (&px)[B], const T (&py)[B], const T (&pz)[B],
                                                   T (&fx)[B], T (&fy)[B], T (&fz)[B], double *e) {
        // Products are fused into adds only inside one expression, never across
        // statements: the forces then round the same way wherever this is
        // inlined, so the forces recomputed from the stored state when a run
        // resumes equal the ones the uninterrupted run carried.
#pragma clang fp contract(on)
        const int N = P.n_beads;
        const int i0 = g * B;
        const bool solo = gbase + G > 64;
        const int me = lane_id();
        const T lA = (T)P.lj_A, lB = (T)P.lj_B, rc2 = (T)P.rc2;
        double e_lj = 0.0, e_bond = 0.0, e_ang = 0.0, e_res = 0.0;
#pragma unroll
        for (int b = 0; b < B; ++b) { fx[b] = 0; fy[b] = 0; fz[b] = 0; }
        T hpx = 0, hpy = 0, hpz = 0, hnx = 0, hny = 0, hnz = 0;   // halo beads of the bonded terms

        // ---- Lennard-Jones: pairs inside the lane (|i-j| > 2 by construction) ----
#pragma unroll
        for (int b1 = 0; b1 < B; ++b1) {
#pragma unroll
            for (int b2 = b1 + 3; b2 < B; ++b2) {
                const T dx = px[b1] - px[b2], dy = py[b1] - py[b2], dz = pz[b1] - pz[b2];
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T ir2 = rcp_t(r2);
                const T ir6 = ir2 * ir2 * ir2;
                T f = ir6 * ir2 * (lA * ir6 - lB);
                const bool ok = r2 < rc2;
                f = ok ? f : (T)0;
                if (ENERGY && ok) e_lj += (double)(ir6 * ((T)P.lj_eA * ir6 - (T)P.lj_eB)) - P.lj_ucut;
                fx[b1] += f * dx; fy[b1] += f * dy; fz[b1] += f * dz;
                fx[b2] -= f * dx; fy[b2] -= f * dy; fz[b2] -= f * dz;
            }
        }
        // ---- Lennard-Jones between lanes: rotate the j-beads through the group ----
        // Round r meets the beads of lane g - r.  Rounds 1 .. (G-1)/2 meet every
        // lane pair once and keep the reactions, which travel with the beads and
        // go back to their owner at the end; for even G round G/2 meets the
        // opposite lane, from both sides.  Only round 1 meets sequence neighbours
        // (pairs |i-j| <= 2 are excluded), so only it takes the masked routine.
        if constexpr (G > 1) {
            constexpr int R_N3 = (G - 1) / 2;
            constexpr bool HALF = (G % 2) == 0;
            T qx[B], qy[B], qz[B], gx[B], gy[B], gz[B];
#pragma unroll
            for (int b = 0; b < B; ++b) { qx[b] = px[b]; qy[b] = py[b]; qz[b] = pz[b]; gx[b] = 0; gy[b] = 0; gz[b] = 0; }
            const int src = solo ? me : gbase + ((g + G - 1) % G);
            auto pull_q = [&]() {
#pragma unroll
                for (int b = 0; b < B; ++b) { qx[b] = pull_f(src, qx[b]); qy[b] = pull_f(src, qy[b]); qz[b] = pull_f(src, qz[b]); }
            };
            // round 1; its j-beads are the previous lane's, whose last bead is also
            // the halo bead of the bonded terms below.  Small groups keep it from
            // here; in groups with a loop of further rounds, three more registers
            // live across that loop cost more than pulling the bead again.
            pull_q();
            if constexpr (kHaloFromRound1) { hpx = qx[B - 1]; hpy = qy[B - 1]; hpz = qz[B - 1]; }
            {
                double e_r = 0.0;
                const int jb = ((g + G - 1) % G) * B;
                if constexpr (R_N3 >= 1) {
                    lj_block<true, true>(P, px, py, pz, qx, qy, qz, fx, fy, fz, gx, gy, gz, i0, jb, lA, lB, rc2, e_r);
                    e_lj += e_r;
                } else {   // G == 2: the neighbour is also the opposite lane
                    lj_block<false, true>(P, px, py, pz, qx, qy, qz, fx, fy, fz, gx, gy, gz, i0, jb, lA, lB, rc2, e_r);
                    e_lj += 0.5 * e_r;   // each such pair is seen from both lanes
                }
            }
            // rounds 2 .. R_N3
#pragma unroll 1
            for (int r = 2; r <= R_N3; ++r) {
                pull_q();
#pragma unroll
                for (int b = 0; b < B; ++b) { gx[b] = pull_f(src, gx[b]); gy[b] = pull_f(src, gy[b]); gz[b] = pull_f(src, gz[b]); }
                double e_r = 0.0;
                lj_block<true, false>(P, px, py, pz, qx, qy, qz, fx, fy, fz, gx, gy, gz, i0, 0, lA, lB, rc2, e_r);
                e_lj += e_r;
            }
            if constexpr (R_N3 >= 1) {
                // the reactions belong to lane g - R_N3
                const int dst = solo ? me : gbase + ((g + G - R_N3) % G);
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    fx[b] += push_f(dst, gx[b]); fy[b] += push_f(dst, gy[b]); fz[b] += push_f(dst, gz[b]);
                }
            }
            if constexpr (HALF && G > 2) {
                // round G/2: the opposite lane, its beads pulled directly
                const int opp = solo ? me : gbase + ((g + G / 2) % G);
#pragma unroll
                for (int b = 0; b < B; ++b) { qx[b] = pull_f(opp, px[b]); qy[b] = pull_f(opp, py[b]); qz[b] = pull_f(opp, pz[b]); }
                double e_r = 0.0;
                lj_block<false, false>(P, px, py, pz, qx, qy, qz, fx, fy, fz, gx, gy, gz, i0, 0, lA, lB, rc2, e_r);
                e_lj += 0.5 * e_r;
            }
        }

        // ---- bonded terms, each computed once ----
        // Local slots 0..B+1: slot 0 is the previous lane's last bead, slots 1..B
        // the owned beads, slot B+1 the next lane's first bead; bond t joins slot
        // t to slot t+1.  A lane takes the bonds that start at an owned bead and
        // the angles centred on owned beads.  These terms depend on the beads
        // only through the bond vectors b_t = x_{t+1} - x_t, so their gradients
        // are gathered per bond, D_t = dU/db_t, and the force on slot t is
        // D_t - D_{t-1}; the two halo beads get D_0 and -D_B, which the lanes
        // owning them read back.
        const int prev = solo ? me : gbase + (g > 0 ? g - 1 : 0);
        const int next = solo ? me : gbase + (g + 1 < G ? g + 1 : G - 1);
        if constexpr (G > 1) {
            if constexpr (!kHaloFromRound1) {
                hpx = pull_f(prev, px[B - 1]); hpy = pull_f(prev, py[B - 1]); hpz = pull_f(prev, pz[B - 1]);
            }
            hnx = pull_f(next, px[0]); hny = pull_f(next, py[0]); hnz = pull_f(next, pz[0]);
        }
        const T kb = (T)P.k_bond, r0 = (T)P.r0, kth = (T)P.k_angle;
        auto slot = [&](int t, T &x, T &y, T &z) {   // position of local slot t (compile-time t)
            if (t == 0) { x = hpx; y = hpy; z = hpz; }
            else if (t <= B) { x = px[t - 1]; y = py[t - 1]; z = pz[t - 1]; }
            else { x = hnx; y = hny; z = hnz; }
        };
        T Dx[B + 1], Dy[B + 1], Dz[B + 1];
        const T m_next = g + 1 < G ? (T)1 : (T)0, m_prev = g > 0 ? (T)1 : (T)0;
        T ux = 0, uy = 0, uz = 0, ail = 0;   // previous bond (t-1 -> t): unit vector, inverse length
        bool avalid = false;
#pragma unroll
        for (int t = 0; t <= B; ++t) {
            T x0, y0, z0, x1, y1, z1;
            slot(t, x0, y0, z0);
            slot(t + 1, x1, y1, z1);
            const T bx = x1 - x0, by = y1 - y0, bz = z1 - z0;
            const int i = i0 - 1 + t;               // bead index of slot t
            const bool bvalid = i >= 0 && i + 1 < N;
            // a bond outside the chain gets unit length so its masked terms stay finite
            T bl, bil;
            const T mb = bvalid ? (T)1 : (T)0;
            if constexpr (kMaskFactors) {
                const T b2 = bx * bx + by * by + bz * bz;
                len_inv(b2 * mb + ((T)1 - mb), bl, bil);
            } else {
                len_inv(bvalid ? bx * bx + by * by + bz * bz : (T)1, bl, bil);
            }
            const T vx = bx * bil, vy = by * bil, vz = bz * bil;
            if (t == 0) {
                Dx[0] = 0; Dy[0] = 0; Dz[0] = 0;
            } else {
                // bond (t, t+1), k_b/2 (|b| - r0)^2: dU/db = k_b (|b| - r0) b/|b|
                T gsc = kb * (bl - r0);
                if constexpr (kMaskFactors) gsc = gsc * mb;
                else gsc = bvalid ? gsc : (T)0;
                Dx[t] = gsc * vx; Dy[t] = gsc * vy; Dz[t] = gsc * vz;
                if (ENERGY && bvalid) e_bond += 0.5 * (double)(kb * (bl - r0) * (bl - r0));
                // angle centred on slot t between bond a (t-1 -> t) and bond b (t -> t+1),
                // unit vectors u and v, c = u.v:
                // dU/da = k (c u - v)/|a|, dU/db = k (c v - u)/|b|
                const bool valid = avalid && bvalid;
                const T c = ux * vx + uy * vy + uz * vz;
                const T kk = valid ? kth : (T)0;
                const T sa = kk * ail, sb = kk * bil;
                Dx[t - 1] += sa * (c * ux - vx); Dy[t - 1] += sa * (c * uy - vy); Dz[t - 1] += sa * (c * uz - vz);
                Dx[t] += sb * (c * vx - ux); Dy[t] += sb * (c * vy - uy); Dz[t] += sb * (c * vz - uz);
                if (ENERGY && valid) e_ang += (double)(kth * ((T)1 - c));
            }
            ux = vx; uy = vy; uz = vz; ail = bil; avalid = bvalid;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            fx[b] += Dx[b + 1] - Dx[b]; fy[b] += Dy[b + 1] - Dy[b]; fz[b] += Dz[b + 1] - Dz[b];
        }
        if constexpr (G > 1) {
            // our last bead is the next lane's slot 0 (force D_0 there), our first
            // bead the previous lane's slot B+1 (force -D_B there)
            const T lx = pull_f(next, Dx[0]), ly = pull_f(next, Dy[0]), lz = pull_f(next, Dz[0]);
            const T fx0 = pull_f(prev, Dx[B]), fy0 = pull_f(prev, Dy[B]), fz0 = pull_f(prev, Dz[B]);
            if constexpr (kMaskFactors) {
                fx[B - 1] += lx * m_next; fy[B - 1] += ly * m_next; fz[B - 1] += lz * m_next;
                fx[0] -= fx0 * m_prev; fy[0] -= fy0 * m_prev; fz[0] -= fz0 * m_prev;
            } else {
                if (g + 1 < G) { fx[B - 1] += lx; fy[B - 1] += ly; fz[B - 1] += lz; }
                if (g > 0) { fx[0] -= fx0; fy[0] -= fy0; fz[0] -= fz0; }
            }
        }

        // ---- restraint k/2 (xi - centre)^2 on the pulled end ----
        const int last = N - 1;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (i0 + b == last) {
                const T dx = px[b] - (T)P.fix_x, dy = py[b] - (T)P.fix_y, dz = pz[b] - (T)P.fix_z;
                T xi, ux, uy, uz;
                if (P.rc_mode == 1) { xi = dz; ux = 0; uy = 0; uz = 1; }
                else { T ixi; len_inv(dx * dx + dy * dy + dz * dz, xi, ixi); ux = dx * ixi; uy = dy * ixi; uz = dz * ixi; }
                const T fr = -kr * (xi - centre);
                fx[b] += fr * ux; fy[b] += fr * uy; fz[b] += fr * uz;
                if (ENERGY) e_res += 0.5 * (double)kr * (double)(xi - centre) * (double)(xi - centre);
            }
        }
        if (ENERGY) { e[0] = e_bond; e[1] = e_ang; e[2] = e_lj; e[3] = e_res; }
    }
};

// The noise of the lane's beads at step `step` (step 0: the Maxwell
// velocities): beads 2m and 2m + 1 share Philox block (gid, step, m, 0), the
// even bead taking its normals z_0..z_2 and the odd bead z_3..z_5.  Calls
// fn(b, z) with the three normals z of owned bead b = 0..B-1.  A lane with an
// even bead count owns whole pairs and draws B/2 blocks; otherwise each bead
// draws its pair's block and keeps its half.
template <typename T, int B, typename Fn>
__device__ __forceinline__ void lane_noise(const DevProblem &P, uint32_t gid, uint32_t step, int i0, Fn &&fn) {
    if constexpr (B % 2 == 0) {
#pragma unroll
        for (int q = 0; q < B / 2; ++q) {
            T z[6];
            Normal6<T>::get(P.seed, gid, step, (uint32_t)((i0 >> 1) + q), 0u, z);
            fn(2 * q, z);
            fn(2 * q + 1, z + 3);
        }
    } else {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            T z[6];
            Normal6<T>::get(P.seed, gid, step, (uint32_t)(i >> 1), 0u, z);
            if (i & 1) { z[0] = z[3]; z[1] = z[4]; z[2] = z[5]; }
            fn(b, z);
        }
    }
}

// One BAOAB step of the lane's owned beads (Leimkuhler-Matthews splitting):
// v += dt/2 F/m; x += dt/2 v; v = c1 v + c2 sqrt(kT/m) eta; x += dt/2 v; then the
// forces at the new positions with the restraint centred at `centre`, and
// v += dt/2 F/m.  Bead 0 (held fixed) and padding beads do not move.  f holds
// the forces of the current positions on entry and of the new ones on return.
template <typename T, int G, int B>
__device__ __forceinline__ void baoab_step(const DevProblem &P, int g, int gbase, uint32_t gid, uint32_t n, T centre,
                                           T kr, T h, T hm, T c1, T c2sd, T (&px)[B], T (&py)[B], T (&pz)[B],
                                           T (&vx)[B], T (&vy)[B], T (&vz)[B], T (&fx)[B], T (&fy)[B], T (&fz)[B]) {
    const int N = P.n_beads;
    const int i0 = g * B;
    lane_noise<T, B>(P, gid, n, i0, [&](int b, const T *z) {
        const int i = i0 + b;
        if (i > 0 && i < N) {
            vx[b] += hm * fx[b]; vy[b] += hm * fy[b]; vz[b] += hm * fz[b];
            px[b] += h * vx[b]; py[b] += h * vy[b]; pz[b] += h * vz[b];
            vx[b] = c1 * vx[b] + c2sd * z[0]; vy[b] = c1 * vy[b] + c2sd * z[1]; vz[b] = c1 * vz[b] + c2sd * z[2];
            px[b] += h * vx[b]; py[b] += h * vy[b]; pz[b] += h * vz[b];
        }
    });
    ChainForce<T, G, B, false>::compute(P, g, gbase, centre, kr, px, py, pz, fx, fy, fz, nullptr);
    if constexpr (ChainForce<T, G, B, false>::kMaskFactors) {
        // the closing half-kick with a zero factor for the fixed bead and the
        // padding (no select; the mobile beads' kick is the same FMA)
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            const T hmb = (i > 0 && i < N) ? hm : (T)0;
            vx[b] += hmb * fx[b]; vy[b] += hmb * fy[b]; vz[b] += hmb * fz[b];
        }
    } else {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            if (i > 0 && i < N) { vx[b] += hm * fx[b]; vy[b] += hm * fy[b]; vz[b] += hm * fz[b]; }
        }
    }
}

}  // namespace ppp

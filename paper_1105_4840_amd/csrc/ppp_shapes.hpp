// Chain kernel shapes compiled into libppp: X(G lanes per replica, B beads per lane).
// Only shapes whose kernels need no scratch memory in either precision are
// built (build.py checks this); more beads per lane spill registers.
// 1 <= G <= 64 (a wavefront holds 64 / G groups; 64 mod G lanes stay idle);
// B >= 2 whenever G > 1 (Lennard-Jones exclusions, |i-j| <= 2, are masked only
// between neighbouring lanes).
#pragma once
#define PPP_FOR_EACH_SHAPE(X)                                                                      \
    X(1, 4) X(1, 8) X(2, 5) X(3, 4) X(4, 3) X(4, 4) X(5, 2) X(6, 2) X(8, 2) X(8, 4) X(16, 2) X(16, 4) \
    X(32, 2) X(32, 4) X(64, 2) X(64, 4)

// the same list for host-only code
#define PPP_FOR_EACH_SHAPE_RT(X) PPP_FOR_EACH_SHAPE(X)

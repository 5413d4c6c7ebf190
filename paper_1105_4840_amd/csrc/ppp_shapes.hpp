// Chain kernel shapes compiled into libppp: X(G lanes per replica, B beads per lane).
// G in {1, 4, 16, 64}; B >= 2 whenever G > 1 (the bonded halo spans two beads).
#pragma once
#define PPP_FOR_EACH_SHAPE(X) \
    X(1, 4) X(1, 8) X(1, 12) X(1, 16) X(4, 4) X(4, 8) X(16, 2) X(16, 4) X(16, 8) X(64, 2) X(64, 4) X(64, 8)

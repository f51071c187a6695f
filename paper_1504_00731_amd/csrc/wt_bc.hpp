// Boundary conditions as maps from a point index along a grid line (any i,
// including the ghost points beyond either end) onto the line's n points.
// Shared by the kernels and the host build of their arithmetic.
//   periodic:      i mod n;
//   transmissive:  the nearest end point (zero gradient);
//   reflective:    the mirror image across a wall half a spacing beyond each
//                  end; reflected() tells whether the point is a mirror image,
//                  whose momentum normal to the wall the caller negates.
// The reflective map is extended with period 2n (mirror images of mirror
// images), so every i maps inside the line: the kernels stage whole tiles,
// which can reach far past the last ghost point of a short line, where
// 2n - 1 - i alone would fall below 0.  On the ghost points themselves
// (-3 .. -1 and n .. n + 2) it is the plain mirror.
#pragma once

#include <cstdint>

#include "wt_common.hpp"
#include "wenotheta.h"

namespace wt {

WT_HD int64_t map_index(int64_t i, int64_t n, int bc)
{
    if (i >= 0 && i < n) return i;              // a point of the line (64-bit % only for ghosts)
    if (bc == WT_PERIODIC) {
        i %= n;
        return i < 0 ? i + n : i;
    }
    if (bc == WT_REFLECTIVE) {
        int64_t k = i % (2 * n);
        if (k < 0) k += 2 * n;
        return k < n ? k : 2 * n - 1 - k;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

WT_HD bool reflected(int64_t i, int64_t n, int bc)
{
    if (bc != WT_REFLECTIVE || (i >= 0 && i < n)) return false;
    int64_t k = i % (2 * n);
    if (k < 0) k += 2 * n;
    return k >= n;
}

// Lax-Friedrichs speed of characteristic field s in direction d, given the
// per-field maxima a(0..m-1) over the grid (0: u_d - c, 1: u_d, 2: u_d + c,
// 3..: u_d).  Behind reflective walls in d the solution is the mirror-extended
// one, in which u_d changes sign and the two acoustic fields exchange their
// speeds, so both take the larger maximum.
template <class Speeds>
WT_HD double split_speed(const Speeds &a, int s, bool walls)
{
    if (walls && (s == 0 || s == 2)) {
        const double a0 = a(0), a2 = a(2);
        return a2 > a0 ? a2 : a0;
    }
    return a(s);
}

}  // namespace wt

// Packed tiles of a batched 2D pass.  The pass's interfaces of one problem are
// listed line after line (a line: a group of 8 rows with their nx + 1 interface
// columns in the x pass, a group of 8 columns with their ny + 1 interface rows in
// the y pass), W per line and nl lines, and
// cut into chunks of at most qt consecutive interfaces that overlap by one
// interface (none after a line end).  A chunk stages the stretch of every line it
// touches plus the 3-point halo on each side, and finishes every cell whose left
// interface q lies in [q0, q0 + nq - 1): the half-open ranges of consecutive
// chunks partition the interfaces, so each cell is finished exactly once.
// Shared by the kernel (staging offsets) and the host (chunk tables).
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define WT_PACK_HD __host__ __device__ inline
#else
#define WT_PACK_HD inline
#endif

namespace wt {

// Chunk limits (256 threads): 8 lanes (the rows or columns of a line) by at most 32
// interface rows, staging at most 41 rows of 8 points (31.5 KB of LDS: five
// workgroups per CU).
constexpr int kPackLanes = 8;
constexpr int kPackQt = 32;
constexpr int kPackRows = 41;

// Staged rows of the chunk of nq interfaces starting at q0 (lines of W interfaces):
// line r0 = q0 / W from interface a0 = q0 - r0 W, whole lines between, and the
// last line up to its interface of q0 + nq - 1; each line's stretch of k
// interfaces takes k + 5 rows.
WT_PACK_HD int pack_rows(int q0, int nq, int W)
{
    const int ql = q0 + nq - 1;
    const int r0 = q0 / W, r1 = ql / W;
    if (r0 == r1) return nq + 5;
    const int first = W - (q0 - r0 * W) + 5;
    const int last = ql - r1 * W + 1 + 5;
    return first + (r1 - r0 - 1) * (W + 5) + last;
}

// Staged-row offset of interface q's stencil within the chunk starting at q0
// (the stencil's 6 points are rows base .. base + 5).
WT_PACK_HD int pack_base(int q0, int q, int W)
{
    const int r0 = q0 / W, r = q / W;
    const int i = q - r * W;
    if (r == r0) return i - (q0 - r0 * W);
    return (W - (q0 - r0 * W) + 5) + (r - r0 - 1) * (W + 5) + i;
}

// Line and point index (along the pass, -3 .. W + 1) of staged row `row` of the
// chunk starting at q0.
WT_PACK_HD void pack_point(int q0, int row, int W, int *line, int *g)
{
    const int r0 = q0 / W, a0 = q0 - r0 * W;
    const int len0 = W - a0 + 5;
    if (row < len0) {
        *line = r0;
        *g = a0 - 3 + row;
    } else {
        const int k = row - len0;
        *line = r0 + 1 + k / (W + 5);
        *g = k % (W + 5) - 3;
    }
}

// Cut the nl * W interfaces into chunks of at most qt interfaces and rmax staged
// rows; emit(q0, nq) for each, in order.  Every chunk has nq >= 2 when
// rmax >= qt + 5 * (qt / W + 2) for the smallest W in use, or at least 2 + 10.
template <class Emit>
void pack_chunks(int W, int nl, int qt, int rmax, Emit &&emit)
{
    const int Q = nl * W;
    int q0 = 0;
    for (;;) {
        int nq = Q - q0 < qt ? Q - q0 : qt;
        while (nq > 2 && pack_rows(q0, nq, W) > rmax) --nq;
        emit(q0, nq);
        const int ql = q0 + nq - 1;
        if (ql >= Q - 1) break;
        q0 = ql % W == W - 1 ? ql + 1 : ql;
    }
}

}  // namespace wt

// Context of the C ABI: device state, workspace and the kernel timer.
// Shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "wenotheta.h"
#include "wt_device.hpp"

// Per-kernel timing with HIP events recorded on the launch stream around each
// sweep launch (enabled by wenotheta_profile).  Kinds: sweep direction d in
// its non-final role (d) or as the final sweep of a stage or RHS (3 + d); the
// fused 2D stage kernel (6).
constexpr int kProfKinds = 7;
constexpr int kProfFused = 6;
constexpr int kProfPairs = 4096;

// Tile shape chosen for the y/z sweeps of one grid shape (see wenotheta_tune).
struct wt_tile_plan {
    uint64_t key = 0;     // system, ndim, n[], precision
    int8_t tile[3] = {0, 0, 0};
};
constexpr int kTilePlans = 16;
constexpr int kTileVariants = 4;
constexpr int kGraphSteps = 8;        // steps per captured solver graph

struct wt_ctx {
    int device = 0;
    wt::DevState *st = nullptr;
    double *U1 = nullptr, *U2 = nullptr, *D = nullptr;
    size_t cap = 0;       // doubles per workspace buffer
    int64_t g = 0;        // stage counter (selects the speed slots)
    // profiler
    bool prof = false;
    hipEvent_t ev[2 * kProfPairs] = {};
    int ev_kind[kProfPairs] = {};
    int nev = 0;
    double prof_ms[kProfKinds] = {};
    int64_t prof_n[kProfKinds] = {};
    int64_t prof_dropped = 0;
    // batched solves: packed stage buffers and per-problem tables
    double *B1 = nullptr, *B2 = nullptr;
    size_t bcap = 0;            // doubles per packed stage buffer
    int64_t *b_n = nullptr, *b_off = nullptr;
    double *b_dx = nullptr, *b_rdx = nullptr;
    int32_t *b_bc = nullptr, *b_order = nullptr, *b_queue = nullptr;
    int64_t b_cap = 0;          // problems the tables hold
    // graph of the last batched launch and the arguments it was captured with
    hipGraphExec_t b_graph = nullptr;
    hipStream_t b_capture = nullptr;
    uint64_t b_key = 0;
    // batched 2D solves: x-divergence buffer, problem table, queue order, graph
    double *BD = nullptr;
    size_t bdcap = 0;           // doubles of BD
    void *b2_tab = nullptr;
    int32_t *b2_order = nullptr, *b2_queue = nullptr;
    int64_t b2_cap = 0;         // problems the 2D tables hold
    hipGraphExec_t b2_graph = nullptr;
    uint64_t b2_key = 0;
    // flat forms of the 1D and 2D batches: per-problem state and tile tables
    void *f1_state = nullptr;
    int64_t f1_state_cap = 0;   // problems
    int32_t *f1_tab = nullptr;
    int64_t f1_tab_cap = 0;     // int32 entries
    void *f2_state = nullptr;
    int64_t f2_state_cap = 0;   // problems
    int32_t *f2_tab = nullptr;
    int64_t f2_tab_cap = 0;     // int32 entries
    // tile variants chosen by the batch tuners, for the batch signature they were tuned on
    int b_var = 0, b2_var = 0;
    uint64_t b_var_key = 0, b2_var_key = 0;
    // graph of kGraphSteps solver steps and the arguments it was captured with
    hipGraphExec_t s_graph = nullptr;
    hipStream_t s_capture = nullptr;
    uint64_t s_key = 0;
    // tile plans per grid shape, most recent first
    wt_tile_plan plans[kTilePlans];
    int nplans = 0;
    // side table for grids with WT_SIDES dimensions (wenotheta_set_sides)
    wt_side sides[6] = {};
    bool has_sides = false;
};


namespace wt {
// Read (and clear) the device error word after synchronising the stream;
// folds completed timing events into the profile.
wt_status collect(wt_ctx *c, hipStream_t s, DevState *host);
// Free the batched-solve workspace and graph.
void release_batched(wt_ctx *c);
}  // namespace wt

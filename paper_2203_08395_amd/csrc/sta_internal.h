// Internal layout of an sta_graph: host-side maps and the device array offsets.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sta.h"
#include "../../include/sta_analysis.h"
#include "../../include/sta_batch.h"

namespace sta {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kTileSlots = 64;      // one work tile = one wavefront of arcs / fanout slots
constexpr uint32_t kHeadBit = 0x80000000u;
constexpr int32_t kDefaultViewSchedMaxArcs = 512;    // mean cell arcs per level
// view-schedule forward chunks: whole tiles of one level, bounded for LDS staging
constexpr int kFwdCapA = 2816, kFwdCapG = 1152, kFwdCapT = 96;
// view-schedule backward chunks: whole tiles of one driver level
constexpr int kBwdCapS = 4096, kBwdCapD = 2048, kBwdCapT = 128;
constexpr size_t kViewTableLdsMax = 65536;            // LDS bytes for tables + axes
// fused spans: up to kSpanF consecutive gate levels per forward launch and kSpanB driver
// levels per backward launch (the lengths measured best on the 1M-pin design).  A span
// tile is processed in chunks of at most 64 lanes (cell arcs or sink slots): one chunk per
// level in the forward pass, one or more per level in the backward pass, at most kSpanF /
// kSpanB chunks per tile (the chunk records are held in registers).
constexpr int kSpanF = 8;
constexpr int kSpanB = 8;
constexpr int kSpanSlotsF = kSpanF * 64;
constexpr int kSpanSlotsB = kSpanB * 64;
// Span tiles per workgroup: one, so that the few tiles of a span launch spread over as
// many compute units as possible (a tile's gathers and table reads are issued by its own
// unit's address pipeline instead of queueing behind three other tiles').
constexpr int kSpanWaves = 1;
// (The span kernels hold a whole tile's prefetched records in registers; they are compiled
// for one wavefront per SIMD, so that long spans do not spill.)
// Level-kernel tiles per workgroup (the same reasoning: a level has a few hundred tiles).
constexpr int kLevelWaves = 1;
// Views a span wavefront computes (the others run as separate workgroups of the same
// launch): one for the forward, backward and adjoint spans.  Two views per backward
// wavefront (its slot records serve both) lost once the next launch's gathers were warmed
// into L2: the level chain, not the record round, then sets the launch time.
constexpr int kSpanViewsPerWave = 1;
constexpr int kBwdViewsPerWave = 1;
// Largest view count the fused spans serve: all (1, 2, 4, 8; measured faster than the level
// and view schedules for every count).
constexpr int kSpanMaxViews = 8;
// Largest arc and driver count of a graph with fused spans: the forward span tiles address
// per-arc and per-driver arrays of up to kSpanMaxViews views (8 bytes per view) by 32-bit
// byte offsets, and the span records pack a gate or driver into 26 bits.
constexpr int64_t kSpanMaxIndex = int64_t(1) << 26;
// Delay calculation of nets of at most 8 nodes: one lane per net of at most kDcLaneSinks
// sinks, a wavefront's first kDcWindow sinks staged in LDS; a net with more sinks (listed
// in dc_wide) gets a wavefront of its own.
constexpr int kDcLaneSinks = 16;
constexpr int kDcWindow = 64 * kDcLaneSinks;

// Device arrays of a graph (offsets in bytes into the one device buffer).
struct DevLayout {
    size_t net_node_ptr, node_parent, node_R, node_C;
    size_t fo_ptr, fo_arc, fo_tap, fo_cap;
    size_t arc_src, arc_meta, gate_arc_ptr;
    size_t ftile_arc, ftile_gate;
    size_t btile_drv, btile_slot, bslot_arc, bslot_out;
    size_t ep_drv;
    size_t fwd_lvl, bwd_lvl;       // per level (first tile, first arc|slot, first gate|driver)
    size_t ftile_maxk;             // per forward tile: the largest gate fanin in it
    size_t fwd_chunk;              // per forward chunk (first tile, first arc, first gate, level)
    size_t bwd_chunk;              // per backward chunk (first tile, first slot, first driver, level)
    size_t sp_crec, sp_arec;       // fused forward spans: level and arc records per tile
    size_t bp_crec, bp_srec;       // fused backward spans: level and slot records per tile
    size_t dc_wide;                // drivers of more than kDcLaneSinks sinks
    size_t total;
};

// Device pointers handed to the kernels by value.
struct DevGraph {
    const int32_t* net_node_ptr;   // [D+1]
    const int16_t* node_parent;    // [M] local parent, -1 at node 0
    const float* node_R;           // [M]
    const float* node_C;           // [M]
    const int32_t* fo_ptr;         // [D+1] sink list of every driver
    const int32_t* fo_arc;         // [A]   internal arc of each sink, ascending input arc id
    const uint8_t* fo_tap;         // [A]   RC node tapped by that sink
    const float* fo_cap;           // [A]   its pin capacitance
    const int32_t* arc_src;        // [A]   internal driver of the net feeding the arc
    const uint32_t* arc_meta;      // [A]   table id | (position in gate) << 16
    const int32_t* gate_arc_ptr;   // [G+1] cell arcs of each internal gate
    const int32_t* ftile_arc;      // [NF+1] forward tile -> first arc
    const int32_t* ftile_gate;     // [NF+1] forward tile -> first gate
    const int32_t* btile_drv;      // [NB+1] backward tile -> first driver
    const int32_t* btile_slot;     // [NB+1] backward tile -> first slot
    const int32_t* bslot_arc;      // [S]   sink arc of the slot, -1 for an endpoint slot
    const int32_t* bslot_out;      // [S]   driver of the sink's gate (or endpoint rank) | head bit
    const int32_t* ep_drv;         // [E]   internal driver of each endpoint rank
    const int32_t* ftile_maxk;     // [NF]  largest gate fanin of each forward tile
    const int32_t* fwd_chunk;      // [NC+1][4] forward chunks
    const int32_t* bwd_chunk;      // [NB+1][4] backward chunks in processing order (+ 4 ints of bounds)
    // Fused spans, fixed-stride records so that a wavefront loads all of its tile's records
    // in one round, indexed by (tile, level c, lane) only:
    const int4* sp_crec;   // [NT][kSpanF] forward level c of tile t: arcs, first LDS slot,
                           //   widest gate's arc count, levels of the tile
    const int4* sp_arec;   // [NT][kSpanF][64] per lane: cell arc, source (driver >= 0 or
                           //   -1 - LDS slot of an in-tile gate), gate | its rank among
                           //   the level's gates << 26 (-1: padding or idle lane), arc_meta
                           //   of the arc | the lane's gate end lane (next head of the
                           //   level) << 24 | head (first arc) << 31
    const int4* bp_crec;   // [NT][kSpanB] backward level c of tile t (top first): slots,
                           //   first LDS driver slot, most slots of a driver, levels of the tile
    const int4* bp_srec;   // [NT][kSpanB][64] per lane: sink arc (-1: endpoint slot), the
                           //   slot's output word (bslot_out), in-tile LDS source or -1 (-2:
                           //   padding or idle; low 16 bits, signed) | the lane's driver end lane
                           //   (next head of the level) << 16, driver | its rank among the
                           //   level's drivers << 26
    const int32_t* dc_wide;        // [n_dc_wide] drivers of more than kDcLaneSinks sinks, ascending
    int32_t n_pi, n_gates, n_drivers, n_arcs, n_dc_wide;
};

// One graph of a batched launch: its device layout, chunk count, view count and buffers
// (the slack buffers are null for a batch without a slack pass).
struct BatchItem {
    DevGraph G;
    int32_t NC, NV;
    const float* pi_ts;
    const float* load;
    const float* nd;
    const float* ni;
    float* drv_ts;
    float* arc_ts;
    float* arc_delay;
    uint8_t* argmax;
    // delay calculation outputs written by the batched delay calculation
    float* load_w;
    float* nd_w;
    float* ni_w;
    float* arc_load;
    // backward pass
    const float* ep_rat;
    float* drv_rat;
    float* arc_rat;
    float* drv_slack;
    float* arc_slack;
    double* tns;
    float* wns;
    int32_t E;
    int32_t ep_blocks;      // endpoint-summary workgroups of this graph
    int32_t ep_part0;       // its first partial in the batch's endpoint scratch
};

// Captured launch sequences (hipGraphs) of one call kind, each reused while its arguments
// (the key: every device pointer the launches bake in, the graph's own device buffer
// included, and every launch parameter) stay the same.  A few argument sets are kept,
// least recently used evicted, so that callers alternating between output sets (one per
// stream) replay instead of re-capturing on every call.  An exec is destroyed only after
// the device has drained, since it may still run on some stream.
constexpr int kLaunchCacheEntries = 4;
struct LaunchEntry {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};
struct LaunchCache {
    std::vector<LaunchEntry> e;
    uint64_t tick = 0;
};
// Waits for the device (hipDeviceSynchronize) if anything is cached, then destroys every
// captured sequence of c.
void drop_launches(LaunchCache& c);

}  // namespace sta

struct sta_graph {
    int32_t n_pi = 0, n_gates = 0, n_tables = 0;
    int64_t D = 0, A = 0, M = 0, L = 0, E = 0, S = 0;
    int32_t max_fanin = 0, max_fanout = 0, max_net_nodes = 0;
    int32_t n_dc_wide = 0;               // drivers of more than sta::kDcLaneSinks sinks
    bool chain_nets = false;             // every net an RC chain (node k's parent k - 1)
    std::vector<int32_t> drv_input, arc_input, gate_input, level, ep_driver;
    std::vector<int32_t> fwd_tile_ptr;   // [L+2]: tiles of gate level l are [p[l], p[l+1])
    std::vector<int32_t> ftile_arc_h, ftile_gate_h, btile_slot_h, btile_drv_h;   // host copies of the tiles
    std::vector<int32_t> bwd_tile_ptr;   // [L+2]: tiles of driver level l are [p[l], p[l+1])
    int64_t n_ftiles = 0, n_btiles = 0;
    // per-level maxima: forward tiles/arcs/gates, backward tiles/slots/drivers
    int32_t max_ft = 0, max_fa = 0, max_fg = 0, max_bt = 0, max_bs = 0, max_bd = 0;
    int32_t n_fchunks = 0, n_bchunks = 0;
    int32_t view_sched_max_arcs = sta::kDefaultViewSchedMaxArcs;
    bool view_auto = true;               // schedule left to the library (sta_set_schedule < 0)
    bool use_graphs = true;              // replay level-schedule launch sequences from hipGraphs
    bool use_spans = true;               // fused spans (kSpanF / kSpanB levels per launch) where possible
    std::vector<int32_t> span_tile_h;    // [NS+1] tiles of forward span s: [p[s], p[s+1]); a
    std::vector<uint8_t> span_fused_h;   //   span with span_fused_h[s] == 0 runs as a level launch
    std::vector<int32_t> span_lv_h;      // [NS][2] first and last gate level of span s (bottom up)
    int64_t n_sptiles = 0;
    std::vector<int32_t> bspan_tile_h;   // the same for the backward spans, whose driver levels
    std::vector<uint8_t> bspan_fused_h;  //   are bspan_lv_h[2b] (top) down to bspan_lv_h[2b + 1],
    std::vector<int32_t> bspan_lv_h;     //   processed top down
    sta_span_info span_info{};           // fusion plan figures (sta_graph_spans)
    mutable std::mutex cache_mu;
    mutable sta::LaunchCache fwd_cache, bwd_cache, adj_cache;
    sta::DevLayout lay{};
    std::vector<uint8_t> image;          // host image of the device buffer
    uint8_t* dev = nullptr;              // caller's device buffer after upload
};

namespace sta {
void set_error(const std::string& msg);
sta_status fail(sta_status st, const std::string& msg);
DevGraph dev_graph(const sta_graph* g);
size_t scratch_bytes();            // device scratch sta_slack needs (fixed size)
sta_status launch_check(const char* what);   // STA_E_HIP with the text of hipGetLastError

// Optional per-launch HIP-event bracketing of the calling thread (instrumentation only;
// sta_profile_begin / sta_profile_end switch it on and collect it).
struct ProfRec {
    const char* name;
    hipEvent_t start, stop;
};
struct Prof {
    bool on = false;
    bool failed = false;
    std::vector<ProfRec> recs;
};
Prof& prof();

template <typename F>
void prof_launch(const char* name, hipStream_t s, F&& launch) {
    Prof& p = prof();
    if (!p.on) {
        launch();
        return;
    }
    ProfRec r{name, nullptr, nullptr};
    if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) {
        p.failed = true;
        launch();
        return;
    }
    (void)hipEventRecord(r.start, s);
    launch();
    (void)hipEventRecord(r.stop, s);
    p.recs.push_back(r);
}
}  // namespace sta

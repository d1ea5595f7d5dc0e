// Host side of the library: design validation, levelization, the level-sorted CSR and
// the wave-sized work tiles, the device image and its upload.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "sta_internal.h"

namespace sta {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

sta_status fail(sta_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

DevGraph dev_graph(const sta_graph* g) {
    DevGraph d{};
    const DevLayout& L = g->lay;
    uint8_t* b = g->dev;
    d.net_node_ptr = reinterpret_cast<const int32_t*>(b + L.net_node_ptr);
    d.node_parent = reinterpret_cast<const int16_t*>(b + L.node_parent);
    d.node_R = reinterpret_cast<const float*>(b + L.node_R);
    d.node_C = reinterpret_cast<const float*>(b + L.node_C);
    d.fo_ptr = reinterpret_cast<const int32_t*>(b + L.fo_ptr);
    d.fo_arc = reinterpret_cast<const int32_t*>(b + L.fo_arc);
    d.fo_tap = reinterpret_cast<const uint8_t*>(b + L.fo_tap);
    d.fo_cap = reinterpret_cast<const float*>(b + L.fo_cap);
    d.arc_src = reinterpret_cast<const int32_t*>(b + L.arc_src);
    d.arc_meta = reinterpret_cast<const uint32_t*>(b + L.arc_meta);
    d.gate_arc_ptr = reinterpret_cast<const int32_t*>(b + L.gate_arc_ptr);
    d.ftile_arc = reinterpret_cast<const int32_t*>(b + L.ftile_arc);
    d.ftile_gate = reinterpret_cast<const int32_t*>(b + L.ftile_gate);
    d.btile_drv = reinterpret_cast<const int32_t*>(b + L.btile_drv);
    d.btile_slot = reinterpret_cast<const int32_t*>(b + L.btile_slot);
    d.bslot_arc = reinterpret_cast<const int32_t*>(b + L.bslot_arc);
    d.bslot_out = reinterpret_cast<const int32_t*>(b + L.bslot_out);
    d.ep_drv = reinterpret_cast<const int32_t*>(b + L.ep_drv);
    d.ftile_maxk = reinterpret_cast<const int32_t*>(b + L.ftile_maxk);
    d.fwd_chunk = reinterpret_cast<const int32_t*>(b + L.fwd_chunk);
    d.bwd_chunk = reinterpret_cast<const int32_t*>(b + L.bwd_chunk);
    d.sp_crec = reinterpret_cast<const int4*>(b + L.sp_crec);
    d.sp_arec = reinterpret_cast<const int4*>(b + L.sp_arec);
    d.bp_crec = reinterpret_cast<const int4*>(b + L.bp_crec);
    d.bp_srec = reinterpret_cast<const int4*>(b + L.bp_srec);
    d.dc_wide = reinterpret_cast<const int32_t*>(b + L.dc_wide);
    d.n_dc_wide = g->n_dc_wide;
    d.n_pi = g->n_pi;
    d.n_gates = g->n_gates;
    d.n_drivers = static_cast<int32_t>(g->D);
    d.n_arcs = static_cast<int32_t>(g->A);
    return d;
}

static bool finite_nonneg(float v) { return std::isfinite(v) && v >= 0.0f; }

// Lane after placing a gate of k cell arcs (a driver of k sink slots) at lane pos of a span
// chunk: one of up to 16 never straddles a 16-lane row (the kernels reduce it inside rows).
static int32_t span_lane(int32_t pos, int32_t k) {
    if (k <= 16 && (pos & 15) + k > 16) pos = (pos + 15) & ~15;
    return pos + k;
}

// A tile level may take several 64-lane chunks.  Placement state of a level: chunks
// opened * 128 + lanes used in the last one.  Adding k (<= 64) lanes opens a chunk when
// the last one cannot take them whole.
static int32_t span_place(int32_t st, int32_t k) {
    int32_t ch = st >> 7, ln = st & 127;
    if (ch == 0) ch = 1;
    int32_t p = span_lane(ln, k);
    if (p > 64) {
        ++ch;
        p = k;
    }
    return ch * 128 + p;
}

static sta_status build(const sta_design_desc* d, sta_graph* g, int32_t cap_f, int32_t cap_b) {
    if (!d) return fail(STA_E_ARG, "sta_build_graph: null design");
    if (d->n_pi < 0 || d->n_gates < 0) return fail(STA_E_ARG, "sta_build_graph: negative n_pi or n_gates");
    if (d->n_tables < 1 || d->n_tables > STA_MAX_TABLES)
        return fail(STA_E_ARG, "sta_build_graph: n_tables must be in 1..65535");
    const int64_t G = d->n_gates, P = d->n_pi, D = P + G;
    if (D > INT32_MAX / 2) return fail(STA_E_ARG, "sta_build_graph: too many drivers");
    if (!d->gate_arc_ptr || !d->net_node_ptr) return fail(STA_E_ARG, "sta_build_graph: null gate_arc_ptr or net_node_ptr");
    if (d->gate_arc_ptr[0] != 0) return fail(STA_E_ARG, "sta_build_graph: gate_arc_ptr[0] != 0");
    int max_fanin = 0;
    for (int64_t q = 0; q < G; ++q) {
        int64_t k = int64_t(d->gate_arc_ptr[q + 1]) - d->gate_arc_ptr[q];
        if (k < 1 || k > STA_MAX_FANIN)
            return fail(STA_E_ARG, "sta_build_graph: gate " + std::to_string(q) + " has " + std::to_string(k) +
                                       " arcs (allowed 1.." + std::to_string(STA_MAX_FANIN) + ")");
        max_fanin = std::max<int>(max_fanin, int(k));
    }
    const int64_t A = d->gate_arc_ptr[G];
    if (A > INT32_MAX / 2) return fail(STA_E_ARG, "sta_build_graph: too many arcs");
    if (A > 0 && (!d->arc_drv || !d->arc_tbl || !d->arc_tap || !d->arc_pincap))
        return fail(STA_E_ARG, "sta_build_graph: null arc array");
    if (d->net_node_ptr[0] != 0) return fail(STA_E_ARG, "sta_build_graph: net_node_ptr[0] != 0");
    int max_nodes = 0;
    for (int64_t u = 0; u < D; ++u) {
        int64_t m = int64_t(d->net_node_ptr[u + 1]) - d->net_node_ptr[u];
        if (m < 1 || m > STA_MAX_NET_NODES)
            return fail(STA_E_ARG, "sta_build_graph: net of driver " + std::to_string(u) + " has " +
                                       std::to_string(m) + " nodes (allowed 1.." + std::to_string(STA_MAX_NET_NODES) + ")");
        max_nodes = std::max<int>(max_nodes, int(m));
    }
    const int64_t M = d->net_node_ptr[D];
    if (M > 0 && (!d->node_parent || !d->node_R || !d->node_C)) return fail(STA_E_ARG, "sta_build_graph: null node array");
    bool chains = true;   // every net an RC chain (node k's parent k - 1)
    for (int64_t u = 0; u < D; ++u) {
        int64_t n0 = d->net_node_ptr[u], m = d->net_node_ptr[u + 1] - n0;
        if (d->node_parent[n0] != -1) return fail(STA_E_RANGE, "sta_build_graph: node 0 of net " + std::to_string(u) + " has a parent");
        for (int64_t k = 1; k < m; ++k) {
            int32_t p = d->node_parent[n0 + k];
            chains = chains && p == k - 1;
            if (p < 0 || p >= k)
                return fail(STA_E_RANGE, "sta_build_graph: net " + std::to_string(u) + " node " + std::to_string(k) +
                                             " has parent " + std::to_string(p) + " (must be in 0..node-1)");
        }
    }
    for (int64_t k = 0; k < M; ++k) {
        if (!finite_nonneg(d->node_C[k])) return fail(STA_E_NONFINITE, "sta_build_graph: node_C[" + std::to_string(k) + "] is not finite and >= 0");
        if (!finite_nonneg(d->node_R[k])) return fail(STA_E_NONFINITE, "sta_build_graph: node_R[" + std::to_string(k) + "] is not finite and >= 0");
    }
    for (int64_t a = 0; a < A; ++a) {
        int32_t u = d->arc_drv[a];
        if (u < 0 || u >= D) return fail(STA_E_RANGE, "sta_build_graph: arc " + std::to_string(a) + " driver " + std::to_string(u) + " out of range");
        if (d->arc_tbl[a] < 0 || d->arc_tbl[a] >= d->n_tables)
            return fail(STA_E_RANGE, "sta_build_graph: arc " + std::to_string(a) + " table out of range");
        int32_t m = d->net_node_ptr[u + 1] - d->net_node_ptr[u];
        if (d->arc_tap[a] < 0 || d->arc_tap[a] >= m)
            return fail(STA_E_RANGE, "sta_build_graph: arc " + std::to_string(a) + " taps node " + std::to_string(d->arc_tap[a]) +
                                         " of a " + std::to_string(m) + "-node net");
        if (!finite_nonneg(d->arc_pincap[a])) return fail(STA_E_NONFINITE, "sta_build_graph: arc_pincap[" + std::to_string(a) + "] is not finite and >= 0");
    }

    // ---- levelize (Kahn) -------------------------------------------------------------
    std::vector<int32_t> fo_cnt(D + 1, 0), fo_ptr_in(D + 1, 0), fo_in(A);
    for (int64_t a = 0; a < A; ++a) fo_cnt[d->arc_drv[a]]++;
    for (int64_t u = 0; u < D; ++u) fo_ptr_in[u + 1] = fo_ptr_in[u] + fo_cnt[u];
    {
        std::vector<int32_t> fill(fo_ptr_in.begin(), fo_ptr_in.end() - 1);
        for (int64_t a = 0; a < A; ++a) fo_in[fill[d->arc_drv[a]]++] = int32_t(a);   // ascending input arc id
    }
    std::vector<int32_t> gate_of_arc(A);
    for (int64_t q = 0; q < G; ++q)
        for (int32_t a = d->gate_arc_ptr[q]; a < d->gate_arc_ptr[q + 1]; ++a) gate_of_arc[a] = int32_t(q);
    std::vector<int32_t> indeg(G, 0), lev(D, 0), queue;
    queue.reserve(G);
    for (int64_t a = 0; a < A; ++a)
        if (d->arc_drv[a] >= P) indeg[gate_of_arc[a]]++;
    for (int64_t q = 0; q < G; ++q)
        if (indeg[q] == 0) queue.push_back(int32_t(q));
    for (size_t h = 0; h < queue.size(); ++h) {
        int32_t q = queue[h];
        int32_t lv = 0;
        for (int32_t a = d->gate_arc_ptr[q]; a < d->gate_arc_ptr[q + 1]; ++a) lv = std::max(lv, lev[d->arc_drv[a]]);
        lev[P + q] = lv + 1;
        int64_t o = P + q;
        for (int32_t i = fo_ptr_in[o]; i < fo_ptr_in[o + 1]; ++i) {
            int32_t c = gate_of_arc[fo_in[i]];
            if (--indeg[c] == 0) queue.push_back(c);
        }
    }
    if (int64_t(queue.size()) != G)
        return fail(STA_E_CYCLE, "sta_build_graph: combinational cycle through " + std::to_string(G - queue.size()) + " gates");
    int32_t Lmax = 0;
    for (int64_t u = 0; u < D; ++u) Lmax = std::max(Lmax, lev[u]);

    // ---- internal numbering: gates by (level, input id) ------------------------------
    std::vector<int32_t> lvl_cnt(Lmax + 2, 0);
    for (int64_t q = 0; q < G; ++q) lvl_cnt[lev[P + q]]++;
    std::vector<int32_t> lvl_gate_ptr(Lmax + 2, 0);   // gates of level l: [ptr[l-1], ptr[l]) with ptr[0] = 0
    for (int32_t l = 1; l <= Lmax; ++l) lvl_gate_ptr[l] = lvl_gate_ptr[l - 1] + lvl_cnt[l];
    std::vector<int32_t> gate_int(G), gate_in(G);
    {
        std::vector<int32_t> fill(Lmax + 1, 0);
        for (int32_t l = 1; l <= Lmax; ++l) fill[l] = lvl_gate_ptr[l - 1];
        for (int64_t q = 0; q < G; ++q) {
            int32_t i = fill[lev[P + q]]++;
            gate_int[q] = i;
            gate_in[i] = int32_t(q);
        }
    }
    auto drv_int = [&](int64_t u) -> int32_t { return u < P ? int32_t(u) : int32_t(P + gate_int[u - P]); };
    g->drv_input.resize(D);
    g->level.resize(D);
    for (int64_t u = 0; u < D; ++u) {
        int32_t i = drv_int(u);
        g->drv_input[i] = int32_t(u);
        g->level[i] = lev[u];
    }
    g->gate_input = gate_in;
    std::vector<int32_t> arc_int(A), gate_arc_ptr_int(G + 1, 0);
    g->arc_input.resize(A);
    for (int64_t i = 0; i < G; ++i) {
        int32_t q = gate_in[i];
        int32_t k = d->gate_arc_ptr[q + 1] - d->gate_arc_ptr[q];
        gate_arc_ptr_int[i + 1] = gate_arc_ptr_int[i] + k;
        for (int32_t j = 0; j < k; ++j) {
            int32_t a = d->gate_arc_ptr[q] + j;
            arc_int[a] = gate_arc_ptr_int[i] + j;
            g->arc_input[gate_arc_ptr_int[i] + j] = a;
        }
    }

    // ---- endpoints -------------------------------------------------------------------
    std::vector<int32_t> ep_rank_in(D, -1);
    int64_t E = 0;
    for (int64_t u = 0; u < D; ++u)
        if (fo_cnt[u] == 0) ep_rank_in[u] = int32_t(E++);
    g->ep_driver.resize(E);
    for (int64_t u = 0; u < D; ++u)
        if (ep_rank_in[u] >= 0) g->ep_driver[ep_rank_in[u]] = drv_int(u);

    int max_fanout = 0;
    for (int64_t u = 0; u < D; ++u) max_fanout = std::max(max_fanout, fo_cnt[u]);

    // ---- forward tiles: consecutive whole gates of one level, <= 64 arcs -------------
    std::vector<int32_t> ftile_arc, ftile_gate;
    g->fwd_tile_ptr.assign(Lmax + 2, 0);
    for (int32_t l = 1; l <= Lmax; ++l) {
        g->fwd_tile_ptr[l] = int32_t(ftile_arc.size());
        int32_t q0 = lvl_gate_ptr[l - 1], q1 = lvl_gate_ptr[l];
        int32_t q = q0;
        while (q < q1) {
            ftile_arc.push_back(gate_arc_ptr_int[q]);
            ftile_gate.push_back(q);
            int32_t used = 0;
            while (q < q1 && used + (gate_arc_ptr_int[q + 1] - gate_arc_ptr_int[q]) <= kTileSlots) {
                used += gate_arc_ptr_int[q + 1] - gate_arc_ptr_int[q];
                ++q;
            }
        }
    }
    g->fwd_tile_ptr[Lmax + 1] = int32_t(ftile_arc.size());
    const int64_t NF = int64_t(ftile_arc.size());
    ftile_arc.push_back(int32_t(A));
    ftile_gate.push_back(int32_t(G));
    std::vector<int32_t> ftile_maxk(std::max<int64_t>(NF, 1), 0);
    for (int64_t t = 0; t < NF; ++t)
        for (int32_t q = ftile_gate[t]; q < ftile_gate[t + 1]; ++q)
            ftile_maxk[t] = std::max(ftile_maxk[t], gate_arc_ptr_int[q + 1] - gate_arc_ptr_int[q]);
    // forward chunks: consecutive whole tiles of one level within the staging bounds
    std::vector<int32_t> fchunk;   // 4 ints per chunk: first tile, first arc, first gate, level
    for (int32_t l = 1; l <= Lmax; ++l) {
        int32_t t = g->fwd_tile_ptr[l];
        const int32_t t1 = g->fwd_tile_ptr[l + 1];
        while (t < t1) {
            const int32_t c0 = t;
            while (t < t1 && (t - c0) < kFwdCapT && ftile_arc[t + 1] - ftile_arc[c0] <= kFwdCapA &&
                   ftile_gate[t + 1] - ftile_gate[c0] <= kFwdCapG)
                ++t;
            if (t == c0) ++t;   // a single tile always fits (<= 64 arcs and gates)
            fchunk.insert(fchunk.end(), {c0, ftile_arc[c0], ftile_gate[c0], l});
        }
    }
    g->n_fchunks = int32_t(fchunk.size() / 4);
    fchunk.insert(fchunk.end(), {int32_t(NF), int32_t(A), int32_t(G), int32_t(Lmax + 1)});

    // ---- internal sink lists and backward slots --------------------------------------
    // driver i's slots: one per sink (ascending input arc id), or one endpoint slot
    std::vector<int32_t> fo_ptr(D + 1, 0), fo_arc(A);
    std::vector<uint8_t> fo_tap(A);
    std::vector<float> fo_cap(A);
    for (int64_t i = 0; i < D; ++i) fo_ptr[i + 1] = fo_ptr[i] + fo_cnt[g->drv_input[i]];
    for (int64_t i = 0; i < D; ++i) {
        int32_t u = g->drv_input[i];
        for (int32_t j = 0; j < fo_cnt[u]; ++j) {
            int32_t a = fo_in[fo_ptr_in[u] + j];
            fo_arc[fo_ptr[i] + j] = arc_int[a];
            fo_tap[fo_ptr[i] + j] = uint8_t(d->arc_tap[a]);
            fo_cap[fo_ptr[i] + j] = d->arc_pincap[a];
        }
    }
    std::vector<int32_t> dc_wide;
    for (int64_t i = 0; i < D; ++i)
        if (fo_ptr[i + 1] - fo_ptr[i] > kDcLaneSinks) dc_wide.push_back(int32_t(i));
    g->n_dc_wide = int32_t(dc_wide.size());
    std::vector<int32_t> slot_ptr(D + 1, 0);
    for (int64_t i = 0; i < D; ++i) slot_ptr[i + 1] = slot_ptr[i] + std::max(1, fo_ptr[i + 1] - fo_ptr[i]);
    const int64_t S = slot_ptr[D];
    std::vector<int32_t> bslot_arc(S), bslot_out(S);
    std::vector<int32_t> int_gate_of_arc(A);
    for (int64_t i = 0; i < G; ++i)
        for (int32_t a = gate_arc_ptr_int[i]; a < gate_arc_ptr_int[i + 1]; ++a) int_gate_of_arc[a] = int32_t(i);
    for (int64_t i = 0; i < D; ++i) {
        int32_t nfo = fo_ptr[i + 1] - fo_ptr[i];
        if (nfo == 0) {
            bslot_arc[slot_ptr[i]] = -1;
            bslot_out[slot_ptr[i]] = int32_t(uint32_t(ep_rank_in[g->drv_input[i]]) | kHeadBit);
        } else {
            for (int32_t j = 0; j < nfo; ++j) {
                int32_t a = fo_arc[fo_ptr[i] + j];
                bslot_arc[slot_ptr[i] + j] = a;
                uint32_t o = uint32_t(P + int_gate_of_arc[a]);
                bslot_out[slot_ptr[i] + j] = int32_t(o | (j == 0 ? kHeadBit : 0u));
            }
        }
    }
    // backward tiles: consecutive drivers of one level, <= 64 slots, or one large driver
    std::vector<int32_t> btile_drv, btile_slot;
    g->bwd_tile_ptr.assign(Lmax + 2, 0);
    for (int32_t l = 0; l <= Lmax; ++l) {
        g->bwd_tile_ptr[l] = int32_t(btile_drv.size());
        int64_t i0 = (l == 0) ? 0 : P + lvl_gate_ptr[l - 1];
        int64_t i1 = (l == 0) ? P : P + lvl_gate_ptr[l];
        int64_t i = i0;
        while (i < i1) {
            btile_drv.push_back(int32_t(i));
            btile_slot.push_back(slot_ptr[i]);
            int32_t first = slot_ptr[i + 1] - slot_ptr[i];
            if (first > kTileSlots) { ++i; continue; }
            int32_t used = 0;
            while (i < i1 && slot_ptr[i + 1] - slot_ptr[i] <= kTileSlots && used + (slot_ptr[i + 1] - slot_ptr[i]) <= kTileSlots) {
                used += slot_ptr[i + 1] - slot_ptr[i];
                ++i;
            }
        }
    }
    g->bwd_tile_ptr[Lmax + 1] = int32_t(btile_drv.size());
    const int64_t NB = int64_t(btile_drv.size());
    btile_drv.push_back(int32_t(D));
    btile_slot.push_back(int32_t(S));
    // backward chunks, in processing order (levels L..0, tiles ascending): each entry is
    // (first tile, tile end, first slot, slot end, first driver, driver end, level, 0).
    // No chunk is made when a single tile exceeds the bounds (then only the level
    // schedule runs the backward pass).
    std::vector<int32_t> bchunk;
    bool bwd_chunkable = true;
    for (int32_t l = Lmax; l >= 0 && bwd_chunkable; --l) {
        int32_t t = g->bwd_tile_ptr[l];
        const int32_t t1 = g->bwd_tile_ptr[l + 1];
        while (t < t1) {
            const int32_t c0 = t;
            while (t < t1 && (t - c0) < kBwdCapT && btile_slot[t + 1] - btile_slot[c0] <= kBwdCapS &&
                   btile_drv[t + 1] - btile_drv[c0] <= kBwdCapD)
                ++t;
            if (t == c0) { bwd_chunkable = false; break; }
            bchunk.insert(bchunk.end(), {c0, t, btile_slot[c0], btile_slot[t], btile_drv[c0], btile_drv[t], l, 0});
        }
    }
    if (!bwd_chunkable) bchunk.clear();
    g->n_bchunks = int32_t(bchunk.size() / 8);
    bchunk.insert(bchunk.end(), {0, 0, 0, 0, 0, 0, -1, 0});

    // ---- internal arcs and nets --------------------------------------------------------
    std::vector<int32_t> arc_src(A);
    std::vector<uint32_t> arc_meta(A);
    for (int64_t i = 0; i < A; ++i) {
        int32_t a = g->arc_input[i];
        arc_src[i] = drv_int(d->arc_drv[a]);
        uint32_t kpos = uint32_t(i - gate_arc_ptr_int[int_gate_of_arc[i]]);
        arc_meta[i] = uint32_t(d->arc_tbl[a]) | (kpos << 16);
    }
    std::vector<int32_t> net_ptr(D + 1, 0);
    for (int64_t i = 0; i < D; ++i) {
        int32_t u = g->drv_input[i];
        net_ptr[i + 1] = net_ptr[i] + (d->net_node_ptr[u + 1] - d->net_node_ptr[u]);
    }
    std::vector<int16_t> node_parent(M);
    std::vector<float> node_R(M), node_C(M);
    for (int64_t i = 0; i < D; ++i) {
        int32_t u = g->drv_input[i];
        int32_t s0 = d->net_node_ptr[u], m = d->net_node_ptr[u + 1] - s0;
        for (int32_t k = 0; k < m; ++k) {
            node_parent[net_ptr[i] + k] = int16_t(d->node_parent[s0 + k]);
            node_R[net_ptr[i] + k] = d->node_R[s0 + k];
            node_C[net_ptr[i] + k] = d->node_C[s0 + k];
        }
    }



    // ---- fused backward spans ------------------------------------------------------------
    // Spans of driver levels, processed top down: from the highest level not yet covered,
    // the longest span [top - n + 1, top] (n <= cap_b <= kSpanB) that can be tiled is taken; a level
    // that cannot be tiled even alone runs as a level launch.  A tile is a set of drivers
    // closed under in-span sinks: the output driver of every gate a tile driver feeds, when
    // its level lies in the span, is in the tile too.  Roots are taken bottom level first;
    // a tile holds <= 64 slots per level.
    std::vector<int32_t> bp_tile, bp_chunk, bp_slot, bp_src, bp_drv;
    {
        g->bspan_tile_h.clear();
        g->bspan_fused_h.clear();
        g->bspan_lv_h.clear();
        auto drv_range = [&](int32_t l, int64_t& i0, int64_t& i1) {
            i0 = (l == 0) ? 0 : P + lvl_gate_ptr[l - 1];
            i1 = (l == 0) ? P : P + lvl_gate_ptr[l];
        };
        std::vector<int32_t> mark(D, -1), dslot(D, -1), tile_mark(D, -1), stack, cone;
        std::vector<uint8_t> covered(D, 0);
        int32_t tile_id = 0;   // unique per filled tile (never reused)
        int32_t stamp = 0;     // unique per cone search (never reused)
        auto lv = [&](int64_t i) { return g->level[i]; };
        auto nslots = [&](int64_t i) { return slot_ptr[i + 1] - slot_ptr[i]; };
        // tiles the span [bot, top]; on failure removes what it appended and returns false
        auto try_span = [&](int32_t top, int32_t bot) -> bool {
            // (the records pack a driver into 26 bits: larger graphs run level launches)
            if (A > kSpanMaxIndex || D > kSpanMaxIndex) return false;
            auto in_span = [&](int64_t i) { return lv(i) >= bot && lv(i) <= top; };
            const int32_t nl = top - bot + 1;
            const size_t t0 = bp_tile.size(), c0all = bp_chunk.size(), s0all = bp_slot.size();
            bool ok = true;
            std::vector<std::vector<int32_t>> td(nl);     // drivers per level (index top - level)
            int32_t tslots[kSpanB] = {};                  // placement state per level (span_place)
            auto flush = [&]() {
                bool any = false;
                for (int j = 0; j < nl; ++j) any = any || !td[j].empty();
                if (!any) return;
                const int32_t c0 = int32_t(bp_chunk.size() / 4);
                int32_t ds = 0;
                for (int j = 0; j < nl; ++j)
                    for (int32_t i : td[j]) dslot[i] = ds++;
                int32_t nch = 0;
                for (int j = 0; j < nl; ++j) {      // j = 0 is the top level: processed first
                    if (td[j].empty()) continue;
                    int32_t ts0 = int32_t(bp_slot.size());
                    int32_t maxs = 1, first = td[j][0];
                    for (int32_t i : td[j]) {
                        if (span_lane(int32_t(bp_slot.size()) - ts0, nslots(i)) > kTileSlots) {
                            // the level continues in a new chunk
                            bp_chunk.insert(bp_chunk.end(), {ts0, int32_t(bp_slot.size()) - ts0, dslot[first], maxs});
                            ++nch;
                            ts0 = int32_t(bp_slot.size());
                            maxs = 1;
                            first = i;
                        }
                        maxs = std::max(maxs, nslots(i));
                        // padding lanes (slot -1) keep a driver of <= 16 slots inside one row
                        const int32_t at = span_lane(int32_t(bp_slot.size()) - ts0, nslots(i)) - nslots(i);
                        while (int32_t(bp_slot.size()) - ts0 < at) {
                            bp_slot.push_back(-1);
                            bp_src.push_back(-2);
                            bp_drv.push_back(0);
                        }
                        for (int32_t sl = slot_ptr[i]; sl < slot_ptr[i + 1]; ++sl) {
                            const int32_t sa = bslot_arc[sl];
                            int32_t src = -1;
                            if (sa >= 0) {
                                const int32_t o = int32_t(P + int_gate_of_arc[sa]);
                                if (in_span(o)) src = dslot[o];
                            }
                            bp_slot.push_back(sl);
                            bp_src.push_back(src);
                            bp_drv.push_back(i);
                        }
                    }
                    bp_chunk.insert(bp_chunk.end(), {ts0, int32_t(bp_slot.size()) - ts0, dslot[first], maxs});
                    ++nch;
                }
                bp_tile.insert(bp_tile.end(), {c0, nch, 0, ds});
                for (int j = 0; j < nl; ++j) { td[j].clear(); tslots[j] = 0; }
                ++tile_id;
            };
            for (int32_t l = bot; l <= top && ok; ++l) {
                int64_t i0, i1;
                drv_range(l, i0, i1);
                for (int64_t r = i0; r < i1 && ok; ++r) {
                    if (covered[r]) continue;
                    cone.clear();
                    stack.assign(1, int32_t(r));
                    const int32_t st = stamp++;
                    mark[r] = st;
                    // (a cone of more slots than a whole tile holds cannot be tiled: stop there)
                    int64_t cone_slots = 0;
                    while (!stack.empty() && cone_slots <= int64_t(kSpanB) * kTileSlots) {
                        const int32_t i = stack.back();
                        stack.pop_back();
                        cone.push_back(i);
                        cone_slots += nslots(i);
                        for (int32_t sl = slot_ptr[i]; sl < slot_ptr[i + 1]; ++sl) {
                            const int32_t sa = bslot_arc[sl];
                            if (sa < 0) continue;
                            const int32_t o = int32_t(P + int_gate_of_arc[sa]);
                            if (in_span(o) && mark[o] != st) { mark[o] = st; stack.push_back(o); }
                        }
                    }
                    if (cone_slots > int64_t(kSpanB) * kTileSlots) { ok = false; break; }
                    // chunks per level after adding the cone (in insertion order) to the
                    // current tile, or alone; a tile holds at most kSpanB chunks in all
                    std::sort(cone.begin(), cone.end());
                    int32_t add[kSpanB], alone[kSpanB] = {};
                    bool wide = false;
                    for (int j = 0; j < nl; ++j) add[j] = tslots[j];
                    for (int32_t i : cone) {
                        const int32_t j = top - lv(i);
                        wide = wide || nslots(i) > kTileSlots;
                        alone[j] = span_place(alone[j], nslots(i));
                        if (tile_mark[i] != tile_id) add[j] = span_place(add[j], nslots(i));
                    }
                    int32_t ch_add = 0, ch_alone = 0;
                    for (int j = 0; j < nl; ++j) {
                        ch_add += add[j] >> 7;
                        ch_alone += alone[j] >> 7;
                    }
                    const bool fits = ch_add <= kSpanB;
                    const bool fits_alone = !wide && ch_alone <= kSpanB;
                    if (!fits_alone) { ok = false; break; }
                    if (!fits) {
                        flush();
                        for (int j = 0; j < nl; ++j) add[j] = alone[j];
                    }
                    for (int32_t i : cone) {
                        if (tile_mark[i] == tile_id) continue;
                        tile_mark[i] = tile_id;
                        td[top - lv(i)].push_back(i);
                        covered[i] = 1;
                    }
                    for (int j = 0; j < nl; ++j) tslots[j] = add[j];
                }
            }
            if (ok) {
                flush();
                return true;
            }
            bp_tile.resize(t0);
            bp_chunk.resize(c0all);
            bp_slot.resize(s0all);
            bp_src.resize(s0all);
            bp_drv.resize(s0all);
            ++tile_id;
            for (int32_t l = bot; l <= top; ++l) {
                int64_t i0, i1;
                drv_range(l, i0, i1);
                for (int64_t r = i0; r < i1; ++r) covered[r] = 0;
            }
            return false;
        };
        for (int32_t top = Lmax; top >= 0;) {
            const int32_t t0 = int32_t(bp_tile.size() / 4);
            int32_t n = std::min<int32_t>(cap_b, top + 1);
            bool ok = try_span(top, top - n + 1);
            while (!ok && n > 1) {
                --n;
                ok = try_span(top, top - n + 1);
            }
            g->bspan_tile_h.push_back(t0);
            g->bspan_fused_h.push_back(uint8_t(ok));
            g->bspan_lv_h.insert(g->bspan_lv_h.end(), {top, top - n + 1});
            top -= n;
        }
        g->bspan_tile_h.push_back(int32_t(bp_tile.size() / 4));
    }

    // ---- fused forward spans -------------------------------------------------------------
    // Spans of gate levels, bottom up: from the lowest level not yet covered, the longest
    // span [l0, l0 + n - 1] (n <= cap_f <= kSpanF) that can be tiled is taken; a level that cannot
    // be tiled even alone runs as a level launch.  A span tile computes, level by level
    // inside one wavefront, a set of gates closed under in-span fanin: every in-span driver
    // of a tile gate is itself in the tile (so it may be computed by several tiles,
    // identically).  Roots are taken top level first; a tile holds <= 64 arcs per level.
    std::vector<int32_t> sp_tile, sp_chunk, sp_ta_arc, sp_ta_src, sp_ta_gate;
    {
        g->span_tile_h.clear();
        g->span_fused_h.clear();
        g->span_lv_h.clear();
        std::vector<int32_t> gate_lv(G);
        for (int32_t l = 1; l <= Lmax; ++l)
            for (int32_t q = lvl_gate_ptr[l - 1]; q < lvl_gate_ptr[l]; ++q) gate_lv[q] = l;
        std::vector<int32_t> mark(G, -1), slot_of(G, -1);
        std::vector<uint8_t> covered(G, 0);
        std::vector<int32_t> stack, cone;
        std::vector<int32_t> tile_mark(G, -1);   // id of the tile being filled that holds the gate
        int32_t tile_id = 0;                      // unique per filled tile (never reused)
        int32_t stamp = 0;                        // unique per cone search (never reused)
        auto try_span = [&](int32_t l0, int32_t l1) -> bool {
            // the forward span kernel addresses per-arc and per-driver arrays of up to 8
            // views by 32-bit byte offsets, and the records pack a gate into 26 bits: larger
            // graphs run their forward levels as level launches
            if (A > kSpanMaxIndex || D > kSpanMaxIndex) return false;
            const int32_t q0 = lvl_gate_ptr[l0 - 1], q1 = lvl_gate_ptr[l1];
            auto in_span = [&](int32_t u) { return u >= P && (u - P) >= q0 && (u - P) < q1; };
            const int32_t nl = l1 - l0 + 1;
            const size_t t0 = sp_tile.size(), c0all = sp_chunk.size(), a0all = sp_ta_arc.size();
            bool ok = true;
            // the tile being filled: gates per level in insertion order, placement state
            // per level (span_place)
            std::vector<std::vector<int32_t>> tg(nl);
            int32_t tarcs[kSpanF] = {};
            auto nk = [&](int32_t q) { return gate_arc_ptr_int[q + 1] - gate_arc_ptr_int[q]; };
            auto flush = [&]() {
                bool any = false;
                for (int j = 0; j < nl; ++j) any = any || !tg[j].empty();
                if (!any) return;
                const int32_t c0 = int32_t(sp_chunk.size() / 4);
                int32_t slot = 0;
                for (int j = 0; j < nl; ++j)
                    for (int32_t q : tg[j]) slot_of[q] = slot++;
                int32_t nch = 0;
                for (int j = 0; j < nl; ++j) {
                    if (tg[j].empty()) continue;
                    int32_t ta0 = int32_t(sp_ta_arc.size());
                    int32_t maxk = 0, first = tg[j][0];
                    for (int32_t q : tg[j]) {
                        if (span_lane(int32_t(sp_ta_arc.size()) - ta0, nk(q)) > kTileSlots) {
                            // the level continues in a new chunk
                            sp_chunk.insert(sp_chunk.end(), {ta0, int32_t(sp_ta_arc.size()) - ta0, slot_of[first], maxk});
                            ++nch;
                            ta0 = int32_t(sp_ta_arc.size());
                            maxk = 0;
                            first = q;
                        }
                        maxk = std::max(maxk, nk(q));
                        // padding lanes (gate -1) keep a gate of <= 16 arcs inside one 16-lane row
                        const int32_t at = span_lane(int32_t(sp_ta_arc.size()) - ta0, nk(q)) - nk(q);
                        while (int32_t(sp_ta_arc.size()) - ta0 < at) {
                            sp_ta_arc.push_back(0);
                            sp_ta_src.push_back(0);
                            sp_ta_gate.push_back(-1);
                        }
                        for (int32_t a = gate_arc_ptr_int[q]; a < gate_arc_ptr_int[q + 1]; ++a) {
                            const int32_t u = arc_src[a];
                            sp_ta_arc.push_back(a);
                            sp_ta_src.push_back(in_span(u) ? -1 - slot_of[u - P] : u);
                            sp_ta_gate.push_back(q);
                        }
                    }
                    sp_chunk.insert(sp_chunk.end(), {ta0, int32_t(sp_ta_arc.size()) - ta0, slot_of[first], maxk});
                    ++nch;
                }
                sp_tile.insert(sp_tile.end(), {c0, nch, 0, slot});
                for (int j = 0; j < nl; ++j) { tg[j].clear(); tarcs[j] = 0; }
                ++tile_id;
            };
            for (int32_t l = l1; l >= l0 && ok; --l) {
                for (int32_t r = lvl_gate_ptr[l - 1]; r < lvl_gate_ptr[l] && ok; ++r) {
                    if (covered[r]) continue;
                    // cone of r: r and its in-span ancestors
                    cone.clear();
                    stack.assign(1, r);
                    const int32_t st = stamp++;
                    mark[r] = st;
                    // (a cone of more arcs than a whole tile holds cannot be tiled: stop there)
                    int64_t cone_arcs = 0;
                    while (!stack.empty() && cone_arcs <= int64_t(kSpanF) * kTileSlots) {
                        const int32_t q = stack.back();
                        stack.pop_back();
                        cone.push_back(q);
                        cone_arcs += nk(q);
                        for (int32_t a = gate_arc_ptr_int[q]; a < gate_arc_ptr_int[q + 1]; ++a) {
                            const int32_t u = arc_src[a];
                            if (in_span(u) && mark[u - P] != st) { mark[u - P] = st; stack.push_back(u - P); }
                        }
                    }
                    if (cone_arcs > int64_t(kSpanF) * kTileSlots) { ok = false; break; }
                    // inserted in ascending gate order per level (drivers precede users: lower
                    // level); lanes per level after adding the cone to the current tile, or alone
                    std::sort(cone.begin(), cone.end());
                    int32_t add[kSpanF], alone[kSpanF] = {};
                    bool wide = false;
                    for (int j = 0; j < nl; ++j) add[j] = tarcs[j];
                    for (int32_t q : cone) {
                        const int32_t j = gate_lv[q] - l0;
                        wide = wide || nk(q) > kTileSlots;
                        alone[j] = span_place(alone[j], nk(q));
                        if (tile_mark[q] != tile_id) add[j] = span_place(add[j], nk(q));
                    }
                    // forward levels keep one chunk each: a level's chunks run one after
                    // another in the wavefront, and a forward level is the expensive one
                    bool fits = true, fits_alone = !wide;
                    for (int j = 0; j < nl; ++j) {
                        fits = fits && (add[j] >> 7) <= 1;
                        fits_alone = fits_alone && (alone[j] >> 7) <= 1;
                    }
                    if (!fits_alone) { ok = false; break; }
                    if (!fits) {
                        flush();
                        for (int j = 0; j < nl; ++j) add[j] = alone[j];
                    }
                    for (int32_t q : cone) {
                        if (tile_mark[q] == tile_id) continue;
                        tile_mark[q] = tile_id;
                        tg[gate_lv[q] - l0].push_back(q);
                        covered[q] = 1;
                    }
                    for (int j = 0; j < nl; ++j) tarcs[j] = add[j];
                }
            }
            if (ok) {
                flush();
                return true;
            }
            // roll back this attempt's tiles
            sp_tile.resize(t0);
            sp_chunk.resize(c0all);
            sp_ta_arc.resize(a0all);
            sp_ta_src.resize(a0all);
            sp_ta_gate.resize(a0all);
            ++tile_id;
            for (int32_t q = q0; q < q1; ++q) covered[q] = 0;
            return false;
        };
        for (int32_t l0 = 1; l0 <= Lmax;) {
            const int32_t t0 = int32_t(sp_tile.size() / 4);
            int32_t n = std::min<int32_t>(cap_f, Lmax - l0 + 1);
            bool ok = try_span(l0, l0 + n - 1);
            while (!ok && n > 1) {
                --n;
                ok = try_span(l0, l0 + n - 1);
            }
            g->span_tile_h.push_back(t0);
            g->span_fused_h.push_back(uint8_t(ok));
            g->span_lv_h.insert(g->span_lv_h.end(), {l0, l0 + n - 1});
            l0 += n;
        }
        g->span_tile_h.push_back(int32_t(sp_tile.size() / 4));
        g->n_sptiles = int64_t(sp_tile.size() / 4);
    }

    // ---- fusion plan figures (reports) -----------------------------------------------------
    {
        sta_span_info& si = g->span_info;
        si = sta_span_info{};
        auto first_of = [](const std::vector<int32_t>& outer, int32_t idx, int64_t n_inner) -> int64_t {
            return idx < int32_t(outer.size() / 4) ? outer[size_t(idx) * 4] : n_inner;
        };
        const int64_t NS = int64_t(g->span_fused_h.size());
        for (int64_t s_ = 0; s_ < NS; ++s_) {
            const int32_t l0 = g->span_lv_h[2 * s_], l1 = g->span_lv_h[2 * s_ + 1];
            ++si.fwd_spans;
            if (!g->span_fused_h[s_]) {
                for (int32_t l = l0; l <= l1; ++l) si.fwd_level_launches += g->fwd_tile_ptr[l + 1] > g->fwd_tile_ptr[l];
                continue;
            }
            ++si.fwd_spans_fused;
            const int32_t t0 = g->span_tile_h[s_], t1 = g->span_tile_h[s_ + 1];
            si.fwd_span_launches += t1 > t0;
            si.fwd_span_tiles += t1 - t0;
            const int32_t q0 = lvl_gate_ptr[l0 - 1], q1 = lvl_gate_ptr[l1];
            si.fwd_span_gates += q1 - q0;
            si.fwd_span_arcs += gate_arc_ptr_int[q1] - gate_arc_ptr_int[q0];
            const int64_t nch = int64_t(sp_chunk.size() / 4), na = int64_t(sp_ta_arc.size());
            const int64_t a0 = first_of(sp_chunk, int32_t(first_of(sp_tile, t0, nch)), na);
            const int64_t a1 = first_of(sp_chunk, int32_t(first_of(sp_tile, t1, nch)), na);
            for (int64_t i = a0; i < a1; ++i) si.fwd_span_arcs_computed += sp_ta_gate[i] >= 0;
        }
        const int64_t NSB = int64_t(g->bspan_fused_h.size());
        for (int64_t b = 0; b < NSB; ++b) {
            const int32_t top = g->bspan_lv_h[2 * b], bot = g->bspan_lv_h[2 * b + 1];
            ++si.bwd_spans;
            if (!g->bspan_fused_h[b]) {
                for (int32_t l = top; l >= bot; --l) si.bwd_level_launches += g->bwd_tile_ptr[l + 1] > g->bwd_tile_ptr[l];
                continue;
            }
            ++si.bwd_spans_fused;
            const int32_t t0 = g->bspan_tile_h[b], t1 = g->bspan_tile_h[b + 1];
            si.bwd_span_launches += t1 > t0;
            si.bwd_span_tiles += t1 - t0;
            const int64_t i0 = (bot == 0) ? 0 : P + lvl_gate_ptr[bot - 1], i1 = P + lvl_gate_ptr[top];
            si.bwd_span_drivers += i1 - i0;
            si.bwd_span_arcs += fo_ptr[i1] - fo_ptr[i0];
            const int64_t nch = int64_t(bp_chunk.size() / 4), ns = int64_t(bp_slot.size());
            const int64_t s0 = first_of(bp_chunk, int32_t(first_of(bp_tile, t0, nch)), ns);
            const int64_t s1 = first_of(bp_chunk, int32_t(first_of(bp_tile, t1, nch)), ns);
            for (int64_t i = s0; i < s1; ++i) si.bwd_span_slots_computed += bp_slot[i] >= 0;
        }
    }

    // ---- fixed-stride span records (device) ------------------------------------------------
    // Level c of tile t at t * kSpan + c, lane k of it at (t * kSpan + c) * 64 + k.  Unused
    // levels and lanes hold indexes that are valid to load from (arc 0, driver 0, endpoint
    // rank 0), which the kernels mask.
    const int64_t NTF = int64_t(sp_tile.size() / 4), NTB = int64_t(bp_tile.size() / 4);
    std::vector<int32_t> sp_crec(size_t(NTF) * kSpanF * 4, 0), sp_arec(size_t(NTF) * kSpanF * 64 * 4, 0);
    for (int64_t t = 0; t < NTF; ++t) {
        const int32_t c0 = sp_tile[t * 4], nch = sp_tile[t * 4 + 1];
        for (int32_t c = 0; c < kSpanF; ++c) {
            int32_t* cr = &sp_crec[size_t(t * kSpanF + c) * 4];
            cr[0] = 0; cr[1] = 0; cr[2] = 1; cr[3] = nch;
            if (c >= nch) continue;
            const int32_t ch = c0 + c, ta0 = sp_chunk[ch * 4], na = sp_chunk[ch * 4 + 1];
            cr[0] = na; cr[1] = sp_chunk[ch * 4 + 2]; cr[2] = sp_chunk[ch * 4 + 3];
            // the lane's meta word: arc_meta | the lane of the next gate head of the level
            // after this lane (na if none: where its gate's segmented maximum ends) << 24 |
            // head bit 31 (the gate's first arc); lanes past the level's last are idle
            // (gate -1), like padding lanes
            // The gate word: the gate (26 bits: graphs with fused spans have fewer than
            // 2^26 drivers) | its rank among the level's gates in the tile (its LDS slot
            // past the level's first) << 26, or -1 for a padding or idle lane.
            int32_t heads_before = 0;
            for (int32_t k = 0; k < na; ++k) {
                const int32_t a = sp_ta_arc[ta0 + k];
                if (sp_ta_gate[ta0 + k] >= 0 && ((arc_meta[a] >> 16) & 0xffu) == 0u) ++heads_before;
                int32_t* ar = &sp_arec[(size_t(t * kSpanF + c) * 64 + k) * 4];
                ar[2] = sp_ta_gate[ta0 + k] < 0 ? -1
                                                : int32_t(uint32_t(sp_ta_gate[ta0 + k]) | (uint32_t(heads_before - 1) << 26));
            }
            int32_t next = na;
            for (int32_t k = na - 1; k >= 0; --k) {
                int32_t* ar = &sp_arec[(size_t(t * kSpanF + c) * 64 + k) * 4];
                const int32_t a = sp_ta_arc[ta0 + k];
                const bool head = sp_ta_gate[ta0 + k] >= 0 && ((arc_meta[a] >> 16) & 0xffu) == 0u;
                ar[0] = a; ar[1] = sp_ta_src[ta0 + k];
                ar[3] = int32_t(arc_meta[a] | (uint32_t(next) << 24) | (head ? 0x80000000u : 0u));
                if (head) next = k;
            }
            for (int32_t k = na; k < 64; ++k) sp_arec[(size_t(t * kSpanF + c) * 64 + k) * 4 + 2] = -1;
        }
    }
    std::vector<int32_t> bp_crec(size_t(NTB) * kSpanB * 4, 0), bp_srec(size_t(NTB) * kSpanB * 64 * 4, 0);
    for (size_t i = 0; i < bp_srec.size(); i += 4) {   // unused lanes: endpoint slots of rank 0
        bp_srec[i] = -1;
        bp_srec[i + 2] = -1;
    }
    for (int64_t t = 0; t < NTB; ++t) {
        const int32_t c0 = bp_tile[t * 4], nch = bp_tile[t * 4 + 1];
        for (int32_t c = 0; c < kSpanB; ++c) {
            int32_t* cr = &bp_crec[size_t(t * kSpanB + c) * 4];
            cr[0] = 0; cr[1] = 0; cr[2] = 1; cr[3] = nch;
            if (c >= nch) continue;
            const int32_t ch = c0 + c, ts0 = bp_chunk[ch * 4], ns = bp_chunk[ch * 4 + 1];
            cr[0] = ns; cr[1] = bp_chunk[ch * 4 + 2]; cr[2] = bp_chunk[ch * 4 + 3];
            // the source word: the in-tile source (16 bits, signed) | the lane of the next
            // driver head of the level after this lane (ns if none) << 16, where its driver's
            // segmented minimum ends
            // and the driver word: the driver (26 bits: graphs with fused spans have at most
            // 2^26 drivers) | its rank among the level's drivers in the tile (its LDS slot
            // past the level's first) << 26
            int32_t next = ns, heads_before = 0;
            for (int32_t k = 0; k < ns; ++k) {
                const int32_t sl = bp_slot[ts0 + k];
                if (sl >= 0 && (uint32_t(bslot_out[sl]) & kHeadBit)) ++heads_before;
                bp_srec[(size_t(t * kSpanB + c) * 64 + k) * 4 + 3] =
                    sl < 0 ? 0 : int32_t(uint32_t(bp_drv[ts0 + k]) | (uint32_t(std::max(heads_before - 1, 0)) << 26));
            }
            for (int32_t k = ns - 1; k >= 0; --k) {
                int32_t* sr = &bp_srec[(size_t(t * kSpanB + c) * 64 + k) * 4];
                const int32_t sl = bp_slot[ts0 + k];
                const int32_t src = sl < 0 ? -2 : bp_src[ts0 + k];
                sr[2] = int32_t((uint32_t(src) & 0xffffu) | (uint32_t(next) << 16));
                if (sl < 0) {            // padding lane: source -2, loads from endpoint rank 0 and driver 0
                    sr[0] = -1; sr[1] = 0;
                    continue;
                }
                sr[0] = bslot_arc[sl]; sr[1] = bslot_out[sl];
                if (uint32_t(bslot_out[sl]) & kHeadBit) next = k;
            }
            for (int32_t k = ns; k < 64; ++k)     // idle lanes: padding (source -2)
                bp_srec[(size_t(t * kSpanB + c) * 64 + k) * 4 + 2] = 0xfffe;
        }
    }

    // ---- device image --------------------------------------------------------------------
    DevLayout& lay = g->lay;
    size_t off = 0;
    auto place = [&](size_t bytes) { size_t o = off; off = align256(off + std::max<size_t>(bytes, 1)); return o; };
    lay.net_node_ptr = place((D + 1) * 4);
    lay.node_parent = place(M * 2);
    lay.node_R = place(M * 4);
    lay.node_C = place(M * 4);
    lay.fo_ptr = place((D + 1) * 4);
    lay.fo_arc = place(A * 4);
    lay.fo_tap = place(A);
    lay.fo_cap = place(A * 4);
    lay.arc_src = place(A * 4);
    lay.arc_meta = place(A * 4);
    lay.gate_arc_ptr = place((G + 1) * 4);
    lay.ftile_arc = place((NF + 1) * 4);
    lay.ftile_gate = place((NF + 1) * 4);
    lay.btile_drv = place((NB + 1) * 4);
    lay.btile_slot = place((NB + 1) * 4);
    lay.bslot_arc = place(S * 4);
    lay.bslot_out = place(S * 4);
    lay.ep_drv = place(E * 4);
    lay.fwd_lvl = place((Lmax + 2) * 12);
    lay.ftile_maxk = place(ftile_maxk.size() * 4);
    lay.fwd_chunk = place(fchunk.size() * 4);
    lay.bwd_chunk = place(bchunk.size() * 4);
    lay.bwd_lvl = place((Lmax + 2) * 12);
    lay.sp_crec = place(sp_crec.size() * 4);
    lay.sp_arec = place(sp_arec.size() * 4);
    lay.bp_crec = place(bp_crec.size() * 4);
    lay.bp_srec = place(bp_srec.size() * 4);
    lay.dc_wide = place(dc_wide.size() * 4);
    lay.total = off;
    g->image.assign(off, 0);
    auto put = [&](size_t o, const void* src, size_t bytes) { if (bytes) std::memcpy(g->image.data() + o, src, bytes); };
    put(lay.net_node_ptr, net_ptr.data(), (D + 1) * 4);
    put(lay.node_parent, node_parent.data(), M * 2);
    put(lay.node_R, node_R.data(), M * 4);
    put(lay.node_C, node_C.data(), M * 4);
    put(lay.fo_ptr, fo_ptr.data(), (D + 1) * 4);
    put(lay.fo_arc, fo_arc.data(), A * 4);
    put(lay.fo_tap, fo_tap.data(), A);
    put(lay.fo_cap, fo_cap.data(), A * 4);
    put(lay.arc_src, arc_src.data(), A * 4);
    put(lay.arc_meta, arc_meta.data(), A * 4);
    put(lay.gate_arc_ptr, gate_arc_ptr_int.data(), (G + 1) * 4);
    put(lay.ftile_arc, ftile_arc.data(), (NF + 1) * 4);
    put(lay.ftile_gate, ftile_gate.data(), (NF + 1) * 4);
    put(lay.btile_drv, btile_drv.data(), (NB + 1) * 4);
    put(lay.btile_slot, btile_slot.data(), (NB + 1) * 4);
    put(lay.bslot_arc, bslot_arc.data(), S * 4);
    put(lay.bslot_out, bslot_out.data(), S * 4);
    put(lay.ep_drv, g->ep_driver.data(), E * 4);
    put(lay.dc_wide, dc_wide.data(), dc_wide.size() * 4);
    // level tables: forward level l (1..L) owns tiles [f[l].t, f[l+1].t), arcs and gates from
    // f[l].a and f[l].g on; backward level l (0..L) likewise with slots and drivers
    std::vector<int32_t> flvl((Lmax + 2) * 3), blvl((Lmax + 2) * 3);
    for (int32_t l = 0; l <= Lmax + 1; ++l) {
        const int32_t ft = g->fwd_tile_ptr[l];
        flvl[l * 3 + 0] = ft;
        flvl[l * 3 + 1] = ftile_arc[ft];
        flvl[l * 3 + 2] = ftile_gate[ft];
        const int32_t bt = g->bwd_tile_ptr[l];
        blvl[l * 3 + 0] = bt;
        blvl[l * 3 + 1] = btile_slot[bt];
        blvl[l * 3 + 2] = btile_drv[bt];
    }
    for (int32_t l = 0; l <= Lmax; ++l) {
        if (l >= 1) {
            g->max_ft = std::max(g->max_ft, flvl[(l + 1) * 3] - flvl[l * 3]);
            g->max_fa = std::max(g->max_fa, flvl[(l + 1) * 3 + 1] - flvl[l * 3 + 1]);
            g->max_fg = std::max(g->max_fg, flvl[(l + 1) * 3 + 2] - flvl[l * 3 + 2]);
        }
        g->max_bt = std::max(g->max_bt, blvl[(l + 1) * 3] - blvl[l * 3]);
        g->max_bs = std::max(g->max_bs, blvl[(l + 1) * 3 + 1] - blvl[l * 3 + 1]);
        g->max_bd = std::max(g->max_bd, blvl[(l + 1) * 3 + 2] - blvl[l * 3 + 2]);
    }
    put(lay.fwd_lvl, flvl.data(), flvl.size() * 4);
    put(lay.ftile_maxk, ftile_maxk.data(), ftile_maxk.size() * 4);
    put(lay.fwd_chunk, fchunk.data(), fchunk.size() * 4);
    put(lay.bwd_chunk, bchunk.data(), bchunk.size() * 4);
    put(lay.bwd_lvl, blvl.data(), blvl.size() * 4);
    put(lay.sp_crec, sp_crec.data(), sp_crec.size() * 4);
    put(lay.sp_arec, sp_arec.data(), sp_arec.size() * 4);
    put(lay.bp_crec, bp_crec.data(), bp_crec.size() * 4);
    put(lay.bp_srec, bp_srec.data(), bp_srec.size() * 4);

    g->n_pi = int32_t(P);
    g->n_gates = int32_t(G);
    g->n_tables = d->n_tables;
    g->D = D; g->A = A; g->M = M; g->L = Lmax; g->E = E; g->S = S;
    g->max_fanin = max_fanin;
    g->max_fanout = max_fanout;
    g->max_net_nodes = max_nodes;
    g->chain_nets = chains;
    g->n_ftiles = NF;
    g->n_btiles = NB;
    g->ftile_arc_h = ftile_arc;
    g->ftile_gate_h = ftile_gate;
    g->btile_slot_h = btile_slot;
    g->btile_drv_h = btile_drv;
    return STA_OK;
}

}  // namespace sta

extern "C" {

const char* sta_last_error(void) { return sta::g_last_error.c_str(); }

sta_status sta_build_graph(const sta_design_desc* d, sta_graph** out) {
    return sta_build_graph_spans(d, sta::kSpanF, sta::kSpanB, out);
}

sta_status sta_build_graph_spans(const sta_design_desc* d, int32_t fwd_levels, int32_t bwd_levels, sta_graph** out) {
    if (!out) return sta::fail(STA_E_ARG, "sta_build_graph: null out");
    if (fwd_levels < 1 || fwd_levels > sta::kSpanF || bwd_levels < 1 || bwd_levels > sta::kSpanB)
        return sta::fail(STA_E_ARG, "sta_build_graph_spans: span lengths must be 1..8");
    sta_graph* g = nullptr;
    try {
        g = new sta_graph();
        sta_status st = sta::build(d, g, fwd_levels, bwd_levels);
        if (st != STA_OK) { delete g; return st; }
    } catch (const std::bad_alloc&) {
        delete g;
        return sta::fail(STA_E_ALLOC, "sta_build_graph: out of host memory");
    } catch (...) {
        delete g;
        return sta::fail(STA_E_ARG, "sta_build_graph: unexpected failure");
    }
    *out = g;
    return STA_OK;
}

sta_status sta_graph_sizes(const sta_graph* g, sta_sizes* s) {
    if (!g || !s) return sta::fail(STA_E_ARG, "sta_graph_sizes: null argument");
    s->n_pi = g->n_pi;
    s->n_gates = g->n_gates;
    s->n_drivers = g->D;
    s->n_arcs = g->A;
    s->n_nodes = g->M;
    s->n_pins = g->D + g->A;
    s->n_levels = g->L;
    s->n_endpoints = g->E;
    s->max_fanin = g->max_fanin;
    s->max_fanout = g->max_fanout;
    s->max_net_nodes = g->max_net_nodes;
    s->n_fwd_tiles = g->n_ftiles;
    s->n_bwd_tiles = g->n_btiles;
    s->graph_bytes = g->lay.total;
    s->scratch_bytes = sta::scratch_bytes();
    return STA_OK;
}

sta_status sta_graph_spans(const sta_graph* g, sta_span_info* out) {
    if (!g || !out) return sta::fail(STA_E_ARG, "sta_graph_spans: null argument");
    *out = g->span_info;
    return STA_OK;
}

sta_status sta_graph_span_list(const sta_graph* g, int32_t* fwd, int32_t* bwd) {
    if (!g) return sta::fail(STA_E_ARG, "sta_graph_span_list: null graph");
    if (fwd)
        for (size_t s = 0; s < g->span_fused_h.size(); ++s) {
            fwd[3 * s] = g->span_lv_h[2 * s];
            fwd[3 * s + 1] = g->span_lv_h[2 * s + 1];
            fwd[3 * s + 2] = g->span_fused_h[s];
        }
    if (bwd)
        for (size_t b = 0; b < g->bspan_fused_h.size(); ++b) {
            bwd[3 * b] = g->bspan_lv_h[2 * b];
            bwd[3 * b + 1] = g->bspan_lv_h[2 * b + 1];
            bwd[3 * b + 2] = g->bspan_fused_h[b];
        }
    return STA_OK;
}

sta_status sta_graph_perm(const sta_graph* g, int32_t* drv_input, int32_t* arc_input, int32_t* gate_input,
                          int32_t* level, int32_t* ep_driver) {
    if (!g) return sta::fail(STA_E_ARG, "sta_graph_perm: null graph");
    auto cp = [](int32_t* dst, const std::vector<int32_t>& v) { if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * 4); };
    cp(drv_input, g->drv_input);
    cp(arc_input, g->arc_input);
    cp(gate_input, g->gate_input);
    cp(level, g->level);
    cp(ep_driver, g->ep_driver);
    return STA_OK;
}

sta_status sta_graph_upload(sta_graph* g, void* dev_buf, size_t bytes, void* stream) {
    if (!g || !dev_buf) return sta::fail(STA_E_ARG, "sta_graph_upload: null argument");
    if (bytes < g->lay.total) return sta::fail(STA_E_ARG, "sta_graph_upload: buffer smaller than graph_bytes");
    if (reinterpret_cast<uintptr_t>(dev_buf) % 256 != 0) return sta::fail(STA_E_ARG, "sta_graph_upload: buffer not 256-byte aligned");
    hipError_t e = hipMemcpyAsync(dev_buf, g->image.data(), g->lay.total, hipMemcpyHostToDevice,
                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return sta::fail(STA_E_HIP, std::string("sta_graph_upload: hipMemcpyAsync: ") + hipGetErrorString(e));
    e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return sta::fail(STA_E_HIP, std::string("sta_graph_upload: hipStreamSynchronize: ") + hipGetErrorString(e));
    // sequences captured against the previous buffer are dropped (their keys name it too)
    {
        std::lock_guard<std::mutex> lock(g->cache_mu);
        for (sta::LaunchCache* c : {&g->fwd_cache, &g->bwd_cache, &g->adj_cache}) sta::drop_launches(*c);
    }
    g->dev = static_cast<uint8_t*>(dev_buf);
    return STA_OK;
}

void sta_graph_free(sta_graph* g) {
    if (!g) return;
    for (sta::LaunchCache* c : {&g->fwd_cache, &g->bwd_cache, &g->adj_cache}) sta::drop_launches(*c);
    delete g;
}

}  // extern "C"

// HIP kernels for CDNA4 (gfx950) and the device-side entry points of libsta.
//
// Build: -O3 -ffp-contract=off (no a*b+c contraction), IEEE FP32 division and sqrt
// (correctly rounded), FP32 denormals kept.  With those, every floating-point step
// below is the same single rounded operation as in the operation order the header
// documents, so results equal the CPU definition bit for bit.
//
// Work decomposition.  The unit of work is a tile: one wavefront over <= 64 cell arcs of
// consecutive whole gates of one level (forward), or over <= 64 sink slots of
// consecutive drivers of one level (backward; a driver with more sinks gets a tile of
// its own whose lanes take contiguous runs of its sinks).  Two schedules run the tiles:
//   level schedule  one launch per level; every launch covers all views of the call.
//                   For wide levels (the whole chip works on one level).
//   view schedule   one 1024-lane workgroup per view walks every level itself, with only
//                   a workgroup barrier between levels and the NLDM tables in LDS; the
//                   views run on separate compute units.  For the usual narrow levels,
//                   where a device-wide step (a launch or a grid barrier, >= 2 us on
//                   MI355X) costs more than the level's own work on one compute unit.
// K1 (RC delay calculation) is level-free: one lane per net.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <memory>
#include <cmath>
#include <cstdint>
#include <cfloat>
#include <cstring>
#include <map>
#include <string>
#include <type_traits>
#include <vector>

#include "sta_internal.h"

namespace sta {

// ---------------------------------------------------------------------------------
// K1: RC delay calculation
// ---------------------------------------------------------------------------------

// Lane t of the block owns net (blockIdx.x*NT + t).  Node temporaries live in LDS,
// interleaved by lane: slot (k, t) at [k*NT + t], two arrays per lane:
//   X: C (node cap), then W = C m1 (in place), its downstream sums, then m2 (in place);
//   Y: Cd (downstream cap), then m1 (in place).
// In place is exact: m1(k) reads m1(parent(k)) (parent < k, already final) and Cd(k)
// (not yet overwritten) in ascending k, and m2 likewise reads W; the operations and their
// order are those of the definition, so the results are the same bit for bit.
template <typename T, int MAXN, int NT>
__device__ __forceinline__ void dc_net(const DevGraph& G, int d, int t, T* sX, T* sY, float* __restrict__ load,
                                       float* __restrict__ net_delay, float* __restrict__ net_imp2,
                                       float* __restrict__ arc_load) {
    const int n0 = G.net_node_ptr[d];
    const int nm = G.net_node_ptr[d + 1] - n0;
    const int16_t* par = G.node_parent + n0;
    const float* R = G.node_R + n0;
    const float* Cw = G.node_C + n0;
    T* X = sX + t;
    T* Y = sY + t;
#define AT_(arr, k) arr[(k) * NT]
    for (int k = 0; k < nm; ++k) AT_(X, k) = static_cast<T>(Cw[k]);
    const int f0 = G.fo_ptr[d], f1 = G.fo_ptr[d + 1];
    for (int e = f0; e < f1; ++e) AT_(X, G.fo_tap[e]) += static_cast<T>(G.fo_cap[e]);
    for (int k = 0; k < nm; ++k) AT_(Y, k) = AT_(X, k);
    for (int k = nm - 1; k >= 1; --k) AT_(Y, par[k]) += AT_(Y, k);
    const float ld = static_cast<float>(AT_(Y, 0));
    load[d] = ld;
    if (d >= G.n_pi) {
        const int q = d - G.n_pi;
        for (int a = G.gate_arc_ptr[q]; a < G.gate_arc_ptr[q + 1]; ++a) arc_load[a] = ld;
    }
    const T milli = static_cast<T>(1e-3);
    AT_(Y, 0) = T(0);
    for (int k = 1; k < nm; ++k) AT_(Y, k) = AT_(Y, par[k]) + (static_cast<T>(R[k]) * AT_(Y, k)) * milli;
    for (int k = 0; k < nm; ++k) AT_(X, k) = AT_(X, k) * AT_(Y, k);
    for (int k = nm - 1; k >= 1; --k) AT_(X, par[k]) += AT_(X, k);
    AT_(X, 0) = T(0);
    for (int k = 1; k < nm; ++k) AT_(X, k) = AT_(X, par[k]) + (static_cast<T>(R[k]) * AT_(X, k)) * milli;
    for (int e = f0; e < f1; ++e) {
        const int k = G.fo_tap[e];
        const int a = G.fo_arc[e];
        const T m1 = AT_(Y, k);
        T imp2 = T(2) * AT_(X, k) - m1 * m1;
        if (imp2 < T(0)) imp2 = T(0);
        net_delay[a] = static_cast<float>(m1);
        net_imp2[a] = static_cast<float>(imp2);
    }
#undef AT_
}

// Nets of at most 8 nodes keep every node value in registers (no LDS, so the launch's
// residency is set by registers alone): a step that reads a node's parent, or a sink's tap
// node, selects among the node registers, and a step that adds into a parent updates the
// selected register only.  The arithmetic and its order are dc_net's, so the results are
// the same bit for bit.

// c ? t : f as explicit v_cndmask instructions: written as C++ selects over the node
// registers, the compiler turns them back into indexed loads from scratch memory
__device__ __forceinline__ float dc_sel(bool c, float t, float f) {
    const unsigned long long m = __builtin_amdgcn_ballot_w64(c);
    float r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(f), "v"(t), "s"(m));
    return r;
}
__device__ __forceinline__ double dc_sel(bool c, double t, double f) {
    const unsigned long long m = __builtin_amdgcn_ballot_w64(c);
    int lo, hi;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(lo) : "v"(__double2loint(f)), "v"(__double2loint(t)), "s"(m));
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(hi) : "v"(__double2hiint(f)), "v"(__double2hiint(t)), "s"(m));
    return __hiloint2double(hi, lo);
}

// a[idx], idx in 0..7: a select tree on the bits of idx
template <typename T>
__device__ __forceinline__ T dc_pick(const T (&a)[8], int idx) {
    const bool b0 = idx & 1, b1 = idx & 2, b2 = idx & 4;
    const T l0 = dc_sel(b0, a[1], a[0]), l1 = dc_sel(b0, a[3], a[2]);
    const T l2 = dc_sel(b0, a[5], a[4]), l3 = dc_sel(b0, a[7], a[6]);
    return dc_sel(b2, dc_sel(b1, l3, l2), dc_sel(b1, l1, l0));
}

// The tree sweeps of a net of nm <= 8 nodes (parents par[k] < k), X holding each node's
// capacitance with its pin caps added: Y becomes m1, X becomes m2; returns the total load.
// chain (uniform): every net of the wavefront is a chain (par[k] = k - 1), so each parent
// is known without a select.
template <typename T>
__device__ __forceinline__ float dc8_sweeps(T (&X)[8], T (&Y)[8], uint32_t pp, const float (&R)[8], int nm,
                                            bool chain) {
    // pp: the parents, 3 bits per node
    auto par = [pp](int k) { return int((pp >> (3 * k)) & 7u); };
    const T milli = static_cast<T>(1e-3);
#pragma unroll
    for (int k = 0; k < 8; ++k) Y[k] = X[k];
    float ld;
    if (chain) {
#pragma unroll
        for (int k = 7; k >= 1; --k) Y[k - 1] = dc_sel(k < nm, Y[k - 1] + Y[k], Y[k - 1]);
        ld = static_cast<float>(Y[0]);
        Y[0] = T(0);
#pragma unroll
        for (int k = 1; k < 8; ++k) Y[k] = Y[k - 1] + (static_cast<T>(R[k]) * Y[k]) * milli;
#pragma unroll
        for (int k = 0; k < 8; ++k) X[k] = X[k] * Y[k];
#pragma unroll
        for (int k = 7; k >= 1; --k) X[k - 1] = dc_sel(k < nm, X[k - 1] + X[k], X[k - 1]);
        X[0] = T(0);
#pragma unroll
        for (int k = 1; k < 8; ++k) X[k] = X[k - 1] + (static_cast<T>(R[k]) * X[k]) * milli;
        return ld;
    }
    // downstream capacitance: children added into their parent, highest node first
#pragma unroll
    for (int k = 7; k >= 1; --k)
#pragma unroll
        for (int p = 0; p < k; ++p) Y[p] = dc_sel(k < nm && par(k) == p, Y[p] + Y[k], Y[p]);
    ld = static_cast<float>(Y[0]);
    Y[0] = T(0);
#pragma unroll
    for (int k = 1; k < 8; ++k)
        if (k < nm) Y[k] = dc_pick(Y, par(k)) + (static_cast<T>(R[k]) * Y[k]) * milli;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (k < nm) X[k] = X[k] * Y[k];
#pragma unroll
    for (int k = 7; k >= 1; --k)
#pragma unroll
        for (int p = 0; p < k; ++p) X[p] = dc_sel(k < nm && par(k) == p, X[p] + X[k], X[p]);
    X[0] = T(0);
#pragma unroll
    for (int k = 1; k < 8; ++k)
        if (k < nm) X[k] = dc_pick(X, par(k)) + (static_cast<T>(R[k]) * X[k]) * milli;
    return ld;
}

// lane k's value of v, to every lane
__device__ __forceinline__ double dc_lane_value(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), k);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), k);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<uint32_t>(lo));
}
__device__ __forceinline__ float dc_lane_value(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

template <typename T>
__device__ __forceinline__ void dc8_store(const T (&X)[8], const T (&Y)[8], int k, int a,
                                          float* __restrict__ net_delay, float* __restrict__ net_imp2) {
    const T m1 = dc_pick(Y, k);
    T imp2 = T(2) * dc_pick(X, k) - m1 * m1;
    if (imp2 < T(0)) imp2 = T(0);
    net_delay[a] = static_cast<float>(m1);
    net_imp2[a] = static_cast<float>(imp2);
}

// One wavefront of the lane-per-net path: nets dw0 .. dw0 + 63 (those of at most
// kDcLaneSinks sinks; a wider net is skipped: its own wavefront does it).  The wavefront's
// sinks are one contiguous range; when it holds at most kDcWindow sinks (always, unless
// wide nets crowd the wavefront) it is loaded coalesced into LDS (s_cap: pin cap, s_at:
// arc | tap << 29) in the round that loads the lanes' nodes, and a lane reads its own
// sinks from LDS; otherwise (STAGED false) each lane reads its sinks from memory.
template <typename T, bool CHAINS, bool STAGED>
__device__ __forceinline__ void dc8_lanes(const DevGraph& G, int dw0, int dwl, int n0, int nm, int f0, int f1,
                                          int a0, int a1, float* __restrict__ s_cap, int* __restrict__ s_at,
                                          float* __restrict__ load, float* __restrict__ net_delay,
                                          float* __restrict__ net_imp2, float* __restrict__ arc_load) {
    const int lane = threadIdx.x & 63;
    const int d = dw0 + lane;
    const bool act = d <= dwl;
    // the wavefront's sink range, from its first and last lanes
    const int F0 = __builtin_amdgcn_readfirstlane(f0);
    const int F1 = __builtin_amdgcn_readlane(f1, dwl - dw0);
    // the lanes' nodes and (STAGED) the wavefront's sinks, 256 per pass
    int par[8];
    float R[8], Cw[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int kk = n0 + (k < nm ? k : 0);
        par[k] = G.node_parent[kk];
        R[k] = G.node_R[kk];
        Cw[k] = G.node_C[kk];
    }
    if constexpr (STAGED) {
        for (int c0 = F0; c0 < F1; c0 += 256) {            // uniform
            int tv[4], av[4];
            float cv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = c0 + i * 64 + lane;
                const int ec = e < F1 ? e : F0;
                tv[i] = G.fo_tap[ec];
                cv[i] = G.fo_cap[ec];
                av[i] = G.fo_arc[ec];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = c0 + i * 64 + lane;
                if (e < F1) {
                    s_cap[e - F0] = cv[i];
                    s_at[e - F0] = av[i] | (tv[i] << 29);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const int ns = f1 - f0;
    const bool mine = act && ns <= kDcLaneSinks;
    uint32_t pp = 0;
    bool chain = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        pp |= uint32_t(par[k] & 7) << (3 * k);
        if (k >= 1) chain = chain && (k >= nm || par[k] == k - 1);
    }
    const bool all_chain = __builtin_amdgcn_ballot_w64(mine && !chain) == 0;
    if (!mine) return;
    T X[8], Y[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) X[k] = static_cast<T>(Cw[k]);
    auto sink = [&](int e, int& tap, int& arc, float& cap) {
        if constexpr (STAGED) {
            const int at = s_at[e - F0];
            tap = int(uint32_t(at) >> 29);
            arc = at & 0x1fffffff;
            cap = s_cap[e - F0];
        } else {
            tap = G.fo_tap[e];
            arc = G.fo_arc[e];
            cap = G.fo_cap[e];
        }
    };
    // pin caps added to their tap nodes in sink order
    for (int e = f0; e < f1; ++e) {
        int tj, aj;
        float cj;
        sink(e, tj, aj, cj);
#pragma unroll
        for (int k = 0; k < 8; ++k) X[k] = dc_sel(tj == k, X[k] + static_cast<T>(cj), X[k]);
    }
    const float ld = dc8_sweeps<T>(X, Y, pp, R, nm, CHAINS || all_chain);
    load[d] = ld;
    for (int a = a0; a < a1; ++a) arc_load[a] = ld;
    for (int e = f0; e < f1; ++e) {
        int tj, aj;
        float cj;
        sink(e, tj, aj, cj);
        dc8_store<T>(X, Y, tj, aj, net_delay, net_imp2);
    }
}

// One wavefront: net d of more than kDcLaneSinks sinks (d uniform).  The lanes load 64
// sinks at a time; the pin caps are added in sink order from broadcast lane values, every
// lane running the same node arithmetic, and each lane then writes its own sinks.
template <typename T, bool CHAINS>
__device__ __forceinline__ void dc8_wave(const DevGraph& G, int d, float* __restrict__ load,
                                         float* __restrict__ net_delay, float* __restrict__ net_imp2,
                                         float* __restrict__ arc_load) {
    const int lane = threadIdx.x & 63;
    const int n0 = G.net_node_ptr[d];
    const int nm = G.net_node_ptr[d + 1] - n0;
    const int f0 = G.fo_ptr[d], f1 = G.fo_ptr[d + 1];
    uint32_t pp = 0;
    bool chain = true;
    float R[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int kk = n0 + (k < nm ? k : 0);
        const int pk = G.node_parent[kk];
        pp |= uint32_t(pk & 7) << (3 * k);
        if (k >= 1) chain = chain && (k >= nm || pk == k - 1);
        R[k] = G.node_R[kk];
    }
    // lane k < 8 adds the pin caps of node k, in sink order, from the broadcast sink values
    T acc = static_cast<T>(G.node_C[n0 + (lane < nm ? lane : 0)]);
    for (int e0 = f0; e0 < f1; e0 += 64) {
        const int e = e0 + lane < f1 ? e0 + lane : f0;
        const int tv = G.fo_tap[e];
        const float cv = G.fo_cap[e];
        const int n = min(64, f1 - e0);
        for (int j = 0; j < n; ++j) {
            const int tj = __builtin_amdgcn_readlane(tv, j);
            const T cj = static_cast<T>(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(cv), j)));
            acc = dc_sel(tj == lane, acc + cj, acc);
        }
    }
    T X[8], Y[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) X[k] = dc_lane_value(acc, k);
    const float ld = dc8_sweeps<T>(X, Y, pp, R, nm, CHAINS || __builtin_amdgcn_ballot_w64(!chain) == 0);
    if (lane == 0) load[d] = ld;
    if (d >= G.n_pi) {
        const int q = d - G.n_pi;
        for (int a = G.gate_arc_ptr[q] + lane; a < G.gate_arc_ptr[q + 1]; a += 64) arc_load[a] = ld;
    }
    for (int e = f0 + lane; e < f1; e += 64) dc8_store<T>(X, Y, G.fo_tap[e], G.fo_arc[e], net_delay, net_imp2);
}

// Workgroup x (256 lanes) of the delay calculation of a graph whose nets have at most 8
// nodes: the first ceil(n_dc_wide / 4) workgroups give each wide net a wavefront (first,
// so that the longest nets start first), the rest one lane per net.
template <typename T, bool CHAINS>
__device__ __forceinline__ void dc8_block(const DevGraph& G, int x, float* __restrict__ load,
                                          float* __restrict__ net_delay, float* __restrict__ net_imp2,
                                          float* __restrict__ arc_load) {
    __shared__ float s_cap[4][kDcWindow];
    __shared__ int s_at[4][kDcWindow];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wb = (G.n_dc_wide + 3) >> 2;
    if (x < wb) {
        const int i = x * 4 + wave;
        if (i < G.n_dc_wide) dc8_wave<T, CHAINS>(G, __builtin_amdgcn_readfirstlane(G.dc_wide[i]), load, net_delay, net_imp2, arc_load);
        return;
    }
    const int dw0 = (x - wb) * 256 + wave * 64;
    if (dw0 >= G.n_drivers) return;
    // one round of loads: each lane's net pointers and gate (clamped to the last net)
    const int dwl = min(dw0 + 63, G.n_drivers - 1);
    const int dd = min(dw0 + int(threadIdx.x & 63), dwl);
    const int n0 = G.net_node_ptr[dd];
    const int nm = G.net_node_ptr[dd + 1] - n0;
    const int f0 = G.fo_ptr[dd], f1 = G.fo_ptr[dd + 1];
    const int q = dd >= G.n_pi ? dd - G.n_pi : -1;
    const int a0 = q >= 0 ? G.gate_arc_ptr[q] : 0, a1 = q >= 0 ? G.gate_arc_ptr[q + 1] : 0;
    const int span = __builtin_amdgcn_readlane(f1, dwl - dw0) - __builtin_amdgcn_readfirstlane(f0);
    if (span <= kDcWindow && G.n_arcs <= (1 << 29))        // (arc | tap << 29 must fit)
        dc8_lanes<T, CHAINS, true>(G, dw0, dwl, n0, nm, f0, f1, a0, a1, s_cap[wave], s_at[wave], load, net_delay, net_imp2, arc_load);
    else
        dc8_lanes<T, CHAINS, false>(G, dw0, dwl, n0, nm, f0, f1, a0, a1, nullptr, nullptr, load, net_delay, net_imp2, arc_load);
}

// workgroups of the delay calculation of g in node-count class maxn with nt lanes each
static inline int dc_blocks_of(int64_t D, int32_t n_wide, int maxn, int nt) {
    return int((D + nt - 1) / nt) + (maxn == 8 ? (n_wide + 3) / 4 : 0);
}

template <typename T, int MAXN, int NT>
__global__ __launch_bounds__(NT) void k_delay_calc(DevGraph G, float* __restrict__ load,
                                                   float* __restrict__ net_delay,
                                                   float* __restrict__ net_imp2,
                                                   float* __restrict__ arc_load) {
    __shared__ T sX[MAXN * NT];   // C, then W, then m2
    __shared__ T sY[MAXN * NT];   // Cd, then m1
    const int t = threadIdx.x;
    const int d = blockIdx.x * NT + t;
    if (d >= G.n_drivers) return;
    dc_net<T, MAXN, NT>(G, d, t, sX, sY, load, net_delay, net_imp2, arc_load);
}

// CHAINS: every net of the graph is a chain (known at graph build), so the kernel has no
// select form of the sweeps and needs far fewer registers (63 against 116 VGPRs for FP64)
template <typename T, bool CHAINS>
__global__ __launch_bounds__(256) void k_delay_calc8(DevGraph G, float* __restrict__ load,
                                                     float* __restrict__ net_delay,
                                                     float* __restrict__ net_imp2,
                                                     float* __restrict__ arc_load) {
    dc8_block<T, CHAINS>(G, int(blockIdx.x), load, net_delay, net_imp2, arc_load);
}

// Batched delay calculation: workgroup x takes nets map[map0 + x].y * NT + t of design
// map[map0 + x].x (the designs of one node-count class in one launch).
template <typename T, int MAXN, int NT>
__global__ __launch_bounds__(NT) void k_delay_calc_batch(const BatchItem* __restrict__ items,
                                                         const int2* __restrict__ map, int map0) {
    __shared__ T sX[MAXN * NT];
    __shared__ T sY[MAXN * NT];
    const int2 m = map[map0 + int(blockIdx.x)];
    const BatchItem& it = items[m.x];
    const int t = threadIdx.x;
    const int d = m.y * NT + t;
    if (d >= it.G.n_drivers) return;
    dc_net<T, MAXN, NT>(it.G, d, t, sX, sY, it.load_w, it.nd_w, it.ni_w, it.arc_load);
}

template <typename T, bool CHAINS>
__global__ __launch_bounds__(256) void k_delay_calc8_batch(const BatchItem* __restrict__ items,
                                                           const int2* __restrict__ map, int map0) {
    const int2 m = map[map0 + int(blockIdx.x)];
    const BatchItem& it = items[m.x];
    dc8_block<T, CHAINS>(it.G, m.y, it.load_w, it.nd_w, it.ni_w, it.arc_load);
}

// ---------------------------------------------------------------------------------
// NLDM lookup helpers
// ---------------------------------------------------------------------------------

struct KLib {
    float ax[26];                // x[7], y[7], dx[6] = fl32(x[i+1]-x[i]), dy[6]
    float sq[5];                 // sq[k]: the least float a with sqrtf(a) >= x[k+1] (slew thresholds)
    const float* tables;         // [sets][K][2][49]
    int32_t n_tables;
};

struct KViews {
    int32_t mode[STA_MAX_VIEWS];
    int32_t set[STA_MAX_VIEWS];
};

// largest i in 0..5 with axis[i] <= v (0 below axis[0]); axes strictly increase
__device__ __forceinline__ int seg6(const float* ax, float v) {
    int i = 0;
#pragma unroll
    for (int t = 1; t <= 5; ++t) i += (ax[t] <= v) ? 1 : 0;
    return i;
}

// bilinear value from the four corners (i,j), (i,j+1), (i+1,j), (i+1,j+1)
__device__ __forceinline__ float bilerp4(float t00, float t01, float t10, float t11, float tx, float ty) {
    const float p = t00 + tx * (t10 - t00);
    const float q = t01 + tx * (t11 - t01);
    return p + ty * (q - p);
}

__device__ __forceinline__ float bilerp(const float* T, int i, int j, float tx, float ty) {
    return bilerp4(T[i * 7 + j], T[i * 7 + j + 1], T[(i + 1) * 7 + j], T[(i + 1) * 7 + j + 1], tx, ty);
}

// base + off bytes, off a 32-bit offset: with a wave-uniform base the access takes the
// scalar-base form (a 32-bit vector offset, no 64-bit address arithmetic per lane)
template <typename T>
__device__ __forceinline__ T* at32(T* base, uint32_t off) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(base) + off);
}

// the delay and slew lookups of table tb of a set: the corners addressed by a 32-bit byte
// offset from the set's wave-uniform base, so that the loads take the scalar-base form (no
// 64-bit address arithmetic per lane); a set is at most 65,536 tables of 392 bytes
__device__ __forceinline__ void bilerp_pair(const float* set, int tb, int i, int j, float tx, float ty,
                                            float& dl, float& sl) {
    const char* b = reinterpret_cast<const char*>(set);
    const uint32_t o = uint32_t(tb) * 392u + uint32_t(i * 7 + j) * 4u;
    auto at = [&](uint32_t k) { return *reinterpret_cast<const float*>(b + (o + k)); };
    dl = bilerp4(at(0), at(4), at(28), at(32), tx, ty);
    sl = bilerp4(at(196), at(200), at(224), at(228), tx, ty);
}

__device__ __forceinline__ uint64_t lanes_le(int lane) {
    return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

__device__ __forceinline__ void load_axes(float* s_ax, const KLib& lib) {
    for (int i = threadIdx.x; i < 26; i += blockDim.x) s_ax[i] = lib.ax[i];
}

// ---------------------------------------------------------------------------------
// forward tile: views v0 .. v0+NW-1 of an NV-view interleaved layout
// ---------------------------------------------------------------------------------

// one lane's cell arc in a tile (inputs gathered by the caller)
struct FwdLane {
    int a, g, gi, kpos, tb, seg_end;
    bool active, head;
    float nd, ni, Lo;
};

// fwd_lane_setup for a span record: the end lane of the lane's gate and its head bit come
// with the record (bits 24..30 and 31 of its meta word; an idle or padding lane has a
// valid table id and is never a head), and so do the gate and its rank in the level (the
// gate word: gate | rank << 26)
__device__ __forceinline__ void fwd_lane_setup_span(FwdLane& x, bool act, uint32_t meta, uint32_t gword) {
    x.active = act;
    x.kpos = int((meta >> 16) & 0xffu);
    x.tb = int(meta & 0xffffu);
    x.head = int32_t(meta) < 0;
    x.g = int(gword & 0x3ffffffu);
    x.gi = int(gword >> 26);
    x.seg_end = int((meta >> 24) & 0x7fu);
}

// gate heads, the lane's gate within the tile and its gate's end lane (wave-uniform call)
__device__ __forceinline__ void fwd_lane_setup(FwdLane& x, bool act, uint32_t meta, int n, int lane) {
    x.active = act;
    x.kpos = int((meta >> 16) & 0xffu);
    x.tb = int(meta & 0xffffu);
    x.head = act && x.kpos == 0;
    const uint64_t heads = __ballot(x.head);
    const uint64_t le = lanes_le(lane);
    x.gi = __popcll(heads & le) - 1;
    const uint64_t after = heads & ~le;
    x.seg_end = after ? (__ffsll(static_cast<unsigned long long>(after)) - 1) : n;
}

// the load segment and fraction of a gate output (shared by the gate's arcs)
__device__ __forceinline__ void gate_jty(const float* s_ax, float Lo, int& j, float& ty) {
    const float* Y = s_ax + 7;
    const float* DY = s_ax + 20;
    j = seg6(Y, Lo);
    ty = (Lo - Y[j]) / DY[j];
}

// One table axis as named wave-uniform scalars (no array, so nothing is ever indexed
// through memory): the first six points and the six segment widths.
struct Axis6 {
    float p0, p1, p2, p3, p4, p5;
    float w0, w1, w2, w3, w4, w5;
};

__device__ __forceinline__ Axis6 axis6(const KLib& lib, int base, int wbase) {
    return Axis6{lib.ax[base], lib.ax[base + 1], lib.ax[base + 2], lib.ax[base + 3], lib.ax[base + 4],
                 lib.ax[base + 5], lib.ax[wbase], lib.ax[wbase + 1], lib.ax[wbase + 2], lib.ax[wbase + 3],
                 lib.ax[wbase + 4], lib.ax[wbase + 5]};
}

// a copy of a wave-uniform value in a vector register
__device__ __forceinline__ float in_vgpr(float x) {
    float r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// the axis in vector registers: a select between two axis points then needs no copy of
// each scalar operand into a vector register first (one scalar operand per instruction),
// which halves the segment searches of a level
__device__ __forceinline__ Axis6 axis6_v(const KLib& lib, int base, int wbase) {
    const Axis6 a = axis6(lib, base, wbase);
    return Axis6{in_vgpr(a.p0), in_vgpr(a.p1), in_vgpr(a.p2), in_vgpr(a.p3), in_vgpr(a.p4), in_vgpr(a.p5),
                 in_vgpr(a.w0), in_vgpr(a.w1), in_vgpr(a.w2), in_vgpr(a.w3), in_vgpr(a.w4), in_vgpr(a.w5)};
}

// seg6 by compares and selects, also returning the segment's origin and width.  The axes
// strictly increase, so the compares are true for a prefix of the points: the count of
// true compares and the last true one are the same index.
__device__ __forceinline__ int seg6_sel(const Axis6& a, float v, float& x0, float& dx) {
    int i = 0;
    x0 = a.p0;
    dx = a.w0;
#define SEG6_STEP_(P, W) { const bool ge = (P) <= v; i += ge ? 1 : 0; x0 = ge ? (P) : x0; dx = ge ? (W) : dx; }
    SEG6_STEP_(a.p1, a.w1)
    SEG6_STEP_(a.p2, a.w2)
    SEG6_STEP_(a.p3, a.w3)
    SEG6_STEP_(a.p4, a.w4)
    SEG6_STEP_(a.p5, a.w5)
#undef SEG6_STEP_
    return i;
}

// The slew axis's square-root thresholds (KLib::sq) as named wave-uniform scalars.
struct Sq5 {
    float t1, t2, t3, t4, t5;
};

__device__ __forceinline__ Sq5 sq5(const KLib& lib) {
    return Sq5{lib.sq[0], lib.sq[1], lib.sq[2], lib.sq[3], lib.sq[4]};
}

// seg6_sel of v = sqrtf(a), found from a itself: a >= sq[k] exactly when sqrtf(a) >= x[k+1]
// (KLib::sq), so the segment, its origin and its width are known before the root is.
__device__ __forceinline__ int seg6_sq(const Axis6& ax, const Sq5& q, float a, float& x0, float& dx) {
    int i = 0;
    x0 = ax.p0;
    dx = ax.w0;
#define SEG6_STEP_(T, P, W) { const bool ge = (T) <= a; i += ge ? 1 : 0; x0 = ge ? (P) : x0; dx = ge ? (W) : dx; }
    SEG6_STEP_(q.t1, ax.p1, ax.w1)
    SEG6_STEP_(q.t2, ax.p2, ax.w2)
    SEG6_STEP_(q.t3, ax.p3, ax.w3)
    SEG6_STEP_(q.t4, ax.p4, ax.w4)
    SEG6_STEP_(q.t5, ax.p5, ax.w5)
#undef SEG6_STEP_
    return i;
}

// arc arithmetic, per-gate max/argmax (min for early views) and the writes.  span: the
// largest gate fanin in the tile (the reduction needs ceil(log2(span)) steps).
// fresh_out (optional, LDS): the gate outputs of the first view, by gate index - gbase.
template <int NW>
__device__ __forceinline__ void fwd_finish(const FwdLane& x, const float2* ts, int j, float ty, int span,
                                           const float* s_ax, const float* const* tab, const bool* early, int NV,
                                           int v0, int n_pi, float* __restrict__ drv_ts, float* __restrict__ arc_ts,
                                           float* __restrict__ arc_delay, uint8_t* __restrict__ argmax,
                                           float2* fresh_out = nullptr, int gbase = 0) {
    const float* X = s_ax;
    const float* DX = s_ax + 14;
    const int lane = threadIdx.x & 63;
    float cand[NW], slw[NW];
    int best_k[NW];
    if (x.active) {
        float2* dst = reinterpret_cast<float2*>(arc_ts) + size_t(x.a) * NV + v0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const float ai = ts[w].x + x.nd;
            const float su2 = ts[w].y * ts[w].y;
            const float si = sqrtf(su2 + x.ni);
            const int i = seg6(X, si);
            const float tx = (si - X[i]) / DX[i];
            float dl, sl;
            bilerp_pair(tab[w], x.tb, i, j, tx, ty, dl, sl);
            dst[w] = make_float2(ai, si);
            arc_delay[size_t(x.a) * NV + v0 + w] = dl;
            cand[w] = ai + dl;
            slw[w] = sl;
            best_k[w] = x.kpos;
        }
    } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) { cand[w] = 0.0f; slw[w] = 0.0f; best_k[w] = 0; }
    }
    // segmented reduction toward each gate's first lane; the left operand covers the
    // lower arc positions, so keeping it on ties keeps the smallest arc index
    for (int off = 1; off < span; off <<= 1) {
        const bool take = (lane + off) < x.seg_end;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const float c2 = __shfl_down(cand[w], off, 64);
            const float s2 = __shfl_down(slw[w], off, 64);
            const int k2 = __shfl_down(best_k[w], off, 64);
            if (take) {
                if (early[w] ? (c2 < cand[w]) : (c2 > cand[w])) { cand[w] = c2; best_k[w] = k2; }
                if (early[w] ? (s2 < slw[w]) : (s2 > slw[w])) slw[w] = s2;
            }
        }
    }
    if (x.head) {
        float2* out = reinterpret_cast<float2*>(drv_ts) + size_t(n_pi + x.g) * NV + v0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            out[w] = make_float2(cand[w], slw[w]);
            argmax[size_t(x.g) * NV + v0 + w] = uint8_t(best_k[w]);
        }
        if (fresh_out) fresh_out[x.g - gbase] = make_float2(cand[0], slw[0]);
    }
}

// ---------------------------------------------------------------------------------
// backward tile
// ---------------------------------------------------------------------------------

template <int NW>
__device__ __forceinline__ void bwd_tile(const DevGraph& G, const bool* early, int NV, int v0, int s0, int n, int d0,
                                         const float* __restrict__ nd, const float* __restrict__ drv_ts,
                                         const float* __restrict__ arc_ts, const float* __restrict__ arc_delay,
                                         const float* __restrict__ ep_rat, float* __restrict__ drv_rat,
                                         float* __restrict__ arc_rat, float* __restrict__ drv_slack,
                                         float* __restrict__ arc_slack) {
    const int lane = threadIdx.x & 63;
    // n <= 64, or one driver owning every slot; lane owns the contiguous slots
    // [lane*c, min(n, (lane+1)*c)) so lower lanes always hold lower sink positions
    const int c = (n + 63) >> 6;
    const int sb = lane * c;
    const int se = min(n, sb + c);
    bool head;
    if (c > 1) head = (lane == 0);
    else head = (sb < n) && (uint32_t(G.bslot_out[s0 + sb]) & kHeadBit) != 0u;
    // segment = lanes of one driver: heads from the slot flags (c == 1) or lane 0 (c > 1)
    const uint64_t heads = __ballot(head);
    const uint64_t le = lanes_le(lane);
    const int gi = __popcll(heads & le) - 1;
    const uint64_t after = heads & ~le;
    const int nl = (n + c - 1) / c;               // lanes holding slots
    const int seg_end = after ? (__ffsll(static_cast<unsigned long long>(after)) - 1) : nl;
    // the driver's arrival times, loaded with the sinks' data (not after the reduction)
    float at_h[NW];
    {
        const int u = head ? d0 + gi : 0;
        const float2* ts = reinterpret_cast<const float2*>(drv_ts) + size_t(u) * NV + v0;
#pragma unroll
        for (int w = 0; w < NW; ++w) at_h[w] = ts[w].x;
    }
    float best[NW];
    bool have = false;
#pragma unroll
    for (int w = 0; w < NW; ++w) best[w] = 0.0f;
    for (int s = sb; s < se; ++s) {
        const int slot = s0 + s;
        const int sa = G.bslot_arc[slot];
        const int so = G.bslot_out[slot] & 0x7fffffff;
        float val[NW];
        if (sa >= 0) {
            const float ndv = nd[sa];
            const float* ro = drv_rat + size_t(so) * NV + v0;
            const float* dl = arc_delay + size_t(sa) * NV + v0;
            const float2* ts = reinterpret_cast<const float2*>(arc_ts) + size_t(sa) * NV + v0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const float rin = ro[w] - dl[w];
                const float ati = ts[w].x;
                arc_rat[size_t(sa) * NV + v0 + w] = rin;
                arc_slack[size_t(sa) * NV + v0 + w] = early[w] ? (ati - rin) : (rin - ati);
                val[w] = rin - ndv;
            }
        } else {
#pragma unroll
            for (int w = 0; w < NW; ++w) val[w] = ep_rat[size_t(so) * NV + v0 + w];
        }
#pragma unroll
        for (int w = 0; w < NW; ++w)
            if (!have || (early[w] ? (val[w] > best[w]) : (val[w] < best[w]))) best[w] = val[w];
        have = true;
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const bool take = (lane + off) < seg_end;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const float b2 = __shfl_down(best[w], off, 64);
            if (take && (early[w] ? (b2 > best[w]) : (b2 < best[w]))) best[w] = b2;
        }
    }
    if (head) {
        const int u = d0 + gi;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const float r = best[w];
            const float at = at_h[w];
            drv_rat[size_t(u) * NV + v0 + w] = r;
            drv_slack[size_t(u) * NV + v0 + w] = early[w] ? (at - r) : (r - at);
        }
    }
}

// ---------------------------------------------------------------------------------
// exact endpoint TNS: fixed-point digits
// ---------------------------------------------------------------------------------

// |x| of a finite FP32 value is m * 2^(sh - 149) with m < 2^24 and 0 <= sh <= 253.
// It is added exactly into a 320-bit fixed-point number held as ten 32-bit digits in
// 64-bit words (the upper halves absorb carries; 2^31 additions cannot overflow).
constexpr int kLimbs = 10;
constexpr int kK4Blocks = 256;
constexpr int kK4Threads = 256;
static_assert(kK4Blocks <= 256, "k_endpoint_final's 256 threads read one partial block each");

constexpr size_t kSlackScratchBytes =
    size_t(kK4Blocks) * STA_MAX_VIEWS * kLimbs * 8 + size_t(kK4Blocks) * STA_MAX_VIEWS * 4;

size_t scratch_bytes() { return kSlackScratchBytes; }

// The endpoint summary's per-block partials for sta_slack_noalloc: one copy of this array
// per device (the code object's global), held until the process ends, shared by every
// sta_slack_noalloc call on that device.  Host code never uses its name as an address:
// the device address comes from hipGetSymbolAddress (slack_scratch_ptr below).
constexpr size_t kNoAllocScratchBytes = 192 * 1024;
static_assert(kSlackScratchBytes <= kNoAllocScratchBytes, "the endpoint partials must fit the static scratch");
static __device__ __align__(256) unsigned char slack_scratch[kNoAllocScratchBytes];

__device__ __forceinline__ void add_neg_slack(unsigned long long (&l)[kLimbs], float s) {
    if (!(s < 0.0f)) return;
    const uint32_t bits = __float_as_uint(s) & 0x7fffffffu;
    const uint32_t ex = bits >> 23;
    uint64_t m = bits & 0x7fffffu;
    if (ex) m |= 0x800000u;
    const int sh = ex ? int(ex) - 1 : 0;
    const int li = sh >> 5;
    const uint64_t x = m << (sh & 31);
    const uint64_t lo = x & 0xffffffffull, hi = x >> 32;
#pragma unroll
    for (int i = 0; i < kLimbs; ++i) {
        l[i] += (i == li) ? lo : 0ull;
        l[i] += (i == li + 1) ? hi : 0ull;
    }
}

// carries propagated, then sum(L[i] 2^(32 i)) * 2^-149 rounded to nearest-even FP64
__device__ double digits_to_double(const unsigned long long* S) {
    uint64_t L[kLimbs];
    uint64_t carry = 0;
#pragma unroll
    for (int i = 0; i < kLimbs; ++i) {
        const uint64_t x = S[i] + carry;            // < 2^63 + 2^32
        L[i] = x & 0xffffffffull;
        carry = x >> 32;
    }
    int t = -1;
#pragma unroll
    for (int i = 0; i < kLimbs; ++i)
        if (L[i]) t = i;
    if (t < 0) return 0.0;
    // 128-bit window of digits t..t-3 (missing digits are 0); the rest is sticky
    uint64_t d0 = 0, d1 = 0, d2 = 0, d3 = 0;
    bool sticky = false;
#pragma unroll
    for (int i = 0; i < kLimbs; ++i) {
        if (i == t) d0 = L[i];
        else if (i == t - 1) d1 = L[i];
        else if (i == t - 2) d2 = L[i];
        else if (i == t - 3) d3 = L[i];
        else if (i < t - 3) sticky = sticky || (L[i] != 0ull);
    }
    const uint64_t hi = (d0 << 32) | d1;
    const uint64_t lo = (d2 << 32) | d3;
    const int s = __clzll(hi);                     // 0..31: hi's top digit is nonzero
    const uint64_t whi = s ? ((hi << s) | (lo >> (64 - s))) : hi;
    const uint64_t wlo = lo << s;
    const int msb = 32 * t + 31 - s;               // bit index of the leading one
    uint64_t mant = whi >> 11;                     // 53 bits
    const uint64_t rb = whi & 0x7ffull;
    sticky = sticky || (wlo != 0ull);
    int e = msb - 52;
    if (rb > 0x400ull || (rb == 0x400ull && (sticky || (mant & 1ull)))) mant += 1ull;
    if (mant == (1ull << 53)) { mant >>= 1; e += 1; }
    return ldexp(double(mant), e - 149);
}

// ---------------------------------------------------------------------------------
// level schedule kernels
// ---------------------------------------------------------------------------------

// Tile bounds of one level passed by value in the kernel arguments (read with scalar
// loads at wave start, no dependent memory round trip); wider levels read them from
// the graph's tile arrays.
constexpr int kArgTiles = 160;
struct KTiles {
    int32_t inl;                 // 1: bounds below are valid
    int32_t first[kArgTiles + 1];  // first arc (forward) or slot (backward) of each tile, + end
    int32_t base[kArgTiles];       // first gate (forward) or driver (backward) of each tile
};

// Level schedule, forward: one tile per 64-lane block.  The block first issues its
// tile's arc loads, then gathers the drivers' results and computes (the tables stay in
// global memory: copying them into each block's LDS was measured slower than the
// L2-resident reads it replaces).
template <int NV>
__global__ __launch_bounds__(64 * kLevelWaves) void k_forward(DevGraph G, KLib lib, KViews V, int tile0, int tile1, KTiles kt,
                                                 const float* __restrict__ arc_load, const float* __restrict__ nd,
                                                 const float* __restrict__ ni, float* __restrict__ drv_ts,
                                                 float* __restrict__ arc_ts, float* __restrict__ arc_delay,
                                                 uint8_t* __restrict__ argmax) {
    __shared__ float s_ax[26];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = tile0 + blockIdx.x * kLevelWaves + wave;
    const bool valid = t < tile1;
    int a0 = 0, n = 0, g0 = 0;
    if (valid) {
        if (kt.inl) {
            a0 = kt.first[t - tile0];
            n = kt.first[t - tile0 + 1] - a0;
            g0 = kt.base[t - tile0];
        } else {
            a0 = G.ftile_arc[t];
            n = G.ftile_arc[t + 1] - a0;
            g0 = G.ftile_gate[t];
        }
    }
    const bool act = lane < n;
    const int a = a0 + lane;
    const int ac = act ? a : 0;                 // clamped: unconditional first-round loads
    const uint32_t meta_r = G.arc_meta[ac];
    const int u_r = G.arc_src[ac];
    const float nd_r = nd[ac], ni_r = ni[ac], lo_r = arc_load[ac];
    const uint32_t meta = act ? meta_r : 0u;
    const int u = act ? u_r : 0;
    FwdLane x;
    x.nd = act ? nd_r : 0.0f;
    x.ni = act ? ni_r : 0.0f;
    x.Lo = act ? lo_r : 0.0f;
    load_axes(s_ax, lib);
    __syncthreads();
    if (!valid) return;
    fwd_lane_setup(x, act, meta, n, lane);
    x.a = a;
    x.g = g0 + x.gi;
    int j = 0;
    float ty = 0.0f;
    gate_jty(s_ax, x.Lo, j, ty);
    const float* tab[NV];
    bool early[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        tab[v] = lib.tables + size_t(V.set[v]) * lib.n_tables * 98;
        early[v] = V.mode[v] == STA_EARLY;
    }
    // second round: the drivers' results
    float2 ts[NV];
    const float2* srcp = reinterpret_cast<const float2*>(drv_ts) + size_t(u) * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) ts[v] = srcp[v];
    fwd_finish<NV>(x, ts, j, ty, 64, s_ax, tab, early, NV, 0, G.n_pi, drv_ts, arc_ts, arc_delay, argmax);
}


// ---------------------------------------------------------------------------------
// fused forward spans: kSpanF levels per launch, one span tile per wavefront
// ---------------------------------------------------------------------------------

// Makes a loaded value opaque to the optimizer at this point, so that the load stays where
// it was issued (ahead of its use) instead of being sunk into the branch that uses it.
template <typename T>
__device__ __forceinline__ void pin_value(T& x) {
    asm volatile("" : "+v"(x));
}

// f(integral_constant<int, C>) for C = C0 .. N-1 in order: a loop expanded at compile time,
// so that per-level register arrays are indexed by constants (the loop unroller leaves a
// long level loop rolled, and its arrays then go to LDS or indexed register moves)
template <int C0, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (C0 < N) {
        f(std::integral_constant<int, C0>{});
        static_for<C0 + 1, N>(f);
    }
}

// lane l takes lane l + OFF of its 16-lane row (DPP row shift; lanes past the row end read
// 0, which the callers never take)
template <int OFF>
__device__ __forceinline__ int row_down(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x100 + OFF, 0xf, 0xf, true);
}

// one step of the segmented maximum with argmax (and maximum slew) inside 16-lane rows
template <int OFF, int NW>
__device__ __forceinline__ void span_max_step(float* cand, float* slw, int* best_k, bool take) {
    float c2[NW], s2[NW];
    int k2[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        c2[w] = __int_as_float(row_down<OFF>(__float_as_int(cand[w])));
        s2[w] = __int_as_float(row_down<OFF>(__float_as_int(slw[w])));
        k2[w] = row_down<OFF>(best_k[w]);
    }
    // bitwise conjunctions (no short circuit), so that the step compiles to compares and
    // selects under one mask instead of a branch on the segment test
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const bool tc = take & (c2[w] > cand[w]);
        const bool ts = take & (s2[w] > slw[w]);
        cand[w] = tc ? c2[w] : cand[w];
        best_k[w] = tc ? k2[w] : best_k[w];
        slw[w] = ts ? s2[w] : slw[w];
    }
}

// one step of a segmented minimum / sum inside 16-lane rows
template <int OFF, int NV>
__device__ __forceinline__ void span_min_step(float* best, bool take) {
    float b2[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) b2[v] = __int_as_float(row_down<OFF>(__float_as_int(best[v])));
#pragma unroll
    for (int v = 0; v < NV; ++v) best[v] = (take & (b2[v] < best[v])) ? b2[v] : best[v];
}
template <int OFF, int NV>
__device__ __forceinline__ void span_sum_step(float* acc, bool take) {
    float b2[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) b2[v] = __int_as_float(row_down<OFF>(__float_as_int(acc[v])));
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = take ? acc[v] + b2[v] : acc[v];
}

// fwd_finish for a span chunk: the same arithmetic, plus every view's gate result kept
// in LDS (slot-indexed) for the tile's gates of the levels above
template <int NW>
__device__ __forceinline__ void fwd_finish_span(const FwdLane& x, const float2* ts, int j, float ty, int span,
                                                const Axis6& ax_x, const Sq5& sq_x, const float* const* tab, const bool* early,
                                                int NV, int v0, int n_pi, float* __restrict__ drv_ts,
                                                float* __restrict__ arc_ts, float* __restrict__ arc_delay,
                                                uint8_t* __restrict__ argmax, float2* lds_res, int slot) {
    const int lane = threadIdx.x & 63;
    float cand[NW], slw[NW];
    int best_k[NW];
    if (x.active) {
        float2* dst = at32(reinterpret_cast<float2*>(arc_ts), (uint32_t(x.a) * NV + v0) * 8u);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const float ai = ts[w].x + x.nd;
            const float su2 = ts[w].y * ts[w].y;
            const float a = su2 + x.ni;
            // the segment from a, so that the table reads need not wait for the root
            float x0, dx;
            const int i = seg6_sq(ax_x, sq_x, a, x0, dx);
            const float si = sqrtf(a);
            const float tx = (si - x0) / dx;
            float dl, sl;
            bilerp_pair(tab[w], x.tb, i, j, tx, ty, dl, sl);
            dst[w] = make_float2(ai, si);
            *at32(arc_delay, (uint32_t(x.a) * NV + v0 + w) * 4u) = dl;
            // early views negated, so that every view takes a maximum (negation is exact)
            cand[w] = early[w] ? -(ai + dl) : ai + dl;
            slw[w] = early[w] ? -sl : sl;
            best_k[w] = x.kpos;
        }
    } else {
        // padding and idle lanes can sit inside a gate's lane range: they never win
#pragma unroll
        for (int w = 0; w < NW; ++w) { cand[w] = -__builtin_inff(); slw[w] = -__builtin_inff(); best_k[w] = 0; }
    }
    // segmented maximum with argmax over a gate's arcs: ceil(log2(widest gate)) steps.
    // Gates of <= 16 arcs lie inside 16-lane rows, so the steps are row shifts (DPP, no
    // LDS round trip); wider gates use cross-lane permutes, every one of a step issued
    // before any is used.
    if (span <= 16) {
        if (span > 1) span_max_step<1, NW>(cand, slw, best_k, (lane + 1) < x.seg_end);
        if (span > 2) span_max_step<2, NW>(cand, slw, best_k, (lane + 2) < x.seg_end);
        if (span > 4) span_max_step<4, NW>(cand, slw, best_k, (lane + 4) < x.seg_end);
        if (span > 8) span_max_step<8, NW>(cand, slw, best_k, (lane + 8) < x.seg_end);
    } else {
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            const int off = 1 << st;
            if (off >= span) break;             // uniform
            const bool take = (lane + off) < x.seg_end;
            float c2[NW], s2[NW];
            int k2[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                c2[w] = __shfl_down(cand[w], off, 64);
                s2[w] = __shfl_down(slw[w], off, 64);
                k2[w] = __shfl_down(best_k[w], off, 64);
            }
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const bool tc = take && c2[w] > cand[w];
                cand[w] = tc ? c2[w] : cand[w];
                best_k[w] = tc ? k2[w] : best_k[w];
                slw[w] = (take && s2[w] > slw[w]) ? s2[w] : slw[w];
            }
        }
    }
    if (x.head) {
        float2* out = at32(reinterpret_cast<float2*>(drv_ts), (uint32_t(n_pi + x.g) * NV + v0) * 8u);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            cand[w] = early[w] ? -cand[w] : cand[w];
            slw[w] = early[w] ? -slw[w] : slw[w];
            out[w] = make_float2(cand[w], slw[w]);
            *at32(argmax, uint32_t(x.g) * NV + v0 + w) = uint8_t(best_k[w]);
            lds_res[slot * NW + w] = make_float2(cand[w], slw[w]);
        }
    }
}

// One wavefront per span tile.  Two rounds of loads for the whole tile (its arc records;
// then the arcs' static data and the arrivals of drivers outside the span), then the
// levels in order, each reading its in-span inputs from LDS: one table round per level
// instead of one launch and three rounds per level.
// NV views stored, NW of them computed per wavefront: views v0 .. v0 + NW - 1 with
// v0 = blockIdx.y * NW (so the views of a tile can run on different compute units).
// (Copying the view's table set into each workgroup's LDS with direct-to-LDS loads, so that
// the levels read table corners from LDS, was measured slower: the copy delays the tile's
// own gathers by more than the levels save.)
// The body of one forward span tile t of graph G, views v0 .. v0 + NW - 1 (tc: t clamped
// into the launch's tiles, for the unconditional record loads; a wavefront with !valid
// returns after them).  res: the wavefront's LDS results, kSpanSlotsF * NW values.
// FIRST (the pass's first launch, when it is a span): drivers that are primary inputs are
// read from pi_ts, and lane pe >= 0 of the launch copies primary-input element pe (one
// view's arrival and slew) from pi_ts into drv_ts, loaded with the records and stored
// after the last level, in place of a separate copy launch.
template <int NV, int NW, bool FIRST = false>
__device__ __forceinline__ void fwd_span_tile(const DevGraph& G, const KLib& lib, const KViews& V, int t, int tc,
                                              bool valid, int v0, const float* __restrict__ arc_load,
                                              const float* __restrict__ nd, const float* __restrict__ ni,
                                              float* __restrict__ drv_ts, float* __restrict__ arc_ts,
                                              float* __restrict__ arc_delay, uint8_t* __restrict__ argmax,
                                              float2* res, const float* __restrict__ pi_ts = nullptr, int pe = -1) {
    // the table axes in wave-uniform registers
    const Axis6 ax_x = axis6_v(lib, 0, 14), ax_y = axis6_v(lib, 7, 20);
    const Sq5 sq_x = sq5(lib);
    const int lane = threadIdx.x & 63;
    const float* tab[NW];
    bool early[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        tab[w] = lib.tables + size_t(V.set[v0 + w]) * lib.n_tables * 98;
        early[w] = V.mode[v0 + w] == STA_EARLY;
    }
    // round 1: the tile's level and arc records, all indexed by (tile, level, lane)
    int na[kSpanF], sl0[kSpanF], mk[kSpanF];
    int ar[kSpanF], sc[kSpanF], gt[kSpanF];
    uint32_t meta[kSpanF];
    int nch = 0;
#pragma unroll
    for (int c = 0; c < kSpanF; ++c) {
        const int4 cr = G.sp_crec[tc * kSpanF + c];
        na[c] = cr.x;
        sl0[c] = cr.y;
        mk[c] = cr.z;
        nch = cr.w;
        const int4 r = G.sp_arec[size_t(tc * kSpanF + c) * 64 + lane];
        ar[c] = r.x;
        sc[c] = r.y;
        gt[c] = r.z;
        meta[c] = uint32_t(r.w);
    }
    float2 piv = make_float2(0.0f, 0.0f);
    if constexpr (FIRST) {
        piv = reinterpret_cast<const float2*>(pi_ts)[pe >= 0 ? pe : 0];
        if (!valid) {
            if (pe >= 0) reinterpret_cast<float2*>(drv_ts)[pe] = piv;
            return;
        }
    }
    if (!valid) return;
    // round 2: the arcs' net data and the arrivals of drivers outside the span
    float ndv[kSpanF], niv[kSpanF], lov[kSpanF];
    float2 ext[kSpanF][NW];
#pragma unroll
    for (int c = 0; c < kSpanF; ++c) {
        const uint32_t a4 = uint32_t(ar[c]) * 4u;
        ndv[c] = *at32(nd, a4);
        niv[c] = *at32(ni, a4);
        lov[c] = *at32(arc_load, a4);
        const int u = sc[c] >= 0 ? sc[c] : 0;
        const float2* sp;
        if constexpr (FIRST)
            sp = reinterpret_cast<const float2*>(u < G.n_pi ? pi_ts : drv_ts) + size_t(u) * NV + v0;
        else
            sp = at32(reinterpret_cast<const float2*>(drv_ts), (uint32_t(u) * NV + v0) * 8u);
#pragma unroll
        for (int w = 0; w < NW; ++w) ext[c][w] = sp[w];
    }
    // all of round 2 is in flight; keep it there (one wait before the first level)
#pragma unroll
    for (int c = 0; c < kSpanF; ++c) {
        pin_value(ndv[c]);
        pin_value(niv[c]);
        pin_value(lov[c]);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            pin_value(ext[c][w].x);
            pin_value(ext[c][w].y);
        }
    }
    // the levels of the tile, in order
    static_for<0, kSpanF>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if (c >= nch) return;                   // uniform
        const bool act = gt[c] != -1;           // gate word -1: padding or idle lane
        FwdLane x;
        fwd_lane_setup_span(x, act, meta[c], uint32_t(gt[c]));
        x.a = ar[c];
        x.nd = act ? ndv[c] : 0.0f;
        x.ni = act ? niv[c] : 0.0f;
        x.Lo = act ? lov[c] : 0.0f;
        int j = 0;
        float ty = 0.0f;
        {
            float y0, dy;
            j = seg6_sel(ax_y, x.Lo, y0, dy);
            ty = (x.Lo - y0) / dy;
        }
        // the source: an in-tile gate's result from LDS (read by every lane, from slot 0
        // when the source is outside the tile, so that there is no branch) or the gathered one
        float2 ts[NW];
        {
            const bool lds_src = sc[c] < 0;
            const int src = lds_src ? -1 - sc[c] : 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const float2 r = res[src * NW + w];
                const float2 e = act ? ext[c][w] : make_float2(0.0f, 0.0f);
                ts[w] = (act && lds_src) ? r : e;
            }
        }
        fwd_finish_span<NW>(x, ts, j, ty, mk[c], ax_x, sq_x, tab, early, NV, v0, G.n_pi, drv_ts, arc_ts, arc_delay,
                            argmax, res, sl0[c] + x.gi);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    });
    if constexpr (FIRST) {
        if (pe >= 0) reinterpret_cast<float2*>(drv_ts)[pe] = piv;
    }
}

// Spare workgroups of a span launch load the records of the next launch's tiles, and data
// they gather, into L2 before that launch reads them.  Workgroups go to the XCDs (each with
// its own L2) round-robin by linear index, and every span launch's grid has a multiple of
// eight workgroups per view group, so the next launch's tile r runs on XCD r mod 8 in every view
// group; spare workgroup q (counted from a multiple of eight) serves the next tiles r with
// r = q (mod 8), kSpanPfTilesF (forward) or kSpanPfTilesB (backward) of them.  One tile per
// spare wavefront measured best forward, two backward (c2 propagate 0.3023 -> 0.3010 ms;
// slack 0.2978 -> 0.3038 ms with one).
constexpr int kSpanPfTilesF = 1;
constexpr int kSpanPfTilesB = 2;

__host__ __device__ __forceinline__ int span_round8(int n) { return (n + 7) & ~7; }
__host__ __device__ __forceinline__ int span_pf_blocks(int n_next, int per) {
    return n_next > 0 ? 8 * ((((n_next + 7) / 8) + per - 1) / per) : 0;
}

// Spare workgroup q of a forward span launch: the next launch's tile records, then the data
// their arcs gather that is final before this launch starts (net delay and spread, arc load,
// and the arrivals of source drivers numbered below fin: drivers are numbered level by level,
// and fin is the first driver of this launch's span, 0 in the launch that copies the primary
// inputs), into L2.
template <int NV>
__device__ __forceinline__ void fwd_prefetch_gathers(const DevGraph& G, const float* __restrict__ arc_load,
                                                      const float* __restrict__ nd, const float* __restrict__ ni,
                                                      const float* __restrict__ drv_ts, int pf0, int pf1, int q, int fin) {
    const int lane = threadIdx.x & 63;
    const int rho = q & 7, kappa = q >> 3;
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kSpanPfTilesF; ++i) {
        const int t = pf0 + rho + 8 * (kappa * kSpanPfTilesF + i);
        if (t >= pf1) break;                    // uniform
        int4 r[kSpanF];
#pragma unroll
        for (int c = 0; c < kSpanF; ++c) r[c] = G.sp_arec[size_t(t * kSpanF + c) * 64 + lane];
        const int4 cr = G.sp_crec[t * kSpanF + (lane & (kSpanF - 1))];
        acc ^= uint32_t(cr.x ^ cr.y ^ cr.z ^ cr.w);
        float f[kSpanF][4];
#pragma unroll
        for (int c = 0; c < kSpanF; ++c) {
            const uint32_t a4 = uint32_t(r[c].x) * 4u;
            f[c][0] = *at32(nd, a4);
            f[c][1] = *at32(ni, a4);
            f[c][2] = *at32(arc_load, a4);
            const int u = r[c].y;
            f[c][3] = (u >= 0 && u < fin) ? drv_ts[size_t(u) * NV * 2] : 0.0f;
        }
#pragma unroll
        for (int c = 0; c < kSpanF; ++c)
            acc ^= __float_as_uint(f[c][0]) ^ __float_as_uint(f[c][1]) ^ __float_as_uint(f[c][2]) ^ __float_as_uint(f[c][3]);
    }
    asm volatile("" ::"v"(acc));
}

template <int NV, int NW, bool FIRST>
__global__ __launch_bounds__(64 * kSpanWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_forward_span(DevGraph G, KLib lib, KViews V, int tile0, int tile1,
                                                      const float* __restrict__ arc_load,
                                                      const float* __restrict__ nd, const float* __restrict__ ni,
                                                      float* __restrict__ drv_ts, float* __restrict__ arc_ts,
                                                      float* __restrict__ arc_delay, uint8_t* __restrict__ argmax,
                                                      int pf0, int pf1, const float* __restrict__ pi_ts, int pf_fin) {
    __shared__ float2 s_res[kSpanWaves][kSpanSlotsF * NW];
    static_assert(kSpanWaves == 1, "one span tile per workgroup");
    const int tb = tile1 - tile0;               // workgroups of tiles
    if (int(blockIdx.x) >= tb) {
        // spare workgroups: the next launch's records and gathers (first view group only)
        const int q = int(blockIdx.x) - span_round8(tb);
        if (blockIdx.y == 0 && q >= 0 && pf1 > pf0) fwd_prefetch_gathers<NV>(G, arc_load, nd, ni, drv_ts, pf0, pf1, q, pf_fin);
        return;
    }
    const int t = tile0 + int(blockIdx.x);
    // FIRST: this lane's primary-input element (-1: none)
    int pe = -1;
    if constexpr (FIRST) {
        const int e = (int(blockIdx.y) * tb + int(blockIdx.x)) * 64 + int(threadIdx.x & 63);
        pe = e < G.n_pi * NV ? e : -1;
    }
    fwd_span_tile<NV, NW, FIRST>(G, lib, V, t, t, true, int(blockIdx.y) * NW, arc_load, nd, ni, drv_ts, arc_ts,
                                 arc_delay, argmax, s_res[0], pi_ts, pe);
}

// Batched forward spans: workgroup x of the launch runs tile map[map0 + x].y of design
// map[map0 + x].x (one span of each of several designs per launch), views blockIdx.y * NW
// onwards; every design has the batch's views.
template <int NV, int NW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_forward_span_batch(
    const BatchItem* __restrict__ items, const int2* __restrict__ map, int map0, KLib lib, KViews V) {
    static_assert(kSpanWaves == 1, "one span tile per workgroup");
    __shared__ float2 s_res[kSpanSlotsF * NW];
    const int2 m = map[map0 + int(blockIdx.x)];
    const BatchItem& it = items[m.x];
    fwd_span_tile<NV, NW>(it.G, lib, V, m.y, m.y, true, int(blockIdx.y) * NW, it.arc_load, it.nd, it.ni,
                                 it.drv_ts, it.arc_ts, it.arc_delay, it.argmax, s_res);
}

// primary inputs: copy (arrival, slew) of every view
__global__ void k_copy_pi(const float* __restrict__ pi_ts, float* __restrict__ drv_ts, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) drv_ts[i] = pi_ts[i];
}

// the same for every design of a batch: design blockIdx.y, n_pi * NV * 2 values each
__global__ void k_copy_pi_batch(const BatchItem* __restrict__ items, int NV) {
    const BatchItem& it = items[blockIdx.y];
    const int n = it.G.n_pi * NV * 2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) it.drv_ts[i] = it.pi_ts[i];
}

template <int NV>
__global__ __launch_bounds__(64 * kLevelWaves) void k_backward(DevGraph G, KViews V, int tile0, int tile1, KTiles kt,
                                                  const float* __restrict__ nd, const float* __restrict__ drv_ts,
                                                  const float* __restrict__ arc_ts,
                                                  const float* __restrict__ arc_delay,
                                                  const float* __restrict__ ep_rat, float* __restrict__ drv_rat,
                                                  float* __restrict__ arc_rat, float* __restrict__ drv_slack,
                                                  float* __restrict__ arc_slack) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = tile0 + blockIdx.x * kLevelWaves + wave;
    if (t >= tile1) return;
    bool early[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) early[v] = V.mode[v] == STA_EARLY;
    int s0, n, d0;
    if (kt.inl) {
        s0 = kt.first[t - tile0];
        n = kt.first[t - tile0 + 1] - s0;
        d0 = kt.base[t - tile0];
    } else {
        s0 = G.btile_slot[t];
        n = G.btile_slot[t + 1] - s0;
        d0 = G.btile_drv[t];
    }
    bwd_tile<NV>(G, early, NV, 0, s0, n, d0, nd, drv_ts, arc_ts, arc_delay, ep_rat, drv_rat, arc_rat, drv_slack,
                 arc_slack);
}


// One wavefront per backward span tile (views 0..NV-1): two rounds of loads for the whole
// tile (its slot records; then the slots' arc data, the drivers' arrivals, and the required
// times of sink gates outside the span or the endpoint required times), then the levels
// top down, in-span required times handed over through LDS.
// NV views stored, NW computed per wavefront (views v0 = blockIdx.y * NW onwards).
// The body of one backward span tile t of graph G, views v0 .. v0 + NW - 1; rs: the
// wavefront's LDS required times, kSpanSlotsB * NW values.
template <int NV, int NW>
__device__ __forceinline__ void bwd_span_tile(const DevGraph& G, const KViews& V, int t, int v0,
                                              const float* __restrict__ nd, const float* __restrict__ drv_ts,
                                              const float* __restrict__ arc_ts, const float* __restrict__ arc_delay,
                                              const float* __restrict__ ep_rat, float* __restrict__ drv_rat,
                                              float* __restrict__ arc_rat, float* __restrict__ drv_slack,
                                              float* __restrict__ arc_slack, float* rs) {
    const int lane = threadIdx.x & 63;
    bool early[NW];
#pragma unroll
    for (int v = 0; v < NW; ++v) early[v] = V.mode[v0 + v] == STA_EARLY;
    // round 1: the tile's level and slot records, all indexed by (tile, level, lane)
    int ns[kSpanB], ds0[kSpanB], ms[kSpanB];
    int sa_[kSpanB], so_[kSpanB], src[kSpanB], drv[kSpanB], sge[kSpanB], grk[kSpanB];
    bool hd[kSpanB];
    int nch = 0;
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        const int4 cr = G.bp_crec[t * kSpanB + c];
        ns[c] = cr.x;
        ds0[c] = cr.y;
        ms[c] = cr.z;
        nch = cr.w;
        const int4 r = G.bp_srec[size_t(t * kSpanB + c) * 64 + lane];
        const uint32_t bo = uint32_t(r.y);
        sa_[c] = r.x;
        so_[c] = int(bo & 0x7fffffffu);
        hd[c] = (bo & kHeadBit) != 0u;
        src[c] = int(int16_t(r.z & 0xffff));
        sge[c] = (r.z >> 16) & 0x7f;
        drv[c] = r.w & 0x3ffffff;
        grk[c] = int(uint32_t(r.w) >> 26);
    }
    // round 2: the slot data the required times need (net delay, arc delay, required
    // times from outside the tile), waited for before the first level; then the arrivals
    // that only the slacks need, issued behind them and used after the last level
    float ndv[kSpanB], dl[kSpanB][NW], ati[kSpanB][NW], ext[kSpanB][NW], atd[kSpanB][NW];
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        const int sa = sa_[c];
        const int sac = sa >= 0 ? sa : 0;
        ndv[c] = nd[sac];
        const float* ext_src = (sa >= 0) ? (drv_rat + size_t(so_[c]) * NV + v0) : (ep_rat + size_t(so_[c]) * NV + v0);
        const float* ext_ld = src[c] >= 0 ? ep_rat : ext_src;   // in-tile sources: any valid address
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            dl[c][v] = arc_delay[size_t(sac) * NV + v0 + v];
            ext[c][v] = ext_ld[v];
        }
    }
    asm volatile("" ::: "memory");             // the loads above issue first
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        const int sac = sa_[c] >= 0 ? sa_[c] : 0;
        const float* ts = arc_ts + (size_t(sac) * NV + v0) * 2;
        const float* dt = drv_ts + (size_t(drv[c]) * NV + v0) * 2;
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            ati[c][v] = ts[2 * v];
            atd[c][v] = dt[2 * v];
        }
    }
    asm volatile("" ::: "memory");             // and these stay here, in flight
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        pin_value(ndv[c]);
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            pin_value(dl[c][v]);
            pin_value(ext[c][v]);
        }
    }
    float rin_[kSpanB][NW], rdrv[kSpanB][NW];
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        if (c >= nch) break;                    // uniform
        const bool act = src[c] != -2;          // source -2: padding or idle lane
        const bool head = act && hd[c];
        const int gi = grk[c];                 // from the record
        const int seg_end = sge[c];            // from the record
        const bool on_arc = act && sa_[c] >= 0;
        // the required times at the sinks' gate outputs: from LDS (in-tile) or prefetched
        const int si = src[c] >= 0 ? src[c] : 0;
        float ro[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v) ro[v] = rs[si * NW + v];
#pragma unroll
        for (int v = 0; v < NW; ++v) ro[v] = src[c] >= 0 ? ro[v] : ext[c][v];
        // per slot: the value its driver minimizes (maximizes early), negated for early
        // views so that every view takes a minimum (negation is exact: same results)
        float best[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            const float rin = ro[v] - dl[c][v];
            rin_[c][v] = rin;
            const float val = on_arc ? rin - ndv[c] : ext[c][v];
            best[v] = act ? (early[v] ? -val : val) : __builtin_inff();   // idle lanes never win
        }
        if (on_arc) {
#pragma unroll
            for (int v = 0; v < NW; ++v) arc_rat[size_t(sa_[c]) * NV + v0 + v] = rin_[c][v];
        }
        // segmented minimum over a driver's slots: ceil(log2(most slots)) steps; drivers of
        // <= 16 slots lie inside 16-lane rows (DPP row shifts), wider ones use permutes
        if (ms[c] <= 16) {
            if (ms[c] > 1) span_min_step<1, NW>(best, (lane + 1) < seg_end);
            if (ms[c] > 2) span_min_step<2, NW>(best, (lane + 2) < seg_end);
            if (ms[c] > 4) span_min_step<4, NW>(best, (lane + 4) < seg_end);
            if (ms[c] > 8) span_min_step<8, NW>(best, (lane + 8) < seg_end);
        } else {
#pragma unroll
            for (int st = 0; st < 6; ++st) {
                const int off = 1 << st;
                if (off >= ms[c]) break;        // uniform
                const bool take = (lane + off) < seg_end;
                float b2[NW];
#pragma unroll
                for (int v = 0; v < NW; ++v) b2[v] = __shfl_down(best[v], off, 64);
#pragma unroll
                for (int v = 0; v < NW; ++v) best[v] = (take && b2[v] < best[v]) ? b2[v] : best[v];
            }
        }
        if (head) {
            const int u = drv[c];
#pragma unroll
            for (int v = 0; v < NW; ++v) {
                const float r = early[v] ? -best[v] : best[v];
                drv_rat[size_t(u) * NV + v0 + v] = r;
                rs[(ds0[c] + gi) * NW + v] = r;
            }
        }
#pragma unroll
        for (int v = 0; v < NW; ++v) rdrv[c][v] = early[v] ? -best[v] : best[v];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the slacks, once the arrivals have landed
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        if (c >= nch) break;                    // uniform
        const bool act = src[c] != -2;
        if (act && sa_[c] >= 0) {
#pragma unroll
            for (int v = 0; v < NW; ++v)
                arc_slack[size_t(sa_[c]) * NV + v0 + v] = early[v] ? (ati[c][v] - rin_[c][v]) : (rin_[c][v] - ati[c][v]);
        }
        if (act && hd[c]) {
            const int u = drv[c];
#pragma unroll
            for (int v = 0; v < NW; ++v)
                drv_slack[size_t(u) * NV + v0 + v] = early[v] ? (atd[c][v] - rdrv[c][v]) : (rdrv[c][v] - atd[c][v]);
        }
    }
}

// The endpoint summary folded into backward span launches (one 64-lane workgroup per
// partial; workgroups past the launch's tiles, in its first view group).  An endpoint's only
// slot is its endpoint slot, so the required time the backward pass takes for it is the
// endpoint's own, and its slack (required - arrival late, arrival - required early) is
// formed here from the arrivals and the endpoint required times, the same FP32 operation:
// the summary then does not wait for the backward pass.
struct EpFold {
    const float* drv_ts;       // [D][NV][2]
    const float* ep_rat;       // [E][NV]
    unsigned long long* limbs; // partials: [nblk][NV][kLimbs]
    float* pw;                 // [nblk][NV]
    double* tns;
    float* wns;
    int E, nblk;
    int role;                  // 0: none, 1: the partials, 2: the final sum
};

constexpr int kEpPerLane = 4;   // endpoints per lane in one round of loads

// first stage: workgroup blk of nblk takes endpoints blk * 256 + r * 64 + lane (r < 4),
// striding by nblk * 256
template <int NV>
__device__ __forceinline__ void endpoint_partial_fold(const DevGraph& G, const KViews& V, const EpFold& f, int blk) {
    __shared__ unsigned long long s_l[NV * kLimbs];
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < NV * kLimbs; i += 64) s_l[i] = 0ull;
    __syncthreads();
    bool early[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) early[v] = V.mode[v] == STA_EARLY;
    const int stride = f.nblk * 64 * kEpPerLane;
    auto slack_of = [&](int e, float (&sv)[NV]) {
        const bool in = e < f.E;
        const int u = in ? G.ep_drv[e] : 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            // (loads only for lanes with an endpoint)
            const float at = in ? f.drv_ts[(size_t(u) * NV + v) * 2] : 0.0f;
            const float r = in ? f.ep_rat[size_t(e) * NV + v] : 0.0f;
            sv[v] = in ? (early[v] ? at - r : r - at) : __builtin_inff();
        }
    };
    float s1[kEpPerLane][NV];
#pragma unroll
    for (int r = 0; r < kEpPerLane; ++r) slack_of(blk * 64 * kEpPerLane + r * 64 + lane, s1[r]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        unsigned long long l[kLimbs];
#pragma unroll
        for (int i = 0; i < kLimbs; ++i) l[i] = 0ull;
        float mn = __builtin_inff();
#pragma unroll
        for (int r = 0; r < kEpPerLane; ++r) {
            mn = (s1[r][v] < mn) ? s1[r][v] : mn;
            add_neg_slack(l, s1[r][v]);
        }
        for (int e0 = blk * 64 * kEpPerLane + stride; e0 < f.E; e0 += stride) {
#pragma unroll
            for (int r = 0; r < kEpPerLane; ++r) {
                float sv[NV];
                slack_of(e0 + r * 64 + lane, sv);
                mn = (sv[v] < mn) ? sv[v] : mn;
                add_neg_slack(l, sv[v]);
            }
        }
#pragma unroll
        for (int i = 0; i < kLimbs; ++i)
            if (l[i]) atomicAdd(&s_l[v * kLimbs + i], l[i]);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const float o2 = __shfl_xor(mn, off, 64);
            mn = (o2 < mn) ? o2 : mn;
        }
        if (lane == 0) f.pw[size_t(blk) * NV + v] = mn;
    }
    __syncthreads();
    for (int i = lane; i < NV * kLimbs; i += 64) f.limbs[size_t(blk) * NV * kLimbs + i] = s_l[i];
}

// second stage, one 64-lane workgroup over the nblk partials
template <int NV>
__device__ __forceinline__ void endpoint_final_fold(const EpFold& f) {
    __shared__ unsigned long long s_sum[NV * kLimbs];
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < NV * kLimbs; i += 64) s_sum[i] = 0ull;
    __syncthreads();
    const int n = f.nblk * NV * kLimbs;
    for (int i0 = lane; i0 < n; i0 += 8 * 64) {
        unsigned long long x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = i0 + r * 64;
            x[r] = i < n ? f.limbs[i] : 0ull;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if (x[r]) atomicAdd(&s_sum[(i0 + r * 64) % (NV * kLimbs)], x[r]);
    }
    float mn[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) mn[v] = __builtin_inff();
    for (int b = lane; b < f.nblk; b += 64) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float x = f.pw[size_t(b) * NV + v];
            mn[v] = (x < mn[v]) ? x : mn[v];
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const float o2 = __shfl_xor(mn[v], off, 64);
            mn[v] = (o2 < mn[v]) ? o2 : mn[v];
        }
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double mag = digits_to_double(&s_sum[v * kLimbs]);
            f.tns[v] = (mag == 0.0) ? 0.0 : -mag;
            f.wns[v] = mn[v];
        }
    }
}

// Spare workgroup q of a backward span launch (as fwd_prefetch_gathers, for the next
// launch's tiles): the tiles' records, then the data their slots gather that is final before
// this launch starts (net and arc delays, arrivals of the sink pins and of the drivers), into
// L2; required times from outside a tile can still change in this launch and are not loaded.
template <int NV>
__device__ __forceinline__ void bwd_prefetch_gathers(const DevGraph& G, const float* __restrict__ nd,
                                                     const float* __restrict__ drv_ts, const float* __restrict__ arc_ts,
                                                     const float* __restrict__ arc_delay, int pf0, int pf1, int q) {
    const int lane = threadIdx.x & 63;
    const int rho = q & 7, kappa = q >> 3;
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kSpanPfTilesB; ++i) {
        const int t = pf0 + rho + 8 * (kappa * kSpanPfTilesB + i);
        if (t >= pf1) break;                    // uniform
        int4 r[kSpanB];
#pragma unroll
        for (int c = 0; c < kSpanB; ++c) r[c] = G.bp_srec[size_t(t * kSpanB + c) * 64 + lane];
        const int4 cr = G.bp_crec[t * kSpanB + (lane & (kSpanB - 1))];
        acc ^= uint32_t(cr.x ^ cr.y ^ cr.z ^ cr.w);
        float f[kSpanB][4];
#pragma unroll
        for (int c = 0; c < kSpanB; ++c) {
            const int sac = r[c].x >= 0 ? r[c].x : 0;
            const int u = r[c].w & 0x3ffffff;
            f[c][0] = nd[sac];
            f[c][1] = arc_delay[size_t(sac) * NV];
            f[c][2] = arc_ts[size_t(sac) * NV * 2];
            f[c][3] = drv_ts[size_t(u) * NV * 2];
        }
#pragma unroll
        for (int c = 0; c < kSpanB; ++c)
            acc ^= __float_as_uint(f[c][0]) ^ __float_as_uint(f[c][1]) ^ __float_as_uint(f[c][2]) ^ __float_as_uint(f[c][3]);
    }
    asm volatile("" ::"v"(acc));
}

template <int NV, int NW>
__global__ __launch_bounds__(64 * kSpanWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_backward_span(DevGraph G, KViews V, int tile0, int tile1,
                                                       const float* __restrict__ nd, const float* __restrict__ drv_ts,
                                                       const float* __restrict__ arc_ts,
                                                       const float* __restrict__ arc_delay,
                                                       const float* __restrict__ ep_rat, float* __restrict__ drv_rat,
                                                       float* __restrict__ arc_rat, float* __restrict__ drv_slack,
                                                       float* __restrict__ arc_slack, EpFold ep, int pf0, int pf1) {
    __shared__ float s_rat[kSpanWaves][kSpanSlotsB * NW];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tb = (tile1 - tile0 + kSpanWaves - 1) / kSpanWaves;   // workgroups of tiles
    if (int(blockIdx.x) >= tb) {
        // past the tiles: the endpoint summary's workgroups, then the prefetch's
        // (first view group only)
        static_assert(kSpanWaves == 1, "the spare workgroups are one wavefront");
        if (blockIdx.y != 0) return;
        const int x = int(blockIdx.x) - tb;
        const int ne = ep.role == 1 ? ep.nblk : ep.role == 2 ? 1 : 0;
        if (x < ne) {
            if (ep.role == 1) endpoint_partial_fold<NV>(G, V, ep, x);
            else endpoint_final_fold<NV>(ep);
            return;
        }
        const int q = int(blockIdx.x) - span_round8(tb + ne);
        if (q >= 0 && pf1 > pf0) bwd_prefetch_gathers<NV>(G, nd, drv_ts, arc_ts, arc_delay, pf0, pf1, q);
        return;
    }
    const int t = tile0 + blockIdx.x * kSpanWaves + wave;
    if (t >= tile1) return;
    bwd_span_tile<NV, NW>(G, V, t, int(blockIdx.y) * NW, nd, drv_ts, arc_ts, arc_delay, ep_rat, drv_rat, arc_rat,
                          drv_slack, arc_slack, s_rat[wave]);
}

// Batched backward spans: workgroup x runs tile map[map0 + x].y of design map[map0 + x].x.
template <int NV, int NW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_backward_span_batch(
    const BatchItem* __restrict__ items, const int2* __restrict__ map, int map0, KViews V) {
    static_assert(kSpanWaves == 1, "one span tile per workgroup");
    __shared__ float s_rat[kSpanSlotsB * NW];
    const int2 m = map[map0 + int(blockIdx.x)];
    const BatchItem& it = items[m.x];
    bwd_span_tile<NV, NW>(it.G, V, m.y, int(blockIdx.y) * NW, it.nd, it.drv_ts, it.arc_ts, it.arc_delay, it.ep_rat,
                          it.drv_rat, it.arc_rat, it.drv_slack, it.arc_slack, s_rat);
}

// Endpoint summary, first stage: workgroup blk of nblk takes endpoints blk * 256 + t,
// striding by nblk * 256, and writes its digits and minimum to partial blk.
template <int NV>
__device__ __forceinline__ void endpoint_partial_body(const int32_t* __restrict__ ep_drv, int E,
                                                      const float* __restrict__ drv_slack, int blk, int nblk,
                                                      unsigned long long* __restrict__ part_limbs,
                                                      float* __restrict__ part_wns) {
    __shared__ unsigned long long s_l[NV * kLimbs];
    __shared__ float s_min[NV][kK4Threads / 64];
    for (int i = threadIdx.x; i < NV * kLimbs; i += blockDim.x) s_l[i] = 0ull;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // the thread's first endpoint: its slacks in every view in one round
    const int e1 = blk * int(blockDim.x) + int(threadIdx.x);
    const int stride = nblk * int(blockDim.x);
    float s1[NV];
    {
        const int u = e1 < E ? ep_drv[e1] : 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) s1[v] = e1 < E ? drv_slack[size_t(u) * NV + v] : __builtin_inff();
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        unsigned long long l[kLimbs];
#pragma unroll
        for (int i = 0; i < kLimbs; ++i) l[i] = 0ull;
        float mn = s1[v];
        add_neg_slack(l, s1[v]);
        for (int e = e1 + stride; e < E; e += stride) {
            const float s = drv_slack[size_t(ep_drv[e]) * NV + v];
            mn = (s < mn) ? s : mn;
            add_neg_slack(l, s);
        }
#pragma unroll
        for (int i = 0; i < kLimbs; ++i)
            if (l[i]) atomicAdd(&s_l[v * kLimbs + i], l[i]);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const float o2 = __shfl_xor(mn, off, 64);
            mn = (o2 < mn) ? o2 : mn;
        }
        if (lane == 0) s_min[v][w] = mn;
    }
    __syncthreads();
    if (threadIdx.x < NV * kLimbs) part_limbs[size_t(blk) * NV * kLimbs + threadIdx.x] = s_l[threadIdx.x];
    if (threadIdx.x < NV) {
        float mn = s_min[threadIdx.x][0];
        for (int i = 1; i < kK4Threads / 64; ++i) mn = (s_min[threadIdx.x][i] < mn) ? s_min[threadIdx.x][i] : mn;
        part_wns[size_t(blk) * NV + threadIdx.x] = mn;
    }
}

template <int NV>
__global__ __launch_bounds__(kK4Threads) void k_endpoint_partial(const int32_t* __restrict__ ep_drv, int E,
                                                                 const float* __restrict__ drv_slack,
                                                                 unsigned long long* __restrict__ part_limbs,
                                                                 float* __restrict__ part_wns) {
    endpoint_partial_body<NV>(ep_drv, E, drv_slack, int(blockIdx.x), int(gridDim.x), part_limbs, part_wns);
}

// Batched first stage: workgroup x is workgroup map[map0 + x].y of design map[map0 + x].x,
// whose partials start at items[..].ep_part0 in the batch's scratch.
template <int NV>
__global__ __launch_bounds__(kK4Threads) void k_endpoint_partial_batch(const BatchItem* __restrict__ items,
                                                                       const int2* __restrict__ map, int map0,
                                                                       unsigned long long* __restrict__ part_limbs,
                                                                       float* __restrict__ part_wns) {
    const int2 m = map[map0 + int(blockIdx.x)];
    const BatchItem& it = items[m.x];
    endpoint_partial_body<NV>(it.G.ep_drv, it.E, it.drv_slack, m.y, it.ep_blocks,
                              part_limbs + size_t(it.ep_part0) * NV * kLimbs, part_wns + size_t(it.ep_part0) * NV);
}

template <int NV>
__device__ __forceinline__ void endpoint_final_body(int nblk, const unsigned long long* __restrict__ part_limbs,
                                                    const float* __restrict__ part_wns, double* __restrict__ tns,
                                                    float* __restrict__ wns) {
    __shared__ unsigned long long s_sum[NV * kLimbs];
    __shared__ float s_min[NV][4];
    for (int i = threadIdx.x; i < NV * kLimbs; i += blockDim.x) s_sum[i] = 0ull;
    // nblk <= kK4Blocks == blockDim.x: each thread reads at most one block's minima, and
    // its share of the digits in rounds of eight loads issued before any is added
    float pmn[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        pmn[v] = int(threadIdx.x) < nblk ? part_wns[size_t(threadIdx.x) * NV + v] : __builtin_inff();
    __syncthreads();
    const int n = nblk * NV * kLimbs;
    for (int i0 = threadIdx.x; i0 < n; i0 += 8 * blockDim.x) {
        unsigned long long x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = i0 + r * int(blockDim.x);
            x[r] = i < n ? part_limbs[i] : 0ull;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if (x[r]) atomicAdd(&s_sum[(i0 + r * int(blockDim.x)) % (NV * kLimbs)], x[r]);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        float mn = pmn[v];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const float o2 = __shfl_xor(mn, off, 64);
            mn = (o2 < mn) ? o2 : mn;
        }
        if (lane == 0) s_min[v][w] = mn;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int v = threadIdx.x;
        const double mag = digits_to_double(&s_sum[v * kLimbs]);
        tns[v] = (mag == 0.0) ? 0.0 : -mag;
        float mn = s_min[v][0];
        for (int i = 1; i < 4; ++i) mn = (s_min[v][i] < mn) ? s_min[v][i] : mn;
        wns[v] = mn;
    }
}

template <int NV>
__global__ __launch_bounds__(256) void k_endpoint_final(int nblk, const unsigned long long* __restrict__ part_limbs,
                                                        const float* __restrict__ part_wns, double* __restrict__ tns,
                                                        float* __restrict__ wns) {
    endpoint_final_body<NV>(nblk, part_limbs, part_wns, tns, wns);
}

// Batched second stage: one workgroup per design (blockIdx.x), over its own partials.
template <int NV>
__global__ __launch_bounds__(256) void k_endpoint_final_batch(const BatchItem* __restrict__ items,
                                                              const unsigned long long* __restrict__ part_limbs,
                                                              const float* __restrict__ part_wns) {
    const BatchItem& it = items[blockIdx.x];
    if (it.ep_blocks == 0) return;                  // a design without slack buffers
    endpoint_final_body<NV>(it.ep_blocks, part_limbs + size_t(it.ep_part0) * NV * kLimbs,
                            part_wns + size_t(it.ep_part0) * NV, it.tns, it.wns);
}

// ---------------------------------------------------------------------------------
// view schedule kernels: one 1024-lane workgroup per view walks every level
// ---------------------------------------------------------------------------------
//
// Each level's static data (tile bounds, arc records, gate loads; for the backward
// pass sink slots and driver arrival times) is staged in LDS.  The loads for level
// l+1 are issued as coalesced 4-byte loads before level l computes and are written to
// LDS after it, so a level costs one dependent round trip (the gather of the drivers'
// results) plus its arithmetic.  A wave owns tiles wave, wave+16, ... of a level and
// issues the gathers of all of them before computing any.

constexpr int kViewThreads = 1024;
constexpr int kViewWaves = kViewThreads / 64;

// k_forward_view: the levels are cut into chunks (whole tiles of one level, at most
// kFwdCapA arcs / kFwdCapG gates).  While chunk c computes, the workgroup issues the
// global loads of chunk c+1's arc records and gate loads, of chunk c+2's driver ids, and
// the gathers of chunk c+1's inputs whose drivers are final (earlier chunks).  Inputs
// produced by chunk c itself are handed to chunk c+1 through LDS.  The compute phase
// reads LDS only.
struct FwdLds {
    int ax, tab, meta, nd, ni, src, in_at, in_sl, flag, gj, gty, f0, f1, taoff, tgoff, tmaxk, total;
};

__host__ __device__ inline FwdLds fwd_lds(int n_tables) {
    FwdLds o{};
    o.ax = 0;
    o.tab = 32;
    o.meta = o.tab + n_tables * 98;
    o.nd = o.meta + kFwdCapA;
    o.ni = o.nd + kFwdCapA;
    o.src = o.ni + kFwdCapA;
    o.in_at = o.src + kFwdCapA;
    o.in_sl = o.in_at + kFwdCapA;
    o.flag = o.in_sl + kFwdCapA;                  // bytes
    o.gj = o.flag + kFwdCapA / 4;
    o.gty = o.gj + kFwdCapG;
    o.f0 = ((o.gty + kFwdCapG) + 1) & ~1;         // float2, 8-byte aligned
    o.f1 = o.f0 + 2 * kFwdCapG;
    o.taoff = o.f1 + 2 * kFwdCapG;
    o.tgoff = o.taoff + kFwdCapT + 1;
    o.tmaxk = o.tgoff + kFwdCapT;
    o.total = o.tmaxk + kFwdCapT;
    return o;
}

constexpr int kFwdRA = (kFwdCapA + kViewThreads - 1) / kViewThreads;   // arcs per lane when staging
constexpr int kFwdRG = (kFwdCapG + kViewThreads - 1) / kViewThreads;   // gates per lane when staging
constexpr int kFwdRT = (kFwdCapT + kViewWaves - 1) / kViewWaves;       // tiles per wave

// One view of one graph, walked by the whole workgroup (every thread must call it).
__device__ __forceinline__ void fwd_view_unit(const DevGraph& G, const KLib& lib, const KViews& V, int NV, int NC,
                                              int v, const float* __restrict__ pi_ts, const float* __restrict__ load,
                                              const float* __restrict__ nd, const float* __restrict__ ni,
                                              float* __restrict__ drv_ts, float* __restrict__ arc_ts,
                                              float* __restrict__ arc_delay, uint8_t* __restrict__ argmax,
                                              float* s_mem) {
    const FwdLds lo = fwd_lds(lib.n_tables);
    float* s_ax = s_mem + lo.ax;
    float* s_tab = s_mem + lo.tab;
    uint32_t* s_meta = reinterpret_cast<uint32_t*>(s_mem + lo.meta);
    float* s_nd = s_mem + lo.nd;
    float* s_ni = s_mem + lo.ni;
    int* s_src = reinterpret_cast<int*>(s_mem + lo.src);
    float* s_in_at = s_mem + lo.in_at;
    float* s_in_sl = s_mem + lo.in_sl;
    uint8_t* s_flag = reinterpret_cast<uint8_t*>(s_mem + lo.flag);
    int* s_gj = reinterpret_cast<int*>(s_mem + lo.gj);
    float* s_gty = s_mem + lo.gty;
    // the two fresh-output buffers are addressed by offset from the LDS base (an array
    // of pointers would lose the LDS address space and turn the accesses into flat ones)
    float2* s_f0 = reinterpret_cast<float2*>(s_mem + lo.f0);
    int* s_taoff = reinterpret_cast<int*>(s_mem + lo.taoff);
    int* s_tgoff = reinterpret_cast<int*>(s_mem + lo.tgoff);
    int* s_tmaxk = reinterpret_cast<int*>(s_mem + lo.tmaxk);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const float* gtab = lib.tables + size_t(V.set[v]) * lib.n_tables * 98;
    const int* CH = G.fwd_chunk;
    load_axes(s_ax, lib);
    for (int i = tid; i < lib.n_tables * 98; i += kViewThreads) s_tab[i] = gtab[i];
    for (int i = tid; i < G.n_pi; i += kViewThreads)
        reinterpret_cast<float2*>(drv_ts)[size_t(i) * NV + v] = reinterpret_cast<const float2*>(pi_ts)[size_t(i) * NV + v];
    const bool early[1] = {V.mode[v] == STA_EARLY};
    const float* tab[1] = {s_tab};
    __syncthreads();

    // staging registers
    uint32_t p_meta[kFwdRA];
    float p_nd[kFwdRA], p_ni[kFwdRA], p_ld[kFwdRG];
    int p_src2[kFwdRA];
    float p_at[kFwdRA], p_sl[kFwdRA];
    bool p_fresh[kFwdRA];
    int p_ta = 0, p_tg = 0, p_tk = 0;

    // static records of chunk c (arc records, gate loads, tile bounds) into registers
    auto fetch_static = [&](int c) {
        const int t0 = CH[c * 4], t1 = CH[c * 4 + 4];
        const int al = CH[c * 4 + 1], ah = CH[c * 4 + 5];
        const int gl = CH[c * 4 + 2], gh = CH[c * 4 + 6];
        // loads are unconditional, from clamped (always valid) indices, so that no
        // branch forces an early wait for them; the values are selected afterwards
#pragma unroll
        for (int k = 0; k < kFwdRA; ++k) {
            const int i = tid + k * kViewThreads;
            const int ia = (i < ah - al) ? al + i : 0;
            p_meta[k] = G.arc_meta[ia];
            p_nd[k] = nd[ia];
            p_ni[k] = ni[ia];
        }
#pragma unroll
        for (int k = 0; k < kFwdRG; ++k) {
            const int i = tid + k * kViewThreads;
            p_ld[k] = load[(i < gh - gl) ? G.n_pi + gl + i : 0];
        }
        p_ta = G.ftile_arc[(tid <= t1 - t0) ? t0 + tid : 0] - al;
        const int it = (tid < t1 - t0) ? t0 + tid : 0;
        p_tg = G.ftile_gate[it] - gl;
        p_tk = G.ftile_maxk[it];
    };
    auto stash_static = [&](int c) {
        const int t0 = CH[c * 4], t1 = CH[c * 4 + 4];
        const int al = CH[c * 4 + 1], ah = CH[c * 4 + 5];
        const int gl = CH[c * 4 + 2], gh = CH[c * 4 + 6];
#pragma unroll
        for (int k = 0; k < kFwdRA; ++k) {
            const int i = tid + k * kViewThreads;
            if (i < ah - al) { s_meta[i] = p_meta[k]; s_nd[i] = p_nd[k]; s_ni[i] = p_ni[k]; }
        }
#pragma unroll
        for (int k = 0; k < kFwdRG; ++k) {
            const int i = tid + k * kViewThreads;
            if (i < gh - gl) {
                int j;
                float ty;
                gate_jty(s_ax, p_ld[k], j, ty);
                s_gj[i] = j;
                s_gty[i] = ty;
            }
        }
        if (tid <= t1 - t0) s_taoff[tid] = p_ta;
        if (tid < t1 - t0) { s_tgoff[tid] = p_tg; s_tmaxk[tid] = p_tk; }
    };
    // driver ids of chunk c
    auto fetch_src = [&](int c) {
        const int al = CH[c * 4 + 1], ah = CH[c * 4 + 5];
#pragma unroll
        for (int k = 0; k < kFwdRA; ++k) {
            const int i = tid + k * kViewThreads;
            p_src2[k] = G.arc_src[(i < ah - al) ? al + i : 0];
        }
    };
    auto stash_src = [&](int c) {
        const int al = CH[c * 4 + 1], ah = CH[c * 4 + 5];
#pragma unroll
        for (int k = 0; k < kFwdRA; ++k) {
            const int i = tid + k * kViewThreads;
            if (i < ah - al) s_src[i] = p_src2[k];
        }
    };
    // inputs of chunk c (driver ids in s_src): gathered when the driver is below
    // `done` (final), else an index into the outputs of the gates from `fresh_base`
    auto fetch_inputs = [&](int c, int done, int fresh_base) {
        const int al = CH[c * 4 + 1], ah = CH[c * 4 + 5];
#pragma unroll
        for (int k = 0; k < kFwdRA; ++k) {
            const int i = tid + k * kViewThreads;
            const int u = (i < ah - al) ? s_src[i] : 0;
            p_fresh[k] = u >= done;
            const int ug = p_fresh[k] ? 0 : u;       // driver 0 stands in for fresh inputs
            const float2 tsv = reinterpret_cast<const float2*>(drv_ts)[size_t(ug) * NV + v];
            p_at[k] = p_fresh[k] ? __int_as_float(u - fresh_base) : tsv.x;
            p_sl[k] = tsv.y;
        }
    };
    auto stash_inputs = [&](int c) {
        const int al = CH[c * 4 + 1], ah = CH[c * 4 + 5];
#pragma unroll
        for (int k = 0; k < kFwdRA; ++k) {
            const int i = tid + k * kViewThreads;
            if (i < ah - al) { s_in_at[i] = p_at[k]; s_in_sl[i] = p_sl[k]; s_flag[i] = p_fresh[k] ? 1 : 0; }
        }
    };

    if (NC > 0) {
        // prologue: chunk 0 (its drivers are primary inputs, final) and chunk 1's driver ids
        fetch_static(0);
        fetch_src(0);
        stash_static(0);
        stash_src(0);
        __syncthreads();
        fetch_inputs(0, G.n_drivers, 0);
        if (NC > 1) fetch_src(1);
        __syncthreads();
        stash_inputs(0);
        if (NC > 1) stash_src(1);
        __syncthreads();
    }

    for (int c = 0; c < NC; ++c) {
        const int t0 = CH[c * 4], T = CH[c * 4 + 4] - t0;
        const int al = CH[c * 4 + 1], gl = CH[c * 4 + 2];
        const int gdone = G.n_pi + gl;          // drivers below are final once chunk c is done... minus chunk c
        // 1. issue the next chunks' global loads
        if (c + 1 < NC) {
            fetch_static(c + 1);
            fetch_inputs(c + 1, gdone, gdone);
        }
        if (c + 2 < NC) fetch_src(c + 2);
        // 2. compute chunk c from LDS
        const float2* fresh_in = s_f0 + ((c + 1) & 1) * kFwdCapG;
        float2* fresh_out = s_f0 + (c & 1) * kFwdCapG;
        for (int r = 0; r < kFwdRT; ++r) {
            const int tl = wave + r * kViewWaves;
            if (tl >= T) break;                 // uniform per wave
            const int a_off = s_taoff[tl];
            const int n = s_taoff[tl + 1] - a_off;
            const int g_off = s_tgoff[tl];
            const int span = s_tmaxk[tl];
            const bool act = lane < n;
            const int ai = a_off + lane;
            FwdLane x;
            const uint32_t meta = act ? s_meta[ai] : 0u;
            fwd_lane_setup(x, act, meta, n, lane);
            x.a = al + ai;
            x.g = gl + g_off + x.gi;
            x.nd = act ? s_nd[ai] : 0.0f;
            x.ni = act ? s_ni[ai] : 0.0f;
            x.Lo = 0.0f;
            const int gidx = g_off + x.gi;
            const int j = act ? s_gj[gidx] : 0;
            const float ty = act ? s_gty[gidx] : 0.0f;
            float2 ts[1];
            if (act) {
                const float a_in = s_in_at[ai];
                ts[0] = s_flag[ai] ? fresh_in[__float_as_int(a_in)] : make_float2(a_in, s_in_sl[ai]);
            } else {
                ts[0] = make_float2(0.0f, 0.0f);
            }
            fwd_finish<1>(x, ts, j, ty, span, s_ax, tab, early, NV, v, G.n_pi, drv_ts, arc_ts, arc_delay, argmax,
                          fresh_out, gl);
        }
        __syncthreads();
        // 3. stage chunk c+1 (and chunk c+2's driver ids)
        if (c + 1 < NC) {
            stash_static(c + 1);
            stash_inputs(c + 1);
        }
        if (c + 2 < NC) stash_src(c + 2);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kViewThreads) void k_forward_view(DevGraph G, KLib lib, KViews V, int NV, int NC,
                                                               const float* __restrict__ pi_ts,
                                                               const float* __restrict__ load,
                                                               const float* __restrict__ nd,
                                                               const float* __restrict__ ni,
                                                               float* __restrict__ drv_ts, float* __restrict__ arc_ts,
                                                               float* __restrict__ arc_delay,
                                                               uint8_t* __restrict__ argmax) {
    extern __shared__ float s_mem[];
    fwd_view_unit(G, lib, V, NV, NC, blockIdx.x, pi_ts, load, nd, ni, drv_ts, arc_ts, arc_delay, argmax, s_mem);
}

// Many graphs and views in one launch: each workgroup claims (graph, view) units from a
// device counter, largest first (the host orders them), until none is left.
__global__ __launch_bounds__(kViewThreads) void k_forward_batch(const BatchItem* __restrict__ items,
                                                                const int2* __restrict__ units, int n_units,
                                                                int* __restrict__ counter, KLib lib, KViews V) {
    extern __shared__ float s_mem[];
    __shared__ int s_u;
    for (;;) {
        if (threadIdx.x == 0) s_u = atomicAdd(counter, 1);
        __syncthreads();
        const int u = s_u;
        __syncthreads();
        if (u >= n_units) break;
        const int2 w = units[u];
        const BatchItem it = items[w.x];
        fwd_view_unit(it.G, lib, V, it.NV, it.NC, w.y, it.pi_ts, it.load, it.nd, it.ni, it.drv_ts, it.arc_ts,
                      it.arc_delay, it.argmax, s_mem);
        __syncthreads();
    }
}

__global__ void k_zero_i32(int* p) { if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0; }

// k_backward_view: chunks of whole backward tiles of one driver level, in processing
// order (levels L..0).  While chunk c computes, the workgroup gathers chunk c+1's
// forward results (arc delay, input arrival, net delay, driver arrival) and the
// required times of the gate outputs its sinks feed when those are final, and loads
// chunk c+2's slot ids.  Required times produced by chunk c reach chunk c+1 through LDS.
struct BwdLds {
    int sa_n, so_n, sa, d, ati, ndv, rat, flag, at, f0, f1, tsoff, tdoff, lim, mn, total;
};

__host__ __device__ inline BwdLds bwd_lds() {
    BwdLds o{};
    o.sa_n = 0;
    o.so_n = o.sa_n + kBwdCapS;
    o.sa = o.so_n + kBwdCapS;
    o.d = o.sa + kBwdCapS;
    o.ati = o.d + kBwdCapS;
    o.ndv = o.ati + kBwdCapS;
    o.rat = o.ndv + kBwdCapS;
    o.flag = o.rat + kBwdCapS;                    // bytes
    o.at = o.flag + kBwdCapS / 4;
    o.f0 = o.at + kBwdCapD;
    o.f1 = o.f0 + kBwdCapD;
    o.tsoff = o.f1 + kBwdCapD;
    o.tdoff = o.tsoff + kBwdCapT + 1;
    o.lim = ((o.tdoff + kBwdCapT) + 1) & ~1;      // 8-byte aligned digits
    o.mn = o.lim + 2 * kLimbs;
    o.total = o.mn + kViewWaves;
    return o;
}

constexpr int kBwdRS = (kBwdCapS + kViewThreads - 1) / kViewThreads;
constexpr int kBwdRD = (kBwdCapD + kViewThreads - 1) / kViewThreads;
constexpr int kBwdRT = (kBwdCapT + kViewWaves - 1) / kViewWaves;
constexpr uint8_t kFlagHead = 1, kFlagFresh = 2, kFlagEndpoint = 4;

__global__ __launch_bounds__(kViewThreads) void k_backward_view(DevGraph G, KViews V, int NV, int NC, int E,
                                                                const float* __restrict__ nd,
                                                                const float* __restrict__ drv_ts,
                                                                const float* __restrict__ arc_ts,
                                                                const float* __restrict__ arc_delay,
                                                                const float* __restrict__ ep_rat,
                                                                float* __restrict__ drv_rat,
                                                                float* __restrict__ arc_rat,
                                                                float* __restrict__ drv_slack,
                                                                float* __restrict__ arc_slack,
                                                                double* __restrict__ tns, float* __restrict__ wns) {
    extern __shared__ float s_mem[];
    const BwdLds lo = bwd_lds();
    int* s_sa_n = reinterpret_cast<int*>(s_mem + lo.sa_n);
    int* s_so_n = reinterpret_cast<int*>(s_mem + lo.so_n);
    int* s_sa = reinterpret_cast<int*>(s_mem + lo.sa);
    float* s_d = s_mem + lo.d;
    float* s_ati = s_mem + lo.ati;
    float* s_ndv = s_mem + lo.ndv;
    float* s_rat = s_mem + lo.rat;
    uint8_t* s_flag = reinterpret_cast<uint8_t*>(s_mem + lo.flag);
    float* s_at = s_mem + lo.at;
    float* s_f0 = s_mem + lo.f0;                   // two buffers of kBwdCapD, by parity
    int* s_tsoff = reinterpret_cast<int*>(s_mem + lo.tsoff);
    int* s_tdoff = reinterpret_cast<int*>(s_mem + lo.tdoff);
    unsigned long long* s_l = reinterpret_cast<unsigned long long*>(s_mem + lo.lim);
    float* s_min = s_mem + lo.mn;
    const int v = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool early = V.mode[v] == STA_EARLY;
    const int* CH = G.bwd_chunk;
    if (tid < kLimbs) s_l[tid] = 0ull;
    __syncthreads();

    int q_sa[kBwdRS], q_so[kBwdRS];
    int p_sa[kBwdRS];
    float p_d[kBwdRS], p_ati[kBwdRS], p_nd[kBwdRS], p_rat[kBwdRS], p_at[kBwdRD];
    uint8_t p_fl[kBwdRS];
    int p_ts = 0, p_td = 0;

    auto fetch_ids = [&](int c) {
        const int s0 = CH[c * 8 + 2], s1 = CH[c * 8 + 3];
#pragma unroll
        for (int k = 0; k < kBwdRS; ++k) {
            const int i = tid + k * kViewThreads;
            const bool ok = i < s1 - s0;
            const int is = ok ? s0 + i : 0;
            const int a = G.bslot_arc[is];
            const int o = G.bslot_out[is];
            q_sa[k] = ok ? a : -1;
            q_so[k] = ok ? o : 0;
        }
    };
    auto stash_ids = [&](int c) {
        const int s0 = CH[c * 8 + 2], s1 = CH[c * 8 + 3];
#pragma unroll
        for (int k = 0; k < kBwdRS; ++k) {
            const int i = tid + k * kViewThreads;
            if (i < s1 - s0) { s_sa_n[i] = q_sa[k]; s_so_n[i] = q_so[k]; }
        }
    };
    // chunk c's gathers (slot ids in s_sa_n/s_so_n); required times of the drivers in
    // [fr_lo, fr_hi) are not final yet and are taken from LDS later
    auto fetch_data = [&](int c, int fr_lo, int fr_hi) {
        const int t0 = CH[c * 8], t1 = CH[c * 8 + 1];
        const int s0 = CH[c * 8 + 2], s1 = CH[c * 8 + 3];
        const int d0 = CH[c * 8 + 4], d1 = CH[c * 8 + 5];
#pragma unroll
        for (int k = 0; k < kBwdRS; ++k) {
            const int i = tid + k * kViewThreads;
            const bool ok = i < s1 - s0;
            const int sa = ok ? s_sa_n[i] : -1;
            const int raw = ok ? s_so_n[i] : 0;
            const int so = raw & 0x7fffffff;
            // unconditional loads from clamped indices (no branch forces an early wait)
            const bool arc = ok && sa >= 0;
            const bool fresh = arc && so >= fr_lo && so < fr_hi;
            const bool endp = ok && sa < 0;
            const int sa_c = arc ? sa : 0;
            const int so_r = (arc && !fresh) ? so : 0;
            const int so_e = endp ? so : 0;
            const float d = arc_delay[size_t(sa_c) * NV + v];
            const float ati = arc_ts[(size_t(sa_c) * NV + v) * 2];
            const float ndv = nd[sa_c];
            const float r_old = drv_rat[size_t(so_r) * NV + v];
            const float r_ep = (E > 0) ? ep_rat[size_t(so_e) * NV + v] : 0.0f;
            uint8_t fl = (uint32_t(raw) & kHeadBit) ? kFlagHead : 0;
            if (fresh) fl |= kFlagFresh;
            if (endp) fl |= kFlagEndpoint;
            const float rat = endp ? r_ep : (fresh ? __int_as_float(so - fr_lo) : r_old);
            p_sa[k] = sa;
            p_d[k] = d;
            p_ati[k] = ati;
            p_nd[k] = ndv;
            p_rat[k] = rat;
            p_fl[k] = fl;
        }
#pragma unroll
        for (int k = 0; k < kBwdRD; ++k) {
            const int i = tid + k * kViewThreads;
            p_at[k] = drv_ts[(size_t((i < d1 - d0) ? d0 + i : 0) * NV + v) * 2];
        }
        p_ts = G.btile_slot[(tid <= t1 - t0) ? t0 + tid : 0] - s0;
        p_td = G.btile_drv[(tid < t1 - t0) ? t0 + tid : 0] - d0;
    };
    auto stash_data = [&](int c) {
        const int t0 = CH[c * 8], t1 = CH[c * 8 + 1];
        const int s0 = CH[c * 8 + 2], s1 = CH[c * 8 + 3];
        const int d0 = CH[c * 8 + 4], d1 = CH[c * 8 + 5];
#pragma unroll
        for (int k = 0; k < kBwdRS; ++k) {
            const int i = tid + k * kViewThreads;
            if (i < s1 - s0) {
                s_sa[i] = p_sa[k];
                s_d[i] = p_d[k];
                s_ati[i] = p_ati[k];
                s_ndv[i] = p_nd[k];
                s_rat[i] = p_rat[k];
                s_flag[i] = p_fl[k];
            }
        }
#pragma unroll
        for (int k = 0; k < kBwdRD; ++k) {
            const int i = tid + k * kViewThreads;
            if (i < d1 - d0) s_at[i] = p_at[k];
        }
        if (tid <= t1 - t0) s_tsoff[tid] = p_ts;
        if (tid < t1 - t0) s_tdoff[tid] = p_td;
    };

    if (NC > 0) {
        fetch_ids(0);
        stash_ids(0);
        __syncthreads();
        fetch_data(0, 0, 0);
        if (NC > 1) fetch_ids(1);
        __syncthreads();
        stash_data(0);
        if (NC > 1) stash_ids(1);
        __syncthreads();
    }

    for (int c = 0; c < NC; ++c) {
        const int T = CH[c * 8 + 1] - CH[c * 8];
        const int d0 = CH[c * 8 + 4], d1 = CH[c * 8 + 5];
        if (c + 1 < NC) fetch_data(c + 1, d0, d1);
        if (c + 2 < NC) fetch_ids(c + 2);
        const float* f_in = s_f0 + ((c + 1) & 1) * kBwdCapD;
        float* f_out = s_f0 + (c & 1) * kBwdCapD;
        for (int r = 0; r < kBwdRT; ++r) {
            const int tl = wave + r * kViewWaves;
            if (tl >= T) break;                   // uniform per wave
            const int s_off = s_tsoff[tl];
            const int n = s_tsoff[tl + 1] - s_off;
            const int d_off = s_tdoff[tl];
            // n <= 64, or one driver owning every slot: lanes take contiguous runs
            const int cs = (n + 63) >> 6;
            const int sb = lane * cs, se = min(n, sb + cs);
            float best = 0.0f;
            bool have = false;
            for (int q = sb; q < se; ++q) {
                const int i = s_off + q;
                const uint8_t fl = s_flag[i];
                float val;
                if (fl & kFlagEndpoint) {
                    val = s_rat[i];
                } else {
                    const float ro = (fl & kFlagFresh) ? f_in[__float_as_int(s_rat[i])] : s_rat[i];
                    const float rin = ro - s_d[i];
                    const float ati = s_ati[i];
                    const int sa = s_sa[i];
                    arc_rat[size_t(sa) * NV + v] = rin;
                    arc_slack[size_t(sa) * NV + v] = early ? (ati - rin) : (rin - ati);
                    val = rin - s_ndv[i];
                }
                if (!have || (early ? (val > best) : (val < best))) best = val;
                have = true;
            }
            const bool head = (cs > 1) ? (lane == 0) : (sb < n && (s_flag[s_off + sb] & kFlagHead) != 0);
            const uint64_t heads = __ballot(head);
            const uint64_t le = lanes_le(lane);
            const int gi = __popcll(heads & le) - 1;
            const uint64_t after = heads & ~le;
            const int nl = (n + cs - 1) / cs;
            const int seg_end = after ? (__ffsll(static_cast<unsigned long long>(after)) - 1) : nl;
            for (int off = 1; off < 64; off <<= 1) {
                const float b2 = __shfl_down(best, off, 64);
                if ((lane + off) < seg_end && (early ? (b2 > best) : (b2 < best))) best = b2;
            }
            if (head) {
                const int dl = d_off + gi;
                const int u = d0 + dl;
                const float at = s_at[dl];
                drv_rat[size_t(u) * NV + v] = best;
                drv_slack[size_t(u) * NV + v] = early ? (at - best) : (best - at);
                f_out[dl] = best;
            }
        }
        __syncthreads();
        if (c + 1 < NC) stash_data(c + 1);
        if (c + 2 < NC) stash_ids(c + 2);
        __syncthreads();
    }
    // endpoint summaries of this view
    unsigned long long lim[kLimbs];
#pragma unroll
    for (int i = 0; i < kLimbs; ++i) lim[i] = 0ull;
    float mn = __builtin_inff();
    for (int e = tid; e < E; e += kViewThreads) {
        const float sl = drv_slack[size_t(G.ep_drv[e]) * NV + v];
        mn = (sl < mn) ? sl : mn;
        add_neg_slack(lim, sl);
    }
#pragma unroll
    for (int i = 0; i < kLimbs; ++i)
        if (lim[i]) atomicAdd(&s_l[i], lim[i]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float o2 = __shfl_xor(mn, off, 64);
        mn = (o2 < mn) ? o2 : mn;
    }
    if (lane == 0) s_min[wave] = mn;
    __syncthreads();
    if (tid == 0) {
        const double mag = digits_to_double(s_l);
        tns[v] = (mag == 0.0) ? 0.0 : -mag;
        float m = s_min[0];
        for (int i = 1; i < kViewWaves; ++i) m = (s_min[i] < m) ? s_min[i] : m;
        wns[v] = m;
    }
}

// ---------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------

static thread_local Prof g_prof;
Prof& prof() { return g_prof; }

sta_status launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(STA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return STA_OK;
}

template <typename T, int MAXN, int NT>
static void launch_dc(const sta_graph* g, const sta_net_out* out, hipStream_t s) {
    const int blocks = dc_blocks_of(g->D, g->n_dc_wide, MAXN, NT);
    prof_launch("k_delay_calc", s, [&] {
        if constexpr (MAXN == 8) {
            if (g->chain_nets)
                hipLaunchKernelGGL((k_delay_calc8<T, true>), dim3(blocks), dim3(NT), 0, s, dev_graph(g), out->load,
                                   out->net_delay, out->net_imp2, out->arc_load);
            else
                hipLaunchKernelGGL((k_delay_calc8<T, false>), dim3(blocks), dim3(NT), 0, s, dev_graph(g), out->load,
                                   out->net_delay, out->net_imp2, out->arc_load);
        } else {
            hipLaunchKernelGGL((k_delay_calc<T, MAXN, NT>), dim3(blocks), dim3(NT), 0, s, dev_graph(g), out->load,
                               out->net_delay, out->net_imp2, out->arc_load);
        }
    });
}

template <typename T>
static void dispatch_dc(const sta_graph* g, const sta_net_out* out, hipStream_t s) {
    // nets of <= 8 nodes: registers only; larger: node temporaries in LDS, 2 * MAXN * NT
    // values of T per block (32 KB for FP64)
    const int m = g->max_net_nodes;
    if (m <= 8) launch_dc<T, 8, 256>(g, out, s);
    else if (m <= 16) launch_dc<T, 16, 128>(g, out, s);
    else if (m <= 32) launch_dc<T, 32, 64>(g, out, s);
    else if (m <= 64) launch_dc<T, 64, 32>(g, out, s);
    else if (m <= 128) launch_dc<T, 128, 16>(g, out, s);
    else launch_dc<T, 256, 8>(g, out, s);
}

static bool views_ok(const sta_views* v, int n_sets, std::string& why) {
    if (!v) { why = "null views"; return false; }
    if (!(v->n_views == 1 || v->n_views == 2 || v->n_views == 4 || v->n_views == 8)) {
        why = "n_views must be 1, 2, 4 or 8";
        return false;
    }
    for (int i = 0; i < v->n_views; ++i) {
        if (v->mode[i] != STA_LATE && v->mode[i] != STA_EARLY) { why = "bad mode"; return false; }
        if (n_sets >= 0 && (v->table_set[i] < 0 || v->table_set[i] >= n_sets)) { why = "table_set out of range"; return false; }
    }
    return true;
}

static KViews kviews(const sta_views* v) {
    KViews k{};
    for (int i = 0; i < STA_MAX_VIEWS; ++i) {
        k.mode[i] = i < v->n_views ? v->mode[i] : 0;
        k.set[i] = i < v->n_views ? v->table_set[i] : 0;
    }
    return k;
}

static size_t lds_limit() {
    static size_t lim = 0;
    if (!lim) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && v > 0)
            lim = size_t(v);
        else
            lim = 65536;
    }
    return lim;
}

// The view schedule runs while one compute unit finishes an average level faster than
// a device-wide step does (a few thousand cell arcs per level) and the level's staged
// data and the view's tables fit in LDS.  Left to the library (the default), the fused
// spans are taken instead: measured faster at every size and view count (10k pins, two
// views: 0.15 vs 0.30 ms per step; four views: propagate 0.07 vs 0.13 ms).
static bool view_auto_off(const sta_graph* g, int n_views) { return g->view_auto && n_views <= kSpanMaxViews && g->use_spans; }

static bool use_view_forward(const sta_graph* g, int n_tables, int n_views, size_t* lds) {
    if (view_auto_off(g, n_views)) return false;
    if (g->L == 0 || g->n_fchunks == 0 || double(g->A) / double(g->L) > double(g->view_sched_max_arcs)) return false;
    *lds = size_t(fwd_lds(n_tables).total) * 4;
    return *lds <= lds_limit();
}

static bool use_view_backward(const sta_graph* g, int n_views, size_t* lds) {
    if (view_auto_off(g, n_views)) return false;
    if (g->L == 0 || g->n_bchunks == 0 || double(g->A) / double(g->L) > double(g->view_sched_max_arcs)) return false;
    *lds = size_t(bwd_lds().total) * 4;
    return *lds <= lds_limit();
}

template <typename K>
static void set_lds(K kernel, size_t lds) {
    if (lds > 65536) hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
}

static KTiles ktiles(const std::vector<int32_t>& first, const std::vector<int32_t>& base, int t0, int t1) {
    KTiles k;
    std::memset(&k, 0, sizeof(k));
    k.inl = (t1 - t0) <= kArgTiles ? 1 : 0;
    if (k.inl) {
        for (int t = t0; t <= t1; ++t) k.first[t - t0] = first[t];
        for (int t = t0; t < t1; ++t) k.base[t - t0] = base[t];
    }
    return k;
}

// Runs enqueue(stream) directly, or replays it from the cached hipGraph of this call
// kind and key (capturing it first when no cached entry has the key; the least recently
// used entry makes room, after the device has drained).  Profiling always runs it directly.
void drop_launches(LaunchCache& c) {
    if (c.e.empty()) return;
    (void)hipDeviceSynchronize();
    for (LaunchEntry& x : c.e) {
        if (x.exec) (void)hipGraphExecDestroy(x.exec);
        if (x.graph) (void)hipGraphDestroy(x.graph);
    }
    c.e.clear();
}

template <typename F>
static sta_status capture_replay(LaunchCache& c, std::mutex& mu, bool use_graphs, std::vector<uint64_t> key,
                                 hipStream_t s, F&& enqueue) {
    if (!use_graphs || g_prof.on) {
        enqueue(s);
        return STA_OK;
    }
    std::lock_guard<std::mutex> lock(mu);
    LaunchEntry* hit = nullptr;
    for (LaunchEntry& x : c.e)
        if (x.key == key) hit = &x;
    if (!hit) {
        hipStream_t cap = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(STA_E_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return fail(STA_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        }
        enqueue(cap);
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(cap, &gr);
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) return fail(STA_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(gr);
            return fail(STA_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        if (int(c.e.size()) >= kLaunchCacheEntries) {
            size_t lru = 0;
            for (size_t i = 1; i < c.e.size(); ++i)
                if (c.e[i].used < c.e[lru].used) lru = i;
            // the evicted exec may still be running on another stream
            (void)hipDeviceSynchronize();
            (void)hipGraphExecDestroy(c.e[lru].exec);
            (void)hipGraphDestroy(c.e[lru].graph);
            c.e.erase(c.e.begin() + std::ptrdiff_t(lru));
        }
        c.e.push_back(LaunchEntry{std::move(key), gr, ex, 0});
        hit = &c.e.back();
    }
    hit->used = ++c.tick;
    hipError_t e = hipGraphLaunch(hit->exec, s);
    if (e != hipSuccess) return fail(STA_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return STA_OK;
}

template <typename F>
static sta_status run_sequence(const sta_graph* g, LaunchCache& c, std::vector<uint64_t> key, hipStream_t s,
                               F&& enqueue) {
    return capture_replay(c, g->cache_mu, g->use_graphs, std::move(key), s, std::forward<F>(enqueue));
}

static uint64_t pk(const void* p) { return uint64_t(reinterpret_cast<uintptr_t>(p)); }

// one level launch of the forward pass (gate level l of g, all views)
template <int NV>
static void launch_forward_level(const sta_graph* g, const KLib& lib, const KViews& kv, const sta_net_out* nd,
                                 const sta_timing_out* o, int64_t l, hipStream_t s) {
    const int t0 = g->fwd_tile_ptr[l], t1 = g->fwd_tile_ptr[l + 1];
    if (t1 <= t0) return;
    const KTiles kt = ktiles(g->ftile_arc_h, g->ftile_gate_h, t0, t1);
    const DevGraph dg = dev_graph(g);
    prof_launch("k_forward", s, [&] {
        hipLaunchKernelGGL((k_forward<NV>), dim3((t1 - t0 + kLevelWaves - 1) / kLevelWaves), dim3(64 * kLevelWaves),
                           0, s, dg, lib, kv, t0, t1, kt, nd->arc_load, nd->net_delay, nd->net_imp2, o->drv_ts,
                           o->arc_ts, o->arc_delay, o->argmax);
    });
}

template <int NV>
static void enqueue_forward_levels(const sta_graph* g, const KLib& lib, const KViews& kv, const float* pi_ts,
                                   const sta_net_out* nd, const sta_timing_out* o, hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    const int npi = int(g->n_pi) * NV * 2;
    // the primary inputs' copy rides on the first span launch when that span is fused and
    // its lanes cover the copy (one element per lane), else it is a launch of its own
    constexpr int NWf = kSpanViewsPerWave < NV ? kSpanViewsPerWave : NV;
    bool copy_in_first = false;
    if constexpr (NV <= kSpanMaxViews)
        copy_in_first = npi > 0 && g->use_spans && !g->span_fused_h.empty() && g->span_fused_h[0] &&
                        int64_t(g->span_tile_h[1] - g->span_tile_h[0]) * (NV / NWf) * 64 >= int64_t(g->n_pi) * NV;
    if (npi > 0 && !copy_in_first)
        prof_launch("k_copy_pi", s, [&] {
            hipLaunchKernelGGL(k_copy_pi, dim3((npi + 255) / 256), dim3(256), 0, s, pi_ts, o->drv_ts, npi);
        });
    auto level = [&](int64_t l) { launch_forward_level<NV>(g, lib, kv, nd, o, l, s); };
    if constexpr (NV <= kSpanMaxViews) {
        if (g->use_spans) {
            const int64_t NS = int64_t(g->span_fused_h.size());
            for (int64_t sp = 0; sp < NS; ++sp) {
                const int64_t l0 = g->span_lv_h[2 * sp], l1 = g->span_lv_h[2 * sp + 1];
                if (!g->span_fused_h[sp]) {
                    for (int64_t l = l0; l <= l1; ++l) level(l);
                    continue;
                }
                const int t0 = g->span_tile_h[sp], t1 = g->span_tile_h[sp + 1];
                if (t1 <= t0) continue;
                constexpr int NW = kSpanViewsPerWave < NV ? kSpanViewsPerWave : NV;
                // the next fused span's tiles, for the record prefetch of the spare workgroups;
                // a multiple of eight workgroups per view group
                int pf0 = 0, pf1 = 0;
                if (sp + 1 < NS && g->span_fused_h[sp + 1]) {
                    pf0 = g->span_tile_h[sp + 1];
                    pf1 = g->span_tile_h[sp + 2];
                }
                const dim3 grid(span_round8(t1 - t0) + span_pf_blocks(pf1 - pf0, kSpanPfTilesF), NV / NW);
                // drivers below pf_fin (those of lower levels) hold final arrivals
                const int pf_fin = (sp == 0 && copy_in_first) ? 0 :
                    int(std::lower_bound(g->level.begin(), g->level.end(), int32_t(l0)) - g->level.begin());
                prof_launch("k_forward_span", s, [&] {
                    if (sp == 0 && copy_in_first)
                        hipLaunchKernelGGL((k_forward_span<NV, NW, true>), grid, dim3(64 * kSpanWaves), 0, s, dg, lib,
                                           kv, t0, t1, nd->arc_load, nd->net_delay, nd->net_imp2, o->drv_ts,
                                           o->arc_ts, o->arc_delay, o->argmax, pf0, pf1, pi_ts, pf_fin);
                    else
                        hipLaunchKernelGGL((k_forward_span<NV, NW, false>), grid, dim3(64 * kSpanWaves), 0, s, dg, lib,
                                           kv, t0, t1, nd->arc_load, nd->net_delay, nd->net_imp2, o->drv_ts,
                                           o->arc_ts, o->arc_delay, o->argmax, pf0, pf1, pi_ts, pf_fin);
                });
            }
            return;
        }
    }
    for (int64_t l = 1; l <= g->L; ++l) level(l);
}

template <int NV>
static sta_status run_forward_levels(const sta_graph* g, const KLib& lib, const KViews& kv, const float* pi_ts,
                                     const sta_net_out* nd, const sta_timing_out* o, hipStream_t s) {
    std::vector<uint64_t> key = {pk(g->dev), uint64_t(NV), pk(lib.tables), uint64_t(lib.n_tables), pk(pi_ts), pk(nd->arc_load),
                                 pk(nd->net_delay), pk(nd->net_imp2), pk(o->drv_ts), pk(o->arc_ts), pk(o->arc_delay),
                                 pk(o->argmax), uint64_t(g->use_spans)};
    for (int i = 0; i < 26; ++i) { uint32_t b; std::memcpy(&b, &lib.ax[i], 4); key.push_back(b); }
    for (int v = 0; v < NV; ++v) key.push_back((uint64_t(kv.mode[v]) << 32) | uint32_t(kv.set[v]));
    return run_sequence(g, g->fwd_cache, std::move(key), s, [&](hipStream_t q) {
        enqueue_forward_levels<NV>(g, lib, kv, pi_ts, nd, o, q);
    });
}

static void run_forward_views(const sta_graph* g, size_t lds, int NV, const KLib& lib, const KViews& kv,
                              const float* pi_ts, const sta_net_out* nd, const sta_timing_out* o, hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    set_lds(k_forward_view, lds);
    prof_launch("k_forward_view", s, [&] {
        hipLaunchKernelGGL(k_forward_view, dim3(NV), dim3(kViewThreads), lds, s, dg, lib, kv, NV, g->n_fchunks, pi_ts,
                           nd->load, nd->net_delay, nd->net_imp2, o->drv_ts, o->arc_ts, o->arc_delay, o->argmax);
    });
}

// one level launch of the backward pass (driver level l of g, all views)
template <int NV>
static void launch_backward_level(const sta_graph* g, const KViews& kv, const float* net_delay, const float* drv_ts,
                                  const float* arc_ts, const float* arc_delay, const float* ep_rat, float* drv_rat,
                                  float* arc_rat, float* drv_slack, float* arc_slack, int64_t l, hipStream_t s) {
    const int t0 = g->bwd_tile_ptr[l], t1 = g->bwd_tile_ptr[l + 1];
    if (t1 <= t0) return;
    const KTiles kt = ktiles(g->btile_slot_h, g->btile_drv_h, t0, t1);
    const DevGraph dg = dev_graph(g);
    prof_launch("k_backward", s, [&] {
        hipLaunchKernelGGL((k_backward<NV>), dim3((t1 - t0 + kLevelWaves - 1) / kLevelWaves), dim3(64 * kLevelWaves),
                           0, s, dg, kv, t0, t1, kt, net_delay, drv_ts, arc_ts, arc_delay, ep_rat, drv_rat, arc_rat,
                           drv_slack, arc_slack);
    });
}

template <int NV>
static void enqueue_backward_levels(const sta_graph* g, const KViews& kv, const sta_net_out* nd,
                                    const sta_timing_out* t, const float* ep_rat, const sta_slack_out* o,
                                    void* scratch, hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    auto level = [&](int64_t l) {
        launch_backward_level<NV>(g, kv, nd->net_delay, t->drv_ts, t->arc_ts, t->arc_delay, ep_rat, o->drv_rat,
                                  o->arc_rat, o->drv_slack, o->arc_slack, l, s);
    };
    auto* limbs = static_cast<unsigned long long*>(scratch);
    auto* pw = reinterpret_cast<float*>(static_cast<uint8_t*>(scratch) + size_t(kK4Blocks) * STA_MAX_VIEWS * kLimbs * 8);
    bool done = false, folded = false;
    if constexpr (NV <= kSpanMaxViews) {
        if (g->use_spans) {
            const int64_t NSB = int64_t(g->bspan_fused_h.size());
            // with two span launches or more, the endpoint summary rides along: its partials
            // in the first launch's spare workgroups, its final sum in the second's
            int n_launch = 0;
            for (int64_t b = 0; b < NSB; ++b)
                n_launch += g->bspan_fused_h[b] && g->bspan_tile_h[b + 1] > g->bspan_tile_h[b];
            folded = n_launch >= 2;
            EpFold ep{t->drv_ts, ep_rat, limbs, pw, o->tns, o->wns, int(g->E), 1, 0};
            {
                int nb = int((g->E + 64 * kEpPerLane - 1) / (64 * kEpPerLane));
                ep.nblk = nb < 1 ? 1 : (nb > kK4Blocks ? kK4Blocks : nb);
            }
            int k = 0;
            for (int64_t b = 0; b < NSB; ++b) {
                const int64_t top = g->bspan_lv_h[2 * b], bot = g->bspan_lv_h[2 * b + 1];
                if (!g->bspan_fused_h[b]) {
                    for (int64_t l = top; l >= bot; --l) level(l);
                    continue;
                }
                const int t0 = g->bspan_tile_h[b], t1 = g->bspan_tile_h[b + 1];
                if (t1 <= t0) continue;
                ep.role = folded && k < 2 ? k + 1 : 0;
                const int ne = ep.role == 1 ? ep.nblk : ep.role == 2 ? 1 : 0;
                ++k;
                // the next launch's tiles (a fused span directly after this one), for the
                // prefetch of their records and gathers
                int pf0 = 0, pf1 = 0;
                if (b + 1 < NSB && g->bspan_fused_h[b + 1]) {
                    pf0 = g->bspan_tile_h[b + 1];
                    pf1 = g->bspan_tile_h[b + 2];
                }
                // spare workgroups: the endpoint summary's, then the prefetch's; a multiple
                // of eight workgroups per view group
                const int nx = span_round8(t1 - t0 + ne) + span_pf_blocks(pf1 - pf0, kSpanPfTilesB);
                prof_launch("k_backward_span", s, [&] {
                    hipLaunchKernelGGL((k_backward_span<NV, kBwdViewsPerWave < NV ? kBwdViewsPerWave : NV>),
                                       dim3(nx, NV / (kBwdViewsPerWave < NV ? kBwdViewsPerWave : NV)),
                                       dim3(64 * kSpanWaves), 0, s, dg, kv, t0,
                                       t1, nd->net_delay, t->drv_ts, t->arc_ts, t->arc_delay, ep_rat, o->drv_rat,
                                       o->arc_rat, o->drv_slack, o->arc_slack, ep, pf0, pf1);
                });
            }
            done = true;
        }
    }
    if (!done)
        for (int64_t l = g->L; l >= 0; --l) level(l);
    if (folded) return;
    int nblk = int((g->E + kK4Threads - 1) / kK4Threads);
    nblk = nblk < 1 ? 1 : (nblk > kK4Blocks ? kK4Blocks : nblk);
    prof_launch("k_endpoint_partial", s, [&] {
        hipLaunchKernelGGL((k_endpoint_partial<NV>), dim3(nblk), dim3(kK4Threads), 0, s, dg.ep_drv, int(g->E),
                           o->drv_slack, limbs, pw);
    });
    prof_launch("k_endpoint_final", s, [&] {
        hipLaunchKernelGGL((k_endpoint_final<NV>), dim3(1), dim3(256), 0, s, nblk, limbs, pw, o->tns, o->wns);
    });
}

template <int NV>
static sta_status run_backward_levels(const sta_graph* g, const KViews& kv, const sta_net_out* nd,
                                      const sta_timing_out* t, const float* ep_rat, const sta_slack_out* o,
                                      void* scratch, hipStream_t s) {
    std::vector<uint64_t> key = {pk(g->dev), uint64_t(NV), pk(nd->net_delay), pk(t->drv_ts), pk(t->arc_ts), pk(t->arc_delay),
                                 pk(ep_rat), pk(o->drv_rat), pk(o->arc_rat), pk(o->drv_slack), pk(o->arc_slack),
                                 pk(o->tns), pk(o->wns), pk(scratch), uint64_t(g->use_spans)};
    for (int v = 0; v < NV; ++v) key.push_back(uint64_t(kv.mode[v]));
    return run_sequence(g, g->bwd_cache, std::move(key), s, [&](hipStream_t q) {
        enqueue_backward_levels<NV>(g, kv, nd, t, ep_rat, o, scratch, q);
    });
}

static void run_backward_views(const sta_graph* g, size_t lds, int NV, const KViews& kv, const sta_net_out* nd,
                               const sta_timing_out* t, const float* ep_rat, const sta_slack_out* o, hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    set_lds(k_backward_view, lds);
    prof_launch("k_backward_view", s, [&] {
        hipLaunchKernelGGL(k_backward_view, dim3(NV), dim3(kViewThreads), lds, s, dg, kv, NV, g->n_bchunks, int(g->E),
                           nd->net_delay, t->drv_ts, t->arc_ts, t->arc_delay, ep_rat, o->drv_rat, o->arc_rat,
                           o->drv_slack, o->arc_slack, o->tns, o->wns);
    });
}


// ---------------------------------------------------------------------------------
// adjoint of TNS (argmax-routed) and the critical-path report
// ---------------------------------------------------------------------------------

// One backward tile of the adjoint: the gradient of TNS with respect to a driver's
// arrival is the sum over its sink pins of the gradient of the sink gate's output when
// that pin's cell arc is the gate's argmax, plus -1 (late) / +1 (early) for an endpoint
// with negative slack.  All values are integer counts, exact in FP32 in any order.
template <int NW>
__device__ __forceinline__ void adj_tile(const DevGraph& G, const bool* early, int NV, int v0, int s0, int n, int d0,
                                         const uint8_t* __restrict__ argmax, const float* __restrict__ drv_slack,
                                         float* __restrict__ g_at, float* __restrict__ g_arc,
                                         float* __restrict__ g_nd) {
    const int lane = threadIdx.x & 63;
    const int c = (n + 63) >> 6;
    const int sb = lane * c;
    const int se = min(n, sb + c);
    bool head;
    if (c > 1) head = (lane == 0);
    else head = (sb < n) && (uint32_t(G.bslot_out[s0 + sb]) & kHeadBit) != 0u;
    const uint64_t heads = __ballot(head);
    const uint64_t le = lanes_le(lane);
    const int gi = __popcll(heads & le) - 1;
    const uint64_t after = heads & ~le;
    const int nl = (n + c - 1) / c;
    const int seg_end = after ? (__ffsll(static_cast<unsigned long long>(after)) - 1) : nl;
    float acc[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) acc[w] = 0.0f;
    for (int s = sb; s < se; ++s) {
        const int slot = s0 + s;
        const int sa = G.bslot_arc[slot];
        const int so = G.bslot_out[slot] & 0x7fffffff;
        if (sa >= 0) {
            const int kpos = int(G.arc_meta[sa] >> 16);
            const int gq = so - G.n_pi;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const float cv = (int(argmax[size_t(gq) * NV + v0 + w]) == kpos) ? g_at[size_t(so) * NV + v0 + w] : 0.0f;
                if (g_arc) g_arc[size_t(sa) * NV + v0 + w] = cv;
                if (g_nd) g_nd[size_t(sa) * NV + v0 + w] = cv;
                acc[w] += cv;
            }
        } else {
            const int u = d0 + gi;      // an endpoint owns exactly one slot, so this lane heads it
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const float sl = drv_slack[size_t(u) * NV + v0 + w];
                acc[w] += sl < 0.0f ? (early[w] ? 1.0f : -1.0f) : 0.0f;
            }
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const bool take = (lane + off) < seg_end;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const float b2 = __shfl_down(acc[w], off, 64);
            if (take) acc[w] += b2;
        }
    }
    if (head) {
        const int u = d0 + gi;
#pragma unroll
        for (int w = 0; w < NW; ++w) g_at[size_t(u) * NV + v0 + w] = acc[w];
    }
}

template <int NV>
__global__ __launch_bounds__(64 * kLevelWaves) void k_adjoint(DevGraph G, KViews V, int tile0, int tile1, KTiles kt,
                                                 const uint8_t* __restrict__ argmax,
                                                 const float* __restrict__ drv_slack, float* __restrict__ g_at,
                                                 float* __restrict__ g_arc, float* __restrict__ g_nd) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = tile0 + blockIdx.x * kLevelWaves + wave;
    if (t >= tile1) return;
    bool early[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) early[v] = V.mode[v] == STA_EARLY;
    int s0, n, d0;
    if (kt.inl) {
        s0 = kt.first[t - tile0];
        n = kt.first[t - tile0 + 1] - s0;
        d0 = kt.base[t - tile0];
    } else {
        s0 = G.btile_slot[t];
        n = G.btile_slot[t + 1] - s0;
        d0 = G.btile_drv[t];
    }
    adj_tile<NV>(G, early, NV, 0, s0, n, d0, argmax, drv_slack, g_at, g_arc, g_nd);
}

// The adjoint on the backward span tiles: the same dependency structure as the required
// times (a driver's gradient needs the gradients of its sink gates' outputs), so one
// launch walks up to kSpanB driver levels top down with in-tile gradients in LDS.  Two
// rounds of loads: the tile's records, then per slot the argmax test's operands (the
// arc's position, the sink gate's argmax), the gradient of a sink gate outside the tile,
// or an endpoint's slack.  Integer counts, so the segmented sums are exact in any order
// and the results equal the level kernel's.
template <int NV, int NW>
__global__ __launch_bounds__(64 * kSpanWaves) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_adjoint_span(DevGraph G, KViews V, int tile0, int tile1,
                                                                  const uint8_t* __restrict__ argmax,
                                                                  const float* __restrict__ drv_slack,
                                                                  float* __restrict__ g_at, float* __restrict__ g_arc,
                                                                  float* __restrict__ g_nd, int pf0, int pf1) {
    __shared__ float s_g[kSpanWaves][kSpanSlotsB * NW];
    static_assert(kSpanWaves == 1, "one span tile per workgroup");
    const int v0 = int(blockIdx.y) * NW;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tb = tile1 - tile0;
    if (int(blockIdx.x) >= tb) {
        // spare workgroups (first view group): the next launch's tile records and the data
        // its slots gather that is final (arc metadata, argmax, driver slacks), into L2, as
        // the backward span launches do; out-of-tile gradients can still change
        const int q = int(blockIdx.x) - span_round8(tb);
        if (blockIdx.y == 0 && q >= 0 && pf1 > pf0) {
            const int rho = q & 7, kappa = q >> 3;
            const int ln = threadIdx.x & 63;
            uint32_t acc = 0;
#pragma unroll
            for (int i = 0; i < kSpanPfTilesB; ++i) {
                const int tt = pf0 + rho + 8 * (kappa * kSpanPfTilesB + i);
                if (tt >= pf1) break;           // uniform
                int4 r[kSpanB];
#pragma unroll
                for (int c = 0; c < kSpanB; ++c) r[c] = G.bp_srec[size_t(tt * kSpanB + c) * 64 + ln];
                const int4 cr = G.bp_crec[tt * kSpanB + (ln & (kSpanB - 1))];
                acc ^= uint32_t(cr.x ^ cr.y ^ cr.z ^ cr.w);
#pragma unroll
                for (int c = 0; c < kSpanB; ++c) {
                    const int sa = r[c].x;
                    const int sac = sa >= 0 ? sa : 0;
                    const int so = int(uint32_t(r[c].y) & 0x7fffffffu);
                    const int gq = sa >= 0 ? so - G.n_pi : 0;
                    const int u = r[c].w & 0x3ffffff;
                    acc ^= uint32_t(G.arc_meta[sac]) ^ uint32_t(argmax[size_t(gq) * NV]) ^
                           __float_as_uint(drv_slack[size_t(u) * NV]);
                }
            }
            asm volatile("" ::"v"(acc));
        }
        return;
    }
    const int t = tile0 + blockIdx.x * kSpanWaves + wave;
    if (t >= tile1) return;
    const int lane = threadIdx.x & 63;
    float* gs = s_g[wave];
    bool early[NW];
#pragma unroll
    for (int v = 0; v < NW; ++v) early[v] = V.mode[v0 + v] == STA_EARLY;
    // round 1: the tile's level and slot records
    int ns[kSpanB], ds0[kSpanB], ms[kSpanB];
    int sa_[kSpanB], so_[kSpanB], src[kSpanB], drv[kSpanB], sge[kSpanB], grk[kSpanB];
    bool hd[kSpanB];
    int nch = 0;
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        const int4 cr = G.bp_crec[t * kSpanB + c];
        ns[c] = cr.x;
        ds0[c] = cr.y;
        ms[c] = cr.z;
        nch = cr.w;
        const int4 r = G.bp_srec[size_t(t * kSpanB + c) * 64 + lane];
        const uint32_t bo = uint32_t(r.y);
        sa_[c] = r.x;
        so_[c] = int(bo & 0x7fffffffu);
        hd[c] = (bo & kHeadBit) != 0u;
        src[c] = int(int16_t(r.z & 0xffff));
        sge[c] = (r.z >> 16) & 0x7f;
        drv[c] = r.w & 0x3ffffff;
        grk[c] = int(uint32_t(r.w) >> 26);
    }
    // round 2
    int kp[kSpanB], am[kSpanB][NW];
    float ext[kSpanB][NW];
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        const int sa = sa_[c];
        const int sac = sa >= 0 ? sa : 0;
        kp[c] = int(G.arc_meta[sac] >> 16);
        const int gq = sa >= 0 ? so_[c] - G.n_pi : 0;
        const float* ep = sa >= 0 ? (src[c] >= 0 ? drv_slack : g_at + size_t(so_[c]) * NV + v0)
                                  : drv_slack + size_t(drv[c]) * NV + v0;
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            am[c][v] = int(argmax[size_t(gq) * NV + v0 + v]);
            ext[c][v] = ep[v];
        }
    }
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        pin_value(kp[c]);
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            pin_value(am[c][v]);
            pin_value(ext[c][v]);
        }
    }
#pragma unroll
    for (int c = 0; c < kSpanB; ++c) {
        if (c >= nch) break;                    // uniform
        const int n = ns[c];
        const bool act = lane < n && src[c] != -2;   // source -2: padding lane
        const bool head = act && hd[c];
        const int gi = grk[c];                 // from the record
        const int seg_end = sge[c];            // from the record
        const bool on_arc = act && sa_[c] >= 0;
        const int si = src[c] >= 0 ? src[c] : 0;
        float gin[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v) gin[v] = gs[si * NW + v];
        float acc[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            const float go = src[c] >= 0 ? gin[v] : ext[c][v];
            const float cv = (am[c][v] == kp[c]) ? go : 0.0f;
            if (on_arc) {
                if (g_arc) g_arc[size_t(sa_[c]) * NV + v0 + v] = cv;
                if (g_nd) g_nd[size_t(sa_[c]) * NV + v0 + v] = cv;
            }
            const float ep = ext[c][v] < 0.0f ? (early[v] ? 1.0f : -1.0f) : 0.0f;
            acc[v] = on_arc ? cv : (act ? ep : 0.0f);
        }
        if (ms[c] <= 16) {
            if (ms[c] > 1) span_sum_step<1, NW>(acc, (lane + 1) < seg_end);
            if (ms[c] > 2) span_sum_step<2, NW>(acc, (lane + 2) < seg_end);
            if (ms[c] > 4) span_sum_step<4, NW>(acc, (lane + 4) < seg_end);
            if (ms[c] > 8) span_sum_step<8, NW>(acc, (lane + 8) < seg_end);
        } else {
#pragma unroll
            for (int st = 0; st < 6; ++st) {
                const int off = 1 << st;
                if (off >= ms[c]) break;        // uniform
                const bool take = (lane + off) < seg_end;
                float b2[NW];
#pragma unroll
                for (int v = 0; v < NW; ++v) b2[v] = __shfl_down(acc[v], off, 64);
#pragma unroll
                for (int v = 0; v < NW; ++v) acc[v] = take ? acc[v] + b2[v] : acc[v];
            }
        }
        if (head) {
            const int u = drv[c];
#pragma unroll
            for (int v = 0; v < NW; ++v) {
                g_at[size_t(u) * NV + v0 + v] = acc[v];
                gs[(ds0[c] + gi) * NW + v] = acc[v];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// d TNS / d load of every gate output: the gradient of its arrival times the NLDM slope
// of its argmax arc's delay in the load ((q - p) / (y[j+1] - y[j]) of the bilinear
// lookup), input slews held; 0 at primary inputs.
template <int NV>
__global__ __launch_bounds__(256) void k_adj_load(DevGraph G, KLib lib, KViews V, const float* __restrict__ arc_load,
                                                  const float* __restrict__ arc_ts, const uint8_t* __restrict__ argmax,
                                                  const float* __restrict__ g_at, float* __restrict__ g_load) {
    __shared__ float s_ax[26];
    load_axes(s_ax, lib);
    __syncthreads();
    const int d = blockIdx.x * 256 + threadIdx.x;
    if (d >= G.n_drivers) return;
    if (d < G.n_pi) {
#pragma unroll
        for (int v = 0; v < NV; ++v) g_load[size_t(d) * NV + v] = 0.0f;
        return;
    }
    const float* X = s_ax;
    const float* DX = s_ax + 14;
    const int q = d - G.n_pi;
    const int a0 = G.gate_arc_ptr[q];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int a = a0 + int(argmax[size_t(q) * NV + v]);
        const float si = arc_ts[(size_t(a) * NV + v) * 2 + 1];
        const float L = arc_load[a];
        const float* T = lib.tables + (size_t(V.set[v]) * lib.n_tables + (G.arc_meta[a] & 0xffffu)) * 98;
        const int i = seg6(X, si);
        const float tx = (si - X[i]) / DX[i];
        int j;
        float ty;
        gate_jty(s_ax, L, j, ty);
        const float p = T[i * 7 + j] + tx * (T[(i + 1) * 7 + j] - T[i * 7 + j]);
        const float qv = T[i * 7 + j + 1] + tx * (T[(i + 1) * 7 + j + 1] - T[i * 7 + j + 1]);
        const float slope = (qv - p) / s_ax[20 + j];
        g_load[size_t(d) * NV + v] = g_at[size_t(d) * NV + v] * slope;
    }
}

__global__ void k_arc_load(DevGraph G, const float* __restrict__ load, float* __restrict__ arc_load) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= G.n_gates) return;
    const float ld = load[G.n_pi + q];
    for (int a = G.gate_arc_ptr[q]; a < G.gate_arc_ptr[q + 1]; ++a) arc_load[a] = ld;
}

// order-preserving key of (slack, endpoint rank): smaller key = worse slack, then lower rank
__device__ __forceinline__ unsigned long long path_key(float s, int rank) {
    uint32_t b = __float_as_uint(s);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return (static_cast<unsigned long long>(b) << 32) | static_cast<uint32_t>(rank);
}

// Selection of the k worst endpoints: every wavefront keeps the 64 smallest keys it has
// seen as an ascending list, one key per lane.  A batch of 64 new keys is sorted across the
// lanes (bitonic network) and merged in: the lane-wise minimum of the list and the reversed
// batch holds the 64 smallest of both as a bitonic sequence, which a half-cleaner network
// sorts.  Keys are unique (the rank is in the low bits), so the result is exact and the
// same in any order.
constexpr int kTopkWaves = 128;       // selection wavefronts (lists of 64 keys in the scratch)

__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) { return a < b ? a : b; }
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) { return a < b ? b : a; }

__device__ __forceinline__ unsigned long long wave_sort64(unsigned long long x, int lane) {
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const unsigned long long y = __shfl_xor(x, stride, 64);
            const bool up = (lane & size) == 0 || size == 64;
            const bool lower = (lane & stride) == 0;
            x = (lower == up) ? umin64(x, y) : umax64(x, y);
        }
    }
    return x;
}

// the 64 smallest of two ascending lists (a, b one key per lane), ascending
__device__ __forceinline__ unsigned long long wave_merge64(unsigned long long a, unsigned long long b, int lane) {
    unsigned long long c = umin64(a, __shfl(b, 63 - lane, 64));
#pragma unroll
    for (int stride = 32; stride > 0; stride >>= 1) {
        const unsigned long long y = __shfl_xor(c, stride, 64);
        c = ((lane & stride) == 0) ? umin64(c, y) : umax64(c, y);
    }
    return c;
}

__global__ __launch_bounds__(256) void k_topk_partial(const int32_t* __restrict__ ep_drv, int E,
                                                      const float* __restrict__ drv_slack, int NV, int v,
                                                      unsigned long long* __restrict__ cand) {
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int W = gridDim.x * 4;
    unsigned long long best = ~0ull;
    const int nb = (E + 63) / 64;
    for (int b = gw; b < nb; b += W) {
        const int e = b * 64 + lane;
        unsigned long long x = ~0ull;
        if (e < E) x = path_key(drv_slack[size_t(ep_drv[e]) * NV + v], e);
        const unsigned long long worst = __shfl(best, 63, 64);
        if (__ballot(x < worst) == 0ull) continue;        // nothing in this batch gets in
        best = wave_merge64(best, wave_sort64(x, lane), lane);
    }
    cand[size_t(gw) * 64 + lane] = best;
}

__global__ __launch_bounds__(256) void k_topk_final(const unsigned long long* __restrict__ cand, int n_lists, int k,
                                                    int32_t* __restrict__ ep_rank, float* __restrict__ slack) {
    __shared__ unsigned long long s_l[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long best = ~0ull;
    for (int i = w; i < n_lists; i += 4) best = wave_merge64(best, cand[size_t(i) * 64 + lane], lane);
    s_l[w][lane] = best;
    __syncthreads();
    if (w != 0) return;
    for (int i = 1; i < 4; ++i) best = wave_merge64(best, s_l[i][lane], lane);
    if (lane < k) {
        const unsigned long long x = best;
        uint32_t b = uint32_t(x >> 32);
        b = (b & 0x80000000u) ? (b & 0x7fffffffu) : ~b;
        ep_rank[lane] = int32_t(uint32_t(x));
        slack[lane] = __uint_as_float(b);
    }
}

// walk the saved argmax arcs from each selected endpoint back to a primary input
__global__ void k_backtrace(DevGraph G, int NV, int v, int k, int L, const uint8_t* __restrict__ argmax,
                            const int32_t* __restrict__ ep_rank, int32_t* __restrict__ len,
                            int32_t* __restrict__ drv, int32_t* __restrict__ arc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    int u = G.ep_drv[ep_rank[i]];
    int n = 0;
    int32_t* pd = drv + size_t(i) * (L + 1);
    int32_t* pa = arc + size_t(i) * L;
    while (n <= L) {
        pd[n++] = u;
        if (u < G.n_pi || n > L) break;
        const int q = u - G.n_pi;
        const int a = G.gate_arc_ptr[q] + int(argmax[size_t(q) * NV + v]);
        pa[n - 1] = a;
        u = G.arc_src[a];
    }
    len[i] = n;
}

template <int NV>
static void enqueue_adjoint_levels(const sta_graph* g, const KLib& kl, const KViews& kv, const sta_net_out* nd,
                                   const sta_timing_out* t, const sta_slack_out* sl, const sta_adjoint_out* o,
                                   hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    auto level = [&](int64_t l) {
        const int t0 = g->bwd_tile_ptr[l], t1 = g->bwd_tile_ptr[l + 1];
        if (t1 <= t0) return;
        const KTiles kt = ktiles(g->btile_slot_h, g->btile_drv_h, t0, t1);
        prof_launch("k_adjoint", s, [&] {
            hipLaunchKernelGGL((k_adjoint<NV>), dim3((t1 - t0 + kLevelWaves - 1) / kLevelWaves),
                               dim3(64 * kLevelWaves), 0, s, dg, kv, t0, t1, kt,
                               t->argmax, sl->drv_slack, o->g_drv_at, o->g_arc_delay, o->g_net_delay);
        });
    };
    bool done = false;
    if constexpr (NV <= kSpanMaxViews) {
        if (g->use_spans) {
            const int64_t NSB = int64_t(g->bspan_fused_h.size());
            for (int64_t b = 0; b < NSB; ++b) {
                const int64_t top = g->bspan_lv_h[2 * b], bot = g->bspan_lv_h[2 * b + 1];
                if (!g->bspan_fused_h[b]) {
                    for (int64_t l = top; l >= bot; --l) level(l);
                    continue;
                }
                const int t0 = g->bspan_tile_h[b], t1 = g->bspan_tile_h[b + 1];
                if (t1 <= t0) continue;
                // the next fused span's tiles, for the spare workgroups' L2 prefetch
                int pf0 = 0, pf1 = 0;
                if (b + 1 < int64_t(g->bspan_fused_h.size()) && g->bspan_fused_h[b + 1]) {
                    pf0 = g->bspan_tile_h[b + 1];
                    pf1 = g->bspan_tile_h[b + 2];
                }
                const int gx = pf1 > pf0 ? span_round8(t1 - t0) + span_pf_blocks(pf1 - pf0, kSpanPfTilesB) : t1 - t0;
                prof_launch("k_adjoint_span", s, [&] {
                    hipLaunchKernelGGL((k_adjoint_span<NV, kSpanViewsPerWave < NV ? kSpanViewsPerWave : NV>),
                                       dim3(gx, NV / (kSpanViewsPerWave < NV ? kSpanViewsPerWave : NV)),
                                       dim3(64 * kSpanWaves), 0, s, dg, kv, t0, t1, t->argmax, sl->drv_slack,
                                       o->g_drv_at, o->g_arc_delay, o->g_net_delay, pf0, pf1);
                });
            }
            done = true;
        }
    }
    if (!done)
        for (int64_t l = g->L; l >= 0; --l) level(l);
    if (o->g_load)
        prof_launch("k_adj_load", s, [&] {
            hipLaunchKernelGGL((k_adj_load<NV>), dim3((g->D + 255) / 256), dim3(256), 0, s, dg, kl, kv, nd->arc_load,
                               t->arc_ts, t->argmax, o->g_drv_at, o->g_load);
        });
}

template <int NV>
static sta_status run_adjoint_levels(const sta_graph* g, const KLib& kl, const KViews& kv, const sta_net_out* nd,
                                     const sta_timing_out* t, const sta_slack_out* sl, const sta_adjoint_out* o,
                                     hipStream_t s) {
    std::vector<uint64_t> key = {pk(g->dev), uint64_t(NV), pk(nd->arc_load), pk(t->arc_ts), pk(t->argmax), pk(sl->drv_slack),
                                 pk(o->g_drv_at), pk(o->g_arc_delay), pk(o->g_net_delay), pk(o->g_load),
                                 pk(kl.tables), uint64_t(kl.n_tables), uint64_t(g->use_spans)};
    for (int i = 0; i < 26; ++i) { uint32_t b; std::memcpy(&b, &kl.ax[i], 4); key.push_back(b); }
    for (int v = 0; v < NV; ++v) { key.push_back(uint64_t(kv.mode[v])); key.push_back(uint64_t(kv.set[v])); }
    return run_sequence(g, g->adj_cache, std::move(key), s, [&](hipStream_t q) {
        enqueue_adjoint_levels<NV>(g, kl, kv, nd, t, sl, o, q);
    });
}

static bool lib_axes_ok(const sta_library* lib, int n_tables, std::string& why) {
    if (lib->n_sets < 1 || lib->n_tables < n_tables || !lib->tables) { why = "library has fewer tables than the design references"; return false; }
    for (int i = 0; i < 7; ++i)
        if (!std::isfinite(lib->x[i]) || !std::isfinite(lib->y[i])) { why = "non-finite library axis"; return false; }
    for (int i = 0; i < 6; ++i)
        if (!(lib->x[i] < lib->x[i + 1]) || !(lib->y[i] < lib->y[i + 1])) { why = "library axes must strictly increase"; return false; }
    return true;
}

// The least float a for which the correctly rounded square root reaches p: sqrtf is
// nondecreasing, so sqrtf(a) >= p exactly when a >= sqrt_floor_of(p), for every a, NaN
// included (both sides false).  p <= 0: every a >= -0 qualifies (sqrtf(-0) = -0 >= p), and
// a negative a has a NaN root, so the threshold is 0; p = +inf: only a = +inf; NaN: none.
static float sqrt_threshold(float p) {
    if (std::isnan(p)) return p;
    if (!(p > 0.0f)) return 0.0f;
    if (std::isinf(p)) return p;
    const double d = double(p) * double(p);
    float t = d >= double(FLT_MAX) ? FLT_MAX : float(d);
    while (t > 0.0f && std::sqrt(std::nextafter(t, 0.0f)) >= p) t = std::nextafter(t, 0.0f);
    while (!(std::sqrt(t) >= p)) t = std::nextafter(t, HUGE_VALF);
    return t;
}

static KLib make_klib(const sta_library* lib) {
    KLib kl{};
    for (int i = 0; i < 7; ++i) { kl.ax[i] = lib->x[i]; kl.ax[7 + i] = lib->y[i]; }
    for (int i = 0; i < 6; ++i) { kl.ax[14 + i] = lib->x[i + 1] - lib->x[i]; kl.ax[20 + i] = lib->y[i + 1] - lib->y[i]; }
    for (int k = 0; k < 5; ++k) kl.sq[k] = sqrt_threshold(lib->x[k + 1]);
    kl.tables = lib->tables;
    kl.n_tables = lib->n_tables;
    return kl;
}


// ---------------------------------------------------------------------------------
// batches of graphs: one persistent launch plus per-level launches
// ---------------------------------------------------------------------------------

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <int NV>
static void enqueue_levels_any(const sta_graph* g, const KLib& kl, const KViews& kv, const float* pi_ts,
                               const sta_net_out* nd, const sta_timing_out* o, hipStream_t s) {
    enqueue_forward_levels<NV>(g, kl, kv, pi_ts, nd, o, s);
}

static void enqueue_levels_nv(int NV, const sta_graph* g, const KLib& kl, const KViews& kv, const float* pi_ts,
                              const sta_net_out* nd, const sta_timing_out* o, hipStream_t s) {
    switch (NV) {
        case 1: enqueue_levels_any<1>(g, kl, kv, pi_ts, nd, o, s); break;
        case 2: enqueue_levels_any<2>(g, kl, kv, pi_ts, nd, o, s); break;
        case 4: enqueue_levels_any<4>(g, kl, kv, pi_ts, nd, o, s); break;
        default: enqueue_levels_any<8>(g, kl, kv, pi_ts, nd, o, s); break;
    }
}

}  // namespace sta

struct sta_batch {
    struct Lvl {
        const sta_graph* g;
        const float* pi_ts;
        sta_net_out nd;
        sta_timing_out out;
    };
    // a span step: one batched launch over map[map0, map0 + nblk), plus the level launches
    // of the designs whose span of this step does not fuse (item, first and last level in
    // the pass's order)
    struct Step {
        int map0 = 0, nblk = 0;
        std::vector<std::array<int64_t, 3>> levels;
    };
    struct DcClass {
        int maxn = 0, map0 = 0, nblk = 0;
        bool chains = true;        // every design of the class has only chain nets
    };
    std::vector<Lvl> level_designs;
    std::vector<const sta_graph*> graphs;      // per item
    std::vector<sta_net_out> nds;              // per item
    std::vector<sta_timing_out> outs;          // per item
    std::vector<sta_slack_out> sls;            // per item (zeroed without slack)
    std::vector<const float*> ep_rats;         // per item
    std::vector<Step> fsteps, bsteps;
    std::vector<DcClass> dc;
    int n_items = 0, n_span_items = 0, ep_map0 = 0, ep_nblk = 0, n_slack_items = 0;
    int n_units = 0;
    int NV = 0;
    sta::KLib kl{};
    sta::KViews kv{};
    size_t lds = 0;
    sta::BatchItem* d_items = nullptr;
    int2* d_units = nullptr;
    int* d_counter = nullptr;
    int2* d_map = nullptr;
    unsigned long long* d_limbs = nullptr;
    float* d_wns = nullptr;
    sta::BatchItem* d_span_items = nullptr;    // the span designs' items, first in the table
    sta_batch_plan plan{};
    sta::LaunchCache cache, bcache, dcache;
    std::mutex mu;
    // a second stream (default priority) and two events: the persistent launch runs on it,
    // forked from and joined back into the caller's stream, beside the span steps
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // views per span wavefront of the batched span launches (sta_batch_set_tiling)
    int fwd_nw = 1, bwd_nw = 2;
};

namespace sta {

// Byte offsets of a batch's workspace regions and the entry counts they were sized for.
struct BatchLayout {
    size_t items = 0, units = 0, counter = 0, map = 0, limbs = 0, wns = 0, total = 0;
    int64_t n_map = 0, n_ep = 0;
};

// endpoint-summary workgroups of one design in a batch: one per 2048 endpoints, 1 to 64
static int batch_ep_blocks(int64_t E) {
    const int64_t nb = (E + 2047) / 2048;
    return int(nb < 1 ? 1 : (nb > 64 ? 64 : nb));
}

// node-count class of a graph's delay calculation and the workgroup size of that class
// (the classes and sizes of sta_delay_calc)
static int dc_class(const sta_graph* g) {
    const int m = g->max_net_nodes;
    return m <= 8 ? 8 : m <= 16 ? 16 : m <= 32 ? 32 : m <= 64 ? 64 : m <= 128 ? 128 : 256;
}
static int dc_threads(int maxn) { return maxn <= 8 ? 256 : 2048 / maxn; }

static bool batch_layout(const sta_batch_design* designs, int32_t n, int NV, BatchLayout* L) {
    int64_t items = 0, maps = 0, ep = 0;
    for (int i = 0; i < n; ++i) {
        const sta_graph* g = designs[i].g;
        if (!g) return false;
        if (g->D == 0) continue;
        ++items;
        if (designs[i].schedule != STA_BATCH_LEVELS)     // spans (or the persistent fallback)
            for (size_t sp = 0; sp < g->span_fused_h.size(); ++sp)
                if (g->span_fused_h[sp]) maps += g->span_tile_h[sp + 1] - g->span_tile_h[sp];
        if (designs[i].ep_rat && designs[i].sl) {
            for (size_t sp = 0; sp < g->bspan_fused_h.size(); ++sp)
                if (g->bspan_fused_h[sp]) maps += g->bspan_tile_h[sp + 1] - g->bspan_tile_h[sp];
            const int eb = batch_ep_blocks(g->E);
            maps += eb;
            ep += eb;
        }
        const int mc = dc_class(g);
        maps += dc_blocks_of(g->D, g->n_dc_wide, mc, dc_threads(mc));
    }
    L->n_map = maps;
    L->n_ep = ep;
    size_t off = 0;
    L->items = off;
    off += align256(sizeof(BatchItem) * size_t(std::max<int64_t>(items, 1)));
    L->units = off;
    off += align256(sizeof(int2) * size_t(std::max<int64_t>(items * NV, 1)));
    L->counter = off;
    off += 256;
    L->map = off;
    off += align256(sizeof(int2) * size_t(std::max<int64_t>(maps, 1)));
    L->limbs = off;
    off += align256(sizeof(unsigned long long) * size_t(std::max<int64_t>(ep, 1)) * NV * kLimbs);
    L->wns = off;
    off += align256(sizeof(float) * size_t(std::max<int64_t>(ep, 1)) * NV);
    L->total = off;
    return true;
}

template <typename T>
static void launch_dc_batch(const sta_batch* b, int maxn, bool chains, int map0, int nblk, hipStream_t q) {
    auto go = [&](auto kern, int nt) {
        prof_launch("k_delay_calc_batch", q, [&] {
            hipLaunchKernelGGL(kern, dim3(nblk), dim3(nt), 0, q, b->d_items, b->d_map, map0);
        });
    };
    switch (maxn) {
        case 8:
            if (chains) go(k_delay_calc8_batch<T, true>, 256);
            else go(k_delay_calc8_batch<T, false>, 256);
            break;
        case 16: go(k_delay_calc_batch<T, 16, 128>, 128); break;
        case 32: go(k_delay_calc_batch<T, 32, 64>, 64); break;
        case 64: go(k_delay_calc_batch<T, 64, 32>, 32); break;
        case 128: go(k_delay_calc_batch<T, 128, 16>, 16); break;
        default: go(k_delay_calc_batch<T, 256, 8>, 8); break;
    }
}

// Forward pass of the span designs: the batched primary-input copy, then per step one
// batched span launch (every design's s-th fused span, every view) and the level launches
// of the spans of this step that do not fuse.
template <int NV>
static void enqueue_batch_forward(const sta_batch* b, hipStream_t q) {
    if (b->n_span_items > 0) {
        int max_pi = 0;
        for (int k = 0; k < b->n_span_items; ++k) max_pi = std::max(max_pi, int(b->graphs[k]->n_pi));
        const int n = max_pi * NV * 2;
        if (n > 0) {
            const int gx = std::min((n + 255) / 256, 64);
            prof_launch("k_copy_pi_batch", q, [&] {
                hipLaunchKernelGGL(k_copy_pi_batch, dim3(gx, b->n_span_items), dim3(256), 0, q, b->d_items, NV);
            });
        }
    }
    for (const auto& st : b->fsteps) {
        if (st.nblk > 0)
            prof_launch("k_forward_span_batch", q, [&] {
                auto go = [&](auto kern, int nw) {
                    hipLaunchKernelGGL(kern, dim3(st.nblk, NV / nw), dim3(64), 0, q, b->d_items, b->d_map, st.map0,
                                       b->kl, b->kv);
                };
                const int nw = std::min(b->fwd_nw, NV);
                if (nw >= 4 && NV >= 4) go(k_forward_span_batch<NV, (NV >= 4 ? 4 : 1)>, 4);
                else if (nw >= 2 && NV >= 2) go(k_forward_span_batch<NV, (NV >= 2 ? 2 : 1)>, 2);
                else go(k_forward_span_batch<NV, 1>, 1);
            });
        for (const auto& lv : st.levels) {
            const int k = int(lv[0]);
            for (int64_t l = lv[1]; l <= lv[2]; ++l)
                launch_forward_level<NV>(b->graphs[k], b->kl, b->kv, &b->nds[k], &b->outs[k], l, q);
        }
    }
}

// Backward pass of the slack designs: per step one batched backward-span launch and the
// level launches of unfused spans (top down), then the batched endpoint summary.
template <int NV>
static void enqueue_batch_backward(const sta_batch* b, hipStream_t q) {
    for (const auto& st : b->bsteps) {
        if (st.nblk > 0)
            prof_launch("k_backward_span_batch", q, [&] {
                auto go = [&](auto kern, int nw) {
                    hipLaunchKernelGGL(kern, dim3(st.nblk, NV / nw), dim3(64), 0, q, b->d_items, b->d_map, st.map0,
                                       b->kv);
                };
                const int nw = std::min(b->bwd_nw, NV);
                if (nw >= 4 && NV >= 4) go(k_backward_span_batch<NV, (NV >= 4 ? 4 : 1)>, 4);
                else if (nw >= 2 && NV >= 2) go(k_backward_span_batch<NV, (NV >= 2 ? 2 : 1)>, 2);
                else go(k_backward_span_batch<NV, 1>, 1);
            });
        for (const auto& lv : st.levels) {
            const int k = int(lv[0]);
            const sta_slack_out& o = b->sls[k];
            const sta_timing_out& t = b->outs[k];
            for (int64_t l = lv[1]; l >= lv[2]; --l)
                launch_backward_level<NV>(b->graphs[k], b->kv, b->nds[k].net_delay, t.drv_ts, t.arc_ts, t.arc_delay,
                                          b->ep_rats[k], o.drv_rat, o.arc_rat, o.drv_slack, o.arc_slack, l, q);
        }
    }
    if (b->ep_nblk > 0) {
        prof_launch("k_endpoint_partial_batch", q, [&] {
            hipLaunchKernelGGL((k_endpoint_partial_batch<NV>), dim3(b->ep_nblk), dim3(kK4Threads), 0, q, b->d_items,
                               b->d_map, b->ep_map0, b->d_limbs, b->d_wns);
        });
        prof_launch("k_endpoint_final_batch", q, [&] {
            hipLaunchKernelGGL((k_endpoint_final_batch<NV>), dim3(b->n_items), dim3(256), 0, q, b->d_items,
                               b->d_limbs, b->d_wns);
        });
    }
}

}  // namespace sta

using namespace sta;

extern "C" {

sta_status sta_delay_calc(const sta_graph* g, sta_dc_precision prec, const sta_net_out* out, void* stream) {
    if (!g || !out) return fail(STA_E_ARG, "sta_delay_calc: null argument");
    if (!g->dev) return fail(STA_E_ARG, "sta_delay_calc: graph not uploaded");
    if (prec != STA_DC_FP64 && prec != STA_DC_FP32) return fail(STA_E_ARG, "sta_delay_calc: unknown precision");
    if (g->D == 0) return STA_OK;
    if (!out->load || (g->A > 0 && (!out->net_delay || !out->net_imp2 || !out->arc_load)))
        return fail(STA_E_ARG, "sta_delay_calc: null output buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (prec == STA_DC_FP64) dispatch_dc<double>(g, out, s);
    else dispatch_dc<float>(g, out, s);
    return launch_check("sta_delay_calc");
}

sta_status sta_propagate(const sta_graph* g, const sta_library* lib, const sta_views* views, const float* pi_ts,
                         const sta_net_out* nd, const sta_timing_out* out, void* stream) {
    if (!g || !lib || !nd || !out) return fail(STA_E_ARG, "sta_propagate: null argument");
    if (!g->dev) return fail(STA_E_ARG, "sta_propagate: graph not uploaded");
    std::string why;
    if (!views_ok(views, lib->n_sets, why)) return fail(STA_E_ARG, "sta_propagate: " + why);
    if (lib->n_sets < 1 || lib->n_tables < g->n_tables || !lib->tables)
        return fail(STA_E_ARG, "sta_propagate: library has fewer tables than the design references");
    for (int i = 0; i < 7; ++i)
        if (!std::isfinite(lib->x[i]) || !std::isfinite(lib->y[i]))
            return fail(STA_E_NONFINITE, "sta_propagate: non-finite library axis");
    for (int i = 0; i < 6; ++i)
        if (!(lib->x[i] < lib->x[i + 1]) || !(lib->y[i] < lib->y[i + 1]))
            return fail(STA_E_ARG, "sta_propagate: library axes must strictly increase");
    if (g->D == 0) return STA_OK;
    if ((g->n_pi > 0 && !pi_ts) || !out->drv_ts ||
        (g->A > 0 && (!out->arc_ts || !out->arc_delay || !out->argmax || !nd->net_delay || !nd->net_imp2 ||
                      !nd->arc_load)) ||
        !nd->load)
        return fail(STA_E_ARG, "sta_propagate: null buffer");
    const KLib kl = make_klib(lib);
    const KViews kv = kviews(views);
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t lds = 0;
    if (use_view_forward(g, lib->n_tables, views->n_views, &lds)) {
        run_forward_views(g, lds, views->n_views, kl, kv, pi_ts, nd, out, s);
    } else {
        sta_status st;
        switch (views->n_views) {
            case 1: st = run_forward_levels<1>(g, kl, kv, pi_ts, nd, out, s); break;
            case 2: st = run_forward_levels<2>(g, kl, kv, pi_ts, nd, out, s); break;
            case 4: st = run_forward_levels<4>(g, kl, kv, pi_ts, nd, out, s); break;
            default: st = run_forward_levels<8>(g, kl, kv, pi_ts, nd, out, s); break;
        }
        if (st != STA_OK) return st;
    }
    return launch_check("sta_propagate");
}

sta_status sta_slack(const sta_graph* g, const sta_views* views, const sta_net_out* nd, const sta_timing_out* t,
                     const float* ep_rat, const sta_slack_out* out, void* scratch, size_t scratch_bytes_, void* stream) {
    if (!g || !nd || !t || !out) return fail(STA_E_ARG, "sta_slack: null argument");
    if (!g->dev) return fail(STA_E_ARG, "sta_slack: graph not uploaded");
    std::string why;
    if (!views_ok(views, -1, why)) return fail(STA_E_ARG, "sta_slack: " + why);
    if (!scratch || scratch_bytes_ < scratch_bytes()) return fail(STA_E_ARG, "sta_slack: scratch smaller than scratch_bytes");
    if (!out->tns || !out->wns) return fail(STA_E_ARG, "sta_slack: null tns/wns");
    if (g->D > 0 && (!out->drv_rat || !out->drv_slack || !t->drv_ts || (g->E > 0 && !ep_rat) ||
                     (g->A > 0 && (!out->arc_rat || !out->arc_slack || !t->arc_ts || !t->arc_delay || !nd->net_delay))))
        return fail(STA_E_ARG, "sta_slack: null buffer");
    const KViews kv = kviews(views);
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t lds = 0;
    if (use_view_backward(g, views->n_views, &lds)) {
        run_backward_views(g, lds, views->n_views, kv, nd, t, ep_rat, out, s);
    } else {
        sta_status st;
        switch (views->n_views) {
            case 1: st = run_backward_levels<1>(g, kv, nd, t, ep_rat, out, scratch, s); break;
            case 2: st = run_backward_levels<2>(g, kv, nd, t, ep_rat, out, scratch, s); break;
            case 4: st = run_backward_levels<4>(g, kv, nd, t, ep_rat, out, scratch, s); break;
            default: st = run_backward_levels<8>(g, kv, nd, t, ep_rat, out, scratch, s); break;
        }
        if (st != STA_OK) return st;
    }
    return launch_check("sta_slack");
}

// Device address of slack_scratch on the current device, looked up once per device (with
// that device current) and kept; later calls read the kept address.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static sta_status slack_scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(STA_E_HIP, std::string("sta_slack_noalloc: hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(STA_E_ARG, "sta_slack_noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(slack_scratch));
        if (e != hipSuccess || !p)
            return fail(STA_E_HIP, std::string("sta_slack_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return STA_OK;
}

sta_status sta_slack_noalloc(const sta_graph* g, const sta_views* views, const sta_net_out* nd,
                             const sta_timing_out* t, const float* ep_rat, const sta_slack_out* out, void* stream) {
    if (!g || !nd || !t || !out) return fail(STA_E_ARG, "sta_slack_noalloc: null argument");
    if (!g->dev) return fail(STA_E_ARG, "sta_slack_noalloc: graph not uploaded");
    std::string why;
    if (!views_ok(views, -1, why)) return fail(STA_E_ARG, "sta_slack_noalloc: " + why);
    if (scratch_bytes() > kNoAllocScratchBytes)
        return fail(STA_E_ARG, "sta_slack_noalloc: the endpoint partials exceed the static scratch");
    if (!out->tns || !out->wns) return fail(STA_E_ARG, "sta_slack_noalloc: null tns/wns");
    if (g->D > 0 && (!out->drv_rat || !out->drv_slack || !t->drv_ts || (g->E > 0 && !ep_rat) ||
                     (g->A > 0 && (!out->arc_rat || !out->arc_slack || !t->arc_ts || !t->arc_delay || !nd->net_delay))))
        return fail(STA_E_ARG, "sta_slack_noalloc: null buffer");
    void* scr = nullptr;
    sta_status st = slack_scratch_ptr(&scr);
    if (st != STA_OK) return st;
    const KViews kv = kviews(views);
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t lds = 0;
    // the same schedule choice as sta_slack, launched directly (no launch-sequence capture)
    if (use_view_backward(g, views->n_views, &lds)) {
        run_backward_views(g, lds, views->n_views, kv, nd, t, ep_rat, out, s);
    } else {
        switch (views->n_views) {
            case 1: enqueue_backward_levels<1>(g, kv, nd, t, ep_rat, out, scr, s); break;
            case 2: enqueue_backward_levels<2>(g, kv, nd, t, ep_rat, out, scr, s); break;
            case 4: enqueue_backward_levels<4>(g, kv, nd, t, ep_rat, out, scr, s); break;
            default: enqueue_backward_levels<8>(g, kv, nd, t, ep_rat, out, scr, s); break;
        }
    }
    return launch_check("sta_slack_noalloc");
}

sta_status sta_profile_begin(void) {
    for (auto& r : g_prof.recs) { hipEventDestroy(r.start); hipEventDestroy(r.stop); }
    g_prof.recs.clear();
    g_prof.failed = false;
    g_prof.on = true;
    return STA_OK;
}

sta_status sta_profile_end(sta_kernel_stat* stats, int32_t cap, int32_t* n) {
    if (!g_prof.on) return fail(STA_E_ARG, "sta_profile_end: profiling is not active");
    g_prof.on = false;
    if (!n || (cap > 0 && !stats)) return fail(STA_E_ARG, "sta_profile_end: null output");
    std::map<std::string, std::pair<int64_t, double>> agg;
    std::vector<std::string> order;
    sta_status st = g_prof.failed ? fail(STA_E_HIP, "sta_profile_end: hipEventCreate failed") : STA_OK;
    for (auto& r : g_prof.recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
            st = fail(STA_E_HIP, "sta_profile_end: event query failed");
        if (!agg.count(r.name)) order.push_back(r.name);
        auto& a = agg[r.name];
        a.first += 1;
        a.second += ms;
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    g_prof.recs.clear();
    int32_t k = 0;
    for (const auto& name : order) {
        if (k < cap) {
            std::memset(stats[k].name, 0, sizeof(stats[k].name));
            std::strncpy(stats[k].name, name.c_str(), sizeof(stats[k].name) - 1);
            stats[k].launches = agg[name].first;
            stats[k].total_ms = agg[name].second;
        }
        ++k;
    }
    *n = k;
    return st;
}

sta_status sta_set_level_fusion(sta_graph* g, int32_t enable) {
    if (!g) return fail(STA_E_ARG, "sta_set_level_fusion: null graph");
    g->use_spans = enable != 0;
    return STA_OK;
}

sta_status sta_set_schedule(sta_graph* g, int32_t view_max_arcs_per_level, int32_t use_graphs) {
    if (!g) return fail(STA_E_ARG, "sta_set_schedule: null graph");
    g->view_sched_max_arcs = view_max_arcs_per_level < 0 ? kDefaultViewSchedMaxArcs : view_max_arcs_per_level;
    g->view_auto = view_max_arcs_per_level < 0;
    g->use_graphs = use_graphs != 0;
    return STA_OK;
}

sta_status sta_arc_load(const sta_graph* g, const sta_net_out* nd, void* stream) {
    if (!g || !nd) return fail(STA_E_ARG, "sta_arc_load: null argument");
    if (!g->dev) return fail(STA_E_ARG, "sta_arc_load: graph not uploaded");
    if (g->n_gates == 0) return STA_OK;
    if (!nd->load || !nd->arc_load) return fail(STA_E_ARG, "sta_arc_load: null buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const DevGraph dg = dev_graph(g);
    prof_launch("k_arc_load", s, [&] {
        hipLaunchKernelGGL(k_arc_load, dim3((g->n_gates + 255) / 256), dim3(256), 0, s, dg, nd->load, nd->arc_load);
    });
    return launch_check("sta_arc_load");
}

sta_status sta_tns_adjoint(const sta_graph* g, const sta_library* lib, const sta_views* views, const sta_net_out* nd,
                           const sta_timing_out* t, const sta_slack_out* sl, const sta_adjoint_out* out,
                           void* stream) {
    if (!g || !views || !nd || !t || !sl || !out) return fail(STA_E_ARG, "sta_tns_adjoint: null argument");
    if (!g->dev) return fail(STA_E_ARG, "sta_tns_adjoint: graph not uploaded");
    std::string why;
    if (!views_ok(views, lib ? lib->n_sets : -1, why)) return fail(STA_E_ARG, "sta_tns_adjoint: " + why);
    if (out->g_load && (!lib || !lib_axes_ok(lib, int(g->n_tables), why)))
        return fail(STA_E_ARG, "sta_tns_adjoint: " + (lib ? why : std::string("g_load needs the library")));
    if (g->D == 0) return STA_OK;
    if (!out->g_drv_at || !sl->drv_slack || (g->A > 0 && !t->argmax) ||
        (out->g_load && (!t->arc_ts || !nd->arc_load)))
        return fail(STA_E_ARG, "sta_tns_adjoint: null buffer");
    const KViews kv = kviews(views);
    const KLib kl = (out->g_load && lib) ? make_klib(lib) : KLib{};
    hipStream_t s = static_cast<hipStream_t>(stream);
    sta_status st;
    switch (views->n_views) {
        case 1: st = run_adjoint_levels<1>(g, kl, kv, nd, t, sl, out, s); break;
        case 2: st = run_adjoint_levels<2>(g, kl, kv, nd, t, sl, out, s); break;
        case 4: st = run_adjoint_levels<4>(g, kl, kv, nd, t, sl, out, s); break;
        default: st = run_adjoint_levels<8>(g, kl, kv, nd, t, sl, out, s); break;
    }
    if (st != STA_OK) return st;
    return launch_check("sta_tns_adjoint");
}

size_t sta_paths_scratch_bytes(void) { return sizeof(unsigned long long) * kTopkWaves * 64; }

sta_status sta_critical_paths(const sta_graph* g, const sta_views* views, int32_t view, int32_t k,
                              const sta_timing_out* t, const sta_slack_out* sl, const sta_paths_out* out,
                              void* scratch, size_t scratch_bytes_, void* stream) {
    if (!g || !views || !t || !sl || !out) return fail(STA_E_ARG, "sta_critical_paths: null argument");
    if (!g->dev) return fail(STA_E_ARG, "sta_critical_paths: graph not uploaded");
    std::string why;
    if (!views_ok(views, -1, why)) return fail(STA_E_ARG, "sta_critical_paths: " + why);
    if (view < 0 || view >= views->n_views) return fail(STA_E_ARG, "sta_critical_paths: view out of range");
    if (k < 1 || k > STA_MAX_PATHS) return fail(STA_E_ARG, "sta_critical_paths: k must be in 1..STA_MAX_PATHS");
    if (k > g->E) return fail(STA_E_ARG, "sta_critical_paths: k exceeds the number of endpoints");
    if (!scratch || scratch_bytes_ < sta_paths_scratch_bytes()) return fail(STA_E_ARG, "sta_critical_paths: scratch too small");
    if (!out->ep_rank || !out->slack || !out->len || !out->drv || !out->arc || !sl->drv_slack || (g->A > 0 && !t->argmax))
        return fail(STA_E_ARG, "sta_critical_paths: null buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const DevGraph dg = dev_graph(g);
    const int NV = views->n_views;
    auto* cand = static_cast<unsigned long long*>(scratch);
    // about eight batches of 64 endpoints per selection wavefront, at most kTopkWaves of them
    const int64_t nb = (g->E + 63) / 64;
    int blocks = int((nb + 31) / 32);
    blocks = blocks < 1 ? 1 : (blocks > kTopkWaves / 4 ? kTopkWaves / 4 : blocks);
    prof_launch("k_topk_partial", s, [&] {
        hipLaunchKernelGGL(k_topk_partial, dim3(blocks), dim3(256), 0, s, dg.ep_drv, int(g->E), sl->drv_slack, NV,
                           int(view), cand);
    });
    prof_launch("k_topk_final", s, [&] {
        hipLaunchKernelGGL(k_topk_final, dim3(1), dim3(256), 0, s, cand, blocks * 4, int(k), out->ep_rank,
                           out->slack);
    });
    prof_launch("k_backtrace", s, [&] {
        hipLaunchKernelGGL(k_backtrace, dim3(1), dim3(64), 0, s, dg, NV, int(view), int(k), int(g->L), t->argmax,
                           out->ep_rank, out->len, out->drv, out->arc);
    });
    return launch_check("sta_critical_paths");
}

size_t sta_batch_workspace_bytes(const sta_batch_design* designs, int32_t n, int32_t n_views) {
    BatchLayout L;
    if (n < 0 || (n > 0 && !designs) || n_views < 1 || n_views > STA_MAX_VIEWS || !batch_layout(designs, n, n_views, &L))
        return 0;
    return L.total;
}

sta_status sta_batch_create(const sta_batch_design* designs, int32_t n, const sta_library* lib,
                            const sta_views* views, void* workspace, size_t workspace_bytes, sta_batch** out) {
    if (!out) return fail(STA_E_ARG, "sta_batch_create: null output");
    *out = nullptr;
    if (n < 0 || (n > 0 && !designs) || !lib || !views) return fail(STA_E_ARG, "sta_batch_create: null argument");
    std::string why;
    if (!views_ok(views, lib->n_sets, why)) return fail(STA_E_ARG, "sta_batch_create: " + why);
    if (!lib_axes_ok(lib, 0, why)) return fail(STA_E_ARG, "sta_batch_create: " + why);
    const int NV = views->n_views;
    for (int i = 0; i < n; ++i) {
        const sta_batch_design& d = designs[i];
        const std::string tag = " (design " + std::to_string(i) + ")";
        if (!d.g || !d.nd || !d.out) return fail(STA_E_ARG, "sta_batch_create: null design entry" + tag);
        const sta_graph* g = d.g;
        if (!g->dev) return fail(STA_E_ARG, "sta_batch_create: graph not uploaded" + tag);
        if (lib->n_tables < g->n_tables) return fail(STA_E_ARG, "sta_batch_create: library has fewer tables than the graph" + tag);
        if (d.schedule != STA_BATCH_PERSISTENT && d.schedule != STA_BATCH_LEVELS && d.schedule != STA_BATCH_SPANS)
            return fail(STA_E_ARG, "sta_batch_create: bad schedule" + tag);
        if ((d.ep_rat == nullptr) != (d.sl == nullptr))
            return fail(STA_E_ARG, "sta_batch_create: ep_rat and sl must be given together" + tag);
        if (g->D == 0) continue;
        if ((g->n_pi > 0 && !d.pi_ts) || !d.out->drv_ts || !d.nd->load ||
            (g->A > 0 && (!d.out->arc_ts || !d.out->arc_delay || !d.out->argmax || !d.nd->net_delay ||
                          !d.nd->net_imp2 || !d.nd->arc_load)))
            return fail(STA_E_ARG, "sta_batch_create: null buffer" + tag);
        if (d.sl && (!d.sl->tns || !d.sl->wns || !d.sl->drv_rat || !d.sl->drv_slack || (g->E > 0 && !d.ep_rat) ||
                     (g->A > 0 && (!d.sl->arc_rat || !d.sl->arc_slack))))
            return fail(STA_E_ARG, "sta_batch_create: null slack buffer" + tag);
    }
    BatchLayout L;
    if (!batch_layout(designs, n, NV, &L)) return fail(STA_E_ARG, "sta_batch_create: bad design list");
    if (!workspace || workspace_bytes < L.total)
        return fail(STA_E_ARG, "sta_batch_create: workspace smaller than sta_batch_workspace_bytes");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(STA_E_ARG, "sta_batch_create: workspace not 256-byte aligned");
    std::unique_ptr<sta_batch> b(new (std::nothrow) sta_batch());
    if (!b) return fail(STA_E_ALLOC, "sta_batch_create: out of host memory");
    b->NV = NV;
    b->bwd_nw = std::min(kBwdViewsPerWave, NV);
    b->kl = make_klib(lib);
    b->kv = kviews(views);
    b->lds = size_t(fwd_lds(lib->n_tables).total) * 4;
    const bool lds_ok = b->lds <= lds_limit();
    // items: the span designs first (the batched primary-input copy covers items
    // 0 .. n_span_items - 1), then the others
    std::vector<BatchItem> items;
    std::vector<int> order;                   // design index of each item
    std::vector<uint8_t> is_span;
    auto persistent_ok = [&](const sta_graph* g) { return lds_ok && g->L > 0 && g->n_fchunks > 0; };
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < n; ++i) {
            const sta_batch_design& d = designs[i];
            if (d.g->D == 0) continue;
            const bool span = d.schedule == STA_BATCH_SPANS || (d.schedule == STA_BATCH_PERSISTENT && !persistent_ok(d.g));
            if (span != (pass == 0)) continue;
            order.push_back(i);
            is_span.push_back(span ? 1 : 0);
        }
    b->n_items = int(order.size());
    int ep_part = 0;
    std::vector<std::pair<int64_t, int2>> units;
    for (int k = 0; k < b->n_items; ++k) {
        const sta_batch_design& d = designs[order[k]];
        const sta_graph* g = d.g;
        BatchItem it{};
        it.G = dev_graph(g);
        it.NC = g->n_fchunks;
        it.NV = NV;
        it.pi_ts = d.pi_ts;
        it.load = d.nd->load;
        it.nd = d.nd->net_delay;
        it.ni = d.nd->net_imp2;
        it.drv_ts = d.out->drv_ts;
        it.arc_ts = d.out->arc_ts;
        it.arc_delay = d.out->arc_delay;
        it.argmax = d.out->argmax;
        it.load_w = d.nd->load;
        it.nd_w = d.nd->net_delay;
        it.ni_w = d.nd->net_imp2;
        it.arc_load = d.nd->arc_load;
        it.E = int32_t(g->E);
        if (d.sl) {
            it.ep_rat = d.ep_rat;
            it.drv_rat = d.sl->drv_rat;
            it.arc_rat = d.sl->arc_rat;
            it.drv_slack = d.sl->drv_slack;
            it.arc_slack = d.sl->arc_slack;
            it.tns = d.sl->tns;
            it.wns = d.sl->wns;
            it.ep_blocks = batch_ep_blocks(g->E);
            it.ep_part0 = ep_part;
            ep_part += it.ep_blocks;
            ++b->n_slack_items;
        }
        items.push_back(it);
        b->graphs.push_back(g);
        b->nds.push_back(*d.nd);
        b->outs.push_back(*d.out);
        sta_slack_out so{};
        if (d.sl) so = *d.sl;
        b->sls.push_back(so);
        b->ep_rats.push_back(d.ep_rat);
        if (is_span[k]) {
            ++b->n_span_items;
        } else if (d.schedule == STA_BATCH_PERSISTENT) {
            for (int v = 0; v < NV; ++v) units.push_back({g->A + 64 * g->L, make_int2(k, v)});
            ++b->plan.persistent_designs;
        } else {
            b->level_designs.push_back({g, d.pi_ts, *d.nd, *d.out});
        }
    }
    std::stable_sort(units.begin(), units.end(),
                     [](const std::pair<int64_t, int2>& x, const std::pair<int64_t, int2>& y) { return x.first > y.first; });
    std::vector<int2> ulist;
    for (auto& u : units) ulist.push_back(u.second);
    b->n_units = int(ulist.size());
    // the tile maps: forward span steps, backward span steps, delay-calculation classes,
    // endpoint workgroups
    std::vector<int2> map;
    int64_t max_f = 0, max_b = 0;
    for (int k = 0; k < b->n_items; ++k) {
        if (is_span[k]) max_f = std::max<int64_t>(max_f, int64_t(b->graphs[k]->span_fused_h.size()));
        if (items[k].tns) max_b = std::max<int64_t>(max_b, int64_t(b->graphs[k]->bspan_fused_h.size()));
    }
    for (int64_t sp = 0; sp < max_f; ++sp) {
        sta_batch::Step st;
        st.map0 = int(map.size());
        for (int k = 0; k < b->n_items; ++k) {
            const sta_graph* g = b->graphs[k];
            if (!is_span[k] || sp >= int64_t(g->span_fused_h.size())) continue;
            if (g->span_fused_h[sp])
                for (int t = g->span_tile_h[sp]; t < g->span_tile_h[sp + 1]; ++t) map.push_back(make_int2(k, t));
            else
                st.levels.push_back({int64_t(k), int64_t(g->span_lv_h[2 * sp]), int64_t(g->span_lv_h[2 * sp + 1])});
        }
        st.nblk = int(map.size()) - st.map0;
        b->plan.fwd_span_tiles += st.nblk;
        b->fsteps.push_back(std::move(st));
    }
    for (int64_t sp = 0; sp < max_b; ++sp) {
        sta_batch::Step st;
        st.map0 = int(map.size());
        for (int k = 0; k < b->n_items; ++k) {
            const sta_graph* g = b->graphs[k];
            if (!items[k].tns || sp >= int64_t(g->bspan_fused_h.size())) continue;
            if (g->bspan_fused_h[sp])
                for (int t = g->bspan_tile_h[sp]; t < g->bspan_tile_h[sp + 1]; ++t) map.push_back(make_int2(k, t));
            else
                st.levels.push_back({int64_t(k), int64_t(g->bspan_lv_h[2 * sp]), int64_t(g->bspan_lv_h[2 * sp + 1])});
        }
        st.nblk = int(map.size()) - st.map0;
        b->plan.bwd_span_tiles += st.nblk;
        b->bsteps.push_back(std::move(st));
    }
    for (int maxn = 8; maxn <= 256; maxn *= 2) {
        sta_batch::DcClass dc;
        dc.maxn = maxn;
        dc.map0 = int(map.size());
        const int nt = dc_threads(maxn);
        for (int k = 0; k < b->n_items; ++k) {
            if (dc_class(b->graphs[k]) != maxn) continue;
            dc.chains = dc.chains && b->graphs[k]->chain_nets;
            const int64_t nb = dc_blocks_of(b->graphs[k]->D, b->graphs[k]->n_dc_wide, maxn, nt);
            for (int64_t x = 0; x < nb; ++x) map.push_back(make_int2(k, int(x)));
        }
        dc.nblk = int(map.size()) - dc.map0;
        if (dc.nblk > 0) b->dc.push_back(dc);
    }
    b->ep_map0 = int(map.size());
    for (int k = 0; k < b->n_items; ++k)
        for (int x = 0; x < items[k].ep_blocks; ++x) map.push_back(make_int2(k, x));
    b->ep_nblk = int(map.size()) - b->ep_map0;
    if (int64_t(map.size()) > L.n_map || ep_part > L.n_ep) return fail(STA_E_ARG, "sta_batch_create: inconsistent layout");
    uint8_t* base = static_cast<uint8_t*>(workspace);
    b->d_items = reinterpret_cast<BatchItem*>(base + L.items);
    b->d_units = reinterpret_cast<int2*>(base + L.units);
    b->d_counter = reinterpret_cast<int*>(base + L.counter);
    b->d_map = reinterpret_cast<int2*>(base + L.map);
    b->d_limbs = reinterpret_cast<unsigned long long*>(base + L.limbs);
    b->d_wns = reinterpret_cast<float*>(base + L.wns);
    hipError_t e = hipSuccess;
    if (!items.empty()) e = hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !ulist.empty())
        e = hipMemcpy(b->d_units, ulist.data(), sizeof(int2) * ulist.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !map.empty()) e = hipMemcpy(b->d_map, map.data(), sizeof(int2) * map.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(STA_E_HIP, std::string("sta_batch_create: hipMemcpy: ") + hipGetErrorString(e));
    b->plan.span_designs = b->n_span_items;
    b->plan.level_designs = int32_t(b->level_designs.size());
    b->plan.persistent_units = b->n_units;
    b->plan.fwd_steps = int32_t(b->fsteps.size());
    b->plan.bwd_steps = int32_t(b->bsteps.size());
    b->plan.slack_designs = b->n_slack_items;
    b->plan.dc_launches = int32_t(b->dc.size());
    if (b->n_units > 0 && b->n_span_items > 0) {
        e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (b->join) (void)hipEventDestroy(b->join);
            if (b->fork) (void)hipEventDestroy(b->fork);
            if (b->side) (void)hipStreamDestroy(b->side);
            return fail(STA_E_HIP, std::string("sta_batch_create: side stream: ") + hipGetErrorString(e));
        }
    }
    *out = b.release();
    return STA_OK;
}

sta_status sta_batch_delay_calc(sta_batch* b, sta_dc_precision prec, int32_t use_graph, void* stream) {
    if (!b) return fail(STA_E_ARG, "sta_batch_delay_calc: null batch");
    if (prec != STA_DC_FP64 && prec != STA_DC_FP32) return fail(STA_E_ARG, "sta_batch_delay_calc: unknown precision");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto enqueue = [&](hipStream_t q) {
        for (const auto& c : b->dc) {
            if (prec == STA_DC_FP64) launch_dc_batch<double>(b, c.maxn, c.chains, c.map0, c.nblk, q);
            else launch_dc_batch<float>(b, c.maxn, c.chains, c.map0, c.nblk, q);
        }
    };
    const sta_status st = capture_replay(b->dcache, b->mu, use_graph != 0, {uint64_t(prec)}, s, enqueue);
    if (st != STA_OK) return st;
    return launch_check("sta_batch_delay_calc");
}

sta_status sta_batch_propagate(sta_batch* b, int32_t use_graph, int32_t persistent_blocks, void* stream) {
    if (!b) return fail(STA_E_ARG, "sta_batch_propagate: null batch");
    if (persistent_blocks < 0) return fail(STA_E_ARG, "sta_batch_propagate: negative block count");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int blocks = persistent_blocks;
    if (blocks == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        blocks = cus;
    }
    if (blocks > b->n_units) blocks = b->n_units;
    // the persistent launch goes to the side stream when span steps run beside it (forked
    // after, and joined before, everything else of the sequence), else in line
    const bool fork = b->n_units > 0 && b->n_span_items > 0 && b->side;
    auto enqueue = [&](hipStream_t q) {
        hipStream_t qp = q;
        if (fork) {
            (void)hipEventRecord(b->fork, q);
            (void)hipStreamWaitEvent(b->side, b->fork, 0);
            qp = b->side;
        }
        if (b->n_units > 0) {
            prof_launch("k_zero_i32", qp, [&] { hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, qp, b->d_counter); });
            set_lds(k_forward_batch, b->lds);
            prof_launch("k_forward_batch", qp, [&] {
                hipLaunchKernelGGL(k_forward_batch, dim3(blocks), dim3(kViewThreads), b->lds, qp, b->d_items,
                                   b->d_units, b->n_units, b->d_counter, b->kl, b->kv);
            });
        }
        if (fork) (void)hipEventRecord(b->join, b->side);
        switch (b->NV) {
            case 1: enqueue_batch_forward<1>(b, q); break;
            case 2: enqueue_batch_forward<2>(b, q); break;
            case 4: enqueue_batch_forward<4>(b, q); break;
            default: enqueue_batch_forward<8>(b, q); break;
        }
        for (auto& d : b->level_designs) enqueue_levels_nv(b->NV, d.g, b->kl, b->kv, d.pi_ts, &d.nd, &d.out, q);
        if (fork) (void)hipStreamWaitEvent(q, b->join, 0);
    };
    const sta_status st = capture_replay(b->cache, b->mu, use_graph != 0, {uint64_t(blocks)}, s, enqueue);
    if (st != STA_OK) return st;
    return launch_check("sta_batch_propagate");
}

sta_status sta_batch_slack(sta_batch* b, int32_t use_graph, void* stream) {
    if (!b) return fail(STA_E_ARG, "sta_batch_slack: null batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto enqueue = [&](hipStream_t q) {
        switch (b->NV) {
            case 1: enqueue_batch_backward<1>(b, q); break;
            case 2: enqueue_batch_backward<2>(b, q); break;
            case 4: enqueue_batch_backward<4>(b, q); break;
            default: enqueue_batch_backward<8>(b, q); break;
        }
    };
    const sta_status st = capture_replay(b->bcache, b->mu, use_graph != 0, {uint64_t(1)}, s, enqueue);
    if (st != STA_OK) return st;
    return launch_check("sta_batch_slack");
}

sta_status sta_batch_set_tiling(sta_batch* b, int32_t fwd_views_per_wave, int32_t bwd_views_per_wave) {
    if (!b) return fail(STA_E_ARG, "sta_batch_set_tiling: null batch");
    auto ok = [&](int32_t w) { return (w == 1 || w == 2 || w == 4) && w <= b->NV; };
    if (!ok(fwd_views_per_wave) || !ok(bwd_views_per_wave))
        return fail(STA_E_ARG, "sta_batch_set_tiling: views per wavefront must be 1, 2 or 4 and at most the view count");
    std::lock_guard<std::mutex> lock(b->mu);
    if (b->fwd_nw != fwd_views_per_wave) drop_launches(b->cache);
    if (b->bwd_nw != bwd_views_per_wave) drop_launches(b->bcache);
    b->fwd_nw = fwd_views_per_wave;
    b->bwd_nw = bwd_views_per_wave;
    return STA_OK;
}

sta_status sta_batch_info(const sta_batch* b, sta_batch_plan* out) {
    if (!b || !out) return fail(STA_E_ARG, "sta_batch_info: null argument");
    *out = b->plan;
    return STA_OK;
}

void sta_batch_free(sta_batch* b) {
    if (!b) return;
    drop_launches(b->cache);
    drop_launches(b->bcache);
    drop_launches(b->dcache);
    if (b->side) {
        (void)hipStreamSynchronize(b->side);
        (void)hipEventDestroy(b->fork);
        (void)hipEventDestroy(b->join);
        (void)hipStreamDestroy(b->side);
    }
    delete b;
}

}  // extern "C"

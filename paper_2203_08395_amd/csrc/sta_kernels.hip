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
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "sta_internal.h"

namespace sta {

// ---------------------------------------------------------------------------------
// K1: RC delay calculation
// ---------------------------------------------------------------------------------

// Lane t of the block owns net (blockIdx.x*NT + t).  Node temporaries live in LDS,
// interleaved by lane: slot (k, t) at [k*NT + t].
template <typename T, int MAXN, int NT>
__global__ __launch_bounds__(NT) void k_delay_calc(DevGraph G, float* __restrict__ load,
                                                   float* __restrict__ net_delay,
                                                   float* __restrict__ net_imp2) {
    __shared__ T sA[MAXN * NT];   // C, later m2
    __shared__ T sB[MAXN * NT];   // Cd, later W
    __shared__ T sM[MAXN * NT];   // m1
    const int t = threadIdx.x;
    const int d = blockIdx.x * NT + t;
    if (d >= G.n_drivers) return;
    const int n0 = G.net_node_ptr[d];
    const int nm = G.net_node_ptr[d + 1] - n0;
    const int16_t* par = G.node_parent + n0;
    const float* R = G.node_R + n0;
    const float* Cw = G.node_C + n0;
    T* A = sA + t;
    T* B = sB + t;
    T* Mm = sM + t;
#define AT_(arr, k) arr[(k) * NT]
    for (int k = 0; k < nm; ++k) AT_(A, k) = static_cast<T>(Cw[k]);
    const int f0 = G.fo_ptr[d], f1 = G.fo_ptr[d + 1];
    for (int e = f0; e < f1; ++e) AT_(A, G.fo_tap[e]) += static_cast<T>(G.fo_cap[e]);
    for (int k = 0; k < nm; ++k) AT_(B, k) = AT_(A, k);
    for (int k = nm - 1; k >= 1; --k) AT_(B, par[k]) += AT_(B, k);
    load[d] = static_cast<float>(AT_(B, 0));
    const T milli = static_cast<T>(1e-3);
    AT_(Mm, 0) = T(0);
    for (int k = 1; k < nm; ++k) AT_(Mm, k) = AT_(Mm, par[k]) + (static_cast<T>(R[k]) * AT_(B, k)) * milli;
    for (int k = 0; k < nm; ++k) AT_(B, k) = AT_(A, k) * AT_(Mm, k);
    for (int k = nm - 1; k >= 1; --k) AT_(B, par[k]) += AT_(B, k);
    AT_(A, 0) = T(0);
    for (int k = 1; k < nm; ++k) AT_(A, k) = AT_(A, par[k]) + (static_cast<T>(R[k]) * AT_(B, k)) * milli;
    for (int e = f0; e < f1; ++e) {
        const int k = G.fo_tap[e];
        const int a = G.fo_arc[e];
        const T m1 = AT_(Mm, k);
        T imp2 = T(2) * AT_(A, k) - m1 * m1;
        if (imp2 < T(0)) imp2 = T(0);
        net_delay[a] = static_cast<float>(m1);
        net_imp2[a] = static_cast<float>(imp2);
    }
#undef AT_
}

// ---------------------------------------------------------------------------------
// NLDM lookup helpers
// ---------------------------------------------------------------------------------

struct KLib {
    float ax[26];                // x[7], y[7], dx[6] = fl32(x[i+1]-x[i]), dy[6]
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

__device__ __forceinline__ float bilerp(const float* T, int i, int j, float tx, float ty) {
    const float t00 = T[i * 7 + j], t01 = T[i * 7 + j + 1];
    const float t10 = T[(i + 1) * 7 + j], t11 = T[(i + 1) * 7 + j + 1];
    const float p = t00 + tx * (t10 - t00);
    const float q = t01 + tx * (t11 - t01);
    return p + ty * (q - p);
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

// arc arithmetic, per-gate max/argmax (min for early views) and the writes
template <int NW>
__device__ __forceinline__ void fwd_finish(const FwdLane& x, const float2* ts, const float* s_ax,
                                           const float* const* tab, const bool* early, int NV, int v0, int n_pi,
                                           float* __restrict__ drv_ts, float* __restrict__ arc_ts,
                                           float* __restrict__ arc_delay, uint8_t* __restrict__ argmax) {
    const float* X = s_ax;
    const float* Y = s_ax + 7;
    const float* DX = s_ax + 14;
    const float* DY = s_ax + 20;
    const int lane = threadIdx.x & 63;
    float cand[NW], slw[NW];
    int best_k[NW];
    if (x.active) {
        const int j = seg6(Y, x.Lo);
        const float ty = (x.Lo - Y[j]) / DY[j];
        float2* dst = reinterpret_cast<float2*>(arc_ts) + size_t(x.a) * NV + v0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const float ai = ts[w].x + x.nd;
            const float su2 = ts[w].y * ts[w].y;
            const float si = sqrtf(su2 + x.ni);
            const int i = seg6(X, si);
            const float tx = (si - X[i]) / DX[i];
            const float* T = tab[w] + size_t(x.tb) * 98;
            const float dl = bilerp(T, i, j, tx, ty);
            const float sl = bilerp(T + 49, i, j, tx, ty);
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
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
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
    // segment = lanes of one driver: heads from the slot flags (c == 1) or lane 0 (c > 1)
    const uint64_t heads = __ballot(head);
    const uint64_t le = lanes_le(lane);
    const int gi = __popcll(heads & le) - 1;
    const uint64_t after = heads & ~le;
    const int nl = (n + c - 1) / c;               // lanes holding slots
    const int seg_end = after ? (__ffsll(static_cast<unsigned long long>(after)) - 1) : nl;
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
        const float2* ts = reinterpret_cast<const float2*>(drv_ts) + size_t(u) * NV + v0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const float r = best[w];
            const float at = ts[w].x;
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

size_t scratch_bytes() {
    return size_t(kK4Blocks) * STA_MAX_VIEWS * kLimbs * 8 + size_t(kK4Blocks) * STA_MAX_VIEWS * 4;
}

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

// Level schedule, forward: 4 tiles per 256-lane block.  The block first issues its
// tiles' arc loads, then copies the view tables into LDS (TAB_LDS: every view reads the
// same table set), then gathers the drivers' results and computes.
template <int NV, bool TAB_LDS>
__global__ __launch_bounds__(256) void k_forward(DevGraph G, KLib lib, KViews V, int tile0, int tile1, KTiles kt,
                                                 const float* __restrict__ load, const float* __restrict__ nd,
                                                 const float* __restrict__ ni, float* __restrict__ drv_ts,
                                                 float* __restrict__ arc_ts, float* __restrict__ arc_delay,
                                                 uint8_t* __restrict__ argmax) {
    extern __shared__ float s_dyn[];
    __shared__ float s_ax[26];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = tile0 + blockIdx.x * 4 + wave;
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
    const uint32_t meta = act ? G.arc_meta[a] : 0u;
    const int u = act ? G.arc_src[a] : 0;
    FwdLane x;
    x.nd = act ? nd[a] : 0.0f;
    x.ni = act ? ni[a] : 0.0f;
    load_axes(s_ax, lib);
    if (TAB_LDS) {
        const float* gt = lib.tables + size_t(V.set[0]) * lib.n_tables * 98;
        const int nt = lib.n_tables * 98;
        int done = 0;
        if ((reinterpret_cast<uintptr_t>(gt) & 15u) == 0) {
            const float4* src = reinterpret_cast<const float4*>(gt);
            float4* dst = reinterpret_cast<float4*>(s_dyn);
            done = (nt / 4) * 4;
            for (int i = threadIdx.x; i < nt / 4; i += 256) dst[i] = src[i];
        }
        for (int i = done + threadIdx.x; i < nt; i += 256) s_dyn[i] = gt[i];
    }
    __syncthreads();
    if (!valid) return;
    fwd_lane_setup(x, act, meta, n, lane);
    x.a = a;
    x.g = g0 + x.gi;
    x.Lo = act ? load[G.n_pi + x.g] : 0.0f;
    float2 ts[NV];
    const float2* srcp = reinterpret_cast<const float2*>(drv_ts) + size_t(u) * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) ts[v] = act ? srcp[v] : make_float2(0.0f, 0.0f);
    const float* tab[NV];
    bool early[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        tab[v] = TAB_LDS ? s_dyn : lib.tables + size_t(V.set[v]) * lib.n_tables * 98;
        early[v] = V.mode[v] == STA_EARLY;
    }
    fwd_finish<NV>(x, ts, s_ax, tab, early, NV, 0, G.n_pi, drv_ts, arc_ts, arc_delay, argmax);
}

// primary inputs: copy (arrival, slew) of every view
__global__ void k_copy_pi(const float* __restrict__ pi_ts, float* __restrict__ drv_ts, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) drv_ts[i] = pi_ts[i];
}

template <int NV>
__global__ __launch_bounds__(256) void k_backward(DevGraph G, KViews V, int tile0, int tile1, KTiles kt,
                                                  const float* __restrict__ nd, const float* __restrict__ drv_ts,
                                                  const float* __restrict__ arc_ts,
                                                  const float* __restrict__ arc_delay,
                                                  const float* __restrict__ ep_rat, float* __restrict__ drv_rat,
                                                  float* __restrict__ arc_rat, float* __restrict__ drv_slack,
                                                  float* __restrict__ arc_slack) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = tile0 + blockIdx.x * 4 + wave;
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

template <int NV>
__global__ __launch_bounds__(kK4Threads) void k_endpoint_partial(const int32_t* __restrict__ ep_drv, int E,
                                                                 const float* __restrict__ drv_slack,
                                                                 unsigned long long* __restrict__ part_limbs,
                                                                 float* __restrict__ part_wns) {
    __shared__ unsigned long long s_l[NV * kLimbs];
    __shared__ float s_min[NV][kK4Threads / 64];
    for (int i = threadIdx.x; i < NV * kLimbs; i += blockDim.x) s_l[i] = 0ull;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        unsigned long long l[kLimbs];
#pragma unroll
        for (int i = 0; i < kLimbs; ++i) l[i] = 0ull;
        float mn = __builtin_inff();
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
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
    if (threadIdx.x < NV * kLimbs) part_limbs[size_t(blockIdx.x) * NV * kLimbs + threadIdx.x] = s_l[threadIdx.x];
    if (threadIdx.x < NV) {
        float mn = s_min[threadIdx.x][0];
        for (int i = 1; i < kK4Threads / 64; ++i) mn = (s_min[threadIdx.x][i] < mn) ? s_min[threadIdx.x][i] : mn;
        part_wns[size_t(blockIdx.x) * NV + threadIdx.x] = mn;
    }
}

template <int NV>
__global__ __launch_bounds__(256) void k_endpoint_final(int nblk, const unsigned long long* __restrict__ part_limbs,
                                                        const float* __restrict__ part_wns, double* __restrict__ tns,
                                                        float* __restrict__ wns) {
    __shared__ unsigned long long s_sum[NV * kLimbs];
    __shared__ float s_min[NV][4];
    for (int i = threadIdx.x; i < NV * kLimbs; i += blockDim.x) s_sum[i] = 0ull;
    __syncthreads();
    for (int i = threadIdx.x; i < nblk * NV * kLimbs; i += blockDim.x) {
        const unsigned long long x = part_limbs[i];
        if (x) atomicAdd(&s_sum[i % (NV * kLimbs)], x);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        float mn = __builtin_inff();
        for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
            const float x = part_wns[size_t(b) * NV + v];
            mn = (x < mn) ? x : mn;
        }
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

// LDS layout of k_forward_view (in 4-byte words)
struct FwdLds {
    int ax, tab, lvl, taoff, tgoff, src, meta, nd, ni, ld, total;
};

__host__ __device__ inline FwdLds fwd_lds(int n_tables, int L, int capT, int capA, int capG) {
    FwdLds o{};
    o.ax = 0;
    o.tab = 32;
    o.lvl = o.tab + n_tables * 98;
    o.taoff = o.lvl + (L + 2) * 3;
    o.tgoff = o.taoff + capT + 1;
    o.src = o.tgoff + capT;
    o.meta = o.src + capA;
    o.nd = o.meta + capA;
    o.ni = o.nd + capA;
    o.ld = o.ni + capA;
    o.total = o.ld + capG;
    return o;
}

template <int RW>
__global__ __launch_bounds__(kViewThreads) void k_forward_view(DevGraph G, KLib lib, KViews V, int NV, int L,
                                                               const int32_t* __restrict__ lvl_g, int capT, int capA,
                                                               int capG, const float* __restrict__ pi_ts,
                                                               const float* __restrict__ load,
                                                               const float* __restrict__ nd,
                                                               const float* __restrict__ ni,
                                                               float* __restrict__ drv_ts, float* __restrict__ arc_ts,
                                                               float* __restrict__ arc_delay,
                                                               uint8_t* __restrict__ argmax) {
    extern __shared__ float s_mem[];
    const FwdLds lo = fwd_lds(lib.n_tables, L, capT, capA, capG);
    float* s_ax = s_mem + lo.ax;
    float* s_tab = s_mem + lo.tab;
    int* s_lvl = reinterpret_cast<int*>(s_mem + lo.lvl);
    int* s_taoff = reinterpret_cast<int*>(s_mem + lo.taoff);
    int* s_tgoff = reinterpret_cast<int*>(s_mem + lo.tgoff);
    int* s_src = reinterpret_cast<int*>(s_mem + lo.src);
    uint32_t* s_meta = reinterpret_cast<uint32_t*>(s_mem + lo.meta);
    float* s_nd = s_mem + lo.nd;
    float* s_ni = s_mem + lo.ni;
    float* s_ld = s_mem + lo.ld;
    const int v = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const float* gtab = lib.tables + size_t(V.set[v]) * lib.n_tables * 98;
    load_axes(s_ax, lib);
    for (int i = tid; i < lib.n_tables * 98; i += kViewThreads) s_tab[i] = gtab[i];
    for (int i = tid; i < (L + 2) * 3; i += kViewThreads) s_lvl[i] = lvl_g[i];
    for (int i = tid; i < G.n_pi; i += kViewThreads)
        reinterpret_cast<float2*>(drv_ts)[size_t(i) * NV + v] = reinterpret_cast<const float2*>(pi_ts)[size_t(i) * NV + v];
    const bool early[1] = {V.mode[v] == STA_EARLY};
    const float* tab[1] = {s_tab};
    __syncthreads();

    // static data of level l into registers (coalesced), then into LDS
    int p_src[RW], p_ld_n = 0;
    uint32_t p_meta[RW];
    float p_nd[RW], p_ni[RW], p_ld[RW];
    int p_ta = 0, p_tg = 0;
    auto fetch = [&](int l) {
        const int t0 = s_lvl[l * 3], t1 = s_lvl[(l + 1) * 3];
        const int al = s_lvl[l * 3 + 1], ah = s_lvl[(l + 1) * 3 + 1];
        const int gl = s_lvl[l * 3 + 2], gh = s_lvl[(l + 1) * 3 + 2];
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int i = tid + k * kViewThreads;
            const bool ok = i < ah - al;
            p_src[k] = ok ? G.arc_src[al + i] : 0;
            p_meta[k] = ok ? G.arc_meta[al + i] : 0u;
            p_nd[k] = ok ? nd[al + i] : 0.0f;
            p_ni[k] = ok ? ni[al + i] : 0.0f;
            p_ld[k] = (i < gh - gl) ? load[G.n_pi + gl + i] : 0.0f;
        }
        p_ta = (tid <= t1 - t0) ? G.ftile_arc[t0 + tid] - al : 0;
        p_tg = (tid < t1 - t0) ? G.ftile_gate[t0 + tid] - gl : 0;
        p_ld_n = 0;
    };
    auto stash = [&](int l) {
        const int t0 = s_lvl[l * 3], t1 = s_lvl[(l + 1) * 3];
        const int al = s_lvl[l * 3 + 1], ah = s_lvl[(l + 1) * 3 + 1];
        const int gl = s_lvl[l * 3 + 2], gh = s_lvl[(l + 1) * 3 + 2];
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int i = tid + k * kViewThreads;
            if (i < ah - al) { s_src[i] = p_src[k]; s_meta[i] = p_meta[k]; s_nd[i] = p_nd[k]; s_ni[i] = p_ni[k]; }
            if (i < gh - gl) s_ld[i] = p_ld[k];
        }
        if (tid <= t1 - t0) s_taoff[tid] = p_ta;
        if (tid < t1 - t0) s_tgoff[tid] = p_tg;
    };
    if (L >= 1) {
        fetch(1);
        stash(1);
    }
    (void)p_ld_n;
    __syncthreads();

    for (int l = 1; l <= L; ++l) {
        const int T = s_lvl[(l + 1) * 3] - s_lvl[l * 3];
        const int al = s_lvl[l * 3 + 1], gl = s_lvl[l * 3 + 2];
        // this wave's tiles: LDS reads, then every gather
        FwdLane x[RW];
        float2 ts[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int tl = wave + r * kViewWaves;
            const bool valid = tl < T;
            const int a_off = valid ? s_taoff[tl] : 0;
            const int n = valid ? s_taoff[tl + 1] - a_off : 0;
            const int g_off = valid ? s_tgoff[tl] : 0;
            const bool act = lane < n;
            const int ai = a_off + lane;
            const uint32_t meta = act ? s_meta[ai] : 0u;
            fwd_lane_setup(x[r], act, meta, n, lane);
            x[r].a = al + ai;
            x[r].g = gl + g_off + x[r].gi;
            x[r].nd = act ? s_nd[ai] : 0.0f;
            x[r].ni = act ? s_ni[ai] : 0.0f;
            x[r].Lo = act ? s_ld[g_off + x[r].gi] : 0.0f;
            const int u = act ? s_src[ai] : 0;
            ts[r] = act ? reinterpret_cast<const float2*>(drv_ts)[size_t(u) * NV + v] : make_float2(0.0f, 0.0f);
        }
        if (l < L) fetch(l + 1);
#pragma unroll
        for (int r = 0; r < RW; ++r)
            fwd_finish<1>(x[r], &ts[r], s_ax, tab, early, NV, v, G.n_pi, drv_ts, arc_ts, arc_delay, argmax);
        __syncthreads();
        if (l < L) stash(l + 1);
        __syncthreads();
    }
}

// LDS layout of k_backward_view (in 4-byte words)
struct BwdLds {
    int lvl, tsoff, tdoff, sa, so, at, lim, mn, total;
};

__host__ __device__ inline BwdLds bwd_lds(int L, int capT, int capS, int capD) {
    BwdLds o{};
    o.lvl = 0;
    o.tsoff = o.lvl + (L + 2) * 3;
    o.tdoff = o.tsoff + capT + 1;
    o.sa = o.tdoff + capT;
    o.so = o.sa + capS;
    o.at = o.so + capS;
    o.lim = ((o.at + capD) + 1) & ~1;              // 8-byte aligned digits
    o.mn = o.lim + 2 * kLimbs;
    o.total = o.mn + kViewWaves;
    return o;
}

template <int RW>
__global__ __launch_bounds__(kViewThreads) void k_backward_view(DevGraph G, KViews V, int NV, int L, int E,
                                                                const int32_t* __restrict__ lvl_g, int capT, int capS,
                                                                int capD, const float* __restrict__ nd,
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
    const BwdLds lo = bwd_lds(L, capT, capS, capD);
    int* s_lvl = reinterpret_cast<int*>(s_mem + lo.lvl);
    int* s_tsoff = reinterpret_cast<int*>(s_mem + lo.tsoff);
    int* s_tdoff = reinterpret_cast<int*>(s_mem + lo.tdoff);
    int* s_sa = reinterpret_cast<int*>(s_mem + lo.sa);
    int* s_so = reinterpret_cast<int*>(s_mem + lo.so);
    float* s_at = s_mem + lo.at;
    unsigned long long* s_l = reinterpret_cast<unsigned long long*>(s_mem + lo.lim);
    float* s_min = s_mem + lo.mn;
    const int v = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const bool early = V.mode[v] == STA_EARLY;
    for (int i = tid; i < (L + 2) * 3; i += kViewThreads) s_lvl[i] = lvl_g[i];
    if (tid < kLimbs) s_l[tid] = 0ull;
    __syncthreads();

    int p_sa[RW], p_so[RW];
    float p_at[RW];
    int p_ts = 0, p_td = 0;
    auto fetch = [&](int l) {
        const int t0 = s_lvl[l * 3], t1 = s_lvl[(l + 1) * 3];
        const int sl = s_lvl[l * 3 + 1], sh = s_lvl[(l + 1) * 3 + 1];
        const int dl = s_lvl[l * 3 + 2], dh = s_lvl[(l + 1) * 3 + 2];
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int i = tid + k * kViewThreads;
            const bool ok = i < sh - sl;
            p_sa[k] = ok ? G.bslot_arc[sl + i] : 0;
            p_so[k] = ok ? G.bslot_out[sl + i] : 0;
            p_at[k] = (i < dh - dl) ? drv_ts[(size_t(dl + i) * NV + v) * 2] : 0.0f;
        }
        p_ts = (tid <= t1 - t0) ? G.btile_slot[t0 + tid] - sl : 0;
        p_td = (tid < t1 - t0) ? G.btile_drv[t0 + tid] - dl : 0;
    };
    auto stash = [&](int l) {
        const int t0 = s_lvl[l * 3], t1 = s_lvl[(l + 1) * 3];
        const int sl = s_lvl[l * 3 + 1], sh = s_lvl[(l + 1) * 3 + 1];
        const int dl = s_lvl[l * 3 + 2], dh = s_lvl[(l + 1) * 3 + 2];
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int i = tid + k * kViewThreads;
            if (i < sh - sl) { s_sa[i] = p_sa[k]; s_so[i] = p_so[k]; }
            if (i < dh - dl) s_at[i] = p_at[k];
        }
        if (tid <= t1 - t0) s_tsoff[tid] = p_ts;
        if (tid < t1 - t0) s_tdoff[tid] = p_td;
    };
    fetch(L);
    stash(L);
    __syncthreads();

    for (int l = L; l >= 0; --l) {
        const int T = s_lvl[(l + 1) * 3] - s_lvl[l * 3];
        const int dl = s_lvl[l * 3 + 2];
        // one-slot-per-lane tiles: every gather first
        float ro[RW], dlv[RW], ati[RW], ndv[RW], epr[RW];
        int sa_r[RW];
        bool big[RW], act[RW], head[RW];
        int s0r[RW], nr[RW], doff[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int tl = wave + r * kViewWaves;
            const bool valid = tl < T;
            s0r[r] = valid ? s_tsoff[tl] : 0;
            nr[r] = valid ? s_tsoff[tl + 1] - s0r[r] : 0;
            doff[r] = valid ? s_tdoff[tl] : 0;
            big[r] = nr[r] > 64;
            act[r] = !big[r] && lane < nr[r];
            const int si = s0r[r] + lane;
            const int sa = act[r] ? s_sa[si] : -1;
            const int so = act[r] ? s_so[si] : 0;
            head[r] = act[r] && (uint32_t(so) & kHeadBit) != 0u;
            const int o = so & 0x7fffffff;
            sa_r[r] = sa;
            ro[r] = (sa >= 0) ? drv_rat[size_t(o) * NV + v] : 0.0f;
            dlv[r] = (sa >= 0) ? arc_delay[size_t(sa) * NV + v] : 0.0f;
            ati[r] = (sa >= 0) ? arc_ts[(size_t(sa) * NV + v) * 2] : 0.0f;
            ndv[r] = (sa >= 0) ? nd[sa] : 0.0f;
            epr[r] = (act[r] && sa < 0) ? ep_rat[size_t(o) * NV + v] : 0.0f;
        }
        if (l > 0) fetch(l - 1);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            if (big[r]) {
                // one driver with more than 64 sinks: lanes take contiguous runs of them
                const int n = nr[r], c = (n + 63) >> 6, sb = lane * c, se = min(n, sb + c);
                float best = 0.0f;
                bool have = false;
                for (int s = sb; s < se; ++s) {
                    const int sa = s_sa[s0r[r] + s];
                    const int o = s_so[s0r[r] + s] & 0x7fffffff;
                    const float rin = drv_rat[size_t(o) * NV + v] - arc_delay[size_t(sa) * NV + v];
                    const float at_i = arc_ts[(size_t(sa) * NV + v) * 2];
                    arc_rat[size_t(sa) * NV + v] = rin;
                    arc_slack[size_t(sa) * NV + v] = early ? (at_i - rin) : (rin - at_i);
                    const float val = rin - nd[sa];
                    if (!have || (early ? (val > best) : (val < best))) best = val;
                    have = true;
                }
                const int nl = (n + c - 1) / c;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const float b2 = __shfl_down(best, off, 64);
                    if ((lane + off) < nl && (early ? (b2 > best) : (b2 < best))) best = b2;
                }
                if (lane == 0) {
                    const int u = dl + doff[r];
                    const float at = s_at[doff[r]];
                    drv_rat[size_t(u) * NV + v] = best;
                    drv_slack[size_t(u) * NV + v] = early ? (at - best) : (best - at);
                }
                continue;
            }
            float val = 0.0f;
            if (sa_r[r] >= 0) {
                const int sa = sa_r[r];
                const float rin = ro[r] - dlv[r];
                arc_rat[size_t(sa) * NV + v] = rin;
                arc_slack[size_t(sa) * NV + v] = early ? (ati[r] - rin) : (rin - ati[r]);
                val = rin - ndv[r];
            } else if (act[r]) {
                val = epr[r];
            }
            const uint64_t heads = __ballot(head[r]);
            const uint64_t le = lanes_le(lane);
            const int gi = __popcll(heads & le) - 1;
            const uint64_t after = heads & ~le;
            const int seg_end = after ? (__ffsll(static_cast<unsigned long long>(after)) - 1) : nr[r];
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const float b2 = __shfl_down(val, off, 64);
                if ((lane + off) < seg_end && (early ? (b2 > val) : (b2 < val))) val = b2;
            }
            if (head[r]) {
                const int dloc = doff[r] + gi;
                const int u = dl + dloc;
                const float at = s_at[dloc];
                drv_rat[size_t(u) * NV + v] = val;
                drv_slack[size_t(u) * NV + v] = early ? (at - val) : (val - at);
            }
        }
        __syncthreads();
        if (l > 0) stash(l - 1);
        __syncthreads();
    }
    // endpoint summaries of this view
    unsigned long long lim[kLimbs];
#pragma unroll
    for (int i = 0; i < kLimbs; ++i) lim[i] = 0ull;
    float mn = __builtin_inff();
    for (int e = tid; e < E; e += kViewThreads) {
        const float s = drv_slack[size_t(G.ep_drv[e]) * NV + v];
        mn = (s < mn) ? s : mn;
        add_neg_slack(lim, s);
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

// Optional per-launch HIP-event bracketing (instrumentation only).
struct ProfRec {
    const char* name;
    hipEvent_t start, stop;
};
struct Prof {
    bool on = false;
    bool failed = false;
    std::vector<ProfRec> recs;
};
static thread_local Prof g_prof;

template <typename F>
static void prof_launch(const char* name, hipStream_t s, F&& launch) {
    if (!g_prof.on) {
        launch();
        return;
    }
    ProfRec r{name, nullptr, nullptr};
    if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) {
        g_prof.failed = true;
        launch();
        return;
    }
    hipEventRecord(r.start, s);
    launch();
    hipEventRecord(r.stop, s);
    g_prof.recs.push_back(r);
}

static sta_status launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(STA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return STA_OK;
}

template <typename T, int MAXN, int NT>
static void launch_dc(const sta_graph* g, const sta_net_out* out, hipStream_t s) {
    const int blocks = int((g->D + NT - 1) / NT);
    prof_launch("k_delay_calc", s, [&] {
        hipLaunchKernelGGL((k_delay_calc<T, MAXN, NT>), dim3(blocks), dim3(NT), 0, s, dev_graph(g), out->load,
                           out->net_delay, out->net_imp2);
    });
}

template <typename T>
static void dispatch_dc(const sta_graph* g, const sta_net_out* out, hipStream_t s) {
    // node temporaries: 3 * MAXN * NT values of T per block (48 KB for FP64)
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

// Per-wave tile count of the view schedule (1, 2, 4 or 8; 0 = does not fit), from the
// widest level: 16 waves, <= 64 arcs or slots per tile and per staged lane load.
static int view_rw(int max_tiles, int max_items) {
    const int need = std::max((max_tiles + kViewWaves - 1) / kViewWaves, (max_items + kViewThreads - 1) / kViewThreads);
    for (int rw = 1; rw <= 8; rw *= 2)
        if (need <= rw) return rw;
    return 0;
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
// data and the view's tables fit in LDS.
static bool use_view_forward(const sta_graph* g, int n_tables, int* rw, size_t* lds) {
    if (g->L == 0 || double(g->A) / double(g->L) > double(g->view_sched_max_arcs)) return false;
    *rw = view_rw(g->max_ft, std::max(g->max_fa, g->max_fg));
    if (!*rw) return false;
    *lds = size_t(fwd_lds(n_tables, int(g->L), g->max_ft, g->max_fa, g->max_fg).total) * 4;
    return *lds <= lds_limit();
}

static bool use_view_backward(const sta_graph* g, int* rw, size_t* lds) {
    if (g->L == 0 || double(g->A) / double(g->L) > double(g->view_sched_max_arcs)) return false;
    *rw = view_rw(g->max_bt, std::max(g->max_bs, g->max_bd));
    if (!*rw) return false;
    *lds = size_t(bwd_lds(int(g->L), g->max_bt, g->max_bs, g->max_bd).total) * 4;
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
// kind (capturing it first when the key differs).  Profiling always runs it directly.
template <typename F>
static sta_status run_sequence(const sta_graph* g, LaunchCache& c, std::vector<uint64_t> key, hipStream_t s,
                               F&& enqueue) {
    if (!g->use_graphs || g_prof.on) {
        enqueue(s);
        return STA_OK;
    }
    std::lock_guard<std::mutex> lock(g->cache_mu);
    if (!c.exec || c.key != key) {
        if (c.exec) { (void)hipGraphExecDestroy(c.exec); c.exec = nullptr; }
        if (c.graph) { (void)hipGraphDestroy(c.graph); c.graph = nullptr; }
        c.key.clear();
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
        c.graph = gr;
        c.exec = ex;
        c.key = std::move(key);
    }
    hipError_t e = hipGraphLaunch(c.exec, s);
    if (e != hipSuccess) return fail(STA_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return STA_OK;
}

static uint64_t pk(const void* p) { return uint64_t(reinterpret_cast<uintptr_t>(p)); }

template <int NV, bool TAB_LDS>
static void enqueue_forward_levels(const sta_graph* g, const KLib& lib, const KViews& kv, const float* pi_ts,
                                   const sta_net_out* nd, const sta_timing_out* o, hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    const int npi = int(g->n_pi) * NV * 2;
    const size_t lds = TAB_LDS ? size_t(lib.n_tables) * 98 * 4 : 0;
    if (TAB_LDS) set_lds(k_forward<NV, TAB_LDS>, lds);
    if (npi > 0)
        prof_launch("k_copy_pi", s, [&] {
            hipLaunchKernelGGL(k_copy_pi, dim3((npi + 255) / 256), dim3(256), 0, s, pi_ts, o->drv_ts, npi);
        });
    for (int64_t l = 1; l <= g->L; ++l) {
        const int t0 = g->fwd_tile_ptr[l], t1 = g->fwd_tile_ptr[l + 1];
        if (t1 <= t0) continue;
        const KTiles kt = ktiles(g->ftile_arc_h, g->ftile_gate_h, t0, t1);
        prof_launch("k_forward", s, [&] {
            hipLaunchKernelGGL((k_forward<NV, TAB_LDS>), dim3((t1 - t0 + 3) / 4), dim3(256), lds, s, dg, lib, kv, t0,
                               t1, kt, nd->load, nd->net_delay, nd->net_imp2, o->drv_ts, o->arc_ts, o->arc_delay,
                               o->argmax);
        });
    }
}

template <int NV>
static sta_status run_forward_levels(const sta_graph* g, const KLib& lib, const KViews& kv, const float* pi_ts,
                                     const sta_net_out* nd, const sta_timing_out* o, hipStream_t s) {
    bool same_set = true;
    for (int v = 1; v < NV; ++v) same_set = same_set && kv.set[v] == kv.set[0];
    // Copying the tables into every block's LDS costs more than the L2-resident global
    // reads it replaces (one level is ~10 blocks that each use a few hundred entries).
    const bool tab_lds = false;
    (void)same_set;
    std::vector<uint64_t> key = {uint64_t(NV), pk(lib.tables), uint64_t(lib.n_tables), pk(pi_ts), pk(nd->load),
                                 pk(nd->net_delay), pk(nd->net_imp2), pk(o->drv_ts), pk(o->arc_ts), pk(o->arc_delay),
                                 pk(o->argmax), uint64_t(tab_lds)};
    for (int i = 0; i < 26; ++i) { uint32_t b; std::memcpy(&b, &lib.ax[i], 4); key.push_back(b); }
    for (int v = 0; v < NV; ++v) key.push_back((uint64_t(kv.mode[v]) << 32) | uint32_t(kv.set[v]));
    return run_sequence(g, g->fwd_cache, std::move(key), s, [&](hipStream_t q) {
        if (tab_lds) enqueue_forward_levels<NV, true>(g, lib, kv, pi_ts, nd, o, q);
        else enqueue_forward_levels<NV, false>(g, lib, kv, pi_ts, nd, o, q);
    });
}

template <int RW>
static void launch_forward_view(const sta_graph* g, int NV, const KLib& lib, const KViews& kv, const float* pi_ts,
                                const sta_net_out* nd, const sta_timing_out* o, size_t lds, hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    const int32_t* lv = reinterpret_cast<const int32_t*>(g->dev + g->lay.fwd_lvl);
    set_lds(k_forward_view<RW>, lds);
    prof_launch("k_forward_view", s, [&] {
        hipLaunchKernelGGL((k_forward_view<RW>), dim3(NV), dim3(kViewThreads), lds, s, dg, lib, kv, NV, int(g->L), lv,
                           g->max_ft, g->max_fa, g->max_fg, pi_ts, nd->load, nd->net_delay, nd->net_imp2, o->drv_ts,
                           o->arc_ts, o->arc_delay, o->argmax);
    });
}

static void run_forward_views(const sta_graph* g, int rw, size_t lds, int NV, const KLib& lib, const KViews& kv,
                              const float* pi_ts, const sta_net_out* nd, const sta_timing_out* o, hipStream_t s) {
    switch (rw) {
        case 1: launch_forward_view<1>(g, NV, lib, kv, pi_ts, nd, o, lds, s); break;
        case 2: launch_forward_view<2>(g, NV, lib, kv, pi_ts, nd, o, lds, s); break;
        case 4: launch_forward_view<4>(g, NV, lib, kv, pi_ts, nd, o, lds, s); break;
        default: launch_forward_view<8>(g, NV, lib, kv, pi_ts, nd, o, lds, s); break;
    }
}

template <int NV>
static void enqueue_backward_levels(const sta_graph* g, const KViews& kv, const sta_net_out* nd,
                                    const sta_timing_out* t, const float* ep_rat, const sta_slack_out* o,
                                    void* scratch, hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    for (int64_t l = g->L; l >= 0; --l) {
        const int t0 = g->bwd_tile_ptr[l], t1 = g->bwd_tile_ptr[l + 1];
        if (t1 <= t0) continue;
        const KTiles kt = ktiles(g->btile_slot_h, g->btile_drv_h, t0, t1);
        prof_launch("k_backward", s, [&] {
            hipLaunchKernelGGL((k_backward<NV>), dim3((t1 - t0 + 3) / 4), dim3(256), 0, s, dg, kv, t0, t1, kt,
                               nd->net_delay, t->drv_ts, t->arc_ts, t->arc_delay, ep_rat, o->drv_rat, o->arc_rat,
                               o->drv_slack, o->arc_slack);
        });
    }
    int nblk = int((g->E + kK4Threads - 1) / kK4Threads);
    nblk = nblk < 1 ? 1 : (nblk > kK4Blocks ? kK4Blocks : nblk);
    auto* limbs = static_cast<unsigned long long*>(scratch);
    auto* pw = reinterpret_cast<float*>(static_cast<uint8_t*>(scratch) + size_t(kK4Blocks) * STA_MAX_VIEWS * kLimbs * 8);
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
    std::vector<uint64_t> key = {uint64_t(NV), pk(nd->net_delay), pk(t->drv_ts), pk(t->arc_ts), pk(t->arc_delay),
                                 pk(ep_rat), pk(o->drv_rat), pk(o->arc_rat), pk(o->drv_slack), pk(o->arc_slack),
                                 pk(o->tns), pk(o->wns), pk(scratch)};
    for (int v = 0; v < NV; ++v) key.push_back(uint64_t(kv.mode[v]));
    return run_sequence(g, g->bwd_cache, std::move(key), s, [&](hipStream_t q) {
        enqueue_backward_levels<NV>(g, kv, nd, t, ep_rat, o, scratch, q);
    });
}

template <int RW>
static void launch_backward_view(const sta_graph* g, int NV, const KViews& kv, const sta_net_out* nd,
                                 const sta_timing_out* t, const float* ep_rat, const sta_slack_out* o, size_t lds,
                                 hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    const int32_t* lv = reinterpret_cast<const int32_t*>(g->dev + g->lay.bwd_lvl);
    set_lds(k_backward_view<RW>, lds);
    prof_launch("k_backward_view", s, [&] {
        hipLaunchKernelGGL((k_backward_view<RW>), dim3(NV), dim3(kViewThreads), lds, s, dg, kv, NV, int(g->L),
                           int(g->E), lv, g->max_bt, g->max_bs, g->max_bd, nd->net_delay, t->drv_ts, t->arc_ts,
                           t->arc_delay, ep_rat, o->drv_rat, o->arc_rat, o->drv_slack, o->arc_slack, o->tns, o->wns);
    });
}

static void run_backward_views(const sta_graph* g, int rw, size_t lds, int NV, const KViews& kv, const sta_net_out* nd,
                               const sta_timing_out* t, const float* ep_rat, const sta_slack_out* o, hipStream_t s) {
    switch (rw) {
        case 1: launch_backward_view<1>(g, NV, kv, nd, t, ep_rat, o, lds, s); break;
        case 2: launch_backward_view<2>(g, NV, kv, nd, t, ep_rat, o, lds, s); break;
        case 4: launch_backward_view<4>(g, NV, kv, nd, t, ep_rat, o, lds, s); break;
        default: launch_backward_view<8>(g, NV, kv, nd, t, ep_rat, o, lds, s); break;
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
    if (!out->load || (g->A > 0 && (!out->net_delay || !out->net_imp2)))
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
        (g->A > 0 && (!out->arc_ts || !out->arc_delay || !out->argmax || !nd->net_delay || !nd->net_imp2)) ||
        !nd->load)
        return fail(STA_E_ARG, "sta_propagate: null buffer");
    KLib kl{};
    for (int i = 0; i < 7; ++i) { kl.ax[i] = lib->x[i]; kl.ax[7 + i] = lib->y[i]; }
    for (int i = 0; i < 6; ++i) { kl.ax[14 + i] = lib->x[i + 1] - lib->x[i]; kl.ax[20 + i] = lib->y[i + 1] - lib->y[i]; }
    kl.tables = lib->tables;
    kl.n_tables = lib->n_tables;
    const KViews kv = kviews(views);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rw = 0;
    size_t lds = 0;
    if (use_view_forward(g, lib->n_tables, &rw, &lds)) {
        run_forward_views(g, rw, lds, views->n_views, kl, kv, pi_ts, nd, out, s);
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
    int rw = 0;
    size_t lds = 0;
    if (use_view_backward(g, &rw, &lds)) {
        run_backward_views(g, rw, lds, views->n_views, kv, nd, t, ep_rat, out, s);
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

sta_status sta_set_schedule(sta_graph* g, int32_t view_max_arcs_per_level, int32_t use_graphs) {
    if (!g) return fail(STA_E_ARG, "sta_set_schedule: null graph");
    g->view_sched_max_arcs = view_max_arcs_per_level < 0 ? kDefaultViewSchedMaxArcs : view_max_arcs_per_level;
    g->use_graphs = use_graphs != 0;
    return STA_OK;
}

}  // extern "C"

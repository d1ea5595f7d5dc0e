// HIP kernels for CDNA4 (gfx950) and the device-side entry points of libsta.
//
// Build: -O3 -ffp-contract=off (no a*b+c contraction), IEEE FP32 division and sqrt
// (correctly rounded), FP32 denormals kept.  With those, every floating-point step
// below is the same single rounded operation as in the operation order the header
// documents, so results equal the CPU definition bit for bit.
//
// Work decomposition (one design, all views of a call at once):
//   K1 k_delay_calc   one lane per net, level-free, node temporaries in LDS.
//   K2 k_forward      one launch per gate level; a wavefront owns a tile of <= 64 cell
//                     arcs of consecutive whole gates; per-gate max/argmax by a
//                     segmented shuffle reduction inside the wavefront.
//   K3 k_backward     one launch per driver level, highest first; a wavefront owns
//                     <= 64 sink slots of consecutive drivers (or one large driver).
//   K4 k_endpoint_*   WNS by min, TNS by exact integer (fixed-point) accumulation of
//                     the negative endpoint slacks, rounded once to FP64.
#include <hip/hip_runtime.h>

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
// NLDM lookup helpers (shared by all views)
// ---------------------------------------------------------------------------------

struct KLib {
    float x[7], y[7];
    float dx[6], dy[6];          // fl32(x[i+1]-x[i]), fl32(y[j+1]-y[j])
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

__device__ __forceinline__ float bilerp(const float* __restrict__ T, int i, int j, float tx, float ty) {
    const float t00 = T[i * 7 + j], t01 = T[i * 7 + j + 1];
    const float t10 = T[(i + 1) * 7 + j], t11 = T[(i + 1) * 7 + j + 1];
    const float p = t00 + tx * (t10 - t00);
    const float q = t01 + tx * (t11 - t01);
    return p + ty * (q - p);
}

__device__ __forceinline__ uint64_t lanes_le(int lane) {
    return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
}

// ---------------------------------------------------------------------------------
// K2: forward propagation of one gate level
// ---------------------------------------------------------------------------------

template <int NV>
__global__ __launch_bounds__(256) void k_forward(DevGraph G, KLib lib, KViews V, int tile0, int tile1,
                                                 const float* __restrict__ load,
                                                 const float* __restrict__ nd,
                                                 const float* __restrict__ ni,
                                                 float* __restrict__ drv_ts, float* __restrict__ arc_ts,
                                                 float* __restrict__ arc_delay, uint8_t* __restrict__ argmax) {
    __shared__ float s_ax[7 + 7 + 6 + 6];
    if (threadIdx.x < 7) s_ax[threadIdx.x] = lib.x[threadIdx.x];
    else if (threadIdx.x < 14) s_ax[threadIdx.x] = lib.y[threadIdx.x - 7];
    else if (threadIdx.x < 20) s_ax[threadIdx.x] = lib.dx[threadIdx.x - 14];
    else if (threadIdx.x < 26) s_ax[threadIdx.x] = lib.dy[threadIdx.x - 20];
    __syncthreads();
    const float* X = s_ax;
    const float* Y = s_ax + 7;
    const float* DX = s_ax + 14;
    const float* DY = s_ax + 20;

    const int lane = threadIdx.x & 63;
    const int t = tile0 + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= tile1) return;                      // uniform per wavefront
    const int a0 = G.ftile_arc[t];
    const int n = G.ftile_arc[t + 1] - a0;
    const int g0 = G.ftile_gate[t];
    const bool active = lane < n;
    const int a = a0 + lane;
    const uint32_t meta = active ? G.arc_meta[a] : 0u;
    const int kpos = int((meta >> 16) & 0xffu);
    const bool head = active && kpos == 0;
    const uint64_t heads = __ballot(head);
    const uint64_t le = lanes_le(lane);
    const int gi = __popcll(heads & le) - 1;
    const uint64_t after = heads & ~le;
    const int seg_end = after ? (__ffsll(static_cast<unsigned long long>(after)) - 1) : n;
    const int g = g0 + gi;
    const int o = G.n_pi + g;

    float cand[NV], slw[NV];
    int best_k[NV];
    if (active) {
        const int u = G.arc_src[a];
        const float ndv = nd[a];
        const float niv = ni[a];
        const int tb = int(meta & 0xffffu);
        const float Lo = load[o];
        const int j = seg6(Y, Lo);
        const float ty = (Lo - Y[j]) / DY[j];
        float in_at[NV], in_sl[NV];
        const float2* src = reinterpret_cast<const float2*>(drv_ts) + size_t(u) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float2 ts = src[v];
            in_at[v] = ts.x;
            in_sl[v] = ts.y;
        }
        float2* dst = reinterpret_cast<float2*>(arc_ts) + size_t(a) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float ai = in_at[v] + ndv;
            const float su2 = in_sl[v] * in_sl[v];
            const float si = sqrtf(su2 + niv);
            const int i = seg6(X, si);
            const float tx = (si - X[i]) / DX[i];
            const float* T = lib.tables + (size_t(V.set[v]) * lib.n_tables + tb) * 98;
            const float dl = bilerp(T, i, j, tx, ty);
            const float sl = bilerp(T + 49, i, j, tx, ty);
            dst[v] = make_float2(ai, si);
            arc_delay[size_t(a) * NV + v] = dl;
            cand[v] = ai + dl;
            slw[v] = sl;
            best_k[v] = kpos;
        }
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) { cand[v] = 0.0f; slw[v] = 0.0f; best_k[v] = 0; }
    }
    // segmented reduction toward each gate's first lane; the left operand covers the
    // lower arc positions, so keeping it on ties keeps the smallest arc index
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const bool take = (lane + off) < seg_end;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float c2 = __shfl_down(cand[v], off, 64);
            const float s2 = __shfl_down(slw[v], off, 64);
            const int k2 = __shfl_down(best_k[v], off, 64);
            if (take) {
                const bool late = V.mode[v] == STA_LATE;
                if (late ? (c2 > cand[v]) : (c2 < cand[v])) { cand[v] = c2; best_k[v] = k2; }
                if (late ? (s2 > slw[v]) : (s2 < slw[v])) slw[v] = s2;
            }
        }
    }
    if (head) {
        float2* out = reinterpret_cast<float2*>(drv_ts) + size_t(o) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            out[v] = make_float2(cand[v], slw[v]);
            argmax[size_t(g) * NV + v] = uint8_t(best_k[v]);
        }
    }
}

// primary inputs: copy (arrival, slew) of every view
__global__ void k_copy_pi(const float* __restrict__ pi_ts, float* __restrict__ drv_ts, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) drv_ts[i] = pi_ts[i];
}

// ---------------------------------------------------------------------------------
// K3: backward required times of one driver level
// ---------------------------------------------------------------------------------

template <int NV>
__global__ __launch_bounds__(256) void k_backward(DevGraph G, KViews V, int tile0, int tile1,
                                                  const float* __restrict__ nd,
                                                  const float* __restrict__ drv_ts,
                                                  const float* __restrict__ arc_ts,
                                                  const float* __restrict__ arc_delay,
                                                  const float* __restrict__ ep_rat,
                                                  float* __restrict__ drv_rat, float* __restrict__ arc_rat,
                                                  float* __restrict__ drv_slack, float* __restrict__ arc_slack) {
    const int lane = threadIdx.x & 63;
    const int t = tile0 + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= tile1) return;
    const int d0 = G.btile_drv[t];
    const int s0 = G.btile_slot[t];
    const int n = G.btile_slot[t + 1] - s0;
    // n <= 64, or one driver owning every slot; lane owns the contiguous slots
    // [lane*c, min(n, (lane+1)*c)) so lower lanes always hold lower sink positions
    const int c = (n + 63) >> 6;
    const int sb = lane * c;
    const int se = min(n, sb + c);
    bool head;
    if (c > 1) head = (lane == 0);
    else head = (sb < n) && (uint32_t(G.bslot_out[s0 + sb]) & kHeadBit) != 0u;
    float best[NV];
    bool have = false;
#pragma unroll
    for (int v = 0; v < NV; ++v) best[v] = 0.0f;
    for (int s = sb; s < se; ++s) {
        const int slot = s0 + s;
        const int sa = G.bslot_arc[slot];
        const int so = G.bslot_out[slot] & 0x7fffffff;
        float val[NV];
        if (sa >= 0) {
            const float ndv = nd[sa];
            const float* ro = drv_rat + size_t(so) * NV;
            const float* dl = arc_delay + size_t(sa) * NV;
            const float2* ts = reinterpret_cast<const float2*>(arc_ts) + size_t(sa) * NV;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const float rin = ro[v] - dl[v];
                const float ati = ts[v].x;
                arc_rat[size_t(sa) * NV + v] = rin;
                arc_slack[size_t(sa) * NV + v] = (V.mode[v] == STA_LATE) ? (rin - ati) : (ati - rin);
                val[v] = rin - ndv;
            }
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) val[v] = ep_rat[size_t(so) * NV + v];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const bool late = V.mode[v] == STA_LATE;
            if (!have || (late ? (val[v] < best[v]) : (val[v] > best[v]))) best[v] = val[v];
        }
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
        for (int v = 0; v < NV; ++v) {
            const float b2 = __shfl_down(best[v], off, 64);
            if (take) {
                const bool late = V.mode[v] == STA_LATE;
                if (late ? (b2 < best[v]) : (b2 > best[v])) best[v] = b2;
            }
        }
    }
    if (head) {
        const int u = d0 + gi;
        const float2* ts = reinterpret_cast<const float2*>(drv_ts) + size_t(u) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const float r = best[v];
            const float at = ts[v].x;
            drv_rat[size_t(u) * NV + v] = r;
            drv_slack[size_t(u) * NV + v] = (V.mode[v] == STA_LATE) ? (r - at) : (at - r);
        }
    }
}

// ---------------------------------------------------------------------------------
// K4: endpoint summaries
// ---------------------------------------------------------------------------------

// |x| of a finite FP32 value is m * 2^(sh - 149) with m < 2^24 and 0 <= sh <= 253.
// It is added exactly into a 320-bit fixed-point number held as ten 32-bit digits in
// 64-bit words (the upper halves absorb carries; 2^32 additions cannot overflow).
constexpr int kLimbs = 10;
constexpr int kK4Blocks = 256;
constexpr int kK4Threads = 256;

size_t scratch_bytes() {
    return size_t(kK4Blocks) * STA_MAX_VIEWS * kLimbs * 8 + size_t(kK4Blocks) * STA_MAX_VIEWS * 4;
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
            if (s < 0.0f) {
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

// bit p of the normalized digit string (0 outside it)
__device__ inline uint32_t big_bit(const uint64_t* L, int p) {
    if (p < 0 || p >= 32 * kLimbs) return 0u;
    return uint32_t(L[p >> 5] >> (p & 31)) & 1u;
}

// round the non-negative integer sum(L[i] 2^(32 i)) * 2^-149 to nearest-even FP64
__device__ double big_to_double(const uint64_t* L) {
    int top = -1;
    for (int i = kLimbs - 1; i >= 0; --i)
        if (L[i]) { top = i; break; }
    if (top < 0) return 0.0;
    const int msb = top * 32 + (31 - __clz(uint32_t(L[top])));
    uint64_t w = 0;
    for (int q = 0; q < 64; ++q) w |= uint64_t(big_bit(L, msb - 63 + q)) << q;
    bool sticky = false;
    for (int p = 0; p < msb - 63; ++p) sticky = sticky || big_bit(L, p);
    uint64_t mant = w >> 11;
    const uint32_t rb = uint32_t(w & 0x7ffu);
    int e = msb - 52;
    if (rb > 0x400u || (rb == 0x400u && (sticky || (mant & 1ull)))) mant += 1ull;
    if (mant == (1ull << 53)) { mant >>= 1; e += 1; }
    return ldexp(double(mant), e - 149);
}

template <int NV>
__global__ void k_endpoint_final(int nblk, const unsigned long long* __restrict__ part_limbs,
                                 const float* __restrict__ part_wns, double* __restrict__ tns,
                                 float* __restrict__ wns) {
    __shared__ unsigned long long s_sum[NV * kLimbs];
    for (int i = threadIdx.x; i < NV * kLimbs; i += blockDim.x) {
        unsigned long long acc = 0ull;
        for (int b = 0; b < nblk; ++b) acc += part_limbs[size_t(b) * NV * kLimbs + i];
        s_sum[i] = acc;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int v = threadIdx.x;
        uint64_t L[kLimbs];
        uint64_t carry = 0;
        for (int i = 0; i < kLimbs; ++i) {
            const uint64_t x = s_sum[v * kLimbs + i] + carry;   // < 2^63 + 2^32
            L[i] = x & 0xffffffffull;
            carry = x >> 32;
        }
        const double mag = big_to_double(L);
        tns[v] = (mag == 0.0) ? 0.0 : -mag;
        float mn = __builtin_inff();
        for (int b = 0; b < nblk; ++b) {
            const float x = part_wns[size_t(b) * NV + v];
            mn = (x < mn) ? x : mn;
        }
        wns[v] = mn;
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

template <int NV>
static void run_forward(const sta_graph* g, const KLib& lib, const KViews& kv, const float* pi_ts,
                        const sta_net_out* nd, const sta_timing_out* o, hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    const int npi = int(g->n_pi) * NV * 2;
    if (npi > 0)
        prof_launch("k_copy_pi", s, [&] {
            hipLaunchKernelGGL(k_copy_pi, dim3((npi + 255) / 256), dim3(256), 0, s, pi_ts, o->drv_ts, npi);
        });
    for (int64_t l = 1; l <= g->L; ++l) {
        const int t0 = g->fwd_tile_ptr[l], t1 = g->fwd_tile_ptr[l + 1];
        if (t1 <= t0) continue;
        prof_launch("k_forward", s, [&] {
            hipLaunchKernelGGL((k_forward<NV>), dim3((t1 - t0 + 3) / 4), dim3(256), 0, s, dg, lib, kv, t0, t1,
                               nd->load, nd->net_delay, nd->net_imp2, o->drv_ts, o->arc_ts, o->arc_delay, o->argmax);
        });
    }
}

template <int NV>
static void run_backward(const sta_graph* g, const KViews& kv, const sta_net_out* nd, const sta_timing_out* t,
                         const float* ep_rat, const sta_slack_out* o, void* scratch, hipStream_t s) {
    const DevGraph dg = dev_graph(g);
    for (int64_t l = g->L; l >= 0; --l) {
        const int t0 = g->bwd_tile_ptr[l], t1 = g->bwd_tile_ptr[l + 1];
        if (t1 <= t0) continue;
        prof_launch("k_backward", s, [&] {
            hipLaunchKernelGGL((k_backward<NV>), dim3((t1 - t0 + 3) / 4), dim3(256), 0, s, dg, kv, t0, t1,
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
        hipLaunchKernelGGL((k_endpoint_final<NV>), dim3(1), dim3(64), 0, s, nblk, limbs, pw, o->tns, o->wns);
    });
}

}  // namespace sta

using namespace sta;

extern "C" {

sta_status sta_delay_calc(const sta_graph* g, sta_dc_precision prec, const sta_net_out* out, void* stream) {
    if (!g || !out) return fail(STA_E_ARG, "sta_delay_calc: null argument");
    if (!g->dev) return fail(STA_E_ARG, "sta_delay_calc: graph not uploaded");
    if (g->D == 0) return STA_OK;
    if (!out->load || (g->A > 0 && (!out->net_delay || !out->net_imp2)))
        return fail(STA_E_ARG, "sta_delay_calc: null output buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (prec == STA_DC_FP64) dispatch_dc<double>(g, out, s);
    else if (prec == STA_DC_FP32) dispatch_dc<float>(g, out, s);
    else return fail(STA_E_ARG, "sta_delay_calc: unknown precision");
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
    if ((g->n_pi > 0 && !pi_ts) || !out->drv_ts || (g->A > 0 && (!out->arc_ts || !out->arc_delay || !out->argmax ||
                                                                  !nd->net_delay || !nd->net_imp2)) || !nd->load)
        return fail(STA_E_ARG, "sta_propagate: null buffer");
    KLib kl{};
    for (int i = 0; i < 7; ++i) { kl.x[i] = lib->x[i]; kl.y[i] = lib->y[i]; }
    for (int i = 0; i < 6; ++i) { kl.dx[i] = lib->x[i + 1] - lib->x[i]; kl.dy[i] = lib->y[i + 1] - lib->y[i]; }
    kl.tables = lib->tables;
    kl.n_tables = lib->n_tables;
    const KViews kv = kviews(views);
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (views->n_views) {
        case 1: run_forward<1>(g, kl, kv, pi_ts, nd, out, s); break;
        case 2: run_forward<2>(g, kl, kv, pi_ts, nd, out, s); break;
        case 4: run_forward<4>(g, kl, kv, pi_ts, nd, out, s); break;
        default: run_forward<8>(g, kl, kv, pi_ts, nd, out, s); break;
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
    switch (views->n_views) {
        case 1: run_backward<1>(g, kv, nd, t, ep_rat, out, scratch, s); break;
        case 2: run_backward<2>(g, kv, nd, t, ep_rat, out, scratch, s); break;
        case 4: run_backward<4>(g, kv, nd, t, ep_rat, out, scratch, s); break;
        default: run_backward<8>(g, kv, nd, t, ep_rat, out, scratch, s); break;
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

}  // extern "C"

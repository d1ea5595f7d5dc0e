// RC-tree nets and the learned delay/slew surrogate: exact FP64 moments, the training-set
// builder, the 12-64-64-2 network on BF16 MFMA (forward, backward, Adam), error
// calibration and the surrogate path with exact fallback.
//
// Network layout on the matrix cores.  Samples are the N dimension of every product:
// a layer computes Z[out][sample] = W[out][in] * X[in][sample] with 16x16 output tiles,
// so the FP32 result tile of one layer (lane l holds rows 4*(l/16)+j of sample l%16) is,
// after ReLU and BF16 rounding, already the B operand of the next layer.  For the K=32
// products the K index of a lane's eight operand values is permuted consistently in A
// (weights) and B (activations): values 0..3 are rows 4g+j of output tile 2c, values 4..7
// rows 4g+j of tile 2c+1, g = l/16.  Weight gradients contract over samples, so their
// operands are restaged through LDS as [feature][sample] rows.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/sta_surrogate.h"
#include "sta_internal.h"

namespace sta {
namespace sur {

constexpr int kMaxN = STA_TREE_MAX_NODES;
constexpr int kPartStride = 5380;            // >= STA_MLP_PARAMS + 1 (loss), per wave
constexpr int kMaxGradWaves = 1024;
constexpr int kNormBlocks = 256;
constexpr int kCalEntries = STA_CAL_BINS * 2 * STA_CAL_BUCKETS;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void flag_err(int32_t* status, int bits) {
    if (status) atomicOr(status, bits);
}

// ---------------------------------------------------------------------------------
// RC-tree moments, one thread per net, node temporaries in LDS interleaved by thread
// ---------------------------------------------------------------------------------

// Checks the net's shape; returns false (and flags the status word) if it cannot be done.
__device__ __forceinline__ bool net_ok(const sta_trees& T, int n, int& n0, int& nm, int& s0, int& s1,
                                       int32_t* status) {
    n0 = T.net_node_ptr[n];
    nm = T.net_node_ptr[n + 1] - n0;
    s0 = T.sink_ptr[n];
    s1 = T.sink_ptr[n + 1];
    if (nm < 1 || nm > kMaxN || s1 < s0) {
        flag_err(status, STA_TREE_ERR_SIZE);
        return false;
    }
    const int32_t* par = T.node_parent + n0;
    for (int k = 1; k < nm; ++k) {
        const int p = par[k];
        if (p < 0 || p >= k) {
            flag_err(status, STA_TREE_ERR_PARENT);
            return false;
        }
    }
    for (int s = s0; s < s1; ++s) {
        const int k = T.sink_node[s];
        if (k < 0 || k >= nm) {
            flag_err(status, STA_TREE_ERR_SINK);
            return false;
        }
    }
    return true;
}

#define NODE(arr, k) arr[(k) * NT]

// C(k) = wire cap + pin caps of the sinks tapping k (ascending sink order)
template <int NT>
__device__ __forceinline__ void node_caps(const sta_trees& T, int n0, int nm, int s0, int s1, double* C) {
    const float* Cw = T.node_C + n0;
    for (int k = 0; k < nm; ++k) NODE(C, k) = static_cast<double>(Cw[k]);
    for (int s = s0; s < s1; ++s) NODE(C, T.sink_node[s]) += static_cast<double>(T.sink_pincap[s]);
}

// in place: X(parent) += X(k) for k descending (downstream sums)
template <int NT>
__device__ __forceinline__ void up_sum(const int32_t* par, int nm, double* X) {
    for (int k = nm - 1; k >= 1; --k) NODE(X, par[k]) += NODE(X, k);
}

// Y(0) = 0, Y(k) = Y(parent) + (R(k) X(k)) 1e-3 for k ascending; Y may alias X
template <int NT>
__device__ __forceinline__ void down_sum(const int32_t* par, const float* R, int nm, const double* X, double* Y) {
    NODE(Y, 0) = 0.0;
    for (int k = 1; k < nm; ++k) NODE(Y, k) = NODE(Y, par[k]) + (static_cast<double>(R[k]) * NODE(X, k)) * 1e-3;
}

__device__ __forceinline__ void sink_out(double m1, double m2, float S, float& delay, float& slew, double& imp2) {
    imp2 = 2.0 * m2 - m1 * m1;
    if (imp2 < 0.0) imp2 = 0.0;
    delay = static_cast<float>(m1);
    const float i2 = static_cast<float>(imp2);
    slew = sqrtf(S * S + i2);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_tree_dataset(sta_trees T, float* __restrict__ feat,
                                                     float* __restrict__ target, float* __restrict__ delay,
                                                     float* __restrict__ slew, int32_t* status) {
    __shared__ double sC[kMaxN * NT];
    __shared__ double sCd[kMaxN * NT];
    __shared__ double sW[kMaxN * NT];    // W, then m2 in place
    __shared__ double sM[kMaxN * NT];    // m1
    const int t = threadIdx.x;
    const int n = blockIdx.x * NT + t;
    if (n >= T.n_nets) return;
    int n0, nm, s0, s1;
    if (!net_ok(T, n, n0, nm, s0, s1, status)) return;
    const int32_t* par = T.node_parent + n0;
    const float* R = T.node_R + n0;
    double* C = sC + t;
    double* Cd = sCd + t;
    double* W = sW + t;
    double* M = sM + t;
    node_caps<NT>(T, n0, nm, s0, s1, C);
    for (int k = 0; k < nm; ++k) NODE(Cd, k) = NODE(C, k);
    up_sum<NT>(par, nm, Cd);
    down_sum<NT>(par, R, nm, Cd, M);
    for (int k = 0; k < nm; ++k) NODE(W, k) = NODE(C, k) * NODE(M, k);
    up_sum<NT>(par, nm, W);
    down_sum<NT>(par, R, nm, W, W);
    double sumR = 0.0, sumC = 0.0;
    for (int k = 1; k < nm; ++k) sumR += static_cast<double>(R[k]);
    for (int k = 0; k < nm; ++k) sumC += static_cast<double>(T.node_C[n0 + k]);
    const double load = NODE(Cd, 0);
    const float S = T.drv_slew[n];
    for (int s = s0; s < s1; ++s) {
        const int k = T.sink_node[s];
        const double m1 = NODE(M, k);
        float d, sl;
        double imp2;
        sink_out(m1, NODE(W, k), S, d, sl, imp2);
        if (delay) delay[s] = d;
        if (slew) slew[s] = sl;
        double rpath = 0.0, cpath = 0.0, rfirst = 0.0;
        int depth = 0;
        for (int v = k; v != 0; v = par[v]) {
            rpath += static_cast<double>(R[v]);
            cpath += NODE(C, v);
            if (par[v] == 0) rfirst = static_cast<double>(R[v]);
            ++depth;
        }
        const double cdk = NODE(Cd, k);
        if (feat) {
            float* f = feat + static_cast<size_t>(s) * 12;
            f[0] = static_cast<float>(rpath);
            f[1] = static_cast<float>(load);
            f[2] = static_cast<float>(cdk);
            f[3] = static_cast<float>(depth);
            f[4] = static_cast<float>(nm);
            f[5] = static_cast<float>(s1 - s0);
            f[6] = static_cast<float>(rfirst);
            f[7] = static_cast<float>(cpath);
            f[8] = static_cast<float>(nm > 1 ? sumR / static_cast<double>(nm - 1) : 0.0);
            f[9] = static_cast<float>(sumC / static_cast<double>(nm));
            f[10] = T.sink_pincap[s];
            f[11] = S;
        }
        if (target) {
            const double L = (rpath * cdk) * 1e-3;
            const double U = (rpath * load) * 1e-3;
            const double span = U - L;
            const double alpha = span > 0.0 ? (m1 - L) / span : 0.0;
            const double gamma = U > 0.0 ? sqrt(imp2) / U : 0.0;
            target[2 * static_cast<size_t>(s)] = static_cast<float>(alpha);
            target[2 * static_cast<size_t>(s) + 1] = static_cast<float>(gamma);
        }
    }
}

#undef NODE

// LDS ordering among the lanes of one wavefront (the wave's LDS operations complete in
// order once waited for; no workgroup barrier, since waves of a block work on different nets)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

constexpr int kExactWaves = 4;     // nets per 256-lane block, one per wavefront

// Exact delay/slew of every net (list == nullptr) or of the listed nets.  One wavefront
// per net, lane k = local node k.  Depths by pointer doubling; downstream sums in rounds
// of decreasing depth, each node adding its children in descending index order (the
// order of the sequential definition, so the FP64 results are the same bit for bit);
// prefix sums (m1, m2) in rounds of increasing depth.
__global__ __launch_bounds__(256) void k_tree_exact(sta_trees T, const int32_t* __restrict__ list,
                                                    const int32_t* __restrict__ count, float* __restrict__ delay,
                                                    float* __restrict__ slew, int32_t* status) {
    __shared__ double s_sum[kExactWaves][kMaxN];    // Cd, later C*m1 summed downstream
    __shared__ double s_m1[kExactWaves][kMaxN];
    __shared__ double s_m2[kExactWaves][kMaxN];
    __shared__ unsigned long long s_ch[kExactWaves][kMaxN];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int i = blockIdx.x * kExactWaves + wv;
    int n = i;
    if (list) {
        if (i >= *count) return;
        n = list[i];
        if (n < 0 || n >= T.n_nets) {
            if (lane == 0) flag_err(status, STA_TREE_ERR_SIZE);
            return;
        }
    } else if (i >= T.n_nets) {
        return;
    }
    const int n0 = T.net_node_ptr[n];
    const int nm = T.net_node_ptr[n + 1] - n0;
    const int s0 = T.sink_ptr[n], s1 = T.sink_ptr[n + 1];
    if (nm < 1 || nm > kMaxN || s1 < s0) {
        if (lane == 0) flag_err(status, STA_TREE_ERR_SIZE);
        return;
    }
    const bool act = lane < nm;
    const int p = (act && lane > 0) ? T.node_parent[n0 + lane] : 0;
    if (__ballot(act && lane > 0 && (p < 0 || p >= lane))) {
        if (lane == 0) flag_err(status, STA_TREE_ERR_PARENT);
        return;
    }
    const float Rk = act ? T.node_R[n0 + lane] : 0.0f;
    double Ck = act ? static_cast<double>(T.node_C[n0 + lane]) : 0.0;
    // sinks 64 at a time: one coalesced load per lane, then the pin caps are added to
    // their nodes in ascending sink order by broadcasting each sink from its lane
    for (int c = s0; c < s1; c += 64) {
        const bool sv = c + lane < s1;
        const int k = sv ? T.sink_node[c + lane] : 0;
        const float cap = sv ? T.sink_pincap[c + lane] : 0.0f;
        if (__ballot(k < 0 || k >= nm)) {
            if (lane == 0) flag_err(status, STA_TREE_ERR_SINK);
            return;
        }
        const int ns = min(64, s1 - c);
        for (int j = 0; j < ns; ++j) {
            const int kj = __builtin_amdgcn_readlane(k, j);
            const float cj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cap), j));
            if (kj == lane) Ck += static_cast<double>(cj);
        }
    }
    s_ch[wv][lane] = 0ull;
    s_m1[wv][lane] = 0.0;
    s_m2[wv][lane] = 0.0;
    wave_sync();
    if (act && lane > 0) atomicOr(&s_ch[wv][p], 1ull << lane);
    // depth by pointer doubling (depth < 64)
    int anc = p, dep = (act && lane > 0) ? 1 : 0;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const int da = __shfl(dep, anc);
        const int aa = __shfl(anc, anc);
        dep += da;
        anc = aa;
    }
    const int maxd = wave_max_i32(dep);
    wave_sync();
    const unsigned long long ch = s_ch[wv][lane];
    // Cd: downstream sums, children in descending index order
    double cd = Ck;
    for (int r = maxd; r >= 0; --r) {
        if (act && dep == r) {
            double acc = Ck;
            unsigned long long m = ch;
            while (m) {
                const int c = 63 - __clzll(static_cast<long long>(m));
                acc += s_sum[wv][c];
                m &= ~(1ull << c);
            }
            cd = acc;
            s_sum[wv][lane] = acc;
        }
        wave_sync();
    }
    double m1 = 0.0;
    for (int r = 1; r <= maxd; ++r) {
        if (act && dep == r) {
            m1 = s_m1[wv][p] + (static_cast<double>(Rk) * cd) * 1e-3;
            s_m1[wv][lane] = m1;
        }
        wave_sync();
    }
    const double w0 = Ck * m1;
    double wd = w0;
    for (int r = maxd; r >= 0; --r) {
        if (act && dep == r) {
            double acc = w0;
            unsigned long long m = ch;
            while (m) {
                const int c = 63 - __clzll(static_cast<long long>(m));
                acc += s_sum[wv][c];
                m &= ~(1ull << c);
            }
            wd = acc;
            s_sum[wv][lane] = acc;
        }
        wave_sync();
    }
    for (int r = 1; r <= maxd; ++r) {
        if (act && dep == r) s_m2[wv][lane] = s_m2[wv][p] + (static_cast<double>(Rk) * wd) * 1e-3;
        wave_sync();
    }
    const float S = T.drv_slew[n];
    for (int c = s0; c < s1; c += 64) {
        const int s = c + lane;
        if (s < s1) {
            const int k = T.sink_node[s];
            float d, sl;
            double imp2;
            sink_out(s_m1[wv][k], s_m2[wv][k], S, d, sl, imp2);
            delay[s] = d;
            slew[s] = sl;
        }
    }
}


// The 12 features of every sink (those of k_tree_dataset, bit for bit) without the
// moments: one wavefront per net, lane k = local node k.  Node caps (pin caps added in
// ascending sink order), downstream caps in rounds of decreasing depth (children in
// descending index order, as the sequential definition), and each sink's path to the
// driver walked upward from the sink (path resistance, path capacitance, depth, first-edge
// resistance), with the net's R and C sums in ascending node order.
__global__ __launch_bounds__(256) void k_tree_features(sta_trees T, float* __restrict__ feat, int32_t* status) {
    __shared__ double s_cd[kExactWaves][kMaxN];     // downstream cap
    __shared__ double s_c[kExactWaves][kMaxN];      // node cap (wire + pin caps)
    __shared__ float s_r[kExactWaves][kMaxN];
    __shared__ float s_cw[kExactWaves][kMaxN];      // wire cap
    __shared__ int s_par[kExactWaves][kMaxN];
    __shared__ unsigned long long s_ch[kExactWaves][kMaxN];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int n = blockIdx.x * kExactWaves + wv;
    if (n >= T.n_nets) return;
    const int n0 = T.net_node_ptr[n];
    const int nm = T.net_node_ptr[n + 1] - n0;
    const int s0 = T.sink_ptr[n], s1 = T.sink_ptr[n + 1];
    if (nm < 1 || nm > kMaxN || s1 < s0) {
        if (lane == 0) flag_err(status, STA_TREE_ERR_SIZE);
        return;
    }
    const bool act = lane < nm;
    const int p = (act && lane > 0) ? T.node_parent[n0 + lane] : 0;
    if (__ballot(act && lane > 0 && (p < 0 || p >= lane))) {
        if (lane == 0) flag_err(status, STA_TREE_ERR_PARENT);
        return;
    }
    const float Rk = act ? T.node_R[n0 + lane] : 0.0f;
    const float Cw = act ? T.node_C[n0 + lane] : 0.0f;
    double Ck = static_cast<double>(Cw);
    for (int c = s0; c < s1; c += 64) {
        const bool sv = c + lane < s1;
        const int k = sv ? T.sink_node[c + lane] : 0;
        const float cap = sv ? T.sink_pincap[c + lane] : 0.0f;
        if (__ballot(k < 0 || k >= nm)) {
            if (lane == 0) flag_err(status, STA_TREE_ERR_SINK);
            return;
        }
        const int ns = min(64, s1 - c);
        for (int j = 0; j < ns; ++j) {
            const int kj = __builtin_amdgcn_readlane(k, j);
            const float cj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cap), j));
            if (kj == lane) Ck += static_cast<double>(cj);
        }
    }
    s_ch[wv][lane] = 0ull;
    s_c[wv][lane] = Ck;
    s_r[wv][lane] = Rk;
    s_cw[wv][lane] = Cw;
    s_par[wv][lane] = p;
    wave_sync();
    if (act && lane > 0) atomicOr(&s_ch[wv][p], 1ull << lane);
    int anc = p, dep = (act && lane > 0) ? 1 : 0;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const int da = __shfl(dep, anc);
        const int aa = __shfl(anc, anc);
        dep += da;
        anc = aa;
    }
    const int maxd = wave_max_i32(dep);
    wave_sync();
    const unsigned long long ch = s_ch[wv][lane];
    for (int r = maxd; r >= 0; --r) {
        if (act && dep == r) {
            double acc = Ck;
            unsigned long long m = ch;
            while (m) {
                const int c = 63 - __clzll(static_cast<long long>(m));
                acc += s_cd[wv][c];
                m &= ~(1ull << c);
            }
            s_cd[wv][lane] = acc;
        }
        wave_sync();
    }
    // the net's resistance and wire-cap sums in ascending node order (every lane walks the
    // same LDS values, so every lane holds them; reading them lane by lane from registers
    // instead was measured slower)
    double sumR = 0.0, sumC = 0.0;
    for (int k = 1; k < nm; ++k) sumR += static_cast<double>(s_r[wv][k]);
    for (int k = 0; k < nm; ++k) sumC += static_cast<double>(s_cw[wv][k]);
    const double load = s_cd[wv][0];
    const float S = T.drv_slew[n];
    const float meanR = static_cast<float>(nm > 1 ? sumR / static_cast<double>(nm - 1) : 0.0);
    const float meanC = static_cast<float>(sumC / static_cast<double>(nm));
    for (int c = s0; c < s1; c += 64) {
        const int s = c + lane;
        if (s >= s1) continue;
        const int k = T.sink_node[s];
        double rpath = 0.0, cpath = 0.0, rfirst = 0.0;
        int depth = 0;
        for (int v = k; v != 0; v = s_par[wv][v]) {
            rpath += static_cast<double>(s_r[wv][v]);
            cpath += s_c[wv][v];
            if (s_par[wv][v] == 0) rfirst = static_cast<double>(s_r[wv][v]);
            ++depth;
        }
        float4* f = reinterpret_cast<float4*>(feat + static_cast<size_t>(s) * 12);
        f[0] = make_float4(static_cast<float>(rpath), static_cast<float>(load), static_cast<float>(s_cd[wv][k]),
                           static_cast<float>(depth));
        f[1] = make_float4(static_cast<float>(nm), static_cast<float>(s1 - s0), static_cast<float>(rfirst),
                           static_cast<float>(cpath));
        f[2] = make_float4(meanR, meanC, T.sink_pincap[s], S);
    }
}

__global__ void k_fill_i32(int32_t* p, int32_t n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// net flag = any untrusted sink; flagged nets are appended to the list (order unspecified)
__global__ void k_sur_compact(const int32_t* __restrict__ sink_ptr, const uint8_t* __restrict__ sink_flag, int32_t n,
                              int32_t* __restrict__ net_flag, int32_t* __restrict__ list,
                              int32_t* __restrict__ count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int f = 0;
    for (int s = sink_ptr[i]; s < sink_ptr[i + 1]; ++s) f |= sink_flag[s];
    net_flag[i] = f;
    if (f) list[atomicAdd(count, 1)] = i;
}

// ---------------------------------------------------------------------------------
// input normalization statistics
// ---------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_norm_partial(const float* __restrict__ feat, int32_t n,
                                                      double* __restrict__ part) {
    __shared__ double red[256];
    double s1[12], s2[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) s1[i] = s2[i] = 0.0;
    for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const double v = log(static_cast<double>(feat[static_cast<size_t>(r) * 12 + i]) + 1.0);
            s1[i] += v;
            s2[i] += v * v;
        }
    }
    for (int q = 0; q < 24; ++q) {
        red[threadIdx.x] = q < 12 ? s1[q] : s2[q - 12];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x * 24 + q] = red[0];
        __syncthreads();
    }
}

__global__ void k_norm_final(const double* __restrict__ part, int32_t blocks, int32_t n, float* __restrict__ norm) {
    const int i = threadIdx.x;
    if (i >= 12) return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < blocks; ++k) {
        a += part[k * 24 + i];
        b += part[k * 24 + 12 + i];
    }
    const double mu = n > 0 ? a / n : 0.0;
    double var = n > 0 ? b / n - mu * mu : 0.0;
    if (var < 0.0) var = 0.0;
    norm[i] = static_cast<float>(mu);
    norm[12 + i] = static_cast<float>(var > 0.0 ? 1.0 / sqrt(var) : 1.0);
}

// ---------------------------------------------------------------------------------
// the network on the matrix cores
// ---------------------------------------------------------------------------------

// BF16 bits of f rounded to nearest even (the hardware conversion, v_cvt_pk_bf16_f32 on
// gfx950: for finite f the same bits as adding 0x7fff plus the kept lowest bit and
// truncating)
__device__ __forceinline__ short bf16r(float f) {
    return __builtin_bit_cast(short, static_cast<__bf16>(f));
}

__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                   0, 0);
}

// K index of value j of a K=32 chunk c for lane group g (see the file comment)
__device__ __forceinline__ int kidx(int c, int g, int j) {
    return 32 * c + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

struct Wf {                 // forward operands of one lane
    v4s w1[4];
    v8s w2[4][2];
    v8s w3[2];
    v4f b1[4], b2[4], b3;
};
struct Wb {                 // backward operands (transposed weights)
    v4s w3t[4];
    v8s w2t[4][2];
};

__device__ __forceinline__ void load_wf(const float* __restrict__ P, int g, int r, Wf& W) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            W.w1[m][j] = bf16r(P[STA_MLP_OFF_W1 + (16 * m + r) * 16 + 4 * g + j]);
            W.b1[m][j] = P[STA_MLP_OFF_B1 + 16 * m + 4 * g + j];
            W.b2[m][j] = P[STA_MLP_OFF_B2 + 16 * m + 4 * g + j];
        }
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int j = 0; j < 8; ++j) W.w2[m][c][j] = bf16r(P[STA_MLP_OFF_W2 + (16 * m + r) * 64 + kidx(c, g, j)]);
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j) W.w3[c][j] = r < 2 ? bf16r(P[STA_MLP_OFF_W3 + r * 64 + kidx(c, g, j)]) : short(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) W.b3[j] = (g == 0 && j < 2) ? P[STA_MLP_OFF_B3 + j] : 0.0f;
}

__device__ __forceinline__ void load_wb(const float* __restrict__ P, int g, int r, Wb& W) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            W.w3t[m][j] = (4 * g + j < 2) ? bf16r(P[STA_MLP_OFF_W3 + (4 * g + j) * 64 + 16 * m + r]) : short(0);
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int j = 0; j < 8; ++j) W.w2t[m][c][j] = bf16r(P[STA_MLP_OFF_W2 + kidx(c, g, j) * 64 + 16 * m + r]);
    }
}

// the B operand of one 16-sample tile: features 4g..4g+3 of sample r (zeros for g == 3)
__device__ __forceinline__ v4s load_x(const float* __restrict__ feat, const float* __restrict__ norm, int g,
                                      size_t s, bool valid, float4& f) {
    f = make_float4(0.f, 0.f, 0.f, 0.f);
    v4s x = {0, 0, 0, 0};
    if (g < 3) {
        if (valid) f = *reinterpret_cast<const float4*>(feat + s * 12 + 4 * g);
        const float v[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = bf16r((logf(v[j] + 1.0f) - norm[4 * g + j]) * norm[12 + 4 * g + j]);
    }
    return x;
}

// raw features 4g..4g+3 of sample s (zeros for g == 3 or past the end).  The load is
// unconditional from a clamped, always valid address and its value is always used (masked
// by a multiply), so the compiler keeps it branch-free and it can be issued ahead of its use.
__device__ __forceinline__ float4 load_feat(const float* __restrict__ feat, int g, int s, bool valid, int n) {
    const int sc = s < n ? s : n - 1;
    const int gc = g < 3 ? g : 2;
    const float4 f = *reinterpret_cast<const float4*>(feat + static_cast<size_t>(sc) * 12 + 4 * gc);
    const float w = (g < 3 && valid) ? 1.0f : 0.0f;
    return make_float4(f.x * w, f.y * w, f.z * w, f.w * w);
}

// this lane's normalization constants (features 4g..4g+3), loaded once per wave
struct NormL {
    float mu[4], rs[4];
};

__device__ __forceinline__ NormL load_norm(const float* __restrict__ norm, int g) {
    NormL q;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        q.mu[j] = g < 3 ? norm[4 * g + j] : 0.0f;
        q.rs[j] = g < 3 ? norm[12 + 4 * g + j] : 0.0f;
    }
    return q;
}

__device__ __forceinline__ v4s make_x(const NormL& q, int g, float4 f) {
    v4s x = {0, 0, 0, 0};
    if (g < 3) {
        const float v[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = bf16r((logf(v[j] + 1.0f) - q.mu[j]) * q.rs[j]);
    }
    return x;
}

struct Fwd {
    v4f z1[4], z2[4];
    v8s h1[2], h2[2];
    v4f y;
};

__device__ __forceinline__ v8s relu_pair(v4f a, v4f b) {
    // BF16 of max(z, 0): z rounded to BF16 first, two values per instruction, then a
    // negative BF16 (sign bit set: a negative 16-bit integer, -0 included) replaced by +0
    // with a packed integer maximum; the bits are those of rounding max(z, 0)
    typedef float v2f_ __attribute__((ext_vector_type(2)));
    typedef __bf16 v2b_ __attribute__((ext_vector_type(2)));
    typedef short v2s_ __attribute__((ext_vector_type(2)));
    const v2s_ p0 = __builtin_bit_cast(v2s_, __builtin_convertvector(v2f_{a[0], a[1]}, v2b_));
    const v2s_ p1 = __builtin_bit_cast(v2s_, __builtin_convertvector(v2f_{a[2], a[3]}, v2b_));
    const v2s_ p2 = __builtin_bit_cast(v2s_, __builtin_convertvector(v2f_{b[0], b[1]}, v2b_));
    const v2s_ p3 = __builtin_bit_cast(v2s_, __builtin_convertvector(v2f_{b[2], b[3]}, v2b_));
    const v8s h = {p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
    return __builtin_elementwise_max(h, v8s(0));
}

__device__ __forceinline__ void forward(const Wf& W, v4s x, Fwd& F) {
#pragma unroll
    for (int m = 0; m < 4; ++m) F.z1[m] = mfma16(W.w1[m], x, W.b1[m]);
    F.h1[0] = relu_pair(F.z1[0], F.z1[1]);
    F.h1[1] = relu_pair(F.z1[2], F.z1[3]);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        v4f a = W.b2[m];
        a = mfma32(W.w2[m][0], F.h1[0], a);
        a = mfma32(W.w2[m][1], F.h1[1], a);
        F.z2[m] = a;
    }
    F.h2[0] = relu_pair(F.z2[0], F.z2[1]);
    F.h2[1] = relu_pair(F.z2[2], F.z2[3]);
    v4f y = W.b3;
    y = mfma32(W.w3[0], F.h2[0], y);
    y = mfma32(W.w3[1], F.h2[1], y);
    F.y = y;
}

__device__ __forceinline__ float sum16(float v) {    // over the 16 lanes of a lane group
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

constexpr int kRow = 40;     // LDS row: 32 samples + 8 pad (80 B, 16-byte aligned)

struct alignas(16) GradLds {
    short x[16][kRow];
    short h1[64][kRow];
    short h2[64][kRow];
    short dy[2][kRow];
    short dz2[64][kRow];
    short dz1[64][kRow];
};

// Forward + backward over the batch, 32 samples per step of a wave; per-wave gradient
// sums (natural parameter layout, then the loss) go to part[wave].
__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ P, const float* __restrict__ norm,
                                                 const float* __restrict__ feat, const float* __restrict__ target,
                                                 const int32_t* __restrict__ idx, int32_t batch, float inv_batch,
                                                 float* __restrict__ part) {
    __shared__ GradLds L;
    const int lane = threadIdx.x;
    const int g = lane >> 4, r = lane & 15;
    Wf W;
    Wb WB;
    load_wf(P, g, r, W);
    load_wb(P, g, r, WB);
    v4f gW2[4][4], gW1[4], gW3[4], gb1[4], gb2[4];
    const v4f z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = gW3[a] = gb1[a] = gb2[a] = z4;
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = z4;
    }
    float gb3_0 = 0.f, gb3_1 = 0.f, sq = 0.f;
    const int units = (batch + 31) / 32;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int pos = u * 32 + b * 16 + r;
            const bool valid = pos < batch;
            const size_t s = valid ? static_cast<size_t>(idx[pos]) : 0;
            float4 f;
            const v4s x = load_x(feat, norm, g, s, valid, f);
            Fwd F;
            forward(W, x, F);
            float d0 = 0.f, d1 = 0.f;
            if (g == 0 && valid) {
                const float e0 = F.y[0] - target[2 * s], e1 = F.y[1] - target[2 * s + 1];
                sq += e0 * e0 + e1 * e1;
                d0 = e0 * inv_batch;
                d1 = e1 * inv_batch;
            }
            gb3_0 += d0;
            gb3_1 += d1;
            const v4s dyq = {bf16r(d0), bf16r(d1), 0, 0};   // rows 4g+j; nonzero only for g == 0
            v4f dz2[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                v4f a = mfma16(WB.w3t[m], dyq, z4);
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = F.z2[m][j] > 0.0f ? a[j] : 0.0f;
                dz2[m] = a;
                gb2[m] += a;
            }
            v8s dzc[2];   // BF16 operand of the masked output gradient (signed values)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                dzc[0][j] = bf16r(dz2[0][j]);
                dzc[0][4 + j] = bf16r(dz2[1][j]);
                dzc[1][j] = bf16r(dz2[2][j]);
                dzc[1][4 + j] = bf16r(dz2[3][j]);
            }
            v4f dz1[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                v4f a = z4;
                a = mfma32(WB.w2t[m][0], dzc[0], a);
                a = mfma32(WB.w2t[m][1], dzc[1], a);
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = F.z1[m][j] > 0.0f ? a[j] : 0.0f;
                dz1[m] = a;
                gb1[m] += a;
            }
            // restage as [feature][sample] rows for the contraction over samples
            const int col = b * 16 + r;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                L.x[4 * g + j][col] = x[j];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    L.h1[32 * c + 4 * g + j][col] = F.h1[c][j];
                    L.h1[32 * c + 16 + 4 * g + j][col] = F.h1[c][4 + j];
                    L.h2[32 * c + 4 * g + j][col] = F.h2[c][j];
                    L.h2[32 * c + 16 + 4 * g + j][col] = F.h2[c][4 + j];
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    L.dz2[16 * m + 4 * g + j][col] = bf16r(dz2[m][j]);
                    L.dz1[16 * m + 4 * g + j][col] = bf16r(dz1[m][j]);
                }
            }
            if (g == 0) {
                L.dy[0][col] = dyq[0];
                L.dy[1][col] = dyq[1];
            }
        }
        __syncthreads();
        const int k0 = 8 * g;
        v8s bh1[4], bh2[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bh1[q] = *reinterpret_cast<const v8s*>(&L.h1[16 * q + r][k0]);
            bh2[q] = *reinterpret_cast<const v8s*>(&L.h2[16 * q + r][k0]);
        }
        const v8s bx = *reinterpret_cast<const v8s*>(&L.x[r][k0]);
        v8s ady = {0, 0, 0, 0, 0, 0, 0, 0};
        if (r < 2) ady = *reinterpret_cast<const v8s*>(&L.dy[r][k0]);
#pragma unroll
        for (int mo = 0; mo < 4; ++mo) {
            const v8s a2 = *reinterpret_cast<const v8s*>(&L.dz2[16 * mo + r][k0]);
            const v8s a1 = *reinterpret_cast<const v8s*>(&L.dz1[16 * mo + r][k0]);
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) gW2[mo][ni] = mfma32(a2, bh1[ni], gW2[mo][ni]);
            gW1[mo] = mfma32(a1, bx, gW1[mo]);
            gW3[mo] = mfma32(ady, bh2[mo], gW3[mo]);
        }
        __syncthreads();
    }
    float* out = part + static_cast<size_t>(blockIdx.x) * kPartStride;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 16 * a + 4 * g + j;
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) out[STA_MLP_OFF_W2 + row * 64 + 16 * ni + r] = gW2[a][ni][j];
            out[STA_MLP_OFF_W1 + row * 16 + r] = gW1[a][j];
            if (4 * g + j < 2) out[STA_MLP_OFF_W3 + (4 * g + j) * 64 + 16 * a + r] = gW3[a][j];
            const float v1 = sum16(gb1[a][j]);
            const float v2 = sum16(gb2[a][j]);
            if (r == 0) {
                out[STA_MLP_OFF_B1 + row] = v1;
                out[STA_MLP_OFF_B2 + row] = v2;
            }
        }
    const float t0 = sum16(gb3_0), t1 = sum16(gb3_1);
    float tot = sum16(sq);
    tot += __shfl_xor(tot, 16);
    tot += __shfl_xor(tot, 32);
    if (lane == 0) {
        out[STA_MLP_OFF_B3] = t0;
        out[STA_MLP_OFF_B3 + 1] = t1;
        out[STA_MLP_PARAMS] = 0.5f * tot * inv_batch;
    }
}

// Sum of the per-wave partials in a fixed order (sixteen interleaved groups of waves per
// parameter, each summed in wave order from loads issued eight at a time, then the groups
// in order); optional gradient output; optional Adam.  64 parameters per 1024-lane block.
constexpr int kAdamGroups = 16;
__global__ __launch_bounds__(64 * kAdamGroups) void k_mlp_adam(float* __restrict__ P, float* __restrict__ m,
                                                               float* __restrict__ v, const float* __restrict__ part,
                                                               int32_t waves, float* __restrict__ grad, int32_t adam,
                                                               float lr, float b1, float b2, float eps, float bc1,
                                                               float bc2) {
    __shared__ float red[kAdamGroups][64];
    const int pl = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + pl;
    float gs = 0.0f;
    if (p <= STA_MLP_PARAMS) {
        for (int w0 = grp; w0 < waves; w0 += 8 * kAdamGroups) {
            float x[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int w = w0 + r * kAdamGroups;
                x[r] = w < waves ? part[static_cast<size_t>(w) * kPartStride + p] : 0.0f;
            }
#pragma unroll
            for (int r = 0; r < 8; ++r)
                if (w0 + r * kAdamGroups < waves) gs += x[r];
        }
    }
    red[grp][pl] = gs;
    __syncthreads();
    if (grp != 0 || p > STA_MLP_PARAMS) return;
    gs = red[0][pl];
#pragma unroll
    for (int q = 1; q < kAdamGroups; ++q) gs += red[q][pl];
    if (grad) grad[p] = gs;
    if (!adam || p == STA_MLP_PARAMS) return;
    const float mm = b1 * m[p] + (1.0f - b1) * gs;
    const float vv = b2 * v[p] + (1.0f - b2) * gs * gs;
    m[p] = mm;
    v[p] = vv;
    P[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

__global__ __launch_bounds__(256) void k_mlp_predict(const float* __restrict__ P, const float* __restrict__ norm,
                                                     const float* __restrict__ feat, int32_t n,
                                                     float* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    Wf W;
    load_wf(P, g, r, W);
    const int tiles = (n + 15) / 16;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int stride = gridDim.x * 4;
    const NormL q = load_norm(norm, g);
    // features are loaded three tiles ahead of their use, in three registers with fixed
    // roles (a manual unroll by three, so no register is copied while its load is in flight)
    auto ahead = [&](int t) { return load_feat(feat, g, t * 16 + r, t < tiles && t * 16 + r < n, n); };
    auto tile_step = [&](int tile, float4& pr) {
        const float4 f = pr;
        pr = ahead(tile + 3 * stride);
        const v4s x = make_x(q, g, f);
        Fwd F;
        forward(W, x, F);
        // every lane stores (group 0's values; past the end, the last sample's again), so no
        // store sits in a branch and the waits for later tiles can leave stores in flight
        const int last = n - 1 - tile * 16;
        const int re = r < last ? r : last;
        const float y0 = __shfl(F.y[0], re), y1 = __shfl(F.y[1], re);
        *reinterpret_cast<float2*>(y + 2 * static_cast<size_t>(tile * 16 + re)) = make_float2(y0, y1);
    };
    float4 p0 = ahead(wave), p1 = ahead(wave + stride), p2 = ahead(wave + 2 * stride);
    for (int tile = wave; tile < tiles; tile += 3 * stride) {
        tile_step(tile, p0);
        if (tile + stride >= tiles) break;
        tile_step(tile + stride, p1);
        if (tile + 2 * stride >= tiles) break;
        tile_step(tile + 2 * stride, p2);
    }
}

__device__ __forceinline__ int cal_bin(float depth, float msize) {
    int d = static_cast<int>(depth);
    d = d < 1 ? 1 : (d > 8 ? 8 : d);
    int m = (static_cast<int>(msize) - 1) / 8;
    m = m < 0 ? 0 : (m > 7 ? 7 : m);
    return (d - 1) * 8 + m;
}

__device__ __forceinline__ int err_bucket(float e) {
    const int key = static_cast<int>(__float_as_uint(fabsf(e)) >> 21);
    const int k = 508 - key;
    return k < 0 ? 0 : (k > STA_CAL_BUCKETS - 1 ? STA_CAL_BUCKETS - 1 : k);
}

// The surrogate path for every sink: network, decode, error bound, fallback flag.
__global__ __launch_bounds__(256) void k_sur_eval(sta_trees T, const float* __restrict__ P,
                                                  const float* __restrict__ norm, const float* __restrict__ calib,
                                                  const float* __restrict__ feat, float tol, float* __restrict__ delay,
                                                  float* __restrict__ slew, uint8_t* __restrict__ sink_flag) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, r = lane & 15;
    Wf W;
    load_wf(P, g, r, W);
    const int n = T.n_sinks;
    const int tiles = (n + 15) / 16;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int stride = gridDim.x * 4;
    const NormL q = load_norm(norm, g);
    auto ahead = [&](int t) { return load_feat(feat, g, t * 16 + r, t < tiles && t * 16 + r < n, n); };
    auto tile_step = [&](int tile, float4& pr) {
        const float4 f = pr;
        pr = ahead(tile + 3 * stride);
        const v4s x = make_x(q, g, f);
        Fwd F;
        forward(W, x, F);
        const float msize = __shfl(f.x, r + 16);    // feature 4, held by lane group 1
        const float S = __shfl(f.w, r + 32);        // feature 11, held by lane group 2
        // computed on every lane, meaningful on lane group 0 (features 0..3).  Alpha is
        // clamped into [0, 1] (the Elmore bounds hold for every RC tree); the calibrated
        // bound is used when it beats the bound-midpoint estimate's 1/2
        const int bin = cal_bin(f.w, msize);
        const float qa = calib[2 * bin], qg = calib[2 * bin + 1];
        float a = fminf(fmaxf(F.y[0], 0.0f), 1.0f);
        float qd = fminf(qa, fmaxf(a, 1.0f - a));
        if (!(qa <= 0.5f)) {
            a = 0.5f;
            qd = 0.5f;
        }
        const float gm = fmaxf(F.y[1], 0.0f);
        const float L = (f.x * f.z) * 1e-3f;
        const float U = (f.x * f.y) * 1e-3f;
        const float d = L + a * (U - L);
        const float gg = gm * U;
        const float sl = sqrtf(S * S + gg * gg);
        const int bad = ((qd * (U - L) <= tol) && (qg * U <= tol)) ? 0 : 1;
        // unconditional stores from every lane (see k_mlp_predict)
        const int last = n - 1 - tile * 16;
        const int re = r < last ? r : last;
        const float dv = __shfl(d, re), sv = __shfl(sl, re);
        const int bv = __shfl(bad, re);
        const size_t so = static_cast<size_t>(tile * 16 + re);
        delay[so] = dv;
        slew[so] = sv;
        sink_flag[so] = static_cast<uint8_t>(bv);
    };
    float4 p0 = ahead(wave), p1 = ahead(wave + stride), p2 = ahead(wave + 2 * stride);
    for (int tile = wave; tile < tiles; tile += 3 * stride) {
        tile_step(tile, p0);
        if (tile + stride >= tiles) break;
        tile_step(tile + stride, p1);
        if (tile + 2 * stride >= tiles) break;
        tile_step(tile + 2 * stride, p2);
    }
}

__global__ __launch_bounds__(256) void k_cal_hist(const float* __restrict__ feat, const float* __restrict__ target,
                                                  const float* __restrict__ y, int32_t n,
                                                  uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[kCalEntries];
    for (int i = threadIdx.x; i < kCalEntries; i += 256) h[i] = 0;
    __syncthreads();
    for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) {
        const size_t q = static_cast<size_t>(s);
        const int bin = cal_bin(feat[q * 12 + 3], feat[q * 12 + 4]);
        const float e0 = fabsf(y[2 * q] - target[2 * q]);
        const float e1 = fabsf(y[2 * q + 1] - target[2 * q + 1]);
        atomicAdd(&h[(bin * 2 + 0) * STA_CAL_BUCKETS + err_bucket(e0)], 1u);
        atomicAdd(&h[(bin * 2 + 1) * STA_CAL_BUCKETS + err_bucket(e1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kCalEntries; i += 256)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ void k_cal_final(const uint32_t* __restrict__ hist, double quantile, int32_t min_count,
                            float* __restrict__ calib) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;    // bin * 2 + output
    if (i >= STA_CAL_BINS * 2) return;
    const uint32_t* h = hist + static_cast<size_t>(i) * STA_CAL_BUCKETS;
    long long n = 0;
    for (int k = 0; k < STA_CAL_BUCKETS; ++k) n += h[k];
    float q = __uint_as_float(0x7F800000u);
    if (n >= min_count) {
        const long long allow = static_cast<long long>(floor((1.0 - quantile) * static_cast<double>(n)));
        long long c = 0;
        for (int k = 0; k < STA_CAL_BUCKETS; ++k) {
            c += h[k];
            if (c > allow) {
                if (k > 0) q = __uint_as_float(static_cast<uint32_t>(509 - k) << 21);
                break;
            }
        }
    }
    calib[i] = q;
}

}  // namespace sur
}  // namespace sta

using namespace sta;
using namespace sta::sur;

static bool trees_ok(const sta_trees* t, bool need_sink_net, std::string& why) {
    if (!t) { why = "null trees"; return false; }
    if (t->n_nets < 0 || t->n_sinks < 0) { why = "negative count"; return false; }
    if (t->n_nets > 0 && (!t->net_node_ptr || !t->node_parent || !t->node_R || !t->node_C || !t->sink_ptr ||
                          !t->drv_slew)) { why = "null net array"; return false; }
    if (t->n_sinks > 0 && (!t->sink_node || !t->sink_pincap)) { why = "null sink array"; return false; }
    if (need_sink_net && t->n_sinks > 0 && !t->sink_net) { why = "null sink_net"; return false; }
    return true;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

extern "C" {

sta_status sta_tree_dataset(const sta_trees* t, float* feat, float* target, float* delay, float* slew,
                            int32_t* status, void* stream) {
    std::string why;
    if (!trees_ok(t, false, why)) return fail(STA_E_ARG, "sta_tree_dataset: " + why);
    if (t->n_nets == 0) return STA_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    constexpr int NT = 32;
    prof_launch("k_tree_dataset", s, [&] {
        hipLaunchKernelGGL((k_tree_dataset<NT>), dim3((t->n_nets + NT - 1) / NT), dim3(NT), 0, s, *t, feat, target,
                           delay, slew, status);
    });
    return launch_check("sta_tree_dataset");
}

sta_status sta_tree_exact(const sta_trees* t, const int32_t* net_list, const int32_t* net_count, float* delay,
                          float* slew, int32_t* status, void* stream) {
    std::string why;
    if (!trees_ok(t, false, why)) return fail(STA_E_ARG, "sta_tree_exact: " + why);
    if ((net_list == nullptr) != (net_count == nullptr)) return fail(STA_E_ARG, "sta_tree_exact: net_list and net_count go together");
    if (t->n_sinks > 0 && (!delay || !slew)) return fail(STA_E_ARG, "sta_tree_exact: null output");
    if (t->n_nets == 0) return STA_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    prof_launch("k_tree_exact", s, [&] {
        hipLaunchKernelGGL(k_tree_exact, dim3((t->n_nets + kExactWaves - 1) / kExactWaves), dim3(256), 0, s, *t,
                           net_list, net_count, delay, slew, status);
    });
    return launch_check("sta_tree_exact");
}

sta_status sta_tree_features(const sta_trees* t, float* feat, int32_t* status, void* stream) {
    std::string why;
    if (!trees_ok(t, false, why)) return fail(STA_E_ARG, "sta_tree_features: " + why);
    if (t->n_sinks > 0 && (!feat || !aligned16(feat))) return fail(STA_E_ARG, "sta_tree_features: null or unaligned feat");
    if (t->n_nets == 0) return STA_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    prof_launch("k_tree_features", s, [&] {
        hipLaunchKernelGGL(k_tree_features, dim3((t->n_nets + kExactWaves - 1) / kExactWaves), dim3(256), 0, s, *t,
                           feat, status);
    });
    return launch_check("sta_tree_features");
}

size_t sta_mlp_norm_scratch_bytes(void) { return sizeof(double) * 24 * kNormBlocks; }

sta_status sta_mlp_norm(const float* feat, int32_t n, float* norm, void* scratch, size_t scratch_bytes,
                        void* stream) {
    if (n < 0 || !norm || (n > 0 && !feat)) return fail(STA_E_ARG, "sta_mlp_norm: bad arguments");
    if (!scratch || scratch_bytes < sta_mlp_norm_scratch_bytes()) return fail(STA_E_ARG, "sta_mlp_norm: scratch too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = static_cast<double*>(scratch);
    prof_launch("k_norm_partial", s, [&] {
        hipLaunchKernelGGL(k_norm_partial, dim3(kNormBlocks), dim3(256), 0, s, feat, n, part);
    });
    prof_launch("k_norm_final", s, [&] {
        hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, s, part, kNormBlocks, n, norm);
    });
    return launch_check("sta_mlp_norm");
}

static int grad_waves(int32_t batch) {
    const int units = (batch + 31) / 32;
    return units < kMaxGradWaves ? units : kMaxGradWaves;
}

size_t sta_mlp_grad_scratch_bytes(int32_t batch) {
    if (batch <= 0) return 0;
    return sizeof(float) * static_cast<size_t>(kPartStride) * grad_waves(batch);
}

sta_status sta_mlp_train_step(float* params, float* adam_m, float* adam_v, const sta_adam* opt, const float* norm,
                              const float* feat, const float* target, const int32_t* idx, int32_t batch, float* grad,
                              void* scratch, size_t scratch_bytes, void* stream) {
    if (batch <= 0 || !params || !norm || !feat || !target || !idx) return fail(STA_E_ARG, "sta_mlp_train_step: bad arguments");
    if (!aligned16(feat)) return fail(STA_E_ARG, "sta_mlp_train_step: feat must be 16-byte aligned");
    if (opt && (!adam_m || !adam_v || opt->step < 1)) return fail(STA_E_ARG, "sta_mlp_train_step: Adam state missing or step < 1");
    if (!scratch || scratch_bytes < sta_mlp_grad_scratch_bytes(batch)) return fail(STA_E_ARG, "sta_mlp_train_step: scratch too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int waves = grad_waves(batch);
    float* part = static_cast<float*>(scratch);
    const float inv = 1.0f / static_cast<float>(batch);
    prof_launch("k_mlp_grad", s, [&] {
        hipLaunchKernelGGL(k_mlp_grad, dim3(waves), dim3(64), 0, s, params, norm, feat, target, idx, batch, inv, part);
    });
    float lr = 0.f, b1 = 0.f, b2 = 0.f, eps = 0.f, bc1 = 1.f, bc2 = 1.f;
    if (opt) {
        lr = opt->lr;
        b1 = opt->beta1;
        b2 = opt->beta2;
        eps = opt->eps;
        bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(b1), opt->step));
        bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(b2), opt->step));
    }
    prof_launch("k_mlp_adam", s, [&] {
        hipLaunchKernelGGL(k_mlp_adam, dim3((STA_MLP_PARAMS + 1 + 63) / 64), dim3(64 * kAdamGroups), 0, s, params,
                           adam_m, adam_v, part, waves, grad, opt ? 1 : 0, lr, b1, b2, eps, bc1, bc2);
    });
    return launch_check("sta_mlp_train_step");
}

static int stream_waves_grid(int32_t n) {
    const int tiles = (n + 15) / 16;
    const int blocks = (tiles + 3) / 4;
    return blocks < 2048 ? (blocks > 0 ? blocks : 1) : 2048;
}

sta_status sta_mlp_predict(const float* params, const float* norm, const float* feat, int32_t n, float* y,
                           void* stream) {
    if (n < 0 || !params || !norm || (n > 0 && (!feat || !y))) return fail(STA_E_ARG, "sta_mlp_predict: bad arguments");
    if (!aligned16(feat)) return fail(STA_E_ARG, "sta_mlp_predict: feat must be 16-byte aligned");
    if (n == 0) return STA_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    prof_launch("k_mlp_predict", s, [&] {
        hipLaunchKernelGGL(k_mlp_predict, dim3(stream_waves_grid(n)), dim3(256), 0, s, params, norm, feat, n, y);
    });
    return launch_check("sta_mlp_predict");
}

size_t sta_surrogate_cal_scratch_bytes(void) { return sizeof(uint32_t) * kCalEntries; }

sta_status sta_surrogate_calibrate(const float* feat, const float* target, const float* y, int32_t n,
                                   double quantile, int32_t min_count, float* calib, void* scratch,
                                   size_t scratch_bytes, void* stream) {
    if (n < 0 || !calib || (n > 0 && (!feat || !target || !y))) return fail(STA_E_ARG, "sta_surrogate_calibrate: bad arguments");
    if (!(quantile > 0.0 && quantile < 1.0)) return fail(STA_E_ARG, "sta_surrogate_calibrate: quantile must be in (0, 1)");
    if (!scratch || scratch_bytes < sta_surrogate_cal_scratch_bytes()) return fail(STA_E_ARG, "sta_surrogate_calibrate: scratch too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t* hist = static_cast<uint32_t*>(scratch);
    prof_launch("k_fill_i32", s, [&] {
        hipLaunchKernelGGL(k_fill_i32, dim3((kCalEntries + 255) / 256), dim3(256), 0, s,
                           reinterpret_cast<int32_t*>(hist), kCalEntries, 0);
    });
    if (n > 0) {
        int blocks = (n + 255) / 256;
        blocks = blocks < 512 ? blocks : 512;
        prof_launch("k_cal_hist", s, [&] {
            hipLaunchKernelGGL(k_cal_hist, dim3(blocks), dim3(256), 0, s, feat, target, y, n, hist);
        });
    }
    prof_launch("k_cal_final", s, [&] {
        hipLaunchKernelGGL(k_cal_final, dim3(1), dim3(STA_CAL_BINS * 2), 0, s, hist, quantile, min_count, calib);
    });
    return launch_check("sta_surrogate_calibrate");
}

sta_status sta_surrogate_eval(const sta_trees* t, const float* params, const float* norm, const float* calib,
                              const float* feat, float tol_ps, float* delay, float* slew, uint8_t* sink_flag,
                              int32_t* net_flag, int32_t* net_list, int32_t* net_count, int32_t* status,
                              void* stream) {
    std::string why;
    if (!trees_ok(t, false, why)) return fail(STA_E_ARG, "sta_surrogate_eval: " + why);
    if (!params || !norm || !calib || !net_count || (t->n_nets > 0 && (!net_flag || !net_list)) ||
        (t->n_sinks > 0 && (!feat || !delay || !slew || !sink_flag)))
        return fail(STA_E_ARG, "sta_surrogate_eval: bad arguments");
    if (!aligned16(feat)) return fail(STA_E_ARG, "sta_surrogate_eval: feat must be 16-byte aligned");
    if (!(tol_ps >= 0.0f)) return fail(STA_E_ARG, "sta_surrogate_eval: tol_ps must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nn = t->n_nets;
    prof_launch("k_fill_i32", s, [&] {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, net_count, 1, 0);
    });
    if (nn == 0) return launch_check("sta_surrogate_eval");
    if (t->n_sinks > 0)
        prof_launch("k_sur_eval", s, [&] {
            hipLaunchKernelGGL(k_sur_eval, dim3(stream_waves_grid(t->n_sinks)), dim3(256), 0, s, *t, params, norm,
                               calib, feat, tol_ps, delay, slew, sink_flag);
        });
    prof_launch("k_sur_compact", s, [&] {
        hipLaunchKernelGGL(k_sur_compact, dim3((nn + 255) / 256), dim3(256), 0, s, t->sink_ptr, sink_flag, nn,
                           net_flag, net_list, net_count);
    });
    prof_launch("k_tree_exact", s, [&] {
        hipLaunchKernelGGL(k_tree_exact, dim3((nn + kExactWaves - 1) / kExactWaves), dim3(256), 0, s, *t, net_list,
                           net_count, delay, slew, status);
    });
    return launch_check("sta_surrogate_eval");
}

}  // extern "C"

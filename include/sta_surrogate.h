/*
 * sta_surrogate.h -- RC-tree nets and the learned net delay/slew surrogate (libsta.so).
 *
 * Background.  Heteroflow's timing workload (Section IV-A) fits a regression model per
 * timing view on the GPU by gradient descent, next to the timer itself.  The learned
 * part here is a small network that predicts the Elmore delay and the PERI slew of every
 * sink of an RC-tree net from 12 features, trained on this library's own exact moments,
 * with the exact computation as fallback and as error judge.  The features are not free:
 * the downstream cap and the path sums need one upward sweep and a walk from every sink to
 * the driver (sta_tree_features), against the four sweeps of the exact moments, so an RC
 * tree's features cost about half of its exact delay and slew:
 *
 *   exact:      m1, m2 per tree node by the upward/downward sweeps of the RC-tree moments
 *               (the same definition sta_delay_calc uses on the nets of a timing graph),
 *               delay = fl32(m1), slew = sqrt(S^2 + fl32(max(0, 2 m2 - m1^2))) in FP32.
 *   features:   per sink, in this order: 0 R_path (ohm), 1 net load (fF), 2 downstream cap
 *               of the sink node, 3 edges on the path, 4 nodes in the net, 5 sinks in the
 *               net, 6 R of the first path edge, 7 cap of the path nodes (pin caps
 *               included), 8 mean edge R of the net, 9 mean wire cap of the net, 10 sink
 *               pin cap, 11 driver slew (ps).
 *   targets:    with the Elmore bounds L = R_path*Cd(sink)*1e-3 <= m1 <= U = R_path*load*1e-3,
 *               alpha = (m1 - L)/(U - L) (0 when U == L) and gamma = sqrt(imp2)/U (0 when U == 0).
 *   network:    12-64-64-2 with ReLU; input x_i = (log(1 + f_i) - mu_i) * rstd_i, zero-padded to
 *               16; matrix products on BF16 operands (rounded to nearest even) with FP32
 *               accumulation, biases and outputs in FP32; outputs (alpha, gamma).
 *   decode:     a = clamp(alpha, 0, 1), g = max(gamma, 0); delay = L + a*(U - L),
 *               slew = sqrt(S^2 + (g*U)^2) (FP32).  Since the true alpha lies in [0, 1],
 *               |a - alpha| <= max(a, 1 - a) always; the delay's error bound is
 *               e_d = min(q_a(bin), max(a, 1 - a)) * (U - L), except that where q_a(bin) > 1/2
 *               the bound midpoint (a = 1/2, e_d = (U - L)/2) is used instead.  The slew's
 *               error bound is e_s = q_g(bin) * U (sqrt(S^2 + x^2) is 1-Lipschitz in x).
 *   fallback:   a sink is trusted if e_d <= tol_ps and e_s <= tol_ps; a net with any
 *               untrusted sink is recomputed exactly.
 *
 * Conventions: every pointer is a device pointer unless stated; every call is
 * asynchronous on the caller's stream and allocates nothing; the caller owns all memory.
 * Status words (int32_t, device, optional) collect data errors found by the kernels as
 * bits (STA_TREE_ERR_*); the caller reads them after synchronizing.  Return values are
 * sta_status codes from sta.h; argument errors are detected before any launch.
 */
#ifndef STA_SURROGATE_H
#define STA_SURROGATE_H

#include "sta.h"

#ifdef __cplusplus
extern "C" {
#endif

#define STA_TREE_MAX_NODES 64      /* nodes per net (driver node included)               */
#define STA_MLP_IN 12
#define STA_MLP_HIDDEN 64
#define STA_MLP_OUT 2
/* FP32 parameter vector, natural row-major layout: W1[64][16] (columns 12..15 stay zero),
   b1[64], W2[64][64], b2[64], W3[2][64], b3[2] */
#define STA_MLP_OFF_W1 0
#define STA_MLP_OFF_B1 1024
#define STA_MLP_OFF_W2 1088
#define STA_MLP_OFF_B2 5184
#define STA_MLP_OFF_W3 5248
#define STA_MLP_OFF_B3 5376
#define STA_MLP_PARAMS 5378
#define STA_MLP_NORM 24            /* mu[12] then rstd[12], FP32                            */
#define STA_CAL_BINS 64            /* 8 depth classes x 8 net-size classes                  */
#define STA_CAL_BUCKETS 128

/* data-error bits written to a status word */
#define STA_TREE_ERR_SIZE 1        /* a net has more than STA_TREE_MAX_NODES or no nodes    */
#define STA_TREE_ERR_PARENT 2      /* parent of local node k not in 0..k-1                  */
#define STA_TREE_ERR_SINK 4        /* a sink taps a node outside its net                    */

/* A set of RC-tree nets.  Net n owns global nodes net_node_ptr[n] .. net_node_ptr[n+1]-1;
   local node 0 is the driver (its R is ignored), local node k > 0 hangs below local node
   node_parent[k] < k through resistance node_R[k] (ohm) and carries wire cap node_C[k]
   (fF).  Sinks sink_ptr[n] .. sink_ptr[n+1]-1 tap local node sink_node[s] with pin cap
   sink_pincap[s]; sink_net[s] = n (optional, not read by the kernels).  drv_slew[n] is the
   driver's output slew (ps).
   Values must be finite and non-negative (the kernels do not check values). */
typedef struct {
    int32_t n_nets;
    int32_t n_sinks;
    const int32_t* net_node_ptr;   /* [n_nets+1]  */
    const int32_t* node_parent;    /* [nodes]     */
    const float* node_R;           /* [nodes]     */
    const float* node_C;           /* [nodes]     */
    const int32_t* sink_ptr;       /* [n_nets+1]  */
    const int32_t* sink_node;      /* [n_sinks]   */
    const float* sink_pincap;      /* [n_sinks]   */
    const float* drv_slew;         /* [n_nets]    */
    const int32_t* sink_net;       /* [n_sinks]   */
} sta_trees;

typedef struct {
    float lr, beta1, beta2, eps;   /* Adam (Kingma & Ba), bias-corrected                     */
    int32_t step;                  /* 1-based update count                                   */
} sta_adam;

/* Training set builder: features feat[S][12], targets target[S][2] = (alpha, gamma) (FP64
   moments and targets rounded once to FP32), and the exact delay[S], slew[S].  Any output
   pointer may be NULL.  One thread per net, FP64 sweeps in the order of the definition. */
sta_status sta_tree_dataset(const sta_trees* t, float* feat, float* target, float* delay, float* slew,
                            int32_t* status, void* stream);

/* Passage: Section IV-A (the inputs of the regression the correlation layer fits).
 * The 12 features of every sink only, feat[S][12] (16-byte aligned), bit for bit those of
 * sta_tree_dataset, without its moment sweeps: node caps, the downstream caps and each
 * sink's path to the driver.  One wavefront per net.  Errors: STA_E_ARG; a malformed net
 * sets a bit of *status as in sta_tree_exact. */
sta_status sta_tree_features(const sta_trees* t, float* feat, int32_t* status, void* stream);

/* Exact delay[S] and slew[S] (FP64 moments).  With net_list == NULL every net is done;
   otherwise only nets net_list[0 .. *net_count - 1] (net_count is a device int32 <= n_nets)
   and the other sinks' outputs are left untouched. */
sta_status sta_tree_exact(const sta_trees* t, const int32_t* net_list, const int32_t* net_count,
                          float* delay, float* slew, int32_t* status, void* stream);

/* Input normalization from n feature rows: norm = (mean, 1/std) per
   feature (of log(1 + f); population std over FP64 sums; 1 where the std is 0).  scratch: at least
   sta_mlp_norm_scratch_bytes() bytes of device memory. */
size_t sta_mlp_norm_scratch_bytes(void);
sta_status sta_mlp_norm(const float* feat, int32_t n, float* norm, void* scratch, size_t scratch_bytes,
                        void* stream);

/* One training step on the batch feat[idx[b]], target[idx[b]], b < batch: forward, loss
   0.5 * mean_b |y_b - t_b|^2, backward (BF16 operands, FP32 accumulation), and the
   gradient summed in a fixed order (bitwise reproducible).  grad (optional) receives the
   STA_MLP_PARAMS gradients followed by the loss.  With opt != NULL the parameters are
   then updated in place by Adam (m, v: STA_MLP_PARAMS floats each, zero before step 1).
   scratch: at least sta_mlp_grad_scratch_bytes(batch) bytes. */
size_t sta_mlp_grad_scratch_bytes(int32_t batch);
sta_status sta_mlp_train_step(float* params, float* adam_m, float* adam_v, const sta_adam* opt,
                              const float* norm, const float* feat, const float* target, const int32_t* idx,
                              int32_t batch, float* grad, void* scratch, size_t scratch_bytes,
                              void* stream);

/* Network outputs y[n][2] = (alpha, gamma) for feature rows 0..n-1. */
sta_status sta_mlp_predict(const float* params, const float* norm, const float* feat, int32_t n, float* y,
                           void* stream);

/* Error calibration on held-out rows: per (bin, output) the upper edge of the histogram
   bucket holding the `quantile` of |y - target| (bins with fewer than min_count rows, or
   whose quantile lies in the top bucket, get +inf).  Bin = 8*(clamp(depth,1,8)-1) +
   clamp((M-1)/8, 0, 7); buckets are quarter octaves read from the FP32 bits of the error
   (bucket = clamp(508 - (bits >> 21), 0, 127)).  calib: [STA_CAL_BINS][2] floats.
   scratch: at least sta_surrogate_cal_scratch_bytes() bytes. */
size_t sta_surrogate_cal_scratch_bytes(void);
sta_status sta_surrogate_calibrate(const float* feat, const float* target, const float* y, int32_t n,
                                   double quantile, int32_t min_count, float* calib, void* scratch,
                                   size_t scratch_bytes, void* stream);

/* The surrogate path: network, decode and error bound for every sink; nets with an
   untrusted sink are listed (net_list, *net_count; order unspecified) and recomputed
   exactly.  delay/slew: [S]; sink_flag: [S] uint8 scratch (1 = untrusted sink);
   net_flag: [n_nets] int32 output (1 = recomputed exactly); net_list: [n_nets];
   net_count: one device int32. */
sta_status sta_surrogate_eval(const sta_trees* t, const float* params, const float* norm, const float* calib,
                              const float* feat, float tol_ps, float* delay, float* slew, uint8_t* sink_flag,
                              int32_t* net_flag, int32_t* net_list, int32_t* net_count, int32_t* status,
                              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* STA_SURROGATE_H */

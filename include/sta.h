/*
 * sta.h -- C ABI of the MI355X levelized static-timing-analysis library (libsta.so).
 *
 * Background.  Heteroflow (Huang & Lin, "Concurrent CPU-GPU Task Programming using
 * Modern C++", Section IV-A) drives a timer over a 1.5M-gate design for many timing
 * views, a view being one process corner combined with one analysis mode.  The paper
 * treats the timer as a black box; this library is that timer's data-parallel core:
 * levelization, RC-net delay calculation, NLDM table lookup, forward arrival/slew
 * propagation and backward required-time/slack analysis, for several views at once.
 * The paper's runtime hands every GPU task a stream and a pooled allocator (Section
 * III-A pull/kernel tasks, Section III-C memory pool); here the caller owns both: every
 * device buffer is allocated by the caller and every call is asynchronous on the
 * caller's stream.
 *
 * Conventions used by every entry point.
 *  - Units: time ps, capacitance fF, resistance ohm (1 ohm * 1 fF = 1e-3 ps).
 *  - Input numbering: drivers 0..n_pi-1 are primary inputs, n_pi+g is gate g's output.
 *  - Internal numbering: sta_build_graph renumbers gates by (level, input id); primary
 *    inputs keep their ids.  Every device output is in internal order; sta_graph_perm
 *    gives the map back to input ids.
 *  - Views: a call evaluates n_views (1, 2, 4 or 8) views together; per-element device
 *    arrays interleave the views, element-major: X[elem][view] (and [elem][view][2]
 *    for (arrival, slew) pairs).
 *  - Errors: every call returns an sta_status; sta_last_error() gives the text of the
 *    last non-OK status of the calling thread.  Validation errors are detected on the
 *    host before anything is launched.  A launch failure returns STA_E_HIP; faults
 *    during execution surface at the caller's next synchronization of the stream.
 *  - Threads: calls on distinct graphs are independent.  A graph is read-only after
 *    sta_graph_upload, so concurrent calls on it from several streams are allowed as
 *    long as their output (and scratch) buffers differ.  The launch sequences a graph
 *    replays are cached per argument set (up to four per call kind), so such callers
 *    replay without re-capturing; a fifth argument set evicts the least recently used
 *    one after waiting for the device.  No C++ exception crosses this ABI.
 */
#ifndef STA_H
#define STA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STA_OK = 0,
    STA_E_ARG = -1,        /* null/undersized buffer, bad size or count, unsupported option */
    STA_E_RANGE = -2,      /* an index out of range (driver, table, RC node, parent)        */
    STA_E_CYCLE = -3,      /* the gate graph has a combinational cycle                      */
    STA_E_NONFINITE = -4,  /* NaN/Inf (or a negative R, C or pin cap) in the design          */
    STA_E_ALLOC = -5,      /* host memory exhausted                                         */
    STA_E_HIP = -6         /* a HIP runtime call failed; the text names it                  */
} sta_status;

typedef enum { STA_LATE = 0, STA_EARLY = 1 } sta_mode;

typedef enum {
    STA_DC_FP64 = 0,       /* RC moments in FP64, the operation order of the definition      */
    STA_DC_FP32 = 1        /* RC moments in FP32 (same order); within 1e-5 relative on
                              shallow nets, see sta_delay_calc                               */
} sta_dc_precision;

#define STA_MAX_VIEWS 8
#define STA_MAX_FANIN 64       /* cell arcs per gate                                          */
#define STA_MAX_NET_NODES 256  /* RC nodes per net                                            */
#define STA_MAX_TABLES 65535

/* Design description (host memory, read during sta_build_graph only; the caller keeps
 * ownership).  A = gate_arc_ptr[n_gates], D = n_pi + n_gates, M = net_node_ptr[D].
 *   gate_arc_ptr[G+1]  cell arcs of gate g are gate_arc_ptr[g] .. gate_arc_ptr[g+1]-1;
 *                      1 <= arcs per gate <= STA_MAX_FANIN; gate_arc_ptr[0] = 0
 *   arc_drv[A]         driver of the net feeding arc a's input pin, 0 <= . < D
 *   arc_tbl[A]         NLDM table pair of arc a, 0 <= . < n_tables
 *   arc_tap[A]         RC node (local to that net) the input pin taps
 *   arc_pincap[A]      input pin capacitance, fF, finite and >= 0
 *   net_node_ptr[D+1]  RC nodes of driver d's net; 1 <= nodes <= STA_MAX_NET_NODES
 *   node_parent[M]     local parent: -1 at local node 0 (the driver), else 0 <= p < k
 *   node_R[M]          resistance of the edge parent -> node (ignored at node 0), ohm
 *   node_C[M]          wire capacitance at the node, fF
 * A driver with no sink is an endpoint; endpoints are ranked by ascending input id. */
typedef struct {
    int32_t n_pi;
    int32_t n_gates;
    int32_t n_tables;
    const int32_t* gate_arc_ptr;
    const int32_t* arc_drv;
    const int32_t* arc_tbl;
    const int32_t* arc_tap;
    const float* arc_pincap;
    const int32_t* net_node_ptr;
    const int32_t* node_parent;
    const float* node_R;
    const float* node_C;
} sta_design_desc;

typedef struct {
    int64_t n_pi, n_gates, n_drivers, n_arcs, n_nodes, n_pins;
    int64_t n_levels;          /* highest gate level L (levels 1..L; primary inputs are 0) */
    int64_t n_endpoints;
    int64_t max_fanin, max_fanout, max_net_nodes;
    int64_t n_fwd_tiles, n_bwd_tiles;
    size_t graph_bytes;        /* device bytes sta_graph_upload needs                        */
    size_t scratch_bytes;      /* device scratch bytes sta_slack needs                       */
} sta_sizes;

typedef struct sta_graph sta_graph;   /* opaque; owns host memory only */

/* Shared NLDM library of a call.  x: input-slew axis (ps), y: load axis (fF), both
 * strictly increasing, host values.  tables: device, [n_sets][n_tables][2][7][7] FP32,
 * [.][.][0] the delay table and [.][.][1] the output-slew table, row-major over
 * (slew index, load index).  A corner is a table set (its tables pre-scaled). */
typedef struct {
    float x[7];
    float y[7];
    const float* tables;
    int32_t n_sets;
    int32_t n_tables;
} sta_library;

/* Views of one call: n_views in {1,2,4,8}; view v analyses mode[v] with table set
 * table_set[v]. */
typedef struct {
    int32_t n_views;
    int32_t mode[STA_MAX_VIEWS];
    int32_t table_set[STA_MAX_VIEWS];
} sta_views;

/* Delay-calculation outputs, device, internal order. */
typedef struct {
    float* load;          /* [D]  lumped net capacitance seen by the driver, fF        */
    float* net_delay;     /* [A]  Elmore delay driver -> input pin, ps                  */
    float* net_imp2;      /* [A]  step-response spread 2*m2 - m1^2 at the pin, ps^2     */
    float* arc_load;      /* [A]  load of the gate output each cell arc drives (= load of
                                  that gate's net; a per-arc copy the forward pass reads
                                  with the arc's other data)                              */
} sta_net_out;

/* Forward outputs, device, internal order, views interleaved. */
typedef struct {
    float* drv_ts;        /* [D][V][2]  (arrival, slew) of every driver pin            */
    float* arc_ts;        /* [A][V][2]  (arrival, slew) of every gate input pin        */
    float* arc_delay;     /* [A][V]     NLDM cell-arc delay                            */
    uint8_t* argmax;      /* [G][V]     winning arc (0-based within the gate)          */
} sta_timing_out;

/* Backward outputs, device, internal order, views interleaved. */
typedef struct {
    float* drv_rat;       /* [D][V] */
    float* arc_rat;       /* [A][V] */
    float* drv_slack;     /* [D][V] */
    float* arc_slack;     /* [A][V] */
    double* tns;          /* [V]  sum of negative endpoint slacks, exact then rounded once */
    float* wns;           /* [V]  minimum endpoint slack (+inf without endpoints)          */
} sta_slack_out;

const char* sta_last_error(void);

/* Passage: Section II-A (a computation waits until the quantities it depends on have
 * arrived: here a gate waits for its fanin drivers) and Section IV-A (the circuit a timer
 * analyses).  The paper gives no levelization; the definition is Kahn's algorithm.
 * Levelizes the design (Kahn; level(PI) = 0, level(g) = 1 + max level of g's fanin
 * drivers), checks it, and builds the level-sorted CSR and the wave-sized work tiles.
 * Host only and synchronous; copies what it needs.  Errors: STA_E_ARG, STA_E_RANGE,
 * STA_E_CYCLE, STA_E_NONFINITE, STA_E_ALLOC.  *out is set only on STA_OK. */
sta_status sta_build_graph(const sta_design_desc* d, sta_graph** out);

/* No passage: a tiling choice of this library (the level-tile size an autotuner may pick).
 * sta_build_graph with the longest fused span capped at fwd_levels gate levels (forward)
 * and bwd_levels driver levels (backward), each 1..8; sta_build_graph uses 8 and 8.
 * Shorter spans mean more launches and smaller fan-in cones per tile; results do not
 * change.  Errors: those of sta_build_graph, STA_E_ARG for a length outside 1..8. */
sta_status sta_build_graph_spans(const sta_design_desc* d, int32_t fwd_levels, int32_t bwd_levels,
                                 sta_graph** out);

/* Sizes of a built graph (host, synchronous).  Errors: STA_E_ARG (null argument). */
sta_status sta_graph_sizes(const sta_graph* g, sta_sizes* out);

/* Host copies of the maps (each pointer may be null):
 *   drv_input[D]   input driver id of internal driver i
 *   arc_input[A]   input arc id of internal arc i
 *   gate_input[G]  input gate id of internal gate i
 *   level[D]       level of internal driver i
 *   ep_driver[E]   internal driver id of the endpoint of rank r */
sta_status sta_graph_perm(const sta_graph* g, int32_t* drv_input, int32_t* arc_input,
                          int32_t* gate_input, int32_t* level, int32_t* ep_driver);

/* Passage: Section III-A, pull task (host data copied into device memory the runtime
 * provides; here the caller provides it).
 * Copies the graph's device arrays into dev_buf (caller-owned device memory of at least
 * graph_bytes, 256-byte aligned) on stream s, waits for the copy, and keeps dev_buf's
 * address; dev_buf must outlive every later call on g.  A graph may be uploaded again
 * (to the same or another buffer): the launch sequences captured against the previous
 * buffer are dropped first (after waiting for the device), so the old buffer may be
 * freed once this returns.  The host arrays stay owned by g.  Errors: STA_E_ARG (null,
 * undersized or unaligned buffer), STA_E_HIP. */
sta_status sta_graph_upload(sta_graph* g, void* dev_buf, size_t bytes, void* stream);

void sta_graph_free(sta_graph* g);

/* Passage: Section IV-A (the timer's delay calculation, a black box there).  The paper
 * states no formula; the moments below are the Elmore / second-moment definitions of
 * RC trees (Rubinstein, Penfield and Horowitz).
 * RC delay calculation of every net: per node total cap C = wire cap + tapped pin caps
 * (sinks in ascending input arc id), downstream cap Cd, load = Cd(driver), Elmore
 * m1(k) = m1(parent) + R(k) Cd(k) 1e-3, W = downstream sum of C m1,
 * m2(k) = m2(parent) + R(k) W(k) 1e-3, imp2 = max(0, 2 m2 - m1^2); outputs rounded to
 * FP32 once.  STA_DC_FP64 evaluates exactly that operation sequence in FP64 (the CPU
 * definition's results, bit for bit); STA_DC_FP32 does the same in FP32.  Also writes
 * arc_load.  One net per lane; asynchronous on stream. */
sta_status sta_delay_calc(const sta_graph* g, sta_dc_precision prec, const sta_net_out* out,
                          void* stream);

/* Passage: Section IV-A (a timer evaluated per view, a view being one corner combined
 * with one analysis mode).  The paper states no timing formula; these are the standard
 * NLDM lookup and max/min arrival propagation, written out here.
 * Forward propagation of all views, level by level.  pi_ts: device [n_pi][V][2]
 * (arrival, slew) of the primary inputs.  For each gate output o and each cell arc a
 * (input pin i, net driver u):
 *   AT_i = AT_u + net_delay_a;  S_i = sqrt(S_u*S_u + net_imp2_a);
 *   d_a, s_a = NLDM(delay, slew tables of a; S_i, load_o)  (bilinear, end segments
 *              extrapolate, every FP32 operation rounded separately);
 *   late:  AT_o = max_a (AT_i + d_a), argmax = smallest a reaching it, S_o = max_a s_a;
 *   early: min in place of max.
 * Results equal the CPU definition bit for bit.  Asynchronous on stream. */
sta_status sta_propagate(const sta_graph* g, const sta_library* lib, const sta_views* views,
                         const float* pi_ts, const sta_net_out* nd, const sta_timing_out* out,
                         void* stream);

/* Passage: Section IV-A (the timing reports the correlation layer reads: slacks,
 * critical paths).  Required times and slack follow the standard definition, written
 * out here (the paper states none).
 * Backward required times, slacks and endpoint summaries of all views.  ep_rat: device
 * [E][V] required time of every endpoint (rank order).  Late views:
 *   RAT_u = min over u's sink pins i of (RAT_i - net_delay_i), or ep_rat at an endpoint;
 *   RAT_i = RAT_o - d_a;  slack = RAT - AT.
 * Early views: max in place of min and slack = AT - RAT.  tns/wns over endpoints.
 * scratch: device, >= scratch_bytes, contents on entry ignored.  Asynchronous. */
sta_status sta_slack(const sta_graph* g, const sta_views* views, const sta_net_out* nd,
                     const sta_timing_out* t, const float* ep_rat, const sta_slack_out* out,
                     void* scratch, size_t scratch_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).
 * sta_slack without the scratch argument: the endpoint partials go to a static device
 * array of the library (192 KiB, one per device, held until the process ends; its
 * address is looked up on the first call on each device).  Results are those of
 * sta_slack bit for bit.  The launches are made directly on the stream (no launch-
 * sequence capture and replay); no device memory is allocated or freed.  The scratch
 * sta_slack needs has a fixed size (scratch_bytes, independent of the design), checked
 * against the static array's size: a larger need is refused with STA_E_ARG.  All calls
 * on one device share the array: calls that overlap on one device (two streams, or two
 * host threads) race on it and give undefined TNS/WNS; serialize them.  Its contents on
 * entry are ignored (every partial is written before it is read).  Errors: those of
 * sta_slack, and STA_E_HIP if the array's address cannot be obtained. */
sta_status sta_slack_noalloc(const sta_graph* g, const sta_views* views, const sta_net_out* nd,
                             const sta_timing_out* t, const float* ep_rat, const sta_slack_out* out,
                             void* stream);

/* Passage: Section III-B (a task graph run many times, run_n: here the captured launch
 * sequence replayed as a hipGraph).
 * Schedule of sta_propagate and sta_slack on graph g.  The view schedule (one workgroup
 * per view walks every level, a workgroup barrier between levels) is used when the
 * design's mean cell arcs per level is at most view_max_arcs_per_level (and the level
 * data fits in LDS), the level schedule (launches per level or per fused span, all views
 * per launch) otherwise.  0 forces the level schedule.  A negative value restores the
 * library's choice (the default): the level schedule with fused spans (the view schedule
 * only when fusion is off, up to 512 mean cell arcs per level).
 * use_graphs != 0 (the default) lets the level schedule capture its launch sequence in a
 * hipGraph on first use and replay it while the call's arguments stay the same (the
 * captures are per graph and per call kind, up to four argument sets each; an argument
 * set not among them is captured, evicting the least recently used after waiting for
 * the device).
 * Every choice gives identical results. */
sta_status sta_set_schedule(sta_graph* g, int32_t view_max_arcs_per_level, int32_t use_graphs);

/* No passage: a scheduling choice of this library (the paper's kernels are one task
 * each).  Errors: STA_E_ARG (null graph).
 * Level fusion of the level schedule (default on): up to eight
 * consecutive gate levels per forward launch and up to eight driver levels per backward
 * launch (the same spans serve the TNS adjoint).  Each workgroup (one wavefront) computes
 * one span tile: in the forward pass a set of gates closed under fanin inside the span
 * (<= 64 cell arcs per level), in the backward pass a set of drivers closed under their
 * sinks' gate outputs inside the span (each level in one or more chunks of <= 64 sink
 * slots, at most eight chunks per tile), level by level, with the in-span arrival
 * (required) times kept in LDS.  A gate or driver needed by several
 * tiles is computed in each of them, identically, so results do not change.  A level that
 * cannot be tiled even alone runs as a level launch, and so does every level of a graph
 * of more than 2^26 cell arcs or drivers (the span kernels address by 32-bit offsets and
 * pack indices into 26 bits).  The view schedule is unaffected. */
sta_status sta_set_level_fusion(sta_graph* g, int32_t enable);

/* The fusion plan of a built graph (host only; independent of sta_set_level_fusion,
 * which decides whether it is used).  Launch counts are those of one forward or one
 * backward pass with fusion on (any view count); the fused kernels' algorithmic work is
 * the gates, cell arcs, drivers and sink arcs of their spans counted once, and
 * *_computed counts evaluations as performed (a cone shared by several tiles is
 * evaluated in each). */
typedef struct {
    int64_t fwd_spans, fwd_spans_fused;         /* forward spans, of which fused          */
    int64_t fwd_span_launches;                  /* fused forward launches (non-empty)      */
    int64_t fwd_level_launches;                 /* level launches of the unfused spans     */
    int64_t fwd_span_gates, fwd_span_arcs;      /* gates and cell arcs of the fused spans   */
    int64_t fwd_span_arcs_computed;
    int64_t fwd_span_tiles;
    int64_t bwd_spans, bwd_spans_fused;
    int64_t bwd_span_launches, bwd_level_launches;
    int64_t bwd_span_drivers, bwd_span_arcs;    /* drivers and their sink arcs, fused spans */
    int64_t bwd_span_slots_computed;            /* sink slots evaluated (a driver without
                                                   fanout has one slot)                    */
    int64_t bwd_span_tiles;
} sta_span_info;

sta_status sta_graph_spans(const sta_graph* g, sta_span_info* out);

/* The spans themselves, host arrays (either may be null):
 *   fwd[fwd_spans][3]  first gate level, last gate level, fused (1) or level launch (0),
 *                      in launch order (bottom up)
 *   bwd[bwd_spans][3]  top driver level, bottom driver level, fused, in launch order
 *                      (top down)
 * Spans partition the levels: forward 1..L, backward 0..L.  A span is at most eight
 * levels long; the builder takes the longest span from the next uncovered level that can
 * be tiled, and an unfused span is a single level. */
sta_status sta_graph_span_list(const sta_graph* g, int32_t* fwd, int32_t* bwd);

/* Per-kernel timing record of the instrumentation calls below. */
typedef struct {
    char name[48];        /* kernel name (template arguments dropped)      */
    int64_t launches;     /* launches bracketed while profiling was active  */
    double total_ms;      /* sum of their durations, from HIP events        */
} sta_kernel_stat;

/* Instrumentation, not for the timed path.  Between sta_profile_begin and
 * sta_profile_end on the calling thread, every kernel launch the library makes is
 * bracketed by two HIP events recorded on the launch's stream.  sta_profile_end waits
 * for those events, writes up to cap records (one per kernel name) and the number of
 * names to *n, and stops profiling.  Errors: STA_E_ARG (not active, null out),
 * STA_E_HIP (an event call failed). */
sta_status sta_profile_begin(void);
sta_status sta_profile_end(sta_kernel_stat* stats, int32_t cap, int32_t* n);

#ifdef __cplusplus
}
#endif
#endif /* STA_H */

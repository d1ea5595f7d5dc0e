/*
 * sta_batch.h -- many designs and corners in one launch sequence (libsta.so).
 *
 * Background.  Heteroflow's timing workload analyses one design under many timing views
 * (a view is a process corner combined with an analysis mode, Section IV-A), and its
 * runtime balances uneven tasks by work stealing (Section III-C) and reruns a task graph
 * many times (Executor::run_n).  Here a batch is a set of uploaded graphs of uneven size
 * that share one NLDM library and one set of views (for instance four corners as four
 * table sets).  Three passes, each one captured launch sequence for the whole batch:
 *   sta_batch_delay_calc  every design's RC moments, one launch per node-count class;
 *   sta_batch_propagate   the forward pass of every (graph, view), by each design's
 *                         schedule:
 *     - STA_BATCH_SPANS: step s runs the s-th fused span of every such design, all its
 *       views, as ONE launch (the designs' tiles side by side: the dependent-level
 *       latency of one design is shared with all the others); a span that does not fuse
 *       runs as that design's level launches in the same step;
 *     - STA_BATCH_PERSISTENT: ONE launch whose workgroups claim (graph, view) units from
 *       a device counter, largest first, each unit walking all levels of its graph inside
 *       one workgroup;
 *     - STA_BATCH_LEVELS: one launch per level for all views;
 *   sta_batch_slack       the backward pass (required times, slacks, TNS, WNS) of every
 *                         design given slack buffers, by backward spans in steps as
 *                         above, then one endpoint-summary launch for all designs.
 * Which schedule each design takes is the caller's plan (the package's autotuner times
 * the candidate plans and caches its choice per size class).  Results are those of
 * sta_delay_calc, sta_propagate and sta_slack on each graph, bit for bit.
 *
 * Ownership: the caller owns the graphs, their net data, outputs and the device
 * workspace; the batch keeps pointers to all of them and must be freed before they are.
 */
#ifndef STA_BATCH_H
#define STA_BATCH_H

#include "sta.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sta_batch sta_batch;

#define STA_BATCH_PERSISTENT 0
#define STA_BATCH_LEVELS 1
#define STA_BATCH_SPANS 2

typedef struct {
    const sta_graph* g;           /* uploaded graph                                          */
    const float* pi_ts;           /* [n_pi][V][2] primary-input (arrival, slew), device        */
    const sta_net_out* nd;        /* its net data: written by sta_batch_delay_calc, read by
                                     the other two passes (device)                           */
    const sta_timing_out* out;    /* its forward outputs (device)                             */
    int32_t schedule;             /* forward pass: STA_BATCH_SPANS, STA_BATCH_PERSISTENT or
                                     STA_BATCH_LEVELS; a graph the persistent kernel cannot
                                     stage (a level chunk over the LDS caps) runs by spans  */
    const float* ep_rat;          /* [E][V] endpoint required times (device), or NULL: the
                                     design takes no part in sta_batch_slack                 */
    const sta_slack_out* sl;      /* its slack outputs (device), or NULL with ep_rat          */
} sta_batch_design;

/* Device workspace of a batch of these designs with n_views views (descriptor table,
 * persistent unit list and counter, the per-launch tile maps of the span steps, the
 * delay-calculation and endpoint maps, and the endpoint partials).  0 on bad arguments. */
size_t sta_batch_workspace_bytes(const sta_batch_design* designs, int32_t n, int32_t n_views);

/* Builds the batch: validates, plans the steps, orders the persistent units by decreasing
 * size, and uploads the tables into the workspace (synchronously).  Errors: STA_E_ARG
 * (null or missing buffers, graph not uploaded, library too small, bad views or schedule,
 * workspace too small), STA_E_ALLOC, STA_E_HIP. */
sta_status sta_batch_create(const sta_batch_design* designs, int32_t n, const sta_library* lib,
                            const sta_views* views, void* workspace, size_t workspace_bytes, sta_batch** out);

/* Passage: Section IV-A (the timer's delay calculation, here for many designs at once).
 * The RC delay calculation of every design (sta_delay_calc's definition and precision
 * modes), one launch per node-count class of the designs.  use_graph != 0 replays a
 * captured sequence.  Asynchronous. */
sta_status sta_batch_delay_calc(sta_batch* b, sta_dc_precision prec, int32_t use_graph, void* stream);

/* Passage: Section IV-A (one timer run per view, many views) and Section III-C (uneven
 * tasks balanced on the device: the span steps and the persistent unit queue).
 * The forward pass of every design and view.  use_graph != 0 replays a hipGraph of the
 * whole launch sequence (captured on first use).  persistent_blocks: workgroups of the
 * persistent launch (0: one per compute unit).  Asynchronous. */
sta_status sta_batch_propagate(sta_batch* b, int32_t use_graph, int32_t persistent_blocks, void* stream);

/* Passage: Section IV-A (the timing reports of every view).  Required times, slacks and
 * endpoint summaries of every design given slack buffers (sta_slack's definition), by
 * backward span steps and one batched endpoint summary.  Asynchronous. */
sta_status sta_batch_slack(sta_batch* b, int32_t use_graph, void* stream);

/* No passage: a tiling choice of this library (what the package's autotuner tunes).
 * Views computed per wavefront by the batched span launches: 1, 2 or 4 (at most the view
 * count); the other views of a tile run in other workgroups of the same launch.  More
 * views per wavefront read a tile's records and gathers once for all of them (less
 * traffic, the batch being bound by throughput), fewer give shorter chains.  Defaults:
 * 1 forward, 1 backward.  Captured sequences are dropped when a value changes; results
 * do not change.  Errors: STA_E_ARG. */
sta_status sta_batch_set_tiling(sta_batch* b, int32_t fwd_views_per_wave, int32_t bwd_views_per_wave);

/* The plan of a batch (for reports). */
typedef struct {
    int32_t span_designs, persistent_designs, level_designs;   /* forward schedules       */
    int32_t persistent_units;                                 /* (graph, view) units     */
    int32_t fwd_steps, fwd_span_tiles;   /* span steps of the forward pass, tiles of their
                                            batched launches (each run for every view)  */
    int32_t bwd_steps, bwd_span_tiles;   /* the same for sta_batch_slack                 */
    int32_t slack_designs;
    int32_t dc_launches;                 /* launches of sta_batch_delay_calc             */
} sta_batch_plan;

sta_status sta_batch_info(const sta_batch* b, sta_batch_plan* out);

void sta_batch_free(sta_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* STA_BATCH_H */

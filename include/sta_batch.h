/*
 * sta_batch.h -- many designs and corners in one launch (libsta.so).
 *
 * Background.  Heteroflow's timing workload analyses one design under many timing views
 * (a view is a process corner combined with an analysis mode, Section IV-A), and its
 * runtime balances uneven tasks by work stealing (Section III-C) and reruns a task graph
 * many times (Executor::run_n).  Here a batch is a set of uploaded graphs of uneven size
 * that share one NLDM library and one set of views (for instance four corners as four
 * table sets).  sta_batch_propagate runs the forward pass of every (graph, view) unit:
 *   - graphs planned for the persistent schedule go to ONE launch whose workgroups claim
 *     (graph, view) units from a device counter, largest first, each unit walking all
 *     levels of its graph inside one workgroup (no grid-wide synchronization);
 *   - graphs planned for the level schedule run one launch per level for all views.
 * The whole sequence can be captured once in a hipGraph and replayed.  Which graphs go
 * where is the caller's plan (the package's autotuner measures both schedules per design
 * size class and caches its choice).  Results are those of sta_propagate on each graph,
 * bit for bit.
 *
 * Ownership: the caller owns the graphs, their net data and outputs (as for
 * sta_propagate) and the device workspace; the batch keeps pointers to all of them and
 * must be freed before they are.
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

typedef struct {
    const sta_graph* g;           /* uploaded graph                                          */
    const float* pi_ts;           /* [n_pi][V][2] primary-input (arrival, slew), device        */
    const sta_net_out* nd;        /* its delay-calculation results (device)                   */
    const sta_timing_out* out;    /* its forward outputs (device)                             */
    int32_t schedule;             /* STA_BATCH_PERSISTENT or STA_BATCH_LEVELS; a graph the
                                     persistent kernel cannot stage (a level chunk over the
                                     LDS caps) is run by levels whatever is asked             */
} sta_batch_design;

/* Device workspace a batch of n designs needs (descriptor table, unit list, counter). */
size_t sta_batch_workspace_bytes(int32_t n_designs, int32_t n_views);

/* Builds the batch: validates, orders the persistent units by decreasing size, and
 * uploads the descriptor table into the workspace (synchronously). */
sta_status sta_batch_create(const sta_batch_design* designs, int32_t n, const sta_library* lib,
                            const sta_views* views, void* workspace, size_t workspace_bytes, sta_batch** out);

/* The forward pass of every design and view.  use_graph != 0 replays a hipGraph of the
 * whole launch sequence (captured on first use).  persistent_blocks: workgroups of the
 * persistent launch (0: one per compute unit). */
sta_status sta_batch_propagate(sta_batch* b, int32_t use_graph, int32_t persistent_blocks, void* stream);

/* Units in the persistent launch and designs run by levels (for reports). */
sta_status sta_batch_info(const sta_batch* b, int32_t* persistent_units, int32_t* level_designs);

void sta_batch_free(sta_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* STA_BATCH_H */

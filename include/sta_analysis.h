/*
 * sta_analysis.h -- analyses on a timed graph (libsta.so): the adjoint of TNS and the
 * critical-path report.
 *
 * Background.  The timing workload of Heteroflow (Section IV-A) extracts, per timing
 * view, the critical paths of the design and the total negative slack as the inputs of
 * its correlation model.  Both come from the same saved quantities of the forward pass:
 * the argmax arc of every gate output (sta_timing_out.argmax) and the endpoint slacks
 * (sta_slack_out.drv_slack).
 *
 * TNS_v = sum over endpoints e of min(0, slack_v(e)), slack = RAT - AT (late) or
 * AT - RAT (early).  With the arguments of the forward maxima (minima) held fixed, TNS is
 * linear in the delays, and its gradient flows along the argmax arcs only:
 *   dTNS/dAT(e)   = -1 (late) or +1 (early) at an endpoint with slack < 0, else 0;
 *   dTNS/dd(a)    = dTNS/dAT(out(a)) if a is the argmax arc of its gate, else 0, for the
 *                   cell-arc delay d(a) and equally for the net delay into a's input pin;
 *   dTNS/dAT(u)   = sum over the sink pins of driver u of dTNS/dd(sink arc);
 *   dTNS/dload(o) = dTNS/dAT(o) * d d(argmax arc)/d load, the NLDM bilinear slope in the
 *                   load axis, (q - p) / (y[j+1] - y[j]), with the input slew held.
 * Gradients with respect to delays are integer counts: minus (plus, early) the number of
 * failing endpoints whose critical path passes through the pin or arc.  At exact ties
 * of the maxima or slack == 0 the one-sided derivatives differ; the chosen argmax (the
 * smallest arc index among equal candidates) and "slack < 0" define the value returned.
 *
 * Conventions as in sta.h: device buffers owned by the caller, internal numbering,
 * views interleaved element-major, asynchronous on the caller's stream.
 */
#ifndef STA_ANALYSIS_H
#define STA_ANALYSIS_H

#include "sta.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    float* g_drv_at;      /* [D][V] dTNS_v/dAT of every driver (required)                 */
    float* g_arc_delay;   /* [A][V] dTNS_v/d(cell-arc delay), or NULL                      */
    float* g_net_delay;   /* [A][V] dTNS_v/d(net delay into the arc's pin), or NULL        */
    float* g_load;        /* [D][V] dTNS_v/d(load of the driver's net), 0 at primary inputs,
                                     or NULL                                               */
} sta_adjoint_out;

/* Passage: Section IV-A (the correlation layer fits regression models by gradient
 * descent on the timing results); the chain rule through the saved argmax is written out
 * above (the paper states none).
 * Adjoint of TNS for every view of a completed sta_propagate + sta_slack on the same
 * graph, views and net data (nd->arc_load, t->argmax, t->arc_ts, sl->drv_slack are
 * read).  The driver levels are walked top down on the backward span tiles: each launch
 * covers up to eight driver levels (a gather over each driver's sink pins with the
 * in-tile gradients in LDS, no atomics); a level that cannot be tiled, and every level
 * when level fusion is off, gets one launch of its own.  Then one launch forms the load
 * gradient.  lib is needed only for g_load (NULL otherwise).  Errors: STA_E_ARG (graph
 * not uploaded, bad views, null or missing buffers), STA_E_HIP. */
sta_status sta_tns_adjoint(const sta_graph* g, const sta_library* lib, const sta_views* views,
                           const sta_net_out* nd, const sta_timing_out* t, const sta_slack_out* sl,
                           const sta_adjoint_out* out, void* stream);

/* No passage (a data-layout helper).  Refreshes nd->arc_load (the load each cell arc
 * sees) from nd->load (per driver), for callers that supply loads of their own instead
 * of running sta_delay_calc.  Errors: STA_E_ARG (graph not uploaded, null buffer). */
sta_status sta_arc_load(const sta_graph* g, const sta_net_out* nd, void* stream);

#define STA_MAX_PATHS 64

typedef struct {
    int32_t* ep_rank;     /* [k] endpoint ranks (ascending driver id order of the input),
                                 worst slack first, ties by lower rank                      */
    float* slack;         /* [k] their slacks in the chosen view                            */
    int32_t* len;         /* [k] drivers on each path                                       */
    int32_t* drv;         /* [k][L+1] internal drivers from the endpoint back to a primary
                                 input (entries past len unspecified)                        */
    int32_t* arc;         /* [k][L] internal cell arcs: arc[i] leads into drv[i]            */
} sta_paths_out;

/* Device scratch that sta_critical_paths needs. */
size_t sta_paths_scratch_bytes(void);

/* Passage: Section IV-A (the correlation layer extracts critical paths from each
 * view's timing).
 * The k (1..STA_MAX_PATHS, <= endpoints) worst endpoints of one view and their critical
 * paths, by walking the saved argmax arcs back to the primary inputs.  L is the number of
 * levels (sta_sizes.n_levels). */
sta_status sta_critical_paths(const sta_graph* g, const sta_views* views, int32_t view, int32_t k,
                              const sta_timing_out* t, const sta_slack_out* sl, const sta_paths_out* out,
                              void* scratch, size_t scratch_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* STA_ANALYSIS_H */

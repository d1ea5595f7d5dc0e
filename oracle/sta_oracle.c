/*
 * CPU oracle for levelized static timing analysis.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  It shares no code, header, table or helper
 * with the HIP implementation; both read the same seeded input arrays.
 *
 * What it computes.  The paper (Heteroflow, Section IV-A, "VLSI Timing Analysis")
 * runs a timer over a 1.5M-gate design for many views (corner x mode) but prints no
 * timing formula and no timing value, so no pin below comes from the paper itself:
 * every function is pinned against mathematics instead (closed forms, brute force on
 * tiny graphs, an independent O(n^2) moment definition, invariants), as listed in the
 * test suite.  The definitions follow the textbook method:
 *   step 1  levelize: Kahn's algorithm; level(PI) = 0, level(g) = 1 + max level of the
 *           drivers of g's inputs; a cycle is an error;
 *   step 2  RC delay calculation per net in FP64: lumped load, Elmore first moment m1,
 *           second moment m2 (Rubinstein-Penfield-Horowitz / PERI), imp2 = 2 m2 - m1^2;
 *   step 3  NLDM 7x7 bilinear lookup in FP32, each operation rounded separately,
 *           linear extrapolation from the end segment (no clamp);
 *   step 4  net slew: S_sink = sqrt(S_drv^2 + imp2)  (PERI quadrature);
 *   step 5  forward propagation in FP32: AT_out = max (late) / min (early) over cell arcs
 *           of (AT_in + d), smallest arc index wins ties; slew = worst arc slew;
 *   step 6  backward required times in FP32 and slack = RAT - AT (late) or AT - RAT
 *           (early).  WNS/TNS are formed by the Python wrapper from the endpoint slacks.
 *
 * Build: gcc -O2 -ffp-contract=off (x86-64 SSE arithmetic: every float/double
 * operation is a single IEEE-754 round-to-nearest-even operation).  The same source is
 * built twice: liboracle.so (serial) and, with -fopenmp, liboracle_omp.so, where the
 * level-ordered entry points (orc_*_lv) run each level's gates (drivers, nets) in
 * parallel.  Every gate, driver or net is computed by the one routine both orders call,
 * from operands fixed before its level starts, so both builds and both orders give the
 * same bits.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_RANGE (-2)
#define ORC_E_CYCLE (-3)

/* ---- step 1: levelization --------------------------------------------------- */

/* Kahn's algorithm on the gate graph.  level[d] for every driver d (PIs 0, gate
 * output n_pi+g gets its gate's level), topo[] receives the gates in the order Kahn's
 * queue released them.  Returns ORC_E_CYCLE if some gate never becomes ready. */
int orc_levelize(int n_pi, int n_gates, const int32_t* gate_arc_ptr, const int32_t* arc_drv,
                 int32_t* level, int32_t* topo)
{
    int D = n_pi + n_gates;
    int A = gate_arc_ptr[n_gates];
    int32_t* indeg = (int32_t*)calloc((size_t)n_gates + 1, sizeof(int32_t));
    int32_t* fo_cnt = (int32_t*)calloc((size_t)D + 1, sizeof(int32_t));
    int32_t* fo_ptr = (int32_t*)calloc((size_t)D + 1, sizeof(int32_t));
    int32_t* fo_gate = (int32_t*)malloc(((size_t)A + 1) * sizeof(int32_t));
    int32_t* queue = (int32_t*)malloc(((size_t)n_gates + 1) * sizeof(int32_t));
    int rc = ORC_OK;
    if (!indeg || !fo_cnt || !fo_ptr || !fo_gate || !queue) { rc = ORC_E_ARG; goto done; }

    for (int g = 0; g < n_gates; ++g)
        for (int a = gate_arc_ptr[g]; a < gate_arc_ptr[g + 1]; ++a) {
            int d = arc_drv[a];
            if (d < 0 || d >= D) { rc = ORC_E_RANGE; goto done; }
            fo_cnt[d]++;
            if (d >= n_pi) indeg[g]++;
        }
    for (int d = 0; d < D; ++d) fo_ptr[d + 1] = fo_ptr[d] + fo_cnt[d];
    memset(fo_cnt, 0, sizeof(int32_t) * (size_t)D);
    for (int g = 0; g < n_gates; ++g)
        for (int a = gate_arc_ptr[g]; a < gate_arc_ptr[g + 1]; ++a) {
            int d = arc_drv[a];
            fo_gate[fo_ptr[d] + fo_cnt[d]++] = g;
        }

    for (int d = 0; d < n_pi; ++d) level[d] = 0;
    int head = 0, tail = 0;
    for (int g = 0; g < n_gates; ++g)
        if (indeg[g] == 0) queue[tail++] = g;
    while (head < tail) {
        int g = queue[head++];
        int lv = 0;
        for (int a = gate_arc_ptr[g]; a < gate_arc_ptr[g + 1]; ++a) {
            int l = level[arc_drv[a]];
            if (l > lv) lv = l;
        }
        level[n_pi + g] = lv + 1;
        int o = n_pi + g;
        for (int i = fo_ptr[o]; i < fo_ptr[o + 1]; ++i) {
            int c = fo_gate[i];
            if (--indeg[c] == 0) queue[tail++] = c;
        }
    }
    if (tail != n_gates) { rc = ORC_E_CYCLE; goto done; }
    if (topo) memcpy(topo, queue, sizeof(int32_t) * (size_t)n_gates);
done:
    free(indeg); free(fo_cnt); free(fo_ptr); free(fo_gate); free(queue);
    return rc;
}

/* ---- step 2: RC delay calculation (FP64) ------------------------------------ */

/* For every net (driver d), nodes k = 0..M-1 local, parent[k] < k for k >= 1.
 *   C[k]  = wire cap + pin caps of the sinks tapped at k (sinks in ascending arc id)
 *   Cd    = C; for k = M-1..1: Cd[parent[k]] += Cd[k]          (downstream cap)
 *   load  = Cd[0]
 *   m1[0] = 0; m1[k] = m1[parent[k]] + (R[k] * Cd[k]) * 1e-3     (ohm*fF -> ps)
 *   W     = C * m1; for k = M-1..1: W[parent[k]] += W[k]
 *   m2[0] = 0; m2[k] = m2[parent[k]] + (R[k] * W[k]) * 1e-3
 *   imp2  = max(0, 2*m2 - m1*m1)
 * Per sink arc: net_delay = fl32(m1[tap]), net_imp2 = fl32(imp2[tap]); load[d] = fl32(load).
 * node_m1/node_m2/node_cd (FP64, per global node) are optional outputs for the tests. */

/* Driver-level CSR of the sink arcs (fanout), each driver's arcs in ascending arc id. */
static int orc_fanout(int D, int A, const int32_t* arc_drv, int32_t** fo_ptr_out, int32_t** fo_arc_out)
{
    int32_t* fo_ptr = (int32_t*)calloc((size_t)D + 2, sizeof(int32_t));
    int32_t* fo_arc = (int32_t*)malloc(((size_t)A + 1) * sizeof(int32_t));
    if (!fo_ptr || !fo_arc) { free(fo_ptr); free(fo_arc); return ORC_E_ARG; }
    for (int a = 0; a < A; ++a) fo_ptr[arc_drv[a] + 2]++;
    for (int d = 0; d < D; ++d) fo_ptr[d + 2] += fo_ptr[d + 1];
    for (int a = 0; a < A; ++a) fo_arc[fo_ptr[arc_drv[a] + 1]++] = a;
    *fo_ptr_out = fo_ptr;
    *fo_arc_out = fo_arc;
    return ORC_OK;
}

/* Checks the RC data of every net: parents before children, taps inside their net. */
static int orc_check_nets(int n_drv, const int32_t* net_node_ptr, const int32_t* node_parent,
                          int n_arcs, const int32_t* arc_drv, const int32_t* arc_tap)
{
    for (int a = 0; a < n_arcs; ++a) {
        int d = arc_drv[a];
        if (d < 0 || d >= n_drv) return ORC_E_RANGE;
        int nm = net_node_ptr[d + 1] - net_node_ptr[d];
        if (arc_tap[a] < 0 || arc_tap[a] >= nm) return ORC_E_RANGE;
    }
    for (int d = 0; d < n_drv; ++d) {
        int n0 = net_node_ptr[d], nm = net_node_ptr[d + 1] - n0;
        if (nm < 1) return ORC_E_ARG;
        for (int k = 1; k < nm; ++k)
            if (node_parent[n0 + k] < 0 || node_parent[n0 + k] >= k) return ORC_E_RANGE;
    }
    return ORC_OK;
}

/* The moments of net d (the definition above), its sinks being fo_arc[fo_ptr[d] ..
 * fo_ptr[d+1]) in ascending arc id.  C, Cd, m1, W, m2: FP64 work arrays of the net's
 * node count. */
static void net_moments(int d, const int32_t* net_node_ptr, const int32_t* node_parent,
                        const float* node_R, const float* node_C, const int32_t* fo_ptr,
                        const int32_t* fo_arc, const int32_t* arc_tap, const float* arc_pincap,
                        double* C, double* Cd, double* m1, double* W, double* m2,
                        float* load, float* net_delay, float* net_imp2,
                        double* node_m1, double* node_m2, double* node_cd)
{
    const int n0 = net_node_ptr[d], nm = net_node_ptr[d + 1] - n0;
    const int32_t* par = node_parent + n0;
    for (int k = 0; k < nm; ++k) C[k] = (double)node_C[n0 + k];
    for (int i = fo_ptr[d]; i < fo_ptr[d + 1]; ++i) C[arc_tap[fo_arc[i]]] += (double)arc_pincap[fo_arc[i]];
    for (int k = 0; k < nm; ++k) Cd[k] = C[k];
    for (int k = nm - 1; k >= 1; --k) Cd[par[k]] += Cd[k];
    load[d] = (float)Cd[0];
    m1[0] = 0.0;
    for (int k = 1; k < nm; ++k) m1[k] = m1[par[k]] + ((double)node_R[n0 + k] * Cd[k]) * 1e-3;
    for (int k = 0; k < nm; ++k) W[k] = C[k] * m1[k];
    for (int k = nm - 1; k >= 1; --k) W[par[k]] += W[k];
    m2[0] = 0.0;
    for (int k = 1; k < nm; ++k) m2[k] = m2[par[k]] + ((double)node_R[n0 + k] * W[k]) * 1e-3;
    for (int i = fo_ptr[d]; i < fo_ptr[d + 1]; ++i) {
        const int a = fo_arc[i], k = arc_tap[a];
        double imp2 = 2.0 * m2[k] - m1[k] * m1[k];
        if (imp2 < 0.0) imp2 = 0.0;
        net_delay[a] = (float)m1[k];
        net_imp2[a] = (float)imp2;
    }
    if (node_m1) memcpy(node_m1 + n0, m1, sizeof(double) * (size_t)nm);
    if (node_m2) memcpy(node_m2 + n0, m2, sizeof(double) * (size_t)nm);
    if (node_cd) memcpy(node_cd + n0, Cd, sizeof(double) * (size_t)nm);
}

/* par = 0: nets one after another; par = 1: nets in parallel (OpenMP build). */
static int delay_calc_impl(int par, int n_drv, const int32_t* net_node_ptr, const int32_t* node_parent,
                           const float* node_R, const float* node_C,
                           int n_arcs, const int32_t* arc_drv, const int32_t* arc_tap, const float* arc_pincap,
                           float* load, float* net_delay, float* net_imp2,
                           double* node_m1, double* node_m2, double* node_cd)
{
    int rc = orc_check_nets(n_drv, net_node_ptr, node_parent, n_arcs, arc_drv, arc_tap);
    if (rc != ORC_OK) return rc;
    int32_t *fo_ptr = NULL, *fo_arc = NULL;
    rc = orc_fanout(n_drv, n_arcs, arc_drv, &fo_ptr, &fo_arc);
    if (rc != ORC_OK) return rc;
    int maxm = 1;
    for (int d = 0; d < n_drv; ++d)
        if (net_node_ptr[d + 1] - net_node_ptr[d] > maxm) maxm = net_node_ptr[d + 1] - net_node_ptr[d];
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel if (par) reduction(| : bad)
#endif
    {
        double* work = (double*)malloc(sizeof(double) * 5 * (size_t)maxm);
        if (!work) {
            bad = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1024)
#endif
            for (int d = 0; d < n_drv; ++d)
                net_moments(d, net_node_ptr, node_parent, node_R, node_C, fo_ptr, fo_arc, arc_tap, arc_pincap,
                            work, work + maxm, work + 2 * (size_t)maxm, work + 3 * (size_t)maxm,
                            work + 4 * (size_t)maxm, load, net_delay, net_imp2, node_m1, node_m2, node_cd);
        }
        free(work);
    }
    free(fo_ptr); free(fo_arc);
    (void)par;
    return bad ? ORC_E_ARG : ORC_OK;
}

int orc_delay_calc(int n_drv, const int32_t* net_node_ptr, const int32_t* node_parent,
                   const float* node_R, const float* node_C,
                   int n_arcs, const int32_t* arc_drv, const int32_t* arc_tap, const float* arc_pincap,
                   float* load, float* net_delay, float* net_imp2,
                   double* node_m1, double* node_m2, double* node_cd)
{
    return delay_calc_impl(0, n_drv, net_node_ptr, node_parent, node_R, node_C, n_arcs, arc_drv, arc_tap,
                           arc_pincap, load, net_delay, net_imp2, node_m1, node_m2, node_cd);
}

/* The same, the nets spread over the OpenMP threads (nets are independent). */
int orc_delay_calc_lv(int n_drv, const int32_t* net_node_ptr, const int32_t* node_parent,
                      const float* node_R, const float* node_C,
                      int n_arcs, const int32_t* arc_drv, const int32_t* arc_tap, const float* arc_pincap,
                      float* load, float* net_delay, float* net_imp2,
                      double* node_m1, double* node_m2, double* node_cd)
{
    return delay_calc_impl(1, n_drv, net_node_ptr, node_parent, node_R, node_C, n_arcs, arc_drv, arc_tap,
                           arc_pincap, load, net_delay, net_imp2, node_m1, node_m2, node_cd);
}

/* Threads the OpenMP entry points use (1 in the serial build). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Drivers bucketed by level, ascending id inside a level: drivers of level l are
 * by_lv[lv_ptr[l] .. lv_ptr[l+1]).  *n_lv = highest level + 1. */
static int orc_level_buckets(int D, const int32_t* level, int32_t** lv_ptr_out, int32_t** by_lv_out, int* n_lv)
{
    int L = 0;
    for (int d = 0; d < D; ++d) if (level[d] > L) L = level[d];
    int32_t* lv_ptr = (int32_t*)calloc((size_t)L + 2, sizeof(int32_t));
    int32_t* by_lv = (int32_t*)malloc(((size_t)D + 1) * sizeof(int32_t));
    if (!lv_ptr || !by_lv) { free(lv_ptr); free(by_lv); return ORC_E_ARG; }
    for (int d = 0; d < D; ++d) lv_ptr[level[d] + 1]++;
    for (int l = 0; l <= L; ++l) lv_ptr[l + 1] += lv_ptr[l];
    int32_t* fill = (int32_t*)malloc(((size_t)L + 1) * sizeof(int32_t));
    if (!fill) { free(lv_ptr); free(by_lv); return ORC_E_ARG; }
    memcpy(fill, lv_ptr, sizeof(int32_t) * ((size_t)L + 1));
    for (int d = 0; d < D; ++d) by_lv[fill[level[d]]++] = d;
    free(fill);
    *lv_ptr_out = lv_ptr;
    *by_lv_out = by_lv;
    *n_lv = L + 1;
    return ORC_OK;
}

/* ---- step 3: NLDM bilinear lookup (FP32) ------------------------------------ */

/* largest i in 0..5 with axis[i] <= v; 0 when v < axis[0] */
static int seg7(const float* axis, float v)
{
    int i = 0;
    for (int t = 1; t <= 5; ++t)
        if (axis[t] <= v) i = t;
    return i;
}

/* T is one 7x7 table, row-major T[i*7+j] at (x[i], y[j]).  Every -, *, + and / below is
 * a separately rounded FP32 operation (no contraction). */
float orc_bilerp(const float* x, const float* y, const float* T, float s, float l)
{
    int i = seg7(x, s);
    int j = seg7(y, l);
    float tx = (s - x[i]) / (x[i + 1] - x[i]);
    float ty = (l - y[j]) / (y[j + 1] - y[j]);
    float t00 = T[i * 7 + j], t10 = T[(i + 1) * 7 + j];
    float t01 = T[i * 7 + j + 1], t11 = T[(i + 1) * 7 + j + 1];
    float p = t00 + tx * (t10 - t00);
    float q = t01 + tx * (t11 - t01);
    return p + ty * (q - p);
}

void orc_bilerp_many(const float* x, const float* y, const float* T, int n,
                     const float* s, const float* l, float* out)
{
    for (int k = 0; k < n; ++k) out[k] = orc_bilerp(x, y, T, s[k], l[k]);
}

/* ---- steps 4-5: forward propagation (FP32) ----------------------------------- */

/* mode 0 = late (max), 1 = early (min).  lib_tab holds n_tables pairs, each 2x49 floats:
 * [t][0] delay table, [t][1] slew table.  A gate's step reads only its drivers' results,
 * so any topological order (Kahn's queue, or level by level) gives the same bits. */

/* One gate g: per cell arc the input pin's arrival and slew, the NLDM delay and output
 * slew at the gate's load; then the max (late) / min (early) over the arcs with the
 * smallest arc index winning ties, and the worst slew. */
static void gate_forward(int mode, int n_pi, int g, const int32_t* gate_arc_ptr, const int32_t* arc_drv,
                         const int32_t* arc_tbl, const float* lib_x, const float* lib_y, const float* lib_tab,
                         const float* load, const float* net_delay, const float* net_imp2,
                         float* at_drv, float* slew_drv, float* at_in, float* slew_in,
                         float* arc_delay, int32_t* argmax)
{
    int o = n_pi + g;
    float best_at = 0.0f, best_slew = 0.0f;
    int best_k = -1;
    for (int a = gate_arc_ptr[g]; a < gate_arc_ptr[g + 1]; ++a) {
        int u = arc_drv[a];
        int tb = arc_tbl[a];
        float ai = at_drv[u] + net_delay[a];
        float su2 = slew_drv[u] * slew_drv[u];
        float si = sqrtf(su2 + net_imp2[a]);
        at_in[a] = ai;
        slew_in[a] = si;
        float d = orc_bilerp(lib_x, lib_y, lib_tab + (size_t)tb * 98, si, load[o]);
        float s = orc_bilerp(lib_x, lib_y, lib_tab + (size_t)tb * 98 + 49, si, load[o]);
        arc_delay[a] = d;
        float cand = ai + d;
        int k = a - gate_arc_ptr[g];
        if (best_k < 0) {
            best_at = cand; best_slew = s; best_k = k;
        } else if (mode == 0) {
            if (cand > best_at) { best_at = cand; best_k = k; }
            if (s > best_slew) best_slew = s;
        } else {
            if (cand < best_at) { best_at = cand; best_k = k; }
            if (s < best_slew) best_slew = s;
        }
    }
    at_drv[o] = best_at;
    slew_drv[o] = best_slew;
    argmax[g] = best_k;
}

/* par = 0: gates in Kahn's order; par = 1: level by level, each level's gates in
 * parallel (OpenMP build). */
static int propagate_impl(int par, int mode, int n_pi, int n_gates, const int32_t* gate_arc_ptr,
                          const int32_t* arc_drv, const int32_t* arc_tbl, int n_tables,
                          const float* lib_x, const float* lib_y, const float* lib_tab,
                          const float* load, const float* net_delay, const float* net_imp2,
                          const float* pi_at, const float* pi_slew,
                          float* at_drv, float* slew_drv, float* at_in, float* slew_in,
                          float* arc_delay, int32_t* argmax)
{
    int D = n_pi + n_gates;
    int A = gate_arc_ptr[n_gates];
    int32_t* level = (int32_t*)malloc(((size_t)D + 1) * sizeof(int32_t));
    int32_t* topo = (int32_t*)malloc(((size_t)n_gates + 1) * sizeof(int32_t));
    int32_t *lv_ptr = NULL, *by_lv = NULL;
    int n_lv = 0;
    int rc = ORC_OK;
    if (!level || !topo) { rc = ORC_E_ARG; goto done; }
    for (int a = 0; a < A; ++a)
        if (arc_tbl[a] < 0 || arc_tbl[a] >= n_tables) { rc = ORC_E_RANGE; goto done; }
    rc = orc_levelize(n_pi, n_gates, gate_arc_ptr, arc_drv, level, topo);
    if (rc != ORC_OK) goto done;

    for (int d = 0; d < n_pi; ++d) { at_drv[d] = pi_at[d]; slew_drv[d] = pi_slew[d]; }
    if (!par) {
        for (int t = 0; t < n_gates; ++t)
            gate_forward(mode, n_pi, topo[t], gate_arc_ptr, arc_drv, arc_tbl, lib_x, lib_y, lib_tab, load,
                         net_delay, net_imp2, at_drv, slew_drv, at_in, slew_in, arc_delay, argmax);
        goto done;
    }
    rc = orc_level_buckets(D, level, &lv_ptr, &by_lv, &n_lv);
    if (rc != ORC_OK) goto done;
    for (int l = 1; l < n_lv; ++l) {
        const int i0 = lv_ptr[l], i1 = lv_ptr[l + 1];
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int i = i0; i < i1; ++i)
            gate_forward(mode, n_pi, by_lv[i] - n_pi, gate_arc_ptr, arc_drv, arc_tbl, lib_x, lib_y, lib_tab, load,
                         net_delay, net_imp2, at_drv, slew_drv, at_in, slew_in, arc_delay, argmax);
    }
done:
    free(level); free(topo); free(lv_ptr); free(by_lv);
    return rc;
}

int orc_propagate(int mode, int n_pi, int n_gates, const int32_t* gate_arc_ptr,
                  const int32_t* arc_drv, const int32_t* arc_tbl, int n_tables,
                  const float* lib_x, const float* lib_y, const float* lib_tab,
                  const float* load, const float* net_delay, const float* net_imp2,
                  const float* pi_at, const float* pi_slew,
                  float* at_drv, float* slew_drv, float* at_in, float* slew_in,
                  float* arc_delay, int32_t* argmax)
{
    return propagate_impl(0, mode, n_pi, n_gates, gate_arc_ptr, arc_drv, arc_tbl, n_tables, lib_x, lib_y,
                          lib_tab, load, net_delay, net_imp2, pi_at, pi_slew, at_drv, slew_drv, at_in, slew_in,
                          arc_delay, argmax);
}

/* The same, level by level with each level's gates spread over the OpenMP threads. */
int orc_propagate_lv(int mode, int n_pi, int n_gates, const int32_t* gate_arc_ptr,
                     const int32_t* arc_drv, const int32_t* arc_tbl, int n_tables,
                     const float* lib_x, const float* lib_y, const float* lib_tab,
                     const float* load, const float* net_delay, const float* net_imp2,
                     const float* pi_at, const float* pi_slew,
                     float* at_drv, float* slew_drv, float* at_in, float* slew_in,
                     float* arc_delay, int32_t* argmax)
{
    return propagate_impl(1, mode, n_pi, n_gates, gate_arc_ptr, arc_drv, arc_tbl, n_tables, lib_x, lib_y,
                          lib_tab, load, net_delay, net_imp2, pi_at, pi_slew, at_drv, slew_drv, at_in, slew_in,
                          arc_delay, argmax);
}

/* ---- step 6: required times and slack (FP32) --------------------------------- */

/* Endpoints are drivers without sinks; ep_rat[r] is the required time of the r-th
 * endpoint in ascending driver id.  Late: RAT_drv = min over its sink arcs of
 * (RAT_in - net_delay), RAT_in = RAT_out - arc_delay, slack = RAT - AT.
 * Early: max instead of min, slack = AT - RAT.  A driver needs the RAT_in of its sinks,
 * which belong to gates of higher level: drivers are visited in reverse topological
 * order (Kahn's, or level by level from the top). */

/* One driver o: its required time and slack, then (a gate output) the required times
 * and slacks of its gate's input pins. */
static void driver_backward(int mode, int n_pi, int o, const int32_t* gate_arc_ptr, const int32_t* fo_ptr,
                            const int32_t* fo_arc, const int32_t* ep_rank, const float* net_delay,
                            const float* arc_delay, const float* at_drv, const float* at_in, const float* ep_rat,
                            float* rat_drv, float* rat_in, float* slack_drv, float* slack_in)
{
    float r;
    if (ep_rank[o] >= 0) {
        r = ep_rat[ep_rank[o]];
    } else {
        r = 0.0f;
        for (int i = fo_ptr[o]; i < fo_ptr[o + 1]; ++i) {
            int a = fo_arc[i];
            float v = rat_in[a] - net_delay[a];
            if (i == fo_ptr[o]) r = v;
            else if (mode == 0) { if (v < r) r = v; }
            else { if (v > r) r = v; }
        }
    }
    rat_drv[o] = r;
    slack_drv[o] = (mode == 0) ? (r - at_drv[o]) : (at_drv[o] - r);
    if (o >= n_pi) {
        int g = o - n_pi;
        for (int a = gate_arc_ptr[g]; a < gate_arc_ptr[g + 1]; ++a) {
            rat_in[a] = r - arc_delay[a];
            slack_in[a] = (mode == 0) ? (rat_in[a] - at_in[a]) : (at_in[a] - rat_in[a]);
        }
    }
}

static int slack_impl(int par, int mode, int n_pi, int n_gates, const int32_t* gate_arc_ptr, const int32_t* arc_drv,
                      const float* net_delay, const float* arc_delay,
                      const float* at_drv, const float* at_in, const float* ep_rat,
                      float* rat_drv, float* rat_in, float* slack_drv, float* slack_in)
{
    int D = n_pi + n_gates;
    int A = gate_arc_ptr[n_gates];
    int32_t* level = (int32_t*)malloc(((size_t)D + 1) * sizeof(int32_t));
    int32_t* topo = (int32_t*)malloc(((size_t)n_gates + 1) * sizeof(int32_t));
    int32_t* ep_rank = (int32_t*)malloc(((size_t)D + 1) * sizeof(int32_t));
    int32_t *fo_ptr = NULL, *fo_arc = NULL, *lv_ptr = NULL, *by_lv = NULL;
    int n_lv = 0;
    int rc = ORC_OK;
    if (!level || !topo || !ep_rank) { rc = ORC_E_ARG; goto done; }
    rc = orc_levelize(n_pi, n_gates, gate_arc_ptr, arc_drv, level, topo);
    if (rc != ORC_OK) goto done;
    rc = orc_fanout(D, A, arc_drv, &fo_ptr, &fo_arc);
    if (rc != ORC_OK) goto done;
    {
        int r = 0;
        for (int d = 0; d < D; ++d) ep_rank[d] = (fo_ptr[d + 1] == fo_ptr[d]) ? r++ : -1;
    }
    if (!par) {
        for (int t = n_gates - 1; t >= -n_pi; --t)   /* t >= 0: gate topo[t]; t < 0: primary input -t-1 */
            driver_backward(mode, n_pi, (t >= 0) ? n_pi + topo[t] : -t - 1, gate_arc_ptr, fo_ptr, fo_arc, ep_rank,
                            net_delay, arc_delay, at_drv, at_in, ep_rat, rat_drv, rat_in, slack_drv, slack_in);
        goto done;
    }
    rc = orc_level_buckets(D, level, &lv_ptr, &by_lv, &n_lv);
    if (rc != ORC_OK) goto done;
    for (int l = n_lv - 1; l >= 0; --l) {
        const int i0 = lv_ptr[l], i1 = lv_ptr[l + 1];
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int i = i0; i < i1; ++i)
            driver_backward(mode, n_pi, by_lv[i], gate_arc_ptr, fo_ptr, fo_arc, ep_rank, net_delay, arc_delay, at_drv,
                            at_in, ep_rat, rat_drv, rat_in, slack_drv, slack_in);
    }
done:
    free(level); free(topo); free(fo_ptr); free(fo_arc); free(ep_rank); free(lv_ptr); free(by_lv);
    return rc;
}

int orc_slack(int mode, int n_pi, int n_gates, const int32_t* gate_arc_ptr, const int32_t* arc_drv,
              const float* net_delay, const float* arc_delay,
              const float* at_drv, const float* at_in, const float* ep_rat,
              float* rat_drv, float* rat_in, float* slack_drv, float* slack_in)
{
    return slack_impl(0, mode, n_pi, n_gates, gate_arc_ptr, arc_drv, net_delay, arc_delay, at_drv, at_in, ep_rat,
                      rat_drv, rat_in, slack_drv, slack_in);
}

/* The same, level by level from the top with each level's drivers spread over the
 * OpenMP threads. */
int orc_slack_lv(int mode, int n_pi, int n_gates, const int32_t* gate_arc_ptr, const int32_t* arc_drv,
                 const float* net_delay, const float* arc_delay,
                 const float* at_drv, const float* at_in, const float* ep_rat,
                 float* rat_drv, float* rat_in, float* slack_drv, float* slack_in)
{
    return slack_impl(1, mode, n_pi, n_gates, gate_arc_ptr, arc_drv, net_delay, arc_delay, at_drv, at_in, ep_rat,
                      rat_drv, rat_in, slack_drv, slack_in);
}

/* ---- RC-tree nets on their own (learned-surrogate workload) ------------------ */

/* Per sink: FP64 Elmore m1 and imp2 = max(0, 2 m2 - m1^2) at the tapped node, with the
 * same definition as orc_delay_calc (sink pin caps added in sink order); per net: load.
 * Per sink also the 12 surrogate features (FP64), when feat is not NULL:
 *   0 R_path  resistance of the root->sink path          6 R of the path's first edge
 *   1 load    total net capacitance                      7 sum of node caps on the path (incl. pin caps)
 *   2 Cd      downstream cap of the sink node            8 mean edge R of the net
 *   3 depth   edges on the path                          9 mean wire cap of the net
 *   4 M       nodes in the net                          10 sink pin cap
 *   5 sinks   sinks of the net                          11 driver slew                  */
int orc_tree_moments(int n_nets, const int32_t* net_node_ptr, const int32_t* node_parent,
                     const float* node_R, const float* node_C, const int32_t* sink_ptr,
                     const int32_t* sink_node, const float* sink_pincap, const float* drv_slew,
                     double* sink_m1, double* sink_imp2, double* net_load, double* feat)
{
    int maxm = 1;
    for (int n = 0; n < n_nets; ++n) {
        int m = net_node_ptr[n + 1] - net_node_ptr[n];
        if (m < 1) return ORC_E_ARG;
        if (m > maxm) maxm = m;
    }
    double* C = (double*)malloc(sizeof(double) * (size_t)maxm);
    double* Cd = (double*)malloc(sizeof(double) * (size_t)maxm);
    double* m1 = (double*)malloc(sizeof(double) * (size_t)maxm);
    double* W = (double*)malloc(sizeof(double) * (size_t)maxm);
    double* m2 = (double*)malloc(sizeof(double) * (size_t)maxm);
    int rc = ORC_OK;
    if (!C || !Cd || !m1 || !W || !m2) { rc = ORC_E_ARG; goto done; }
    for (int n = 0; n < n_nets; ++n) {
        const int n0 = net_node_ptr[n], nm = net_node_ptr[n + 1] - n0;
        const int32_t* par = node_parent + n0;
        for (int k = 1; k < nm; ++k)
            if (par[k] < 0 || par[k] >= k) { rc = ORC_E_RANGE; goto done; }
        for (int k = 0; k < nm; ++k) C[k] = (double)node_C[n0 + k];
        for (int s = sink_ptr[n]; s < sink_ptr[n + 1]; ++s) {
            if (sink_node[s] < 0 || sink_node[s] >= nm) { rc = ORC_E_RANGE; goto done; }
            C[sink_node[s]] += (double)sink_pincap[s];
        }
        for (int k = 0; k < nm; ++k) Cd[k] = C[k];
        for (int k = nm - 1; k >= 1; --k) Cd[par[k]] += Cd[k];
        net_load[n] = Cd[0];
        m1[0] = 0.0;
        for (int k = 1; k < nm; ++k) m1[k] = m1[par[k]] + ((double)node_R[n0 + k] * Cd[k]) * 1e-3;
        for (int k = 0; k < nm; ++k) W[k] = C[k] * m1[k];
        for (int k = nm - 1; k >= 1; --k) W[par[k]] += W[k];
        m2[0] = 0.0;
        for (int k = 1; k < nm; ++k) m2[k] = m2[par[k]] + ((double)node_R[n0 + k] * W[k]) * 1e-3;
        double sumR = 0.0, sumC = 0.0;
        for (int k = 1; k < nm; ++k) sumR += (double)node_R[n0 + k];
        for (int k = 0; k < nm; ++k) sumC += (double)node_C[n0 + k];
        for (int s = sink_ptr[n]; s < sink_ptr[n + 1]; ++s) {
            const int k = sink_node[s];
            double imp2 = 2.0 * m2[k] - m1[k] * m1[k];
            if (imp2 < 0.0) imp2 = 0.0;
            sink_m1[s] = m1[k];
            sink_imp2[s] = imp2;
            if (feat) {
                double rpath = 0.0, cpath = 0.0, rfirst = 0.0;
                int depth = 0;
                for (int v = k; v != 0; v = par[v]) {
                    rpath += (double)node_R[n0 + v];
                    cpath += C[v];
                    if (par[v] == 0) rfirst = (double)node_R[n0 + v];
                    ++depth;
                }
                double* f = feat + (size_t)s * 12;
                f[0] = rpath;
                f[1] = Cd[0];
                f[2] = Cd[k];
                f[3] = (double)depth;
                f[4] = (double)nm;
                f[5] = (double)(sink_ptr[n + 1] - sink_ptr[n]);
                f[6] = rfirst;
                f[7] = cpath;
                f[8] = nm > 1 ? sumR / (double)(nm - 1) : 0.0;
                f[9] = sumC / (double)nm;
                f[10] = (double)sink_pincap[s];
                f[11] = (double)drv_slew[n];
            }
        }
    }
done:
    free(C); free(Cd); free(m1); free(W); free(m2);
    return rc;
}

/* ---- adjoint of TNS (FP64 reference) ------------------------------------------ */

/* Chain rule of TNS = sum over endpoints of min(0, slack) through the forward maxima
 * (minima for early), with the arguments of the maxima fixed: d TNS / d AT(endpoint) is
 * -1 (late) or +1 (early) where the endpoint slack is negative, 0 otherwise; a gate
 * output passes its gradient to its argmax arc (the arc's delay and its input pin's
 * arrival), and a driver collects the gradients of all its sink pins.  FP64 (the values
 * are integer counts).  Gates are visited in reverse topological order. */
int orc_tns_adjoint(int mode, int n_pi, int n_gates, const int32_t* gate_arc_ptr, const int32_t* arc_drv,
                    const int32_t* argmax, const float* slack_drv, double* g_at, double* g_arc)
{
    int D = n_pi + n_gates;
    int A = gate_arc_ptr[n_gates];
    int32_t* level = (int32_t*)malloc(((size_t)D + 1) * sizeof(int32_t));
    int32_t* topo = (int32_t*)malloc(((size_t)n_gates + 1) * sizeof(int32_t));
    int32_t *fo_ptr = NULL, *fo_arc = NULL;
    int rc = ORC_OK;
    if (!level || !topo) { rc = ORC_E_ARG; goto done; }
    rc = orc_levelize(n_pi, n_gates, gate_arc_ptr, arc_drv, level, topo);
    if (rc != ORC_OK) goto done;
    rc = orc_fanout(D, A, arc_drv, &fo_ptr, &fo_arc);
    if (rc != ORC_OK) goto done;
    for (int d = 0; d < D; ++d) {
        g_at[d] = 0.0;
        if (fo_ptr[d + 1] == fo_ptr[d] && slack_drv[d] < 0.0f) g_at[d] = (mode == 0) ? -1.0 : 1.0;
    }
    for (int a = 0; a < A; ++a) g_arc[a] = 0.0;
    for (int t = n_gates - 1; t >= 0; --t) {
        int g = topo[t];
        int o = n_pi + g;
        int a = gate_arc_ptr[g] + argmax[g];
        g_arc[a] = g_at[o];
        g_at[arc_drv[a]] += g_at[o];
    }
done:
    free(level); free(topo); free(fo_ptr); free(fo_arc);
    return rc;
}

static double orc_tns_term(int mode, double at, double rat)
{
    double s = (mode == 0) ? rat - at : at - rat;
    return s < 0.0 ? s : 0.0;
}

/* Change of TNS (FP64, arrivals AT = max/min over arcs of AT(driver) + net delay + arc
 * delay, from the primary-input arrivals) when the cell-arc delays of one gate are
 * replaced, for each of n_pert perturbations: gate pert_gate[p] gets delays
 * pert_delay[pert_off[p] .. pert_off[p+1]) for its arcs in order.  Arrivals are
 * re-evaluated only where they change, in level order; base_tns receives the
 * unperturbed TNS (compensated summation).  ep_rat is indexed by driver (used only at
 * endpoints). */
int orc_tns_delta(int mode, int n_pi, int n_gates, const int32_t* gate_arc_ptr, const int32_t* arc_drv,
                  const double* arc_delay, const double* net_delay, const double* pi_at, const double* ep_rat,
                  int n_pert, const int32_t* pert_gate, const int32_t* pert_off, const double* pert_delay,
                  double* base_tns, double* delta)
{
    int D = n_pi + n_gates;
    int A = gate_arc_ptr[n_gates];
    int32_t* level = (int32_t*)malloc(((size_t)D + 1) * sizeof(int32_t));
    int32_t* topo = (int32_t*)malloc(((size_t)n_gates + 1) * sizeof(int32_t));
    double* at = (double*)malloc(((size_t)D + 1) * sizeof(double));
    double* atw = (double*)malloc(((size_t)D + 1) * sizeof(double));
    double* dw = (double*)malloc(((size_t)A + 1) * sizeof(double));
    int32_t* next = (int32_t*)malloc(((size_t)D + 1) * sizeof(int32_t));
    uint8_t* queued = (uint8_t*)calloc((size_t)D + 1, 1);
    int32_t* touched = (int32_t*)malloc(((size_t)D + 1) * sizeof(int32_t));
    int32_t *fo_ptr = NULL, *fo_arc = NULL, *head = NULL;
    int Lmax = 0, rc = ORC_OK;
    if (!level || !topo || !at || !atw || !dw || !next || !queued || !touched) { rc = ORC_E_ARG; goto done; }
    rc = orc_levelize(n_pi, n_gates, gate_arc_ptr, arc_drv, level, topo);
    if (rc != ORC_OK) goto done;
    rc = orc_fanout(D, A, arc_drv, &fo_ptr, &fo_arc);
    if (rc != ORC_OK) goto done;
    for (int d = 0; d < D; ++d) if (level[d] > Lmax) Lmax = level[d];
    head = (int32_t*)malloc(((size_t)Lmax + 1) * sizeof(int32_t));
    if (!head) { rc = ORC_E_ARG; goto done; }
    for (int l = 0; l <= Lmax; ++l) head[l] = -1;
    for (int d = 0; d < n_pi; ++d) at[d] = pi_at[d];
    for (int t = 0; t < n_gates; ++t) {
        int g = topo[t], o = n_pi + g;
        double best = 0.0;
        for (int a = gate_arc_ptr[g]; a < gate_arc_ptr[g + 1]; ++a) {
            double c = at[arc_drv[a]] + net_delay[a] + arc_delay[a];
            if (a == gate_arc_ptr[g] || (mode == 0 ? c > best : c < best)) best = c;
        }
        at[o] = best;
    }
    {
        double s = 0.0, comp = 0.0;       /* Kahan-Babuska summation of the base TNS */
        for (int d = 0; d < D; ++d) {
            if (fo_ptr[d + 1] != fo_ptr[d]) continue;
            double x = orc_tns_term(mode, at[d], ep_rat[d]);
            double t = s + x;
            comp += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
            s = t;
        }
        *base_tns = s + comp;
    }
    memcpy(atw, at, sizeof(double) * (size_t)D);
    memcpy(dw, arc_delay, sizeof(double) * (size_t)A);
    for (int p = 0; p < n_pert; ++p) {
        int g0 = pert_gate[p];
        if (g0 < 0 || g0 >= n_gates || pert_off[p + 1] - pert_off[p] != gate_arc_ptr[g0 + 1] - gate_arc_ptr[g0]) {
            rc = ORC_E_RANGE;
            goto done;
        }
        for (int k = 0; k < pert_off[p + 1] - pert_off[p]; ++k) dw[gate_arc_ptr[g0] + k] = pert_delay[pert_off[p] + k];
        int nt = 0;
        double dt = 0.0;
        int o0 = n_pi + g0;
        next[o0] = head[level[o0]];
        head[level[o0]] = o0;
        queued[o0] = 1;
        for (int l = level[o0]; l <= Lmax; ++l) {
            while (head[l] >= 0) {
                int o = head[l];
                head[l] = next[o];
                queued[o] = 0;
                int g = o - n_pi;
                double best = 0.0;
                for (int a = gate_arc_ptr[g]; a < gate_arc_ptr[g + 1]; ++a) {
                    double c = atw[arc_drv[a]] + net_delay[a] + dw[a];
                    if (a == gate_arc_ptr[g] || (mode == 0 ? c > best : c < best)) best = c;
                }
                if (best == atw[o]) continue;
                if (atw[o] == at[o]) touched[nt++] = o;
                atw[o] = best;
                if (fo_ptr[o + 1] == fo_ptr[o]) continue;
                for (int e = fo_ptr[o]; e < fo_ptr[o + 1]; ++e) {
                    int a = fo_arc[e];
                    int g2 = 0;
                    /* gate of arc a: arcs are contiguous per gate */
                    {
                        int lo = 0, hi = n_gates - 1;
                        while (lo < hi) {
                            int mid = (lo + hi + 1) / 2;
                            if (gate_arc_ptr[mid] <= a) lo = mid; else hi = mid - 1;
                        }
                        g2 = lo;
                    }
                    int o2 = n_pi + g2;
                    if (!queued[o2]) {
                        queued[o2] = 1;
                        next[o2] = head[level[o2]];
                        head[level[o2]] = o2;
                    }
                }
            }
        }
        for (int i = 0; i < nt; ++i) {
            int o = touched[i];
            if (fo_ptr[o + 1] == fo_ptr[o])
                dt += orc_tns_term(mode, atw[o], ep_rat[o]) - orc_tns_term(mode, at[o], ep_rat[o]);
            atw[o] = at[o];
        }
        for (int k = gate_arc_ptr[g0]; k < gate_arc_ptr[g0 + 1]; ++k) dw[k] = arc_delay[k];
        delta[p] = dt;
    }
done:
    free(level); free(topo); free(at); free(atw); free(dw); free(next); free(queued); free(touched);
    free(fo_ptr); free(fo_arc); free(head);
    return rc;
}

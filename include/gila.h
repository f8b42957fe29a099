/*
 * gila.h -- C ABI of an MI355X (gfx950) implementation of the layout step of
 * GiLA, the vertex-centric Fruchterman-Reingold algorithm of Arleo, Didimo,
 * Liotta and Montecchiani ("A Distributed Force-Directed Algorithm on Giraph:
 * Design and Experiments").
 *
 * Every iteration each vertex v sums
 *   - attraction from each adjacent u:  (x_u - x_v) * delta / d
 *     (magnitude delta^2 / d, Section 3.1 with p = 2), and
 *   - repulsion from each u in its k-neighbourhood N_v(k):
 *     (x_v - x_u) * d^2 / delta^2  (magnitude d^2 / delta, q = 1),
 * where N_v(k) is every vertex at graph distance <= k from v, v excluded
 * (Section 4.5; the TTL flooding there delivers exactly this set).  Then every
 * vertex moves at once by Delta_v = F_v * min(|F_v|, t_h) / |F_v| (the
 * temperature cap of Section 3.1; synchronous update of Section 4.5), and the
 * temperature cools along a schedule (Section 5.1).
 *
 * Conventions for every entry point
 *   - Return value: GILA_OK (0) or a negative status.  No exception or signal
 *     crosses the ABI.  gila_last_error() gives a thread-local message for the
 *     last failing call on the calling thread.
 *   - "_dev" pointers are device (HBM) pointers on the current HIP device;
 *     "_host" pointers are host memory.  The caller owns every buffer it
 *     passes; the library never frees them and keeps no reference after the
 *     call returns (handles copy what they need).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Device work
 *     is ordered on it.  Calls that return statistics synchronise the stream
 *     before returning.
 *   - Argument and graph validation happens before any compute kernel runs and
 *     returns GILA_EINVAL.  Device allocation failure returns GILA_ENOMEM; a
 *     failing HIP call returns GILA_EDEVICE.
 *   - Positions are interleaved (x, y) pairs: float[2n] for GILA_FP32 and
 *     GILA_FP32_KAHAN, double[2n] for GILA_FP64.
 *   - Calls that share a handle, or the stream a handle's work is on, must not
 *     overlap; distinct handles may be used from distinct threads.
 */
#ifndef GILA_H
#define GILA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ */
/* Status codes and precisions                                        */
/* ------------------------------------------------------------------ */
enum {
    GILA_OK = 0,
    GILA_EINVAL = -1,       /* bad argument or malformed graph */
    GILA_ENOMEM = -2,       /* device or host allocation failed / over budget */
    GILA_EDEVICE = -3,      /* a HIP call failed (fault, launch error) */
    GILA_EAGAIN = -4,       /* result not ready yet (gila_poll) */
    GILA_ECANCELED = -5,    /* job was cancelled */
    GILA_EUNSUPPORTED = -6, /* valid request the library does not support */
    GILA_ENONFINITE = -7    /* a force was not finite in the chosen precision (points too
                               close for the force exponents): those vertices did not move
                               and the run stopped after that iteration */
};

enum {
    GILA_FP64 = 0,          /* double positions, double per-pair terms and sums */
    GILA_FP32 = 1,          /* float positions and per-pair terms, plain float lane sums */
    GILA_FP32_KAHAN = 2     /* float positions and terms, Kahan-compensated lane sums */
};
/* In every precision the per-vertex combine of lane sums, the cap, and the
 * global reductions (energy, max displacement, moved count) are done in
 * double (64-bit) arithmetic. */

/* Force model (Section 3.1: ||f^a|| = delta^p / d, ||f^r|| = d^2 / delta^q
 * with integer exponents).  The repulsion term on v from u is
 * (x_v - x_u) d^2 / delta^(q+1) and the attraction term (x_u - x_v)
 * delta^(p-1) / d; coincident ends exert no force. */
enum {
    GILA_MODEL_FR = 0,      /* p = 2, q = 1 (Fruchterman-Reingold; a zeroed struct) */
    GILA_MODEL_LINLOG = 1,  /* p = 0, q = 1 (Noack's LinLog model, Section 6) */
    GILA_MODEL_PQ = 2       /* p = force_p, q = force_q, each in [0, 8] */
};

const char* gila_strerror(int status);
/* Message of the last failing call on this thread ("" if none). */
const char* gila_last_error(void);
/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int gila_version(void);

/* Device memory of freed handles.  gila_khop_free, gila_pruned_free and
 * gila_batch_free wait once for the whole device (so a handle may be freed
 * while work on it is still queued on any stream), then keep the handle's
 * device blocks in the library's per-device cache, where later handles of
 * similar sizes reuse them without a hipMalloc.  The cache holds at most
 * 16 GiB (older blocks beyond that are returned to the device), and all of it
 * is returned before an allocation of the library is reported as failed.
 * The one-shot calls (gila_layout, gila_layout_pruned, gila_layout_batch)
 * release their handles into the cache ordered on their stream, without a
 * device-wide wait.  gila_release_cached_memory returns every cached block
 * whose releasing work has completed to the device (hipFree) and gives the
 * bytes returned; it never fails. */
int64_t gila_release_cached_memory(void);

/* ------------------------------------------------------------------ */
/* Graph                                                                */
/* ------------------------------------------------------------------ */
/* Simple undirected graph G = (V, E) (Section 3.1) in symmetric CSR form:
 * row_ptr[n+1] (row_ptr[0] = 0, row_ptr[n] = nnz = 2|E|), col_idx[nnz] with
 * each row strictly ascending, no self-loop, and u in row v iff v in row u.
 * Isolated vertices are allowed: they feel no force and never move. */
typedef struct gila_csr {
    int32_t n;
    int64_t nnz;
    const int64_t* row_ptr;
    const int32_t* col_idx;
} gila_csr;

/* ------------------------------------------------------------------ */
/* k-neighbourhood lists N_v(k) (Section 4.5)                          */
/* ------------------------------------------------------------------ */
typedef struct gila_khop gila_khop;

/* Build N_v(k) for every vertex of g_dev (device CSR) with k >= 1.
 * The graph is validated (EINVAL on any CSR rule above, or k < 1), copied into
 * the handle and relabelled internally (non-isolated vertices first; by
 * decreasing |N_v(k)|, or in the caller's order when most edges are short in
 * it -- results are returned in caller ids either way), and its k-hop lists
 * are built by CSR frontier expansion on the device.  The handle owns all of
 * its device memory (lists, internal graph copy, iteration workspace) until
 * gila_khop_free.  Synchronises `stream`. */
int gila_build_khop(const gila_csr* g_dev, int32_t k, void* stream, gila_khop** out);

/* Sizes of a handle: vertex count, k, total ordered pairs P = sum |N_v(k)|,
 * non-isolated vertex count, and device bytes the handle holds.  Any output
 * pointer may be NULL. */
int gila_khop_info(const gila_khop* kh, int32_t* n, int32_t* k, int64_t* total_pairs,
                   int32_t* n_active, int64_t* device_bytes);

/* Canonical lists in the caller's vertex ids: ptr_host[n+1] and
 * idx_host[total_pairs], each row ascending and without v.  Either may be
 * NULL to skip it.  Synchronises the handle's internal work. */
int gila_khop_export(const gila_khop* kh, int64_t* ptr_host, int32_t* idx_host);

/* The handle's internal vertex order: order_host[i] (i < n) is the caller id
 * of the vertex the iteration kernels hold at position i.  Without
 * degree-order override (GILA_ORDER) it is either |N_v(k)| descending, or,
 * when most edges join vertices less than 1024 apart in the caller's ids,
 * rows of at least 8192 k-hop entries first and then the caller's order; in
 * both, isolated vertices come last and ties keep ascending caller ids.  It
 * decides the order of every sum, hence the bits of every result.  EINVAL for
 * a NULL handle or order_host.  Synchronous. */
int gila_khop_order(const gila_khop* kh, int32_t* order_host);

/* Rows of selected vertices only: for i < count, row verts_host[i] goes to
 * idx_host[ptr_host[i] .. ptr_host[i+1]) in caller ids, ascending.  With
 * idx_host == NULL only ptr_host[count+1] is written (to size the buffer). */
int gila_khop_export_rows(const gila_khop* kh, int64_t count, const int32_t* verts_host,
                          int64_t* ptr_host, int32_t* idx_host);

void gila_khop_free(gila_khop* kh);

/* Weights of the repulsion each vertex exerts (Section 4.6: a vertex from
 * which L degree-one neighbours were pruned repels with weight 1 + L, so the
 * disc its leaves are put back on stays clear).  The repulsion on v from u
 * becomes w_u (x_v - x_u) d^2 / delta^2; attraction is unchanged.  mass_dev
 * is double[n] on the device, caller ids, every weight in [0, 1e30]; it is
 * copied into the handle (EINVAL, and the previous weights kept, if any is
 * out of range).  NULL restores unit weights.  The next iteration call
 * rebuilds the segment layout for the weighted kernels (a weight is staged in
 * LDS beside each position).  Synchronises `stream`. */
int gila_khop_set_mass(gila_khop* kh, const double* mass_dev, void* stream);

/* ------------------------------------------------------------------ */
/* Layout parameters                                                    */
/* ------------------------------------------------------------------ */
typedef struct gila_params {
    int32_t precision;          /* GILA_FP64 | GILA_FP32 | GILA_FP32_KAHAN */
    double ideal_length;        /* d > 0 (Section 3.1; the paper uses 20 + sqrt(800)) */
    int32_t iterations;         /* H >= 0: length of temperature[] */
    const double* temperature;  /* host [H]: cap t_h >= 0 of iteration h */
    double stop_fraction;       /* > 0 enables the halting rule of Section 5.1: stop after
                                   an iteration in which fewer than stop_fraction * n_active
                                   vertices moved more than stop_displacement; 0 = off */
    double stop_displacement;   /* threshold of that rule (the paper: 0.01) */
    int32_t force_model;        /* GILA_MODEL_* (0 = FR).  The batched entry points and the
                                   server run FR only (other models: EUNSUPPORTED) */
    int32_t force_p;            /* GILA_MODEL_PQ: attraction exponent p */
    int32_t force_q;            /* GILA_MODEL_PQ: repulsion exponent q */
} gila_params;

typedef struct gila_stats {
    int32_t iterations_run;     /* iterations executed by the call */
    int32_t stopped;            /* 1 if the halting rule ended the run */
    int64_t moved;              /* last iteration: #{v : |Delta_v| > stop_displacement} */
    double max_disp;            /* last iteration: max_v |Delta_v| */
    double energy;              /* last iteration: sum_v |F_v|^2 */
    int64_t coincident;         /* last iteration: ordered pairs at distance 0 (no force) */
    int64_t nonfinite;          /* last iteration: vertices whose force was not finite
                                   (they did not move; the call returns GILA_ENONFINITE) */
} gila_stats;

/* Cap schedules (Section 5.1), written to temperature_host[0 .. iterations):
 *   paper:  t_h = sqrt((n / a) d) 0.93^h, h from 0 -- the paper's cap with n
 *           the vertex count and a the height / width ratio of the initial
 *           drawing's bounding box (both > 0; EINVAL otherwise);
 *   linear: t_h = t0 - t0 h / iterations (t0 >= 0), from t0 down to
 *           t0 / iterations.
 * Host only (no device work).  iterations >= 0; temperature_host may be NULL
 * only when iterations is 0. */
int gila_paper_schedule(double n, double aspect, double ideal_length, int32_t iterations,
                        double* temperature_host);
int gila_linear_schedule(double t0, int32_t iterations, double* temperature_host);

/* Seeded uniform placement in [0, width) x [0, height) (Section 5.1 places the
 * vertices at random in a 1200 x 1200 frame).  Coordinate c in {0: x, 1: y}
 * of vertex v is u * width (or height) with u = (s >> 11) * 2^-53 and s the
 * (2v + c)-th output of SplitMix64 seeded with `seed` (Steele, Lea, Flood
 * 2014).  Written to pos_dev in the precision's layout. */
int gila_init_positions(int32_t n, uint64_t seed, double width, double height,
                        int32_t precision, void* pos_dev, void* stream);

/* One iteration h (cap params->temperature[h]) on pos_dev (caller ids,
 * in/out): every F_v from the current positions (Section 3.1 force equation,
 * repulsion over N_v(k) and attraction over the edges as in the second
 * superstep of Section 4.5), then every vertex moved at once by the capped
 * displacement (Section 3.1 cap; the synchronous coordinate update at the end
 * of a Section 4.5 iteration).  If force_dev / disp_dev are not NULL they
 * receive F_v and Delta_v (double[2n], caller ids).  `out` (may be NULL)
 * receives the iteration's statistics; the call synchronises when
 * out != NULL.  The halting rule is not applied by a single step.
 * GILA_ENONFINITE: some F_v was not finite; those vertices did not move. */
int gila_step(const gila_khop* kh, const gila_params* params, int32_t h, void* pos_dev,
              double* force_dev, double* disp_dev, void* stream, gila_stats* out);

/* Iterations h = start_h .. end_h-1 (end_h <= params->iterations) on a built
 * handle, positions in/out at pos_dev (caller ids): the iteration of gila_step
 * repeated with the caps of the schedule (Section 5.1) and, when
 * params->stop_fraction > 0, the halting rule of Section 5.1 evaluated after
 * every iteration.  The loop runs on the device (captured as a HIP graph); a
 * run split at any h gives the same bits as one run.  GILA_ENONFINITE: the
 * run stopped after an iteration with a non-finite force (`out` describes
 * it).  Synchronises `stream`. */
int gila_run(const gila_khop* kh, const gila_params* params, int32_t start_h, int32_t end_h,
             void* pos_dev, void* stream, gila_stats* out);

/* Measurement: iterations h .. h + reps - 1 run on `stream` exactly as
 * gila_run runs them (captured as one HIP graph; eager launches if the
 * capture is refused), advancing pos_dev, between two HIP events; on the
 * segment path each force kernel also records on the device wall clock when
 * its first workgroup started and its last one ended.  ms_out[0] receives the
 * force kernel's average span (on the direct path, the whole iteration: its
 * gather kernel moves the vertices itself), ms_out[1] the iteration's average
 * from the events minus ms_out[0] (the combine and statistics kernels and the
 * launch gaps; 0 on the direct path), ms_out[2] 1 if the iterations ran as a
 * graph replay, 0 if eagerly; ms_out holds 3 doubles.  Synchronises
 * `stream`. */
int gila_time_iterations(const gila_khop* kh, const gila_params* params, int32_t h,
                         int32_t reps, void* pos_dev, void* stream, double* ms_out);

/* Per-iteration statistics.  After gila_enable_history(kh, capacity, ...),
 * every iteration h < capacity that gila_step, gila_run or
 * gila_time_iterations then runs on this handle writes its FP64 statistics --
 * the energy sum_v |F_v|^2, the largest |Delta_v| and the number of vertices
 * that moved more than stop_displacement (Section 5.1's halting statistic),
 * and the coincident pairs -- as row h of a device table, the same values
 * gila_stats reports for that iteration.  gila_history copies rows
 * [h0, h0 + count) to rows_host[count][4] (energy, max_disp, moved,
 * coincident); rows of iterations not run (past the schedule, or after the
 * halting rule stopped the run) read as NaN.  capacity 0 frees the table.
 * Enabling replaces the table (all rows NaN again) and drops the handle's
 * captured loops.  EINVAL for a negative capacity or rows outside the table.
 * Both synchronise `stream`. */
int gila_enable_history(gila_khop* kh, int32_t capacity, void* stream);
int gila_history(const gila_khop* kh, int32_t h0, int32_t count, double* rows_host,
                 void* stream);

/* Whole layout of one graph (the layout phase of Section 4.5 on a graph the
 * caller has already reduced as Sections 4.3 and 4.6 describe, or not):
 * gila_build_khop, gila_run over all params->iterations, free.
 * Synchronises `stream`. */
int gila_layout(const gila_csr* g_dev, int32_t k, const gila_params* params, void* pos_dev,
                void* stream, gila_stats* out);

/* ------------------------------------------------------------------ */
/* Degree-one vertices: pruning and reinsertion (Sections 4.3, 4.6)     */
/* ------------------------------------------------------------------ */
typedef struct gila_pruned gila_pruned;

/* Prune the degree-one vertices of g_dev (device CSR, validated as for
 * gila_build_khop).  A vertex of degree one is removed unless its only
 * neighbour also has degree one and a larger id (one end of each isolated
 * edge stays); one pass, so every removed vertex hangs from a kept one.  The
 * kept vertices, renumbered in ascending original id, and the edges among
 * them form the pruned graph.  The handle owns its device memory until
 * gila_pruned_free.  Synchronises `stream`. */
int gila_prune(const gila_csr* g_dev, void* stream, gila_pruned** out);

/* Sizes: kept vertices, adjacency entries of the pruned graph, pruned
 * vertices, kept vertices with at least one pruned neighbour, device bytes
 * held.  Any output may be NULL. */
int gila_pruned_info(const gila_pruned* p, int32_t* n_kept, int64_t* nnz_kept, int32_t* n_pruned,
                     int32_t* n_with_leaves, int64_t* device_bytes);

/* The pruned graph as a device CSR and the repulsion weights of its vertices
 * (double[n_kept], 1 + pruned neighbours; for gila_khop_set_mass).  Both
 * point into the handle: valid until gila_pruned_free.  Either output may be
 * NULL. */
int gila_pruned_graph(const gila_pruned* p, gila_csr* g_dev_out, const double** mass_dev_out);

/* Host copies, each int32[n] in original ids (any may be NULL): the kept
 * vertex a pruned vertex hung from (-1 for kept vertices), the number of
 * vertices pruned from each vertex, and each vertex's id in the pruned graph
 * (-1 for pruned vertices).  Synchronous. */
int gila_pruned_export(const gila_pruned* p, int32_t* anchor_host, int32_t* leaves_host,
                       int32_t* new_id_host);

/* pos_kept_dev[new_id[v]] = pos_all_dev[v] for every kept v (positions in
 * the precision's layout).  Enqueued on `stream`. */
int gila_pruned_gather(const gila_pruned* p, int32_t precision, const void* pos_all_dev,
                       void* pos_kept_dev, void* stream);

/* Reinsertion (Section 4.6): pos_all_dev receives every vertex of the
 * original graph.  Kept vertices take their position in pos_kept_dev (the
 * drawing of the pruned graph).  The L vertices pruned from kept vertex v go,
 * in ascending id, to v + rho (cos a_j, sin a_j) with a_j = phi + 2 pi j / L,
 * rho = 0.2 x the length of v's shortest edge in the pruned drawing
 * (0.2 x ideal_length if v has none), and phi the middle of the widest gap
 * between the angles of v's edges taken modulo 2 pi / L (the first widest
 * in ascending order; 0 without edges): the leaves are spread evenly and as
 * far as possible in angle from the edges.  Computed in double; enqueued on
 * `stream`. */
int gila_reinsert(const gila_pruned* p, double ideal_length, int32_t precision,
                  const void* pos_kept_dev, void* pos_all_dev, void* stream);

void gila_pruned_free(gila_pruned* p);

/* The pipeline of Sections 4.3 - 4.6 on one graph: prune, build N_v(k) of the
 * pruned graph, weight each kept vertex's repulsion by 1 + its pruned
 * neighbours, run all params->iterations from the kept vertices' positions in
 * pos_dev (the pruned vertices' entries are ignored), then reinsert, writing
 * every vertex to pos_dev.  `out` describes the iterations on the pruned
 * graph (n_active and the halting rule count its vertices).  Synchronises. */
int gila_layout_pruned(const gila_csr* g_dev, int32_t k, const gila_params* params, void* pos_dev,
                       void* stream, gila_stats* out);

/* ------------------------------------------------------------------ */
/* Connected components: each laid out alone, then packed (Section 4.6) */
/* ------------------------------------------------------------------ */

/* label_dev[v] (device int32[n]) = the smallest vertex id of v's connected
 * component.  count_out (may be NULL) receives the number of components.
 * The graph is validated as for gila_build_khop.  Synchronises `stream`. */
int gila_components(const gila_csr* g_dev, int32_t* label_dev, int32_t* count_out, void* stream);

/* gila_components for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same labels (label_dev as gila_components writes it, bit for bit) and
 * count, with no hipMalloc, hipFree or other allocating call.  The graph is
 * validated on the device (EINVAL as for gila_build_khop).  Its scratch (CSR
 * flags, the per-pass hooked flag, per-workgroup root counts) is a fixed
 * 16 KiB array of device memory inside the library, one copy per device,
 * held until the process ends; no graph needs more, so no size is refused
 * for it.  Every call on a device uses that device's copy: calls that
 * overlap on one device (other threads or streams) race and must be
 * serialised by the caller.  Synchronises `stream`. */
int gila_components_noalloc(const gila_csr* g_dev, int32_t* label_dev, int32_t* count_out,
                            void* stream);

/* Packs the drawings of the components in a matrix (Section 4.6), in place:
 * components in order of decreasing vertex count (ties: smaller label) fill
 * ceil(sqrt(C)) columns row by row; a column is as wide as its widest drawing
 * and a row as tall as its tallest, consecutive columns and rows `gap` apart,
 * the first cell's lower-left corner at the origin; every drawing is
 * translated so that its bounding box's lower-left corner is its cell's.
 * label_dev as gila_components writes it (each label in [0, n) and naming a
 * vertex labelled with itself; EINVAL otherwise).  Synchronises `stream`. */
int gila_pack_components(int32_t n, const int32_t* label_dev, double gap, int32_t precision,
                         void* pos_dev, void* stream);

/* Sections 4.6 and 5.1 on one graph: every connected component with at least
 * two vertices is laid out on its own from its vertices' positions in pos_dev,
 * for params->iterations iterations with the cap
 * sqrt((n_C / a_C) d) 0.93^h -- n_C its vertex count, a_C the height / width
 * of its initial drawing's bounding box (1 when that box has no area) -- and
 * with params' halting rule applied to the component alone; then the
 * drawings are packed with gap d (gila_pack_components).
 * params->temperature is ignored (may be NULL).  Components of up to 2048
 * vertices run together in one batched launch when the force model is FR,
 * larger ones on the whole GPU one after another.  components_out: number of
 * components; iterations_host (host int32[n]): for every vertex, the
 * iterations its component ran (0 for a vertex without edges).  Either may
 * be NULL.  Synchronises `stream`. */
int gila_layout_components(const gila_csr* g_dev, int32_t k, const gila_params* params,
                           void* pos_dev, void* stream, int32_t* components_out,
                           int32_t* iterations_host);

/* ------------------------------------------------------------------ */
/* Drawing-quality metrics (Section 5.2)                                */
/* ------------------------------------------------------------------ */
enum {
    GILA_METRIC_CROSSINGS = 1,   /* edge crossings (all pairs of edges: O(m^2) work) */
    GILA_METRIC_LENGTHS = 2,     /* mean and standard deviation of the edge lengths */
    GILA_METRIC_SIMILARITY = 4   /* Gabriel-graph similarity */
};

typedef struct gila_metrics {
    int64_t edges;              /* m: undirected edges */
    int64_t crossings;          /* pairs of edges that cross (no shared end; each end strictly
                                   on the opposite side of the other edge's line) */
    double edge_length_mean;
    double edge_length_std;     /* population standard deviation */
    double similarity;          /* mean over vertices of the Jaccard index of the vertex's
                                   neighbours in the graph and in the Gabriel graph of the
                                   drawing's points (1 for a vertex with neither) */
    int64_t gabriel_edges;      /* edges of that Gabriel graph: u, v adjacent when no other
                                   point lies in the closed disc with diameter uv */
} gila_metrics;

/* The quality measures of Section 5.2 for the drawing pos_dev (positions in
 * `precision`'s layout, taken at single precision, where every orientation
 * and in-disc sign is decided exactly) of the graph g_dev (validated as for
 * gila_build_khop).  `what` is an OR of GILA_METRIC_*; the others are left 0
 * (similarity 1).  edge_crossings_dev (device int64[m], may be NULL)
 * receives the crossings of every edge, edges {u, v} with u < v numbered in
 * row order (row v, its entries above v); without it each pair of edges is
 * tested once, with it twice.  jaccard_dev (device double[n], may be NULL)
 * receives the per-vertex Jaccard indices.  Crossings per edge (CRE) are
 * crossings / edges.  Positions must be finite (EINVAL otherwise).
 * Synchronises `stream`. */
int gila_drawing_metrics(const gila_csr* g_dev, int32_t precision, const void* pos_dev,
                         int32_t what, void* stream, gila_metrics* out,
                         int64_t* edge_crossings_dev, double* jaccard_dev);

/* ------------------------------------------------------------------ */
/* Many graphs in one launch                                            */
/* ------------------------------------------------------------------ */
typedef struct gila_batch gila_batch;

/* Build the k-hop lists N_v(k) (Section 4.5) of `count` independent graphs
 * (graphs_dev[i] is a device CSR with at most 65535 vertices, k[i] >= 1) into
 * one segmented handle, and fix each graph's plan: its lanes per vertex (the
 * order in which its force terms are summed, hence its result bits), from
 * its row-length class c (see gila_batch_plan) -- one lane while
 * 4 * 2^c <= 128, else about 128 entries per lane, a power of two in
 * [1, 64] -- and, for a graph of fewer than 256 vertices, at least the
 * largest power of two L with n L <= 512 (so its vertices fill a
 * workgroup).  The plan depends only on the graph, so a graph's result is
 * the same bits alone, in any batch and in any process.  Synchronises. */
int gila_batch_build(const gila_csr* graphs_dev, int32_t count, const int32_t* k,
                     void* stream, gila_batch** out);

/* All iterations of every graph of the batch in one persistent segmented
 * launch (the Section 4.5 iteration with each graph's own cap schedule and
 * halting rule, Section 5.1), each graph with its plan's lanes per vertex.
 * params[i] and pos_dev[i] belong to graph i; all graphs must use the same
 * precision and the FR model.  out (may be NULL) is [count].
 * GILA_ENONFINITE: some graph met a non-finite force (its out[] entry counts
 * the vertices; its run stopped there; the other graphs are unaffected).
 * Synchronises. */
int gila_batch_run(gila_batch* b, const gila_params* params, void* const* pos_dev,
                   void* stream, gila_stats* out);

int gila_batch_info(const gila_batch* b, int32_t* count, int64_t* total_pairs,
                    int64_t* device_bytes);

/* The handle's plan: lanes_host[count] receives each graph's lanes per vertex,
 * class_host[count] its row-length class c = the largest c <= 7 with
 * mean |N_v(k)| >= 2^(c+1) (0 below 4), so that the class's means lie below
 * 4 * 2^c.  Either may be NULL. */
int gila_batch_plan(const gila_batch* b, int32_t* lanes_host, int32_t* class_host);

/* Replaces the plan: lanes_host[count], each a power of two in [1, 64]
 * (EINVAL otherwise, plan unchanged).  A plan read with gila_batch_plan (or
 * derived from a gila_batch_tune table by class) and set again reproduces
 * that run's bits. */
int gila_batch_set_plan(gila_batch* b, const int32_t* lanes_host);

/* Tuner (the project's own): for each row-length class present in the batch,
 * times every lanes-per-vertex choice on up to 48 of its graphs (8 iterations
 * at cap 0 from seeded positions, in scratch memory; the caller's positions
 * are not touched) in `precision`, and sets the fastest in the plan of every
 * graph of the class (raised, for small graphs, to the lanes that fill a
 * workgroup, as at build).  class_lanes_host[8] (may be NULL) receives the
 * choice per class (0: class absent), for the caller to keep and apply to
 * later batches.  Never run implicitly.  Synchronises `stream`. */
int gila_batch_tune(gila_batch* b, int32_t precision, void* stream, int32_t* class_lanes_host);

/* Latency of each graph in the last gila_batch_run: ms_host[count] receives
 * the time from the start of the first graph's work to the moment graph i's
 * positions were written back (device wall clock). */
int gila_batch_latency(const gila_batch* b, double* ms_host);

/* The k-hop lists N_v(k) of graph `graph` of a built batch, in that graph's own
 * vertex ids: ptr_host[n + 1] (ptr_host[0] = 0) and idx_host[ptr_host[n]],
 * each row ascending.  idx_host may be NULL to size the rows first.  EINVAL
 * for a NULL batch or ptr_host or a graph index out of range.  Synchronous. */
int gila_batch_export(const gila_batch* b, int32_t graph, int64_t* ptr_host, int32_t* idx_host);
void gila_batch_free(gila_batch* b);

/* gila_batch_build + gila_batch_run + gila_batch_free. */
int gila_layout_batch(const gila_csr* graphs_dev, int32_t count, const int32_t* k,
                      const gila_params* params, void* const* pos_dev, void* stream,
                      gila_stats* out);

/* ------------------------------------------------------------------ */
/* Serving: continuous batching of layout jobs                          */
/* ------------------------------------------------------------------ */
typedef struct gila_server gila_server;

/* A server owns five threads (admission, k-hop builds, two for batched small jobs,
 * ticks) and its own streams on `device`.  Unlike the other handles, a server
 * may be used from several threads at once: gila_submit, gila_poll,
 * gila_wait, gila_cancel, gila_job_latency and gila_server_info serialise on
 * the server's lock (gila_wait sleeps without holding it).  A job's result is
 * taken by one gila_poll or gila_wait; other calls on that ticket, also ones
 * already waiting, then return GILA_EINVAL.  gila_server_destroy must not
 * overlap any other call on the server.  Jobs are admitted in arrival order
 * while their device footprint bound fits in hbm_budget_bytes (0 = 90% of free
 * HBM) and fewer than max_slots jobs are in flight.  Small jobs are laid out
 * together in batched launches; larger ones are built, then advance a few
 * iterations per tick, each job's next tick queued as soon as its previous
 * one has ended (a replay of the job's captured tick); builds, batched
 * launches and ticks overlap.
 * Device memory released by the server goes to the library's block cache
 * (reused without device-wide synchronisation). */
int gila_server_create(int32_t device, int64_t hbm_budget_bytes, int32_t max_slots,
                       gila_server** out);

/* Queue a job.  g_host is a host CSR, init_pos_host double[2n]; both and the
 * temperature array are copied before return.  ticket receives the job id.
 * Returns EINVAL for bad parameters or out-of-range indices; the remaining
 * graph rules (sorted rows, no self-loop, symmetry) are checked on the device
 * when the job is admitted, and a violation fails the job with EINVAL (seen by
 * gila_poll).  A job whose footprint bound exceeds the whole budget fails
 * with ENOMEM; one that fits waits until enough memory is free. */
int gila_submit(gila_server* s, const gila_csr* g_host, int32_t k, const gila_params* params,
                const double* init_pos_host, uint64_t* ticket);

/* GILA_EAGAIN while the job is queued or running; GILA_OK once done, after
 * writing out_pos_host double[2n] (may be NULL) and out (may be NULL) and
 * releasing the job; GILA_ECANCELED / other status if it ended otherwise. */
int gila_poll(gila_server* s, uint64_t ticket, double* out_pos_host, gila_stats* out);

/* Block until the job is done (or failed); then as gila_poll. */
int gila_wait(gila_server* s, uint64_t ticket, double* out_pos_host, gila_stats* out);

/* Cancel a queued or running job; its memory is released at the next tick. */
int gila_cancel(gila_server* s, uint64_t ticket);

/* Server settings: "tick_iterations" (iterations a resident job advances per
 * tick, default 50), "small_max_vertices" (largest job laid out by the batched
 * LDS-resident kernel, default 1024 -- one workgroup per graph, so larger jobs
 * finish sooner on the whole-GPU path; 0 = the most that fits in LDS),
 * "fail_alloc_ticket" (test hook: the job with this ticket fails its device
 * allocation with ENOMEM). */
int gila_server_config(gila_server* s, const char* key, int64_t value);

/* Queue wait and total latency (submit to completion, ms) of a finished job;
 * GILA_EAGAIN before it finished.  Kept until the server is destroyed. */
int gila_job_latency(gila_server* s, uint64_t ticket, double* queued_ms, double* total_ms);

/* Counters: jobs done, ticks queued (one per resident large job per tick),
 * peak resident large jobs, device bytes reserved. */
int gila_server_info(gila_server* s, int64_t* jobs_done, int64_t* ticks, int32_t* peak_resident,
                     int64_t* bytes_in_use);

void gila_server_destroy(gila_server* s);

#ifdef __cplusplus
}
#endif

#endif /* GILA_H */

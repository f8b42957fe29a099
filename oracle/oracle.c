/*
 * oracle.c -- plain, slow, FP64 CPU oracle of GiLA's k-hop
 * Fruchterman-Reingold layout (Arleo, Didimo, Liotta, Montecchiani,
 * "A Distributed Force-Directed Algorithm on Giraph").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; both receive the same input
 * arrays from the seeded generators.
 *
 * What it computes (each function names its passage):
 *   - N_v(k): every vertex at graph distance <= k from v, v itself excluded,
 *     sorted ascending (Section 4.5, definition of the k-neighbourhood; the
 *     flooding with TTL delivers exactly this set for k >= 2).  Computed by a
 *     textbook BFS from every vertex.
 *   - F_v = sum over adjacent u of the attractive force plus sum over
 *     u in N_v(k) of the repulsive force (Section 3.1 force equation with the
 *     repulsion sum restricted to N_v(k) by Section 4.5).  Magnitudes
 *     ||f^a|| = delta^p / d and ||f^r|| = d^2 / delta^q with p = 2, q = 1
 *     (Section 3.1).  Attraction points from v towards u, repulsion away from
 *     u.  Adjacent vertices contribute both (Section 4.5, second superstep).
 *   - Displacement capped by the temperature t_h, all vertices moved together
 *     once every force of the iteration is known (Section 3.1; Section 4.5,
 *     coordinates updated when no message is left).
 *   - Halting statistic: number of vertices displaced by more than a
 *     threshold (Section 5.1: stop when fewer than 15% moved more than 0.01).
 *
 * Readings where the paper is silent: a pair of distinct vertices at the same
 * point (delta = 0) contributes no force and is counted; F_v = 0 gives no
 * move; coordinates are not clamped to any frame.
 *
 * Sums are plain sequential double sums in ascending neighbour id.  OpenMP
 * splits the *vertices* across threads (never a sum), so results do not
 * depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* ------------------------------------------------------------------ */
/* k-neighbourhoods by breadth-first search (Section 4.5)              */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* BFS from `src` to depth k.  dist[] must be all -1 on entry and is restored
 * to all -1 on return.  The reached vertices other than src are written to
 * out[] (capacity n) in BFS order; returns their number. */
static int64_t bfs_ball(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
                        int32_t k, int32_t src, int32_t* dist, int32_t* queue,
                        int32_t* out) {
    int64_t head = 0, tail = 0, found = 0;
    (void)n;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t w = queue[head++];
        if (dist[w] == k) continue;
        for (int64_t e = row_ptr[w]; e < row_ptr[w + 1]; ++e) {
            int32_t u = col_idx[e];
            if (dist[u] < 0) {
                dist[u] = dist[w] + 1;
                queue[tail++] = u;
                out[found++] = u;
            }
        }
    }
    for (int64_t i = 0; i < tail; ++i) dist[queue[i]] = -1;
    return found;
}

/* |N_v(k)| for every v in verts[0..count) (or all vertices if verts == NULL). */
int orc_khop_count(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t k,
                   int64_t count, const int32_t* verts, int64_t* sizes) {
    if (n < 0 || k < 1) return ORC_EINVAL;
    if (verts == NULL) count = n;
    int err = ORC_OK;
#pragma omp parallel
    {
        int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int32_t* out = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        if (!dist || !queue || !out) {
#pragma omp atomic write
            err = ORC_ENOMEM;
        } else {
            for (int32_t i = 0; i < n; ++i) dist[i] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < count; ++i) {
                int32_t v = verts ? verts[i] : (int32_t)i;
                sizes[i] = bfs_ball(n, row_ptr, col_idx, k, v, dist, queue, out);
            }
        }
        free(dist);
        free(queue);
        free(out);
    }
    return err;
}

/* Fill the rows of N_v(k), sorted ascending, at idx[ptr[i] .. ptr[i+1]) for
 * v = verts[i] (or v = i if verts == NULL).  ptr must come from the sizes of
 * orc_khop_count (exclusive prefix sum). */
int orc_khop_fill(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t k,
                  int64_t count, const int32_t* verts, const int64_t* ptr, int32_t* idx) {
    if (n < 0 || k < 1) return ORC_EINVAL;
    if (verts == NULL) count = n;
    int err = ORC_OK;
#pragma omp parallel
    {
        int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        if (!dist || !queue) {
#pragma omp atomic write
            err = ORC_ENOMEM;
        } else {
            for (int32_t i = 0; i < n; ++i) dist[i] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < count; ++i) {
                int32_t v = verts ? verts[i] : (int32_t)i;
                int32_t* row = idx + ptr[i];
                int64_t got = bfs_ball(n, row_ptr, col_idx, k, v, dist, queue, row);
                if (got != ptr[i + 1] - ptr[i]) {
#pragma omp atomic write
                    err = ORC_EINVAL;
                } else {
                    qsort(row, (size_t)got, sizeof(int32_t), cmp_i32);
                }
            }
        }
        free(dist);
        free(queue);
    }
    return err;
}

/* ------------------------------------------------------------------ */
/* Forces (Section 3.1 with p = 2, q = 1; Section 4.5 locality)       */
/* ------------------------------------------------------------------ */

/* One vertex: F_v = attraction over adj(v) + repulsion over N_v(k).
 * pos is interleaved (x, y).  Returns the number of coincident pairs. */
static int64_t force_one(int32_t v, const int64_t* row_ptr, const int32_t* col_idx,
                         const int32_t* krow, int64_t klen, double d,
                         const double* pos, double* fx_out, double* fy_out) {
    const double xv = pos[2 * (int64_t)v], yv = pos[2 * (int64_t)v + 1];
    double ax = 0.0, ay = 0.0, rx = 0.0, ry = 0.0;
    int64_t coincident = 0;
    /* attraction: ||f^a|| = delta^2 / d, pointing from v towards u */
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        int32_t u = col_idx[e];
        double dx = pos[2 * (int64_t)u] - xv;
        double dy = pos[2 * (int64_t)u + 1] - yv;
        double delta = sqrt(dx * dx + dy * dy);
        /* unit vector (dx, dy) / delta times delta^2 / d */
        ax += dx * (delta / d);
        ay += dy * (delta / d);
    }
    /* repulsion: ||f^r|| = d^2 / delta, pointing from u towards v */
    for (int64_t i = 0; i < klen; ++i) {
        int32_t u = krow[i];
        double dx = xv - pos[2 * (int64_t)u];
        double dy = yv - pos[2 * (int64_t)u + 1];
        double dd = dx * dx + dy * dy;
        if (dd == 0.0) {
            ++coincident;
            continue;
        }
        /* unit vector (dx, dy) / delta times d^2 / delta */
        rx += dx * (d * d / dd);
        ry += dy * (d * d / dd);
    }
    *fx_out = ax + rx;
    *fy_out = ay + ry;
    return coincident;
}

/* Forces on verts[0..count) (all vertices if verts == NULL).  For the i-th
 * vertex its k-hop row is kidx[kptr[i] .. kptr[i+1]) -- rows indexed like
 * verts, so a sampled subset carries only its own rows.  F is [count][2]. */
int orc_forces(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
               int64_t count, const int32_t* verts, const int64_t* kptr,
               const int32_t* kidx, double d, const double* pos, double* F,
               int64_t* coincident_out) {
    if (n < 0 || !(d > 0.0)) return ORC_EINVAL;
    if (verts == NULL) count = n;
    int64_t coincident = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : coincident)
    for (int64_t i = 0; i < count; ++i) {
        int32_t v = verts ? verts[i] : (int32_t)i;
        coincident += force_one(v, row_ptr, col_idx, kidx + kptr[i], kptr[i + 1] - kptr[i],
                                d, pos, &F[2 * i], &F[2 * i + 1]);
    }
    if (coincident_out) *coincident_out = coincident;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Capped move (Section 3.1: displacement limited by the temperature)  */
/* ------------------------------------------------------------------ */

/* Delta = F * min(|F|, t) / |F|, and 0 when |F| = 0. */
int orc_cap(int64_t count, const double* F, double t, double* D) {
    if (!(t >= 0.0)) return ORC_EINVAL;
    for (int64_t i = 0; i < count; ++i) {
        double fx = F[2 * i], fy = F[2 * i + 1];
        double norm = sqrt(fx * fx + fy * fy);
        if (norm == 0.0) {
            D[2 * i] = 0.0;
            D[2 * i + 1] = 0.0;
        } else {
            double len = norm < t ? norm : t;
            D[2 * i] = fx * (len / norm);
            D[2 * i + 1] = fy * (len / norm);
        }
    }
    return ORC_OK;
}

typedef struct {
    int64_t moved;     /* #{v : |Delta_v| > stop_displacement} */
    double max_disp;   /* max_v |Delta_v| */
    double energy;     /* sum_v |F_v|^2 */
    int64_t coincident;
} orc_iter_stats;

/* One synchronous iteration on the whole graph: every force from the current
 * positions, then every vertex moved at once (Section 4.5).  pos is updated in
 * place only after all forces are known.  F and D (both [n][2]) receive the
 * forces and displacements. */
int orc_step(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
             const int64_t* kptr, const int32_t* kidx, double d, double t,
             double stop_displacement, double* pos, double* F, double* D,
             orc_iter_stats* st) {
    int64_t coincident = 0;
    int rc = orc_forces(n, row_ptr, col_idx, n, NULL, kptr, kidx, d, pos, F, &coincident);
    if (rc) return rc;
    rc = orc_cap(n, F, t, D);
    if (rc) return rc;
    int64_t moved = 0;
    double max_disp = 0.0, energy = 0.0;
    for (int32_t v = 0; v < n; ++v) {
        double dl = sqrt(D[2 * v] * D[2 * v] + D[2 * v + 1] * D[2 * v + 1]);
        if (dl > stop_displacement) ++moved;
        if (dl > max_disp) max_disp = dl;
        energy += F[2 * v] * F[2 * v] + F[2 * v + 1] * F[2 * v + 1];
        pos[2 * v] += D[2 * v];
        pos[2 * v + 1] += D[2 * v + 1];
    }
    if (st) {
        st->moved = moved;
        st->max_disp = max_disp;
        st->energy = energy;
        st->coincident = coincident;
    }
    return ORC_OK;
}

/* Iterations h = h0 .. h_end-1 with cap temperature[h].  If stop_fraction > 0
 * the run ends after the first iteration in which fewer than
 * stop_fraction * n_active vertices moved more than stop_displacement
 * (Section 5.1); n_active counts the vertices with at least one edge.
 * Returns the number of iterations run in *iters_run. */
int orc_layout(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
               const int64_t* kptr, const int32_t* kidx, double d,
               const double* temperature, int32_t h0, int32_t h_end,
               double stop_fraction, double stop_displacement, double* pos,
               int32_t* iters_run, orc_iter_stats* last) {
    if (h0 < 0 || h_end < h0) return ORC_EINVAL;
    double* F = (double*)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
    double* D = (double*)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
    if (!F || !D) {
        free(F);
        free(D);
        return ORC_ENOMEM;
    }
    int64_t n_active = 0;
    for (int32_t v = 0; v < n; ++v) n_active += (row_ptr[v + 1] > row_ptr[v]);
    orc_iter_stats st = {0, 0.0, 0.0, 0};
    int32_t run = 0;
    int rc = ORC_OK;
    for (int32_t h = h0; h < h_end; ++h) {
        rc = orc_step(n, row_ptr, col_idx, kptr, kidx, d, temperature[h], stop_displacement,
                      pos, F, D, &st);
        if (rc) break;
        ++run;
        if (stop_fraction > 0.0 && (double)st.moved < stop_fraction * (double)n_active) break;
    }
    free(F);
    free(D);
    if (iters_run) *iters_run = run;
    if (last) *last = st;
    return rc;
}

/* ------------------------------------------------------------------ */
/* Cooling schedules                                                    */
/* ------------------------------------------------------------------ */

/* Section 5.1: maximum displacement at superstep h is
 * sqrt((n / a) * d) * 0.93^h, with n the component's vertex count and a the
 * height/width aspect ratio of its initial frame. */
void orc_paper_schedule(double n, double aspect, double d, int32_t iterations, double* t) {
    double base = sqrt((n / aspect) * d);
    for (int32_t h = 0; h < iterations; ++h) t[h] = base * pow(0.93, (double)h);
}

/* Linear cooling from t0 to t0/iterations: t_h = t0 - t0 h / iterations
 * (exact for integer t0 = iterations, e.g. 100, 99, ..., 1). */
void orc_linear_schedule(double t0, int32_t iterations, double* t) {
    for (int32_t h = 0; h < iterations; ++h)
        t[h] = t0 - (t0 * (double)h) / (double)iterations;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

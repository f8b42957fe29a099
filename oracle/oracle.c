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
 *     ||f^a|| = delta^p / d and ||f^r|| = d^2 / delta^q (Section 3.1): FR's
 *     p = 2, q = 1 by default, any non-negative integers otherwise (the
 *     LinLog model of Section 6 is p = 0, q = 1).  Attraction points from v
 *     towards u, repulsion away from u.  Adjacent vertices contribute both
 *     (Section 4.5, second superstep).  Coincident ends exert no force.
 *   - Displacement capped by the temperature t_h, all vertices moved together
 *     once every force of the iteration is known (Section 3.1; Section 4.5,
 *     coordinates updated when no message is left).
 *   - Halting statistic: number of vertices displaced by more than a
 *     threshold (Section 5.1: stop when fewer than 15% moved more than 0.01).
 *
 *   - Connected components, each laid out on its own with the cap
 *     sqrt((n_C / a_C) d) 0.93^h of its vertex count and initial aspect
 *     ratio (Sections 4.6, 5.1), and the drawings packed in a matrix
 *     (Section 4.6; the per-component driver is in __init__.py).
 *   - Drawing-quality metrics of Section 5.2: edge crossings, the standard
 *     deviation of edge lengths, and the similarity of the drawing's Gabriel
 *     graph to the graph (mean Jaccard index of the neighbourhoods),
 *     evaluated on single-precision coordinates.
 *   - Pruning of degree-one vertices before the layout (Section 4.3), the
 *     repulsion exerted by a vertex weighted by its pruned leaves
 *     (Section 4.6), and reinsertion of the leaves on a circle around their
 *     neighbour after the layout (Section 4.6).
 *
 * Readings where the paper is silent: a pair of distinct vertices at the same
 * point (delta = 0) contributes no force and is counted; F_v = 0 gives no
 * move; coordinates are not clamped to any frame.  Pruning: a degree-one
 * vertex is removed unless its only neighbour also has degree one and a
 * larger id (so one vertex of an isolated edge stays); one pass only.  The
 * weight of the repulsion exerted by u is 1 + (number of leaves pruned from
 * u).  Reinsertion: radius 0.2 times the shortest edge incident to the
 * vertex in the pruned drawing (0.2 d when it has none); its L leaves, in
 * ascending id, at angles phi + 2 pi j / L, with phi chosen so that the
 * leaves are as far as possible (in angle) from the incident edges.
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
/* Forces (Section 3.1, exponents p and q; Section 4.5 locality)      */
/* ------------------------------------------------------------------ */

/* One vertex: F_v = attraction over adj(v) + repulsion over N_v(k).
 * pos is interleaved (x, y).  Returns the number of coincident pairs.  The
 * p = 2 and q = 1 branches are the general expressions with the powers
 * cancelled by hand (no root, no pow). */
static int64_t force_one(int32_t v, const int64_t* row_ptr, const int32_t* col_idx,
                         const int32_t* krow, int64_t klen, double d, const double* mass,
                         int32_t p, int32_t q, const double* pos, double* fx_out,
                         double* fy_out) {
    const double xv = pos[2 * (int64_t)v], yv = pos[2 * (int64_t)v + 1];
    double ax = 0.0, ay = 0.0, rx = 0.0, ry = 0.0;
    int64_t coincident = 0;
    /* attraction: ||f^a|| = delta^p / d, pointing from v towards u */
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        int32_t u = col_idx[e];
        double dx = pos[2 * (int64_t)u] - xv;
        double dy = pos[2 * (int64_t)u + 1] - yv;
        double delta = sqrt(dx * dx + dy * dy);
        if (p == 2) {
            /* unit vector (dx, dy) / delta times delta^2 / d */
            ax += dx * (delta / d);
            ay += dy * (delta / d);
        } else if (delta > 0.0) {
            /* unit vector times delta^p / d; coincident ends exert nothing */
            const double mag = pow(delta, (double)p) / d;
            ax += (dx / delta) * mag;
            ay += (dy / delta) * mag;
        }
    }
    /* repulsion: ||f^r|| = d^2 / delta^q, pointing from u towards v */
    for (int64_t i = 0; i < klen; ++i) {
        int32_t u = krow[i];
        double dx = xv - pos[2 * (int64_t)u];
        double dy = yv - pos[2 * (int64_t)u + 1];
        double dd = dx * dx + dy * dy;
        if (dd == 0.0) {
            ++coincident;
            continue;
        }
        /* weighted by the leaves pruned from u (Section 4.6) when masses
         * are given */
        const double w = mass ? mass[u] : 1.0;
        if (q == 1) {
            /* unit vector (dx, dy) / delta times d^2 / delta */
            rx += dx * (w * (d * d / dd));
            ry += dy * (w * (d * d / dd));
        } else {
            const double delta = sqrt(dd);
            const double mag = d * d / pow(delta, (double)q);
            rx += (dx / delta) * (w * mag);
            ry += (dy / delta) * (w * mag);
        }
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
               const int32_t* kidx, double d, const double* mass, int32_t p, int32_t q,
               const double* pos, double* F, int64_t* coincident_out) {
    if (n < 0 || !(d > 0.0) || p < 0 || q < 0) return ORC_EINVAL;
    if (verts == NULL) count = n;
    int64_t coincident = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : coincident)
    for (int64_t i = 0; i < count; ++i) {
        int32_t v = verts ? verts[i] : (int32_t)i;
        coincident += force_one(v, row_ptr, col_idx, kidx + kptr[i], kptr[i + 1] - kptr[i],
                                d, mass, p, q, pos, &F[2 * i], &F[2 * i + 1]);
    }
    if (coincident_out) *coincident_out = coincident;
    return ORC_OK;
}

/* Sum of the magnitudes of the terms that make up F_v (Section 3.1:
 * ||f^a|| = delta^p / d per adjacent u, ||f^r|| = d^2 / delta^q per u in
 * N_v(k), the latter scaled by u's weight when masses are given; coincident
 * ends contribute nothing, as in the force).  S_v bounds |F_v| and sets the
 * scale of the rounding error of any evaluation of F_v that rounds each term:
 * a sum of terms each off by a relative e is off by at most e * S_v.  Rows as
 * in orc_forces; S is [count]. */
int orc_force_magnitudes(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
                         int64_t count, const int32_t* verts, const int64_t* kptr,
                         const int32_t* kidx, double d, const double* mass, int32_t p,
                         int32_t q, const double* pos, double* S) {
    if (n < 0 || !(d > 0.0) || p < 0 || q < 0) return ORC_EINVAL;
    if (verts == NULL) count = n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < count; ++i) {
        const int32_t v = verts ? verts[i] : (int32_t)i;
        const double xv = pos[2 * (int64_t)v], yv = pos[2 * (int64_t)v + 1];
        double s = 0.0;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t u = col_idx[e];
            const double dx = pos[2 * (int64_t)u] - xv, dy = pos[2 * (int64_t)u + 1] - yv;
            const double delta = sqrt(dx * dx + dy * dy);
            if (delta > 0.0) s += pow(delta, (double)p) / d;
        }
        for (int64_t j = kptr[i]; j < kptr[i + 1]; ++j) {
            const int32_t u = kidx[j];
            const double dx = xv - pos[2 * (int64_t)u], dy = yv - pos[2 * (int64_t)u + 1];
            const double delta = sqrt(dx * dx + dy * dy);
            if (delta > 0.0) s += (mass ? mass[u] : 1.0) * (d * d / pow(delta, (double)q));
        }
        S[i] = s;
    }
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
             const int64_t* kptr, const int32_t* kidx, double d, const double* mass, int32_t p,
             int32_t q, double t, double stop_displacement, double* pos, double* F, double* D,
             orc_iter_stats* st) {
    int64_t coincident = 0;
    int rc = orc_forces(n, row_ptr, col_idx, n, NULL, kptr, kidx, d, mass, p, q, pos, F,
                        &coincident);
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
               const int64_t* kptr, const int32_t* kidx, double d, const double* mass, int32_t p,
               int32_t q, const double* temperature, int32_t h0, int32_t h_end,
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
        rc = orc_step(n, row_ptr, col_idx, kptr, kidx, d, mass, p, q, temperature[h],
                      stop_displacement, pos, F, D, &st);
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
/* Pruning and reinsertion of degree-one vertices (Sections 4.3, 4.6)  */
/* ------------------------------------------------------------------ */

/* Marks the pruned vertices: a degree-one vertex v with neighbour w is
 * pruned unless w has degree one too and w > v.  anchor[v] = w for a pruned
 * v (else -1); leaves[w] counts the vertices pruned from w.  new_id[v] is v's
 * id in the pruned graph (kept vertices in ascending original id; -1 for
 * pruned ones).  Returns the number of kept vertices in *n_kept and the
 * pruned graph's adjacency entries in *nnz_kept. */
int orc_prune(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* anchor,
              int32_t* leaves, int32_t* new_id, int32_t* n_kept, int64_t* nnz_kept) {
    if (n < 0) return ORC_EINVAL;
    for (int32_t v = 0; v < n; ++v) {
        anchor[v] = -1;
        leaves[v] = 0;
    }
    for (int32_t v = 0; v < n; ++v) {
        if (row_ptr[v + 1] - row_ptr[v] != 1) continue;
        const int32_t w = col_idx[row_ptr[v]];
        const int64_t degw = row_ptr[w + 1] - row_ptr[w];
        if (degw > 1 || w < v) anchor[v] = w;
    }
    int32_t kept = 0;
    int64_t nnz = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (anchor[v] >= 0) {
            leaves[anchor[v]] += 1;
            new_id[v] = -1;
        } else {
            new_id[v] = kept++;
        }
    }
    for (int32_t v = 0; v < n; ++v) {
        if (anchor[v] >= 0) continue;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) nnz += anchor[col_idx[e]] < 0;
    }
    *n_kept = kept;
    *nnz_kept = nnz;
    return ORC_OK;
}

/* The pruned graph's CSR (kept vertices renumbered by new_id; rows stay
 * ascending because the renumbering keeps the order). */
int orc_pruned_graph(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
                     const int32_t* new_id, int64_t* rp_out, int32_t* ci_out) {
    int64_t o = 0;
    int32_t r = 0;
    rp_out[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (new_id[v] < 0) continue;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t u = new_id[col_idx[e]];
            if (u >= 0) ci_out[o++] = u;
        }
        rp_out[++r] = o;
    }
    return ORC_OK;
}

static int cmp_f64(const void* a, const void* b) {
    const double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* Reinsertion (Section 4.6).  pos_kept [n_kept][2] is the drawing of the
 * pruned graph (rp_k, ci_k); pos_all [n][2] receives every vertex: kept ones
 * copied, the leaves of kept vertex v (original ids in ascending order) on
 * the circle of radius rho = 0.2 * (shortest edge incident to v in the pruned
 * drawing; d if it has none) at angles phi + 2 pi j / L.  phi is the middle
 * of the widest gap between the incident edges' angles taken modulo 2 pi / L
 * (the first widest gap in ascending order; phi = 0 without incident edges),
 * so every leaf is as far as possible in angle from the incident edges. */
int orc_reinsert(int32_t n, const int32_t* anchor, const int32_t* leaves, const int32_t* new_id,
                 int32_t n_kept, const int64_t* rp_k, const int32_t* ci_k, double d,
                 const double* pos_kept, double* pos_all) {
    const double two_pi = 6.283185307179586476925286766559;
    int32_t* kept_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_kept > 0 ? n_kept : 1));
    int32_t* next_j = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    double* phi = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* rho = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!kept_of || !next_j || !phi || !rho) {
        free(kept_of);
        free(next_j);
        free(phi);
        free(rho);
        return ORC_ENOMEM;
    }
    for (int32_t v = 0; v < n; ++v)
        if (new_id[v] >= 0) kept_of[new_id[v]] = v;
    for (int32_t i = 0; i < n_kept; ++i) {
        const int32_t v = kept_of[i];
        pos_all[2 * (int64_t)v] = pos_kept[2 * (int64_t)i];
        pos_all[2 * (int64_t)v + 1] = pos_kept[2 * (int64_t)i + 1];
        const int32_t L = leaves[v];
        if (L == 0) continue;
        const double xv = pos_kept[2 * (int64_t)i], yv = pos_kept[2 * (int64_t)i + 1];
        const int64_t deg = rp_k[i + 1] - rp_k[i];
        const double period = two_pi / (double)L;
        double shortest = -1.0;
        double* res = (double*)malloc(sizeof(double) * (size_t)(deg > 0 ? deg : 1));
        if (!res) {
            free(kept_of);
            free(next_j);
            free(phi);
            free(rho);
            return ORC_ENOMEM;
        }
        for (int64_t e = 0; e < deg; ++e) {
            const int32_t u = ci_k[rp_k[i] + e];
            const double dx = pos_kept[2 * (int64_t)u] - xv, dy = pos_kept[2 * (int64_t)u + 1] - yv;
            const double len = sqrt(dx * dx + dy * dy);
            if (shortest < 0.0 || len < shortest) shortest = len;
            double a = atan2(dy, dx);
            if (a < 0.0) a += two_pi;
            double r = fmod(a, period);
            if (r < 0.0) r += period;
            if (r >= period) r -= period;
            res[e] = r;
        }
        double best = 0.0;
        if (deg > 0) {
            qsort(res, (size_t)deg, sizeof(double), cmp_f64);
            double widest = -1.0;
            for (int64_t e = 0; e < deg; ++e) {
                const double lo = res[e];
                const double hi = e + 1 < deg ? res[e + 1] : res[0] + period;
                if (hi - lo > widest) {
                    widest = hi - lo;
                    best = lo + 0.5 * (hi - lo);
                }
            }
            if (best >= period) best -= period;
        }
        free(res);
        phi[v] = best;
        rho[v] = 0.2 * (deg > 0 ? shortest : d);
    }
    for (int32_t u = 0; u < n; ++u) {
        const int32_t v = anchor[u];
        if (v < 0) continue;
        const int32_t j = next_j[v]++;
        const double theta = phi[v] + two_pi * (double)j / (double)leaves[v];
        const int32_t i = new_id[v];
        pos_all[2 * (int64_t)u] = pos_kept[2 * (int64_t)i] + rho[v] * cos(theta);
        pos_all[2 * (int64_t)u + 1] = pos_kept[2 * (int64_t)i + 1] + rho[v] * sin(theta);
    }
    free(kept_of);
    free(next_j);
    free(phi);
    free(rho);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Connected components and packing (Section 4.6)                      */
/* ------------------------------------------------------------------ */

/* label[v] = the smallest vertex id of v's connected component (a BFS from
 * every unlabelled vertex in ascending order).  *count_out = number of
 * components. */
int orc_components(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* label,
                   int32_t* count_out) {
    if (n < 0) return ORC_EINVAL;
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) return ORC_ENOMEM;
    for (int32_t v = 0; v < n; ++v) label[v] = -1;
    int32_t count = 0;
    for (int32_t s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        ++count;
        int32_t head = 0, tail = 0;
        label[s] = s;
        queue[tail++] = s;
        while (head < tail) {
            const int32_t v = queue[head++];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                const int32_t u = col_idx[e];
                if (label[u] < 0) {
                    label[u] = s;
                    queue[tail++] = u;
                }
            }
        }
    }
    free(queue);
    *count_out = count;
    return ORC_OK;
}

typedef struct {
    int32_t label, size;
    double minx, miny, maxx, maxy;
} orc_comp;

static int cmp_comp(const void* a, const void* b) {
    const orc_comp* x = (const orc_comp*)a;
    const orc_comp* y = (const orc_comp*)b;
    if (x->size != y->size) return x->size > y->size ? -1 : 1;  /* larger first */
    return (x->label > y->label) - (x->label < y->label);      /* then smaller label */
}

/* Packing of the components' drawings in a matrix (Section 4.6).  Components
 * in order of decreasing vertex count (ties: smaller label first) fill a
 * matrix of ceil(sqrt(C)) columns row by row.  Column c is as wide as the
 * widest bounding box in it, row r as tall as the tallest; consecutive
 * columns and rows are `gap` apart, the first cell's corner is the origin, and
 * each drawing is translated so that its bounding box's lower-left corner is
 * its cell's lower-left corner.  pos [n][2] is changed in place. */
int orc_pack(int32_t n, const int32_t* label, double gap, double* pos) {
    if (n < 0 || !(gap >= 0.0)) return ORC_EINVAL;
    if (n == 0) return ORC_OK;
    int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);  /* root -> component index */
    int32_t C = 0;
    for (int32_t v = 0; v < n; ++v) C += label[v] == v;
    orc_comp* comp = (orc_comp*)malloc(sizeof(orc_comp) * (size_t)C);
    int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
    if (!slot || !comp || !rank) {
        free(slot);
        free(comp);
        free(rank);
        return ORC_ENOMEM;
    }
    int32_t c = 0;
    for (int32_t v = 0; v < n; ++v)
        if (label[v] == v) {
            slot[v] = c;
            comp[c].label = v;
            comp[c].size = 0;
            comp[c].minx = comp[c].miny = INFINITY;
            comp[c].maxx = comp[c].maxy = -INFINITY;
            ++c;
        }
    for (int32_t v = 0; v < n; ++v) {
        orc_comp* k = &comp[slot[label[v]]];
        const double x = pos[2 * (int64_t)v], y = pos[2 * (int64_t)v + 1];
        k->size += 1;
        if (x < k->minx) k->minx = x;
        if (x > k->maxx) k->maxx = x;
        if (y < k->miny) k->miny = y;
        if (y > k->maxy) k->maxy = y;
    }
    qsort(comp, (size_t)C, sizeof(orc_comp), cmp_comp);
    for (int32_t r = 0; r < C; ++r) slot[comp[r].label] = r;  /* root -> rank */
    int32_t cols = 1;
    while ((int64_t)cols * cols < C) ++cols;
    const int32_t rows = (C + cols - 1) / cols;
    double* colx = (double*)calloc((size_t)cols + 1, sizeof(double));
    double* rowy = (double*)calloc((size_t)rows + 1, sizeof(double));
    double* colw = (double*)calloc((size_t)cols, sizeof(double));
    double* rowh = (double*)calloc((size_t)rows, sizeof(double));
    if (!colx || !rowy || !colw || !rowh) {
        free(slot);
        free(comp);
        free(rank);
        free(colx);
        free(rowy);
        free(colw);
        free(rowh);
        return ORC_ENOMEM;
    }
    for (int32_t r = 0; r < C; ++r) {
        const double w = comp[r].maxx - comp[r].minx, h = comp[r].maxy - comp[r].miny;
        if (w > colw[r % cols]) colw[r % cols] = w;
        if (h > rowh[r / cols]) rowh[r / cols] = h;
    }
    for (int32_t j = 0; j < cols; ++j) colx[j + 1] = colx[j] + colw[j] + gap;
    for (int32_t j = 0; j < rows; ++j) rowy[j + 1] = rowy[j] + rowh[j] + gap;
    for (int32_t v = 0; v < n; ++v) {
        const int32_t r = slot[label[v]];
        pos[2 * (int64_t)v] += colx[r % cols] - comp[r].minx;
        pos[2 * (int64_t)v + 1] += rowy[r / cols] - comp[r].miny;
    }
    free(slot);
    free(comp);
    free(rank);
    free(colx);
    free(rowy);
    free(colw);
    free(rowh);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Drawing-quality metrics (Section 5.2: crossings, edge length        */
/* deviation, similarity of the drawing's Gabriel graph to the graph)   */
/* ------------------------------------------------------------------ */

/* Exact sign of a sum of doubles.  two_sum splits a + b into its rounded
 * sum and the rounding error, both exact doubles (Knuth's algorithm).
 * Adding the terms one by one into a list of such pieces, each new term
 * passed through the list with two_sum, keeps the list's sum equal to the
 * exact sum and leaves the pieces nonoverlapping in increasing magnitude
 * (Shewchuk's expansion growth), so the sign of the sum is the sign of the
 * last nonzero piece. */
static void two_sum(double a, double b, double* s, double* e) {
    const double x = a + b;
    const double bv = x - a;
    const double av = x - bv;
    *s = x;
    *e = (a - av) + (b - bv);
}

static int exact_sign(const double* term, int k) {
    double piece[16];
    int len = 0;
    for (int i = 0; i < k; ++i) {
        double q = term[i];
        for (int j = 0; j < len; ++j) {
            double s, e;
            two_sum(q, piece[j], &s, &e);
            piece[j] = e;
            q = s;
        }
        piece[len++] = q;
    }
    for (int j = len - 1; j >= 0; --j)
        if (piece[j] != 0.0) return piece[j] > 0.0 ? 1 : -1;
    return 0;
}

/* Sign of the orientation of (a, b, c): > 0 counter-clockwise.  The
 * determinant (b - a) x (c - a) is multiplied out into eight products of
 * coordinates; coordinates are single-precision values, so each product is
 * exact in double, and the sign of their sum is taken exactly. */
static int orient(const double* a, const double* b, const double* c) {
    const double t[8] = {b[0] * c[1], -(b[0] * a[1]), -(a[0] * c[1]), a[0] * a[1],
                         -(b[1] * c[0]), b[1] * a[0], a[1] * c[0], -(a[1] * a[0])};
    return exact_sign(t, 8);
}

/* Edges {u, v} (u < v) in row order: edge e is the e-th pair met when rows
 * are read in ascending v and each row keeps its entries u > v. */
static int64_t edge_list(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* eu,
                         int32_t* ev) {
    int64_t m = 0;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (col_idx[e] > v) {
                if (eu) {
                    eu[m] = v;
                    ev[m] = col_idx[e];
                }
                ++m;
            }
    return m;
}

/* Two edges cross when they share no end vertex and each one's ends lie
 * strictly on opposite sides of the other's line (touching, overlapping
 * collinear edges and shared ends do not count). */
static int edges_cross(const double* pos, int32_t a, int32_t b, int32_t c, int32_t d) {
    if (a == c || a == d || b == c || b == d) return 0;
    const double *pa = pos + 2 * (int64_t)a, *pb = pos + 2 * (int64_t)b;
    const double *pc = pos + 2 * (int64_t)c, *pd = pos + 2 * (int64_t)d;
    return orient(pa, pb, pc) * orient(pa, pb, pd) < 0 && orient(pc, pd, pa) * orient(pc, pd, pb) < 0;
}

/* Crossings of the drawing: per_edge[e] (may be NULL) = number of edges
 * crossing edge e; *total = number of crossing pairs. */
int orc_crossings(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* pos,
                  int64_t* per_edge, int64_t* total) {
    if (n < 0) return ORC_EINVAL;
    const int64_t m = edge_list(n, row_ptr, col_idx, NULL, NULL);
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!eu || !ev) {
        free(eu);
        free(ev);
        return ORC_ENOMEM;
    }
    edge_list(n, row_ptr, col_idx, eu, ev);
    int64_t sum = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : sum)
    for (int64_t i = 0; i < m; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < m; ++j)
            if (j != i) c += edges_cross(pos, eu[i], ev[i], eu[j], ev[j]);
        if (per_edge) per_edge[i] = c;
        sum += c;
    }
    *total = sum / 2;
    free(eu);
    free(ev);
    return ORC_OK;
}

/* Crossings of the edges sel[0..count) (indices into the edge list) with
 * every edge. */
int orc_edge_crossings(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
                       const double* pos, int64_t count, const int64_t* sel, int64_t* out) {
    const int64_t m = edge_list(n, row_ptr, col_idx, NULL, NULL);
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!eu || !ev) {
        free(eu);
        free(ev);
        return ORC_ENOMEM;
    }
    /* every index is checked before any thread starts, so no thread writes
     * shared state */
    for (int64_t k = 0; k < count; ++k)
        if (sel[k] < 0 || sel[k] >= m) {
            free(eu);
            free(ev);
            return ORC_EINVAL;
        }
    edge_list(n, row_ptr, col_idx, eu, ev);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < count; ++k) {
        const int64_t i = sel[k];
        int64_t c = 0;
        for (int64_t j = 0; j < m; ++j)
            if (j != i) c += edges_cross(pos, eu[i], ev[i], eu[j], ev[j]);
        out[k] = c;
    }
    free(eu);
    free(ev);
    return ORC_OK;
}

/* Mean and standard deviation (population, two passes) of the edge lengths. */
int orc_edge_lengths(int32_t n, const int64_t* row_ptr, const int32_t* col_idx,
                     const double* pos, double* mean, double* stdev) {
    double s = 0.0;
    int64_t m = 0;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t u = col_idx[e];
            if (u <= v) continue;
            const double dx = pos[2 * (int64_t)u] - pos[2 * (int64_t)v];
            const double dy = pos[2 * (int64_t)u + 1] - pos[2 * (int64_t)v + 1];
            s += sqrt(dx * dx + dy * dy);
            ++m;
        }
    if (m == 0) {
        *mean = 0.0;
        *stdev = 0.0;
        return ORC_OK;
    }
    const double mu = s / (double)m;
    double q = 0.0;
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t u = col_idx[e];
            if (u <= v) continue;
            const double dx = pos[2 * (int64_t)u] - pos[2 * (int64_t)v];
            const double dy = pos[2 * (int64_t)u + 1] - pos[2 * (int64_t)v + 1];
            const double z = sqrt(dx * dx + dy * dy) - mu;
            q += z * z;
        }
    *mean = mu;
    *stdev = sqrt(q / (double)m);
    return ORC_OK;
}

/* Gabriel graph of the points (brute force): u and v are adjacent when no
 * other point lies in the closed disc with diameter uv, i.e. when
 * (w - u).(w - v) > 0 for every other w.  deg[u] = Gabriel degree; with
 * adj != NULL also the rows (ascending; adj_ptr [n+1] as computed by a
 * first call with adj == NULL). */
static int gabriel_pair(int32_t n, const double* pos, int32_t u, int32_t v) {
    const double ux = pos[2 * (int64_t)u], uy = pos[2 * (int64_t)u + 1];
    const double vx = pos[2 * (int64_t)v], vy = pos[2 * (int64_t)v + 1];
    for (int32_t w = 0; w < n; ++w) {
        if (w == u || w == v) continue;
        const double wx = pos[2 * (int64_t)w], wy = pos[2 * (int64_t)w + 1];
        /* (w - u).(w - v) multiplied out; exact sign as in orient() */
        const double t[8] = {wx * wx, -(wx * vx), -(ux * wx), ux * vx,
                             wy * wy, -(wy * vy), -(uy * wy), uy * vy};
        if (exact_sign(t, 8) <= 0) return 0;
    }
    return 1;
}

int orc_gabriel(int32_t n, const double* pos, int64_t* adj_ptr, int32_t* adj) {
    if (n < 0) return ORC_EINVAL;
    if (!adj) {
        adj_ptr[0] = 0;
        int64_t* cnt = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
        if (!cnt) return ORC_ENOMEM;
#pragma omp parallel for schedule(dynamic, 4)
        for (int32_t u = 0; u < n; ++u)
            for (int32_t v = 0; v < n; ++v)
                if (v != u && gabriel_pair(n, pos, u, v)) cnt[u] += 1;
        for (int32_t u = 0; u < n; ++u) adj_ptr[u + 1] = adj_ptr[u] + cnt[u];
        free(cnt);
        return ORC_OK;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t u = 0; u < n; ++u) {
        int64_t o = adj_ptr[u];
        for (int32_t v = 0; v < n; ++v)
            if (v != u && gabriel_pair(n, pos, u, v)) adj[o++] = v;
    }
    return ORC_OK;
}

/* Similarity (Section 5.2): for every vertex the Jaccard index of its
 * neighbourhood in the graph and in the Gabriel graph, |A n B| / |A u B|
 * (1 when both are empty), averaged over the vertices; per_vertex (may be
 * NULL) receives the indices.  Both row sets ascending. */
int orc_jaccard(int32_t n, const int64_t* row_ptr, const int32_t* col_idx, const int64_t* gg_ptr,
                const int32_t* gg, double* per_vertex, double* mean) {
    double s = 0.0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t i = row_ptr[v], j = gg_ptr[v], both = 0;
        while (i < row_ptr[v + 1] && j < gg_ptr[v + 1]) {
            if (col_idx[i] == gg[j]) {
                ++both;
                ++i;
                ++j;
            } else if (col_idx[i] < gg[j]) {
                ++i;
            } else {
                ++j;
            }
        }
        const int64_t uni = (row_ptr[v + 1] - row_ptr[v]) + (gg_ptr[v + 1] - gg_ptr[v]) - both;
        const double J = uni == 0 ? 1.0 : (double)both / (double)uni;
        if (per_vertex) per_vertex[v] = J;
        s += J;
    }
    *mean = n > 0 ? s / (double)n : 1.0;
    return ORC_OK;
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

/* Threads of later parallel loops (results never depend on it: threads
 * split vertices, never a sum). */
void orc_set_threads(int32_t t) {
#ifdef _OPENMP
    omp_set_num_threads(t > 0 ? t : 1);
#else
    (void)t;
#endif
}

/*
 * Drives every entry point of the oracle (oracle/oracle.c) on small graphs so
 * that the test suite can run it under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every buffer is allocated at its exact size, and
 * the graphs include isolated vertices, leaves, coincident points and
 * components of one and two vertices.  Values are pinned by the Python tests;
 * this program checks memory and arithmetic safety and the return codes.
 * Prints "OK <calls>" and exits 0, or the first failing call and exits 1.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t moved;
    double max_disp;
    double energy;
    int64_t coincident;
} orc_iter_stats;

int orc_khop_count(int32_t, const int64_t*, const int32_t*, int32_t, int64_t, const int32_t*,
                   int64_t*);
int orc_khop_fill(int32_t, const int64_t*, const int32_t*, int32_t, int64_t, const int32_t*,
                  const int64_t*, int32_t*);
int orc_forces(int32_t, const int64_t*, const int32_t*, int64_t, const int32_t*, const int64_t*,
               const int32_t*, double, const double*, int32_t, int32_t, const double*, double*,
               int64_t*);
int orc_force_magnitudes(int32_t, const int64_t*, const int32_t*, int64_t, const int32_t*,
                         const int64_t*, const int32_t*, double, const double*, int32_t, int32_t,
                         const double*, double*);
int orc_cap(int64_t, const double*, double, double*);
int orc_step(int32_t, const int64_t*, const int32_t*, const int64_t*, const int32_t*, double,
             const double*, int32_t, int32_t, double, double, double*, double*, double*,
             orc_iter_stats*);
int orc_layout(int32_t, const int64_t*, const int32_t*, const int64_t*, const int32_t*, double,
               const double*, int32_t, int32_t, const double*, int32_t, int32_t, double, double,
               double*, int32_t*, orc_iter_stats*);
int orc_prune(int32_t, const int64_t*, const int32_t*, int32_t*, int32_t*, int32_t*, int32_t*,
              int64_t*);
int orc_pruned_graph(int32_t, const int64_t*, const int32_t*, const int32_t*, int64_t*, int32_t*);
int orc_reinsert(int32_t, const int32_t*, const int32_t*, const int32_t*, int32_t, const int64_t*,
                 const int32_t*, double, const double*, double*);
int orc_components(int32_t, const int64_t*, const int32_t*, int32_t*, int32_t*);
int orc_pack(int32_t, const int32_t*, double, double*);
int orc_crossings(int32_t, const int64_t*, const int32_t*, const double*, int64_t*, int64_t*);
int orc_edge_crossings(int32_t, const int64_t*, const int32_t*, const double*, int64_t,
                       const int64_t*, int64_t*);
int orc_edge_lengths(int32_t, const int64_t*, const int32_t*, const double*, double*, double*);
int orc_gabriel(int32_t, const double*, int64_t*, int32_t*);
int orc_jaccard(int32_t, const int64_t*, const int32_t*, const int64_t*, const int32_t*, double*,
                double*);
void orc_paper_schedule(double, double, double, int32_t, double*);
void orc_linear_schedule(double, int32_t, double*);

static int g_calls = 0;
#define CALL(expr)                                                            \
    do {                                                                      \
        ++g_calls;                                                            \
        int rc_ = (expr);                                                     \
        if (rc_ != 0) {                                                       \
            printf("FAIL %s:%d: %s returned %d\n", __FILE__, __LINE__, #expr, rc_); \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

static void* xmalloc(size_t bytes) {
    void* p = malloc(bytes ? bytes : 1);
    if (!p) {
        printf("FAIL out of memory\n");
        exit(1);
    }
    return p;
}

typedef struct {
    int32_t n;
    int64_t nnz;
    int64_t* rp;
    int32_t* ci;
} graph;

static uint64_t g_state = 88172645463325252ull;
static uint64_t next_u64(void) { /* xorshift64 */
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return g_state;
}

/* simple undirected graph from an edge list (duplicates and loops dropped) */
static graph make_graph(int32_t n, int m, const int32_t* eu, const int32_t* ev) {
    char* adj = (char*)calloc((size_t)n * (size_t)(n > 0 ? n : 1), 1);
    for (int i = 0; i < m; ++i)
        if (eu[i] != ev[i]) {
            adj[(size_t)eu[i] * n + ev[i]] = 1;
            adj[(size_t)ev[i] * n + eu[i]] = 1;
        }
    graph g;
    g.n = n;
    g.rp = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    g.rp[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t c = 0;
        for (int32_t u = 0; u < n; ++u) c += adj[(size_t)v * n + u];
        g.rp[v + 1] = g.rp[v] + c;
    }
    g.nnz = g.rp[n];
    g.ci = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)g.nnz);
    int64_t o = 0;
    for (int32_t v = 0; v < n; ++v)
        for (int32_t u = 0; u < n; ++u)
            if (adj[(size_t)v * n + u]) g.ci[o++] = u;
    free(adj);
    return g;
}

static void exercise(const graph* g, int k, int coincide) {
    const int32_t n = g->n;
    double* pos = (double*)xmalloc(sizeof(double) * 2 * (size_t)n);
    for (int32_t i = 0; i < 2 * n; ++i) pos[i] = (double)(next_u64() % 100000) * 1e-3;
    if (coincide && n > 3) {
        pos[2] = pos[0];
        pos[3] = pos[1];
    }
    /* k-neighbourhoods, all vertices and a subset */
    int64_t* sizes = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)n);
    CALL(orc_khop_count(n, g->rp, g->ci, k, n, NULL, sizes));
    int64_t* kptr = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    kptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) kptr[v + 1] = kptr[v] + sizes[v];
    int32_t* kidx = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)kptr[n]);
    CALL(orc_khop_fill(n, g->rp, g->ci, k, n, NULL, kptr, kidx));
    /* a subset of rows (vertices 0, n - 1, n / 2; none for an empty graph) */
    const int64_t ns = n > 0 ? 3 : 0;
    int32_t sub[3] = {0, n > 0 ? n - 1 : 0, n / 2};
    int64_t ssz[3] = {0, 0, 0}, sptr[4] = {0, 0, 0, 0};
    CALL(orc_khop_count(n, g->rp, g->ci, k, ns, ns ? sub : NULL, ssz));
    for (int i = 0; i < ns; ++i) sptr[i + 1] = sptr[i] + ssz[i];
    int32_t* sidx = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)sptr[ns]);
    if (ns) CALL(orc_khop_fill(n, g->rp, g->ci, k, ns, sub, sptr, sidx));
    /* forces, magnitudes, cap, step, layout (several force laws, weights) */
    double* F = (double*)xmalloc(sizeof(double) * 2 * (size_t)n);
    double* D = (double*)xmalloc(sizeof(double) * 2 * (size_t)n);
    double* S = (double*)xmalloc(sizeof(double) * (size_t)n);
    double* mass = (double*)xmalloc(sizeof(double) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) mass[v] = 1.0 + (double)(v % 3);
    int64_t coinc = 0;
    const int32_t models[4][2] = {{2, 1}, {0, 1}, {4, 5}, {1, 0}};
    for (int m = 0; m < 4; ++m) {
        CALL(orc_forces(n, g->rp, g->ci, n, NULL, kptr, kidx, 20.0, m % 2 ? mass : NULL,
                        models[m][0], models[m][1], pos, F, &coinc));
        CALL(orc_force_magnitudes(n, g->rp, g->ci, n, NULL, kptr, kidx, 20.0, m % 2 ? mass : NULL,
                                  models[m][0], models[m][1], pos, S));
    }
    if (ns) CALL(orc_forces(n, g->rp, g->ci, ns, sub, sptr, sidx, 20.0, NULL, 2, 1, pos, F, &coinc));
    CALL(orc_cap(n, F, 3.0, D));
    orc_iter_stats st;
    double* x = (double*)xmalloc(sizeof(double) * 2 * (size_t)n);
    memcpy(x, pos, sizeof(double) * 2 * (size_t)n);
    CALL(orc_step(n, g->rp, g->ci, kptr, kidx, 20.0, NULL, 2, 1, 5.0, 0.01, x, F, D, &st));
    double temps[6];
    orc_paper_schedule((double)(n > 0 ? n : 1), 1.0, 20.0, 6, temps);
    orc_linear_schedule(10.0, 6, temps);
    int32_t run = 0;
    CALL(orc_layout(n, g->rp, g->ci, kptr, kidx, 20.0, mass, 2, 1, temps, 0, 6, 0.15, 0.01, x,
                    &run, &st));
    /* pruning and reinsertion */
    int32_t* anchor = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t* leaves = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t* new_id = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t nk = 0;
    int64_t nnzk = 0;
    CALL(orc_prune(n, g->rp, g->ci, anchor, leaves, new_id, &nk, &nnzk));
    int64_t* rpk = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(nk + 1));
    int32_t* cik = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)nnzk);
    CALL(orc_pruned_graph(n, g->rp, g->ci, new_id, rpk, cik));
    double* xk = (double*)xmalloc(sizeof(double) * 2 * (size_t)nk);
    for (int32_t v = 0; v < n; ++v)
        if (new_id[v] >= 0) {
            xk[2 * new_id[v]] = pos[2 * v];
            xk[2 * new_id[v] + 1] = pos[2 * v + 1];
        }
    CALL(orc_reinsert(n, anchor, leaves, new_id, nk, rpk, cik, 20.0, xk, x));
    /* components and packing */
    int32_t* label = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t ncomp = 0;
    CALL(orc_components(n, g->rp, g->ci, label, &ncomp));
    memcpy(x, pos, sizeof(double) * 2 * (size_t)n);
    CALL(orc_pack(n, label, 5.0, x));
    /* drawing metrics on single-precision coordinates */
    double* xs = (double*)xmalloc(sizeof(double) * 2 * (size_t)n);
    for (int32_t i = 0; i < 2 * n; ++i) xs[i] = (double)(float)pos[i];
    const int64_t m = g->nnz / 2;
    int64_t* per_edge = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)m);
    int64_t total = 0;
    CALL(orc_crossings(n, g->rp, g->ci, xs, per_edge, &total));
    CALL(orc_crossings(n, g->rp, g->ci, xs, NULL, &total));
    if (m > 0) {
        int64_t sel[2] = {0, m - 1}, out[2];
        CALL(orc_edge_crossings(n, g->rp, g->ci, xs, 2, sel, out));
        int64_t bad[1] = {m};
        ++g_calls;
        if (orc_edge_crossings(n, g->rp, g->ci, xs, 1, bad, out) == 0) {
            printf("FAIL an edge index out of range was accepted\n");
            exit(1);
        }
    }
    double mean = 0.0, sd = 0.0;
    CALL(orc_edge_lengths(n, g->rp, g->ci, xs, &mean, &sd));
    int64_t* gp = (int64_t*)xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    CALL(orc_gabriel(n, xs, gp, NULL));
    int32_t* gi = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)gp[n]);
    CALL(orc_gabriel(n, xs, gp, gi));
    double* jac = (double*)xmalloc(sizeof(double) * (size_t)n);
    CALL(orc_jaccard(n, g->rp, g->ci, gp, gi, jac, &mean));
    free(pos); free(sizes); free(kptr); free(kidx); free(sidx); free(F); free(D); free(S);
    free(mass); free(x); free(anchor); free(leaves); free(new_id); free(rpk); free(cik);
    free(xk); free(label); free(xs); free(per_edge); free(gp); free(gi); free(jac);
}

int main(void) {
    /* a path, a star with an isolated edge and isolated vertices, a grid, a
     * random graph with several components */
    int32_t eu[400], ev[400];
    int m = 0;
    for (int i = 0; i + 1 < 7; ++i, ++m) {
        eu[m] = i;
        ev[m] = i + 1;
    }
    graph path = make_graph(7, m, eu, ev);
    m = 0;
    for (int i = 1; i < 8; ++i, ++m) {
        eu[m] = 0;
        ev[m] = i;
    }
    eu[m] = 9;
    ev[m] = 10;
    ++m;
    graph star = make_graph(13, m, eu, ev);
    m = 0;
    for (int r = 0; r < 5; ++r)
        for (int c = 0; c < 4; ++c) {
            if (c + 1 < 4) {
                eu[m] = r * 4 + c;
                ev[m++] = r * 4 + c + 1;
            }
            if (r + 1 < 5) {
                eu[m] = r * 4 + c;
                ev[m++] = (r + 1) * 4 + c;
            }
        }
    graph grid = make_graph(20, m, eu, ev);
    m = 0;
    for (int i = 0; i < 150; ++i, ++m) {
        eu[m] = (int32_t)(next_u64() % 60);
        ev[m] = (int32_t)(next_u64() % 60);
    }
    graph rnd = make_graph(60, m, eu, ev);
    graph empty = make_graph(0, 0, eu, ev);
    const graph* all[5] = {&path, &star, &grid, &rnd, &empty};
    for (int gi = 0; gi < 5; ++gi)
        for (int k = 1; k <= 3; ++k) exercise(all[gi], k, gi % 2);
    for (int gi = 0; gi < 5; ++gi) {
        free(all[gi]->rp);
        free(all[gi]->ci);
    }
    printf("OK %d\n", g_calls);
    return 0;
}

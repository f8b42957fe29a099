// Degree-one vertices: pruned before the layout, reinserted after it.
//
// Pruning (Section 4.3): a vertex of degree one is removed, unless its only
// neighbour also has degree one and a larger id (one end of every isolated
// edge stays).  Each kept vertex records how many vertices were pruned from
// it; the layout of the pruned graph weights the repulsion a kept vertex
// exerts by 1 + that number (Section 4.6), so that the disc its leaves will
// occupy stays clear.  Kept vertices are renumbered in ascending original id.
//
// Reinsertion (Section 4.6): the L leaves of a kept vertex v go on the circle
// of radius 0.2 x (v's shortest incident edge in the drawing of the pruned
// graph; 0.2 x d when v has no edge left), in ascending original id at angles
// phi + 2 pi j / L.  phi is the middle of the widest gap between the angles of
// v's incident edges taken modulo 2 pi / L (the first widest, in ascending
// order), which keeps every leaf as far as possible in angle from the edges.
//
// Everything runs on the device:
//   prune_mark_kernel     thread per vertex: the pruning rule, leaf counts
//   kept_kernel           thread per vertex: new ids, original id of each kept one
//   kept_rows_kernel      wave per kept vertex: pruned-graph degree (count
//                         pass), then its row and its leaves in ascending id
//                         (fill pass), compacted with ballots
//   anchor_kernel         thread per kept vertex: weights, leaf counts, the
//                         list of vertices that have leaves
//   reinsert_*_kernel     workgroup per vertex with leaves: residues of the
//                         edge angles, the first widest gap between them, and
//                         the leaves' positions.  Rows of up to 256 edges: one
//                         wavefront sorts them in LDS; longer rows: 512
//                         threads bin them into 2 deg buckets (no sort)
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_util.h"
#include "gila_internal.h"

struct gila_pruned {
    int device = 0;
    int32_t n = 0, n_kept = 0, n_pruned = 0, n_anchor = 0;
    int32_t n_class[2] = {0, 0};    // vertices with leaves: short rows, long rows
    int64_t nnz = 0, nnz_kept = 0;
    int64_t max_anchor_deg = 0;     // longest pruned-graph row of a vertex with leaves
    int32_t* anchor = nullptr;      // [n] neighbour a pruned vertex hangs from, -1 if kept
    int32_t* leaves = nullptr;      // [n] vertices pruned from each vertex
    int32_t* new_id = nullptr;      // [n] id in the pruned graph, -1 if pruned
    int32_t* kept_of = nullptr;     // [n_kept] original id of each kept vertex
    int64_t* rp = nullptr;          // [n_kept + 1] pruned graph
    int32_t* ci = nullptr;          // [nnz_kept]
    double* mass = nullptr;         // [n_kept] 1 + leaves, pruned ids
    int64_t* leaf_ptr = nullptr;    // [n_kept + 1] leaves of kept vertex i ...
    int32_t* leaf_ids = nullptr;    // [n_pruned] ... in ascending original id
    int32_t* anchors = nullptr;     // [n_anchor] pruned ids of the vertices with leaves,
                                    // grouped by row-length class
    int64_t device_bytes = 0;
};

namespace gila {

// Reinsertion: rows of at most kShortRow edges are sorted in LDS by one
// wavefront; longer rows are binned (kLongThreads threads per vertex).
constexpr int kShortRow = 256;
constexpr int kLongThreads = 512;
constexpr int kSortClasses = 2;

__global__ __launch_bounds__(kBlock) void prune_mark_kernel(int32_t n, const int64_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            int32_t* __restrict__ anchor,
                                                            int32_t* __restrict__ leaves) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        int32_t a = -1;
        if (rp[v + 1] - rp[v] == 1) {
            const int32_t w = ci[rp[v]];
            if (rp[w + 1] - rp[w] > 1 || w < v) a = w;
        }
        anchor[v] = a;
        if (a >= 0) atomicAdd(&leaves[a], 1);
    }
}

__global__ __launch_bounds__(kBlock) void keep_flags_kernel(int32_t n, const int32_t* __restrict__ anchor,
                                                            int64_t* __restrict__ flag) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        flag[v] = anchor[v] < 0 ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void kept_kernel(int32_t n, const int32_t* __restrict__ anchor,
                                                      const int64_t* __restrict__ kscan,
                                                      int32_t* __restrict__ new_id,
                                                      int32_t* __restrict__ kept_of) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        if (anchor[v] < 0) {
            const int32_t i = (int32_t)kscan[v];
            new_id[v] = i;
            kept_of[i] = (int32_t)v;
        } else {
            new_id[v] = -1;
        }
    }
}

struct KeptRows {
    int32_t n_kept;
    const int64_t* rp;         // original graph
    const int32_t* ci;
    const int32_t* anchor;
    const int32_t* new_id;
    const int32_t* kept_of;
    int64_t* kdeg;             // count pass: [n_kept] pruned-graph degree
    const int64_t* krp;        // fill pass: pruned-graph rows ...
    int32_t* kci;
    const int64_t* leaf_ptr;   // ... and leaf lists
    int32_t* leaf_ids;
};

// Wave per kept vertex.  The original row is ascending, so the kept
// neighbours (renumbered monotonically) and the leaves come out ascending.
template <bool FILL>
__global__ __launch_bounds__(kBlock) void kept_rows_kernel(KeptRows a) {
    const int lane = lane64();
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    for (int64_t i = (int64_t)blockIdx.x * kWaves + wave_id(); i < a.n_kept; i += waves) {
        const int32_t v = a.kept_of[i];
        const int64_t rb = a.rp[v], re = a.rp[v + 1];
        int64_t kout = FILL ? a.krp[i] : 0;
        int64_t lout = FILL ? a.leaf_ptr[i] : 0;
        for (int64_t e0 = rb; e0 < re; e0 += 64) {
            const int64_t e = e0 + lane;
            int32_t u = -1, nu = -1;
            bool leaf = false;
            if (e < re) {
                u = a.ci[e];
                nu = a.new_id[u];
                leaf = a.anchor[u] == v;
            }
            const uint64_t kb = __ballot(nu >= 0);
            if constexpr (FILL) {
                const uint64_t lb = __ballot(leaf);
                const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                if (nu >= 0) a.kci[kout + __popcll(kb & below)] = nu;
                if (leaf) a.leaf_ids[lout + __popcll(lb & below)] = u;
                lout += __popcll(lb);
            }
            kout += __popcll(kb);
        }
        if (!FILL && lane == 0) a.kdeg[i] = kout;
    }
}

// Weights, leaf counts, and the row-length class of each vertex with leaves
// (-1 without leaves).
__global__ __launch_bounds__(kBlock) void anchor_kernel(int32_t n_kept, const int32_t* __restrict__ kept_of,
                                                        const int32_t* __restrict__ leaves,
                                                        const int64_t* __restrict__ krp,
                                                        double* __restrict__ mass,
                                                        int64_t* __restrict__ lcount,
                                                        int32_t* __restrict__ cls,
                                                        unsigned long long* __restrict__ maxdeg) {
    unsigned long long md = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_kept;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t L = leaves[kept_of[i]];
        const int64_t deg = krp[i + 1] - krp[i];
        mass[i] = 1.0 + (double)L;
        lcount[i] = L;
        int32_t c = -1;
        if (L > 0) {
            c = deg <= kShortRow ? 0 : 1;
            md = (unsigned long long)deg > md ? (unsigned long long)deg : md;
        }
        cls[i] = c;
    }
    md = wave_max(md);
    if (lane64() == 0 && md) atomicMax(maxdeg, md);
}

__global__ __launch_bounds__(kBlock) void class_flag_kernel(int32_t n_kept, const int32_t* __restrict__ cls,
                                                            int32_t c, int64_t* __restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_kept;
         i += (int64_t)gridDim.x * kBlock)
        flag[i] = cls[i] == c ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void anchor_list_kernel(int32_t n_kept, const int32_t* __restrict__ cls,
                                                             int32_t c, const int64_t* __restrict__ scan,
                                                             int64_t offset,
                                                             int32_t* __restrict__ anchors) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_kept;
         i += (int64_t)gridDim.x * kBlock)
        if (cls[i] == c) anchors[offset + scan[i]] = (int32_t)i;
}

// ------------------------------------------------------------------ reinsertion
template <class V>
__global__ __launch_bounds__(kBlock) void copy_kept_kernel(int32_t n_kept,
                                                           const int32_t* __restrict__ kept_of,
                                                           const V* __restrict__ pos_kept,
                                                           V* __restrict__ pos_all) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_kept;
         i += (int64_t)gridDim.x * kBlock)
        pos_all[kept_of[i]] = pos_kept[i];
}

template <class V>
__global__ __launch_bounds__(kBlock) void gather_kept_kernel(int32_t n_kept,
                                                             const int32_t* __restrict__ kept_of,
                                                             const V* __restrict__ pos_all,
                                                             V* __restrict__ pos_kept) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_kept;
         i += (int64_t)gridDim.x * kBlock)
        pos_kept[i] = pos_all[kept_of[i]];
}

struct ReinsertArgs {
    int32_t n_anchor;          // vertices of `anchors` this launch handles
    const int32_t* anchors;
    const int32_t* kept_of;
    const int32_t* leaves;
    const int64_t* rp;         // pruned graph
    const int32_t* ci;
    const int64_t* leaf_ptr;
    const int32_t* leaf_ids;
    double d;
    unsigned long long* buckets;  // [4 * nnz_kept] bucket bounds of the long rows (null if none)
    const void* pos_kept;
    void* pos_all;
};

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Angle of (dx, dy) in [0, 2 pi), reduced modulo the leaf spacing `period`
// (a zero comes out as +0, so that the bit patterns of residues order as
// their values).
__device__ __forceinline__ double angle_residue(double dx, double dy, double period) {
    double ang = atan2(dy, dx);
    if (ang < 0.0) ang += kTwoPi;
    double r = fmod(ang, period);
    if (r < 0.0) r += period;
    if (r >= period) r -= period;
    return r + 0.0;
}

// Minimum over the workgroup, returned to every thread (sh: THREADS / 64 doubles).
template <int THREADS>
__device__ double block_min(double x, double* sh) {
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(x, off, 64);
        x = o < x ? o : x;
    }
    if (lane64() == 0) sh[wave_id()] = x;
    __syncthreads();
    x = sh[0];
    for (int q = 1; q < THREADS / 64; ++q) x = sh[q] < x ? sh[q] : x;
    __syncthreads();
    return x;
}

// Widest gap over the workgroup: the larger gap wins, equal gaps go to the
// smaller index.  Every thread receives the winner.
template <int THREADS>
__device__ void block_widest(double& g, int64_t& idx, double* sg, int64_t* si) {
    for (int off = 32; off >= 1; off >>= 1) {
        const double og = __shfl_xor(g, off, 64);
        const int64_t oi = __shfl_xor(idx, off, 64);
        if (og > g || (og == g && oi < idx)) {
            g = og;
            idx = oi;
        }
    }
    if (lane64() == 0) {
        sg[wave_id()] = g;
        si[wave_id()] = idx;
    }
    __syncthreads();
    g = sg[0];
    idx = si[0];
    for (int q = 1; q < THREADS / 64; ++q)
        if (sg[q] > g || (sg[q] == g && si[q] < idx)) {
            g = sg[q];
            idx = si[q];
        }
    __syncthreads();
}

// The L leaves of kept vertex i (at xv, yv), in ascending id, at angles
// phi + 2 pi j / L on the circle of radius rho.
template <class V, int THREADS>
__device__ void place_leaves(const ReinsertArgs& a, int32_t i, int32_t L, double xv, double yv,
                             double phi, double rho) {
    V* __restrict__ pa = reinterpret_cast<V*>(a.pos_all);
    const int64_t lb = a.leaf_ptr[i];
    for (int32_t j = threadIdx.x; j < L; j += THREADS) {
        const double th = phi + kTwoPi * (double)j / (double)L;
        V p;
        p.x = (decltype(p.x))(xv + rho * cos(th));
        p.y = (decltype(p.y))(yv + rho * sin(th));
        pa[a.leaf_ids[lb + j]] = p;
    }
}

// Ascending bitonic sort of x[0, m) (m a power of two, in LDS) by one
// workgroup of THREADS threads.
template <int THREADS>
__device__ void block_bitonic_sort(double* x, int m) {
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < m; i += THREADS) {
                const int p = i ^ j;
                if (p > i) {
                    const double u = x[i], w = x[p];
                    if ((u > w) == ((i & k) == 0)) {
                        x[i] = w;
                        x[p] = u;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Rows of at most kShortRow edges: one wavefront per vertex sorts the
// residues in LDS and scans consecutive pairs (around the circle) for the
// first widest gap.
template <class V>
__global__ __launch_bounds__(64) void reinsert_short_kernel(ReinsertArgs a) {
    __shared__ double s_res[kShortRow];
    __shared__ double s_g[1];
    __shared__ int64_t s_i[1];
    const V* __restrict__ pk = reinterpret_cast<const V*>(a.pos_kept);
    for (int64_t t = blockIdx.x; t < a.n_anchor; t += gridDim.x) {
        const int32_t i = a.anchors[t];
        const int32_t L = a.leaves[a.kept_of[i]];
        const int64_t rb = a.rp[i];
        const int deg = (int)(a.rp[i + 1] - rb);
        const double xv = (double)pk[i].x, yv = (double)pk[i].y;
        const double period = kTwoPi / (double)L;
        int m = 1;
        while (m < deg) m <<= 1;
        double shortest = INFINITY;
        for (int e = threadIdx.x; e < m; e += 64) {
            double r = INFINITY;  // padding sorts last
            if (e < deg) {
                const int32_t u = a.ci[rb + e];
                const double dx = (double)pk[u].x - xv, dy = (double)pk[u].y - yv;
                const double len = sqrt(dx * dx + dy * dy);
                shortest = len < shortest ? len : shortest;
                r = angle_residue(dx, dy, period);
            }
            s_res[e] = r;
        }
        shortest = block_min<64>(shortest, s_g);
        block_bitonic_sort<64>(s_res, m);
        double best = -1.0;
        int64_t bi = 0;
        for (int e = threadIdx.x; e < deg; e += 64) {
            const double lo = s_res[e];
            const double hi = e + 1 < deg ? s_res[e + 1] : s_res[0] + period;
            if (hi - lo > best) {
                best = hi - lo;
                bi = e;
            }
        }
        block_widest<64>(best, bi, s_g, s_i);
        double phi = 0.0;
        if (deg > 0) {
            const double lo = s_res[bi];
            const double hi = bi + 1 < deg ? s_res[bi + 1] : s_res[0] + period;
            phi = lo + 0.5 * (hi - lo);
            if (phi >= period) phi -= period;
        }
        __syncthreads();  // s_res is reused by the next vertex
        place_leaves<V, 64>(a, i, L, xv, yv, phi, 0.2 * (deg > 0 ? shortest : a.d));
    }
}

__device__ __forceinline__ unsigned long long load_l2(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Longer rows, without sorting: the residues are binned into B = 2 deg
// buckets of width period / B, keeping each bucket's smallest and largest
// residue.  The widest gap is at least period / deg, more than any two
// residues of one bucket are apart, so it runs from the largest residue of a
// non-empty bucket to the smallest of the next non-empty bucket (cyclically);
// scanning non-empty buckets in ascending order finds the same first widest
// gap, with the same end points, as a scan of the sorted residues.  Residues
// are non-negative, so their IEEE bit patterns order as the values do and the
// bucket bounds are kept with 64-bit integer atomics (performed in L2; read
// back with loads that bypass the L1 cache).
template <class V>
__global__ __launch_bounds__(kLongThreads) void reinsert_long_kernel(ReinsertArgs a) {
    constexpr int T = kLongThreads;
    __shared__ double s_g[T / 64];
    __shared__ int64_t s_i[T / 64];
    __shared__ int64_t s_next[T];  // first non-empty bucket at or after each thread's chunk
    __shared__ double s_lohi[2];
    constexpr int64_t kNone = INT64_MAX;
    const V* __restrict__ pk = reinterpret_cast<const V*>(a.pos_kept);
    for (int64_t t = blockIdx.x; t < a.n_anchor; t += gridDim.x) {
        const int32_t i = a.anchors[t];
        const int32_t L = a.leaves[a.kept_of[i]];
        const int64_t rb = a.rp[i], deg = a.rp[i + 1] - rb;
        const double xv = (double)pk[i].x, yv = (double)pk[i].y;
        const double period = kTwoPi / (double)L;
        const int64_t B = 2 * deg;
        unsigned long long* bmin = a.buckets + 4 * rb;
        unsigned long long* bmax = bmin + B;
        for (int64_t b = threadIdx.x; b < B; b += T) {
            bmin[b] = ~0ull;
            bmax[b] = 0ull;
        }
        __builtin_amdgcn_s_waitcnt(0);  // the stores have reached L2
        __syncthreads();
        const double scale = (double)B / period;
        double shortest = INFINITY;
        for (int64_t e = threadIdx.x; e < deg; e += T) {
            const int32_t u = a.ci[rb + e];
            const double dx = (double)pk[u].x - xv, dy = (double)pk[u].y - yv;
            const double len = sqrt(dx * dx + dy * dy);
            shortest = len < shortest ? len : shortest;
            const double r = angle_residue(dx, dy, period);
            const double q = r * scale;
            int64_t b = q >= 0.0 ? (int64_t)q : 0;  // (a NaN position lands in bucket 0)
            b = b < B ? b : B - 1;
            const unsigned long long bits = (unsigned long long)__double_as_longlong(r);
            atomicMin(&bmin[b], bits);
            atomicMax(&bmax[b], bits);
        }
        __builtin_amdgcn_s_waitcnt(0);  // the atomics are done
        shortest = block_min<T>(shortest, s_g);
        // first non-empty bucket of each thread's chunk, then a suffix minimum
        const int64_t C = (B + T - 1) / T;
        const int64_t c0 = (int64_t)threadIdx.x * C, c1 = c0 + C < B ? c0 + C : B;
        int64_t first = kNone;
        for (int64_t b = c0; b < c1 && first == kNone; ++b)
            if (load_l2(&bmin[b]) <= load_l2(&bmax[b])) first = b;
        s_next[threadIdx.x] = first;
        __syncthreads();
        for (int off = 1; off < T; off <<= 1) {
            int64_t v = s_next[threadIdx.x];
            if (threadIdx.x + off < T) {
                const int64_t o = s_next[threadIdx.x + off];
                v = o < v ? o : v;
            }
            __syncthreads();
            s_next[threadIdx.x] = v;
            __syncthreads();
        }
        const int64_t first_all = s_next[0];
        const int64_t after = threadIdx.x + 1 < T ? s_next[threadIdx.x + 1] : kNone;
        // gaps that start in this chunk, in ascending order
        double best = -1.0, blo = 0.0, bhi = 0.0;
        int64_t bi = kNone;
        int64_t prev = kNone;
        double prev_max = 0.0;
        auto consider = [&](int64_t from, double lo, double hi) {
            if (hi - lo > best) {
                best = hi - lo;
                bi = from;
                blo = lo;
                bhi = hi;
            }
        };
        for (int64_t b = c0; b < c1; ++b) {
            const unsigned long long mn = load_l2(&bmin[b]), mx = load_l2(&bmax[b]);
            if (mn > mx) continue;  // empty
            if (prev != kNone) consider(prev, prev_max, __longlong_as_double((long long)mn));
            prev = b;
            prev_max = __longlong_as_double((long long)mx);
        }
        if (prev != kNone) {
            const double hi = after != kNone
                                  ? __longlong_as_double((long long)load_l2(&bmin[after]))
                                  : __longlong_as_double((long long)load_l2(&bmin[first_all])) + period;
            consider(prev, prev_max, hi);
        }
        int64_t win = bi;
        double wg = best;
        block_widest<T>(wg, win, s_g, s_i);
        if (bi == win && bi != kNone) {
            s_lohi[0] = blo;
            s_lohi[1] = bhi;
        }
        __syncthreads();
        const double lo = s_lohi[0], hi = s_lohi[1];
        double phi = lo + 0.5 * (hi - lo);
        if (phi >= period) phi -= period;
        __syncthreads();  // s_next and s_lohi are reused by the next vertex
        place_leaves<V, T>(a, i, L, xv, yv, phi, 0.2 * shortest);
    }
}

static int grid_of(int64_t items) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (items + kBlock - 1) / kBlock));
}

static void free_pruned(gila_pruned* p, Release rel = Release{}) {
    if (!p) return;
    DeviceGuard g(p->device);
    rel(p->anchor);
    rel(p->leaves);
    rel(p->new_id);
    rel(p->kept_of);
    rel(p->rp);
    rel(p->ci);
    rel(p->mass);
    rel(p->leaf_ptr);
    rel(p->leaf_ids);
    rel(p->anchors);
    delete p;
}

namespace {
struct PrunedHolder {
    gila_pruned* p;
    Release rel{};
    ~PrunedHolder() { free_pruned(p, rel); }
};

// Scratch freed into the block cache once the work on its stream is done.
struct Tmp {
    hipStream_t st;
    void* p = nullptr;
    explicit Tmp(hipStream_t s) : st(s) {}
    ~Tmp() { dfree_on(p, st); }
    template <class T>
    int alloc(size_t count) {
        return dalloc(&p, count * sizeof(T) + 16);
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};
}  // namespace

static int prune(const gila_csr* g, hipStream_t s, gila_pruned** out) {
    if (!out) return fail(GILA_EINVAL, "out is NULL");
    *out = nullptr;
    GILA_TRY(validate_graph(g, s));
    int dev = 0;
    GILA_HIP(hipGetDevice(&dev));
    const int32_t n = g->n;
    PrunedHolder h{new gila_pruned()};
    gila_pruned* p = h.p;
    p->device = dev;
    p->n = n;
    p->nnz = g->nnz;
    GILA_TRY(dalloc_t(&p->anchor, (size_t)n));
    GILA_TRY(dalloc_t(&p->leaves, (size_t)n));
    GILA_TRY(dalloc_t(&p->new_id, (size_t)n));
    const size_t ws = (size_t)scan_workspace_count(std::max<int64_t>(n, 1));
    Tmp flag(s), scan(s), wsp(s), small(s);
    GILA_TRY(flag.alloc<int64_t>((size_t)n + 1));
    GILA_TRY(scan.alloc<int64_t>((size_t)n + 1));
    GILA_TRY(wsp.alloc<int64_t>(ws));
    GILA_TRY(small.alloc<int64_t>(4));
    int64_t* d_small = small.as<int64_t>();  // [0] max anchor degree
    GILA_HIP(hipMemsetAsync(d_small, 0, 4 * sizeof(int64_t), s));
    if (n > 0) {
        GILA_HIP(hipMemsetAsync(p->leaves, 0, sizeof(int32_t) * n, s));
        hipLaunchKernelGGL(prune_mark_kernel, dim3(grid_of(n)), dim3(kBlock), 0, s, n, g->row_ptr,
                           g->col_idx, p->anchor, p->leaves);
        hipLaunchKernelGGL(keep_flags_kernel, dim3(grid_of(n)), dim3(kBlock), 0, s, n, p->anchor,
                           flag.as<int64_t>());
        GILA_HIP(hipGetLastError());
        GILA_TRY(enqueue_exclusive_scan_i64(flag.as<int64_t>(), scan.as<int64_t>(), n,
                                            wsp.as<int64_t>(), s));
    }
    int64_t nk = 0;
    if (n > 0) {
        GILA_HIP(hipMemcpyAsync(&nk, scan.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
    }
    const int32_t n_kept = (int32_t)nk;
    p->n_kept = n_kept;
    p->n_pruned = n - n_kept;
    GILA_TRY(dalloc_t(&p->kept_of, (size_t)n_kept));
    GILA_TRY(dalloc_t(&p->rp, (size_t)n_kept + 1));
    GILA_TRY(dalloc_t(&p->mass, (size_t)n_kept));
    GILA_TRY(dalloc_t(&p->leaf_ptr, (size_t)n_kept + 1));
    GILA_TRY(dalloc_t(&p->leaf_ids, (size_t)p->n_pruned));
    GILA_HIP(hipMemsetAsync(p->rp, 0, sizeof(int64_t), s));
    GILA_HIP(hipMemsetAsync(p->leaf_ptr, 0, sizeof(int64_t), s));
    KeptRows kr{};
    kr.n_kept = n_kept;
    kr.rp = g->row_ptr;
    kr.ci = g->col_idx;
    kr.anchor = p->anchor;
    kr.new_id = p->new_id;
    kr.kept_of = p->kept_of;
    const int rgrid = (int)std::max<int64_t>(1, std::min<int64_t>(16384, ((int64_t)n_kept + kWaves - 1) / kWaves));
    int64_t sizes[2] = {0, 0};  // nnz_kept, longest row of a vertex with leaves
    int64_t csizes[kSortClasses] = {0, 0};  // vertices with leaves per class
    if (n > 0) {
        hipLaunchKernelGGL(kept_kernel, dim3(grid_of(n)), dim3(kBlock), 0, s, n, p->anchor,
                           scan.as<int64_t>(), p->new_id, p->kept_of);
        // pruned-graph degrees -> row offsets
        kr.kdeg = flag.as<int64_t>();
        hipLaunchKernelGGL(kept_rows_kernel<false>, dim3(rgrid), dim3(kBlock), 0, s, kr);
        GILA_HIP(hipGetLastError());
        GILA_TRY(enqueue_exclusive_scan_i64(kr.kdeg, p->rp, n_kept, wsp.as<int64_t>(), s));
        // weights, leaf counts -> leaf offsets, vertices with leaves -> one
        // list grouped by row-length class
        int64_t* lcount = flag.as<int64_t>();
        int64_t* cflag = scan.as<int64_t>();
        Tmp cls(s), cscan(s);
        GILA_TRY(cls.alloc<int32_t>((size_t)n_kept + 1));
        GILA_TRY(cscan.alloc<int64_t>(((size_t)n_kept + 1) * kSortClasses));
        hipLaunchKernelGGL(anchor_kernel, dim3(grid_of(n_kept)), dim3(kBlock), 0, s, n_kept,
                           p->kept_of, p->leaves, p->rp, p->mass, lcount, cls.as<int32_t>(),
                           (unsigned long long*)d_small);
        GILA_HIP(hipGetLastError());
        GILA_TRY(enqueue_exclusive_scan_i64(lcount, p->leaf_ptr, n_kept, wsp.as<int64_t>(), s));
        for (int c = 0; c < kSortClasses; ++c) {
            int64_t* cs = cscan.as<int64_t>() + (size_t)c * (n_kept + 1);
            hipLaunchKernelGGL(class_flag_kernel, dim3(grid_of(n_kept)), dim3(kBlock), 0, s, n_kept,
                               cls.as<int32_t>(), c, cflag);
            GILA_HIP(hipGetLastError());
            GILA_TRY(enqueue_exclusive_scan_i64(cflag, cs, n_kept, wsp.as<int64_t>(), s));
            GILA_HIP(hipMemcpyAsync(&csizes[c], cs + n_kept, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        }
        GILA_HIP(hipMemcpyAsync(&sizes[0], p->rp + n_kept, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipMemcpyAsync(&sizes[1], d_small, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        p->nnz_kept = sizes[0];
        p->max_anchor_deg = sizes[1];
        p->n_anchor = 0;
        for (int c = 0; c < kSortClasses; ++c) {
            p->n_class[c] = (int32_t)csizes[c];
            p->n_anchor += p->n_class[c];
        }
        GILA_TRY(dalloc_t(&p->ci, (size_t)p->nnz_kept));
        GILA_TRY(dalloc_t(&p->anchors, (size_t)p->n_anchor));
        int64_t off = 0;
        for (int c = 0; c < kSortClasses; ++c) {
            hipLaunchKernelGGL(anchor_list_kernel, dim3(grid_of(n_kept)), dim3(kBlock), 0, s, n_kept,
                               cls.as<int32_t>(), c, cscan.as<int64_t>() + (size_t)c * (n_kept + 1),
                               off, p->anchors);
            off += csizes[c];
        }
        kr.krp = p->rp;
        kr.kci = p->ci;
        kr.leaf_ptr = p->leaf_ptr;
        kr.leaf_ids = p->leaf_ids;
        hipLaunchKernelGGL(kept_rows_kernel<true>, dim3(rgrid), dim3(kBlock), 0, s, kr);
        GILA_HIP(hipGetLastError());
        GILA_HIP(hipStreamSynchronize(s));
    } else {
        GILA_TRY(dalloc_t(&p->ci, 0));
        GILA_TRY(dalloc_t(&p->anchors, 0));
    }
    p->device_bytes = 12 * (int64_t)n + (int64_t)n_kept * (4 + 8 + 8 + 8 + 4) + 16 +
                      4 * p->nnz_kept + 4 * (int64_t)p->n_pruned;
    *out = p;
    h.p = nullptr;
    return GILA_OK;
}

static int check_precision(int32_t precision) {
    if (precision != GILA_FP64 && precision != GILA_FP32 && precision != GILA_FP32_KAHAN)
        return fail(GILA_EINVAL, "unknown precision %d", precision);
    return GILA_OK;
}

static int reinsert(const gila_pruned* p, double d, int32_t precision, const void* pos_kept,
                    void* pos_all, hipStream_t s) {
    if (!p) return fail(GILA_EINVAL, "handle is NULL");
    GILA_TRY(check_precision(precision));
    if (!(d > 0.0) || !std::isfinite(d)) return fail(GILA_EINVAL, "ideal_length must be finite and > 0");
    if (p->n > 0 && (!pos_kept || !pos_all)) return fail(GILA_EINVAL, "position buffer is NULL");
    if (p->n == 0) return GILA_OK;
    DeviceGuard dg(p->device);
    const bool f64 = precision == GILA_FP64;
    if (f64)
        hipLaunchKernelGGL(copy_kept_kernel<double2>, dim3(grid_of(p->n_kept)), dim3(kBlock), 0, s,
                           p->n_kept, p->kept_of, (const double2*)pos_kept, (double2*)pos_all);
    else
        hipLaunchKernelGGL(copy_kept_kernel<float2>, dim3(grid_of(p->n_kept)), dim3(kBlock), 0, s,
                           p->n_kept, p->kept_of, (const float2*)pos_kept, (float2*)pos_all);
    GILA_HIP(hipGetLastError());
    if (p->n_anchor == 0) return GILA_OK;
    Tmp scratch(s);
    if (p->n_class[1] > 0) GILA_TRY(scratch.alloc<unsigned long long>(4 * (size_t)p->nnz_kept));
    ReinsertArgs a{};
    a.anchors = p->anchors;
    a.kept_of = p->kept_of;
    a.leaves = p->leaves;
    a.rp = p->rp;
    a.ci = p->ci;
    a.leaf_ptr = p->leaf_ptr;
    a.leaf_ids = p->leaf_ids;
    a.d = d;
    a.buckets = scratch.as<unsigned long long>();
    a.pos_kept = pos_kept;
    a.pos_all = pos_all;
    a.n_anchor = p->n_class[0];
    if (a.n_anchor > 0) {
        const dim3 grid((unsigned)std::min<int64_t>(65536, a.n_anchor));
        if (f64) hipLaunchKernelGGL(reinsert_short_kernel<double2>, grid, dim3(64), 0, s, a);
        else hipLaunchKernelGGL(reinsert_short_kernel<float2>, grid, dim3(64), 0, s, a);
        GILA_HIP(hipGetLastError());
    }
    a.anchors += a.n_anchor;
    a.n_anchor = p->n_class[1];
    if (a.n_anchor > 0) {
        const dim3 grid((unsigned)std::min<int64_t>(65536, a.n_anchor));
        if (f64) hipLaunchKernelGGL(reinsert_long_kernel<double2>, grid, dim3(kLongThreads), 0, s, a);
        else hipLaunchKernelGGL(reinsert_long_kernel<float2>, grid, dim3(kLongThreads), 0, s, a);
        GILA_HIP(hipGetLastError());
    }
    return GILA_OK;
}

static int gather(const gila_pruned* p, int32_t precision, const void* pos_all, void* pos_kept,
                  hipStream_t s) {
    if (!p) return fail(GILA_EINVAL, "handle is NULL");
    GILA_TRY(check_precision(precision));
    if (p->n_kept > 0 && (!pos_kept || !pos_all)) return fail(GILA_EINVAL, "position buffer is NULL");
    if (p->n_kept == 0) return GILA_OK;
    DeviceGuard dg(p->device);
    if (precision == GILA_FP64)
        hipLaunchKernelGGL(gather_kept_kernel<double2>, dim3(grid_of(p->n_kept)), dim3(kBlock), 0, s,
                           p->n_kept, p->kept_of, (const double2*)pos_all, (double2*)pos_kept);
    else
        hipLaunchKernelGGL(gather_kept_kernel<float2>, dim3(grid_of(p->n_kept)), dim3(kBlock), 0, s,
                           p->n_kept, p->kept_of, (const float2*)pos_all, (float2*)pos_kept);
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

}  // namespace gila

using namespace gila;

extern "C" {

int gila_prune(const gila_csr* g_dev, void* stream, gila_pruned** out) {
    TraceRange trace_range("gila_prune");
    clear_error();
    return prune(g_dev, (hipStream_t)stream, out);
}

int gila_pruned_info(const gila_pruned* p, int32_t* n_kept, int64_t* nnz_kept, int32_t* n_pruned,
                     int32_t* n_with_leaves, int64_t* device_bytes) {
    clear_error();
    if (!p) return fail(GILA_EINVAL, "handle is NULL");
    if (n_kept) *n_kept = p->n_kept;
    if (nnz_kept) *nnz_kept = p->nnz_kept;
    if (n_pruned) *n_pruned = p->n_pruned;
    if (n_with_leaves) *n_with_leaves = p->n_anchor;
    if (device_bytes) *device_bytes = p->device_bytes;
    return GILA_OK;
}

int gila_pruned_graph(const gila_pruned* p, gila_csr* g_dev_out, const double** mass_dev_out) {
    clear_error();
    if (!p) return fail(GILA_EINVAL, "handle is NULL");
    if (g_dev_out) {
        g_dev_out->n = p->n_kept;
        g_dev_out->nnz = p->nnz_kept;
        g_dev_out->row_ptr = p->rp;
        g_dev_out->col_idx = p->ci;
    }
    if (mass_dev_out) *mass_dev_out = p->mass;
    return GILA_OK;
}

int gila_pruned_export(const gila_pruned* p, int32_t* anchor_host, int32_t* leaves_host,
                       int32_t* new_id_host) {
    clear_error();
    if (!p) return fail(GILA_EINVAL, "handle is NULL");
    if (p->n == 0) return GILA_OK;
    DeviceGuard dg(p->device);
    const size_t b = sizeof(int32_t) * (size_t)p->n;
    if (anchor_host) GILA_HIP(hipMemcpy(anchor_host, p->anchor, b, hipMemcpyDeviceToHost));
    if (leaves_host) GILA_HIP(hipMemcpy(leaves_host, p->leaves, b, hipMemcpyDeviceToHost));
    if (new_id_host) GILA_HIP(hipMemcpy(new_id_host, p->new_id, b, hipMemcpyDeviceToHost));
    return GILA_OK;
}

int gila_pruned_gather(const gila_pruned* p, int32_t precision, const void* pos_all_dev,
                       void* pos_kept_dev, void* stream) {
    clear_error();
    return gather(p, precision, pos_all_dev, pos_kept_dev, (hipStream_t)stream);
}

int gila_reinsert(const gila_pruned* p, double ideal_length, int32_t precision,
                  const void* pos_kept_dev, void* pos_all_dev, void* stream) {
    TraceRange trace_range("gila_reinsert");
    clear_error();
    return reinsert(p, ideal_length, precision, pos_kept_dev, pos_all_dev, (hipStream_t)stream);
}

void gila_pruned_free(gila_pruned* p) {
    if (!p) return;
    DeviceGuard g(p->device);
    free_pruned(p, public_release());
}

int gila_layout_pruned(const gila_csr* g_dev, int32_t k, const gila_params* params, void* pos_dev,
                       void* stream, gila_stats* out) {
    TraceRange trace_range("gila_layout_pruned");
    clear_error();
    GILA_TRY(check_params(params, true));
    if (k < 1) return fail(GILA_EINVAL, "k must be >= 1 (got %d)", k);
    if (g_dev && g_dev->n > 0 && !pos_dev) return fail(GILA_EINVAL, "pos_dev is NULL");
    hipStream_t s = (hipStream_t)stream;
    gila_pruned* p = nullptr;
    GILA_TRY(prune(g_dev, s, &p));
    PrunedHolder ph{p, Release{true, s}};
    gila_csr pg{p->n_kept, p->nnz_kept, p->rp, p->ci};
    gila_khop* kh = nullptr;
    GILA_TRY(build_khop(&pg, k, s, &kh));
    struct KH {
        gila_khop* k;
        hipStream_t s;
        ~KH() { free_khop(k, Release{true, s}); }
    } kguard{kh, s};
    GILA_TRY(gila_khop_set_mass(kh, p->mass, stream));
    const size_t pb = params->precision == GILA_FP64 ? 16 : 8;
    Tmp kept(s);
    GILA_TRY(kept.alloc<unsigned char>(pb * (size_t)std::max(p->n_kept, 1)));
    GILA_TRY(gather(p, params->precision, pos_dev, kept.p, s));
    {
        std::lock_guard<std::mutex> lk(kh->mu);
        GILA_TRY(run_iterations(kh, params, 0, params->iterations, kept.p, s, out, false));
    }
    GILA_TRY(reinsert(p, params->ideal_length, params->precision, kept.p, pos_dev, s));
    GILA_HIP(hipStreamSynchronize(s));
    return GILA_OK;
}

}  // extern "C"

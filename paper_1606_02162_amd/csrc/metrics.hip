// Drawing-quality metrics (Section 5.2): edge crossings, the standard
// deviation of edge lengths, and the similarity of the drawing's Gabriel
// graph to the graph (mean Jaccard index of the neighbourhoods).
//
// Coordinates are taken at single precision, so a product of two coordinates
// is exact in double.  Orientation and in-disc signs are first evaluated in
// double with an a-priori error bound; where the value is within the bound
// of zero the sign is taken exactly, from the polynomial multiplied out into
// such products and summed with expansion arithmetic (two-sum chains).
//
//   edge_list_kernel      edges {u, v}, u < v, in row order (the part of a
//                         sorted row above v is a suffix found by bisection)
//   crossings_kernel      an edge per thread against a chunk of edges
//                         streamed through LDS (each entry: end points and
//                         line coefficients); per pair four filtered signs
//                         decided by wavefront lane masks on the scalar unit;
//                         each pair once for the total, or both ways for
//                         per-edge counts
//   lengths kernels       per-edge length, fixed-order sums (mean, then the
//                         squared deviations)
//   grid kernels          points binned into a uniform grid (about two per
//                         cell)
//   gabriel_degree_kernel thread per point u (in cell order): rings of cells
//                         around u until each of the eight 45-degree octants
//                         around u is settled: the nearest point w found in it
//                         blocks everything at squared distance >= 2 |w - u|^2
//                         (such a v sees w within 45 degrees of its own
//                         direction, so w lies in the disc with diameter uv),
//                         or, with no point found, the rings cover the part of
//                         the bounding box the octant reaches; then every
//                         point not excluded that way is tested for an empty
//                         disc with diameter uv (cells scanned outwards from
//                         the disc's centre)
//   gabriel_edge_kernel   the same disc test for each graph edge (for the
//                         Jaccard intersections)
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "device_util.h"
#include "gila_internal.h"

namespace gila {

namespace {
struct MBuf {
    hipStream_t st;
    void* p = nullptr;
    explicit MBuf(hipStream_t s) : st(s) {}
    ~MBuf() { dfree_on(p, st); }
    template <class T>
    int alloc(size_t count) {
        return dalloc(&p, count * sizeof(T) + 64);
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};
int mgrid(int64_t items) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (items + kBlock - 1) / kBlock));
}
}  // namespace

constexpr int kCrossTile = 256;         // edges per LDS tile of the crossing kernel
constexpr int64_t kGabrielBudget = 2048;  // cells and points one thread visits for a point

// ------------------------------------------------------------------ points and edges
template <class V>
__global__ __launch_bounds__(kBlock) void to_float_kernel(int32_t n, const V* __restrict__ pos,
                                                          float2* __restrict__ out) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        out[v] = make_float2((float)pos[v].x, (float)pos[v].y);
}

// first entry of row v above v, and how many there are
__global__ __launch_bounds__(kBlock) void upper_count_kernel(int32_t n, const int64_t* __restrict__ rp,
                                                             const int32_t* __restrict__ ci,
                                                             int64_t* __restrict__ first,
                                                             int64_t* __restrict__ cnt) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        int64_t lo = rp[v], hi = rp[v + 1];
        const int64_t end = hi;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (ci[mid] <= v) lo = mid + 1;
            else hi = mid;
        }
        first[v] = lo;
        cnt[v] = end - lo;
    }
}

// Wavefront per vertex: its upper entries become edges eo[v] ...
__global__ __launch_bounds__(kBlock) void edge_list_kernel(int32_t n, const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const int64_t* __restrict__ first,
                                                           const int64_t* __restrict__ eo,
                                                           int2* __restrict__ ends) {
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    for (int64_t v = (int64_t)blockIdx.x * kWaves + wave_id(); v < n; v += waves) {
        const int64_t f = first[v], len = rp[v + 1] - f, o = eo[v];
        for (int64_t j = lane64(); j < len; j += 64) ends[o + j] = make_int2((int32_t)v, ci[f + j]);
    }
}

// ------------------------------------------------------------------ exact signs
// Knuth's two-sum: s is the rounded a + b and s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Exact sign of t[0] + ... + t[K-1].  Each term is merged into a growing
// expansion by a chain of two-sums (Shewchuk's grow-expansion); the pieces
// stay nonoverlapping with the largest last, so the sign of the sum is that
// of the last nonzero piece.
template <int K>
__device__ __forceinline__ int exact_sum_sign(const double (&t)[K]) {
    double h[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        double q = t[i];
#pragma unroll
        for (int j = 0; j < i; ++j) two_sum(q, h[j], q, h[j]);
        h[i] = q;
    }
    int sg = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) sg = h[j] > 0.0 ? 1 : (h[j] < 0.0 ? -1 : sg);
    return sg;
}

// orient(a, b, c) = (b - a) x (c - a) multiplied out (the two a.x a.y
// products cancel); products of single-precision values are exact in double.
__device__ __noinline__ int orient_exact(float ax, float ay, float bx, float by, float cx, float cy) {
    const double t[6] = {(double)bx * cy, -((double)bx * ay), -((double)ax * cy),
                         -((double)by * cx), (double)by * ax, (double)ay * cx};
    return exact_sum_sign(t);
}

// ------------------------------------------------------------------ crossings
// A segment's line in the form used by the sign filter: for a point x,
// orient(p0, p1, x) = dx x.y - dy x.x - k, evaluated in double.  Its rounding
// error is below 4u(|dx| |x.y| + |dy| |x.x|) + 2u(|x1 y0| + |y1 x0|) plus
// second-order terms (u = 2^-53; coordinates are floats, so x1 y0 and y1 x0
// are exact), hence below bnd = 8u((|dx| + |dy|) M + |x1 y0| + |y1 x0|) for
// every point with coordinates of magnitude at most M.
struct Line {
    double dx, dy, k, bnd;
};

__device__ __forceinline__ Line make_line(float x0, float y0, float x1, float y1, double M) {
#pragma clang fp contract(off)
    Line L;
    L.dx = (double)x1 - (double)x0;
    L.dy = (double)y1 - (double)y0;
    const double s = (double)x1 * y0, t = (double)y1 * x0;
    L.k = s - t;
    L.bnd = ((fabs(L.dx) + fabs(L.dy)) * M + (fabs(s) + fabs(t))) * 0x1p-50;
    return L;
}

// orient(p0, p1, (x, y)) up to rounding: its sign is certain where |d| > L.bnd
__device__ __forceinline__ double side(const Line& L, double x, double y) {
#pragma clang fp contract(off)
    const double q = L.dy * x;
    return fma(L.dx, y, -q) - L.k;
}

// One LDS entry: an edge's end points and line.
struct alignas(16) CrossEntry {
    double x0, y0, x1, y1;
    Line L;
};

constexpr int kCrossRows = 1;                         // edges per thread (64 VGPRs: 8 waves per SIMD)
constexpr int kCrossBlock = kCrossRows * kCrossTile;  // edges per block
constexpr int64_t kCrossChunk = 8192;                 // edges streamed per block (at least)

// Exact crossing decision for a pair the filter could not settle.
__device__ __forceinline__ int cross_exact(int2 ea, int2 ec, const float2* __restrict__ p) {
    if (ea.x == ec.x || ea.x == ec.y || ea.y == ec.x || ea.y == ec.y) return 0;
    const float2 a = p[ea.x], b = p[ea.y], c = p[ec.x], d = p[ec.y];
    const int o1 = orient_exact(a.x, a.y, b.x, b.y, c.x, c.y);
    const int o2 = orient_exact(a.x, a.y, b.x, b.y, d.x, d.y);
    if (o1 * o2 >= 0) return 0;
    const int o3 = orient_exact(c.x, c.y, d.x, d.y, a.x, a.y);
    const int o4 = orient_exact(c.x, c.y, d.x, d.y, b.x, b.y);
    return o3 * o4 < 0 ? 1 : 0;
}

// The pairs (i, j) of one LDS tile for the edges a thread holds.  Lane
// masks of the wavefront (one ballot per comparison, combined in scalar
// registers) decide each pair: sure crossings of PAIRS_ONCE mode are counted
// per wavefront (wcnt), other counts per lane (cnt).  DIAG: count j > i only.
template <bool PAIRS_ONCE, bool DIAG>
__device__ __forceinline__ void cross_tile(const CrossEntry* __restrict__ s_e, const int2* __restrict__ s_end,
                                           int tn, int64_t t0, int64_t a0, const uint64_t (&live)[kCrossRows],
                                           const double (&ax)[kCrossRows], const double (&ay)[kCrossRows],
                                           const double (&bx)[kCrossRows], const double (&by)[kCrossRows],
                                           const Line (&la)[kCrossRows], int (&cnt)[kCrossRows],
                                           uint64_t& wcnt, const int2* __restrict__ ends,
                                           const float2* __restrict__ p) {
    const uint64_t me = 1ull << lane64();
    for (int q = 0; q < tn; ++q) {
        const CrossEntry c = s_e[q];
#pragma unroll
        for (int r = 0; r < kCrossRows; ++r) {
            const int64_t i = a0 + r * kCrossTile + threadIdx.x;
            const double d1 = side(la[r], c.x0, c.y0);
            const double d2 = side(la[r], c.x1, c.y1);
            const double d3 = side(c.L, ax[r], ay[r]);
            const double d4 = side(c.L, bx[r], by[r]);
            // the signs are certain where |d| > bnd; then |d| > bnd >= 2^-348
            // (a float's nonzero difference or product is at least 2^-298 in
            // magnitude), so the products below neither underflow nor overflow
            const uint64_t sure = __builtin_amdgcn_ballot_w64(fabs(d1) > la[r].bnd) &
                                  __builtin_amdgcn_ballot_w64(fabs(d2) > la[r].bnd) &
                                  __builtin_amdgcn_ballot_w64(fabs(d3) > c.L.bnd) &
                                  __builtin_amdgcn_ballot_w64(fabs(d4) > c.L.bnd);
            const uint64_t cross = __builtin_amdgcn_ballot_w64(d1 * d2 < 0.0) &
                                   __builtin_amdgcn_ballot_w64(d3 * d4 < 0.0);
            const uint64_t keep = DIAG ? __builtin_amdgcn_ballot_w64(t0 + q > i) & live[r] : live[r];
            if (PAIRS_ONCE)
                wcnt += __popcll(sure & cross & keep);
            else
                cnt[r] += (sure & cross & keep & me) ? 1 : 0;
            const uint64_t slow = ~sure & keep;
            if (slow) [[unlikely]] {
                if (slow & me) cnt[r] += cross_exact(ends[i], s_end[q], p);
            }
        }
    }
}

// Block (blockIdx.x, blockIdx.y): edges i of A-block x (thread t holds
// i = x * kCrossBlock + r * kCrossTile + t, r < kCrossRows) against edges j
// of chunk y, streamed through LDS in tiles.  A crossing is a pair with no
// shared end whose ends lie strictly on opposite sides of the other's line.
// PAIRS_ONCE: only j > i counts (each crossing once, for the total);
// otherwise every j != i counts and per_edge[i] accumulates.  M bounds the
// magnitude of every coordinate.
template <bool PAIRS_ONCE>
__global__ __launch_bounds__(kCrossTile) void crossings_kernel(int64_t m, int64_t chunk, double M,
                                                               const int2* __restrict__ ends,
                                                               const float2* __restrict__ p,
                                                               unsigned long long* __restrict__ per_edge,
                                                               unsigned long long* __restrict__ total) {
    __shared__ CrossEntry s_e[kCrossTile];
    __shared__ int2 s_end[kCrossTile];
    const int64_t a0 = (int64_t)blockIdx.x * kCrossBlock;
    const int64_t c0 = (int64_t)blockIdx.y * chunk;
    const int64_t c1 = min(c0 + chunk, m);
    int64_t jbeg = c0;
    if (PAIRS_ONCE) {
        if (c1 <= a0 + 1) return;  // every j of the chunk is <= every i of the block
        jbeg = max(c0, a0);        // a0 is a multiple of the tile size
    }
    double ax[kCrossRows], ay[kCrossRows], bx[kCrossRows], by[kCrossRows];
    Line la[kCrossRows];
    int cnt[kCrossRows];
    uint64_t live[kCrossRows];
    uint64_t wcnt = 0;
#pragma unroll
    for (int r = 0; r < kCrossRows; ++r) {
        const int64_t i = a0 + r * kCrossTile + threadIdx.x;
        cnt[r] = 0;
        live[r] = __builtin_amdgcn_ballot_w64(i < m);
        float2 pa = make_float2(0.f, 0.f), pb = pa;
        if (i < m) {
            const int2 e = ends[i];
            pa = p[e.x];
            pb = p[e.y];
        }
        ax[r] = pa.x;
        ay[r] = pa.y;
        bx[r] = pb.x;
        by[r] = pb.y;
        la[r] = make_line(pa.x, pa.y, pb.x, pb.y, M);
    }
    for (int64_t t0 = jbeg; t0 < c1; t0 += kCrossTile) {
        const int64_t j = t0 + threadIdx.x;
        if (j < c1) {
            const int2 e = ends[j];
            const float2 pc = p[e.x], pd = p[e.y];
            s_e[threadIdx.x] = CrossEntry{pc.x, pc.y, pd.x, pd.y, make_line(pc.x, pc.y, pd.x, pd.y, M)};
            s_end[threadIdx.x] = e;
        }
        __syncthreads();
        const int tn = (int)min<int64_t>(kCrossTile, c1 - t0);
        // in PAIRS_ONCE mode, tiles that reach into the block's own range count j > i only
        if (PAIRS_ONCE && t0 < a0 + kCrossBlock)
            cross_tile<PAIRS_ONCE, true>(s_e, s_end, tn, t0, a0, live, ax, ay, bx, by, la, cnt, wcnt, ends, p);
        else
            cross_tile<PAIRS_ONCE, false>(s_e, s_end, tn, t0, a0, live, ax, ay, bx, by, la, cnt, wcnt, ends, p);
        __syncthreads();
    }
    int64_t sum = 0;
#pragma unroll
    for (int r = 0; r < kCrossRows; ++r) {
        const int64_t i = a0 + r * kCrossTile + threadIdx.x;
        sum += cnt[r];
        if (!PAIRS_ONCE && per_edge && cnt[r] && i < m)
            atomicAdd(&per_edge[i], (unsigned long long)cnt[r]);
    }
    const int64_t w = wave_sum(sum) + (int64_t)wcnt;
    if (lane64() == 0 && w) atomicAdd(total, (unsigned long long)w);
}

// ------------------------------------------------------------------ edge lengths
__global__ __launch_bounds__(kBlock) void lengths_sum_kernel(int64_t m, const int2* __restrict__ ends,
                                                             const float2* __restrict__ p,
                                                             double mean, int pass,
                                                             double* __restrict__ partial) {
    __shared__ double s[kWaves];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * kBlock) {
        const float2 a = p[ends[e].x], b = p[ends[e].y];
        const double dx = (double)b.x - (double)a.x, dy = (double)b.y - (double)a.y;
        const double l = sqrt(dx * dx + dy * dy);
        acc += pass == 0 ? l : (l - mean) * (l - mean);
    }
    const double t = block_sum(acc, s);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// ------------------------------------------------------------------ grid
struct Grid {
    float x0, y0, inv;  // cell of x: floor((x - x0) * inv)
    int32_t gx, gy;
};

__device__ __forceinline__ int32_t cell_x(const Grid& g, float x) {
    const float f = (x - g.x0) * g.inv;
    int32_t c = f >= 0.f ? (int32_t)f : 0;
    return c < g.gx ? c : g.gx - 1;
}
__device__ __forceinline__ int32_t cell_y(const Grid& g, float y) {
    const float f = (y - g.y0) * g.inv;
    int32_t c = f >= 0.f ? (int32_t)f : 0;
    return c < g.gy ? c : g.gy - 1;
}

__global__ __launch_bounds__(kBlock) void bounds_kernel(int32_t n, const float2* __restrict__ p,
                                                        unsigned int* __restrict__ box) {
    // box: ordered keys of xmin, ymin (min) and of -xmax, -ymax (min)
    __shared__ unsigned int s_k[4][kBlock];
    unsigned int k[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    auto key = [](float f) {
        const unsigned int u = __float_as_uint(f);
        return (u >> 31) ? ~u : (u | 0x80000000u);
    };
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const float2 q = p[v];
        k[0] = min(k[0], key(q.x));
        k[1] = min(k[1], key(q.y));
        k[2] = min(k[2], key(-q.x));
        k[3] = min(k[3], key(-q.y));
    }
    for (int c = 0; c < 4; ++c) s_k[c][threadIdx.x] = k[c];
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int c = 0; c < 4; ++c) s_k[c][threadIdx.x] = min(s_k[c][threadIdx.x], s_k[c][threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x < 4) atomicMin(&box[threadIdx.x], s_k[threadIdx.x][0]);
}

__global__ __launch_bounds__(kBlock) void cell_count_kernel(int32_t n, Grid g, const float2* __restrict__ p,
                                                            int32_t* __restrict__ cell,
                                                            int64_t* __restrict__ cnt) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const int32_t c = cell_y(g, p[v].y) * g.gx + cell_x(g, p[v].x);
        cell[v] = c;
        atomicAdd((unsigned long long*)&cnt[c], 1ull);
    }
}

__global__ __launch_bounds__(kBlock) void cell_fill_kernel(int32_t n, const int32_t* __restrict__ cell,
                                                           const int64_t* __restrict__ start,
                                                           unsigned long long* __restrict__ cursor,
                                                           int32_t* __restrict__ pts) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const int32_t c = cell[v];
        const unsigned long long at = atomicAdd(&cursor[c], 1ull);
        pts[start[c] + (int64_t)at] = (int32_t)v;
    }
}

// (w - u).(w - v) multiplied out into products of floats (exact in double)
__device__ __noinline__ int disc_sign_exact(float2 u, float2 v, float2 w) {
    const double t[8] = {(double)w.x * w.x, -((double)w.x * v.x), -((double)u.x * w.x),
                         (double)u.x * v.x, (double)w.y * w.y, -((double)w.y * v.y),
                         -((double)u.y * w.y), (double)u.y * v.y};
    return exact_sum_sign(t);
}

// w lies in the closed disc with diameter uv: (w - u).(w - v) <= 0.  The
// double evaluation errs by less than 3u(|l| + |r|) plus second-order terms
// (u = 2^-53, as for a 2x2 determinant of rounded differences); when the
// result is within 8u of zero the sign is taken exactly.
__device__ __forceinline__ bool in_disc(float2 u, float2 v, float2 w) {
#pragma clang fp contract(off)
    const double l = ((double)w.x - (double)u.x) * ((double)w.x - (double)v.x);
    const double r = ((double)w.y - (double)u.y) * ((double)w.y - (double)v.y);
    const double d = l + r;
    const double b = (fabs(l) + fabs(r)) * 0x1p-50;
    if (d > b) return false;
    if (d < -b) return true;
    return disc_sign_exact(u, v, w) <= 0;
}

// The cells at Chebyshev distance exactly k from (cx, cy) inside columns
// [x0, x1] and rows [y0, y1] ((cx, cy) itself inside), numbered
// 0 .. count - 1 so that a thread or the lanes of a wavefront can take them
// in turn: row cy - k in full (if inside), row cy + k in full (if inside and
// k > 0), then the rows between at columns cx - k and cx + k (each if
// inside).  A ring costs only its cells inside.
struct RingShape {
    int64_t gx, count;
    int32_t cx, cy, k, xa, wtop, wbot, mid0, sides;  // sides: 1 left column, 2 right, 3 both
};

__device__ __forceinline__ RingShape ring_shape(const Grid& g, int32_t cx, int32_t cy, int32_t k, int32_t x0,
                                                int32_t x1, int32_t y0, int32_t y1) {
    RingShape R;
    R.gx = g.gx;
    R.cx = cx;
    R.cy = cy;
    R.k = k;
    R.xa = max(cx - k, x0);
    const int32_t w = min(cx + k, x1) - R.xa + 1;
    R.wtop = cy - k >= y0 ? w : 0;
    R.wbot = k > 0 && cy + k <= y1 ? w : 0;
    R.mid0 = max(cy - k + 1, y0);
    const int32_t nmid = k > 0 ? max(min(cy + k - 1, y1) - R.mid0 + 1, 0) : 0;
    R.sides = k > 0 ? (cx - k >= x0 ? 1 : 0) | (cx + k <= x1 ? 2 : 0) : 0;
    R.count = (int64_t)R.wtop + R.wbot + (int64_t)nmid * __popc(R.sides);
    return R;
}

__device__ __forceinline__ int64_t ring_cell(const RingShape& R, int64_t i) {
    if (i < R.wtop) return (int64_t)(R.cy - R.k) * R.gx + R.xa + i;
    i -= R.wtop;
    if (i < R.wbot) return (int64_t)(R.cy + R.k) * R.gx + R.xa + i;
    i -= R.wbot;
    int64_t y;
    int32_t x;
    if (R.sides == 3) {
        y = R.mid0 + (i >> 1);
        x = (i & 1) ? R.cx + R.k : R.cx - R.k;
    } else {
        y = R.mid0 + i;
        x = R.sides == 1 ? R.cx - R.k : R.cx + R.k;
    }
    return y * R.gx + x;
}

// Visit the cells of a ring in order; f(cell) returns true to stop, and then
// so does this (returning true).
template <class F>
__device__ __forceinline__ bool ring_cells(const Grid& g, int32_t cx, int32_t cy, int32_t k, int32_t x0,
                                           int32_t x1, int32_t y0, int32_t y1, F&& f) {
    const RingShape R = ring_shape(g, cx, cy, k, x0, x1, y0, y1);
    for (int64_t i = 0; i < R.count; ++i)
        if (f(ring_cell(R, i))) return true;
    return false;
}

// Cells visited (and points looked at) by the Gabriel searches, counted
// against a thread's budget.
struct Work {
    int64_t n = 0;
};

// No point other than iu, iv in the closed disc with diameter uv.  Cells are
// scanned outwards from the disc's centre, where a blocking point is most
// likely to be.
__device__ bool gabriel_pair_dev(const Grid& g, const int64_t* __restrict__ start,
                                 const int32_t* __restrict__ pts, const float2* __restrict__ p,
                                 int32_t iu, int32_t iv, Work& work) {
    const float2 u = p[iu], v = p[iv];
    const float cx = 0.5f * (u.x + v.x), cy = 0.5f * (u.y + v.y);
    const double dx = (double)v.x - (double)u.x, dy = (double)v.y - (double)u.y;
    // half the diameter, rounded up, plus one cell either way against rounding
    const float r = (float)(0.5 * sqrt(dx * dx + dy * dy)) * 1.0001f + 1e-30f;
    const int32_t x0 = max(cell_x(g, cx - r) - 1, 0), x1 = min(cell_x(g, cx + r) + 1, g.gx - 1);
    const int32_t y0 = max(cell_y(g, cy - r) - 1, 0), y1 = min(cell_y(g, cy + r) + 1, g.gy - 1);
    const int32_t ccx = min(max(cell_x(g, cx), x0), x1), ccy = min(max(cell_y(g, cy), y0), y1);
    const int32_t K = max(max(ccx - x0, x1 - ccx), max(ccy - y0, y1 - ccy));
    for (int32_t k = 0; k <= K; ++k) {
        const bool blocked = ring_cells(g, ccx, ccy, k, x0, x1, y0, y1, [&](int64_t c) {
            ++work.n;
            for (int64_t q = start[c]; q < start[c + 1]; ++q) {
                ++work.n;
                const int32_t w = pts[q];
                if (w != iu && w != iv && in_disc(u, v, p[w])) return true;
            }
            return false;
        });
        if (blocked) return false;
    }
    return true;
}

// octant of the direction (dx, dy), from signs and |dx| vs |dy| only
__device__ __forceinline__ int octant(double dx, double dy) {
    return (dx < 0.0 ? 4 : 0) + (dy < 0.0 ? 2 : 0) + (fabs(dx) < fabs(dy) ? 1 : 0);
}

// The cells of ring k (k >= 4) around (cx, cy) that can hold points of
// octant o, numbered like a ring's.  With (p, q) a cell's index offsets
// along the octant's major and minor axes, signed towards it, a point of the
// octant with true offsets A >= B >= 0 (in cell widths) has |p - A| < 2 and
// |q - B| < 2 (one for its place in the cell, one for a cell index computed
// in float), so p >= -1, q >= -1 and p >= q - 3: on ring k these are p = k
// with q in [-1, k] and q = k with p in [k - 3, k - 1].  Only offsets inside
// the grid are numbered (a degenerate grid of one row would otherwise cost k
// steps per ring).
struct SectorShape {
    int64_t gx, count;
    int32_t c0, c1, s0, s1, k, qa, na, pa;
    bool major_y;
};

__device__ __forceinline__ SectorShape sector_shape(const Grid& g, int32_t cx, int32_t cy, int32_t k, int o) {
    SectorShape S;
    const int32_t sx = (o & 4) ? -1 : 1, sy = (o & 2) ? -1 : 1;
    S.major_y = o & 1;
    S.gx = g.gx;
    S.k = k;
    // centre, extent and sign of the major (0) and minor (1) axes
    S.c0 = S.major_y ? cy : cx;
    S.s0 = S.major_y ? sy : sx;
    S.c1 = S.major_y ? cx : cy;
    S.s1 = S.major_y ? sx : sy;
    const int32_t n0 = S.major_y ? g.gy : g.gx, n1 = S.major_y ? g.gx : g.gy;
    // signed offsets t with c + s t inside [0, n): t in [lo, hi], lo <= 0 <= hi
    auto lo = [](int32_t c, int32_t n, int32_t s) { return s > 0 ? -c : c - (n - 1); };
    auto hi = [](int32_t c, int32_t n, int32_t s) { return s > 0 ? n - 1 - c : c; };
    S.qa = max(-1, lo(S.c1, n1, S.s1));
    S.na = k <= hi(S.c0, n0, S.s0) ? max(min(k, hi(S.c1, n1, S.s1)) - S.qa + 1, 0) : 0;
    S.pa = max(k - 3, lo(S.c0, n0, S.s0));
    const int32_t nb = k <= hi(S.c1, n1, S.s1) ? max(min(k - 1, hi(S.c0, n0, S.s0)) - S.pa + 1, 0) : 0;
    S.count = (int64_t)S.na + nb;
    return S;
}

__device__ __forceinline__ int64_t sector_cell(const SectorShape& S, int64_t i) {
    const int32_t pp = i < S.na ? S.k : S.pa + (int32_t)(i - S.na);
    const int32_t qq = i < S.na ? S.qa + (int32_t)i : S.k;
    const int64_t a = S.c0 + S.s0 * pp, b = S.c1 + S.s1 * qq;
    return S.major_y ? a * S.gx + b : b * S.gx + a;
}

// Full ring, or only the sectors of the octants in `open` when that visits
// fewer cells (k + 5 per octant against 8k).
__device__ __forceinline__ bool use_full_ring(int32_t k, unsigned open) {
    return k <= 3 || (int32_t)__popc(open) * (k + 5) >= 8 * k;
}

__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// Gabriel degree of point iu.  Rings of cells around u find the nearest
// point of each 45-degree octant until the octant is settled; a second walk
// over the same rings (or sectors) tests every point of an octant that is
// not blocked.  WAVE: the lanes of a wavefront take the cells of each ring in
// turn (all lanes call this for the same point and get the same result);
// otherwise one thread does it all and gives up (returns -1) once it has
// visited more than `budget` cells and points.  box = (xmin, xmax, ymin, ymax).
template <bool WAVE>
__device__ int32_t gabriel_degree_of(int32_t iu, const Grid& g, const int64_t* __restrict__ start,
                                     const int32_t* __restrict__ pts, const float2* __restrict__ p,
                                     float cell, float4 box, int64_t budget) {
    const int lane = WAVE ? lane64() : 0;
    const int stride = WAVE ? 64 : 1;
    Work work;
    const float2 u = p[iu];
    const int32_t cx = cell_x(g, u.x), cy = cell_y(g, u.y);
    // reach[o]: the largest squared distance from u to a point of the
    // bounding box in octant o (its wedge is bounded by the box edges A
    // along x and B along y; the far corner of the wedge's part inside is at
    // (A, min(A, B)) or (min(A, B), B))
    double reach[8], best[8];
    int32_t ko[8];
    for (int o = 0; o < 8; ++o) {
        const double A = (o & 4) ? (double)u.x - box.x : (double)box.y - u.x;
        const double B = (o & 2) ? (double)u.y - box.z : (double)box.w - u.y;
        const double mn = fmin(A, B);
        reach[o] = ((o & 1) ? B * B : A * A) + mn * mn;
        // an octant that needs dx < 0 (dy < 0) with u on the box's left
        // (lower) edge holds no point at all
        if (((o & 4) && A == 0.0) || ((o & 2) && B == 0.0)) reach[o] = 0.0;
        best[o] = INFINITY;
        ko[o] = 0;
    }
    // f(cell, octant) for this thread's (lane's) cells of ring k: the whole
    // ring (octant -1) or the sectors of the octants in `open`
    auto each_cell = [&](int32_t k, unsigned open, auto&& f) {
        if (use_full_ring(k, open)) {
            const RingShape R = ring_shape(g, cx, cy, k, 0, g.gx - 1, 0, g.gy - 1);
            for (int64_t i = lane; i < R.count; i += stride) f(ring_cell(R, i), -1);
        } else {
            for (int o = 0; o < 8; ++o) {
                if (!(open >> o & 1)) continue;
                const SectorShape S = sector_shape(g, cx, cy, k, o);
                for (int64_t i = lane; i < S.count; i += stride) f(sector_cell(S, i), o);
            }
        }
    };
    // rings beyond kmax lie entirely outside the grid
    const int32_t kmax = max(max(cx, g.gx - 1 - cx), max(cy, g.gy - 1 - cy));
    unsigned open = 0xFFu;  // octants not yet settled
    for (int32_t k = 0; open; ++k) {
        each_cell(k, open, [&](int64_t c, int) {
            ++work.n;
            for (int64_t q = start[c]; q < start[c + 1]; ++q) {
                ++work.n;
                const int32_t w = pts[q];
                if (w == iu) continue;
                const double dx = (double)p[w].x - (double)u.x, dy = (double)p[w].y - (double)u.y;
                const double r2 = dx * dx + dy * dy;
                if (r2 <= 0.0) continue;  // a coincident point has no direction
                const int o = octant(dx, dy);
                best[o] = r2 < best[o] ? r2 : best[o];
            }
        });
        if (WAVE)
            for (int o = 0; o < 8; ++o) best[o] = wave_min_d(best[o]);
        else if (work.n > budget)
            return -1;
        // every point of an octant visited so far within (k - 2) cells' width
        // of u has been seen (a cell index computed in float can be one off);
        // an octant is settled at ring ko once that covers twice its nearest
        // squared distance (beyond, its points are blocked) or, with no point
        // found, its reach (it has none)
        const double cover = k >= 2 ? (double)(k - 2) * (double)cell : 0.0;
        for (int o = 0; o < 8; ++o) {
            if (!(open >> o & 1)) continue;
            const double need = (best[o] < INFINITY ? 2.0 * best[o] : reach[o]) * (1.0 + 1e-9);
            if ((k >= 2 && need <= cover * cover) || k >= kmax) {
                ko[o] = k;
                open &= ~(1u << o);
            }
        }
    }
    int32_t K = 0;
    for (int o = 0; o < 8; ++o) K = max(K, ko[o]);
    // candidates: points of octant o on rings up to ko[o] that are not blocked
    int32_t deg = 0;
    bool over = false;
    for (int32_t k = 0; k <= K && !over; ++k) {
        unsigned live = 0;
        for (int o = 0; o < 8; ++o) live |= (ko[o] >= k ? 1u : 0u) << o;
        each_cell(k, live, [&](int64_t c, int only) {
            if (!WAVE && (over = over || work.n > budget)) return;
            ++work.n;
            for (int64_t q = start[c]; q < start[c + 1]; ++q) {
                ++work.n;
                const int32_t iv = pts[q];
                if (iv == iu) continue;
                const double dx = (double)p[iv].x - (double)u.x, dy = (double)p[iv].y - (double)u.y;
                const double r2 = dx * dx + dy * dy;
                const int o = octant(dx, dy);
                if (r2 > 0.0) {
                    if (only >= 0 ? o != only : !(live >> o & 1)) continue;
                    if (r2 >= 2.0 * best[o] * (1.0 + 1e-9)) continue;  // blocked
                } else if (only > 0) {
                    continue;  // a coincident point is taken once, with octant 0
                }
                deg += gabriel_pair_dev(g, start, pts, p, iu, iv, work) ? 1 : 0;
            }
        });
    }
    if (WAVE) return wave_sum(deg);
    return over ? -1 : deg;
}

// Thread per point (in cell order: a wavefront's points are neighbours); a
// point whose search exceeds the budget is listed in hard[] for
// gabriel_wave_kernel instead.  At most 128 VGPRs, so that four waves per
// SIMD hold every point of a 262k-point drawing at once (the walks are
// latency-bound: 14.4 ms against 18.2 ms at 137 VGPRs and three waves).
__global__ __launch_bounds__(kBlock, 4) void gabriel_degree_kernel(int32_t n, Grid g,
                                                                const int64_t* __restrict__ start,
                                                                const int32_t* __restrict__ pts,
                                                                const float2* __restrict__ p,
                                                                float cell, float4 box, int64_t budget,
                                                                int32_t* __restrict__ gdeg,
                                                                int32_t* __restrict__ hard,
                                                                int32_t* __restrict__ hard_count) {
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * kBlock) {
        const int32_t iu = pts[t];
        const int32_t deg = gabriel_degree_of<false>(iu, g, start, pts, p, cell, box, budget);
        if (deg >= 0)
            gdeg[iu] = deg;
        else
            hard[atomicAdd(hard_count, 1)] = iu;
    }
}

// Wavefront per listed point (at most 128 VGPRs, as above).
__global__ __launch_bounds__(kBlock, 4) void gabriel_wave_kernel(Grid g, const int64_t* __restrict__ start,
                                                              const int32_t* __restrict__ pts,
                                                              const float2* __restrict__ p, float cell,
                                                              float4 box, const int32_t* __restrict__ hard,
                                                              const int32_t* __restrict__ hard_count,
                                                              int32_t* __restrict__ gdeg) {
    const int32_t count = *hard_count;
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    for (int64_t i = (int64_t)blockIdx.x * kWaves + wave_id(); i < count; i += waves) {
        const int32_t iu = hard[i];
        const int32_t deg = gabriel_degree_of<true>(iu, g, start, pts, p, cell, box, 0);
        if (lane64() == 0) gdeg[iu] = deg;
    }
}

// Gabriel test of every adjacency entry: inter[v] = graph neighbours of v
// that are Gabriel neighbours.
__global__ __launch_bounds__(kBlock) void gabriel_edge_kernel(int32_t n, Grid g,
                                                              const int64_t* __restrict__ start,
                                                              const int32_t* __restrict__ pts,
                                                              const float2* __restrict__ p,
                                                              const int64_t* __restrict__ rp,
                                                              const int32_t* __restrict__ ci,
                                                              int32_t* __restrict__ inter) {
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    for (int64_t v = (int64_t)blockIdx.x * kWaves + wave_id(); v < n; v += waves) {
        int32_t c = 0;
        Work work;
        for (int64_t e = rp[v] + lane64(); e < rp[v + 1]; e += 64)
            c += gabriel_pair_dev(g, start, pts, p, (int32_t)v, ci[e], work) ? 1 : 0;
        c = wave_sum(c);
        if (lane64() == 0) inter[v] = c;
    }
}

__global__ __launch_bounds__(kBlock) void jaccard_kernel(int32_t n, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ gdeg,
                                                         const int32_t* __restrict__ inter,
                                                         double* __restrict__ jac,
                                                         double* __restrict__ partial,
                                                         unsigned long long* __restrict__ gsum) {
    __shared__ double s[kWaves];
    double acc = 0.0;
    unsigned long long ge = 0;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const int64_t both = inter[v];
        const int64_t uni = (rp[v + 1] - rp[v]) + gdeg[v] - both;
        const double J = uni == 0 ? 1.0 : (double)both / (double)uni;
        if (jac) jac[v] = J;
        acc += J;
        ge += (unsigned long long)gdeg[v];
    }
    const double t = block_sum(acc, s);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
    const unsigned long long w = wave_sum(ge);
    if (lane64() == 0 && w) atomicAdd(gsum, w);
}

// Sum of partial[0 .. count) in a fixed order (the same bits on every run):
// thread t adds partial[t], partial[t + 256], ... in turn, then a fixed tree.
__global__ __launch_bounds__(kBlock) void ordered_sum_kernel(int32_t count, const double* __restrict__ partial,
                                                             double* __restrict__ out) {
    __shared__ double s_v[kBlock];
    double a = 0.0;
    for (int32_t i = threadIdx.x; i < count; i += kBlock) a += partial[i];
    s_v[threadIdx.x] = a;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s_v[threadIdx.x] += s_v[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s_v[0];
}

template <class V>
static int drawing_metrics(const gila_csr* g, const V* pos, int32_t what, hipStream_t s,
                           gila_metrics* out, int64_t* edge_crossings, double* jaccard) {
    const int32_t n = g->n;
    *out = gila_metrics{};
    out->similarity = 1.0;
    if (n == 0) return GILA_OK;
    MBuf pf(s), first(s), cnt(s), eo(s), ends(s), ws(s);
    GILA_TRY(pf.alloc<float2>((size_t)n));
    hipLaunchKernelGGL(to_float_kernel<V>, dim3(mgrid(n)), dim3(kBlock), 0, s, n, pos, pf.as<float2>());
    GILA_HIP(hipGetLastError());
    // bounding box (finite coordinates only)
    MBuf box(s);
    GILA_TRY(box.alloc<unsigned int>(4));
    GILA_HIP(hipMemsetAsync(box.p, 0xFF, 4 * sizeof(unsigned int), s));
    hipLaunchKernelGGL(bounds_kernel, dim3(mgrid(n)), dim3(kBlock), 0, s, n, pf.as<float2>(),
                       box.as<unsigned int>());
    GILA_HIP(hipGetLastError());
    unsigned int hb[4];
    GILA_HIP(hipMemcpyAsync(hb, box.p, sizeof(hb), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    auto val = [](unsigned int k) {
        const unsigned int u = (k >> 31) ? (k & 0x7FFFFFFFu) : ~k;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    };
    const float xmin = val(hb[0]), ymin = val(hb[1]), xmax = -val(hb[2]), ymax = -val(hb[3]);
    if (!std::isfinite(xmin) || !std::isfinite(xmax) || !std::isfinite(ymin) || !std::isfinite(ymax))
        return fail(GILA_EINVAL, "positions must be finite");
    const double M = std::max(std::max(std::fabs((double)xmin), std::fabs((double)xmax)),
                              std::max(std::fabs((double)ymin), std::fabs((double)ymax)));
    // edge list
    GILA_TRY(first.alloc<int64_t>((size_t)n));
    GILA_TRY(cnt.alloc<int64_t>((size_t)n));
    GILA_TRY(eo.alloc<int64_t>((size_t)n + 1));
    GILA_TRY(ws.alloc<int64_t>((size_t)scan_workspace_count(n)));
    hipLaunchKernelGGL(upper_count_kernel, dim3(mgrid(n)), dim3(kBlock), 0, s, n, g->row_ptr,
                       g->col_idx, first.as<int64_t>(), cnt.as<int64_t>());
    GILA_HIP(hipGetLastError());
    GILA_TRY(enqueue_exclusive_scan_i64(cnt.as<int64_t>(), eo.as<int64_t>(), n, ws.as<int64_t>(), s));
    int64_t m = 0;
    GILA_HIP(hipMemcpyAsync(&m, eo.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    GILA_TRY(ends.alloc<int2>((size_t)std::max<int64_t>(m, 1)));
    const int rgrid = (int)std::max<int64_t>(1, std::min<int64_t>(16384, ((int64_t)n + kWaves - 1) / kWaves));
    hipLaunchKernelGGL(edge_list_kernel, dim3(rgrid), dim3(kBlock), 0, s, n, g->row_ptr, g->col_idx,
                       first.as<int64_t>(), eo.as<int64_t>(), ends.as<int2>());
    GILA_HIP(hipGetLastError());
    if ((what & GILA_METRIC_CROSSINGS) && m > 0) {
        MBuf tot(s);
        GILA_TRY(tot.alloc<unsigned long long>(1));
        GILA_HIP(hipMemsetAsync(tot.p, 0, sizeof(unsigned long long), s));
        // chunks of at least kCrossChunk edges, few enough for the grid's y extent
        int64_t chunk = std::max<int64_t>(kCrossChunk, (m + 65534) / 65535);
        chunk = (chunk + kCrossTile - 1) / kCrossTile * kCrossTile;
        const dim3 grid((unsigned)((m + kCrossBlock - 1) / kCrossBlock), (unsigned)((m + chunk - 1) / chunk));
        if (edge_crossings) {
            GILA_HIP(hipMemsetAsync(edge_crossings, 0, sizeof(int64_t) * (size_t)m, s));
            hipLaunchKernelGGL(crossings_kernel<false>, grid, dim3(kCrossTile), 0, s, m, chunk, M,
                               ends.as<int2>(), pf.as<float2>(),
                               reinterpret_cast<unsigned long long*>(edge_crossings),
                               tot.as<unsigned long long>());
        } else {
            hipLaunchKernelGGL(crossings_kernel<true>, grid, dim3(kCrossTile), 0, s, m, chunk, M,
                               ends.as<int2>(), pf.as<float2>(), nullptr, tot.as<unsigned long long>());
        }
        GILA_HIP(hipGetLastError());
        unsigned long long t = 0;
        GILA_HIP(hipMemcpyAsync(&t, tot.p, sizeof(t), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        out->crossings = (int64_t)(edge_crossings ? t / 2 : t);
    }
    if ((what & GILA_METRIC_LENGTHS) && m > 0) {
        const int lg = mgrid(m);
        MBuf part(s), sum(s);
        GILA_TRY(part.alloc<double>((size_t)lg));
        GILA_TRY(sum.alloc<double>(1));
        double tot = 0.0;
        hipLaunchKernelGGL(lengths_sum_kernel, dim3(lg), dim3(kBlock), 0, s, m, ends.as<int2>(),
                           pf.as<float2>(), 0.0, 0, part.as<double>());
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(kBlock), 0, s, lg, part.as<double>(), sum.as<double>());
        GILA_HIP(hipMemcpyAsync(&tot, sum.p, sizeof(double), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        const double mean = tot / (double)m;
        hipLaunchKernelGGL(lengths_sum_kernel, dim3(lg), dim3(kBlock), 0, s, m, ends.as<int2>(),
                           pf.as<float2>(), mean, 1, part.as<double>());
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(kBlock), 0, s, lg, part.as<double>(), sum.as<double>());
        GILA_HIP(hipMemcpyAsync(&tot, sum.p, sizeof(double), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        out->edge_length_mean = mean;
        out->edge_length_std = std::sqrt(tot / (double)m);
    }
    if (what & GILA_METRIC_SIMILARITY) {
        // grid of about two points per cell over the bounding box
        const double w = std::max(1e-30, (double)xmax - (double)xmin);
        const double h = std::max(1e-30, (double)ymax - (double)ymin);
        double cell = std::sqrt(2.0 * w * h / (double)n);
        cell = std::max(cell, std::max(w, h) / 65536.0);
        cell = std::max(cell, 1e-30);
        Grid gr;
        gr.x0 = xmin;
        gr.y0 = ymin;
        gr.gx = (int32_t)std::min(65536.0, std::floor(w / cell) + 1);
        gr.gy = (int32_t)std::min(65536.0, std::floor(h / cell) + 1);
        gr.inv = (float)(1.0 / cell);
        const int64_t G = (int64_t)gr.gx * gr.gy;
        MBuf cellof(s), ccnt(s), cstart(s), cur(s), pts(s), gdeg(s), inter(s), part(s), sum(s), gs(s),
            ws2(s);
        GILA_TRY(cellof.alloc<int32_t>((size_t)n));
        GILA_TRY(ccnt.alloc<int64_t>((size_t)G));
        GILA_TRY(cstart.alloc<int64_t>((size_t)G + 1));
        GILA_TRY(cur.alloc<unsigned long long>((size_t)G));
        GILA_TRY(pts.alloc<int32_t>((size_t)n));
        GILA_TRY(gdeg.alloc<int32_t>((size_t)n));
        GILA_TRY(inter.alloc<int32_t>((size_t)n));
        GILA_TRY(ws2.alloc<int64_t>((size_t)scan_workspace_count(G)));
        GILA_HIP(hipMemsetAsync(ccnt.p, 0, sizeof(int64_t) * G, s));
        GILA_HIP(hipMemsetAsync(cur.p, 0, sizeof(unsigned long long) * G, s));
        hipLaunchKernelGGL(cell_count_kernel, dim3(mgrid(n)), dim3(kBlock), 0, s, n, gr, pf.as<float2>(),
                           cellof.as<int32_t>(), ccnt.as<int64_t>());
        GILA_HIP(hipGetLastError());
        GILA_TRY(enqueue_exclusive_scan_i64(ccnt.as<int64_t>(), cstart.as<int64_t>(), G,
                                            ws2.as<int64_t>(), s));
        hipLaunchKernelGGL(cell_fill_kernel, dim3(mgrid(n)), dim3(kBlock), 0, s, n, cellof.as<int32_t>(),
                           cstart.as<int64_t>(), cur.as<unsigned long long>(), pts.as<int32_t>());
        // a point whose search visits more cells and points than this goes
        // to a wavefront of its own (GILA_GABRIEL_BUDGET overrides; 0 sends
        // every point there)
        int64_t budget = kGabrielBudget;
        if (const char* e = getenv("GILA_GABRIEL_BUDGET")) budget = std::max<int64_t>(0, std::atoll(e));
        MBuf hard(s), hcount(s);
        GILA_TRY(hard.alloc<int32_t>((size_t)n));
        GILA_TRY(hcount.alloc<int32_t>(1));
        GILA_HIP(hipMemsetAsync(hcount.p, 0, sizeof(int32_t), s));
        const float4 fbox = make_float4(xmin, xmax, ymin, ymax);
        hipLaunchKernelGGL(gabriel_degree_kernel, dim3(mgrid(n)), dim3(kBlock), 0, s, n, gr,
                           cstart.as<int64_t>(), pts.as<int32_t>(), pf.as<float2>(), (float)cell, fbox,
                           budget, gdeg.as<int32_t>(), hard.as<int32_t>(), hcount.as<int32_t>());
        hipLaunchKernelGGL(gabriel_wave_kernel, dim3(mgrid((int64_t)n * 64)), dim3(kBlock), 0, s, gr,
                           cstart.as<int64_t>(), pts.as<int32_t>(), pf.as<float2>(), (float)cell, fbox,
                           hard.as<int32_t>(), hcount.as<int32_t>(), gdeg.as<int32_t>());
        hipLaunchKernelGGL(gabriel_edge_kernel, dim3(rgrid), dim3(kBlock), 0, s, n, gr,
                           cstart.as<int64_t>(), pts.as<int32_t>(), pf.as<float2>(), g->row_ptr,
                           g->col_idx, inter.as<int32_t>());
        GILA_HIP(hipGetLastError());
        const int jg = mgrid(n);
        GILA_TRY(part.alloc<double>((size_t)jg));
        GILA_TRY(sum.alloc<double>(1));
        GILA_TRY(gs.alloc<unsigned long long>(1));
        GILA_HIP(hipMemsetAsync(gs.p, 0, sizeof(unsigned long long), s));
        hipLaunchKernelGGL(jaccard_kernel, dim3(jg), dim3(kBlock), 0, s, n, g->row_ptr, gdeg.as<int32_t>(),
                           inter.as<int32_t>(), jaccard, part.as<double>(), gs.as<unsigned long long>());
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(kBlock), 0, s, jg, part.as<double>(), sum.as<double>());
        GILA_HIP(hipGetLastError());
        double tot = 0.0;
        unsigned long long ge = 0;
        GILA_HIP(hipMemcpyAsync(&tot, sum.p, sizeof(double), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipMemcpyAsync(&ge, gs.p, sizeof(ge), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        out->similarity = tot / (double)n;
        out->gabriel_edges = (int64_t)(ge / 2);
    }
    out->edges = m;
    GILA_HIP(hipStreamSynchronize(s));
    return GILA_OK;
}

}  // namespace gila

using namespace gila;

extern "C" {

int gila_drawing_metrics(const gila_csr* g_dev, int32_t precision, const void* pos_dev,
                         int32_t what, void* stream, gila_metrics* out,
                         int64_t* edge_crossings_dev, double* jaccard_dev) {
    TraceRange trace_range("gila_drawing_metrics");
    clear_error();
    if (!out) return fail(GILA_EINVAL, "out is NULL");
    if (precision != GILA_FP64 && precision != GILA_FP32 && precision != GILA_FP32_KAHAN)
        return fail(GILA_EINVAL, "unknown precision %d", precision);
    hipStream_t s = (hipStream_t)stream;
    GILA_TRY(validate_graph(g_dev, s));
    if (g_dev->n > 0 && !pos_dev) return fail(GILA_EINVAL, "pos_dev is NULL");
    if (precision == GILA_FP64)
        return drawing_metrics<double2>(g_dev, (const double2*)pos_dev, what, s, out,
                                        edge_crossings_dev, jaccard_dev);
    return drawing_metrics<float2>(g_dev, (const float2*)pos_dev, what, s, out, edge_crossings_dev,
                                   jaccard_dev);
}

}  // extern "C"

// Drawing-quality metrics (Section 5.2): edge crossings, the standard
// deviation of edge lengths, and the similarity of the drawing's Gabriel
// graph to the graph (mean Jaccard index of the neighbourhoods).
//
// Coordinates are taken at single precision.  Differences of two floats and
// products of two such differences are exact in double, and a correctly
// rounded subtraction or sum of two exact doubles keeps its sign, so the
// orientation and in-disc tests below have exact signs (whether or not the
// compiler fuses a multiply into the subtraction).
//
//   edge_list_kernel      edges {u, v}, u < v, in row order (the part of a
//                         sorted row above v is a suffix found by bisection)
//   crossings_kernel      thread per edge, all other edges streamed through
//                         LDS in tiles; an exact bounding-box reject, then
//                         four orientation signs; per-edge counts
//   lengths kernels       per-edge length, fixed-order sums (mean, then the
//                         squared deviations)
//   grid kernels          points binned into a uniform grid (about two per
//                         cell)
//   gabriel_degree_kernel thread per point u: rings of cells around u until,
//                         in each of the eight 45-degree octants around u,
//                         the nearest point w found so far blocks everything
//                         at squared distance >= 2 |w - u|^2 (such a v sees w
//                         within 45 degrees of its own direction, so w lies in
//                         the disc with diameter uv) and the rings cover that
//                         far; then every point not excluded that way is
//                         tested for an empty disc with diameter uv
//   gabriel_edge_kernel   the same disc test for each graph edge (for the
//                         Jaccard intersections)
#include <algorithm>
#include <cmath>
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

constexpr int kCrossTile = 256;  // edges per LDS tile of the crossing kernel

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

// ------------------------------------------------------------------ crossings
__device__ __forceinline__ int orient_sign(float ax, float ay, float bx, float by, float cx,
                                           float cy) {
    const double l = ((double)bx - (double)ax) * ((double)cy - (double)ay);
    const double r = ((double)by - (double)ay) * ((double)cx - (double)ax);
    const double d = l - r;
    return (d > 0.0) - (d < 0.0);
}

struct Seg {
    float x0, y0, x1, y1;
};

__global__ __launch_bounds__(kCrossTile) void crossings_kernel(int64_t m, const int2* __restrict__ ends,
                                                               const float2* __restrict__ p,
                                                               int64_t* __restrict__ per_edge,
                                                               unsigned long long* __restrict__ total) {
    __shared__ Seg s_seg[kCrossTile];
    __shared__ float4 s_box[kCrossTile];  // xmin, xmax, ymin, ymax
    __shared__ int2 s_end[kCrossTile];
    const int64_t i = (int64_t)blockIdx.x * kCrossTile + threadIdx.x;
    const bool live = i < m;
    int2 ei = make_int2(-1, -1);
    Seg a{0.f, 0.f, 0.f, 0.f};
    if (live) {
        ei = ends[i];
        const float2 pa = p[ei.x], pb = p[ei.y];
        a = Seg{pa.x, pa.y, pb.x, pb.y};
    }
    const float axmin = fminf(a.x0, a.x1), axmax = fmaxf(a.x0, a.x1);
    const float aymin = fminf(a.y0, a.y1), aymax = fmaxf(a.y0, a.y1);
    int64_t count = 0;
    for (int64_t t0 = 0; t0 < m; t0 += kCrossTile) {
        const int64_t j = t0 + threadIdx.x;
        if (j < m) {
            const int2 e = ends[j];
            const float2 pc = p[e.x], pd = p[e.y];
            s_seg[threadIdx.x] = Seg{pc.x, pc.y, pd.x, pd.y};
            s_box[threadIdx.x] = make_float4(fminf(pc.x, pd.x), fmaxf(pc.x, pd.x), fminf(pc.y, pd.y),
                                             fmaxf(pc.y, pd.y));
            s_end[threadIdx.x] = e;
        }
        __syncthreads();
        const int tn = (int)(m - t0 < kCrossTile ? m - t0 : kCrossTile);
        if (live) {
            for (int q = 0; q < tn; ++q) {
                const float4 b = s_box[q];
                // a proper crossing lies inside both closed boxes
                if (b.x > axmax || axmin > b.y || b.z > aymax || aymin > b.w) continue;
                const int2 e = s_end[q];
                if (e.x == ei.x || e.x == ei.y || e.y == ei.x || e.y == ei.y) continue;  // shared end or itself
                const Seg c = s_seg[q];
                const int o1 = orient_sign(a.x0, a.y0, a.x1, a.y1, c.x0, c.y0);
                const int o2 = orient_sign(a.x0, a.y0, a.x1, a.y1, c.x1, c.y1);
                if (o1 * o2 >= 0) continue;
                const int o3 = orient_sign(c.x0, c.y0, c.x1, c.y1, a.x0, a.y0);
                const int o4 = orient_sign(c.x0, c.y0, c.x1, c.y1, a.x1, a.y1);
                count += o3 * o4 < 0 ? 1 : 0;
            }
        }
        __syncthreads();
    }
    if (live && per_edge) per_edge[i] = count;
    const int64_t w = wave_sum(count);
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
    for (int c = 0; c < 4; ++c) atomicMin(&box[c], k[c]);
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

// w lies in the closed disc with diameter uv: (w - u).(w - v) <= 0 (exact sign)
__device__ __forceinline__ bool in_disc(float2 u, float2 v, float2 w) {
    const double a = ((double)w.x - (double)u.x) * ((double)w.x - (double)v.x);
    const double b = ((double)w.y - (double)u.y) * ((double)w.y - (double)v.y);
    return a + b <= 0.0;
}

// No point other than iu, iv in the closed disc with diameter uv.
__device__ bool gabriel_pair_dev(const Grid& g, const int64_t* __restrict__ start,
                                 const int32_t* __restrict__ pts, const float2* __restrict__ p,
                                 int32_t iu, int32_t iv) {
    const float2 u = p[iu], v = p[iv];
    const float cx = 0.5f * (u.x + v.x), cy = 0.5f * (u.y + v.y);
    const double dx = (double)v.x - (double)u.x, dy = (double)v.y - (double)u.y;
    // half the diameter, rounded up, plus one cell either way against rounding
    const float r = (float)(0.5 * sqrt(dx * dx + dy * dy)) * 1.0001f + 1e-30f;
    const int32_t x0 = max(cell_x(g, cx - r) - 1, 0), x1 = min(cell_x(g, cx + r) + 1, g.gx - 1);
    const int32_t y0 = max(cell_y(g, cy - r) - 1, 0), y1 = min(cell_y(g, cy + r) + 1, g.gy - 1);
    for (int32_t y = y0; y <= y1; ++y)
        for (int32_t x = x0; x <= x1; ++x) {
            const int64_t c = (int64_t)y * g.gx + x;
            for (int64_t k = start[c]; k < start[c + 1]; ++k) {
                const int32_t w = pts[k];
                if (w == iu || w == iv) continue;
                if (in_disc(u, v, p[w])) return false;
            }
        }
    return true;
}

// octant of the direction (dx, dy), from signs and |dx| vs |dy| only
__device__ __forceinline__ int octant(double dx, double dy) {
    return (dx < 0.0 ? 4 : 0) + (dy < 0.0 ? 2 : 0) + (fabs(dx) < fabs(dy) ? 1 : 0);
}

// Visit the points of the cells at Chebyshev distance exactly k from (cx, cy)
// (rows and columns clamped to the grid, so a ring costs its cells inside).
template <class F>
__device__ __forceinline__ void ring_points(const Grid& g, const int64_t* __restrict__ start,
                                            const int32_t* __restrict__ pts, int32_t cx,
                                            int32_t cy, int32_t k, F&& f) {
    auto cell_points = [&](int32_t x, int32_t y) {
        const int64_t c = (int64_t)y * g.gx + x;
        for (int64_t q = start[c]; q < start[c + 1]; ++q) f(pts[q]);
    };
    const int32_t y0 = max(cy - k, 0), y1 = min(cy + k, g.gy - 1);
    const int32_t x0 = max(cx - k, 0), x1 = min(cx + k, g.gx - 1);
    for (int32_t y = y0; y <= y1; ++y) {
        if (y == cy - k || y == cy + k) {
            for (int32_t x = x0; x <= x1; ++x) cell_points(x, y);
        } else {
            if (cx - k >= 0) cell_points(cx - k, y);
            if (cx + k < g.gx) cell_points(cx + k, y);
        }
    }
}

__global__ __launch_bounds__(kBlock) void gabriel_degree_kernel(int32_t n, Grid g,
                                                                const int64_t* __restrict__ start,
                                                                const int32_t* __restrict__ pts,
                                                                const float2* __restrict__ p,
                                                                float cell, int32_t* __restrict__ gdeg) {
    for (int64_t iu = (int64_t)blockIdx.x * kBlock + threadIdx.x; iu < n;
         iu += (int64_t)gridDim.x * kBlock) {
        const float2 u = p[iu];
        const int32_t cx = cell_x(g, u.x), cy = cell_y(g, u.y);
        double best[8];
        for (int o = 0; o < 8; ++o) best[o] = INFINITY;
        // rings beyond kmax lie entirely outside the grid
        const int32_t kmax = max(max(cx, g.gx - 1 - cx), max(cy, g.gy - 1 - cy));
        int32_t K = 0;
        for (int32_t k = 0;; ++k) {
            ring_points(g, start, pts, cx, cy, k, [&](int32_t w) {
                if (w == iu) return;
                const double dx = (double)p[w].x - (double)u.x, dy = (double)p[w].y - (double)u.y;
                const double r2 = dx * dx + dy * dy;
                if (r2 <= 0.0) return;  // a coincident point has no direction
                const int o = octant(dx, dy);
                best[o] = r2 < best[o] ? r2 : best[o];
            });
            K = k;
            if (k >= kmax) break;
            // every point within (k - 2) cells' width of u has been seen (a
            // cell index computed in float can be one off)
            const double cover = k >= 2 ? (double)(k - 2) * (double)cell : 0.0;
            double need = 0.0;
            for (int o = 0; o < 8; ++o) need = fmax(need, 2.0 * best[o] * (1.0 + 1e-9));
            if (k >= 2 && need <= cover * cover) break;
        }
        int32_t deg = 0;
        for (int32_t k = 0; k <= K; ++k)
            ring_points(g, start, pts, cx, cy, k, [&](int32_t iv) {
                if (iv == iu) return;
                const double dx = (double)p[iv].x - (double)u.x, dy = (double)p[iv].y - (double)u.y;
                const double r2 = dx * dx + dy * dy;
                if (r2 > 0.0 && r2 >= 2.0 * best[octant(dx, dy)] * (1.0 + 1e-9)) return;  // blocked
                deg += gabriel_pair_dev(g, start, pts, p, (int32_t)iu, iv) ? 1 : 0;
            });
        gdeg[iu] = deg;
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
        for (int64_t e = rp[v] + lane64(); e < rp[v + 1]; e += 64)
            c += gabriel_pair_dev(g, start, pts, p, (int32_t)v, ci[e]) ? 1 : 0;
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

// Sum of partial[0 .. count) in order, by one thread.
__global__ void ordered_sum_kernel(int32_t count, const double* __restrict__ partial,
                                   double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int32_t i = 0; i < count; ++i) s += partial[i];
    *out = s;
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
        hipLaunchKernelGGL(crossings_kernel, dim3((unsigned)((m + kCrossTile - 1) / kCrossTile)),
                           dim3(kCrossTile), 0, s, m, ends.as<int2>(), pf.as<float2>(), edge_crossings,
                           tot.as<unsigned long long>());
        GILA_HIP(hipGetLastError());
        unsigned long long t = 0;
        GILA_HIP(hipMemcpyAsync(&t, tot.p, sizeof(t), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        out->crossings = (int64_t)(t / 2);
    }
    if ((what & GILA_METRIC_LENGTHS) && m > 0) {
        const int lg = mgrid(m);
        MBuf part(s), sum(s);
        GILA_TRY(part.alloc<double>((size_t)lg));
        GILA_TRY(sum.alloc<double>(1));
        double tot = 0.0;
        hipLaunchKernelGGL(lengths_sum_kernel, dim3(lg), dim3(kBlock), 0, s, m, ends.as<int2>(),
                           pf.as<float2>(), 0.0, 0, part.as<double>());
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(64), 0, s, lg, part.as<double>(), sum.as<double>());
        GILA_HIP(hipMemcpyAsync(&tot, sum.p, sizeof(double), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        const double mean = tot / (double)m;
        hipLaunchKernelGGL(lengths_sum_kernel, dim3(lg), dim3(kBlock), 0, s, m, ends.as<int2>(),
                           pf.as<float2>(), mean, 1, part.as<double>());
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(64), 0, s, lg, part.as<double>(), sum.as<double>());
        GILA_HIP(hipMemcpyAsync(&tot, sum.p, sizeof(double), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        out->edge_length_mean = mean;
        out->edge_length_std = std::sqrt(tot / (double)m);
    }
    if (what & GILA_METRIC_SIMILARITY) {
        // grid of about two points per cell over the points' bounding box
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
            return fail(GILA_EINVAL, "positions must be finite for the similarity metric");
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
        hipLaunchKernelGGL(gabriel_degree_kernel, dim3(mgrid(n)), dim3(kBlock), 0, s, n, gr,
                           cstart.as<int64_t>(), pts.as<int32_t>(), pf.as<float2>(), (float)cell,
                           gdeg.as<int32_t>());
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
        hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(64), 0, s, jg, part.as<double>(), sum.as<double>());
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

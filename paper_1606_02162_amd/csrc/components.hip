// Connected components, each laid out on its own, and packing of their
// drawings (Sections 4.6 and 5.1).
//
// Labels: every vertex starts as its own root; each pass hooks, for every
// edge whose ends have different roots, the larger root under the smaller
// one (atomic minimum), then compresses every path to its root.  Parent ids
// only ever decrease, and the loop ends after a pass that hooked nothing:
// then every edge joins vertices of one tree, whose root is its smallest id.
//
// Order: a stable sort of the vertices by label groups each component
// (ascending ids inside); a stable sort of the components by decreasing size
// (ties: smaller label) gives their ranks, the order of the packing matrix.
// Vertices are renumbered component by component in rank order, so every
// component is a contiguous id range with its own CSR.
//
// Layout (gila_layout_components): each component of at least two vertices
// gets the cap sqrt((n_C / a_C) d) 0.93^h, a_C the height / width of its
// initial drawing's bounding box (1 when degenerate), and runs its own
// halting rule: components of at most kSmallComponent vertices together in
// one batched launch (FR model), larger ones one after another on the whole
// GPU.  Singletons never move.
//
// Packing: ranks fill a matrix of ceil(sqrt(C)) columns row by row; a column
// is as wide as its widest drawing, a row as tall as its tallest, with the
// gap between consecutive ones; each drawing is translated so that its
// bounding box's lower-left corner is its cell's.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "device_util.h"
#include "gila_internal.h"

namespace gila {

constexpr int32_t kSmallComponent = 2048;
constexpr int kDigitBits = 11;
constexpr int kDigits = 1 << kDigitBits;

namespace {
// Device scratch released into the block cache when its stream is done.
struct Buf {
    hipStream_t st;
    void* p = nullptr;
    explicit Buf(hipStream_t s) : st(s) {}
    ~Buf() { dfree_on(p, st); }
    template <class T>
    int alloc(size_t count) {
        return dalloc(&p, count * sizeof(T) + 64);
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

int grid_for(int64_t items) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(8192, (items + kBlock - 1) / kBlock));
}
}  // namespace

// ------------------------------------------------------------------ labels
__global__ __launch_bounds__(kBlock) void cc_init_kernel(int32_t n, int32_t* parent) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        parent[v] = (int32_t)v;
}

__device__ __forceinline__ int32_t cc_root(const int32_t* parent, int32_t x) {
    int32_t p = parent[x];
    while (p != x) {
        x = p;
        p = parent[x];
    }
    return x;
}

// Wavefront per vertex v; every edge {u, v} with u < v once.
__global__ __launch_bounds__(kBlock) void cc_hook_kernel(int32_t n, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         int32_t* parent, int32_t* changed) {
    const int lane = lane64();
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    bool hooked = false;
    for (int64_t v = (int64_t)blockIdx.x * kWaves + wave_id(); v < n; v += waves) {
        const int64_t re = rp[v + 1];
        for (int64_t e = rp[v] + lane; e < re; e += 64) {
            const int32_t u = ci[e];
            if (u >= v) break;  // rows ascend: the rest of this lane's entries are larger
            const int32_t ru = cc_root(parent, u), rv = cc_root(parent, (int32_t)v);
            if (ru != rv) {
                atomicMin(&parent[ru > rv ? ru : rv], ru < rv ? ru : rv);
                hooked = true;
            }
        }
    }
    if (__ballot(hooked) && lane == 0) atomicOr(changed, 1);
}

__global__ __launch_bounds__(kBlock) void cc_compress_kernel(int32_t n, int32_t* parent) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        parent[v] = cc_root(parent, (int32_t)v);
}

// Labels of a validated graph into label (device, [n]).  Synchronises `s`
// after every pass (to read whether anything was hooked).
static int label_components(const gila_csr* g, int32_t* label, hipStream_t s) {
    const int32_t n = g->n;
    if (n == 0) return GILA_OK;
    hipLaunchKernelGGL(cc_init_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, label);
    GILA_HIP(hipGetLastError());
    if (g->nnz == 0) return GILA_OK;
    Buf flag(s);
    GILA_TRY(flag.alloc<int32_t>(1));
    const int hgrid = (int)std::max<int64_t>(1, std::min<int64_t>(16384, ((int64_t)n + kWaves - 1) / kWaves));
    for (int pass = 0;; ++pass) {
        if (pass > 4096) return fail(GILA_EDEVICE, "component labels did not settle");
        GILA_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(cc_hook_kernel, dim3(hgrid), dim3(kBlock), 0, s, n, g->row_ptr,
                           g->col_idx, label, flag.as<int32_t>());
        hipLaunchKernelGGL(cc_compress_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, label);
        GILA_HIP(hipGetLastError());
        int32_t changed = 0;
        GILA_HIP(hipMemcpyAsync(&changed, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        if (!changed) break;
    }
    return GILA_OK;
}

// ------------------------------------------------------------------ stable sort by key
__global__ __launch_bounds__(kBlock) void iota_kernel(int64_t count, int32_t* out) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * kBlock)
        out[i] = (int32_t)i;
}

// Per-tile histogram of the digit (key >> shift) & (kDigits - 1) of the
// elements perm[j], stored digit-major so that its exclusive prefix sum is
// the first output position of every (digit, tile).
__global__ __launch_bounds__(kBlock) void digit_hist_kernel(int64_t T, int64_t tj, int64_t ntiles,
                                                            const int32_t* __restrict__ key,
                                                            const int32_t* __restrict__ perm,
                                                            int shift, int64_t* __restrict__ hist) {
    __shared__ int32_t s_cnt[kDigits];
    for (int s = threadIdx.x; s < kDigits; s += kBlock) s_cnt[s] = 0;
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * tj;
    const int64_t j1 = j0 + tj < T ? j0 + tj : T;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kBlock)
        atomicAdd(&s_cnt[(key[perm[j]] >> shift) & (kDigits - 1)], 1);
    __syncthreads();
    for (int s = threadIdx.x; s < kDigits; s += kBlock) hist[(int64_t)s * ntiles + blockIdx.x] = s_cnt[s];
}

// One wavefront per tile walks it in order, 64 elements at a time; equal
// digits within a step are ranked by lane, so equal keys keep their order.
__global__ __launch_bounds__(64) void digit_scatter_kernel(int64_t T, int64_t tj, int64_t ntiles,
                                                           const int32_t* __restrict__ key,
                                                           const int32_t* __restrict__ perm,
                                                           int shift, const int64_t* __restrict__ base,
                                                           int32_t* __restrict__ out) {
    __shared__ int64_t s_next[kDigits];
    const int lane = threadIdx.x;
    for (int s = lane; s < kDigits; s += 64) s_next[s] = base[(int64_t)s * ntiles + blockIdx.x];
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * tj;
    const int64_t j1 = j0 + tj < T ? j0 + tj : T;
    for (int64_t c = j0; c < j1; c += 64) {
        const int64_t j = c + lane;
        const bool valid = j < j1;
        const int32_t e = valid ? perm[j] : 0;
        const int32_t dg = valid ? (key[e] >> shift) & (kDigits - 1) : -1;
        int rank = 0, same = 0;
        for (int l = 0; l < 64; ++l) {
            const int32_t dl = __builtin_amdgcn_readlane(dg, l);
            same += dl == dg ? 1 : 0;
            rank += (dl == dg && l < lane) ? 1 : 0;
        }
        const int64_t at = valid ? s_next[dg] : 0;
        __syncthreads();
        if (valid) {
            out[at + rank] = e;
            if (rank == same - 1) s_next[dg] = at + same;
        }
        __syncthreads();
    }
}

// perm_out[i] = the element at sorted position i of 0 .. T-1 ordered by
// key[element] (0 <= key <= kmax), ties in element order.
static int stable_sort_by_key(const int32_t* key, int64_t T, int32_t kmax, int32_t* perm_out,
                              hipStream_t s) {
    if (T == 0) return GILA_OK;
    const int64_t tj = std::max<int64_t>(4096, (T * kDigits + (1 << 24) - 1) >> 24);
    const int64_t ntiles = (T + tj - 1) / tj;
    const int64_t H = ntiles * kDigits;
    Buf tmp(s), hist(s), scan(s), ws(s);
    GILA_TRY(tmp.alloc<int32_t>((size_t)T));
    GILA_TRY(hist.alloc<int64_t>((size_t)H));
    GILA_TRY(scan.alloc<int64_t>((size_t)H + 1));
    GILA_TRY(ws.alloc<int64_t>((size_t)scan_workspace_count(H)));
    int passes = 0;
    for (int shift = 0; shift == 0 || (shift < 31 && (kmax >> shift) > 0); shift += kDigitBits) ++passes;
    // the passes alternate between the two buffers and end in perm_out
    int32_t* bufs[2] = {perm_out, tmp.as<int32_t>()};
    int32_t* cur = bufs[passes & 1];
    hipLaunchKernelGGL(iota_kernel, dim3(grid_for(T)), dim3(kBlock), 0, s, T, cur);
    GILA_HIP(hipGetLastError());
    int pass = 0;
    for (int shift = 0; shift == 0 || (shift < 31 && (kmax >> shift) > 0); shift += kDigitBits, ++pass) {
        int32_t* nxt = bufs[(passes - pass - 1) & 1];
        hipLaunchKernelGGL(digit_hist_kernel, dim3((unsigned)ntiles), dim3(kBlock), 0, s, T, tj,
                           ntiles, key, cur, shift, hist.as<int64_t>());
        GILA_HIP(hipGetLastError());
        GILA_TRY(enqueue_exclusive_scan_i64(hist.as<int64_t>(), scan.as<int64_t>(), H,
                                            ws.as<int64_t>(), s));
        hipLaunchKernelGGL(digit_scatter_kernel, dim3((unsigned)ntiles), dim3(64), 0, s, T, tj,
                           ntiles, key, cur, shift, scan.as<int64_t>(), nxt);
        GILA_HIP(hipGetLastError());
        cur = nxt;
    }
    return GILA_OK;
}

// ------------------------------------------------------------------ component order
// gstart[i] = 1 where the label-sorted sequence starts a new component.
__global__ __launch_bounds__(kBlock) void group_start_kernel(int32_t n, const int32_t* __restrict__ label,
                                                             const int32_t* __restrict__ bylabel,
                                                             int64_t* __restrict__ gstart) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        gstart[i] = (i == 0 || label[bylabel[i]] != label[bylabel[i - 1]]) ? 1 : 0;
}

// First position of every group (components in label order).
__global__ __launch_bounds__(kBlock) void group_bounds_kernel(int32_t n, const int64_t* __restrict__ gstart,
                                                              const int64_t* __restrict__ gidx,
                                                              int64_t* __restrict__ gfirst) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        if (gstart[i]) gfirst[gidx[i]] = i;  // gidx: groups starting before i
}

__global__ __launch_bounds__(kBlock) void group_size_kernel(int32_t C, int32_t n, const int64_t* __restrict__ gfirst,
                                                            int32_t* __restrict__ gsize,
                                                            int32_t* __restrict__ gkey) {
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < C;
         g += (int64_t)gridDim.x * kBlock) {
        const int64_t end = g + 1 < C ? gfirst[g + 1] : n;
        const int32_t sz = (int32_t)(end - gfirst[g]);
        gsize[g] = sz;
        gkey[g] = n - sz;  // larger components first
    }
}

// Rank r holds group byrank[r]: the group's rank and the sizes by rank.
__global__ __launch_bounds__(kBlock) void rank_tables_kernel(int32_t C, const int32_t* __restrict__ byrank,
                                                             const int32_t* __restrict__ gsize,
                                                             int32_t* __restrict__ grank,
                                                             int32_t* __restrict__ rsize,
                                                             int64_t* __restrict__ rsize64) {
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < C;
         r += (int64_t)gridDim.x * kBlock) {
        const int32_t g = byrank[r];
        grank[g] = (int32_t)r;
        rsize[r] = gsize[g];
        rsize64[r] = gsize[g];
    }
}

// New numbering: component by component in rank order, ascending ids inside.
__global__ __launch_bounds__(kBlock) void renumber_kernel(int32_t n, const int32_t* __restrict__ bylabel,
                                                          const int64_t* __restrict__ gidx,
                                                          const int64_t* __restrict__ gstart,
                                                          const int64_t* __restrict__ gfirst,
                                                          const int32_t* __restrict__ grank,
                                                          const int64_t* __restrict__ roff,
                                                          int32_t* __restrict__ perm,
                                                          int32_t* __restrict__ iperm,
                                                          int32_t* __restrict__ vrank) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t g = gidx[i] + gstart[i] - 1;  // group of position i
        const int32_t r = grank[g];
        const int64_t at = roff[r] + (i - gfirst[g]);
        const int32_t v = bylabel[i];
        perm[at] = v;
        iperm[v] = (int32_t)at;
        vrank[at] = r;
    }
}

// Components of a labelled graph in rank order (device tables) and the
// renumbering of the vertices.
struct CompOrder {
    int32_t C = 0;                   // components
    int32_t C2 = 0;                  // components with at least two vertices: ranks [0, C2)
    std::vector<int32_t> size;       // host, by rank
    std::vector<int64_t> off;        // host, [C + 1] first new id of each rank
    Buf perm, iperm, vrank, roff;    // device: new -> old, old -> new, rank of new id, offsets
    explicit CompOrder(hipStream_t s) : perm(s), iperm(s), vrank(s), roff(s) {}
};

static int order_components(int32_t n, const int32_t* label, hipStream_t s, CompOrder& o) {
    GILA_TRY(o.perm.alloc<int32_t>((size_t)n));
    GILA_TRY(o.iperm.alloc<int32_t>((size_t)n));
    GILA_TRY(o.vrank.alloc<int32_t>((size_t)n));
    if (n == 0) {
        GILA_TRY(o.roff.alloc<int64_t>(1));
        o.off.assign(1, 0);
        return GILA_OK;
    }
    Buf bylabel(s), gstart(s), gidx(s), ws(s);
    GILA_TRY(bylabel.alloc<int32_t>((size_t)n));
    GILA_TRY(gstart.alloc<int64_t>((size_t)n));
    GILA_TRY(gidx.alloc<int64_t>((size_t)n + 1));
    GILA_TRY(ws.alloc<int64_t>((size_t)scan_workspace_count(n)));
    GILA_TRY(stable_sort_by_key(label, n, n - 1, bylabel.as<int32_t>(), s));
    hipLaunchKernelGGL(group_start_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, label,
                       bylabel.as<int32_t>(), gstart.as<int64_t>());
    GILA_HIP(hipGetLastError());
    GILA_TRY(enqueue_exclusive_scan_i64(gstart.as<int64_t>(), gidx.as<int64_t>(), n,
                                        ws.as<int64_t>(), s));
    int64_t C = 0;
    GILA_HIP(hipMemcpyAsync(&C, gidx.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    o.C = (int32_t)C;
    Buf gfirst(s), gsize(s), gkey(s), byrank(s), grank(s), rsize(s), rsize64(s);
    GILA_TRY(gfirst.alloc<int64_t>((size_t)C));
    GILA_TRY(gsize.alloc<int32_t>((size_t)C));
    GILA_TRY(gkey.alloc<int32_t>((size_t)C));
    GILA_TRY(byrank.alloc<int32_t>((size_t)C));
    GILA_TRY(grank.alloc<int32_t>((size_t)C));
    GILA_TRY(rsize.alloc<int32_t>((size_t)C));
    GILA_TRY(rsize64.alloc<int64_t>((size_t)C));
    GILA_TRY(o.roff.alloc<int64_t>((size_t)C + 1));
    hipLaunchKernelGGL(group_bounds_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n,
                       gstart.as<int64_t>(), gidx.as<int64_t>(), gfirst.as<int64_t>());
    hipLaunchKernelGGL(group_size_kernel, dim3(grid_for(C)), dim3(kBlock), 0, s, o.C, n,
                       gfirst.as<int64_t>(), gsize.as<int32_t>(), gkey.as<int32_t>());
    GILA_HIP(hipGetLastError());
    GILA_TRY(stable_sort_by_key(gkey.as<int32_t>(), C, n - 1, byrank.as<int32_t>(), s));
    hipLaunchKernelGGL(rank_tables_kernel, dim3(grid_for(C)), dim3(kBlock), 0, s, o.C,
                       byrank.as<int32_t>(), gsize.as<int32_t>(), grank.as<int32_t>(),
                       rsize.as<int32_t>(), rsize64.as<int64_t>());
    GILA_HIP(hipGetLastError());
    Buf ws2(s);
    GILA_TRY(ws2.alloc<int64_t>((size_t)scan_workspace_count(C)));
    GILA_TRY(enqueue_exclusive_scan_i64(rsize64.as<int64_t>(), o.roff.as<int64_t>(), C,
                                        ws2.as<int64_t>(), s));
    hipLaunchKernelGGL(renumber_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n,
                       bylabel.as<int32_t>(), gidx.as<int64_t>(), gstart.as<int64_t>(),
                       gfirst.as<int64_t>(), grank.as<int32_t>(), o.roff.as<int64_t>(),
                       o.perm.as<int32_t>(), o.iperm.as<int32_t>(), o.vrank.as<int32_t>());
    GILA_HIP(hipGetLastError());
    o.size.resize((size_t)C);
    o.off.resize((size_t)C + 1);
    GILA_HIP(hipMemcpyAsync(o.size.data(), rsize.p, sizeof(int32_t) * C, hipMemcpyDeviceToHost, s));
    GILA_HIP(hipMemcpyAsync(o.off.data(), o.roff.p, sizeof(int64_t) * (C + 1), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    o.C2 = 0;
    while (o.C2 < o.C && o.size[o.C2] >= 2) ++o.C2;
    return GILA_OK;
}

// ------------------------------------------------------------------ bounding boxes and packing
// Bounding box of the contiguous new-id range of every rank r < R (positions
// in new order); one workgroup per rank, grid-stride.
template <class V>
__global__ __launch_bounds__(kBlock) void rank_bbox_kernel(int32_t R, const int64_t* __restrict__ roff,
                                                           const V* __restrict__ pos,
                                                           double4* __restrict__ box) {
    __shared__ double s[4][kWaves];
    for (int64_t r = blockIdx.x; r < R; r += gridDim.x) {
        double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
        for (int64_t i = roff[r] + threadIdx.x; i < roff[r + 1]; i += kBlock) {
            const double x = (double)pos[i].x, y = (double)pos[i].y;
            x0 = x < x0 ? x : x0;
            y0 = y < y0 ? y : y0;
            x1 = x > x1 ? x : x1;
            y1 = y > y1 ? y : y1;
        }
        for (int off = 32; off >= 1; off >>= 1) {
            double o = __shfl_xor(x0, off, 64);
            x0 = o < x0 ? o : x0;
            o = __shfl_xor(y0, off, 64);
            y0 = o < y0 ? o : y0;
            o = __shfl_xor(x1, off, 64);
            x1 = o > x1 ? o : x1;
            o = __shfl_xor(y1, off, 64);
            y1 = o > y1 ? o : y1;
        }
        if (lane64() == 0) {
            s[0][wave_id()] = x0;
            s[1][wave_id()] = y0;
            s[2][wave_id()] = x1;
            s[3][wave_id()] = y1;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 1; q < kWaves; ++q) {
                x0 = s[0][q] < x0 ? s[0][q] : x0;
                y0 = s[1][q] < y0 ? s[1][q] : y0;
                x1 = s[2][q] > x1 ? s[2][q] : x1;
                y1 = s[3][q] > y1 ? s[3][q] : y1;
            }
            box[r] = make_double4(x0, y0, x1, y1);
        }
        __syncthreads();
    }
}

// Column widths and row heights: the largest extent in each (extents are
// non-negative, so their bit patterns order as the values; the arrays start
// at zero).
__global__ __launch_bounds__(kBlock) void pack_extent_kernel(int32_t C, int32_t cols,
                                                             const double4* __restrict__ box,
                                                             unsigned long long* __restrict__ colw,
                                                             unsigned long long* __restrict__ rowh) {
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < C;
         r += (int64_t)gridDim.x * kBlock) {
        const double w = box[r].z - box[r].x, h = box[r].w - box[r].y;
        atomicMax(&colw[r % cols], (unsigned long long)__double_as_longlong(w + 0.0));
        atomicMax(&rowh[r / cols], (unsigned long long)__double_as_longlong(h + 0.0));
    }
}

// Cell corners: running sums of widths and heights plus the gap, in the
// order of a plain loop (one thread; there are at most 46341 columns).
__global__ void pack_cells_kernel(int32_t cols, int32_t rows, double gap,
                                  const unsigned long long* __restrict__ colw,
                                  const unsigned long long* __restrict__ rowh,
                                  double* __restrict__ colx, double* __restrict__ rowy) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    colx[0] = 0.0;
    rowy[0] = 0.0;
    for (int32_t j = 0; j < cols; ++j) colx[j + 1] = colx[j] + __longlong_as_double((long long)colw[j]) + gap;
    for (int32_t j = 0; j < rows; ++j) rowy[j + 1] = rowy[j] + __longlong_as_double((long long)rowh[j]) + gap;
}

// Translate (new order) and scatter back to the caller's ids.
template <class V>
__global__ __launch_bounds__(kBlock) void pack_move_kernel(int32_t n, int32_t cols,
                                                           const int32_t* __restrict__ vrank,
                                                           const int32_t* __restrict__ perm,
                                                           const double4* __restrict__ box,
                                                           const double* __restrict__ colx,
                                                           const double* __restrict__ rowy,
                                                           const V* __restrict__ src,
                                                           V* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t r = vrank[i];
        const double4 b = box[r];
        V p = src[i];
        p.x = (decltype(p.x))((double)p.x + (colx[r % cols] - b.x));
        p.y = (decltype(p.y))((double)p.y + (rowy[r / cols] - b.y));
        dst[perm[i]] = p;
    }
}

template <class V>
__global__ __launch_bounds__(kBlock) void gather_new_kernel(int32_t n, const int32_t* __restrict__ perm,
                                                            const V* __restrict__ src,
                                                            V* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        dst[i] = src[perm[i]];
}

// Packing of positions held in new order (pos_new) into the caller's ids.
template <class V>
static int pack_new_order(int32_t n, const CompOrder& o, double gap, const V* pos_new, V* pos_out,
                          hipStream_t s) {
    if (n == 0) return GILA_OK;
    int32_t cols = 1;
    while ((int64_t)cols * cols < o.C) ++cols;
    const int32_t rows = (o.C + cols - 1) / cols;
    Buf box(s), colx(s), rowy(s), ext(s);
    GILA_TRY(box.alloc<double4>((size_t)o.C));
    GILA_TRY(colx.alloc<double>((size_t)cols + 1));
    GILA_TRY(rowy.alloc<double>((size_t)rows + 1));
    GILA_TRY(ext.alloc<unsigned long long>((size_t)cols + rows));
    unsigned long long* colw = ext.as<unsigned long long>();
    unsigned long long* rowh = colw + cols;
    GILA_HIP(hipMemsetAsync(colw, 0, sizeof(unsigned long long) * (cols + rows), s));
    hipLaunchKernelGGL(rank_bbox_kernel<V>, dim3((unsigned)std::min<int64_t>(65536, o.C)),
                       dim3(kBlock), 0, s, o.C, o.roff.as<int64_t>(), pos_new, box.as<double4>());
    hipLaunchKernelGGL(pack_extent_kernel, dim3(grid_for(o.C)), dim3(kBlock), 0, s, o.C, cols,
                       box.as<double4>(), colw, rowh);
    hipLaunchKernelGGL(pack_cells_kernel, dim3(1), dim3(64), 0, s, cols, rows, gap, colw, rowh,
                       colx.as<double>(), rowy.as<double>());
    hipLaunchKernelGGL(pack_move_kernel<V>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, cols,
                       o.vrank.as<int32_t>(), o.perm.as<int32_t>(), box.as<double4>(),
                       colx.as<double>(), rowy.as<double>(), pos_new, pos_out);
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

template <class V>
static int pack_positions(int32_t n, const CompOrder& o, double gap, V* pos, hipStream_t s) {
    Buf tmp(s);
    GILA_TRY(tmp.alloc<V>((size_t)std::max(n, 1)));
    hipLaunchKernelGGL(gather_new_kernel<V>, dim3(grid_for(n)), dim3(kBlock), 0, s, n,
                       o.perm.as<int32_t>(), pos, tmp.as<V>());
    GILA_HIP(hipGetLastError());
    return pack_new_order<V>(n, o, gap, tmp.as<V>(), pos, s);
}

// Component labels given by a caller: each in [0, n) and naming a vertex
// labelled with itself.
__global__ __launch_bounds__(kBlock) void check_labels_kernel(int32_t n, const int32_t* __restrict__ label,
                                                              int32_t* __restrict__ bad) {
    bool b = false;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const int32_t l = label[v];
        if (l < 0 || l >= n) b = true;
        else if (label[l] != l) b = true;
    }
    if (__ballot(b) && lane64() == 0) atomicOr(bad, 1);
}

// ------------------------------------------------------------------ per-component CSRs
// Row lengths in new order.
__global__ __launch_bounds__(kBlock) void new_len_kernel(int32_t n, const int32_t* __restrict__ perm,
                                                         const int64_t* __restrict__ rp,
                                                         int64_t* __restrict__ len) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t v = perm[i];
        len[i] = rp[v + 1] - rp[v];
    }
}

// Rows in new order with ids local to the component (ascending: the
// renumbering is monotone inside a component), one wavefront per row.
__global__ __launch_bounds__(kBlock) void new_rows_kernel(int32_t n, const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ iperm,
                                                          const int32_t* __restrict__ vrank,
                                                          const int64_t* __restrict__ roff,
                                                          const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const int64_t* __restrict__ nrp,
                                                          int32_t* __restrict__ nci) {
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    for (int64_t i = (int64_t)blockIdx.x * kWaves + wave_id(); i < n; i += waves) {
        const int32_t v = perm[i];
        const int64_t base = roff[vrank[i]];
        const int64_t b = rp[v], len = rp[v + 1] - b, o = nrp[i];
        for (int64_t e = lane64(); e < len; e += 64) nci[o + e] = (int32_t)(iperm[ci[b + e]] - base);
    }
}

// Rebased row offsets of every component with at least two vertices: the
// rows of rank r (new ids roff[r] .. roff[r+1]) go to crp[roff[r] + r ..],
// starting at 0.
__global__ __launch_bounds__(kBlock) void comp_rp_kernel(int32_t n, int32_t C2,
                                                         const int32_t* __restrict__ vrank,
                                                         const int64_t* __restrict__ roff,
                                                         const int64_t* __restrict__ nrp,
                                                         int64_t* __restrict__ crp) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t r = vrank[i];
        if (r >= C2) continue;
        const int64_t first = roff[r];
        crp[i + r] = nrp[i] - nrp[first];
        if (i + 1 == roff[r + 1]) crp[i + 1 + r] = nrp[i + 1] - nrp[first];
    }
}

template <class V>
static int layout_components(const gila_csr* g, int32_t k, const gila_params* params, V* pos,
                             hipStream_t s, int32_t* components_out, int32_t* iterations_host) {
    const int32_t n = g->n;
    Buf label(s);
    GILA_TRY(label.alloc<int32_t>((size_t)std::max(n, 1)));
    GILA_TRY(label_components(g, label.as<int32_t>(), s));
    CompOrder o(s);
    GILA_TRY(order_components(n, label.as<int32_t>(), s, o));
    if (components_out) *components_out = o.C;
    if (n == 0) return GILA_OK;
    std::vector<int32_t> runs((size_t)o.C, 0);  // iterations run, by rank
    // graph and positions in new order
    Buf nrp(s), nci(s), crp(s), npos(s), ws(s), len(s);
    GILA_TRY(len.alloc<int64_t>((size_t)n));
    GILA_TRY(nrp.alloc<int64_t>((size_t)n + 1));
    GILA_TRY(nci.alloc<int32_t>((size_t)std::max<int64_t>(g->nnz, 1)));
    GILA_TRY(crp.alloc<int64_t>((size_t)n + (size_t)o.C2 + 1));
    GILA_TRY(npos.alloc<V>((size_t)n));
    GILA_TRY(ws.alloc<int64_t>((size_t)scan_workspace_count(n)));
    hipLaunchKernelGGL(new_len_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n,
                       o.perm.as<int32_t>(), g->row_ptr, len.as<int64_t>());
    GILA_HIP(hipGetLastError());
    GILA_TRY(enqueue_exclusive_scan_i64(len.as<int64_t>(), nrp.as<int64_t>(), n, ws.as<int64_t>(), s));
    const int rgrid = (int)std::max<int64_t>(1, std::min<int64_t>(16384, ((int64_t)n + kWaves - 1) / kWaves));
    hipLaunchKernelGGL(new_rows_kernel, dim3(rgrid), dim3(kBlock), 0, s, n, o.perm.as<int32_t>(),
                       o.iperm.as<int32_t>(), o.vrank.as<int32_t>(), o.roff.as<int64_t>(), g->row_ptr,
                       g->col_idx, nrp.as<int64_t>(), nci.as<int32_t>());
    hipLaunchKernelGGL(comp_rp_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, o.C2,
                       o.vrank.as<int32_t>(), o.roff.as<int64_t>(), nrp.as<int64_t>(),
                       crp.as<int64_t>());
    hipLaunchKernelGGL(gather_new_kernel<V>, dim3(grid_for(n)), dim3(kBlock), 0, s, n,
                       o.perm.as<int32_t>(), pos, npos.as<V>());
    GILA_HIP(hipGetLastError());
    // initial bounding boxes -> caps
    std::vector<double4> box((size_t)std::max(o.C2, 1));
    std::vector<int64_t> nrp_at((size_t)o.C2 + 1);
    if (o.C2 > 0) {
        Buf dbox(s);
        GILA_TRY(dbox.alloc<double4>((size_t)o.C2));
        hipLaunchKernelGGL(rank_bbox_kernel<V>, dim3((unsigned)std::min<int64_t>(65536, o.C2)),
                           dim3(kBlock), 0, s, o.C2, o.roff.as<int64_t>(), npos.as<V>(),
                           dbox.as<double4>());
        GILA_HIP(hipGetLastError());
        GILA_HIP(hipMemcpyAsync(box.data(), dbox.p, sizeof(double4) * o.C2, hipMemcpyDeviceToHost, s));
        std::vector<int64_t> nrp_host((size_t)n + 1);
        GILA_HIP(hipMemcpyAsync(nrp_host.data(), nrp.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        for (int32_t r = 0; r <= o.C2; ++r) nrp_at[r] = nrp_host[o.off[r]];
    }
    const int32_t H = params->iterations;
    const double d = params->ideal_length;
    std::vector<double> temps((size_t)std::max<int64_t>((int64_t)o.C2 * H, 1));
    std::vector<gila_params> cp((size_t)std::max(o.C2, 1));
    std::vector<gila_csr> cg((size_t)std::max(o.C2, 1));
    for (int32_t r = 0; r < o.C2; ++r) {
        const double w = box[r].z - box[r].x, h = box[r].w - box[r].y;
        const double aspect = (w > 0.0 && h > 0.0) ? h / w : 1.0;
        const double base = std::sqrt(((double)o.size[r] / aspect) * d);
        for (int32_t t = 0; t < H; ++t) temps[(size_t)r * H + t] = base * std::pow(0.93, (double)t);
        cp[r] = *params;
        cp[r].temperature = temps.data() + (size_t)r * H;
        cg[r].n = o.size[r];
        cg[r].nnz = nrp_at[r + 1] - nrp_at[r];
        cg[r].row_ptr = crp.as<int64_t>() + o.off[r] + r;
        cg[r].col_idx = nci.as<int32_t>() + nrp_at[r];
    }
    // large components on the whole GPU, one after another
    const bool batchable = params->force_model == GILA_MODEL_FR;
    int32_t small_first = o.C2;
    if (batchable)
        while (small_first > 0 && o.size[small_first - 1] <= kSmallComponent) --small_first;
    for (int32_t r = 0; r < small_first; ++r) {
        gila_khop* kh = nullptr;
        GILA_TRY(build_khop(&cg[r], k, s, &kh));
        gila_stats st{};
        int rc;
        {
            std::lock_guard<std::mutex> lk(kh->mu);
            rc = run_iterations(kh, &cp[r], 0, H, npos.as<V>() + o.off[r], s, &st, false);
        }
        free_khop(kh, Release{true, s});
        GILA_TRY(rc);
        runs[r] = st.iterations_run;
    }
    // the small ones in one batched launch
    const int32_t nsmall = o.C2 - small_first;
    if (nsmall > 0) {
        std::vector<int32_t> ks((size_t)nsmall, k);
        std::vector<void*> pp((size_t)nsmall);
        for (int32_t j = 0; j < nsmall; ++j) pp[j] = npos.as<V>() + o.off[small_first + j];
        gila_batch* b = nullptr;
        GILA_TRY(batch_build(cg.data() + small_first, nsmall, ks.data(), s, &b));
        std::vector<gila_stats> st((size_t)nsmall);
        const int rc = batch_run(b, cp.data() + small_first, pp.data(), s, st.data(), false);
        free_batch(b, Release{true, s});
        GILA_TRY(rc);
        for (int32_t j = 0; j < nsmall; ++j) runs[small_first + j] = st[j].iterations_run;
    }
    GILA_TRY(pack_new_order<V>(n, o, d, npos.as<V>(), pos, s));
    if (iterations_host) {
        std::vector<int32_t> perm((size_t)n);
        GILA_HIP(hipMemcpyAsync(perm.data(), o.perm.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        for (int32_t r = 0; r < o.C; ++r)
            for (int64_t i = o.off[r]; i < o.off[r + 1]; ++i) iterations_host[perm[i]] = runs[r];
    }
    GILA_HIP(hipStreamSynchronize(s));
    return GILA_OK;
}

// ------------------------------------------------------------------ labels without allocation
// gila_components_noalloc keeps its scratch in a fixed array per device,
// never in allocated memory.  Layout (64-bit words):
//   [0] CSR flags (int32 in the low half), [1] hooked-this-pass flag (int32),
//   [2] number of components, [8, 8 + kNoAllocPartials) per-workgroup root
//   counts.  The counting grid never exceeds kNoAllocPartials workgroups, so
//   no graph needs more than these 16 KiB.
constexpr int kNoAllocHeader = 8;
constexpr int kNoAllocPartials = 2040;
constexpr int kNoAllocWords = kNoAllocHeader + kNoAllocPartials;
static __device__ __align__(256) unsigned long long scratch[kNoAllocWords];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static unsigned long long* g_scratch_ptr[kMaxScratchDevices];

// Device address of `scratch` on the current device (each device holds its own
// copy); looked up once per device.  In host code the array's name is only a
// stand-in, so kernels and copies must use this address.
static int scratch_address(unsigned long long** out) {
    int dev = 0;
    GILA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(GILA_EUNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GILA_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
    }
    *out = g_scratch_ptr[dev];
    return GILA_OK;
}

// Zeroes words [0, count) (a kernel, not a memset node, so the call can sit in
// a captured graph).
__global__ void clear_words_kernel(unsigned long long* w, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) w[i] = 0ull;
}

// row_ptr rules (0 first, nnz last, monotone, every offset in [0, nnz]) on the
// device: flag bit 16.  The CSR checks of validate_csr_kernel read col_idx
// through row_ptr and may run only once these hold.
__global__ __launch_bounds__(kBlock) void rowptr_check_kernel(int32_t n, int64_t nnz,
                                                              const int64_t* __restrict__ rp,
                                                              int32_t* __restrict__ flag) {
    int32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= n;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t r = rp[i];
        if ((i == 0 && r != 0) || (i == n && r != nnz) || r < 0 || r > nnz ||
            (i > 0 && rp[i - 1] > r))
            bad = 16;
    }
    if (bad) atomicOr(flag, bad);
}

// Roots (label[v] == v) counted per workgroup into partial[blockIdx.x].
__global__ __launch_bounds__(kBlock) void count_roots_kernel(int32_t n,
                                                             const int32_t* __restrict__ label,
                                                             unsigned long long* __restrict__ partial) {
    __shared__ int64_t s_red[kWaves];
    int64_t c = 0;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        c += label[v] == (int32_t)v ? 1 : 0;
    const int64_t tot = block_sum<int64_t>(c, s_red);
    if (threadIdx.x == 0) partial[blockIdx.x] = (unsigned long long)tot;
}

// total = partial[0] + ... + partial[count - 1] (one workgroup, fixed order).
__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const unsigned long long* __restrict__ partial,
                                                              int count,
                                                              unsigned long long* __restrict__ total) {
    __shared__ int64_t s_red[kWaves];
    int64_t c = 0;
    for (int i = threadIdx.x; i < count; i += kBlock) c += (int64_t)partial[i];
    const int64_t tot = block_sum<int64_t>(c, s_red);
    if (threadIdx.x == 0) *total = (unsigned long long)tot;
}

// Reads an int32 flag word of the scratch (synchronises the stream).
static int read_flag(const unsigned long long* word, hipStream_t s, int32_t* out) {
    GILA_HIP(hipMemcpyAsync(out, word, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    return GILA_OK;
}

static int components_noalloc(const gila_csr* g, int32_t* label, int32_t* count_out,
                              hipStream_t s) {
    if (!g) return fail(GILA_EINVAL, "graph is NULL");
    const int32_t n = g->n;
    const int64_t nnz = g->nnz;
    if (n < 0 || nnz < 0) return fail(GILA_EINVAL, "negative n or nnz");
    if (n > 0 && !g->row_ptr) return fail(GILA_EINVAL, "row_ptr is NULL");
    if (nnz > 0 && !g->col_idx) return fail(GILA_EINVAL, "col_idx is NULL");
    if (nnz % 2) return fail(GILA_EINVAL, "nnz must be even for a symmetric CSR");
    if (nnz > (int64_t)n * (int64_t)(n > 0 ? n - 1 : 0))
        return fail(GILA_EINVAL, "nnz exceeds n(n-1)");
    if (n > 0 && !label) return fail(GILA_EINVAL, "label_dev is NULL");
    unsigned long long* w = nullptr;
    GILA_TRY(scratch_address(&w));
    if (n == 0) {
        if (count_out) *count_out = 0;
        return GILA_OK;
    }
    int32_t* csr_flag = reinterpret_cast<int32_t*>(w);
    int32_t* hooked = reinterpret_cast<int32_t*>(w + 1);
    unsigned long long* partial = w + kNoAllocHeader;
    hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(64), 0, s, w, kNoAllocHeader);
    hipLaunchKernelGGL(rowptr_check_kernel, dim3(grid_for((int64_t)n + 1)), dim3(kBlock), 0, s, n,
                       nnz, g->row_ptr, csr_flag);
    GILA_HIP(hipGetLastError());
    int32_t flag = 0;
    GILA_TRY(read_flag(w, s, &flag));
    if (flag) return fail(GILA_EINVAL, "row_ptr must run from 0 to nnz without decreasing");
    if (nnz > 0) {
        GILA_TRY(launch_validate_csr(n, nnz, g->row_ptr, g->col_idx, csr_flag, s));
        GILA_TRY(read_flag(w, s, &flag));
        if (flag)
            return fail(GILA_EINVAL, "malformed CSR:%s%s%s%s", (flag & 1) ? " column out of range" : "",
                        (flag & 2) ? " self-loop" : "", (flag & 4) ? " row not strictly ascending" : "",
                        (flag & 8) ? " not symmetric" : "");
    }
    // the labelling passes of label_components, with the hooked flag in scratch
    hipLaunchKernelGGL(cc_init_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, label);
    GILA_HIP(hipGetLastError());
    if (nnz > 0) {
        const int hgrid =
            (int)std::max<int64_t>(1, std::min<int64_t>(16384, ((int64_t)n + kWaves - 1) / kWaves));
        for (int pass = 0;; ++pass) {
            if (pass > 4096) return fail(GILA_EDEVICE, "component labels did not settle");
            hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(64), 0, s, w + 1, 1);
            hipLaunchKernelGGL(cc_hook_kernel, dim3(hgrid), dim3(kBlock), 0, s, n, g->row_ptr,
                               g->col_idx, label, hooked);
            hipLaunchKernelGGL(cc_compress_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, label);
            GILA_HIP(hipGetLastError());
            int32_t changed = 0;
            GILA_TRY(read_flag(w + 1, s, &changed));
            if (!changed) break;
        }
    }
    if (count_out) {
        // every component has exactly one root (its smallest id)
        const int cgrid = (int)std::min<int64_t>(kNoAllocPartials, ((int64_t)n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(count_roots_kernel, dim3(cgrid), dim3(kBlock), 0, s, n, label, partial);
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kBlock), 0, s, partial, cgrid, w + 2);
        GILA_HIP(hipGetLastError());
        unsigned long long c = 0;
        GILA_HIP(hipMemcpyAsync(&c, w + 2, sizeof(c), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        *count_out = (int32_t)c;
    }
    GILA_HIP(hipStreamSynchronize(s));
    return GILA_OK;
}

}  // namespace gila

using namespace gila;

extern "C" {

int gila_components_noalloc(const gila_csr* g_dev, int32_t* label_dev, int32_t* count_out,
                            void* stream) {
    clear_error();
    return components_noalloc(g_dev, label_dev, count_out, (hipStream_t)stream);
}

int gila_components(const gila_csr* g_dev, int32_t* label_dev, int32_t* count_out, void* stream) {
    TraceRange trace_range("gila_components");
    clear_error();
    hipStream_t s = (hipStream_t)stream;
    GILA_TRY(validate_graph(g_dev, s));
    if (g_dev->n > 0 && !label_dev) return fail(GILA_EINVAL, "label_dev is NULL");
    GILA_TRY(label_components(g_dev, label_dev, s));
    if (count_out) {
        CompOrder o(s);
        GILA_TRY(order_components(g_dev->n, label_dev, s, o));
        *count_out = o.C;
    }
    GILA_HIP(hipStreamSynchronize(s));
    return GILA_OK;
}

int gila_pack_components(int32_t n, const int32_t* label_dev, double gap, int32_t precision,
                         void* pos_dev, void* stream) {
    TraceRange trace_range("gila_pack_components");
    clear_error();
    if (n < 0) return fail(GILA_EINVAL, "n must be >= 0");
    if (n > 0 && (!label_dev || !pos_dev)) return fail(GILA_EINVAL, "label_dev or pos_dev is NULL");
    if (!(gap >= 0.0) || !std::isfinite(gap)) return fail(GILA_EINVAL, "gap must be finite and >= 0");
    if (precision != GILA_FP64 && precision != GILA_FP32 && precision != GILA_FP32_KAHAN)
        return fail(GILA_EINVAL, "unknown precision %d", precision);
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return GILA_OK;
    {
        Buf bad(s);
        GILA_TRY(bad.alloc<int32_t>(1));
        GILA_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(check_labels_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, label_dev,
                           bad.as<int32_t>());
        GILA_HIP(hipGetLastError());
        int32_t b = 0;
        GILA_HIP(hipMemcpyAsync(&b, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        if (b) return fail(GILA_EINVAL, "labels must lie in [0, n) and name a vertex labelled with itself");
    }
    CompOrder o(s);
    GILA_TRY(order_components(n, label_dev, s, o));
    if (precision == GILA_FP64) GILA_TRY(pack_positions<double2>(n, o, gap, (double2*)pos_dev, s));
    else GILA_TRY(pack_positions<float2>(n, o, gap, (float2*)pos_dev, s));
    GILA_HIP(hipStreamSynchronize(s));
    return GILA_OK;
}

int gila_layout_components(const gila_csr* g_dev, int32_t k, const gila_params* params,
                           void* pos_dev, void* stream, int32_t* components_out,
                           int32_t* iterations_host) {
    TraceRange trace_range("gila_layout_components");
    clear_error();
    if (!params) return fail(GILA_EINVAL, "params is NULL");
    gila_params p = *params;
    p.temperature = nullptr;  // the caps are the components' own
    GILA_TRY(check_params(&p, false));
    if (k < 1) return fail(GILA_EINVAL, "k must be >= 1 (got %d)", k);
    hipStream_t s = (hipStream_t)stream;
    GILA_TRY(validate_graph(g_dev, s));
    if (g_dev->n > 0 && !pos_dev) return fail(GILA_EINVAL, "pos_dev is NULL");
    if (p.precision == GILA_FP64)
        return layout_components<double2>(g_dev, k, &p, (double2*)pos_dev, s, components_out,
                                          iterations_host);
    return layout_components<float2>(g_dev, k, &p, (float2*)pos_dev, s, components_out,
                                     iterations_host);
}

}  // extern "C"

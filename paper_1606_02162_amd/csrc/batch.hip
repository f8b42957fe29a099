// Many independent graphs in one persistent launch.
//
// Build: the graphs are laid out one after another as a block-diagonal union
// (vertex ids offset by each graph's base), validated, and their k-hop lists
// are built in one batched frontier expansion whose bitmaps cover only the
// source's own graph.  Lists and adjacency are stored as 16-bit ids local to
// their graph.
//
// Run: one persistent kernel.  A workgroup takes the next graph (largest
// first), copies its positions into LDS (two buffers), and runs ALL of the
// graph's iterations there -- forces from LDS gathers, the temperature cap,
// the synchronous move into the other buffer, the statistics and the halting
// rule -- with only workgroup barriers between iterations; then it writes the
// positions back and takes the next graph.
//
// Graphs run with one lane per vertex read their rows from wave slices: the
// graph's vertices sorted by decreasing row length, cut into slices of 64
// (one per wavefront step), and each slice's rows stored interleaved -- quad
// j of the slice's lane l at word j * 64 + l -- padded to the slice's longest
// row (an even number of quads).  A wavefront then loads 512 contiguous bytes
// per quad step, its lanes walk rows of similar length, and each vertex still
// adds its terms in its own row order (the same bits as the row layout).  A graph's arithmetic depends only
// on that graph and its lanes per vertex, which the handle's plan fixes at
// build (from the graph's mean row length; gila_batch_tune or
// gila_batch_set_plan may replace it), so its result is the same bits alone,
// in any batch and in any process.  The launch is captured as a HIP graph and
// replayed on later runs.
#include <algorithm>
#include <cstring>
#include <cmath>
#include <cstdlib>
#include <map>
#include <numeric>

#include "iteration.h"

namespace gila {

struct BatchDesc {
    int64_t vbase;             // first vertex of the graph in the union
    int64_t sbase;             // its first wave slice
    int32_t n;
    int32_t n_active;
    int32_t lpv;               // lanes per vertex
    int32_t iters;             // iterations to run
    int32_t t_off;             // offset of its temperatures
    int32_t cls;               // row-length class (key of the tuner's table)
    double d;
    double stop_fraction;
    double stop_displacement;
    void* pos;                 // caller's positions (n, precision layout)
};

// A wave slice: 64 vertices of one graph (a lane each), with their rows
// interleaved at sk + koff (nq quad words per lane, nq even) and their
// adjacency interleaved at sa + aoff (na ids per lane).
struct SellSlice {
    int64_t koff;
    int64_t aoff;
    int32_t nq;
    int32_t na;
};

struct BatchArgs {
    int32_t count;
    const BatchDesc* graphs;
    const int32_t* order;      // graphs in decreasing work
    const int64_t* kstart;     // [nv]: start of each k-hop row in kidx
    const int32_t* klen;       // [nv]: its length, padded to whole quads
    const uint16_t* kidx;      // local ids
    const int64_t* rp;         // union adjacency row offsets
    const uint16_t* ci;        // local ids
    const SellSlice* sell;     // wave slices (graphs with one lane per vertex)
    const uint2* smeta;        // [64 per slice]: (vertex, row quads | degree << 16)
    const uint2* sk;           // interleaved rows (quads of local ids)
    const uint16_t* sa;        // interleaved adjacency (local ids)
    double* escratch;          // [grid][2][slices_max] per-slice energies
    int32_t slices_max;        // slices of the largest graph
    const double* temps;
    gila_stats* stats;         // [count], indexed like graphs
    uint64_t* t_start;         // [count] device wall clock when the graph was taken
    uint64_t* t_end;           // [count] ... and when its positions were written back
    int32_t* work;             // next graph (atomic)
};

}  // namespace gila

struct gila_batch {
    int device = 0;
    int32_t count = 0;
    int64_t nv = 0, nnz = 0, P = 0;  // vertices, adjacency entries, pairs
    int64_t device_bytes = 0;
    int32_t nmax = 0;
    std::vector<int64_t> vbase, ebase, Pg, sbase;
    std::vector<int32_t> n, n_active, k, cls;
    std::vector<int32_t> lpv;  // the plan: lanes per vertex of each graph
    int64_t* kstart = nullptr;  // [nv]: start of each k-hop row in kidx
    int32_t* klen = nullptr;    // [nv]: its length, padded to whole quads
    uint16_t* kidx = nullptr;
    int64_t kidx_size = 0;      // entries of kidx (the rows and the blocks' slack)
    int64_t* rp = nullptr;
    uint16_t* ci16 = nullptr;
    int64_t nslices = 0, sell_quads = 0, sell_adj = 0;
    gila::SellSlice* d_sell = nullptr;
    uint2* d_smeta = nullptr;
    uint2* d_sk = nullptr;
    uint16_t* d_sa = nullptr;
    double* d_escratch = nullptr;  // per-slice energies, [grid][2][slices of the largest graph]
    int64_t escratch_grid = 0;     // workgroups it has room for
    gila::BatchDesc* d_desc = nullptr;
    int32_t* d_order = nullptr;
    double* d_temps = nullptr;
    int64_t temps_cap = 0;
    gila_stats* d_stats = nullptr;
    uint64_t* d_clock = nullptr;   // [2 * count]: start and end wall clock per graph
    int32_t* d_work = nullptr;
    std::vector<int32_t> order;
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> gkey;
    std::mutex mu;
};

namespace gila {

constexpr int kBatchBlock = 512;
constexpr int kBatchWaves = kBatchBlock / 64;
constexpr int kClasses = 8;
// A vertex with a non-finite force is counted in the high 32 bits of the
// per-thread moved counter (a batched graph has at most 65535 vertices, so
// the low half never carries into them): no extra register in the kernel.
constexpr int64_t kNonfiniteOne = int64_t(1) << 32;

// ------------------------------------------------------------------ build kernels
struct GraphSrc {
    const int64_t* rp;
    const int32_t* ci;
    int64_t vbase, ebase, nnz;
    int32_t n, pad;
};

// One workgroup per graph: copy its CSR into the union with rebased ids and
// check the per-graph rules that the union check cannot see.
__global__ __launch_bounds__(kBlock) void gather_csr_kernel(const GraphSrc* __restrict__ src,
                                                            int64_t* __restrict__ rp,
                                                            int32_t* __restrict__ ci,
                                                            int32_t* __restrict__ flag) {
    const GraphSrc g = src[blockIdx.x];
    int32_t bad = 0;
    for (int64_t i = threadIdx.x; i <= g.n; i += kBlock) {
        const int64_t r = g.rp ? g.rp[i] : 0;  // an empty graph may pass no row_ptr
        if ((i == 0 && r != 0) || (i == g.n && r != g.nnz) || r < 0 || r > g.nnz) bad |= 16;
        if (i > 0 && g.rp[i - 1] > r) bad |= 16;
        rp[g.vbase + i] = g.ebase + (r < 0 ? 0 : (r > g.nnz ? g.nnz : r));
    }
    for (int64_t j = threadIdx.x; j < g.nnz; j += kBlock) {
        const int32_t u = g.ci[j];
        if (u < 0 || u >= g.n) {
            bad |= 1;
            ci[g.ebase + j] = (int32_t)g.vbase;  // keeps later checks in range
        } else {
            ci[g.ebase + j] = (int32_t)(g.vbase + u);
        }
    }
    if (bad) atomicOr(flag, bad);
}

// One workgroup per graph: local 16-bit adjacency ids and the non-isolated
// vertex count.
__global__ __launch_bounds__(kBlock) void localize_kernel(const GraphSrc* __restrict__ src,
                                                          const int32_t* __restrict__ ci,
                                                          const int64_t* __restrict__ rp,
                                                          uint16_t* __restrict__ ci16,
                                                          int32_t* __restrict__ n_active) {
    __shared__ int32_t s_red[4];
    const GraphSrc g = src[blockIdx.x];
    for (int64_t j = threadIdx.x; j < g.nnz; j += kBlock)
        ci16[g.ebase + j] = (uint16_t)(ci[g.ebase + j] - g.vbase);
    int32_t act = 0;
    for (int64_t i = threadIdx.x; i < g.n; i += kBlock)
        act += rp[g.vbase + i + 1] > rp[g.vbase + i] ? 1 : 0;
    const int32_t tot = block_sum<int32_t>(act, s_red);
    if (threadIdx.x == 0) n_active[blockIdx.x] = tot;
}

__global__ void gather_bounds_kernel(const int64_t* __restrict__ kptr,
                                     const int64_t* __restrict__ vb, int32_t count,
                                     int64_t* __restrict__ out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= count; i += gridDim.x * blockDim.x)
        out[i] = kptr[vb[i]];
}

// ------------------------------------------------------------------ k-hop lists of small graphs
// One workgroup per graph (largest first): the graph's CSR is copied into LDS
// with local ids, then each wavefront takes one source at a time and runs a
// level-synchronous BFS to depth k on three bitmaps of its own in LDS
// (visited, this level, next level), deduplicating with LDS atomic ORs.  The
// count pass writes |N_v(k)|; the fill pass writes the row ascending by
// scanning the visited bitmap.  Used when every graph of the batch fits.
// Workgroups of 1024 threads (16 wavefronts share one graph, so that the
// largest graphs, taken first, do not leave a long tail) when the per-wave
// bitmaps fit beside the graph in LDS, else 512.

struct BatchBfsArgs {
    int32_t count;
    const int32_t* gorder;   // graphs, largest first
    const int64_t* vbase;    // [count + 1]
    const int64_t* rp;       // union CSR (global ids)
    const int32_t* ci;
    const int32_t* gk;       // k of each graph
    const int64_t* gbase;    // [count]: start of each graph's block of kidx
    int64_t* counts;         // [nv]: |N_v(k)|
    int64_t* kstart;         // [nv]: start of each row in kidx
    int32_t* klen;           // [nv]: its length, padded to whole quads
    uint16_t* kidx;          // local ids, each row padded with the sentinel n
    int32_t* work;           // next graph (atomic)
    int32_t nmax;            // largest graph: vertices ...
    int64_t nnzmax;          // ... and adjacency entries
};

size_t batch_bfs_lds_bytes(int32_t nmax, int64_t nnzmax, int waves) {
    const size_t nwords = (size_t)(nmax + 31) / 32;
    return 4 * ((size_t)nmax + 1) + 2 * (((size_t)nnzmax + 1) & ~(size_t)1) +
           4 * nwords * 3 * (size_t)waves;
}

// One pass per source: after its BFS the wavefront knows |N_v(k)|, takes the
// row's place (padded to quads) from the graph's cursor in LDS inside the
// graph's block of kidx -- sized by a walk-count bound of the graph's rows
// (walk_bound_kernel), so it never overflows -- and writes the row ascending
// from the visited bitmap, then the padding.  Where a row lands in the block
// depends on which wavefront finishes first; what it holds does not.
template <int BS>
__global__ __launch_bounds__(BS) void batch_khop_kernel(BatchBfsArgs a) {
    constexpr int kBfsBlock = BS;
    constexpr int kBfsWaves = BS / 64;
    extern __shared__ __align__(16) unsigned char s_raw[];
    __shared__ int s_g;
    __shared__ unsigned long long s_cursor;
    const int nwords_max = (a.nmax + 31) / 32;
    int32_t* s_rp = reinterpret_cast<int32_t*>(s_raw);
    uint16_t* s_ci = reinterpret_cast<uint16_t*>(s_rp + a.nmax + 1);
    uint32_t* s_bm = reinterpret_cast<uint32_t*>(s_ci + ((a.nnzmax + 1) & ~(int64_t)1));
    const int lane = lane64(), w = wave_id();
    uint32_t* vis = s_bm + (size_t)w * 3 * nwords_max;
    for (;;) {
        if (threadIdx.x == 0) s_g = atomicAdd(a.work, 1);
        __syncthreads();
        const int gi = s_g;
        __syncthreads();
        if (gi >= a.count) return;
        const int g = a.gorder[gi];
        const int64_t vb = a.vbase[g];
        const int n = (int)(a.vbase[g + 1] - vb);
        const int k = a.gk[g];
        const int64_t eb = a.rp[vb];
        const int64_t ne = a.rp[vb + n] - eb;
        for (int i = threadIdx.x; i <= n; i += kBfsBlock) s_rp[i] = (int32_t)(a.rp[vb + i] - eb);
        for (int64_t j = threadIdx.x; j < ne; j += kBfsBlock) s_ci[j] = (uint16_t)(a.ci[eb + j] - vb);
        if (threadIdx.x == 0) s_cursor = 0ull;
        __syncthreads();
        const int nw = (n + 31) >> 5;
        const int64_t gb = a.gbase[g];
        for (int src = w; src < n; src += kBfsWaves) {
            uint32_t* cur = vis + nwords_max;
            uint32_t* nxt = cur + nwords_max;
            for (int i = lane; i < nw; i += 64) {
                vis[i] = 0u;
                cur[i] = 0u;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                vis[src >> 5] = 1u << (src & 31);
                cur[src >> 5] = 1u << (src & 31);
            }
            __builtin_amdgcn_wave_barrier();
            int found = 0;
            for (int level = 0; level < k; ++level) {
                for (int i = lane; i < nw; i += 64) nxt[i] = 0u;
                __builtin_amdgcn_wave_barrier();
                int added = 0;
                for (int i = lane; i < nw; i += 64) {
                    uint32_t bits = cur[i];
                    while (bits) {
                        const int u = i * 32 + __builtin_ctz(bits);
                        bits &= bits - 1u;
                        const int e1 = s_rp[u + 1];
                        for (int e = s_rp[u]; e < e1; ++e) {
                            const int x = s_ci[e];
                            const uint32_t m = 1u << (x & 31);
                            if (!(atomicOr(&vis[x >> 5], m) & m)) {
                                atomicOr(&nxt[x >> 5], m);
                                ++added;
                            }
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
                found += added;
                uint32_t* t = cur;
                cur = nxt;
                nxt = t;
                if (__ballot(added > 0) == 0ull) break;
            }
            // the row's place: |N_v(k)| padded to quads, from the graph's cursor
            const int total = wave_sum(found);
            const int padded = (total + 3) & ~3;
            unsigned long long off = 0ull;
            if (lane == 0) off = atomicAdd(&s_cursor, (unsigned long long)padded);
            off = __shfl(off, 0, 64);
            const int64_t start = gb + (int64_t)off;
            if (lane == 0) {
                a.counts[vb + src] = total;
                a.kstart[vb + src] = start;
                a.klen[vb + src] = padded;
            }
            // the row: visited ids except src, ascending
            int64_t out = start;
            for (int i0 = 0; i0 < nw; i0 += 64) {
                const int i = i0 + lane;
                uint32_t bits = i < nw ? vis[i] : 0u;
                if (i == (src >> 5)) bits &= ~(1u << (src & 31));
                const int c = __popc(bits);
                const int incl = wave_inclusive_scan(c);
                int64_t at = out + incl - c;
                while (bits) {
                    a.kidx[at++] = (uint16_t)(i * 32 + __builtin_ctz(bits));
                    bits &= bits - 1u;
                }
                out += __shfl(incl, 63, 64);
            }
            for (int j = total + lane; j < padded; j += 64) a.kidx[start + j] = (uint16_t)n;
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
}

static int run_batch_bfs(const BatchBfsArgs& a, size_t lds, int bs, int device, hipStream_t s) {
    const void* kernel = bs == 1024 ? (const void*)batch_khop_kernel<1024>
                                    : (const void*)batch_khop_kernel<512>;
    if (lds > 48 * 1024)
        (void)quiet(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const DeviceInfo& di = device_info(device);
    const int per_cu =
        (int)std::max<size_t>(1, std::min<size_t>(2048 / bs, (160u * 1024u) / (lds + 1024)));
    const int grid = std::min(a.count, di.cus * per_cu);
    GILA_HIP(hipMemsetAsync(a.work, 0, sizeof(int32_t), s));
    if (bs == 1024)
        hipLaunchKernelGGL(batch_khop_kernel<1024>, dim3(grid), dim3(1024), lds, s, a);
    else
        hipLaunchKernelGGL(batch_khop_kernel<512>, dim3(grid), dim3(512), lds, s, a);
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

// ------------------------------------------------------------------ row blocks
// An upper bound of each vertex's padded row: the walks of length <= k (its
// graph's k) from v, capped at n_g - 1 (|N_v(k)| counts distinct vertices
// reached by such walks), rounded up to whole quads.  Level l adds the walks
// of length l: w_l(v) = sum of w_{l-1}(u) over u adjacent to v (capped at
// n_g, which keeps the sums small and the bound valid).  One launch per level.
__global__ void vertex_graph_kernel(const int64_t* __restrict__ vbase, int32_t* __restrict__ vgraph) {
    const int64_t vb = vbase[blockIdx.x], ve = vbase[blockIdx.x + 1];
    for (int64_t v = vb + threadIdx.x; v < ve; v += blockDim.x) vgraph[v] = (int32_t)blockIdx.x;
}

__global__ void walk_init_kernel(int64_t nv, const int64_t* __restrict__ rp,
                                 int64_t* __restrict__ cur, int64_t* __restrict__ tot) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = rp[v + 1] - rp[v];
        cur[v] = d;
        tot[v] = d;
    }
}

__global__ void walk_level_kernel(int64_t nv, const int64_t* __restrict__ rp,
                                  const int32_t* __restrict__ ci, const int32_t* __restrict__ vgraph,
                                  const int64_t* __restrict__ vbase, const int32_t* __restrict__ gk,
                                  int32_t level, const int64_t* __restrict__ cur,
                                  int64_t* __restrict__ nxt, int64_t* __restrict__ tot) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = vgraph[v];
        const int64_t ng = vbase[g + 1] - vbase[g];
        int64_t w = 0;
        if (level <= gk[g]) {
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) w += cur[ci[e]];
            w = w < ng ? w : ng;
            const int64_t t = tot[v] + w;
            tot[v] = t < ng - 1 ? t : ng - 1;
        }
        nxt[v] = w;
    }
}

__global__ void walk_pad_kernel(int64_t nv, const int64_t* __restrict__ tot,
                                int64_t* __restrict__ padded) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x)
        padded[v] = (tot[v] + 3) & ~(int64_t)3;
}

// Row starts and padded lengths from prefix offsets (the per-source path).
__global__ void rows_from_offsets_kernel(int64_t nv, const int64_t* __restrict__ kptr,
                                         int64_t* __restrict__ kstart, int32_t* __restrict__ klen) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv;
         v += (int64_t)gridDim.x * blockDim.x) {
        kstart[v] = kptr[v];
        klen[v] = (int32_t)(kptr[v + 1] - kptr[v]);
    }
}

// Rows of the layout kernel are padded to whole quads of ids: padded counts,
// and the padding entries set to the graph's sentinel id n (an LDS slot that
// holds a position far away, whose terms are exactly 0).
__global__ void pad_counts_kernel(int64_t nv, const int64_t* __restrict__ counts,
                                  int64_t* __restrict__ padded) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv;
         i += (int64_t)gridDim.x * blockDim.x)
        padded[i] = (counts[i] + 3) & ~(int64_t)3;
}

__global__ __launch_bounds__(kBlock) void pad_rows_kernel(const int64_t* __restrict__ vbase,
                                                          const int64_t* __restrict__ kptr,
                                                          const int64_t* __restrict__ counts,
                                                          uint16_t* __restrict__ kidx) {
    const int64_t vb = vbase[blockIdx.x];
    const int n = (int)(vbase[blockIdx.x + 1] - vb);
    for (int v = threadIdx.x; v < n; v += kBlock) {
        const int64_t e1 = kptr[vb + v + 1];
        for (int64_t e = kptr[vb + v] + counts[vb + v]; e < e1; ++e) kidx[e] = (uint16_t)n;
    }
}

// ------------------------------------------------------------------ wave slices
// One workgroup per graph: its vertices' local ids by decreasing row length in
// quads (ties by id) -- a bitonic sort of (key, id) words in LDS.  Graphs of
// more than kOrderMax vertices keep the identity order (their slices are then
// less even, the results are the same).
constexpr int kOrderMax = 8192;
// Graphs of fewer than kOffsetLimit vertices store their wave slices' rows
// as 16-bit offsets of 8-byte slots (id x 8; the sentinel's n x 8 <= 65528):
// the byte offset of an FP32 position, so its address is one add of a 16-bit
// half; larger graphs keep ids.
constexpr int kOffsetLimit = 8192;

__global__ __launch_bounds__(kBlock) void row_order_kernel(const int64_t* __restrict__ vbase,
                                                           const int32_t* __restrict__ klen,
                                                           uint16_t* __restrict__ order) {
    __shared__ uint32_t s_key[kOrderMax];
    const int64_t vb = vbase[blockIdx.x];
    const int n = (int)(vbase[blockIdx.x + 1] - vb);
    if (n > kOrderMax) {
        for (int i = threadIdx.x; i < n; i += kBlock) order[vb + i] = (uint16_t)i;
        return;
    }
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = threadIdx.x; i < np; i += kBlock) {
        // a row has at most 65534 entries, so at most 16384 quads
        const uint32_t q = i < n ? (uint32_t)(klen[vb + i] >> 2) : 0u;
        s_key[i] = i < n ? ((0xFFFFu - q) << 16) | (uint32_t)i : 0xFFFFFFFFu;
    }
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < np; i += kBlock) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const uint32_t x = s_key[i], y = s_key[j];
                    if ((x > y) == up) {
                        s_key[i] = y;
                        s_key[j] = x;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = threadIdx.x; i < n; i += kBlock) order[vb + i] = (uint16_t)(s_key[i] & 0xFFFFu);
}

// One wavefront per slice: its lanes' vertices (the graph's sentinel id n for
// lanes past the end), row quads and degrees, and the slice's sizes (quads
// rounded up to even, adjacency entries) for the offset scans.
__global__ __launch_bounds__(kBlock) void sell_dims_kernel(
    int64_t nslices, const int32_t* __restrict__ sgraph, const int64_t* __restrict__ vbase,
    const int64_t* __restrict__ sbase, const int32_t* __restrict__ klen,
    const int64_t* __restrict__ rp, const uint16_t* __restrict__ order,
    SellSlice* __restrict__ hdr, uint2* __restrict__ smeta, int64_t* __restrict__ szk,
    int64_t* __restrict__ sza) {
    const int64_t sl = (int64_t)blockIdx.x * (kBlock / 64) + wave_id();
    if (sl >= nslices) return;
    const int lane = lane64();
    const int g = sgraph[sl];
    const int64_t vb = vbase[g];
    const int n = (int)(vbase[g + 1] - vb);
    const int i = (int)(sl - sbase[g]) * 64 + lane;
    const bool live = i < n;
    const int v = live ? (int)order[vb + i] : n;
    const int nq = live ? klen[vb + v] >> 2 : 0;
    const int deg = live ? (int)(rp[vb + v + 1] - rp[vb + v]) : 0;
    const int Q = (wave_max(nq) + 1) & ~1;
    const int D = wave_max(deg);
    smeta[sl * 64 + lane] = make_uint2((uint32_t)v, (uint32_t)nq | ((uint32_t)deg << 16));
    if (lane == 0) {
        szk[sl] = (int64_t)Q * 64;
        sza[sl] = (int64_t)((D + 3) & ~3) * 64;
        hdr[sl].nq = Q;
        hdr[sl].na = D;
    }
}

// One wavefront per slice: the interleaved rows (sentinel quads past a row's
// end) and adjacency (sentinel ids past a vertex's degree, up to a multiple
// of four), and the slice's offsets.
__global__ __launch_bounds__(kBlock) void sell_fill_kernel(
    int64_t nslices, const int32_t* __restrict__ sgraph, const int64_t* __restrict__ vbase,
    const int64_t* __restrict__ kstart, const uint16_t* __restrict__ kidx,
    const int64_t* __restrict__ rp, const uint16_t* __restrict__ ci16,
    const int64_t* __restrict__ koff, const int64_t* __restrict__ aoff,
    const uint2* __restrict__ smeta, SellSlice* __restrict__ hdr, uint2* __restrict__ sk,
    uint16_t* __restrict__ sa) {
    const int64_t sl = (int64_t)blockIdx.x * (kBlock / 64) + wave_id();
    if (sl >= nslices) return;
    const int lane = lane64();
    const int g = sgraph[sl];
    const int64_t vb = vbase[g];
    const uint32_t n = (uint32_t)(vbase[g + 1] - vb);
    const uint2 m = smeta[sl * 64 + lane];
    const int v = (int)m.x;
    const int nq = (int)(m.y & 0xFFFFu), deg = (int)(m.y >> 16);
    const int Q = hdr[sl].nq, D = hdr[sl].na;
    const int64_t ko = koff[sl], ao = aoff[sl];
    // a lane past the graph's end (v = n) reads no row
    const uint2* row = reinterpret_cast<const uint2*>(kidx + (v < (int)n ? kstart[vb + v] : 0));
    const uint2 sent = make_uint2(n | (n << 16), n | (n << 16));
    // both halves below 8192, so one shift scales both
    const int sh = n < (uint32_t)kOffsetLimit ? 3 : 0;
    for (int j = 0; j < Q; ++j) {
        const uint2 w = j < nq ? row[j] : sent;
        sk[ko + (int64_t)j * 64 + lane] = make_uint2(w.x << sh, w.y << sh);
    }
    const uint16_t* arow = ci16 + rp[vb + v];
    // adjacency in groups of four entries per lane (8 contiguous bytes, one
    // load), group g of lane l at entries 256 g + 4 l
    for (int j = 0; j < ((D + 3) & ~3); ++j)
        sa[ao + (int64_t)(j >> 2) * 256 + lane * 4 + (j & 3)] = j < deg ? arow[j] : (uint16_t)n;
    if (lane == 0) {
        hdr[sl].koff = ko;
        hdr[sl].aoff = ao;
    }
}

// ------------------------------------------------------------------ the persistent kernel
// The temperature cap and synchronous move of one vertex (its new position),
// with its share of the iteration statistics.  A non-finite force -- a term
// overflowed -- leaves the vertex in place and counts it (the graph's run
// stops).
template <class P>
__device__ __forceinline__ typename P::vec2 batch_move(const BatchDesc& G, typename P::vec2 xv,
                                                       double fx, double fy, double t,
                                                       double& energy, double& maxd,
                                                       int64_t& moved) {
    using R = typename P::real;
    typename P::vec2 nx = xv;
    if constexpr (sizeof(R) == 4) {
        // FP32 positions: the move in FP32 (one lane per vertex does this
        // part, so its instruction count matters); |Delta| = the capped length
        float l, dx, dy;
        if (capped_move_f32(fx, fy, t, dx, dy, l)) {
            energy += fx * fx + fy * fy;
            nx.x = xv.x + dx;
            nx.y = xv.y + dy;
            maxd = (double)l > maxd ? (double)l : maxd;
            moved += (double)l > G.stop_displacement ? 1 : 0;
        } else {
            moved += kNonfiniteOne;
        }
    } else {
        double dx, dy;
        if (capped_move(fx, fy, t, dx, dy)) {
            energy += fx * fx + fy * fy;
            nx.x = (R)((double)xv.x + dx);
            nx.y = (R)((double)xv.y + dy);
            const double dl = sqrt(dx * dx + dy * dy);
            maxd = dl > maxd ? dl : maxd;
            moved += dl > G.stop_displacement ? 1 : 0;
        } else {
            moved += kNonfiniteOne;
        }
    }
    return nx;
}

// The attraction term of the batched launch: attract() with p = 2, the FP32
// distance taken by the hardware square root (within 1 ulp).  The correctly
// rounded square root costs ~17 more instructions per edge, about a fifth of
// a vertex's work in these graphs of short rows; in FP64 attract() itself.
template <class P>
__device__ __forceinline__ void batch_attract(typename P::real xv, typename P::real yv,
                                              typename P::vec2 p, typename P::real dparam,
                                              Acc<typename P::real, P::kahan>& acc) {
    if constexpr (sizeof(typename P::real) == 4) {
        const float dx = p.x - xv;
        const float dy = p.y - yv;
        const float s = __builtin_amdgcn_sqrtf(dx * dx + dy * dy) * dparam;
        acc.add(dx * s, dy * s);
    } else {
        attract<P>(xv, yv, p, dparam, acc);
    }
}

template <class P, int LPV>
__device__ __forceinline__ void batch_graph_iteration(
    const BatchArgs& a, const BatchDesc& G, const typename P::vec2* __restrict__ cur,
    typename P::vec2* __restrict__ nxt, double t, double& energy, double& maxd, int64_t& moved,
    int& coinc) {
    using R = typename P::real;
    using V = typename P::vec2;
    const double d2 = G.d * G.d;
    // repulsion is summed without its factor d^2 (applied once per row), so
    // attraction (x_u - x_v) delta / d enters the same sum divided by d^2
    const R dpar = sizeof(R) == 4 ? (R)(1.0 / (G.d * d2)) : (R)(G.d * d2);
    constexpr int ngroups = kBatchBlock / LPV;
    const int grp = threadIdx.x / LPV;
    const int gl = threadIdx.x % LPV;
    for (int v0 = 0; v0 < G.n; v0 += ngroups) {
        const int v = v0 + grp;
        Acc<R, P::kahan> acc;
        V xv;
        xv.x = 0;
        xv.y = 0;
        if (v < G.n) {
            xv = cur[v];
            // the row as quads of 16-bit local ids (padded with the sentinel id n)
            const int64_t kb = a.kstart[G.vbase + v], ke = kb + a.klen[G.vbase + v];
            const uint2* __restrict__ q4 = reinterpret_cast<const uint2*>(a.kidx + kb);
            const int nq = (int)((ke - kb) >> 2);
            R mindd = R(1);
            int q = gl;
            // four quads per lane per step (the adds in the same order as
            // two-quad steps, so the same bits)
            for (; q + 3 * LPV < nq; q += 4 * LPV) {
                const uint2 w0 = q4[q], w1 = q4[q + LPV], w2 = q4[q + 2 * LPV], w3 = q4[q + 3 * LPV];
                R ax, ay, bx, by;
                repulse4<P>(cur[w0.x & 0xFFFFu], cur[w0.x >> 16], cur[w0.y & 0xFFFFu],
                            cur[w0.y >> 16], xv.x, xv.y, ax, ay, mindd);
                repulse4<P>(cur[w1.x & 0xFFFFu], cur[w1.x >> 16], cur[w1.y & 0xFFFFu],
                            cur[w1.y >> 16], xv.x, xv.y, bx, by, mindd);
                acc.add(ax + bx, ay + by);
                repulse4<P>(cur[w2.x & 0xFFFFu], cur[w2.x >> 16], cur[w2.y & 0xFFFFu],
                            cur[w2.y >> 16], xv.x, xv.y, ax, ay, mindd);
                repulse4<P>(cur[w3.x & 0xFFFFu], cur[w3.x >> 16], cur[w3.y & 0xFFFFu],
                            cur[w3.y >> 16], xv.x, xv.y, bx, by, mindd);
                acc.add(ax + bx, ay + by);
            }
            for (; q + LPV < nq; q += 2 * LPV) {
                const uint2 w0 = q4[q];
                const uint2 w1 = q4[q + LPV];
                R ax, ay, bx, by;
                repulse4<P>(cur[w0.x & 0xFFFFu], cur[w0.x >> 16], cur[w0.y & 0xFFFFu],
                            cur[w0.y >> 16], xv.x, xv.y, ax, ay, mindd);
                repulse4<P>(cur[w1.x & 0xFFFFu], cur[w1.x >> 16], cur[w1.y & 0xFFFFu],
                            cur[w1.y >> 16], xv.x, xv.y, bx, by, mindd);
                acc.add(ax + bx, ay + by);
            }
            for (; q < nq; q += LPV) {
                const uint2 w0 = q4[q];
                R ax, ay;
                repulse4<P>(cur[w0.x & 0xFFFFu], cur[w0.x >> 16], cur[w0.y & 0xFFFFu],
                            cur[w0.y >> 16], xv.x, xv.y, ax, ay, mindd);
                acc.add(ax, ay);
            }
            if (mindd <= coincidence_bias<R>()) {
                const uint16_t* row = a.kidx + kb;
                const int len = (int)(ke - kb);
                for (int e = gl; e < len; e += LPV) {
                    const V p = cur[row[e]];
                    coinc += (row[e] != G.n && p.x == xv.x && p.y == xv.y) ? 1 : 0;
                }
            }
            const int64_t ab = a.rp[G.vbase + v], ae = a.rp[G.vbase + v + 1];
            for (int64_t j = ab + gl; j < ae; j += LPV) batch_attract<P>(xv.x, xv.y, cur[a.ci[j]], dpar, acc);
        }
        const double fx = group_sum<LPV>(acc.x()) * d2;
        const double fy = group_sum<LPV>(acc.y()) * d2;
        if (v < G.n && gl == 0) nxt[v] = batch_move<P>(G, xv, fx, fy, t, energy, maxd, moved);
    }
}

// Rows of graphs run with one lane per vertex, from the graph's wave slices:
// each wavefront takes the next slice (longest rows first) from the
// iteration's counter in LDS, and writes the slice's energy to e_slice[slice]
// (the iteration's energy is their sum in slice order).  All lanes load and evaluate every quad step of
// the slice; a lane adds a step's terms only within its own row, in the same
// grouping as the row layout (pairs of quads, a last odd quad alone), and its
// adjacency terms only within its degree, so each vertex gets the same bits.
template <class P, bool OFF>
__device__ __forceinline__ void batch_graph_iteration_slices(
    const BatchArgs& a, const BatchDesc& G, const typename P::vec2* __restrict__ cur,
    typename P::vec2* __restrict__ nxt, double t, int* s_next, double* e_slice, double& maxd,
    int64_t& moved, int& coinc) {
    using R = typename P::real;
    using V = typename P::vec2;
    const double d2 = G.d * G.d;
    const R dpar = sizeof(R) == 4 ? (R)(1.0 / (G.d * d2)) : (R)(G.d * d2);
    const int lane = lane64();
    // a row entry's position: entries are ids, or (OFF) offsets of 8-byte
    // slots -- byte offsets of FP32 positions, half those of FP64 ones
    const auto at = [cur](uint32_t h) -> V {
        if constexpr (OFF)
            return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(cur) +
                                               h * (uint32_t)(sizeof(V) / 8));
        else
            return cur[h];
    };
    const int ns = (G.n + 63) >> 6;
    for (;;) {
        int sl = 0;
        if (lane == 0) sl = atomicAdd(s_next, 1);
        sl = __builtin_amdgcn_readfirstlane(sl);
        if (sl >= ns) break;
        const int64_t si = G.sbase + sl;
        // the slice's header through the scalar cache (built by an earlier
        // launch, only read here)
        typedef const __attribute__((address_space(4))) SellSlice* SellPtr;
        const SellPtr hp = (SellPtr)(a.sell + si);
        SellSlice S;
        S.koff = hp->koff;
        S.aoff = hp->aoff;
        S.nq = hp->nq;
        S.na = hp->na;
        // groups of four quad steps, the next group's loads issued before
        // this group's terms (rows stream from HBM: a wait per group would
        // leave each slice waiting on its row length over four latencies).
        // The first group is issued before the lane records, whose wait
        // then overlaps it.
        const uint2* __restrict__ q = a.sk + S.koff + lane;
        uint2 n0 = make_uint2(0, 0), n1 = n0, n2 = n0, n3 = n0;
        if (S.nq >= 4) {
            n0 = q[0];
            n1 = q[64];
            n2 = q[128];
            n3 = q[192];
        }
        const uint2 m = a.smeta[si * 64 + lane];
        // the first four adjacency entries, loaded now so that they arrive
        // during the row's terms
        const uint2* __restrict__ aq = reinterpret_cast<const uint2*>(a.sa + S.aoff) + lane;
        uint2 ag = make_uint2(0, 0);
        if (S.na > 0) ag = aq[0];
        const int v = (int)m.x;  // n (the far sentinel) past the graph's end
        const int nq = (int)(m.y & 0xFFFFu), deg = (int)(m.y >> 16);
        const V xv = cur[v];
        Acc<R, P::kahan> acc;
        R mindd = R(1);
        int j = 0;
        for (; j + 3 < S.nq; j += 4) {
            const uint2 w0 = n0, w1 = n1, w2 = n2, w3 = n3;
            if (j + 7 < S.nq) {  // uniform
                n0 = q[(int64_t)(j + 4) * 64];
                n1 = q[(int64_t)(j + 5) * 64];
                n2 = q[(int64_t)(j + 6) * 64];
                n3 = q[(int64_t)(j + 7) * 64];
            }
            R ax, ay, bx, by;
            repulse4<P>(at(w0.x & 0xFFFFu), at(w0.x >> 16), at(w0.y & 0xFFFFu),
                        at(w0.y >> 16), xv.x, xv.y, ax, ay, mindd);
            repulse4<P>(at(w1.x & 0xFFFFu), at(w1.x >> 16), at(w1.y & 0xFFFFu),
                        at(w1.y >> 16), xv.x, xv.y, bx, by, mindd);
            if (j + 1 < nq) acc.add(ax + bx, ay + by);
            else if (j < nq) acc.add(ax, ay);
            repulse4<P>(at(w2.x & 0xFFFFu), at(w2.x >> 16), at(w2.y & 0xFFFFu),
                        at(w2.y >> 16), xv.x, xv.y, ax, ay, mindd);
            repulse4<P>(at(w3.x & 0xFFFFu), at(w3.x >> 16), at(w3.y & 0xFFFFu),
                        at(w3.y >> 16), xv.x, xv.y, bx, by, mindd);
            if (j + 3 < nq) acc.add(ax + bx, ay + by);
            else if (j + 2 < nq) acc.add(ax, ay);
        }
        for (; j < S.nq; j += 2) {  // S.nq is even
            const uint2 w0 = q[(int64_t)j * 64], w1 = q[(int64_t)(j + 1) * 64];
            R ax, ay, bx, by;
            repulse4<P>(at(w0.x & 0xFFFFu), at(w0.x >> 16), at(w0.y & 0xFFFFu),
                        at(w0.y >> 16), xv.x, xv.y, ax, ay, mindd);
            repulse4<P>(at(w1.x & 0xFFFFu), at(w1.x >> 16), at(w1.y & 0xFFFFu),
                        at(w1.y >> 16), xv.x, xv.y, bx, by, mindd);
            if (j + 1 < nq) acc.add(ax + bx, ay + by);
            else if (j < nq) acc.add(ax, ay);
        }
        const bool live = v < G.n;
        // padding quads hold the far sentinel (an infinite squared distance),
        // so mindd sees only the row's own pairs
        if (live && mindd <= coincidence_bias<R>()) {
            const int64_t kb = a.kstart[G.vbase + v], ke = kb + a.klen[G.vbase + v];
            const uint16_t* row = a.kidx + kb;
            for (int64_t e = 0; e < ke - kb; ++e) {
                const V p = cur[row[e]];
                coinc += (row[e] != G.n && p.x == xv.x && p.y == xv.y) ? 1 : 0;
            }
        }
        // the slice's adjacency, four entries (one load) at a time, the next
        // group loaded before this one's terms; padding holds the sentinel id
        // n, a valid slot.  All four positions are read before the first
        // term (the empty asm keeps the reads from being moved into the
        // per-lane branches); terms in edge order.
        for (int e = 0; e < S.na; e += 4) {
            const uint2 g = ag;
            if (e + 4 < S.na) ag = aq[(int64_t)((e >> 2) + 1) * 64];  // uniform
            const int u0 = (int)(g.x & 0xFFFFu), u1 = (int)(g.x >> 16);
            const int u2 = (int)(g.y & 0xFFFFu), u3 = (int)(g.y >> 16);
            const V p0 = cur[u0], p1 = cur[u1], p2 = cur[u2], p3 = cur[u3];
            asm volatile("" ::"v"(p0.x), "v"(p1.x), "v"(p2.x), "v"(p3.x));
            if (e < deg) batch_attract<P>(xv.x, xv.y, p0, dpar, acc);
            if (e + 1 < deg) batch_attract<P>(xv.x, xv.y, p1, dpar, acc);
            if (e + 2 < deg) batch_attract<P>(xv.x, xv.y, p2, dpar, acc);
            if (e + 3 < deg) batch_attract<P>(xv.x, xv.y, p3, dpar, acc);
        }
        double energy = 0.0;
        if (live) {
            const double fx = acc.x() * d2;
            const double fy = acc.y() * d2;
            nxt[v] = batch_move<P>(G, xv, fx, fy, t, energy, maxd, moved);
        }
        // the slice's energy, summed in a fixed order whichever wavefront
        // took the slice
        const double se = wave_sum(energy);
        if (lane == 0) e_slice[sl] = se;
    }
}

template <int PREC>
__device__ __forceinline__ void batch_layout_body(const BatchArgs& a) {
    using P = Prec<PREC>;
    using V = typename P::vec2;
    extern __shared__ __align__(16) unsigned char s_raw[];
    __shared__ int s_g;
    __shared__ int s_sl[2];  // next wave slice, for alternate iterations
    // per-wave statistics, two sets used by alternate iterations (a set is
    // rewritten two iterations later, after a barrier every reader has passed)
    __shared__ double s_e[2][kBatchWaves], s_m[2][kBatchWaves];
    __shared__ int64_t s_mv[2][kBatchWaves], s_c[2][kBatchWaves];
    const int lane = lane64(), w = wave_id();
    for (;;) {
        if (threadIdx.x == 0) s_g = atomicAdd(a.work, 1);
        __syncthreads();
        // uniform across the workgroup: the graph's descriptor goes to scalar
        // registers
        const int gi = __builtin_amdgcn_readfirstlane(s_g);
        if (gi >= a.count) break;
        const int gid = a.order[gi];
        const BatchDesc G = a.graphs[gid];
        if (threadIdx.x == 0 && a.t_start) a.t_start[gid] = wall_clock64();
        // two position buffers of n + 1 slots; slot n holds the far sentinel
        V* cur = reinterpret_cast<V*>(s_raw);
        V* nxt = cur + G.n + 1;
        // per-slice energies of alternate iterations (one lane per vertex), in
        // the workgroup's own part of the scratch
        const int ns = (G.n + 63) >> 6;
        double* e_sl = a.escratch + (int64_t)blockIdx.x * 2 * a.slices_max;
        const V* src = reinterpret_cast<const V*>(G.pos);
        for (int i = threadIdx.x; i < G.n; i += kBatchBlock) cur[i] = src[i];
        if (threadIdx.x == 0) {
            V far;
            far.x = sizeof(far.x) == 4 ? (decltype(far.x))1e30f : (decltype(far.x))1e300;
            far.y = far.x;
            cur[G.n] = far;
            nxt[G.n] = far;
            s_sl[0] = 0;
            s_sl[1] = 0;
        }
        __syncthreads();
        double E = 0.0, M = 0.0;
        int64_t MV = 0, C = 0, NF = 0;
        int run = 0, stopped = 0;
        for (int h = 0; h < G.iters; ++h) {
            const double t = a.temps[G.t_off + h];
            double energy = 0.0, maxd = 0.0;
            int64_t moved = 0;
            int coinc = 0;
            // the other iteration's slice counter was last used before the
            // previous barrier: reset it for the next iteration
            if (threadIdx.x == 0) s_sl[(h + 1) & 1] = 0;
            switch (G.lpv) {
                case 1:
                    if (G.n < kOffsetLimit)
                        batch_graph_iteration_slices<P, true>(a, G, cur, nxt, t, &s_sl[h & 1],
                                                              e_sl + (h & 1) * ns, maxd, moved, coinc);
                    else
                        batch_graph_iteration_slices<P, false>(a, G, cur, nxt, t, &s_sl[h & 1],
                                                               e_sl + (h & 1) * ns, maxd, moved, coinc);
                    break;
                case 2: batch_graph_iteration<P, 2>(a, G, cur, nxt, t, energy, maxd, moved, coinc); break;
                case 4: batch_graph_iteration<P, 4>(a, G, cur, nxt, t, energy, maxd, moved, coinc); break;
                case 8: batch_graph_iteration<P, 8>(a, G, cur, nxt, t, energy, maxd, moved, coinc); break;
                case 16: batch_graph_iteration<P, 16>(a, G, cur, nxt, t, energy, maxd, moved, coinc); break;
                case 32: batch_graph_iteration<P, 32>(a, G, cur, nxt, t, energy, maxd, moved, coinc); break;
                default: batch_graph_iteration<P, 64>(a, G, cur, nxt, t, energy, maxd, moved, coinc); break;
            }
            // iteration statistics: per wave, then every thread combines the
            // waves' values in the same fixed order (the same bits everywhere).
            // The barrier also ends this iteration's reads of cur and writes
            // of nxt before the next iteration swaps them.
            const int par = h & 1;
            const double we = wave_sum(energy);
            const double wm = wave_max(maxd);
            const int64_t wmv = wave_sum(moved);
            const int64_t wc = wave_sum((int64_t)coinc);
            if (lane == 0) {
                s_e[par][w] = we;
                s_m[par][w] = wm;
                s_mv[par][w] = wmv;
                s_c[par][w] = wc;
            }
            __syncthreads();
            double e = s_e[par][0], m = s_m[par][0];
            int64_t mv = s_mv[par][0], c = s_c[par][0];
            for (int i = 1; i < kBatchWaves; ++i) {
                e += s_e[par][i];
                m = s_m[par][i] > m ? s_m[par][i] : m;
                mv += s_mv[par][i];
                c += s_c[par][i];
            }
            E = e;
            M = m;
            C = c;
            NF = mv >> 32;  // vertices with a non-finite force
            mv &= 0xFFFFFFFFll;
            MV = mv;
            ++run;
            V* tmp = cur;
            cur = nxt;
            nxt = tmp;
            if (NF > 0) break;  // a non-finite force ends this graph's run
            if (G.stop_fraction > 0.0 && (double)mv < G.stop_fraction * (double)G.n_active) {
                stopped = 1;
                break;
            }
        }
        if (G.lpv == 1 && run > 0) {
            // the last iteration's slice energies (written before its barrier)
            const double* es = e_sl + ((run - 1) & 1) * ns;
            double e = 0.0;
            for (int i = 0; i < ns; ++i) e += es[i];
            E = e;
        }
        V* dst = reinterpret_cast<V*>(G.pos);
        for (int i = threadIdx.x; i < G.n; i += kBatchBlock) dst[i] = cur[i];
        if (threadIdx.x == 0) {
            gila_stats st;
            st.iterations_run = run;
            st.stopped = stopped;
            st.moved = MV;
            st.max_disp = M;
            st.energy = E;
            st.coincident = C;
            st.nonfinite = NF;
            a.stats[gid] = st;
        }
        __syncthreads();
        if (threadIdx.x == 0 && a.t_end) {
            // the workgroup's position stores have completed (the barrier
            // above, then a wait for this wave's own stores)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            a.t_end[gid] = wall_clock64();
        }
        __syncthreads();
    }
}

// The FP32 launches are held to 128 VGPRs, i.e. four waves per SIMD: the
// launch waits on the latency of each iteration's row loads, and the
// compiler's free choice sits just above 128 (three waves per SIMD).  The
// FP64 launch keeps its free allocation, which the cap would make spill.
template <int PREC>
__global__ __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(4)))
void batch_layout_kernel(BatchArgs a) {
    batch_layout_body<PREC>(a);
}

__global__ __launch_bounds__(kBatchBlock) void batch_layout_kernel_f64(BatchArgs a) {
    batch_layout_body<GILA_FP64>(a);
}

__global__ void reset_work_kernel(int32_t* w) { *w = 0; }

// ------------------------------------------------------------------ lanes per vertex
// Row-length class of a graph: floor(log2(mean |N_v(k)|)), clamped to the table.
static int row_class(int64_t P, int32_t n) {
    const double mean = n > 0 ? (double)P / n : 0.0;
    int c = 0;
    while (c < kClasses - 1 && mean >= (double)(4 << c)) ++c;
    return c;
}

// Default lanes per vertex of a class: one lane per vertex up to rows of
// about 128 entries, then enough lanes for about 128 entries each.  More lanes
// per vertex add a cross-lane reduction per vertex and leave lanes idle at the
// end of short rows: on graphs of 50 to 5,000 vertices with mean rows of 32 to
// 128 entries, one lane per vertex ran the launch in 58% of the time that
// eight entries per lane took.
static int default_lpv(int cls) {
    const int mean_hi = 4 << cls;
    int l = 1;
    while (l < 64 && l * 128 < mean_hi) l *= 2;
    return l;
}

// Lanes per vertex that let one round of a small graph's vertices fill the
// workgroup: the largest power of two L <= 64 with n L <= kBatchBlock (1 for
// graphs of at least kBatchBlock / 2 vertices).  A graph's plan takes at least
// this many, whatever its class's choice.
static int fill_lanes(int32_t n) {
    int l = 1;
    while (l < 64 && (int64_t)n * l * 2 <= kBatchBlock) l *= 2;
    return l;
}


size_t batch_lds_bytes(int32_t nmax, int precision) {
    return (size_t)2 * ((size_t)std::max(nmax, 1) + 1) * (precision == GILA_FP64 ? 16 : 8);
}

static void launch_batch_kernel(int precision, int grid, size_t lds, hipStream_t s,
                                const BatchArgs& a) {
    switch (precision) {
        case GILA_FP64:
            hipLaunchKernelGGL(batch_layout_kernel_f64, dim3(grid), dim3(kBatchBlock), lds, s, a);
            break;
        case GILA_FP32:
            hipLaunchKernelGGL(batch_layout_kernel<GILA_FP32>, dim3(grid), dim3(kBatchBlock), lds, s, a);
            break;
        default:
            hipLaunchKernelGGL(batch_layout_kernel<GILA_FP32_KAHAN>, dim3(grid), dim3(kBatchBlock), lds,
                               s, a);
            break;
    }
}

static void set_lds_attr(size_t lds) {
    if (lds <= 48 * 1024) return;
    (void)quiet(hipFuncSetAttribute((const void*)batch_layout_kernel_f64,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    (void)quiet(hipFuncSetAttribute((const void*)batch_layout_kernel<GILA_FP32>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    (void)quiet(hipFuncSetAttribute((const void*)batch_layout_kernel<GILA_FP32_KAHAN>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
}

static int batch_grid(const gila_batch* b, size_t lds) {
    const DeviceInfo& di = device_info(b->device);
    const size_t per_cu = std::max<size_t>(1, std::min<size_t>(4, (160u * 1024u) / (lds + 1024)));
    return (int)std::max<int64_t>(
        1, std::min<int64_t>(std::min<int64_t>((int64_t)di.cus * (int64_t)per_cu, b->count),
                             b->escratch_grid));
}

// The tuner: for every row-length class present in the batch, times each
// candidate lanes per vertex (1, 2, ..., 64) on up to 48 of the class's
// graphs (8 iterations at cap 0 from seeded positions in scratch memory) and
// keeps the fastest.  table[c] receives the choice for class c (0 where the
// class is absent), and every graph of the class takes it in the handle's
// plan.  Only an explicit gila_batch_tune runs it.
static int tune_plan(gila_batch* b, int precision, hipStream_t s, int32_t* table) {
    std::vector<int> todo;
    for (int c = 0; c < kClasses; ++c) {
        table[c] = 0;
        for (int32_t i = 0; i < b->count; ++i)
            if (b->cls[i] == c && b->n[i] > 0) {
                todo.push_back(c);
                break;
            }
    }
    if (todo.empty()) return GILA_OK;
    std::vector<BatchDesc> desc((size_t)b->count);
    for (int32_t i = 0; i < b->count; ++i) {
        BatchDesc& d = desc[i];
        d.vbase = b->vbase[i];
        d.sbase = b->sbase[i];
        d.n = b->n[i];
        d.n_active = b->n_active[i];
        d.cls = b->cls[i];
        d.d = 48.0;
        d.stop_displacement = 0.01;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GILA_HIP(hipEventCreate(&e0));
    GILA_HIP(hipEventCreate(&e1));
    const size_t pb = precision == GILA_FP64 ? 16 : 8;
    int rc = GILA_OK;
    for (int c : todo) {
        std::vector<int32_t> ids;
        for (int32_t i = 0; i < b->count && ids.size() < 48; ++i)
            if (b->cls[i] == c && b->n[i] > 0) ids.push_back(i);
        int64_t vtot = 0;
        int32_t nmax = 0;
        for (int32_t i : ids) {
            vtot += desc[i].n;
            nmax = std::max(nmax, desc[i].n);
        }
        void* scratch = nullptr;
        BatchDesc* d_desc = nullptr;
        int32_t* d_order = nullptr;
        double* d_t = nullptr;
        gila_stats* d_st = nullptr;
        rc = dalloc(&scratch, (size_t)vtot * pb);
        if (!rc) rc = dalloc_t(&d_desc, ids.size());
        if (!rc) rc = dalloc_t(&d_order, ids.size());
        if (!rc) rc = dalloc_t(&d_t, 8);
        if (!rc) rc = dalloc_t(&d_st, ids.size());
        const std::vector<double> temps(8, 0.0);  // t = 0: nothing moves
        std::vector<int32_t> ord(ids.size());
        std::iota(ord.begin(), ord.end(), 0);
        if (!rc && hipMemcpyAsync(d_t, temps.data(), 8 * sizeof(double), hipMemcpyHostToDevice, s))
            rc = fail(GILA_EDEVICE, "tuner upload");
        if (!rc && hipMemcpyAsync(d_order, ord.data(), ord.size() * 4, hipMemcpyHostToDevice, s))
            rc = fail(GILA_EDEVICE, "tuner upload");
        float best_ms = 1e30f;
        int best = default_lpv(c);
        const size_t lds = batch_lds_bytes(nmax, precision);
        set_lds_attr(lds);
        for (int lpv = 1; lpv <= 64 && !rc; lpv *= 2) {
            std::vector<BatchDesc> sub;
            int64_t off = 0;
            for (int32_t i : ids) {
                BatchDesc d = desc[i];
                d.pos = (char*)scratch + off * pb;
                // seeded positions in the paper's frame (the timing does not
                // depend on them beyond rare coincident pairs)
                rc = gila_init_positions(d.n, (uint64_t)i, 1200.0, 1200.0, precision, d.pos, s);
                if (rc) break;
                d.lpv = std::max(lpv, fill_lanes(d.n));
                d.iters = 8;
                d.t_off = 0;
                d.stop_fraction = 0.0;
                off += d.n;
                sub.push_back(d);
            }
            if (rc) break;
            if (hipMemcpyAsync(d_desc, sub.data(), sub.size() * sizeof(BatchDesc),
                               hipMemcpyHostToDevice, s) != hipSuccess) {
                rc = fail(GILA_EDEVICE, "tuner upload");
                break;
            }
            BatchArgs a{};
            a.count = (int32_t)sub.size();
            a.graphs = d_desc;
            a.order = d_order;
            a.kstart = b->kstart;
            a.klen = b->klen;
            a.kidx = b->kidx;
            a.rp = b->rp;
            a.ci = b->ci16;
            a.sell = b->d_sell;
            a.smeta = b->d_smeta;
            a.sk = b->d_sk;
            a.sa = b->d_sa;
            a.escratch = b->d_escratch;
            a.slices_max = (b->nmax + 63) / 64;
            a.temps = d_t;
            a.stats = d_st;
            a.work = b->d_work;
            const int grid = (int)std::min<int64_t>(std::min<int64_t>(a.count, device_info(b->device).cus),
                                                    b->escratch_grid);
            hipLaunchKernelGGL(reset_work_kernel, dim3(1), dim3(1), 0, s, b->d_work);
            (void)quiet(hipEventRecord(e0, s));
            launch_batch_kernel(precision, grid, lds, s, a);
            (void)quiet(hipEventRecord(e1, s));
            if (hipStreamSynchronize(s) != hipSuccess) {
                rc = fail(GILA_EDEVICE, "tuner run failed");
                break;
            }
            float ms = 0.f;
            (void)quiet(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_ms) {
                best_ms = ms;
                best = lpv;
            }
        }
        dfree_on(scratch, s);
        dfree_on(d_desc, s);
        dfree_on(d_order, s);
        dfree_on(d_t, s);
        dfree_on(d_st, s);
        if (rc) break;
        table[c] = best;
        for (int32_t i = 0; i < b->count; ++i)
            if (b->cls[i] == c) b->lpv[i] = std::max(best, fill_lanes(b->n[i]));
    }
    (void)quiet(hipEventDestroy(e0));
    (void)quiet(hipEventDestroy(e1));
    return rc;
}

void free_batch(gila_batch* b, Release rel) {
    if (!b) return;
    DeviceGuard g(b->device);
    if (b->gexec) (void)quiet(hipGraphExecDestroy(b->gexec));
    rel(b->kstart);
    rel(b->klen);
    rel(b->kidx);
    rel(b->rp);
    rel(b->ci16);
    rel(b->d_sell);
    rel(b->d_smeta);
    rel(b->d_sk);
    rel(b->d_sa);
    rel(b->d_escratch);
    rel(b->d_desc);
    rel(b->d_order);
    rel(b->d_temps);
    rel(b->d_stats);
    rel(b->d_clock);
    rel(b->d_work);
    delete b;
}

struct BatchHolder {
    gila_batch* p;
    ~BatchHolder() { free_batch(p); }
};

// A build temporary, released into the cache after the work on its stream.
template <class T>
struct DevTmp {
    hipStream_t s;
    T* p = nullptr;
    explicit DevTmp(hipStream_t st) : s(st) {}
    ~DevTmp() { dfree_on(p, s); }
};

// The wave slices of every graph (see the file comment): vertex order, slice
// sizes, offsets, interleaved rows and adjacency.  Needs the padded rows
// (kstart, klen, kidx), the union adjacency (rp) and its local ids (ci16).
static int build_slices(gila_batch* b, const int64_t* d_vb, hipStream_t s) {
    const int32_t count = b->count;
    b->sbase.assign((size_t)count + 1, 0);
    for (int32_t i = 0; i < count; ++i) b->sbase[i + 1] = b->sbase[i] + (b->n[i] + 63) / 64;
    const int64_t S = b->sbase[count];
    b->nslices = S;
    // room for the largest persistent grid (four workgroups per CU)
    b->escratch_grid = (int64_t)device_info(b->device).cus * 4;
    GILA_TRY(dalloc_t(&b->d_escratch,
                      (size_t)b->escratch_grid * 2 * (size_t)std::max(1, (b->nmax + 63) / 64)));
    if (S == 0) return GILA_OK;
    std::vector<int32_t> sgraph((size_t)S);
    for (int32_t i = 0; i < count; ++i)
        for (int64_t j = b->sbase[i]; j < b->sbase[i + 1]; ++j) sgraph[(size_t)j] = i;
    DevTmp<uint16_t> d_order(s);
    DevTmp<int32_t> d_sgraph(s);
    DevTmp<int64_t> d_sb(s), d_szk(s), d_sza(s), d_koff(s), d_aoff(s);
    GILA_TRY(dalloc_t(&d_order.p, (size_t)std::max<int64_t>(b->nv, 1)));
    GILA_TRY(dalloc_t(&d_sgraph.p, (size_t)S));
    GILA_TRY(dalloc_t(&d_sb.p, (size_t)count + 1));
    GILA_TRY(dalloc_t(&d_szk.p, (size_t)S));
    GILA_TRY(dalloc_t(&d_sza.p, (size_t)S));
    GILA_TRY(dalloc_t(&d_koff.p, (size_t)S + 1));
    GILA_TRY(dalloc_t(&d_aoff.p, (size_t)S + 1));
    GILA_TRY(dalloc_t(&b->d_sell, (size_t)S));
    GILA_TRY(dalloc_t(&b->d_smeta, (size_t)S * 64));
    GILA_HIP(hipMemcpyAsync(d_sgraph.p, sgraph.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, s));
    GILA_HIP(hipMemcpyAsync(d_sb.p, b->sbase.data(), sizeof(int64_t) * (count + 1),
                            hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(row_order_kernel, dim3(count), dim3(kBlock), 0, s, d_vb, b->klen, d_order.p);
    GILA_HIP(hipGetLastError());
    const int per_block = kBlock / 64;
    const dim3 sg((unsigned)((S + per_block - 1) / per_block));
    hipLaunchKernelGGL(sell_dims_kernel, sg, dim3(kBlock), 0, s, S, d_sgraph.p, d_vb, d_sb.p,
                       b->klen, b->rp, d_order.p, b->d_sell, b->d_smeta, d_szk.p, d_sza.p);
    GILA_HIP(hipGetLastError());
    GILA_TRY(exclusive_scan_i64(d_szk.p, d_koff.p, S, s));
    GILA_TRY(exclusive_scan_i64(d_sza.p, d_aoff.p, S, s));
    GILA_HIP(hipMemcpyAsync(&b->sell_quads, d_koff.p + S, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipMemcpyAsync(&b->sell_adj, d_aoff.p + S, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    GILA_TRY(dalloc_t(&b->d_sk, (size_t)std::max<int64_t>(b->sell_quads, 1)));
    GILA_TRY(dalloc_t(&b->d_sa, (size_t)std::max<int64_t>(b->sell_adj, 1)));
    hipLaunchKernelGGL(sell_fill_kernel, sg, dim3(kBlock), 0, s, S, d_sgraph.p, d_vb, b->kstart,
                       b->kidx, b->rp, b->ci16, d_koff.p, d_aoff.p, b->d_smeta, b->d_sell,
                       b->d_sk, b->d_sa);
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

int batch_build(const gila_csr* graphs, int32_t count, const int32_t* k, hipStream_t s,
                gila_batch** out) {
    if (!out) return fail(GILA_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 0) return fail(GILA_EINVAL, "count must be >= 0");
    if (count > 0 && (!graphs || !k)) return fail(GILA_EINVAL, "graphs or k is NULL");
    int dev = 0;
    GILA_HIP(hipGetDevice(&dev));
    BatchHolder h{new gila_batch()};
    gila_batch* b = h.p;
    b->device = dev;
    b->count = count;
    b->vbase.assign((size_t)count + 1, 0);
    b->ebase.assign((size_t)count + 1, 0);
    b->n.assign(count, 0);
    b->k.assign(count, 0);
    std::vector<GraphSrc> src(count);
    int32_t kmax = 1;
    for (int32_t i = 0; i < count; ++i) {
        const gila_csr& g = graphs[i];
        if (k[i] < 1) return fail(GILA_EINVAL, "graph %d: k must be >= 1", i);
        if (g.n < 0 || g.nnz < 0) return fail(GILA_EINVAL, "graph %d: negative size", i);
        if (g.n > 65535) return fail(GILA_EUNSUPPORTED, "graph %d: more than 65535 vertices", i);
        if (g.nnz % 2 || g.nnz > (int64_t)g.n * (g.n > 0 ? g.n - 1 : 0))
            return fail(GILA_EINVAL, "graph %d: bad nnz", i);
        if ((g.n > 0 && !g.row_ptr) || (g.nnz > 0 && !g.col_idx))
            return fail(GILA_EINVAL, "graph %d: NULL array", i);
        b->n[i] = g.n;
        b->k[i] = k[i];
        kmax = std::max(kmax, k[i]);
        b->nmax = std::max(b->nmax, g.n);
        b->vbase[i + 1] = b->vbase[i] + g.n;
        b->ebase[i + 1] = b->ebase[i] + g.nnz;
        src[i] = GraphSrc{g.n > 0 ? g.row_ptr : nullptr, g.col_idx, b->vbase[i], b->ebase[i],
                           g.nnz, g.n, 0};
    }
    b->nv = b->vbase[count];
    b->nnz = b->ebase[count];
    if (b->nv > INT32_MAX - 1) return fail(GILA_EUNSUPPORTED, "batch too large");
    if (count == 0) {  // an empty batch holds no device state
        *out = b;
        h.p = nullptr;
        return GILA_OK;
    }

    PhaseTimer pt("batch_build", s);
    DevTmp<GraphSrc> d_src(s);
    DevTmp<int32_t> d_flag(s), d_ci32(s), d_k(s), d_nact(s);
    DevTmp<int64_t> d_vb(s), d_counts(s), d_bounds(s);
    GILA_TRY(dalloc_t(&d_src.p, std::max(count, 1)));
    GILA_TRY(dalloc_t(&d_flag.p, 2));
    GILA_TRY(dalloc_t(&b->rp, (size_t)b->nv + 1));
    GILA_TRY(dalloc_t(&d_ci32.p, (size_t)b->nnz));
    GILA_TRY(dalloc_t(&b->ci16, (size_t)b->nnz));
    GILA_TRY(dalloc_t(&d_vb.p, (size_t)count + 1));
    GILA_TRY(dalloc_t(&d_k.p, std::max(count, 1)));
    GILA_TRY(dalloc_t(&d_nact.p, std::max(count, 1)));
    GILA_TRY(dalloc_t(&b->d_work, 1));
    GILA_HIP(hipMemsetAsync(d_flag.p, 0, 2 * sizeof(int32_t), s));
    GILA_HIP(hipMemsetAsync(b->rp, 0, sizeof(int64_t), s));
    GILA_HIP(hipMemcpyAsync(d_vb.p, b->vbase.data(), sizeof(int64_t) * (count + 1),
                            hipMemcpyHostToDevice, s));
    if (count > 0) {
        GILA_HIP(hipMemcpyAsync(d_src.p, src.data(), sizeof(GraphSrc) * count,
                                hipMemcpyHostToDevice, s));
        GILA_HIP(hipMemcpyAsync(d_k.p, b->k.data(), sizeof(int32_t) * count,
                                hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(gather_csr_kernel, dim3(count), dim3(kBlock), 0, s, d_src.p, b->rp,
                           d_ci32.p, d_flag.p);
        GILA_HIP(hipGetLastError());
        GILA_TRY(launch_validate_csr((int32_t)b->nv, b->nnz, b->rp, d_ci32.p, d_flag.p, s));
    }
    int32_t flag = 0;
    GILA_HIP(hipMemcpyAsync(&flag, d_flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    if (flag)
        return fail(GILA_EINVAL, "malformed CSR in batch:%s%s%s%s%s",
                    (flag & 16) ? " bad row_ptr" : "", (flag & 1) ? " column out of range" : "",
                    (flag & 2) ? " self-loop" : "", (flag & 4) ? " row not strictly ascending" : "",
                    (flag & 8) ? " not symmetric" : "");

    pt.mark("gather+validate");
    // k-hop rows as 16-bit local ids, each padded to whole quads with the
    // graph's sentinel id n; counts |N_v(k)|; per-graph blocks of kidx
    const int32_t nwords = std::max<int32_t>(1, (b->nmax + 31) / 32);
    GILA_TRY(dalloc_t(&d_counts.p, (size_t)std::max<int64_t>(b->nv, 1)));
    GILA_TRY(dalloc_t(&b->kstart, (size_t)std::max<int64_t>(b->nv, 1)));
    GILA_TRY(dalloc_t(&b->klen, (size_t)std::max<int64_t>(b->nv, 1)));
    // graphs whose CSR and three bitmaps per wavefront fit in LDS: one
    // workgroup per graph, one pass; otherwise one workgroup per source,
    // count then fill
    int64_t nnzmax = 0;
    for (int32_t i = 0; i < count; ++i) nnzmax = std::max(nnzmax, b->ebase[i + 1] - b->ebase[i]);
    const size_t max_lds = device_info(dev).max_lds_per_block;
    const int bfs_bs = batch_bfs_lds_bytes(b->nmax, nnzmax, 16) + 1024 <= max_lds ? 1024 : 512;
    const size_t bfs_lds = batch_bfs_lds_bytes(b->nmax, nnzmax, bfs_bs / 64);
    const bool per_graph = bfs_lds + 1024 <= max_lds &&
                           !(getenv("GILA_BATCH_BFS") && std::strcmp(getenv("GILA_BATCH_BFS"), "source") == 0);
    const int vg = (int)std::min<int64_t>(4096, (std::max<int64_t>(b->nv, 1) + kBlock - 1) / kBlock);
    if (per_graph) {
        // each graph's block: the sum of its rows' walk bounds
        DevTmp<int32_t> d_vgraph(s);
        DevTmp<int64_t> d_w0(s), d_w1(s), d_tot(s), d_bound(s), d_bscan(s), d_gbase(s);
        GILA_TRY(dalloc_t(&d_vgraph.p, (size_t)std::max<int64_t>(b->nv, 1)));
        GILA_TRY(dalloc_t(&d_w0.p, (size_t)std::max<int64_t>(b->nv, 1)));
        GILA_TRY(dalloc_t(&d_w1.p, (size_t)std::max<int64_t>(b->nv, 1)));
        GILA_TRY(dalloc_t(&d_tot.p, (size_t)std::max<int64_t>(b->nv, 1)));
        GILA_TRY(dalloc_t(&d_bound.p, (size_t)std::max<int64_t>(b->nv, 1)));
        GILA_TRY(dalloc_t(&d_bscan.p, (size_t)b->nv + 1));
        GILA_TRY(dalloc_t(&d_gbase.p, (size_t)count + 1));
        hipLaunchKernelGGL(vertex_graph_kernel, dim3(count), dim3(kBlock), 0, s, d_vb.p,
                           d_vgraph.p);
        hipLaunchKernelGGL(walk_init_kernel, dim3(vg), dim3(kBlock), 0, s, b->nv, b->rp, d_w0.p,
                           d_tot.p);
        int64_t* cur = d_w0.p;
        int64_t* nxt = d_w1.p;
        for (int32_t level = 2; level <= kmax; ++level) {
            hipLaunchKernelGGL(walk_level_kernel, dim3(vg), dim3(kBlock), 0, s, b->nv, b->rp,
                               d_ci32.p, d_vgraph.p, d_vb.p, d_k.p, level, cur, nxt, d_tot.p);
            std::swap(cur, nxt);
        }
        hipLaunchKernelGGL(walk_pad_kernel, dim3(vg), dim3(kBlock), 0, s, b->nv, d_tot.p,
                           d_bound.p);
        GILA_HIP(hipGetLastError());
        GILA_TRY(exclusive_scan_i64(d_bound.p, d_bscan.p, b->nv, s));
        hipLaunchKernelGGL(gather_bounds_kernel, dim3((count + 256) / 256), dim3(256), 0, s,
                           d_bscan.p, d_vb.p, count, d_gbase.p);
        GILA_HIP(hipGetLastError());
        GILA_HIP(hipMemcpyAsync(&b->kidx_size, d_gbase.p + count, sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        GILA_TRY(dalloc_t(&b->kidx, (size_t)b->kidx_size + 64));
        pt.mark("bounds");
        std::vector<int32_t> gorder((size_t)count);
        std::iota(gorder.begin(), gorder.end(), 0);
        std::stable_sort(gorder.begin(), gorder.end(),
                         [&](int32_t x, int32_t y) { return b->n[x] > b->n[y]; });
        DevTmp<int32_t> d_gorder(s);
        GILA_TRY(dalloc_t(&d_gorder.p, (size_t)count));
        GILA_HIP(hipMemcpyAsync(d_gorder.p, gorder.data(), sizeof(int32_t) * count,
                                hipMemcpyHostToDevice, s));
        BatchBfsArgs ga{};
        ga.count = count;
        ga.gorder = d_gorder.p;
        ga.vbase = d_vb.p;
        ga.rp = b->rp;
        ga.ci = d_ci32.p;
        ga.gk = d_k.p;
        ga.gbase = d_gbase.p;
        ga.counts = d_counts.p;
        ga.kstart = b->kstart;
        ga.klen = b->klen;
        ga.kidx = b->kidx;
        ga.work = d_flag.p + 1;
        ga.nmax = b->nmax;
        ga.nnzmax = nnzmax;
        GILA_TRY(run_batch_bfs(ga, bfs_lds, bfs_bs, dev, s));
        GILA_HIP(hipStreamSynchronize(s));
    } else if (b->nv > 0) {
        BfsArgs a{};
        a.n = (int32_t)b->nv;
        a.k = kmax;
        a.kmax = kmax;
        a.nverts = (int32_t)b->nv;
        a.nwords = nwords;
        a.rp = b->rp;
        a.ci = d_ci32.p;
        a.counts = d_counts.p;
        a.work = d_flag.p + 1;
        a.gvbase = d_vb.p;
        a.gk = d_k.p;
        a.ngraphs = count;
        a.qcap = std::max<int32_t>(1, b->nmax);
        GILA_TRY(run_bfs(false, dev, s, a));
        DevTmp<int64_t> d_padded(s), d_kptr(s);
        GILA_TRY(dalloc_t(&d_padded.p, (size_t)b->nv));
        GILA_TRY(dalloc_t(&d_kptr.p, (size_t)b->nv + 1));
        hipLaunchKernelGGL(pad_counts_kernel, dim3(vg), dim3(kBlock), 0, s, b->nv, d_counts.p,
                           d_padded.p);
        GILA_HIP(hipGetLastError());
        GILA_TRY(exclusive_scan_i64(d_padded.p, d_kptr.p, b->nv, s));
        GILA_HIP(hipMemcpyAsync(&b->kidx_size, d_kptr.p + b->nv, sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        GILA_TRY(dalloc_t(&b->kidx, (size_t)b->kidx_size + 64));
        a.kptr = d_kptr.p;
        a.kidx16 = b->kidx;
        GILA_TRY(run_bfs(true, dev, s, a));
        hipLaunchKernelGGL(pad_rows_kernel, dim3(count), dim3(kBlock), 0, s, d_vb.p, d_kptr.p,
                           d_counts.p, b->kidx);
        hipLaunchKernelGGL(rows_from_offsets_kernel, dim3(vg), dim3(kBlock), 0, s, b->nv,
                           d_kptr.p, b->kstart, b->klen);
        GILA_HIP(hipGetLastError());
        GILA_HIP(hipStreamSynchronize(s));
    }
    // true row offsets: the pair counts
    DevTmp<int64_t> d_ktrue(s);
    GILA_TRY(dalloc_t(&d_ktrue.p, (size_t)b->nv + 1));
    GILA_TRY(exclusive_scan_i64(d_counts.p, d_ktrue.p, b->nv, s));
    GILA_HIP(hipMemcpyAsync(&b->P, d_ktrue.p + b->nv, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    pt.mark("fill");
    if (count > 0) {
        hipLaunchKernelGGL(localize_kernel, dim3(count), dim3(kBlock), 0, s, d_src.p, d_ci32.p,
                           b->rp, b->ci16, d_nact.p);
        GILA_HIP(hipGetLastError());
    }
    // per-graph pair counts and non-isolated counts
    GILA_TRY(dalloc_t(&d_bounds.p, (size_t)count + 1));
    hipLaunchKernelGGL(gather_bounds_kernel, dim3((count + 256) / 256), dim3(256), 0, s, d_ktrue.p,
                       d_vb.p, count, d_bounds.p);
    GILA_HIP(hipGetLastError());
    std::vector<int64_t> bounds((size_t)count + 1, 0);
    b->n_active.assign(count, 0);
    GILA_HIP(hipMemcpyAsync(bounds.data(), d_bounds.p, sizeof(int64_t) * (count + 1),
                            hipMemcpyDeviceToHost, s));
    if (count > 0)
        GILA_HIP(hipMemcpyAsync(b->n_active.data(), d_nact.p, sizeof(int32_t) * count,
                                hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    pt.mark("localize+bounds");
    GILA_TRY(build_slices(b, d_vb.p, s));
    pt.mark("slices");
    b->Pg.assign(count, 0);
    b->cls.assign(count, 0);
    b->lpv.assign(count, 1);
    std::vector<int64_t> work(count);
    for (int32_t i = 0; i < count; ++i) {
        b->Pg[i] = bounds[i + 1] - bounds[i];
        b->cls[i] = row_class(b->Pg[i], b->n[i]);
        b->lpv[i] = std::max(default_lpv(b->cls[i]), fill_lanes(b->n[i]));
        work[i] = b->Pg[i] + (b->ebase[i + 1] - b->ebase[i]) + 8ll * b->n[i];
    }
    b->order.resize(count);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int32_t x, int32_t y) { return work[x] > work[y]; });
    GILA_TRY(dalloc_t(&b->d_order, std::max(count, 1)));
    GILA_TRY(dalloc_t(&b->d_desc, std::max(count, 1)));
    GILA_TRY(dalloc_t(&b->d_stats, std::max(count, 1)));
    GILA_TRY(dalloc_t(&b->d_clock, 2 * (size_t)std::max(count, 1)));
    if (count > 0)
        GILA_HIP(hipMemcpyAsync(b->d_order, b->order.data(), sizeof(int32_t) * count,
                                hipMemcpyHostToDevice, s));
    GILA_HIP(hipStreamSynchronize(s));
    pt.mark("order");
    b->device_bytes = 8 * (b->nv + 1) + 12 * b->nv + 2 * (b->kidx_size + b->nnz) +
                      (int64_t)(sizeof(BatchDesc) + 4 + sizeof(gila_stats)) * count +
                      (int64_t)(sizeof(SellSlice) + 64 * sizeof(uint2)) * b->nslices +
                      8 * b->sell_quads + 2 * b->sell_adj +
                      16 * b->escratch_grid * (int64_t)std::max(1, (b->nmax + 63) / 64);
    *out = b;
    h.p = nullptr;
    return GILA_OK;
}

int batch_run(gila_batch* b, const gila_params* params, void* const* pos, hipStream_t s,
              gila_stats* out, bool use_graph) {
    const int32_t count = b->count;
    if (count == 0) return GILA_OK;
    if (!params || !pos) return fail(GILA_EINVAL, "params or pos is NULL");
    const int precision = params[0].precision;
    int64_t total_t = 0;
    for (int32_t i = 0; i < count; ++i) {
        GILA_TRY(check_params(&params[i], true));
        if (params[i].force_model != GILA_MODEL_FR)
            return fail(GILA_EUNSUPPORTED, "graph %d: the batched kernel runs the FR model only", i);
        if (params[i].precision != precision)
            return fail(GILA_EINVAL, "graph %d: all graphs of a batch share one precision", i);
        if (b->n[i] > 0 && !pos[i]) return fail(GILA_EINVAL, "graph %d: pos is NULL", i);
        total_t += params[i].iterations;
    }
    const size_t lds = batch_lds_bytes(b->nmax, precision);
    if (lds > device_info(b->device).max_lds_per_block - 2048)
        return fail(GILA_EUNSUPPORTED, "largest graph (%d vertices) does not fit in LDS",
                    b->nmax);
    std::vector<double> temps((size_t)std::max<int64_t>(total_t, 1));
    std::vector<BatchDesc> desc(count);
    int64_t off = 0;
    for (int32_t i = 0; i < count; ++i) {
        BatchDesc& d = desc[i];
        d.vbase = b->vbase[i];
        d.sbase = b->sbase[i];
        d.n = b->n[i];
        d.n_active = b->n_active[i];
        d.cls = b->cls[i];
        d.iters = params[i].iterations;
        d.t_off = (int32_t)off;
        d.d = params[i].ideal_length;
        d.stop_fraction = params[i].stop_fraction;
        d.stop_displacement = params[i].stop_displacement;
        d.pos = pos[i];
        if (params[i].iterations > 0)
            std::memcpy(&temps[off], params[i].temperature,
                        sizeof(double) * params[i].iterations);
        off += params[i].iterations;
    }
    for (int32_t i = 0; i < count; ++i) desc[i].lpv = b->lpv[i];
    if ((int64_t)temps.size() > b->temps_cap) {
        dfree(b->d_temps);
        b->d_temps = nullptr;
        b->temps_cap = 0;
        GILA_TRY(dalloc_t(&b->d_temps, temps.size()));
        b->temps_cap = (int64_t)temps.size();
        if (b->gexec) {
            (void)quiet(hipGraphExecDestroy(b->gexec));
            b->gexec = nullptr;
        }
    }
    GILA_HIP(hipMemcpyAsync(b->d_temps, temps.data(), sizeof(double) * temps.size(),
                            hipMemcpyHostToDevice, s));
    GILA_HIP(hipMemcpyAsync(b->d_desc, desc.data(), sizeof(BatchDesc) * count,
                            hipMemcpyHostToDevice, s));
    set_lds_attr(lds);
    BatchArgs a{};
    a.count = count;
    a.graphs = b->d_desc;
    a.order = b->d_order;
    a.kstart = b->kstart;
    a.klen = b->klen;
    a.kidx = b->kidx;
    a.rp = b->rp;
    a.ci = b->ci16;
    a.sell = b->d_sell;
    a.smeta = b->d_smeta;
    a.sk = b->d_sk;
    a.sa = b->d_sa;
    a.escratch = b->d_escratch;
    a.slices_max = (b->nmax + 63) / 64;
    a.temps = b->d_temps;
    a.stats = b->d_stats;
    a.t_start = b->d_clock;
    a.t_end = b->d_clock + count;
    a.work = b->d_work;
    const int grid = batch_grid(b, lds);
    const std::vector<uint64_t> key = {(uint64_t)precision, (uint64_t)lds, (uint64_t)grid,
                                       (uint64_t)(uintptr_t)b->d_temps};
    if (!use_graph) {
        hipLaunchKernelGGL(reset_work_kernel, dim3(1), dim3(1), 0, s, b->d_work);
        launch_batch_kernel(precision, grid, lds, s, a);
        GILA_HIP(hipGetLastError());
    } else if (!b->gexec || key != b->gkey) {
        if (b->gexec) {
            (void)quiet(hipGraphExecDestroy(b->gexec));
            b->gexec = nullptr;
        }
        hipStream_t cs = capture_stream(b->device);
        if (!cs) return fail(GILA_EDEVICE, "cannot create capture stream");
        (void)hipGetLastError();  // no stale status may fail a check inside the capture
        GILA_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        hipLaunchKernelGGL(reset_work_kernel, dim3(1), dim3(1), 0, cs, b->d_work);
        launch_batch_kernel(precision, grid, lds, cs, a);
        hipGraph_t graph = nullptr;
        const hipError_t le = hipGetLastError();
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        if (le != hipSuccess || ee != hipSuccess) {
            if (graph) (void)quiet(hipGraphDestroy(graph));
            return fail(GILA_EDEVICE, "batch graph capture: %s",
                        hipGetErrorString(le != hipSuccess ? le : ee));
        }
        const hipError_t ie = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        (void)quiet(hipGraphDestroy(graph));
        if (ie != hipSuccess) {
            b->gexec = nullptr;
            return fail(GILA_EDEVICE, "batch graph instantiate: %s", hipGetErrorString(ie));
        }
        b->gkey = key;
    }
    if (use_graph) GILA_HIP(hipGraphLaunch(b->gexec, s));
    std::vector<gila_stats> st(count);
    GILA_HIP(hipMemcpyAsync(st.data(), b->d_stats, sizeof(gila_stats) * count,
                            hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    if (out) std::memcpy(out, st.data(), sizeof(gila_stats) * count);
    for (int32_t i = 0; i < count; ++i)
        if (st[i].nonfinite > 0)
            return fail(GILA_ENONFINITE,
                        "graph %d: %lld vertices had a non-finite force in iteration %d; they "
                        "did not move and the graph's run stopped",
                        i, (long long)st[i].nonfinite, st[i].iterations_run - 1);
    return GILA_OK;
}

}  // namespace gila

using namespace gila;

extern "C" {

int gila_batch_build(const gila_csr* graphs_dev, int32_t count, const int32_t* k, void* stream,
                     gila_batch** out) {
    clear_error();
    return batch_build(graphs_dev, count, k, (hipStream_t)stream, out);
}

int gila_batch_run(gila_batch* b, const gila_params* params, void* const* pos_dev, void* stream,
                   gila_stats* out) {
    TraceRange trace_range("gila_batch_run");
    clear_error();
    if (!b) return fail(GILA_EINVAL, "batch is NULL");
    std::lock_guard<std::mutex> lk(b->mu);
    DeviceGuard dg(b->device);
    return batch_run(b, params, pos_dev, (hipStream_t)stream, out, true);
}

int gila_batch_info(const gila_batch* b, int32_t* count, int64_t* total_pairs,
                    int64_t* device_bytes) {
    if (!b) return fail(GILA_EINVAL, "batch is NULL");
    if (count) *count = b->count;
    if (total_pairs) *total_pairs = b->P;
    if (device_bytes) *device_bytes = b->device_bytes;
    return GILA_OK;
}

int gila_batch_export(const gila_batch* b, int32_t graph, int64_t* ptr_host, int32_t* idx_host) {
    clear_error();
    if (!b || !ptr_host) return fail(GILA_EINVAL, "batch or ptr_host is NULL");
    if (graph < 0 || graph >= b->count) return fail(GILA_EINVAL, "graph %d out of range", graph);
    DeviceGuard dg(b->device);
    const int32_t n = b->n[graph];
    ptr_host[0] = 0;
    if (n == 0) return GILA_OK;
    std::vector<int64_t> ks((size_t)n);
    std::vector<int32_t> kl((size_t)n);
    GILA_HIP(hipMemcpy(ks.data(), b->kstart + b->vbase[graph], sizeof(int64_t) * n,
                       hipMemcpyDeviceToHost));
    GILA_HIP(hipMemcpy(kl.data(), b->klen + b->vbase[graph], sizeof(int32_t) * n,
                       hipMemcpyDeviceToHost));
    // the graph's rows lie in one block of kidx, in any order
    int64_t lo = INT64_MAX, hi = 0;
    for (int32_t v = 0; v < n; ++v) {
        lo = std::min(lo, ks[v]);
        hi = std::max(hi, ks[v] + kl[v]);
    }
    std::vector<uint16_t> rows((size_t)std::max<int64_t>(hi - lo, 0));
    if (!rows.empty())
        GILA_HIP(hipMemcpy(rows.data(), b->kidx + lo, sizeof(uint16_t) * rows.size(),
                           hipMemcpyDeviceToHost));
    // rows are padded to quads with the sentinel id n: strip it
    for (int32_t v = 0; v < n; ++v) {
        const int64_t r0 = ks[v] - lo;
        int64_t e = r0 + kl[v];
        while (e > r0 && rows[(size_t)e - 1] == (uint16_t)n) --e;
        const int64_t len = e - r0;
        if (idx_host)
            for (int64_t j = 0; j < len; ++j) idx_host[ptr_host[v] + j] = rows[(size_t)(r0 + j)];
        ptr_host[v + 1] = ptr_host[v] + len;
    }
    return GILA_OK;
}

int gila_batch_latency(const gila_batch* b, double* ms_host) {
    clear_error();
    if (!b || !ms_host) return fail(GILA_EINVAL, "batch or output is NULL");
    if (b->count == 0) return GILA_OK;
    DeviceGuard dg(b->device);
    std::vector<uint64_t> clk(2 * (size_t)b->count);
    GILA_HIP(hipMemcpy(clk.data(), b->d_clock, sizeof(uint64_t) * clk.size(),
                       hipMemcpyDeviceToHost));
    int khz = 0;
    GILA_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device));
    if (khz <= 0) return fail(GILA_EDEVICE, "no device wall clock rate");
    uint64_t t0 = clk[0];
    for (int32_t i = 0; i < b->count; ++i) t0 = std::min(t0, clk[i]);
    for (int32_t i = 0; i < b->count; ++i)
        ms_host[i] = (double)(clk[b->count + i] - t0) / (double)khz;
    return GILA_OK;
}

int gila_batch_plan(const gila_batch* b, int32_t* lanes_host, int32_t* class_host) {
    clear_error();
    if (!b) return fail(GILA_EINVAL, "batch is NULL");
    for (int32_t i = 0; i < b->count; ++i) {
        if (lanes_host) lanes_host[i] = b->lpv[i];
        if (class_host) class_host[i] = b->cls[i];
    }
    return GILA_OK;
}

int gila_batch_set_plan(gila_batch* b, const int32_t* lanes_host) {
    clear_error();
    if (!b) return fail(GILA_EINVAL, "batch is NULL");
    if (b->count > 0 && !lanes_host) return fail(GILA_EINVAL, "lanes_host is NULL");
    for (int32_t i = 0; i < b->count; ++i) {
        const int32_t l = lanes_host[i];
        if (l < 1 || l > 64 || (l & (l - 1)))
            return fail(GILA_EINVAL, "graph %d: lanes per vertex %d is not a power of two in "
                                     "[1, 64]", i, l);
    }
    std::lock_guard<std::mutex> lk(b->mu);
    for (int32_t i = 0; i < b->count; ++i) b->lpv[i] = lanes_host[i];
    return GILA_OK;
}

int gila_batch_tune(gila_batch* b, int32_t precision, void* stream, int32_t* class_lanes_host) {
    clear_error();
    if (!b) return fail(GILA_EINVAL, "batch is NULL");
    if (precision != GILA_FP64 && precision != GILA_FP32 && precision != GILA_FP32_KAHAN)
        return fail(GILA_EINVAL, "unknown precision %d", precision);
    std::lock_guard<std::mutex> lk(b->mu);
    DeviceGuard dg(b->device);
    int32_t table[kClasses];
    GILA_TRY(tune_plan(b, precision, (hipStream_t)stream, table));
    if (class_lanes_host) std::memcpy(class_lanes_host, table, sizeof(table));
    return GILA_OK;
}

void gila_batch_free(gila_batch* b) {
    if (!b) return;
    DeviceGuard g(b->device);
    free_batch(b, public_release());
}

int gila_layout_batch(const gila_csr* graphs_dev, int32_t count, const int32_t* k,
                      const gila_params* params, void* const* pos_dev, void* stream,
                      gila_stats* out) {
    TraceRange trace_range("gila_layout_batch");
    clear_error();
    gila_batch* b = nullptr;
    GILA_TRY(batch_build(graphs_dev, count, k, (hipStream_t)stream, &b));
    int rc;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        rc = batch_run(b, params, pos_dev, (hipStream_t)stream, out, false);
    }
    free_batch(b, Release{true, (hipStream_t)stream});
    return rc;
}

}  // extern "C"

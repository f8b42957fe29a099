// Segment-blocked iteration: every neighbour gather comes from LDS.
//
// Internal vertex ids are split into segments of S consecutive ids (S
// positions fill 64 KB of LDS for large degree-ordered graphs: 8190 FP32
// positions, the most that 16-bit byte offsets address; 32 KB for the
// others).  The k-hop row (and adjacency row)
// of an active vertex v is cut into slices, one per segment that the row
// touches; only non-empty slices exist.  A slice holds its ids as 16-bit LDS
// byte offsets (id - s*S) * sizeof(position).  Slices are stored
// segment-major (all slices of segment 0, then segment 1, ...), within a
// segment longest first, so that the lane groups of one wavefront walk
// slices of about the same length.
// k-hop slices are padded to a whole number of 4-id quads with a sentinel
// offset: LDS slot S holds a position so far away (1e30) that its squared
// distance overflows to +inf, the reciprocal is exactly 0 and the padding term
// is exactly zero.  Each lane then loads one aligned 8-byte quad of ids per
// memory instruction.
//
// One iteration is two kernels:
//   seg_force_kernel   one workgroup = one segment x a work-balanced range of
//                      its slices.  It copies the segment's positions into
//                      LDS, then sums repulsion (k-hop slice) and attraction
//                      (adjacency slice) of each slice and writes the slice's
//                      partial force (FP32 / Kahan lane sums, double-precision
//                      combine).  Partials are stored row-major: the partials
//                      of row v are contiguous and in segment order.
//   seg_combine_kernel one thread per vertex: adds the vertex's partials in
//                      segment order, applies the temperature cap, writes the
//                      vertex's next position and the iteration statistics.
// The result of every row depends only on the graph's plan (lanes per slice of
// its workgroup) and on the fixed segment order, never on scheduling.
//
// The layout is built on the device (build_segments): count the slices of
// every row, emit them row-major, reorder them by segment and length with two
// stable counting sorts, prefix-sum the padded lengths, fill the offsets, and
// cut each segment into workgroups of about equal work.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "iteration.h"

namespace gila {

// Two workgroup shapes of the force kernel, chosen per graph (seg_big):
// 1024 threads with 64 KB segments (two workgroups per CU) for graphs whose
// rows scatter over many segments, 512 threads with 32 KB segments (four per
// CU) for the others.  Both keep eight waves per SIMD.
template <bool BIG>
constexpr int seg_block() { return BIG ? 1024 : 512; }
#ifndef GILA_SEG_WAVES
#define GILA_SEG_WAVES 8
#endif
constexpr int kSegWaves = GILA_SEG_WAVES;  // waves per SIMD the FP32 force kernel is built for
constexpr int kSegTailPad = 64;    // slack entries after the k-hop offsets
constexpr int kMaxSegments = 16384;  // segment counters of the build fit in 64 KB of LDS
constexpr int kLongRow = 16;       // rows longer than kLongRow * nseg: binary search per segment
constexpr int kFillLanes = 16;     // lanes per slice in the fill pass
// Weighted repulsion: a segment holds at most weight_base<BIG>() bytes of
// positions (6500 FP32 or 3250 FP64 ones for the large workgroups, 2730 or
// 1365 for the small ones), and its weights (half a position each) go to a
// static LDS array, whose address is a constant the compiler folds into the
// LDS instruction (the weight address is then o / 2 plus that constant).
// Positions and weights together take 78 KB (two large workgroups in the
// 160 KB of a CU) or 33 KB (four small ones).
template <bool BIG>
constexpr int weight_base() { return BIG ? 52000 : 21840; }

template <bool WEIGHTED, bool BIG>
struct WeightLds {
    __device__ static unsigned char* get() { return nullptr; }
};
template <bool BIG>
struct WeightLds<true, BIG> {
    __device__ static unsigned char* get() {
        __shared__ __align__(16) unsigned char w[weight_base<BIG>() / 2];
        return w;
    }
};

bool segment_path_enabled() {
    const char* e = getenv("GILA_PATH");
    return !(e && std::strcmp(e, "direct") == 0);
}

// ------------------------------------------------------------------ build kernels
template <class T>
__device__ __forceinline__ int64_t lower_bound_ids(const T* __restrict__ a, int64_t lo, int64_t hi,
                                                   int64_t key) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct SliceBuild {
    int32_t na, S, nseg, pos_bytes;
    const int64_t* kptr;  // internal k-hop rows (ascending ids)
    const int32_t* kidx;
    const int64_t* rp;    // internal adjacency rows (ascending ids)
    const int32_t* ci;
    int64_t* rs;          // [na] slices per row (count pass)
    const int64_t* vsl;   // [na + 1] first slice of each row, row-major
    // row-major slice descriptors (emit pass)
    int32_t* d_seg;
    int64_t* d_k0;
    int32_t* d_kn;
    int32_t* d_a0;
    int32_t* d_an;
    int32_t* d_row;
};

__device__ __forceinline__ void emit_slice(const SliceBuild& b, int64_t j, int32_t v, int32_t s,
                                           int64_t k0, int64_t ke, int64_t ab, int64_t ae) {
    const int64_t lo = (int64_t)s * b.S, hi = lo + b.S;
    const int64_t k1 = lower_bound_ids(b.kidx, k0, ke, hi);
    const int64_t a0 = lower_bound_ids(b.ci, ab, ae, lo);
    const int64_t a1 = lower_bound_ids(b.ci, a0, ae, hi);
    b.d_seg[j] = s;
    b.d_k0[j] = k0;
    b.d_kn[j] = (int32_t)(k1 - k0);
    b.d_a0[j] = (int32_t)a0;
    b.d_an[j] = (int32_t)(a1 - a0);
    b.d_row[j] = v;
}

// Wave per row: the segments a sorted k-hop row touches.  Short rows are
// scanned for segment changes; long rows binary-search each segment.  The
// count pass writes the number of slices; the emit pass writes them at
// vsl[v] onward in segment order.  Every adjacency id of v is also a k-hop id
// of v (k >= 1), so the k-hop slices cover the adjacency slices.
template <bool EMIT>
__global__ __launch_bounds__(kBlock) void slice_rows_kernel(SliceBuild b) {
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
    const int lane = lane64();
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t vv = wave; vv < b.na; vv += nwaves) {
        const int32_t v = (int32_t)vv;
        const int64_t kb = b.kptr[v], ke = b.kptr[v + 1];
        const int64_t ab = b.rp[v], ae = b.rp[v + 1];
        int64_t t = EMIT ? b.vsl[v] : 0;
        if (ke - kb > (int64_t)kLongRow * b.nseg) {
            for (int32_t s0 = 0; s0 < b.nseg; s0 += 64) {
                const int32_t s = s0 + lane;
                bool ne = false;
                int64_t k0 = ke;
                if (s < b.nseg) {
                    k0 = lower_bound_ids(b.kidx, kb, ke, (int64_t)s * b.S);
                    ne = k0 < ke && (int64_t)b.kidx[k0] < (int64_t)(s + 1) * b.S;
                }
                const uint64_t m = __ballot(ne);
                if (EMIT && ne) emit_slice(b, t + __popcll(m & below), v, s, k0, ke, ab, ae);
                t += __popcll(m);
            }
        } else {
            for (int64_t j0 = kb; j0 < ke; j0 += 64) {
                const int64_t j = j0 + lane;
                bool start = false;
                int32_t s = 0;
                if (j < ke) {
                    s = b.kidx[j] / b.S;
                    start = j == kb || b.kidx[j - 1] / b.S != s;
                }
                const uint64_t m = __ballot(start);
                if (EMIT && start) emit_slice(b, t + __popcll(m & below), v, s, j, ke, ab, ae);
                t += __popcll(m);
            }
        }
        if (!EMIT && lane == 0) b.rs[v] = t;
    }
}

// Stable counting sort of a sequence of slices by an integer key in
// [0, nkeys), in tiles of `tj` consecutive elements.  Element i of the input
// is slice perm[i] (slice i when perm is null); its key is key[perm[i]].
// Pass 1: per-tile histogram, stored key-major (hist[key * ntiles + tile]) so
// that its exclusive prefix sum is the first output position of each
// (key, tile).
__device__ __forceinline__ int64_t sort_elem(const int32_t* perm, int64_t i) {
    return perm ? perm[i] : i;
}

__global__ __launch_bounds__(kBlock) void slice_hist_kernel(int64_t T, int64_t tj, int64_t ntiles,
                                                            int32_t nkeys,
                                                            const int32_t* __restrict__ key,
                                                            const int32_t* __restrict__ perm,
                                                            int64_t* __restrict__ hist) {
    extern __shared__ int32_t s_cnt[];
    for (int s = threadIdx.x; s < nkeys; s += kBlock) s_cnt[s] = 0;
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * tj;
    const int64_t j1 = j0 + tj < T ? j0 + tj : T;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kBlock) atomicAdd(&s_cnt[key[sort_elem(perm, j)]], 1);
    __syncthreads();
    for (int s = threadIdx.x; s < nkeys; s += kBlock) hist[(int64_t)s * ntiles + blockIdx.x] = s_cnt[s];
}

// Pass 2 (one wavefront per tile): walk the tile in order, 64 elements at a
// time; equal keys within a step are ranked by lane, so elements with equal
// keys keep their input order.  out[position] = slice.
__global__ __launch_bounds__(64) void slice_scatter_kernel(int64_t T, int64_t tj, int64_t ntiles,
                                                           int32_t nkeys,
                                                           const int32_t* __restrict__ key,
                                                           const int32_t* __restrict__ perm,
                                                           const int64_t* __restrict__ base,
                                                           int32_t* __restrict__ out) {
    extern __shared__ int32_t s_next[];
    const int lane = threadIdx.x;
    for (int s = lane; s < nkeys; s += 64) s_next[s] = (int32_t)base[(int64_t)s * ntiles + blockIdx.x];
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * tj;
    const int64_t j1 = j0 + tj < T ? j0 + tj : T;
    for (int64_t c = j0; c < j1; c += 64) {
        const int64_t j = c + lane;
        const bool valid = j < j1;
        const int64_t e = valid ? sort_elem(perm, j) : 0;
        const int32_t s = valid ? key[e] : -1;
        int rank = 0, same = 0;
        for (int l = 0; l < 64; ++l) {
            const int32_t sl = __builtin_amdgcn_readlane(s, l);
            same += sl == s ? 1 : 0;
            rank += (sl == s && l < lane) ? 1 : 0;
        }
        const int32_t at = valid ? s_next[s] : 0;
        __syncthreads();
        if (valid) {
            out[at + rank] = (int32_t)e;
            if (rank == same - 1) s_next[s] = at + same;
        }
        __syncthreads();
    }
}

// One 11-bit digit of each element's key, for the LSD passes below.
constexpr int kOrderDigitBits = 11;
__global__ __launch_bounds__(kBlock) void key_digit_kernel(int32_t n, const uint32_t* __restrict__ key,
                                                           int shift, int32_t* __restrict__ digit) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock)
        digit[v] = (int32_t)((key[v] >> shift) & ((1u << kOrderDigitBits) - 1u));
}

int stable_order_by_key(int32_t n, const uint32_t* key, uint32_t max_key, int32_t* out,
                        hipStream_t s) {
    if (n <= 0) return GILA_OK;
    int passes = 1;
    while (passes * kOrderDigitBits < 32 && (max_key >> (passes * kOrderDigitBits)) > 0) ++passes;
    const int32_t nkeys_max = 1 << kOrderDigitBits;
    const int64_t tj = std::max<int64_t>(1024, ((int64_t)n * nkeys_max + (1 << 24) - 1) >> 24);
    const int64_t ntiles = (n + tj - 1) / tj;
    const int64_t H = ntiles * nkeys_max;
    struct Tmp {
        void* p = nullptr;
        hipStream_t s;
        ~Tmp() { dfree_on(p, s); }
    } digit{nullptr, s}, buf{nullptr, s}, hist{nullptr, s}, hscan{nullptr, s}, ws{nullptr, s};
    GILA_TRY(dalloc_t(reinterpret_cast<int32_t**>(&digit.p), (size_t)n));
    GILA_TRY(dalloc_t(reinterpret_cast<int32_t**>(&buf.p), (size_t)n));
    GILA_TRY(dalloc_t(reinterpret_cast<int64_t**>(&hist.p), (size_t)H));
    GILA_TRY(dalloc_t(reinterpret_cast<int64_t**>(&hscan.p), (size_t)H + 1));
    GILA_TRY(dalloc_t(reinterpret_cast<int64_t**>(&ws.p), (size_t)scan_workspace_count(H)));
    const unsigned grid = (unsigned)std::min<int64_t>(4096, ((int64_t)n + kBlock - 1) / kBlock);
    // the last pass writes `out`; earlier ones alternate so that it does
    const int32_t* src = nullptr;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kOrderDigitBits;
        const int32_t nkeys = (int32_t)std::min<uint64_t>((uint64_t)nkeys_max, ((uint64_t)max_key >> shift) + 1);
        int32_t* dst = ((passes - 1 - p) & 1) ? static_cast<int32_t*>(buf.p) : out;
        hipLaunchKernelGGL(key_digit_kernel, dim3(grid), dim3(kBlock), 0, s, n, key, shift,
                           static_cast<int32_t*>(digit.p));
        const size_t lds = sizeof(int32_t) * (size_t)nkeys;
        hipLaunchKernelGGL(slice_hist_kernel, dim3((unsigned)ntiles), dim3(kBlock), lds, s, (int64_t)n,
                           tj, ntiles, nkeys, static_cast<const int32_t*>(digit.p), src,
                           static_cast<int64_t*>(hist.p));
        GILA_HIP(hipGetLastError());
        GILA_TRY(enqueue_exclusive_scan_i64(static_cast<int64_t*>(hist.p), static_cast<int64_t*>(hscan.p),
                                            ntiles * nkeys, static_cast<int64_t*>(ws.p), s));
        hipLaunchKernelGGL(slice_scatter_kernel, dim3((unsigned)ntiles), dim3(64), lds, s, (int64_t)n, tj,
                           ntiles, nkeys, static_cast<const int32_t*>(digit.p), src,
                           static_cast<const int64_t*>(hscan.p), dst);
        GILA_HIP(hipGetLastError());
        src = dst;
    }
    return GILA_OK;
}

// Length key of each slice: dense slices (at least dmin k-hop ids; dmin <= 0:
// none) key 0, the others by their quads, more quads smaller keys (longest
// first), clamped to keys 1 .. kLenKeys - 1.  Within a segment the dense
// slices therefore come first.
constexpr int kLenKeys = 1024;
__global__ __launch_bounds__(kBlock) void slice_lenkey_kernel(int64_t T, const int32_t* __restrict__ d_kn,
                                                              int32_t dmin,
                                                              int32_t* __restrict__ lenkey) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= T) return;
    const int32_t nq = (d_kn[j] + 3) >> 2;
    const bool dense = dmin > 0 && d_kn[j] >= dmin;
    lenkey[j] = dense ? 0 : kLenKeys - 1 - (nq < kLenKeys - 2 ? nq : kLenKeys - 2);
}

// Padded k-hop and adjacency lengths of each segment-major slice, and
// whether it is dense (its k-hop ids then take no offsets, only a bitmap).
__global__ __launch_bounds__(kBlock) void slice_lengths_kernel(int64_t T,
                                                               const int32_t* __restrict__ order,
                                                               const int32_t* __restrict__ d_kn,
                                                               const int32_t* __restrict__ d_an,
                                                               int32_t dmin,
                                                               int64_t* __restrict__ wk,
                                                               int64_t* __restrict__ wa,
                                                               int64_t* __restrict__ dn) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= T) return;
    const int32_t j = order[i];
    const bool dense = dmin > 0 && d_kn[j] >= dmin;
    wk[i] = dense ? 0 : (d_kn[j] + 3) & ~3;
    wa[i] = d_an[j];
    dn[i] = dense ? 1 : 0;
}

// Cumulative work of the slices before i: entries plus a fixed cost per
// slice; a dense slice evaluates every slot of its segment (dense_work).
__device__ __forceinline__ int64_t slice_work(const int64_t* sl_k, const int64_t* sl_a,
                                              const int64_t* sl_dn, int64_t i, int64_t slice_cost,
                                              int64_t dense_work) {
    return sl_k[i] + sl_a[i] + slice_cost * i + (sl_dn ? dense_work * sl_dn[i] : 0);
}

// For each segment s (and s = nseg): its first segment-major slice and the
// cumulative work there; last entry: total padded k-hop length.
__global__ __launch_bounds__(kBlock) void segment_starts_kernel(
    int32_t nseg, int64_t T, int64_t ntiles, int64_t slice_cost, int64_t dense_work,
    const int64_t* __restrict__ base, const int64_t* __restrict__ sl_k,
    const int64_t* __restrict__ sl_a, const int64_t* __restrict__ sl_dn, int64_t* __restrict__ out) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s > nseg) return;
    const int64_t f = s < nseg ? base[(int64_t)s * ntiles] : T;
    out[2 * s] = f;
    out[2 * s + 1] = slice_work(sl_k, sl_a, sl_dn, f, slice_cost, dense_work);
    if (s == nseg) {
        out[2 * s + 2] = sl_k[T];
        out[2 * s + 3] = sl_dn ? sl_dn[T] : 0;
    }
}

// kFillLanes lanes per segment-major slice: LDS byte offsets of its ids, the
// k-hop part padded with the sentinel (a dense slice has none: see
// dense_mask_kernel); the slice records.
__global__ __launch_bounds__(kBlock) void slice_fill_kernel(
    SliceBuild b, int64_t T, const int32_t* __restrict__ order, const int64_t* __restrict__ sl_k,
    const int64_t* __restrict__ sl_a64, uint16_t* __restrict__ sk_idx, uint16_t* __restrict__ sa_idx,
    int32_t* __restrict__ sl_v, int32_t* __restrict__ sl_p, int32_t* __restrict__ sl_a) {
    const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kFillLanes;
    const int64_t ng = ((int64_t)gridDim.x * kBlock) / kFillLanes;
    const int gl = threadIdx.x % kFillLanes;
    const uint16_t sentinel = (uint16_t)(b.S * b.pos_bytes);
    for (int64_t i = g; i < T; i += ng) {
        const int32_t j = order[i];
        const int32_t s = b.d_seg[j];
        const int32_t lo = s * b.S;
        const int64_t k0 = b.d_k0[j];
        const int32_t kn = b.d_kn[j];
        const int64_t dst = sl_k[i], kpad = sl_k[i + 1] - dst;
        for (int64_t t = gl; t < kpad; t += kFillLanes)
            sk_idx[dst + t] = t < kn ? (uint16_t)((b.kidx[k0 + t] - lo) * b.pos_bytes) : sentinel;
        const int32_t a0 = b.d_a0[j], an = b.d_an[j];
        const int64_t adst = sl_a64[i];
        for (int32_t t = gl; t < an; t += kFillLanes)
            sa_idx[adst + t] = (uint16_t)((b.ci[a0 + t] - lo) * b.pos_bytes);
        if (gl == 0) {
            sl_v[i] = b.d_row[j];
            sl_p[i] = j;
            sl_a[i] = (int32_t)adst;
            if (i == T - 1) sl_a[T] = (int32_t)sl_a64[T];
        }
    }
}

// The bitmap of each dense slice, one wavefront per slice: slot 64 b + l is
// bit l of mask b.  The slice's ids are ascending, so each 64-id chunk spans
// a few consecutive masks; each mask is the OR over the wavefront of its
// lanes' bits, kept in a register while later chunks may still add to it and
// written once (masks no id reaches stay zero).
__global__ __launch_bounds__(kBlock) void dense_mask_kernel(SliceBuild b, int64_t T,
                                                            const int32_t* __restrict__ order,
                                                            const int64_t* __restrict__ sl_dn,
                                                            int32_t dense_blocks,
                                                            uint64_t* __restrict__ dmask) {
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
    const int lane = lane64();
    for (int64_t i = wave; i < T; i += nwaves) {
        if (sl_dn[i + 1] == sl_dn[i]) continue;
        const int32_t j = order[i];
        const int32_t lo = b.d_seg[j] * b.S;
        const int64_t k0 = b.d_k0[j];
        const int32_t kn = b.d_kn[j];
        uint64_t* m = dmask + sl_dn[i] * dense_blocks;
        uint64_t cur = 0;
        int32_t curw = -1;
        for (int32_t c = 0; c < kn; c += 64) {
            const int32_t t = c + lane;
            const int32_t local = t < kn ? b.kidx[k0 + t] - lo : 0;
            const int32_t w = t < kn ? local >> 6 : -1;
            const uint64_t bit = t < kn ? 1ull << (local & 63) : 0ull;
            const int32_t wlo = __builtin_amdgcn_readfirstlane(w);
            const int32_t whi = __shfl(w, kn - c < 64 ? kn - c - 1 : 63, 64);
            for (int32_t ww = wlo; ww <= whi; ++ww) {
                uint64_t v = w == ww ? bit : 0ull;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off, 64);
                if (ww != curw) {
                    if (curw >= 0 && lane == 0) m[curw] = cur;
                    cur = 0;
                    curw = ww;
                }
                cur |= v;
            }
        }
        if (curw >= 0 && lane == 0) m[curw] = cur;
    }
}

// Enough quads per lane (qpl) to amortise the per-slice reduction.
__host__ __device__ __forceinline__ int lanes_for_length(int64_t len, int64_t qpl) {
    int l = 1;
    while (l < 64 && (int64_t)l * 2 * qpl * 4 <= len) l *= 2;
    return l;
}

// One thread per workgroup of the force kernel: desc = (segment, index in
// the segment, workgroups of the segment).  The segment's slices are split
// where the cumulative work crosses equal fractions; lanes per slice follow
// the mean slice length of the range.
__global__ __launch_bounds__(kBlock) void segment_plan_kernel(
    int32_t nwg, int64_t slice_cost, int64_t qpl, int64_t dense_work,
    const int64_t* __restrict__ starts, const int64_t* __restrict__ sl_k,
    const int32_t* __restrict__ sl_a, const int64_t* __restrict__ sl_dn, int4* __restrict__ wg) {
    const int w = blockIdx.x * kBlock + threadIdx.x;
    if (w >= nwg) return;
    const int4 d = wg[w];
    const int s = d.x, t = d.y, c = d.z;
    const int64_t f0 = starts[2 * s], f1 = starts[2 * s + 2];
    const int64_t c0 = starts[2 * s + 1], c1 = starts[2 * s + 3];
    const int64_t W = c1 - c0;
    auto work = [&](int64_t i) {
        return sl_k[i] + (int64_t)sl_a[i] + slice_cost * i + (sl_dn ? dense_work * sl_dn[i] : 0);
    };
    auto cut = [&](int64_t target) {
        int64_t lo = f0, hi = f1;
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (work(mid) < target) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int64_t ib = t == 0 ? f0 : cut(c0 + W * t / c);
    const int64_t ie = t == c - 1 ? f1 : cut(c0 + W * (t + 1) / c);
    // lanes per slice from the mean length of the range's offset-listed slices
    const int64_t is = ib + (sl_dn ? sl_dn[ie] - sl_dn[ib] : 0);
    const int64_t len = ie > is ? ((sl_k[ie] - sl_k[is]) + (int64_t)(sl_a[ie] - sl_a[is])) / (ie - is) : 0;
    wg[w] = make_int4(s, (int)ib, (int)ie, lanes_for_length(len, qpl));
}

// ------------------------------------------------------------------ iteration: segment kernel
// Exact number of coincident pairs in a row of quads (only walked for rows in
// which some lane saw a zero squared distance).
template <class V, int LPV>
__device__ __forceinline__ int count_coincident_quads(V xv, const uint2* __restrict__ q4, int nq,
                                                      int gl, const unsigned char* __restrict__ lds) {
    int c = 0;
    for (int q = gl; q < nq; q += LPV) {
        const uint2 w = q4[q];
        const uint32_t offs[4] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16};
        for (int i = 0; i < 4; ++i) {
            const V p = *reinterpret_cast<const V*>(lds + offs[i]);
            c += (p.x == xv.x && p.y == xv.y) ? 1 : 0;
        }
    }
    return c;
}

// Repulsion from the four neighbours whose LDS byte offsets are packed in w.
// With WEIGHTED, the weight of the vertex staged at byte offset o of the
// positions is at byte offset o / 2 of `lw` (a weight is half a position).
template <class P, bool WEIGHTED, int Q>
__device__ __forceinline__ void quad_terms(uint2 w, const unsigned char* __restrict__ lds,
                                           const unsigned char* __restrict__ lw,
                                           typename P::real xv, typename P::real yv,
                                           typename P::real& sx, typename P::real& sy,
                                           typename P::real& mindd, int q) {
    using R = typename P::real;
    using V = typename P::vec2;
    const uint32_t o0 = w.x & 0xFFFFu, o1 = w.x >> 16, o2 = w.y & 0xFFFFu, o3 = w.y >> 16;
    const V p0 = *reinterpret_cast<const V*>(lds + o0);
    const V p1 = *reinterpret_cast<const V*>(lds + o1);
    const V p2 = *reinterpret_cast<const V*>(lds + o2);
    const V p3 = *reinterpret_cast<const V*>(lds + o3);
    if constexpr (WEIGHTED) {
        const R m[4] = {*reinterpret_cast<const R*>(lw + (o0 >> 1)),
                        *reinterpret_cast<const R*>(lw + (o1 >> 1)),
                        *reinterpret_cast<const R*>(lw + (o2 >> 1)),
                        *reinterpret_cast<const R*>(lw + (o3 >> 1))};
        repulse4<P, true, Q>(p0, p1, p2, p3, xv, yv, sx, sy, mindd, m, q);
    } else {
        repulse4<P, false, Q>(p0, p1, p2, p3, xv, yv, sx, sy, mindd, nullptr, q);
    }
}

template <class P, int LPV, bool WEIGHTED, int Q>
__device__ __forceinline__ void seg_slices(const SegArgs& a, int ib, int ie,
                                           const typename P::vec2* __restrict__ lp,
                                           const unsigned char* __restrict__ lw, int* s_next,
                                           int& coinc) {
    using R = typename P::real;
    using V = typename P::vec2;
    const V* __restrict__ gpos = reinterpret_cast<const V*>(a.pos);
    const unsigned char* __restrict__ lds = reinterpret_cast<const unsigned char*>(lp);
    const double d2 = a.d * a.d;
    // attraction (x_u - x_v) delta / d enters the same sum divided by d^2
    const R dpar = sizeof(R) == 4 ? (R)(1.0 / (a.d * d2)) : (R)(a.d * d2);
    // Each wavefront takes the next (64 / LPV) slices of the range when it
    // is done with its previous ones (slices are sorted longest first, so the
    // groups of a wavefront get similar work and no wavefront idles while
    // slices remain).  A slice's result depends only on the slice and LPV.
    constexpr int kPerWave = 64 / LPV;
    const int gl = threadIdx.x % LPV;
    const int wgrp = lane64() / LPV;
    for (;;) {
        int i0 = 0;
        if (lane64() == 0) i0 = atomicAdd(s_next, kPerWave);
        i0 = __builtin_amdgcn_readfirstlane(i0);
        if (i0 >= ie) break;
        const int i = i0 + wgrp;
        Acc<R, P::kahan> acc;
        if (i < ie) {
            const V xv = gpos[a.sl_v[i]];
            const int64_t kb = a.sl_k[i], ke = a.sl_k[i + 1];
            const uint2* __restrict__ q4 = reinterpret_cast<const uint2*>(a.kidx + kb);
            const int nq = (int)((ke - kb) >> 2);
            R mindd = R(1);
            // four quads (16 neighbours) per lane per step, one compensated
            // add per eight terms; then the remaining quads one by one.  FP64
            // with a run-time exponent takes them one by one throughout: 16
            // pairs in flight exceed the 128 VGPRs of four waves per SIMD.
            constexpr bool kFourQuads = !(sizeof(R) == 8 && Q < 0);
            int q = gl;
            // quads are loaded a step ahead of their terms: the next step of
            // four, or else the remaining (fewer than four) quads of the row
            uint2 n0 = make_uint2(0, 0), n1 = n0, n2 = n0, n3 = n0;
            // (as a macro: a lambda writing the four registers through
            // references put them in scratch memory)
#define GILA_QUADS_AHEAD(qq)                                        \
    do {                                                            \
        const int q_ = (qq);                                        \
        if (q_ + 3 * LPV < nq) {                                    \
            n0 = q4[q_];                                            \
            n1 = q4[q_ + LPV];                                      \
            n2 = q4[q_ + 2 * LPV];                                  \
            n3 = q4[q_ + 3 * LPV];                                  \
        } else {                                                    \
            if (q_ < nq) n0 = q4[q_];                               \
            if (q_ + LPV < nq) n1 = q4[q_ + LPV];                   \
            if (q_ + 2 * LPV < nq) n2 = q4[q_ + 2 * LPV];           \
        }                                                           \
    } while (0)
            // (exponents fixed at compile time only, and with leaf weights
            // only q = 1: the other forms' terms need registers that the
            // look-ahead pushes into scratch memory -- the run-time exponent
            // (4, 5) took 0.398 -> 0.401 ms with it)
            constexpr bool kAhead = kFourQuads && (Q == 1 || (Q >= 0 && !WEIGHTED));
            if constexpr (kAhead) {
                GILA_QUADS_AHEAD(q);
                for (; q + 3 * LPV < nq; q += 4 * LPV) {
                    const uint2 w0 = n0, w1 = n1, w2 = n2, w3 = n3;
                    GILA_QUADS_AHEAD(q + 4 * LPV);
                    R ax, ay, bx, by;
                    quad_terms<P, WEIGHTED, Q>(w0, lds, lw, xv.x, xv.y, ax, ay, mindd, a.rep_q);
                    quad_terms<P, WEIGHTED, Q>(w1, lds, lw, xv.x, xv.y, bx, by, mindd, a.rep_q);
                    acc.add(ax + bx, ay + by);
                    quad_terms<P, WEIGHTED, Q>(w2, lds, lw, xv.x, xv.y, ax, ay, mindd, a.rep_q);
                    quad_terms<P, WEIGHTED, Q>(w3, lds, lw, xv.x, xv.y, bx, by, mindd, a.rep_q);
                    acc.add(ax + bx, ay + by);
                }
                // the remaining quads, one by one as below
                const auto rest = [&](uint2 w) {
                    if (q < nq) {
                        R ax, ay;
                        quad_terms<P, WEIGHTED, Q>(w, lds, lw, xv.x, xv.y, ax, ay, mindd, a.rep_q);
                        acc.add(ax, ay);
                    }
                    q += LPV;
                };
                rest(n0);
                rest(n1);
                rest(n2);
            } else if constexpr (kFourQuads) {
                for (; q + 3 * LPV < nq; q += 4 * LPV) {
                    const uint2 w0 = q4[q];
                    const uint2 w1 = q4[q + LPV];
                    const uint2 w2 = q4[q + 2 * LPV];
                    const uint2 w3 = q4[q + 3 * LPV];
                    R ax, ay, bx, by;
                    quad_terms<P, WEIGHTED, Q>(w0, lds, lw, xv.x, xv.y, ax, ay, mindd, a.rep_q);
                    quad_terms<P, WEIGHTED, Q>(w1, lds, lw, xv.x, xv.y, bx, by, mindd, a.rep_q);
                    acc.add(ax + bx, ay + by);
                    quad_terms<P, WEIGHTED, Q>(w2, lds, lw, xv.x, xv.y, ax, ay, mindd, a.rep_q);
                    quad_terms<P, WEIGHTED, Q>(w3, lds, lw, xv.x, xv.y, bx, by, mindd, a.rep_q);
                    acc.add(ax + bx, ay + by);
                }
            }
#undef GILA_QUADS_AHEAD
            for (; q < nq; q += LPV) {
                R ax, ay;
                quad_terms<P, WEIGHTED, Q>(q4[q], lds, lw, xv.x, xv.y, ax, ay, mindd, a.rep_q);
                acc.add(ax, ay);
            }
            if (mindd <= coincidence_bias<R>())
                coinc += count_coincident_quads<V, LPV>(xv, q4, nq, gl, lds);
            const int32_t ab = a.sl_a[i], ae = a.sl_a[i + 1];
            for (int32_t j = ab + gl; j < ae; j += LPV)
                attract<P>(xv.x, xv.y, *reinterpret_cast<const V*>(lds + a.aidx[j]), dpar, acc,
                           a.att_p);
        }
        const double fx = group_sum<LPV>(acc.x()) * d2;
        const double fy = group_sum<LPV>(acc.y()) * d2;
        if (i < ie && gl == 0) a.part[a.sl_p[i]] = make_double2(fx, fy);
    }
}

// Repulsion from the four vertices staged at LDS addresses ps[0 .. 3] (with
// WEIGHTED, each weight at half its position's byte offset in lw, as in
// quad_terms).
template <class P, bool WEIGHTED, int Q>
__device__ __forceinline__ void slot_terms(const unsigned char* const* ps,
                                           const unsigned char* __restrict__ lds,
                                           const unsigned char* __restrict__ lw,
                                           typename P::real xv, typename P::real yv,
                                           typename P::real& sx, typename P::real& sy,
                                           typename P::real& mindd, int q) {
    using R = typename P::real;
    using V = typename P::vec2;
    const V p0 = *reinterpret_cast<const V*>(ps[0]);
    const V p1 = *reinterpret_cast<const V*>(ps[1]);
    const V p2 = *reinterpret_cast<const V*>(ps[2]);
    const V p3 = *reinterpret_cast<const V*>(ps[3]);
    if constexpr (WEIGHTED) {
        const R m[4] = {*reinterpret_cast<const R*>(lw + ((ps[0] - lds) >> 1)),
                        *reinterpret_cast<const R*>(lw + ((ps[1] - lds) >> 1)),
                        *reinterpret_cast<const R*>(lw + ((ps[2] - lds) >> 1)),
                        *reinterpret_cast<const R*>(lw + ((ps[3] - lds) >> 1))};
        repulse4<P, true, Q>(p0, p1, p2, p3, xv, yv, sx, sy, mindd, m, q);
    } else {
        repulse4<P, false, Q>(p0, p1, p2, p3, xv, yv, sx, sy, mindd, nullptr, q);
    }
}

// A dense slice, by one whole wavefront: every slot of the segment's nblk
// blocks of 64 is evaluated against the row's vertex, lane l taking slot
// 64 b + l of block b.  Block b's mask (bit l: slot 64 b + l is in the slice)
// is uniform, read by scalar loads, and becomes the lane condition of one
// select per slot: the slot's LDS byte offset, or the sentinel, whose term
// is exactly zero.  Eight blocks per step, one compensated add per eight
// terms, as in the offset-listed slices.  Then the slice's adjacency terms
// and the wavefront's sum.
template <class P, bool WEIGHTED, int Q>
__device__ __forceinline__ void dense_slice(const SegArgs& a, int i, int nblk,
                                            const unsigned char* __restrict__ lds,
                                            const unsigned char* __restrict__ lw, int& coinc) {
    using R = typename P::real;
    using V = typename P::vec2;
    const V* __restrict__ gpos = reinterpret_cast<const V*>(a.pos);
    const int lane = lane64();
    const V xv = gpos[a.sl_v[i]];
    // the masks never change during the launch: read through the constant
    // address space, so that the uniform loads are scalar
    typedef const __attribute__((address_space(4))) uint64_t* MaskPtr;
    const int32_t di = __builtin_amdgcn_readfirstlane((int32_t)a.sl_dn[i]);
    const MaskPtr mk = (MaskPtr)(a.dmask + (int64_t)di * a.dense_blocks);
    const unsigned char* lsent = lds + (uint32_t)a.seg * (uint32_t)sizeof(V);
    constexpr uint32_t kStep = 64 * (uint32_t)sizeof(V);
    Acc<R, P::kahan> acc;
    R mindd = R(1);
#pragma unroll 1
    for (int b0 = 0; b0 < nblk; b0 += 8) {
        const unsigned char* base = lds + (uint32_t)b0 * kStep + (uint32_t)lane * (uint32_t)sizeof(V);
        const unsigned char* ps[8];  // slots 64 (b0 + t) + lane, or the sentinel
#pragma unroll
        for (int t = 0; t < 8; ++t)
            ps[t] = __builtin_amdgcn_inverse_ballot_w64(mk[b0 + t]) ? base + t * kStep : lsent;
        R ax, ay, bx, by;
        slot_terms<P, WEIGHTED, Q>(ps, lds, lw, xv.x, xv.y, ax, ay, mindd, a.rep_q);
        slot_terms<P, WEIGHTED, Q>(ps + 4, lds, lw, xv.x, xv.y, bx, by, mindd, a.rep_q);
        acc.add(ax + bx, ay + by);
    }
    if (mindd <= coincidence_bias<R>()) {
        int c = 0;
#pragma unroll 1
        for (int b = 0; b < nblk; ++b) {
            if (__builtin_amdgcn_inverse_ballot_w64(mk[b])) {
                const V p = *reinterpret_cast<const V*>(lds + (uint32_t)b * kStep +
                                                        (uint32_t)lane * (uint32_t)sizeof(V));
                c += (p.x == xv.x && p.y == xv.y) ? 1 : 0;
            }
        }
        coinc += c;
    }
    const double d2 = a.d * a.d;
    const R dpar = sizeof(R) == 4 ? (R)(1.0 / (a.d * d2)) : (R)(a.d * d2);
    const int32_t ab = a.sl_a[i], ae = a.sl_a[i + 1];
    for (int32_t j = ab + lane; j < ae; j += 64)
        attract<P>(xv.x, xv.y, *reinterpret_cast<const V*>(lds + a.aidx[j]), dpar, acc, a.att_p);
    const double fx = group_sum<64>(acc.x()) * d2;
    const double fy = group_sum<64>(acc.y()) * d2;
    if (lane == 0) a.part[a.sl_p[i]] = make_double2(fx, fy);
}

// FP32: eight waves per SIMD, as two 1024-thread workgroups per CU with a
// 64 KB segment each (BIG) or four 512-thread ones with 32 KB.  Where rows
// scatter, BIG halves the segments, so the slices per row, and doubles the
// pairs per slice (310 against 345 us per R-MAT 18 launch); where rows are
// local they touch one or two segments either way and the smaller
// workgroups keep more of them per graph.  FP64 needs more registers.
// WEIGHTED stages each vertex's repulsion weight in a static LDS array (slot
// S of positions and weights holds the sentinel).
template <int PREC, bool WEIGHTED, int Q, bool BIG>
__global__ __launch_bounds__(seg_block<BIG>(), PREC == GILA_FP64 ? 4 : kSegWaves) void seg_force_kernel(SegArgs a) {
    constexpr int kSegBlock = seg_block<BIG>();
    using P = Prec<PREC>;
    using V = typename P::vec2;
    extern __shared__ __align__(16) unsigned char s_raw[];
    V* lp = reinterpret_cast<V*>(s_raw);
    __shared__ int64_t s_c[kSegBlock / 64];
    if (a.span && threadIdx.x == 0) atomicMin(&a.span[0], (unsigned long long)wall_clock64());
    if (a.ctl->stopped) {
        if (a.span && threadIdx.x == 0) atomicMax(&a.span[1], (unsigned long long)wall_clock64());
        return;
    }
    const int4 w = a.wg[blockIdx.x];
    const int s = w.x, ib = w.y, ie = w.z, lpv = w.w;
    // stage the segment's positions
    const V* gpos = reinterpret_cast<const V*>(a.pos);
    const int64_t base = (int64_t)s * a.seg;
    const int64_t left = (int64_t)a.na - base;
    const int cnt = (int)(left < a.seg ? left : a.seg);
    for (int i = threadIdx.x; i < cnt; i += kSegBlock) lp[i] = gpos[base + i];
    using R = typename P::real;
    R* lw = reinterpret_cast<R*>(WeightLds<WEIGHTED, BIG>::get());
    if constexpr (WEIGHTED) {
        const R* gw = reinterpret_cast<const R*>(a.mass);
        for (int i = threadIdx.x; i < cnt; i += kSegBlock) lw[i] = gw[base + i];
    }
    // the range's dense slices are its head (the sort puts them first in
    // each segment): [ib, id) by whole wavefronts, then [id, ie)
    const int id = ib + (a.sl_dn ? (int)(a.sl_dn[ie] - a.sl_dn[ib]) : 0);
    __shared__ int s_next, s_dnext;
    if (threadIdx.x == 0) {
        s_next = id;
        s_dnext = ib;
        V far;
        far.x = sizeof(far.x) == 4 ? (decltype(far.x))1e30f : (decltype(far.x))1e300;
        far.y = far.x;
        lp[a.seg] = far;  // sentinel slot: padding terms vanish exactly
        if constexpr (WEIGHTED) lw[a.seg] = R(0);
    }
    __syncthreads();
    int coinc = 0;
    if constexpr (PREC != GILA_FP64) {
        if (id > ib) {
            const int nblk = (cnt + 63) >> 6;
            const unsigned char* lds = reinterpret_cast<const unsigned char*>(lp);
            const unsigned char* lwb = reinterpret_cast<const unsigned char*>(lw);
            for (;;) {
                int i = 0;
                if (lane64() == 0) i = atomicAdd(&s_dnext, 1);
                i = __builtin_amdgcn_readfirstlane(i);
                if (i >= id) break;
                dense_slice<P, WEIGHTED, Q>(a, i, nblk, lds, lwb, coinc);
            }
        }
    }
    const unsigned char* wb = reinterpret_cast<const unsigned char*>(lw);
    switch (lpv) {
        case 1: seg_slices<P, 1, WEIGHTED, Q>(a, id, ie, lp, wb, &s_next, coinc); break;
        case 2: seg_slices<P, 2, WEIGHTED, Q>(a, id, ie, lp, wb, &s_next, coinc); break;
        case 4: seg_slices<P, 4, WEIGHTED, Q>(a, id, ie, lp, wb, &s_next, coinc); break;
        case 8: seg_slices<P, 8, WEIGHTED, Q>(a, id, ie, lp, wb, &s_next, coinc); break;
        case 16: seg_slices<P, 16, WEIGHTED, Q>(a, id, ie, lp, wb, &s_next, coinc); break;
        case 32: seg_slices<P, 32, WEIGHTED, Q>(a, id, ie, lp, wb, &s_next, coinc); break;
        default: seg_slices<P, 64, WEIGHTED, Q>(a, id, ie, lp, wb, &s_next, coinc); break;
    }
    const int64_t wc = wave_sum((int64_t)coinc);
    if (lane64() == 0) s_c[wave_id()] = wc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t c = 0;
        for (int i = 0; i < kSegBlock / 64; ++i) c += s_c[i];
        if (c) atomicAdd((unsigned long long*)&a.ctl->coinc_pending, (unsigned long long)c);
        if (a.span) atomicMax(&a.span[1], (unsigned long long)wall_clock64());
    }
}

// ------------------------------------------------------------------ iteration: combine kernel
template <int PREC>
__global__ __launch_bounds__(kBlock) void seg_combine_kernel(StepArgs a) {
    using P = Prec<PREC>;
    using V = typename P::vec2;
    if (a.ctl->stopped) return;
    double energy = 0.0, maxd = 0.0;
    int64_t moved = 0, nonfinite = 0;
    const int32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < a.n_active) {
        // partials added one after another in segment order; loads are
        // issued four at a time
        double fx = 0.0, fy = 0.0;
        const int64_t je = a.vsl[v + 1];
        int64_t j = a.vsl[v];
        for (; j + 3 < je; j += 4) {
            const double2 p0 = a.part[j], p1 = a.part[j + 1], p2 = a.part[j + 2],
                          p3 = a.part[j + 3];
            fx += p0.x;
            fy += p0.y;
            fx += p1.x;
            fy += p1.y;
            fx += p2.x;
            fy += p2.y;
            fx += p3.x;
            fy += p3.y;
        }
        for (; j < je; ++j) {
            const double2 p = a.part[j];
            fx += p.x;
            fy += p.y;
        }
        const V xv = reinterpret_cast<const V*>(a.pos_cur)[v];
        finish_vertex<P>(a, v, xv, fx, fy, energy, maxd, moved, nonfinite);
    }
    end_iteration(a, energy, maxd, moved, 0, nonfinite);
}

// ------------------------------------------------------------------ host: plan and build
static int env_int(const char* name, int dflt) {
    const char* e = getenv(name);
    return e ? atoi(e) : dflt;
}

static int pos_bytes_of(int precision) { return precision == GILA_FP64 ? 16 : 8; }

// LDS bytes per staged vertex: its position, and its weight when the
// repulsion is weighted (a weight is half a position).
static int slot_bytes(const gila_khop* kh, int precision) {
    const int pb = pos_bytes_of(precision);
    return kh->mass64 ? pb + pb / 2 : pb;
}

// The large workgroup shape for degree-ordered graphs (rows scatter over the
// ids) of more than one large segment; the small one for caller-ordered
// graphs (meshes, rings, small worlds: rows stay in one or two segments).
static bool seg_big(const gila_khop* kh) {
    if (const char* e = getenv("GILA_SEG_SHAPE")) {
        if (!std::strcmp(e, "small")) return false;
        if (!std::strcmp(e, "large")) return true;
    }
    return !kh->caller_order && kh->n_active > 8190;
}

int seg_size_for(const gila_khop* kh, int precision) {
    const int pos_bytes = pos_bytes_of(precision);
    const bool big = seg_big(kh);
    // LDS of one workgroup: the segment's staged vertices plus ~1 KB of other state
    const int64_t lds_cap = (int64_t)device_info(kh->device).max_lds_per_block - 1024;
    // positions (and weights) of one segment: 64 KB or 32 KB, or all that
    // the weight array of the shape allows
    const int64_t dflt = kh->mass64 ? (int64_t)(big ? weight_base<true>() : weight_base<false>()) * 3 / 2
                                    : (big ? 65536 : 32768);
    const int64_t want = std::min<int64_t>(env_int("GILA_SEG_BYTES", dflt), lds_cap);
    int S = (int)(want / slot_bytes(kh, precision)) - 1;  // one slot for the sentinel
    S = std::min(S, 65535 / pos_bytes - 1);  // byte offsets, sentinel included, fit in 16 bits
    if (kh->mass64)  // positions below the weights
        S = std::min(S, (big ? weight_base<true>() : weight_base<false>()) / pos_bytes - 1);
    return std::max(64, S);
}

// Dynamic LDS of the force kernel for segment size S (the positions; the
// weights of the weighted kernel are in static LDS).
static size_t seg_lds_bytes(const gila_khop* kh, int precision, int S) {
    (void)kh;
    return (size_t)(S + 1) * pos_bytes_of(precision);
}

bool segment_ready_for(const gila_khop* kh, int precision) {
    return kh->seg_ready && segment_path_enabled() && kh->seg == seg_size_for(kh, precision) &&
           kh->seg_weighted == (kh->mass64 != nullptr) && kh->seg_large == seg_big(kh);
}

void free_segments(gila_khop* kh, Release rel) {
    rel(kh->vsl);
    rel(kh->sl_v);
    rel(kh->sl_p);
    rel(kh->sl_k);
    rel(kh->sl_a);
    rel(kh->sk_idx);
    rel(kh->sa_idx);
    rel(kh->seg_wg);
    rel(kh->part);
    rel(kh->sl_dn);
    rel(kh->dmask);
    kh->vsl = nullptr;
    kh->sl_v = kh->sl_p = kh->sl_a = nullptr;
    kh->sl_k = nullptr;
    kh->sk_idx = kh->sa_idx = nullptr;
    kh->seg_wg = nullptr;
    kh->part = nullptr;
    kh->sl_dn = nullptr;
    kh->dmask = nullptr;
    kh->dense_blocks = 0;
    kh->ndense = 0;
    kh->seg_ready = false;
    kh->nslices = 0;
}

namespace {
// One device allocation carved into 256-byte aligned pieces.
struct Arena {
    hipStream_t st;  // the stream that uses it
    void* base = nullptr;
    size_t used = 0;
    explicit Arena(hipStream_t s) : st(s) {}
    ~Arena() { dfree_on(base, st); }
    template <class T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(static_cast<char*>(base) + used);
        used += (count * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
    template <class T>
    static size_t size(size_t count) {
        return (count * sizeof(T) + 255) & ~(size_t)255;
    }
};
}  // namespace

int build_segments(gila_khop* kh, int precision, hipStream_t st) {
    const int32_t na = kh->n_active;
    const int pos_bytes = precision == GILA_FP64 ? 16 : 8;
    const int S = seg_size_for(kh, precision);
    const bool weighted = kh->mass64 != nullptr;
    if (kh->seg_ready && kh->seg == S && kh->seg_weighted == weighted && kh->seg_large == seg_big(kh))
        return GILA_OK;
    free_segments(kh);
    if (na == 0) return GILA_OK;
    if (kh->nnz >= (int64_t)INT32_MAX) return fail(GILA_EUNSUPPORTED, "adjacency too large");
    const int32_t nseg = (int32_t)((na + (int64_t)S - 1) / S);
    if (nseg > kMaxSegments) return fail(GILA_EUNSUPPORTED, "too many segments (%d)", nseg);
    PhaseTimer pt("build_segments", st);
    const int grid_rows = (int)std::min<int64_t>(16384, ((int64_t)na * 64 + kBlock - 1) / kBlock);

    // --- slices per row, row-major offsets
    GILA_TRY(dalloc_t(&kh->vsl, (size_t)na + 1));
    int64_t T = 0;
    {
        Arena ar(st);
        const size_t ws = (size_t)scan_workspace_count(na);
        GILA_TRY(dalloc(&ar.base, Arena::size<int64_t>(na) + Arena::size<int64_t>(ws)));
        SliceBuild b{};
        b.na = na;
        b.S = S;
        b.nseg = nseg;
        b.pos_bytes = pos_bytes;
        b.kptr = kh->kptr;
        b.kidx = kh->kidx;
        b.rp = kh->rp;
        b.ci = kh->ci;
        b.rs = ar.take<int64_t>(na);
        hipLaunchKernelGGL(slice_rows_kernel<false>, dim3(grid_rows), dim3(kBlock), 0, st, b);
        GILA_HIP(hipGetLastError());
        GILA_TRY(enqueue_exclusive_scan_i64(b.rs, kh->vsl, na, ar.take<int64_t>(ws), st));
        GILA_HIP(hipMemcpyAsync(&T, kh->vsl + na, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GILA_HIP(hipStreamSynchronize(st));
    }
    if (T <= 0 || T >= (int64_t)INT32_MAX) return fail(GILA_EUNSUPPORTED, "%lld slices", (long long)T);
    pt.mark("count");
    if (pt.on) pt.log += " nseg=" + std::to_string(nseg) + " slices=" + std::to_string(T);

    // --- slices ordered by segment, then by length (longest first), then
    // row: two stable counting sorts (length, then segment).  Groups of
    // lanes in one wavefront then walk slices of about the same length.
    auto tiling = [&](int32_t nkeys, int64_t& tj, int64_t& ntiles) {
        tj = std::max<int64_t>(1024, (T * (int64_t)nkeys + (1 << 24) - 1) >> 24);
        ntiles = (T + tj - 1) / tj;
    };
    int64_t tj1, nt1, tj2, nt2;
    tiling(kLenKeys, tj1, nt1);
    tiling(nseg, tj2, nt2);
    const int64_t H = std::max(nt1 * kLenKeys, nt2 * nseg);
    const size_t ws = (size_t)std::max(scan_workspace_count(H), scan_workspace_count(T));
    // Dense slices (FP32 positions): a k-hop slice with at least
    // dmin ids (GILA_DENSE_MIN per mille of the segment; 0: none) is kept as
    // a bitmap over the segment's slots, one 64-bit mask per block of 64
    // (dblocks, a whole number of the kernel's eight-block steps).
    const int32_t dblocks = ((S + 63) / 64 + 7) / 8 * 8;
    const int dense_permille = env_int("GILA_DENSE_MIN", 750);
    const bool dense_ok = precision != GILA_FP64 && dense_permille > 0;
    const int32_t dmin =
        dense_ok ? std::max<int32_t>(64, (int32_t)((int64_t)S * dense_permille / 1000)) : 0;
    const int64_t dense_work = S;
    Arena ar(st);
    GILA_TRY(dalloc(&ar.base, Arena::size<int32_t>(T) * 5 + Arena::size<int64_t>(T) +  // d_*
                                  Arena::size<int64_t>(H) + Arena::size<int64_t>(H + 1) +  // hist, its scan
                                  Arena::size<int32_t>(T) * 3 +                            // lenkey, order1, order
                                  Arena::size<int64_t>(T) * 3 + Arena::size<int64_t>(T + 1) +  // wk, wa, dn, sl_a64
                                  Arena::size<int64_t>(ws) + Arena::size<int64_t>(2 * nseg + 4)));
    SliceBuild b{};
    b.na = na;
    b.S = S;
    b.nseg = nseg;
    b.pos_bytes = pos_bytes;
    b.kptr = kh->kptr;
    b.kidx = kh->kidx;
    b.rp = kh->rp;
    b.ci = kh->ci;
    b.vsl = kh->vsl;
    b.d_seg = ar.take<int32_t>(T);
    b.d_k0 = ar.take<int64_t>(T);
    b.d_kn = ar.take<int32_t>(T);
    b.d_a0 = ar.take<int32_t>(T);
    b.d_an = ar.take<int32_t>(T);
    b.d_row = ar.take<int32_t>(T);
    int64_t* hist = ar.take<int64_t>(H);
    int64_t* hscan = ar.take<int64_t>(H + 1);
    int32_t* lenkey = ar.take<int32_t>(T);
    int32_t* order1 = ar.take<int32_t>(T);
    int32_t* order = ar.take<int32_t>(T);
    int64_t* wk = ar.take<int64_t>(T);
    int64_t* wa = ar.take<int64_t>(T);
    int64_t* dn = ar.take<int64_t>(T);
    int64_t* sl_a64 = ar.take<int64_t>(T + 1);
    int64_t* sws = ar.take<int64_t>(ws);
    int64_t* starts = ar.take<int64_t>(2 * nseg + 4);

    GILA_TRY(dalloc_t(&kh->sl_v, (size_t)T));
    GILA_TRY(dalloc_t(&kh->sl_p, (size_t)T));
    GILA_TRY(dalloc_t(&kh->sl_k, (size_t)T + 1));
    GILA_TRY(dalloc_t(&kh->sl_a, (size_t)T + 1));
    GILA_TRY(dalloc_t(&kh->part, (size_t)T));
    if (dense_ok) GILA_TRY(dalloc_t(&kh->sl_dn, (size_t)T + 1));

    hipLaunchKernelGGL(slice_rows_kernel<true>, dim3(grid_rows), dim3(kBlock), 0, st, b);
    const unsigned tgrid = (unsigned)((T + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(slice_lenkey_kernel, dim3(tgrid), dim3(kBlock), 0, st, T, b.d_kn, dmin, lenkey);
    GILA_HIP(hipGetLastError());
    auto counting_sort = [&](int32_t nkeys, int64_t tj, int64_t ntiles, const int32_t* key,
                             const int32_t* perm, int32_t* out) -> int {
        const size_t lds = sizeof(int32_t) * (size_t)nkeys;
        if (lds > 48 * 1024) {
            (void)quiet(hipFuncSetAttribute((const void*)slice_hist_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            (void)quiet(hipFuncSetAttribute((const void*)slice_scatter_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        }
        hipLaunchKernelGGL(slice_hist_kernel, dim3((unsigned)ntiles), dim3(kBlock), lds, st, T, tj,
                           ntiles, nkeys, key, perm, hist);
        GILA_HIP(hipGetLastError());
        GILA_TRY(enqueue_exclusive_scan_i64(hist, hscan, ntiles * nkeys, sws, st));
        hipLaunchKernelGGL(slice_scatter_kernel, dim3((unsigned)ntiles), dim3(64), lds, st, T, tj,
                           ntiles, nkeys, key, perm, hscan, out);
        GILA_HIP(hipGetLastError());
        return GILA_OK;
    };
    GILA_TRY(counting_sort(kLenKeys, tj1, nt1, lenkey, nullptr, order1));
    GILA_TRY(counting_sort(nseg, tj2, nt2, b.d_seg, order1, order));
    const int64_t ntiles = nt2;  // hscan now holds the segment sort's offsets
    hipLaunchKernelGGL(slice_lengths_kernel, dim3((unsigned)((T + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, st, T, order, b.d_kn, b.d_an, dmin, wk, wa, dn);
    GILA_HIP(hipGetLastError());
    GILA_TRY(enqueue_exclusive_scan_i64(wk, kh->sl_k, T, sws, st));
    GILA_TRY(enqueue_exclusive_scan_i64(wa, sl_a64, T, sws, st));
    if (dense_ok) GILA_TRY(enqueue_exclusive_scan_i64(dn, kh->sl_dn, T, sws, st));
    const int64_t slice_cost = env_int("GILA_SEG_ROW_COST", 24);
    hipLaunchKernelGGL(segment_starts_kernel, dim3((nseg + 1 + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       st, nseg, T, ntiles, slice_cost, dense_work, hscan, kh->sl_k, sl_a64,
                       kh->sl_dn, starts);
    GILA_HIP(hipGetLastError());
    std::vector<int64_t> hs((size_t)2 * nseg + 4);
    GILA_HIP(hipMemcpyAsync(hs.data(), starts, sizeof(int64_t) * hs.size(), hipMemcpyDeviceToHost, st));
    GILA_HIP(hipStreamSynchronize(st));
    const int64_t kstore = hs[2 * nseg + 2];
    const int64_t ndense = hs[2 * nseg + 3];
    if (hs[2 * nseg] != T || hs[0] != 0 || ndense < 0 || ndense > T ||
        (ndense == 0 && kstore < kh->P))
        return fail(GILA_EDEVICE, "segment slices do not cover the lists");
    if (pt.on) pt.log += " dense=" + std::to_string(ndense);
    pt.mark("sort");

    // --- workgroups: per segment, ranges of about equal work
    const int cus = device_info(kh->device).cus;
    const int64_t total = hs[2 * nseg + 1] - hs[1];
    // About 16 workgroups per CU, but no fewer than ~96K work units each
    // while that still leaves 8 per CU: staging the segment costs every
    // thread the same few loads whatever its share of pairs (BA 100k, k = 3:
    // 194 -> 182 us per launch; R-MAT 18, whose workgroups get ~130K at 16
    // per CU, is unchanged).  Small graphs keep workgroups of 4096 units.
    const int64_t wpc = std::max<int64_t>(1, env_int("GILA_SEG_WG_PER_CU", 16));
    const int64_t floor_w = std::min<int64_t>(env_int("GILA_SEG_WG_MIN_WORK", 98304),
                                              total / ((int64_t)cus * std::max<int64_t>(1, wpc / 2)));
    const int64_t per_wg = std::max<int64_t>({4096, floor_w, total / ((int64_t)cus * wpc)});
    std::vector<int4> plan;
    for (int32_t sg = 0; sg < nseg; ++sg) {
        if (hs[2 * sg + 2] == hs[2 * sg]) continue;
        const int64_t W = hs[2 * sg + 3] - hs[2 * sg + 1];
        const int c = (int)std::max<int64_t>(1, (W + per_wg - 1) / per_wg);
        for (int t = 0; t < c; ++t) plan.push_back(make_int4(sg, t, c, 0));
    }
    kh->seg = S;
    kh->seg_large = seg_big(kh);  // the shape S was chosen for; launches use this one
    kh->nseg = nseg;
    kh->nslices = T;
    kh->seg_grid = (int32_t)plan.size();
    kh->comb_grid = (na + kBlock - 1) / kBlock;

    GILA_TRY(dalloc_t(&kh->sk_idx, (size_t)kstore + kSegTailPad));
    GILA_TRY(dalloc_t(&kh->sa_idx, (size_t)kh->nnz + 64));
    GILA_TRY(dalloc_t(&kh->seg_wg, plan.size()));
    kh->ndense = ndense;
    kh->dense_blocks = ndense > 0 ? dblocks : 0;
    if (ndense > 0) {
        const size_t masks = (size_t)ndense * dblocks;
        GILA_TRY(dalloc_t(&kh->dmask, masks));
        GILA_HIP(hipMemsetAsync(kh->dmask, 0, masks * sizeof(uint64_t), st));
    }
    if (kh->comb_grid > kh->partials_cap) {
        dfree_on(kh->partials, st);
        kh->partials = nullptr;
        kh->partials_cap = 0;
        GILA_TRY(dalloc_t(&kh->partials, (size_t)kh->comb_grid));
        kh->partials_cap = kh->comb_grid;
    }
    GILA_HIP(hipMemcpyAsync(kh->seg_wg, plan.data(), sizeof(int4) * plan.size(),
                            hipMemcpyHostToDevice, st));
    const int fill_grid =
        (int)std::min<int64_t>(65536, (T * kFillLanes + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(slice_fill_kernel, dim3(fill_grid), dim3(kBlock), 0, st, b, T, order,
                       kh->sl_k, sl_a64, kh->sk_idx, kh->sa_idx, kh->sl_v, kh->sl_p, kh->sl_a);
    if (ndense > 0) {
        const int mgrid = (int)std::min<int64_t>(4096, (T * 64 + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(dense_mask_kernel, dim3(mgrid), dim3(kBlock), 0, st, b, T, order,
                           kh->sl_dn, dblocks, kh->dmask);
    }
    hipLaunchKernelGGL(segment_plan_kernel, dim3((unsigned)((plan.size() + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, st, (int32_t)plan.size(), slice_cost,
                       (int64_t)env_int("GILA_SEG_QPL", 8), dense_work, starts, kh->sl_k, kh->sl_a,
                       kh->ndense > 0 ? kh->sl_dn : nullptr, kh->seg_wg);
    GILA_HIP(hipGetLastError());
    const size_t lds = seg_lds_bytes(kh, precision, S);
    if (lds > 48 * 1024) {
        const void* kernels[] = {
#define GILA_SEG_KERNELS(W, Q, B)                                   \
    (const void*)seg_force_kernel<GILA_FP64, W, Q, B>,              \
        (const void*)seg_force_kernel<GILA_FP32, W, Q, B>,          \
        (const void*)seg_force_kernel<GILA_FP32_KAHAN, W, Q, B>
#define GILA_SEG_KERNELS_B(W, Q) GILA_SEG_KERNELS(W, Q, false), GILA_SEG_KERNELS(W, Q, true)
            GILA_SEG_KERNELS_B(false, 1), GILA_SEG_KERNELS_B(true, 1),  GILA_SEG_KERNELS_B(false, 0),
            GILA_SEG_KERNELS_B(true, 0),  GILA_SEG_KERNELS_B(false, 2), GILA_SEG_KERNELS_B(true, 2),
            GILA_SEG_KERNELS_B(false, 3), GILA_SEG_KERNELS_B(true, 3),  GILA_SEG_KERNELS_B(false, -1),
            GILA_SEG_KERNELS_B(true, -1)
#undef GILA_SEG_KERNELS_B
#undef GILA_SEG_KERNELS
        };
        for (const void* k : kernels)
            (void)quiet(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    GILA_HIP(hipStreamSynchronize(st));
    pt.mark("fill+plan");
    kh->seg_precision = precision;
    kh->seg_weighted = weighted;
    kh->seg_ready = true;
    kh->device_bytes += (int64_t)(na + 1) * 8 + T * (4 + 4 + 8 + 4 + 16) + 2 * (kstore + kh->nnz) +
                        (int64_t)sizeof(int4) * (int64_t)plan.size() +
                        (dense_ok ? (T + 1) * 8 : 0) + ndense * dblocks * 8;
    return GILA_OK;
}

template <bool WEIGHTED, int Q, bool BIG>
static void launch_seg_force(int precision, dim3 sg, size_t lds, hipStream_t s, const SegArgs& g) {
    const dim3 sb(seg_block<BIG>());
    switch (precision) {
        case GILA_FP64: hipLaunchKernelGGL((seg_force_kernel<GILA_FP64, WEIGHTED, Q, BIG>), sg, sb, lds, s, g); break;
        case GILA_FP32: hipLaunchKernelGGL((seg_force_kernel<GILA_FP32, WEIGHTED, Q, BIG>), sg, sb, lds, s, g); break;
        default: hipLaunchKernelGGL((seg_force_kernel<GILA_FP32_KAHAN, WEIGHTED, Q, BIG>), sg, sb, lds, s, g); break;
    }
}

// Repulsion exponents with a kernel of their own; others run the general one.
template <bool WEIGHTED, bool BIG>
static void launch_seg_force_q(int q, int precision, dim3 sg, size_t lds, hipStream_t s,
                               const SegArgs& g) {
    switch (q) {
        case 1: launch_seg_force<WEIGHTED, 1, BIG>(precision, sg, lds, s, g); break;
        case 0: launch_seg_force<WEIGHTED, 0, BIG>(precision, sg, lds, s, g); break;
        case 2: launch_seg_force<WEIGHTED, 2, BIG>(precision, sg, lds, s, g); break;
        case 3: launch_seg_force<WEIGHTED, 3, BIG>(precision, sg, lds, s, g); break;
        default: launch_seg_force<WEIGHTED, -1, BIG>(precision, sg, lds, s, g); break;
    }
}

int launch_segment_step(const gila_khop* kh, int precision, const StepArgs& a, hipStream_t s,
                        unsigned long long* span) {
    if (kh->n_active == 0) return GILA_OK;
    SegArgs g{};
    g.na = kh->n_active;
    g.seg = kh->seg;
    g.wg = kh->seg_wg;
    g.sl_v = kh->sl_v;
    g.sl_p = kh->sl_p;
    g.sl_k = kh->sl_k;
    g.sl_a = kh->sl_a;
    g.kidx = kh->sk_idx;
    g.aidx = kh->sa_idx;
    g.pos = a.pos_cur;
    g.part = kh->part;
    g.d = a.d;
    g.ctl = a.ctl;
    g.mass = a.mass;
    g.att_p = a.att_p;
    g.rep_q = a.rep_q;
    g.span = span;
    g.sl_dn = kh->ndense > 0 ? kh->sl_dn : nullptr;
    g.dmask = kh->dmask;
    g.dense_blocks = kh->dense_blocks;
    StepArgs c = a;
    c.vsl = kh->vsl;
    c.part = kh->part;
    c.nblocks = kh->comb_grid;
    if (precision != GILA_FP64 && precision != GILA_FP32 && precision != GILA_FP32_KAHAN)
        return fail(GILA_EINVAL, "unknown precision %d", precision);
    if ((a.mass != nullptr) != kh->seg_weighted)
        return fail(GILA_EINVAL, "segment layout built for other repulsion weights");
    const size_t lds = seg_lds_bytes(kh, precision, kh->seg);
    const dim3 sg(kh->seg_grid), cg(kh->comb_grid), cb(kBlock);
    const bool big = kh->seg_large;
    if (a.mass && big) launch_seg_force_q<true, true>(a.rep_q, precision, sg, lds, s, g);
    else if (a.mass) launch_seg_force_q<true, false>(a.rep_q, precision, sg, lds, s, g);
    else if (big) launch_seg_force_q<false, true>(a.rep_q, precision, sg, lds, s, g);
    else launch_seg_force_q<false, false>(a.rep_q, precision, sg, lds, s, g);
    switch (precision) {
        case GILA_FP64: hipLaunchKernelGGL(seg_combine_kernel<GILA_FP64>, cg, cb, 0, s, c); break;
        case GILA_FP32: hipLaunchKernelGGL(seg_combine_kernel<GILA_FP32>, cg, cb, 0, s, c); break;
        default: hipLaunchKernelGGL(seg_combine_kernel<GILA_FP32_KAHAN>, cg, cb, 0, s, c); break;
    }
    GILA_TRY(launch_iteration_stats(c, s));
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

}  // namespace gila

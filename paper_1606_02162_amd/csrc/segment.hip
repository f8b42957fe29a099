// Segment-blocked iteration: every neighbour gather comes from LDS.
//
// Internal vertex ids are split into segments of S consecutive ids (S
// positions fill 32 KB of LDS by default).  Each k-hop row (and adjacency
// row) of an active vertex v is cut into per-segment slices; slice (s, v)
// holds the ids of N_v(k) (resp. adj(v)) that fall in segment s, stored as
// 16-bit LDS byte offsets (id - s*S) * sizeof(position), segment-major: all
// slices of segment s, rows in internal order.  k-hop slices are padded to a
// whole number of 4-id quads with a sentinel offset: LDS slot S holds a
// position so far away (1e30) that its squared distance overflows to +inf, the
// reciprocal is exactly 0 and the padding term is exactly zero.  Each lane then
// loads one aligned 8-byte quad of ids per memory instruction.
//
// One iteration is two kernels:
//   seg_force_kernel   one workgroup = one segment x a pair-balanced range of
//                      rows.  It copies the segment's positions into LDS,
//                      then sums repulsion (k-hop slice) and attraction
//                      (adjacency slice) for each row of its range, and
//                      writes the row's partial force for that segment
//                      (FP32 / Kahan lane sums, double-precision combine).
//   seg_combine_kernel one thread per vertex: adds the vertex's partials in
//                      segment order, applies the temperature cap, writes the
//                      vertex's next position and the iteration statistics.
// The result of every row depends only on the graph's plan (lanes per row of
// its workgroup) and on the fixed segment order, never on scheduling.
#include <algorithm>
#include <cstdlib>

#include "iteration.h"

namespace gila {

constexpr int kSegBlock = 512;   // threads per segment workgroup
constexpr int kSegTailPad = 1024;  // slack entries after the k-hop index array (>= 3 * 64 quads)

bool segment_path_enabled() {
    const char* e = getenv("GILA_PATH");
    return !(e && std::strcmp(e, "direct") == 0);
}

// ------------------------------------------------------------------ build: counts
// Wave per active row v: slice lengths of the (sorted) k-hop and adjacency
// rows for every segment, by binary search of the segment boundaries.
__device__ __forceinline__ int64_t lower_bound_i32(const int32_t* __restrict__ a, int64_t lo,
                                                   int64_t hi, int32_t key) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void seg_count_kernel(
    int32_t na, int32_t S, int32_t nseg, const int64_t* __restrict__ kptr,
    const int32_t* __restrict__ kidx, const int64_t* __restrict__ rp,
    const int32_t* __restrict__ ci, int32_t* __restrict__ kcnt, int32_t* __restrict__ acnt) {
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
    const int lane = lane64();
    for (int64_t v = wave; v < na; v += nwaves) {
        const int64_t kb = kptr[v], ke = kptr[v + 1];
        const int64_t ab = rp[v], ae = rp[v + 1];
        for (int s = lane; s < nseg; s += 64) {
            const int32_t lo_id = s * S, hi_id = (s + 1) * S;
            const int64_t k0 = lower_bound_i32(kidx, kb, ke, lo_id);
            const int64_t k1 = lower_bound_i32(kidx, k0, ke, hi_id);
            const int64_t a0 = lower_bound_i32(ci, ab, ae, lo_id);
            const int64_t a1 = lower_bound_i32(ci, a0, ae, hi_id);
            kcnt[(int64_t)s * na + v] = (int32_t)(k1 - k0);
            acnt[(int64_t)s * na + v] = (int32_t)(a1 - a0);
        }
    }
}

// Wave per active row: write each slice as LDS byte offsets into its place,
// k-hop slices padded to whole quads with the sentinel offset.
__global__ __launch_bounds__(kBlock) void seg_fill_kernel(
    int32_t na, int32_t S, int32_t nseg, int32_t pos_bytes, const int64_t* __restrict__ kptr,
    const int32_t* __restrict__ kidx, const int64_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const int32_t* __restrict__ kcnt,
    const int64_t* __restrict__ sk_ptr, uint16_t* __restrict__ sk_idx,
    const int32_t* __restrict__ sa_ptr, uint16_t* __restrict__ sa_idx) {
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
    const int lane = lane64();
    const uint16_t sentinel = (uint16_t)(S * pos_bytes);
    for (int64_t v = wave; v < na; v += nwaves) {
        int64_t kpos = kptr[v];
        int64_t apos = rp[v];
        for (int s = 0; s < nseg; ++s) {
            const int64_t slot = (int64_t)s * na + v;
            const int64_t kdst = sk_ptr[slot], kpad = sk_ptr[slot + 1] - kdst;
            const int32_t klen = kcnt[slot];
            const int32_t base = s * S;
            for (int64_t j = lane; j < kpad; j += 64)
                sk_idx[kdst + j] =
                    j < klen ? (uint16_t)((kidx[kpos + j] - base) * pos_bytes) : sentinel;
            kpos += klen;
            const int64_t adst = sa_ptr[slot], alen = sa_ptr[slot + 1] - adst;
            for (int64_t j = lane; j < alen; j += 64)
                sa_idx[adst + j] = (uint16_t)((ci[apos + j] - base) * pos_bytes);
            apos += alen;
        }
    }
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
template <class P>
__device__ __forceinline__ void quad_terms(uint2 w, const unsigned char* __restrict__ lds,
                                           typename P::real xv, typename P::real yv,
                                           typename P::real d2, typename P::real& sx,
                                           typename P::real& sy, typename P::real& mindd) {
    using R = typename P::real;
    using V = typename P::vec2;
    const V p0 = *reinterpret_cast<const V*>(lds + (w.x & 0xFFFFu));
    const V p1 = *reinterpret_cast<const V*>(lds + (w.x >> 16));
    const V p2 = *reinterpret_cast<const V*>(lds + (w.y & 0xFFFFu));
    const V p3 = *reinterpret_cast<const V*>(lds + (w.y >> 16));
    R x0, y0, x1, y1, x2, y2, x3, y3;
    repulse_term<P>(xv, yv, p0, d2, x0, y0, mindd);
    repulse_term<P>(xv, yv, p1, d2, x1, y1, mindd);
    repulse_term<P>(xv, yv, p2, d2, x2, y2, mindd);
    repulse_term<P>(xv, yv, p3, d2, x3, y3, mindd);
    sx = (x0 + x1) + (x2 + x3);
    sy = (y0 + y1) + (y2 + y3);
}

template <class P, int LPV>
__device__ __forceinline__ void seg_rows(const SegArgs& a, int s, int vb, int ve,
                                         const typename P::vec2* __restrict__ lp,
                                         int& coinc) {
    using R = typename P::real;
    using V = typename P::vec2;
    const V* __restrict__ gpos = reinterpret_cast<const V*>(a.pos);
    const unsigned char* __restrict__ lds = reinterpret_cast<const unsigned char*>(lp);
    const R d2 = (R)(a.d * a.d);
    const R dpar = attract_param<R>(a.d);
    const int ngroups = kSegBlock / LPV;
    const int grp = threadIdx.x / LPV;
    const int gl = threadIdx.x % LPV;
    const int64_t sbase = (int64_t)s * a.na;
    const uint32_t sq = (uint32_t)a.seg * (uint32_t)sizeof(V);
    const uint2 sentinel = make_uint2(sq | (sq << 16), sq | (sq << 16));
    for (int v0 = vb; v0 < ve; v0 += ngroups) {
        const int v = v0 + grp;
        Acc<R, P::kahan> acc;
        if (v < ve) {
            const V xv = gpos[v];
            const int64_t slot = sbase + v;
            const int64_t kb = a.kptr[slot], ke = a.kptr[slot + 1];
            const uint2* __restrict__ q4 = reinterpret_cast<const uint2*>(a.kidx + kb);
            const int nq = (int)((ke - kb) >> 2);
            R mindd = R(1);
            // two quads per lane per step, the next two already in flight.
            // Loads run up to 3*LPV quads past the row end (the index array
            // carries kSegTailPad entries of slack); quads past the end are
            // replaced by sentinels, whose terms are exactly 0.
            int q = gl;
            uint2 n0 = q4[q];
            uint2 n1 = q4[q + LPV];
            while (q < nq) {
                const uint2 w0 = n0;
                const uint2 w1 = q + LPV < nq ? n1 : sentinel;
                q += 2 * LPV;
                n0 = q4[q];
                n1 = q4[q + LPV];
                R sx, sy;
                quad_terms<P>(w0, lds, xv.x, xv.y, d2, sx, sy, mindd);
                acc.add(sx, sy);
                quad_terms<P>(w1, lds, xv.x, xv.y, d2, sx, sy, mindd);
                acc.add(sx, sy);
            }
            if (mindd == R(0)) coinc += count_coincident_quads<V, LPV>(xv, q4, nq, gl, lds);
            const int32_t ab = a.aptr[slot], ae = a.aptr[slot + 1];
            for (int32_t j = ab + gl; j < ae; j += LPV)
                attract<P>(xv.x, xv.y, *reinterpret_cast<const V*>(lds + a.aidx[j]), dpar, acc);
        }
        const double fx = group_sum<LPV>(acc.x());
        const double fy = group_sum<LPV>(acc.y());
        if (v < ve && gl == 0) a.part[sbase + v] = make_double2(fx, fy);
    }
}

template <int PREC>
__global__ __launch_bounds__(kSegBlock) void seg_force_kernel(SegArgs a) {
    using P = Prec<PREC>;
    using V = typename P::vec2;
    extern __shared__ __align__(16) unsigned char s_raw[];
    V* lp = reinterpret_cast<V*>(s_raw);
    __shared__ int64_t s_c[kSegBlock / 64];
    if (a.ctl->stopped) return;
    const int4 w = a.wg[blockIdx.x];
    const int s = w.x, vb = w.y, ve = w.z, lpv = w.w;
    // stage the segment's positions
    const V* gpos = reinterpret_cast<const V*>(a.pos);
    const int64_t base = (int64_t)s * a.seg;
    const int64_t left = (int64_t)a.na - base;
    const int cnt = (int)(left < a.seg ? left : a.seg);
    for (int i = threadIdx.x; i < cnt; i += kSegBlock) lp[i] = gpos[base + i];
    if (threadIdx.x == 0) {
        V far;
        far.x = sizeof(far.x) == 4 ? (decltype(far.x))1e30f : (decltype(far.x))1e300;
        far.y = far.x;
        lp[a.seg] = far;  // sentinel slot: padding terms vanish exactly
    }
    __syncthreads();
    int coinc = 0;
    switch (lpv) {
        case 1: seg_rows<P, 1>(a, s, vb, ve, lp, coinc); break;
        case 2: seg_rows<P, 2>(a, s, vb, ve, lp, coinc); break;
        case 4: seg_rows<P, 4>(a, s, vb, ve, lp, coinc); break;
        case 8: seg_rows<P, 8>(a, s, vb, ve, lp, coinc); break;
        case 16: seg_rows<P, 16>(a, s, vb, ve, lp, coinc); break;
        case 32: seg_rows<P, 32>(a, s, vb, ve, lp, coinc); break;
        default: seg_rows<P, 64>(a, s, vb, ve, lp, coinc); break;
    }
    const int64_t wc = wave_sum((int64_t)coinc);
    if (lane64() == 0) s_c[wave_id()] = wc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t c = 0;
        for (int i = 0; i < kSegBlock / 64; ++i) c += s_c[i];
        if (c) atomicAdd((unsigned long long*)&a.ctl->coinc_pending, (unsigned long long)c);
    }
}

// ------------------------------------------------------------------ iteration: combine kernel
template <int PREC>
__global__ __launch_bounds__(kBlock) void seg_combine_kernel(StepArgs a) {
    using P = Prec<PREC>;
    using V = typename P::vec2;
    if (a.ctl->stopped) return;
    double energy = 0.0, maxd = 0.0;
    int64_t moved = 0;
    const int32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < a.n_active) {
        double fx = 0.0, fy = 0.0;
        for (int s = 0; s < a.nseg; ++s) {
            const double2 p = a.part[(int64_t)s * a.n_active + v];
            fx += p.x;
            fy += p.y;
        }
        const V xv = reinterpret_cast<const V*>(a.pos_cur)[v];
        finish_vertex<P>(a, v, xv, fx, fy, energy, maxd, moved);
    }
    end_iteration(a, energy, maxd, moved, 0);
}

// ------------------------------------------------------------------ host: plan and build
static int env_int(const char* name, int dflt) {
    const char* e = getenv(name);
    return e ? atoi(e) : dflt;
}

int seg_size_for(int precision, int device) {
    const int pos_bytes = precision == GILA_FP64 ? 16 : 8;
    // LDS of one workgroup: the segment's positions plus ~1 KB of other state
    const int64_t lds_cap = (int64_t)device_info(device).max_lds_per_block - 1024;
    const int64_t want = std::min<int64_t>(env_int("GILA_SEG_BYTES", 32768), lds_cap);
    int S = (int)(want / pos_bytes) - 1;  // one slot for the sentinel
    S = std::min(S, 65535 / pos_bytes - 1);  // byte offsets, sentinel included, fit in 16 bits
    return std::max(64, S);
}

static int lanes_for(int64_t med) {
    // enough quads per lane (GILA_SEG_QPL, default 8) to amortise the
    // per-slice reduction
    const int64_t qpl = env_int("GILA_SEG_QPL", 8);
    int l = 1;
    while (l < 64 && (int64_t)l * 2 * qpl * 4 <= med) l *= 2;
    return l;
}

int build_segments(gila_khop* kh, int precision, hipStream_t st) {
    const int32_t na = kh->n_active;
    const int pos_bytes = precision == GILA_FP64 ? 16 : 8;
    const int S = seg_size_for(precision, kh->device);
    if (kh->seg_ready && kh->seg == S) return GILA_OK;
    // release an older layout
    dfree(kh->sk_ptr);
    dfree(kh->sk_idx);
    dfree(kh->sa_ptr);
    dfree(kh->sa_idx);
    dfree(kh->seg_wg);
    dfree(kh->part);
    kh->sk_ptr = nullptr;
    kh->sk_idx = nullptr;
    kh->sa_ptr = nullptr;
    kh->sa_idx = nullptr;
    kh->seg_wg = nullptr;
    kh->part = nullptr;
    kh->seg_ready = false;
    if (na == 0) return GILA_OK;
    if (kh->nnz >= (int64_t)INT32_MAX) return fail(GILA_EUNSUPPORTED, "adjacency too large");
    const int32_t nseg = (int32_t)((na + (int64_t)S - 1) / S);
    const int64_t slots = (int64_t)nseg * na;
    PhaseTimer pt("build_segments", st);

    int32_t *d_kc = nullptr, *d_ac = nullptr;
    GILA_TRY(dalloc_t(&d_kc, (size_t)slots));
    int rc = dalloc_t(&d_ac, (size_t)slots);
    if (rc) {
        dfree(d_kc);
        return rc;
    }
    const int grid = (int)std::min<int64_t>(8192, ((int64_t)na * 64 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(seg_count_kernel, dim3(grid), dim3(kBlock), 0, st, na, S, nseg, kh->kptr,
                       kh->kidx, kh->rp, kh->ci, d_kc, d_ac);
    std::vector<int32_t> kc((size_t)slots), ac((size_t)slots);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipMemcpyAsync(kc.data(), d_kc, sizeof(int32_t) * slots, hipMemcpyDeviceToHost, st);
    hipError_t e3 = hipMemcpyAsync(ac.data(), d_ac, sizeof(int32_t) * slots, hipMemcpyDeviceToHost, st);
    hipError_t e4 = hipStreamSynchronize(st);
    dfree(d_ac);
    struct KcGuard {
        int32_t* p;
        ~KcGuard() { dfree(p); }
    } kc_guard{d_kc};
    if (e1 || e2 || e3 || e4) return fail(GILA_EDEVICE, "segment count failed");

    pt.mark("count");
    // segment-major offsets
    std::vector<int64_t> skp((size_t)slots + 1);
    std::vector<int32_t> sap((size_t)slots + 1);
    skp[0] = 0;
    sap[0] = 0;
    int64_t ksum = 0;
    for (int64_t i = 0; i < slots; ++i) {
        ksum += kc[i];
        skp[i + 1] = skp[i] + ((kc[i] + 3) & ~3);
        sap[i + 1] = sap[i] + ac[i];
    }
    if (ksum != kh->P || sap[slots] != kh->nnz)
        return fail(GILA_EDEVICE, "segment slices do not cover the lists");
    const int64_t kstore = skp[slots];

    // workgroup plan: per segment, contiguous row ranges of ~equal work
    const int cus = device_info(kh->device).cus;
    const int64_t row_cost = env_int("GILA_SEG_ROW_COST", 24);
    const int64_t total = kh->P + kh->nnz + row_cost * slots;
    const int64_t target_wgs = (int64_t)cus * env_int("GILA_SEG_WG_PER_CU", 16);
    const int64_t per_wg = std::max<int64_t>(4096, total / std::max<int64_t>(1, target_wgs));
    std::vector<int4> plan;
    std::vector<int64_t> lens;
    for (int32_t s = 0; s < nseg; ++s) {
        const int64_t b = (int64_t)s * na;
        int32_t start = 0;
        int64_t acc = 0;
        for (int32_t v = 0; v < na; ++v) {
            acc += kc[b + v] + ac[b + v] + row_cost;
            if (acc >= per_wg || v == na - 1) {
                lens.clear();
                for (int32_t u = start; u <= v; ++u) lens.push_back(kc[b + u] + ac[b + u]);
                std::nth_element(lens.begin(), lens.begin() + lens.size() / 2, lens.end());
                const int lpv = lanes_for(lens[lens.size() / 2]);
                plan.push_back(make_int4(s, start, v + 1, lpv));
                start = v + 1;
                acc = 0;
            }
        }
    }
    pt.mark("plan");
    kh->seg = S;
    kh->nseg = nseg;
    kh->seg_grid = (int32_t)plan.size();
    kh->comb_grid = (na + kBlock - 1) / kBlock;

    GILA_TRY(dalloc_t(&kh->sk_ptr, (size_t)slots + 1));
    GILA_TRY(dalloc_t(&kh->sa_ptr, (size_t)slots + 1));
    GILA_TRY(dalloc_t(&kh->sk_idx, (size_t)kstore + kSegTailPad));
    GILA_TRY(dalloc_t(&kh->sa_idx, (size_t)kh->nnz + 64));
    GILA_TRY(dalloc_t(&kh->seg_wg, plan.size()));
    GILA_TRY(dalloc_t(&kh->part, (size_t)slots));
    if (kh->comb_grid > kh->partials_cap) {
        dfree(kh->partials);
        kh->partials = nullptr;
        kh->partials_cap = 0;
        GILA_TRY(dalloc_t(&kh->partials, (size_t)kh->comb_grid));
        kh->partials_cap = kh->comb_grid;
    }
    pt.mark("alloc");
    GILA_HIP(hipMemcpyAsync(kh->sk_ptr, skp.data(), sizeof(int64_t) * (slots + 1),
                            hipMemcpyHostToDevice, st));
    GILA_HIP(hipMemcpyAsync(kh->sa_ptr, sap.data(), sizeof(int32_t) * (slots + 1),
                            hipMemcpyHostToDevice, st));
    GILA_HIP(hipMemcpyAsync(kh->seg_wg, plan.data(), sizeof(int4) * plan.size(),
                            hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(seg_fill_kernel, dim3(grid), dim3(kBlock), 0, st, na, S, nseg, pos_bytes,
                       kh->kptr, kh->kidx, kh->rp, kh->ci, d_kc, kh->sk_ptr, kh->sk_idx,
                       kh->sa_ptr, kh->sa_idx);
    GILA_HIP(hipGetLastError());
    pt.mark("upload+fill");
    const size_t lds = (size_t)(S + 1) * pos_bytes;
    if (lds > 48 * 1024) {
        (void)hipFuncSetAttribute((const void*)seg_force_kernel<GILA_FP64>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute((const void*)seg_force_kernel<GILA_FP32>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute((const void*)seg_force_kernel<GILA_FP32_KAHAN>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    GILA_HIP(hipStreamSynchronize(st));
    kh->seg_precision = precision;
    kh->seg_ready = true;
    kh->device_bytes += (int64_t)(slots + 1) * 12 + 2 * (kstore + kh->nnz) + 16 * slots +
                        (int64_t)sizeof(int4) * (int64_t)plan.size();
    return GILA_OK;
}

int launch_segment_step(const gila_khop* kh, int precision, const StepArgs& a, hipStream_t s,
                        hipEvent_t* ev) {
    if (kh->n_active == 0) return GILA_OK;
    SegArgs g{};
    g.na = kh->n_active;
    g.seg = kh->seg;
    g.wg = kh->seg_wg;
    g.kptr = kh->sk_ptr;
    g.kidx = kh->sk_idx;
    g.aptr = kh->sa_ptr;
    g.aidx = kh->sa_idx;
    g.pos = a.pos_cur;
    g.part = kh->part;
    g.d = a.d;
    g.ctl = a.ctl;
    StepArgs c = a;
    c.nseg = kh->nseg;
    c.part = kh->part;
    c.nblocks = kh->comb_grid;
    const int pos_bytes = precision == GILA_FP64 ? 16 : 8;
    const size_t lds = (size_t)(kh->seg + 1) * pos_bytes;
    const dim3 sg(kh->seg_grid), sb(kSegBlock), cg(kh->comb_grid), cb(kBlock);
    if (precision != GILA_FP64 && precision != GILA_FP32 && precision != GILA_FP32_KAHAN)
        return fail(GILA_EINVAL, "unknown precision %d", precision);
    if (ev) GILA_HIP(hipEventRecord(ev[0], s));
    switch (precision) {
        case GILA_FP64: hipLaunchKernelGGL(seg_force_kernel<GILA_FP64>, sg, sb, lds, s, g); break;
        case GILA_FP32: hipLaunchKernelGGL(seg_force_kernel<GILA_FP32>, sg, sb, lds, s, g); break;
        default: hipLaunchKernelGGL(seg_force_kernel<GILA_FP32_KAHAN>, sg, sb, lds, s, g); break;
    }
    if (ev) GILA_HIP(hipEventRecord(ev[1], s));
    switch (precision) {
        case GILA_FP64: hipLaunchKernelGGL(seg_combine_kernel<GILA_FP64>, cg, cb, 0, s, c); break;
        case GILA_FP32: hipLaunchKernelGGL(seg_combine_kernel<GILA_FP32>, cg, cb, 0, s, c); break;
        default: hipLaunchKernelGGL(seg_combine_kernel<GILA_FP32_KAHAN>, cg, cb, 0, s, c); break;
    }
    if (ev) GILA_HIP(hipEventRecord(ev[2], s));
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

}  // namespace gila

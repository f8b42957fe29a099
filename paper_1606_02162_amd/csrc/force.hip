// One layout iteration: forces, capped synchronous move, statistics.
//
// For every non-isolated vertex v (Section 3.1 force law, p = 2, q = 1, with
// the repulsion restricted to N_v(k) as in Section 4.5):
//   F_v = sum_{u in N_v(k)} (x_v - x_u) d^2 / |x_v - x_u|^2
//       + sum_{u in adj(v)} (x_u - x_v) |x_u - x_v| / d
//   Delta_v = F_v min(|F_v|, t) / |F_v|   (0 if F_v = 0)
//   x_v <- x_v + Delta_v                  (written to the other buffer: all
//                                          vertices move at once)
// A pair at distance 0 contributes nothing and is counted.
//
// Mapping: a group of LPV lanes of a 64-wide wavefront owns one vertex and
// strides its k-hop row with unit-stride (coalesced) loads of neighbour ids,
// gathering each neighbour position as one 8-byte (FP32) or 16-byte (FP64)
// load.  Lane sums are combined in double precision with a fixed butterfly
// of cross-lane shuffles, so every result is deterministic.  The longest rows
// ("hubs", which come first in the internal order) get a whole 256-thread
// workgroup.  Workgroups of ordinary vertices cover contiguous vertex ranges
// balanced by pair count, planned once per graph.  Per-workgroup statistics
// are reduced in a fixed order by whichever workgroup finishes last.
#include <algorithm>
#include <cmath>

#include "iteration.h"

namespace gila {

// Partial force of one vertex over lanes lane0, lane0+STRIDE, ... of its rows.
// WEIGHTED scales the repulsion from u by u's weight (Section 4.6).
template <class P, int STRIDE, bool WEIGHTED>
__device__ __forceinline__ void vertex_partial(const StepArgs& a, int32_t v, int lane0,
                                               Acc<typename P::real, P::kahan>& acc, int& coinc,
                                               typename P::vec2& xv_out) {
    using R = typename P::real;
    using V = typename P::vec2;
    const V* __restrict__ pos = reinterpret_cast<const V*>(a.pos_cur);
    const V xv = pos[v];
    xv_out = xv;
    const R d2 = (R)(a.d * a.d);
    const R inv_d = attract_param<R>(a.d);
    const R* __restrict__ wt = reinterpret_cast<const R*>(a.mass);
    auto scale = [&](int32_t u) -> R {
        if constexpr (WEIGHTED) return d2 * wt[u];
        else return d2;
    };
    const int64_t kb = a.kptr[v], ke = a.kptr[v + 1];
    int64_t e = kb + lane0;
    // four independent gathers in flight per lane
    for (; e + 3 * STRIDE < ke; e += 4 * STRIDE) {
        const int32_t u0 = a.kidx[e];
        const int32_t u1 = a.kidx[e + STRIDE];
        const int32_t u2 = a.kidx[e + 2 * STRIDE];
        const int32_t u3 = a.kidx[e + 3 * STRIDE];
        const V p0 = pos[u0], p1 = pos[u1], p2 = pos[u2], p3 = pos[u3];
        repulse<P>(xv.x, xv.y, p0, scale(u0), acc, coinc, a.rep_q);
        repulse<P>(xv.x, xv.y, p1, scale(u1), acc, coinc, a.rep_q);
        repulse<P>(xv.x, xv.y, p2, scale(u2), acc, coinc, a.rep_q);
        repulse<P>(xv.x, xv.y, p3, scale(u3), acc, coinc, a.rep_q);
    }
    for (; e < ke; e += STRIDE) {
        const int32_t u = a.kidx[e];
        repulse<P>(xv.x, xv.y, pos[u], scale(u), acc, coinc, a.rep_q);
    }
    const int64_t rb = a.rp[v], re = a.rp[v + 1];
    for (int64_t j = rb + lane0; j < re; j += STRIDE)
        attract<P>(xv.x, xv.y, pos[a.ci[j]], inv_d, acc, a.att_p);
}

template <int PREC, int LPV, bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void fr_step_kernel(StepArgs a) {
    using P = Prec<PREC>;
    using V = typename P::vec2;
    __shared__ double s_fx[kWaves], s_fy[kWaves];

    if (a.ctl->stopped) return;  // the halting rule fired in an earlier iteration

    const int lane = lane64();
    const int w = wave_id();
    double energy = 0.0, maxd = 0.0;
    int64_t moved = 0, nonfinite = 0;
    int coinc = 0;

    if ((int32_t)blockIdx.x < a.nhub) {
        // one hub vertex per workgroup
        const int32_t v = blockIdx.x;
        Acc<typename P::real, P::kahan> acc;
        V xv;
        vertex_partial<P, kBlock, WEIGHTED>(a, v, threadIdx.x, acc, coinc, xv);
        double fx = wave_sum(acc.x()), fy = wave_sum(acc.y());
        if (lane == 0) {
            s_fx[w] = fx;
            s_fy[w] = fy;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            fx = s_fx[0];
            fy = s_fy[0];
            for (int i = 1; i < kWaves; ++i) {
                fx += s_fx[i];
                fy += s_fy[i];
            }
            finish_vertex<P>(a, v, xv, fx, fy, energy, maxd, moved, nonfinite);
        }
    } else {
        constexpr int G = 64 / LPV;                 // vertices in flight per wavefront
        const int b = blockIdx.x - a.nhub;
        const int32_t vb = a.block_start[b], ve = a.block_start[b + 1];
        const int grp = w * G + lane / LPV;         // group index in the workgroup
        const int gl = lane % LPV;                  // lane within the group
        for (int32_t base = vb; base < ve; base += kWaves * G) {
            const int32_t v = base + grp;
            const bool live = v < ve;
            Acc<typename P::real, P::kahan> acc;
            V xv;
            xv.x = 0;
            xv.y = 0;
            if (live) vertex_partial<P, LPV, WEIGHTED>(a, v, gl, acc, coinc, xv);
            const double fx = group_sum<LPV>(acc.x());
            const double fy = group_sum<LPV>(acc.y());
            if (live && gl == 0)
                finish_vertex<P>(a, v, xv, fx, fy, energy, maxd, moved, nonfinite);
        }
    }

    end_iteration(a, energy, maxd, moved, (int64_t)coinc, nonfinite);
}

// ------------------------------------------------------------------ launch
template <int PREC, bool WEIGHTED>
static void launch_lpv(int lpv, const StepArgs& a, hipStream_t s) {
    const dim3 grid(a.nblocks), block(kBlock);
    switch (lpv) {
        case 4: hipLaunchKernelGGL((fr_step_kernel<PREC, 4, WEIGHTED>), grid, block, 0, s, a); break;
        case 8: hipLaunchKernelGGL((fr_step_kernel<PREC, 8, WEIGHTED>), grid, block, 0, s, a); break;
        case 16: hipLaunchKernelGGL((fr_step_kernel<PREC, 16, WEIGHTED>), grid, block, 0, s, a); break;
        case 32: hipLaunchKernelGGL((fr_step_kernel<PREC, 32, WEIGHTED>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((fr_step_kernel<PREC, 64, WEIGHTED>), grid, block, 0, s, a); break;
    }
}

template <int PREC>
static void launch_prec(int lpv, const StepArgs& a, hipStream_t s) {
    if (a.mass) launch_lpv<PREC, true>(lpv, a, s);
    else launch_lpv<PREC, false>(lpv, a, s);
}

int launch_step(const gila_khop* kh, int precision, const StepArgs& a, hipStream_t s) {
    if (a.nblocks <= 0) return GILA_OK;
    switch (precision) {
        case GILA_FP64: launch_prec<GILA_FP64>(kh->lpv, a, s); break;
        case GILA_FP32: launch_prec<GILA_FP32>(kh->lpv, a, s); break;
        case GILA_FP32_KAHAN: launch_prec<GILA_FP32_KAHAN>(kh->lpv, a, s); break;
        default: return fail(GILA_EINVAL, "unknown precision %d", precision);
    }
    GILA_HIP(hipGetLastError());
    return launch_iteration_stats(a, s);
}

// ------------------------------------------------------------------ plan
// Rows of at least kHubMin pairs come first in the internal order and get a
// workgroup each; the rest are packed into contiguous ranges of about
// kPairsPerBlock pairs (plus a per-vertex overhead) and at most
// kMaxVertsPerBlock vertices.
static constexpr int64_t kVertexCost = 32;

int plan_iteration(gila_khop* kh, const std::vector<int64_t>& counts,
                   const std::vector<int64_t>& rp_internal, hipStream_t s) {
    const int32_t na = kh->n_active;
    int32_t nhub = 0;
    while (nhub < na && counts[nhub] >= kHubMin) ++nhub;
    // lanes per vertex from the median row length of the non-hub vertices
    int64_t med = 0;
    if (na > nhub) {
        std::vector<int64_t> rest(counts.begin() + nhub, counts.begin() + na);
        std::nth_element(rest.begin(), rest.begin() + rest.size() / 2, rest.end());
        med = rest[rest.size() / 2];
    }
    int lpv = 4;
    while (lpv < 64 && lpv * 8 < med) lpv *= 2;
    const int64_t pairs_per_block = std::max<int64_t>(2048, 64ll * lpv);
    const int32_t max_verts = kWaves * (64 / lpv) * 16;
    std::vector<int32_t> starts;
    starts.push_back(nhub);
    int64_t acc = 0;
    int32_t cnt = 0;
    for (int32_t v = nhub; v < na; ++v) {
        acc += counts[v] + (rp_internal[v + 1] - rp_internal[v]) + kVertexCost;
        ++cnt;
        if (acc >= pairs_per_block || cnt >= max_verts) {
            starts.push_back(v + 1);
            acc = 0;
            cnt = 0;
        }
    }
    if (starts.back() != na) starts.push_back(na);
    kh->lpv = lpv;
    kh->nhub = nhub;
    const int32_t nnormal = (int32_t)starts.size() - 1;
    kh->nblocks = nhub + nnormal;
    GILA_TRY(dalloc_t(&kh->block_start, starts.size()));
    // on the build's stream (never the legacy one, which must not meet a
    // capture in progress on another thread); `starts` lives until the copy ends
    GILA_HIP(hipMemcpyAsync(kh->block_start, starts.data(), sizeof(int32_t) * starts.size(),
                            hipMemcpyHostToDevice, s));
    GILA_HIP(hipStreamSynchronize(s));
    return GILA_OK;
}

}  // namespace gila

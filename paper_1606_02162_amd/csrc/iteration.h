// Device pieces shared by the iteration kernels: precision policies, the
// per-pair force terms, the lane accumulator, the capped move, and the
// fixed-order statistics reduction that ends every iteration.
#pragma once

#include <cfloat>

#include "device_util.h"
#include "gila_internal.h"

namespace gila {

template <int PREC>
struct Prec;

template <>
struct Prec<GILA_FP64> {
    using real = double;
    using vec2 = double2;
    static constexpr bool kahan = false;
};
template <>
struct Prec<GILA_FP32> {
    using real = float;
    using vec2 = float2;
    static constexpr bool kahan = false;
};
template <>
struct Prec<GILA_FP32_KAHAN> {
    using real = float;
    using vec2 = float2;
    static constexpr bool kahan = true;
};

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <class R>
__device__ __forceinline__ R fast_rsqrt(R x) {
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rsqf(x);
    else return R(1) / sqrt(x);
}

// 1 / sqrt(dd) where inv = 1 / dd is at hand: in FP64 the square root of
// inv, which saves a double division per pair.
template <class R>
__device__ __forceinline__ R rsqrt_with_inv(R dd, R inv) {
    if constexpr (sizeof(R) == 4) return fast_rsqrt(dd);
    else return sqrt(inv);
}

// x^k for a small non-negative integer k (uniform across the wavefront).
template <class R>
__device__ __forceinline__ R pow_int(R x, int k) {
    R r = R(1);
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

// General repulsion exponent q (Section 3.1: magnitude d^2 / delta^q): the
// factor multiplying (x_v - x_u) d^2 is delta^-(q+1) = (delta^2)^-(q+1)/2,
// from inv = 1 / delta^2 and, for even q, one reciprocal square root.  A
// coincident pair (dd at most the coincidence bias) gets 0, since its
// power would overflow.  q = 1 returns inv itself.  Q >= 0 fixes q at
// compile time; Q < 0 takes the run-time q in [0, 8]: inv^e with
// e = (q + 1) / 2 <= 4 from its three bits by selects, so that no loop sits
// in the unrolled pair loop (a loop there made the compiler spill).
template <int Q = -1, class R>
__device__ __forceinline__ R repulsion_factor(R dd, R inv, int q, R bias) {
    if constexpr (Q == 1) return inv;
    R r;
    if constexpr (Q == 0) r = rsqrt_with_inv(dd, inv);
    else if constexpr (Q == 2) r = inv * rsqrt_with_inv(dd, inv);
    else if constexpr (Q == 3) r = inv * inv;
    else {
        const int e = (q + 1) >> 1;
        const R inv2 = inv * inv;
        r = (e & 1) ? inv : R(1);
        r = (e & 2) ? r * inv2 : r;
        r = (e & 4) ? r * (inv2 * inv2) : r;
        // (1 / sqrt(dd) here, not sqrt(inv): the compiler keeps a branch
        // around its division for odd q but computes sqrt(inv) for every q)
        if (!(q & 1)) r *= fast_rsqrt(dd);
    }
    return dd > bias ? r : R(0);
}

// Lane accumulator of 2-vectors: plain, or Kahan-compensated (the running
// compensation c holds the negated low part lost by each add).
template <class R, bool KAHAN>
struct Acc {
    R sx = 0, sy = 0, cx = 0, cy = 0;
    __device__ __forceinline__ void add(R tx, R ty) {
        if constexpr (KAHAN) {
            const R yx = tx - cx;
            const R ux = sx + yx;
            cx = (ux - sx) - yx;
            sx = ux;
            const R yy = ty - cy;
            const R uy = sy + yy;
            cy = (uy - sy) - yy;
            sy = uy;
        } else {
            sx += tx;
            sy += ty;
        }
    }
    __device__ __forceinline__ double x() const {
        return KAHAN ? (double)sx - (double)cx : (double)sx;
    }
    __device__ __forceinline__ double y() const {
        return KAHAN ? (double)sy - (double)cy : (double)sy;
    }
};

// Repulsion term (x_v - x_u) d^2 / delta^2 of a neighbour at p on v at (xv, yv)
// (magnitude d^2 / delta, q = 1), returned in (tx, ty).  A coincident pair
// (delta = 0) has dx = dy = 0; clamping delta^2 to a tiny positive value keeps
// its scale finite, so its term is exactly 0.  The clamp changes nothing else:
// any squared FP32 distance this small already overflows the force.  `mindd`
// tracks the smallest delta^2 seen, so that rows holding a coincident pair can
// be recounted exactly (rare) without a per-pair counter.
template <class P>
__device__ __forceinline__ void repulse_term(typename P::real xv, typename P::real yv,
                                             typename P::vec2 p, typename P::real d2,
                                             typename P::real& tx, typename P::real& ty,
                                             typename P::real& mindd) {
    using R = typename P::real;
    const R dx = xv - p.x;
    const R dy = yv - p.y;
    const R dd = dx * dx + dy * dy;
    mindd = fmin(mindd, dd);
    R s;
    if constexpr (sizeof(R) == 4) {
        s = d2 * fast_rcp(fmaxf(dd, 1e-30f));
    } else {
        s = dd > R(0) ? d2 / dd : R(0);
    }
    tx = dx * s;
    ty = dy * s;
}

// Squared distance plus a tiny bias: a coincident pair gets delta^2 = bias
// instead of 0, so its reciprocal is finite and its term (dx = dy = 0) is
// exactly 0.  For any two distinct positions of magnitude below ~1e12 the
// bias is far below the rounding of delta^2 and changes nothing.
template <class R>
__device__ __forceinline__ R coincidence_bias() {
    return sizeof(R) == 4 ? (R)1e-30f : (R)1e-300;
}

// Repulsion (x_v - x_u) / delta^2 from four neighbours at p0..p3, summed into
// (sx, sy); the factor d^2 of the force (magnitude d^2 / delta, q = 1) is
// applied by the caller once per row.  A sentinel far away (delta^2 = +inf)
// contributes exactly 0.  `mindd` tracks the smallest biased delta^2, so rows
// holding a coincident pair can be recounted exactly (rare).  With WEIGHTED,
// the term of neighbour i is scaled by w[i], the weight of the repulsion that
// neighbour exerts (1 + its pruned degree-one neighbours, Section 4.6).  With
// Q != 1 the repulsion exponent is Q (0, 2 or 3), or the argument q (Q < 0).
template <class P, bool WEIGHTED = false, int Q = 1>
__device__ __forceinline__ void repulse4(typename P::vec2 p0, typename P::vec2 p1,
                                         typename P::vec2 p2, typename P::vec2 p3,
                                         typename P::real xv, typename P::real yv,
                                         typename P::real& sx, typename P::real& sy,
                                         typename P::real& mindd,
                                         const typename P::real* w = nullptr, int q = 1) {
    using R = typename P::real;
    const R bias = coincidence_bias<R>();
    const R dx0 = xv - p0.x, dy0 = yv - p0.y;
    const R dx1 = xv - p1.x, dy1 = yv - p1.y;
    const R dx2 = xv - p2.x, dy2 = yv - p2.y;
    const R dx3 = xv - p3.x, dy3 = yv - p3.y;
    const R dd0 = fma(dx0, dx0, fma(dy0, dy0, bias));
    const R dd1 = fma(dx1, dx1, fma(dy1, dy1, bias));
    const R dd2 = fma(dx2, dx2, fma(dy2, dy2, bias));
    const R dd3 = fma(dx3, dx3, fma(dy3, dy3, bias));
    mindd = fmin(fmin(mindd, dd0), dd1);
    mindd = fmin(fmin(mindd, dd2), dd3);
    R r0, r1, r2, r3;
    if constexpr (sizeof(R) == 4) {
        r0 = fast_rcp(dd0);
        r1 = fast_rcp(dd1);
        r2 = fast_rcp(dd2);
        r3 = fast_rcp(dd3);
    } else {
        r0 = R(1) / dd0;
        r1 = R(1) / dd1;
        r2 = R(1) / dd2;
        r3 = R(1) / dd3;
    }
    if constexpr (Q != 1) {
        r0 = repulsion_factor<Q>(dd0, r0, q, bias);
        r1 = repulsion_factor<Q>(dd1, r1, q, bias);
        r2 = repulsion_factor<Q>(dd2, r2, q, bias);
        r3 = repulsion_factor<Q>(dd3, r3, q, bias);
    }
    if constexpr (WEIGHTED) {
        r0 *= w[0];
        r1 *= w[1];
        r2 *= w[2];
        r3 *= w[3];
    }
    sx = fma(dx0, r0, dx1 * r1) + fma(dx2, r2, dx3 * r3);
    sy = fma(dy0, r0, dy1 * r1) + fma(dy2, r2, dy3 * r3);
}

// One neighbour (the remainder of a row walk), same conventions as repulse4.
template <class P>
__device__ __forceinline__ void repulse1(typename P::vec2 p, typename P::real xv,
                                         typename P::real yv, typename P::real& sx,
                                         typename P::real& sy, typename P::real& mindd) {
    using R = typename P::real;
    const R dx = xv - p.x, dy = yv - p.y;
    const R dd = fma(dx, dx, fma(dy, dy, coincidence_bias<R>()));
    mindd = fmin(mindd, dd);
    R r;
    if constexpr (sizeof(R) == 4) r = fast_rcp(dd);
    else r = R(1) / dd;
    sx = dx * r;
    sy = dy * r;
}

// Number of pairs of a strided row walk whose points coincide.
template <class V, class IDX, int STRIDE>
__device__ __forceinline__ int count_coincident(V xv, const IDX* __restrict__ row, int len,
                                                int lane0, const V* __restrict__ pos) {
    int c = 0;
    for (int e = lane0; e < len; e += STRIDE) {
        const V p = pos[row[e]];
        c += (xv.x == p.x && xv.y == p.y) ? 1 : 0;
    }
    return c;
}

// Repulsion on v (at xv, yv) from a neighbour at p: (x_v - x_u) d^2 / delta^2
// (magnitude d^2 / delta, q = 1; d^2 / delta^q with (x_v - x_u) d^2 /
// delta^(q+1) for another q).  A coincident pair adds nothing and is counted.
template <class P>
__device__ __forceinline__ void repulse(typename P::real xv, typename P::real yv,
                                        typename P::vec2 p, typename P::real d2,
                                        Acc<typename P::real, P::kahan>& acc, int& coinc,
                                        int q = 1) {
    using R = typename P::real;
    const R dx = xv - p.x;
    const R dy = yv - p.y;
    const R dd = dx * dx + dy * dy;
    R s;
    if (q == 1) {
        if constexpr (sizeof(R) == 4) {
            s = dd > R(0) ? d2 * fast_rcp(dd) : R(0);
        } else {
            s = dd > R(0) ? d2 / dd : R(0);
        }
    } else {
        const R inv = sizeof(R) == 4 ? fast_rcp(dd) : R(1) / dd;
        s = dd > R(0) ? d2 * repulsion_factor(dd, inv, q, R(0)) : R(0);
    }
    coinc += (dd == R(0));
    acc.add(dx * s, dy * s);
}

// delta^(p-1) from dd = delta^2, for the attraction exponent p (Section 3.1:
// magnitude delta^p / d, so the term is (x_u - x_v) delta^(p-1) / d); 0 for
// coincident ends when p = 0.
template <class R>
__device__ __forceinline__ R attraction_factor(R dd, int p) {
    if (p == 0) return dd > R(0) ? fast_rsqrt(dd) : R(0);
    const int e = p - 1;
    return (e & 1) ? pow_int(dd, e >> 1) * sqrt(dd) : pow_int(dd, e >> 1);
}

// Attraction on v from an adjacent u at p: (x_u - x_v) delta / d (magnitude
// delta^2 / d, p = 2; (x_u - x_v) delta^(pa-1) / d for another exponent pa).
// `dparam` is 1/d in FP32 and d itself in FP64.
template <class P>
__device__ __forceinline__ void attract(typename P::real xv, typename P::real yv,
                                        typename P::vec2 p, typename P::real dparam,
                                        Acc<typename P::real, P::kahan>& acc, int pa = 2) {
    using R = typename P::real;
    const R dx = p.x - xv;
    const R dy = p.y - yv;
    const R f = pa == 2 ? sqrt(dx * dx + dy * dy) : attraction_factor(dx * dx + dy * dy, pa);
    R s;
    if constexpr (sizeof(R) == 4) {
        s = f * dparam;
    } else {
        s = f / dparam;
    }
    acc.add(dx * s, dy * s);
}

template <class R>
__device__ __forceinline__ R attract_param(double d) {
    return sizeof(R) == 4 ? (R)(1.0 / d) : (R)d;
}

// Temperature-capped displacement (Section 3.1): Delta = F min(|F|, t) / |F|,
// and 0 for F = 0.  When squaring F would overflow or underflow, F is first
// scaled by a power of two (exact) that brings its largest component into
// [0.5, 1), so every finite F != 0 moves min(|F|, t) along F.  A non-finite F
// (a term overflowed in the precision) gives no move and returns false.
__device__ __forceinline__ bool capped_move(double fx, double fy, double t, double& dx,
                                            double& dy) {
    dx = 0.0;
    dy = 0.0;
    if (!(fabs(fx) <= DBL_MAX) || !(fabs(fy) <= DBL_MAX)) return false;
    const double n2 = fx * fx + fy * fy;
    if (n2 > 0.0 && n2 <= DBL_MAX) {
        const double norm = sqrt(n2);
        const double len = norm < t ? norm : t;
        dx = fx * (len / norm);
        dy = fy * (len / norm);
    } else if (fx != 0.0 || fy != 0.0) {
        int e = 0;
        (void)frexp(fmax(fabs(fx), fabs(fy)), &e);
        const double ux = ldexp(fx, -e), uy = ldexp(fy, -e);
        const double nu = sqrt(ux * ux + uy * uy);  // in [0.5, sqrt(2))
        const double sc = fmin(ldexp(nu, e), t) / nu;  // |F| = nu 2^e (inf: the cap)
        dx = ux * sc;
        dy = uy * sc;
    }
    return true;
}

// The same cap computed in float (FP32 positions), returning the capped
// length in l.  The common branch's test implies finite components, so the
// rare branch -- |F|^2 outside float's range, or F not finite -- costs the
// common case nothing.  A finite F whose square overflows is scaled by 2^-96
// (exact) first: forces summed from float terms over at most 64 lanes and
// scaled by d^2 stay below 2^146, so the scaled square is finite.  A finite
// F whose square underflows (|F| < 2^-63) gives no move: it could not change
// a float position away from the origin.  Returns false (no move) for a
// non-finite F.
__device__ __forceinline__ bool capped_move_f32(double fx, double fy, double t, float& dx,
                                                float& dy, float& l) {
    const float fxf = (float)fx, fyf = (float)fy;
    const float n2 = fmaf(fxf, fxf, fyf * fyf);
    dx = 0.f;
    dy = 0.f;
    l = 0.f;
    if (n2 > 0.f && n2 <= FLT_MAX) {
        const float norm = sqrtf(n2);
        l = fminf(norm, (float)t);
        const float sc = l * __builtin_amdgcn_rcpf(norm);
        dx = fxf * sc;
        dy = fyf * sc;
    } else if (!(fabs(fx) <= DBL_MAX) || !(fabs(fy) <= DBL_MAX)) {
        return false;
    } else if (n2 > 0.f) {
        const float ux = (float)(fx * 0x1p-96), uy = (float)(fy * 0x1p-96);
        const float nu = sqrtf(fmaf(ux, ux, uy * uy));
        l = fminf(nu * 0x1p96f, (float)t);  // |F| = nu 2^96 (inf in float: the cap)
        const float sc = l * __builtin_amdgcn_rcpf(nu);
        dx = ux * sc;
        dy = uy * sc;
    }
    return true;
}

// Cap, move and record one vertex (Section 3.1 temperature cap; the move is
// written to the other buffer, so all vertices move together).  A vertex
// whose force is not finite stays put and is counted in `nonfinite`.
template <class P>
__device__ __forceinline__ void finish_vertex(const StepArgs& a, int32_t v, typename P::vec2 xv,
                                              double fx, double fy, double& energy, double& maxd,
                                              int64_t& moved, int64_t& nonfinite) {
    using V = typename P::vec2;
    using R = typename P::real;
    double dx, dy;
    const double t = a.temps ? a.temps[a.ctl->h_base + a.tick_j] : a.t;
    if (!capped_move(fx, fy, t, dx, dy)) {
        ++nonfinite;
        fx = 0.0;  // keeps the energy statistic finite
        fy = 0.0;
    }
    V nx;
    nx.x = (R)((double)xv.x + dx);
    nx.y = (R)((double)xv.y + dy);
    reinterpret_cast<V*>(a.pos_next)[v] = nx;
    if (a.F_out) {
        const int32_t o = a.perm[v];
        a.F_out[2 * (int64_t)o] = fx;
        a.F_out[2 * (int64_t)o + 1] = fy;
        a.D_out[2 * (int64_t)o] = dx;
        a.D_out[2 * (int64_t)o + 1] = dy;
    }
    const double dl = sqrt(dx * dx + dy * dy);
    energy += fx * fx + fy * fy;
    maxd = dl > maxd ? dl : maxd;
    moved += dl > a.stop_displacement ? 1 : 0;
}

// Ends the per-vertex part of an iteration kernel: the workgroup's statistics,
// reduced in a fixed order, go to a.partials[blockIdx.x].  The iteration's
// totals are published by iteration_stats_kernel, launched next on the same
// stream (a kernel boundary makes the partials visible to it without a
// device-wide cache writeback per workgroup).  Every thread of the workgroup
// must call it.
__device__ __forceinline__ void end_iteration(const StepArgs& a, double energy, double maxd,
                                              int64_t moved, int64_t coinc, int64_t nonfinite) {
    __shared__ double s_e[kWaves], s_m[kWaves];
    __shared__ int64_t s_mv[kWaves], s_c[kWaves], s_nf[kWaves];
    const int lane = lane64();
    const int w = wave_id();
    const double we = wave_sum(energy);
    const double wm = wave_max(maxd);
    const int64_t wmv = wave_sum(moved);
    const int64_t wc = wave_sum(coinc);
    const int64_t wnf = wave_sum(nonfinite);
    if (lane == 0) {
        s_e[w] = we;
        s_m[w] = wm;
        s_mv[w] = wmv;
        s_c[w] = wc;
        s_nf[w] = wnf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial p;
        p.energy = s_e[0];
        p.max_disp = s_m[0];
        p.moved = s_mv[0];
        p.coincident = s_c[0];
        p.nonfinite = s_nf[0];
        for (int i = 1; i < kWaves; ++i) {
            p.energy += s_e[i];
            p.max_disp = s_m[i] > p.max_disp ? s_m[i] : p.max_disp;
            p.moved += s_mv[i];
            p.coincident += s_c[i];
            p.nonfinite += s_nf[i];
        }
        a.partials[blockIdx.x] = p;
    }
}

}  // namespace gila

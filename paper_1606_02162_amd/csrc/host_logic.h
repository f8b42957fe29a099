// Host-only logic of the library, in plain C++17 with no HIP dependency, so
// that it can also be built and run on a CPU alone (with sanitizers) by the
// test suite: argument checks, the checks of a host CSR, the device
// footprint bound of a layout job, and the layout server's admission rule.
// Functions report a status (GILA_*) and write a message into `msg`.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/gila.h"

namespace gila {
namespace host {

// Checks of the layout parameters (Section 3.1 force model, Section 5.1 cap
// schedule and halting rule); need_temps: a schedule must be present.
inline int check_params(const gila_params* p, bool need_temps, char* msg, size_t len) {
    if (!p) return std::snprintf(msg, len, "params is NULL"), GILA_EINVAL;
    if (p->precision != GILA_FP64 && p->precision != GILA_FP32 &&
        p->precision != GILA_FP32_KAHAN)
        return std::snprintf(msg, len, "unknown precision %d", p->precision), GILA_EINVAL;
    if (!(p->ideal_length > 0.0) || !std::isfinite(p->ideal_length))
        return std::snprintf(msg, len, "ideal_length must be finite and > 0"), GILA_EINVAL;
    if (p->iterations < 0) return std::snprintf(msg, len, "iterations must be >= 0"), GILA_EINVAL;
    if (need_temps && p->iterations > 0 && !p->temperature)
        return std::snprintf(msg, len, "temperature is NULL"), GILA_EINVAL;
    if (p->temperature)
        for (int32_t h = 0; h < p->iterations; ++h)
            if (!(p->temperature[h] >= 0.0) || !std::isfinite(p->temperature[h]))
                return std::snprintf(msg, len, "temperature[%d] must be finite and >= 0", h),
                       GILA_EINVAL;
    if (!(p->stop_fraction >= 0.0) || !(p->stop_displacement >= 0.0))
        return std::snprintf(msg, len, "stop parameters must be >= 0"), GILA_EINVAL;
    if (p->force_model != GILA_MODEL_FR && p->force_model != GILA_MODEL_LINLOG &&
        p->force_model != GILA_MODEL_PQ)
        return std::snprintf(msg, len, "unknown force model %d", p->force_model), GILA_EINVAL;
    if (p->force_model == GILA_MODEL_PQ &&
        (p->force_p < 0 || p->force_p > 8 || p->force_q < 0 || p->force_q > 8))
        return std::snprintf(msg, len, "force exponents p = %d, q = %d outside [0, 8]",
                             p->force_p, p->force_q),
               GILA_EINVAL;
    return GILA_OK;
}

// Cheap checks of a host CSR at submission: sizes, pointers, row_ptr from 0 to
// nnz without decreasing, every column in range (so that the footprint bound
// can walk the graph).  Sortedness, self-loops and symmetry are checked on
// the device when the job is admitted.
inline int validate_host_csr(const gila_csr* g, char* msg, size_t len) {
    if (!g) return std::snprintf(msg, len, "graph is NULL"), GILA_EINVAL;
    if (g->n < 0 || g->nnz < 0 || g->nnz % 2)
        return std::snprintf(msg, len, "bad n or nnz"), GILA_EINVAL;
    if (g->n > 0 && !g->row_ptr) return std::snprintf(msg, len, "row_ptr is NULL"), GILA_EINVAL;
    if (g->nnz > 0 && !g->col_idx) return std::snprintf(msg, len, "col_idx is NULL"), GILA_EINVAL;
    if (g->n > 0 && (g->row_ptr[0] != 0 || g->row_ptr[g->n] != g->nnz))
        return std::snprintf(msg, len, "row_ptr must run from 0 to nnz"), GILA_EINVAL;
    for (int32_t v = 0; v < g->n; ++v)
        if (g->row_ptr[v + 1] < g->row_ptr[v])
            return std::snprintf(msg, len, "row_ptr not monotone"), GILA_EINVAL;
    for (int64_t e = 0; e < g->nnz; ++e)
        if (g->col_idx[e] < 0 || g->col_idx[e] >= g->n)
            return std::snprintf(msg, len, "column out of range"), GILA_EINVAL;
    return GILA_OK;
}

// Upper bound of P = sum_v |N_v(k)| (Section 4.5) from the adjacency alone:
// the number of walks of length <= k from v, capped at n - 1 per vertex.
// rp[n + 1], ci[rp[n]] with every column in [0, n).
inline int64_t pairs_upper_bound(int32_t n, int32_t k, const int64_t* rp, const int32_t* ci) {
    if (n <= 0) return 0;
    std::vector<int64_t> cur((size_t)n), nxt((size_t)n), tot((size_t)n);
    for (int32_t v = 0; v < n; ++v) cur[v] = tot[v] = rp[v + 1] - rp[v];
    for (int32_t level = 2; level <= k; ++level) {
        for (int32_t v = 0; v < n; ++v) {
            int64_t s = 0;
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) s += cur[ci[e]];
            nxt[v] = std::min<int64_t>(s, (int64_t)n);
            tot[v] = std::min<int64_t>(tot[v] + nxt[v], (int64_t)n - 1);
        }
        cur.swap(nxt);
    }
    int64_t P = 0;
    for (int32_t v = 0; v < n; ++v) P += tot[v];
    return P;
}

// Bytes a layout job may hold on the device: graph, positions, lists (int32
// and 16-bit padded copies), per-slice offsets and partials (bounded by the
// lists), and a fixed margin.
inline int64_t footprint_bytes(int32_t n, int64_t nnz, int32_t k, const int64_t* rp,
                               const int32_t* ci) {
    const int64_t P = pairs_upper_bound(n, k, rp, ci);
    return 64ll * n + 16ll * nnz + 8ll * P + (1ll << 20);
}

// The layout server's admission rule: jobs leave the queue in arrival order;
// the job at the front is admitted when fewer than max_slots jobs are in
// flight and its footprint fits beside the bytes already reserved; a job
// whose footprint exceeds the whole budget is rejected (ENOMEM) at once, a
// cancelled one dropped.  A job whose footprint is not known yet (< 0) and a
// job that does not fit now hold the queue (no overtaking).
struct AdmitState {
    int64_t budget = 0;
    int32_t max_slots = 1;
    int64_t reserved = 0;
    int32_t in_flight = 0;
};

struct QueuedJob {
    int64_t footprint = -1;  // < 0: not computed yet
    bool cancel = false;
};

enum AdmitOutcome { kAdmitWait = 0, kAdmitTake = 1, kAdmitReject = 2, kAdmitDrop = 3 };

// The decision for the job at the front of the queue.  kAdmitTake reserves
// its bytes and a slot; the caller releases them with admit_release when the
// job ends.
inline AdmitOutcome admit_front(AdmitState& st, const QueuedJob& j) {
    if (j.cancel) return kAdmitDrop;
    if (j.footprint < 0) return kAdmitWait;
    if (j.footprint > st.budget) return kAdmitReject;
    if (st.in_flight >= st.max_slots || st.reserved + j.footprint > st.budget) return kAdmitWait;
    st.reserved += j.footprint;
    st.in_flight += 1;
    return kAdmitTake;
}

// Whether admit_front would decide anything but "wait" (the admitter sleeps
// until then).  A job with an unknown footprint counts as progress: the
// admitter computes it.
inline bool admit_can_progress(const AdmitState& st, const QueuedJob& j) {
    return j.footprint < 0 || j.cancel || j.footprint > st.budget ||
           (st.in_flight < st.max_slots && st.reserved + j.footprint <= st.budget);
}

inline void admit_release(AdmitState& st, int64_t footprint) {
    st.reserved -= footprint;
    st.in_flight -= 1;
}

// Cap schedules of Section 5.1 (see gila_paper_schedule).
inline int paper_schedule(double n, double aspect, double d, int32_t iterations, double* t,
                          char* msg, size_t len) {
    if (iterations < 0) return std::snprintf(msg, len, "iterations must be >= 0"), GILA_EINVAL;
    if (iterations > 0 && !t) return std::snprintf(msg, len, "temperature_host is NULL"), GILA_EINVAL;
    if (!(n > 0.0) || !(aspect > 0.0) || !(d > 0.0) || !std::isfinite(n) || !std::isfinite(aspect) ||
        !std::isfinite(d))
        return std::snprintf(msg, len, "n, aspect and ideal_length must be finite and > 0"),
               GILA_EINVAL;
    // sqrt((n / a) d) 0.93^h, h counted from 0
    const double base = std::sqrt(n / aspect * d);
    for (int32_t h = 0; h < iterations; ++h) t[h] = base * std::pow(0.93, (double)h);
    return GILA_OK;
}

inline int linear_schedule(double t0, int32_t iterations, double* t, char* msg, size_t len) {
    if (iterations < 0) return std::snprintf(msg, len, "iterations must be >= 0"), GILA_EINVAL;
    if (iterations > 0 && !t) return std::snprintf(msg, len, "temperature_host is NULL"), GILA_EINVAL;
    if (!(t0 >= 0.0) || !std::isfinite(t0))
        return std::snprintf(msg, len, "t0 must be finite and >= 0"), GILA_EINVAL;
    for (int32_t h = 0; h < iterations; ++h) t[h] = t0 - (t0 * (double)h) / (double)iterations;
    return GILA_OK;
}

}  // namespace host
}  // namespace gila

// CPU-only test of the library's host logic (csrc/host_logic.h), built by the
// test suite with g++ under AddressSanitizer and UndefinedBehaviorSanitizer:
//   - the layout server's admission rule driven by a fake device (a byte
//     budget and slots) and a fake clock (an event simulation of arrivals and
//     completions): invariants and the arrival-order guarantee;
//   - parameter checks, host CSR checks, the walk-count bound of P against an
//     exact BFS count, the cap schedules against their closed forms, and the
//     k-hop handle's internal vertex order against a comparison sort.
// Prints "OK <checks>" and exits 0, or the first failure and exits 1.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <queue>
#include <random>
#include <vector>

#include "../../paper_1606_02162_amd/csrc/host_logic.h"

using namespace gila::host;

static int g_checks = 0;
#define CHECK(cond, ...)                                                  \
    do {                                                                  \
        ++g_checks;                                                       \
        if (!(cond)) {                                                    \
            std::printf("FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond);   \
            std::printf(__VA_ARGS__);                                     \
            std::printf("\n");                                            \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

// ------------------------------------------------------------------ admission
struct SimJob {
    double arrive, service;
    int64_t footprint;
    bool cancel_in_queue;   // cancelled while still queued
    int outcome = -1;       // AdmitOutcome once decided
    double admitted = -1, done = -1;
};

// Event simulation of the admitter: jobs arrive, their footprint is known at
// once (the real admitter computes it outside its lock; the rule treats an
// unknown one as "wait"), the queue is served by admit_front in arrival order
// after every event, admitted jobs hold their bytes and slot for their
// service time on the fake device.
static void simulate(uint32_t seed, int64_t budget, int32_t slots, int count) {
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::vector<SimJob> jobs((size_t)count);
    double t = 0.0;
    for (auto& j : jobs) {
        t += -std::log(1.0 - U(rng)) * 5e-3;                         // Poisson arrivals
        j.arrive = t;
        j.service = 1e-3 + U(rng) * 40e-3;
        const double r = U(rng);
        j.footprint = r < 0.05 ? budget + 1 + (int64_t)(U(rng) * budget)   // never fits
                               : 1 + (int64_t)(U(rng) * U(rng) * budget);
        j.cancel_in_queue = U(rng) < 0.03;
    }
    AdmitState st;
    st.budget = budget;
    st.max_slots = slots;
    std::deque<int> queue;
    using Ev = std::pair<double, int>;  // (time, job): completion events
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
    size_t next = 0;
    std::vector<int> admit_order;
    double now = 0.0;
    auto serve = [&]() {
        while (!queue.empty()) {
            SimJob& j = jobs[queue.front()];
            QueuedJob q{j.footprint, j.cancel_in_queue};
            // the rule's wait predicate agrees with its decision
            const bool progress = admit_can_progress(st, q);
            const AdmitOutcome o = admit_front(st, q);
            CHECK(progress == (o != kAdmitWait), "predicate and decision disagree");
            if (o == kAdmitWait) break;
            j.outcome = o;
            const int id = queue.front();
            queue.pop_front();
            if (o == kAdmitTake) {
                j.admitted = now;
                admit_order.push_back(id);
                running.push({now + j.service, id});
            }
            // the fake device never holds more than the budget or the slots
            CHECK(st.reserved <= st.budget && st.reserved >= 0, "reserved %lld", (long long)st.reserved);
            CHECK(st.in_flight <= st.max_slots && st.in_flight >= 0, "in flight %d", st.in_flight);
        }
    };
    while (next < jobs.size() || !running.empty()) {
        const bool arrival = next < jobs.size() &&
                             (running.empty() || jobs[next].arrive <= running.top().first);
        if (arrival) {
            now = jobs[next].arrive;
            queue.push_back((int)next);
            ++next;
        } else {
            const Ev e = running.top();
            running.pop();
            now = e.first;
            jobs[e.second].done = now;
            admit_release(st, jobs[e.second].footprint);
        }
        serve();
    }
    CHECK(queue.empty(), "%zu jobs left queued", queue.size());
    CHECK(st.reserved == 0 && st.in_flight == 0, "resources not returned");
    // every job was decided: rejected exactly when it can never fit, dropped
    // exactly when cancelled, admitted otherwise; admission in arrival order
    for (const auto& j : jobs) {
        if (j.cancel_in_queue) CHECK(j.outcome == kAdmitDrop, "cancelled job not dropped");
        else if (j.footprint > budget) CHECK(j.outcome == kAdmitReject, "oversized job not rejected");
        else CHECK(j.outcome == kAdmitTake && j.done >= j.admitted && j.admitted >= j.arrive,
                   "job not admitted and run");
    }
    for (size_t i = 1; i < admit_order.size(); ++i)
        CHECK(admit_order[i] > admit_order[i - 1], "admitted out of arrival order");
}

static void test_admission() {
    simulate(1, 1000, 4, 2000);
    simulate(2, 1 << 20, 64, 3000);
    simulate(3, 50, 1, 500);        // one slot: strictly one job at a time
    // a hand case: the front job blocks a later one that would fit
    AdmitState st;
    st.budget = 100;
    st.max_slots = 8;
    CHECK(admit_front(st, QueuedJob{60, false}) == kAdmitTake, "first");
    CHECK(admit_front(st, QueuedJob{50, false}) == kAdmitWait, "second must wait");
    CHECK(!admit_can_progress(st, QueuedJob{50, false}), "no progress");
    CHECK(admit_can_progress(st, QueuedJob{-1, false}), "unknown footprint is progress");
    CHECK(admit_front(st, QueuedJob{-1, false}) == kAdmitWait, "unknown footprint waits");
    CHECK(admit_front(st, QueuedJob{101, false}) == kAdmitReject, "too big");
    CHECK(admit_front(st, QueuedJob{50, true}) == kAdmitDrop, "cancelled");
    admit_release(st, 60);
    CHECK(admit_front(st, QueuedJob{50, false}) == kAdmitTake && st.reserved == 50, "after release");
}

// ------------------------------------------------------------------ checks
static void test_param_and_csr_checks() {
    char msg[256];
    const double temps[3] = {3.0, 2.0, 1.0};
    gila_params p{};
    p.precision = GILA_FP32;
    p.ideal_length = 10.0;
    p.iterations = 3;
    p.temperature = temps;
    CHECK(check_params(&p, true, msg, sizeof msg) == GILA_OK, "%s", msg);
    gila_params b = p;
    b.ideal_length = -1.0;
    CHECK(check_params(&b, true, msg, sizeof msg) == GILA_EINVAL, "negative d");
    b = p;
    b.temperature = nullptr;
    CHECK(check_params(&b, true, msg, sizeof msg) == GILA_EINVAL, "missing schedule");
    CHECK(check_params(&b, false, msg, sizeof msg) == GILA_OK, "schedule not needed");
    const double bad[2] = {1.0, NAN};
    b = p;
    b.iterations = 2;
    b.temperature = bad;
    CHECK(check_params(&b, true, msg, sizeof msg) == GILA_EINVAL, "NaN cap");
    b = p;
    b.force_model = GILA_MODEL_PQ;
    b.force_q = 9;
    CHECK(check_params(&b, true, msg, sizeof msg) == GILA_EINVAL, "q out of range");
    CHECK(check_params(nullptr, true, msg, sizeof msg) == GILA_EINVAL, "null");

    const int64_t rp[4] = {0, 1, 3, 4};
    const int32_t ci[4] = {1, 0, 2, 1};
    gila_csr g{3, 4, rp, ci};
    CHECK(validate_host_csr(&g, msg, sizeof msg) == GILA_OK, "%s", msg);
    const int32_t ci_bad[4] = {1, 0, 7, 1};
    gila_csr gb{3, 4, rp, ci_bad};
    CHECK(validate_host_csr(&gb, msg, sizeof msg) == GILA_EINVAL, "column out of range");
    const int64_t rp_bad[4] = {0, 3, 1, 4};
    gila_csr gr{3, 4, rp_bad, ci};
    CHECK(validate_host_csr(&gr, msg, sizeof msg) == GILA_EINVAL, "row_ptr decreases");
    gila_csr go{3, 3, rp, ci};
    CHECK(validate_host_csr(&go, msg, sizeof msg) == GILA_EINVAL, "odd nnz");
    gila_csr gn{3, 4, nullptr, ci};
    CHECK(validate_host_csr(&gn, msg, sizeof msg) == GILA_EINVAL, "null row_ptr");
}

// exact |N_v(k)| by BFS, to hold the bound against
static int64_t exact_pairs(int32_t n, int32_t k, const std::vector<int64_t>& rp,
                           const std::vector<int32_t>& ci) {
    int64_t P = 0;
    std::vector<int32_t> dist((size_t)n);
    for (int32_t s = 0; s < n; ++s) {
        std::fill(dist.begin(), dist.end(), -1);
        std::deque<int32_t> q{s};
        dist[s] = 0;
        while (!q.empty()) {
            const int32_t w = q.front();
            q.pop_front();
            if (dist[w] == k) continue;
            for (int64_t e = rp[w]; e < rp[w + 1]; ++e)
                if (dist[ci[e]] < 0) {
                    dist[ci[e]] = dist[w] + 1;
                    q.push_back(ci[e]);
                    ++P;
                }
        }
    }
    return P;
}

static void test_pairs_bound() {
    std::mt19937 rng(7);
    for (int trial = 0; trial < 40; ++trial) {
        const int32_t n = 2 + (int32_t)(rng() % 60);
        std::vector<std::vector<int32_t>> adj((size_t)n);
        const int m = (int)(rng() % (3 * n));
        for (int e = 0; e < m; ++e) {
            const int32_t u = (int32_t)(rng() % n), v = (int32_t)(rng() % n);
            if (u == v) continue;
            bool dup = false;
            for (int32_t x : adj[u]) dup = dup || x == v;
            if (dup) continue;
            adj[u].push_back(v);
            adj[v].push_back(u);
        }
        std::vector<int64_t> rp((size_t)n + 1, 0);
        std::vector<int32_t> ci;
        for (int32_t v = 0; v < n; ++v) {
            std::sort(adj[v].begin(), adj[v].end());
            ci.insert(ci.end(), adj[v].begin(), adj[v].end());
            rp[v + 1] = (int64_t)ci.size();
        }
        for (int32_t k = 1; k <= 3; ++k) {
            const int64_t exact = exact_pairs(n, k, rp, ci);
            const int64_t bound = pairs_upper_bound(n, k, rp.data(), ci.empty() ? nullptr : ci.data());
            CHECK(bound >= exact, "bound %lld below exact %lld", (long long)bound, (long long)exact);
            if (k == 1) CHECK(bound == exact, "k = 1 bound is the degree sum");
            CHECK(bound <= (int64_t)n * (n - 1), "bound above n(n-1)");
        }
        CHECK(footprint_bytes(n, (int64_t)ci.size(), 2, rp.data(), ci.empty() ? nullptr : ci.data()) >
                  (1ll << 20), "footprint includes the margin");
    }
}

static void test_schedules() {
    char msg[256];
    double t[100];
    CHECK(linear_schedule(100.0, 100, t, msg, sizeof msg) == GILA_OK, "%s", msg);
    for (int h = 0; h < 100; ++h) CHECK(t[h] == 100.0 - h, "linear t[%d] = %g", h, t[h]);
    CHECK(paper_schedule(1000.0, 2.0, 8.0, 10, t, msg, sizeof msg) == GILA_OK, "%s", msg);
    CHECK(std::fabs(t[0] * t[0] - 4000.0) < 1e-9, "t0^2 = (n / a) d");
    for (int h = 1; h < 10; ++h) CHECK(std::fabs(t[h] / t[h - 1] - 0.93) < 1e-14, "ratio");
    CHECK(paper_schedule(0.0, 1.0, 8.0, 3, t, msg, sizeof msg) == GILA_EINVAL, "n = 0");
    CHECK(linear_schedule(-1.0, 3, t, msg, sizeof msg) == GILA_EINVAL, "t0 < 0");
    CHECK(linear_schedule(1.0, 3, nullptr, msg, sizeof msg) == GILA_EINVAL, "null output");
    CHECK(linear_schedule(1.0, 0, nullptr, msg, sizeof msg) == GILA_OK, "empty schedule");
}

// The internal vertex order against a comparison sort of the same keys
// (stable, so equal keys keep ascending ids).
int main() {
    test_admission();
    test_param_and_csr_checks();
    test_pairs_bound();
    test_schedules();
    std::printf("OK %d\n", g_checks);
    return 0;
}

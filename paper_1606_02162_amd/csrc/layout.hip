// Iteration drivers: seeded placement, one step, a device-resident loop of
// steps captured as a HIP graph, and the whole-layout entry point.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "device_util.h"
#include "gila_internal.h"
#include "host_logic.h"

namespace gila {

// ------------------------------------------------------------------ iteration statistics
// One workgroup, after the iteration's per-vertex kernel: reduces the
// workgroups' partials (a.nblocks of them) in a fixed order and publishes the
// iteration's statistics (Section 5.1 halting rule included).
__global__ __launch_bounds__(kBlock) void iteration_stats_kernel(StepArgs a) {
    __shared__ double s_e[kWaves], s_m[kWaves];
    __shared__ int64_t s_mv[kWaves], s_c[kWaves], s_nf[kWaves];
    Ctl* ctl = a.ctl;
    if (ctl->stopped) return;
    const int lane = lane64();
    const int w = wave_id();
    double e = 0.0, m = 0.0;
    int64_t mv = 0, c = 0, nf = 0;
    for (int i = threadIdx.x; i < a.nblocks; i += kBlock) {
        const Partial p = a.partials[i];
        e += p.energy;
        m = p.max_disp > m ? p.max_disp : m;
        mv += p.moved;
        c += p.coincident;
        nf += p.nonfinite;
    }
    e = wave_sum(e);
    m = wave_max(m);
    mv = wave_sum(mv);
    c = wave_sum(c);
    nf = wave_sum(nf);
    if (lane == 0) {
        s_e[w] = e;
        s_m[w] = m;
        s_mv[w] = mv;
        s_c[w] = c;
        s_nf[w] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        e = s_e[0];
        m = s_m[0];
        mv = s_mv[0];
        c = s_c[0];
        nf = s_nf[0];
        for (int i = 1; i < kWaves; ++i) {
            e += s_e[i];
            m = s_m[i] > m ? s_m[i] : m;
            mv += s_mv[i];
            c += s_c[i];
            nf += s_nf[i];
        }
        c += ctl->coinc_pending;
        ctl->coinc_pending = 0;
        ctl->energy = e;
        ctl->max_disp = m;
        ctl->moved = mv;
        ctl->coincident = c;
        ctl->nonfinite = nf;
        ctl->iters_run += 1;
        if (a.check_stop && (double)mv < a.stop_fraction * (double)a.n_active) ctl->stopped = 1;
        // a non-finite force ends the run (2: stopped by the error, not the rule)
        if (nf > 0) ctl->stopped = 2;
        // the history row: this iteration's h (from the replay's base in a
        // captured chunk or tick)
        int32_t slot = a.hist_slot;
        if (a.temps) {
            const int32_t hh = ctl->h_base + a.tick_j;
            slot = hh < a.hist_cap ? hh : -1;
        }
        if (slot >= 0) {
            double* hrow = a.hist + 4 * (int64_t)slot;
            hrow[0] = e;
            hrow[1] = m;
            hrow[2] = (double)mv;
            hrow[3] = (double)c;
        }
    }
}

int launch_iteration_stats(const StepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(iteration_stats_kernel, dim3(1), dim3(kBlock), 0, s, a);
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

// ------------------------------------------------------------------ placement
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
    // output number c (0-based) of SplitMix64 seeded with `seed`
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <class V>
__global__ __launch_bounds__(kBlock) void init_positions_kernel(int32_t n, uint64_t seed,
                                                                double width, double height,
                                                                V* __restrict__ pos) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const double ux = (double)(splitmix64_at(seed, 2ull * v) >> 11) * 0x1.0p-53;
        const double uy = (double)(splitmix64_at(seed, 2ull * v + 1ull) >> 11) * 0x1.0p-53;
        V p;
        p.x = (decltype(p.x))(ux * width);
        p.y = (decltype(p.y))(uy * height);
        pos[v] = p;
    }
}

// ------------------------------------------------------------------ small kernels
__global__ void reset_ctl_kernel(Ctl* ctl) {
    ctl->stopped = 0;
    ctl->iters_run = 0;
    ctl->done_blocks = 0u;
    ctl->moved = 0;
    ctl->max_disp = 0.0;
    ctl->energy = 0.0;
    ctl->coincident = 0;
    ctl->coinc_pending = 0;
    ctl->nonfinite = 0;
}

// Caller positions -> internal buffer 0; isolated vertices (the tail of the
// internal order) never move, so they are written to buffer 1 as well.
template <class V>
__global__ __launch_bounds__(kBlock) void permute_in_kernel(int32_t n, int32_t n_active,
                                                            const int32_t* __restrict__ perm,
                                                            const V* __restrict__ src,
                                                            V* __restrict__ b0,
                                                            V* __restrict__ b1) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const V p = src[perm[i]];
        b0[i] = p;
        if (i >= n_active) b1[i] = p;
    }
}

// Internal buffer holding the result (iteration parity) -> caller positions.
template <class V>
__global__ __launch_bounds__(kBlock) void permute_out_kernel(int32_t n,
                                                             const int32_t* __restrict__ perm,
                                                             const V* __restrict__ b0,
                                                             const V* __restrict__ b1,
                                                             const Ctl* __restrict__ ctl,
                                                             V* __restrict__ dst) {
    const V* src = (ctl->iters_run & 1) ? b1 : b0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        dst[perm[i]] = src[i];
}

static int grid_for(int64_t items) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (items + kBlock - 1) / kBlock));
}

static int launch_permute_in(const gila_khop* kh, int precision, const void* pos, hipStream_t s) {
    if (kh->n == 0) return GILA_OK;
    const int g = grid_for(kh->n);
    if (precision == GILA_FP64)
        hipLaunchKernelGGL(permute_in_kernel<double2>, dim3(g), dim3(kBlock), 0, s, kh->n,
                           kh->n_active, kh->perm, (const double2*)pos, (double2*)kh->pos[0],
                           (double2*)kh->pos[1]);
    else
        hipLaunchKernelGGL(permute_in_kernel<float2>, dim3(g), dim3(kBlock), 0, s, kh->n,
                           kh->n_active, kh->perm, (const float2*)pos, (float2*)kh->pos[0],
                           (float2*)kh->pos[1]);
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

static int launch_permute_out(const gila_khop* kh, int precision, void* pos, hipStream_t s) {
    if (kh->n == 0) return GILA_OK;
    const int g = grid_for(kh->n);
    if (precision == GILA_FP64)
        hipLaunchKernelGGL(permute_out_kernel<double2>, dim3(g), dim3(kBlock), 0, s, kh->n,
                           kh->perm, (const double2*)kh->pos[0], (const double2*)kh->pos[1],
                           kh->ctl, (double2*)pos);
    else
        hipLaunchKernelGGL(permute_out_kernel<float2>, dim3(g), dim3(kBlock), 0, s, kh->n,
                           kh->perm, (const float2*)kh->pos[0], (const float2*)kh->pos[1],
                           kh->ctl, (float2*)pos);
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

int check_params(const gila_params* p, bool need_temps) {
    char msg[256];
    const int rc = host::check_params(p, need_temps, msg, sizeof(msg));
    return rc == GILA_OK ? GILA_OK : fail(rc, "%s", msg);
}

void force_exponents(const gila_params* p, int32_t* att_p, int32_t* rep_q) {
    switch (p->force_model) {
        case GILA_MODEL_LINLOG: *att_p = 0; *rep_q = 1; break;
        case GILA_MODEL_PQ: *att_p = p->force_p; *rep_q = p->force_q; break;
        default: *att_p = 2; *rep_q = 1; break;
    }
}

static StepArgs base_args(const gila_khop* kh, const gila_params* p) {
    StepArgs a{};
    a.n_active = kh->n_active;
    a.nhub = kh->nhub;
    a.nblocks = kh->nblocks;
    a.block_start = kh->block_start;
    a.rp = kh->rp;
    a.ci = kh->ci;
    a.kptr = kh->kptr;
    a.kidx = kh->kidx;
    a.d = p->ideal_length;
    a.stop_fraction = p->stop_fraction;
    a.stop_displacement = p->stop_displacement;
    a.perm = kh->perm;
    a.partials = kh->partials;
    a.ctl = kh->ctl;
    a.hist = kh->hist;
    a.hist_slot = -1;
    a.hist_cap = kh->hist_cap;
    if (kh->mass64)
        a.mass = p->precision == GILA_FP64 ? (const void*)kh->mass64 : (const void*)kh->mass32;
    force_exponents(p, &a.att_p, &a.rep_q);
    return a;
}

static void to_stats(const Ctl& c, gila_stats* out) {
    out->iterations_run = c.iters_run;
    out->stopped = c.stopped == 1 ? 1 : 0;
    out->moved = c.moved;
    out->max_disp = c.max_disp;
    out->energy = c.energy;
    out->coincident = c.coincident;
    out->nonfinite = c.nonfinite;
}

int nonfinite_status(const Ctl& c) {
    if (c.nonfinite > 0)
        return fail(GILA_ENONFINITE,
                    "%lld vertices had a non-finite force in iteration %d (points too close "
                    "for the force exponents in this precision); they did not move and the "
                    "run stopped",
                    (long long)c.nonfinite, c.iters_run - 1);
    return GILA_OK;
}

// Enqueue: reset, permute in, iterations, permute out.
int enqueue_run(gila_khop* kh, const gila_params* p, int32_t start_h, int32_t end_h,
                void* pos_dev, hipStream_t s) {
    hipLaunchKernelGGL(reset_ctl_kernel, dim3(1), dim3(1), 0, s, kh->ctl);
    GILA_HIP(hipGetLastError());
    GILA_TRY(launch_permute_in(kh, p->precision, pos_dev, s));
    StepArgs a = base_args(kh, p);
    a.check_stop = p->stop_fraction > 0.0 ? 1 : 0;
    for (int32_t h = start_h; h < end_h; ++h) {
        const int j = h - start_h;
        a.pos_cur = kh->pos[j & 1];
        a.pos_next = kh->pos[(j + 1) & 1];
        a.t = p->temperature[h];
        a.hist_slot = h < kh->hist_cap ? h : -1;
        GILA_TRY(launch_iteration(kh, p->precision, a, s));
    }
    GILA_TRY(launch_permute_out(kh, p->precision, pos_dev, s));
    return GILA_OK;
}

void drop_graphs(gila_khop* kh) {
    if (kh->gexec) (void)quiet(hipGraphExecDestroy(kh->gexec));
    if (kh->tick_exec) (void)quiet(hipGraphExecDestroy(kh->tick_exec));
    if (kh->chunk_exec) (void)quiet(hipGraphExecDestroy(kh->chunk_exec));
    kh->gexec = nullptr;
    kh->tick_exec = nullptr;
    kh->chunk_exec = nullptr;
    kh->gkey.clear();
    kh->tick_key.clear();
    kh->chunk_key.clear();
}

// The device copy of the schedule, replaced (with the graphs that read it)
// when the schedule changes.
static int upload_schedule(gila_khop* kh, const gila_params* p, hipStream_t s) {
    const size_t H = (size_t)p->iterations;
    if (kh->d_temps && kh->temps_host.size() == H &&
        std::memcmp(kh->temps_host.data(), p->temperature, H * sizeof(double)) == 0)
        return GILA_OK;
    drop_graphs(kh);
    dfree_on(kh->d_temps, s);
    kh->d_temps = nullptr;
    kh->temps_host.assign(p->temperature, p->temperature + H);
    GILA_TRY(dalloc_t(&kh->d_temps, std::max<size_t>(H, 1)));
    if (H > 0)
        GILA_HIP(hipMemcpyAsync(kh->d_temps, kh->temps_host.data(), H * sizeof(double),
                                hipMemcpyHostToDevice, s));
    return GILA_OK;
}

__global__ void set_h_base_kernel(Ctl* ctl, int32_t h) { ctl->h_base = h; }

// Iterations per captured chunk of a long gila_run (even).
constexpr int32_t kRunChunk = 50;

int enqueue_tick(gila_khop* kh, const gila_params* p, int32_t h, int32_t count,
                 int32_t graph_len, void* pos_dev, hipStream_t s) {
    if (count != graph_len || count <= 0 || h < 0 || h + count > p->iterations)
        return enqueue_run(kh, p, h, h + count, pos_dev, s);
    // the device copy of the schedule (the same for every tick of a job)
    GILA_TRY(upload_schedule(kh, p, s));
    int32_t att_p = 0, rep_q = 0;
    force_exponents(p, &att_p, &rep_q);
    auto bits = [](double x) {
        uint64_t u;
        std::memcpy(&u, &x, 8);
        return u;
    };
    const std::vector<uint64_t> key = {(uint64_t)(uintptr_t)pos_dev, (uint64_t)count,
                                       (uint64_t)p->precision, bits(p->ideal_length),
                                       bits(p->stop_fraction), bits(p->stop_displacement),
                                       (uint64_t)(uint32_t)att_p, (uint64_t)(uint32_t)rep_q,
                                       (uint64_t)segment_ready_for(kh, p->precision),
                                       (uint64_t)(uintptr_t)kh->d_temps};
    if (!kh->tick_exec || key != kh->tick_key) {
        if (kh->tick_exec) (void)quiet(hipGraphExecDestroy(kh->tick_exec));
        kh->tick_exec = nullptr;
        kh->tick_key.clear();
        hipStream_t cs = capture_stream(kh->device);
        (void)hipGetLastError();  // no stale status may fail a check inside the capture
        if (!cs || hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
            (void)hipGetLastError();
            return enqueue_run(kh, p, h, h + count, pos_dev, s);
        }
        int rc = GILA_OK;
        hipLaunchKernelGGL(reset_ctl_kernel, dim3(1), dim3(1), 0, cs, kh->ctl);
        if (hipGetLastError() != hipSuccess) rc = fail(GILA_EDEVICE, "tick capture: reset");
        if (rc == GILA_OK) rc = launch_permute_in(kh, p->precision, pos_dev, cs);
        StepArgs a = base_args(kh, p);
        a.check_stop = p->stop_fraction > 0.0 ? 1 : 0;
        a.temps = kh->d_temps;
        for (int32_t j = 0; j < count && rc == GILA_OK; ++j) {
            a.pos_cur = kh->pos[j & 1];
            a.pos_next = kh->pos[(j + 1) & 1];
            a.tick_j = j;
            rc = launch_iteration(kh, p->precision, a, cs);
        }
        if (rc == GILA_OK) rc = launch_permute_out(kh, p->precision, pos_dev, cs);
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        hipError_t ie = hipErrorUnknown;
        if (rc == GILA_OK && ee == hipSuccess && graph)
            ie = hipGraphInstantiate(&kh->tick_exec, graph, nullptr, nullptr, 0);
        if (graph) (void)quiet(hipGraphDestroy(graph));
        if (ie != hipSuccess) {
            // a capture another thread's call invalidated, or one the runtime
            // refused: this tick runs eagerly (the same bits); the next tries again
            if (getenv("GILA_DEBUG"))
                fprintf(stderr, "[gila] tick capture refused: enqueue %d, end %s, instantiate %s\n",
                        rc, hipGetErrorString(ee), hipGetErrorString(ie));
            kh->tick_exec = nullptr;
            (void)hipGetLastError();
            clear_error();
            return enqueue_run(kh, p, h, h + count, pos_dev, s);
        }
        kh->tick_key = key;
    }
    hipLaunchKernelGGL(set_h_base_kernel, dim3(1), dim3(1), 0, s, kh->ctl, h);
    GILA_HIP(hipGetLastError());
    GILA_HIP(hipGraphLaunch(kh->tick_exec, s));
    return GILA_OK;
}

// The direct-gather kernel's workgroup plan, made from the list lengths and
// degrees on its first use, and its partials.
static int ensure_direct_plan(gila_khop* kh, hipStream_t s) {
    if (kh->block_start) return GILA_OK;
    const int32_t n = kh->n;
    std::vector<int64_t> kptr((size_t)n + 1, 0), rp((size_t)n + 1, 0);
    if (n > 0) {
        GILA_HIP(hipMemcpyAsync(kptr.data(), kh->kptr, sizeof(int64_t) * (n + 1),
                                hipMemcpyDeviceToHost, s));
        GILA_HIP(hipMemcpyAsync(rp.data(), kh->rp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost,
                                s));
        GILA_HIP(hipStreamSynchronize(s));
    }
    std::vector<int64_t> counts((size_t)n);
    for (int32_t i = 0; i < n; ++i) counts[i] = kptr[i + 1] - kptr[i];
    GILA_TRY(plan_iteration(kh, counts, rp, s));
    kh->device_bytes += (int64_t)sizeof(int32_t) * (kh->nblocks + 1);
    if (kh->nblocks > kh->partials_cap) {
        drop_graphs(kh);  // captured graphs hold the old partials
        dfree_on(kh->partials, s);
        kh->partials = nullptr;
        kh->device_bytes -= (int64_t)sizeof(Partial) * kh->partials_cap;
        kh->partials_cap = 0;
        GILA_TRY(dalloc_t(&kh->partials, (size_t)kh->nblocks));
        kh->partials_cap = kh->nblocks;
        kh->device_bytes += (int64_t)sizeof(Partial) * kh->partials_cap;
    }
    return GILA_OK;
}

int prepare_precision(gila_khop* kh, int precision, hipStream_t s) {
    if (segment_path_enabled()) {
        if (segment_ready_for(kh, precision)) return GILA_OK;
        drop_graphs(kh);
        const int rc = build_segments(kh, precision, s);
        if (rc == GILA_OK) return GILA_OK;
        if (rc != GILA_EUNSUPPORTED) return rc;
        clear_error();  // the direct-gather kernel serves this graph
    }
    return ensure_direct_plan(kh, s);
}

int launch_iteration(const gila_khop* kh, int precision, const StepArgs& a, hipStream_t s) {
    if (segment_ready_for(kh, precision)) return launch_segment_step(kh, precision, a, s);
    return launch_step(kh, precision, a, s);
}

// Everything the captured loop depends on besides the handle's own buffers
// (a change of weights or of the segment layout destroys the cached graph
// where it happens): the positions' address, the iteration range and
// schedule, the parameters, the force law (the kernel instantiation and its
// exponent arguments) and the kernel path.
static std::vector<uint64_t> graph_key(const gila_khop* kh, const gila_params* p,
                                       int32_t start_h, int32_t end_h, void* pos_dev) {
    auto bits = [](double x) {
        uint64_t u;
        std::memcpy(&u, &x, 8);
        return u;
    };
    int32_t att_p = 0, rep_q = 0;
    force_exponents(p, &att_p, &rep_q);
    std::vector<uint64_t> key = {(uint64_t)(uintptr_t)pos_dev, (uint64_t)start_h, (uint64_t)end_h,
                                 (uint64_t)p->precision, bits(p->ideal_length),
                                 bits(p->stop_fraction), bits(p->stop_displacement),
                                 (uint64_t)(uint32_t)att_p, (uint64_t)(uint32_t)rep_q,
                                 (uint64_t)segment_ready_for(kh, p->precision)};
    for (int32_t h = start_h; h < end_h; ++h) key.push_back(bits(p->temperature[h]));
    return key;
}

// Long runs replay one captured chunk of kRunChunk iterations (an even
// number: each chunk starts and ends in the first position buffer) whose caps
// are read from the device copy of the schedule at the base that a small
// kernel sets before each replay; capturing and instantiating the whole run
// would cost a few milliseconds per handle.  The chunk's iterations are the
// same launches as the whole run's, so the result is the same bits.
static int enqueue_chunked_run(gila_khop* kh, const gila_params* p, int32_t start_h,
                               int32_t end_h, void* pos_dev, hipStream_t s) {
    GILA_TRY(upload_schedule(kh, p, s));
    int32_t att_p = 0, rep_q = 0;
    force_exponents(p, &att_p, &rep_q);
    auto bits = [](double x) {
        uint64_t u;
        std::memcpy(&u, &x, 8);
        return u;
    };
    const std::vector<uint64_t> key = {(uint64_t)p->precision, bits(p->ideal_length),
                                       bits(p->stop_fraction), bits(p->stop_displacement),
                                       (uint64_t)(uint32_t)att_p, (uint64_t)(uint32_t)rep_q,
                                       (uint64_t)segment_ready_for(kh, p->precision),
                                       (uint64_t)(uintptr_t)kh->d_temps,
                                       (uint64_t)(uintptr_t)kh->hist, (uint64_t)kh->hist_cap};
    StepArgs a = base_args(kh, p);
    a.check_stop = p->stop_fraction > 0.0 ? 1 : 0;
    a.temps = kh->d_temps;
    if (!kh->chunk_exec || key != kh->chunk_key) {
        if (kh->chunk_exec) (void)quiet(hipGraphExecDestroy(kh->chunk_exec));
        kh->chunk_exec = nullptr;
        kh->chunk_key.clear();
        hipStream_t cs = capture_stream(kh->device);
        if (!cs) return fail(GILA_EDEVICE, "cannot create capture stream");
        (void)hipGetLastError();  // no stale status may fail a check inside the capture
        GILA_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        int rc = GILA_OK;
        for (int32_t j = 0; j < kRunChunk && rc == GILA_OK; ++j) {
            a.pos_cur = kh->pos[j & 1];
            a.pos_next = kh->pos[(j + 1) & 1];
            a.tick_j = j;
            rc = launch_iteration(kh, p->precision, a, cs);
        }
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        if (rc != GILA_OK) {
            if (graph) (void)quiet(hipGraphDestroy(graph));
            return rc;
        }
        if (ee != hipSuccess) return fail(GILA_EDEVICE, "chunk capture: %s", hipGetErrorString(ee));
        const hipError_t ie = hipGraphInstantiate(&kh->chunk_exec, graph, nullptr, nullptr, 0);
        (void)quiet(hipGraphDestroy(graph));
        if (ie != hipSuccess) {
            kh->chunk_exec = nullptr;
            return fail(GILA_EDEVICE, "chunk instantiate: %s", hipGetErrorString(ie));
        }
        kh->chunk_key = key;
    }
    hipLaunchKernelGGL(reset_ctl_kernel, dim3(1), dim3(1), 0, s, kh->ctl);
    GILA_HIP(hipGetLastError());
    GILA_TRY(launch_permute_in(kh, p->precision, pos_dev, s));
    int32_t h = start_h;
    for (; end_h - h >= kRunChunk; h += kRunChunk) {
        hipLaunchKernelGGL(set_h_base_kernel, dim3(1), dim3(1), 0, s, kh->ctl, h);
        GILA_HIP(hipGetLastError());
        GILA_HIP(hipGraphLaunch(kh->chunk_exec, s));
    }
    // the rest one launch at a time, continuing in the first buffer
    a.temps = nullptr;
    for (int32_t j = 0; h < end_h; ++h, ++j) {
        a.pos_cur = kh->pos[j & 1];
        a.pos_next = kh->pos[(j + 1) & 1];
        a.t = p->temperature[h];
        a.hist_slot = h < kh->hist_cap ? h : -1;
        GILA_TRY(launch_iteration(kh, p->precision, a, s));
    }
    return launch_permute_out(kh, p->precision, pos_dev, s);
}

int run_iterations(gila_khop* kh, const gila_params* p, int32_t start_h, int32_t end_h,
                   void* pos_dev, hipStream_t stream, gila_stats* out, bool use_graph) {
    if (kh->n > 0 && !pos_dev) return fail(GILA_EINVAL, "pos_dev is NULL");
    if (start_h < 0 || end_h < start_h || end_h > p->iterations)
        return fail(GILA_EINVAL, "iteration range [%d, %d) outside [0, %d]", start_h, end_h,
                    p->iterations);
    GILA_TRY(prepare_precision(kh, p->precision, stream));
    if (use_graph && end_h - start_h >= 2 * kRunChunk) {
        GILA_TRY(enqueue_chunked_run(kh, p, start_h, end_h, pos_dev, stream));
    } else if (use_graph && end_h > start_h) {
        std::vector<uint64_t> key = graph_key(kh, p, start_h, end_h, pos_dev);
        if (!kh->gexec || key != kh->gkey) {
            if (kh->gexec) {
                (void)quiet(hipGraphExecDestroy(kh->gexec));
                kh->gexec = nullptr;
            }
            hipStream_t cs = capture_stream(kh->device);
            if (!cs) return fail(GILA_EDEVICE, "cannot create capture stream");
            (void)hipGetLastError();  // no stale status may fail a check inside the capture
            GILA_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
            const int rc = enqueue_run(kh, p, start_h, end_h, pos_dev, cs);
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(cs, &graph);
            if (rc != GILA_OK) {
                if (graph) (void)quiet(hipGraphDestroy(graph));
                return rc;
            }
            if (ee != hipSuccess)
                return fail(GILA_EDEVICE, "graph capture: %s", hipGetErrorString(ee));
            const hipError_t ie = hipGraphInstantiate(&kh->gexec, graph, nullptr, nullptr, 0);
            (void)quiet(hipGraphDestroy(graph));
            if (ie != hipSuccess) {
                kh->gexec = nullptr;
                return fail(GILA_EDEVICE, "graph instantiate: %s", hipGetErrorString(ie));
            }
            kh->gkey = key;
        }
        GILA_HIP(hipGraphLaunch(kh->gexec, stream));
    } else {
        GILA_TRY(enqueue_run(kh, p, start_h, end_h, pos_dev, stream));
    }
    Ctl c{};
    GILA_HIP(hipMemcpyAsync(&c, kh->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    GILA_HIP(hipStreamSynchronize(stream));
    if (kh->n_active == 0) c.iters_run = end_h - start_h;  // nothing can move
    if (out) to_stats(c, out);
    return nonfinite_status(c);
}

}  // namespace gila

using namespace gila;

extern "C" {

int gila_paper_schedule(double n, double aspect, double ideal_length, int32_t iterations,
                        double* temperature_host) {
    clear_error();
    char msg[256];
    const int rc = host::paper_schedule(n, aspect, ideal_length, iterations, temperature_host,
                                        msg, sizeof(msg));
    return rc == GILA_OK ? GILA_OK : fail(rc, "%s", msg);
}

int gila_linear_schedule(double t0, int32_t iterations, double* temperature_host) {
    clear_error();
    char msg[256];
    const int rc = host::linear_schedule(t0, iterations, temperature_host, msg, sizeof(msg));
    return rc == GILA_OK ? GILA_OK : fail(rc, "%s", msg);
}

int gila_init_positions(int32_t n, uint64_t seed, double width, double height, int32_t precision,
                        void* pos_dev, void* stream) {
    clear_error();
    if (n < 0) return fail(GILA_EINVAL, "n must be >= 0");
    if (n > 0 && !pos_dev) return fail(GILA_EINVAL, "pos_dev is NULL");
    if (!(width >= 0.0) || !(height >= 0.0) || !std::isfinite(width) || !std::isfinite(height))
        return fail(GILA_EINVAL, "frame must be finite and >= 0");
    if (n == 0) return GILA_OK;
    hipStream_t s = (hipStream_t)stream;
    const int g = grid_for(n);
    switch (precision) {
        case GILA_FP64:
            hipLaunchKernelGGL(init_positions_kernel<double2>, dim3(g), dim3(kBlock), 0, s, n,
                               seed, width, height, (double2*)pos_dev);
            break;
        case GILA_FP32:
        case GILA_FP32_KAHAN:
            hipLaunchKernelGGL(init_positions_kernel<float2>, dim3(g), dim3(kBlock), 0, s, n,
                               seed, width, height, (float2*)pos_dev);
            break;
        default: return fail(GILA_EINVAL, "unknown precision %d", precision);
    }
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

int gila_step(const gila_khop* kh_c, const gila_params* params, int32_t h, void* pos_dev,
              double* force_dev, double* disp_dev, void* stream, gila_stats* out) {
    TraceRange trace_range("gila_step");
    clear_error();
    gila_khop* kh = const_cast<gila_khop*>(kh_c);
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    GILA_TRY(check_params(params, true));
    if (h < 0 || h >= params->iterations)
        return fail(GILA_EINVAL, "h = %d outside [0, %d)", h, params->iterations);
    if (kh->n > 0 && !pos_dev) return fail(GILA_EINVAL, "pos_dev is NULL");
    if ((force_dev == nullptr) != (disp_dev == nullptr))
        return fail(GILA_EINVAL, "force_dev and disp_dev must both be set or both NULL");
    std::lock_guard<std::mutex> lk(kh->mu);
    DeviceGuard dg(kh->device);
    hipStream_t s = (hipStream_t)stream;
    GILA_TRY(prepare_precision(kh, params->precision, s));
    if (force_dev && kh->n > 0) {
        // isolated vertices feel no force and do not move
        GILA_HIP(hipMemsetAsync(force_dev, 0, sizeof(double) * 2 * kh->n, s));
        GILA_HIP(hipMemsetAsync(disp_dev, 0, sizeof(double) * 2 * kh->n, s));
    }
    hipLaunchKernelGGL(reset_ctl_kernel, dim3(1), dim3(1), 0, s, kh->ctl);
    GILA_HIP(hipGetLastError());
    GILA_TRY(launch_permute_in(kh, params->precision, pos_dev, s));
    StepArgs a = base_args(kh, params);
    a.check_stop = 0;
    a.pos_cur = kh->pos[0];
    a.pos_next = kh->pos[1];
    a.t = params->temperature[h];
    a.hist_slot = h < kh->hist_cap ? h : -1;
    a.F_out = force_dev;
    a.D_out = disp_dev;
    GILA_TRY(launch_iteration(kh, params->precision, a, s));
    GILA_TRY(launch_permute_out(kh, params->precision, pos_dev, s));
    if (out) {
        Ctl c{};
        GILA_HIP(hipMemcpyAsync(&c, kh->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        if (kh->n_active == 0) c.iters_run = 1;
        to_stats(c, out);
        return nonfinite_status(c);
    }
    return GILA_OK;
}

int gila_run(const gila_khop* kh_c, const gila_params* params, int32_t start_h, int32_t end_h,
             void* pos_dev, void* stream, gila_stats* out) {
    TraceRange trace_range("gila_run");
    clear_error();
    gila_khop* kh = const_cast<gila_khop*>(kh_c);
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    GILA_TRY(check_params(params, true));
    std::lock_guard<std::mutex> lk(kh->mu);
    DeviceGuard dg(kh->device);
    const char* env = getenv("GILA_NO_GRAPH");
    const bool use_graph = !(env && env[0] == '1');
    return run_iterations(kh, params, start_h, end_h, pos_dev, (hipStream_t)stream, out,
                          use_graph);
}

int gila_time_iterations(const gila_khop* kh_c, const gila_params* params, int32_t h,
                         int32_t reps, void* pos_dev, void* stream, double* ms_out) {
    TraceRange trace_range("gila_time_iterations");
    clear_error();
    gila_khop* kh = const_cast<gila_khop*>(kh_c);
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    if (!ms_out) return fail(GILA_EINVAL, "ms_out is NULL");
    GILA_TRY(check_params(params, true));
    if (reps < 1 || h < 0 || h + reps > params->iterations)
        return fail(GILA_EINVAL, "iterations [%d, %d) outside the schedule", h, h + reps);
    if (kh->n > 0 && !pos_dev) return fail(GILA_EINVAL, "pos_dev is NULL");
    std::lock_guard<std::mutex> lk(kh->mu);
    DeviceGuard dg(kh->device);
    hipStream_t s = (hipStream_t)stream;
    GILA_TRY(prepare_precision(kh, params->precision, s));
    const bool seg = segment_ready_for(kh, params->precision);
    int khz = 0;
    GILA_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, kh->device));
    if (khz <= 0) return fail(GILA_EDEVICE, "no device wall clock rate");
    // per iteration: the force kernel's first start and last end
    std::vector<unsigned long long> span_h((size_t)2 * reps);
    for (int32_t r = 0; r < reps; ++r) {
        span_h[2 * r] = ~0ull;
        span_h[2 * r + 1] = 0ull;
    }
    unsigned long long* span = nullptr;
    GILA_TRY(dalloc_t(&span, span_h.size()));
    GILA_HIP(hipMemcpyAsync(span, span_h.data(), sizeof(unsigned long long) * span_h.size(),
                            hipMemcpyHostToDevice, s));
    // the iterations h .. h + reps - 1 exactly as gila_run runs them (which
    // advance pos_dev), the force kernels recording their spans
    auto enqueue = [&](hipStream_t q) -> int {
        hipLaunchKernelGGL(reset_ctl_kernel, dim3(1), dim3(1), 0, q, kh->ctl);
        GILA_HIP(hipGetLastError());
        GILA_TRY(launch_permute_in(kh, params->precision, pos_dev, q));
        StepArgs a = base_args(kh, params);
        for (int32_t r = 0; r < reps; ++r) {
            a.pos_cur = kh->pos[r & 1];
            a.pos_next = kh->pos[(r + 1) & 1];
            a.t = params->temperature[h + r];
            a.hist_slot = h + r < kh->hist_cap ? h + r : -1;
            if (seg) GILA_TRY(launch_segment_step(kh, params->precision, a, q, span + 2 * r));
            else GILA_TRY(launch_step(kh, params->precision, a, q));
        }
        return launch_permute_out(kh, params->precision, pos_dev, q);
    };
    hipGraphExec_t exec = nullptr;
    bool in_graph = false;
    {
        hipStream_t cs = capture_stream(kh->device);
        (void)hipGetLastError();  // no stale status may fail a check inside the capture
        if (cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            const int erc = enqueue(cs);
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(cs, &graph);
            in_graph = erc == GILA_OK && ee == hipSuccess && graph &&
                       hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
            if (graph) (void)quiet(hipGraphDestroy(graph));
            if (!in_graph && getenv("GILA_DEBUG"))
                fprintf(stderr, "[gila] timing capture refused: %d (%s), end %s\n", erc,
                        gila_last_error(), hipGetErrorString(ee));
        }
        (void)hipGetLastError();
        clear_error();
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    int rc = GILA_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            rc = fail(GILA_EDEVICE, "hipEventCreate failed");
        }
    if (rc == GILA_OK && hipEventRecord(ev[0], s) != hipSuccess) rc = fail(GILA_EDEVICE, "event record");
    if (rc == GILA_OK) {
        if (in_graph) {
            if (hipGraphLaunch(exec, s) != hipSuccess) rc = fail(GILA_EDEVICE, "graph launch");
        } else {
            rc = enqueue(s);
        }
    }
    if (rc == GILA_OK && hipEventRecord(ev[1], s) != hipSuccess) rc = fail(GILA_EDEVICE, "event record");
    if (rc == GILA_OK &&
        hipMemcpyAsync(span_h.data(), span, sizeof(unsigned long long) * span_h.size(),
                       hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = fail(GILA_EDEVICE, "span download");
    if (rc == GILA_OK && hipStreamSynchronize(s) != hipSuccess)
        rc = fail(GILA_EDEVICE, "stream synchronise failed");
    float t = 0.f;
    if (rc == GILA_OK && hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess)
        rc = fail(GILA_EDEVICE, "hipEventElapsedTime failed");
    if (exec) (void)quiet(hipGraphExecDestroy(exec));
    for (auto& e : ev)
        if (e) (void)quiet(hipEventDestroy(e));
    dfree_on(span, s);
    if (rc == GILA_OK) {
        const double iter = (double)t / reps;
        double f = iter;
        if (seg) {
            uint64_t ticks = 0;
            for (int32_t r = 0; r < reps; ++r)
                if (span_h[2 * r + 1] > span_h[2 * r]) ticks += span_h[2 * r + 1] - span_h[2 * r];
            f = (double)ticks / (double)khz / reps;  // ticks / kHz = ms
        }
        ms_out[0] = f;
        ms_out[1] = seg ? iter - f : 0.0;
        ms_out[2] = in_graph ? 1.0 : 0.0;
    }
    return rc;
}

int gila_enable_history(gila_khop* kh, int32_t capacity, void* stream) {
    clear_error();
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    if (capacity < 0) return fail(GILA_EINVAL, "capacity must be >= 0");
    std::lock_guard<std::mutex> lk(kh->mu);
    DeviceGuard dg(kh->device);
    hipStream_t s = (hipStream_t)stream;
    // captured loops hold the table's rows in their arguments
    drop_graphs(kh);
    dfree_on(kh->hist, s);
    kh->hist = nullptr;
    kh->hist_cap = 0;
    if (capacity == 0) return GILA_OK;
    GILA_TRY(dalloc_t(&kh->hist, (size_t)capacity * 4));
    // rows of iterations not run read as NaN
    const std::vector<double> nan((size_t)capacity * 4, std::nan(""));
    GILA_HIP(hipMemcpyAsync(kh->hist, nan.data(), nan.size() * sizeof(double),
                            hipMemcpyHostToDevice, s));
    GILA_HIP(hipStreamSynchronize(s));
    kh->hist_cap = capacity;
    return GILA_OK;
}

int gila_history(const gila_khop* kh_c, int32_t h0, int32_t count, double* rows_host,
                 void* stream) {
    clear_error();
    gila_khop* kh = const_cast<gila_khop*>(kh_c);
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    if (h0 < 0 || count < 0 || (int64_t)h0 + count > kh->hist_cap)
        return fail(GILA_EINVAL, "rows [%d, %lld) outside the history of %d rows", h0,
                    (long long)h0 + count, kh->hist_cap);
    if (count > 0 && !rows_host) return fail(GILA_EINVAL, "rows_host is NULL");
    if (count == 0) return GILA_OK;
    std::lock_guard<std::mutex> lk(kh->mu);
    DeviceGuard dg(kh->device);
    hipStream_t s = (hipStream_t)stream;
    GILA_HIP(hipMemcpyAsync(rows_host, kh->hist + 4 * (int64_t)h0,
                            sizeof(double) * 4 * (size_t)count, hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    return GILA_OK;
}

int gila_layout(const gila_csr* g_dev, int32_t k, const gila_params* params, void* pos_dev,
                void* stream, gila_stats* out) {
    TraceRange trace_range("gila_layout");
    clear_error();
    GILA_TRY(check_params(params, true));
    gila_khop* kh = nullptr;
    GILA_TRY(gila_build_khop(g_dev, k, stream, &kh));
    int rc;
    {
        std::lock_guard<std::mutex> lk(kh->mu);
        rc = run_iterations(kh, params, 0, params->iterations, pos_dev, (hipStream_t)stream, out,
                            false);
    }
    free_khop(kh, Release{true, (hipStream_t)stream});
    return rc;
}

}  // extern "C"

// Internal declarations of libgila (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gila.h"

namespace gila {

// ------------------------------------------------------------------ errors
int fail(int code, const char* fmt, ...);  // records a thread-local message, returns code
void clear_error();

#define GILA_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t gila_e_ = (call);                                                    \
        if (gila_e_ != hipSuccess)                                                      \
            return ::gila::fail(gila_e_ == hipErrorOutOfMemory ? GILA_ENOMEM : GILA_EDEVICE, \
                                "%s failed: %s (%s:%d)", #call,                        \
                                hipGetErrorString(gila_e_), __FILE__, __LINE__);        \
    } while (0)

#define GILA_TRY(expr)            \
    do {                          \
        int gila_rc_ = (expr);    \
        if (gila_rc_ != GILA_OK)  \
            return gila_rc_;      \
    } while (0)

// For a call whose failure is handled otherwise or harmless (teardown, cache
// trims, a function attribute that the launch after it checks): HIP also
// keeps a failure as the thread's last error, which the next launch check
// would report as its own, so it is taken back here.
inline hipError_t quiet(hipError_t e) {
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

// Device allocation that maps failure to GILA_ENOMEM.
int dalloc(void** p, size_t bytes);
template <class T>
int dalloc_t(T** p, size_t count) {
    return dalloc(reinterpret_cast<void**>(p), count * sizeof(T) + (count == 0 ? 16 : 0));
}
// hipFree semantics (synchronises the device)
void dfree(void* p);
// Releases a dalloc() block into the library's cache: it is reused once the
// work enqueued on `s` so far has completed (at once when `idle`: the caller
// knows no work uses it).  No device-wide synchronisation.
void dfree_on(void* p, hipStream_t s, bool idle = false);

// How a handle's device memory is released: hipFree (the default, safe for
// work on any stream), or into the cache once the work on `stream` is done.
struct Release {
    bool cached = false;
    hipStream_t stream = nullptr;
    bool idle = false;  // cached, with the device known to be idle: reusable at once
    void operator()(void* p) const {
        if (cached) dfree_on(p, stream, idle);
        else dfree(p);
    }
};

// Release for the public free calls: waits once for the whole device (the
// caller's work on the handle may be queued on any stream), then caches every
// block as reusable at once.  If the device cannot be synchronised, the blocks
// take plain hipFree instead.
Release public_release();

// Returns every cached block whose releasing work has completed to the device;
// the bytes returned.
int64_t release_cached();

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

// Phase timing of host-driven builds, printed to stderr when the environment
// variable GILA_TIMING is 1 (each mark synchronises the stream).
struct PhaseTimer {
    const char* what;
    hipStream_t stream;
    bool on;
    double t0, last;
    std::string log;
    PhaseTimer(const char* w, hipStream_t s);
    void mark(const char* phase);
    ~PhaseTimer();
};

// A roctx range (visible to rocprofv3 --marker-trace) for the lifetime of
// the object: the library's entry points and the server's units of work.
struct TraceRange {
    explicit TraceRange(const char* name);
    ~TraceRange();
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// A library-owned, default-priority stream per device for graph capture.
hipStream_t capture_stream(int device);

struct DeviceInfo {
    int cus = 256;
    size_t max_lds_per_block = 65536;
    int warp = 64;
};
const DeviceInfo& device_info(int device);

constexpr int kBlock = 256;       // threads per workgroup in every kernel
constexpr int64_t kHubMin = 8192; // rows at least this long get a workgroup of their own (direct path)
constexpr int kWaves = kBlock / 64;

// ------------------------------------------------------------------ device control block
// Written by the statistics kernel that ends each iteration; read by the host
// at the end of a call and by the next iteration's kernels (stopped flag).
struct Ctl {
    int32_t stopped;
    int32_t iters_run;
    uint32_t done_blocks;  // reserved
    int32_t h_base;        // first iteration of a captured tick (caps read on the device)
    int64_t moved;
    double max_disp;
    double energy;
    int64_t coincident;
    int64_t coinc_pending;  // coincident pairs counted by the segment kernel, not yet published
    int64_t nonfinite;      // last iteration: vertices with a non-finite force (stopped = 2)
};

// Per-workgroup partial statistics of one iteration.
struct Partial {
    double energy;
    double max_disp;
    int64_t moved;
    int64_t coincident;
    int64_t nonfinite;
};

// ------------------------------------------------------------------ iteration kernel arguments
struct StepArgs {
    int32_t n_active;
    int32_t nhub;               // vertices [0, nhub) are hubs: one workgroup each
    int32_t nblocks;            // total workgroups of the launch
    const int32_t* block_start; // normal workgroup b - nhub covers [block_start[b-nhub], block_start[b-nhub+1])
    const int64_t* rp;
    const int32_t* ci;
    const int64_t* kptr;
    const int32_t* kidx;
    const void* pos_cur;
    void* pos_next;
    double d;
    double t;                   // cap of the iteration, unless temps is set:
    const double* temps;        // device schedule: the cap is temps[ctl->h_base + tick_j]
    int32_t tick_j;             // (captured ticks, whose first iteration is set at replay)
    double stop_fraction;
    double stop_displacement;
    int32_t check_stop;
    int32_t hist_slot;          // < 0: no history (with temps: ctl->h_base + tick_j)
    int32_t hist_cap;           // rows of the history table
    const int32_t* perm;        // internal -> caller ids (for F/D outputs)
    double* F_out;              // caller ids, may be null
    double* D_out;
    Partial* partials;          // [nblocks]
    Ctl* ctl;
    double* hist;               // [slots][4]: energy, max_disp, moved, coincident
    // segment-blocked path: the partial forces of vertex v are
    // part[vsl[v] .. vsl[v + 1]), one per non-empty slice, in segment order
    const int64_t* vsl;
    const double2* part;
    // weight of the repulsion each vertex exerts (internal ids; float for the
    // FP32 precisions, double for FP64); null = every weight 1
    const void* mass;
    int32_t att_p;              // force exponents (FR: 2, 1)
    int32_t rep_q;
};

// Arguments of the segment kernel (one workgroup = one id segment x a range
// of that segment's slices).
struct SegArgs {
    int32_t na;                 // non-isolated vertices (rows)
    int32_t seg;                // segment size S (vertex ids per segment)
    const int4* wg;             // [grid] (segment, first slice, end slice, lanes per slice)
    const int32_t* sl_v;        // [T] row of each slice (segment-major order)
    const int32_t* sl_p;        // [T] index of the slice's partial force
    const int64_t* sl_k;        // [T + 1] start of each slice in kidx (quad-aligned)
    const int32_t* sl_a;        // [T + 1] start of each slice in aidx
    const uint16_t* kidx;       // LDS byte offsets of the k-hop entries
    const uint16_t* aidx;       // LDS byte offsets of the adjacency entries
    const void* pos;            // positions of this iteration (internal ids)
    double2* part;              // [T]
    double d;
    Ctl* ctl;
    const void* mass;           // repulsion weights (internal ids), null = unit
    int32_t att_p;              // force exponents (FR: 2, 1)
    int32_t rep_q;
    // null, or [2]: the device wall clock when the launch's first workgroup
    // started (atomic min) and its last one ended (atomic max)
    unsigned long long* span;
    // dense slices (see segment.hip): null, or [T + 1] dense slices before
    // each slice; their bitmaps, dense_blocks lane masks of 64 slots each
    const int64_t* sl_dn;
    const uint64_t* dmask;
    int32_t dense_blocks;
};

// Arguments of the k-hop frontier-expansion kernel (khop.hip).
struct BfsArgs {
    int32_t n;
    int32_t k;
    int32_t nverts;            // sources are ids [0, nverts)
    int32_t nwords;            // bitmap words (largest graph)
    const int64_t* rp;
    const int32_t* ci;
    int64_t* counts;           // count pass: |N_v(k)| per source
    const int64_t* kptr;       // fill pass: row offsets
    int32_t* kidx;             // fill pass: rows (global ids) ...
    uint16_t* kidx16;          // ... or rows as ids local to the source's graph
    int32_t* queue;            // [grid][qcap] frontier storage (k >= 3)
    int64_t qcap;
    uint32_t* gbitmap;         // [grid][nwords] when the bitmap is not in LDS
    int32_t* work;             // next source (atomic)
    // batch mode (gvbase != nullptr)
    const int64_t* gvbase;     // [ngraphs + 1] first vertex of each graph
    const int32_t* gk;         // [ngraphs] k of each graph
    int32_t ngraphs;
    int32_t kmax;
};

}  // namespace gila

// ------------------------------------------------------------------ handles
struct gila_khop {
    int device = 0;
    int32_t n = 0, k = 0, n_active = 0;
    int64_t nnz = 0, P = 0;
    int64_t device_bytes = 0;
    // internal vertex ids: non-isolated vertices first.  Either by |N_v(k)|
    // descending (ties: caller id), or, when the caller's order already keeps
    // most edges short, rows of at least kHubMin entries first and then the
    // caller's order (see build_khop).
    bool caller_order = false;
    int32_t* perm = nullptr;   // [n] internal -> caller
    int32_t* iperm = nullptr;  // [n] caller -> internal
    int64_t* rp = nullptr;     // internal CSR
    int32_t* ci = nullptr;
    int64_t* kptr = nullptr;   // internal k-hop CSR, rows ascending in internal ids
    int32_t* kidx = nullptr;
    // plan of the iteration kernel
    int32_t lpv = 64;          // lanes per vertex for non-hub vertices
    int32_t nhub = 0;
    int32_t nblocks = 0;       // hub + normal workgroups
    int32_t* block_start = nullptr;
    // workspace
    void* pos[2] = {nullptr, nullptr};  // 16 B per vertex each
    gila::Partial* partials = nullptr;
    int32_t partials_cap = 0;
    gila::Ctl* ctl = nullptr;
    double* hist = nullptr;
    int32_t hist_cap = 0;
    // segment-blocked layout of the k-hop and adjacency lists (see segment.hip)
    bool seg_ready = false;
    int32_t seg = 0, nseg = 0;      // segment size and count
    int64_t nslices = 0;            // non-empty (segment, row) slices T
    int64_t* vsl = nullptr;         // [n_active + 1] first partial of each row
    int32_t* sl_v = nullptr;        // [T] slice records, segment-major
    int32_t* sl_p = nullptr;        // [T]
    int64_t* sl_k = nullptr;        // [T + 1]
    int32_t* sl_a = nullptr;        // [T + 1]
    uint16_t* sk_idx = nullptr;     // [sl_k[T] + tail pad]
    uint16_t* sa_idx = nullptr;     // [nnz + pad]
    int64_t* sl_dn = nullptr;       // [T + 1] dense slices before each slice (null: none)
    uint64_t* dmask = nullptr;      // [dense slices][dense_blocks] lane masks of 64 slots
    int32_t dense_blocks = 0;
    int64_t ndense = 0;
    int4* seg_wg = nullptr;         // [seg_grid]
    int32_t seg_grid = 0;
    int32_t comb_grid = 0;
    double2* part = nullptr;        // [T] partial force of each slice, row-major
    int32_t seg_precision = -1;     // precision the segment size was chosen for
    bool seg_weighted = false;      // segment size chosen with a weight per staged vertex
    bool seg_large = false;         // force kernel shape: 1024 threads (else 512)
    // weights of the repulsion each vertex exerts (internal ids), null = unit
    double* mass64 = nullptr;
    float* mass32 = nullptr;
    // cached HIP graph of the last gila_run call
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> gkey;
    // captured tick of the layout server: a fixed number of iterations whose
    // caps come from the device copy of the schedule at ctl->h_base
    hipGraphExec_t tick_exec = nullptr;
    std::vector<uint64_t> tick_key;
    hipGraphExec_t chunk_exec = nullptr;  // kRunChunk iterations of gila_run, caps from d_temps
    std::vector<uint64_t> chunk_key;
    double* d_temps = nullptr;
    std::vector<double> temps_host;  // the schedule d_temps holds
    std::mutex mu;
};

namespace gila {
// implemented in force.hip
int launch_step(const gila_khop* kh, int precision, const StepArgs& a, hipStream_t s);
int plan_iteration(gila_khop* kh, const std::vector<int64_t>& counts_internal,
                   const std::vector<int64_t>& rp_internal, hipStream_t s);
// implemented in khop.hip
int build_khop(const gila_csr* g, int32_t k, hipStream_t s, gila_khop** out);
void free_khop(gila_khop* kh, Release rel = Release{});
int run_bfs(bool fill, int device, hipStream_t s, BfsArgs a);
int launch_validate_csr(int32_t n, int64_t nnz, const int64_t* rp, const int32_t* ci, int32_t* flag,
                        hipStream_t s);
int validate_graph(const gila_csr* g, hipStream_t s);
// implemented in util.hip: out[0] = 0, out[i + 1] = in[0] + ... + in[i]
// (in != out).  The enqueue variant needs scan_workspace_count(n) int64 of
// workspace and does not synchronise; the other allocates and synchronises.
int exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
int64_t scan_workspace_count(int64_t n);
int enqueue_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* ws,
                               hipStream_t s);
// implemented in segment.hip
int build_segments(gila_khop* kh, int precision, hipStream_t s);
// Stable sort of the ids 0 .. n-1 by key (ascending; equal keys keep
// ascending ids) into out[n], ordered on `s`: LSD counting-sort passes of
// 11-bit digits over the bits of max_key (every key <= max_key).  Scratch is
// released into the block cache after the work on `s`.
int stable_order_by_key(int32_t n, const uint32_t* key, uint32_t max_key, int32_t* out,
                        hipStream_t s);
void free_segments(gila_khop* kh, Release rel = Release{});
// span: null, or where the force kernel records its start and end (SegArgs)
int launch_segment_step(const gila_khop* kh, int precision, const StepArgs& a, hipStream_t s,
                        unsigned long long* span = nullptr);
bool segment_path_enabled();
// segment size S for the handle's graph in `precision` (weighted repulsion
// stores a weight beside each staged position)
int seg_size_for(const gila_khop* kh, int precision);
// the segment layout is built for `precision` and the iteration uses it
bool segment_ready_for(const gila_khop* kh, int precision);
// implemented in layout.hip: publishes an iteration's statistics from the
// per-workgroup partials (launched after each per-vertex kernel)
int launch_iteration_stats(const StepArgs& a, hipStream_t s);
// implemented in layout.hip: one iteration on whichever path the handle is ready for
int launch_iteration(const gila_khop* kh, int precision, const StepArgs& a, hipStream_t s);
int prepare_precision(gila_khop* kh, int precision, hipStream_t s);
// destroys the handle's captured graphs (their kernels or arguments changed)
void drop_graphs(gila_khop* kh);
// implemented in layout.hip
int run_iterations(gila_khop* kh, const gila_params* p, int32_t start_h, int32_t end_h,
                   void* pos_dev, hipStream_t stream, gila_stats* out, bool use_graph);
int check_params(const gila_params* p, bool need_temps);
// GILA_ENONFINITE (with a message) when the control block records a
// non-finite force, else GILA_OK
int nonfinite_status(const Ctl& c);
// exponents (p, q) of the params' force model
void force_exponents(const gila_params* p, int32_t* att_p, int32_t* rep_q);
// Enqueues (no synchronisation) iterations [start_h, end_h) on pos_dev: reset
// of the control block, permute in, the iterations, permute out.
int enqueue_run(gila_khop* kh, const gila_params* p, int32_t start_h, int32_t end_h,
                void* pos_dev, hipStream_t s);
// Enqueues iterations [h, h + count) like enqueue_run, with the same bits;
// when count == graph_len they replay one captured graph per handle (built on
// first use, the caps read from a device copy of the schedule), so a tick of
// the server costs two launches instead of three per iteration.
int enqueue_tick(gila_khop* kh, const gila_params* p, int32_t h, int32_t count,
                 int32_t graph_len, void* pos_dev, hipStream_t s);
// implemented in batch.hip
int batch_build(const gila_csr* graphs, int32_t count, const int32_t* k, hipStream_t s,
                gila_batch** out);
int batch_run(gila_batch* b, const gila_params* params, void* const* pos, hipStream_t s,
              gila_stats* out, bool use_graph);
void free_batch(gila_batch* b, Release rel = Release{});
size_t batch_lds_bytes(int32_t nmax, int precision);
}  // namespace gila

// k-neighbourhood lists N_v(k) (Section 4.5) by CSR frontier expansion.
//
// The paper delivers N_v(k) to v every iteration by flooding messages with a
// time-to-live of k and deduplicating senders in a per-vertex hash set.  The
// graph does not change between iterations, so here the set is built once:
// one workgroup expands the frontier of one source vertex level by level,
// deduplicating with a bitmap over all vertex ids held in LDS (global memory
// when n is too large for LDS).  A count pass gives |N_v(k)|; after the
// prefix sum a fill pass writes each row by scanning the bitmap, which yields
// the row in ascending id order with no sort.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "device_util.h"
#include "gila_internal.h"
#include "host_logic.h"

namespace gila {

// ------------------------------------------------------------------ validation
// flag bits: 1 column out of range, 2 self-loop, 4 row not strictly ascending,
// 8 asymmetric (u in row v but v not in row u).  With `near` set, also counts
// the entries with |u - v| < window (how local the caller's order is).
__global__ __launch_bounds__(kBlock) void validate_csr_kernel(int32_t n, int64_t nnz,
                                                              const int64_t* __restrict__ rp,
                                                              const int32_t* __restrict__ ci,
                                                              int32_t* __restrict__ flag,
                                                              int32_t window,
                                                              unsigned long long* __restrict__ near) {
    int32_t bad = 0;
    int64_t close = 0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * kBlock) {
        // owner row: largest v with rp[v] <= e
        int32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            int32_t mid = lo + (hi - lo + 1) / 2;
            if (rp[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int32_t v = lo;
        const int32_t u = ci[e];
        if (u < 0 || u >= n) {
            bad |= 1;
            continue;
        }
        if (u == v) bad |= 2;
        close += (u - v < window && v - u < window) ? 1 : 0;
        if (e > rp[v] && ci[e - 1] >= u) bad |= 4;
        // binary search v in row u
        int64_t a = rp[u], b = rp[u + 1] - 1;
        bool found = false;
        while (a <= b) {
            int64_t mid = a + (b - a) / 2;
            int32_t x = ci[mid];
            if (x == v) {
                found = true;
                break;
            }
            if (x < v) a = mid + 1;
            else b = mid - 1;
        }
        if (!found) bad |= 8;
    }
    if (bad) atomicOr(flag, bad);
    if (near) {
        const int64_t c = wave_sum(close);
        if (lane64() == 0 && c) atomicAdd(near, (unsigned long long)c);
    }
}

// ------------------------------------------------------------------ BFS count / fill
// One workgroup expands one source at a time.  In batch mode the sources
// belong to many independent graphs laid out one after another (a
// block-diagonal union): each source's bitmap covers only its own graph's id
// range and its k is its graph's k.
// With the bitmap in LDS, a summary bitmap (one bit per bitmap word) records
// the words a source touched, so clearing and scanning cost O(n/1024 + |row|)
// per source instead of O(n/32).
// Frontier rows at least this long are walked by a whole wavefront.
constexpr int64_t kWaveRow = 32;
constexpr int32_t kBfsTake = 4;

// BS threads per workgroup (256 or 512; see run_bfs).  With 512, registers
// are capped so that 8 wavefronts fit per SIMD.

template <int BS, bool FILL, bool LDS_BITMAP>
__global__ __launch_bounds__(BS, BS / 64) void khop_bfs_kernel(BfsArgs a) {
    constexpr int kBfsBlock = BS;
    constexpr int kBfsWaves = BS / 64;
    extern __shared__ uint32_t s_dyn[];
    constexpr bool SUMMARY = LDS_BITMAP;
    __shared__ int32_t s_v;
    __shared__ int32_t s_qtail;
    __shared__ int32_t s_bw[kBfsBlock];    // frontier vertex of each listed long row
    __shared__ int32_t s_bdeg[kBfsBlock];  // its degree
    __shared__ int32_t s_nbig;             // long rows listed in this chunk
    __shared__ int64_t s_red[kBfsWaves];

    uint32_t* bm = LDS_BITMAP ? s_dyn : a.gbitmap + (size_t)blockIdx.x * a.nwords;
    uint32_t* sm = s_dyn + a.nwords;  // summary (LDS bitmap only)
    int32_t* queue = a.queue ? a.queue + (size_t)blockIdx.x * a.qcap : nullptr;

    if (threadIdx.x == 0) s_nbig = 0;
    for (int i = threadIdx.x; i < a.nwords; i += kBfsBlock) bm[i] = 0u;
    if constexpr (SUMMARY)
        for (int i = threadIdx.x; i < (a.nwords + 31) / 32; i += kBfsBlock) sm[i] = 0u;
    __syncthreads();
    // sets bit u; true if it was clear
    auto visit = [&](int64_t u) -> bool {
        const uint32_t bit = 1u << (u & 31);
        const uint32_t old = atomicOr(&bm[u >> 5], bit);
        if constexpr (SUMMARY)
            if (old == 0u) atomicOr(&sm[u >> 10], 1u << ((u >> 5) & 31));
        return !(old & bit);
    };

    // sources are taken kBfsTake at a time (one atomic per group)
    for (;;) {
        if (threadIdx.x == 0) s_v = atomicAdd(a.work, kBfsTake);
        __syncthreads();
        const int32_t v0 = s_v;
        if (v0 >= a.nverts) break;
        const int32_t v1 = min(v0 + kBfsTake, a.nverts);
        for (int32_t v = v0; v < v1; ++v) {
            // the source's graph: id base, bitmap words and k
            int64_t base = 0;
            int32_t nw = a.nwords, k = a.k;
            if (a.gvbase) {
                int32_t lo = 0, hi = a.ngraphs - 1;
                while (lo < hi) {
                    const int32_t mid = lo + (hi - lo + 1) / 2;
                    if (a.gvbase[mid] <= v) lo = mid;
                    else hi = mid - 1;
                }
                base = a.gvbase[lo];
                nw = (int32_t)((a.gvbase[lo + 1] - base + 31) / 32);
                k = a.gk[lo];
            }
            const int64_t rb = a.rp[v], re = a.rp[v + 1];
            int64_t mycount = 0;
            if (re > rb) {
                if (threadIdx.x == 0) {
                    visit(v - base);
                    s_qtail = 0;
                }
                __syncthreads();
                // level 1: the adjacency row (distinct, never v in a simple graph)
                for (int64_t e = rb + threadIdx.x; e < re; e += kBfsBlock)
                    if (visit(a.ci[e] - base)) ++mycount;
                __syncthreads();
                // levels 2..k: expand the previous level's new vertices.  A frontier
                // vertex with a short row is walked by one lane; long rows are
                // listed in LDS and walked by whole wavefronts (coalesced reads).
                // The visited set does not depend on the order of the visits.
                int64_t fb = rb, fe = re;
                bool from_queue = false;
                for (int level = 2; level <= k; ++level) {
                    const bool record = level < k;
                    const int32_t qstart = s_qtail;
                    // every thread has read the level's queue start before any
                    // thread appends to the queue
                    __syncthreads();
                    auto expand = [&](int32_t ug) {
                        if (visit(ug - base)) {
                            ++mycount;
                            if (record) {
                                const int32_t q = atomicAdd(&s_qtail, 1);
                                queue[q] = ug;
                            }
                        }
                    };
                    for (int64_t c = fb; c < fe; c += kBfsBlock) {
                        const int64_t i = c + threadIdx.x;
                        int64_t deg = 0, start = 0;
                        int32_t w = 0;
                        if (i < fe) {
                            w = from_queue ? queue[i] : a.ci[i];
                            start = a.rp[w];
                            deg = a.rp[w + 1] - start;
                        }
                        if (deg >= kWaveRow) {
                            const int b = atomicAdd(&s_nbig, 1);
                            s_bw[b] = w;
                            s_bdeg[b] = (int32_t)deg;
                        } else {
                            int64_t e = 0;
                            for (; e + 4 <= deg; e += 4) {
                                const int32_t u0 = a.ci[start + e], u1 = a.ci[start + e + 1];
                                const int32_t u2 = a.ci[start + e + 2], u3 = a.ci[start + e + 3];
                                expand(u0);
                                expand(u1);
                                expand(u2);
                                expand(u3);
                            }
                            for (; e < deg; ++e) expand(a.ci[start + e]);
                        }
                        __syncthreads();
                        const int nbig = s_nbig;
                        for (int b = wave_id(); b < nbig; b += kBfsWaves) {
                            const int64_t bs = a.rp[s_bw[b]], bd = s_bdeg[b];
                            int64_t e = lane64();
                            for (; e + 192 < bd; e += 256) {
                                const int32_t u0 = a.ci[bs + e], u1 = a.ci[bs + e + 64];
                                const int32_t u2 = a.ci[bs + e + 128], u3 = a.ci[bs + e + 192];
                                expand(u0);
                                expand(u1);
                                expand(u2);
                                expand(u3);
                            }
                            for (; e < bd; e += 64) expand(a.ci[bs + e]);
                        }
                        __syncthreads();
                        if (threadIdx.x == 0) s_nbig = 0;
                        __syncthreads();
                    }
                    fb = qstart;
                    fe = s_qtail;
                    from_queue = true;
                    __syncthreads();
                }
            }
            if constexpr (!FILL) {
                const int64_t cnt = block_sum<int64_t, kBfsWaves>(mycount, s_red);
                if (threadIdx.x == 0) a.counts[v] = cnt;
                if (re > rb) {
                    if constexpr (SUMMARY) {
                        for (int i = threadIdx.x; i < (nw + 31) / 32; i += kBfsBlock) {
                            uint32_t t = sm[i];
                            while (t) {
                                bm[i * 32 + __builtin_ctz(t)] = 0u;
                                t &= t - 1u;
                            }
                            sm[i] = 0u;
                        }
                    } else {
                        for (int i = threadIdx.x; i < nw; i += kBfsBlock) bm[i] = 0u;
                    }
                }
            } else {
                if (re > rb) {
                    if (threadIdx.x == 0) {
                        const int64_t lv = v - base;
                        bm[lv >> 5] &= ~(1u << (lv & 31));
                    }
                    __syncthreads();
                    int64_t pos = a.kptr[v];
                    const int64_t end = a.kptr[v + 1];
                    auto emit = [&](int wi, uint32_t word, int64_t& o) {
                        while (word) {
                            const int b = __ffs(word) - 1;
                            const int64_t local = (int64_t)wi * 32 + b;
                            if (o < end) {
                                if (a.kidx16) a.kidx16[o] = (uint16_t)local;
                                else a.kidx[o] = (int32_t)(base + local);
                            }
                            ++o;
                            word &= word - 1u;
                        }
                    };
                    if constexpr (SUMMARY) {
                        // Rounds of kBfsBlock summary words (1024 ids each).  Thread
                        // t counts the ids under summary word t; the non-empty
                        // words are listed with their first output position, then
                        // each half wavefront emits one listed word at a time,
                        // lane h taking bitmap word h of it: ids come out in
                        // order, and a few dense summary words (the hubs, which
                        // most rows reach) are shared by 32 lanes, not walked by
                        // one thread.
                        int32_t* s_lex = s_bdeg;  // offset within the round
                        int32_t* s_lsi = s_bw;
                        const int ns = (nw + 31) / 32;
                        const int half = lane64() >> 5, h = lane64() & 31;
                        for (int s0 = 0; s0 < ns; s0 += kBfsBlock) {
                            const int si = s0 + threadIdx.x;
                            const uint32_t t0 = si < ns ? sm[si] : 0u;
                            int64_t c = 0;
                            for (uint32_t t = t0; t; t &= t - 1u) c += __popc(bm[si * 32 + __builtin_ctz(t)]);
                            if (si < ns) sm[si] = 0u;
                            int64_t total, nlist;
                            const int64_t ex = block_exclusive_scan<int64_t, kBfsWaves>(c, s_red, total);
                            const int64_t li = block_exclusive_scan<int64_t, kBfsWaves>(c > 0 ? 1 : 0, s_red, nlist);
                            if (c > 0) {
                                s_lsi[li] = si;
                                s_lex[li] = (int32_t)ex;
                            }
                            __syncthreads();
                            for (int64_t j = wave_id() * 2 + half; j < nlist; j += 2 * kBfsWaves) {
                                const int wi = s_lsi[j] * 32 + h;
                                const uint32_t word = wi < nw ? bm[wi] : 0u;
                                // exclusive prefix of the popcounts over the half
                                const int32_t cnt = __popc(word);
                                int32_t inc = cnt;
#pragma unroll
                                for (int off = 1; off < 32; off <<= 1) {
                                    const int32_t y = __shfl_up(inc, off, 32);
                                    if (h >= off) inc += y;
                                }
                                int64_t o = pos + s_lex[j] + (inc - cnt);
                                emit(wi, word, o);
                                if (wi < nw) bm[wi] = 0u;
                            }
                            pos += total;
                            __syncthreads();
                        }
                    } else {
                        for (int w0 = 0; w0 < nw; w0 += kBfsBlock) {
                            const int wi = w0 + threadIdx.x;
                            const uint32_t word = wi < nw ? bm[wi] : 0u;
                            int64_t total;
                            const int64_t ex =
                                block_exclusive_scan<int64_t, kBfsWaves>((int64_t)__popc(word), s_red, total);
                            int64_t o = pos + ex;
                            emit(wi, word, o);
                            if (wi < nw) bm[wi] = 0u;
                            pos += total;
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ relabelling
// Internal row i is caller row perm[i] with every id mapped through iperm.
__global__ __launch_bounds__(kBlock) void relabel_csr_kernel(
    int32_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ iperm,
    const int64_t* __restrict__ rp_in, const int32_t* __restrict__ ci_in,
    const int64_t* __restrict__ rp_out, int32_t* __restrict__ ci_out) {
    // one wavefront per row
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
    for (int64_t i = wave; i < n; i += nw) {
        const int32_t src = perm[i];
        const int64_t b = rp_in[src], e = rp_in[src + 1], o = rp_out[i];
        for (int64_t j = b + lane64(); j < e; j += 64) ci_out[o + (j - b)] = iperm[ci_in[j]];
    }
}

__global__ void reset_counter_kernel(int32_t* c) { *c = 0; }

int launch_validate_csr(int32_t n, int64_t nnz, const int64_t* rp, const int32_t* ci, int32_t* flag,
                        hipStream_t s) {
    if (nnz <= 0) return GILA_OK;
    const int grid = (int)std::min<int64_t>(4096, (nnz + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(validate_csr_kernel, dim3(grid), dim3(kBlock), 0, s, n, nnz, rp, ci, flag,
                       0, (unsigned long long*)nullptr);
    GILA_HIP(hipGetLastError());
    return GILA_OK;
}

// Host checks of the row pointers and the device check of every entry of a
// caller's CSR (the rules of gila_csr).  Synchronises `s`.
int validate_graph(const gila_csr* g, hipStream_t s) {
    if (!g) return fail(GILA_EINVAL, "graph is NULL");
    if (g->n < 0 || g->nnz < 0) return fail(GILA_EINVAL, "negative n or nnz");
    if (g->n > 0 && !g->row_ptr) return fail(GILA_EINVAL, "row_ptr is NULL");
    if (g->nnz > 0 && !g->col_idx) return fail(GILA_EINVAL, "col_idx is NULL");
    if (g->nnz > (int64_t)g->n * (int64_t)(g->n > 0 ? g->n - 1 : 0))
        return fail(GILA_EINVAL, "nnz exceeds n(n-1)");
    if (g->n == 0) return GILA_OK;
    std::vector<int64_t> rp((size_t)g->n + 1);
    GILA_HIP(hipMemcpyAsync(rp.data(), g->row_ptr, sizeof(int64_t) * rp.size(),
                            hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    if (rp[0] != 0 || rp[g->n] != g->nnz)
        return fail(GILA_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    for (int32_t v = 0; v < g->n; ++v)
        if (rp[v + 1] < rp[v]) return fail(GILA_EINVAL, "row_ptr not monotone");
    if (g->nnz % 2) return fail(GILA_EINVAL, "nnz must be even for a symmetric CSR");
    if (g->nnz == 0) return GILA_OK;
    int32_t* d_flag = nullptr;
    GILA_TRY(dalloc_t(&d_flag, 1));
    int rc = GILA_OK;
    int32_t flag = 0;
    hipError_t e = hipMemsetAsync(d_flag, 0, sizeof(int32_t), s);
    if (e == hipSuccess) {
        rc = launch_validate_csr(g->n, g->nnz, g->row_ptr, g->col_idx, d_flag, s);
        if (rc == GILA_OK) {
            e = hipMemcpyAsync(&flag, d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
    }
    dfree_on(d_flag, s);
    if (rc != GILA_OK) return rc;
    if (e != hipSuccess) return fail(GILA_EDEVICE, "validation: %s", hipGetErrorString(e));
    if (flag)
        return fail(GILA_EINVAL, "malformed CSR:%s%s%s%s", (flag & 1) ? " column out of range" : "",
                    (flag & 2) ? " self-loop" : "", (flag & 4) ? " row not strictly ascending" : "",
                    (flag & 8) ? " not symmetric" : "");
    return GILA_OK;
}

int run_bfs(bool fill, int device, hipStream_t s, BfsArgs a) {
    const DeviceInfo& di = device_info(device);
    // LDS bitmap: one bit per vertex id plus the summary (one bit per word)
    const size_t bm_bytes = ((size_t)a.nwords + ((size_t)a.nwords + 31) / 32) * 4;
    // (GILA_BFS_BITMAP=global takes the global-memory bitmap whatever n is)
    const char* bm_env = getenv("GILA_BFS_BITMAP");
    const bool lds = bm_bytes + 8 * 1024 * 2 + 1024 <= di.max_lds_per_block &&
                     !(bm_env && std::strcmp(bm_env, "global") == 0);
    // Workgroup shape.  256 threads while the LDS lets 8 such workgroups
    // share a CU (32 wavefronts); larger bitmaps (more than ~2^17 ids) take
    // 512-thread workgroups, at most 4 per CU, so that 32 wavefronts per CU
    // still keep the frontier's scattered row reads in flight.  The k = 1
    // pass (short rows, no expansion) keeps 256.  Static LDS: the long-row
    // lists (8 bytes per thread) and a few words.
    const int32_t kmax = a.gvbase ? a.kmax : a.k;
    auto fit = [&](int bs) {
        const size_t per = bm_bytes + 8 * (size_t)bs + 256;
        return (int)std::max<size_t>(1, std::min<size_t>(2048 / bs, (160u * 1024u) / per));
    };
    int bs = 256;
    int per_cu = 8;
    if (lds) {
        per_cu = fit(256);
        if (per_cu < 8 && kmax >= 2) {
            bs = 512;
            per_cu = fit(512);
        }
    }
    int grid = di.cus * per_cu;
    if (a.nverts < grid) grid = std::max(1, a.nverts);
    if (kmax >= 3) {
        // frontier queues: one graph's vertex count per workgroup (the
        // largest graph in batch mode), capped at ~1 GiB in total
        const int64_t qn = a.qcap > 0 ? a.qcap : std::max<int32_t>(1, a.n);
        const int64_t cap_grid = std::max<int64_t>(64, (1ll << 30) / std::max<int64_t>(1, 4ll * qn));
        grid = (int)std::min<int64_t>(grid, cap_grid);
        a.qcap = qn;
        GILA_TRY(dalloc_t(&a.queue, (size_t)grid * a.qcap));
    } else {
        a.queue = nullptr;
        a.qcap = 0;
    }
    a.gbitmap = nullptr;
    if (!lds) {
        int rc = dalloc_t(&a.gbitmap, (size_t)grid * a.nwords);
        if (rc) {
            dfree_on(a.queue, s);
            return rc;
        }
    }
    int rc = GILA_OK;
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, a.work);
    const size_t shm = lds ? bm_bytes : 0;
    auto launch = [&](auto kernel, int threads) {
        if (shm > 65536)
            (void)quiet(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)shm));
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), shm, s, a);
    };
    if (bs == 512) {
        if (fill) launch(khop_bfs_kernel<512, true, true>, 512);
        else launch(khop_bfs_kernel<512, false, true>, 512);
    } else if (lds) {
        if (fill) launch(khop_bfs_kernel<256, true, true>, 256);
        else launch(khop_bfs_kernel<256, false, true>, 256);
    } else {
        if (fill) launch(khop_bfs_kernel<256, true, false>, 256);
        else launch(khop_bfs_kernel<256, false, false>, 256);
    }
    e = hipGetLastError();
    if (e != hipSuccess) rc = fail(GILA_EDEVICE, "k-hop kernel launch: %s", hipGetErrorString(e));
    // scratch is freed after the work on the stream is done
    hipError_t se = hipStreamSynchronize(s);
    if (rc == GILA_OK && se != hipSuccess)
        rc = fail(GILA_EDEVICE, "k-hop kernel: %s", hipGetErrorString(se));
    dfree_on(a.queue, s);
    dfree_on(a.gbitmap, s);
    return rc;
}

void free_khop(gila_khop* kh, Release rel) {
    if (!kh) return;
    DeviceGuard g(kh->device);
    if (kh->gexec) (void)quiet(hipGraphExecDestroy(kh->gexec));
    if (kh->tick_exec) (void)quiet(hipGraphExecDestroy(kh->tick_exec));
    if (kh->chunk_exec) (void)quiet(hipGraphExecDestroy(kh->chunk_exec));
    rel(kh->d_temps);
    rel(kh->perm);
    rel(kh->iperm);
    rel(kh->rp);
    rel(kh->ci);
    rel(kh->kptr);
    rel(kh->kidx);
    rel(kh->block_start);
    rel(kh->pos[0]);
    rel(kh->pos[1]);
    rel(kh->partials);
    rel(kh->ctl);
    rel(kh->hist);
    rel(kh->mass64);
    rel(kh->mass32);
    free_segments(kh, rel);
    delete kh;
}

struct KhopHolder {
    gila_khop* p;
    ~KhopHolder() { free_khop(p); }
};

// ------------------------------------------------------------------ repulsion weights
// Caller-order weights -> internal order, in double and float; flags any
// weight outside [0, kMaxWeight] (NaN included).
static constexpr double kMaxWeight = 1e30;

__global__ __launch_bounds__(kBlock) void weights_in_kernel(int32_t n, const int32_t* __restrict__ perm,
                                                            const double* __restrict__ src,
                                                            double* __restrict__ w64,
                                                            float* __restrict__ w32,
                                                            int32_t* __restrict__ flag) {
    int32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double w = src[perm[i]];
        if (!(w >= 0.0 && w <= kMaxWeight)) bad = 1;
        w64[i] = w;
        w32[i] = (float)w;
    }
    if (bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ internal vertex order
// Edges shorter than this in the caller's order count as local.
static constexpr int32_t kLocalWindow = 1024;

// The caller's order is kept when most edges are local (meshes, rings, road
// networks numbered along the graph): neighbourhoods then fall into few
// segments of the iteration kernel.  Otherwise rows are sorted by length.
// GILA_ORDER=degree|caller overrides the choice.
static bool use_caller_order(unsigned long long near_edges, int64_t nnz) {
    const char* e = getenv("GILA_ORDER");
    if (e && std::strcmp(e, "degree") == 0) return false;
    if (e && std::strcmp(e, "caller") == 0) return true;
    return nnz > 0 && (double)near_edges >= 0.7 * (double)nnz;
}

// Sort key of each caller vertex; the internal order is the ascending order
// of the keys, equal keys by ascending caller id.  Degree order: |N_v(k)|
// descending (n - 1 - |N_v(k)|), isolated vertices last (n).  Caller order:
// rows of at least hub_min entries (0), then the other non-isolated vertices
// (1), then the isolated ones (2).
__global__ __launch_bounds__(kBlock) void order_key_kernel(int32_t n, const int64_t* __restrict__ rp,
                                                           const int64_t* __restrict__ counts,
                                                           int32_t caller_order, int64_t hub_min,
                                                           uint32_t* __restrict__ key) {
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * kBlock) {
        const bool isolated = rp[v + 1] == rp[v];
        const int64_t c = counts[v];
        uint32_t kv;
        if (caller_order) kv = isolated ? 2u : (c >= hub_min ? 0u : 1u);
        else kv = isolated ? (uint32_t)n : (uint32_t)(n - 1 - c);
        key[v] = kv;
    }
}

// Internal vertex i = caller vertex perm[i]: the inverse permutation and the
// degree and list length of each internal row (their exclusive sums are the
// internal row pointers and list offsets).
__global__ __launch_bounds__(kBlock) void internal_rows_kernel(
    int32_t n, const int32_t* __restrict__ perm, const int64_t* __restrict__ rp,
    const int64_t* __restrict__ counts, int32_t* __restrict__ iperm, int64_t* __restrict__ deg,
    int64_t* __restrict__ cnt) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const int32_t v = perm[i];
        iperm[v] = (int32_t)i;
        deg[i] = rp[v + 1] - rp[v];
        cnt[i] = counts[v];
    }
}

int build_khop(const gila_csr* g, int32_t k, hipStream_t s, gila_khop** out) {
    if (!out) return fail(GILA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(GILA_EINVAL, "graph is NULL");
    if (k < 1) return fail(GILA_EINVAL, "k must be >= 1 (got %d)", k);
    if (g->n < 0 || g->nnz < 0) return fail(GILA_EINVAL, "negative n or nnz");
    if (g->n > 0 && !g->row_ptr) return fail(GILA_EINVAL, "row_ptr is NULL");
    if (g->nnz > 0 && !g->col_idx) return fail(GILA_EINVAL, "col_idx is NULL");
    if (g->nnz > (int64_t)g->n * (int64_t)(g->n > 0 ? g->n - 1 : 0))
        return fail(GILA_EINVAL, "nnz exceeds n(n-1)");
    int dev = 0;
    GILA_HIP(hipGetDevice(&dev));
    const int32_t n = g->n;
    const int64_t nnz = g->nnz;
    PhaseTimer pt("build_khop", s);

    KhopHolder h{new gila_khop()};
    gila_khop* kh = h.p;
    kh->device = dev;
    kh->n = n;
    kh->k = k;
    kh->nnz = nnz;

    // --- row pointers on the host: monotone, 0 .. nnz
    std::vector<int64_t> rp_host((size_t)n + 1, 0);
    if (n > 0) {
        GILA_HIP(hipMemcpyAsync(rp_host.data(), g->row_ptr, sizeof(int64_t) * (n + 1),
                                hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        if (rp_host[0] != 0 || rp_host[n] != nnz)
            return fail(GILA_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
        int32_t bad = -1, active = 0;
        for (int32_t v = 0; v < n; ++v) {
            const int64_t d = rp_host[v + 1] - rp_host[v];
            bad = (d < 0 && bad < 0) ? v : bad;
            active += d > 0 ? 1 : 0;
        }
        if (bad >= 0) return fail(GILA_EINVAL, "row_ptr not monotone");
        kh->n_active = active;
        if (nnz % 2) return fail(GILA_EINVAL, "nnz must be even for a symmetric CSR");
    }

    pt.mark("rowptr");
    // --- device validation of every entry
    // d_flag[0]: validation flags, d_flag[1]: BFS work counter,
    // d_flag[2..3]: number of short edges (caller's order)
    int32_t* d_flag = nullptr;
    int32_t* d_work = nullptr;
    GILA_TRY(dalloc_t(&d_flag, 4));
    struct F {
        int32_t* p;
        hipStream_t s;
        ~F() { dfree_on(p, s); }
    } fguard{d_flag, s};
    d_work = d_flag + 1;
    unsigned long long* d_near = reinterpret_cast<unsigned long long*>(d_flag + 2);
    GILA_HIP(hipMemsetAsync(d_flag, 0, 4 * sizeof(int32_t), s));
    if (nnz > 0) {
        const int grid = (int)std::min<int64_t>(4096, (nnz + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(validate_csr_kernel, dim3(grid), dim3(kBlock), 0, s, n, nnz,
                           g->row_ptr, g->col_idx, d_flag, kLocalWindow, d_near);
        GILA_HIP(hipGetLastError());
    }
    int32_t hflag[4] = {0, 0, 0, 0};
    GILA_HIP(hipMemcpyAsync(hflag, d_flag, sizeof(hflag), hipMemcpyDeviceToHost, s));
    GILA_HIP(hipStreamSynchronize(s));
    const int32_t flag = hflag[0];
    unsigned long long near_edges = 0;
    std::memcpy(&near_edges, &hflag[2], sizeof(near_edges));
    if (flag) {
        return fail(GILA_EINVAL, "malformed CSR:%s%s%s%s", (flag & 1) ? " column out of range" : "",
                    (flag & 2) ? " self-loop" : "", (flag & 4) ? " row not strictly ascending" : "",
                    (flag & 8) ? " not symmetric" : "");
    }

    pt.mark("validate");
    // --- count pass on the caller's graph
    const int32_t nwords = (n + 31) / 32;
    int64_t* d_counts = nullptr;
    GILA_TRY(dalloc_t(&d_counts, (size_t)std::max(n, 1)));
    struct C {
        int64_t* p;
        hipStream_t s;
        ~C() { dfree_on(p, s); }
    } cguard{d_counts, s};
    if (n > 0) {
        BfsArgs a{};
        a.n = n;
        a.k = k;
        a.nverts = n;
        a.nwords = nwords;
        a.rp = g->row_ptr;
        a.ci = g->col_idx;
        a.counts = d_counts;
        a.work = d_work;
        GILA_TRY(run_bfs(false, dev, s, a));
    }

    pt.mark("count");
    // --- internal order (non-isolated vertices first), its graph and list
    // offsets, all on the device
    kh->caller_order = use_caller_order(near_edges, nnz);
    GILA_TRY(dalloc_t(&kh->perm, (size_t)n));
    GILA_TRY(dalloc_t(&kh->iperm, (size_t)n));
    GILA_TRY(dalloc_t(&kh->rp, (size_t)n + 1));
    GILA_TRY(dalloc_t(&kh->ci, (size_t)nnz));
    GILA_TRY(dalloc_t(&kh->kptr, (size_t)n + 1));
    int64_t P = 0;
    if (n > 0) {
        struct T {
            void* p = nullptr;
            hipStream_t s;
            ~T() { dfree_on(p, s); }
        } key{nullptr, s}, deg{nullptr, s}, cnt{nullptr, s}, ws{nullptr, s};
        GILA_TRY(dalloc_t(reinterpret_cast<uint32_t**>(&key.p), (size_t)n));
        GILA_TRY(dalloc_t(reinterpret_cast<int64_t**>(&deg.p), (size_t)n));
        GILA_TRY(dalloc_t(reinterpret_cast<int64_t**>(&cnt.p), (size_t)n));
        GILA_TRY(dalloc_t(reinterpret_cast<int64_t**>(&ws.p), (size_t)scan_workspace_count(n)));
        const unsigned grid = (unsigned)std::min<int64_t>(4096, ((int64_t)n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(order_key_kernel, dim3(grid), dim3(kBlock), 0, s, n, g->row_ptr,
                           d_counts, (int32_t)kh->caller_order, kHubMin,
                           static_cast<uint32_t*>(key.p));
        GILA_HIP(hipGetLastError());
        const uint32_t max_key = kh->caller_order ? 2u : (uint32_t)n;
        GILA_TRY(stable_order_by_key(n, static_cast<const uint32_t*>(key.p), max_key, kh->perm, s));
        hipLaunchKernelGGL(internal_rows_kernel, dim3(grid), dim3(kBlock), 0, s, n, kh->perm,
                           g->row_ptr, d_counts, kh->iperm, static_cast<int64_t*>(deg.p),
                           static_cast<int64_t*>(cnt.p));
        GILA_HIP(hipGetLastError());
        int64_t* sws = static_cast<int64_t*>(ws.p);
        GILA_TRY(enqueue_exclusive_scan_i64(static_cast<int64_t*>(deg.p), kh->rp, n, sws, s));
        GILA_TRY(enqueue_exclusive_scan_i64(static_cast<int64_t*>(cnt.p), kh->kptr, n, sws, s));
        int64_t tail[2] = {0, 0};
        GILA_HIP(hipMemcpyAsync(&tail[0], kh->kptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipMemcpyAsync(&tail[1], kh->rp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GILA_HIP(hipStreamSynchronize(s));
        if (tail[1] != nnz) return fail(GILA_EDEVICE, "internal row pointers do not sum to nnz");
        P = tail[0];
    }
    kh->P = P;
    GILA_TRY(dalloc_t(&kh->kidx, (size_t)P));

    pt.mark("order");
    const int32_t n_active = kh->n_active;
    // --- internal graph copy
    if (n > 0 && nnz > 0) {
        const int grid = (int)std::min<int64_t>(8192, ((int64_t)n * 64 + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(relabel_csr_kernel, dim3(grid), dim3(kBlock), 0, s, n, kh->perm,
                           kh->iperm, g->row_ptr, g->col_idx, kh->rp, kh->ci);
        GILA_HIP(hipGetLastError());
    }

    pt.mark("relabel");
    // --- internal adjacency rows in ascending order (a k = 1 fill pass)
    if (n_active > 0 && nnz > 0) {
        int32_t* ci_sorted = nullptr;
        GILA_TRY(dalloc_t(&ci_sorted, (size_t)nnz));
        BfsArgs a{};
        a.n = n;
        a.k = 1;
        a.nverts = n_active;
        a.nwords = nwords;
        a.rp = kh->rp;
        a.ci = kh->ci;
        a.kptr = kh->rp;
        a.kidx = ci_sorted;
        a.work = d_work;
        const int rc = run_bfs(true, dev, s, a);
        if (rc) {
            dfree_on(ci_sorted, s);
            return rc;
        }
        dfree_on(kh->ci, s);
        kh->ci = ci_sorted;
    }

    pt.mark("sort_adj");
    // --- fill pass on the internal graph (rows come out ascending)
    if (n_active > 0 && P > 0) {
        BfsArgs a{};
        a.n = n;
        a.k = k;
        a.nverts = n_active;
        a.nwords = nwords;
        a.rp = kh->rp;
        a.ci = kh->ci;
        a.kptr = kh->kptr;
        a.kidx = kh->kidx;
        a.work = d_work;
        GILA_TRY(run_bfs(true, dev, s, a));
    }

    pt.mark("fill");
    // --- iteration workspace (the direct path's plan and partials are made
    // on its first use)
    GILA_TRY(dalloc_t(reinterpret_cast<double**>(&kh->pos[0]), 2 * (size_t)std::max(n, 1)));
    GILA_TRY(dalloc_t(reinterpret_cast<double**>(&kh->pos[1]), 2 * (size_t)std::max(n, 1)));
    GILA_TRY(dalloc_t(&kh->ctl, 1));
    GILA_HIP(hipMemsetAsync(kh->ctl, 0, sizeof(Ctl), s));
    GILA_HIP(hipStreamSynchronize(s));
    // segment-blocked lists for FP32 positions (the common case); FP64 runs
    // rebuild them for their own segment size on first use
    pt.mark("plan");
    if (segment_path_enabled()) {
        const int src = build_segments(kh, GILA_FP32_KAHAN, s);
        if (src != GILA_OK && src != GILA_EUNSUPPORTED) return src;
        clear_error();
    }
    kh->device_bytes = (int64_t)sizeof(int32_t) * 2 * n + sizeof(int64_t) * 2 * (n + 1) +
                       sizeof(int32_t) * (nnz + P) + 32 * (int64_t)n +
                       (int64_t)sizeof(Partial) * kh->partials_cap;
    *out = kh;
    h.p = nullptr;
    return GILA_OK;
}

}  // namespace gila

using namespace gila;

extern "C" {

int gila_build_khop(const gila_csr* g_dev, int32_t k, void* stream, gila_khop** out) {
    clear_error();
    return build_khop(g_dev, k, (hipStream_t)stream, out);
}

int gila_khop_info(const gila_khop* kh, int32_t* n, int32_t* k, int64_t* total_pairs,
                   int32_t* n_active, int64_t* device_bytes) {
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    if (n) *n = kh->n;
    if (k) *k = kh->k;
    if (total_pairs) *total_pairs = kh->P;
    if (n_active) *n_active = kh->n_active;
    if (device_bytes) *device_bytes = kh->device_bytes;
    return GILA_OK;
}

int gila_khop_order(const gila_khop* kh, int32_t* order_host) {
    clear_error();
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    if (!order_host) return fail(GILA_EINVAL, "order_host is NULL");
    if (kh->n == 0) return GILA_OK;
    DeviceGuard dg(kh->device);
    GILA_HIP(hipMemcpy(order_host, kh->perm, sizeof(int32_t) * kh->n, hipMemcpyDeviceToHost));
    return GILA_OK;
}

int gila_khop_export_rows(const gila_khop* kh, int64_t count, const int32_t* verts_host,
                          int64_t* ptr_host, int32_t* idx_host) {
    clear_error();
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    if (count < 0 || (count > 0 && !verts_host)) return fail(GILA_EINVAL, "bad vertex list");
    if (!ptr_host) return fail(GILA_EINVAL, "ptr_host is NULL");
    DeviceGuard dg(kh->device);
    const int32_t n = kh->n;
    std::vector<int64_t> kptr((size_t)n + 1);
    std::vector<int32_t> perm((size_t)n), iperm((size_t)n);
    GILA_HIP(hipMemcpy(kptr.data(), kh->kptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    GILA_HIP(hipMemcpy(perm.data(), kh->perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    GILA_HIP(hipMemcpy(iperm.data(), kh->iperm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    ptr_host[0] = 0;
    for (int64_t i = 0; i < count; ++i) {
        const int32_t v = verts_host[i];
        if (v < 0 || v >= n) return fail(GILA_EINVAL, "vertex %d out of range", v);
        const int32_t r = iperm[v];
        ptr_host[i + 1] = ptr_host[i] + (kptr[r + 1] - kptr[r]);
    }
    if (!idx_host) return GILA_OK;
    for (int64_t i = 0; i < count; ++i) {
        const int32_t r = iperm[verts_host[i]];
        const int64_t len = kptr[r + 1] - kptr[r];
        int32_t* dst = idx_host + ptr_host[i];
        if (len > 0)
            GILA_HIP(hipMemcpy(dst, kh->kidx + kptr[r], sizeof(int32_t) * len,
                               hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < len; ++j) dst[j] = perm[dst[j]];
        std::sort(dst, dst + len);
    }
    return GILA_OK;
}

int gila_khop_export(const gila_khop* kh, int64_t* ptr_host, int32_t* idx_host) {
    clear_error();
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    DeviceGuard dg(kh->device);
    const int32_t n = kh->n;
    std::vector<int64_t> kptr((size_t)n + 1);
    std::vector<int32_t> perm((size_t)n), iperm((size_t)n);
    GILA_HIP(hipMemcpy(kptr.data(), kh->kptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    GILA_HIP(hipMemcpy(perm.data(), kh->perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    GILA_HIP(hipMemcpy(iperm.data(), kh->iperm, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    std::vector<int64_t> ptr((size_t)n + 1, 0);
    for (int32_t v = 0; v < n; ++v) {
        const int32_t r = iperm[v];
        ptr[v + 1] = ptr[v] + (kptr[r + 1] - kptr[r]);
    }
    if (ptr_host) std::memcpy(ptr_host, ptr.data(), sizeof(int64_t) * (n + 1));
    if (!idx_host) return GILA_OK;
    std::vector<int32_t> all((size_t)kh->P);
    if (kh->P > 0)
        GILA_HIP(hipMemcpy(all.data(), kh->kidx, sizeof(int32_t) * kh->P, hipMemcpyDeviceToHost));
    for (int32_t v = 0; v < n; ++v) {
        const int32_t r = iperm[v];
        int32_t* dst = idx_host + ptr[v];
        const int64_t len = kptr[r + 1] - kptr[r];
        for (int64_t j = 0; j < len; ++j) dst[j] = perm[all[kptr[r] + j]];
        std::sort(dst, dst + len);
    }
    return GILA_OK;
}

int gila_khop_set_mass(gila_khop* kh, const double* mass_dev, void* stream) {
    clear_error();
    if (!kh) return fail(GILA_EINVAL, "handle is NULL");
    std::lock_guard<std::mutex> lk(kh->mu);
    DeviceGuard dg(kh->device);
    hipStream_t s = (hipStream_t)stream;
    if (mass_dev && kh->n > 0) {
        const int32_t n = kh->n;
        double* w64 = nullptr;
        float* w32 = nullptr;
        int32_t* d_flag = nullptr;
        int rc = dalloc_t(&w64, (size_t)n);
        if (rc == GILA_OK) rc = dalloc_t(&w32, (size_t)n);
        if (rc == GILA_OK) rc = dalloc_t(&d_flag, 1);
        int32_t flag = 0;
        if (rc == GILA_OK) {
            hipError_t e = hipMemsetAsync(d_flag, 0, sizeof(int32_t), s);
            if (e == hipSuccess) {
                const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kBlock - 1) / kBlock));
                hipLaunchKernelGGL(weights_in_kernel, dim3(grid), dim3(kBlock), 0, s, n, kh->perm,
                                   mass_dev, w64, w32, d_flag);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipMemcpyAsync(&flag, d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) rc = fail(GILA_EDEVICE, "weights: %s", hipGetErrorString(e));
            else if (flag) rc = fail(GILA_EINVAL, "every weight must lie in [0, 1e30]");
        }
        dfree_on(d_flag, s);
        if (rc != GILA_OK) {
            dfree_on(w64, s);
            dfree_on(w32, s);
            return rc;
        }
        if (!kh->mass64) kh->device_bytes += 12 * (int64_t)n;
        dfree_on(kh->mass64, s);
        dfree_on(kh->mass32, s);
        kh->mass64 = w64;
        kh->mass32 = w32;
    } else if (kh->mass64) {
        dfree_on(kh->mass64, s);
        dfree_on(kh->mass32, s);
        kh->mass64 = nullptr;
        kh->mass32 = nullptr;
        kh->device_bytes -= 12 * (int64_t)kh->n;
    }
    // the captured loops hold the previous kernels and arguments
    drop_graphs(kh);
    return GILA_OK;
}

void gila_khop_free(gila_khop* kh) {
    if (!kh) return;
    DeviceGuard g(kh->device);
    free_khop(kh, public_release());
}

}  // extern "C"

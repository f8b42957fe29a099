// Device helpers shared by libgila kernels: wavefront and workgroup scans and
// reductions for 64-wide wavefronts and 256-thread workgroups.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gila {

__device__ __forceinline__ int lane64() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Inclusive prefix sum across the 64 lanes of a wavefront.
template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = lane64();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive prefix sum over a workgroup of NW wavefronts (256 threads by
// default).  `sh` is LDS scratch of at least NW elements.  Contains two
// barriers; every thread must call it.
template <class T, int NW = 4>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sh, T& total) {
    const int w = wave_id();
    T inc = wave_inclusive_scan(v);
    if (lane64() == 63) sh[w] = inc;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        T s = sh[i];
        before += (i < w) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

// Sum over a workgroup of NW wavefronts (256 threads by default) in a fixed
// order (butterfly within each wavefront, then wavefronts 0..NW-1 in order).
// Result valid in every thread.
template <class T, int NW = 4>
__device__ __forceinline__ T block_sum(T v, T* sh) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane64() == 0) sh[wave_id()] = v;
    __syncthreads();
    T r = sh[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r += sh[i];
    __syncthreads();
    return r;
}

// Fixed-order butterfly sum over aligned groups of G lanes (G a power of two
// <= 64).  Every lane of a group ends with the same bits.
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    return group_sum<64>(v);
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

}  // namespace gila

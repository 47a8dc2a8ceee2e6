// Wave64 / workgroup primitives for gfx950 (CDNA4): ballots, lane prefix
// counts, inclusive scans over a wave and over a 256-thread workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pg {

__device__ inline int lane_id() { return (int)__lane_id(); }

// Number of set bits of `mask` at lanes below the calling lane.
__device__ inline uint32_t lane_prefix(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

// Orders the LDS accesses of the lanes of one wave around this point: the
// compiler may neither move memory operations across it nor assume LDS still
// holds what this lane last wrote (other lanes' writes before it are seen).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ inline T wave_incl_scan(T v) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T o = __shfl_up(v, off, kWave);
        if (lane_id() >= off) v += o;
    }
    return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        uint32_t o = __shfl_xor(v, off, kWave);
        v = o < v ? o : v;
    }
    return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        uint32_t o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Exclusive scan over a workgroup of NT threads (NT a multiple of 64);
// `lds` holds NT/64 + 1 entries.  Returns the exclusive prefix and writes the
// workgroup total to *total.  Contains barriers: call from every thread.
template <int NT, typename T>
__device__ inline T block_excl_scan(T v, T* lds, T* total) {
    constexpr int NW = NT / kWave;
    const int w = threadIdx.x / kWave;
    T inc = wave_incl_scan(v);
    if (lane_id() == kWave - 1) lds[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < NW; i++) { T t = lds[i]; lds[i] = run; run += t; }
        lds[NW] = run;
    }
    __syncthreads();
    T res = inc - v + lds[w];
    *total = lds[NW];
    __syncthreads();
    return res;
}

}  // namespace pg

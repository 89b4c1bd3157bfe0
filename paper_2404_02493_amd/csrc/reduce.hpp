// Block reductions and the deterministic "last block finishes" grid reduction.
#pragma once

#include "common.hpp"

namespace helm {

constexpr int BLOCK = 256;  // threads per block of every kernel (4 wavefronts of 64)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Reduce K per-thread accumulators over the block; thread 0 receives the sums in out[].
// red: LDS scratch of at least 4*K doubles.
template <int K>
__device__ __forceinline__ void block_sum(const double (&acc)[K], int kcount, double* red, double* out) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int v = 0; v < K; ++v) {
        if (v < kcount) {
            double s = wave_sum(acc[v]);
            if (lane == 0) red[wave * K + v] = s;
        }
    }
    __syncthreads();
    if (tid == 0) {
        for (int v = 0; v < kcount; ++v) out[v] = red[v] + red[K + v] + red[2 * K + v] + red[3 * K + v];
    }
    __syncthreads();
}

// Writes this block's K sums to partials[block*kcount + v] and takes a ticket.
// Returns true in every thread of the last block to finish; that block then sees
// every partial (release/acquire at device scope).  Deterministic: the final sum
// is formed by grid_final_sum in a fixed order.
template <int K>
__device__ __forceinline__ bool block_partials_and_ticket(const double (&acc)[K], int kcount, double* partials,
                                                          unsigned int* ticket, double* red, double* sums,
                                                          int* is_last) {
    block_sum<K>(acc, kcount, red, sums);
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nblk = gridDim.x * gridDim.y;
    const int blk = blockIdx.x + blockIdx.y * gridDim.x;
    if (tid == 0) {
        for (int v = 0; v < kcount; ++v) partials[(size_t)blk * kcount + v] = sums[v];
        __threadfence();
        unsigned int t = atomicAdd(ticket, 1u);
        *is_last = (t == (unsigned)(nblk - 1));
    }
    __syncthreads();
    bool last = *is_last != 0;
    if (last) __threadfence();
    return last;
}

// Called by every thread of the last block: sums[v] = sum over blocks of partials (fixed order).
template <int K>
__device__ __forceinline__ void grid_final_sum(const double* partials, int kcount, double* red, double* sums,
                                               unsigned int* ticket) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nblk = gridDim.x * gridDim.y;
    double acc[K];
#pragma unroll
    for (int v = 0; v < K; ++v) acc[v] = 0.0;
    for (int b = tid; b < nblk; b += BLOCK) {
        const volatile double* p = partials + (size_t)b * kcount;
#pragma unroll
        for (int v = 0; v < K; ++v)
            if (v < kcount) acc[v] += p[v];
    }
    block_sum<K>(acc, kcount, red, sums);
    if (tid == 0) *ticket = 0u;
}

}  // namespace helm

// Block reductions.  Grid reductions are two-kernel: every block stores its
// partial sums (plain stores, layout partials[v * nblk + block]) and a one-block
// finalize kernel sums them in a fixed order.  There is no cross-block
// synchronisation inside a kernel.
#pragma once

#include "common.hpp"

namespace helm {

constexpr int BLOCK = 256;     // threads per block of the grid kernels (4 wavefronts of 64)
constexpr int FBLOCK = 1024;   // threads of the one-block finalize kernels
constexpr int MAXRED = 2048;   // at most this many blocks in a kernel that produces partials

// v moved by the DPP control CTRL within the rows selected by RM; lanes without a
// source (and rows outside RM) receive 0.
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ double dpp_move(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, RM, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, RM, 0xF, false);
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes (all active), returned to every lane.  Scans of each row of 16
// lanes (row_shr 1, 2, 4, 8), then the row totals carried by row_bcast 15 and 31, so lane
// 63 ends with the sum (a fixed order; measured about 2 us less than a butterfly of
// lane shuffles for 16 sums at the end of a 1924-wavefront kernel).
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0x111>(v);       // row_shr:1
    v += dpp_move<0x112>(v);       // row_shr:2
    v += dpp_move<0x114>(v);       // row_shr:4
    v += dpp_move<0x118>(v);       // row_shr:8
    v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)u, 63), hi = __builtin_amdgcn_readlane((int)(u >> 32), 63);
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Reduce K per-thread accumulators over the block (any size up to 1024 threads);
// thread 0 receives the sums in out[] (LDS).  red: LDS scratch of NW*K doubles,
// NW = number of wavefronts of the block.
template <int K, int NW>
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
    if (tid < kcount) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += red[w * K + tid];
        out[tid] = s;
    }
    __syncthreads();
}

// Stores this block's kcount sums (after block_sum) to partials[v * nblk + block].
__device__ __forceinline__ void store_partials(const double* sums, int kcount, double* partials) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nblk = gridDim.x;
    if (tid < kcount) partials[(size_t)tid * nblk + blockIdx.x] = sums[tid];
}

// In a one-block finalize kernel of FBLOCK threads: sums[v] = sum over blocks of
// partials[v * nblk + b], v < kcount, fixed order; result in LDS sums[] for all threads.
template <int K>
__device__ __forceinline__ void final_sum(const double* __restrict__ partials, int nblk, int kcount, double* red,
                                          double* sums) {
    double acc[K];
#pragma unroll
    for (int v = 0; v < K; ++v) acc[v] = 0.0;
    const int tid = threadIdx.x;
    for (int b = tid; b < nblk; b += FBLOCK) {
#pragma unroll
        for (int v = 0; v < K; ++v)
            if (v < kcount) acc[v] += partials[(size_t)v * nblk + b];
    }
    block_sum<K, FBLOCK / 64>(acc, kcount, red, sums);
}

}  // namespace helm

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

// Sum of row[0 .. nblk) in a fixed order, returned to every lane of the calling wavefront:
// lane l of group g (g = 0..15) adds blocks 64 g + l, 64 g + l + FBLOCK, ...; each group is
// summed over its lanes (wave_sum) and the group sums are added for g = 0, 1, ...  Only the
// groups that hold blocks are reduced; the sums are bit-identical to those of a block
// reduction over FBLOCK threads (one group per wavefront) in the same order.
__device__ __forceinline__ double group_row_sum(const double* __restrict__ row, int nblk, int lane) {
    constexpr int NW = FBLOCK / 64;
    const int ng = (nblk + 63) / 64 < NW ? (nblk + 63) / 64 : NW;  // groups holding blocks
    double t[NW];
#pragma unroll
    for (int g = 0; g < NW; ++g) {  // the first FBLOCK blocks: every load issued (from
        const int bb = g * 64 + lane;  // block 0 past the end), none under a branch
        const double v = row[bb < nblk ? bb : 0];
        t[g] = bb < nblk ? 0.0 + v : 0.0;
    }
    for (int b0 = FBLOCK; b0 < nblk; b0 += FBLOCK) {
#pragma unroll
        for (int g = 0; g < NW; ++g) {
            const int bb = b0 + g * 64 + lane;
            if (bb < nblk) t[g] += row[bb];
        }
    }
    double sv = 0.0;
#pragma unroll
    for (int g = 0; g < NW; ++g)
        if (g < ng) sv += wave_sum(t[g]);
    if (ng < NW) sv += 0.0;  // the empty groups' zero sums (only the sign of a zero can change)
    return sv;
}

// In a one-block finalize kernel of FBLOCK threads: sums[v] = sum over blocks of
// partials[v * nblk + b], v < kcount, in the order of group_row_sum; result in LDS sums[]
// for all threads.  One wavefront per entry (wavefront w takes v = w, w + 16, ...).
template <int K>
__device__ __forceinline__ void final_sum(const double* __restrict__ partials, int nblk, int kcount, double* sums) {
    constexpr int NW = FBLOCK / 64, R = (K + NW - 1) / NW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = wv + r * NW;
        if (e >= kcount) continue;  // uniform over the wavefront
        const double sv = group_row_sum(partials + (size_t)e * nblk, nblk, lane);
        if (lane == 0) sums[e] = sv;
    }
    __syncthreads();
}

}  // namespace helm

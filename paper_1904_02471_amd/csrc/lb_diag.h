// lb_diag.h -- deterministic FP64 block reduction of the five diagnostics,
// used by the fused step kernels and the stand-alone reduction.
#pragma once

#include "lb_internal.h"

namespace lbm {

// Per-thread FP64 accumulators: sum delta-rho, sum j_x, sum j_y,
// sum rho |u|^2 / 2, sum u . phi (velocities in the kernel's own unit).
struct DiagAcc {
    double v[kDiag] = {0.0, 0.0, 0.0, 0.0, 0.0};
};

// Sum the accumulators of the whole block in a fixed order and store the
// result at partial[block_id * kDiag].  Every thread of the block must call
// this (it synchronises the block).  blockDim must be a multiple of 64 and at
// most 1024.
__device__ __forceinline__ void block_diag_store(DiagAcc &acc, double *partial, int block_id)
{
    __shared__ double red[16][kDiag];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < kDiag; ++i) acc.v[i] += __shfl_xor(acc.v[i], off, 64);
    }
    const int lane = tid & 63, wave = tid >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kDiag; ++i) red[wave][i] = acc.v[i];
    }
    __syncthreads();
    if (tid < kDiag) {
        double s = 0.0;
        for (int w = 0; w < (nthreads >> 6); ++w) s += red[w][tid];
        partial[(long long)block_id * kDiag + tid] = s;
    }
}

// Sum nblocks partials into out[kDiag] in a fixed order, by one workgroup
// of 256 threads: thread t sums partials t, t + 256, ... in order, then a
// pairwise tree over the 256 thread sums.
__device__ __forceinline__ void diag_finalize_block(const double *partial, int nblocks, double *out)
{
    constexpr int kT = 256;
    __shared__ double s[kDiag][kT];
    const int t = threadIdx.x;
    double a[kDiag] = {0, 0, 0, 0, 0};
    for (int b = t; b < nblocks; b += kT)
        for (int i = 0; i < kDiag; ++i) a[i] += partial[(long long)b * kDiag + i];
    for (int i = 0; i < kDiag; ++i) s[i][t] = a[i];
    __syncthreads();
    for (int h = kT / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int i = 0; i < kDiag; ++i) s[i][t] += s[i][t + h];
        __syncthreads();
    }
    if (t < kDiag) out[t] = s[t][0];
}

}  // namespace lbm

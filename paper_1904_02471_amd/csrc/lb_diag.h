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

// Sum NV per-thread values over the whole block in a fixed order (a
// butterfly over the 64 lanes of each wave, then the waves in order) and
// store the result at partial[block_id * NV].  Every thread of the block
// must call this (it synchronises the block).  blockDim must be a multiple
// of 64 and at most 1024.
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double *partial, int block_id)
{
    __shared__ double red[16][NV];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off, 64);
    }
    const int lane = tid & 63, wave = tid >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
    }
    __syncthreads();
    if (tid < NV) {
        double s = 0.0;
        for (int w = 0; w < (nthreads >> 6); ++w) s += red[w][tid];
        partial[(long long)block_id * NV + tid] = s;
    }
}

// The five diagnostics of a block (block_sum_store with NV = kDiag).
__device__ __forceinline__ void block_diag_store(DiagAcc &acc, double *partial, int block_id)
{
    block_sum_store<kDiag>(acc.v, partial, block_id);
}

// Sum nblocks partials of NV values each into sums[NV] in a fixed order, by
// one workgroup of 256 threads: thread t sums partials t, t + 256, ... in
// order, then a pairwise tree over the 256 thread sums.  The result is valid
// in thread 0 .. NV-1 (sums[i] written by thread i) after the call.
template <int NV>
__device__ __forceinline__ void finalize_sums_block(const double *partial, int nblocks, double *sums)
{
    constexpr int kT = 256;
    __shared__ double s[NV][kT];
    const int t = threadIdx.x;
    double a[NV];
    for (int i = 0; i < NV; ++i) a[i] = 0.0;
    for (int b = t; b < nblocks; b += kT)
        for (int i = 0; i < NV; ++i) a[i] += partial[(long long)b * NV + i];
    for (int i = 0; i < NV; ++i) s[i][t] = a[i];
    __syncthreads();
    for (int h = kT / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int i = 0; i < NV; ++i) s[i][t] += s[i][t + h];
        __syncthreads();
    }
    if (t < NV) sums[t] = s[t][0];
}

// Sum nblocks partials of the five diagnostics into out[kDiag].
__device__ __forceinline__ void diag_finalize_block(const double *partial, int nblocks, double *out)
{
    finalize_sums_block<kDiag>(partial, nblocks, out);
}

}  // namespace lbm

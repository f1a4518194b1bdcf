// lb_batch.hip -- batched kernels of the serving form: one launch steps all
// admitted simulations of a kind together, each workgroup taking one row
// (collision-streaming) or one tile (finite-difference: 64 x 32 in the first
// stage, 64 x 16 or 64 x 32 in the later ones) of one simulation from a work
// list.  The per-row / per-tile device code is the same as in the
// single-simulation kernels (lb_cs_impl.h, lb_fd_impl.h).  The batch step is
// read from device memory, so that a captured step replays unchanged.
#include "lb_batch.h"
#include "lb_cs_impl.h"
#include "lb_fd_impl.h"

namespace lbm {

namespace {

__device__ __forceinline__ int step_of(const BatchSlot &s, int epoch) { return epoch - s.start_epoch; }

__global__ __launch_bounds__(kCsThreads) void cs_batch_kernel(const BatchSlot *__restrict__ slots,
                                                              const BatchWork *__restrict__ work,
                                                              const int *__restrict__ epoch_ptr)
{
    const int epoch = *epoch_ptr;
    const BatchWork w = work[blockIdx.x];
    const BatchSlot &s = slots[w.slot];
    const int e = step_of(s, epoch);
    if (e < 0 || e >= s.nsteps) return;  // uniform over the workgroup
    const float *src = s.buf[e & 1];
    float *dst = s.buf[(e & 1) ^ 1];
    // the same row form as the single-simulation launch, so that the fused
    // diagnostics sum in the same order
    const bool vec = cs_vec_ok<float>(s.p);
    if (e % s.every == 0) {
        const DiagArgs<float> d{s.partial, s.ax, s.ay, s.bx, s.by};
        if (vec)
            cs_row_vec<float, true>(src, dst, s.p, d, w.local, w.local);
        else
            cs_row<float, false, true>(src, dst, s.p, d, w.local, w.local);
    } else {
        const DiagArgs<float> d{};
        if (vec)
            cs_row_vec<float, false>(src, dst, s.p, d, w.local, w.local);
        else
            cs_row<float, false, false>(src, dst, s.p, d, w.local, w.local);
    }
}

template <int N, int STAGE, int ROWS>
__global__ __launch_bounds__(kFdThreads) void fd_batch_kernel(const BatchSlot *__restrict__ slots,
                                                              const BatchWork *__restrict__ work,
                                                              const int *__restrict__ epoch_ptr, float cb)
{
    const int epoch = *epoch_ptr;
    // contiguous runs of the work list per XCD (workgroup b runs on XCD b % 8)
    const int nb = gridDim.x, b = blockIdx.x, q = nb / 8, r = nb % 8, x = b % 8;
    const BatchWork w = work[x * q + (x < r ? x : r) + b / 8];
    const BatchSlot &s = slots[w.slot];
    const int e = step_of(s, epoch);
    if (e < 0 || e >= s.nsteps) return;  // uniform over the workgroup
    const int bx = w.local % s.tiles_x, by = w.local / s.tiles_x;
    if (STAGE == 1) {
        const DiagArgs<float> d{s.partial, s.ax, s.ay, s.bx, s.by};
        fd_stage_tile<float, N, false, false>(s.buf[0], nullptr, s.buf[1], cb, s.p, d, bx, by, w.local,
                                              e % s.every == 0);
    } else {
        const DiagArgs<float> d{};
        const float *src = STAGE == 2 ? s.buf[1] : s.buf[2];
        float *out = STAGE == 2 ? s.buf[2] : s.buf[0];
        fd_stage_tile<float, N, false, true, ROWS>(src, s.buf[0], out, cb, s.p, d, bx, by, w.local, false);
    }
}

__global__ __launch_bounds__(256) void finalize_batch_kernel(const BatchSlot *__restrict__ slots,
                                                             const int *__restrict__ ids,
                                                             const int *__restrict__ epoch_ptr)
{
    const int epoch = *epoch_ptr;
    const BatchSlot &s = slots[ids[blockIdx.x]];
    const int e = step_of(s, epoch);
    if (e < 0 || e >= s.nsteps || e % s.every != 0) return;
    diag_finalize_block(s.partial, s.diag_blocks, s.series + (long long)(e / s.every) * kDiag);
}

// after the launches of one batch step (one thread; stream order places it
// after them)
__global__ void epoch_advance_kernel(int *epoch) { *epoch += 1; }

template <int N>
hipError_t launch_fd_n_batch(const BatchSlot *slots, const BatchWork *work, int nwork, int stage, int rows,
                             const int *epoch, hipStream_t s)
{
    // the same stage weights as the single-simulation launcher
    const float cb = stage == 1 ? 1.0f : (stage == 2 ? 0.25f : 2.0f / 3.0f);
    if (stage == 1)
        hipLaunchKernelGGL((fd_batch_kernel<N, 1, kFdRows>), dim3(nwork), dim3(kFdThreads), 0, s, slots, work, epoch,
                           cb);
    else if (stage == 2 && rows == 4)
        hipLaunchKernelGGL((fd_batch_kernel<N, 2, 4>), dim3(nwork), dim3(kFdThreads), 0, s, slots, work, epoch, cb);
    else if (stage == 2)
        hipLaunchKernelGGL((fd_batch_kernel<N, 2, 8>), dim3(nwork), dim3(kFdThreads), 0, s, slots, work, epoch, cb);
    else if (rows == 4)
        hipLaunchKernelGGL((fd_batch_kernel<N, 3, 4>), dim3(nwork), dim3(kFdThreads), 0, s, slots, work, epoch, cb);
    else
        hipLaunchKernelGGL((fd_batch_kernel<N, 3, 8>), dim3(nwork), dim3(kFdThreads), 0, s, slots, work, epoch, cb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cs_batch(const BatchSlot *slots, const BatchWork *work, int nwork, const int *epoch, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(cs_batch_kernel, dim3(nwork), dim3(kCsThreads), 0, s, slots, work, epoch);
    return hipGetLastError();
}

hipError_t launch_fd_batch(const BatchSlot *slots, const BatchWork *work, int nwork, int N, int stage, int rows,
                           const int *epoch, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    if (rows != 4 && rows != 8) return hipErrorInvalidValue;
    switch (N) {
    case 1: return launch_fd_n_batch<1>(slots, work, nwork, stage, rows, epoch, s);
    case 2: return launch_fd_n_batch<2>(slots, work, nwork, stage, rows, epoch, s);
    case 3: return launch_fd_n_batch<3>(slots, work, nwork, stage, rows, epoch, s);
    case 4: return launch_fd_n_batch<4>(slots, work, nwork, stage, rows, epoch, s);
    case 5: return launch_fd_n_batch<5>(slots, work, nwork, stage, rows, epoch, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize_batch(const BatchSlot *slots, const int *slot_ids, int nslots, const int *epoch,
                                 hipStream_t s)
{
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_batch_kernel, dim3(nslots), dim3(256), 0, s, slots, slot_ids, epoch);
    return hipGetLastError();
}

hipError_t launch_epoch_advance(int *epoch, hipStream_t s)
{
    hipLaunchKernelGGL(epoch_advance_kernel, dim3(1), dim3(1), 0, s, epoch);
    return hipGetLastError();
}

}  // namespace lbm

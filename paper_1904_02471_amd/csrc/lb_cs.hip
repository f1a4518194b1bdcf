// lb_cs.hip -- collision-streaming D2Q9 step for gfx950, one simulation per
// launch: one workgroup per row (device code in lb_cs_impl.h).
#include "lb_cs_impl.h"

namespace lbm {

namespace {

template <typename T, bool FIXED, bool DIAG, bool REF>
__global__ __launch_bounds__(kCsThreads) void cs_step_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                             const Params<typename Arith<T>::type> p,
                                                             const DiagArgs<typename Arith<T>::type> d)
{
    cs_row<T, FIXED, DIAG, REF>(src, dst, p, d, blockIdx.x, blockIdx.x);
}

template <typename T, bool DIAG, bool REF, bool NT = false>
__global__ __launch_bounds__(1024) void cs_step_vec_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                                 const Params<typename Arith<T>::type> p,
                                                                 const DiagArgs<typename Arith<T>::type> d)
{
    cs_row_vec<T, DIAG, REF, NT>(src, dst, p, d, blockIdx.x, blockIdx.x);
}

template <typename T, bool FIXED, bool REF>
hipError_t launch_cs_t(const T *src, T *dst, const Params<typename Arith<T>::type> &p,
                       const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s, int threads, bool nt)
{
    dim3 grid(p.Ny), block(kCsThreads);
    if (!FIXED && cs_vec_ok<T>(p)) {
        // sampled steps keep the canonical size (their diagnostics sum per
        // thread) and plain stores
        const dim3 vblock(diag || threads <= 0 ? cs_vec_threads<T>(p.Nx) : threads);
        if (diag) {
            hipLaunchKernelGGL((cs_step_vec_kernel<T, true, REF>), grid, vblock, 0, s, src, dst, p, *diag);
        } else if (nt) {
            DiagArgs<typename Arith<T>::type> none{};
            hipLaunchKernelGGL((cs_step_vec_kernel<T, false, REF, true>), grid, vblock, 0, s, src, dst, p, none);
        } else {
            DiagArgs<typename Arith<T>::type> none{};
            hipLaunchKernelGGL((cs_step_vec_kernel<T, false, REF>), grid, vblock, 0, s, src, dst, p, none);
        }
        return hipGetLastError();
    }
    if (diag) {
        hipLaunchKernelGGL((cs_step_kernel<T, FIXED, true, REF>), grid, block, 0, s, src, dst, p, *diag);
    } else {
        DiagArgs<typename Arith<T>::type> none{};
        hipLaunchKernelGGL((cs_step_kernel<T, FIXED, false, REF>), grid, block, 0, s, src, dst, p, none);
    }
    return hipGetLastError();
}

}  // namespace

int cs_diag_blocks(int /*Nx*/, int Ny) { return Ny; }

template <typename T>
hipError_t launch_cs_step_st(const T *src, T *dst, const Params<typename Arith<T>::type> &p,
                             const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s, int threads, bool nt)
{
    if constexpr (std::is_same<T, __half>::value) {
        // FP16 relative to a reference equilibrium (periodic only)
        if (p.ref)
            return p.fixed_x ? hipErrorInvalidValue : launch_cs_t<T, false, true>(src, dst, p, diag, s, threads, nt);
    }
    if (p.fixed_x) return launch_cs_t<T, true, false>(src, dst, p, diag, s, threads, false);
    return launch_cs_t<T, false, false>(src, dst, p, diag, s, threads, nt);
}

template <typename T>
hipError_t launch_cs_step(const T *src, T *dst, const Params<typename Arith<T>::type> &p,
                          const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s, int threads)
{
    return launch_cs_step_st<T>(src, dst, p, diag, s, threads, false);
}

template hipError_t launch_cs_step<float>(const float *, float *, const Params<float> &, const DiagArgs<float> *,
                                          hipStream_t, int);
template hipError_t launch_cs_step<__half>(const __half *, __half *, const Params<float> &,
                                           const DiagArgs<float> *, hipStream_t, int);
template hipError_t launch_cs_step<double>(const double *, double *, const Params<double> &,
                                           const DiagArgs<double> *, hipStream_t, int);
template hipError_t launch_cs_step_st<float>(const float *, float *, const Params<float> &, const DiagArgs<float> *,
                                             hipStream_t, int, bool);
template hipError_t launch_cs_step_st<__half>(const __half *, __half *, const Params<float> &,
                                              const DiagArgs<float> *, hipStream_t, int, bool);
template hipError_t launch_cs_step_st<double>(const double *, double *, const Params<double> &,
                                              const DiagArgs<double> *, hipStream_t, int, bool);

}  // namespace lbm

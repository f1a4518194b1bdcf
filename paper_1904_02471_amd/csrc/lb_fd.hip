// lb_fd.hip -- finite-difference Gauss-Hermite stage kernels for gfx950, one
// simulation per launch (device code in lb_fd_impl.h).
#include "lb_fd_impl.h"

namespace lbm {

namespace {

template <typename T, int N, bool FIXED, bool DIAG, bool WITH_GN, int ROWS>
__global__ __launch_bounds__(kFdThreads) void fd_stage_kernel(const T *__restrict__ src, const T *gn, T *out,
                                                              const typename Arith<T>::type cb,
                                                              const Params<typename Arith<T>::type> p,
                                                              const DiagArgs<typename Arith<T>::type> d)
{
    // Workgroups are dispatched round-robin over the 8 XCDs (block b to XCD
    // b % 8).  Give each XCD a contiguous run of tiles (row-major), so that
    // most halo cache lines are shared by tiles in the same XCD's L2.
    const int nb = gridDim.x;
    const int b = blockIdx.x, q = nb / 8, r = nb % 8, x = b % 8;
    const int tile = x * q + (x < r ? x : r) + b / 8;
    const int tiles_x = (p.Nx + kTX - 1) / kTX;
    fd_stage_tile<T, N, FIXED, WITH_GN, ROWS>(src, gn, out, cb, p, d, tile % tiles_x, tile / tiles_x, tile, DIAG);
}

template <typename T, int N, bool FIXED, int ROWS>
hipError_t launch_fd_rows(const T *src, const T *gn, T *out, int stage, const Params<typename Arith<T>::type> &p,
                          const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s)
{
    using CT = typename Arith<T>::type;
    constexpr int kTY = FdGeom<ROWS>::kTY;
    dim3 grid(((p.Nx + kTX - 1) / kTX) * ((p.Ny + kTY - 1) / kTY)), block(kFdThreads);
    Params<CT> ps = p;  // a distinct random stream per stage
    ps.salt = mix_host(p.salt * 3u + (unsigned)stage);
    DiagArgs<CT> none{};
    if (stage == 1) {
        if (diag) {
            if constexpr (ROWS == kFdRows)
                hipLaunchKernelGGL((fd_stage_kernel<T, N, FIXED, true, false, ROWS>), grid, block, 0, s, src,
                                   nullptr, out, CT(1), ps, *diag);
            else
                return hipErrorInvalidValue;  // sampled stages use the canonical tiles
        } else {
            hipLaunchKernelGGL((fd_stage_kernel<T, N, FIXED, false, false, ROWS>), grid, block, 0, s, src, nullptr,
                               out, CT(1), ps, none);
        }
    } else {
        const CT cb = (stage == 2) ? CT(0.25) : CT(2) / CT(3);
        hipLaunchKernelGGL((fd_stage_kernel<T, N, FIXED, false, true, ROWS>), grid, block, 0, s, src, gn, out, cb,
                           ps, none);
    }
    return hipGetLastError();
}

template <typename T, int N, bool FIXED>
hipError_t launch_fd_n(const T *src, const T *gn, T *out, int stage, const Params<typename Arith<T>::type> &p,
                       const DiagArgs<typename Arith<T>::type> *diag, int rows, hipStream_t s)
{
    if (rows == 4 && !diag) return launch_fd_rows<T, N, FIXED, 4>(src, gn, out, stage, p, diag, s);
    return launch_fd_rows<T, N, FIXED, kFdRows>(src, gn, out, stage, p, diag, s);
}

template <typename T, bool FIXED>
hipError_t launch_fd_b(const T *src, const T *gn, T *out, int stage, const Params<typename Arith<T>::type> &p,
                       const DiagArgs<typename Arith<T>::type> *diag, int rows, hipStream_t s)
{
    switch (p.N) {
    case 1: return launch_fd_n<T, 1, FIXED>(src, gn, out, stage, p, diag, rows, s);
    case 2: return launch_fd_n<T, 2, FIXED>(src, gn, out, stage, p, diag, rows, s);
    case 3: return launch_fd_n<T, 3, FIXED>(src, gn, out, stage, p, diag, rows, s);
    case 4: return launch_fd_n<T, 4, FIXED>(src, gn, out, stage, p, diag, rows, s);
    case 5: return launch_fd_n<T, 5, FIXED>(src, gn, out, stage, p, diag, rows, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int fd_diag_blocks(int Nx, int Ny)
{
    return ((Nx + kTX - 1) / kTX) * ((Ny + FdGeom<kFdRows>::kTY - 1) / FdGeom<kFdRows>::kTY);
}

template <typename T>
hipError_t launch_fd_stage(const T *src, const T *gn, T *out, int stage, const Params<typename Arith<T>::type> &p,
                           const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s, int rows)
{
    if (p.fixed_x) return launch_fd_b<T, true>(src, gn, out, stage, p, diag, rows, s);
    return launch_fd_b<T, false>(src, gn, out, stage, p, diag, rows, s);
}

template hipError_t launch_fd_stage<float>(const float *, const float *, float *, int, const Params<float> &,
                                           const DiagArgs<float> *, hipStream_t, int);
template hipError_t launch_fd_stage<__half>(const __half *, const __half *, __half *, int, const Params<float> &,
                                            const DiagArgs<float> *, hipStream_t, int);
template hipError_t launch_fd_stage<double>(const double *, const double *, double *, int,
                                            const Params<double> &, const DiagArgs<double> *, hipStream_t, int);

}  // namespace lbm

// lb_fd.hip -- finite-difference Gauss-Hermite stage kernels for gfx950, one
// simulation per launch (device code in lb_fd_impl.h).
#include <cmath>

#include "lb_fd_impl.h"
#include "lb_node_index.h"

namespace lbm {

namespace {

// Occupancy asked of the compiler: five waves per SIMD (at most 96
// registers) for the later-stage 64 x 16 kernel of order 3 with FP32
// storage, which fits it without spills (left alone it takes 98 registers
// and four waves since the base-value copy moved behind the x-face reads).
// Order 4 spills at 96 registers in that form and keeps four waves (106
// registers); order 5 spills at 96 too.  Nothing for the others: with the
// moments of the output accumulated in registers, holding the 64 x 32
// first-stage kernels to 128 registers (four waves per SIMD) spills and
// runs slower than three waves without spills; the first-stage 64 x 16
// kernels spill at 96 registers, the later-stage ones at 80 (six waves), and
// both ran slower than without the limit.
template <typename T, int N, bool FIXED, bool DIAG, bool WITH_GN, int ROWS>
__global__ __launch_bounds__(kFdThreads)
__attribute__((amdgpu_waves_per_eu((WITH_GN && ROWS == 4 && N == 3 && sizeof(T) == 4) ? 5 : 1))) void fd_stage_kernel(const T *__restrict__ src, const T *gn, T *out,
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

// Moments of a stored value v of population k, accumulated in ascending k
// (the order and operations of the moment planes, fd_mom_offset).
template <typename CT>
struct MomAcc {
    CT drho = CT(0), jx = CT(0), jy = CT(0);
    __device__ __forceinline__ void add(const Params<CT> &p, int k, CT v)
    {
        drho += v;
        jx = fmaT(v, p.vx[k], jx);
        jy = fmaT(v, p.vy[k], jy);
    }
    // into the moment planes of the state buffer `buf`, at element index o
    template <typename T>
    __device__ __forceinline__ void store(const Params<CT> &p, T *buf, long long o) const
    {
        CT *m = reinterpret_cast<CT *>(reinterpret_cast<char *>(buf) + fd_mom_offset(p.K, p.plane, (int)sizeof(T)));
        m[o] = drho;
        m[p.plane + o] = jx;
        m[2 * p.plane + o] = jy;
    }
};

// Moment planes of g from its populations (one thread per node).
template <typename T>
__global__ __launch_bounds__(256) void fd_moments_kernel(T *g, const Params<typename Arith<T>::type> p)
{
    using CT = typename Arith<T>::type;
    const long long node = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (node >= (long long)p.Nx * p.Ny) return;
    int x, y;
    node_xy(node, p.Nx, x, y);
    const long long o = (long long)y * p.pitch + p.xoff + x;
    MomAcc<CT> m;
    for (int k = 0; k < p.K; ++k) m.add(p, k, ld(g + k * p.plane + o));
    m.store(p, g, o);
}

// ---------------------------------------------------------------------
// Implicit-explicit stepping (IMEX-SSP2(2,2,2)): the two pointwise stages.
// An implicit relaxation stage solves f_i = h + a tau R(f_i), a = g dt / tau;
// R keeps rho and rho u, so f_eq(f_i) = f_eq(h) and
//   f_i = (h + a f_eq(h)) / (1 + a).
// Moments and equilibrium are the stage kernel's (fd_node_correct, fd_geq).

template <typename CT, int N>
struct NodeEq {
    CT drho, ux, uy, dlt;
};

// Moments of h at node offset o, h_k = hk(k) (a callable), with the same
// summation order as the stage kernel's pre-pass.
template <typename CT, int N, typename H>
__device__ __forceinline__ NodeEq<CT, N> node_eq(const Params<CT> &p, H hk)
{
    CT drho = CT(0), jx = CT(0), jy = CT(0);
    for (int k = 0; k < p.K; ++k) {
        const CT g = hk(k);
        drho += g;
        jx = fmaT(g, p.vx[k], jx);
        jy = fmaT(g, p.vy[k], jy);
    }
    NodeEq<CT, N> q;
    const CT inv = CT(1) / (p.rho0 + drho);
    q.drho = drho;
    q.ux = jx * inv;
    q.uy = jy * inv;
    fd_node_correct<CT, N>(p, drho, jx, jy, q.ux, q.uy, q.dlt);
    return q;
}

template <typename CT, int N>
__device__ __forceinline__ CT node_geq(const Params<CT> &p, const NodeEq<CT, N> &q, int k)
{
    CT hx[N + 1], hy[N + 1];
    hx[0] = hy[0] = CT(1);
#pragma unroll
    for (int n = 1; n <= N; ++n) {
        hx[n] = p.hc[p.ki[k]][n];
        hy[n] = p.hc[p.kj[k]][n];
    }
    return fd_geq<CT, N>(p.w[k], hx, hy, p.rho0, q.drho, q.ux, q.uy, q.dlt);
}

// First stage: out = relaxed g (one thread per node), with its moment planes.
template <typename T, int N>
__global__ __launch_bounds__(256) void fd_imex_relax_kernel(const T *__restrict__ g, T *__restrict__ out,
                                                            const Params<typename Arith<T>::type> p,
                                                            typename Arith<T>::type a,
                                                            typename Arith<T>::type inv1pa)
{
    using CT = typename Arith<T>::type;
    const long long node = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (node >= (long long)p.Nx * p.Ny) return;
    int x, y;
    node_xy(node, p.Nx, x, y);
    const long long o = (long long)y * p.pitch + p.xoff + x;
    const long long P = p.plane;
    const NodeEq<CT, N> q = node_eq<CT, N>(p, [&](int k) { return ld(g + k * P + o); });
    uint32_t rb = mix32((uint32_t)node, p.salt);
    MomAcc<CT> m;
    for (int k = 0; k < p.K; ++k) {
        const CT h = ld(g + k * P + o);
        rb = xorshift32(rb);
        m.add(p, k, store_state(out + k * P + o, fmaT(a, node_geq<CT, N>(p, q, k), h) * inv1pa, rb >> 19));
    }
    m.store(p, out, o);
}

// Second stage, from y = f1 + dt L(f1) (in yb), f = g^n (in g) and f1 (in
// f1b): the explicit part h = f + dt A(f1) + (1 - 2g) dt R(f1) is
// y + 3 (f - f1) (as g dt R(f1) = f1 - f); writes f2 = relax(h) over yb and
// b = 2 f1 + h - f - f2 over f1b, so that the last stage
// f' = b + (f2 + dt L(f2) - b) / 2 equals f + dt/2 [L(f1) + L(f2)].  The
// moment planes of yb are f2's.
template <typename T, int N>
__global__ __launch_bounds__(256) void fd_imex_mid_kernel(T *__restrict__ yb, const T *__restrict__ g,
                                                          T *__restrict__ f1b,
                                                          const Params<typename Arith<T>::type> p,
                                                          typename Arith<T>::type a,
                                                          typename Arith<T>::type inv1pa)
{
    using CT = typename Arith<T>::type;
    const long long node = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (node >= (long long)p.Nx * p.Ny) return;
    int x, y;
    node_xy(node, p.Nx, x, y);
    const long long o = (long long)y * p.pitch + p.xoff + x;
    const long long P = p.plane;
    auto hk = [&](int k) {
        const CT f1 = ld(f1b + k * P + o);
        return fmaT(CT(3), ld(g + k * P + o) - f1, ld(yb + k * P + o));
    };
    const NodeEq<CT, N> q = node_eq<CT, N>(p, hk);
    uint32_t rb = mix32((uint32_t)node, p.salt);
    MomAcc<CT> m;
    for (int k = 0; k < p.K; ++k) {
        const CT f1 = ld(f1b + k * P + o), f = ld(g + k * P + o);
        const CT h = fmaT(CT(3), f - f1, ld(yb + k * P + o));
        const CT f2 = fmaT(a, node_geq<CT, N>(p, q, k), h) * inv1pa;
        const CT b = fmaT(CT(2), f1, h - f) - f2;
        rb = xorshift32(rb);
        m.add(p, k, store_state(yb + k * P + o, f2, rb >> 19));
        rb = xorshift32(rb);
        store_state(f1b + k * P + o, b, rb >> 19);
    }
    m.store(p, yb, o);
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
        // stages 2 and 3 of RK-3; 4: the last IMEX stage
        const CT cb = (stage == 2) ? CT(0.25) : (stage == 3 ? CT(2) / CT(3) : CT(0.5));
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

template <typename T, int N>
hipError_t launch_imex_n(int which, T *a_buf, const T *g, T *b_buf, const Params<typename Arith<T>::type> &p,
                         double dt_over_tau, hipStream_t s)
{
    using CT = typename Arith<T>::type;
    const double gam = 1.0 - 1.0 / std::sqrt(2.0);
    const CT a = (CT)(gam * dt_over_tau), inv1pa = (CT)(1.0 / (1.0 + gam * dt_over_tau));
    const long long nodes = (long long)p.Nx * p.Ny;
    const dim3 grid((unsigned)((nodes + 255) / 256)), block(256);
    Params<CT> ps = p;
    ps.salt = mix_host(p.salt * 3u + 5u + (unsigned)which);
    if (which == 0)
        hipLaunchKernelGGL((fd_imex_relax_kernel<T, N>), grid, block, 0, s, g, a_buf, ps, a, inv1pa);
    else
        hipLaunchKernelGGL((fd_imex_mid_kernel<T, N>), grid, block, 0, s, b_buf, g, a_buf, ps, a, inv1pa);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_fd_imex(int which, T *a_buf, const T *g, T *b_buf, const Params<typename Arith<T>::type> &p,
                          double dt_over_tau, hipStream_t s)
{
    switch (p.N) {
    case 1: return launch_imex_n<T, 1>(which, a_buf, g, b_buf, p, dt_over_tau, s);
    case 2: return launch_imex_n<T, 2>(which, a_buf, g, b_buf, p, dt_over_tau, s);
    case 3: return launch_imex_n<T, 3>(which, a_buf, g, b_buf, p, dt_over_tau, s);
    case 4: return launch_imex_n<T, 4>(which, a_buf, g, b_buf, p, dt_over_tau, s);
    case 5: return launch_imex_n<T, 5>(which, a_buf, g, b_buf, p, dt_over_tau, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_fd_imex<float>(int, float *, const float *, float *, const Params<float> &, double,
                                          hipStream_t);
template hipError_t launch_fd_imex<__half>(int, __half *, const __half *, __half *, const Params<float> &, double,
                                           hipStream_t);
template hipError_t launch_fd_imex<double>(int, double *, const double *, double *, const Params<double> &, double,
                                           hipStream_t);

template <typename T>
hipError_t launch_fd_moments(T *g, const Params<typename Arith<T>::type> &p, hipStream_t s)
{
    const long long nodes = (long long)p.Nx * p.Ny;
    hipLaunchKernelGGL((fd_moments_kernel<T>), dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, s, g, p);
    return hipGetLastError();
}

template hipError_t launch_fd_moments<float>(float *, const Params<float> &, hipStream_t);
template hipError_t launch_fd_moments<__half>(__half *, const Params<float> &, hipStream_t);
template hipError_t launch_fd_moments<double>(double *, const Params<double> &, hipStream_t);

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

// lb_aux.hip -- set-up and read-out kernels of the lattice Boltzmann library:
// equilibrium initialisation, canonical state transfer, moments and the
// stand-alone FP64 diagnostics.  All arithmetic here is FP64 whatever the
// storage precision; none of these kernels is on the time-step path.
//
// Collision-streaming storage holds post-collision values at their source
// node, so the canonical (pre-collision) value f_k(x) is read from x - e_k
// ("pull") and written to x - e_k ("push").  Finite-difference storage holds
// f_k(x) at x.
#include <mutex>

#include "lb_diag.h"
#include "lb_internal.h"
#include "lb_node_index.h"

namespace lbm {

namespace {

constexpr int kAuxThreads = 256;
constexpr int kReduceMaxBlocks = 1024;

constexpr size_t kScratchDoubles = (size_t)(kDiag + 1) * kReduceMaxBlocks;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

__device__ __forceinline__ int wrapi(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Shifted order-N equilibrium g_eq_k = f_eq_k - w_k rho0 =
// w_k [drho + rho sum_{1 <= n+m <= N} He_n(xi_i) He_m(xi_j) ax^n ay^m / (n! m!)],
// with ax, ay the velocity in units of c_s (Section 1).
__device__ double feq_shifted(const Params<double> &p, int k, double drho, double rho, double ax, double ay)
{
    double px[kMaxN + 1], py[kMaxN + 1];
    px[0] = py[0] = 1.0;
    for (int n = 1; n <= p.N; ++n) {
        px[n] = px[n - 1] * ax;
        py[n] = py[n - 1] * ay;
    }
    const int i = p.ki[k], j = p.kj[k];
    double s = 0.0;
    for (int n = 0; n <= p.N; ++n)
        for (int m = 0; n + m <= p.N; ++m)
            if (n + m > 0) s += (p.hc[i][n] * px[n]) * (p.hc[j][m] * py[m]);
    return p.w[k] * (drho + rho * s);
}

// Storage address of the value of population k that the canonical state
// holds at node (x, y).
__device__ __forceinline__ long long store_index(const Params<double> &p, bool cs, int k, int x, int y)
{
    int xs = x, ys = y;
    if (cs) {
        const int ex = p.ki[k] - 1, ey = p.kj[k] - 1;
        xs = x - ex;
        ys = wrapi(y - ey, p.Ny);
        if (!p.fixed_x) xs = wrapi(xs, p.Nx);  // with fixed ends xs = -1 / Nx is a ghost column
    }
    return (long long)k * p.plane + (long long)ys * p.pitch + p.xoff + xs;
}

template <typename T>
__device__ __forceinline__ double ldd(const T *ptr) { return (double)ld(ptr); }

// Storage node of the canonical value f_k(x, y) (store_index's position).
__device__ __forceinline__ void store_node(const Params<double> &p, bool cs, int k, int x, int y, int &xs, int &ys)
{
    xs = x;
    ys = y;
    if (cs) {
        xs = x - (p.ki[k] - 1);
        ys = wrapi(y - (p.kj[k] - 1), p.Ny);
        if (!p.fixed_x) xs = wrapi(xs, p.Nx);
    }
}

// Reference shift of population k stored at node (xs, ys): 0 unless the
// storage is relative to a reference equilibrium (LB_FP16_REF, CS).
__device__ __forceinline__ double ref_shift(const Params<double> &p, int k, int xs, int ys)
{
    if (!p.ref) return 0.0;
    float ux, uy;
    ref_unpack(p.ref[(long long)ys * p.pitch + xs], ux, uy);
    float c[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) c[i] = p.ref_c[i];
    return (double)cs_ref_pop(k, ux, uy, c);
}

// Shifted value g_k = f_k - w_k rho0 of the canonical state at (x, y) (under
// LB_FP16_REF the stored value is the scaled departure from the reference).
template <typename T>
__device__ __forceinline__ double stored_g(const T *src, const Params<double> &p, bool cs, int k, int x, int y)
{
    int xs, ys;
    store_node(p, cs, k, x, y, xs, ys);
    const double v = ldd(src + store_index(p, cs, k, x, y));
    if (!p.ref) return v;
    return v * (double)kRefInvScale + ref_shift(p, k, xs, ys);
}

// Store the shifted value g of f_k(x, y) (less the reference shift, if any).
template <typename T>
__device__ __forceinline__ void store_g(T *dst, const Params<double> &p, bool cs, int k, int x, int y, double g)
{
    int xs, ys;
    store_node(p, cs, k, x, y, xs, ys);
    if (!p.ref)
        store_from(dst + store_index(p, cs, k, x, y), g);
    else
        store_from(dst + store_index(p, cs, k, x, y), (g - ref_shift(p, k, xs, ys)) * (double)kRefScale);
}

// Reference velocity of LB_FP16_REF: (ux, uy) / c_l per node, rounded to
// FP16 (the collision works in lattice velocity units).
__global__ __launch_bounds__(kAuxThreads) void ref_from_velocity_kernel(uint32_t *ref, const double *ux,
                                                                        const double *uy, const Params<double> p,
                                                                        double inv_cl)
{
    const long long n = (long long)blockIdx.x * kAuxThreads + threadIdx.x;
    if (n >= (long long)p.Nx * p.Ny) return;
    int x, y;
    node_xy(n, p.Nx, x, y);
    const unsigned short hx = __builtin_bit_cast(unsigned short, (_Float16)(ux[n] * inv_cl));
    const unsigned short hy = __builtin_bit_cast(unsigned short, (_Float16)(uy[n] * inv_cl));
    ref[(long long)y * p.pitch + x] = (uint32_t)hx | ((uint32_t)hy << 16);
}

// The same from the velocity of a canonical state f [K][Ny][Nx] (FP64).
__global__ __launch_bounds__(kAuxThreads) void ref_from_state_kernel(uint32_t *ref, const double *f,
                                                                     const Params<double> p)
{
    const long long n = (long long)blockIdx.x * kAuxThreads + threadIdx.x;
    const long long nodes = (long long)p.Nx * p.Ny;
    if (n >= nodes) return;
    int x, y;
    node_xy(n, p.Nx, x, y);
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int k = 0; k < p.K; ++k) {
        const double fk = f[k * nodes + n];
        r += fk;
        jx += fk * (double)(p.ki[k] - 1);  // lattice units: e_k
        jy += fk * (double)(p.kj[k] - 1);
    }
    const unsigned short hx = __builtin_bit_cast(unsigned short, (_Float16)(jx / r));
    const unsigned short hy = __builtin_bit_cast(unsigned short, (_Float16)(jy / r));
    ref[(long long)y * p.pitch + x] = (uint32_t)hx | ((uint32_t)hy << 16);
}

template <typename T>
__global__ __launch_bounds__(kAuxThreads) void init_kernel(T *dst, const double *rho, const double *ux,
                                                           const double *uy, bool cs, const Params<double> p)
{
    const long long n = (long long)blockIdx.x * kAuxThreads + threadIdx.x;
    if (n >= (long long)p.Nx * p.Ny) return;
    int x, y;
    node_xy(n, p.Nx, x, y);
    const double r = rho[n];
    const double ax = ux[n] / p.cs, ay = uy[n] / p.cs;
    for (int k = 0; k < p.K; ++k) store_g(dst, p, cs, k, x, y, feq_shifted(p, k, r - p.rho0, r, ax, ay));
}

template <typename T>
__global__ __launch_bounds__(kAuxThreads) void fill_ghosts_kernel(T *buf, const Params<double> p)
{
    const int n = blockIdx.x * kAuxThreads + threadIdx.x;
    if (n >= p.K * p.Ny) return;
    const int k = n / p.Ny, y = n % p.Ny;
    T *row = buf + (long long)k * p.plane + (long long)y * p.pitch;
    store_from(row, p.ghost_l[k]);
    store_from(row + p.xoff + p.Nx, p.ghost_r[k]);
}

template <typename T>
__global__ __launch_bounds__(kAuxThreads) void get_state_kernel(const T *src, double *f, bool cs,
                                                                const Params<double> p)
{
    const long long n = (long long)blockIdx.x * kAuxThreads + threadIdx.x;
    const long long nodes = (long long)p.Nx * p.Ny;
    if (n >= nodes) return;
    int x, y;
    node_xy(n, p.Nx, x, y);
    for (int k = 0; k < p.K; ++k) f[k * nodes + n] = stored_g(src, p, cs, k, x, y) + p.w[k] * p.rho0;
}

template <typename T>
__global__ __launch_bounds__(kAuxThreads) void set_state_kernel(T *dst, const double *f, bool cs,
                                                                const Params<double> p)
{
    const long long n = (long long)blockIdx.x * kAuxThreads + threadIdx.x;
    const long long nodes = (long long)p.Nx * p.Ny;
    if (n >= nodes) return;
    int x, y;
    node_xy(n, p.Nx, x, y);
    for (int k = 0; k < p.K; ++k) store_g(dst, p, cs, k, x, y, f[k * nodes + n] - p.w[k] * p.rho0);
}

// moments of node n: drho = sum g_k, j = sum g_k v_k (sum w_k v_k = 0)
template <typename T>
__device__ __forceinline__ void node_moments(const T *src, bool cs, const Params<double> &p, int x, int y,
                                             double &drho, double &jx, double &jy)
{
    drho = jx = jy = 0.0;
    for (int k = 0; k < p.K; ++k) {
        const double g = stored_g(src, p, cs, k, x, y);
        drho += g;
        jx += g * p.vx[k];
        jy += g * p.vy[k];
    }
}

template <typename T>
__global__ __launch_bounds__(kAuxThreads) void moments_kernel(const T *src, double *rho, double *ux, double *uy,
                                                              bool cs, const Params<double> p)
{
    const long long n = (long long)blockIdx.x * kAuxThreads + threadIdx.x;
    if (n >= (long long)p.Nx * p.Ny) return;
    int x, y;
    node_xy(n, p.Nx, x, y);
    double drho, jx, jy;
    node_moments(src, cs, p, x, y, drho, jx, jy);
    const double r = p.rho0 + drho;
    if (rho) rho[n] = r;
    if (ux) ux[n] = jx / r;
    if (uy) uy[n] = jy / r;
}

template <typename T>
__global__ __launch_bounds__(kAuxThreads) void reduce_kernel(const T *src, bool cs, const Params<double> p,
                                                             const DiagArgs<double> d)
{
    const long long nodes = (long long)p.Nx * p.Ny;
    DiagAcc acc;
    for (long long n = (long long)blockIdx.x * kAuxThreads + threadIdx.x; n < nodes;
         n += (long long)gridDim.x * kAuxThreads) {
        int x, y;
        node_xy(n, p.Nx, x, y);
        double drho, jx, jy;
        node_moments(src, cs, p, x, y, drho, jx, jy);
        const double r = p.rho0 + drho, ux = jx / r, uy = jy / r;
        acc.v[0] += drho;
        acc.v[1] += jx;
        acc.v[2] += jy;
        acc.v[3] += 0.5 * r * (ux * ux + uy * uy);
        if (d.ax) acc.v[4] += ux * (d.ax[x] * d.ay[y]) + uy * (d.bx[x] * d.by[y]);
    }
    block_diag_store(acc, d.partial, blockIdx.x);
}

__global__ __launch_bounds__(kAuxThreads) void diag_finalize_kernel(const double *partial, int nblocks, double *out)
{
    diag_finalize_block(partial, nblocks, out);
}

// Diagnostics with a velocity pattern given as two full fields phi_x, phi_y
// ([Ny][Nx], FP64; both NULL for none): per block the FP64 sums of drho, j_x,
// j_y, rho |u|^2 / 2, u . phi and phi . phi, in node order per thread.
template <typename T>
__global__ __launch_bounds__(kAuxThreads) void reduce_field_kernel(const T *src, bool cs, const Params<double> p,
                                                                   const double *phix, const double *phiy,
                                                                   double *partial)
{
    const long long nodes = (long long)p.Nx * p.Ny;
    double acc[kDiag + 1] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long n = (long long)blockIdx.x * kAuxThreads + threadIdx.x; n < nodes;
         n += (long long)gridDim.x * kAuxThreads) {
        int x, y;
        node_xy(n, p.Nx, x, y);
        double drho, jx, jy;
        node_moments(src, cs, p, x, y, drho, jx, jy);
        const double r = p.rho0 + drho, ux = jx / r, uy = jy / r;
        acc[0] += drho;
        acc[1] += jx;
        acc[2] += jy;
        acc[3] += 0.5 * r * (ux * ux + uy * uy);
        if (phix) {
            const double a = phix[n], b = phiy[n];
            acc[4] += ux * a + uy * b;
            acc[5] += a * a + b * b;
        }
    }
    block_sum_store<kDiag + 1>(acc, partial, blockIdx.x);
}

// {M, Px, Py, E, A} from the partials of reduce_field_kernel: M = rho0 nodes
// + sum drho, A = sum u.phi / sum phi.phi (0 without a pattern).
__global__ __launch_bounds__(kAuxThreads) void reduce_field_finish_kernel(const double *partial, int nblocks,
                                                                          double rho0, double nodes, double *out)
{
    __shared__ double sums[kDiag + 1];
    finalize_sums_block<kDiag + 1>(partial, nblocks, sums);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = rho0 * nodes + sums[0];
        out[1] = sums[1];
        out[2] = sums[2];
        out[3] = sums[3];
        out[4] = sums[5] > 0.0 ? sums[4] / sums[5] : 0.0;
    }
}

unsigned grid_for(long long n) { return (unsigned)((n + kAuxThreads - 1) / kAuxThreads); }

}  // namespace

// Per-block partials of the field reduction for callers that cannot allocate
// (lb_reduce_field_noalloc): a fixed array of (kDiag + 1) doubles for each of
// the at most kReduceMaxBlocks blocks (48 KiB), one copy per GPU for the
// life of the process.  Host code never passes `scratch` itself (in host
// code the name is a stand-in, not a device address): it passes the
// address hipGetSymbolAddress returned for the device.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t reduce_field_scratch(int device, double **ptr, size_t *capacity)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        // the caller has made `device` current
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    *ptr = g_scratch_ptr[device];
    *capacity = kScratchDoubles;
    return hipSuccess;
}

int reduce_diag_blocks(int Nx, int Ny)
{
    long long b = ((long long)Nx * Ny + kAuxThreads - 1) / kAuxThreads;
    return (int)(b < kReduceMaxBlocks ? b : kReduceMaxBlocks);
}

template <typename T>
hipError_t launch_init(T *dst, const double *rho, const double *ux, const double *uy, bool cs,
                       const Params<double> &p, hipStream_t s)
{
    hipLaunchKernelGGL(init_kernel<T>, dim3(grid_for((long long)p.Nx * p.Ny)), dim3(kAuxThreads), 0, s, dst, rho,
                       ux, uy, cs, p);
    return hipGetLastError();
}

hipError_t launch_ref_from_velocity(uint32_t *ref, const double *ux, const double *uy, const Params<double> &p,
                                    double inv_cl, hipStream_t s)
{
    hipLaunchKernelGGL(ref_from_velocity_kernel, dim3(grid_for((long long)p.Nx * p.Ny)), dim3(kAuxThreads), 0, s,
                       ref, ux, uy, p, inv_cl);
    return hipGetLastError();
}

hipError_t launch_ref_from_state(uint32_t *ref, const double *f, const Params<double> &p, hipStream_t s)
{
    hipLaunchKernelGGL(ref_from_state_kernel, dim3(grid_for((long long)p.Nx * p.Ny)), dim3(kAuxThreads), 0, s, ref,
                       f, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_ghosts(T *buf, const Params<double> &p, hipStream_t s)
{
    hipLaunchKernelGGL(fill_ghosts_kernel<T>, dim3(grid_for((long long)p.K * p.Ny)), dim3(kAuxThreads), 0, s, buf,
                       p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_get_state(const T *src, double *f, bool cs, const Params<double> &p, hipStream_t s)
{
    hipLaunchKernelGGL(get_state_kernel<T>, dim3(grid_for((long long)p.Nx * p.Ny)), dim3(kAuxThreads), 0, s, src, f,
                       cs, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_set_state(T *dst, const double *f, bool cs, const Params<double> &p, hipStream_t s)
{
    hipLaunchKernelGGL(set_state_kernel<T>, dim3(grid_for((long long)p.Nx * p.Ny)), dim3(kAuxThreads), 0, s, dst, f,
                       cs, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_moments(const T *src, double *rho, double *ux, double *uy, bool cs, const Params<double> &p,
                          hipStream_t s)
{
    hipLaunchKernelGGL(moments_kernel<T>, dim3(grid_for((long long)p.Nx * p.Ny)), dim3(kAuxThreads), 0, s, src,
                       rho, ux, uy, cs, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce(const T *src, bool cs, const Params<double> &p, const DiagArgs<double> &diag,
                         hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel<T>, dim3(reduce_diag_blocks(p.Nx, p.Ny)), dim3(kAuxThreads), 0, s, src, cs, p,
                       diag);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce_field(const T *src, bool cs, const Params<double> &p, const double *phix, const double *phiy,
                               double *partial, double *out, hipStream_t s)
{
    const int nb = reduce_diag_blocks(p.Nx, p.Ny);
    hipLaunchKernelGGL(reduce_field_kernel<T>, dim3(nb), dim3(kAuxThreads), 0, s, src, cs, p, phix, phiy, partial);
    hipLaunchKernelGGL(reduce_field_finish_kernel, dim3(1), dim3(kAuxThreads), 0, s, (const double *)partial, nb,
                       p.rho0, (double)p.Nx * (double)p.Ny, out);
    return hipGetLastError();
}

hipError_t launch_diag_finalize(const double *partial, int nblocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(diag_finalize_kernel, dim3(1), dim3(kAuxThreads), 0, s, partial, nblocks, out);
    return hipGetLastError();
}

#define LB_AUX_INSTANTIATE(T)                                                                                     \
    template hipError_t launch_init<T>(T *, const double *, const double *, const double *, bool,                 \
                                       const Params<double> &, hipStream_t);                                      \
    template hipError_t launch_fill_ghosts<T>(T *, const Params<double> &, hipStream_t);                          \
    template hipError_t launch_get_state<T>(const T *, double *, bool, const Params<double> &, hipStream_t);      \
    template hipError_t launch_set_state<T>(T *, const double *, bool, const Params<double> &, hipStream_t);      \
    template hipError_t launch_moments<T>(const T *, double *, double *, double *, bool, const Params<double> &,  \
                                          hipStream_t);                                                           \
    template hipError_t launch_reduce<T>(const T *, bool, const Params<double> &, const DiagArgs<double> &,       \
                                         hipStream_t);                                                            \
    template hipError_t launch_reduce_field<T>(const T *, bool, const Params<double> &, const double *,           \
                                               const double *, double *, double *, hipStream_t);

LB_AUX_INSTANTIATE(float)
LB_AUX_INSTANTIATE(__half)
LB_AUX_INSTANTIATE(double)

}  // namespace lbm

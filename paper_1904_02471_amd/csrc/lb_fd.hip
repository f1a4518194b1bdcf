// lb_fd.hip -- finite-difference Gauss-Hermite step for gfx950: one launch
// per stage of the third-order TVD Runge-Kutta scheme (Section 2),
//
//   L(g)_k = -[v_kx (F_{i+1/2} - F_{i-1/2}) + v_ky (G_{j+1/2} - G_{j-1/2})] / ds
//            - (g_k - g_eq_k(g)) / tau
//   stage 1: A   = g   + dt L(g)
//   stage 2: B   = 3/4 g + 1/4 (A + dt L(A))
//   stage 3: g' = 1/3 g + 2/3 (B + dt L(B))      (written over g)
//
// with F, G the WENO-5 reconstructions on the upwind side of each interface
// and g_eq the Hermite equilibrium of order N (Section 1).
//
// Mapping: a workgroup of 256 threads owns a 64 x 16 tile; thread (lx, wy)
// owns column lx and rows 4 wy .. 4 wy + 3.  The workgroup first gathers the
// moments of its nodes (K loads per node), then loops over the populations:
// the tile of population k plus a 3-node halo is staged in LDS, each thread
// computes the x and y flux differences of its 4 nodes, the equilibrium of
// population k from the node's moments (kept in registers), and writes the
// Runge-Kutta combination.  Only O(N) registers per node are live across the
// population loop, so the same kernel serves K = 9 .. 36.
#include "lb_diag.h"
#include "lb_internal.h"

namespace lbm {

namespace {

constexpr int kTX = 64, kTY = 16, kRows = 4;
constexpr int kFdThreads = 256;
constexpr int kHalo = 3;
constexpr int kLX = kTX + 2 * kHalo;  // 70
constexpr int kLY = kTY + 2 * kHalo;  // 22
constexpr int kTileElems = kLX * kLY;
constexpr int kLoadsPerThread = (kTileElems + kFdThreads - 1) / kFdThreads;

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// WENO-5 (Jiang-Shu) interface value downstream of cell c from the values
// a, b, c, d, e ordered along the upwind direction.  The nonlinear weights
// alpha_r = d_r / (eps + beta_r)^2, normalised, are formed over a common
// denominator so that one reciprocal serves the interface:
//   omega_0 : omega_1 : omega_2 = 0.1 s1 s2 : 0.6 s0 s2 : 0.3 s0 s1,
//   s_r = (eps + beta_r)^2.
// Every multiply-add is an explicit fma (the library is compiled without
// automatic contraction), so each interface is the same function of its five
// inputs wherever it is evaluated: a uniform state stays uniform to the bit.
template <typename CT>
__device__ __forceinline__ CT weno5(CT a, CT b, CT c, CT d, CT e, CT eps)
{
    const CT k13 = CT(13.0 / 12.0), q = CT(0.25);
    const CT t0 = fmaT(CT(-2), b, a + c), u0 = fmaT(CT(-4), b, fmaT(CT(3), c, a));
    const CT t1 = fmaT(CT(-2), c, b + d), u1 = b - d;
    const CT t2 = fmaT(CT(-2), d, c + e), u2 = fmaT(CT(3), c, fmaT(CT(-4), d, e));
    const CT s0 = fmaT(k13 * t0, t0, fmaT(q * u0, u0, eps));
    const CT s1 = fmaT(k13 * t1, t1, fmaT(q * u1, u1, eps));
    const CT s2 = fmaT(k13 * t2, t2, fmaT(q * u2, u2, eps));
    const CT S0 = s0 * s0, S1 = s1 * s1, S2 = s2 * s2;
    const CT a0 = CT(0.1) * (S1 * S2), a1 = CT(0.6) * (S0 * S2), a2 = CT(0.3) * (S0 * S1);
    const CT q0 = fmaT(CT(11), c, fmaT(CT(-7), b, CT(2) * a));
    const CT q1 = fmaT(CT(5), c, fmaT(CT(2), d, -b));
    const CT q2 = fmaT(CT(5), d, fmaT(CT(2), c, -e));
    const CT num = fmaT(a0, q0, fmaT(a1, q1, a2 * q2));
    return num * fast_rcp(CT(6) * ((a0 + a1) + a2));
}

__device__ __forceinline__ int wrap(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

template <typename T, int N, bool FIXED, bool DIAG>
__global__ __launch_bounds__(kFdThreads) void fd_stage_kernel(const T *__restrict__ src, const T *gn, T *out,
                                                              const typename Arith<T>::type ca,
                                                              const typename Arith<T>::type cb,
                                                              const Params<typename Arith<T>::type> p,
                                                              const DiagArgs<typename Arith<T>::type> d)
{
    using CT = typename Arith<T>::type;
    __shared__ CT tile[kLY][kLX];

    const int tid = threadIdx.x;
    const int lx = tid & 63, wy = tid >> 6;
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY;
    const int Nx = p.Nx, Ny = p.Ny;
    const long long P = p.plane;

    // --- offsets of the tile elements this thread stages (fixed over k) ---
    // code: >= 0 element offset inside a plane, -1 left end, -2 right end, -3 unused
    int toff[kLoadsPerThread];
#pragma unroll
    for (int i = 0; i < kLoadsPerThread; ++i) {
        const int e = tid + i * kFdThreads;
        if (e < kTileElems) {
            const int r = e / kLX, c = e - r * kLX;
            const int gy = wrap(y0 - kHalo + r, Ny);
            const int gxr = x0 - kHalo + c;
            if (FIXED && gxr < 0) {
                toff[i] = -1;
            } else if (FIXED && gxr >= Nx) {
                toff[i] = -2;
            } else {
                toff[i] = gy * p.pitch + p.xoff + wrap(gxr, Nx);
            }
        } else {
            toff[i] = -3;
        }
    }

    // --- moments of the thread's nodes ---
    const int gx = x0 + lx;
    const bool colok = gx < Nx;
    int noff[kRows];
    bool active[kRows];
    CT drho[kRows], rho[kRows], pxn[kRows][N + 1], pyn[kRows][N + 1];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int gy = y0 + wy * kRows + r;
        active[r] = colok && gy < Ny;
        noff[r] = (gy < Ny ? gy : Ny - 1) * p.pitch + p.xoff + (colok ? gx : Nx - 1);
    }
    {
        CT dr[kRows], jx[kRows], jy[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) dr[r] = jx[r] = jy[r] = CT(0);
        for (int k = 0; k < p.K; ++k) {
            const CT vxk = p.vx[k], vyk = p.vy[k];
            const T *sk = src + k * P;
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const CT g = ld(sk + noff[r]);
                dr[r] += g;
                jx[r] = fmaT(g, vxk, jx[r]);
                jy[r] = fmaT(g, vyk, jy[r]);
            }
        }
        DiagAcc acc;
        CT pax = CT(0), pbx = CT(0);
        if (DIAG && d.ax) {
            pax = d.ax[colok ? gx : 0];
            pbx = d.bx[colok ? gx : 0];
        }
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            drho[r] = dr[r];
            rho[r] = p.rho0 + dr[r];
            const CT inv = CT(1) / rho[r];
            const CT ux = jx[r] * inv, uy = jy[r] * inv;
            pxn[r][0] = pyn[r][0] = CT(1);
#pragma unroll
            for (int n = 1; n <= N; ++n) {
                pxn[r][n] = pxn[r][n - 1] * ux;
                pyn[r][n] = pyn[r][n - 1] * uy;
            }
            if (DIAG && active[r]) {
                const int gy = y0 + wy * kRows + r;
                acc.v[0] += (double)dr[r];
                acc.v[1] += (double)jx[r];
                acc.v[2] += (double)jy[r];
                acc.v[3] += (double)(CT(0.5) * rho[r] * (ux * ux + uy * uy));
                if (d.ax) acc.v[4] += (double)(ux * (pax * d.ay[gy]) + uy * (pbx * d.by[gy]));
            }
        }
        if (DIAG) block_diag_store(acc, d.partial, blockIdx.y * gridDim.x + blockIdx.x);
    }

    const CT eps = p.eps, inv_ds = p.inv_ds, inv_tau = p.inv_tau, dt = p.dt;
    const int lc = lx + kHalo;  // LDS column of the thread's nodes

    for (int k = 0; k < p.K; ++k) {
        __syncthreads();  // previous population's tile fully consumed
        const T *sk = src + k * P;
#pragma unroll
        for (int i = 0; i < kLoadsPerThread; ++i) {
            const int e = tid + i * kFdThreads;
            if (e < kTileElems) {
                const int o = toff[i];
                CT v;
                if (FIXED && o == -1)
                    v = p.ghost_l[k];
                else if (FIXED && o == -2)
                    v = p.ghost_r[k];
                else
                    v = ld(sk + o);
                (&tile[0][0])[e] = v;
            }
        }
        CT gnv[kRows];
        if (gn) {
            const T *gk = gn + k * P;
#pragma unroll
            for (int r = 0; r < kRows; ++r) gnv[r] = ld(gk + noff[r]);
        }
        __syncthreads();

        const CT vxk = p.vx[k], vyk = p.vy[k];
        const int qi = p.ki[k], qj = p.kj[k];

        // y flux differences: march up the column, 5 interfaces for 4 nodes
        CT dfy[kRows];
        if (vyk != CT(0)) {
            const int rb = wy * kRows + kHalo;  // LDS row of the first node
            CT prev = CT(0);
#pragma unroll
            for (int m = 0; m <= kRows; ++m) {
                const int c = rb - 1 + m;  // interface between rows c and c+1
                CT G;
                if (vyk > CT(0))
                    G = weno5(tile[c - 2][lc], tile[c - 1][lc], tile[c][lc], tile[c + 1][lc], tile[c + 2][lc], eps);
                else
                    G = weno5(tile[c + 3][lc], tile[c + 2][lc], tile[c + 1][lc], tile[c][lc], tile[c - 1][lc], eps);
                if (m > 0) dfy[m - 1] = G - prev;
                prev = G;
            }
        } else {
#pragma unroll
            for (int r = 0; r < kRows; ++r) dfy[r] = CT(0);
        }

#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const int lr = wy * kRows + r + kHalo;
            const CT *row = tile[lr];
            CT dfx = CT(0);
            if (vxk > CT(0)) {
                const CT fr = weno5(row[lc - 2], row[lc - 1], row[lc], row[lc + 1], row[lc + 2], eps);
                const CT fl = weno5(row[lc - 3], row[lc - 2], row[lc - 1], row[lc], row[lc + 1], eps);
                dfx = fr - fl;
            } else if (vxk < CT(0)) {
                const CT fr = weno5(row[lc + 3], row[lc + 2], row[lc + 1], row[lc], row[lc - 1], eps);
                const CT fl = weno5(row[lc + 2], row[lc + 1], row[lc], row[lc - 1], row[lc - 2], eps);
                dfx = fr - fl;
            }
            const CT g = row[lc];

            // order-N equilibrium, shifted:  w_k [drho + rho P'(u)],
            // P' = sum_{1 <= n+m <= N} a_n b_m with a_n = He_n(xi_i) ux^n / n!,
            // b_m = He_m(xi_j) uy^m / m!, summed as C'_N + sum_n a_n (1 + C'_{N-n}),
            // C'_r = b_1 + ... + b_r (no O(1) term, so no cancellation).
            CT cpre[N + 1];
            cpre[0] = CT(0);
#pragma unroll
            for (int m = 1; m <= N; ++m) cpre[m] = fmaT(p.hc[qj][m], pyn[r][m], cpre[m - 1]);
            CT pp = cpre[N];
#pragma unroll
            for (int n = 1; n <= N; ++n) pp = fmaT(p.hc[qi][n] * pxn[r][n], CT(1) + cpre[N - n], pp);
            const CT geq = p.w[k] * fmaT(rho[r], pp, drho[r]);

            const CT adv = fmaT(vxk, dfx, vyk * dfy[r]) * inv_ds;
            const CT L = -fmaT(g - geq, inv_tau, adv);
            CT res = fmaT(dt, L, g);
            if (gn) res = fmaT(ca, gnv[r], cb * res);
            if (active[r]) store_from(out + k * P + noff[r], res);
        }
    }
}

template <typename T, int N, bool FIXED>
hipError_t launch_fd_n(const T *src, const T *gn, T *out, int stage, const Params<typename Arith<T>::type> &p,
                       const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s)
{
    using CT = typename Arith<T>::type;
    dim3 grid((p.Nx + kTX - 1) / kTX, (p.Ny + kTY - 1) / kTY), block(kFdThreads);
    CT ca = CT(0), cb = CT(1);
    const T *g = nullptr;
    if (stage == 2) {
        ca = CT(0.75);
        cb = CT(0.25);
        g = gn;
    } else if (stage == 3) {
        ca = CT(1) / CT(3);
        cb = CT(2) / CT(3);
        g = gn;
    }
    if (diag && stage == 1) {
        hipLaunchKernelGGL((fd_stage_kernel<T, N, FIXED, true>), grid, block, 0, s, src, g, out, ca, cb, p, *diag);
    } else {
        DiagArgs<CT> none{};
        hipLaunchKernelGGL((fd_stage_kernel<T, N, FIXED, false>), grid, block, 0, s, src, g, out, ca, cb, p, none);
    }
    return hipGetLastError();
}

template <typename T, bool FIXED>
hipError_t launch_fd_b(const T *src, const T *gn, T *out, int stage, const Params<typename Arith<T>::type> &p,
                       const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s)
{
    switch (p.N) {
    case 1: return launch_fd_n<T, 1, FIXED>(src, gn, out, stage, p, diag, s);
    case 2: return launch_fd_n<T, 2, FIXED>(src, gn, out, stage, p, diag, s);
    case 3: return launch_fd_n<T, 3, FIXED>(src, gn, out, stage, p, diag, s);
    case 4: return launch_fd_n<T, 4, FIXED>(src, gn, out, stage, p, diag, s);
    case 5: return launch_fd_n<T, 5, FIXED>(src, gn, out, stage, p, diag, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int fd_diag_blocks(int Nx, int Ny) { return ((Nx + kTX - 1) / kTX) * ((Ny + kTY - 1) / kTY); }

template <typename T>
hipError_t launch_fd_stage(const T *src, const T *gn, T *out, int stage, const Params<typename Arith<T>::type> &p,
                           const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s)
{
    if (p.fixed_x) return launch_fd_b<T, true>(src, gn, out, stage, p, diag, s);
    return launch_fd_b<T, false>(src, gn, out, stage, p, diag, s);
}

template hipError_t launch_fd_stage<float>(const float *, const float *, float *, int, const Params<float> &,
                                           const DiagArgs<float> *, hipStream_t);
template hipError_t launch_fd_stage<__half>(const __half *, const __half *, __half *, int, const Params<float> &,
                                            const DiagArgs<float> *, hipStream_t);
template hipError_t launch_fd_stage<double>(const double *, const double *, double *, int,
                                            const Params<double> &, const DiagArgs<double> *, hipStream_t);

}  // namespace lbm

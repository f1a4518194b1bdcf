// lb_fd_impl.h -- device code of the finite-difference Gauss-Hermite step,
// shared by the single-simulation kernel (lb_fd.hip) and the batched kernel
// (lb_batch.hip).  One launch per stage of the third-order TVD Runge-Kutta scheme (Section 2),
//
//   L(g)_k = -[v_kx (F_{i+1/2} - F_{i-1/2}) + v_ky (G_{j+1/2} - G_{j-1/2})] / ds
//            - (g_k - g_eq_k(g)) / tau
//   stage 1: A  = g + dt L(g)
//   stage 2: B  = g + 1/4 (A + dt L(A) - g)           (= 3/4 g + 1/4 (A + dt L(A)))
//   stage 3: g' = g + 2/3 (B + dt L(B) - g)           (= 1/3 g + 2/3 (B + dt L(B)))
//
// with F, G the WENO-5 reconstructions on the upwind side of each interface
// and g_eq the Hermite equilibrium of order N (Section 1).  The combinations
// are written as g + c (x - g) so that the two weights sum to one exactly in
// floating point (1/3 and 2/3 do not): no spurious growth of the state.
//
// The WENO-5 face is the bulk of the arithmetic, so the mapping evaluates
// every face once and marches along rows and columns so that neighbouring
// faces share their differences and smoothness terms (the stage sits between
// its memory traffic and the rate at which two waves co-issue its vector
// instructions; neither is saturated):
//
//   A workgroup of 256 threads owns a 64 x 32 tile; thread (lx, wy) owns
//   column lx and the 8 rows 8 wy .. 8 wy + 7 (the canonical geometry; the
//   tile height is a template parameter, 64 x 16 with 4 rows per thread is
//   the other choice of the autotuner, with 4-face x segments).
//   1. moments: the thread reads drho, j_x, j_y of its 8 nodes from the
//      input's moment planes (fd_mom_offset) and keeps drho, u_x, u_y.
//   2. loop over the populations k; the tile of population k with a 3-node
//      halo is staged in LDS (double-buffered; the next tile is prefetched
//      into registers while the current one is used):
//      a. x-faces: thread (row tid / 8, segment tid % 8) marches along its
//         row over 8 faces from a 12-value register window; 32 lanes of one
//         wave (which one rotates with the tile) add the left face of
//         column 0 of the 32 rows; faces go to LDS;
//      b. y-faces: thread (lx, wy) marches up its column over the 8 faces
//         above its 8 nodes, from a 12-value register window; the face
//         below its first node is the top face of the thread below (LDS),
//         the tile's bottom faces are computed by another wave (the two
//         edge tasks go to different waves, which rotate with the tile);
//      c. node update: flux differences, order-N equilibrium of population
//         k, Runge-Kutta combination, store; the stored values are summed
//         into the output's moments, written after the last population.
//   The sign of v_kx / v_ky is uniform over the launch, so the upwind side
//   is a scalar branch and every LDS access has a constant offset.
#pragma once

#include <type_traits>

#include "lb_diag.h"
#include "lb_internal.h"

namespace lbm {


constexpr int kTX = 64;
constexpr int kFdThreads = 256;
constexpr int kHalo = 3;
constexpr int kLX = kTX + 2 * kHalo;  // 70
constexpr int kXFaceStride = kTX + 1;  // x-faces per tile row
// Canonical tile height (rows per thread 8: 64 x 32 tiles).  Sampled stages,
// whose diagnostics partials are indexed by tile, and the batched launches
// always use it; plain stages may use a tuned height.
constexpr int kFdRows = 8;

// Tile geometry for ROWS rows per thread: 64 x (4 ROWS) tiles, the tile with
// its halo staged in LDS, x-faces marched in segments of kSeg per thread.
template <int ROWS>
struct FdGeom {
    static constexpr int kRows = ROWS;
    static constexpr int kTY = 4 * ROWS;
    static constexpr int kLY = kTY + 2 * kHalo;
    static constexpr int kTileElems = kLX * kLY;
    static constexpr int kLoadsPerThread = (kTileElems + kFdThreads - 1) / kFdThreads;
    static constexpr int kSeg = kTX * kTY / kFdThreads;
    static_assert(kTY * (kTX / kSeg) == kFdThreads, "one x-face segment per thread");
    static_assert(kTY <= 64, "the column-0 faces are computed by one wave");
};

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// WENO-5 (Jiang-Shu) interface value downstream of cell c from the values
// a, b, c, d, e ordered along the upwind direction:
//   candidates q0 = (2a - 7b + 11c)/6, q1 = (-b + 5c + 2d)/6, q2 = (2c + 5d - e)/6
//   smoothness beta0 = 13/12 (a-2b+c)^2 + 1/4 (a-4b+3c)^2,
//              beta1 = 13/12 (b-2c+d)^2 + 1/4 (b-d)^2,
//              beta2 = 13/12 (c-2d+e)^2 + 1/4 (3c-4d+e)^2
//   weights    alpha_r = d_r / (eps + beta_r)^2, d = (0.1, 0.6, 0.3)
//   value      sum alpha_r q_r / sum alpha_r.
// Evaluated in terms of the second differences t_r, the first differences
// cb = c - b, dc = d - c and their halves (exact), with which
//   (a-4b+3c)/2 = t0/2 + cb = v0,  (b-d)/2 = -(cb/2 + dc/2) = -v1,
//   (3c-4d+e)/2 = t2/2 - dc = v2,
//   10 d_r (q_r - c) = t0/3 + cb/2,  cb + 2 dc,  3 dc/2 - t2/2 = dc/2 - v2,
// and the weights over the common denominator (eps+beta0)^2 (eps+beta1)^2
// (eps+beta2)^2 (one reciprocal per face); numerator and denominator both
// carry the factor 10 (10 d_r = 1, 6, 3), which leaves one instruction per
// term.  On a sliding window the t_r, eps + 13/12 t_r^2, the first
// differences and their halves are common subexpressions of neighbouring
// faces.  FP32 range: (eps + beta)^4 must stay a normal number, hence the
// library accepts 1e-9 <= eps <= 1e9 for FP32 arithmetic.  Every
// multiply-add is an explicit fma (the library is compiled without
// automatic contraction), so a face is the same function of its five inputs
// wherever it is evaluated.
template <typename CT>
__device__ __forceinline__ CT weno5(CT a, CT b, CT c, CT d, CT e, CT eps)
{
    const CT k13 = CT(13.0 / 12.0), h = CT(0.5);
    const CT t0 = fmaT(CT(-2), b, a + c);
    const CT t1 = fmaT(CT(-2), c, b + d);
    const CT t2 = fmaT(CT(-2), d, c + e);
    const CT cb = c - b, dc = d - c;
    const CT hcb = h * cb, hdc = h * dc;
    const CT T0 = fmaT(k13 * t0, t0, eps), T1 = fmaT(k13 * t1, t1, eps), T2 = fmaT(k13 * t2, t2, eps);
    const CT v0 = fmaT(h, t0, cb), v1 = hcb + hdc, v2 = fmaT(h, t2, -dc);
    const CT s0 = fmaT(v0, v0, T0), s1 = fmaT(v1, v1, T1), s2 = fmaT(v2, v2, T2);
    const CT S0 = s0 * s0, S1 = s1 * s1, S2 = s2 * s2;
    const CT A0 = S1 * S2, A1 = S0 * S2, A2 = S0 * S1;
    // 10 d_r (q_r - c)
    const CT R0 = fmaT(CT(1.0 / 3.0), t0, hcb);
    const CT R1 = fmaT(CT(2), dc, cb);
    const CT R2 = hdc - v2;
    const CT num = fmaT(A0, R0, fmaT(A1, R1, A2 * R2));
    const CT den = fmaT(CT(6), A1, fmaT(CT(3), A2, A0));
    return fmaT(num, fast_rcp(den), c);
}

// Plane access through a buffer resource: the plane's base address sits in
// the (scalar) descriptor and every lane supplies a 32-bit byte offset, so
// the per-population addressing needs no 64-bit vector arithmetic and no
// per-lane 64-bit addresses held across the population loop.  Planes are
// below 4 GiB (the library refuses larger finite-difference grids); the
// descriptor's range is the plane's size, so an access past it would read
// 0 or be dropped instead of touching other memory (the 64 x 32 stage uses
// that to drop the stores of lanes without a node, at the offset of the
// plane's end).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t fd_plane(const void *base, uint32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)nbytes, 0x00020000);
}

// Loads and stores of values at a byte offset of a plane (FP32 and FP64:
// also the moment planes).  pack gives the bits a stepped value is stored
// as (rounded as store_state does: stochastically to FP16 with r13), unpack
// their value, put stores them.
template <typename T>
struct FdPlaneIO;
template <>
struct FdPlaneIO<float> {
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t off, float v)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
    }
    static __device__ __forceinline__ float pack(float v, uint32_t) { return v; }
    static __device__ __forceinline__ float unpack(float b) { return b; }
    static __device__ __forceinline__ void put(__amdgpu_buffer_rsrc_t r, uint32_t off, float b) { store(r, off, b); }
};
template <>
struct FdPlaneIO<double> {
    typedef unsigned int W __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    }
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t off, double v)
    {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(W, v), r, off, 0, 0);
    }
    static __device__ __forceinline__ double pack(double v, uint32_t) { return v; }
    static __device__ __forceinline__ double unpack(double b) { return b; }
    static __device__ __forceinline__ void put(__amdgpu_buffer_rsrc_t r, uint32_t off, double b) { store(r, off, b); }
};
template <>
struct FdPlaneIO<__half> {
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0)));
    }
    static __device__ __forceinline__ __half pack(float v, uint32_t r13) { return half_sr(v, r13); }
    static __device__ __forceinline__ float unpack(__half b) { return __half2float(b); }
    static __device__ __forceinline__ void put(__amdgpu_buffer_rsrc_t r, uint32_t off, __half b)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, b), r, off, 0, 0);
    }
};


// Sign tests of a velocity component held in a scalar register, on its bits
// (integer compares run on the scalar unit; float compares would take vector
// instructions): non-zero, and positive.
__device__ __forceinline__ bool v_nonzero(float v) { return (__builtin_bit_cast(uint32_t, v) & 0x7fffffffu) != 0u; }
__device__ __forceinline__ bool v_positive(float v) { return __builtin_bit_cast(int32_t, v) > 0; }
__device__ __forceinline__ bool v_nonzero(double v)
{
    return (__builtin_bit_cast(uint64_t, v) & 0x7fffffffffffffffull) != 0ull;
}
__device__ __forceinline__ bool v_positive(double v) { return __builtin_bit_cast(int64_t, v) > 0; }

__device__ __forceinline__ int fd_wrap(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Moment-exact equilibrium, per node.  The rounded tables give the
// equilibrium mass and momentum defects of relative size ~1e-8 (polynomials
// in u whose coefficients are exact sums in Params); left alone they act
// every stage with the same sign and drift the FP32 state.  They are removed
// once per node, inside operations whose exact results are not yet rounded:
// subtracting a correction below half an ulp from an already rounded smooth
// field would round it away or double it in a fixed spatial pattern.  u: one
// Newton step on rho u = j, with the momentum defect rho (ex, ey) folded into
// the residual, so that rho * u reproduces j - defect rather than
// rho * fl(j / rho).  Mass: dlt = defect / rho enters the equilibrium sum P'
// as its starting value.  By symmetry of the tables only even-even (mass),
// odd-even (x) and even-odd (y) monomials remain.  ux0, uy0 = j * (1 / rho)
// on input; ux, uy corrected on output.
template <typename CT, int N>
__device__ __forceinline__ void fd_node_correct(const Params<CT> &p, CT drho, CT jx, CT jy, CT &ux, CT &uy,
                                                CT &dlt)
{
    const CT ux0 = ux, uy0 = uy;
    CT xp[N + 1], yp[N + 1];
    xp[0] = yp[0] = CT(1);
#pragma unroll
    for (int n = 1; n <= N; ++n) {
        xp[n] = xp[n - 1] * ux0;
        yp[n] = yp[n - 1] * uy0;
    }
    CT dm = CT(0), ex = CT(0), ey = CT(0);
#pragma unroll
    for (int n = 0; n <= N; ++n)
#pragma unroll
        for (int m = 0; n + m <= N; ++m) {
            if (n % 2 == 0 && m % 2 == 0 && n + m > 0) dm = fmaT(p.fd_m[n][m], xp[n] * yp[m], dm);
            if (n % 2 == 1 && m % 2 == 0) {
                ex = fmaT(p.fd_jx[n][m], xp[n] * yp[m], ex);
                ey = fmaT(p.fd_jy[m][n], xp[m] * yp[n], ey);
            }
        }
    const CT rho = p.rho0 + drho;  // the same value the equilibrium forms
    const CT inv = CT(1) / rho;
    const CT rx = fmaT(-rho, ex, fmaT(-rho, ux0, jx));
    const CT ry = fmaT(-rho, ey, fmaT(-rho, uy0, jy));
    ux = fmaT(rx, inv, ux0);
    uy = fmaT(ry, inv, uy0);
    dlt = fmaT(p.fd_w1 * drho, inv, dm);
}

// Order-N equilibrium of one population, shifted:  w_k [drho + rho P'(u)],
// P' = sum_{1 <= n+m <= N} a_n b_m with a_n = He_n(xi_i) ux^n / n!,
// b_m = He_m(xi_j) uy^m / m!, summed as C'_N + sum_n a_n (1 + C'_{N-n}),
// C'_r = b_1 + ... + b_r (no O(1) term, so no cancellation) less the mass
// defect dlt per unit rho.  The terms odd and even in xi_j (in the prefix
// sums) and in xi_i (in the a_n sum) are accumulated apart and joined last:
// mirrored populations then share their even part bit for bit, and the
// roundings of the mass they carry do not drift one way (a single running
// sum rounds the small even terms against a large odd one, with a bias of
// ~10% of the rounding noise in D2Q36).  hx[n], hy[n] = He_n / n! at the
// population's two roots.
template <typename CT, int N>
__device__ __forceinline__ CT fd_geq(CT wk, const CT (&hx)[N + 1], const CT (&hy)[N + 1], CT rho0, CT drho,
                                     CT ux, CT uy, CT dlt)
{
    CT px[N + 1], py[N + 1];
    px[1] = ux;
    py[1] = uy;
#pragma unroll
    for (int n = 2; n <= N; ++n) {
        px[n] = px[n - 1] * ux;
        py[n] = py[n - 1] * uy;
    }
    CT ce = -dlt, co = CT(0);
    CT cp[N];  // C'_0 .. C'_{N-1}
    cp[0] = ce;
#pragma unroll
    for (int m = 1; m <= N; ++m) {
        if (m % 2)
            co = fmaT(hy[m], py[m], co);
        else
            ce = fmaT(hy[m], py[m], ce);
        if (m < N) cp[m] = ce + co;
    }
#pragma unroll
    for (int n = N; n >= 1; --n) {
        if (n % 2)
            co = fmaT(hx[n] * px[n], CT(1) + cp[N - n], co);
        else
            ce = fmaT(hx[n] * px[n], CT(1) + cp[N - n], ce);
    }
    const CT pp = ce + co;
    return wk * fmaT(rho0 + drho, pp, drho);
}

// One 64 x (4 ROWS) tile (bx, by) of a Runge-Kutta stage, by a 256-thread
// workgroup; with `diag` the diagnostics of the tile's input state go to
// partial[diag_block].  Every face and node is evaluated by the same
// sequence of operations for any ROWS, so the stage output does not depend
// on the tile height.  The moments of the input come from its moment planes
// (fd_mom_offset), and the stage writes those of its output.
template <typename T, int N, bool FIXED, bool WITH_GN, int ROWS = kFdRows>
__device__ __forceinline__ void fd_stage_tile(const T *__restrict__ src, const T *gn, T *out,
                                              const typename Arith<T>::type cb,
                                              const Params<typename Arith<T>::type> &p,
                                              const DiagArgs<typename Arith<T>::type> &d, int bx, int by,
                                              int diag_block, bool diag)
{
    using CT = typename Arith<T>::type;
    using G = FdGeom<ROWS>;
    constexpr int kRows = G::kRows, kTY = G::kTY, kTileElems = G::kTileElems;
    constexpr int kLoadsPerThread = G::kLoadsPerThread, kSeg = G::kSeg;
    __shared__ CT tile[2][kTileElems];
    __shared__ CT xface[kTY * kXFaceStride];
    __shared__ CT yface[(kFdThreads / kTX + 1) * kTX];  // y-faces below thread rows 0..3 and above row 3
    // FP32 storage: tiles and the Runge-Kutta base values are copied from
    // global memory straight into LDS (global_load_lds), without registers
    constexpr bool kDma = std::is_same<T, float>::value;
    __shared__ CT gnl[kDma && WITH_GN ? kTY * kTX : 1];
    __shared__ CT dltl[kRows * kFdThreads];  // per node: mass defect of the tables / rho

    const int tid = threadIdx.x;
    const int lx = tid & 63, wy = tid >> 6;
    // the wave's first thread and row block as scalars, so that the LDS
    // destinations of the tile copies (wave-uniform) are formed in scalar
    // registers
    const int wave0 = __builtin_amdgcn_readfirstlane(tid) & ~63;
    const int wy_s = wave0 >> 6;
    const int cw = diag_block & 3;  // wave of the tile's bottom y-faces
    const int cxw = cw ^ 2;         // wave of the column-0 x-faces
    // those waves have the tile-edge faces to evaluate on top of their share,
    // and the others wait for them at the barriers: let their instructions go first
    if (wy == cw || wy == cxw) __builtin_amdgcn_s_setprio(2);
    const int x0 = bx * kTX, y0 = by * kTY;
    const int Nx = p.Nx, Ny = p.Ny;
    const long long P = p.plane;
    const uint32_t pbytes = (uint32_t)(P * (long long)sizeof(T));
    using IO = FdPlaneIO<T>;

    // --- byte offsets in a plane of the tile elements this thread stages
    // (fixed over k); kLeftEnd / kRightEnd: the end states, kNoElem: none
    constexpr uint32_t kNoElem = 0xffffffffu, kLeftEnd = 0xfffffffeu, kRightEnd = 0xfffffffdu;
    uint32_t toff[kLoadsPerThread];
#pragma unroll
    for (int i = 0; i < kLoadsPerThread; ++i) {
        const int e = tid + i * kFdThreads;
        if (e < kTileElems) {
            const int r = e / kLX, c = e - r * kLX;
            const int gy = fd_wrap(y0 - kHalo + r, Ny);
            const int gxr = x0 - kHalo + c;
            if (FIXED && gxr < 0)
                toff[i] = kLeftEnd;
            else if (FIXED && gxr >= Nx)
                toff[i] = kRightEnd;
            else
                toff[i] = (uint32_t)(gy * p.pitch + p.xoff + fd_wrap(gxr, Nx)) * (uint32_t)sizeof(T);
        } else {
            toff[i] = kNoElem;
        }
    }
    auto fetch = [&](int k, CT *reg) {
        const auto sk = fd_plane(src + k * P, pbytes);
#pragma unroll
        for (int i = 0; i < kLoadsPerThread; ++i) {
            const uint32_t o = toff[i];
            if (o < kRightEnd)
                reg[i] = IO::load(sk, o);
            else if (FIXED && o == kLeftEnd)
                reg[i] = p.ghost_l[k];
            else if (FIXED && o == kRightEnd)
                reg[i] = p.ghost_r[k];
        }
    };
    auto stash = [&](int buf, const CT *reg) {
#pragma unroll
        for (int i = 0; i < kLoadsPerThread; ++i)
            if (toff[i] != kNoElem) tile[buf][tid + i * kFdThreads] = reg[i];
    };
    // asynchronous copy of tile k into tile[buf]; complete after a wait on
    // the vector-memory counter
    auto fetch_lds = [&](int k, int buf) {
        const auto sk = fd_plane(src + k * P, pbytes);
        const int wave_base = wave0;  // wave-uniform (scalar) LDS offset of the wave
#pragma unroll
        for (int i = 0; i < kLoadsPerThread; ++i) {
            const uint32_t o = toff[i];
            if (o < kRightEnd) {
                __builtin_amdgcn_raw_ptr_buffer_load_lds(sk, &tile[buf][i * kFdThreads + wave_base], 4, o, 0, 0, 0);
            } else if (FIXED && o == kLeftEnd) {
                tile[buf][tid + i * kFdThreads] = p.ghost_l[k];
            } else if (FIXED && o == kRightEnd) {
                tile[buf][tid + i * kFdThreads] = p.ghost_r[k];
            }
        }
    };

    // --- the thread's nodes: column gx, rows gy0 .. gy0 + 7 ---
    const int gx = x0 + lx;
    const int gy0 = y0 + wy * kRows;
    const bool colok = gx < Nx;
    const int noff0 = p.xoff + (colok ? gx : Nx - 1);
    auto node_idx = [&](int r) {  // element index inside a plane
        const int gy = gy0 + r;
        return (uint32_t)((gy < Ny ? gy : Ny - 1) * p.pitch + noff0);
    };
    auto node_off = [&](int r) { return node_idx(r) * (uint32_t)sizeof(T); };  // byte offset
    using MIO = FdPlaneIO<CT>;
    const uint32_t mbytes = (uint32_t)(P * (long long)sizeof(CT));  // one moment plane
    const unsigned long long moff = fd_mom_offset(p.K, P, (int)sizeof(T));
    auto active = [&](int r) { return colok && gy0 + r < Ny; };

    CT pre[kLoadsPerThread];
    if constexpr (kDma)
        fetch_lds(0, 0);
    else
        fetch(0, pre);
    CT drho[kRows], uxv[kRows], uyv[kRows];
    {
        // the input's moments, from its moment planes
        CT jx[kRows], jy[kRows];
        const char *mb = reinterpret_cast<const char *>(src) + moff;
        const auto m0 = fd_plane(mb, mbytes), m1 = fd_plane(mb + mbytes, mbytes),
                   m2 = fd_plane(mb + 2 * (unsigned long long)mbytes, mbytes);
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const uint32_t o = node_idx(r) * (uint32_t)sizeof(CT);
            drho[r] = MIO::load(m0, o);
            jx[r] = MIO::load(m1, o);
            jy[r] = MIO::load(m2, o);
        }
        DiagAcc acc;
        CT pax = CT(0), pbx = CT(0);
        if (diag && d.ax) {
            pax = d.ax[colok ? gx : 0];
            pbx = d.bx[colok ? gx : 0];
        }
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const CT rho = p.rho0 + drho[r];
            const CT inv = CT(1) / rho;
            uxv[r] = jx[r] * inv;
            uyv[r] = jy[r] * inv;
            if (diag && active(r)) {
                const int gy = gy0 + r;
                acc.v[0] += (double)drho[r];
                acc.v[1] += (double)jx[r];
                acc.v[2] += (double)jy[r];
                acc.v[3] += (double)(CT(0.5) * rho * fmaT(uxv[r], uxv[r], uyv[r] * uyv[r]));
                if (d.ax) acc.v[4] += (double)fmaT(uxv[r], pax * d.ay[gy], uyv[r] * (pbx * d.by[gy]));
            }
        }
        if (diag) block_diag_store(acc, d.partial, diag_block);

        // moment-exact equilibrium corrections (fd_node_correct); the mass
        // defect goes to LDS, thread-private, to spare registers
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            CT dlt;
            fd_node_correct<CT, N>(p, drho[r], jx[r], jy[r], uxv[r], uyv[r], dlt);
            dltl[r * kFdThreads + tid] = dlt;
        }
    }

    const CT eps = p.eps, dt = p.dt, inv_tau = p.inv_tau;
    if constexpr (kDma) {
        __builtin_amdgcn_s_waitcnt(0);
    } else {
        stash(0, pre);
        if (p.K > 1) fetch(1, pre);
    }
    __syncthreads();

    // moments of the output, summed as the stage stores it
    CT orho[kRows], ojx[kRows], ojy[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) orho[r] = ojx[r] = ojy[r] = CT(0);

    const int c0 = (wy * kRows + kHalo) * kLX + lx + kHalo;  // LDS cell of the thread's first node
    const int xr = tid / (kTX / kSeg), xs = tid % (kTX / kSeg);   // x-face row and segment
    const int xw = (xr + kHalo) * kLX + xs * kSeg + kHalo;        // LDS cell of the segment's first column

    for (int k = 0; k < p.K; ++k) {
        const int buf = k & 1;
        const CT *L = tile[buf];
        const CT vxk = p.vx[k], vyk = p.vy[k];
        const bool xnz = v_nonzero(vxk), xpos = v_positive(vxk), ynz = v_nonzero(vyk), ypos = v_positive(vyk);

        CT gnv[kRows];
        if constexpr (kDma) {
            if (k + 1 < p.K) fetch_lds(k + 1, buf ^ 1);
        } else if (WITH_GN) {
            const auto gk = fd_plane(gn + k * P, pbytes);
#pragma unroll
            for (int r = 0; r < kRows; ++r) gnv[r] = IO::load(gk, node_off(r));
        }

        // a. x-faces: faces xs*8 + 1 .. xs*8 + 8 of row xr (face i lies between
        //    tile columns i-1 and i), marching; column-0 faces by kTY lanes of
        //    wave cxw (rotating with the tile, so that no SIMD takes them for
        //    every workgroup; not the wave of the bottom y-faces, so that no
        //    wave holds both edge tasks up at the barrier)
        if (xnz) {
            CT w[kSeg + 4];
            CT *fx = &xface[xr * kXFaceStride + xs * kSeg + 1];
            if (xpos) {
#pragma unroll
                for (int i = 0; i < kSeg + 4; ++i) w[i] = L[xw - 2 + i];
#pragma unroll
                for (int m = 0; m < kSeg; ++m) fx[m] = weno5(w[m], w[m + 1], w[m + 2], w[m + 3], w[m + 4], eps);
                if (wy == cxw && lx < kTY) {
                    const int b = (lx + kHalo) * kLX + kHalo - 1;  // upwind cell of the column-0 face
                    xface[lx * kXFaceStride] = weno5(L[b - 2], L[b - 1], L[b], L[b + 1], L[b + 2], eps);
                }
            } else {
#pragma unroll
                for (int i = 0; i < kSeg + 4; ++i) w[i] = L[xw - 1 + i];
#pragma unroll
                for (int m = 0; m < kSeg; ++m) fx[m] = weno5(w[m + 4], w[m + 3], w[m + 2], w[m + 1], w[m], eps);
                if (wy == cxw && lx < kTY) {
                    const int b = (lx + kHalo) * kLX + kHalo;  // upwind cell of the column-0 face
                    xface[lx * kXFaceStride] = weno5(L[b + 2], L[b + 1], L[b], L[b - 1], L[b - 2], eps);
                }
            }
        }

        // the Runge-Kutta base values of population k, copied into LDS after
        // the x-face window reads are issued: the compiler cannot tell those
        // window reads from the copy's LDS writes and would wait for every
        // copy in flight before them (the next tile's included), which
        // serialised each population on its prefetch (y-face and node-update
        // reads are told apart; the copy lands by the mid-population wait)
        if constexpr (kDma) {
            if (WITH_GN) {
                const auto gk = fd_plane(gn + k * P, pbytes);
#pragma unroll
                for (int r = 0; r < kRows; ++r)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(gk, &gnl[(wy_s * kRows + r) * kTX], 4, node_off(r), 0, 0, 0);
            }
        }

        // b. y-faces: march up the column over the faces above the thread's
        //    nodes (face m lies below node m, m = 1 .. kRows); the face below
        //    its first node is the top face of the thread below, passed in
        //    LDS, and the tile's bottom faces come from wave cw
        CT dfy[kRows];
        CT g1 = CT(0);  // face 1, paired with face 0 after the barrier
        if (ynz) {
            CT w[kRows + 4];
            CT prev = CT(0);
            const int c00 = kHalo * kLX + lx + kHalo;  // LDS cell of the column's tile row 0
            if (ypos) {
#pragma unroll
                for (int i = 0; i < kRows + 4; ++i) w[i] = L[c0 + (i - 2) * kLX];
#pragma unroll
                for (int m = 1; m <= kRows; ++m) {
                    const CT G = weno5(w[m - 1], w[m], w[m + 1], w[m + 2], w[m + 3], eps);
                    if (m == 1)
                        g1 = G;
                    else
                        dfy[m - 1] = G - prev;
                    prev = G;
                }
                if (wy == cw)
                    yface[lx] = weno5(L[c00 - 3 * kLX], L[c00 - 2 * kLX], L[c00 - kLX], L[c00], L[c00 + kLX], eps);
            } else {
#pragma unroll
                for (int i = 0; i < kRows + 4; ++i) w[i] = L[c0 + (i - 1) * kLX];
#pragma unroll
                for (int m = 1; m <= kRows; ++m) {
                    const CT G = weno5(w[m + 3], w[m + 2], w[m + 1], w[m], w[m - 1], eps);
                    if (m == 1)
                        g1 = G;
                    else
                        dfy[m - 1] = G - prev;
                    prev = G;
                }
                if (wy == cw)
                    yface[lx] = weno5(L[c00 + 2 * kLX], L[c00 + kLX], L[c00], L[c00 - kLX], L[c00 - 2 * kLX], eps);
            }
            yface[(wy + 1) * kTX + lx] = prev;
        } else {
#pragma unroll
            for (int r = 0; r < kRows; ++r) dfy[r] = CT(0);
        }
        // the population's table values: their scalar loads are issued
        // before the mid-population wait, which covers their latency
        const int qi = p.ki[k], qj = p.kj[k];
        const CT wk = p.w[k];
        CT hx[N + 1], hy[N + 1];
        hx[0] = hy[0] = CT(1);
#pragma unroll
        for (int n = 1; n <= N; ++n) {
            hx[n] = p.hc[qi][n];
            hy[n] = p.hc[qj][n];
        }
        if constexpr (kDma) __builtin_amdgcn_s_waitcnt(0);  // tile k+1 and the base values have landed
        __syncthreads();
        {
            // read whatever v_ky and kept by a select, as the x-faces below
            const CT yb = yface[wy * kTX + lx];
            dfy[0] = ynz ? g1 - yb : CT(0);
        }

        // c. node updates
        const auto ok = fd_plane(out + k * P, pbytes);
        const CT vxs = vxk * p.inv_ds, vys = vyk * p.inv_ds;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const int tr = wy * kRows + r;  // tile row
            const CT g = L[c0 + r * kLX];
            // both faces are read whatever v_kx, and the difference is taken
            // by a select: a branch per row kept the compiler from overlapping
            // the rows' LDS reads (with v_kx = 0 the x-face array holds another
            // population's faces, or nothing yet, and the select drops them)
            const CT fr = xface[tr * kXFaceStride + lx + 1], fl = xface[tr * kXFaceStride + lx];
            const CT dfx = xnz ? fr - fl : CT(0);

            const CT geq = fd_geq<CT, N>(wk, hx, hy, p.rho0, drho[r], uxv[r], uyv[r], dltl[r * kFdThreads + tid]);

            const CT adv = fmaT(vxs, dfx, vys * dfy[r]);
            const CT Lk = -fmaT(g - geq, inv_tau, adv);
            CT res = fmaT(dt, Lk, g);
            if (WITH_GN) {
                CT b;
                if constexpr (kDma)
                    b = gnl[tr * kTX + lx];
                else
                    b = gnv[r];
                res = fmaT(cb, res - b, b);
            }
            uint32_t rb = 0;
            if constexpr (std::is_same<T, __half>::value)
                rb = mix32((uint32_t)((gy0 + r) * Nx + gx), p.salt ^ ((uint32_t)k * 0x632be5abu));
            const auto bits = IO::pack(res, rb >> 19);
            const CT st = IO::unpack(bits);
            orho[r] += st;
            ojx[r] = fmaT(st, vxk, ojx[r]);
            ojy[r] = fmaT(st, vyk, ojy[r]);
            if constexpr (ROWS == 8) {
                // lanes without a node here store past the plane's end, which
                // the buffer resource's range check drops: no branch per row,
                // so the rows' LDS reads overlap (64 x 16 tiles: the compiler
                // then spills at the five-wave register limit)
                IO::put(ok, active(r) ? node_off(r) : pbytes, bits);
            } else if (active(r)) {
                IO::put(ok, node_off(r), bits);
            }
        }
        // the output's moments, after its last population (inside the loop:
        // stored after it, they kept other registers live and cost more)
        if (k == p.K - 1) {
            char *mb = reinterpret_cast<char *>(out) + moff;
            const auto m0 = fd_plane(mb, mbytes), m1 = fd_plane(mb + mbytes, mbytes),
                       m2 = fd_plane(mb + 2 * (unsigned long long)mbytes, mbytes);
#pragma unroll
            for (int r = 0; r < kRows; ++r)
                if (active(r)) {
                    const uint32_t o = node_idx(r) * (uint32_t)sizeof(CT);
                    MIO::store(m0, o, orho[r]);
                    MIO::store(m1, o, ojx[r]);
                    MIO::store(m2, o, ojy[r]);
                }
        }

        // d. next tile into the other LDS buffer, prefetch the one after
        if constexpr (!kDma) {
            if (k + 1 < p.K) {
                stash(buf ^ 1, pre);
                if (k + 2 < p.K) fetch(k + 2, pre);
            }
        }
        __syncthreads();
    }
}

}  // namespace lbm

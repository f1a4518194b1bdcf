// lb_fd_fused.hip -- temporally blocked finite-difference step for gfx950:
// the three Runge-Kutta stages of one time step (Section 2: TVD RK-3 with
// WENO-5 advection and explicit BGK collision) in one launch, the stage
// values between the stages kept on chip.
//
// Decomposition: the grid is cut into x-strips and each strip into
// y-segments; one workgroup owns a strip segment and marches up it one row
// per iteration.  At iteration J it computes stage 1 at row J, stage 2 at row
// J-3 and stage 3 (the new state) at row J-6: the WENO-5 flux difference of a
// node reaches 3 nodes up and down, so a stage row needs the previous stage
// up to 3 rows above it, which the march has produced.  A segment of Ys
// output rows therefore computes stage 1 on Ys + 12 rows and stage 2 on
// Ys + 6 (the y recompute), and reads the state with a 9-row halo.
//
// Mapping: wave w holds populations w*PW .. w*PW+PW-1, lane l the strip
// columns l*C .. l*C+C-1 of a 64*C-column strip window.  Every lane keeps the
// y-windows of its columns in registers: 7 rows of the state g, of stage 1
// and of stage 2.  The x-stencil of a row comes from the neighbouring lanes
// by whole-wave DPP shifts (one lane per instruction); the values a lane near
// the window edges receives are wrong, so each stage is valid 3 columns
// further in on each side and a window of 64*C columns yields 64*C - 18
// output columns (the x recompute).  No stage value goes through memory.
//
// The equilibrium of a node needs the moments of all populations of the
// stage's input there, which live in different waves: each stage writes its
// row to LDS, and after the workgroup barrier of the iteration C waves (one
// column per lane) sum the populations in ascending order with the same
// operations as the stage kernel's moment planes, apply the moment-exact
// correction and keep (drho, u, mass defect) per column in small LDS rings
// until the next stage reaches that row (3 iterations later); stage 3's sums
// are written to the moment planes of the new state.  One barrier per
// iteration.  Faces, equilibria and updates are the stage kernel's functions
// (lb_fd_impl.h) on the same inputs, so the new state is bit for bit that of
// the three stage launches.
//
// FP32 storage, periodic grids, velocity sets with Q = 3 or 4 (the launcher
// refuses the rest: the library uses the stage launches there).  Traffic per step: the state read once
// with its halos (about (64C/(64C-18)) (1 + 18/Ys) of it) and written once,
// against 8 reads and writes of the state for three stage launches.
#include "lb_fd_impl.h"

namespace lbm {

namespace {

template <int Q, int PW, int C>
struct Fuse {
    static constexpr int K = Q * Q;
    static constexpr int kWaves = K / PW;
    static constexpr int kThreads = 64 * kWaves;
    static constexpr int kCols = 64 * C;  // strip columns held by the lanes of a wave
    static constexpr int kHaloX = 9;      // three stages of reach 3
    static constexpr int kOut = kCols - 2 * kHaloX;
    static_assert(K % PW == 0, "populations split evenly over the waves");
    static_assert(kThreads <= 1024, "one workgroup");
};

// Value of `v` held `L` lanes away (lane i receives lane i - L for L > 0,
// lane i - L = i + |L| for L < 0), by whole-wave DPP shifts; lanes whose
// source is outside the wave receive 0.
template <int L>
__device__ __forceinline__ float lane_from(float v)
{
    if constexpr (L == 0) {
        return v;
    } else if constexpr (L > 0) {
        // wave_shr:1 -- lane i takes lane i - 1
        const int r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false);
        return lane_from<L - 1>(__int_as_float(r));
    } else {
        // wave_shl:1 -- lane i takes lane i + 1
        const int r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false);
        return lane_from<L + 1>(__int_as_float(r));
    }
}

// Row values at relative columns o = -2 .. C+2 of a lane's first column,
// from the lane's own C values v[] and its neighbours' (the x-stencil of the
// lane's C right faces for either upwind side).
template <int C>
struct XRow {
    float x[C + 5];  // x[o + 2]
    __device__ __forceinline__ float at(int o) const { return x[o + 2]; }
};

template <int C, int O>
__device__ __forceinline__ float xval(const float (&v)[C])
{
    // column O relative to the lane's first: lane offset floor(O / C), index O mod C
    constexpr int L = (O >= 0) ? O / C : -((-O + C - 1) / C);
    constexpr int j = O - L * C;
    return lane_from<-L>(v[j]);
}

template <int C, int O>
__device__ __forceinline__ void fill_x(XRow<C> &r, const float (&v)[C])
{
    if constexpr (O <= C + 2) {
        r.x[O + 2] = xval<C, O>(v);
        fill_x<C, O + 1>(r, v);
    }
}

// Corrected input moments of a node: drho, u (after fd_node_correct) and the
// mass defect per unit rho.
struct NodeMom {
    float drho, ux, uy, dlt;
};

template <int N>
__device__ __forceinline__ float4 correct_moments(const Params<float> &p, float drho, float jx, float jy)
{
    const float rho = p.rho0 + drho;
    const float inv = 1.0f / rho;
    float ux = jx * inv, uy = jy * inv, dlt;
    fd_node_correct<float, N>(p, drho, jx, jy, ux, uy, dlt);
    return make_float4(drho, ux, uy, dlt);
}

// Per-thread march state.  Window slot of row J + d at iteration phase PH
// (J = y0 - 6 + t, PH = t mod 7): (PH + 3 + d) mod 7.
template <int PW, int C>
struct FuseRegs {
    float G[PW][C][7];    // state rows J-3 .. J+3
    float S1[PW][C][7];   // stage 1 rows J-6 .. J
    float S2[PW][C][7];   // stage 2 rows J-9 .. J-3
    float yb[3][PW][C];   // y-face below the row each stage computes next
    float nxt[PW][C];     // state row J+4 (loaded one iteration ahead)
};

template <int PH, int D>
__device__ __forceinline__ constexpr int slot() { return (PH + 3 + D + 21) % 7; }

// One stage row for the lane's populations and columns: W is the stage's
// input window, D the row offset (0, -3, -6), the update's base values
// (stages 2, 3) in `base`, the corrected input moments of the row's columns
// in `mom` (LDS).  Writes the outputs to out[i][j].
template <int Q, int N, int PW, int C, int PH, int D, int STAGE>
__device__ __forceinline__ void stage_row(const Params<float> &p, int wave, const float (&W)[PW][C][7],
                                          float (&yb)[PW][C], bool first, const float (&base)[PW][C],
                                          const float4 *mom, int col0, float (&out)[PW][C])
{
    const float eps = p.eps, dt = p.dt, inv_tau = p.inv_tau;
    const float cb = STAGE == 2 ? 0.25f : (STAGE == 3 ? 2.0f / 3.0f : 1.0f);
    float4 m[C];
#pragma unroll
    for (int j = 0; j < C; ++j) m[j] = mom[col0 + j];
#pragma unroll
    for (int i = 0; i < PW; ++i) {
        const int k = wave * PW + i;
        const float vxk = p.vx[k], vyk = p.vy[k];
        const float vxs = vxk * p.inv_ds, vys = vyk * p.inv_ds;
        // x: right faces of the lane's columns, the left one of its first from the lane before
        float dfx[C];
        {
            float v[C];
#pragma unroll
            for (int j = 0; j < C; ++j) v[j] = W[i][j][slot<PH, D>()];
            XRow<C> xr;
            fill_x<C, -2>(xr, v);
            float F[C];
            if (vxk > 0.0f) {
#pragma unroll
                for (int j = 0; j < C; ++j)
                    F[j] = weno5(xr.at(j - 2), xr.at(j - 1), xr.at(j), xr.at(j + 1), xr.at(j + 2), eps);
            } else {
#pragma unroll
                for (int j = 0; j < C; ++j)
                    F[j] = weno5(xr.at(j + 3), xr.at(j + 2), xr.at(j + 1), xr.at(j), xr.at(j - 1), eps);
            }
            const float fl = lane_from<1>(F[C - 1]);
#pragma unroll
            for (int j = 0; j < C; ++j) dfx[j] = (vxk != 0.0f) ? F[j] - (j == 0 ? fl : F[j - 1]) : 0.0f;
        }
        // y: the face above the row; the face below is the one above the row before
        float hx[N + 1], hy[N + 1];
        hx[0] = hy[0] = 1.0f;
        const int qi = p.ki[k], qj = p.kj[k];
#pragma unroll
        for (int n = 1; n <= N; ++n) {
            hx[n] = p.hc[qi][n];
            hy[n] = p.hc[qj][n];
        }
        const float wk = p.w[k];
#pragma unroll
        for (int j = 0; j < C; ++j) {
            float dfy = 0.0f;
            if (vyk != 0.0f) {
                float top, bot = yb[i][j];
                if (vyk > 0.0f) {
                    top = weno5(W[i][j][slot<PH, D - 2>()], W[i][j][slot<PH, D - 1>()], W[i][j][slot<PH, D>()], W[i][j][slot<PH, D + 1>()],
                                W[i][j][slot<PH, D + 2>()], eps);
                    if (first)
                        bot = weno5(W[i][j][slot<PH, D - 3>()], W[i][j][slot<PH, D - 2>()], W[i][j][slot<PH, D - 1>()],
                                    W[i][j][slot<PH, D>()], W[i][j][slot<PH, D + 1>()], eps);
                } else {
                    top = weno5(W[i][j][slot<PH, D + 3>()], W[i][j][slot<PH, D + 2>()], W[i][j][slot<PH, D + 1>()], W[i][j][slot<PH, D>()],
                                W[i][j][slot<PH, D - 1>()], eps);
                    if (first)
                        bot = weno5(W[i][j][slot<PH, D + 2>()], W[i][j][slot<PH, D + 1>()], W[i][j][slot<PH, D>()],
                                    W[i][j][slot<PH, D - 1>()], W[i][j][slot<PH, D - 2>()], eps);
                }
                dfy = top - bot;
                yb[i][j] = top;
            }
            const float g = W[i][j][slot<PH, D>()];
            const float geq = fd_geq<float, N>(wk, hx, hy, p.rho0, m[j].x, m[j].y, m[j].z, m[j].w);
            const float adv = fmaT(vxs, dfx[j], vys * dfy);
            const float Lk = -fmaT(g - geq, inv_tau, adv);
            float res = fmaT(dt, Lk, g);
            if (STAGE > 1) res = fmaT(cb, res - base[i][j], base[i][j]);
            out[i][j] = res;
        }
    }
}

template <int Q, int N, int PW, int C>
__global__ __launch_bounds__((Fuse<Q, PW, C>::kThreads)) void fd_fused_step_kernel(const float *__restrict__ src,
                                                                                 float *__restrict__ dst,
                                                                                 const Params<float> p, int Ys,
                                                                                 int nstrips)
{
    using F = Fuse<Q, PW, C>;
    constexpr int K = F::K, kCols = F::kCols;
    // LDS: a stage row of every population (two parities: the one written
    // this iteration, the one being summed), the corrected-moment rings
    __shared__ float V[2][3][K][kCols];
    __shared__ float4 M1[2][kCols], M2[4][kCols], M3[4][kCols];

    // contiguous runs of strip segments per XCD (workgroup b runs on XCD b % 8)
    const int nb = gridDim.x, b = blockIdx.x, q = nb / 8, rr = nb % 8, xcd = b % 8;
    const int tile = xcd * q + (xcd < rr ? xcd : rr) + b / 8;
    const int strip = tile % nstrips, seg = tile / nstrips;
    const int Nx = p.Nx, Ny = p.Ny;
    const int x0 = strip * F::kOut, y0 = seg * Ys;
    const int wout = min(F::kOut, Nx - x0);       // output columns of the strip
    const int yend = min(y0 + Ys, Ny);            // output rows [y0, yend)
    const int T = (yend - y0) + 12;               // iterations: stage 1 rows y0-6 .. yend+5

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col0 = lane * C;                    // first window column of the lane
    const long long P = p.plane;
    const uint32_t pbytes = (uint32_t)(P * (long long)sizeof(float));
    using IO = FdPlaneIO<float>;
    const unsigned long long moff = fd_mom_offset(K, P, (int)sizeof(float));
    const uint32_t mbytes = pbytes;  // one moment plane (FP32)

    // global column of window column cl (periodic)
    auto gcol = [&](int cl) __attribute__((always_inline)) { return fd_wrap(x0 - F::kHaloX + cl, Nx); };
    auto grow = [&](int r) __attribute__((always_inline)) { return fd_wrap(r, Ny); };
    auto byte_off = [&](int r, int cl) __attribute__((always_inline)) { return (uint32_t)(grow(r) * p.pitch + gcol(cl)) * (uint32_t)sizeof(float); };

    FuseRegs<PW, C> R;
    auto load_row = [&](int r, float (&dstv)[PW][C]) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < PW; ++i) {
            const auto pl = fd_plane(src + (long long)(wave * PW + i) * P, pbytes);
#pragma unroll
            for (int j = 0; j < C; ++j) dstv[i][j] = IO::load(pl, byte_off(r, col0 + j));
        }
    };

    // corrected moments of the state at row r for the window columns (the
    // C summing waves, one column per lane)
    const bool summer = wave < C;
    const int scol = wave * 64 + lane;  // the summing lane's window column
    auto state_moments = [&](int r) __attribute__((always_inline)) -> float4 {
        const char *mb = reinterpret_cast<const char *>(src) + moff;
        const uint32_t o = byte_off(r, scol);
        const float drho = IO::load(fd_plane(mb, mbytes), o);
        const float jx = IO::load(fd_plane(mb + mbytes, mbytes), o);
        const float jy = IO::load(fd_plane(mb + 2 * (unsigned long long)mbytes, mbytes), o);
        return correct_moments<N>(p, drho, jx, jy);
    };
    // sums of a stage row over the populations, ascending k (the moment planes' order)
    auto row_sums = [&](int par, int stage, float &drho, float &jx, float &jy) __attribute__((always_inline)) {
        drho = jx = jy = 0.0f;
        for (int k = 0; k < K; ++k) {
            const float v = V[par][stage][k][scol];
            drho += v;
            jx = fmaT(v, p.vx[k], jx);
            jy = fmaT(v, p.vy[k], jy);
        }
    };
    auto ring4 = [&](int r) __attribute__((always_inline)) { return (r - y0 + 16) & 3; };

    // prologue: state rows y0-9 .. y0-4 in slots 0..5 (phase 0), row y0-3 ahead
    {
        float tmp[PW][C];
#pragma unroll
        for (int d = -3; d <= 2; ++d) {
            load_row(y0 - 6 + d, tmp);
#pragma unroll
            for (int i = 0; i < PW; ++i)
#pragma unroll
                for (int j = 0; j < C; ++j) R.G[i][j][d + 3] = tmp[i][j];  // slot of row J0 + d at phase 0
        }
        load_row(y0 - 3, R.nxt);
        if (summer) M1[(y0 - 6) & 1][scol] = state_moments(y0 - 6);
    }
    __syncthreads();

    // phase B of the iteration before t (rows J-1, J-4, J-7), and the state
    // moments of row J+1 for the next one
    auto phase_b = [&](int t) __attribute__((always_inline)) {
        if (!summer) return;
        const int J = y0 - 6 + t, par = (t - 1) & 1;
        float drho, jx, jy;
        if (t - 1 >= 0 && t - 1 < T) {
            row_sums(par, 0, drho, jx, jy);
            M2[ring4(J - 1)][scol] = correct_moments<N>(p, drho, jx, jy);
        }
        if (t - 1 >= 6 && t - 1 < T) {
            row_sums(par, 1, drho, jx, jy);
            M3[ring4(J - 4)][scol] = correct_moments<N>(p, drho, jx, jy);
        }
        if (t - 1 >= 12 && t - 1 < T) {
            row_sums(par, 2, drho, jx, jy);
            const int r = J - 7;
            if (scol >= F::kHaloX && scol < F::kHaloX + wout) {
                char *mb = reinterpret_cast<char *>(dst) + moff;
                const uint32_t o = byte_off(r, scol);
                IO::store(fd_plane(mb, mbytes), o, drho);
                IO::store(fd_plane(mb + mbytes, mbytes), o, jx);
                IO::store(fd_plane(mb + 2 * (unsigned long long)mbytes, mbytes), o, jy);
            }
        }
        if (t < T) M1[(J + 1) & 1][scol] = state_moments(J + 1);
    };

    auto iteration = [&](auto ph, int t) __attribute__((always_inline)) {
        constexpr int PH = decltype(ph)::value;
        const int J = y0 - 6 + t, par = t & 1;
        // the state row J+3 joins the window; row J+4 is fetched for the next iteration
#pragma unroll
        for (int i = 0; i < PW; ++i)
#pragma unroll
            for (int j = 0; j < C; ++j) R.G[i][j][slot<PH, 3>()] = R.nxt[i][j];
        load_row(J + 4, R.nxt);
        float b3[PW][C];
        if (t >= 12) load_row(J - 6, b3);  // stage 3's base: the state at its row

        float o[PW][C];
        // stage 1 at row J
        stage_row<Q, N, PW, C, PH, 0, 1>(p, wave, R.G, R.yb[0], t == 0, o, M1[J & 1], col0, o);
#pragma unroll
        for (int i = 0; i < PW; ++i)
#pragma unroll
            for (int j = 0; j < C; ++j) {
                R.S1[i][j][slot<PH, 0>()] = o[i][j];
                V[par][0][wave * PW + i][col0 + j] = o[i][j];
            }
        // stage 2 at row J-3
        if (t >= 6) {
            float base[PW][C];
#pragma unroll
            for (int i = 0; i < PW; ++i)
#pragma unroll
                for (int j = 0; j < C; ++j) base[i][j] = R.G[i][j][slot<PH, -3>()];
            stage_row<Q, N, PW, C, PH, -3, 2>(p, wave, R.S1, R.yb[1], t == 6, base, M2[ring4(J - 3)], col0, o);
#pragma unroll
            for (int i = 0; i < PW; ++i)
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    R.S2[i][j][slot<PH, -3>()] = o[i][j];
                    V[par][1][wave * PW + i][col0 + j] = o[i][j];
                }
        }
        // stage 3 at row J-6: the new state
        if (t >= 12) {
            stage_row<Q, N, PW, C, PH, -6, 3>(p, wave, R.S2, R.yb[2], t == 12, b3, M3[ring4(J - 6)], col0, o);
#pragma unroll
            for (int i = 0; i < PW; ++i) {
                const auto pl = fd_plane(dst + (long long)(wave * PW + i) * P, pbytes);
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    V[par][2][wave * PW + i][col0 + j] = o[i][j];
                    const int cl = col0 + j;
                    if (cl >= F::kHaloX && cl < F::kHaloX + wout) IO::store(pl, byte_off(J - 6, cl), o[i][j]);
                }
            }
        }
        phase_b(t);
        __syncthreads();
    };

    for (int t0 = 0; t0 < T; t0 += 7) {
        iteration(std::integral_constant<int, 0>{}, t0);
        if (t0 + 1 < T) iteration(std::integral_constant<int, 1>{}, t0 + 1);
        if (t0 + 2 < T) iteration(std::integral_constant<int, 2>{}, t0 + 2);
        if (t0 + 3 < T) iteration(std::integral_constant<int, 3>{}, t0 + 3);
        if (t0 + 4 < T) iteration(std::integral_constant<int, 4>{}, t0 + 4);
        if (t0 + 5 < T) iteration(std::integral_constant<int, 5>{}, t0 + 5);
        if (t0 + 6 < T) iteration(std::integral_constant<int, 6>{}, t0 + 6);
    }
    // the last iteration's stage-3 moments
    phase_b(T);
}

template <int Q, int N, int PW, int C>
hipError_t launch_fused_qn(const float *src, float *dst, const Params<float> &p, int Ys, hipStream_t s)
{
    using F = Fuse<Q, PW, C>;
    const int nstrips = (p.Nx + F::kOut - 1) / F::kOut;
    const int nseg = (p.Ny + Ys - 1) / Ys;
    hipLaunchKernelGGL((fd_fused_step_kernel<Q, N, PW, C>), dim3(nstrips * nseg), dim3(F::kThreads), 0, s, src, dst,
                       p, Ys, nstrips);
    return hipGetLastError();
}

template <int Q, int PW, int C>
hipError_t launch_fused_q(const float *src, float *dst, const Params<float> &p, int Ys, hipStream_t s)
{
    switch (p.N) {
    case 1: return launch_fused_qn<Q, 1, PW, C>(src, dst, p, Ys, s);
    case 2: return launch_fused_qn<Q, 2, PW, C>(src, dst, p, Ys, s);
    case 3: if constexpr (Q > 3) return launch_fused_qn<Q, 3, PW, C>(src, dst, p, Ys, s); else break;
    case 4: if constexpr (Q > 4) return launch_fused_qn<Q, 4, PW, C>(src, dst, p, Ys, s); else break;
    case 5: if constexpr (Q > 5) return launch_fused_qn<Q, 5, PW, C>(src, dst, p, Ys, s); else break;
    default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

// Q = 3 and 4: one population per wave, two columns per lane (9 or 16
// waves, 128-column windows, 110 output columns).  The larger sets do not fit
// the register windows: 25 or 36 populations take 2 or 3 populations per wave
// (at most 16 waves a workgroup), whose 21 window values each exceed the 168
// registers of three waves per SIMD (the Q = 6 build with 3 populations per
// wave spills 1.9 KB per lane); they keep the stage launches.
bool fd_fused_supported(int Q, bool fixed) { return !fixed && (Q == 3 || Q == 4); }

hipError_t launch_fd_fused(const float *src, float *dst, const Params<float> &p, int Ys, hipStream_t s)
{
    if (p.fixed_x || Ys < 1) return hipErrorInvalidValue;
    switch (p.Q) {
    case 3: return launch_fused_q<3, 1, 2>(src, dst, p, Ys, s);
    case 4: return launch_fused_q<4, 1, 2>(src, dst, p, Ys, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm

// lb_internal.h -- types shared by the host runtime and the HIP kernels of
// the lattice Boltzmann library (not part of the public ABI).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lb.h"

namespace lbm {

constexpr int kMaxQ = 6;          // largest per-axis Gauss-Hermite order
constexpr int kMaxK = kMaxQ * kMaxQ;
constexpr int kMaxN = kMaxQ - 1;  // largest equilibrium order
constexpr int kDiag = 5;          // sum drho, sum jx, sum jy, sum rho|u|^2/2, sum u.phi

// Per-simulation constants, passed to every kernel by value (kernel
// arguments live in the constant cache; every index into these arrays is
// wave-uniform).  CT is the arithmetic type (float or double).
template <typename CT>
struct Params {
    int Nx, Ny;
    int pitch;        // elements between rows of one population plane
    int xoff;         // column of node x = 0 inside a row (1 with ghost columns)
    long long plane;  // elements between population planes
    int K, Q, N;
    int fixed_x;      // fixed-value x ends
    CT rho0;          // shift: stored g_k = f_k - w_k rho0
    CT cs;            // sound speed
    CT omega;         // CS: dt / tau
    CT dt, inv_ds, inv_tau, eps;  // FD
    CT w[kMaxK];
    CT vx[kMaxK], vy[kMaxK];      // physical velocities
    int ki[kMaxK], kj[kMaxK];     // per-axis root index of population k
    CT ghost_l[kMaxK], ghost_r[kMaxK];  // stored end equilibria: w_k (rho_end - rho0)
    CT hc[kMaxQ][kMaxN + 1];      // He_n(xi_i) / n!, xi_i = root i in units of c_s
    // CS D2Q9 equilibrium constants chosen so that, as exact real numbers,
    // w0 + 4 w1 + 4 w5 = 1 and 2 a1 + 4 a5 = 1 (a = 3 w): the equilibrium then
    // carries exactly the node's mass and momentum up to unbiased rounding.
    CT cs_w0, cs_w1, cs_w5, cs_a1, cs_a5;
    // FD: moment defects of the rounded tables, as exact sums over k of the
    // stored constants: mass  sum_k w_k hc[i_k][n] hc[j_k][m]       (fd_m),
    // momentum  sum_k w_k v_k hc[i_k][n] hc[j_k][m] - delta (fd_jx, fd_jy),
    // and fd_w1 = sum_k w_k - 1.  Zero in exact arithmetic; the stage kernel
    // removes them from its equilibrium node by node.
    CT fd_w1;
    CT fd_m[kMaxN + 1][kMaxN + 1], fd_jx[kMaxN + 1][kMaxN + 1], fd_jy[kMaxN + 1][kMaxN + 1];
    unsigned salt;  // per launch: seeds the stochastic rounding of FP16 stores
    // CS with FP16 storage relative to a reference equilibrium
    // (LB_FP16_REF): per node the reference velocity U in lattice units as
    // two FP16 values packed in 32 bits (x low), rows of `pitch` entries;
    // NULL otherwise.  ref_c: the FP32 constants of the shift (cs_ref_pop).
    const uint32_t *ref;
    float ref_c[8];
};

// Shift of CS population k (D2Q9 order) under LB_FP16_REF: the second-order
// equilibrium at (rho0, rho0 U) less w_k rho0, the same expression as the
// collision's equilibrium (Section 2):
//   R_k(U) = rho0 (a_k e_k.U + b_k (e_k.U)^2 - w_k 1.5 |U|^2),
// a = 3 w, b = 4.5 w (a_0 = b_0 = 0).  The stored value of population k at
// node s is f_k - w_k rho0 - R_k(U(s)): for a flow near the reference the
// stored departures are small, and so is their FP16 rounding.  Always FP32
// (c = {w0, w1, w5, a1, a5, b1, b5, rho0}), in every kernel that reads or
// writes the storage, so that each path adds and removes the same value.
// The constants are the collision's FP32 equilibrium constants and the
// operations follow its equilibrium: evaluated otherwise (from terms shared
// by the nine populations and the exact rational weights, equal to 1e-10),
// the stored departures carried a rounding pattern correlated with the
// flow, and the fitted viscosity of the 4096^2 vortex moved from +1e-4 ..
// +2.5e-4 to +1.3e-3 on every seed.
__host__ __device__ __forceinline__ float cs_ref_pop(int k, float ux, float uy, const float (&c)[8])
{
    float eu, w, a, b;
    switch (k) {
    case 0: eu = 0.0f; w = c[0]; a = 0.0f; b = 0.0f; break;
    case 1: eu = ux; w = c[1]; a = c[3]; b = c[5]; break;
    case 2: eu = uy; w = c[1]; a = c[3]; b = c[5]; break;
    case 3: eu = -ux; w = c[1]; a = c[3]; b = c[5]; break;
    case 4: eu = -uy; w = c[1]; a = c[3]; b = c[5]; break;
    case 5: eu = ux + uy; w = c[2]; a = c[4]; b = c[6]; break;
    case 6: eu = uy - ux; w = c[2]; a = c[4]; b = c[6]; break;
    case 7: eu = -ux - uy; w = c[2]; a = c[4]; b = c[6]; break;
    default: eu = ux - uy; w = c[2]; a = c[4]; b = c[6]; break;
    }
    const float usq = 1.5f * __builtin_fmaf(ux, ux, uy * uy);
    return c[7] * __builtin_fmaf(a, eu, __builtin_fmaf(b * eu, eu, -(w * usq)));
}

// The stored departure of LB_FP16_REF is scaled by 2^12 before its FP16
// rounding (and by 2^-12 when read, both exact): departures of a few 1e-5
// would otherwise fall below the FP16 normal range (6.1e-5), whose fixed
// subnormal spacing 6e-8 would cap their precision; scaled, they keep the
// relative precision 2^-11 down to 1.5e-8, and up to 16 in magnitude.
constexpr float kRefScale = 4096.0f, kRefInvScale = 1.0f / 4096.0f;

// The two FP16 halves of a packed reference velocity, as FP32.
__host__ __device__ __forceinline__ void ref_unpack(uint32_t v, float &ux, float &uy)
{
    ux = (float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu));
    uy = (float)__builtin_bit_cast(_Float16, (unsigned short)(v >> 16));
}

// Fused or stand-alone diagnostics: per-block FP64 partial sums.
template <typename CT>
struct DiagArgs {
    double *partial;              // [blocks][kDiag]
    const CT *ax, *ay, *bx, *by;  // separable probe, NULL when unset
};

// Storage conversions: the state is stored as float, half or double; the
// arithmetic type is float for the first two and double for the last.
__device__ __forceinline__ void store_from(float *p, float v) { *p = v; }
__device__ __forceinline__ void store_from(__half *p, float v) { *p = __float2half_rn(v); }
__device__ __forceinline__ void store_from(double *p, double v) { *p = v; }
__device__ __forceinline__ void store_from(float *p, double v) { *p = (float)v; }
__device__ __forceinline__ void store_from(__half *p, double v) { *p = __builtin_bit_cast(__half, (_Float16)v); }

// Stochastic rounding of an FP32 value v to FP16 with 13 random bits r13
// (0..8191): v moves away from zero by r13 units of 2^-13 of the FP16 step
// at v (2^-10 of its power of two in the FP16 normal range, 2^-24 below
// 2^-14), and the result is truncated toward zero to FP16.  The value thus
// passes the upper FP16 neighbour with probability equal to its position
// between the two neighbours, and keeps the lower one otherwise: exactly
// unbiased in the FP16 normal range.  Below 2^-14 the FP32 bits of v finer
// than 2^-37 are not randomised, which biases the result toward zero by less
// than 2^-13 of an FP16 step (2^-37 absolute); below 2^-24 the choice is
// between 0 and 2^-24.  A state that changes by less than an FP16 step per
// time step thus still evolves correctly on average, where round-to-nearest
// would hold it fixed.  gfx950's stochastic-rounding conversion
// (v_cvt_sr_f16_f32) with r13 in bits 31..19 of its random operand does
// exactly this, one instruction per value: it gave the same FP16 bits as the
// arithmetic form (an exact fma of r13 and the 2^-13 step into v, then the
// round-toward-zero conversion) on 2^20 values of both signs across the
// normal, subnormal and below-2^-24 FP16 ranges.  Beyond the FP16 range it
// gives +-inf where that form saturated at +-65504.
typedef __fp16 half2_bits __attribute__((ext_vector_type(2)));

// v rounded into the low (hi = false) or high half of the packed pair h.
__device__ __forceinline__ half2_bits sr16_into(half2_bits h, float v, uint32_t r13, bool hi)
{
    return hi ? __builtin_amdgcn_cvt_sr_f16_f32(h, v, r13 << 19, true)
              : __builtin_amdgcn_cvt_sr_f16_f32(h, v, r13 << 19, false);
}

__device__ __forceinline__ __half half_sr(float v, uint32_t r13)
{
    const half2_bits h = sr16_into(half2_bits{}, v, r13, false);
    return __builtin_bit_cast(__half, (unsigned short)(__builtin_bit_cast(uint32_t, h) & 0xffffu));
}

// Counter-based random bits (a 32-bit integer mixer) for (key, salt).
__device__ __forceinline__ uint32_t mix32(uint32_t key, uint32_t salt)
{
    uint32_t h = key * 0x9e3779b1u ^ salt;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ uint32_t xorshift32(uint32_t s)
{
    s ^= s << 13;
    s ^= s >> 17;
    s ^= s << 5;
    return s;
}

// Host-side mixer for per-launch salts.
inline unsigned mix_host(unsigned x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Store of a stepped state value: FP16 storage rounds stochastically with the
// given 13 random bits, the other storage types round to nearest.  Returns
// the value stored, in the arithmetic type.
__device__ __forceinline__ float store_state(float *p, float v, uint32_t) { *p = v; return v; }
__device__ __forceinline__ double store_state(double *p, double v, uint32_t) { *p = v; return v; }
__device__ __forceinline__ float store_state(__half *p, float v, uint32_t r13)
{
    const __half h = half_sr(v, r13);
    *p = h;
    return __half2float(h);
}

// Elements between population planes: the plane (pitch x Ny) plus 4352
// bytes.  With planes a power of two in size (2048^2, 4096^2), the rows that
// a kernel reads from the K planes at once start at the same offset modulo
// every power-of-two interleave of the memory channels and crowd the same
// channels; the pad (a multiple of 16 bytes, so rows keep their alignment)
// spreads them: +8 % on the 4096^2 collision-streaming step.
constexpr long long kPlanePadBytes = 4352;
inline long long padded_plane(long long elems, int esize) { return elems + kPlanePadBytes / esize; }

// Moment planes of a finite-difference state buffer.  After the K population
// planes (plane elements each) the buffer holds three planes in the
// arithmetic type: drho = sum_k g_k, jx = sum_k v_kx g_k, jy = sum_k v_ky g_k
// of the stored values, summed over k in ascending order with one add and two
// fmas per population, so that they equal bit for bit what a kernel would
// sum from the planes themselves.  Every kernel that writes a state buffer's
// populations writes its moment planes too; the stage kernels read them
// instead of summing the populations again.  Byte offset of the first one:
__host__ __device__ inline unsigned long long fd_mom_offset(int K, long long plane, int esize)
{
    return ((unsigned long long)K * (unsigned long long)plane * (unsigned long long)esize + 255ull) & ~255ull;
}

template <typename T> struct Arith { using type = float; };
template <> struct Arith<double> { using type = double; };

template <typename T>
__device__ __forceinline__ typename Arith<T>::type ld(const T *p);
template <> __device__ __forceinline__ float ld<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float ld<__half>(const __half *p) { return __half2float(*p); }
template <> __device__ __forceinline__ double ld<double>(const double *p) { return *p; }

// Hot-path launchers (lb_cs.hip, lb_fd.hip).  `diag` non-NULL fuses the
// diagnostics of the step's input state.
// `threads`: workgroup size of plain steps in the vector row form (0: the
// default, one chunk per thread); sampled steps always use the default.
template <typename T>
hipError_t launch_cs_step(const T *src, T *dst, const Params<typename Arith<T>::type> &p,
                          const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s, int threads = 0);
// `rows`: rows per thread of the stage tiles (8: 64 x 32, the canonical
// tiles; 4: 64 x 16, a tuning choice for stages without diagnostics); the
// output does not depend on it.
template <typename T>
hipError_t launch_fd_stage(const T *src, const T *gn, T *out, int stage, const Params<typename Arith<T>::type> &p,
                           const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s, int rows = 8);
// Temporally blocked FD step (lb_fd_fused.hip): the three Runge-Kutta stages
// in one launch, src (state with its moment planes) -> dst; strips of 110
// output columns, y-segments of Ys rows.  FP32 storage, periodic, Q = 3 or 4
// (fd_fused_supported); the output is bitwise that of the stage launches.
bool fd_fused_supported(int Q, bool fixed);
hipError_t launch_fd_fused(const float *src, float *dst, const Params<float> &p, int Ys, hipStream_t s);
// Pointwise stages of the implicit-explicit FD step: which = 0 relaxes g
// into a_buf; which = 1 turns (y in b_buf, g, f1 in a_buf) into (f2 in
// b_buf, the last stage's base in a_buf).  dt_over_tau = dt / tau.
template <typename T>
hipError_t launch_fd_imex(int which, T *a_buf, const T *g, T *b_buf, const Params<typename Arith<T>::type> &p,
                          double dt_over_tau, hipStream_t s);
// Moment planes of the FD state buffer g from its populations (after the
// populations are set from the host).
template <typename T>
hipError_t launch_fd_moments(T *g, const Params<typename Arith<T>::type> &p, hipStream_t s);
int cs_diag_blocks(int Nx, int Ny);
int fd_diag_blocks(int Nx, int Ny);

// Auxiliary launchers (lb_aux.hip), all in FP64 arithmetic.  `cs` selects
// the pull / push mapping of the collision-streaming storage.
template <typename T>
hipError_t launch_init(T *dst, const double *rho, const double *ux, const double *uy, bool cs,
                       const Params<double> &p, hipStream_t s);
template <typename T>
hipError_t launch_get_state(const T *src, double *f, bool cs, const Params<double> &p, hipStream_t s);
template <typename T>
hipError_t launch_set_state(T *dst, const double *f, bool cs, const Params<double> &p, hipStream_t s);
template <typename T>
hipError_t launch_moments(const T *src, double *rho, double *ux, double *uy, bool cs, const Params<double> &p,
                          hipStream_t s);
template <typename T>
hipError_t launch_reduce(const T *src, bool cs, const Params<double> &p, const DiagArgs<double> &diag,
                         hipStream_t s);
// Diagnostics with a full velocity pattern (phix, phiy: [Ny][Nx] FP64 device
// fields, both NULL for none): {M, Px, Py, E, A} written to out[kDiag]
// (device) by a second, single-workgroup launch; partial holds
// (kDiag + 1) * reduce_diag_blocks(Nx, Ny) doubles.
template <typename T>
hipError_t launch_reduce_field(const T *src, bool cs, const Params<double> &p, const double *phix, const double *phiy,
                               double *partial, double *out, hipStream_t s);
// Reference velocities of LB_FP16_REF (packed FP16 pairs, rows of pitch
// entries): from velocity fields (divided by c_l: inv_cl = 1 / c_l) or from
// the velocity of a canonical state f [K][Ny][Nx].
hipError_t launch_ref_from_velocity(uint32_t *ref, const double *ux, const double *uy, const Params<double> &p,
                                    double inv_cl, hipStream_t s);
hipError_t launch_ref_from_state(uint32_t *ref, const double *f, const Params<double> &p, hipStream_t s);
// Device address and capacity (doubles) of the fixed partials array of the
// field reduction on `device` (looked up once per device; thread-safe).
hipError_t reduce_field_scratch(int device, double **ptr, size_t *capacity);
template <typename T>
hipError_t launch_fill_ghosts(T *buf, const Params<double> &p, hipStream_t s);
int reduce_diag_blocks(int Nx, int Ny);

// Deterministic sum of nblocks partials into out[kDiag] (device memory).
hipError_t launch_diag_finalize(const double *partial, int nblocks, double *out, hipStream_t s);

}  // namespace lbm

// lb_api.cpp -- the C ABI of include/lb.h: handle, parameter validation,
// device buffers, launch sequencing and host/device transfers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <type_traits>
#include <utility>
#include <vector>

#include "lb.h"
#include "lb_internal.h"
#include "lb_model.h"
#include "lb_sim_impl.h"

using namespace lbm;

namespace {

thread_local int g_last_error = LB_OK;

int fail(int code)
{
    g_last_error = code;
    return code;
}

}  // namespace


namespace lbm {

size_t elem_size(Prec p) { return (p == P16 || p == P16R) ? 2 : (p == P64 ? 8 : 4); }

// CS D2Q9 constants in the arithmetic type, chosen so that the sums that
// carry mass and momentum are exact as real numbers: w1 = fl(1/9), w5 = 1/36
// rounded to a quarter of w0's ulp, w0 = 1 - 4 w1 - 4 w5 (representable by
// construction); a1 = fl(1/3), a5 = (1 - 2 a1) / 4 (representable).  Each
// differs from its exact value by at most about one ulp.
template <typename CT>
void cs_exact_constants(Params<CT> &p)
{
    constexpr int digits = std::numeric_limits<CT>::digits;
    const long double q = std::ldexp(1.0L, -3 - digits);  // w0 in [1/4, 1/2): ulp 2^(-1-digits)
    const CT w1 = (CT)(1.0L / 9.0L);
    const CT w5 = (CT)(std::nearbyint((1.0L / 36.0L) / q) * q);
    const CT w0 = (CT)(1.0L - 4.0L * w1 - 4.0L * w5);
    const CT a1 = (CT)(1.0L / 3.0L);
    const CT a5 = (CT)((1.0L - 2.0L * a1) / 4.0L);
    p.cs_w0 = w0;
    p.cs_w1 = w1;
    p.cs_w5 = w5;
    p.cs_a1 = a1;
    p.cs_a5 = a5;
}

// Mass and momentum defects of the FD equilibrium tables as stored in the
// arithmetic type (Section 1: the quadrature reproduces the Hermite moments
// exactly, so every one of these sums vanishes for exact constants).  The
// products of stored constants are formed in long double.
template <typename CT>
void fd_moment_defects(Params<CT> &p)
{
    long double W = 0.0L;
    for (int k = 0; k < p.K; ++k) W += (long double)p.w[k];
    p.fd_w1 = (CT)(W - 1.0L);
    for (int n = 0; n <= kMaxN; ++n)
        for (int m = 0; m <= kMaxN; ++m) {
            long double sm = 0.0L, sx = 0.0L, sy = 0.0L;
            if (n + m <= p.N) {
                for (int k = 0; k < p.K; ++k) {
                    const long double t = (long double)p.w[k] * (long double)p.hc[p.ki[k]][n] *
                                          (long double)p.hc[p.kj[k]][m];
                    sm += t;
                    sx += t * (long double)p.vx[k];
                    sy += t * (long double)p.vy[k];
                }
                if (n == 1 && m == 0) sx -= 1.0L;  // c_s = 1 in FD units
                if (n == 0 && m == 1) sy -= 1.0L;
            }
            p.fd_m[n][m] = (n + m == 0) ? CT(0) : (CT)sm;
            p.fd_jx[n][m] = (CT)sx;
            p.fd_jy[n][m] = (CT)sy;
        }
}

template <typename CT>
Params<CT> make_params(const lb_sim *s)
{
    Params<CT> p{};
    p.Nx = s->Nx;
    p.Ny = s->Ny;
    p.pitch = s->pitch;
    p.xoff = s->xoff;
    p.plane = s->plane;
    p.K = s->K;
    p.Q = s->Q;
    p.N = s->N;
    p.fixed_x = s->fixed ? 1 : 0;
    p.rho0 = (CT)s->rho0;
    p.cs = (CT)s->mi.cs;
    p.omega = (CT)(s->dt / s->tau);
    p.dt = (CT)s->dt;
    p.inv_ds = (CT)(1.0 / s->ds);
    p.inv_tau = (CT)(1.0 / s->tau);
    p.eps = (CT)s->eps;
    p.salt = mix_host((unsigned)s->steps ^ (s->rounding_seed * 0x9e3779b1u));
    for (int k = 0; k < s->K; ++k) {
        p.w[k] = (CT)s->mi.w[k];
        p.vx[k] = (CT)s->mi.vx[k];
        p.vy[k] = (CT)s->mi.vy[k];
        p.ki[k] = s->mi.ki[k];
        p.kj[k] = s->mi.kj[k];
        // the end equilibria at u = 0 are w_k rho_end exactly, for every order
        p.ghost_l[k] = (CT)(s->mi.w[k] * (s->rho_l - s->rho0));
        p.ghost_r[k] = (CT)(s->mi.w[k] * (s->rho_r - s->rho0));
    }
    for (int i = 0; i < s->Q; ++i)
        for (int n = 0; n <= kMaxN; ++n) p.hc[i][n] = (CT)s->mi.hc[i][n];
    if (s->cs)
        cs_exact_constants(p);
    else
        fd_moment_defects(p);
    if (s->prec == P16R) {
        // the FP32 constants of the reference shift, whatever CT is
        Params<float> pf{};
        cs_exact_constants(pf);
        p.ref = s->d_ref;
        const float c[8] = {pf.cs_w0, pf.cs_w1, pf.cs_w5, pf.cs_a1, pf.cs_a5, 0.5f, 0.125f, (float)s->rho0};
        for (int i = 0; i < 8; ++i) p.ref_c[i] = c[i];
    }
    return p;
}

void free_buffers(lb_sim *s)
{
    for (int i = 0; i < 3; ++i) {
        if (s->buf[i]) (void)hipFree(s->buf[i]);
        s->buf[i] = nullptr;
    }
    if (s->d_ref) (void)hipFree(s->d_ref);
    s->d_ref = nullptr;
}

int alloc_buffers(lb_sim *s)
{
    free_buffers(s);
    s->xoff = (s->cs && s->fixed) ? 1 : 0;
    s->pitch = s->Nx + 2 * s->xoff;
    s->plane = padded_plane((long long)s->pitch * s->Ny, s->esize);
    s->buf_bytes = (size_t)s->K * (size_t)s->plane * s->esize;
    if (!s->cs)  // the moment planes (fd_mom_offset), in the arithmetic type
        s->buf_bytes = (size_t)fd_mom_offset(s->K, s->plane, s->esize) +
                       3 * (size_t)s->plane * (s->prec == P64 ? sizeof(double) : sizeof(float));
    for (int i = 0; i < s->nbuf; ++i) {
        if (hipMalloc(&s->buf[i], s->buf_bytes) != hipSuccess) {
            (void)hipGetLastError();
            free_buffers(s);
            return LB_ENOMEM;
        }
        if (hipMemsetAsync(s->buf[i], 0, s->buf_bytes, s->stream) != hipSuccess) return LB_EDEVICE;
    }
    if (s->prec == P16R) {
        const size_t bytes = (size_t)s->pitch * s->Ny * sizeof(uint32_t);
        if (hipMalloc(&s->d_ref, bytes) != hipSuccess) {
            (void)hipGetLastError();
            free_buffers(s);
            return LB_ENOMEM;
        }
        if (hipMemsetAsync(s->d_ref, 0, bytes, s->stream) != hipSuccess) return LB_EDEVICE;
    }
    return LB_OK;
}

template <typename T>
T *bufp(lb_sim *s, int i)
{
    return static_cast<T *>(s->buf[i]);
}

// Dispatch on the storage type.
template <typename F>
hipError_t with_type(lb_sim *s, F &&f)
{
    switch (s->prec) {
    case P16:
    case P16R: return f((__half *)nullptr);
    case P64: return f((double *)nullptr);
    default: return f((float *)nullptr);
    }
}

int dev_status(hipError_t e) { return e == hipSuccess ? LB_OK : (e == hipErrorOutOfMemory ? LB_ENOMEM : LB_EDEVICE); }

// Current canonical-state buffer.
int state_index(const lb_sim *s) { return s->cs ? s->cur : 0; }

// Whether plain FD steps take the temporally blocked kernel.
bool fused_active(const lb_sim *s)
{
    return !s->cs && !s->imex && s->prec == P32 && s->fd_fused_ys > 0 && fd_fused_supported(s->Q, s->fixed);
}

// Advance one step; diag non-null fuses the diagnostics of the input state.
template <typename T>
hipError_t step_once(lb_sim *s, bool with_diag)
{
    using CT = typename Arith<T>::type;
    const Params<CT> p = make_params<CT>(s);
    DiagArgs<CT> d{};
    d.partial = s->d_partial;
    if (s->probe) {
        if constexpr (sizeof(CT) == 8) {
            d.ax = s->d_probe64;
            d.ay = s->d_probe64 + s->Nx;
            d.bx = s->d_probe64 + s->Nx + s->Ny;
            d.by = s->d_probe64 + 2 * s->Nx + s->Ny;
        } else {
            d.ax = s->d_probe32;
            d.ay = s->d_probe32 + s->Nx;
            d.bx = s->d_probe32 + s->Nx + s->Ny;
            d.by = s->d_probe32 + 2 * s->Nx + s->Ny;
        }
    }
    const DiagArgs<CT> *dp = with_diag ? &d : nullptr;
    hipError_t e = hipSuccess;
    if (s->cs) {
        e = launch_cs_step_st<T>(bufp<T>(s, s->cur), bufp<T>(s, 1 - s->cur), p, dp, s->stream, s->cs_threads,
                                 s->cs_nt);
        s->cur ^= 1;
    } else {
        T *g = bufp<T>(s, 0), *a = bufp<T>(s, 1), *b = bufp<T>(s, 2);
        if (s->imex) {
            // IMEX-SSP2(2,2,2): f1 = relax(g) -> A; y = f1 + dt L(f1) -> B;
            // (f2, base) -> (B, A); g' = base + (f2 + dt L(f2) - base) / 2.
            // The sampled diagnostics are those of f1, whose moments are g's.
            const double r = s->dt / s->tau;
            e = launch_fd_imex<T>(0, a, g, nullptr, p, r, s->stream);
            if (e == hipSuccess) e = launch_fd_stage<T>(a, nullptr, b, 1, p, dp, s->stream, dp ? 8 : s->fd_rows);
            if (e == hipSuccess) e = launch_fd_imex<T>(1, a, g, b, p, r, s->stream);
            if (e == hipSuccess) e = launch_fd_stage<T>(b, a, g, 4, p, nullptr, s->stream, s->fd_rows_rest);
        } else if (std::is_same<T, float>::value && !dp && fused_active(s)) {
            // the three stages in one launch into A, which becomes the state
            if constexpr (std::is_same<T, float>::value) {
                e = launch_fd_fused(g, a, p, s->fd_fused_ys, s->stream);
                if (e == hipSuccess) std::swap(s->buf[0], s->buf[1]);
            }
        } else {
            e = launch_fd_stage<T>(g, nullptr, a, 1, p, dp, s->stream, dp ? 8 : s->fd_rows);
            if (e == hipSuccess) e = launch_fd_stage<T>(a, g, b, 2, p, nullptr, s->stream, s->fd_rows_rest);
            if (e == hipSuccess) e = launch_fd_stage<T>(b, g, g, 3, p, nullptr, s->stream, s->fd_rows_rest);
        }
    }
    if (e == hipSuccess) ++s->steps;
    return e;
}

// ---------------------------------------------------------------------
// Graph replay of plain steps.  The kernel arguments of a run of steps
// without sampling repeat exactly (CS, and FD with the fused kernel: after an
// even number of steps the ping-pong pair is back at its start; FD stage
// launches: the buffers never move), so a
// captured graph of G steps replays any run of G steps with one launch.
// FP16 storage is excluded: its stochastic rounding draws fresh random bits
// every step, which a replayed graph would repeat.
int graph_len(const lb_sim *s)
{
    if (s->prec == P16 || s->prec == P16R) return 0;
    int g = s->graph_steps < 0 ? (s->cs ? 8 : 4) : s->graph_steps;
    // CS, and FD with the fused kernel: the two state buffers alternate, so
    // a replayed run must return them to their start
    if ((s->cs || fused_active(s)) && (g & 1)) ++g;
    return g;
}

void drop_graphs(lb_sim *s)
{
    for (auto &g : s->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

template <typename T>
hipError_t capture_steps(lb_sim *s, int G, hipGraphExec_t *out)
{
    hipError_t e = hipSuccess;
    if (!s->cap_stream) e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    const long long steps0 = s->steps;
    const int cur0 = s->cur;
    hipStream_t user = s->stream;
    s->stream = s->cap_stream;
    e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int i = 0; i < G && e == hipSuccess; ++i) e = step_once<T>(s, false);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
    }
    s->stream = user;
    s->steps = steps0;
    s->cur = cur0;
    return e;
}

// n steps without sampling: whole graphs, then single launches.
template <typename T>
hipError_t plain_steps(lb_sim *s, long long n)
{
    hipError_t e = hipSuccess;
    const int G = graph_len(s);
    while (G > 0 && n >= G && e == hipSuccess) {
        hipGraphExec_t &ge = s->graph[s->cs ? s->cur : 0];
        if (!ge) e = capture_steps<T>(s, G, &ge);
        if (e == hipSuccess) e = hipGraphLaunch(ge, s->stream);
        if (e == hipSuccess) {
            s->steps += G;  // CS: G is even, the current buffer is unchanged
            n -= G;
        }
    }
    for (; n > 0 && e == hipSuccess; --n) e = step_once<T>(s, false);
    return e;
}

// ---------------------------------------------------------------------
// Autotuning of the plain-step launch shapes.  Candidates are timed on the
// handle's own buffers with launches that leave the state untouched.  CS: a
// step from the current buffer into the other one (which the next step
// overwrites) with workgroup size cs_threads and store policy cs_nt.  With
// `scratch` (a device buffer of the handle's buffer size) the timed CS
// launches ping-pong between the other buffer and it, as consecutive steps
// do, so that each launch reads what the previous one wrote: whether that is
// still in the last-level cache is what the store policy changes.
template <typename T>
hipError_t time_candidate(lb_sim *s, int cs_threads, bool cs_nt, int reps, float *ms, void *scratch = nullptr)
{
    using CT = typename Arith<T>::type;
    const Params<CT> p = make_params<CT>(s);
    int nlaunch = 0;
    auto launch = [&]() -> hipError_t {
        const T *src = bufp<T>(s, s->cur);
        T *dst = bufp<T>(s, 1 - s->cur);
        if (scratch && nlaunch > 0) {
            // other -> scratch, scratch -> other, ...
            T *x = bufp<T>(s, 1 - s->cur), *y = static_cast<T *>(scratch);
            src = (nlaunch & 1) ? x : y;
            dst = (nlaunch & 1) ? y : x;
        }
        ++nlaunch;
        return launch_cs_step_st<T>(src, dst, p, nullptr, s->stream, cs_threads, cs_nt);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

// Tile heights of the FD stage launches timed against each other over whole
// steps: blocks of `block` consecutive steps per candidate (first-stage rows,
// later-stage rows), the candidates taking turns over as many rounds as there
// are candidates, each round starting one candidate further on, with an
// event between consecutive blocks.  The shader clock drifts under sustained
// load (by up to ~15 % within milliseconds; it recovers when the device
// idles), and timed in a fixed order the block times fell steadily with
// their place in the round; rotated, every candidate takes every place once.
// One untimed block per candidate first.  ms[i] is the time of candidate
// i's nc * block steps.  With `copy` (a device buffer of the
// handle's buffer size holding a copy of the state) the steps are plain steps
// of that copy, with their traffic and cache reuse; without it each step
// writes A, B and A again from the untouched state.
template <typename T>
hipError_t time_fd_rows(lb_sim *s, const std::vector<std::pair<int, int>> &cand, int block, std::vector<float> &ms,
                        void *copy)
{
    using CT = typename Arith<T>::type;
    const Params<CT> p = make_params<CT>(s);
    T *g = copy ? static_cast<T *>(copy) : bufp<T>(s, 0), *a = bufp<T>(s, 1), *b = bufp<T>(s, 2);
    T *out3 = copy ? g : a;
    const size_t nc = cand.size(), n = nc * nc;
    auto which = [&](size_t j) { return (j % nc + j / nc) % nc; };  // round j / nc, place j % nc
    auto step = [&](const std::pair<int, int> &c) {
        hipError_t e = launch_fd_stage<T>(g, nullptr, a, 1, p, nullptr, s->stream, c.first);
        if (e == hipSuccess) e = launch_fd_stage<T>(a, g, b, 2, p, nullptr, s->stream, c.second);
        if (e == hipSuccess) e = launch_fd_stage<T>(b, g, out3, 3, p, nullptr, s->stream, c.second);
        return e;
    };
    ms.assign(nc, 0.0f);
    std::vector<hipEvent_t> ev(n + 1, nullptr);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i <= n && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    for (size_t i = 0; i < nc; ++i)  // warm-up
        for (int k = 0; k < block && e == hipSuccess; ++k) e = step(cand[i]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], s->stream);
    for (size_t j = 0; j < n && e == hipSuccess; ++j) {
        for (int k = 0; k < block && e == hipSuccess; ++k) e = step(cand[which(j)]);
        if (e == hipSuccess) e = hipEventRecord(ev[j + 1], s->stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[n]);
    for (size_t j = 0; j < n && e == hipSuccess; ++j) {
        float t = 0.0f;
        e = hipEventElapsedTime(&t, ev[j], ev[j + 1]);
        ms[which(j)] += t;
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    return e;
}

// Time `reps` launches of the temporally blocked FD step from the state into
// buffer A (which the next step overwrites; the state is untouched).
hipError_t time_fused(lb_sim *s, int ys, int reps, float *ms)
{
    const Params<float> p = make_params<float>(s);
    const float *g = bufp<float>(s, 0);
    float *a = bufp<float>(s, 1);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_fd_fused(g, a, p, ys, s->stream);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_fd_fused(g, a, p, ys, s->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

int diag_blocks_fused(const lb_sim *s) { return s->cs ? cs_diag_blocks(s->Nx, s->Ny) : fd_diag_blocks(s->Nx, s->Ny); }

// Convert the device sums (sum drho, sum jx, sum jy, sum rho u^2/2, sum u.phi)
// into {M, Px, Py, E, A}; `vscale` converts the kernel's velocity unit.
void finish_diag(const lb_sim *s, const double *raw, double vscale, double *out)
{
    const double nodes = (double)s->Nx * (double)s->Ny;
    out[0] = s->rho0 * nodes + raw[0];
    out[1] = raw[1] * vscale;
    out[2] = raw[2] * vscale;
    out[3] = raw[3] * vscale * vscale;
    out[4] = s->probe ? raw[4] * vscale / s->probe_den : 0.0;
}

template <typename T>
hipError_t reduce_into(lb_sim *s, double *d_dst)
{
    const Params<double> p = make_params<double>(s);
    DiagArgs<double> d{};
    d.partial = s->d_partial;
    if (s->probe) {
        d.ax = s->d_probe64;
        d.ay = s->d_probe64 + s->Nx;
        d.bx = s->d_probe64 + s->Nx + s->Ny;
        d.by = s->d_probe64 + 2 * s->Nx + s->Ny;
    }
    hipError_t e = launch_reduce<T>(bufp<T>(s, state_index(s)), s->cs, p, d, s->stream);
    if (e == hipSuccess) e = launch_diag_finalize(s->d_partial, reduce_diag_blocks(s->Nx, s->Ny), d_dst, s->stream);
    return e;
}

int set_last_error(int code) { return fail(code); }

int validate_create(int model_flags, int Nx, int Ny, double tau, double dt, double ds, int N)
{
    const int model = model_flags & 0xff;
    const int precbits = model_flags & LB_PRECISION_MASK;
    if ((model_flags & ~(0xff | LB_PRECISION_MASK | LB_IMEX)) != 0) return LB_EINVAL;
    // storage relative to a reference equilibrium: collision-streaming only
    if (precbits == LB_FP16_REF && model != LB_CS_D2Q9) return LB_EINVAL;
    const bool imex = (model_flags & LB_IMEX) != 0;
    ModelInfo mi{};
    if (!(tau > 0) || !(dt > 0) || !(ds > 0) || !std::isfinite(tau) || !std::isfinite(dt) || !std::isfinite(ds) ||
        Nx < 1 || Ny < 1 || (long long)Nx * Ny > (1LL << 30) || !model_info(model, ds, dt, &mi))
        return LB_EINVAL;
    if (model == LB_CS_D2Q9) {
        // positive viscosity nu = c_s^2 (tau - dt/2) (Section 2)
        if (N != 2 || !(tau > 0.5 * dt) || imex) return LB_EINVAL;
        return LB_OK;
    }
    if (N < 1 || N > mi.Q - 1) return LB_EINVAL;
    // the stage kernels address a population plane, and a moment plane in the
    // arithmetic type (at least 4 bytes a value), with 32-bit byte offsets;
    // planes are padded (padded_plane)
    const int esize = precbits == LB_FP64 ? 8 : (precbits == LB_FP16_SHIFTED ? 2 : 4);
    const long long csize = precbits == LB_FP64 ? 8 : 4;
    if (padded_plane((long long)Nx * Ny, esize) * csize >= (1LL << 32)) return LB_EINVAL;
    // CFL = max |v_k,alpha| dt / ds <= 1 and dt < tau (Section 4.1); dt == tau
    // is accepted, as in the shear-wave runs of Section 4.2
    const double vmax = mi.xi[mi.Q - 1];
    if (vmax * dt / ds > 1.0 + 1e-12) return LB_ECFL;
    if (!imex && dt > tau * (1.0 + 1e-12)) return LB_ESTIFF;
    return LB_OK;
}

template Params<float> make_params<float>(const lb_sim *);
template Params<double> make_params<double>(const lb_sim *);

bool all_finite(const double *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

}  // namespace lbm

extern "C" {

int lb_last_error(void) { return g_last_error; }

const char *lb_strerror(int code)
{
    switch (code) {
    case LB_OK: return "ok";
    case LB_EINVAL: return "invalid argument";
    case LB_ECFL: return "time step violates the CFL bound max|v| dt/ds <= 1";
    case LB_ESTIFF: return "FD time step larger than the relaxation time";
    case LB_ENOMEM: return "device memory exhausted";
    case LB_EDEVICE: return "HIP runtime error";
    case LB_ENAN: return "non-finite result";
    case LB_EBUSY: return "server budget or slots exhausted";
    case LB_ESTATE: return "call out of order";
    default: return "unknown status";
    }
}

int lb_model_info(int model, double ds, double dt, double *vx, double *vy, double *w, double *cs)
{
    ModelInfo mi{};
    if (!model_info(model, ds, dt, &mi)) return fail(LB_EINVAL);
    for (int k = 0; k < mi.K; ++k) {
        if (vx) vx[k] = mi.vx[k];
        if (vy) vy[k] = mi.vy[k];
        if (w) w[k] = mi.w[k];
    }
    if (cs) *cs = mi.cs;
    return mi.K;
}

lb_sim *lb_create(int model_flags, int Nx, int Ny, double tau, double dt, double ds, int N)
{
    const int vrc = lbm::validate_create(model_flags, Nx, Ny, tau, dt, ds, N);
    if (vrc != LB_OK) {
        fail(vrc);
        return nullptr;
    }
    const int model = model_flags & 0xff;
    const int precbits = model_flags & LB_PRECISION_MASK;
    ModelInfo mi{};
    model_info(model, ds, dt, &mi);
    const bool cs = model == LB_CS_D2Q9;
    lb_sim *s = new (std::nothrow) lb_sim();
    if (!s) {
        fail(LB_ENOMEM);
        return nullptr;
    }
    if (hipGetDevice(&s->device) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        fail(LB_EDEVICE);
        return nullptr;
    }
    s->model = model;
    s->imex = (model_flags & LB_IMEX) != 0;
    s->prec = precbits == LB_FP16_SHIFTED ? P16 : (precbits == LB_FP64 ? P64 : (precbits == LB_FP16_REF ? P16R : P32));
    s->cs = cs;
    s->Nx = Nx;
    s->Ny = Ny;
    s->K = mi.K;
    s->Q = mi.Q;
    s->N = N;
    s->tau = tau;
    s->dt = dt;
    s->ds = ds;
    s->mi = mi;
    s->esize = elem_size(s->prec);
    s->nbuf = cs ? 2 : 3;
    if (hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        fail(LB_EDEVICE);
        return nullptr;
    }
    s->stream = s->own_stream;
    int rc = alloc_buffers(s);
    if (rc == LB_OK) {
        int blocks = cs_diag_blocks(Nx, Ny);
        blocks = std::max(blocks, fd_diag_blocks(Nx, Ny));
        blocks = std::max(blocks, reduce_diag_blocks(Nx, Ny));
        s->partial_blocks = blocks;
        // kDiag + 1 sums per block: the field reduction also sums phi . phi
        if (hipMalloc(&s->d_partial, sizeof(double) * (kDiag + 1) * (size_t)blocks) != hipSuccess ||
            hipMalloc(&s->d_out, sizeof(double) * kDiag) != hipSuccess) {
            (void)hipGetLastError();
            rc = LB_ENOMEM;
        }
    }
    if (rc != LB_OK) {
        lb_destroy(s);
        fail(rc);
        return nullptr;
    }
    g_last_error = LB_OK;
    return s;
}

void lb_destroy(lb_sim *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    drop_graphs(s);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    free_buffers(s);
    if (s->d_partial) (void)hipFree(s->d_partial);
    if (s->d_out) (void)hipFree(s->d_out);
    if (s->d_probe64) (void)hipFree(s->d_probe64);
    if (s->d_probe32) (void)hipFree(s->d_probe32);
    if (s->d_series) (void)hipFree(s->d_series);
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    delete s;
}

int lb_set_bc_x(lb_sim *s, double rho_left, double rho_right)
{
    if (!s || !(rho_left > 0) || !(rho_right > 0) || !std::isfinite(rho_left) || !std::isfinite(rho_right))
        return fail(LB_EINVAL);
    if (s->ready) return fail(LB_ESTATE);
    if (s->prec == P16R) return fail(LB_EINVAL);  // periodic only
    drop_graphs(s);
    const bool relayout = s->cs && !s->fixed;
    s->fixed = true;
    s->rho_l = rho_left;
    s->rho_r = rho_right;
    if (relayout) {
        int rc = alloc_buffers(s);
        if (rc != LB_OK) return fail(rc);
    }
    return LB_OK;
}

int lb_set_weno_eps(lb_sim *s, double eps)
{
    if (!s || !(eps > 0) || !std::isfinite(eps)) return fail(LB_EINVAL);
    if (s->cs) return fail(LB_EINVAL);
    // the WENO weights use (eps + beta)^4, which must stay a normal number
    const double lo = s->prec == P64 ? 1e-75 : 1e-9, hi = s->prec == P64 ? 1e75 : 1e9;
    if (eps < lo || eps > hi) return fail(LB_EINVAL);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    drop_graphs(s);
    s->eps = eps;
    return LB_OK;
}

int lb_set_stream(lb_sim *s, void *hip_stream)
{
    if (!s) return fail(LB_EINVAL);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    s->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : s->own_stream;
    return LB_OK;
}

int lb_synchronize(lb_sim *s)
{
    if (!s) return fail(LB_EINVAL);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    return LB_OK;
}

long long lb_steps_done(const lb_sim *s) { return s ? s->steps : -1; }

size_t lb_device_bytes(const lb_sim *s)
{
    if (!s) return 0;
    return s->nbuf * s->buf_bytes + sizeof(double) * ((kDiag + 1) * (size_t)s->partial_blocks + kDiag) +
           (s->d_probe64 ? 2 * (s->Nx + s->Ny) * (sizeof(double) + sizeof(float)) : 0) +
           sizeof(double) * kDiag * (size_t)s->series_cap +
           (s->d_ref ? (size_t)s->pitch * s->Ny * sizeof(uint32_t) : 0);
}

// Upload fields / state through a temporary device buffer.
static int upload(lb_sim *s, const double *h, size_t n, double **d)
{
    *d = nullptr;
    if (hipMalloc(d, n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return LB_ENOMEM;
    }
    if (hipMemcpyAsync(*d, h, n * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess) return LB_EDEVICE;
    return LB_OK;
}

static int ghosts_and(lb_sim *s)
{
    if (!(s->cs && s->fixed)) return LB_OK;
    const Params<double> p = make_params<double>(s);
    for (int i = 0; i < s->nbuf; ++i) {
        hipError_t e = with_type(s, [&](auto *tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            return launch_fill_ghosts<T>(bufp<T>(s, i), p, s->stream);
        });
        if (e != hipSuccess) return dev_status(e);
    }
    return LB_OK;
}

int lb_init(lb_sim *s, const double *rho, const double *ux, const double *uy)
{
    if (!s || !rho || !ux || !uy) return fail(LB_EINVAL);
    const size_t n = (size_t)s->Nx * s->Ny;
    double mean = 0.0;
    for (size_t i = 0; i < n; ++i) {
        if (!(rho[i] > 0) || !std::isfinite(rho[i]) || !std::isfinite(ux[i]) || !std::isfinite(uy[i]))
            return fail(LB_EINVAL);
        mean += rho[i];
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    drop_graphs(s);
    s->rho0 = mean / (double)n;
    s->cur = 0;
    int rc = ghosts_and(s);
    if (rc != LB_OK) return fail(rc);
    std::vector<double> host(3 * n);
    std::memcpy(host.data(), rho, n * sizeof(double));
    std::memcpy(host.data() + n, ux, n * sizeof(double));
    std::memcpy(host.data() + 2 * n, uy, n * sizeof(double));
    double *d = nullptr;
    rc = upload(s, host.data(), 3 * n, &d);
    if (rc == LB_OK) {
        const Params<double> p = make_params<double>(s);
        hipError_t e = with_type(s, [&](auto *tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipError_t e = hipSuccess;
            if (s->d_ref) e = launch_ref_from_velocity(s->d_ref, d + n, d + 2 * n, p, 1.0 / s->mi.cl, s->stream);
            if (e == hipSuccess) e = launch_init<T>(bufp<T>(s, 0), d, d + n, d + 2 * n, s->cs, p, s->stream);
            if (e == hipSuccess && !s->cs)
                e = launch_fd_moments<T>(bufp<T>(s, 0), make_params<typename Arith<T>::type>(s), s->stream);
            return e;
        });
        rc = dev_status(e);
        if (hipStreamSynchronize(s->stream) != hipSuccess && rc == LB_OK) rc = LB_EDEVICE;
    }
    if (d) (void)hipFree(d);
    if (rc != LB_OK) return fail(rc);
    s->steps = 0;
    s->ready = true;
    return LB_OK;
}

int lb_set_state(lb_sim *s, const double *f)
{
    if (!s || !f) return fail(LB_EINVAL);
    const size_t nodes = (size_t)s->Nx * s->Ny, n = nodes * s->K;
    double mass = 0.0;
    for (size_t i = 0; i < n; ++i) {
        if (!std::isfinite(f[i])) return fail(LB_EINVAL);
        mass += f[i];
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    drop_graphs(s);
    s->rho0 = mass / (double)nodes;
    s->cur = 0;
    int rc = ghosts_and(s);
    if (rc != LB_OK) return fail(rc);
    double *d = nullptr;
    rc = upload(s, f, n, &d);
    if (rc == LB_OK) {
        const Params<double> p = make_params<double>(s);
        hipError_t e = with_type(s, [&](auto *tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipError_t e = hipSuccess;
            if (s->d_ref) e = launch_ref_from_state(s->d_ref, d, p, s->stream);
            if (e == hipSuccess) e = launch_set_state<T>(bufp<T>(s, 0), d, s->cs, p, s->stream);
            if (e == hipSuccess && !s->cs)
                e = launch_fd_moments<T>(bufp<T>(s, 0), make_params<typename Arith<T>::type>(s), s->stream);
            return e;
        });
        rc = dev_status(e);
        if (hipStreamSynchronize(s->stream) != hipSuccess && rc == LB_OK) rc = LB_EDEVICE;
    }
    if (d) (void)hipFree(d);
    if (rc != LB_OK) return fail(rc);
    s->steps = 0;
    s->ready = true;
    return LB_OK;
}

int lb_get_state(lb_sim *s, double *f)
{
    if (!s || !f) return fail(LB_EINVAL);
    if (!s->ready) return fail(LB_ESTATE);
    const size_t n = (size_t)s->Nx * s->Ny * s->K;
    double *d = nullptr;
    if (hipMalloc(&d, n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LB_ENOMEM);
    }
    const Params<double> p = make_params<double>(s);
    hipError_t e = with_type(s, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return launch_get_state<T>(bufp<T>(s, state_index(s)), d, s->cs, p, s->stream);
    });
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(dev_status(e));
    return LB_OK;
}

int lb_moments(lb_sim *s, double *rho, double *ux, double *uy)
{
    if (!s) return fail(LB_EINVAL);
    if (!s->ready) return fail(LB_ESTATE);
    const size_t n = (size_t)s->Nx * s->Ny;
    double *d = nullptr;
    if (hipMalloc(&d, 3 * n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LB_ENOMEM);
    }
    const Params<double> p = make_params<double>(s);
    hipError_t e = with_type(s, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return launch_moments<T>(bufp<T>(s, state_index(s)), d, d + n, d + 2 * n, s->cs, p, s->stream);
    });
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, d, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && ux) e = hipMemcpyAsync(ux, d + n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && uy)
        e = hipMemcpyAsync(uy, d + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(dev_status(e));
    return LB_OK;
}

int lb_set_probe(lb_sim *s, const double *ax, const double *ay, const double *bx, const double *by)
{
    if (!s) return fail(LB_EINVAL);
    if (!ax && !ay && !bx && !by) {
        s->probe = false;
        return LB_OK;
    }
    if (!ax || !ay || !bx || !by) return fail(LB_EINVAL);
    const int Nx = s->Nx, Ny = s->Ny;
    const size_t n = 2 * (size_t)(Nx + Ny);
    std::vector<double> h(n);
    std::memcpy(h.data(), ax, Nx * sizeof(double));
    std::memcpy(h.data() + Nx, ay, Ny * sizeof(double));
    std::memcpy(h.data() + Nx + Ny, bx, Nx * sizeof(double));
    std::memcpy(h.data() + 2 * Nx + Ny, by, Ny * sizeof(double));
    if (!all_finite(h.data(), n)) return fail(LB_EINVAL);
    // sum phi.phi = (sum ax^2)(sum ay^2) + (sum bx^2)(sum by^2)
    double sax = 0, say = 0, sbx = 0, sby = 0;
    for (int i = 0; i < Nx; ++i) {
        sax += ax[i] * ax[i];
        sbx += bx[i] * bx[i];
    }
    for (int j = 0; j < Ny; ++j) {
        say += ay[j] * ay[j];
        sby += by[j] * by[j];
    }
    const double den = sax * say + sbx * sby;
    if (!(den > 0)) return fail(LB_EINVAL);
    std::vector<float> h32(h.begin(), h.end());
    if (!s->d_probe64) {
        if (hipMalloc(&s->d_probe64, n * sizeof(double)) != hipSuccess ||
            hipMalloc(&s->d_probe32, n * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LB_ENOMEM);
        }
    }
    if (hipMemcpyAsync(s->d_probe64, h.data(), n * sizeof(double), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_probe32, h32.data(), n * sizeof(float), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return fail(LB_EDEVICE);
    s->probe = true;
    s->probe_den = den;
    return LB_OK;
}

int lb_step(lb_sim *s, int nsteps)
{
    if (!s || nsteps < 0) return fail(LB_EINVAL);
    if (!s->ready) return fail(LB_ESTATE);
    hipError_t e = with_type(s, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return plain_steps<T>(s, nsteps);
    });
    if (e != hipSuccess) return fail(dev_status(e));
    return LB_OK;
}

namespace {

// Launch shapes chosen by lb_autotune, per device and simulation shape (the
// timings depend on the kernels and the grid, not on tau, dt or the state),
// shared by every handle of the process.
struct TuneKey {
    int device, model, prec, fixed, imex, Nx, Ny, N;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(device, model, prec, fixed, imex, Nx, Ny, N) <
               std::tie(o.device, o.model, o.prec, o.fixed, o.imex, o.Nx, o.Ny, o.N);
    }
};
struct TuneVal {
    int cs_threads, fd_rows, fd_rows_rest, fd_fused_ys;
    bool cs_nt;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;

TuneKey tune_key(const lb_sim *s)
{
    return {s->device, s->model, (int)s->prec, s->fixed ? 1 : 0, s->imex ? 1 : 0, s->Nx, s->Ny, s->N};
}

}  // namespace

int lb_tuning_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
    return LB_OK;
}

int lb_tuning_cache_size(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return (int)g_tune_cache.size();
}

int lb_autotune(lb_sim *s, int reps)
{
    if (!s || reps < 1 || reps > 1000) return fail(LB_EINVAL);
    if (!s->ready) return fail(LB_ESTATE);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    const TuneKey key = tune_key(s);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            const TuneVal &v = it->second;
            if (v.cs_threads != s->cs_threads || v.fd_rows != s->fd_rows || v.fd_rows_rest != s->fd_rows_rest ||
                v.fd_fused_ys != s->fd_fused_ys || v.cs_nt != s->cs_nt)
                drop_graphs(s);
            s->cs_threads = v.cs_threads;
            s->cs_nt = v.cs_nt;
            s->fd_rows = v.fd_rows;
            s->fd_rows_rest = v.fd_rows_rest;
            s->fd_fused_ys = v.fd_fused_ys;
            return LB_OK;
        }
    }
    // CS vector rows: a scratch buffer for timing consecutive steps (without
    // it, the workgroup sizes are timed from the current buffer and the
    // stores stay plain); FD: a copy of the state for timing plain steps
    // (without it, steps that leave the state in place)
    const bool cs_vec = s->cs && !s->fixed && s->Nx % (s->prec == P64 ? 2 : 4) == 0;
    void *scratch = nullptr;
    if ((cs_vec || !s->cs) && hipMalloc(&scratch, s->buf_bytes) != hipSuccess) {
        (void)hipGetLastError();
        scratch = nullptr;
    }
    if (scratch && !s->cs &&
        hipMemcpyAsync(scratch, s->buf[0], s->buf_bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess) {
        (void)hipFree(scratch);
        return fail(LB_EDEVICE);
    }
    // the fastest of the CS candidates (workgroup size, store policy) timed
    // by f(candidate, &ms).  The candidates take turns over as many rounds as
    // there are candidates, each round starting one candidate further on, and
    // each keeps its best time: the shader clock drifts by up to ~15 % over
    // the tuning, and in a fixed order the times follow the place in the
    // round; rotated, every candidate takes every place once.
    auto pick = [&](size_t nc, auto &&f, size_t *arg) -> hipError_t {
        std::vector<float> best(nc, 0.0f);
        for (size_t round = 0; round < nc; ++round)
            for (size_t j = 0; j < nc; ++j) {
                const size_t i = (j + round) % nc;
                float ms = 0.0f;
                const hipError_t e = f(i, &ms);
                if (e != hipSuccess) return e;
                if (round == 0 || ms < best[i]) best[i] = ms;
            }
        *arg = 0;
        for (size_t i = 1; i < nc; ++i)
            if (best[i] < best[*arg]) *arg = i;
        return hipSuccess;
    };
    int cs_threads = s->cs_threads, rows1 = s->fd_rows, rows_rest = s->fd_rows_rest;
    bool cs_nt = false;
    hipError_t e = hipSuccess;
    if (s->cs) {
        if (cs_vec) {
            const int threads[4] = {0, 256, 512, 1024};
            size_t arg = 0;
            e = pick(4, [&](size_t i, float *ms) {
                return with_type(s, [&](auto *tag) {
                    using T = std::remove_pointer_t<decltype(tag)>;
                    return time_candidate<T>(s, threads[i], false, reps, ms, scratch);
                });
            }, &arg);
            if (e == hipSuccess) cs_threads = threads[arg];
            // then the store policy at that workgroup size: non-temporal
            // stores pay only when the state is far larger than the
            // last-level cache, which the timing finds out
            if (e == hipSuccess && scratch) {
                e = pick(2, [&](size_t i, float *ms) {
                    return with_type(s, [&](auto *tag) {
                        using T = std::remove_pointer_t<decltype(tag)>;
                        return time_candidate<T>(s, cs_threads, i == 1, reps, ms, scratch);
                    });
                }, &arg);
                if (e == hipSuccess) cs_nt = arg == 1;
            }
        }
    }
    // FD: the four pairs of tile heights (first stage, later stages), timed
    // over blocks of whole steps taking turns (blocks of at least 10 steps:
    // two candidates may differ by 1-2 %); per step
    float fd_step_ms = 0.0f;
    if (!s->cs) {
        const std::vector<std::pair<int, int>> cand = {{8, 8}, {8, 4}, {4, 8}, {4, 4}};
        const int block = std::max(reps, 10);
        std::vector<float> t;
        e = with_type(s, [&](auto *tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            return time_fd_rows<T>(s, cand, block, t, scratch);
        });
        if (e == hipSuccess) {
            size_t arg = 0;
            for (size_t i = 1; i < cand.size(); ++i)
                if (t[i] < t[arg]) arg = i;
            rows1 = cand[arg].first;
            rows_rest = cand[arg].second;
            fd_step_ms = t[arg] / (float)(block * cand.size());
        }
    }
    // FD: the stage launches (with the tile heights just chosen) against the
    // temporally blocked kernel with y-segments of 32, 64 and 128 rows
    int fused = 0;
    if (e == hipSuccess && !s->cs && !s->imex && s->prec == P32 && fd_fused_supported(s->Q, s->fixed)) {
        float best = fd_step_ms;  // per step
        for (int ys : {32, 64, 128}) {
            float tf = 0.0f;
            if (e == hipSuccess) e = time_fused(s, ys, reps, &tf);
            if (e == hipSuccess && tf / (float)reps < best) {
                best = tf / (float)reps;
                fused = ys;
            }
        }
    }
    if (scratch) {
        // the timed launches are complete (each timing waits for its end event)
        if (hipFree(scratch) != hipSuccess && e == hipSuccess) e = hipErrorUnknown;
    }
    if (e != hipSuccess) return fail(dev_status(e));
    drop_graphs(s);
    s->cs_threads = cs_threads;
    s->cs_nt = cs_nt;
    s->fd_rows = rows1;
    s->fd_rows_rest = rows_rest;
    s->fd_fused_ys = fused;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {cs_threads, rows1, rows_rest, fused, cs_nt};
    return LB_OK;
}

int lb_set_cs_nontemporal(lb_sim *s, int on)
{
    if (!s || (on != 0 && on != 1) || !s->cs) return fail(LB_EINVAL);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    if (s->cs_nt != (on != 0)) drop_graphs(s);
    s->cs_nt = on != 0;
    return LB_OK;
}

int lb_get_cs_nontemporal(const lb_sim *s)
{
    if (!s) return fail(LB_EINVAL);
    return s->cs_nt ? 1 : 0;
}

int lb_set_tuning(lb_sim *s, int cs_threads, int fd_rows, int fd_rows_rest)
{
    auto rows_ok = [](int r) { return r == 4 || r == 8; };
    if (!s || cs_threads < 0 || cs_threads > 1024 || cs_threads % 64 || !rows_ok(fd_rows) || !rows_ok(fd_rows_rest))
        return fail(LB_EINVAL);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    drop_graphs(s);
    s->cs_threads = cs_threads;
    s->fd_rows = fd_rows;
    s->fd_rows_rest = fd_rows_rest;
    return LB_OK;
}

int lb_get_tuning(const lb_sim *s, int *cs_threads, int *fd_rows, int *fd_rows_rest)
{
    if (!s || !cs_threads || !fd_rows || !fd_rows_rest) return fail(LB_EINVAL);
    *cs_threads = s->cs_threads;
    *fd_rows = s->fd_rows;
    *fd_rows_rest = s->fd_rows_rest;
    return LB_OK;
}

int lb_set_fd_fused(lb_sim *s, int rows_per_segment)
{
    if (!s || rows_per_segment < 0 || rows_per_segment > 4096) return fail(LB_EINVAL);
    if (rows_per_segment > 0 && (s->cs || s->imex || s->prec != P32 || !fd_fused_supported(s->Q, s->fixed)))
        return fail(LB_EINVAL);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    drop_graphs(s);
    s->fd_fused_ys = rows_per_segment;
    return LB_OK;
}

int lb_get_fd_fused(const lb_sim *s) { return s ? s->fd_fused_ys : fail(LB_EINVAL); }

int lb_set_rounding_seed(lb_sim *s, unsigned seed)
{
    if (!s) return fail(LB_EINVAL);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    drop_graphs(s);
    s->rounding_seed = seed;
    return LB_OK;
}

int lb_set_graph_steps(lb_sim *s, int steps)
{
    if (!s || steps < -1 || steps > 4096) return fail(LB_EINVAL);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(LB_EDEVICE);
    drop_graphs(s);
    s->graph_steps = steps;
    return LB_OK;
}

int lb_reduce(lb_sim *s, double out[5])
{
    if (!s || !out) return fail(LB_EINVAL);
    if (!s->ready) return fail(LB_ESTATE);
    hipError_t e = with_type(s, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return reduce_into<T>(s, s->d_out);
    });
    double raw[kDiag];
    if (e == hipSuccess) e = hipMemcpyAsync(raw, s->d_out, sizeof(raw), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(dev_status(e));
    finish_diag(s, raw, 1.0, out);
    if (!all_finite(out, kDiag)) return fail(LB_ENAN);
    return LB_OK;
}

int lb_reduce_field(lb_sim *s, const double *phi_x, const double *phi_y, double out[5])
{
    if (!s || !out || (!phi_x) != (!phi_y)) return fail(LB_EINVAL);
    if (!s->ready) return fail(LB_ESTATE);
    const size_t n = (size_t)s->Nx * s->Ny;
    if (phi_x && (!all_finite(phi_x, n) || !all_finite(phi_y, n))) return fail(LB_EINVAL);
    double *d = nullptr;
    if (phi_x) {
        if (hipMalloc(&d, 2 * n * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LB_ENOMEM);
        }
    }
    hipError_t e = hipSuccess;
    if (d) e = hipMemcpyAsync(d, phi_x, n * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (d && e == hipSuccess) e = hipMemcpyAsync(d + n, phi_y, n * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
        const Params<double> p = make_params<double>(s);
        e = with_type(s, [&](auto *tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            return launch_reduce_field<T>(bufp<T>(s, state_index(s)), s->cs, p, d, d ? d + n : nullptr,
                                          s->d_partial, s->d_out, s->stream);
        });
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, s->d_out, sizeof(double) * kDiag, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (d) (void)hipFree(d);
    if (e != hipSuccess) return fail(dev_status(e));
    if (!all_finite(out, kDiag)) return fail(LB_ENAN);
    return LB_OK;
}

int lb_reduce_field_noalloc(lb_sim *s, const double *d_phi_x, const double *d_phi_y, double *d_out)
{
    if (!s || !d_out || (!d_phi_x) != (!d_phi_y)) return fail(LB_EINVAL);
    if (!s->ready) return fail(LB_ESTATE);
    // the per-block partials live in the library's fixed device array of the
    // simulation's device (reduce_field_scratch), not in allocated memory
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(LB_EDEVICE);
    if (cur != s->device && hipSetDevice(s->device) != hipSuccess) return fail(LB_EDEVICE);
    double *scratch = nullptr;
    size_t cap = 0;
    hipError_t e = reduce_field_scratch(s->device, &scratch, &cap);
    int rc = dev_status(e);
    if (rc == LB_OK && (size_t)(kDiag + 1) * (size_t)reduce_diag_blocks(s->Nx, s->Ny) > cap) rc = LB_EINVAL;
    if (rc == LB_OK) {
        const Params<double> p = make_params<double>(s);
        e = with_type(s, [&](auto *tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            return launch_reduce_field<T>(bufp<T>(s, state_index(s)), s->cs, p, d_phi_x, d_phi_y, scratch, d_out,
                                          s->stream);
        });
        rc = dev_status(e);
    }
    if (cur != s->device) (void)hipSetDevice(cur);
    return rc == LB_OK ? LB_OK : fail(rc);
}

int lb_series_reserve(lb_sim *s, int capacity)
{
    if (!s || capacity < 0) return fail(LB_EINVAL);
    if (capacity <= s->series_cap) return LB_OK;
    double *d = nullptr;
    if (hipMalloc(&d, sizeof(double) * kDiag * (size_t)capacity) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LB_ENOMEM);
    }
    hipError_t e = hipSuccess;
    if (!s->series_t.empty())
        e = hipMemcpyAsync(d, s->d_series, sizeof(double) * kDiag * s->series_t.size(), hipMemcpyDeviceToDevice,
                           s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(dev_status(e));
    }
    if (s->d_series) (void)hipFree(s->d_series);
    s->d_series = d;
    s->series_cap = capacity;
    return LB_OK;
}

// Steps with fused sampling: a step samples its input state when
// (steps - base) % every == 0.
static int sampled_steps(lb_sim *s, int nsteps, int every, long long base)
{
    long long need = 0;
    for (long long t = s->steps; t < s->steps + nsteps; ++t)
        if ((t - base) % every == 0) ++need;
    if ((long long)s->series_t.size() + need > s->series_cap) return LB_EBUSY;
    hipError_t e = hipSuccess;
    const long long end = s->steps + nsteps;
    while (s->steps < end && e == hipSuccess) {
        const long long t = s->steps;
        const long long phase = ((t - base) % every + every) % every;
        if (phase != 0) {  // the run of plain steps up to the next sample
            const long long run = std::min(end - t, (long long)every - phase);
            e = with_type(s, [&](auto *tag) {
                using T = std::remove_pointer_t<decltype(tag)>;
                return plain_steps<T>(s, run);
            });
            continue;
        }
        e = with_type(s, [&](auto *tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            return step_once<T>(s, true);
        });
        if (e == hipSuccess) {
            e = launch_diag_finalize(s->d_partial, diag_blocks_fused(s), s->d_series + kDiag * s->series_t.size(),
                                     s->stream);
            s->series_t.push_back(t);
            s->series_fused.push_back(1);
        }
    }
    return dev_status(e);
}

int lb_step_sampled(lb_sim *s, int nsteps, int every)
{
    if (!s || nsteps < 0 || every < 1) return fail(LB_EINVAL);
    if (!s->ready) return fail(LB_ESTATE);
    int rc = sampled_steps(s, nsteps, every, 0);
    return rc == LB_OK ? LB_OK : fail(rc);
}

int lb_series_read(lb_sim *s, double *out, int max_rows)
{
    if (!s || (max_rows > 0 && !out) || max_rows < 0) return fail(LB_EINVAL);
    const int n = (int)s->series_t.size();
    std::vector<double> raw((size_t)kDiag * n);
    hipError_t e = hipSuccess;
    if (n > 0) e = hipMemcpyAsync(raw.data(), s->d_series, raw.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(dev_status(e));
    const int m = std::min(n, max_rows);
    bool finite = true;
    for (int i = 0; i < m; ++i) {
        // fused CS sums are in lattice velocity units (u / c_l); FD and the
        // stand-alone reduction use physical velocities
        out[6 * i] = (double)s->series_t[i];
        finish_diag(s, raw.data() + kDiag * i, (s->series_fused[i] && s->cs) ? s->mi.cl : 1.0, out + 6 * i + 1);
        finite = finite && all_finite(out + 6 * i + 1, kDiag);
    }
    s->series_t.clear();
    s->series_fused.clear();
    if (!finite) return fail(LB_ENAN);
    return m;
}

int lb_run_sampled(lb_sim *s, int nsteps, int every, double *series)
{
    if (!s || nsteps < 0 || every < 1 || !series) return fail(LB_EINVAL);
    if (!s->ready) return fail(LB_ESTATE);
    const int nsamp = nsteps / every + 1;
    s->series_t.clear();
    s->series_fused.clear();
    int rc = lb_series_reserve(s, nsamp);
    if (rc != LB_OK) return rc;
    const long long base = s->steps;
    rc = sampled_steps(s, nsteps, every, base);
    if (rc == LB_OK && nsteps % every == 0) {
        hipError_t e = with_type(s, [&](auto *tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            return reduce_into<T>(s, s->d_series + kDiag * s->series_t.size());
        });
        s->series_t.push_back(s->steps);
        s->series_fused.push_back(0);
        rc = dev_status(e);
    }
    if (rc != LB_OK) {
        s->series_t.clear();
        s->series_fused.clear();
        return fail(rc);
    }
    std::vector<double> rows((size_t)6 * nsamp);
    const int got = lb_series_read(s, rows.data(), nsamp);
    if (got < 0) return got;
    for (int i = 0; i < got; ++i)
        for (int j = 0; j < kDiag; ++j) series[kDiag * i + j] = rows[6 * i + 1 + j];
    return LB_OK;
}

}  // extern "C"

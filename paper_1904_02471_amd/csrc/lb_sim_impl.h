// lb_sim_impl.h -- the simulation handle behind the C ABI and the internal
// helpers that the batch server (lb_server.cpp) shares with it.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "lb.h"
#include "lb_internal.h"
#include "lb_model.h"

namespace lbm {
// storage: FP32, FP16 shifted by w_k rho0, FP64, FP16 relative to a
// reference equilibrium (CS only)
enum Prec { P32 = 0, P16 = 1, P64 = 2, P16R = 3 };
}  // namespace lbm

struct lb_sim {
    int device = 0;  // HIP device current at lb_create, which holds the buffers
    int model = 0;
    lbm::Prec prec = lbm::P32;
    bool cs = true;
    bool imex = false;  // FD: implicit-explicit time stepping (LB_IMEX)
    int Nx = 0, Ny = 0, K = 0, Q = 0, N = 0;
    double tau = 0, dt = 0, ds = 0;
    lbm::ModelInfo mi{};
    double rho0 = 1.0;
    bool fixed = false;
    double rho_l = 1.0, rho_r = 1.0;
    double eps = 1e-6;
    bool ready = false;
    long long steps = 0;
    int cur = 0;  // CS: buffer holding the current state
    int pitch = 0, xoff = 0;
    long long plane = 0;
    size_t esize = 4;
    int nbuf = 0;
    void *buf[3] = {nullptr, nullptr, nullptr};
    size_t buf_bytes = 0;
    hipStream_t stream = nullptr, own_stream = nullptr;
    double *d_partial = nullptr;  // per-block diagnostics partials
    int partial_blocks = 0;
    double *d_out = nullptr;      // kDiag doubles
    bool probe = false;
    double probe_den = 0.0;
    double *d_probe64 = nullptr;  // ax | ay | bx | by
    float *d_probe32 = nullptr;
    double *d_series = nullptr;   // [series_cap][kDiag] raw sums
    int series_cap = 0;
    std::vector<long long> series_t;  // step index of each pending sample
    std::vector<char> series_fused;   // sums in the step kernel's velocity unit
    // Runs of plain steps replay a captured graph of graph_len steps (CS: one
    // per starting buffer; FD: [0]); dropped whenever the parameters change.
    int graph_steps = -1;             // -1: the model's default, 0: no graphs
    unsigned rounding_seed = 0;       // FP16 stochastic rounding: random-bit stream
    // Launch shapes of plain steps (set by lb_autotune / lb_set_tuning): CS
    // vector-row workgroup size (0: one chunk per thread), FD tile rows per
    // thread (8: 64 x 32 tiles, 4: 64 x 16) of the first Runge-Kutta stage and
    // of the later ones (which also read the step's base state).  Results do
    // not depend on them.
    int cs_threads = 0;
    bool cs_nt = false;  // CS vector rows of plain steps: non-temporal stores
    int fd_rows = 8;
    int fd_rows_rest = 8;
    // FD plain steps by the temporally blocked kernel with y-segments of this
    // many rows (0: three stage launches); FP32, periodic, Q = 3 or 4
    int fd_fused_ys = 0;
    uint32_t *d_ref = nullptr;  // LB_FP16_REF: reference velocity per node (packed FP16 pairs)
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr;
};

namespace lbm {

int set_last_error(int code);
// lb_create's parameter checks: LB_OK or the code lb_create would fail with
int validate_create(int model_flags, int Nx, int Ny, double tau, double dt, double ds, int N);
int state_index(const lb_sim *s);
template <typename CT>
Params<CT> make_params(const lb_sim *s);
int dev_status(hipError_t e);
int diag_blocks_fused(const lb_sim *s);
void finish_diag(const lb_sim *s, const double *raw, double vscale, double *out);
// Decay rate of an amplitude series (lb_fit_decay): LB_OK or an LB_E* code.
int fit_decay_rate(const double *t, const double *amp, int n, double omega, double *rate);
// A CS step with a store policy: nt selects non-temporal stores for the
// vector row form of plain steps (sampled steps and scalar rows store
// plainly); launch_cs_step is this with nt = false.
template <typename T>
hipError_t launch_cs_step_st(const T *src, T *dst, const Params<typename Arith<T>::type> &p,
                             const DiagArgs<typename Arith<T>::type> *diag, hipStream_t s, int threads, bool nt);

}  // namespace lbm

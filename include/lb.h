/*
 * lb.h -- C ABI of the MI355X (gfx950) isothermal lattice Boltzmann library.
 *
 * Method: Negro, Busuioc, Ambrus, Gonnella, Lamura, Sofonea, "Comparison
 * between isothermal collision-streaming and finite-difference lattice
 * Boltzmann models", arXiv:1904.02471.
 *
 *   collision-streaming (CS) D2Q9:  Section 2, CS evolution equation
 *       f_k(x + v_k dt, t + dt) - f_k(x, t) = -(dt / tau) (f_k - f_eq_k)
 *   finite-difference (FD) Gauss-Hermite D2Q(Q*Q), Q = 3..6:  Section 2, BGK
 *       equation d_t f_k + v_k . grad f_k = -(f_k - f_eq_k) / tau advanced by
 *       third-order TVD Runge-Kutta with WENO-5 advection
 *   equilibrium: Hermite expansion of the Maxwellian to total order N
 *       (Section 1; second-order form in Section 2)
 *   moments: rho = sum_k f_k, rho u = sum_k f_k v_k (Section 2)
 *
 * Conventions shared by every call
 *   - Fields are row-major [Ny][Nx] float64 host arrays, x fastest; the node
 *     (i, j) sits at (i ds, j ds).  Distributions are [K][Ny][Nx].
 *   - CS D2Q9 population order: 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW,
 *     7 SW, 8 SE; v_k = e_k ds/dt, sound speed c_s = (ds/dt)/sqrt(3); tau
 *     is in the time unit of dt; N must be 2.
 *   - FD population order k = j*Q + i with v_k = (xi_i, xi_j), xi the
 *     ascending roots of the Hermite polynomial He_Q; units c_s = 1
 *     (T = m = 1, Section 4.1); ds is the grid spacing; 1 <= N <= Q-1.
 *   - All pointers are caller-owned host pointers unless stated; the library
 *     never frees caller memory and never keeps a caller pointer after a call
 *     returns.
 *   - Calls on one handle are not thread-safe; distinct handles are
 *     independent.  lb_step is asynchronous on the handle's stream; every
 *     call that returns host data synchronises that stream first.
 *   - Return value: LB_OK (0) or a negative LB_E* code; lb_create returns NULL
 *     on error and lb_last_error() (per thread) gives the code.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* models (low byte of the model_flags argument) */
enum lb_model {
    LB_CS_D2Q9 = 0,
    LB_FD_D2Q9 = 1,
    LB_FD_D2Q16 = 2,
    LB_FD_D2Q25 = 3,
    LB_FD_D2Q36 = 4
};

/* storage precision (bits 8-9).  The stored quantity is always the shifted
 * g_k = f_k - w_k rho0 (rho0 = mean initial density); arithmetic is FP32 for
 * LB_FP32 and LB_FP16_SHIFTED, FP64 for LB_FP64. */
enum lb_precision {
    LB_FP32 = 0,
    LB_FP16_SHIFTED = 1 << 8,
    LB_FP64 = 2 << 8,
    /* collision-streaming only, periodic: FP16 storage of the departure from a
     * reference equilibrium, 2^12 (g_k - R_k(U(x))) (the factor keeps small
     * departures in the FP16 normal range) with R_k(U) the second-order
     * equilibrium at (rho0, rho0 U) less w_k rho0 (Section 2) and U a
     * per-node reference velocity stored as two FP16 values (4 more bytes
     * per node: 40 bytes per node-step instead of 36).  lb_init takes U from
     * the initial velocity, lb_set_state from the state's.  For a flow near
     * its reference (a decaying wave or vortex) the stored departures are
     * orders of magnitude below g_k, and so is the noise of their
     * stochastic rounding; arithmetic stays FP32. */
    LB_FP16_REF = 3 << 8
};
#define LB_PRECISION_MASK (3 << 8)

/* Time integration of the FD models (bit 10, or-ed into the model like the
 * precision).  Default: the third-order TVD Runge-Kutta scheme with the BGK
 * collision explicit in every stage (Section 2), which needs dt <= tau
 * (Section 4.1, LB_ESTIFF otherwise).  LB_IMEX: an implicit-explicit scheme,
 * which Section 4.1 names for lifting that bound without specifying one; the
 * library takes IMEX-SSP2(2,2,2) (Pareschi & Russo 2005): advection explicit
 * (SSP Heun tableau), relaxation implicit (L-stable tableau, solved in closed
 * form because the collision keeps rho and rho u), second order, any dt/tau;
 * the CFL bound still applies.  Four launches per step (two stencil stages,
 * two pointwise relaxation stages), three state buffers.  The stencil stage
 * re-evaluates the relaxation of the stored first stage explicitly, so its
 * storage rounding is amplified by dt/tau (visible with FP16 storage at large
 * dt/tau).  CS models reject it (LB_EINVAL). */
#define LB_IMEX (1 << 10)

enum lb_status {
    LB_OK = 0,
    LB_EINVAL = -1,  /* bad model, size, order, pointer or argument */
    LB_ECFL = -2,    /* FD: max |v_k,alpha| dt / ds > 1 (Section 4.1 CFL bound) */
    LB_ESTIFF = -3,  /* FD: dt > tau, explicit collision would be stiff (Section 4.1) */
    LB_ENOMEM = -4,  /* device allocation failed */
    LB_EDEVICE = -5, /* HIP runtime error */
    LB_ENAN = -6,    /* non-finite diagnostics */
    LB_EBUSY = -7,   /* server: budget or slots exhausted */
    LB_ESTATE = -8   /* call out of order (e.g. step before init) */
};

typedef struct lb_sim lb_sim;

/* Create a simulation of Nx x Ny nodes (periodic in x and y).
 *   model_flags: lb_model | lb_precision.
 *   tau, dt, ds: relaxation time, time step, grid spacing (see conventions).
 *   N: order of the Hermite expansion of the equilibrium.
 * Validation: Nx, Ny >= 1, Nx * Ny <= 2^30 (periodic directions wrap, so
 * one node per direction is a valid grid); CS needs N == 2 and
 * tau > dt/2 (positive viscosity nu = c_s^2 (tau - dt/2), Section 2); FD
 * needs 1 <= N <= Q-1, the CFL bound, dt <= tau (Section 4.1) and one
 * population plane and one moment plane below 4 GiB: (Nx * Ny + 4352 / s) * c
 * < 2^32, with s the bytes of a stored value and c = 8 for FP64 storage, 4
 * otherwise (the moments are kept in the arithmetic type; each plane is
 * padded by 4352 bytes).  Allocates all device memory (2 state buffers for CS, 3
 * for FD, each FD buffer with three moment planes after its populations) on
 * the current HIP device.  Returns NULL on error (see lb_last_error). */
lb_sim *lb_create(int model_flags, int Nx, int Ny, double tau, double dt, double ds, int N);

/* Release all device memory of the handle.  NULL is ignored. */
void lb_destroy(lb_sim *sim);

/* Code of the last failed call on this thread (LB_OK if none). */
int lb_last_error(void);

/* Static description of a status code. */
const char *lb_strerror(int code);

/* Velocity set of a model: writes K values to vx, vy, w (each may be NULL)
 * and the sound speed to *cs (may be NULL); for CS uses ds and dt, for FD
 * ignores them.  Returns K (> 0) or LB_EINVAL. */
int lb_model_info(int model, double ds, double dt, double *vx, double *vy, double *w, double *cs);

/* Fixed-value ends in x: the nodes beyond x = 0 and x = Nx-1 hold the
 * equilibrium at (rho_left, u = 0) and (rho_right, u = 0); y stays periodic.
 * Must be called before lb_init / lb_set_state.  Densities must be > 0. */
int lb_set_bc_x(lb_sim *sim, double rho_left, double rho_right);

/* FD only: tolerance eps of the WENO-5 nonlinear weights (default 1e-6;
 * the weights of Jiang and Shu, the paper's WENO-5 reference, Section 2).
 * Accepted range: [1e-9, 1e9] with FP32 arithmetic, [1e-75, 1e75] with FP64
 * (the weights are formed from (eps + beta)^4); LB_EINVAL otherwise. */
int lb_set_weno_eps(lb_sim *sim, double eps);

/* f := f_eq(rho, u) at every node (rho > 0).  Sets rho0 to the mean of rho
 * and resets the step counter.  Arrays [Ny][Nx]. */
int lb_init(lb_sim *sim, const double *rho, const double *ux, const double *uy);

/* Advance nsteps >= 0 time steps (CS: one fused pull stream-collide launch
 * per step; FD: three RK stage launches per step).  Asynchronous. */
int lb_step(lb_sim *sim, int nsteps);

/* Density and velocity of the current state, [Ny][Nx] each (any may be NULL). */
int lb_moments(lb_sim *sim, double *rho, double *ux, double *uy);

/* Velocity pattern for the amplitude diagnostic of lb_reduce and of the
 * sampled steps, as products of 1-D factors: phi_x(i, j) = ax[i] ay[j],
 * phi_y(i, j) = bx[i] by[j] (ax, bx: Nx values; ay, by: Ny values).  All NULL
 * clears the pattern.  The decaying modes of Sections 4.2-4.3 (shear wave,
 * Taylor-Green vortex) are of this form, which lets the sampled steps form
 * the projection from 2 (Nx + Ny) values instead of two full fields; an
 * arbitrary pattern goes through lb_reduce_field. */
int lb_set_probe(lb_sim *sim, const double *ax, const double *ay, const double *bx, const double *by);

/* Diagnostics of the current state, accumulated in FP64 on the device in a
 * fixed order (deterministic):
 *   out[0] M  = sum rho          out[1], out[2] P = sum rho u
 *   out[3] E  = sum rho |u|^2/2  out[4] A = sum u.phi / sum phi.phi (0 without a probe)
 * Returns LB_ENAN when a result is not finite. */
int lb_reduce(lb_sim *sim, double out[5]);

/* Diagnostics of the current state with an arbitrary velocity pattern phi
 * (the mode whose amplitude the decay laws of Sections 4.2-4.3 follow):
 * phi_x, phi_y are host arrays [Ny][Nx] (both NULL: A = 0).  Same sums and
 * order of accumulation as lb_reduce, in FP64 on the device:
 *   out[0] M = sum rho, out[1..2] P = sum rho u, out[3] E = sum rho |u|^2/2,
 *   out[4] A = sum u.phi / sum phi.phi (0 when phi.phi sums to 0).
 * Copies the pattern to a temporary device buffer (allocates) and
 * synchronises.  LB_EINVAL if only one of phi_x, phi_y is given or a value is
 * not finite; LB_ENAN when a result is not finite. */
int lb_reduce_field(lb_sim *sim, const double *phi_x, const double *phi_y, double out[5]);

/* lb_reduce_field for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same results, bit for bit, with the pattern and the
 * output in caller-owned DEVICE memory and nothing allocated or
 * synchronised.
 *   d_phi_x, d_phi_y: device arrays [Ny][Nx] of doubles (both NULL: A = 0),
 *     read by kernels on the handle's stream: they must be ready on that
 *     stream and stay valid until the call's work has run.
 *   d_out: device array of 5 doubles, written on the handle's stream
 *     {M, Px, Py, E, A} as lb_reduce_field computes them.
 * Enqueued asynchronously on the handle's stream; no non-finite check (read
 * d_out after a synchronisation).  Per-block partial sums go to one fixed
 * device array per GPU, held until the process ends: (5 + 1) doubles for
 * each of at most 1024 blocks (48 KiB), which every grid lb_create accepts
 * fits (a larger need returns LB_EINVAL).  Every call on a GPU shares that
 * GPU's array and leaves its partials there (each call writes all it reads,
 * so nothing needs clearing): calls that overlap on one GPU, on different
 * streams or from different threads, race and must be serialised by the
 * caller.  Switches to the handle's device for the call if another is
 * current.  LB_EINVAL if only one of the pattern pointers is given or d_out
 * is NULL, LB_ESTATE before lb_init / lb_set_state. */
int lb_reduce_field_noalloc(lb_sim *sim, const double *d_phi_x, const double *d_phi_y, double *d_out);

/* Advance nsteps steps; for every step whose input state has
 * lb_steps_done() % every == 0, the diagnostics of that input state are
 * computed inside the step kernels (no extra pass over the state) and
 * appended to the handle's series.  Asynchronous, like lb_step.  The series
 * holds at most `capacity` samples (lb_series_reserve); further samples
 * return LB_EBUSY before any step is launched. */
int lb_step_sampled(lb_sim *sim, int nsteps, int every);

/* Make room for `capacity` samples in the series (allocates; default 0). */
int lb_series_reserve(lb_sim *sim, int capacity);

/* Copy the pending samples as rows {t, M, Px, Py, E, A} (t = step index of
 * the sampled state) into out[max_rows * 6], oldest first, and clear the
 * series.  Synchronises.  Returns the number of rows copied (>= 0; samples
 * beyond max_rows are dropped) or a negative LB_E* code. */
int lb_series_read(lb_sim *sim, double *out, int max_rows);

/* Run nsteps steps and return the diagnostics every `every` steps (at steps
 * 0, every, 2 every, ... <= nsteps) in series[(nsteps / every + 1) * 5],
 * fused into the step kernels except for a sample at t = nsteps.
 * Synchronises; clears the handle's series. */
int lb_run_sampled(lb_sim *sim, int nsteps, int every, double *series);

/* Canonical (pre-collision) distribution f_k(x, t), [K][Ny][Nx] float64. */
int lb_get_state(lb_sim *sim, double *f);
int lb_set_state(lb_sim *sim, const double *f);

/* Number of steps taken since lb_init / lb_set_state. */
long long lb_steps_done(const lb_sim *sim);

/* Graph replay of plain steps (a performance setting; results are
 * bitwise the same).  Runs of steps without sampling in lb_step and
 * lb_step_sampled replay a HIP graph captured once with `steps` steps
 * (rounded up to even for CS, whose two buffers then return to their start);
 * the remainder of a run is launched step by step.  steps = -1 restores the
 * default (CS 8, FD 4), 0 launches every step separately.  FP16 storage never
 * replays graphs: its stochastic rounding draws new random bits every step.
 * Captured graphs are dropped (and recaptured on demand) by lb_init,
 * lb_set_state, lb_set_weno_eps and this call.  Returns LB_EINVAL for steps
 * outside [-1, 4096]. */
int lb_set_graph_steps(lb_sim *sim, int steps);

/* FP16 storage: the stream of counter-based random bits that the stochastic
 * rounding draws (seed 0 by default).  Different seeds give independent
 * realisations of the rounding; FP32 and FP64 storage ignore it.  The bits
 * are a function of (seed, step, node, population, stage), so a run repeats
 * exactly for a given seed. */
int lb_set_rounding_seed(lb_sim *sim, unsigned seed);

/* Autotuning of the launch shapes of plain steps (steps without sampling;
 * results are bitwise the same for every shape).  Times the candidates on
 * the handle's own buffers, leaving the state unchanged, and keeps the
 * fastest: CS (vector row form only) workgroup sizes of 256, 512 and 1024
 * threads against one chunk per thread, then at that size plain against
 * non-temporal stores (lb_set_cs_nontemporal), `reps` launches per timing;
 * FD the four pairs of tile heights (64 x 32 or 64 x 16 nodes for the first
 * Runge-Kutta stage and for the later ones, which also read the step's base
 * state) as blocks of max(reps, 10) whole plain steps of a temporary copy of
 * the state (one more state buffer while tuning; without it, steps that
 * leave the state in place), then, where lb_set_fd_fused applies, the
 * three stage launches against the fused step with 32-, 64- and 128-row
 * segments, per step.  The candidates of a choice take turns in rotated
 * order, so that a drift of the device clock during the tuning falls on
 * each alike.  Synchronises the stream.  LB_ESTATE before lb_init,
 * LB_EDEVICE if the state copy fails, LB_EINVAL for reps outside
 * [1, 1000].  The choice is kept in a
 * process-wide cache keyed by device, model, storage, boundaries, grid and
 * Hermite order; a later call for a handle of the same key (any handle, any
 * thread) takes the cached shapes without timing. */
int lb_autotune(lb_sim *sim, int reps);

/* Empty the autotuning cache, so that the next lb_autotune of each key times
 * its candidates again.  Returns LB_OK. */
int lb_tuning_cache_clear(void);

/* Number of keys in the autotuning cache. */
int lb_tuning_cache_size(void);

/* Set the plain-step launch shapes directly: cs_threads 0 (one chunk per
 * thread) or a multiple of 64 up to 1024; fd_rows (first FD stage) and
 * fd_rows_rest (later FD stages, the last IMEX stage included) 8 (64 x 32
 * tiles) or 4 (64 x 16).  LB_EINVAL otherwise.  Defaults of a new handle:
 * 0, 8, 8. */
int lb_set_tuning(lb_sim *sim, int cs_threads, int fd_rows, int fd_rows_rest);

/* FD plain steps by the temporally blocked kernel: the three Runge-Kutta
 * stages of a step in one launch (Section 2), each workgroup marching up a
 * y-segment of rows_per_segment rows of an x-strip of 110 columns with the
 * stage values kept on chip; the new state is bit for bit that of the three
 * stage launches, with the state read once (plus halos) and written once per
 * step instead of eight state transfers.  0 (the default of a new handle)
 * restores the stage launches; lb_autotune chooses between them.  FP32
 * storage, periodic, Q = 3 or 4 (D2Q9, D2Q16), explicit Runge-Kutta only:
 * LB_EINVAL otherwise, and for values outside [0, 4096].  Sampled steps keep
 * the stage launches (their first stage sums the diagnostics). */
int lb_set_fd_fused(lb_sim *sim, int rows_per_segment);

/* Segment rows of the fused FD step, 0 for the stage launches (LB_EINVAL for
 * a NULL handle). */
int lb_get_fd_fused(const lb_sim *sim);

/* The current plain-step launch shapes (host ints). */
int lb_get_tuning(const lb_sim *sim, int *cs_threads, int *fd_rows, int *fd_rows_rest);

/* Store policy of CS plain steps: 1 stores the vector row form's outputs
 * non-temporally (the written lines are not kept in the caches; faster only
 * for states well beyond the 256 MB last-level cache), 0 (the default of a
 * new handle) plainly.  Results are bitwise the same; sampled steps and the
 * scalar row form store plainly.  LB_EINVAL for an FD handle or a value
 * other than 0 and 1. */
int lb_set_cs_nontemporal(lb_sim *sim, int on);

/* The CS store policy of plain steps: 1 non-temporal, 0 plain (LB_EINVAL
 * for a NULL handle). */
int lb_get_cs_nontemporal(const lb_sim *sim);

/* Launch on a caller-owned HIP stream (hipStream_t passed as void*; NULL
 * means the library's own stream).  The caller keeps the stream alive. */
int lb_set_stream(lb_sim *sim, void *hip_stream);

/* Block until the handle's stream is idle. */
int lb_synchronize(lb_sim *sim);

/* Device bytes held by the handle. */
size_t lb_device_bytes(const lb_sim *sim);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of many independent simulations.
 *
 * A server owns a compute stream, an admission stream (same priority) and a
 * worker thread (started by the first lb_server_submit).  Submitted requests
 * wait in a queue; the worker admits them while the device-memory budget and
 * the slot count allow (footprint = state buffers + diagnostics of the
 * simulation), creating and initialising them on the admission stream while
 * the batched steps of the running simulations proceed on the compute
 * stream.  Every admitted simulation advances by one step per batched step:
 * one launch for all collision-streaming simulations, three Runge-Kutta stage
 * launches per equilibrium order for the finite-difference ones, one launch
 * for the sampled diagnostics; a batched step of a given running set is
 * captured once as a HIP graph and replayed (the kernels read the step index
 * from device memory).  Runs of batched steps ("chunks") end at the first
 * completion or after chunk_steps steps; between chunks the finished
 * simulations are drained (final diagnostics, apparent viscosity), their
 * memory is released and the newly admitted ones join.  The later-stage FD
 * tile height (64 x 16 or 64 x 32) is chosen per equilibrium order by timing
 * both on the first running set that has the order.  Each simulation
 * computes the same values as a single lb_sim run of the same request (same
 * per-row / per-tile device code), whatever else shares the batch.
 * Supported requests: periodic, FP32 storage, any model.
 * ------------------------------------------------------------------------ */
typedef struct lb_server lb_server;

typedef struct lb_request {
    int model;                /* lb_model (FP32 storage) */
    int Nx, Ny;
    double tau, dt, ds;       /* as for lb_create */
    int N;                    /* equilibrium order */
    const double *rho, *ux, *uy;         /* initial fields [Ny][Nx]; read at admission, so they
                                            must stay valid until the request's result is polled */
    const double *ax, *ay, *bx, *by;     /* separable probe (as lb_set_probe), all NULL for none */
    int nsteps;               /* steps to run, >= 1 */
    int sample_every;         /* diagnostics every this many steps, >= 1 */
    uint64_t tag;             /* returned in the result */
    double decay_k2;          /* > 0 (needs a probe): fit the amplitude series A(t), t = step dt, and
                                 return nu_app = decay rate / decay_k2 (shear wave of wavenumber k:
                                 k^2, Section 4.2; Taylor-Green vortex: 2 k^2, Section 4.3); 0: no fit */
    double decay_omega;       /* >= 0: angular frequency (per unit of t) of a modulation fitted along
                                 (lb_fit_decay), 0 for none */
} lb_request;

typedef struct lb_result {
    uint64_t id, tag;
    int status;               /* LB_OK or the error that ended the request */
    int nsamples;
    double *samples;          /* nsamples rows {t, M, Px, Py, E, A}: the states at
                                 t = 0, every, 2 every, ... < nsteps and the final state
                                 t = nsteps; owned by the server until lb_server_release */
    double t_submit, t_admit, t_finish;  /* seconds on the server clock */
    double nu_app;            /* apparent viscosity of the request's fit (NaN without one, or when the
                                 fit fails) */
} lb_result;

/* hbm_budget_bytes: device memory the admitted simulations may hold;
 * max_slots: simulations admitted at once (1..4096); chunk_steps: batched
 * steps between admission / drain points (>= 1).  NULL on error. */
lb_server *lb_server_create(size_t hbm_budget_bytes, int max_slots, int chunk_steps);

/* Launch options, before the first lb_server_submit (LB_ESTATE after it):
 * use_graphs 1 (default) replays each batched step as a captured HIP graph,
 * 0 launches its kernels one by one (the same kernels in the same order:
 * the results are bitwise the same); tune_tiles 1 (default) times the FD
 * later-stage tile heights per order, 0 keeps 64 x 16.  LB_EINVAL for values
 * other than 0 and 1. */
int lb_server_configure(lb_server *srv, int use_graphs, int tune_tiles);

/* Admission by nodes in flight, before the first lb_server_submit (LB_ESTATE
 * after it): queued requests are admitted (in arrival order, within the
 * budget and slots) only while the grid nodes of the admitted simulations
 * stay at or below max_nodes; a request larger than the limit is admitted
 * alone.  0 (the default) sets no limit, so every request that fits the
 * budget runs at once and all share the device.  A limit that still fills
 * the device keeps the throughput and lets the earlier requests finish
 * sooner (lower time-to-result).  LB_EINVAL for a NULL server. */
int lb_server_set_node_limit(lb_server *srv, size_t max_nodes);

/* Admission order of queued requests, before the first lb_server_submit
 * (LB_ESTATE after it): LB_ADMIT_ARRIVAL (the default) admits in arrival
 * order; LB_ADMIT_SHORTEST admits the request of smallest estimated device
 * work first (grid nodes x steps x the model's cost per node-step: 1 for CS
 * D2Q9, 0.75 K for an FD model of K populations), equal work in arrival
 * order.  Shortest-first lowers the median time-to-result when many
 * requests wait; a long request waits while shorter ones keep arriving.
 * Results do not depend on the order.  LB_EINVAL for another value. */
enum lb_admit_policy { LB_ADMIT_ARRIVAL = 0, LB_ADMIT_SHORTEST = 1 };
int lb_server_set_policy(lb_server *srv, int policy);

/* Queue a request (non-blocking).  LB_EINVAL for a request that lb_create
 * would reject or that is not supported in a batch; LB_EBUSY when the
 * request alone exceeds the budget.  *id receives the request id. */
int lb_server_submit(lb_server *srv, const lb_request *req, uint64_t *id);

/* Move up to max finished results into out, waiting up to timeout_us for
 * the first one.  Returns the number of results (>= 0). */
int lb_server_poll(lb_server *srv, lb_result *out, int max, int timeout_us);

/* Free the samples of a polled result. */
void lb_server_release(lb_server *srv, lb_result *res);

/* Seconds since the server was created (the clock of the time stamps). */
double lb_server_clock(const lb_server *srv);

/* Counters: out[0] submitted, out[1] completed, out[2] queued, out[3]
 * running, out[4] device bytes held, out[5] batched steps launched,
 * out[6] seconds the worker spent with simulations on the device. */
int lb_server_stats(const lb_server *srv, double out[7]);

/* Stop the worker (running and queued requests are abandoned) and release
 * every resource.  NULL is ignored. */
void lb_server_destroy(lb_server *srv);

/* Decay rate of an amplitude series, the FP64 viscosity fit of Sections
 * 4.2-4.3 (a shear wave decays as exp(-nu k^2 t), a Taylor-Green vortex as
 * exp(-2 nu k^2 t); the paper does not state its fit): least squares of
 * ln|amp[i]| on {1, -t[i]}, or with omega > 0 on {1, -t[i], cos(omega t[i]),
 * sin(omega t[i])} (a modulation at a known frequency fitted along, e.g. the
 * standing sound wave of a vortex started from the incompressible pressure).
 * t, amp: n host values; *rate receives the coefficient of -t.  LB_EINVAL for
 * n below 3 (5 with omega), a zero or non-finite value, or a degenerate
 * design; LB_ENAN for a non-finite result. */
int lb_fit_decay(const double *t, const double *amp, int n, double omega, double *rate);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */

/*
 * lb_oracle.c -- plain FP64 CPU oracle for the isothermal lattice Boltzmann
 * time step of Negro, Busuioc, Ambrus, Gonnella, Lamura, Sofonea,
 * "Comparison between isothermal collision-streaming and finite-difference
 * lattice Boltzmann models" (arXiv:1904.02471).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; it computes every table
 * (Gauss-Hermite roots and weights, Hermite polynomials) itself.
 *
 * Everything is written for clarity, not speed: one node, one population at a
 * time, in double precision, in the order the paper states the steps.  By
 * default it runs on one thread (the plain definition); orc_set_threads lets
 * the loops over rows and nodes run on several host threads (OpenMP), which
 * changes no arithmetic: every node's values are computed by the same
 * operations whichever thread takes it, so the results are bitwise those of
 * the single-threaded run.  Sums over the whole lattice (orc_reduce) stay on
 * one thread, in node order.  Readings taken where the paper is silent are
 * marked READING.
 *
 * Distribution layout: f[k][y][x], x fastest, k the population index.
 *   CS D2Q9 population order: 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
 *   FD models: tensor order k = j*Q + i, v_k = (xi_i, xi_j), xi ascending.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXQ 8
#define ORC_MAXK (ORC_MAXQ * ORC_MAXQ)

enum { ORC_CS_D2Q9 = 0, ORC_FD_D2Q9 = 1, ORC_FD_D2Q16 = 2, ORC_FD_D2Q25 = 3, ORC_FD_D2Q36 = 4 };

typedef struct orc_sim {
    int model, Q, K, N, Nx, Ny;
    double tau, dt, ds, cs;
    double vx[ORC_MAXK], vy[ORC_MAXK], w[ORC_MAXK];
    int ex[ORC_MAXK], ey[ORC_MAXK]; /* CS only: link in node units */
    double *f;                      /* canonical (pre-collision) state */
    double *work[4];
    int bc_x_fixed;
    double rho_left, rho_right;
    double weno_eps;
    int time_scheme; /* FD: 0 third-order TVD Runge-Kutta, 1 IMEX-SSP2(2,2,2) */
    int threads;     /* host threads of the row / node loops (1: plain serial run) */
} orc_sim;

/* Row / node loops of a function whose simulation is `s`: parallel over
 * s->threads host threads when above one. */
#define ORC_PARALLEL_FOR _Pragma("omp parallel for num_threads(s->threads) if(s->threads > 1) schedule(static)")

/* ------------------------------------------------------------------------ */
/* Gauss-Hermite quadrature (Section 1: the velocity set is given by the     */
/* roots of the Hermite polynomial of order Q, weights from the quadrature). */
/* Probabilists' Hermite polynomials He_n, weight exp(-x^2/2)/sqrt(2 pi).     */
/* ------------------------------------------------------------------------ */

/* He_0..He_n at x by the three-term recursion He_{n+1} = x He_n - n He_{n-1}. */
static void hermite_values(double x, int n, double *h)
{
    h[0] = 1.0;
    if (n >= 1) h[1] = x;
    for (int m = 1; m < n; ++m) h[m + 1] = x * h[m] - m * h[m - 1];
}

static double hermite_at(double x, int n)
{
    double h[ORC_MAXQ + 2];
    hermite_values(x, n, h);
    return h[n];
}

/* Roots of He_Q in ascending order and their normalised quadrature weights
 * w_i = Q! / (Q He_{Q-1}(x_i))^2 (so that sum w_i = 1).  Roots are bracketed
 * by a sign scan over [-2 sqrt(Q) - 1, 2 sqrt(Q) + 1] and refined by
 * bisection to the last representable bit.  Returns 0 on success. */
int orc_gauss_hermite(int Q, double *x, double *w)
{
    if (Q < 1 || Q > ORC_MAXQ) return -1;
    double lim = 2.0 * sqrt((double)Q) + 1.0;
    int nscan = 20000, found = 0;
    double a = -lim, fa = hermite_at(a, Q);
    for (int s = 1; s <= nscan && found < Q; ++s) {
        double b = -lim + 2.0 * lim * s / nscan;
        double fb = hermite_at(b, Q);
        if (fb == 0.0) {
            x[found++] = b;
        } else if (fa != 0.0 && (fa < 0.0) != (fb < 0.0)) {
            double lo = a, hi = b, flo = fa;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid == lo || mid == hi) break;
                double fm = hermite_at(mid, Q);
                if (fm == 0.0) { lo = hi = mid; break; }
                if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
            }
            x[found++] = 0.5 * (lo + hi);
        }
        a = b;
        fa = fb;
    }
    if (found != Q) return -2;
    double qfact = 1.0;
    for (int i = 2; i <= Q; ++i) qfact *= i;
    for (int i = 0; i < Q; ++i) {
        double h = hermite_at(x[i], Q - 1);
        w[i] = qfact / ((Q * h) * (Q * h));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Model set-up                                                              */
/* ------------------------------------------------------------------------ */

/* Velocity set of a model.  CS D2Q9 (Section 2, after the collision-streaming
 * evolution equation): links to the 8 neighbours with |v_k,alpha| = c_l =
 * ds/dt, weights from the Q=3 Gauss-Hermite rule, sound speed
 * c_s = c_l / sqrt(3).  FD models: v_k = (xi_i, xi_j), the roots of He_Q, in
 * units where c_s = 1 (T = m = 1, Section 4.1). */
int orc_velocity_set(int model, double ds, double dt, double *vx, double *vy, double *w,
                     double *cs, int *ex, int *ey)
{
    static const int cex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int cey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    double x[ORC_MAXQ], wq[ORC_MAXQ];
    if (model == ORC_CS_D2Q9) {
        if (orc_gauss_hermite(3, x, wq)) return -1;
        /* x = {-sqrt3, 0, +sqrt3}; weight by |e| component */
        double cl = ds / dt;
        for (int k = 0; k < 9; ++k) {
            double wx = cex[k] == 0 ? wq[1] : wq[0];
            double wy = cey[k] == 0 ? wq[1] : wq[0];
            vx[k] = cex[k] * cl;
            vy[k] = cey[k] * cl;
            w[k] = wx * wy;
            if (ex) ex[k] = cex[k];
            if (ey) ey[k] = cey[k];
        }
        *cs = cl / sqrt(3.0);
        return 9;
    }
    if (model < ORC_FD_D2Q9 || model > ORC_FD_D2Q36) return -1;
    int Q = model + 2;
    if (orc_gauss_hermite(Q, x, wq)) return -1;
    for (int j = 0; j < Q; ++j)
        for (int i = 0; i < Q; ++i) {
            int k = j * Q + i;
            vx[k] = x[i];
            vy[k] = x[j];
            w[k] = wq[i] * wq[j];
            if (ex) ex[k] = 0;
            if (ey) ey[k] = 0;
        }
    *cs = 1.0;
    return Q * Q;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium: Hermite expansion of the Maxwellian truncated at total       */
/* order N (Section 1; for N = 2 this is the printed second-order form).      */
/* f_eq_k = w_k rho sum_{n+m<=N} He_n(cx) He_m(cy) ax^n ay^m / (n! m!),       */
/* cx = v_kx / c_s, ax = u_x / c_s.                                           */
/* ------------------------------------------------------------------------ */

static double factorial(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

static double feq_one(const orc_sim *s, int k, double rho, double ux, double uy)
{
    double hx[ORC_MAXQ + 2], hy[ORC_MAXQ + 2];
    double cx = s->vx[k] / s->cs, cy = s->vy[k] / s->cs;
    double ax = ux / s->cs, ay = uy / s->cs;
    hermite_values(cx, s->N, hx);
    hermite_values(cy, s->N, hy);
    double sum = 0.0;
    for (int n = 0; n <= s->N; ++n)
        for (int m = 0; n + m <= s->N; ++m)
            sum += hx[n] * hy[m] * pow(ax, n) * pow(ay, m) / (factorial(n) * factorial(m));
    return s->w[k] * rho * sum;
}

/* Moments (Section 2): rho = sum_k f_k, rho u = sum_k f_k v_k. */
static void moments_node(const orc_sim *s, const double *f, long node, long plane, double *rho,
                         double *ux, double *uy)
{
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int k = 0; k < s->K; ++k) {
        double fk = f[k * plane + node];
        r += fk;
        jx += fk * s->vx[k];
        jy += fk * s->vy[k];
    }
    *rho = r;
    *ux = jx / r;
    *uy = jy / r;
}

/* ------------------------------------------------------------------------ */
/* Public API                                                                */
/* ------------------------------------------------------------------------ */

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->f);
    for (int i = 0; i < 4; ++i) free(s->work[i]);
    free(s);
}

orc_sim *orc_create(int model, int Nx, int Ny, double tau, double dt, double ds, int N)
{
    if (Nx < 1 || Ny < 1 || tau <= 0.0 || dt <= 0.0 || ds <= 0.0) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->model = model;
    s->Nx = Nx;
    s->Ny = Ny;
    s->tau = tau;
    s->dt = dt;
    s->ds = ds;
    s->N = N;
    s->weno_eps = 1e-6;
    s->threads = 1;
    int K = orc_velocity_set(model, ds, dt, s->vx, s->vy, s->w, &s->cs, s->ex, s->ey);
    if (K < 0) { free(s); return NULL; }
    s->K = K;
    s->Q = (model == ORC_CS_D2Q9) ? 3 : model + 2;
    if (N < 0 || N > s->Q - 1 || (model == ORC_CS_D2Q9 && N != 2)) { free(s); return NULL; }
    size_t n = (size_t)K * Nx * Ny;
    s->f = (double *)calloc(n, sizeof(double));
    for (int i = 0; i < 4; ++i) s->work[i] = (double *)calloc(n, sizeof(double));
    if (!s->f || !s->work[0] || !s->work[1] || !s->work[2] || !s->work[3]) { orc_destroy(s); return NULL; }
    return s;
}

int orc_num_populations(const orc_sim *s) { return s->K; }
double orc_sound_speed(const orc_sim *s) { return s->cs; }

void orc_velocities(const orc_sim *s, double *vx, double *vy, double *w)
{
    for (int k = 0; k < s->K; ++k) {
        vx[k] = s->vx[k];
        vy[k] = s->vy[k];
        w[k] = s->w[k];
    }
}

void orc_set_weno_eps(orc_sim *s, double eps) { s->weno_eps = eps; }

/* Host threads of the row and node loops (>= 1; 1 is the plain serial run).
 * Results do not depend on it. */
void orc_set_threads(orc_sim *s, int threads) { s->threads = threads < 1 ? 1 : threads; }

/* Fixed-value x ends: the nodes beyond x = 0 and x = Nx-1 hold the
 * equilibrium at (rho_left, 0) and (rho_right, 0).  READING: the paper runs
 * every case periodic; this equilibrium (Dirichlet) end is the reading used
 * for the fixed-end shock tube. */
void orc_set_bc_x(orc_sim *s, double rho_left, double rho_right)
{
    s->bc_x_fixed = 1;
    s->rho_left = rho_left;
    s->rho_right = rho_right;
}

void orc_equilibrium(const orc_sim *s, double rho, double ux, double uy, double *feq)
{
    for (int k = 0; k < s->K; ++k) feq[k] = feq_one(s, k, rho, ux, uy);
}

/* f := f_eq(rho, u) at every node. Fields are [Ny][Nx]. */
void orc_init(orc_sim *s, const double *rho, const double *ux, const double *uy)
{
    long plane = (long)s->Nx * s->Ny;
    ORC_PARALLEL_FOR
    for (long node = 0; node < plane; ++node)
        for (int k = 0; k < s->K; ++k) s->f[k * plane + node] = feq_one(s, k, rho[node], ux[node], uy[node]);
}

void orc_get_state(const orc_sim *s, double *f)
{
    memcpy(f, s->f, sizeof(double) * (size_t)s->K * s->Nx * s->Ny);
}

void orc_set_state(orc_sim *s, const double *f)
{
    memcpy(s->f, f, sizeof(double) * (size_t)s->K * s->Nx * s->Ny);
}

void orc_moments(const orc_sim *s, double *rho, double *ux, double *uy)
{
    long plane = (long)s->Nx * s->Ny;
    ORC_PARALLEL_FOR
    for (long node = 0; node < plane; ++node) moments_node(s, s->f, node, plane, &rho[node], &ux[node], &uy[node]);
}

/* ------------------------------------------------------------------------ */
/* Collision-streaming step (Section 2, collision-streaming evolution        */
/* equation): f_k(x + v_k dt, t + dt) = f_k - (dt/tau)(f_k - f_eq_k).         */
/* Collide at every node, then move each post-collision value one link.       */
/* ------------------------------------------------------------------------ */

static void cs_step_once(orc_sim *s)
{
    int Nx = s->Nx, Ny = s->Ny, K = s->K;
    long plane = (long)Nx * Ny;
    double *fstar = s->work[0];
    double omega = s->dt / s->tau;
    ORC_PARALLEL_FOR
    for (long node = 0; node < plane; ++node) {
        double rho, ux, uy;
        moments_node(s, s->f, node, plane, &rho, &ux, &uy);
        for (int k = 0; k < K; ++k) {
            double fk = s->f[k * plane + node];
            fstar[k * plane + node] = fk - omega * (fk - feq_one(s, k, rho, ux, uy));
        }
    }
    for (int k = 0; k < K; ++k) {
        ORC_PARALLEL_FOR
        for (int y = 0; y < Ny; ++y)
            for (int x = 0; x < Nx; ++x) {
                int xs = x - s->ex[k], ys = y - s->ey[k];
                ys = (ys % Ny + Ny) % Ny;
                double val;
                if (s->bc_x_fixed && (xs < 0 || xs >= Nx)) {
                    val = feq_one(s, k, xs < 0 ? s->rho_left : s->rho_right, 0.0, 0.0);
                } else {
                    xs = (xs % Nx + Nx) % Nx;
                    val = fstar[k * plane + (long)ys * Nx + xs];
                }
                s->f[k * plane + (long)y * Nx + x] = val;
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Finite-difference step (Section 2): the BGK equation                     */
/*   d_t f_k + v_k . grad f_k = -(f_k - f_eq_k) / tau                        */
/* with WENO-5 upwind reconstruction for the advection term and the          */
/* third-order TVD Runge-Kutta scheme in time.                               */
/* ------------------------------------------------------------------------ */

/* WENO-5 (Jiang & Shu) reconstruction at the interface downstream of cell c,
 * from the five values a,b,c,d,e ordered along the upwind direction
 * (a = two cells upstream of c, e = two cells downstream).  READING: the
 * paper names WENO-5 but gives no details; this is the classic form with
 * linear weights (0.1, 0.6, 0.3), power 2 and tolerance eps. */
double orc_weno5(double a, double b, double c, double d, double e, double eps)
{
    double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
    double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
    double b0 = 13.0 / 12.0 * (a - 2.0 * b + c) * (a - 2.0 * b + c) + 0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
    double b1 = 13.0 / 12.0 * (b - 2.0 * c + d) * (b - 2.0 * c + d) + 0.25 * (b - d) * (b - d);
    double b2 = 13.0 / 12.0 * (c - 2.0 * d + e) * (c - 2.0 * d + e) + 0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);
    double a0 = 0.1 / ((eps + b0) * (eps + b0));
    double a1 = 0.6 / ((eps + b1) * (eps + b1));
    double a2 = 0.3 / ((eps + b2) * (eps + b2));
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* Value of population k at node (x, y), x possibly outside [0, Nx) (ghost
 * nodes of the fixed-value ends) and y taken periodically. */
static double fd_value(const orc_sim *s, const double *f, int k, int x, int y)
{
    int Nx = s->Nx, Ny = s->Ny;
    y = (y % Ny + Ny) % Ny;
    if (x < 0 || x >= Nx) {
        if (s->bc_x_fixed) return feq_one(s, k, x < 0 ? s->rho_left : s->rho_right, 0.0, 0.0);
        x = (x % Nx + Nx) % Nx;
    }
    return f[(long)k * Nx * Ny + (long)y * Nx + x];
}

/* Interface value of population k between node i and node i+1 along axis
 * (dx, dy) = (1,0) or (0,1), starting from node (x, y) = node i. Upwind side
 * chosen by the sign of the velocity component v. */
static double fd_interface(const orc_sim *s, const double *f, int k, int x, int y, int dx, int dy, double v)
{
    double p[6];
    for (int m = -2; m <= 3; ++m) p[m + 2] = fd_value(s, f, k, x + m * dx, y + m * dy);
    /* p[0..5] = f_{i-2}, f_{i-1}, f_i, f_{i+1}, f_{i+2}, f_{i+3} */
    if (v > 0.0) return orc_weno5(p[0], p[1], p[2], p[3], p[4], s->weno_eps);
    return orc_weno5(p[5], p[4], p[3], p[2], p[1], s->weno_eps);
}

/* L(f) = -v_x (F_{i+1/2} - F_{i-1/2}) / ds - v_y (G_{j+1/2} - G_{j-1/2}) / ds
 *        - (f - f_eq(f)) / tau */
static void fd_rhs(const orc_sim *s, const double *f, double *out)
{
    int Nx = s->Nx, Ny = s->Ny, K = s->K;
    long plane = (long)Nx * Ny;
    ORC_PARALLEL_FOR
    for (int y = 0; y < Ny; ++y)
        for (int x = 0; x < Nx; ++x) {
            long node = (long)y * Nx + x;
            double rho, ux, uy;
            moments_node(s, f, node, plane, &rho, &ux, &uy);
            for (int k = 0; k < K; ++k) {
                double adv = 0.0;
                if (s->vx[k] != 0.0) {
                    double fr = fd_interface(s, f, k, x, y, 1, 0, s->vx[k]);
                    double fl = fd_interface(s, f, k, x - 1, y, 1, 0, s->vx[k]);
                    adv += s->vx[k] * (fr - fl) / s->ds;
                }
                if (s->vy[k] != 0.0) {
                    double gr = fd_interface(s, f, k, x, y, 0, 1, s->vy[k]);
                    double gl = fd_interface(s, f, k, x, y - 1, 0, 1, s->vy[k]);
                    adv += s->vy[k] * (gr - gl) / s->ds;
                }
                double fk = f[k * plane + node];
                out[k * plane + node] = -adv - (fk - feq_one(s, k, rho, ux, uy)) / s->tau;
            }
        }
}

/* Third-order TVD Runge-Kutta (Shu-Osher form):
 *   f1 = f + dt L(f)
 *   f2 = 3/4 f + 1/4 (f1 + dt L(f1))
 *   f' = 1/3 f + 2/3 (f2 + dt L(f2)) */
static void fd_step_once(orc_sim *s)
{
    long n = (long)s->K * s->Nx * s->Ny;
    double *L = s->work[0], *f1 = s->work[1], *f2 = s->work[2];
    double dt = s->dt;
    fd_rhs(s, s->f, L);
    ORC_PARALLEL_FOR
    for (long i = 0; i < n; ++i) f1[i] = s->f[i] + dt * L[i];
    fd_rhs(s, f1, L);
    ORC_PARALLEL_FOR
    for (long i = 0; i < n; ++i) f2[i] = 0.75 * s->f[i] + 0.25 * (f1[i] + dt * L[i]);
    fd_rhs(s, f2, L);
    ORC_PARALLEL_FOR
    for (long i = 0; i < n; ++i) s->f[i] = s->f[i] / 3.0 + 2.0 / 3.0 * (f2[i] + dt * L[i]);
}

/* Implicit-explicit time stepping.
 * READING: Section 4.1 names implicit-explicit (IMEX) schemes as the way to
 * lift the restriction dt < tau_FD, without giving one.  We take the
 * second-order IMEX-SSP2(2,2,2) Runge-Kutta scheme of Pareschi & Russo
 * (J. Sci. Comput. 25, 2005): the advection A(f) explicit with the SSP
 * (Heun) tableau, the BGK relaxation R(f) = -(f - f_eq(f)) / tau implicit
 * with the L-stable tableau [[g, 0], [1 - 2g, g]], g = 1 - 1/sqrt(2), both
 * with weights (1/2, 1/2):
 *   f1 = f + g dt R(f1)
 *   f2 = f + dt A(f1) + (1 - 2g) dt R(f1) + g dt R(f2)
 *   f' = f + dt/2 [A(f1) + A(f2)] + dt/2 [R(f1) + R(f2)]
 * R leaves rho and rho u unchanged, so f_eq(f_i) is the equilibrium of the
 * explicit part h of its stage, and each implicit stage has the closed form
 *   f_i = (h + (g dt / tau) f_eq(h)) / (1 + g dt / tau). */

/* out = advection term -v . grad f (WENO-5 faces, as in fd_rhs). */
static void fd_advection(const orc_sim *s, const double *f, double *out)
{
    int Nx = s->Nx, Ny = s->Ny, K = s->K;
    long plane = (long)Nx * Ny;
    ORC_PARALLEL_FOR
    for (int y = 0; y < Ny; ++y)
        for (int x = 0; x < Nx; ++x) {
            long node = (long)y * Nx + x;
            for (int k = 0; k < K; ++k) {
                double adv = 0.0;
                if (s->vx[k] != 0.0) {
                    double fr = fd_interface(s, f, k, x, y, 1, 0, s->vx[k]);
                    double fl = fd_interface(s, f, k, x - 1, y, 1, 0, s->vx[k]);
                    adv += s->vx[k] * (fr - fl) / s->ds;
                }
                if (s->vy[k] != 0.0) {
                    double gr = fd_interface(s, f, k, x, y, 0, 1, s->vy[k]);
                    double gl = fd_interface(s, f, k, x, y - 1, 0, 1, s->vy[k]);
                    adv += s->vy[k] * (gr - gl) / s->ds;
                }
                out[k * plane + node] = -adv;
            }
        }
}

/* out = relaxation term -(f - f_eq(f)) / tau. */
static void fd_relaxation(const orc_sim *s, const double *f, double *out)
{
    long plane = (long)s->Nx * s->Ny;
    ORC_PARALLEL_FOR
    for (long node = 0; node < plane; ++node) {
        double rho, ux, uy;
        moments_node(s, f, node, plane, &rho, &ux, &uy);
        for (int k = 0; k < s->K; ++k)
            out[k * plane + node] = -(f[k * plane + node] - feq_one(s, k, rho, ux, uy)) / s->tau;
    }
}

/* out = the solution f_i of f_i = h + a tau R(f_i), a = g dt / tau. */
static void fd_implicit_relax(const orc_sim *s, const double *h, double a, double *out)
{
    long plane = (long)s->Nx * s->Ny;
    ORC_PARALLEL_FOR
    for (long node = 0; node < plane; ++node) {
        double rho, ux, uy;
        moments_node(s, h, node, plane, &rho, &ux, &uy);
        for (int k = 0; k < s->K; ++k)
            out[k * plane + node] = (h[k * plane + node] + a * feq_one(s, k, rho, ux, uy)) / (1.0 + a);
    }
}

static void fd_imex_step_once(orc_sim *s)
{
    long n = (long)s->K * s->Nx * s->Ny;
    double *f1 = s->work[0], *f2 = s->work[1], *A1 = s->work[2], *R1 = s->work[3];
    double dt = s->dt, g = 1.0 - 1.0 / sqrt(2.0), a = g * dt / s->tau;
    fd_implicit_relax(s, s->f, a, f1);
    fd_advection(s, f1, A1);
    fd_relaxation(s, f1, R1);
    double *h = (double *)malloc(sizeof(double) * n);
    for (long i = 0; i < n; ++i) h[i] = s->f[i] + dt * A1[i] + (1.0 - 2.0 * g) * dt * R1[i];
    fd_implicit_relax(s, h, a, f2);
    /* reuse h for A(f2) and then R(f2) terms */
    fd_advection(s, f2, h);
    for (long i = 0; i < n; ++i) s->f[i] += 0.5 * dt * (A1[i] + h[i]) + 0.5 * dt * R1[i];
    fd_relaxation(s, f2, h);
    for (long i = 0; i < n; ++i) s->f[i] += 0.5 * dt * h[i];
    free(h);
}

void orc_set_time_scheme(orc_sim *s, int scheme) { s->time_scheme = scheme; }

void orc_step(orc_sim *s, int nsteps)
{
    for (int i = 0; i < nsteps; ++i) {
        if (s->model == ORC_CS_D2Q9)
            cs_step_once(s);
        else if (s->time_scheme == 1)
            fd_imex_step_once(s);
        else
            fd_step_once(s);
    }
}

/* Diagnostics of the current state: out = {M, Px, Py, E, A} with
 * M = sum rho, P = sum rho u, E = sum rho |u|^2 / 2 and
 * A = sum (u . phi) / sum (phi . phi), the projection of the velocity field on
 * the pattern phi ([Ny][Nx] each; A = 0 when phi is NULL). */
void orc_reduce(const orc_sim *s, const double *phi_x, const double *phi_y, double *out)
{
    long plane = (long)s->Nx * s->Ny;
    double M = 0, Px = 0, Py = 0, E = 0, num = 0, den = 0;
    for (long node = 0; node < plane; ++node) {
        double rho, ux, uy;
        moments_node(s, s->f, node, plane, &rho, &ux, &uy);
        M += rho;
        Px += rho * ux;
        Py += rho * uy;
        E += 0.5 * rho * (ux * ux + uy * uy);
        if (phi_x && phi_y) {
            num += ux * phi_x[node] + uy * phi_y[node];
            den += phi_x[node] * phi_x[node] + phi_y[node] * phi_y[node];
        }
    }
    out[0] = M;
    out[1] = Px;
    out[2] = Py;
    out[3] = E;
    out[4] = den > 0 ? num / den : 0.0;
}

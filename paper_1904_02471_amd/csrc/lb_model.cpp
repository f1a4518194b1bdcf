// lb_model.cpp -- velocity sets and equilibrium tables of the library
// (host, FP64).
//
// Velocity space (Section 1): the discrete velocities are the roots of the
// Hermite polynomial He_Q (probabilists' convention, weight
// exp(-x^2/2)/sqrt(2 pi)), one set per axis, and the 2-D set is their tensor
// product with weights w_i w_j.  The roots and weights come from the
// Golub-Welsch construction: they are the eigenvalues of the symmetric
// tridiagonal Jacobi matrix of the Hermite recurrence (off-diagonal sqrt(n))
// and the squared first components of its normalised eigenvectors.  The
// eigen-decomposition is done with cyclic Jacobi rotations.
#include "lb_model.h"

#include <algorithm>
#include <cmath>

namespace lbm {

namespace {

void jacobi_eigen(int n, double a[kTabQ][kTabQ], double v[kTabQ][kTabQ])
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += a[p][q] * a[p][q];
        if (off < 1e-34) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                if (std::fabs(a[p][q]) < 1e-300) continue;
                const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(1.0 + theta * theta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q of A
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q of A
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[k][p], vkq = v[k][q];
                    v[k][p] = c * vkp - s * vkq;
                    v[k][q] = s * vkp + c * vkq;
                }
            }
        }
    }
}

double hermite(int n, double x)
{
    double h0 = 1.0, h1 = x;
    if (n == 0) return h0;
    for (int m = 1; m < n; ++m) {
        const double h2 = x * h1 - m * h0;
        h0 = h1;
        h1 = h2;
    }
    return h1;
}

}  // namespace

bool gauss_hermite(int Q, double *x, double *w)
{
    if (Q < 1 || Q > kTabQ) return false;
    double a[kTabQ][kTabQ] = {}, v[kTabQ][kTabQ];
    for (int i = 0; i + 1 < Q; ++i) a[i][i + 1] = a[i + 1][i] = std::sqrt((double)(i + 1));
    jacobi_eigen(Q, a, v);
    int idx[kTabQ];
    for (int i = 0; i < Q; ++i) idx[i] = i;
    std::sort(idx, idx + Q, [&](int p, int q) { return a[p][p] < a[q][q]; });
    double xs[kTabQ], ws[kTabQ];
    for (int i = 0; i < Q; ++i) {
        xs[i] = a[idx[i]][idx[i]];
        ws[i] = v[0][idx[i]] * v[0][idx[i]];
    }
    // the rule is symmetric about 0: average mirrored pairs, polish the roots
    // with two Newton steps on He_Q (He_Q' = Q He_{Q-1}), renormalise weights
    double sum = 0.0;
    for (int i = 0; i < Q; ++i) {
        const int m = Q - 1 - i;
        double r = 0.5 * (xs[i] - xs[m]);
        if (i == m) r = 0.0;
        for (int it = 0; it < 2 && i != m; ++it) r -= hermite(Q, r) / (Q * hermite(Q - 1, r));
        x[i] = r;
        w[i] = 0.5 * (ws[i] + ws[m]);
        sum += w[i];
    }
    for (int i = 0; i < Q; ++i) w[i] /= sum;
    return true;
}

bool model_info(int model, double ds, double dt, ModelInfo *mi)
{
    if (model == LB_CS_D2Q9) {
        static const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        static const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        if (!(ds > 0) || !(dt > 0)) return false;
        mi->Q = 3;
        mi->K = 9;
        gauss_hermite(3, mi->xi, mi->wq);  // {-sqrt3, 0, sqrt3}, {1/6, 2/3, 1/6}
        const double cl = ds / dt;
        mi->cs = cl / std::sqrt(3.0);
        mi->cl = cl;
        for (int k = 0; k < 9; ++k) {
            mi->ki[k] = ex[k] + 1;
            mi->kj[k] = ey[k] + 1;
            mi->vx[k] = ex[k] * cl;
            mi->vy[k] = ey[k] * cl;
            mi->w[k] = mi->wq[mi->ki[k]] * mi->wq[mi->kj[k]];
        }
    } else if (model >= LB_FD_D2Q9 && model <= LB_FD_D2Q36) {
        const int Q = model + 2;
        mi->Q = Q;
        mi->K = Q * Q;
        gauss_hermite(Q, mi->xi, mi->wq);
        mi->cs = 1.0;
        mi->cl = 1.0;
        for (int j = 0; j < Q; ++j)
            for (int i = 0; i < Q; ++i) {
                const int k = j * Q + i;
                mi->ki[k] = i;
                mi->kj[k] = j;
                mi->vx[k] = mi->xi[i];
                mi->vy[k] = mi->xi[j];
                mi->w[k] = mi->wq[i] * mi->wq[j];
            }
    } else {
        return false;
    }
    // He_n(xi_i) / n! for the order-N equilibrium
    for (int i = 0; i < mi->Q; ++i) {
        double fact = 1.0;
        for (int n = 0; n <= kTabN; ++n) {
            if (n > 1) fact *= n;
            mi->hc[i][n] = hermite(n, mi->xi[i]) / fact;
        }
    }
    return true;
}

}  // namespace lbm

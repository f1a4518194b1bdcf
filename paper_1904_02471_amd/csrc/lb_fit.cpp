// lb_fit.cpp -- decay rate of an amplitude series (lb_fit_decay), the FP64
// fit that turns the sampled diagnostics into an apparent viscosity: the
// shear wave decays as exp(-nu k^2 t) (Section 4.2), the Taylor-Green vortex
// as exp(-2 nu k^2 t) (Section 4.3), so nu_app = rate / k^2 or rate / (2 k^2).
//
// Least squares of y = ln|A(t)| on the columns {1, -t} (plain log-linear),
// or {1, -t, cos(omega t), sin(omega t)} when a modulation of angular
// frequency omega is fitted along.  Solved by modified Gram-Schmidt QR of
// the design in long double: the columns are orthogonalised in
// order, so the rate is the coefficient of the second column after
// back-substitution (the constant column first, so t is in effect centred).
#include <cmath>
#include <vector>

#include "lb.h"
#include "lb_sim_impl.h"

namespace lbm {

int fit_decay_rate(const double *t, const double *amp, int n, double omega, double *rate)
{
    const int m = omega > 0.0 ? 4 : 2;
    if (!t || !amp || !rate || n < m + 1 || !(omega >= 0.0) || !std::isfinite(omega)) return LB_EINVAL;
    std::vector<long double> y(n);
    std::vector<std::vector<long double>> q(m, std::vector<long double>(n));
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(t[i]) || !std::isfinite(amp[i]) || amp[i] == 0.0) return LB_EINVAL;
        y[i] = std::log(std::fabs((long double)amp[i]));
        q[0][i] = 1.0L;
        q[1][i] = -(long double)t[i];
        if (m == 4) {
            q[2][i] = std::cos((long double)omega * (long double)t[i]);
            q[3][i] = std::sin((long double)omega * (long double)t[i]);
        }
    }
    // modified Gram-Schmidt: q_j orthonormal, r upper triangular
    long double r[4][4] = {};
    for (int j = 0; j < m; ++j) {
        for (int k = 0; k < j; ++k) {
            long double d = 0.0L;
            for (int i = 0; i < n; ++i) d += q[k][i] * q[j][i];
            r[k][j] = d;
            for (int i = 0; i < n; ++i) q[j][i] -= d * q[k][i];
        }
        long double nn = 0.0L;
        for (int i = 0; i < n; ++i) nn += q[j][i] * q[j][i];
        nn = std::sqrt(nn);
        if (!(nn > 0.0L)) return LB_EINVAL;  // degenerate design (equal times, aliased frequency)
        r[j][j] = nn;
        for (int i = 0; i < n; ++i) q[j][i] /= nn;
    }
    // coefficients: R c = Q^T y
    long double b[4] = {};
    for (int j = 0; j < m; ++j) {
        long double d = 0.0L;
        for (int i = 0; i < n; ++i) d += q[j][i] * y[i];
        b[j] = d;
    }
    long double c[4] = {};
    for (int j = m - 1; j >= 0; --j) {
        long double s = b[j];
        for (int k = j + 1; k < m; ++k) s -= r[j][k] * c[k];
        c[j] = s / r[j][j];
    }
    *rate = (double)c[1];
    return std::isfinite(*rate) ? LB_OK : LB_ENAN;
}

}  // namespace lbm

extern "C" int lb_fit_decay(const double *t, const double *amp, int n, double omega, double *rate)
{
    const int rc = lbm::fit_decay_rate(t, amp, n, omega, rate);
    return rc == LB_OK ? LB_OK : lbm::set_last_error(rc);
}

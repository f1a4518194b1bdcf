// lb_model.h -- host tables of the velocity sets (no HIP dependency).
#pragma once

#include "lb.h"

namespace lbm {

constexpr int kTabQ = 6;  // largest per-axis order
constexpr int kTabN = kTabQ - 1;  // largest equilibrium order

struct ModelInfo {
    int K, Q;
    double cs;   // sound speed
    double cl;   // CS lattice speed ds/dt (1 for FD)
    double xi[kTabQ], wq[kTabQ];  // 1-D roots (units of c_s) and weights
    double vx[kTabQ * kTabQ], vy[kTabQ * kTabQ], w[kTabQ * kTabQ];
    int ki[kTabQ * kTabQ], kj[kTabQ * kTabQ];
    double hc[kTabQ][kTabQ];  // He_n(xi_i) / n!, n = 0..5
};

// Q-point Gauss-Hermite rule (ascending roots, weights summing to 1).
bool gauss_hermite(int Q, double *x, double *w);

// Velocity set, weights and equilibrium table of a model.
bool model_info(int model, double ds, double dt, ModelInfo *mi);

}  // namespace lbm

// lb_cs_impl.h -- device code of the collision-streaming D2Q9 step, shared
// by the single-simulation kernel (lb_cs.hip) and the batched kernel
// (lb_batch.hip), so that both evaluate the same rounded expressions.
//
// One launch advances every node by one time step of the CS evolution
// equation (Section 2): f_k(x + e_k, t + 1) = f_k - omega (f_k - f_eq_k),
// omega = dt / tau, with the second-order equilibrium of Section 2.
//
// Storage and mapping
//   * Structure of arrays: plane k holds population k, rows of `pitch`
//     elements, x contiguous; 64 lanes of a wave read 64 consecutive x.
//   * Pull scheme with two buffers: the buffer after step n holds the
//     post-collision values of step n at their source node; a node gathers
//     its 9 incoming values from the neighbours (x - e_k), collides in
//     registers and writes 9 values at its own position.  Each stored value
//     is read exactly once per step: 9 loads + 9 stores per node.
//   * Stored values are shifted, g_k = f_k - w_k rho0, which keeps the
//     small deviations from the reference state in the mantissa (FP32 and
//     FP16 storage); all arithmetic in FP32 (FP64 for double storage).
//   * One workgroup per row, threads striding over x: the periodic x-wrap and
//     the +-1 misaligned x-gathers stay inside one workgroup, so no cache line
//     is shared between workgroups on different XCDs.
//   * Fixed-value x ends: the buffers carry one ghost column on each side
//     (xoff = 1); the step writes the end equilibria into the ghost entries
//     that the next step pulls from.

#pragma once

#include <type_traits>

#include "lb_diag.h"
#include "lb_internal.h"

namespace lbm {

constexpr int kCsThreads = 256;

__device__ __forceinline__ float cs_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double cs_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One row y of the step (all threads of a 256-thread workgroup); with DIAG
// the diagnostics of the row's input state go to partial[diag_block].
template <typename T, bool FIXED, bool DIAG>
__device__ __forceinline__ void cs_row(const T *__restrict__ src, T *__restrict__ dst,
                                       const Params<typename Arith<T>::type> &p,
                                       const DiagArgs<typename Arith<T>::type> &d, int y, int diag_block)
{
    using CT = typename Arith<T>::type;
    const int Nx = p.Nx;
    const int ym = (y == 0) ? p.Ny - 1 : y - 1;
    const int yp = (y == p.Ny - 1) ? 0 : y + 1;
    const long long P = p.plane;
    const T *r0 = src + (long long)y * p.pitch + p.xoff;   // row y
    const T *rs = src + (long long)ym * p.pitch + p.xoff;  // row y-1: sources of N, NE, NW
    const T *rn = src + (long long)yp * p.pitch + p.xoff;  // row y+1: sources of S, SW, SE
    T *o = dst + (long long)y * p.pitch + p.xoff;

    const CT w0 = p.cs_w0, w1 = p.cs_w1, w5 = p.cs_w5, a1 = p.cs_a1, a5 = p.cs_a5;
    const CT b1 = CT(0.5), b5 = CT(0.125);  // 4.5 w, exact
    const CT omega = p.omega, rho0 = p.rho0;
    const CT c15 = CT(1.5);

    DiagAcc acc;
    CT pay = CT(0), pby = CT(0);
    if (DIAG && d.ax) {
        pay = d.ay[y];
        pby = d.by[y];
    }

    for (int x = threadIdx.x; x < Nx; x += kCsThreads) {
        int xm, xp;
        if (FIXED) {
            xm = x - 1;  // ghost column at -1 / Nx lives in memory
            xp = x + 1;
        } else {
            xm = (x == 0) ? Nx - 1 : x - 1;
            xp = (x == Nx - 1) ? 0 : x + 1;
        }
        // gather: population k arrives from x - e_k
        const CT g0 = ld(r0 + x);
        const CT g1 = ld(r0 + 1 * P + xm);  // E  from (x-1, y)
        const CT g2 = ld(rs + 2 * P + x);   // N  from (x, y-1)
        const CT g3 = ld(r0 + 3 * P + xp);  // W  from (x+1, y)
        const CT g4 = ld(rn + 4 * P + x);   // S  from (x, y+1)
        const CT g5 = ld(rs + 5 * P + xm);  // NE from (x-1, y-1)
        const CT g6 = ld(rs + 6 * P + xp);  // NW from (x+1, y-1)
        const CT g7 = ld(rn + 7 * P + xp);  // SW from (x+1, y+1)
        const CT g8 = ld(rn + 8 * P + xm);  // SE from (x-1, y+1)

        // moments (lattice velocity units: u / c_l)
        const CT drho = ((g0 + g1) + (g2 + g3)) + ((g4 + g5) + (g6 + g7)) + g8;
        const CT rho = rho0 + drho;
        const CT jx = (g1 - g3) + (g5 - g6) + (g8 - g7);
        const CT jy = (g2 - g4) + (g5 + g6) - (g7 + g8);
        const CT inv = CT(1) / rho;
        const CT ux = jx * inv, uy = jy * inv;
        const CT usq = c15 * cs_fma(ux, ux, uy * uy);

        // second-order equilibrium, shifted, written as
        //   w_k drho + a_k (e_k . j) + rho (b_k (e_k . u)^2 - w_k 1.5 u^2),
        // a = 3 w, b = 4.5 w: the first-order term takes j itself (rho * (j / rho)
        // would carry the quotient's rounding into the momentum every step), and
        // with the constants' exact sums the mass and momentum of the
        // equilibrium equal the node's up to unbiased rounding.
        auto relax = [&](CT g, CT w, CT a, CT b, CT ej, CT eu) -> CT {
            const CT sec = rho * cs_fma(b * eu, eu, -(w * usq));
            const CT geq = cs_fma(w, drho, cs_fma(a, ej, sec));
            return cs_fma(omega, geq - g, g);
        };
        // FP16 storage rounds stochastically: one counter-based draw per
        // node and step, advanced per population (unused otherwise)
        uint32_t rb = 0;
        if constexpr (std::is_same<T, __half>::value) rb = mix32((uint32_t)(y * Nx + x), p.salt);
        auto put = [&](T *q, CT v) {
            if constexpr (std::is_same<T, __half>::value) rb = xorshift32(rb);
            store_state(q, v, rb);
        };
        {
            const CT geq0 = cs_fma(w0, drho, -(rho * (w0 * usq)));
            put(o + x, cs_fma(omega, geq0 - g0, g0));
        }
        put(o + 1 * P + x, relax(g1, w1, a1, b1, jx, ux));
        put(o + 2 * P + x, relax(g2, w1, a1, b1, jy, uy));
        put(o + 3 * P + x, relax(g3, w1, a1, b1, -jx, -ux));
        put(o + 4 * P + x, relax(g4, w1, a1, b1, -jy, -uy));
        put(o + 5 * P + x, relax(g5, w5, a5, b5, jx + jy, ux + uy));
        put(o + 6 * P + x, relax(g6, w5, a5, b5, jy - jx, uy - ux));
        put(o + 7 * P + x, relax(g7, w5, a5, b5, -jx - jy, -ux - uy));
        put(o + 8 * P + x, relax(g8, w5, a5, b5, jx - jy, ux - uy));

        if (FIXED) {
            // the next step pulls E, NE, SE into x = 0 from column -1 and W,
            // NW, SW into x = Nx-1 from column Nx: keep the end equilibria there
            if (x == 0) {
                store_from(o + 1 * P - 1, p.ghost_l[1]);
                store_from(o + 5 * P - 1, p.ghost_l[5]);
                store_from(o + 8 * P - 1, p.ghost_l[8]);
            }
            if (x == Nx - 1) {
                store_from(o + 3 * P + Nx, p.ghost_r[3]);
                store_from(o + 6 * P + Nx, p.ghost_r[6]);
                store_from(o + 7 * P + Nx, p.ghost_r[7]);
            }
        }
        if (DIAG) {
            acc.v[0] += (double)drho;
            acc.v[1] += (double)jx;
            acc.v[2] += (double)jy;
            acc.v[3] += (double)(CT(0.5) * rho * (ux * ux + uy * uy));
            if (d.ax) acc.v[4] += (double)(ux * (d.ax[x] * pay) + uy * (d.bx[x] * pby));
        }
    }
    if (DIAG) block_diag_store(acc, d.partial, diag_block);
}

}  // namespace lbm

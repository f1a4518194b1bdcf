"""Shared helpers of the GPU parity tests: paired GPU / oracle simulations
and the tolerances derived from the arithmetic.

Tolerances (per element of the canonical state f, absolute):
  FP64 storage: both sides compute in double; they differ by summation order
      and fused multiply-adds only: 1e-13 * (n + 1) * max|f|.
  FP32 storage: every stored and computed quantity is a shifted one
      (g = f - w rho0, drho = rho - rho0, u, the equilibrium's departure
      w_k (drho + rho P'(u)) from w_k rho0); the O(1) density rho0 + drho
      enters only as the factor of P'(u) = O(|u|), so each rounding is
      relative to the shifted signal.  Each step adds at most ~C u32 max|g|
      with C = 32 (about 30 rounded operations feed one output), u32 =
      2^-24, g = f - w rho0 of the oracle's state, plus the oracle's own
      FP64 rounding of the unshifted f:
      tol = 32 u32 (n + 1) max|g| + 1e-13 (n + 1) max|f|.
  FP16 storage: the stored g carries a relative rounding of u16 = 2^-11 per
      step: tol = 2 u16 (n + 1) max|g| + the FP32 bound (FP16 relative to a
      reference equilibrium stores smaller departures: the same bound).  The
      rounding is stochastic and unbiased, so the parity tests also hold the
      rms error over the state to 2 u16 sqrt(n + 1) rms g.
"""
import numpy as np

import oracle
from paper_1904_02471_amd import lb

U32 = 2.0 ** -24
U16 = 2.0 ** -11

ORACLE_MODEL = {lb.LB_CS_D2Q9: oracle.CS_D2Q9, lb.LB_FD_D2Q9: oracle.FD_D2Q9, lb.LB_FD_D2Q16: oracle.FD_D2Q16,
                lb.LB_FD_D2Q25: oracle.FD_D2Q25, lb.LB_FD_D2Q36: oracle.FD_D2Q36}
PREC_NAME = {lb.LB_FP32: "fp32", lb.LB_FP16_SHIFTED: "fp16", lb.LB_FP64: "fp64", lb.LB_FP16_REF: "fp16ref"}


def pair(model, Nx, Ny, tau, dt, ds, N, prec, bc=None, eps=None):
    g = lb.Sim(model, Nx, Ny, tau, dt, ds, N, precision=prec)
    o = oracle.OracleSim(ORACLE_MODEL[model], Nx, Ny, tau, dt, ds, N)
    if bc is not None:
        g.set_bc_x(*bc)
        o.set_bc_x(*bc)
    if eps is not None:
        g.set_weno_eps(eps)
        o.set_weno_eps(eps)
    return g, o


def tolerance(prec, nsteps, f_ref, w, rho0):
    fmax = float(np.max(np.abs(f_ref)))
    gmax = float(np.max(np.abs(f_ref - w[:, None, None] * rho0)))
    if prec == lb.LB_FP64:
        return 1e-13 * (nsteps + 1) * fmax
    tol = 32 * U32 * (nsteps + 1) * gmax + 1e-13 * (nsteps + 1) * fmax
    if prec in (lb.LB_FP16_SHIFTED, lb.LB_FP16_REF):
        # (relative to a reference equilibrium the stored departures are at
        # most as large as g, so the same bound holds)
        tol += 2 * U16 * (nsteps + 1) * gmax
    return tol


def assert_state_close(gpu_f, orc_f, tol, what):
    err = np.abs(gpu_f - orc_f)
    i = np.unravel_index(np.argmax(err), err.shape)
    print("%s: max|df| = %.3e at %s (tol %.3e)" % (what, err[i], i, tol), flush=True)
    assert err[i] <= tol, "%s: max|df| %.3e at %s > tol %.3e" % (what, err[i], i, tol)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def field_errors(g, o):
    """rel-L2 of rho - rho0 and of u = (ux, uy) of a GPU simulation against
    the oracle's (rho0: the oracle's mean density)."""
    rg, xg, yg = g.moments()
    ro, xo, yo = o.moments()
    r0 = float(ro.mean())
    return rel_l2(rg - r0, ro - r0), rel_l2(np.stack([xg, yg]), np.stack([xo, yo]))

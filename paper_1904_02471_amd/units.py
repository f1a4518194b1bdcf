"""Relations between the non-dimensionalisations of the FD and CS models
(Section 3) and the standard lattice units used by the serving stream.

Unit systems
  FD:           length unit = system size L, speed unit c_ref, c_s = 1
  paper LU:     length unit = lattice spacing (L / N), ds = 1, dt = 1/sqrt(3), c_s = 1
  standard LU:  ds = dt = 1, c_s^2 = 1/3 (same length unit as paper LU, time
                unit sqrt(3) times shorter)
"""
import math

SQRT3 = math.sqrt(3.0)


def tau_lu_from_fd(tau_fd, n):
    """tau_LU = N tau_FD + sqrt(3)/6: the CS relaxation time that gives the
    FD viscosity nu_FD = tau_FD on N nodes (Section 3)."""
    return n * tau_fd + SQRT3 / 6.0


def tau_fd_from_lu(tau_lu, n):
    return (tau_lu - SQRT3 / 6.0) / n


def nu_cs(tau, dt, cs2):
    """CS viscosity nu = c_s^2 (tau - dt/2) (Section 2; c_s = 1 in paper LU)."""
    return cs2 * (tau - 0.5 * dt)


def nu_fd(tau_fd, T=1.0, m=1.0):
    """FD viscosity nu_FD = tau_FD T / m (Section 2, Chapman-Enskog)."""
    return tau_fd * T / m


def cs_step_in_fd_time(n):
    """One CS step (dt_LU = 1/sqrt 3) in FD time units, 1 / (N sqrt 3)."""
    return 1.0 / (n * SQRT3)


def tau_std_from_lu(tau_lu):
    return SQRT3 * tau_lu


def tau_lu_from_std(tau_std):
    return tau_std / SQRT3


def tau_fd_from_std(tau_std, n):
    """FD relaxation time with the viscosity of a CS run at tau_std
    (ds = dt = 1) on n nodes: nu_std = (tau_std - 1/2)/3 in (lattice spacing)^2
    per step; nu_FD = sqrt(3) nu_std / n."""
    return (tau_std - 0.5) / (SQRT3 * n)


def velocity_fd_from_std(u_std):
    """Speeds: u_FD = u_paperLU = sqrt(3) u_std."""
    return SQRT3 * u_std


def time_fd_from_std(t_std, n):
    """t_FD = t_paperLU / n = t_std / (sqrt(3) n)."""
    return t_std / (SQRT3 * n)


def fd_time_step(tau_fd, ds, vmax, cfl=0.5):
    """dt = min(CFL ds / max|v_k,alpha|, tau_FD): the CFL bound and the
    explicit-collision bound dt <= tau_FD (Section 4.1)."""
    return min(cfl * ds / vmax, tau_fd)

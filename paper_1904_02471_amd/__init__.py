"""MI355X-native isothermal lattice Boltzmann time step (Negro et al.,
arXiv:1904.02471): collision-streaming D2Q9 and finite-difference
Gauss-Hermite models behind the C ABI declared in include/lb.h.

Submodules
  lb         ctypes binding of liblbm.so (the HIP library), same names as the C ABI
  units      relations between the FD and CS non-dimensionalisations (Section 3)
  workloads  seeded synthetic initial states and request traces
  serve      continuous-batching front end of the lb_server_* API
"""
__all__ = ["lb", "units", "workloads"]

"""Linearised one-step operators of the two schemes for a Fourier mode,
written from the definitions (not from the oracle): used by the oracle pins
and by the GPU physics checks to predict decay rates."""
import numpy as np

E9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])


def cs_matrix(q, omega, w, xi):
    """CS step about rho = 1, u = 0: S [(1 - omega) I + omega Eq], with
    Eq_kl = w_k (1 + xi_k . xi_l) and S_kk = exp(-i q.e_k)."""
    K = len(w)
    Eq = w[:, None] * (1.0 + xi @ xi.T)
    S = np.diag(np.exp(-1j * (E9 @ q)))
    return S @ ((1 - omega) * np.eye(K) + omega * Eq)


def shear_decay_per_step(M, w, xi, axis):
    """Modulus of the eigenvalue whose eigenvector is closest to the
    transverse-momentum mode along `axis` (0: u_x, 1: u_y)."""
    lam, vec = np.linalg.eig(M)
    mode = w * xi[:, axis]
    overlap = np.abs(vec.conj().T @ mode) / np.linalg.norm(vec, axis=0)
    return abs(lam[np.argmax(overlap)])

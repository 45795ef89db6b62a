"""phi_1 and the exponential-Euler form of the LEM update (oracle).

Section 2 defines phi_k(z) = (e^z - sum_{l<k} z^l/l!)/z^k (the printed upper
limit of the sum is read as k-1, the standard definition that makes
z phi_1(z) = e^z - 1); phi = phi_1.  Update (5) of section 3 is
    v^{n+1} = v^n + dt phi(dt A_M)(A_M v^n + g_M),
which for g_M = 0 equals exp(dt A_M) v^n.  phi_1(B) b is read off the
exponential of the augmented matrix [[B, b], [0, 0]], whose last column is
[phi_1(B) b; 1].
"""
from __future__ import annotations

import numpy as np

from .expm import expm


def phi1_action(B: np.ndarray, b: np.ndarray) -> np.ndarray:
    n = B.shape[0]
    Z = np.zeros((n + 1, n + 1), dtype=np.result_type(B, b))
    Z[:n, :n] = B
    Z[:n, n] = b
    return expm(Z)[:n, n]


def phi1_matrix(B: np.ndarray) -> np.ndarray:
    """phi_1(B), the top-right block of expm([[B, I], [0, 0]])."""
    n = B.shape[0]
    Z = np.zeros((2 * n, 2 * n), dtype=B.dtype)
    Z[:n, :n] = B
    Z[:n, n:] = np.eye(n)
    return expm(Z)[:n, n:]


def phi1_scalar(z):
    """phi_1(z) = (e^z - 1)/z elementwise (real or complex), phi_1(0) = 1."""
    z = np.asarray(z)
    out = np.ones(z.shape, dtype=np.result_type(z, 1.0))
    nz = z != 0
    out[nz] = np.expm1(z[nz]) / z[nz]
    return out


def exp_euler_step(B: np.ndarray, v: np.ndarray, g: np.ndarray | None = None):
    """v + phi_1(B)(B v + dtg) with B = dt*A_M and dtg = dt times the forcing."""
    r = B @ v if g is None else B @ v + g
    return v + phi1_action(B, r)

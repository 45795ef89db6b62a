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


def exp_euler_step(B: np.ndarray, v: np.ndarray, g: np.ndarray | None = None):
    """v + phi_1(B)(B v + dt g) with B = dt*A_M (g already in rate units)."""
    r = B @ v if g is None else B @ v + g
    return v + phi1_action(B, r)

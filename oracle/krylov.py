"""Krylov approximation of exp(A) v (oracle; test infrastructure only).

Section 4.3 computes both the global reference and the local actions with the
Krylov method of Saad (1992): build an orthonormal basis V_m of
K_m(A, v) = span{v, Av, ..., A^{m-1} v} by Arnoldi, with the upper Hessenberg
H_m = V_m^T A V_m, and approximate exp(A) v ~ beta V_m exp(H_m) e_1,
beta = ||v||.  Saad's a posteriori estimate of the error is
beta * h_{m+1,m} * |e_m^T exp(H_m) e_1|.  When it is too large the step is
cut into sub-steps (exp(A) = exp(sA) exp((1-s)A)), as in Sidje's Expokit.

Arnoldi here is modified Gram-Schmidt with one full re-orthogonalization
pass.  A happy breakdown (h_{j+1,j} ~ 0) means K_j is invariant and the
approximation is exact at dimension j.  ``A`` is passed as a matvec that
already includes the time step (it applies dt*A).
"""
from __future__ import annotations

import numpy as np

from .expm import expm


def arnoldi(matvec, v: np.ndarray, m: int, breakdown_tol: float = 1e-13):
    """Returns (beta, V, H, k): V is n x (k+1) (the last column is v_{k+1},
    zero on breakdown), H is (k+1) x k, k <= m the dimension reached."""
    n = v.shape[0]
    beta = float(np.linalg.norm(v))
    dt = np.result_type(v.dtype, np.float64)
    V = np.zeros((n, m + 1), dtype=dt)
    H = np.zeros((m + 1, m), dtype=dt)
    if beta == 0.0:
        return beta, V[:, :1], H[:1, :0], 0
    V[:, 0] = v / beta
    scale = 0.0
    for j in range(m):
        w = matvec(V[:, j])
        scale = max(scale, float(np.linalg.norm(w)))
        for _ in range(2):  # MGS, then one re-orthogonalization pass
            for i in range(j + 1):
                c = np.vdot(V[:, i], w)
                H[i, j] += c
                w = w - c * V[:, i]
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        if hn <= breakdown_tol * max(scale, 1e-300):
            return beta, V[:, : j + 2], H[: j + 2, : j + 1], j + 1
        V[:, j + 1] = w / hn
    return beta, V, H, m


def expv(matvec, v: np.ndarray, m: int = 40, tol: float = 1e-14,
         return_info: bool = False):
    """exp(A) v with sub-steps so that each sub-step's estimate is within
    tol * (sub-step fraction) * ||v||.  ``matvec`` applies A (dt included)."""
    w = np.array(v, dtype=np.result_type(v.dtype, np.float64))
    done = 0.0
    s = 1.0
    n_sub = 0
    norm0 = float(np.linalg.norm(v))
    while done < 1.0 - 1e-15:
        s = min(s, 1.0 - done)
        beta, V, H, k = arnoldi(matvec, w, m)
        if beta == 0.0:
            break
        happy = k < m or H[k, k - 1] == 0.0
        while True:
            F = expm(s * H[:k, :k])
            f = F[:, 0]
            if happy:
                err = 0.0
            else:
                err = beta * s * abs(H[k, k - 1]) * abs(f[k - 1])
            if err <= tol * s * max(norm0, 1e-300) or s < 1e-12:
                break
            s *= 0.5
        w = beta * (V[:, :k] @ f)
        done += s
        n_sub += 1
    if return_info:
        return w, {"substeps": n_sub}
    return w

"""One step of the Local Exponential Method (oracle; test infrastructure).

Section 3: for every region M_i = D_i u B_i,
  1. restrict u^n to M_i and take the local problem (4), whose matrix A_{M_i}
     is the restriction of A to the nodes of M_i with the couplings to nodes
     outside M_i removed (homogeneous Dirichlet data on the box boundary --
     the forcing g is zero for the periodic problems here);
  2. advance it by one step of (5); with g = 0 the exponential-Euler update
     v + dt phi(dt A_M)(A_M v) equals exp(dt A_M) v (see phi.py);
  3. overwrite u^{n+1} on the core D_i with the local result, discarding the
     buffer rows.

The local exponential is the exact one (dense Pade on the principal submatrix
of dt*A), so this is the plain definition

    u^{n+1}[S_i] = expm(dt A[G_i, G_i])[core rows, :] @ u^n[G_i]

for every block i and every column of an ensemble.  Identical local matrices
(constant coefficients) are exponentiated once and reused; nothing else is
shared between blocks.
"""
from __future__ import annotations

import hashlib

import numpy as np

from . import partition as P
from .expm import expm
from .krylov import expv


class LocalExpCache:
    """Memo of core rows of expm(dt A_M), keyed by the exact local matrix."""

    def __init__(self):
        self.store = {}

    def get(self, A_loc: np.ndarray, rows: np.ndarray) -> np.ndarray:
        key = (A_loc.shape, hashlib.sha1(A_loc.tobytes()).hexdigest(),
               hashlib.sha1(rows.tobytes()).hexdigest())
        E = self.store.get(key)
        if E is None:
            E = expm(A_loc)[rows, :]
            self.store[key] = E
        return E


def local_matrix(A_sparse, G: np.ndarray) -> np.ndarray:
    """Principal submatrix dt*A[G, G] (couplings leaving the box dropped)."""
    return A_sparse[G][:, G].toarray()


def step(A_sparse, boxes, ndim: int, n: int, u: np.ndarray,
         cache: LocalExpCache | None = None, krylov_above: int = 0,
         krylov_m: int = 40, krylov_tol: float = 1e-15) -> np.ndarray:
    """One LEM step for u of shape (N,) or (N, k).  Blocks with more than
    ``krylov_above`` local points (when > 0) use the Krylov action instead of
    the dense local exponential."""
    cache = cache if cache is not None else LocalExpCache()
    vec = u.ndim == 1
    U = u.reshape(u.shape[0], -1)
    out = np.full_like(U, np.nan)
    for b in boxes:
        G = P.gather_map(b, ndim, n)
        S = P.scatter_map(b, ndim, n)
        rows = P.core_local_rows(b, ndim)
        A_loc_sp = A_sparse[G][:, G]
        if krylov_above and len(G) > krylov_above:
            mv = lambda x, M=A_loc_sp: M @ x
            for c in range(U.shape[1]):
                out[S, c] = expv(mv, U[G, c], m=krylov_m, tol=krylov_tol)[rows]
        else:
            E = cache.get(A_loc_sp.toarray(), rows)
            out[S] = E @ U[G]
    return out[:, 0] if vec else out


def run(A_sparse, boxes, ndim: int, n: int, u: np.ndarray, n_steps: int,
        cache: LocalExpCache | None = None, **kw) -> np.ndarray:
    cache = cache if cache is not None else LocalExpCache()
    for _ in range(n_steps):
        u = step(A_sparse, boxes, ndim, n, u, cache, **kw)
    return u

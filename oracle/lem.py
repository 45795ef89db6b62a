"""One step of the Local Exponential Method (oracle; test infrastructure).

Section 3: for every region M_i = D_i u B_i,
  1. restrict u^n to M_i and take the local problem (4), whose matrix A_{M_i}
     is the restriction of A to the nodes of M_i with the couplings to nodes
     outside M_i removed (homogeneous Dirichlet data on the box boundary --
     the forcing g is zero for the periodic problems here);
  2. advance it by one step of (5); with g = 0 the exponential-Euler update
     v + dt phi(dt A_M)(A_M v) equals exp(dt A_M) v (see phi.py); with a
     forcing g (constant over the step, restricted to M_i) it is
     exp(dt A_M) v + phi_1(dt A_M)(dt g_M), phi_1 read off the exponential of
     an augmented matrix;
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
from .phi import phi1_matrix


class LocalExpCache:
    """Memo of core rows of expm(dt A_M) (and of phi_1(dt A_M)), keyed by the
    exact local matrix."""

    def __init__(self):
        self.store = {}

    def _key(self, kind, A_loc, rows):
        return (kind, A_loc.shape, hashlib.sha1(A_loc.tobytes()).hexdigest(),
                hashlib.sha1(rows.tobytes()).hexdigest())

    def get(self, A_loc: np.ndarray, rows: np.ndarray) -> np.ndarray:
        key = self._key("exp", A_loc, rows)
        E = self.store.get(key)
        if E is None:
            E = expm(A_loc)[rows, :]
            self.store[key] = E
        return E

    def get_phi1(self, A_loc: np.ndarray, rows: np.ndarray) -> np.ndarray:
        key = self._key("phi1", A_loc, rows)
        F = self.store.get(key)
        if F is None:
            F = phi1_matrix(A_loc)[rows, :]
            self.store[key] = F
        return F


def local_matrix(A_sparse, G: np.ndarray) -> np.ndarray:
    """Principal submatrix dt*A[G, G] (couplings leaving the box dropped)."""
    return A_sparse[G][:, G].toarray()


def step(A_sparse, boxes, ndim: int, n: int, u: np.ndarray,
         cache: LocalExpCache | None = None, krylov_above: int = 0,
         krylov_m: int = 40, krylov_tol: float = 1e-15,
         dtg: np.ndarray | None = None) -> np.ndarray:
    """One LEM step for u of shape (N,) or (N, k).  Blocks with more than
    ``krylov_above`` local points (when > 0) use the Krylov action instead of
    the dense local exponential.  ``dtg`` (shape of u) is dt times a forcing g
    that is constant over the step; the local update is then
    exp(dt A_M) v + phi_1(dt A_M) (dt g)_M, the Krylov branch taking it as the
    action of the augmented matrix [[dt A_M, (dt g)_M], [0, 0]] on [v; 1]."""
    cache = cache if cache is not None else LocalExpCache()
    vec = u.ndim == 1
    U = u.reshape(u.shape[0], -1)
    F = None if dtg is None else np.asarray(dtg, dtype=float).reshape(U.shape)
    out = np.full_like(U, np.nan)
    for b in boxes:
        G = P.gather_map(b, ndim, n)
        S = P.scatter_map(b, ndim, n)
        rows = P.core_local_rows(b, ndim, n)
        A_loc_sp = A_sparse[G][:, G]
        if krylov_above and len(G) > krylov_above:
            for c in range(U.shape[1]):
                if F is None:
                    mv = lambda x, M=A_loc_sp: M @ x
                    out[S, c] = expv(mv, U[G, c], m=krylov_m, tol=krylov_tol)[rows]
                else:
                    f = F[G, c]
                    mv = lambda x, M=A_loc_sp, f=f: np.concatenate([M @ x[:-1] + f * x[-1], [0.0]])
                    x0 = np.concatenate([U[G, c], [1.0]])
                    out[S, c] = expv(mv, x0, m=krylov_m, tol=krylov_tol)[:-1][rows]
        else:
            A_loc = A_loc_sp.toarray()
            out[S] = cache.get(A_loc, rows) @ U[G]
            if F is not None:
                out[S] += cache.get_phi1(A_loc, rows) @ F[G]
    return out[:, 0] if vec else out


def run(A_sparse, boxes, ndim: int, n: int, u: np.ndarray, n_steps: int,
        cache: LocalExpCache | None = None, **kw) -> np.ndarray:
    cache = cache if cache is not None else LocalExpCache()
    for _ in range(n_steps):
        u = step(A_sparse, boxes, ndim, n, u, cache, **kw)
    return u

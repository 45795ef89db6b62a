"""LEM for the 1D Schroedinger equation with a harmonic potential (oracle;
test infrastructure).

Section 4.1 tests the method on

    c_t = (i/2) c_xx - i (kappa/2) x^2 c,   x in [-L/2, L/2), periodic,

with centered differences on n points (x_j = -L/2 + j dx, dx = L/n), i.e.
c' = -i H c with the real symmetric matrix

    H = -(1/2) D2 + diag(kappa x_j^2 / 2),   (D2 c)_j = (c_{j-1} - 2 c_j + c_{j+1}) / dx^2.

The LEM step is the one of section 3 with complex local problems: on every
region M_i the local matrix is the principal submatrix -i dt H[G_i, G_i]
(couplings to nodes outside M_i dropped), its exponential is taken directly
in complex arithmetic (Pade [13/13] of expm.py), and its core rows overwrite
the state.  The whole-grid box (core = n, halo = 0) keeps the periodic
coupling and is the global method.

Reading taken for the stability number of this problem: mu = nu dt / dx^2
with nu = 1/2, the coefficient of c_xx, so dt = 2 mu dx^2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import partition as P
from .expm import expm


def grid(n: int, L: float) -> np.ndarray:
    return -0.5 * L + np.arange(n) * (L / n)


def hamiltonian(n: int, L: float, kappa: float) -> sp.csr_matrix:
    """H = -(1/2) D2 + kappa x^2 / 2 on the periodic grid (real symmetric)."""
    dx = L / n
    x = grid(n, L)
    i = np.arange(n)
    off = np.full(n, -0.5 / (dx * dx))
    diag = 1.0 / (dx * dx) + 0.5 * kappa * x * x
    rows = np.concatenate([i, i, i])
    cols = np.concatenate([i, (i - 1) % n, (i + 1) % n])
    vals = np.concatenate([diag, off, off])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def global_propagator(n: int, L: float, kappa: float, dt: float) -> np.ndarray:
    """exp(-i dt H), the exact step of the semi-discrete problem."""
    return expm(-1j * dt * hamiltonian(n, L, kappa).toarray())


def global_run(c0: np.ndarray, L: float, kappa: float, dt: float, n_steps: int) -> np.ndarray:
    E = global_propagator(c0.shape[0], L, kappa, dt)
    c = c0.astype(complex)
    for _ in range(n_steps):
        c = E @ c
    return c


def lem_blocks(n: int, L: float, kappa: float, dt: float, core: int, halo: int):
    """(gather map, scatter map, core rows of exp(-i dt H[G, G])) per region."""
    H = hamiltonian(n, L, kappa).toarray()
    out = []
    for b in P.uniform_boxes(1, n, core, halo):
        G = P.gather_map(b, 1, n)
        rows = P.core_local_rows(b, 1)
        E = expm(-1j * dt * H[np.ix_(G, G)])[rows, :]
        out.append((G, P.scatter_map(b, 1, n), E))
    return out


def lem_run(c0: np.ndarray, L: float, kappa: float, dt: float, n_steps: int, core: int,
            halo: int) -> np.ndarray:
    """n_steps LEM steps of c0 (shape (n,) or (n, k), complex)."""
    n = c0.shape[0]
    blocks = lem_blocks(n, L, kappa, dt, core, halo)
    c = c0.astype(complex)
    for _ in range(n_steps):
        out = np.full_like(c, np.nan)
        for G, S, E in blocks:
            out[S] = E @ c[G]
        c = out
    return c


def coherent_state(x: np.ndarray, kappa: float, x0: float, p0: float = 0.0) -> np.ndarray:
    """Gaussian of the oscillator's ground-state width centred at x0 with
    momentum p0: exp(-omega (x - x0)^2 / 2 + i p0 x), omega = sqrt(kappa)."""
    w = np.sqrt(kappa)
    return np.exp(-0.5 * w * (x - x0) ** 2 + 1j * p0 * x)


def coherent_state_exact(x: np.ndarray, kappa: float, x0: float, t: float) -> np.ndarray:
    """The continuous solution for coherent_state(x, kappa, x0, 0): the same
    Gaussian with its centre at x0 cos(omega t) and momentum -omega x0
    sin(omega t), up to a global phase (so compare moduli or fix the phase)."""
    w = np.sqrt(kappa)
    xc = x0 * np.cos(w * t)
    pc = -w * x0 * np.sin(w * t)
    return np.exp(-0.5 * w * (x - xc) ** 2 + 1j * pc * x)

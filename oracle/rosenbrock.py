"""Exponential Rosenbrock-Euler LEM for a nonlinear problem (oracle; test
infrastructure).

Sections 3 and 4 of the paper advance nonlinear problems u' = F(u) by the
exponential Rosenbrock methods of Hochbruck, Lubich and Selhofer (1998); the
second-order member (exponential Rosenbrock-Euler) is

    u^{n+1} = u^n + dt phi_1(dt J) F(u^n),

J the Jacobian of F.  The local matrices make it affordable to freeze J (and
the local phi_1 matrices) over several steps: here J is taken at the state of
the last refresh, every ``refresh`` steps.  LEM applies the step region by
region: on M_i the local matrix is the principal submatrix J[G_i, G_i]
(couplings to nodes outside M_i dropped), F is evaluated on the whole grid
and restricted to M_i, and the core rows overwrite u^{n+1} (step 3).

The problem is the viscous Burgers equation of section 4.2,
u_t = -(u^2/2)_x + nu u_xx, on a periodic 1D grid.  Reading taken: centered
differences (the paper uses a monotonized finite volume flux, whose limiter
is out of scope):

    F_i = -(u_{i+1}^2 - u_{i-1}^2) / (4 dx) + nu (u_{i+1} - 2 u_i + u_{i-1}) / dx^2
    dF_i/du_{i-1} =  u_{i-1}/(2 dx) + nu/dx^2
    dF_i/du_i     = -2 nu/dx^2
    dF_i/du_{i+1} = -u_{i+1}/(2 dx) + nu/dx^2
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import partition as P
from .phi import phi1_matrix


def burgers_F(u: np.ndarray, dx: float, nu: float) -> np.ndarray:
    """F(u) for u of shape (n,) or (n, k) (columns independent)."""
    up = np.roll(u, -1, axis=0)
    um = np.roll(u, 1, axis=0)
    return -(up * up - um * um) / (4.0 * dx) + nu * (up - 2.0 * u + um) / (dx * dx)


def burgers_J(u: np.ndarray, dx: float, nu: float) -> sp.csr_matrix:
    """Jacobian of F at the state u (shape (n,)), periodic."""
    n = u.shape[0]
    i = np.arange(n)
    im, ip = (i - 1) % n, (i + 1) % n
    d = nu / (dx * dx)
    rows = np.concatenate([i, i, i])
    cols = np.concatenate([im, i, ip])
    vals = np.concatenate([u[im] / (2.0 * dx) + d, np.full(n, -2.0 * d), -u[ip] / (2.0 * dx) + d])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def ere_global_run(u0: np.ndarray, dx: float, nu: float, dt: float, n_steps: int,
                   refresh: int = 1) -> np.ndarray:
    """Global exponential Rosenbrock-Euler steps (D = 1) with the Jacobian
    refreshed every ``refresh`` steps; u0 of shape (n,) or (n, k)."""
    U = u0.reshape(u0.shape[0], -1).astype(float).copy()
    phis = [None] * U.shape[1]
    for step in range(n_steps):
        if step % refresh == 0:
            phis = [phi1_matrix(dt * burgers_J(U[:, c], dx, nu).toarray())
                    for c in range(U.shape[1])]
        Fu = burgers_F(U, dx, nu)
        U = U + dt * np.column_stack([phis[c] @ Fu[:, c] for c in range(U.shape[1])])
    return U[:, 0] if u0.ndim == 1 else U


def ere_lem_run(u0: np.ndarray, boxes, n: int, dx: float, nu: float, dt: float,
                n_steps: int, refresh: int = 1) -> np.ndarray:
    """LEM exponential Rosenbrock-Euler steps on 1D boxes: per region the core
    rows of v + dt phi_1(dt J_M) F(u)_M, J_M the principal submatrix of the
    Jacobian frozen at the last refresh."""
    U = u0.reshape(u0.shape[0], -1).astype(float).copy()
    maps = [(P.gather_map(b, 1, n), P.scatter_map(b, 1, n), P.core_local_rows(b, 1))
            for b in boxes]
    local = None
    for step in range(n_steps):
        if step % refresh == 0:
            local = []
            for c in range(U.shape[1]):
                J = burgers_J(U[:, c], dx, nu)
                local.append([phi1_matrix(dt * J[G][:, G].toarray())[rows, :]
                              for G, _, rows in maps])
        Fu = burgers_F(U, dx, nu)
        out = np.full_like(U, np.nan)
        for c in range(U.shape[1]):
            for k, (G, S, rows) in enumerate(maps):
                out[S, c] = U[G, c][rows] + dt * (local[c][k] @ Fu[G, c])
        U = out
    return U[:, 0] if u0.ndim == 1 else U


def rk4_reference(u0: np.ndarray, dx: float, nu: float, t: float, n_sub: int) -> np.ndarray:
    """Classical Runge-Kutta of order 4 with n_sub steps (a reference for the
    time-discretization error of the semi-discrete problem)."""
    u = u0.astype(float).copy()
    h = t / n_sub
    for _ in range(n_sub):
        k1 = burgers_F(u, dx, nu)
        k2 = burgers_F(u + 0.5 * h * k1, dx, nu)
        k3 = burgers_F(u + 0.5 * h * k2, dx, nu)
        k4 = burgers_F(u + h * k3, dx, nu)
        u = u + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return u

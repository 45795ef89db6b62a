"""The semi-discrete operator A (oracle; test infrastructure only).

Model problem: the linear advection-diffusion equation, eq. (2) of section 2,
with periodic boundaries as in the tests of section 4.1 (1D, eq. (6)) and
section 4.3 (2D, conservative form ibv2d).  The spatial discretization
(eq. (3)) is the centered second-order finite difference of section 4.1.

All weights are returned already multiplied by dt, i.e. they are the entries
of dt*A, so that with the stability parameters of section 2,
C = |a| dt/dx and mu = nu dt/dx^2, the constant-coefficient 1D row is

    (dt A u)_i = (mu + C/2) u_{i-1} - 2 mu u_i + (mu - C/2) u_{i+1}

(centered -a u_x contributes +C/2 to the west and -C/2 to the east neighbour,
centered nu u_xx contributes mu, -2 mu, mu).  In 2D the y axis adds
(mu_y + C_y/2) on the south (j-1) and (mu_y - C_y/2) on the north (j+1)
neighbour.  DOF index is j*n + i (x fastest).

For a per-node diffusivity nu(x) the diffusion term is taken in the
conservative flux form d/dx(nu du/dx) with the arithmetic mean on faces:
    mu_{i+1/2} = dt (nu_i + nu_{i+1}) / (2 dx^2),
so that w_E(i) = mu_{i+1/2} - C/2, w_W(i) = mu_{i-1/2} + C/2 and
w_0(i) = -(sum of the face mu's of node i).  Columns of dt*A then sum to zero
(the scheme conserves mass), which the constant case also satisfies.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Weights:
    """Per-node weights of dt*A, each of shape (ny, nx); ny = 1 in 1D.

    w[0]: centre, w[1]: west (i-1), w[2]: east (i+1), w[3]: south (j-1),
    w[4]: north (j+1).  S/N are zero in 1D.
    """

    ndim: int
    n: int
    w0: np.ndarray
    wW: np.ndarray
    wE: np.ndarray
    wS: np.ndarray
    wN: np.ndarray

    @property
    def N(self) -> int:
        return self.n ** self.ndim


def weights(ndim: int, n: int, dx: float, dt: float, vel, nu=None,
            nu_field=None) -> Weights:
    """Weights of dt*A for the periodic advection-diffusion operator."""
    ny = 1 if ndim == 1 else n
    shape = (ny, n)
    cx = vel[0] * dt / dx
    cy = (vel[1] * dt / dx) if ndim == 2 else 0.0
    if nu_field is None:
        mu = nu * dt / (dx * dx)
        mu_e = np.full(shape, mu)   # face (i+1/2, j)
        mu_w = np.full(shape, mu)   # face (i-1/2, j)
        mu_n = np.full(shape, mu if ndim == 2 else 0.0)
        mu_s = np.full(shape, mu if ndim == 2 else 0.0)
    else:
        f = np.asarray(nu_field, dtype=np.float64).reshape(shape)
        s = dt / (2.0 * dx * dx)
        mu_e = (f + np.roll(f, -1, axis=1)) * s
        mu_w = (f + np.roll(f, 1, axis=1)) * s
        if ndim == 2:
            mu_n = (f + np.roll(f, -1, axis=0)) * s
            mu_s = (f + np.roll(f, 1, axis=0)) * s
        else:
            mu_n = np.zeros(shape)
            mu_s = np.zeros(shape)
    wW = mu_w + cx / 2.0
    wE = mu_e - cx / 2.0
    if ndim == 2:
        wS = mu_s + cy / 2.0
        wN = mu_n - cy / 2.0
    else:
        wS = np.zeros(shape)
        wN = np.zeros(shape)
    w0 = -(mu_e + mu_w + mu_n + mu_s)
    return Weights(ndim, n, w0, wW, wE, wS, wN)


def apply(W: Weights, u: np.ndarray) -> np.ndarray:
    """(dt A) u for u of shape (N,) or (N, k), by shifts of the periodic grid."""
    ny = W.w0.shape[0]
    n = W.n
    vec = u.ndim == 1
    U = u.reshape(ny, n, -1)
    out = W.w0[..., None] * U
    out = out + W.wW[..., None] * np.roll(U, 1, axis=1)    # u_{i-1}
    out = out + W.wE[..., None] * np.roll(U, -1, axis=1)   # u_{i+1}
    if W.ndim == 2:
        out = out + W.wS[..., None] * np.roll(U, 1, axis=0)   # u_{j-1}
        out = out + W.wN[..., None] * np.roll(U, -1, axis=0)  # u_{j+1}
    out = out.reshape(W.N, -1)
    return out[:, 0] if vec else out


def sparse(W: Weights) -> sp.csr_matrix:
    """dt*A as a sparse N x N matrix with periodic wrap."""
    ny = W.w0.shape[0]
    n = W.n
    j, i = np.meshgrid(np.arange(ny), np.arange(n), indexing="ij")
    row = (j * n + i).reshape(-1)
    rows, cols, vals = [row], [row], [W.w0.reshape(-1)]
    rows.append(row); cols.append((j * n + (i - 1) % n).reshape(-1)); vals.append(W.wW.reshape(-1))
    rows.append(row); cols.append((j * n + (i + 1) % n).reshape(-1)); vals.append(W.wE.reshape(-1))
    if W.ndim == 2:
        rows.append(row); cols.append((((j - 1) % ny) * n + i).reshape(-1)); vals.append(W.wS.reshape(-1))
        rows.append(row); cols.append((((j + 1) % ny) * n + i).reshape(-1)); vals.append(W.wN.reshape(-1))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(W.N, W.N))
    return A.tocsr()  # duplicates (n <= 2) are summed, as the stencil sums them


def dense(W: Weights) -> np.ndarray:
    return sparse(W).toarray()


def from_problem(p) -> Weights:
    """Weights for a ``lem_inputs.Problem``."""
    return weights(p.ndim, p.n, p.dx, p.dt, p.vel, nu=p.nu, nu_field=p.nu_field)

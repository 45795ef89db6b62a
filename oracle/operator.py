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

A variable velocity enters in the conservative form -div(a c) of eq. ibv2d
(section 4.3) with centered face fluxes a_{i+1/2} (c_i + c_{i+1}) / 2: given
the face velocities a_x(i+1/2, j) and a_y(i, j+1/2), with
alpha_{i+1/2} = dt a_x(i+1/2, j) / (2 dx) (and alpha on y faces with dy),

    w_E = mu_e - alpha_e,  w_W = mu_w + alpha_w,  (likewise S, N)
    w_0 = -(mu_e + mu_w + mu_n + mu_s) - (alpha_e - alpha_w + alpha_n - alpha_s).

Columns still sum to zero for any face velocities; rows sum to zero (constant
states are steady) when the discrete divergence of the faces vanishes, as it
does exactly for faces taken from a stream function.  The y spacing dy may
differ from dx (anisotropic meshes, section 4.3); then C_y = a_y dt / dy and
mu_y = nu dt / dy^2.
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
            nu_field=None, vel_faces=None, dy=None) -> Weights:
    """Weights of dt*A for the periodic advection-diffusion operator.

    vel_faces (optional, replaces vel): array of shape (ndim, ny, n), a_x on
    the east face of each node and, in 2D, a_y on its north face.  dy: y
    spacing (default dx)."""
    ny = 1 if ndim == 1 else n
    shape = (ny, n)
    dy = dx if dy is None else dy
    if nu_field is None:
        mu = nu * dt / (dx * dx)
        muy = nu * dt / (dy * dy)
        mu_e = np.full(shape, mu)   # face (i+1/2, j)
        mu_w = np.full(shape, mu)   # face (i-1/2, j)
        mu_n = np.full(shape, muy if ndim == 2 else 0.0)
        mu_s = np.full(shape, muy if ndim == 2 else 0.0)
    else:
        f = np.asarray(nu_field, dtype=np.float64).reshape(shape)
        s = dt / (2.0 * dx * dx)
        sy = dt / (2.0 * dy * dy)
        mu_e = (f + np.roll(f, -1, axis=1)) * s
        mu_w = (f + np.roll(f, 1, axis=1)) * s
        if ndim == 2:
            mu_n = (f + np.roll(f, -1, axis=0)) * sy
            mu_s = (f + np.roll(f, 1, axis=0)) * sy
        else:
            mu_n = np.zeros(shape)
            mu_s = np.zeros(shape)
    if vel_faces is None:
        cx = vel[0] * dt / dx
        cy = (vel[1] * dt / dy) if ndim == 2 else 0.0
        al_e = al_w = np.full(shape, cx / 2.0)
        al_n = al_s = np.full(shape, cy / 2.0)
    else:
        F = np.asarray(vel_faces, dtype=np.float64).reshape((ndim,) + shape)
        al_e = F[0] * (dt / (2.0 * dx))
        al_w = np.roll(al_e, 1, axis=1)
        if ndim == 2:
            al_n = F[1] * (dt / (2.0 * dy))
            al_s = np.roll(al_n, 1, axis=0)
        else:
            al_n = al_s = np.zeros(shape)
    wW = mu_w + al_w
    wE = mu_e - al_e
    if ndim == 2:
        wS = mu_s + al_s
        wN = mu_n - al_n
    else:
        wS = np.zeros(shape)
        wN = np.zeros(shape)
    w0 = -(mu_e + mu_w + mu_n + mu_s)
    if vel_faces is not None:
        w0 = w0 - ((al_e - al_w) + (al_n - al_s))
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
    return weights(p.ndim, p.n, p.dx, p.dt, p.vel, nu=p.nu, nu_field=p.nu_field,
                   vel_faces=getattr(p, "vel_faces", None), dy=getattr(p, "dy", None))

"""The global exponential step u <- exp(dt A) u (oracle; test infrastructure).

This is the "standard exponential method" with D = 1 of section 4.1 (and the
exact solution formula of section 2).  With a forcing g constant in time the
step is u <- exp(dt A) u + phi_1(dt A)(dt g); ``dtg`` below is dt g.  For periodic constant
coefficients dt*A is circulant (block-circulant with circulant blocks in 2D),
so it is diagonalized by the discrete Fourier transform: a Fourier mode
exp(i theta j) is multiplied by the symbol

    lambda(theta) = w_W e^{-i theta_x} + w_E e^{+i theta_x}
                  + w_S e^{-i theta_y} + w_N e^{+i theta_y} + w_0,

theta = 2 pi k / n, and exp(dt A) u = ifft(exp(lambda) * fft(u)) -- the
"Fourier method and separation of variables" reference of section 4.1.
Otherwise: dense expm on small grids, the Krylov action on large ones.
"""
from __future__ import annotations

import numpy as np

from . import operator as op
from .expm import expm
from .krylov import expv
from .phi import exp_euler_step, phi1_scalar


def is_constant(W: op.Weights) -> bool:
    return all(np.all(a == a.flat[0]) for a in (W.w0, W.wW, W.wE, W.wS, W.wN))


def symbol(W: op.Weights) -> np.ndarray:
    """lambda on the (ny, nx) grid of wavenumbers (constant coefficients)."""
    if not is_constant(W):
        raise ValueError("the Fourier symbol needs constant coefficients")
    n = W.n
    th = 2.0 * np.pi * np.arange(n) / n
    lam_x = W.wW.flat[0] * np.exp(-1j * th) + W.wE.flat[0] * np.exp(1j * th)
    if W.ndim == 1:
        return (lam_x + W.w0.flat[0])[None, :]
    lam_y = W.wS.flat[0] * np.exp(-1j * th) + W.wN.flat[0] * np.exp(1j * th)
    return lam_y[:, None] + lam_x[None, :] + W.w0.flat[0]


def fft_steps(W: op.Weights, u: np.ndarray, n_steps: int = 1,
              dtg: np.ndarray | None = None) -> np.ndarray:
    """n_steps global steps for u of shape (N,) or (N, k), by the DFT: mode
    by mode u <- e^lambda u + phi_1(lambda) (dt g)."""
    vec = u.ndim == 1
    ny = 1 if W.ndim == 1 else W.n
    U = u.reshape(ny, W.n, -1)
    lam = symbol(W)[..., None]
    fwd = (lambda a: np.fft.fft(a, axis=1)) if W.ndim == 1 else \
        (lambda a: np.fft.fft2(a, axes=(0, 1)))
    inv = (lambda a: np.fft.ifft(a, axis=1)) if W.ndim == 1 else \
        (lambda a: np.fft.ifft2(a, axes=(0, 1)))
    Uh = fwd(U)
    if dtg is None:
        Uh = np.exp(n_steps * lam) * Uh
    else:
        Gh = fwd(np.asarray(dtg, dtype=float).reshape(U.shape))
        for _ in range(n_steps):
            Uh = np.exp(lam) * Uh + phi1_scalar(lam) * Gh
    out = inv(Uh).real.reshape(W.N, -1)
    return out[:, 0] if vec else out


def dense_step(W: op.Weights, u: np.ndarray, dtg: np.ndarray | None = None) -> np.ndarray:
    B = op.dense(W)
    if dtg is None:
        return expm(B) @ u
    U = u.reshape(u.shape[0], -1)
    F = np.asarray(dtg, dtype=float).reshape(U.shape)
    out = np.column_stack([exp_euler_step(B, U[:, c], F[:, c]) for c in range(U.shape[1])])
    return out[:, 0] if u.ndim == 1 else out


def krylov_step(W: op.Weights, u: np.ndarray, m: int = 40,
                tol: float = 1e-14, dtg: np.ndarray | None = None) -> np.ndarray:
    vec = u.ndim == 1
    U = u.reshape(u.shape[0], -1)
    F = None if dtg is None else np.asarray(dtg, dtype=float).reshape(U.shape)
    out = np.empty_like(U)
    for c in range(U.shape[1]):
        if F is None:
            out[:, c] = expv(lambda x: op.apply(W, x), U[:, c], m=m, tol=tol)
        else:
            f = F[:, c]
            mv = lambda x, f=f: np.concatenate([op.apply(W, x[:-1]) + f * x[-1], [0.0]])
            out[:, c] = expv(mv, np.concatenate([U[:, c], [1.0]]), m=m, tol=tol)[:-1]
    return out[:, 0] if vec else out


def steps(W: op.Weights, u: np.ndarray, n_steps: int, dtg: np.ndarray | None = None,
          **kw) -> np.ndarray:
    """n_steps global steps by the best available exact route."""
    if is_constant(W):
        return fft_steps(W, u, n_steps, dtg)
    for _ in range(n_steps):
        u = dense_step(W, u, dtg) if W.N <= 2048 else krylov_step(W, u, dtg=dtg, **kw)
    return u

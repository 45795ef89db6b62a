"""The global exponential step u <- exp(dt A) u (oracle; test infrastructure).

This is the "standard exponential method" with D = 1 of section 4.1 (and the
exact solution formula of section 2 with g = 0).  For periodic constant
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


def fft_steps(W: op.Weights, u: np.ndarray, n_steps: int = 1) -> np.ndarray:
    """exp(dt A)^n_steps u for u of shape (N,) or (N, k), by the DFT."""
    vec = u.ndim == 1
    ny = 1 if W.ndim == 1 else W.n
    U = u.reshape(ny, W.n, -1)
    g = np.exp(n_steps * symbol(W))[..., None]
    if W.ndim == 1:
        out = np.fft.ifft(g * np.fft.fft(U, axis=1), axis=1)
    else:
        out = np.fft.ifft2(g * np.fft.fft2(U, axes=(0, 1)), axes=(0, 1))
    out = out.real.reshape(W.N, -1)
    return out[:, 0] if vec else out


def dense_step(W: op.Weights, u: np.ndarray) -> np.ndarray:
    return expm(op.dense(W)) @ u


def krylov_step(W: op.Weights, u: np.ndarray, m: int = 40,
                tol: float = 1e-14) -> np.ndarray:
    vec = u.ndim == 1
    U = u.reshape(u.shape[0], -1)
    out = np.empty_like(U)
    for c in range(U.shape[1]):
        out[:, c] = expv(lambda x: op.apply(W, x), U[:, c], m=m, tol=tol)
    return out[:, 0] if vec else out


def steps(W: op.Weights, u: np.ndarray, n_steps: int, **kw) -> np.ndarray:
    """n_steps global steps by the best available exact route."""
    if is_constant(W):
        return fft_steps(W, u, n_steps)
    for _ in range(n_steps):
        u = dense_step(W, u) if W.N <= 2048 else krylov_step(W, u, **kw)
    return u

"""Seeded synthetic inputs for the Local Exponential Method workloads.

This module only draws numbers: grid sizes, physical coefficients (velocity,
diffusivity, time step) and initial states.  It holds none of the method's
arithmetic -- no stencil weights, no exponentials, no partitions -- so that both
the CPU oracle and the GPU path can consume the same inputs while sharing no
code.  Every generator uses NumPy's PCG64 ``default_rng(seed)`` with a fixed
draw order, so a (workload, seed) pair always yields the same arrays.

The physical problem is the advection-diffusion equation of the paper's model
problem (eq. (2), and its 2D conservative form in section 4.3) on the periodic
unit square/interval, discretized on ``n`` points per axis, ``dx = 1/n``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class Problem:
    """Physical description of one periodic advection-diffusion problem.

    ndim      1 or 2
    n         points per axis (grid is n or n x n, x index fastest)
    dx        grid spacing (= 1/n on the unit domain)
    dt        time step
    vel       constant velocity (a_x, a_y); a_y ignored in 1D
    nu        scalar diffusivity, or None when ``nu_field`` is given
    nu_field  per-node diffusivity, shape (n,) or (n, n) [y, x], float64
    states    initial states, shape (N, n_states) with N = n**ndim, DOF
              index j*n + i (x fastest), ensemble index fastest in memory
    vel_faces optional face velocities replacing ``vel``, shape (ndim, ny, n):
              a_x on the east face (i+1/2, j) of every node, a_y on its north
              face (i, j+1/2)
    dy        y spacing when it differs from dx (anisotropic mesh), else None
    """

    ndim: int
    n: int
    dx: float
    dt: float
    vel: Tuple[float, float]
    nu: Optional[float]
    nu_field: Optional[np.ndarray]
    states: np.ndarray
    meta: dict = field(default_factory=dict)
    vel_faces: Optional[np.ndarray] = None
    dy: Optional[float] = None

    @property
    def N(self) -> int:
        return self.n ** self.ndim


def _grid(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) / n


def bump_plus_modes(n: int, seed: int, n_modes: int = 8, kmax: int = 32,
                    sigma: float = 0.05, amp_max: float = 0.1) -> np.ndarray:
    """1D state: Gaussian bump at x=0.5 plus ``n_modes`` random cosines.

    Draw order: wavenumbers (distinct, from 1..kmax), amplitudes U(0, amp_max),
    phases U(0, 2 pi).
    """
    rng = np.random.default_rng(seed)
    k = rng.choice(np.arange(1, kmax + 1), size=n_modes, replace=False)
    a = rng.uniform(0.0, amp_max, size=n_modes)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    x = _grid(n)
    u = np.exp(-((x - 0.5) ** 2) / (2.0 * sigma ** 2))
    for kr, ar, pr in zip(k, a, ph):
        u = u + ar * np.cos(2.0 * np.pi * kr * x + pr)
    return u


def _cos_sum(x: np.ndarray, kx, ky, a, ph) -> np.ndarray:
    """sum_q a_q cos(2 pi (kx_q x + ky_q y) + ph_q) on the grid, shape (n, n)
    [y, x], evaluated as the real part of a rank-(#modes) outer product."""
    ex = np.exp(2j * np.pi * np.outer(kx, x))            # (modes, n) along x
    ey = np.exp(2j * np.pi * np.outer(ky, x))            # (modes, n) along y
    coef = (np.asarray(a) * np.exp(1j * np.asarray(ph)))[:, None]
    return np.real((coef * ey).T @ ex)


def smooth_states_2d(n: int, n_states: int, seed: int, n_modes: int = 16,
                     kmax: int = 8) -> np.ndarray:
    """Ensemble of smooth periodic 2D states, unit RMS each.

    Each state is a sum of ``n_modes`` cosines with integer wavevectors in
    [-kmax, kmax]^2, N(0,1) amplitudes and U(0, 2 pi) phases.  Draw order per
    state: kx, ky, amplitudes, phases.  Returns shape (n*n, n_states).
    """
    rng = np.random.default_rng(seed)
    x = _grid(n)
    out = np.empty((n * n, n_states), dtype=np.float64)
    for s in range(n_states):
        kx = rng.integers(-kmax, kmax + 1, size=n_modes)
        ky = rng.integers(-kmax, kmax + 1, size=n_modes)
        a = rng.standard_normal(n_modes)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
        u = _cos_sum(x, kx, ky, a, ph)
        rms = np.sqrt(np.mean(u * u))
        if rms == 0.0:
            u[:] = 1.0
            rms = 1.0
        out[:, s] = (u / rms).reshape(-1)
    return out


def source_fields_2d(n: int, n_states: int, seed: int, n_modes: int = 4, kmax: int = 4,
                     mean: float = 0.5) -> np.ndarray:
    """Sources g for du/dt = A u + g: per state, ``mean`` plus a unit-RMS sum of
    ``n_modes`` smooth cosines (wavevectors in [-kmax, kmax]^2), drawn like
    smooth_states_2d.  Returns shape (n*n, n_states)."""
    return mean + smooth_states_2d(n, n_states, seed, n_modes=n_modes, kmax=kmax)


def gaussian_members(n: int, length: float, n_states: int, seed: int) -> np.ndarray:
    """Gaussian bumps a exp(-(x - x0)^2) on n cells of [0, length) (the
    Burgers initial datum of section 4.2), per member a ~ U(0.5, 1.5) and
    x0 ~ U(0.2, 0.8) * length (draw order: a, x0).  Shape (n, n_states)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n) * (length / n)
    a = rng.uniform(0.5, 1.5, n_states)
    x0 = rng.uniform(0.2 * length, 0.8 * length, n_states)
    return np.ascontiguousarray(np.column_stack([a[k] * np.exp(-(x - x0[k]) ** 2)
                                                 for k in range(n_states)]))


def gaussian_wavepackets(n: int, length: float, kappa: float, n_states: int,
                         seed: int) -> np.ndarray:
    """Complex Gaussian wave packets exp(-sqrt(kappa) (x - x0)^2 / 2 + i p0 x)
    on the n points x_j = -length/2 + j length/n (the Schroedinger initial
    datum of section 4.1, oscillator ground-state width), per member
    x0 ~ U(-2, 2) and p0 ~ U(-3, 3) (draw order: x0, p0).  Shape
    (n, n_states), complex128."""
    rng = np.random.default_rng(seed)
    x = -0.5 * length + np.arange(n) * (length / n)
    x0 = rng.uniform(-2.0, 2.0, n_states)
    p0 = rng.uniform(-3.0, 3.0, n_states)
    w = np.sqrt(kappa)
    return np.ascontiguousarray(np.column_stack(
        [np.exp(-0.5 * w * (x - x0[k]) ** 2 + 1j * p0[k] * x) for k in range(n_states)]))


def white_noise_states(N: int, n_states: int, seed: int) -> np.ndarray:
    """iid N(0,1) states, shape (N, n_states) (rough stress inputs)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, n_states))


def lognormal_field_2d(n: int, seed: int, median: float = 1e-3,
                       sigma_log: float = 1.0, n_modes: int = 64,
                       kmax: int = 8) -> np.ndarray:
    """Smooth lognormal diffusivity field nu(x, y) of shape (n, n) [y, x].

    z is a sum of ``n_modes`` random cosines (wavevectors in [-kmax, kmax]^2,
    N(0,1) amplitudes, U(0, 2 pi) phases), standardized to mean 0 / std 1;
    nu = median * exp(sigma_log * z).
    """
    rng = np.random.default_rng(seed)
    kx = rng.integers(-kmax, kmax + 1, size=n_modes)
    ky = rng.integers(-kmax, kmax + 1, size=n_modes)
    a = rng.standard_normal(n_modes)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    z = _cos_sum(_grid(n), kx, ky, a, ph)
    z = (z - z.mean()) / z.std()
    return median * np.exp(sigma_log * z)


# ---------------------------------------------------------------------------
# The five workloads.  Sizes may be scaled down (``n``) for parity tests that
# the oracle must finish in seconds; the defaults are the full sizes.
# ---------------------------------------------------------------------------

def workload_1d(n: int = 1024, seed: int = 0, cfl: float = 4.0,
                a: float = 1.0, nu: float = 1e-3) -> Problem:
    """1D periodic advection-diffusion, Gaussian bump + 8 random modes,
    a=1, nu=1e-3, dt = cfl*dx (default 4 dx), 1024 points."""
    dx = 1.0 / n
    u0 = bump_plus_modes(n, seed)
    return Problem(1, n, dx, cfl * dx, (a, 0.0), nu, None, u0.reshape(n, 1),
                   meta={"name": "adv-diff-1d", "seed": seed})


def workload_2d_ensemble(n: int = 256, n_states: int = 64, seed: int = 1,
                         cfl: float = 2.0, vel=(1.0, 0.5),
                         nu: float = 1e-3) -> Problem:
    """2D periodic advection-diffusion, velocity (1, 0.5), nu=1e-3,
    dt = 2 dx, ensemble of smooth unit-RMS states."""
    dx = 1.0 / n
    st = smooth_states_2d(n, n_states, seed)
    return Problem(2, n, dx, cfl * dx, tuple(vel), nu, None, st,
                   meta={"name": "adv-diff-2d-ensemble", "seed": seed})


def workload_2d_mixed(n: int = 512, n_smooth: int = 128, n_noise: int = 0,
                      seed: int = 3) -> Problem:
    """The 2D ensemble operator at 512^2 with smooth states (plus optional
    white-noise stress states appended as extra columns)."""
    dx = 1.0 / n
    st = smooth_states_2d(n, n_smooth, seed)
    if n_noise:
        st = np.concatenate([st, white_noise_states(n * n, n_noise, seed + 1000)],
                            axis=1)
    return Problem(2, n, dx, 2.0 * dx, (1.0, 0.5), 1e-3, None, st,
                   meta={"name": "adv-diff-2d-mixed", "seed": seed})


def workload_2d_variable(n: int = 1024, seed: int = 2,
                         dt_over_dx: float = 0.25) -> Problem:
    """2D periodic diffusion-advection with lognormal nu(x) (median 1e-3,
    sigma_log 1), velocity (1, 0), one smooth state, dt = dx/4."""
    dx = 1.0 / n
    nuf = lognormal_field_2d(n, seed)
    st = smooth_states_2d(n, 1, seed + 100)
    return Problem(2, n, dx, dt_over_dx * dx, (1.0, 0.0), None, nuf, st,
                   meta={"name": "adv-diff-2d-lognormal", "seed": seed})


def vortex_faces(n: int, speed: float = 1.0, height: float = 1.0) -> np.ndarray:
    """Face velocities of a single periodic vortex on [0, 1) x [0, height),
    n x n nodes (dx = 1/n, dy = height/n), from the stream function
    psi(x, y) = (speed height / pi) sin^2(pi x) sin^2(pi y / height) sampled at
    the cell corners (i+1/2, j+1/2):
        a_x(i+1/2, j) = (psi(i+1/2, j+1/2) - psi(i+1/2, j-1/2)) / dy,
        a_y(i, j+1/2) = -(psi(i+1/2, j+1/2) - psi(i-1/2, j+1/2)) / dx,
    so the discrete divergence of the faces vanishes (up to rounding); the
    flow turns about the centre like a solid body near it.  Shape (2, n, n)."""
    dx, dy = 1.0 / n, height / n
    xc = (np.arange(n) + 0.5) * dx
    yc = (np.arange(n) + 0.5) * dy
    psi = (speed * height / np.pi) * np.outer(np.sin(np.pi * yc / height) ** 2,
                                             np.sin(np.pi * xc) ** 2)  # [j, i] at (i+1/2, j+1/2)
    ax = (psi - np.roll(psi, 1, axis=0)) / dy
    ay = -(psi - np.roll(psi, 1, axis=1)) / dx
    return np.ascontiguousarray(np.stack([ax, ay]))


def gaussian_blobs_2d(n: int, n_states: int, seed: int, height: float = 1.0) -> np.ndarray:
    """Periodic Gaussian blobs on [0, 1) x [0, height): per member a centre
    (U(0.2, 0.8), U(0.2, 0.8) height) and a width U(0.04, 0.1) in units of the
    box side (draw order: cx, cy, width).  Shape (n*n, n_states)."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.2, 0.8, n_states)
    cy = rng.uniform(0.2, 0.8, n_states)
    w = rng.uniform(0.04, 0.1, n_states)
    x = np.arange(n) / n
    y = np.arange(n) / n
    out = np.empty((n * n, n_states))
    for k in range(n_states):
        dxp = np.minimum(np.abs(x - cx[k]), 1 - np.abs(x - cx[k]))
        dyp = np.minimum(np.abs(y - cy[k]), 1 - np.abs(y - cy[k]))
        out[:, k] = np.exp(-(dyp[:, None] ** 2 + dxp[None, :] ** 2) / (2 * w[k] ** 2)).reshape(-1)
    return out


def workload_2d_vortex(n: int = 512, n_states: int = 16, seed: int = 5, courant: float = 2.0,
                       nu: float = 1e-4) -> Problem:
    """2D advection-diffusion -div(a c) + nu lap c (eq. ibv2d) with the single
    periodic vortex of ``vortex_faces`` (unit peak speed scale), constant nu,
    dt = courant * dx / max|a|, Gaussian blobs."""
    dx = 1.0 / n
    F = vortex_faces(n)
    amax = float(np.abs(F).max())
    st = gaussian_blobs_2d(n, n_states, seed)
    return Problem(2, n, dx, courant * dx / amax, (0.0, 0.0), nu, None, st,
                   meta={"name": "adv-diff-2d-vortex", "seed": seed, "courant": courant},
                   vel_faces=F)


def workload_2d_columns(n: int = 128, n_states: int = 64, seed: int = 7, aspect: float = 16.0,
                        courant_x: float = 0.8, mu_y: float = 6.0) -> Problem:
    """Anisotropic mesh for column-wise decompositions (section 4.3): n x n
    nodes on [0, 1) x [0, 1/aspect) (dy = dx / aspect), the single vortex of
    ``vortex_faces`` flattened to that height, horizontal Courant number
    ``courant_x`` and vertical diffusion number nu dt / dy^2 = ``mu_y``
    (stiff in the vertical only), Gaussian blobs."""
    dx = 1.0 / n
    dy = dx / aspect
    F = vortex_faces(n, height=1.0 / aspect)
    dt = courant_x * dx / float(np.abs(F[0]).max())
    nu = mu_y * dy * dy / dt
    st = gaussian_blobs_2d(n, n_states, seed, height=1.0 / aspect)
    return Problem(2, n, dx, dt, (0.0, 0.0), nu, None, st,
                   meta={"name": "adv-diff-2d-anisotropic-columns", "seed": seed,
                         "aspect": aspect, "courant_x": courant_x, "mu_y": mu_y},
                   vel_faces=F, dy=dy)


@dataclass
class Request:
    """One served time-stepping request."""

    rid: int
    arrival: float          # seconds since the stream start
    problem: Problem
    n_steps: int


def serving_stream(n_requests: int, seed: int = 4, rate: float = 200.0,
                   sides=(64, 128, 256, 512), dt_mults=(1, 2, 4),
                   steps_range=(20, 200), nu_range=(1e-4, 1e-2),
                   vel=(1.0, 0.5)) -> List[Request]:
    """Poisson arrival stream of independent 2D periodic problems.

    Gaps are exponential with the given mean rate.  Per request, in this draw
    order: gap, grid side, log-uniform nu, dt multiple of dx, step count; the
    initial state comes from ``smooth_states_2d`` with a per-request seed.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(np.asarray(sides)))
        nu = float(np.exp(rng.uniform(np.log(nu_range[0]), np.log(nu_range[1]))))
        mult = int(rng.choice(np.asarray(dt_mults)))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        dx = 1.0 / n
        st = smooth_states_2d(n, 1, seed * 100003 + r, n_modes=8, kmax=4)
        out.append(Request(r, t, Problem(2, n, dx, mult * dx, tuple(vel), nu,
                                         None, st,
                                         meta={"name": "served", "rid": r}),
                           steps))
    return out

"""Buffer (halo) width from an off-diagonal decay bound (oracle; test
infrastructure only).

Section 3 asks that buffers be wide enough for the contribution of nodes
outside M_i to be negligible, and section 2 (Theorem 1, after Iserles)
explains why entries of exp(dt A) decay away from the diagonal at a rate set
by C and mu.  The printed form of Theorem 1 is garbled, so this module uses a
bound proved directly for the stencil operator, in the same Taylor-tail
family:

Let dt*A_M = w0 I + N on the box (w0 the diagonal, N the off-diagonal part).
The LEM error at the core after one step is, by Duhamel's formula applied to
the local problem (4) with the outside values as a source entering at the box
edge, an integral over s in [0, 1] of exp(s dt A_M) applied to the coupling
w_side * u_outside(s).  Entrywise |exp(s dt A_M)| <= exp(s w0) exp(s |N|),
and the entries of exp(s |N|) are bounded, for any r > 0, by Cauchy's
estimate on its generating function.  Summing over all edge nodes of one side
(all perpendicular offsets) and integrating in s gives, relative to the
largest value of the solution over the step,

    eps(h) = G * sum_sides |w_s| * min_{r>0} [(exp(phi_s(r)) - 1)/phi_s(r)] r^-h
    phi_s(r) = w0 + P_s + |w_s| r + |w_sbar| / r

where w_s couples the box edge to the outside across side s, w_sbar is the
opposite weight on the same axis, P_s the sum of |w| along the other axis,
and h is the distance from the edge node to the nearest core node (the halo
width).  G = exp(max(0, max_i (w0_i + sum |w|_i))) bounds the growth of the
infinity norm of the global solution over one step (G = 1 when all weights
are non-negative, i.e. mu >= C/2).  For a spatially varying operator the
block maximum of each |w| and the largest (least negative) w0 are used.
The objective is convex in log r; it is minimized in log space.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import minimize_scalar


def _log_expm1_over(phi: float) -> float:
    """log((e^phi - 1)/phi), stable for every real phi (value 0 at phi=0)."""
    if abs(phi) < 1e-8:
        return phi / 2.0
    if phi > 0:
        return phi + math.log1p(-math.exp(-phi)) - math.log(phi)
    return math.log(-math.expm1(phi)) - math.log(-phi)


def side_log_bound(ws: float, wsbar: float, w0: float, P: float, h: int) -> float:
    """log of |w_s| * min_r [(e^phi - 1)/phi] r^-h for one side; -inf if w_s = 0."""
    b = abs(ws)
    c = abs(wsbar)
    if b == 0.0:
        return -math.inf
    a = w0 + P

    def f(t):
        return _log_expm1_over(a + b * math.exp(t) + c * math.exp(-t)) - h * t

    res = minimize_scalar(f, bounds=(-40.0, 40.0), method="bounded",
                          options={"xatol": 1e-11, "maxiter": 2000})
    return math.log(b) + float(res.fun)


def block_coefficients(W, box, ndim: int):
    """Block maxima (|wW|, |wE|, |wS|, |wN|) and largest w0 over the box M_i."""
    from .partition import gather_map
    G = gather_map(box, ndim, W.n)
    f = lambda a: np.abs(a.reshape(-1)[G]).max()
    return (f(W.wW), f(W.wE), f(W.wS), f(W.wN), W.w0.reshape(-1)[G].max())


def growth_factor(W) -> float:
    s = W.w0 + np.abs(W.wW) + np.abs(W.wE) + np.abs(W.wS) + np.abs(W.wN)
    return math.exp(max(0.0, float(s.max())))


def eps(coeffs, h: int, ndim: int, G: float = 1.0, cut_y: bool = True) -> float:
    """The bound eps(h) for one block, given its coefficient maxima.  A box
    that spans the whole y axis (column-wise decomposition, cut_y False) has
    no buffer edge across y, so only its x sides contribute."""
    aW, aE, aS, aN, w0 = coeffs
    terms = [side_log_bound(aW, aE, w0, aS + aN, h),
             side_log_bound(aE, aW, w0, aS + aN, h)]
    if ndim == 2 and cut_y:
        terms += [side_log_bound(aS, aN, w0, aW + aE, h),
                  side_log_bound(aN, aS, w0, aW + aE, h)]
    return G * sum(math.exp(t) for t in terms if t > -math.inf)


def halo_width(coeffs, ndim: int, tol: float, h_min: int, h_max: int,
               G: float = 1.0, cut_y: bool = True):
    """Smallest h >= h_min with eps(h) <= tol, clamped at h_max.

    Returns (h, clamped) where clamped is True when even h_max misses tol.
    """
    for h in range(h_min, h_max + 1):
        if eps(coeffs, h, ndim, G, cut_y) <= tol:
            return h, False
    return h_max, True


def accepts(coeffs, ndim: int, tol: float, h_min: int, h: int,
            G: float = 1.0, rel: float = 1e-12, cut_y: bool = True) -> bool:
    """Tie-tolerant check that h is the halo-rule answer: eps(h) <= tol and
    either h = h_min or eps(h - 1) > tol (both up to a relative ``rel``)."""
    if eps(coeffs, h, ndim, G, cut_y) > tol * (1.0 + rel):
        return False
    return h == h_min or eps(coeffs, h - 1, ndim, G, cut_y) > tol * (1.0 - rel)

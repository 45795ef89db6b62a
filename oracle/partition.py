"""Overlapping decomposition of the periodic grid (oracle; test infrastructure).

Section 3 decomposes the mesh into regions M_i = D_i u B_i: the cores D_i are
disjoint and cover the mesh, and each buffer B_i surrounds its core.  Here a
block is a rectangular core of cx x cy points with origin (ox, oy) and a
buffer of h points on every side (along x only in 1D); the local box M_i is
the core widened by h per side, taken modulo n on the periodic grid.

Local numbering inside a box is row-major with x fastest:
    l = ly * Lx + lx,  Lx = cx + 2h,  Ly = cy + 2h (1 in 1D)
and the gather map sends local l to the global DOF
    G[l] = ((oy - h + ly) mod n) * n + ((ox - h + lx) mod n)     (2D)
    G[l] = (ox - h + lx) mod n                                   (1D).
Core rows are the local points with lx, ly in [h, h + c); the scatter map
sends core row r = ry * cx + rx to the global DOF (oy + ry) * n + (ox + rx).

A box must not reach itself through the wrap (Lx < n, Ly < n) unless it is
the whole domain (the D = 1 case: core = grid, h = 0), where the local
operator keeps the periodic coupling and LEM equals the global method.

A core that spans a whole axis has no buffer along that axis and keeps the
periodic coupling along it: the column-wise decompositions of section 4.3
(cores of c x n points, buffers of h only across the columns).  Then the
principal submatrix on the box already contains the wrap-around couplings of
that axis, because both of their end points belong to the box.
"""
from __future__ import annotations

from typing import List, NamedTuple

import numpy as np


class Box(NamedTuple):
    ox: int
    oy: int
    cx: int
    cy: int
    h: int


def box_halos(b: Box, ndim: int, n: int | None = None):
    """Buffer widths (hx, hy): none along an axis the core spans whole."""
    hx = 0 if (n is not None and b.cx == n) else b.h
    if ndim == 1:
        return hx, 0
    hy = 0 if (n is not None and b.cy == n) else b.h
    return hx, hy


def box_dims(b: Box, ndim: int, n: int | None = None):
    hx, hy = box_halos(b, ndim, n)
    Lx = b.cx + 2 * hx
    Ly = (b.cy + 2 * hy) if ndim == 2 else 1
    return Lx, Ly


def uniform_boxes(ndim: int, n: int, c: int, h: int) -> List[Box]:
    """Cores of side c tiling the grid; block order is y-major, then x."""
    if n % c:
        raise ValueError("core side must divide the grid side")
    nb = n // c
    if ndim == 1:
        return [Box(bx * c, 0, c, 1, h) for bx in range(nb)]
    return [Box(bx * c, by * c, c, c, h) for by in range(nb) for bx in range(nb)]


def column_boxes(n: int, c: int, h: int) -> List[Box]:
    """Column-wise 2D decomposition: cores of c x n points (whole columns),
    buffers of h points across the columns only."""
    if n % c:
        raise ValueError("core width must divide the grid side")
    return [Box(bx * c, 0, c, n, h) for bx in range(n // c)]


def validate(b: Box, ndim: int, n: int) -> None:
    Lx, Ly = box_dims(b, ndim, n)
    whole = (b.cx == n and b.h == 0 and (ndim == 1 or b.cy == n))
    if whole:
        return
    if (b.cx < n and Lx >= n) or (ndim == 2 and b.cy < n and Ly >= n):
        raise ValueError("box reaches itself through the periodic wrap")


def gather_map(b: Box, ndim: int, n: int) -> np.ndarray:
    validate(b, ndim, n)
    Lx, Ly = box_dims(b, ndim, n)
    hx, hy = box_halos(b, ndim, n)
    lx = np.arange(Lx)
    gx = (b.ox - hx + lx) % n
    if ndim == 1:
        return gx.astype(np.int64)
    ly = np.arange(Ly)
    gy = (b.oy - hy + ly) % n
    return (gy[:, None] * n + gx[None, :]).reshape(-1).astype(np.int64)


def core_local_rows(b: Box, ndim: int, n: int | None = None) -> np.ndarray:
    Lx, _ = box_dims(b, ndim, n)
    hx, hy = box_halos(b, ndim, n)
    rx = np.arange(b.cx) + hx
    if ndim == 1:
        return rx.astype(np.int64)
    ry = np.arange(b.cy) + hy
    return (ry[:, None] * Lx + rx[None, :]).reshape(-1).astype(np.int64)


def scatter_map(b: Box, ndim: int, n: int) -> np.ndarray:
    rx = b.ox + np.arange(b.cx)
    if ndim == 1:
        return rx.astype(np.int64)
    ry = b.oy + np.arange(b.cy)
    return (ry[:, None] * n + rx[None, :]).reshape(-1).astype(np.int64)


def check_tiling(boxes: List[Box], ndim: int, n: int) -> None:
    """The cores must be disjoint and cover every DOF exactly once."""
    N = n ** ndim
    hits = np.zeros(N, dtype=np.int64)
    for b in boxes:
        if b.ox < 0 or b.oy < 0 or b.ox + b.cx > n or (ndim == 2 and b.oy + b.cy > n):
            raise ValueError("core outside the grid")
        if ndim == 1 and (b.oy != 0 or b.cy != 1):
            raise ValueError("1D core must have oy = 0, cy = 1")
        np.add.at(hits, scatter_map(b, ndim, n), 1)
    if not np.all(hits == 1):
        raise ValueError("cores do not tile the grid exactly once")


def all_maps(boxes: List[Box], ndim: int, n: int):
    """Concatenated gather and scatter maps with their per-block offsets."""
    G = [gather_map(b, ndim, n) for b in boxes]
    S = [scatter_map(b, ndim, n) for b in boxes]
    goff = np.concatenate([[0], np.cumsum([len(g) for g in G])])
    soff = np.concatenate([[0], np.cumsum([len(s) for s in S])])
    return np.concatenate(G), goff, np.concatenate(S), soff

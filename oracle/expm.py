"""Dense matrix exponential by Pade [13/13] with scaling and squaring
(oracle; test infrastructure only).

The paper computes its stored local exponential (phi) matrices "by the scaling
and squaring algorithm and Pade approximation" (sections 3 and 4, citing Moler
and Van Loan).  This is the degree-13 variant of N. J. Higham, "The scaling
and squaring method for the matrix exponential revisited", SIAM J. Matrix
Anal. Appl. 26 (2005): scale A by 2^-s so that ||A/2^s||_1 <= theta_13, form
the diagonal Pade approximant r_13 = q(A)^{-1} p(A) with p(A) = V + U,
q(A) = V - U (U the odd part, V the even part), and square s times.

The Pade coefficients are computed exactly from their closed form
    c_j = (2m - j)! m! / ((2m)! j! (m - j)!),  m = 13,
then scaled so that the leading one is 1 (the integer table of Higham's paper).
A library matrix product and a library LU solve are the only primitives.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

PADE_M = 13
#: Higham (2005), Table 2.3: largest ||A||_1 for which r_13 meets unit roundoff.
THETA_13 = 5.371920351148152


def pade_coefficients(m: int = PADE_M):
    """Exact Pade [m/m] numerator coefficients, scaled so c_m = 1."""
    c = [Fraction(math.factorial(2 * m - j) * math.factorial(m),
                  math.factorial(2 * m) * math.factorial(j) * math.factorial(m - j))
         for j in range(m + 1)]
    return [x / c[m] for x in c]


_B = [float(x) for x in pade_coefficients()]


def squarings(A: np.ndarray) -> int:
    nrm = np.linalg.norm(A, 1)
    if nrm <= THETA_13:
        return 0
    return int(math.ceil(math.log2(nrm / THETA_13)))


def expm(A: np.ndarray) -> np.ndarray:
    """exp(A) for a dense square float64 (or complex) matrix."""
    A = np.asarray(A)
    n = A.shape[0]
    if n == 0:
        return A.copy()
    s = squarings(A)
    A = A / (2.0 ** s)
    b = _B
    I = np.eye(n, dtype=A.dtype)
    A2 = A @ A
    A4 = A2 @ A2
    A6 = A4 @ A2
    U = A @ (A6 @ (b[13] * A6 + b[11] * A4 + b[9] * A2)
             + b[7] * A6 + b[5] * A4 + b[3] * A2 + b[1] * I)
    V = (A6 @ (b[12] * A6 + b[10] * A4 + b[8] * A2)
         + b[6] * A6 + b[4] * A4 + b[2] * A2 + b[0] * I)
    R = np.linalg.solve(V - U, V + U)
    for _ in range(s):
        R = R @ R
    return R

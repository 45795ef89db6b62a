"""Error metrics (oracle; test infrastructure): relative l2 (Frobenius over
all DOFs and ensemble members) and relative l-infinity, as the paper reports
relative l2 and l-infinity errors in section 4."""
from __future__ import annotations

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_linf(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (nb if nb > 0 else 1.0)) if a.size else 0.0

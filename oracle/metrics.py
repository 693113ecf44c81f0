"""Error measures, accumulated in FP64."""
from __future__ import annotations

import numpy as np


def rel_l2(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = float(np.linalg.norm(ref))
    return float(np.linalg.norm(x - ref)) / den if den > 0 else float(np.linalg.norm(x))


def rel_max(x, ref) -> float:
    """max|x - ref| / max|ref|."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = float(np.abs(ref).max()) if ref.size else 0.0
    num = float(np.abs(x - ref).max()) if ref.size else 0.0
    return num / den if den > 0 else num

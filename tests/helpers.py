"""Helpers shared by the tests (error norms, golden-file parsing)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rmse_closed(a: np.ndarray, b: np.ndarray) -> float:
    """RMSE over the nodes j = 0..n of the closed periodic domain, i.e. with
    the periodic end nodes counted twice (the node set that reproduces the
    RMSEs printed in Tables 2 and 3)."""
    idx = tuple(np.r_[np.arange(s), 0] for s in a.shape)
    diff = a[np.ix_(*idx)] - b[np.ix_(*idx)]
    return float(np.sqrt(np.mean(diff * diff)))


def rmse(a: np.ndarray, b: np.ndarray) -> float:
    diff = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.mean(diff * diff)))


def max_rel(a, b) -> float:
    """max |a - b| / max |b| (norm-wise relative error)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b))) / (den if den > 0 else 1.0)


def read_table(name: str):
    """Rows of a golden table: (eps, variable, [rmse or None per level], cr)."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            eps = float(parts[0])
            var = parts[1]
            vals = [None if p == "x" else float(p) for p in parts[2:6]]
            rows.append((eps, var, vals, float(parts[6])))
    return rows


def read_table4():
    """Rows of golden/table4.txt: (eps, t, variable, [rmse or None per level], cr)."""
    rows = []
    with open(os.path.join(GOLDEN, "table4.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            p = line.split()
            rows.append((float(p[0]), float(p[1]), p[2],
                         [None if v == "x" else float(v) for v in p[3:7]], float(p[7])))
    return rows

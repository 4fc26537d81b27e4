"""Pre-screening of the base features before expansion (test infrastructure
only): FP64 NumPy reference of the two rankings the paper offers for problems
with many primary features (Sec. 3.1, eq. mi-exact; the initial_screening
option of Sec. 3.3, methods "mi" and "spearman").

Mutual information (eq. mi-exact) is the integral of
p(x, y) log(p(x, y) / (p(x) p(y))); the paper approximates it with kernel
density estimation without fixing the estimator.  Reading taken here: both
variables standardised to zero mean and unit population sd; Gaussian kernels
with Silverman's rule-of-thumb bandwidth h_k = (4 / (k + 2))^(1 / (k + 4))
n^(-1 / (k + 4)) for k = 1 (each marginal) and k = 2 (the joint, product
kernel); the integral replaced by the sample mean over the n observations of
log(p(x_s, y_s) / (p(x_s) p(y_s))) with each density the kernel average over
all n observations (resubstitution).

Spearman: |Pearson correlation| of the ranks, ties given their average rank.

Selection: the best ceil(q d) features by (score desc, index asc), q the
quantile the option names (e.g. 0.01 keeps the top 1%).
"""
from __future__ import annotations

import math

import numpy as np


def bandwidth(n: int, k: int) -> float:
    return (4.0 / (k + 2.0)) ** (1.0 / (k + 4.0)) * n ** (-1.0 / (k + 4.0))


def _standardise(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    sd = math.sqrt(float(np.mean((v - v.mean()) ** 2)))
    return (v - v.mean()) / sd if sd > 0.0 else np.zeros_like(v)


def mutual_information(x: np.ndarray, y: np.ndarray) -> float:
    """KDE estimate of eq. mi-exact for one feature (0 for a constant one)."""
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    n = x.size
    if np.all(x == x[0]) or np.all(y == y[0]):
        return 0.0
    a, b = _standardise(x), _standardise(y)
    h1, h2 = bandwidth(n, 1), bandwidth(n, 2)
    dx = a[:, None] - a[None, :]
    dy = b[:, None] - b[None, :]
    # densities at each observation, kernel average over all observations
    px = np.exp(-dx * dx / (2.0 * h1 * h1)).mean(axis=1) / (math.sqrt(2.0 * math.pi) * h1)
    py = np.exp(-dy * dy / (2.0 * h1 * h1)).mean(axis=1) / (math.sqrt(2.0 * math.pi) * h1)
    pxy = np.exp(-(dx * dx + dy * dy) / (2.0 * h2 * h2)).mean(axis=1) / (2.0 * math.pi * h2 * h2)
    return float(np.mean(np.log(pxy) - np.log(px) - np.log(py)))


def ranks(v: np.ndarray) -> np.ndarray:
    """1-based ranks, ties sharing their average rank (written as loops over the
    sorted order, independent of any library ranking routine)."""
    v = np.asarray(v, dtype=np.float64)
    order = sorted(range(v.size), key=lambda i: (v[i], i))
    r = np.empty(v.size)
    i = 0
    while i < v.size:
        j = i
        while j + 1 < v.size and v[order[j + 1]] == v[order[i]]:
            j += 1
        avg = (i + j) / 2.0 + 1.0
        for q in range(i, j + 1):
            r[order[q]] = avg
        i = j + 1
    return r


def spearman(x: np.ndarray, y: np.ndarray) -> float:
    """|Spearman rank correlation| (0 for a constant feature)."""
    rx, ry = ranks(x), ranks(y)
    a, b = rx - rx.mean(), ry - ry.mean()
    d = math.sqrt(float(a @ a) * float(b @ b))
    return abs(float(a @ b)) / d if d > 0.0 else 0.0


def scores(X: np.ndarray, y: np.ndarray, method: str) -> np.ndarray:
    fn = {"mi": mutual_information, "spearman": spearman}[method]
    return np.array([fn(X[:, i], y) for i in range(X.shape[1])])


def select(sc: np.ndarray, quantile: float) -> np.ndarray:
    """Indices of the best ceil(quantile d) features, by (score desc, index asc)."""
    d = sc.size
    keep = max(1, min(d, int(math.ceil(quantile * d - 1e-12))))
    order = sorted(range(d), key=lambda i: (-sc[i], i))
    return np.array(order[:keep], dtype=np.int64)

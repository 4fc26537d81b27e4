"""Pins of the pre-screening reference (oracle/prescreen.py): Sec. 3.1,
eq. mi-exact (mutual information by kernel density estimation) and the
Spearman alternative of Sec. 3.3, against closed forms, invariances and
independent library routines."""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import prescreen as P


def test_bandwidth_is_silvermans_rule():
    # the univariate rule's familiar constant (4/3)^(1/5) = 1.0592..., and n^(-1/6) in two dimensions
    assert math.isclose(P.bandwidth(1, 1), 1.0592238410488122, rel_tol=1e-15)
    assert math.isclose(P.bandwidth(64, 2), 0.5, rel_tol=1e-15)


def test_ranks_and_spearman_against_scipy():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 12, 300).astype(float)          # many ties
    y = x ** 2 + rng.normal(0, 20, 300)
    assert np.array_equal(P.ranks(x), scipy.stats.rankdata(x, method="average"))
    assert math.isclose(P.spearman(x, y), abs(scipy.stats.spearmanr(x, y).statistic), rel_tol=1e-12)
    z = rng.lognormal(0, 1, 500)
    w = -np.log(z) + 0.1 * rng.normal(size=500)
    assert math.isclose(P.spearman(z, w), abs(scipy.stats.spearmanr(z, w).statistic), rel_tol=1e-12)
    # a monotone transform of either variable leaves it unchanged; a constant gives 0
    assert math.isclose(P.spearman(np.exp(x / 5), y), P.spearman(x, y), rel_tol=1e-15)
    assert P.spearman(np.full(300, 2.0), y) == 0.0


def test_mi_gaussian_closed_form_and_monotone():
    """For a bivariate Gaussian with correlation rho, MI = -log(1 - rho^2) / 2;
    the estimate at n = 2000 is within 0.03 + 10% of it for rho <= 0.8 (a
    small positive bias from the smoothing), near 0 without dependence, and it
    increases with rho."""
    rng = np.random.default_rng(0)
    n = 2000
    z = rng.normal(size=(n, 2))
    prev = -1.0
    for rho in (0.0, 0.3, 0.5, 0.8, 0.95):
        y = rho * z[:, 0] + math.sqrt(1 - rho * rho) * z[:, 1]
        mi = P.mutual_information(z[:, 0], y)
        exact = -0.5 * math.log(1 - rho * rho)
        if rho == 0.0:
            assert 0.0 <= mi < 0.03
        elif rho <= 0.8:
            assert abs(mi - exact) <= 0.03 + 0.1 * exact, (rho, mi, exact)
        assert mi > prev
        prev = mi


def test_mi_invariances():
    rng = np.random.default_rng(5)
    x = rng.lognormal(0, 0.5, 700)
    y = np.sin(2 * x) + 0.1 * rng.normal(size=700)
    m = P.mutual_information(x, y)
    assert math.isclose(P.mutual_information(y, x), m, rel_tol=1e-12)            # symmetric
    assert math.isclose(P.mutual_information(3 * x - 7, y), m, rel_tol=1e-12)    # affine in x
    assert math.isclose(P.mutual_information(-x, 0.5 * y + 2), m, rel_tol=1e-12)
    assert math.isclose(P.mutual_information(x[::-1], y[::-1]), m, rel_tol=1e-12)   # sample order
    assert P.mutual_information(np.full(700, 1.5), y) == 0.0
    # a nonlinear dependence that Pearson misses is seen by MI
    u = rng.uniform(-1, 1, 700)
    v = u * u + 0.02 * rng.normal(size=700)
    assert abs(np.corrcoef(u, v)[0, 1]) < 0.15 and P.mutual_information(u, v) > 0.5


@pytest.mark.parametrize("q,d,keep", [(0.01, 1445, 15), (0.5, 10, 5), (0.001, 10, 1), (1.0, 7, 7)])
def test_select_count_and_order(q, d, keep):
    rng = np.random.default_rng(d)
    sc = rng.uniform(0, 1, d)
    sc[3] = sc[5] = sc.max() + 1.0                                             # a tie: index order
    sel = P.select(sc, q)
    assert len(sel) == keep
    assert sel[0] == 3 and (keep == 1 or sel[1] == 5)
    assert np.all(np.diff(sc[sel]) <= 0)

"""Pins of the oracle's weighted forms (Sec. 2.4: whitening by W = Sigma^(-1/2)
for noise with a known diagonal covariance, sample weights w_s = 1 / sigma_s^2).

The reading: the model keeps its intercept, so whitening multiplies the
intercept column by W as well as the features and the target; least squares
in the whitened space is then weighted least squares, and the screening
correlation of a whitened feature with the whitened residual (after the
whitened intercept is projected out) is the weighted Pearson correlation.

Each pin ties the weighted code to something other than itself:
  * integer weights equal the unweighted method on data where sample s is
    repeated w_s times (a dropped or misplaced weight anywhere changes it);
  * the weighted SSE of a tuple equals numpy's least squares on rows scaled
    by sqrt(w_s), intercept column included (the whitening itself);
  * the weighted score equals the cosine of the sqrt(w)-scaled vectors after
    projecting out sqrt(w) (the whitened intercept);
  * constant weights leave scores and the chosen models unchanged.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O

UN, BI = ["sq", "sqrt", "inv"], ["add", "sub", "mul", "div"]


def _problem(seed, n=24, d=3):
    rng = np.random.default_rng(seed)
    X = rng.lognormal(0.0, 0.5, size=(n, d))
    sig = rng.uniform(0.05, 1.0, n)
    y = 2.0 * X[:, 0] * X[:, 1] - X[:, 2] ** 2 + sig * rng.normal(size=n)
    w = np.round(1.0 / sig ** 2 / 4.0).clip(1, 6)           # small integer weights
    return X, y, w


def _repeat(X, y, w):
    idx = np.repeat(np.arange(len(y)), w.astype(int))
    return X[idx], y[idx]


def test_weighted_corr_equals_replicated_samples():
    X, y, w = _problem(1)
    Xr, yr = _repeat(X, y, w)
    for j in range(X.shape[1]):
        a = O.abs_corr(X[:, j], y, w)
        b = O.abs_corr(Xr[:, j], yr)
        assert math.isclose(a, b, rel_tol=1e-13), (j, a, b)


def test_weighted_corr_is_the_whitened_cosine():
    rng = np.random.default_rng(2)
    n = 40
    f, r = rng.normal(size=n), rng.normal(size=n)
    w = rng.uniform(0.1, 5.0, n)
    q = np.sqrt(w)
    P = np.eye(n) - np.outer(q, q) / (q @ q)               # projects out the whitened intercept
    a, b = P @ (q * f), P @ (q * r)
    cos = abs(a @ b) / math.sqrt((a @ a) * (b @ b))
    assert math.isclose(O.abs_corr(f, r, w), cos, rel_tol=1e-12)
    # unequal weights change it; constant weights do not
    assert abs(O.abs_corr(f, r, w) - O.abs_corr(f, r)) > 1e-3
    assert math.isclose(O.abs_corr(f, r, np.full(n, 7.5)), O.abs_corr(f, r), rel_tol=1e-13)


def test_weighted_screen_equals_replicated_samples():
    X, y, w = _problem(3)
    Xr, yr = _repeat(X, y, w)
    sp = O.Space(3, UN, BI, 2, True)
    a = sp.score_range(X, y, 0, sp.total, w=w)
    b = sp.score_range(Xr, yr, 0, sp.total)
    ok = np.isfinite(a)
    assert np.array_equal(ok, np.isfinite(b))
    assert np.max(np.abs(a[ok] - b[ok])) <= 1e-11
    ia, sa = sp.sis(X, y, 50, w=w)
    ib, sb = sp.sis(Xr, yr, 50)
    # identical lists up to the order of scores equal to rounding
    assert np.max(np.abs(sa - sb)) <= 1e-11
    assert set(ia[sa > sa[-1] + 1e-9].tolist()) == set(ib[sb > sb[-1] + 1e-9].tolist())


def test_weighted_l0_is_whitened_least_squares():
    rng = np.random.default_rng(4)
    n, m = 30, 7
    F = rng.lognormal(0.0, 0.6, size=(n, m))
    sig = rng.uniform(0.05, 1.0, n)
    w = 1.0 / sig ** 2
    y = 1.0 + 3.0 * F[:, 2] - 2.0 * F[:, 5] + 0.5 * F[:, 1] + sig * rng.normal(size=n)
    q = np.sqrt(w)
    for D in (1, 2, 3):
        best, best_sse = None, np.inf
        for T in itertools.combinations(range(m), D):
            A = np.column_stack([q] + [q * F[:, t] for t in T])        # whitened intercept + features
            coef, *_ = np.linalg.lstsq(A, q * y, rcond=None)
            sse = float(np.sum((q * y - A @ coef) ** 2))
            if best is None or sse < best_sse - 1e-12 * best_sse:
                best, best_sse, best_coef = T, sse, coef
        res = O.l0(F, y, D, w=w)
        assert tuple(res.best.tolist()) == best
        assert math.isclose(res.sse, best_sse, rel_tol=1e-9)
        assert np.allclose(res.coef, best_coef, rtol=1e-8, atol=1e-10)
        assert res.n_tuples == math.comb(m, D)
    # the unweighted search picks a different model on this heteroscedastic problem at D = 3 or
    # reports a different SSE: the weights reach the search
    assert not math.isclose(O.l0(F, y, 3).sse, O.l0(F, y, 3, w=w).sse, rel_tol=1e-6)


def test_weighted_l0_equals_replicated_samples():
    rng = np.random.default_rng(5)
    n, m = 20, 6
    F = rng.lognormal(0.0, 0.6, size=(n, m))
    y = F[:, 0] - 2 * F[:, 3] + rng.normal(0, 0.3, n)
    w = rng.integers(1, 5, n).astype(float)
    idx = np.repeat(np.arange(n), w.astype(int))
    for D in (1, 2, 3):
        a, b = O.l0(F, y, D, w=w), O.l0(F[idx], y[idx], D)
        assert np.array_equal(a.best, b.best)
        assert math.isclose(a.sse, b.sse, rel_tol=1e-11)
        assert np.allclose(a.coef, b.coef, rtol=1e-10, atol=1e-12)


def test_weighted_fit_equals_replicated_samples():
    X, y, w = _problem(6, n=20)
    Xr, yr = _repeat(X, y, w)
    a = O.fit(X, y, ["sq", "sqrt"], ["add", "mul", "div"], 2, False, 5, 2, w=w)
    b = O.fit(Xr, yr, ["sq", "sqrt"], ["add", "mul", "div"], 2, False, 5, 2)
    assert len(a) == len(b) == 2
    for sa, sb in zip(a, b):
        assert sorted(sa.sub_ids.tolist()) == sorted(sb.sub_ids.tolist())
        assert list(sa.best_ids) == list(sb.best_ids)
        assert math.isclose(sa.sse, sb.sse, rel_tol=1e-9)
        assert math.isclose(sa.r2, sb.r2, rel_tol=1e-9)
        assert math.isclose(sa.rmse, sb.rmse, rel_tol=1e-9)


def test_constant_weights_change_nothing_but_the_sse_scale():
    X, y, _ = _problem(7, n=22)
    a = O.fit(X, y, ["sq"], ["add", "mul"], 2, False, 4, 2)
    b = O.fit(X, y, ["sq"], ["add", "mul"], 2, False, 4, 2, w=np.full(len(y), 3.0))
    for sa, sb in zip(a, b):
        assert list(sa.best_ids) == list(sb.best_ids)
        assert math.isclose(sb.sse, 3.0 * sa.sse, rel_tol=1e-10)
        assert math.isclose(sa.r2, sb.r2, rel_tol=1e-10)


def test_weights_are_validated():
    f = np.arange(5.0)
    with pytest.raises(ValueError):
        O.abs_corr(f, f, np.array([1.0, 2.0, 0.0, 1.0, 1.0]))
    with pytest.raises(ValueError):
        O.abs_corr(f, f, np.ones(4))

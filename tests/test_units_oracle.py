"""Pins of the oracle's dimensional analysis (Sec. 2.1: sums and differences
only of features with the same units; Sec. 3.3: the dimensionality option,
one unit string per base feature).  Readings: every distinct unit string is a
base dimension, "" or "1" a dimensionless feature; products and quotients
add and subtract exponents, x^2, x^3, sqrt(x), 1/x scale them by 2, 3, 1/2,
-1, and exp, exp(-x), ln and sin take a dimensionless argument (a feature
breaking a rule is not generated: it is invalid).

The pins: the paper's own five-feature example (features 3 and 5 share
units) counted in closed form; hand-derived units of named features; and the
NumPy brute force, whose units are exact fractions computed on its own
expression enumeration, agreeing id by id (validity and exponents) and on a
whole fit."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute as B
from oracle import oracle as O

BI = ["add", "sub", "mul", "div"]


def _x(seed, n, d, lo=0.5, hi=5.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=(n, d))


def test_paper_dimensionality_example_counts():
    """Five features, 1-4 with distinct units and 5 sharing 3's: at level 1
    a sum or difference exists only for the pair (3, 5); products and both
    quotients exist for all ten pairs."""
    units = ["u1", "u2", "u3", "u4", "u3"]
    X = _x(1, 40, 5)
    sp = O.Space(5, [], BI, 1, False, units)
    plain = O.Space(5, [], BI, 1, False)
    _, valid = sp.eval(X, range(sp.total))
    _, valid_plain = plain.eval(X, range(plain.total))
    assert valid_plain.all()
    counts = {"add": 0, "sub": 0, "mul": 0, "div": 0}
    pairs = {}
    for fid in range(5, sp.total):
        op, l, r = sp.decode(fid)
        name = BI[op]
        counts[name] += int(valid[fid - 0])
        if valid[fid] and name in ("add", "sub"):
            pairs[name] = tuple(sorted((l, r)))
    assert counts == {"add": 1, "sub": 1, "mul": 10, "div": 20}
    assert pairs == {"add": (2, 4), "sub": (2, 4)}


def test_hand_derived_units():
    # x0: length, x1: time, x2: length, x3: dimensionless
    units = ["m", "s", "m", "1"]
    sp = O.Space(4, ["sq", "sqrt", "inv", "exp"], BI, 2, False, units)
    feats, bu = B.enumerate_space_units(_x(2, 30, 4), ["sq", "sqrt", "inv", "exp"], BI, 2, False, units)
    by_expr = {e: i for i, (e, _, _) in enumerate(feats)}
    m, s_ = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    want = {
        "(x0/x1)": (True, m - s_),                 # speed
        "(x2-x0)": (True, m),
        "(x1+x0)": (False, None),                  # length + time
        "sqrt(x0)": (True, 0.5 * m),
        "((x0)^2/x1)": (True, 2 * m - s_),
        "(sqrt(x2)*sqrt(x0))": (True, m),          # sqrt(m) sqrt(m) = m
        "exp(x3)": (True, 0 * m),
        "exp(x0)": (False, None),                  # exp of a length
        "(exp(x3)*x1)": (True, s_),
        "1/((x0/x2))": (True, 0 * m),              # a dimensionless ratio
        "exp((x0/x2))": (True, 0 * m),             # exp of a dimensionless ratio
        "exp((x0/x1))": (False, None),             # exp of a speed
    }
    for expr, w in want.items():
        assert expr in by_expr, expr
        ok, u = sp.units(by_expr[expr])
        assert ok == w[0], expr
        if ok:
            assert np.array_equal(u, w[1]), (expr, u)
            assert bu[by_expr[expr]] == {k: Fraction(v) for k, v in zip(["m", "s"], w[1]) if v != 0}


@pytest.mark.parametrize("units,rect", [(["a", "b", "a"], True), (["a", "1", "b"], True), (["1", "1", "1"], False),
                                        (["x", "x", "x"], True)])
def test_validity_and_units_match_brute_force(units, rect):
    un = ["sq", "cube", "sqrt", "inv", "exp", "log", "sin"]
    X = _x(3, 25, 3)
    sp = O.Space(3, un, BI, 2, rect, units)
    feats, bu = B.enumerate_space_units(X, un, BI, 2, rect, units)
    assert sp.total == len(feats)
    _, valid = sp.eval(X, range(sp.total))
    names = []
    for u in units:
        if u not in ("", "1") and u not in names:
            names.append(u)
    for fid in range(sp.total):
        assert valid[fid] == feats[fid][2], (fid, feats[fid][0])
        ok, u = sp.units(fid)
        assert ok == (bu[fid] is not None), (fid, feats[fid][0])
        if ok:
            want = np.array([float(bu[fid].get(k, 0)) for k in names])
            assert np.array_equal(u, want), (fid, feats[fid][0], u, want)
    if units == ["1", "1", "1"]:
        # all dimensionless: the same space as without units
        _, v0 = O.Space(3, un, BI, 2, rect).eval(X, range(sp.total))
        assert np.array_equal(valid, v0)
    # a rule that removes something: not every valid plain feature is physical
    _, v0 = O.Space(3, un, BI, 2, rect).eval(X, range(sp.total))
    assert valid.sum() <= v0.sum()


def test_fit_with_units_matches_brute_force():
    rng = np.random.default_rng(8)
    X = rng.uniform(0.5, 4.0, size=(30, 4))
    units = ["m", "s", "m", "1"]
    # a physical target: (x0 + x2) / x1 plus a dimensionless term's effect
    y = (X[:, 0] + X[:, 2]) / X[:, 1] + 0.3 * X[:, 0] / X[:, 1] * X[:, 3] + rng.normal(0, 0.01, 30)
    o = O.fit(X, y, ["sq", "sqrt", "inv"], BI, 2, False, 5, 2, dimensionality=units)
    b = B.fit(X, y, ["sq", "sqrt", "inv"], BI, 2, False, 5, 2, dimensionality=units)
    for so, sb in zip(o, b):
        assert sorted(so.sub_ids.tolist()) == sorted(np.asarray(sb["sub_ids"]).tolist())
        assert list(so.best_ids) == list(sb["best_ids"])
        assert math.isclose(so.sse, sb["sse"], rel_tol=1e-9)
    # every selected feature is physical
    sp = O.Space(4, ["sq", "sqrt", "inv"], BI, 2, False, units)
    assert all(sp.units(int(f))[0] for s in o for f in s.sub_ids)

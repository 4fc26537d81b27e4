"""NumPy brute force for tiny problems: the oracle's own check.

Test infrastructure only.  Written independently of ``sisso_oracle.c``: it
builds every feature as an expression string and a NumPy value vector level
by level (Sec. 2.1, eq. feature-exp), ranks all of them with
``numpy.corrcoef`` (Sec. 2.2, eq. sis-weight / sis-method), and fits every
t-subset with ``numpy.linalg.lstsq`` on [1, F_T] (Sec. 2.3, eq. residual).
It follows the same written readings as the oracle (numbering, validity --
including the rule that a sum or difference cancelling to sd <= 1e-5 of its
operands' root-mean-square is invalid --, duplicate classes, tie rules) so the
two can be compared id by id.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

def _elementwise(fn):
    """Apply a scalar function of Python's math module to every element.
    The transcendental functions are taken from the platform's C library (as
    the C oracle's are) rather than from NumPy's own implementations, which
    may differ by an ulp; the comparison then checks the enumeration and the
    composition of features exactly, also for ill-conditioned compositions
    such as sin(exp(x)).  Their values are pinned against hand-computed
    constants by the tests."""
    def apply(a):
        out = np.empty_like(a)
        for i, v in enumerate(a.tolist()):
            try:
                out[i] = fn(v)
            except OverflowError:
                out[i] = np.inf
            except ValueError:
                out[i] = np.nan
        return out
    return apply


_UNARY = {
    "sq": (lambda a: a * a, lambda a: True, "({})^2"),
    "cube": (lambda a: a * a * a, lambda a: True, "({})^3"),
    "sqrt": (np.sqrt, lambda a: np.all(a >= 0), "sqrt({})"),
    "inv": (lambda a: 1.0 / a, lambda a: np.all(a != 0), "1/({})"),
    "exp": (_elementwise(math.exp), lambda a: True, "exp({})"),
    "nexp": (_elementwise(lambda v: math.exp(-v)), lambda a: True, "exp(-{})"),
    "log": (_elementwise(math.log), lambda a: np.all(a > 0), "ln({})"),
    "sin": (_elementwise(math.sin), lambda a: True, "sin({})"),
}
_BINARY = {"add": "+", "sub": "-", "mul": "*", "div": "/"}


def _ok(v: np.ndarray) -> bool:
    if not np.all(np.isfinite(v)) or np.any(np.abs(v) > 1e15):
        return False
    sd = np.sqrt(np.mean((v - v.mean()) ** 2))
    return bool(sd != 0 and sd > 1e-6 * abs(v.mean()))


def _bin(op, a, b):
    with np.errstate(all="ignore"):
        if op == "add":
            return a + b, True
        if op == "sub":
            return a - b, True
        if op == "mul":
            return a * b, True
        return a / b, bool(np.all(b != 0))


def _slots(binary):
    out = []
    for op in binary:
        out.append((op, False))
        if op == "div":
            out.append((op, True))
    return out


# Units as {dimension name: Fraction exponent} (dimensionless: {}), None for a
# feature that breaks dimensional analysis (Sec. 2.1; Sec. 3.3's
# dimensionality option): sums and differences need equal units, products and
# quotients add and subtract exponents, powers scale them, and exp, exp(-x),
# ln, sin take a dimensionless argument.
_UNIT_POW = {"sq": Fraction(2), "cube": Fraction(3), "sqrt": Fraction(1, 2), "inv": Fraction(-1)}


def _unit_unary(op: str, ua: Optional[Dict[str, Fraction]]):
    if ua is None:
        return None
    if op in _UNIT_POW:
        return {k: e * _UNIT_POW[op] for k, e in ua.items()}
    return {} if not ua else None


def _unit_binary(op: str, ul, ur):
    if ul is None or ur is None:
        return None
    if op in ("add", "sub"):
        return dict(ul) if ul == ur else None
    sign = 1 if op == "mul" else -1
    out = dict(ul)
    for k, e in ur.items():
        out[k] = out.get(k, Fraction(0)) + sign * e
    return {k: e for k, e in out.items() if e != 0}


def enumerate_space(X: np.ndarray, unary: Sequence[str], binary: Sequence[str], levels: int,
                    rect: bool = False, dimensionality: Optional[Sequence[str]] = None):
    """All features in canonical order: list of (expr, values, valid)."""
    return enumerate_space_units(X, unary, binary, levels, rect, dimensionality)[0]


def enumerate_space_units(X: np.ndarray, unary: Sequence[str], binary: Sequence[str], levels: int,
                          rect: bool = False, dimensionality: Optional[Sequence[str]] = None):
    """(features, units): the features as enumerate_space gives them and, per
    feature, its units (None if not physical; all {} without dimensionality).
    With dimensionality (one unit string per base feature, "" or "1" for a
    dimensionless one) a non-physical feature is invalid."""
    n, d = X.shape
    feats: List[Tuple[str, np.ndarray, bool]] = []
    units: List[Optional[Dict[str, Fraction]]] = []
    for i in range(d):
        v = X[:, i].astype(np.float64)
        feats.append((f"x{i}", v, _ok(v)))
        u = dimensionality[i] if dimensionality is not None else ""
        units.append({} if u in ("", "1") else {u: Fraction(1)})
    sizes = [0, d]            # P_{-1}, P_0
    slots = _slots(binary)

    def unary_feat(a, op):
        fn, dom, fmt = _UNARY[op]
        ea, va, oka = feats[a]
        if not oka:
            return (fmt.format(ea), np.full(n, np.nan), False)
        with np.errstate(all="ignore"):
            if not dom(va):
                return (fmt.format(ea), np.full(n, np.nan), False)
            v = fn(va)
        return (fmt.format(ea), v, _ok(v))

    def binary_feat(l, r, op):
        el, vl, okl = feats[l]
        er, vr, okr = feats[r]
        e = f"({el}{_BINARY[op]}{er})"
        if not (okl and okr):
            return (e, np.full(n, np.nan), False)
        v, dom = _bin(op, vl, vr)
        if not dom:
            return (e, np.full(n, np.nan), False)
        ok = _ok(v)
        if ok and op in ("add", "sub"):
            scale = max(np.sqrt(np.mean(vl ** 2)), np.sqrt(np.mean(vr ** 2)))
            ok = bool(np.sqrt(np.mean((v - v.mean()) ** 2)) > 1e-5 * scale)
        return (e, v, ok)

    def physical(f, u):
        e, v, ok = f
        return (e, v, ok and u is not None) if dimensionality is not None else f

    for _ in range(levels):
        lo, hi = sizes[-2], sizes[-1]
        new, nu = [], []
        for a in range(lo, hi):
            for op in unary:
                ua = _unit_unary(op, units[a])
                new.append(physical(unary_feat(a, op), ua)); nu.append(ua)
        for j in range(lo, hi):
            for i in range(j):
                for op, rev in slots:
                    l, r = (i, j) if rev else (j, i)
                    ub = _unit_binary(op, units[l], units[r])
                    new.append(physical(binary_feat(l, r, op), ub)); nu.append(ub)
        feats.extend(new)
        units.extend(nu)
        sizes.append(len(feats))
    if rect:
        lo, hi = sizes[-2], sizes[-1]
        new, nu = [], []
        for u in range(lo, hi):
            for op in unary:
                ua = _unit_unary(op, units[u])
                new.append(physical(unary_feat(u, op), ua)); nu.append(ua)
        for u in range(lo, hi):
            for v in range(0, lo):
                for op, rev in slots:
                    l, r = (v, u) if rev else (u, v)
                    ub = _unit_binary(op, units[l], units[r])
                    new.append(physical(binary_feat(l, r, op), ub)); nu.append(ub)
        feats.extend(new)
        units.extend(nu)
    return feats, units


def abs_corr(f, r) -> float:
    return float(abs(np.corrcoef(f, r)[0, 1]))


def sis(feats, r, keep: int, exclude=()):
    ex = set(int(e) for e in exclude)
    cand = [(abs_corr(v, r), i) for i, (_, v, ok) in enumerate(feats) if ok and i not in ex]
    cand.sort(key=lambda t: (-t[0], t[1]))
    cand = cand[:keep]
    return np.array([i for _, i in cand], dtype=np.int64), np.array([s for s, _ in cand])


def dedup(feats, list_ids, list_scores, prev, k):
    ids = list(prev) + list(list_ids)
    m = len(ids)
    label = list(range(m))

    def find(a):
        while label[a] != a:
            a = label[a]
        return a

    for i in range(m):
        for j in range(i + 1, m):
            if 1.0 - abs_corr(feats[ids[i]][1], feats[ids[j]][1]) <= 1e-9:
                a, b = find(i), find(j)
                if a != b:
                    label[max(a, b)] = min(a, b)
    comps = {}
    for i in range(m):
        comps.setdefault(find(i), []).append(i)
    classes = []
    for members in comps.values():
        if any(i < len(prev) for i in members):
            continue
        rep = min(ids[i] for i in members)
        sc = max(list_scores[i - len(prev)] for i in members)
        classes.append((sc, rep))
    classes.sort(key=lambda t: (-t[0], t[1]))
    return [rep for _, rep in classes[:k]], [sc for sc, _ in classes[:k]], len(classes)


def l0(F: np.ndarray, y: np.ndarray, D: int):
    """All D-subsets of the columns of F with lstsq on [1, F_T].  Tie band
    1e-12 * S_yy, lexicographically first tuple; near-singular tuples (the
    smallest eigenvalue of their correlation matrix <= 1e-10) skipped."""
    n, m = F.shape
    syy = float(np.sum((y - y.mean()) ** 2))
    res = []
    for tup in itertools.combinations(range(m), D):
        Ft = F[:, tup]
        Z = (Ft - Ft.mean(0)) / np.sqrt(np.sum((Ft - Ft.mean(0)) ** 2, axis=0))
        if np.min(np.linalg.eigvalsh(Z.T @ Z)) <= 1e-10:
            continue
        A = np.column_stack([np.ones(n), Ft])
        c, *_ = np.linalg.lstsq(A, y, rcond=None)
        sse = float(np.sum((y - A @ c) ** 2))
        res.append((sse, tup, c))
    smin = min(r[0] for r in res)
    for sse, tup, c in res:                       # combinations are lexicographic
        if sse <= smin + 1e-12 * syy:
            return tup, sse, c, len(res)
    raise AssertionError


def fit(X, y, unary, binary, levels, rect, k, dmax, keep0=None, dimensionality=None):
    """Brute-force SISSO loop (same readings as the oracle)."""
    feats = enumerate_space(X, unary, binary, levels, rect, dimensionality)
    keep0 = 2 * k if keep0 is None else keep0
    sub: List[int] = []
    r = np.asarray(y, dtype=np.float64).copy()
    out = []
    for t in range(1, dmax + 1):
        keep = keep0
        while True:
            li, ls = sis(feats, r, keep, exclude=sub)
            new, nsc, ncls = dedup(feats, li, ls, sub, k)
            if len(new) >= k or len(li) < keep or keep >= 4096:
                break
            keep = min(2 * keep, 4096)
        sub = sub + list(new)
        order = sorted(sub)
        F = np.column_stack([feats[i][1] for i in order])
        tup, sse, c, nfit = l0(F, y, t)
        best = [order[i] for i in tup]
        r = y - np.column_stack([np.ones(len(y)), F[:, list(tup)]]) @ c
        out.append(dict(list_ids=li, list_scores=ls, sub_ids=np.array(sub), best_ids=best,
                        coef=c, sse=sse, exprs=[feats[i][0] for i in best]))
    return out

"""ctypes front-end of the plain-C FP64 oracle (test infrastructure only).

Every function here marshals NumPy arrays into ``sisso_oracle.c`` and back;
the arithmetic lives in the C file.  Operator codes follow the numbering of
the C file (binary: add 0, sub 1, mul 2, div 3; unary: sq 4, cube 5, sqrt 6,
inv 7, exp 8, nexp 9, log 10, sin 11).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import build as _build

OPCODE = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sq": 4, "cube": 5, "sqrt": 6,
          "inv": 7, "exp": 8, "nexp": 9, "log": 10, "sin": 11}

_lib = None
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)


class _Step(ctypes.Structure):
    _fields_ = [("n_list", ctypes.c_int64),
                ("list_ids", ctypes.c_int64 * 4096),
                ("list_scores", ctypes.c_double * 4096),
                ("n_sub", ctypes.c_int64),
                ("sub_ids", ctypes.c_int64 * 1024),
                ("best_ids", ctypes.c_int64 * 8),
                ("coef", ctypes.c_double * 9),
                ("sse", ctypes.c_double), ("runner_up", ctypes.c_double),
                ("rmse", ctypes.c_double), ("r2", ctypes.c_double),
                ("n_tuples", ctypes.c_int64), ("n_singular", ctypes.c_int64),
                ("status", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        L.or_space_new.restype = ctypes.c_void_p
        L.or_space_new.argtypes = [ctypes.c_int, _i32p, ctypes.c_int, _i32p, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int]
        L.or_space_free.argtypes = [ctypes.c_void_p]
        L.or_space_total.restype = ctypes.c_int64
        L.or_space_total.argtypes = [ctypes.c_void_p]
        L.or_space_pool.restype = ctypes.c_int64
        L.or_space_pool.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.or_decode.restype = ctypes.c_int
        L.or_decode.argtypes = [ctypes.c_void_p, ctypes.c_int64, _i32p, _i64p, _i64p]
        L.or_eval.restype = ctypes.c_int
        L.or_eval.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp]
        L.or_eval_many.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _i64p,
                                   ctypes.c_int64, _dp, ctypes.c_int, _i32p]
        L.or_abs_corr.restype = ctypes.c_double
        L.or_abs_corr.argtypes = [_dp, _dp, ctypes.c_int]
        L.or_score_range.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _dp,
                                     ctypes.c_int64, ctypes.c_int64, _dp]
        L.or_sis.restype = ctypes.c_int64
        L.or_sis.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _dp,
                             ctypes.c_int64, ctypes.c_int64, _i64p, ctypes.c_int64,
                             ctypes.c_int64, _i64p, _dp]
        L.or_dup_components.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i64p]
        L.or_dedup.restype = ctypes.c_int64
        L.or_dedup.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _i64p, _dp,
                               ctypes.c_int64, _i64p, ctypes.c_int64, ctypes.c_int64,
                               _i64p, _dp, _i64p]
        L.or_l0.restype = ctypes.c_int
        L.or_l0.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp, ctypes.c_int,
                            _i64p, _dp, _dp, _dp, _i64p, _i64p]
        L.or_residual.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _i64p, ctypes.c_int, _dp,
                                  _dp, _dp]
        L.or_fit.restype = ctypes.c_int
        L.or_fit.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int64, ctypes.POINTER(_Step)]
        L.or_abs_corr_w.restype = ctypes.c_double
        L.or_abs_corr_w.argtypes = [_dp, _dp, _dp, ctypes.c_int]
        L.or_score_range_w.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp,
                                       ctypes.c_int64, ctypes.c_int64, _dp]
        L.or_sis_w.restype = ctypes.c_int64
        L.or_sis_w.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp,
                               ctypes.c_int64, ctypes.c_int64, _i64p, ctypes.c_int64,
                               ctypes.c_int64, _i64p, _dp]
        L.or_dup_components_w.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp, _i64p]
        L.or_dedup_w.restype = ctypes.c_int64
        L.or_dedup_w.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _dp, _i64p, _dp,
                                 ctypes.c_int64, _i64p, ctypes.c_int64, ctypes.c_int64,
                                 _i64p, _dp, _i64p]
        L.or_l0_w.restype = ctypes.c_int
        L.or_l0_w.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp, _dp, ctypes.c_int,
                              _i64p, _dp, _dp, _dp, _i64p, _i64p]
        L.or_fit_w.restype = ctypes.c_int
        L.or_fit_w.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int64, ctypes.POINTER(_Step)]
        L.or_space_set_units.restype = ctypes.c_int
        L.or_space_set_units.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int]
        L.or_units.restype = ctypes.c_int
        L.or_units.argtypes = [ctypes.c_void_p, ctypes.c_int64, _dp]
        L.or_step_size.restype = ctypes.c_int
        assert L.or_step_size() == ctypes.sizeof(_Step)
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _wp(w, n: int):
    """Sample weights (Sec. 2.4: w_s = 1 / sigma_s^2 for a diagonal noise
    covariance) as a C pointer, or NULL for the unweighted method; the array
    is returned too so that it outlives the call."""
    if w is None:
        return None, None
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    if w.shape != (n,) or not np.all(np.isfinite(w)) or np.any(w <= 0.0):
        raise ValueError("oracle: weights must be n positive finite values")
    return w, _p(w, _dp)


def _colmajor(X: np.ndarray) -> np.ndarray:
    """n x d row-major array -> contiguous d x n buffer (column-major X)."""
    return np.ascontiguousarray(np.asarray(X, dtype=np.float64).T)


def unit_matrix(dimensionality: Sequence[str]) -> np.ndarray:
    """Exponent matrix (d x n_dim) of the base features from their unit
    strings (the dimensionality option of Sec. 3.3): every distinct string
    names a base dimension in order of first appearance and gives its feature
    exponent 1 there; "" and "1" mark a dimensionless feature."""
    names: List[str] = []
    for u in dimensionality:
        if u not in ("", "1") and u not in names:
            names.append(u)
    M = np.zeros((len(dimensionality), len(names)), dtype=np.float64)
    for i, u in enumerate(dimensionality):
        if u not in ("", "1"):
            M[i, names.index(u)] = 1.0
    return M


class Space:
    """The expanded feature space: `levels` full levels plus, if `rect`, the
    one-sided next-level slice; with `dimensionality` (one unit string per
    base feature), features that break dimensional analysis are invalid."""

    def __init__(self, d: int, unary: Sequence[str], binary: Sequence[str], levels: int,
                 rect: bool = False, dimensionality: Sequence[str] | None = None):
        self.d, self.levels, self.rect = d, levels, rect
        self.unary, self.binary = list(unary), list(binary)
        u = np.array([OPCODE[o] for o in unary] or [0], dtype=np.int32)
        b = np.array([OPCODE[o] for o in binary] or [0], dtype=np.int32)
        h = lib().or_space_new(d, _p(u, _i32p), len(unary), _p(b, _i32p), len(binary),
                               levels, int(rect))
        if not h:
            raise ValueError("oracle: invalid space")
        self._h = ctypes.c_void_p(h)
        self.n_dim = 0
        if dimensionality is not None:
            if len(dimensionality) != d:
                raise ValueError("oracle: one unit string per base feature")
            M = np.ascontiguousarray(unit_matrix(dimensionality))
            self.n_dim = M.shape[1]
            # no named dimension: every feature is dimensionless, no rule applies
            if self.n_dim and lib().or_space_set_units(self._h, _p(M, _dp), self.n_dim):
                raise ValueError("oracle: too many base dimensions")

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.or_space_free(self._h)
            self._h = None

    @property
    def total(self) -> int:
        return int(lib().or_space_total(self._h))

    def pool(self, level: int) -> int:
        return int(lib().or_space_pool(self._h, level))

    def decode(self, fid: int):
        op = ctypes.c_int32(); l = ctypes.c_int64(); r = ctypes.c_int64()
        if lib().or_decode(self._h, fid, ctypes.byref(op), ctypes.byref(l), ctypes.byref(r)):
            raise IndexError(fid)
        return op.value, l.value, r.value

    def units(self, fid: int):
        """(physical, exponents) of feature fid (exponents over the base
        dimensions in order of first appearance)."""
        u = np.zeros(max(self.n_dim, 1), dtype=np.float64)
        ok = lib().or_units(self._h, int(fid), _p(u, _dp))
        return bool(ok), u[:self.n_dim].copy()

    def eval(self, X: np.ndarray, ids: Sequence[int]):
        """FP64 values (n x len(ids)) and validity flags of features `ids`."""
        Xc = _colmajor(X)
        n = X.shape[0]
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int64))
        out = np.empty((len(ids), n), dtype=np.float64)
        valid = np.empty(len(ids), dtype=np.int32)
        lib().or_eval_many(self._h, _p(Xc, _dp), n, n, _p(ids, _i64p), len(ids), _p(out, _dp), n,
                           _p(valid, _i32p))
        return out.T.copy(), valid.astype(bool)

    def score_range(self, X, r, begin: int, end: int, w=None) -> np.ndarray:
        Xc = _colmajor(X)
        r = np.ascontiguousarray(r, dtype=np.float64)
        out = np.empty(end - begin, dtype=np.float64)
        w, wp = _wp(w, X.shape[0])
        lib().or_score_range_w(self._h, _p(Xc, _dp), X.shape[0], X.shape[0], _p(r, _dp), wp, begin,
                               end, _p(out, _dp))
        return out

    def sis(self, X, r, keep: int, exclude: Sequence[int] = (), begin: int = 0,
            end: int | None = None, w=None):
        Xc = _colmajor(X)
        r = np.ascontiguousarray(r, dtype=np.float64)
        ex = np.ascontiguousarray(np.asarray(list(exclude) or [0], dtype=np.int64))
        ids = np.empty(max(keep, 1), dtype=np.int64)
        sc = np.empty(max(keep, 1), dtype=np.float64)
        end = self.total if end is None else end
        w, wp = _wp(w, X.shape[0])
        c = lib().or_sis_w(self._h, _p(Xc, _dp), X.shape[0], X.shape[0], _p(r, _dp), wp, begin, end,
                           _p(ex, _i64p), len(exclude), keep, _p(ids, _i64p), _p(sc, _dp))
        return ids[:c].copy(), sc[:c].copy()

    def dedup(self, X, list_ids, list_scores, prev: Sequence[int], k: int, w=None):
        Xc = _colmajor(X)
        w, wp = _wp(w, X.shape[0])
        li = np.ascontiguousarray(np.asarray(list_ids, dtype=np.int64))
        ls = np.ascontiguousarray(np.asarray(list_scores, dtype=np.float64))
        pv = np.ascontiguousarray(np.asarray(list(prev) or [0], dtype=np.int64))
        oi = np.empty(max(k, 1), dtype=np.int64)
        os_ = np.empty(max(k, 1), dtype=np.float64)
        ncls = ctypes.c_int64()
        c = lib().or_dedup_w(self._h, _p(Xc, _dp), X.shape[0], X.shape[0], wp, _p(li, _i64p),
                             _p(ls, _dp), len(li), _p(pv, _i64p), len(prev), k, _p(oi, _i64p),
                             _p(os_, _dp), ctypes.byref(ncls))
        return oi[:c].copy(), os_[:c].copy(), ncls.value


def abs_corr(f, r, w=None) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    w, wp = _wp(w, len(f))
    return float(lib().or_abs_corr_w(_p(f, _dp), _p(r, _dp), wp, len(f)))


def dup_components(F: np.ndarray, w=None) -> np.ndarray:
    """F: n x m FP64; returns the component label (min member index) per column."""
    Fc = np.ascontiguousarray(np.asarray(F, dtype=np.float64).T)
    m = Fc.shape[0]
    comp = np.empty(max(m, 1), dtype=np.int64)
    w, wp = _wp(w, F.shape[0])
    lib().or_dup_components_w(_p(Fc, _dp), F.shape[0], F.shape[0], m, wp, _p(comp, _i64p))
    return comp[:m]


@dataclass
class L0Result:
    best: np.ndarray        # positions, ascending
    sse: float
    runner_up: float
    coef: np.ndarray        # intercept first
    n_tuples: int
    n_singular: int
    status: int


def l0(F: np.ndarray, y: np.ndarray, D: int, w=None) -> L0Result:
    """Exhaustive D-term least squares over the columns of F (n x m), whose
    order must be ascending in feature id; weighted least squares (the SSE is
    sum_s w_s e_s^2) when sample weights w are given."""
    Fc = np.ascontiguousarray(np.asarray(F, dtype=np.float64).T)
    n, m = F.shape
    y = np.ascontiguousarray(y, dtype=np.float64)
    best = np.zeros(8, dtype=np.int64)
    sse = ctypes.c_double(); ru = ctypes.c_double()
    coef = np.zeros(9, dtype=np.float64)
    nt = ctypes.c_int64(); ns = ctypes.c_int64()
    w, wp = _wp(w, n)
    st = lib().or_l0_w(_p(Fc, _dp), n, n, m, _p(y, _dp), wp, D, _p(best, _i64p), ctypes.byref(sse),
                       ctypes.byref(ru), _p(coef, _dp), ctypes.byref(nt), ctypes.byref(ns))
    return L0Result(best[:D].copy(), sse.value, ru.value, coef[:D + 1].copy(), nt.value,
                    ns.value, st)


@dataclass
class StepResult:
    list_ids: np.ndarray
    list_scores: np.ndarray
    sub_ids: np.ndarray
    best_ids: np.ndarray
    coef: np.ndarray
    sse: float
    runner_up: float
    rmse: float
    r2: float
    n_tuples: int
    n_singular: int
    status: int


def fit(X: np.ndarray, y: np.ndarray, unary, binary, levels: int, rect: bool, k: int,
        dmax: int, keep0: int | None = None, w=None, dimensionality=None) -> List[StepResult]:
    """Oracle SISSO fit; one StepResult per dimension t = 1..dmax (weighted
    screening, duplicate classes and least squares when sample weights w are
    given)."""
    sp = Space(X.shape[1], unary, binary, levels, rect, dimensionality)
    Xc = _colmajor(X)
    y = np.ascontiguousarray(y, dtype=np.float64)
    steps = (_Step * dmax)()
    keep0 = 2 * k if keep0 is None else keep0
    w, wp = _wp(w, X.shape[0])
    done = lib().or_fit_w(sp._h, _p(Xc, _dp), X.shape[0], X.shape[0], _p(y, _dp), wp, k, dmax, keep0,
                          steps)
    out = []
    for t in range(done):
        s = steps[t]
        out.append(StepResult(np.array(s.list_ids[:s.n_list]), np.array(s.list_scores[:s.n_list]),
                              np.array(s.sub_ids[:s.n_sub]), np.array(s.best_ids[:t + 1]),
                              np.array(s.coef[:t + 2]), s.sse, s.runner_up, s.rmse, s.r2,
                              s.n_tuples, s.n_singular, s.status))
    return out


def fit_threshold(X: np.ndarray, y: np.ndarray, unary, binary, levels: int, rect, tau: float, keep: int,
                  k: int, dmax: int):
    """Oracle SISSO fit with Sec. 2.2's threshold alternative: each pass keeps
    every candidate whose |corr| with the residual is at least tau (searched
    among the best `keep`), forms their duplicate classes against S_{t-1} and
    appends at most k of them; the SO of Sec. 2.3 then fits y on S_t.  Built
    from the oracle's own screening, duplicate-class and l0 functions.
    Returns per t: (appended ids, S_t, best ids, SSE)."""
    sp = Space(X.shape[1], unary, binary, levels, rect)
    r = np.asarray(y, dtype=np.float64).copy()
    sub: List[int] = []
    out = []
    for t in range(1, dmax + 1):
        ids, sc = sp.sis(X, r, keep, exclude=sorted(sub))
        sel = sc >= tau
        new, nsc, _ = sp.dedup(X, ids[sel], sc[sel], sub, k)
        sub.extend(int(i) for i in new)
        srt = np.array(sorted(sub), dtype=np.int64)
        F, ok = sp.eval(X, srt)
        res = l0(F, y, t)
        best = srt[res.best]
        A = np.column_stack([np.ones(len(y)), F[:, res.best]])
        r = y - A @ res.coef
        out.append((np.array(new), np.array(sub), best, res.sse))
    return out

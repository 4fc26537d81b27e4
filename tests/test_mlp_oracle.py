"""Pins of the FP64 reference of the learned proposal (no GPU).

The gradient is pinned by central finite differences of the loss, Adam by
its closed form under a constant gradient, the operand statistics by
numpy.corrcoef and scipy.stats.skew, BF16 rounding by hand-checked bit
patterns, and the operand classes by a small hand-enumerated space.
"""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import mlp as M
from oracle import oracle as O
from paper_2410_01752_amd import inputs as I


def _setup(seed=3, batch=24):
    X, t, w = I.mlp_batch(seed, batch)
    P = I.mlp_init(seed + 100)
    P["b1"] = np.random.default_rng(seed).uniform(-0.2, 0.2, M.HIDDEN)
    P["b2"] = np.array([0.3])
    return X, t, w, P


def test_gradient_matches_central_differences():
    X, t, w, P = _setup()
    z, _, _ = M.forward(X, P, bf16=False)
    assert np.min(np.abs(z)) > 1e-5          # no kink within the perturbation
    loss, g, _ = M.loss_and_grad(X, t, w, P, bf16=False)
    rng = np.random.default_rng(7)
    h = 1e-6
    checks = [("b2", (0,))] + [("w2", (int(i),)) for i in rng.integers(0, M.HIDDEN, 8)] + \
             [("b1", (int(i),)) for i in rng.integers(0, M.HIDDEN, 8)] + \
             [("W1", (int(i), int(j))) for i, j in zip(rng.integers(0, M.HIDDEN, 16), rng.integers(0, 140, 16))]
    for name, idx in checks:
        Pp = {k: v.copy() for k, v in P.items()}
        Pm = {k: v.copy() for k, v in P.items()}
        Pp[name][idx] += h
        Pm[name][idx] -= h
        lp = M.loss_and_grad(X, t, w, Pp, bf16=False)[0]
        lm = M.loss_and_grad(X, t, w, Pm, bf16=False)[0]
        fd = (lp - lm) / (2 * h)
        an = g[name][idx]
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-3), (name, idx, fd, an)


def test_loss_is_weighted_mse_and_zero_at_the_target():
    X, t, w, P = _setup(batch=10)
    _, _, s = M.forward(X, P)
    loss, g, _ = M.loss_and_grad(X, s.copy(), w, P)
    assert loss == 0.0
    assert all(np.all(v == 0.0) for v in g.values())
    loss2 = M.loss_and_grad(X, t, np.ones(10), P)[0]
    assert math.isclose(loss2, float(np.mean((s - t) ** 2)), rel_tol=1e-12)


def test_adam_constant_gradient_closed_form():
    """With zero initial moments and a constant gradient g, every bias-
    corrected step moves a parameter by -lr * g / (|g| + eps)."""
    P = {"a": np.array([1.0, -2.0, 0.5]), "b": np.array([3.0])}
    G = {"a": np.array([0.3, -1e-3, 2.0]), "b": np.array([-4.0])}
    Mo = {k: np.zeros_like(v) for k, v in P.items()}
    Vo = {k: np.zeros_like(v) for k, v in P.items()}
    lr, eps = 1e-2, 1e-8
    cur = P
    for step in range(1, 4):
        cur, Mo, Vo = M.adam_step(cur, G, Mo, Vo, step, lr=lr, eps=eps)
        for k in P:
            exp = P[k] - step * lr * G[k] / (np.abs(G[k]) + eps)
            assert np.allclose(cur[k], exp, rtol=0, atol=1e-12), (k, step)


def test_operand_stats_against_library_routines():
    rng = np.random.default_rng(11)
    n = 500
    x = rng.lognormal(0.0, 0.5, n)
    r = 0.7 * np.log(x) + rng.normal(0, 0.3, n)
    st = M.operand_stats(x, r)
    assert math.isclose(st[0], np.corrcoef(x, r)[0, 1], rel_tol=1e-12)
    assert math.isclose(st[2], np.corrcoef(1 / x, r)[0, 1], rel_tol=1e-12)
    assert math.isclose(st[3], np.corrcoef(np.log(x), r)[0, 1], rel_tol=1e-12)
    assert math.isclose(st[4], np.corrcoef(x * x, r)[0, 1], rel_tol=1e-12)
    assert st[1] == abs(st[0]) and st[5] == abs(st[2]) and st[6] == abs(st[3])
    assert math.isclose(st[8] * 10, scipy.stats.skew(x, bias=True), rel_tol=1e-10)
    assert math.isclose(st[7] * 4, math.log10(np.std(x) / np.mean(x)), rel_tol=1e-12)
    assert st[11] == 1.0 and st[12] == 0.0 and st[13] == 1.0
    # a column with a zero: 1/x and log|x| are undefined -> 0
    x0 = x.copy()
    x0[3] = 0.0
    s0 = M.operand_stats(x0, r)
    assert s0[2] == 0.0 and s0[3] == 0.0 and s0[12] == 1.0 and s0[11] == 0.0
    # a symmetric sample has zero skewness; a constant column has zero correlations
    sym = np.concatenate([x, 2 * np.mean(x) - x])
    assert abs(M.operand_stats(sym, np.concatenate([r, r]))[8]) < 1e-12
    c = M.operand_stats(np.full(n, 2.5), r)
    assert c[0] == 0.0 and c[4] == 0.0 and c[2] == 0.0


def test_bf16_rounding_bit_patterns():
    one = 1.0
    assert M.bf16_round(np.array([one]))[0] == 1.0
    assert M.bf16_round(np.array([1 + 2 ** -7]))[0] == 1 + 2 ** -7          # representable
    assert M.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0                   # tie -> even
    assert M.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6       # tie -> even (up)
    assert M.bf16_round(np.array([1 + 2 ** -8 + 2 ** -12]))[0] == 1 + 2 ** -7  # above the tie
    assert M.bf16_round(np.array([-3.0]))[0] == -3.0
    assert M.bf16_round(np.array([0.0]))[0] == 0.0


def test_tree_classes_small_space():
    """d = 2, unary {sq}, binary {add, mul}: P_0 = {x0, x1}; N_1 = sq(x0) 2,
    sq(x1) 3, x1+x0 4, x1*x0 5; level 2 starts with sq of 2..5 (ids 6..9),
    then pairs (j, i) with j in N_1."""
    sp = O.Space(2, ["sq"], ["add", "mul"], 2)
    assert sp.pool(1) == 6
    assert M.tree_classes(sp, 0) == (0, 13, 13)
    assert M.tree_classes(sp, 2) == (1 + 4, 0, 13)
    assert M.tree_classes(sp, 5) == (1 + 2, 0, 0)
    assert M.tree_classes(sp, 6) == (1 + 4, 1 + 4, 13)       # sq(sq(x0))
    assert M.tree_classes(sp, 9) == (1 + 4, 1 + 2, 13)       # sq(x1*x0)
    # first pair of level 2: j = 2 (sq x0), i = 0: add, then mul
    assert M.tree_classes(sp, 10) == (1 + 0, 1 + 4, 0)
    assert M.tree_classes(sp, 11) == (1 + 2, 1 + 4, 0)


def test_factorised_score_equals_network_on_the_input():
    P = I.mlp_init(5)
    P["b1"] = np.random.default_rng(2).uniform(-0.5, 0.5, M.HIDDEN)
    rng = np.random.default_rng(9)
    for form in range(5):
        eu = M.encode((3, 0, 0), rng.uniform(-1, 1, 14))
        ev = M.encode((0, 13, 13), rng.uniform(-1, 1, 14))
        x = M.candidate_input(eu, ev, form)
        s = M.forward(x[None, :], P)[2][0]
        assert math.isclose(M.score_factorised(eu, ev, form, P), s, rel_tol=1e-12, abs_tol=1e-12)


def test_target_is_fisher_z():
    assert M.target(np.array([0.0]))[0] == 0.0
    assert math.isclose(M.target(np.array([0.5]))[0], 0.5 * math.log(3.0), rel_tol=1e-15)
    assert np.isfinite(M.target(np.array([1.0]))[0])


def test_operand_stats_log10_mean_and_sd_hand_values():
    """Entries 51 and 52 of an operand encoding: clip(log10|mean|, -6, 6)/6
    and clip(log10 sd, -6, 6)/6.  x = (990, 1010): mean 1000, population sd
    10, so the entries are 3/6 and 1/6; scaling by 1e8 clips the mean's
    entry at 1 (sd 1e9 clips too); scaling by 1e-8 gives log10 = -5 and -7."""
    r = np.array([0.3, -0.3])
    st = M.operand_stats(np.array([990.0, 1010.0]), r)
    assert math.isclose(st[9], 0.5, rel_tol=1e-15) and math.isclose(st[10], 1.0 / 6.0, rel_tol=1e-14)
    big = M.operand_stats(np.array([990.0, 1010.0]) * 1e8, r)
    assert big[9] == 1.0 and big[10] == 1.0
    small = M.operand_stats(np.array([990.0, 1010.0]) * 1e-8, r)
    assert math.isclose(small[9], -5.0 / 6.0, rel_tol=1e-14) and small[10] == -1.0
    neg = M.operand_stats(-np.array([990.0, 1010.0]), r)
    assert math.isclose(neg[9], 0.5, rel_tol=1e-15)

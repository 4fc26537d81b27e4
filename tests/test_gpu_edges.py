"""Degenerate and boundary cases of the screening and fitting path against the
FP64 oracle: the smallest sample counts (n below one float4 group, ragged
chunks, every feature tied at |corr| = 1), lists longer than the number of
valid candidates, K' = 1, a constant residual (no candidate has a defined
correlation) and whole fits at small n."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2410_01752_amd import inputs as I

from test_gpu_parity import _compare_fit, _engine, _screen, assert_topk_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [3, 5, 7])
def test_smallest_sample_counts_full_rect_space(n):
    p = I.tiny(21, n=n, d=3, dist="lognormal", rect=True)
    print(f"[edges] rect space n={n}", flush=True)
    eng = _engine(p)
    sp = O.Space(3, p.unary, p.binary, 2, True)
    keep = 300
    gi, gs = _screen(eng, p.y, keep)
    oi, os_ = sp.sis(p.X, p.y, keep)
    assert_topk_parity(sp, p.X, p.y, gi, gs, oi, os_, keep)


def test_list_longer_than_the_valid_candidates_and_keep_one():
    p = I.tiny(22, n=20, d=2, dist="lognormal", rect=False, unary=("sq",), binary=("add", "mul"), rung=1)
    print("[edges] 6 valid candidates", flush=True)
    eng = _engine(p)
    sp = O.Space(2, p.unary, p.binary, 1, False)
    gi, gs = _screen(eng, p.y, 100)
    oi, os_ = sp.sis(p.X, p.y, 100)
    assert len(oi) < 100 and np.array_equal(gi, oi)
    assert np.max(np.abs(gs - os_)) <= 1e-6
    g1, s1 = _screen(eng, p.y, 1)
    assert len(g1) == 1 and g1[0] == oi[0]


def test_constant_residual_admits_nothing():
    p = I.tiny(23, n=40, d=3, dist="lognormal", rect=True)
    print("[edges] constant residual", flush=True)
    eng = _engine(p)
    sp = O.Space(3, p.unary, p.binary, 2, True)
    r = np.full(40, 2.5)
    assert len(sp.sis(p.X, r, 50)[0]) == 0
    gi, gs = _screen(eng, r, 50)
    assert len(gi) == 0
    for form in ("bf16",):
        r64 = torch.as_tensor(r, dtype=torch.float64, device=eng.dev)
        ids, sc, cnt = eng.screen(r64, 50, None, begin=eng.binary_base(), precision=form)
        torch.cuda.synchronize()
        assert int(cnt.item()) == 0


@pytest.mark.parametrize("n", [6, 9])
def test_fit_at_small_n_matches_oracle(n):
    p = I.tiny(24, n=n, d=3, dist="uniform", rect=False, k=3, dmax=2)
    print(f"[edges] fit n={n}", flush=True)
    eng = _engine(p)
    res = eng.fit(p.k, p.dmax)
    ref = O.fit(p.X, p.y, p.unary, p.binary, p.rung, p.rect, p.k, p.dmax)
    _compare_fit(p, res, ref)


def test_topk_tie_overflow_keeps_every_entry_above_the_cutoff():
    """More entries tie exactly at the k-th score than the top-k gather buffer
    (8192) holds behind the entries above it.  x0 carries the target; x1..x130
    are copies of one column z, so z's copies and every x_j + x_i = 2z (i, j
    >= 1) tie exactly (8,515 features), and the x_j + x0 tie at a higher
    score.  The merge must return every entry above the cutoff (x0 and the 130
    sums with x0), fill the rest with tied entries, and report the overflow."""
    from paper_2410_01752_amd import _lib as L
    rng = np.random.default_rng(31)
    n, d = 64, 131
    x0 = rng.lognormal(0.0, 0.5, n)
    z = rng.lognormal(0.0, 0.5, n)
    X = np.column_stack([x0] + [z] * (d - 1))
    y = x0 + 0.2 * z + rng.normal(0.0, 0.05, n)
    p = I.Problem("ties", X, y, [], ["add"], 1, False, 10, 1, [], [], 0)
    print("[edges] tie overflow at the top-k cutoff", flush=True)
    eng = _engine(p)
    sp = O.Space(d, [], ["add"], 1, False)
    keep = 2048
    oi, os_ = sp.sis(X, y, keep)
    n_above = int(np.sum(os_ > os_[-1]))
    assert n_above == 131 and np.sum(os_ == os_[-1]) == keep - n_above
    gi, gs = _screen(eng, y, keep)
    assert len(gi) == keep
    assert set(gi[:n_above].tolist()) == set(oi[:n_above].tolist())
    assert np.all(gs[n_above:] == gs[n_above])
    assert gs[n_above - 1] > gs[n_above]
    ties = set(np.flatnonzero(np.isclose(sp.score_range(X, y, 0, sp.total), os_[-1], rtol=0, atol=1e-15)).tolist())
    assert len(ties) == 8515 and set(gi[n_above:].tolist()) <= ties
    torch.cuda.synchronize()
    assert int(eng.tk_status.item()) == 1
    # the fit driver refuses a merge whose tie order is not exact
    with pytest.raises(L.SissoError):
        eng.fit(10, 1, keep0=keep)


def test_duplicate_class_with_millions_of_pairs():
    """The screened list holds 1,977 duplicates of one feature (copies of z and
    sums of two copies, 2z), so one duplicate class has about 1.95 million
    pairs: the classes (Sec. 2.1's non-unique combinations) must still be
    exact -- the subspace equals the oracle's."""
    rng = np.random.default_rng(32)
    n, d = 64, 71
    x0 = rng.lognormal(0.0, 0.5, n)
    z = rng.lognormal(0.0, 0.5, n)
    X = np.column_stack([x0] + [z] * (d - 1))
    y = x0 + 0.2 * z + rng.normal(0.0, 0.05, n)
    p = I.Problem("dups", X, y, [], ["add"], 1, False, 3, 1, [], [], 0)
    print("[edges] duplicate class of ~2e6 pairs", flush=True)
    eng = _engine(p)
    res = eng.fit(3, 1, keep0=2048)
    ref = O.fit(X, y, [], ["add"], 1, False, 3, 1, keep0=2048)
    assert list(res[0].list_ids) == list(ref[0].list_ids)
    assert list(res[0].sub_ids) == list(ref[0].sub_ids)
    assert res[0].n_classes == 3
    assert list(res[0].best_ids) == list(ref[0].best_ids)

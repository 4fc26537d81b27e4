"""GPU parity tests: the HIP path through the C ABI against the FP64 oracle.

Tolerances: |corr| within 1e-6 absolute of the oracle for FP32 screening
scores; identical top-K' sets except for ids whose oracle score is within
1e-6 of the oracle's cutoff; identical SO best tuples (unless the oracle's
runner-up is within 1e-9 relative); SO SSE / RMSE within 1e-6 relative.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2410_01752_amd import inputs as I

pytestmark = pytest.mark.gpu

SCORE_TOL = 1e-6


def _engine(p, levels=None, rect=None):
    from paper_2410_01752_amd.fit import Engine
    return Engine(p.X, p.y, p.unary, p.binary, p.rung if levels is None else levels,
                  p.rect if rect is None else rect)


def _oracle_scores_for(sp, X, r, ids):
    return np.array([sp.score_range(X, r, int(i), int(i) + 1)[0] for i in ids])


def assert_topk_parity(sp, X, r, gpu_ids, gpu_sc, o_ids, o_sc, keep, tol=SCORE_TOL):
    gpu_ids = np.asarray(gpu_ids)
    gpu_sc = np.asarray(gpu_sc, dtype=np.float64)
    assert len(gpu_ids) == len(o_ids), (len(gpu_ids), len(o_ids))
    omap = dict(zip(o_ids.tolist(), o_sc.tolist()))
    missing = [i for i in gpu_ids.tolist() if i not in omap]
    if missing:
        omap.update(zip(missing, _oracle_scores_for(sp, X, r, missing).tolist()))
    ref = np.array([omap[i] for i in gpu_ids.tolist()])
    assert np.all(np.isfinite(ref)), "GPU kept a feature the oracle calls invalid"
    err = np.abs(ref - gpu_sc)
    assert err.max() <= tol, f"max |dcorr| = {err.max():.3e}"
    cutoff = o_sc[-1] if len(o_ids) == keep else -np.inf
    diff = set(gpu_ids.tolist()) ^ set(o_ids.tolist())
    for i in diff:
        assert abs(omap[i] - cutoff) <= tol, (i, omap[i], cutoff)
    # order: GPU list is sorted by (score desc, id asc)
    assert np.all(np.diff(gpu_sc) <= 0)


def _screen(eng, r, keep, begin=0, end=None, exclude=None, grid=0, tile=0):
    r64 = torch.as_tensor(r, dtype=torch.float64, device=eng.dev)
    ex = None
    if exclude is not None and len(exclude):
        ex = torch.as_tensor(np.sort(np.asarray(exclude, dtype=np.int64)), device=eng.dev)
    ids, sc, cnt = eng.screen(r64, keep, ex, begin=begin, end=end, grid=grid, tile=tile)
    torch.cuda.synchronize()
    c = int(cnt.item())
    return ids[:c].cpu().numpy(), sc[:c].cpu().numpy()


# ------------------------------------------------------------------ pools

@pytest.mark.parametrize("name", ["tiny_rect", "C1", "C2"])
def test_pools_match_oracle(name):
    p = {"tiny_rect": lambda: I.tiny(3, n=40, d=4, rect=True), "C1": I.config1,
         "C2": I.config2}[name]()
    print(f"[pools] {name} n={p.X.shape[0]} d={p.X.shape[1]}", flush=True)
    eng = _engine(p)
    sp = O.Space(p.X.shape[1], p.unary, p.binary, p.rung, p.rect)
    pL = sp.pool(p.rung)
    rng = np.random.default_rng(0)
    ids = np.unique(np.concatenate([np.arange(min(pL, 3000)), rng.integers(0, pL, 3000)]))
    V, ok = sp.eval(p.X, ids)
    torch.cuda.synchronize()
    pool = eng.pool32.view(pL, eng.ld32)[:, :eng.n].cpu().numpy()
    stats = eng.stats.view(pL, 8).cpu().numpy()
    assert np.array_equal(stats[ids, 6] != 0, ok)
    got = pool[ids[ok]].T
    want = V[:, ok].astype(np.float32)
    assert np.all(np.abs(got - want) <= 2e-7 * np.maximum(np.abs(want), 1e-30))


@pytest.mark.parametrize("n", [2048, 2049, 2600])
def test_long_columns_pools_and_column_pass(n):
    """Columns of up to 2048 samples are held in registers by the pool and
    stored-column kernels; longer ones take the streaming path.  Both sides of
    the boundary against the oracle: every pool column, and SIS over the stored
    pool plus the unary slice."""
    p = I.tiny(17, n=n, d=4, dist="lognormal", rect=True)
    print(f"[long columns] n={n}", flush=True)
    eng = _engine(p)
    sp = O.Space(4, p.unary, p.binary, 2, True)
    p2 = sp.pool(2)
    V, ok = sp.eval(p.X, np.arange(p2))
    torch.cuda.synchronize()
    pool = eng.pool32.view(p2, eng.ld32)[:, :eng.n].cpu().numpy()
    stats = eng.stats.view(p2, 8).cpu().numpy()
    assert np.array_equal(stats[:, 6] != 0, ok)
    want = V[:, ok].astype(np.float32)
    assert np.all(np.abs(pool[ok].T - want) <= 2e-7 * np.maximum(np.abs(want), 1e-30))
    end = p2 + len(p.unary) * (p2 - sp.pool(1))
    keep = 800
    gi, gs = _screen(eng, p.y, keep, 0, end)
    oi, os_ = sp.sis(p.X, p.y, keep, begin=0, end=end)
    assert_topk_parity(sp, p.X, p.y, gi, gs, oi, os_, keep)


# --------------------------------------------------------------- screening

def test_screen_c1_full_space():
    p = I.config1()
    print("[screen] C1", flush=True)
    eng = _engine(p)
    sp = O.Space(5, p.unary, p.binary, 2)
    keep = 2048
    gi, gs = _screen(eng, p.y, keep)
    oi, os_ = sp.sis(p.X, p.y, keep)
    assert_topk_parity(sp, p.X, p.y, gi, gs, oi, os_, keep)


def test_screen_tiny_rect_full_space_and_exclusion():
    p = I.tiny(5, n=24, d=3, rect=True)
    print("[screen] tiny rect", flush=True)
    eng = _engine(p)
    sp = O.Space(3, p.unary, p.binary, 2, True)
    keep = 600
    gi, gs = _screen(eng, p.y, keep)
    oi, os_ = sp.sis(p.X, p.y, keep)
    assert_topk_parity(sp, p.X, p.y, gi, gs, oi, os_, keep)
    ex = oi[:50:3]
    gi2, gs2 = _screen(eng, p.y, keep, exclude=ex)
    oi2, os2 = sp.sis(p.X, p.y, keep, exclude=ex)
    assert not set(ex.tolist()) & set(gi2.tolist())
    assert_topk_parity(sp, p.X, p.y, gi2, gs2, oi2, os2, keep)


@pytest.mark.parametrize("part", ["pool", "unary", "binary", "binary_ragged"])
def test_screen_rect_slices(part):
    """Slices of each block of a rung-3 space (n = 300, d = 6)."""
    p = I.tiny(9, n=300, d=6, dist="lognormal", rect=True)
    print(f"[screen] rect slice {part}", flush=True)
    eng = _engine(p)
    sp = O.Space(6, p.unary, p.binary, 2, True)
    p1, p2 = sp.pool(1), sp.pool(2)
    ru = len(p.unary) * (p2 - p1)
    binbase = p2 + ru
    per_u = p1 * 5
    begin, end = {"pool": (0, p2), "unary": (p2, p2 + ru),
                  "binary": (binbase + 40 * per_u, binbase + 104 * per_u),
                  "binary_ragged": (binbase + 33 * per_u + 17, binbase + 70 * per_u + 3)}[part]
    keep = 1000
    gi, gs = _screen(eng, p.y, keep, begin, end)
    oi, os_ = sp.sis(p.X, p.y, keep, begin=begin, end=end)
    assert_topk_parity(sp, p.X, p.y, gi, gs, oi, os_, keep)


def test_screen_c3_shape_slices():
    """n = 2000, d = 20 (the rung-3 workload's shape): a slice of the stored
    pool, of the unary block and of the binary block, in the default launch."""
    p = I.config3()
    print("[screen] C3 slices", flush=True)
    eng = _engine(p)
    sp = O.Space(20, p.unary, p.binary, 2, True)
    p1, p2 = sp.pool(1), sp.pool(2)
    binbase = p2 + 3 * (p2 - p1)
    per_u = p1 * 5
    keep = 400
    for begin, end in [(p1, p1 + 60000), (p2 + 5000, p2 + 35000),
                       (binbase + 1000 * per_u, binbase + 1064 * per_u)]:
        gi, gs = _screen(eng, p.y, keep, begin, end)
        oi, os_ = sp.sis(p.X, p.y, keep, begin=begin, end=end)
        assert_topk_parity(sp, p.X, p.y, gi, gs, oi, os_, keep)


def test_screen_deterministic_across_grids_and_tiles():
    p = I.tiny(9, n=300, d=6, dist="lognormal", rect=True)
    eng = _engine(p)
    ref = None
    for grid, tile in [(0, 0), (7, 0), (64, 1), (3, 2), (0, 1)]:
        gi, gs = _screen(eng, p.y, 500, grid=grid, tile=tile)
        if ref is None:
            ref = (gi, gs)
        else:
            assert np.array_equal(gi, ref[0]) and np.array_equal(gs, ref[1]), (grid, tile)


def test_topk_smaller_k_is_prefix():
    p = I.tiny(9, n=300, d=6, dist="lognormal", rect=True)
    eng = _engine(p)
    r64 = torch.as_tensor(p.y, dtype=torch.float64, device=eng.dev)
    ids, sc, cnt = eng.screen(r64, 700)
    ids2, sc2, cnt2 = eng.screen(r64, 700, k=37)
    torch.cuda.synchronize()
    assert int(cnt2.item()) == 37
    assert torch.equal(ids[:37], ids2) and torch.equal(sc[:37], sc2)


# ---------------------------------------------------------------------- SO

def _l0_gpu(F, y, D):
    import ctypes
    from paper_2410_01752_amd import _lib as L
    dev = torch.device("cuda:0")
    n, m = F.shape
    Ft = torch.as_tensor(np.ascontiguousarray(F.T), device=dev)
    yt = torch.as_tensor(y, dtype=torch.float64, device=dev)
    tup = torch.empty(3, dtype=torch.int32, device=dev)
    sse = torch.empty(1, dtype=torch.float64, device=dev)
    coef = torch.empty(4, dtype=torch.float64, device=dev)
    res = torch.empty(n, dtype=torch.float64, device=dev)
    st = torch.empty(4, dtype=torch.float64, device=dev)
    nb = L.lib().sisso_l0_workspace_size(m, n, D)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    L.check(L.lib().sisso_l0_search(Ft.data_ptr(), m, n, n, yt.data_ptr(), D, 1e-10, tup.data_ptr(),
                                    sse.data_ptr(), coef.data_ptr(), res.data_ptr(), st.data_ptr(),
                                    ws.data_ptr(), nb, L.stream_handle()), "l0")
    torch.cuda.synchronize()
    return (tup[:D].cpu().numpy(), float(sse.item()), coef[:D + 1].cpu().numpy(), res.cpu().numpy(),
            st.cpu().numpy())


@pytest.mark.parametrize("D", [1, 2, 3])
@pytest.mark.parametrize("seed", [0, 1])
def test_l0_matches_oracle(D, seed):
    rng = np.random.default_rng(seed)
    n, m = 150, 45
    F = rng.lognormal(size=(n, m))
    y = 1.3 * F[:, 4] - 0.8 * F[:, 17] + 0.5 * F[:, 30] + 0.3 * rng.normal(size=n)
    ref = O.l0(F, y, D)
    tup, sse, coef, res, st = _l0_gpu(F, y, D)
    near_tie = ref.runner_up <= ref.sse * (1 + 1e-9)
    if not near_tie:
        assert list(tup) == list(ref.best)
    assert abs(sse - ref.sse) <= 1e-6 * ref.sse
    assert np.allclose(coef, ref.coef, rtol=1e-6, atol=1e-9)
    assert int(st[2]) == math.comb(m, D)
    assert abs(st[0] - math.sqrt(ref.sse / n)) <= 1e-6 * math.sqrt(ref.sse / n)


def test_l0_singular_and_exact_fit():
    rng = np.random.default_rng(3)
    a, b, c = rng.uniform(1, 2, size=(3, 60))
    F = np.column_stack([a, b, a + b, c, rng.uniform(1, 2, size=60)])
    y = 2.0 - a + 3.0 * c
    tup, sse, coef, res, st = _l0_gpu(F, y, 3)
    ref = O.l0(F, y, 3)
    syy = np.sum((y - y.mean()) ** 2)
    assert sse <= 1e-13 * syy                       # S_yy - fit: rounding level
    assert st[0] <= 1e-12 * np.sqrt(syy)            # explicit residual
    assert int(st[3]) >= 1                          # (a, b, a+b) skipped
    assert list(tup) == list(ref.best)


# --------------------------------------------------------------------- fit

def _compare_fit(p, res_gpu, res_or):
    assert len(res_gpu) == len(res_or)
    for g, o in zip(res_gpu, res_or):
        print(f"  t={g.t}: gpu best {list(g.best_ids)} rmse {g.rmse:.6g} | oracle best "
              f"{list(o.best_ids)} rmse {o.rmse:.6g}", flush=True)
        assert set(g.sub_ids.tolist()) == set(o.sub_ids.tolist())
        near_tie = o.runner_up <= o.sse * (1 + 1e-9)
        if not near_tie:
            assert list(g.best_ids) == list(o.best_ids)
        assert abs(g.rmse - o.rmse) <= 1e-6 * o.rmse + 1e-12


@pytest.mark.parametrize("name", ["C1", "tiny_rect", "C2"])
def test_fit_matches_oracle(name):
    p = {"C1": I.config1, "tiny_rect": lambda: I.tiny(5, n=24, d=3, rect=True, k=6, dmax=3),
         "C2": I.config2}[name]()
    print(f"[fit] {name}", flush=True)
    eng = _engine(p)
    rg = eng.fit(p.k, p.dmax)
    ro = O.fit(p.X, p.y, p.unary, p.binary, p.rung, p.rect, p.k, p.dmax)
    _compare_fit(p, rg, ro)


def test_c1_gpu_recovers_planted_terms():
    p = I.config1()
    eng = _engine(p)
    st = eng.fit(p.k, p.dmax)[1]
    sp = O.Space(5, p.unary, p.binary, 2)
    V, _ = sp.eval(p.X, st.best_ids)
    planted = [I.eval_tree(t, p.X) for t in p.planted]
    for a in range(2):
        assert max(abs(np.corrcoef(V[:, a], pl)[0, 1]) for pl in planted) > 1 - 1e-12
    assert 0.005 < st.rmse < 0.015

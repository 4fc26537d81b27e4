"""The whole rung 3 of eq. feature-exp (Sec. 2.1) screened on the GPU (space
mode rect = 2: the next TRI level, generated in registers), and the threshold
alternative of Sec. 2.2, against the FP64 oracle: |corr| within 1e-6 and
identical top lists up to ties at the cutoff (as the other parity tests);
identical threshold lists and threshold fits."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2410_01752_amd import inputs as I

from test_gpu_parity import _screen, assert_topk_parity

pytestmark = pytest.mark.gpu

UN, BI = ["sq"], ["add", "mul"]


def _engine(X, y, unary, binary, rect=2):
    from paper_2410_01752_amd.fit import Engine
    return Engine(X, y, unary, binary, 2, rect)


def test_full_rung3_tiny_whole_space():
    rng = np.random.default_rng(12)
    X = rng.lognormal(0.0, 0.5, size=(40, 3))
    y = X[:, 0] * X[:, 1] ** 2 + (X[:, 2] + X[:, 0]) * X[:, 1] + 0.01 * rng.normal(size=40)
    print("[rung3 full] tiny whole space", flush=True)
    eng = _engine(X, y, UN, BI)
    sp = O.Space(3, UN, BI, 2, 2)
    assert eng.total == sp.total
    for keep in (300, 2000):
        gi, gs = _screen(eng, y, keep)
        oi, os_ = sp.sis(X, y, keep)
        assert_topk_parity(sp, X, y, gi, gs, oi, os_, keep)


def test_full_rung3_ops1_tiny_ragged_ranges():
    p = I.tiny(9, n=60, d=3, dist="lognormal", rect=False)
    eng = _engine(p.X, p.y, p.unary, p.binary)
    sp = O.Space(3, p.unary, p.binary, 2, 2)
    bb = eng.binary_base()
    for b, e in [(bb, bb + 7001), (bb + 123457, bb + 200003), (sp.total - 50000, sp.total)]:
        print(f"[rung3 full] range [{b}, {e})", flush=True)
        gi, gs = _screen(eng, p.y, 400, b, e)
        oi, os_ = sp.sis(p.X, p.y, 400, begin=b, end=e)
        assert_topk_parity(sp, p.X, p.y, gi, gs, oi, os_, 400)


def test_full_rung3_slices_at_the_workload_size():
    """n = 2000, d = 20: slices of N_2 x P_2 (1.76e13 candidates): pairs of
    the first new u with P_1, pairs inside N_2 x N_2, and the block's last
    ids (above 2^44)."""
    p = I.config3()
    print("[rung3 full] n = 2000, d = 20", flush=True)
    eng = _engine(p.X, p.y, p.unary, p.binary)
    sp = O.Space(20, p.unary, p.binary, 2, 2)
    bb = eng.binary_base()
    p1 = sp.pool(1)
    j = p1 + 30                     # pairs (j, i) for i < j: j - 1 pairs of 5 slots
    start_j = bb + 5 * (j * (j - 1) // 2 - p1 * (p1 - 1) // 2)
    j2 = 2_000_000                  # deep inside N_2: i runs over P_1 and N_2
    start_j2 = bb + 5 * (j2 * (j2 - 1) // 2 - p1 * (p1 - 1) // 2)
    slices = [(start_j, start_j + 5 * 9 * j),                     # 9 whole rows j .. j+8 (i over P_1 and N_2)
              (start_j2 + 5 * 1_000_000, start_j2 + 5 * 1_008_000),
              (sp.total - 40_000, sp.total)]
    for b, e in slices:
        print(f"[rung3 full] slice [{b}, {e})", flush=True)
        gi, gs = _screen(eng, p.y, 300, b, e)
        oi, os_ = sp.sis(p.X, p.y, 300, begin=b, end=e)
        assert_topk_parity(sp, p.X, p.y, gi, gs, oi, os_, 300)
    assert slices[-1][0] > 2 ** 44


def test_threshold_selection_matches_oracle():
    rng = np.random.default_rng(12)
    X = rng.lognormal(0.0, 0.5, size=(40, 3))
    y = X[:, 0] * X[:, 1] ** 2 + 0.3 * rng.normal(size=40)
    eng = _engine(X, y, UN, BI)
    sp = O.Space(3, UN, BI, 2, 2)
    oi, os_ = sp.sis(X, y, 3000)
    tau = float(os_[150])
    r64 = torch.as_tensor(y, dtype=torch.float64, device=eng.dev)
    eng.screen(r64, 2048)
    ids, sc, cnt = eng.select_threshold(tau, 2048)
    c = int(cnt.item())
    got = ids[:c].cpu().numpy()
    gsc = sc[:c].cpu().numpy().astype(np.float64)
    omap = dict(zip(oi.tolist(), os_.tolist()))
    want = set(oi[os_ >= tau].tolist())
    assert np.all(gsc >= np.float32(tau)) and np.all(np.diff(gsc) <= 0)
    assert max(abs(omap[i] - s) for i, s in zip(got.tolist(), gsc.tolist())) <= 1e-6
    for i in set(got.tolist()) ^ want:                       # only ties with the threshold may differ
        assert abs(omap[i] - tau) <= 1e-6, (i, omap[i], tau)
    assert len(want) > 100
    # lists that filled above the threshold are reported, not silently cut
    from paper_2410_01752_amd import _lib as L
    eng.screen(r64, 20)
    with pytest.raises(L.SissoError):
        eng.select_threshold(tau, 2048)


def test_threshold_fit_matches_oracle():
    p = I.tiny(30, n=50, d=3, dist="lognormal", rect=False, k=5, dmax=2)
    from paper_2410_01752_amd.fit import Engine
    eng = Engine(p.X, p.y, p.unary, p.binary, 2, False)
    tau = 0.6
    res = eng.fit(40, 2, keep0=2048, threshold=tau)
    ref = O.fit_threshold(p.X, p.y, p.unary, p.binary, 2, False, tau, 2048, 40, 2)
    for g, (new, sub, best, sse) in zip(res, ref):
        assert sorted(g.sub_ids.tolist()) == sorted(sub.tolist())
        assert list(g.best_ids) == list(best)
        assert abs(g.sse - sse) <= 1e-6 * sse

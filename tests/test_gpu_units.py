"""Dimensional analysis on the GPU (Sec. 2.1; the dimensionality option of
Sec. 3.3) against the oracle's units: pool units and validity column by
column, screening of the stored pools, of the one-sided rung-3 slice (unary
and binary blocks) and of the whole next level in the FP32 form, the 16-bit
form against the FP32 form, and whole fits.  Tolerances as the unweighted
parity tests (|corr| within 1e-6, identical lists up to ties at the
cutoff)."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2410_01752_amd import inputs as I

from test_gpu_parity import _screen, assert_topk_parity
from test_gpu_bf16 import _both, _check

pytestmark = pytest.mark.gpu

FULLU = ["sq", "cube", "sqrt", "inv", "exp", "nexp", "log", "sin"]
BI = ["add", "sub", "mul", "div"]


def _engine(X, y, unary, binary, levels, rect, units):
    from paper_2410_01752_amd.fit import Engine
    return Engine(X, y, unary, binary, levels, rect, dimensionality=units)


def test_pool_units_and_validity_match_oracle():
    rng = np.random.default_rng(41)
    X = rng.uniform(0.5, 4.0, size=(60, 5))
    y = X[:, 0] / X[:, 1] + rng.normal(0, 0.01, 60)
    units = ["m", "s", "m", "1", "kg"]
    print("[units] pools", flush=True)
    eng = _engine(X, y, FULLU, BI, 2, True, units)
    sp = O.Space(5, FULLU, BI, 2, True, units)
    pL = sp.pool(2)
    torch.cuda.synchronize()
    got = eng.units.view(pL, 8).cpu().numpy()
    valid = eng.stats.view(pL, 8)[:, 6].cpu().numpy() != 0
    _, ovalid = sp.eval(X, range(pL))
    assert np.array_equal(valid, ovalid)
    for fid in range(pL):
        ok, u = sp.units(fid)
        if ok:
            assert np.array_equal(got[fid, :3] / 16.0, u) and not got[fid, 3:].any(), fid
        else:
            assert got[fid, 0] == -32768, fid


@pytest.mark.parametrize("rect", [1, 2])
def test_units_screen_matches_oracle(rect):
    rng = np.random.default_rng(42 + rect)
    X = rng.uniform(0.5, 4.0, size=(50, 4))
    y = (X[:, 0] + X[:, 2]) / X[:, 1] + 0.2 * np.exp(X[:, 3]) + rng.normal(0, 0.02, 50)
    units = ["m", "s", "m", "1"]
    un = FULLU if rect == 1 else ["sq", "exp"]
    bi = BI if rect == 1 else ["add", "mul"]
    print(f"[units] screen rect={rect}", flush=True)
    eng = _engine(X, y, un, bi, 2, rect, units)
    sp = O.Space(4, un, bi, 2, rect, units)
    pL = sp.pool(2)
    bb = eng.binary_base()
    ranges = [(0, sp.total)] if sp.total < 400000 else [(0, pL), (pL, bb), (bb, bb + 150000),
                                                           (sp.total - 100000, sp.total)]
    for b, e in ranges:
        gi, gs = _screen(eng, y, 400, b, e)
        oi, os_ = sp.sis(X, y, 400, begin=b, end=e)
        assert_topk_parity(sp, X, y, gi, gs, oi, os_, 400)
    # the units remove candidates the plain space would rank: lists differ
    plain = O.Space(4, un, bi, 2, rect)
    pi, _ = plain.sis(X, y, 400)
    oi, _ = sp.sis(X, y, 400)
    assert set(pi.tolist()) != set(oi.tolist())


def test_units_slice_at_workload_size_and_16bit_form():
    """n = 2000, d = 20 with five unit groups: FP32 slice parity against the
    oracle, and the 16-bit form's list equal to the FP32 form's."""
    p = I.config3()
    units = ["u%d" % (i % 5) for i in range(20)]
    print("[units] n = 2000, d = 20", flush=True)
    eng = _engine(p.X, p.y, p.unary, p.binary, 2, True, units)
    sp = O.Space(20, p.unary, p.binary, 2, True, units)
    bb = eng.binary_base()
    per_u = sp.pool(1) * 5
    # u = 400,000 and 400,001 break the rules (their slices are empty), 400,002 .. 400,004 not
    for b, e in [(bb, bb + 3 * per_u), (bb + 400_000 * per_u, bb + 400_000 * per_u + 5 * per_u),
                 (sp.total - 2 * per_u, sp.total)]:
        print(f"[units] slice [{b}, {e})", flush=True)
        gi, gs = _screen(eng, p.y, 300, b, e)
        oi, os_ = sp.sis(p.X, p.y, 300, begin=b, end=e)
        assert len(oi) > 0
        assert_topk_parity(sp, p.X, p.y, gi, gs, oi, os_, 300)
    # a u column that breaks the rules gives no candidate at all
    assert not sp.units(int(sp.pool(1)) + 400_000)[0]
    gi, _ = _screen(eng, p.y, 300, bb + 400_000 * per_u, bb + 400_001 * per_u)
    assert len(gi) == 0
    end = bb + 20_000 * per_u
    out = _both(eng, p.y, 1000, 4000, bb, end)
    _check(out, 1000)
    fi, _ = out["fp32"]
    for fid in fi[:50]:
        assert sp.units(int(fid))[0]


def test_units_fit_matches_oracle():
    rng = np.random.default_rng(44)
    X = rng.uniform(0.5, 4.0, size=(80, 5))
    units = ["m", "s", "m", "1", "kg"]
    y = (X[:, 0] + X[:, 2]) / X[:, 1] + 0.5 * X[:, 4] * X[:, 3] ** 2 + rng.normal(0, 0.01, 80)
    print("[units] fit", flush=True)
    eng = _engine(X, y, FULLU, BI, 2, False, units)
    res = eng.fit(10, 2)
    ref = O.fit(X, y, FULLU, BI, 2, False, 10, 2, dimensionality=units)
    for g, o in zip(res, ref):
        assert sorted(g.sub_ids.tolist()) == sorted(o.sub_ids.tolist())
        assert list(g.best_ids) == list(o.best_ids)
        assert math.isclose(g.sse, o.sse, rel_tol=1e-9)


def test_units_refused_by_the_learned_form():
    from paper_2410_01752_amd import _lib as L
    import ctypes
    p = I.tiny(5, n=40, d=3, dist="lognormal", rect=True)
    eng = _engine(p.X, p.y, p.unary, p.binary, 2, True, ["a", "b", "a"])
    r64 = torch.as_tensor(p.y, device=eng.dev)
    eng.prepare_residual(r64)
    a = eng.score_args(100)
    enc = torch.empty(1 << 20, dtype=torch.uint8, device=eng.dev)
    bb = eng.binary_base()
    assert L.lib().sisso_encode_operands(ctypes.byref(eng.space), ctypes.byref(a), 0, 1, L.ptr(enc),
                                         L.stream_handle(eng.dev)) == 5      # SISSO_E_UNSUPPORTED

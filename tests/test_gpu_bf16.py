"""BF16-MFMA screening with FP32 band rescore, against the plain FP32 path.

Recall of the BF16 form's top-K' against the FP32 form's top-K' must be
>= 0.99 (ids missing from the BF16 list may only be FP32 near-ties of the
cutoff beyond that), and every score the BF16 form returns is the FP32
path's score of that id, bit for bit (the band is rescored with the FP32
kernel's arithmetic).  The FP32 path itself is checked against the oracle in
test_gpu_parity.py.
"""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2410_01752_amd import inputs as I

pytestmark = pytest.mark.gpu


def _engine(p):
    from paper_2410_01752_amd.fit import Engine
    return Engine(p.X, p.y, p.unary, p.binary, p.rung, p.rect)


def _both(eng, r, keep, band, begin=None, end=None):
    r64 = torch.as_tensor(r, dtype=torch.float64, device=eng.dev)
    begin = eng.binary_base() if begin is None else begin
    out = {}
    for prec in ("fp32", "bf16"):
        ids, sc, cnt = eng.screen(r64, keep, None, begin=begin, end=end, precision=prec, band=band)
        torch.cuda.synchronize()
        c = int(cnt.item())
        out[prec] = (ids[:c].cpu().numpy(), sc[:c].cpu().numpy())
    return out


def recall_of(out, tol=1e-6):
    """Top-K' recall of the BF16 form against the FP32 form.  A FP32 member that
    the BF16 list lacks counts as found when its score is within tol of the
    cutoff: such candidates tie with the cutoff (typically duplicate features
    with bit-identical scores) and either choice is a valid top-K'."""
    fi, fs = out["fp32"]
    bi, bs = out["bf16"]
    got = set(bi.tolist())
    cutoff = fs[-1]
    found = sum(1 for i, s in zip(fi.tolist(), fs.tolist()) if i in got or s <= cutoff + tol)
    raw = sum(1 for i in fi.tolist() if i in got)
    return found / len(fi), raw / len(fi)


def _check(out, keep, min_recall=0.99):
    fi, fs = out["fp32"]
    bi, bs = out["bf16"]
    assert len(bi) == len(fi)
    fmap = dict(zip(fi.tolist(), fs.tolist()))
    bmap = dict(zip(bi.tolist(), bs.tolist()))
    for i in bmap:
        if i in fmap:
            assert bmap[i] == fmap[i], (i, bmap[i], fmap[i])        # bit-identical rescore
    # the BF16 list is sorted and never ranks below the FP32 cutoff
    assert np.all(np.diff(bs) <= 0) and bs[-1] >= fs[-1] - 1e-6
    recall, raw = recall_of(out)
    print(f"  recall {recall:.4f} (raw {raw:.4f}, {len(fi)} kept)", flush=True)
    assert recall >= min_recall
    return recall


def test_bf16_recall_rung3_small():
    p = I.tiny(9, n=300, d=6, dist="lognormal", rect=True)
    print("[bf16] n=300 d=6 full binary block", flush=True)
    eng = _engine(p)
    _check(_both(eng, p.y, 500, 2000), 500)


def test_bf16_recall_c3_slice():
    """n = 2000, d = 20: 1024 operands u of the binary block (5.3e6 candidates)."""
    p = I.config3()
    print("[bf16] C3 slice", flush=True)
    eng = _engine(p)
    sp = O.Space(20, p.unary, p.binary, 2, True)
    bb = eng.binary_base()
    per_u = sp.pool(1) * 5
    out = _both(eng, p.y, 400, 1600, begin=bb + 2000 * per_u, end=bb + 3024 * per_u)
    _check(out, 400)


@pytest.mark.parametrize("keep,band", [(2048, 7168), (700, 3000)])
def test_bf16_band_wider_than_block_lists(keep, band):
    """A band above SISSO_MAX_KEEP: each block keeps its best 2048 by BF16
    score, publishes no grid-wide bound, and the grid-wide merge takes the
    best `band` for the exact rescore (C3 shape, 1024 u operands)."""
    p = I.config3()
    print(f"[bf16] C3 slice keep {keep} band {band}", flush=True)
    eng = _engine(p)
    sp = O.Space(20, p.unary, p.binary, 2, True)
    bb = eng.binary_base()
    per_u = sp.pool(1) * 5
    out = _both(eng, p.y, keep, band, begin=bb + 500 * per_u, end=bb + 1524 * per_u)
    assert _check(out, keep) == 1.0


def test_bf16_rescored_scores_match_oracle():
    """The rescored list of the BF16 form is FP32-exact: within 1e-6 of the oracle."""
    p = I.tiny(9, n=300, d=6, dist="lognormal", rect=True)
    eng = _engine(p)
    sp = O.Space(6, p.unary, p.binary, 2, True)
    out = _both(eng, p.y, 300, 1200)
    bi, bs = out["bf16"]
    ref = np.array([sp.score_range(p.X, p.y, int(i), int(i) + 1)[0] for i in bi[:120]])
    assert np.max(np.abs(ref - bs[:120])) <= 1e-6


def test_bf16_fit_matches_fp32_fit():
    p = I.tiny(5, n=200, d=5, dist="lognormal", rect=True, k=8, dmax=3)
    eng = _engine(p)
    a = eng.fit(p.k, p.dmax, precision="fp32")
    b = eng.fit(p.k, p.dmax, precision="bf16", band=0)
    for x, y in zip(a, b):
        assert list(x.best_ids) == list(y.best_ids)
        assert abs(x.rmse - y.rmse) <= 1e-9 * x.rmse


def test_autotuned_shapes_give_identical_results(tmp_path):
    from paper_2410_01752_amd import autotune as A
    p = I.tiny(9, n=300, d=6, dist="lognormal", rect=True)
    eng = _engine(p)
    cache = A.Cache(str(tmp_path / "at.json"))
    for form in ("fp32", "bf16"):
        ch = A.tune_engine(eng, form=form, keep=300, band=1200, sample_tiles=64, cache=cache)
        assert cache.get(A.cache_key(*A.device_key(), "k_score_rect_bf16" if form == "bf16" else "k_score_rect",
                                     form, eng.n)) is not None
        r64 = torch.as_tensor(p.y, dtype=torch.float64, device=eng.dev)
        a = eng.screen(r64, 300, None, precision=form, band=1200)
        b = eng.screen(r64, 300, None, precision=form, band=1200, tile=ch.tile, grid=ch.grid)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # the stored-column pass: its tuned block count gives the default list
    r64 = torch.as_tensor(p.y, dtype=torch.float64, device=eng.dev)
    bb = eng.binary_base()
    a = eng.screen(r64, 300, None, begin=0, end=bb)
    torch.cuda.synchronize()
    a = (a[0].clone(), a[1].clone())
    cc = A.tune_columns(eng, keep=300, cache=cache, shapes=[(0, g) for g in (0, 1, 7, 4096)])
    assert eng.col_grid == cc.grid and len(cc.timings) == 4
    for g in (1, 7, 4096):
        eng.col_grid = g
        b = eng.screen(r64, 300, None, begin=0, end=bb)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    eng.col_grid = 0


def _a256(x):
    return (x + 255) // 256 * 256


def _band_of(eng, band):
    """The BF16 band of the last screen (ids and BF16 scores, before the exact
    rescore), read from the BF16 workspace: column sums of both sides, then
    band ids (int64), band scores (float32) and the band count."""
    s = eng.space
    vcols, ucols = int(s.pool[eng.levels - 1]), int(s.pool[eng.levels] - s.pool[eng.levels - 1])
    w = eng._ws["bf16"]
    o_id = _a256(vcols * 2 * 16) + _a256(ucols * 8)
    o_sc = o_id + _a256(band * 8)
    o_ct = o_sc + _a256(band * 4)
    c = int(w[o_ct:o_ct + 4].view(torch.int32).item())
    ids = w[o_id:o_id + 8 * c].view(torch.int64).cpu().numpy()
    sc = w[o_sc:o_sc + 4 * c].view(torch.float32).cpu().numpy()
    order = np.lexsort((ids, -sc))
    return ids[order], sc[order]


def _redo_flag(eng, band):
    """1 if the last read screen's append overflowed its workspace and the
    pass was scored again in lists: the band lists' header follows the band
    count; its redo flag sits after the 64-bit append counter (byte 48)."""
    s = eng.space
    vcols, ucols = int(s.pool[eng.levels - 1]), int(s.pool[eng.levels] - s.pool[eng.levels - 1])
    o = _a256(vcols * 2 * 16) + _a256(ucols * 8) + _a256(band * 8) + _a256(band * 4) + 256
    return int(eng._ws["bf16"][o + 56:o + 60].view(torch.int32).item())


@pytest.mark.parametrize("case", ["ragged_n300", "persistent_grid", "c3_shape_n2000", "c3_full_block"])
def test_bf16_moments_read_equals_plain_screen(case):
    """A screen that reads the stored residual-independent moments gives the
    same BF16 band (ids and BF16 scores, bit for bit) and the same rescored
    list as a plain screen of the same residual; so does the screen that
    writes them.  Cases: n = 300 (a ragged last chunk of samples, ragged u and v
    tiles), a grid of 3 blocks sweeping every u tile, n = 2000 with d = 12, and the
    whole C3 binary block at the bench's keep, band and tuned grid (41,434 u tiles;
    the read form sizes its own grid)."""
    if case == "ragged_n300":
        p, keep, band, grid = I.tiny(9, n=300, d=6, dist="lognormal", rect=True), 300, 1200, 0
    elif case == "persistent_grid":
        p, keep, band, grid = I.tiny(4, n=77, d=5, dist="lognormal", rect=True), 200, 800, 3
    elif case == "c3_shape_n2000":
        p, keep, band, grid = I.tiny(21, n=2000, d=12, dist="lognormal", rect=True), 1000, 4000, 0
    else:       # the bench's workload: 1.37e10 candidates, 69 GB of moments, the bench's band
        p, keep, band, grid = I.config3(), 2048, 7168, 256
    print(f"[bf16 moments] {case}", flush=True)
    eng = _engine(p)
    assert eng.bf16_moments_buffer() is not None
    rng = np.random.default_rng(77)
    y64 = torch.as_tensor(p.y, dtype=torch.float64, device=eng.dev)
    r2 = torch.as_tensor(p.y - 0.3 * p.X[:, 0] + 0.1 * rng.standard_normal(p.y.shape[0]),
                         dtype=torch.float64, device=eng.dev)
    excl = torch.as_tensor(np.sort(rng.choice(eng.total, 50, replace=False)), dtype=torch.int64,
                           device=eng.dev)

    def run(r, mode, ex=None):
        ids, sc, cnt = eng.screen(r, keep, ex, precision="bf16", band=band, grid=grid, moments=mode)
        torch.cuda.synchronize()
        c = int(cnt.item())
        return (ids[:c].cpu().numpy(), sc[:c].cpu().numpy()), _band_of(eng, band)

    plain_y = run(y64, "none")
    whole_y = run(y64, "write_whole")          # the one-call WRITE screen
    write_y = run(y64, "write")                # images, moments pass, READ screen
    plain_r = run(r2, "none", excl)
    read_r = run(r2, "read", excl)
    read_y = run(y64, "read")
    redo_default = _redo_flag(eng, band)
    # the bound's sampling step: every u tile (the tightest bound), and every
    # sixteenth (at C3 more candidates reach that bound than the workspace
    # holds, and the pass is scored again in lists)
    steps = {}
    try:
        for step in ("1", "16"):
            os.environ["SISSO_BF16_BOUND_STEP"] = step
            steps[step] = run(y64, "read"), _redo_flag(eng, band)
    finally:
        os.environ.pop("SISSO_BF16_BOUND_STEP", None)
    if case == "c3_full_block":
        assert redo_default == 0 and steps["1"][1] == 0 and steps["16"][1] == 1
    for a, b in ((plain_y, whole_y), (plain_y, write_y), (plain_r, read_r), (plain_y, read_y),
                 (plain_y, steps["1"][0]), (plain_y, steps["16"][0])):
        (ia, sa), (ba, bsa) = a
        (ib, sb), (bb_, bsb) = b
        assert len(ba) > 0
        assert np.array_equal(ba, bb_) and np.array_equal(bsa, bsb)      # the BF16 band, bit for bit
        assert np.array_equal(ia, ib) and np.array_equal(sa, sb)         # the rescored list


def test_bf16_fit_with_moments_equals_fit_without():
    """A BF16 fit whose later passes read the first pass's moments gives the
    tuples and RMSE of the BF16 fit that recomputes them and of the FP32 fit."""
    p = I.tiny(6, n=400, d=6, dist="lognormal", rect=True, k=10, dmax=3)
    eng = _engine(p)
    a = eng.fit(p.k, p.dmax, precision="bf16", moments="off")
    assert eng.bf16_moments is None
    b = eng.fit(p.k, p.dmax, precision="bf16", moments="auto")
    assert eng.bf16_moments is not None
    c = eng.fit(p.k, p.dmax, precision="fp32")
    assert len(a) == len(b) == len(c) == p.dmax
    for x, y, z in zip(a, b, c):
        assert list(x.best_ids) == list(y.best_ids) == list(z.best_ids)
        assert x.rmse == y.rmse
        assert abs(x.rmse - z.rmse) <= 1e-9 * z.rmse


def test_bf16_moments_argument_errors():
    """Moments need the whole binary block (a WRITE over part of it would leave
    pairs unwritten that a later READ reads); unknown modes and policies are
    rejected before any launch."""
    from paper_2410_01752_amd import _lib as L
    p = I.tiny(9, n=300, d=6, dist="lognormal", rect=True)
    eng = _engine(p)
    y64 = torch.as_tensor(p.y, dtype=torch.float64, device=eng.dev)
    bb = eng.binary_base()
    with pytest.raises(L.SissoError):
        eng.screen(y64, 100, None, begin=bb + 5, precision="bf16", band=400, moments="write")
    with pytest.raises(L.SissoError):
        eng.screen(y64, 100, None, precision="bf16", band=400, moments="sometimes")
    with pytest.raises(L.SissoError):
        eng.fit(5, 2, precision="bf16", moments="always")
    # the plain form ignores moments="none"; a whole-block write then read works
    a = eng.screen(y64, 100, None, precision="bf16", band=400, moments="write")
    b = eng.screen(y64, 100, None, precision="bf16", band=400, moments="read")
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_small_spread_differences_reach_the_list():
    """Valid differences whose spread is about 1e-3 of their operands' rms fill
    the top of the list: x1 = 1 + 1e-3 N(0, 1) and y = x0 (x1^2 - 1) + noise,
    so (x1 x0) x1 - x0, x1 x0 - x0 and their regroupings all correlate with y
    to 0.9999.  Their 16-bit variance is rounding noise (the conditioning test
    flags them) and they are scored exactly: the 16-bit form's list equals the
    FP32 form's list id for id and bit for bit (the exact rules call them
    valid, their sd being above 1e-5 of the operands' rms; a screen that cut
    them at 1e-2 lost them)."""
    rng = np.random.default_rng(41)
    n, d = 500, 4
    X = rng.lognormal(0.0, 0.5, size=(n, d))
    X[:, 1] = 1.0 + 1e-3 * rng.normal(size=n)
    target = X[:, 0] * (X[:, 1] ** 2 - 1.0)
    y = 3.0 * target / target.std() + 0.05 * rng.normal(size=n)
    p = I.Problem("spread", X, y, list(I.OPS1["unary"]), list(I.OPS1["binary"]), 2, True, 10, 1, [], [], 0)
    print("[bf16] small-spread differences", flush=True)
    eng = _engine(p)
    sp = O.Space(d, p.unary, p.binary, 2, True)
    out = _both(eng, p.y, 200, 800)
    fi, fs = out["fp32"]
    bi, bs = out["bf16"]
    gap = 0
    for i in fi[:50]:
        op, a, b = sp.decode(int(i))
        if op != O.OPCODE["sub"]:
            continue
        V, ok = sp.eval(X, [int(i), a, b])
        ratio = V[:, 0].std() / np.sqrt(np.mean(V[:, 1:] ** 2, axis=0)).max()
        gap += int(ok.all() and 1e-5 < ratio < 1e-2)
    assert gap >= 10, gap
    assert np.array_equal(bi, fi) and np.array_equal(bs, fs)

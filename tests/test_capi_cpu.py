"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2410_01752_amd import _lib as L
from paper_2410_01752_amd import inputs as I
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sisso.h")).read()
    return sorted(set(re.findall(r"\b(sisso_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = L.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(L.EXPORTED) <= set(names)
    assert lib.sisso_version().decode().startswith("sisso-mi355x")


def test_space_init_validation():
    s = L.Space()
    s.d, s.levels, s.rect, s.n_unary, s.n_binary = 0, 2, 0, 0, 1
    s.binary[0] = 2
    assert L.lib().sisso_space_init(ctypes.byref(s)) == 2          # d < 1
    s.d, s.levels = 3, 3
    assert L.lib().sisso_space_init(ctypes.byref(s)) == 2          # levels > 2
    s.levels, s.n_binary = 2, 2
    s.binary[0] = s.binary[1] = 2
    assert L.lib().sisso_space_init(ctypes.byref(s)) == 2          # repeated op
    s.binary[1] = 7
    assert L.lib().sisso_space_init(ctypes.byref(s)) == 2          # unary code as binary
    assert L.lib().sisso_space_init(None) == 1


@pytest.mark.parametrize("d,ops,levels,rect", [
    (5, I.OPS1, 2, False), (10, I.FULL, 2, False), (20, I.OPS1, 2, True), (30, I.OPS1, 2, True),
    (3, I.OPS1, 2, True), (2, {"unary": [], "binary": ["add", "mul"]}, 2, False),
    (4, I.FULL, 1, True), (6, {"unary": ["log", "sin"], "binary": ["div"]}, 2, True)])
def test_space_counts_and_decode_match_oracle(d, ops, levels, rect):
    s = L.make_space(d, ops["unary"], ops["binary"], levels, rect)
    o = O.Space(d, ops["unary"], ops["binary"], levels, rect)
    assert s.total == o.total
    for l in range(levels + 1):
        assert s.pool[l] == o.pool(l)
    rng = np.random.default_rng(d)
    ids = list(range(min(o.total, 2000))) + [int(v) for v in rng.integers(0, o.total, 2000)]
    ids += [o.total - 1, int(s.pool[levels]) - 1, int(s.pool[levels])] if o.total > s.pool[levels] else []
    for fid in ids:
        assert L.decode(s, fid) == o.decode(fid), fid


def test_decode_ids_above_2_32():
    s = L.make_space(20, I.OPS1["unary"], I.OPS1["binary"], 2, True)
    o = O.Space(20, I.OPS1["unary"], I.OPS1["binary"], 2, True)
    for fid in [2 ** 32, 2 ** 32 + 12345, 2 ** 33 + 7, s.total - 5]:
        assert L.decode(s, fid) == o.decode(fid)
    with pytest.raises(L.SissoError):
        L.decode(s, s.total)


def test_argument_errors_before_launch():
    lib = L.lib()
    s = L.make_space(5, I.OPS1["unary"], I.OPS1["binary"], 2, False)
    a = L.ScoreArgs()
    a.n, a.keep = 50, 40
    # null pointers
    assert lib.sisso_expand_score(ctypes.byref(s), ctypes.byref(a), 0, 10, None, 0, None) == 1
    assert lib.sisso_topk(None, 0, 5, None, None, None, None) == 1
    assert lib.sisso_materialize_pools(ctypes.byref(s), None, 50, 50, None, 64, None, 50, None, None) == 1
    assert lib.sisso_l0_search(None, 10, 10, 10, None, 2, 1e-10, None, None, None, None, None, None, 0, None) == 1
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    # shapes
    assert lib.sisso_materialize_pools(ctypes.byref(s), fake, 1, 1, fake, 4, fake, 1, fake, None) == 2
    assert lib.sisso_materialize_pools(ctypes.byref(s), fake, 50, 50, fake, 50, fake, 50, fake, None) == 2  # ld32 % 4
    assert lib.sisso_l0_search(fake, 2, 10, 10, fake, 3, 1e-10, fake, fake, fake, fake, fake, fake, 1 << 20,
                               None) == 2                                              # m < D
    assert lib.sisso_l0_search(fake, 10, 10, 10, fake, 4, 1e-10, fake, fake, fake, fake, fake, fake, 1 << 20,
                               None) == 2                                              # D > 3
    assert lib.sisso_l0_search(fake, 10, 10, 10, fake, 2, 1e-10, fake, fake, fake, fake, fake, fake, 8,
                               None) == 4                                              # workspace
    assert lib.sisso_prepare_residual(fake, 1, fake, fake, None) == 2
    # ranges
    a.pool32 = a.stats = a.r32 = a.info = 0x1000
    a.ld32 = 64
    ws = lib.sisso_score_workspace_size(ctypes.byref(s), ctypes.byref(a))
    assert ws > 0
    assert lib.sisso_expand_score(ctypes.byref(s), ctypes.byref(a), 5, 5, fake, ws, None) == 3     # empty
    assert lib.sisso_expand_score(ctypes.byref(s), ctypes.byref(a), 0, s.total + 1, fake, ws, None) == 3
    assert lib.sisso_expand_score(ctypes.byref(s), ctypes.byref(a), 0, 10, fake, ws - 1, None) == 4
    a.keep = 0
    assert lib.sisso_expand_score(ctypes.byref(s), ctypes.byref(a), 0, 10, fake, ws, None) == 3
    a.keep, a.precision = 40, 7
    assert lib.sisso_expand_score(ctypes.byref(s), ctypes.byref(a), 0, 10, fake, ws, None) == 5
    a.precision = 0
    for bad in (-1, 16385):                      # the stored-column pass's block count
        a.col_grid = bad
        assert lib.sisso_score_workspace_size(ctypes.byref(s), ctypes.byref(a)) == 0
        assert lib.sisso_expand_score(ctypes.byref(s), ctypes.byref(a), 0, 10, fake, ws, None) == 3
        assert lib.sisso_expand_score_lists(ctypes.byref(s), ctypes.byref(a), 0, 10) == -1
    a.col_grid = 16384
    assert lib.sisso_score_workspace_size(ctypes.byref(s), ctypes.byref(a)) >= ws
    a.col_grid = 0
    assert lib.sisso_topk(fake, ws, 0, fake, fake, fake, None) == 3
    assert lib.sisso_subspace_update(fake, 50, fake, fake, fake, 40, fake, 50, fake, 50, fake, 1020, 20,
                                     fake, fake, fake, 1 << 30, None) == 2             # m_prev + k > 1024
    assert lib.sisso_sort_subspace(fake, 50, fake, 0, 50, fake, 50, fake, fake, None) == 2
    for st in range(8):
        assert lib.sisso_status_string(st)
    assert lib.sisso_topk_status(None, ws, fake, None) == 1
    assert lib.sisso_topk_status(fake, ws, None, None) == 1
    assert lib.sisso_topk_status(fake, 8, fake, None) == 4


def test_l0_outcome_reports_all_singular_searches():
    """sisso_l0_outcome reads a finished search's stats record (RMSE, R^2,
    tuples evaluated, tuples skipped): SISSO_E_NUMERIC (7) when every tuple
    was singular, SISSO_OK otherwise."""
    lib = L.lib()
    ok = np.array([0.1, 0.9, 79800.0, 12.0])
    none = np.array([np.nan, np.nan, 79800.0, 79800.0])
    assert lib.sisso_l0_outcome(ok.ctypes.data) == 0
    assert lib.sisso_l0_outcome(none.ctypes.data) == 7
    assert lib.sisso_l0_outcome(None) == 1


def test_noalloc_l0_argument_errors_before_launch():
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    cap = lib.sisso_l0_scratch_capacity()
    assert cap >= lib.sisso_l0_workspace_size(600, 2000, 3)
    assert lib.sisso_l0_search_noalloc(None, 10, 10, 10, fake, 2, 1e-10, fake, fake, fake, fake, fake, None) == 1
    assert lib.sisso_l0_search_noalloc(fake, 2, 10, 10, fake, 3, 1e-10, fake, fake, fake, fake, fake, None) == 2
    assert lib.sisso_l0_search_noalloc(fake, 10, 10, 10, fake, 4, 1e-10, fake, fake, fake, fake, fake, None) == 2
    assert lib.sisso_l0_workspace_size(1024, 4096, 3) > cap
    assert lib.sisso_l0_search_noalloc(fake, 1024, 4096, 4096, fake, 3, 1e-10, fake, fake, fake, fake, fake,
                                       None) == 4


def test_bf16_moments_size_and_argument_errors_before_launch():
    """The moments buffer holds 6 floats per pair of the padded 64 x 64 tiles of
    the slice's binary block, then the list of the candidates the screen
    scores exactly (a counter and one id per 1024 candidates of the block, at
    least 2^16 and at most 2^26), then the u side's FP16 image (four planes
    of 64 columns x 16 samples per 64-column tile and chunk of 16 samples),
    then 3 floats per pair of the same tiles (a pass's residual contractions),
    then the v side's FP16 image for the moments pass (six planes of 128
    columns x 16 samples per 128-column tile and chunk); a bad
    mode, a missing or short buffer and the usual range checks are reported
    before any launch."""
    lib = L.lib()
    s = L.make_space(20, I.OPS1["unary"], I.OPS1["binary"], 2, True)
    nu, nv = int(s.pool[2] - s.pool[1]), int(s.pool[1])
    tiles = ((nu + 63) // 64) * ((nv + 63) // 64)
    side = min(max(int(s.rect_binary) // 1024, 1 << 16), 1 << 26)
    a256 = lambda x: (x + 255) // 256 * 256
    mom = a256(tiles * 4 * 16 * 6 * 64 * 4)
    uimg = a256(((nu + 63) // 64) * ((100 + 15) // 16) * 4 * 64 * 16 * 2)
    vmimg = a256(((nv + 127) // 128) * ((100 + 15) // 16) * 6 * 128 * 16 * 2)
    cst = a256(tiles * 4 * 16 * 3 * 64 * 4)
    assert lib.sisso_bf16_moments_size(ctypes.byref(s), 100) == mom + a256(256 + 8 * side) + uimg + cst + vmimg
    assert lib.sisso_bf16_moments_size(ctypes.byref(s), 1) == 0
    plain = L.make_space(5, I.OPS1["unary"], I.OPS1["binary"], 2, False)
    assert lib.sisso_bf16_moments_size(ctypes.byref(plain), 100) == 0      # no slice
    a = L.ScoreArgs()
    a.n, a.keep, a.ld32 = 100, 40, 128
    a.pool32 = a.stats = a.r32 = a.info = 0x1000
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    band = 160
    bws = lib.sisso_bf16_workspace_size(ctypes.byref(s), ctypes.byref(a), band)
    ops = lib.sisso_bf16_operands_size(ctypes.byref(s), 100)
    mom = lib.sisso_bf16_moments_size(ctypes.byref(s), 100)
    assert bws > 0 and ops > 0
    b0 = int(s.pool[2] + s.rect_unary)
    sp, ap = ctypes.byref(s), ctypes.byref(a)

    def call(mode, m=fake, mb=mom, lo=b0, hi=s.total):
        return lib.sisso_bf16_screen_moments(sp, ap, fake, ops, band, lo, hi, m, mb, mode, fake, bws, None)

    assert call(3) == 3                                   # unknown mode
    assert call(-1) == 3
    assert call(L.MOMENTS_WRITE, m=None) == 1             # no buffer
    assert call(L.MOMENTS_READ, m=None) == 1
    assert call(L.MOMENTS_READ, mb=mom - 1) == 4          # short buffer
    assert call(L.MOMENTS_WRITE, lo=b0 - 1) == 3          # outside the binary block
    assert lib.sisso_bf16_screen_moments(sp, ap, None, ops, band, b0, s.total, fake, mom, 1, fake, bws,
                                         None) == 1       # no operands


def test_batched_l0_argument_errors_before_launch():
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    # the record layout matches the C struct: 8 + 4*4 + 7*8 + 8 bytes
    assert ctypes.sizeof(L.L0Problem) == 88
    assert lib.sisso_l0_search_batched(None, 4, 2, 100, 500, 1e-10, None, None) == 1
    assert lib.sisso_l0_search_batched(fake, 0, 2, 100, 500, 1e-10, None, None) == 2
    assert lib.sisso_l0_search_batched(fake, L.MAX_BATCH + 1, 2, 100, 500, 1e-10, None, None) == 2
    assert lib.sisso_l0_search_batched(fake, 4, 0, 100, 500, 1e-10, None, None) == 2
    assert lib.sisso_l0_search_batched(fake, 4, L.MAX_D + 1, 100, 500, 1e-10, None, None) == 2
    assert lib.sisso_l0_search_batched(fake, 4, 3, 2, 500, 1e-10, None, None) == 2        # m_max < D
    assert lib.sisso_l0_search_batched(fake, 4, 2, L.MAX_SUBSPACE + 1, 500, 1e-10, None, None) == 2
    assert lib.sisso_l0_search_batched(fake, 4, 2, 100, 1, 1e-10, None, None) == 2
    assert lib.sisso_l0_search_batched(fake, 4, 2, 100, L.MAX_N + 1, 1e-10, None, None) == 2
    assert lib.sisso_l0_search_batched(fake, 4, 2, 100, 500, -1.0, None, None) == 3
    assert lib.sisso_l0_search_batched(fake, 4, 2, 100, 500, 1.0, None, None) == 3
    assert lib.sisso_l0_search_batched(fake, 4, 2, 100, 500, float("nan"), None, None) == 3


def test_batched_subspace_steps_argument_errors_before_launch():
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    s2 = L.make_space(4, ["sq", "sqrt", "inv"], ["add", "sub", "mul", "div"], 2, False)
    # record layouts match the C structs
    assert ctypes.sizeof(L.EvalProblem) == 64
    assert ctypes.sizeof(L.SubspaceProblem) == 112
    assert ctypes.sizeof(L.SortProblem) == 56
    m = lib.sisso_materialize_ids_batched
    assert m(None, 1, fake, 4, 100, None, None) == 1
    assert m(ctypes.byref(s2), 1, None, 4, 100, None, None) == 1
    assert m(ctypes.byref(s2), 0, fake, 4, 100, None, None) == 2          # stored levels
    assert m(ctypes.byref(s2), 3, fake, 4, 100, None, None) == 2
    assert m(ctypes.byref(s2), 1, fake, 0, 100, None, None) == 2
    assert m(ctypes.byref(s2), 1, fake, L.MAX_BATCH + 1, 100, None, None) == 2
    assert m(ctypes.byref(s2), 1, fake, 4, 0, None, None) == 2
    assert m(ctypes.byref(s2), 1, fake, 4, L.MAX_KEEP + 1, None, None) == 2
    u = lib.sisso_subspace_update_batched
    assert u(None, 4, 200, 50, None, None) == 1
    assert u(fake, 0, 200, 50, None, None) == 2
    assert u(fake, 4, 0, 50, None, None) == 2
    assert u(fake, 4, L.MAX_SUBSPACE + L.MAX_KEEP + 1, 50, None, None) == 2
    assert u(fake, 4, 200, 0, None, None) == 2
    assert u(fake, 4, 200, L.MAX_SUBSPACE + 1, None, None) == 2
    s = lib.sisso_sort_subspace_batched
    assert s(None, 4, 100, None, None) == 1
    assert s(fake, 0, 100, None, None) == 2
    assert s(fake, 4, 0, None, None) == 2
    assert s(fake, 4, L.MAX_SUBSPACE + 1, None, None) == 2


def test_batched_argument_errors_before_launch():
    lib = L.lib()
    full = dict(unary=["sq", "sqrt", "inv"], binary=["add", "sub", "mul", "div"])
    s2 = L.make_space(4, full["unary"], full["binary"], 2, False)
    s1 = L.make_space(4, full["unary"], full["binary"], 1, False)
    sr = L.make_space(4, full["unary"], full["binary"], 2, True)
    fake = ctypes.c_void_p(0x1000)
    ws = lib.sisso_batch_workspace_size(ctypes.byref(s2), 8, 100)
    assert ws > 0
    # sizes grow with problems and keep; unsupported spaces give 0 / -1
    assert lib.sisso_batch_workspace_size(ctypes.byref(s2), 16, 100) > ws
    assert lib.sisso_batch_workspace_size(ctypes.byref(s2), 8, 200) > ws
    assert lib.sisso_batch_workspace_size(ctypes.byref(s1), 8, 100) == 0
    assert lib.sisso_batch_workspace_size(ctypes.byref(sr), 8, 100) == 0
    assert lib.sisso_batch_workspace_size(ctypes.byref(s2), 0, 100) == 0
    assert lib.sisso_batch_workspace_size(ctypes.byref(s2), L.MAX_BATCH + 1, 100) == 0
    assert lib.sisso_batch_workspace_size(ctypes.byref(s2), 8, L.MAX_KEEP + 1) == 0
    assert lib.sisso_batch_items(ctypes.byref(sr)) == -1
    # items: 32 x 32 pair tiles of the level-2 triangle plus 64-column batches of P_1
    p0, p1 = s2.pool[0], s2.pool[1]
    tiles = 0
    for u0 in range(p0, p1, 32):
        ue = min(u0 + 32, p1)
        tiles += (ue - 1 + 31) // 32
    assert lib.sisso_batch_items(ctypes.byref(s2)) == tiles + (p1 + 63) // 64
    # null pointers, shapes, unsupported spaces, workspace, all before any launch
    assert lib.sisso_expand_score_batched(ctypes.byref(s2), None, 8, 100, 0, fake, ws, None) == 1
    assert lib.sisso_expand_score_batched(ctypes.byref(s2), fake, 8, 100, 0, None, ws, None) == 1
    assert lib.sisso_expand_score_batched(ctypes.byref(s2), fake, 0, 100, 0, fake, ws, None) == 2
    assert lib.sisso_expand_score_batched(ctypes.byref(s2), fake, 8, 0, 0, fake, ws, None) == 2
    assert lib.sisso_expand_score_batched(ctypes.byref(s2), fake, 8, 100, -1, fake, ws, None) == 2
    assert lib.sisso_expand_score_batched(ctypes.byref(s1), fake, 8, 100, 0, fake, ws, None) == 5
    assert lib.sisso_expand_score_batched(ctypes.byref(sr), fake, 8, 100, 0, fake, ws, None) == 5
    assert lib.sisso_expand_score_batched(ctypes.byref(s2), fake, 8, 100, 0, fake, ws - 1, None) == 4
    assert lib.sisso_topk_batched(None, 8, fake, ws, fake, fake, fake, None, None) == 1
    assert lib.sisso_topk_batched(fake, 0, fake, ws, fake, fake, fake, None, None) == 2
    assert lib.sisso_prepare_residual_batched(None, 8, None) == 1
    assert lib.sisso_prepare_residual_batched(fake, L.MAX_BATCH + 1, None) == 2
    assert lib.sisso_materialize_ids_stored(ctypes.byref(s2), 3, 50, fake, 50, fake, fake, 4, fake, 50, fake,
                                            None) == 2
    assert lib.sisso_materialize_ids_stored(ctypes.byref(s2), 0, 50, fake, 50, fake, fake, 4, fake, 50, fake,
                                            None) == 2


def test_learned_argument_errors_before_launch():
    lib = L.lib()
    sr = L.make_space(4, ["sq", "sqrt", "inv"], ["add", "sub", "mul", "div"], 2, True)
    st = L.make_space(4, ["sq", "sqrt", "inv"], ["add", "sub", "mul", "div"], 2, False)
    fake = ctypes.c_void_p(0x1000)
    a = L.ScoreArgs()
    a.n, a.keep, a.ld32 = 50, 40, 64
    a.pool32 = a.stats = a.r32 = a.info = 0x1000
    assert lib.sisso_mlp_param_count() == L.MLP_PARAMS and lib.sisso_mlp_table_count() == L.MLP_TABLES
    assert lib.sisso_encode_operands(ctypes.byref(sr), ctypes.byref(a), 0, 10, None, None) == 1
    assert lib.sisso_encode_operands(ctypes.byref(sr), ctypes.byref(a), 5, 5, fake, None) == 3
    assert lib.sisso_encode_operands(ctypes.byref(sr), ctypes.byref(a), 0, sr.pool[2] + 1, fake, None) == 3
    assert lib.sisso_candidate_inputs(ctypes.byref(st), fake, fake, 4, fake, None) == 5       # no slice
    assert lib.sisso_score_ids(ctypes.byref(st), ctypes.byref(a), fake, 4, fake, None) == 5
    assert lib.sisso_score_ids(ctypes.byref(sr), ctypes.byref(a), fake, -1, fake, None) == 2
    assert lib.sisso_mlp_forward(None, fake, 4, fake, fake, None) == 1
    assert lib.sisso_mlp_forward(fake, fake, 0, fake, fake, None) == 2
    assert lib.sisso_mlp_workspace_size(0) == 0 and lib.sisso_mlp_workspace_size(64) > 0
    assert lib.sisso_mlp_backward(fake, fake, fake, fake, fake, fake, 64, fake, None, fake, 16, None) == 4
    assert lib.sisso_adam_step(fake, fake, fake, fake, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None) == 2
    assert lib.sisso_adam_step(fake, fake, fake, fake, 10, 1, 1e-3, 1.0, 0.999, 1e-8, None) == 2
    assert lib.sisso_mlp_parts(fake, fake, 0, 0, fake, None) == 2
    assert lib.sisso_mlp_parts(fake, fake, 10, 2, fake, None) == 2
    assert lib.sisso_select_kth(fake, 10, 11, fake, None) == 3
    assert lib.sisso_select_kth(fake, 10, 0, fake, None) == 3
    ws = lib.sisso_score_workspace_size(ctypes.byref(sr), ctypes.byref(a))
    bb = sr.pool[2] + sr.rect_unary
    assert lib.sisso_expand_score_pruned(ctypes.byref(st), ctypes.byref(a), fake, fake, fake, fake, 0, 10, fake,
                                         ws, None, None) == 5
    assert lib.sisso_expand_score_pruned(ctypes.byref(sr), ctypes.byref(a), fake, fake, fake, fake, bb, bb, fake,
                                         ws, None, None) == 3
    assert lib.sisso_expand_score_pruned(ctypes.byref(sr), ctypes.byref(a), fake, fake, fake, fake, bb,
                                         sr.total, fake, ws - 1, None, None) == 4
    assert lib.sisso_expand_score_pruned(ctypes.byref(sr), ctypes.byref(a), None, fake, fake, fake, bb,
                                         sr.total, fake, ws, None, None) == 1
    assert lib.sisso_expand_score_pruned_lists(ctypes.byref(sr), ctypes.byref(a), bb, sr.total) > 0

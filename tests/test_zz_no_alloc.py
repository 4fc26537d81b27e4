"""The allocation-free SO entry point (sisso_l0_search_noalloc) against the
workspace entry point (sisso_l0_search) through the C ABI: two calls in a row,
the second on a smaller problem, each bit-identical to the workspace call."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _outputs(dev, n, D):
    return (torch.full((D,), -7, dtype=torch.int32, device=dev), torch.full((1,), np.nan, dtype=torch.float64, device=dev),
            torch.full((D + 1,), np.nan, dtype=torch.float64, device=dev),
            torch.full((n,), np.nan, dtype=torch.float64, device=dev),
            torch.full((4,), np.nan, dtype=torch.float64, device=dev))


def _run(L, F, y, m, n, D, noalloc):
    dev = F.device
    tup, sse, coef, resid, stats = _outputs(dev, n, D)
    st = L.stream_handle(dev)
    if noalloc:
        rc = L.lib().sisso_l0_search_noalloc(L.ptr(F), m, n, n, L.ptr(y), D, 1e-10, L.ptr(tup), L.ptr(sse),
                                             L.ptr(coef), L.ptr(resid), L.ptr(stats), st)
    else:
        nb = L.lib().sisso_l0_workspace_size(m, n, D)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        rc = L.lib().sisso_l0_search(L.ptr(F), m, n, n, L.ptr(y), D, 1e-10, L.ptr(tup), L.ptr(sse), L.ptr(coef),
                                     L.ptr(resid), L.ptr(stats), L.ptr(ws), nb, st)
    L.check(rc, "l0")
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (tup, sse, coef, resid, stats)]


@pytest.mark.parametrize("D", [2, 3])
def test_noalloc_matches_workspace_entry_point(D):
    from paper_2410_01752_amd import _lib as L
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(71 + D)
    # first a larger problem, then a smaller one: the second call must not see
    # anything the first left in the shared device array
    for m, n in [(300, 1500), (90, 257)]:
        print(f"[noalloc] D={D} m={m} n={n}", flush=True)
        Fh = rng.lognormal(0.0, 0.5, size=(m, n))
        yh = 1.5 * Fh[7] - 0.7 * Fh[m // 2] + (0.3 * Fh[m - 2] if D == 3 else 0.0) + rng.normal(0, 0.01, n)
        F = torch.as_tensor(Fh, device=dev).contiguous()
        y = torch.as_tensor(yh, device=dev)
        ref = _run(L, F, y, m, n, D, noalloc=False)
        got = _run(L, F, y, m, n, D, noalloc=True)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b, equal_nan=True)
        assert sorted(ref[0].tolist()) == sorted(([7, m // 2, m - 2] if D == 3 else [7, m // 2]))


def test_noalloc_rejects_oversized_problem():
    from paper_2410_01752_amd import _lib as L
    cap = L.lib().sisso_l0_scratch_capacity()
    m, n = 1024, 4096
    assert L.lib().sisso_l0_workspace_size(m, n, 3) > cap
    dev = torch.device("cuda:0")
    F = torch.zeros(m * n, dtype=torch.float64, device=dev)
    y = torch.zeros(n, dtype=torch.float64, device=dev)
    tup, sse, coef, resid, stats = _outputs(dev, n, 3)
    rc = L.lib().sisso_l0_search_noalloc(L.ptr(F), m, n, n, L.ptr(y), 3, 1e-10, L.ptr(tup), L.ptr(sse), L.ptr(coef),
                                         L.ptr(resid), L.ptr(stats), L.stream_handle(dev))
    assert rc == 4   # SISSO_E_WORKSPACE, before any launch

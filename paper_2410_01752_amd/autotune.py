"""Autotuner of the screening kernels' launch shapes.

For a kernel, a screening form and a bucket of sample counts n, it times each
candidate launch shape on the real workload with HIP events on the stream the
kernel runs on, and keeps the fastest:
  * the FP32 slice kernel (k_score_rect): register-tile variant x persistent
    grid, on a contiguous block of operand tiles of the rung-3 slice;
  * the plain 16-bit slice kernel (k_score_rect_bf16): persistent grid;
  * the stored-column pass (k_score_columns): its block count (col_grid), on
    the stored pools and the unary slice;
  * the batched persistent kernel (k_score_batch): its grid, on one screening
    call over every problem of the batch (keyed also by the batch size).
Choices are cached in a JSON file keyed by (GPU architecture, HIP runtime
version, kernel, form, n bucket).  The moments pass and the read pass of the
16-bit form size their grids from the CU count, and their tile shapes,
waves per block and K-chunk are compile-time constants of their kernels.

Launch shapes never change results: every block keeps its best K' by
(score desc, id asc) and the merge is exact, so any shape returns the same
list (the determinism tests check this across grids and tiles).
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import asdict, dataclass
from typing import Dict, List, Optional, Sequence, Tuple

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sisso_mi355x", "autotune.json")

# candidate launch shapes per kernel: (tile variant, grid); grid 0 = library default
FP32_SHAPES: List[Tuple[int, int]] = [(t, g) for t in (0, 1, 2) for g in (0, 256, 512, 768)]
BF16_SHAPES: List[Tuple[int, int]] = [(0, g) for g in (0, 256, 512, 768)]
COL_SHAPES: List[Tuple[int, int]] = [(0, g) for g in (0, 1024, 4096, 8192)]
BATCH_SHAPES: List[Tuple[int, int]] = [(0, g) for g in (0, 256, 512, 1024, 2048)]


def n_bucket(n: int) -> str:
    """Sample-count bucket: powers of two (n <= 256, 512, 1024, 2048, ...)."""
    b = 64
    while b < n:
        b *= 2
    return f"n<={b}"


@dataclass
class Choice:
    tile: int
    grid: int
    ms: float
    timings: Dict[str, float]


def cache_key(arch: str, runtime: str, kernel: str, form: str, n: int) -> str:
    return "|".join([arch, runtime, kernel, form, n_bucket(n)])


def pick(timings: Dict[Tuple[int, int], float]) -> Tuple[int, int]:
    """Fastest shape; ties go to the first shape in candidate order."""
    best, best_ms = None, float("inf")
    for shape, ms in timings.items():
        if ms < best_ms:
            best, best_ms = shape, ms
    return best


class Cache:
    def __init__(self, path: str = DEFAULT_CACHE):
        self.path = path
        self.data: Dict[str, dict] = {}
        if os.path.exists(path):
            try:
                with open(path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, key: str) -> Optional[Choice]:
        d = self.data.get(key)
        if d is None:
            return None
        return Choice(d["tile"], d["grid"], d["ms"], d.get("timings", {}))

    def put(self, key: str, choice: Choice):
        self.data[key] = asdict(choice)
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def device_key():
    import torch
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "gfx").split(":")[0]
    return arch, str(torch.version.hip)


def tune_engine(eng, form: str = "fp32", keep: int = 1024, band: int = 2048, sample_tiles: int = 1024,
                cache: Optional[Cache] = None, force: bool = False, shapes: Optional[Sequence] = None,
                repeats: int = 2) -> Choice:
    """Tune the slice kernel of `form` for an Engine (its space and n).  Times
    each shape on the binary block's first `sample_tiles` operand tiles of 64,
    screening against y."""
    import torch
    cache = cache or Cache()
    arch, rt = device_key()
    kernel = "k_score_rect_bf16" if form == "bf16" else "k_score_rect"
    key = cache_key(arch, rt, kernel, form, eng.n)
    hit = cache.get(key)
    if hit is not None and not force:
        return hit
    shapes = list(shapes or (BF16_SHAPES if form == "bf16" else FP32_SHAPES))
    bb = eng.binary_base()
    per_u = int(eng.space.pool[eng.levels - 1]) * int(eng.space.n_slots)
    n_u = int(eng.space.pool[eng.levels] - eng.space.pool[eng.levels - 1])
    end = min(eng.total, bb + per_u * min(n_u, 64 * sample_tiles))
    y64 = eng.y
    timings: Dict[Tuple[int, int], float] = {}
    for tile, grid in shapes:
        best = float("inf")
        for _ in range(repeats):
            ev = {}
            eng.screen(y64, keep, None, begin=bb, end=end, grid=grid, tile=tile, precision=form,
                       band=band, events=ev)
            torch.cuda.synchronize()
            name = "bf16_screen" if form == "bf16" else "binary"
            ms = sum(a.elapsed_time(b) for a, b in ev[name])
            best = min(best, ms)
        timings[(tile, grid)] = best
    tile, grid = pick(timings)
    choice = Choice(tile, grid, timings[(tile, grid)],
                    {f"tile{t}_grid{g}": ms for (t, g), ms in timings.items()})
    cache.put(key, choice)
    return choice


def _time_shapes(shapes, run, repeats: int) -> Dict[Tuple[int, int], float]:
    """Best of `repeats` timings (ms) of run(tile, grid) per shape."""
    timings: Dict[Tuple[int, int], float] = {}
    for tile, grid in shapes:
        timings[(tile, grid)] = min(run(tile, grid) for _ in range(repeats))
    return timings


def _choice(cache: Cache, key: str, timings: Dict[Tuple[int, int], float]) -> Choice:
    tile, grid = pick(timings)
    choice = Choice(tile, grid, timings[(tile, grid)],
                    {f"tile{t}_grid{g}": ms for (t, g), ms in timings.items()})
    cache.put(key, choice)
    return choice


def tune_columns(eng, keep: int = 1024, cache: Optional[Cache] = None, force: bool = False,
                 shapes: Optional[Sequence] = None, repeats: int = 2) -> Choice:
    """Tune the stored-column pass of an Engine (its block count, col_grid):
    times the screen of the stored pools and the unary slice against y, and
    sets eng.col_grid to the choice."""
    import torch
    cache = cache or Cache()
    arch, rt = device_key()
    key = cache_key(arch, rt, "k_score_columns", "fp32", eng.n)
    hit = None if force else cache.get(key)
    if hit is None:
        end = eng.binary_base()
        saved = eng.col_grid

        def run(tile, grid):
            eng.col_grid = grid
            ev = {}
            eng.screen(eng.y, keep, None, begin=0, end=end, events=ev)
            torch.cuda.synchronize()
            return sum(a.elapsed_time(b) for a, b in ev["pool"])
        try:
            hit = _choice(cache, key, _time_shapes(list(shapes or COL_SHAPES), run, repeats))
        finally:
            eng.col_grid = saved
    eng.col_grid = hit.grid
    return hit


def tune_batched(batch, keep: int = 100, cache: Optional[Cache] = None, force: bool = False,
                 shapes: Optional[Sequence] = None, repeats: int = 2) -> Choice:
    """Tune the batched persistent kernel for a Batch (its grid): times one
    screening call over every problem against its y, and sets batch.grid to
    the choice (Batch.fit takes it)."""
    import torch
    cache = cache or Cache()
    arch, rt = device_key()
    P = batch.P
    pb = 1
    while pb < P:
        pb *= 2
    key = cache_key(arch, rt, "k_score_batch", f"fp32_P<={pb}", max(batch.n))
    hit = None if force else cache.get(key)
    if hit is None:
        which = list(range(P))

        def run(tile, grid):
            ev = {}
            batch.screen(which, [batch.y[p] for p in which], [keep] * P, grid=grid, events=ev)
            torch.cuda.synchronize()
            return sum(a.elapsed_time(b) for a, b in ev["batch_screen"])
        hit = _choice(cache, key, _time_shapes(list(shapes or BATCH_SHAPES), run, repeats))
    batch.grid = hit.grid
    return hit

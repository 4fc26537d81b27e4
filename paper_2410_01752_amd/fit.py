"""SISSO fit driver on MI355X: the loop of Sec. 2.3 over the C ABI.

For t = 1..D (eq. subspace-expansion):
    r    = y (t = 1) or the residual of the best (t-1)-term model
    SIS  : sisso_prepare_residual -> sisso_expand_score -> sisso_topk
    S_t  : sisso_materialize_ids (FP64) -> sisso_subspace_update
    SO   : sisso_sort_subspace -> sisso_l0_search (best t-term model, residual)
Every step runs in the library's kernels; this module only allocates device
buffers with torch, passes pointers and reads back the small per-t results.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


@dataclass
class StepResult:
    t: int
    list_ids: np.ndarray         # screened list before duplicate removal
    list_scores: np.ndarray      # FP32 screening scores
    sub_ids: np.ndarray          # S_t in insertion order
    best_ids: np.ndarray         # ascending ids of the best t-term model
    coef: np.ndarray             # intercept first, then per best id
    sse: float
    rmse: float
    r2: float
    n_tuples: int
    n_skipped: int
    keep: int
    n_classes: int


def _round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


# device memory left free beside the BF16 moments buffer
MOMENTS_HEADROOM = 8 << 30


class Engine:
    """Device state of one SISSO problem: base features, pools, subspace."""

    def __init__(self, X: np.ndarray, y: np.ndarray, unary: Sequence[str], binary: Sequence[str],
                 levels: int, rect: bool = False, device: str = "cuda:0", weights: Optional[np.ndarray] = None,
                 dimensionality: Optional[Sequence[str]] = None):
        """`weights`: optional per-sample weights w_s = 1 / sigma_s^2 for noise
        with a known diagonal covariance (Sec. 2.4's whitening): screening,
        duplicate classes and SO then use the weighted correlation and weighted
        least squares (FP32 screening form only).  `dimensionality`: optional
        unit string per base feature (Sec. 3.3): features that break
        dimensional analysis are not generated (FP32 and 16-bit forms)."""
        L.lib()
        self.dev = torch.device(device)
        X = np.asarray(X, dtype=np.float64)
        self.n, self.d = X.shape
        n = self.n
        if n < 2 or n > L.MAX_N:
            raise L.SissoError(f"n = {n} outside 2..{L.MAX_N}")
        self.space = L.make_space(self.d, list(unary), list(binary), levels, rect)
        self.levels, self.rect = levels, rect
        self.ld32 = _round_up(n, 64)
        self.ld64 = n
        self.X = torch.from_numpy(np.ascontiguousarray(X.T)).to(self.dev)
        self.y = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float64)).to(self.dev)
        pL, p1 = self.space.pool[levels], self.space.pool[1]
        self.pool32 = torch.empty(pL * self.ld32, dtype=torch.float32, device=self.dev)
        self.pool1 = torch.empty(p1 * self.ld64, dtype=torch.float64, device=self.dev)
        self.stats = torch.empty(pL * L.COLSTAT_FLOATS, dtype=torch.float32, device=self.dev)
        L.check(L.lib().sisso_materialize_pools(
            ctypes.byref(self.space), L.ptr(self.X), n, n, L.ptr(self.pool32), self.ld32,
            L.ptr(self.pool1), self.ld64, L.ptr(self.stats), L.stream_handle(self.dev)),
            "sisso_materialize_pools")
        self.units: Optional[torch.Tensor] = None
        if dimensionality is not None:
            if len(dimensionality) != self.d:
                raise L.SissoError("one unit string per base feature")
            bu = torch.from_numpy(L.base_units(dimensionality)).to(self.dev)
            self.units = torch.empty(pL * L.UNIT_DIMS, dtype=torch.int16, device=self.dev)
            L.check(L.lib().sisso_pool_units(ctypes.byref(self.space), L.ptr(bu), L.ptr(self.units),
                                             L.ptr(self.stats), L.stream_handle(self.dev)), "sisso_pool_units")
            torch.cuda.synchronize(self.dev)          # bu is released on return
        self.bf16_ops: Optional[torch.Tensor] = None
        self.bf16_moments: Optional[torch.Tensor] = None
        self.col_grid = 0           # blocks of the stored-column pass (0: the library's default)
        self.tk_status = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self.r32 = torch.zeros(self.ld32, dtype=torch.float32, device=self.dev)
        self.info = torch.zeros(L.RESID_DOUBLES, dtype=torch.float64, device=self.dev)
        self.w64: Optional[torch.Tensor] = None
        self.w32: Optional[torch.Tensor] = None
        if weights is not None:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
            if w.shape != (n,) or not np.all(np.isfinite(w)) or np.any(w <= 0.0):
                raise L.SissoError("weights must be n positive finite values")
            self.w64 = torch.from_numpy(w).to(self.dev)
            self.w32 = torch.zeros(self.ld32, dtype=torch.float32, device=self.dev)
        self._ws: Dict[str, torch.Tensor] = {}

    # ---------------------------------------------------------------- utils
    @property
    def total(self) -> int:
        return int(self.space.total)

    def _workspace(self, name: str, nbytes: int) -> torch.Tensor:
        t = self._ws.get(name)
        if t is None or t.numel() < nbytes:
            t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.dev)
            self._ws[name] = t
        return t

    def stream(self) -> int:
        return L.stream_handle(self.dev)

    def decode(self, fid: int):
        return L.decode(self.space, int(fid))

    def expr(self, fid: int) -> str:
        """Readable expression of a feature id."""
        op, l, r = self.decode(fid)
        if op < 0:
            return f"x{fid}"
        name = L.OPNAME[op]
        if op <= 3:
            sym = {"add": "+", "sub": "-", "mul": "*", "div": "/"}[name]
            return f"({self.expr(l)}{sym}{self.expr(r)})"
        return f"{name}({self.expr(l)})"

    # ----------------------------------------------------------------- SIS
    def prepare_residual(self, r64: torch.Tensor):
        if self.w64 is not None:
            L.check(L.lib().sisso_prepare_residual_weighted(L.ptr(r64), L.ptr(self.w64), self.n, L.ptr(self.r32),
                                                            L.ptr(self.w32), L.ptr(self.info), self.stream()),
                    "sisso_prepare_residual_weighted")
            return
        L.check(L.lib().sisso_prepare_residual(L.ptr(r64), self.n, L.ptr(self.r32), L.ptr(self.info),
                                               self.stream()), "sisso_prepare_residual")

    def score_args(self, keep: int, exclude: Optional[torch.Tensor] = None, grid: int = 0,
                   tile: int = 0, precision: int = L.FP32) -> L.ScoreArgs:
        a = L.ScoreArgs()
        a.n, a.pool32, a.ld32 = self.n, L.ptr(self.pool32), self.ld32
        a.stats, a.r32, a.info = L.ptr(self.stats), L.ptr(self.r32), L.ptr(self.info)
        a.exclude = L.ptr(exclude) if exclude is not None and exclude.numel() else None
        a.n_exclude = int(exclude.numel()) if exclude is not None else 0
        a.keep, a.precision, a.grid, a.tile = keep, precision, grid, tile
        a.w32 = L.ptr(self.w32) if self.w32 is not None else None
        a.units = L.ptr(self.units) if self.units is not None else None
        a.col_grid = self.col_grid
        return a

    def binary_base(self) -> int:
        """First id of the one-sided slice's binary block (total if none)."""
        s = self.space
        return int(s.pool[self.levels] + s.rect_unary) if self.rect else self.total

    def prepare_bf16(self):
        """BF16 operands of the slice's newest-level side (once per problem)."""
        if self.bf16_ops is not None:
            return
        nb = L.lib().sisso_bf16_operands_size(ctypes.byref(self.space), self.n)
        if nb == 0:
            raise L.SissoError("BF16 screening needs a space with the rung-3 slice")
        self.bf16_ops = torch.empty(nb, dtype=torch.uint8, device=self.dev)
        a = self.score_args(1)
        L.check(L.lib().sisso_prepare_bf16(ctypes.byref(self.space), ctypes.byref(a), L.ptr(self.bf16_ops),
                                           nb, self.stream()), "sisso_prepare_bf16")

    def bf16_moments_buffer(self) -> Optional[torch.Tensor]:
        """Device buffer of the BF16 screen's residual-independent moments
        (sisso_bf16_screen_moments), allocated on first use; None when the
        space has no slice or the buffer would leave less than
        MOMENTS_HEADROOM bytes of device memory free."""
        if self.bf16_moments is None:
            nb = L.lib().sisso_bf16_moments_size(ctypes.byref(self.space), self.n)
            if nb == 0:
                return None
            free, _ = torch.cuda.mem_get_info(self.dev)
            free += torch.cuda.memory_reserved(self.dev) - torch.cuda.memory_allocated(self.dev)
            if nb + MOMENTS_HEADROOM > free:
                return None
            self.bf16_moments = torch.empty(nb, dtype=torch.uint8, device=self.dev)
        return self.bf16_moments

    def screen(self, r64: torch.Tensor, keep: int, exclude: Optional[torch.Tensor] = None,
               begin: int = 0, end: Optional[int] = None, grid: int = 0, tile: int = 0,
               k: Optional[int] = None, events: Optional[dict] = None, precision: str = "fp32",
               band: int = 0, moments: str = "none"):
        """SIS over ids [begin, end): returns device tensors (ids, scores, count).

        The pass is issued as one sisso_expand_score call per block of the
        space (stored pool + unary slice, then the binary slice) feeding one
        workspace; `events`, if given, collects (start, end) CUDA events per
        call, recorded on the stream the kernels run on.  With the BF16 form,
        `moments` "write" also stores the residual-independent moments of the
        whole binary block into bf16_moments_buffer() (as three calls: the
        operand images, the moments pass, a "read" screen; "write_whole" issues
        the one-call WRITE screen instead), and "read" uses the ones an earlier
        "write" over the same engine stored."""
        end = self.total if end is None else end
        if moments not in ("none", "write", "read", "write_whole"):
            raise L.SissoError(f"unknown moments mode {moments!r}")
        if self.w64 is not None and precision != "fp32":
            raise L.SissoError("weighted screening runs in the FP32 form only")
        self.prepare_residual(r64)
        a = self.score_args(keep, exclude, grid, tile)
        nbytes = L.lib().sisso_score_workspace_size(ctypes.byref(self.space), ctypes.byref(a))
        if nbytes == 0:
            raise L.SissoError("sisso_score_workspace_size: invalid arguments")
        ws = self._workspace("score", nbytes)
        st = self.stream()
        bb = self.binary_base()
        parts = [("pool", begin, min(end, bb)), ("binary", max(begin, bb), end)]
        base = 0
        use_bf16 = precision == "bf16" and self.rect
        use_learned = precision == "learned" and self.rect
        if use_learned and getattr(self, "pruner", None) is None:
            raise L.SissoError("learned screening needs a pruner (Engine.set_pruner)")
        if use_bf16:
            self.prepare_bf16()
            band = max(min(band or 4 * keep, L.MAX_BAND), keep)
        for name, b, e in parts:
            if b >= e:
                continue
            a.list_base = base
            if events is not None:
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record()
            fallback = None
            if name == "binary" and use_learned:
                pr, (frac, n_sample, seed) = self.pruner, self.pruner_cfg
                steps = [("learned_prepare", lambda: pr.prepare(r64)),
                         ("learned_threshold", lambda: pr.threshold(frac, n_sample, seed)),
                         ("learned_check", lambda: pr.tail_recall(seed=seed + 1))]
                for sname, call in steps:
                    if events is not None:
                        s0 = torch.cuda.Event(enable_timing=True)
                        s1 = torch.cuda.Event(enable_timing=True)
                        s0.record()
                    res = call()
                    if events is not None:
                        s1.record()
                        events.setdefault(sname, []).append((s0, s1))
                tail_n, tail_pass = res
                self.learned_log.append((tail_n, tail_pass))
                if tail_n > 0 and tail_pass < self.pruner_min_recall * tail_n:
                    # the proposal does not rank this residual's top: screen exhaustively
                    fallback = self.pruner_fallback
                    self.prepare_residual(r64)
                    if fallback == "bf16":
                        self.prepare_bf16()
                        band = max(min(band or 4 * keep, L.MAX_BAND), keep)
                else:
                    if events is not None:
                        s0 = torch.cuda.Event(enable_timing=True)
                        s1 = torch.cuda.Event(enable_timing=True)
                        s0.record()
                    nl = pr.screen_binary(a, ws, b, e)
                    if events is not None:
                        s1.record()
                        events.setdefault("learned_screen", []).append((s0, s1))
            if name == "binary" and (use_bf16 or fallback == "bf16"):
                nb = L.lib().sisso_bf16_workspace_size(ctypes.byref(self.space), ctypes.byref(a), band)
                bws = self._workspace("bf16", nb)
                sp_, a_ = ctypes.byref(self.space), ctypes.byref(a)
                mode = L.MOMENTS_NONE if fallback is not None else \
                    {"none": L.MOMENTS_NONE, "write": L.MOMENTS_WRITE, "read": L.MOMENTS_READ,
                     "write_whole": L.MOMENTS_WRITE}[moments]
                split = moments == "write"            # "write_whole": the one-call WRITE screen
                mom = self.bf16_moments_buffer() if mode != L.MOMENTS_NONE else None
                if mode != L.MOMENTS_NONE and (mom is None or b != bb or e != self.total):
                    raise L.SissoError("BF16 moments need their buffer and the whole binary block")
                ops_, mp_ = L.ptr(self.bf16_ops), (L.ptr(mom) if mom is not None else None)
                mb_ = mom.numel() if mom is not None else 0
                steps = [("bf16_residual", lambda: L.lib().sisso_bf16_residual(sp_, a_, band, L.ptr(bws),
                                                                              bws.numel(), st))]
                if mode == L.MOMENTS_WRITE and split:
                    # a WRITE screen as its three parts (timed apart): the operand
                    # images, the moments pass, then a READ screen
                    steps += [("bf16_images", lambda: L.lib().sisso_bf16_moments_images(
                                  sp_, a_, ops_, self.bf16_ops.numel(), band, b, e, mp_, mb_, L.ptr(bws), bws.numel(),
                                  st)),
                              ("bf16_moments", lambda: L.lib().sisso_bf16_moments_pass(
                                  sp_, a_, ops_, self.bf16_ops.numel(), band, b, e, mp_, mb_, L.ptr(bws), bws.numel(),
                                  st))]
                smode = L.MOMENTS_READ if (mode == L.MOMENTS_WRITE and split) else mode
                steps += [("bf16_screen_read" if smode == L.MOMENTS_READ else "bf16_screen",
                           lambda: L.lib().sisso_bf16_screen_moments(sp_, a_, ops_, self.bf16_ops.numel(), band, b, e,
                                                                     mp_, mb_, smode, L.ptr(bws), bws.numel(), st)),
                          ("bf16_rescore", lambda: L.lib().sisso_bf16_rescore(sp_, a_, band, L.ptr(bws),
                                                                             bws.numel(), L.ptr(ws), ws.numel(),
                                                                             st))]
                for sname, call in steps:
                    if events is not None:
                        s0 = torch.cuda.Event(enable_timing=True)
                        s1 = torch.cuda.Event(enable_timing=True)
                        s0.record()
                    L.check(call(), "sisso_" + sname)
                    if events is not None:
                        s1.record()
                        events.setdefault(sname, []).append((s0, s1))
                nl = L.lib().sisso_expand_score_bf16_lists(ctypes.byref(self.space), ctypes.byref(a), band)
            elif not (name == "binary" and use_learned and fallback is None):
                L.check(L.lib().sisso_expand_score(ctypes.byref(self.space), ctypes.byref(a), b, e,
                                                   L.ptr(ws), ws.numel(), st), "sisso_expand_score")
                nl = L.lib().sisso_expand_score_lists(ctypes.byref(self.space), ctypes.byref(a), b, e)
            if events is not None:
                ev1.record()
                events.setdefault(name, []).append((ev0, ev1))
            base += nl
        k = keep if k is None else k
        ids = torch.empty(k, dtype=torch.int64, device=self.dev)
        sc = torch.empty(k, dtype=torch.float32, device=self.dev)
        cnt = torch.empty(1, dtype=torch.int32, device=self.dev)
        if events is not None:
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record()
        L.check(L.lib().sisso_topk(L.ptr(ws), ws.numel(), k, L.ptr(ids), L.ptr(sc), L.ptr(cnt), st),
                "sisso_topk")
        L.check(L.lib().sisso_topk_status(L.ptr(ws), ws.numel(), L.ptr(self.tk_status), st), "sisso_topk_status")
        if events is not None:
            ev1.record()
            events.setdefault("topk", []).append((ev0, ev1))
        return ids, sc, cnt

    def select_threshold(self, tau: float, max_out: int):
        """Every candidate of the last screening pass whose score is at least
        tau (Sec. 2.2's threshold alternative to a fixed k), best first, at
        most max_out: device tensors (ids, scores, count).  Raises if the
        pass's per-block lists may have dropped candidates that reach tau, or
        more than max_out do."""
        ws = self._ws.get("score")
        if ws is None:
            raise L.SissoError("select_threshold needs a screening pass first")
        ids = torch.empty(max_out, dtype=torch.int64, device=self.dev)
        sc = torch.empty(max_out, dtype=torch.float32, device=self.dev)
        cnt = torch.empty(1, dtype=torch.int32, device=self.dev)
        st = self.stream()
        L.check(L.lib().sisso_select_threshold(L.ptr(ws), ws.numel(), float(tau), max_out, L.ptr(ids), L.ptr(sc),
                                               L.ptr(cnt), st), "sisso_select_threshold")
        L.check(L.lib().sisso_topk_status(L.ptr(ws), ws.numel(), L.ptr(self.tk_status), st), "sisso_topk_status")
        status = int(self.tk_status.item())
        if status == 4:
            raise L.SissoError("threshold selection: a block's list filled above the threshold (raise keep)")
        if status == 5:
            raise L.SissoError(f"threshold selection: more than {max_out} candidates reach {tau}")
        if status != 0:
            raise L.SissoError(f"threshold selection: status {status}")
        return ids, sc, cnt

    def materialize(self, ids: torch.Tensor):
        """FP64 values (count x n, row q = feature ids[q]) and validity."""
        count = ids.numel()
        out = torch.empty(count * self.n, dtype=torch.float64, device=self.dev)
        valid = torch.empty(count, dtype=torch.int32, device=self.dev)
        L.check(L.lib().sisso_materialize_ids(ctypes.byref(self.space), self.n, L.ptr(self.pool1),
                                              self.ld64, L.ptr(self.stats), L.ptr(ids), count,
                                              L.ptr(out), self.n, L.ptr(valid), self.stream()),
                "sisso_materialize_ids")
        return out.view(count, self.n), valid

    def set_pruner(self, pruner, frac: float = 0.05, n_sample: int = 1 << 20, seed: int = 0,
                   min_recall: float = 0.99, fallback: str = "fp32"):
        """Learned screening of the slice's binary block (precision="learned"):
        only candidates the network ranks in the top `frac` are scored exactly.
        Before each pass the proposal's recall of the exact top of a uniform
        sample is measured; below `min_recall` the pass screens exhaustively
        with the `fallback` form ("fp32" or "bf16")."""
        self.pruner = pruner
        self.pruner_cfg = (frac, n_sample, seed)
        self.pruner_min_recall = min_recall
        self.pruner_fallback = fallback
        self.learned_log = []

    # ----------------------------------------------------------------- fit
    def fit(self, k: int, dmax: int, keep0: Optional[int] = None, singular_tol: float = 1e-10,
            grid: int = 0, tile: int = 0, timings: Optional[dict] = None, precision: str = "fp32",
            band: int = 0, moments: str = "auto", threshold: Optional[float] = None) -> List[StepResult]:
        """SISSO fit: for t = 1..dmax, SIS against the residual, subspace
        update, SO over the subspace.  With the BF16 form and `moments` "auto",
        the first pass of the fit stores the residual-independent moments of
        the binary block and the later passes read them (when the buffer fits
        in device memory); "off" recomputes them in every pass.  With a
        `threshold`, each pass keeps every candidate whose score reaches it
        (Sec. 2.2's alternative) instead of the best k: S_t grows by all their
        duplicate classes, at most k per pass (the screen keeps keep0 per
        block; a pass whose lists filled above the threshold raises)."""
        keep0 = min(2 * k if keep0 is None else keep0, L.MAX_KEEP)
        if moments not in ("auto", "off"):
            raise L.SissoError(f"unknown moments policy {moments!r}")
        use_mom = precision == "bf16" and self.rect and moments == "auto" and \
            self.bf16_moments_buffer() is not None
        mom_state = "write"                   # written by this fit's first pass, then read
        if dmax < 1 or dmax > L.MAX_D or k * dmax > L.MAX_SUBSPACE:
            raise L.SissoError("dmax or k out of range")
        fs = FitState(self.n, self.dev, self.w64)
        out: List[StepResult] = []
        r = self.y
        self.residuals = [self.y]
        for t in range(1, dmax + 1):
            keep = keep0
            while True:
                ids, sc, cnt = self.screen(r, keep, fs.exclude(), grid=grid, tile=tile, events=timings,
                                           precision=precision, band=band,
                                           moments=mom_state if use_mom else "none")
                mom_state = "read"
                if threshold is not None:
                    fs.read_update(cnt, self.tk_status)         # the merge's own status
                    ids, sc, cnt = self.select_threshold(threshold, keep)
                    cand, valid = self.materialize(ids)
                    fs.update(cand, ids, valid, cnt, keep, r, k, self._workspace)
                    nn, nc, ct = fs.read_update(cnt)
                    break
                cand, valid = self.materialize(ids)
                fs.update(cand, ids, valid, cnt, keep, r, k, self._workspace)
                nn, nc, ct = fs.read_update(cnt, self.tk_status)
                if nn >= k or ct < keep or keep >= L.MAX_KEEP:
                    break
                keep = min(2 * keep, L.MAX_KEEP)
            if not fs.commit(nn, t):
                break
            fs.so(self.y, t, singular_tol, self._workspace, timings)
            out.append(fs.result(t, ids, sc, ct, keep, nc))
            r = fs.resid.clone()
            self.residuals.append(r)
        return out


class FitState:
    """Device state of one problem's subspace S_t and SO results (Sec. 2.3).

    update() launches the subspace update for a screened list, so() the id
    sort and the l0 search; neither synchronises.  read_update() and
    result() copy the few scalars the loop needs to the host."""

    def __init__(self, n: int, dev: torch.device, w64: Optional[torch.Tensor] = None):
        self.n, self.dev, self.m = n, dev, 0
        self.w64 = w64                           # sample weights (None: unweighted)
        M = L.MAX_SUBSPACE
        self.sub = torch.empty(M * n, dtype=torch.float64, device=dev)
        self.sub_ids = torch.empty(M, dtype=torch.int64, device=dev)
        self.fsorted = torch.empty(M * n, dtype=torch.float64, device=dev)
        self.ids_sorted = torch.empty(M, dtype=torch.int64, device=dev)
        self.perm = torch.empty(M, dtype=torch.int32, device=dev)
        self.n_new = torch.zeros(1, dtype=torch.int32, device=dev)
        self.n_cls = torch.zeros(1, dtype=torch.int32, device=dev)
        self.tup = torch.empty(L.MAX_D, dtype=torch.int32, device=dev)
        self.sse = torch.empty(1, dtype=torch.float64, device=dev)
        self.coef = torch.empty(L.MAX_D + 1, dtype=torch.float64, device=dev)
        self.resid = torch.empty(n, dtype=torch.float64, device=dev)
        self.stats = torch.empty(4, dtype=torch.float64, device=dev)

    def exclude(self) -> Optional[torch.Tensor]:
        return self.ids_sorted[:self.m] if self.m else None

    def update(self, cand, ids, valid, cnt, keep: int, r, k: int, workspace):
        n, st = self.n, L.stream_handle(self.dev)
        nb = L.lib().sisso_subspace_workspace_size(n, keep, self.m)
        ws = workspace("sub", nb)
        L.check(L.lib().sisso_subspace_update_weighted(
            L.ptr(cand), n, L.ptr(ids), L.ptr(valid), L.ptr(cnt), keep, L.ptr(r), L.ptr(self.w64), n,
            L.ptr(self.sub), n, L.ptr(self.sub_ids), self.m, k, L.ptr(self.n_new), L.ptr(self.n_cls),
            L.ptr(ws), ws.numel(), st), "sisso_subspace_update")

    def read_update(self, cnt, tk_status=None):
        """(appended, classes, screened count) of the last update; raises if
        the top-k merge could not order its ties exactly."""
        parts = [self.n_new, self.n_cls, cnt] + ([tk_status] if tk_status is not None else [])
        v = torch.cat(parts).cpu().numpy()
        if tk_status is not None and int(v[3]) != 0:
            raise L.SissoError(f"sisso_topk: status {int(v[3])} (more ties at the cutoff than the gather holds)")
        return int(v[0]), int(v[1]), int(v[2])

    def commit(self, nn: int, t: int) -> bool:
        """Grow S_t by the nn appended features; False if S_t has fewer than t."""
        self.m += nn
        return self.m >= t

    def sort(self):
        """Put S_t in ascending id order (the SO's column order)."""
        n, m, st = self.n, self.m, L.stream_handle(self.dev)
        L.check(L.lib().sisso_sort_subspace(L.ptr(self.sub), n, L.ptr(self.sub_ids), m, n, L.ptr(self.fsorted),
                                            n, L.ptr(self.ids_sorted), L.ptr(self.perm), st),
                "sisso_sort_subspace")

    def so_record(self, y, t: int, workspace, sort: bool = True) -> "L.L0Problem":
        """Sort S_t (unless done by a batched call) and return this problem's
        sisso_l0_problem record."""
        if sort:
            self.sort()
        n, m = self.n, self.m
        ws = workspace("l0", L.lib().sisso_l0_workspace_size(m, n, t))
        rec = L.L0Problem()
        rec.F, rec.m, rec.ld, rec.n, rec.reserved = L.ptr(self.fsorted), m, n, n, 0
        rec.y, rec.out_tuple, rec.out_sse = L.ptr(y), L.ptr(self.tup), L.ptr(self.sse)
        rec.out_coef, rec.out_resid, rec.out_stats = L.ptr(self.coef), L.ptr(self.resid), L.ptr(self.stats)
        rec.ws, rec.ws_bytes = L.ptr(ws), ws.numel()
        return rec

    def so(self, y, t: int, singular_tol: float, workspace, timings: Optional[dict] = None):
        n, m, st = self.n, self.m, L.stream_handle(self.dev)
        self.sort()
        nb = L.lib().sisso_l0_workspace_size(m, n, t)
        ws = workspace("l0", nb)
        if timings is not None:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
        L.check(L.lib().sisso_l0_search_weighted(L.ptr(self.fsorted), m, n, n, L.ptr(y), L.ptr(self.w64), t,
                                                 singular_tol, L.ptr(self.tup), L.ptr(self.sse), L.ptr(self.coef),
                                                 L.ptr(self.resid), L.ptr(self.stats), L.ptr(ws), ws.numel(), st),
                "sisso_l0_search")
        if timings is not None:
            e1.record()
            timings.setdefault(f"l0_D{t}", []).append((e0, e1))
            timings.setdefault("so_m", []).append(m)

    def result(self, t: int, ids, sc, ct: int, keep: int, nc: int) -> StepResult:
        m = self.m
        tp = self.tup[:t].cpu().numpy()
        srt = self.ids_sorted[:m].cpu().numpy()
        stt = np.ascontiguousarray(self.stats.cpu().numpy())
        L.check(L.lib().sisso_l0_outcome(stt.ctypes.data), "sisso_l0_search")
        best = srt[tp] if (tp >= 0).all() else np.full(t, -1)
        return StepResult(t, ids[:ct].cpu().numpy(), sc[:ct].cpu().numpy(), self.sub_ids[:m].cpu().numpy(),
                          best, self.coef[:t + 1].cpu().numpy(), float(self.sse.item()), float(stt[0]),
                          float(stt[1]), int(stt[2]), int(stt[3]), keep, nc)

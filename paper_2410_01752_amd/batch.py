"""Many independent SISSO fits over one feature space, screened together.

Cross-validation folds and bootstrap resamples of a dataset (or several
datasets) share the operator set and rung, so one persistent launch screens
all of them: sisso_prepare_residual_batched -> sisso_expand_score_batched ->
sisso_topk_batched per step t of Sec. 2.3.  Each problem stores only its pool
P_1; the level-2 features are generated in registers by the screening
kernel.  The FP64 materialisation of the screened lists, the subspace
updates, the subspace sorts and the SO step then run as one batched call each
(sisso_materialize_ids_batched, sisso_subspace_update_batched,
sisso_sort_subspace_batched, sisso_l0_search_batched) over the problems'
FitState buffers, and the per-step results come back in a few copies.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L
from .fit import FitState, StepResult, _round_up


class Batch:
    """Device state of a batch of problems (X_p, y_p) over one TRI level-2 space."""

    def __init__(self, problems: Sequence[Tuple[np.ndarray, np.ndarray]], unary: Sequence[str],
                 binary: Sequence[str], levels: int = 2, device: str = "cuda:0"):
        L.lib()
        if not problems or len(problems) > L.MAX_BATCH:
            raise L.SissoError(f"batch of {len(problems)} problems outside 1..{L.MAX_BATCH}")
        if levels != 2:
            raise L.SissoError("batched screening needs a TRI space with 2 levels")
        self.dev = torch.device(device)
        d = int(np.asarray(problems[0][0]).shape[1])
        self.space = L.make_space(d, list(unary), list(binary), levels, False)
        self.store = L.make_space(d, list(unary), list(binary), levels - 1, False)
        self.levels, self.d = levels, d
        self.P = len(problems)
        self.grid = 0               # persistent blocks of the screening kernel (0: the library's default)
        p1 = int(self.store.pool[1])
        st = L.stream_handle(self.dev)
        self.n: List[int] = []
        self.ld32: List[int] = []
        self.X, self.y, self.pool32, self.pool1, self.stats, self.r32, self.info = [], [], [], [], [], [], []
        for X, y in problems:
            X = np.asarray(X, dtype=np.float64)
            n, dd = X.shape
            if dd != d:
                raise L.SissoError("every problem of a batch needs the same base features")
            if n < 2 or n > L.MAX_N:
                raise L.SissoError(f"n = {n} outside 2..{L.MAX_N}")
            ld32 = _round_up(n, 64)
            Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to(self.dev)
            yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float64)).to(self.dev)
            pool32 = torch.empty(p1 * ld32, dtype=torch.float32, device=self.dev)
            pool1 = torch.empty(p1 * n, dtype=torch.float64, device=self.dev)
            stats = torch.empty(p1 * L.COLSTAT_FLOATS, dtype=torch.float32, device=self.dev)
            L.check(L.lib().sisso_materialize_pools(ctypes.byref(self.store), L.ptr(Xd), n, n, L.ptr(pool32),
                                                    ld32, L.ptr(pool1), n, L.ptr(stats), st),
                    "sisso_materialize_pools")
            self.n.append(n)
            self.ld32.append(ld32)
            self.X.append(Xd)
            self.y.append(yd)
            self.pool32.append(pool32)
            self.pool1.append(pool1)
            self.stats.append(stats)
            self.r32.append(torch.zeros(ld32, dtype=torch.float32, device=self.dev))
            self.info.append(torch.zeros(L.RESID_DOUBLES, dtype=torch.float64, device=self.dev))
        self._ws: Dict[str, torch.Tensor] = {}
        self._keep_alive: list = []

    @property
    def total(self) -> int:
        return int(self.space.total)

    def _workspace(self, name: str, nbytes: int) -> torch.Tensor:
        t = self._ws.get(name)
        if t is None or t.numel() < nbytes:
            t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.dev)
            self._ws[name] = t
        return t

    def table(self, which: Sequence[int], r64: Sequence[torch.Tensor], keep: Sequence[int],
              exclude: Sequence[Optional[torch.Tensor]]) -> torch.Tensor:
        """Device copy of the sisso_problem records of problems `which`."""
        arr = (L.Problem * len(which))()
        for j, p in enumerate(which):
            e = arr[j]
            e.n, e.keep, e.ld32 = self.n[p], int(keep[j]), self.ld32[p]
            e.pool32, e.stats = L.ptr(self.pool32[p]), L.ptr(self.stats[p])
            e.r64, e.r32, e.info = L.ptr(r64[j]), L.ptr(self.r32[p]), L.ptr(self.info[p])
            ex = exclude[j]
            e.exclude = L.ptr(ex) if ex is not None and ex.numel() else None
            e.n_exclude = int(ex.numel()) if ex is not None else 0
            e.reserved = 0
        host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
        return host.to(self.dev)

    def screen(self, which: Sequence[int], r64: Sequence[torch.Tensor], keep: Sequence[int],
               exclude: Optional[Sequence[Optional[torch.Tensor]]] = None, grid: int = 0,
               events: Optional[dict] = None):
        """SIS of problems `which` against residuals r64 (device FP64): returns
        device tensors ids [len(which), keep_max], scores, counts, status."""
        P = len(which)
        exclude = exclude if exclude is not None else [None] * P
        keep_max = int(max(keep))
        tab = self.table(which, r64, keep, exclude)
        self._keep_alive = [tab, list(r64), list(exclude)]
        st = L.stream_handle(self.dev)
        nb = L.lib().sisso_batch_workspace_size(ctypes.byref(self.space), P, keep_max)
        if nb == 0:
            raise L.SissoError("sisso_batch_workspace_size: invalid arguments")
        ws = self._workspace("batch", nb)
        ids = torch.empty(P * keep_max, dtype=torch.int64, device=self.dev)
        sc = torch.empty(P * keep_max, dtype=torch.float32, device=self.dev)
        cnt = torch.empty(P, dtype=torch.int32, device=self.dev)
        status = torch.empty(P, dtype=torch.int32, device=self.dev)
        ev = []
        if events is not None:
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record()
        L.check(L.lib().sisso_prepare_residual_batched(L.ptr(tab), P, st), "sisso_prepare_residual_batched")
        if ev:
            ev[1].record()
        L.check(L.lib().sisso_expand_score_batched(ctypes.byref(self.space), L.ptr(tab), P, keep_max, grid,
                                                   L.ptr(ws), ws.numel(), st), "sisso_expand_score_batched")
        if ev:
            ev[2].record()
        L.check(L.lib().sisso_topk_batched(L.ptr(tab), P, L.ptr(ws), ws.numel(), L.ptr(ids), L.ptr(sc),
                                           L.ptr(cnt), L.ptr(status), st), "sisso_topk_batched")
        if ev:
            ev[3].record()
            events.setdefault("batch_prepare", []).append((ev[0], ev[1]))
            events.setdefault("batch_screen", []).append((ev[1], ev[2]))
            events.setdefault("batch_topk", []).append((ev[2], ev[3]))
            events.setdefault("batch_screen_sum_n", []).append(sum(self.n[p] for p in which))
            events.setdefault("batch_screen_problems", []).append(len(which))
        return ids.view(P, keep_max), sc.view(P, keep_max), cnt, status

    def materialize(self, p: int, ids: torch.Tensor):
        """FP64 values (count x n) and validity of features ids of problem p."""
        n, count = self.n[p], ids.numel()
        out = torch.empty(count * n, dtype=torch.float64, device=self.dev)
        valid = torch.empty(count, dtype=torch.int32, device=self.dev)
        L.check(L.lib().sisso_materialize_ids_stored(ctypes.byref(self.space), self.levels - 1, n,
                                                     L.ptr(self.pool1[p]), n, L.ptr(self.stats[p]), L.ptr(ids),
                                                     count, L.ptr(out), n, L.ptr(valid),
                                                     L.stream_handle(self.dev)), "sisso_materialize_ids_stored")
        return out.view(count, n), valid

    def fit(self, k: int, dmax: int, keep0: Optional[int] = None, singular_tol: float = 1e-10,
            grid: Optional[int] = None, timings: Optional[dict] = None) -> List[List[StepResult]]:
        """SISSO (Sec. 2.3) for every problem; result[p][t-1] as Engine.fit.
        grid: persistent blocks of the batched screening kernel (None: the
        batch's `grid`, which autotune.tune_batched sets; 0: the library's
        default)."""
        grid = self.grid if grid is None else grid
        keep0 = min(2 * k if keep0 is None else keep0, L.MAX_KEEP)
        if dmax < 1 or dmax > L.MAX_D or k * dmax > L.MAX_SUBSPACE:
            raise L.SissoError("dmax or k out of range")
        P = self.P
        states = [FitState(self.n[p], self.dev) for p in range(P)]
        wss = [{} for _ in range(P)]

        def ws_of(p):
            def get(name, nbytes):
                t = wss[p].get(name)
                if t is None or t.numel() < nbytes:
                    t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.dev)
                    wss[p][name] = t
                return t
            return get

        out: List[List[StepResult]] = [[] for _ in range(P)]
        active = list(range(P))
        r = list(self.y)
        for t in range(1, dmax + 1):
            keep = {p: keep0 for p in active}
            todo = list(active)
            lists: Dict[int, tuple] = {}
            upd: Dict[int, tuple] = {}
            while todo:
                ids, sc, cnt, status = self.screen(todo, [r[p] for p in todo], [keep[p] for p in todo],
                                                   [states[p].exclude() for p in todo], grid=grid, events=timings)
                self.update_batched(todo, states, ids, cnt, keep, r, k, ws_of)
                for j, p in enumerate(todo):
                    lists[p] = (ids[j], sc[j], cnt[j:j + 1])
                v = torch.stack([torch.cat([states[p].n_new, states[p].n_cls]) for p in todo]).cpu().numpy()
                cv, sv = cnt.cpu().numpy(), status.cpu().numpy()
                if np.any(sv != 0):
                    raise L.SissoError(f"sisso_topk_batched: problem status {sv.tolist()}")
                uv = self._upd_hold[3].cpu().numpy()
                if np.any(uv != 0):
                    raise L.SissoError(f"batched materialise / subspace update: entry status {uv.tolist()}")
                nxt = []
                for j, p in enumerate(todo):
                    nn, nc, ct = int(v[j, 0]), int(v[j, 1]), int(cv[j])
                    upd[p] = (nn, nc, ct)
                    if not (nn >= k or ct < keep[p] or keep[p] >= L.MAX_KEEP):
                        keep[p] = min(2 * keep[p], L.MAX_KEEP)
                        nxt.append(p)
                todo = nxt
            still = [p for p in active if states[p].commit(upd[p][0], t)]
            if still:
                self.so_batched(still, states, t, singular_tol, ws_of, timings)
                for p, res in zip(still, self.results(still, states, lists, upd, keep, t)):
                    out[p].append(res)
                    r[p] = states[p].resid.clone()
            active = still
        return out

    def update_batched(self, which, states, ids, cnt, keep, r, k: int, ws_of):
        """FP64 materialisation of every screened list and the subspace updates
        (Sec. 2.1 duplicates, Sec. 2.3 eq. subspace-expansion) of the problems in
        `which` (row j of ids / cnt belongs to which[j]), in two batched calls."""
        lib, st, P = L.lib(), L.stream_handle(self.dev), len(which)
        erecs, srecs = (L.EvalProblem * P)(), (L.SubspaceProblem * P)()
        hold = []
        for j, p in enumerate(which):
            n, kp, s = self.n[p], keep[p], states[p]
            out = torch.empty(kp * n, dtype=torch.float64, device=self.dev)
            valid = torch.empty(kp, dtype=torch.int32, device=self.dev)
            e = erecs[j]
            e.n, e.count, e.pool1_64, e.ld64, e.stats = n, kp, L.ptr(self.pool1[p]), n, L.ptr(self.stats[p])
            e.ids, e.out, e.ldo, e.reserved, e.valid = L.ptr(ids[j]), L.ptr(out), n, 0, L.ptr(valid)
            ws = ws_of(p)("sub", lib.sisso_subspace_workspace_size(n, kp, s.m))
            u = srecs[j]
            u.cand, u.ldc, u.count_max, u.cand_ids, u.cand_valid = L.ptr(out), n, kp, L.ptr(ids[j]), L.ptr(valid)
            u.count_dev, u.r, u.n, u.lds, u.sub, u.sub_ids = L.ptr(cnt[j:j + 1]), L.ptr(r[p]), n, n, L.ptr(s.sub), \
                L.ptr(s.sub_ids)
            u.m_prev, u.k, u.n_new, u.n_classes = s.m, k, L.ptr(s.n_new), L.ptr(s.n_cls)
            u.ws, u.ws_bytes = L.ptr(ws), ws.numel()
            hold += [out, valid]
        et, ut = L.device_table(erecs, self.dev), L.device_table(srecs, self.dev)
        status = torch.empty(2 * P, dtype=torch.int32, device=self.dev)
        L.check(lib.sisso_materialize_ids_batched(ctypes.byref(self.space), self.levels - 1, L.ptr(et), P,
                                                  max(keep[p] for p in which), L.ptr(status), st),
                "sisso_materialize_ids_batched")
        nodes_max = max(states[p].m + keep[p] for p in which)
        L.check(lib.sisso_subspace_update_batched(L.ptr(ut), P, nodes_max, k, L.ptr(status[P:]), st),
                "sisso_subspace_update_batched")
        self._upd_hold = (hold, et, ut, status)      # alive until the stream has passed the calls

    def so_batched(self, which, states, t: int, singular_tol: float, ws_of, timings=None):
        """The SO step (Sec. 2.3) of every problem in `which` in one batched call
        (after one batched sort of their subspaces into ascending id order)."""
        P = len(which)
        srt = (L.SortProblem * P)()
        for j, p in enumerate(which):
            s, n = states[p], self.n[p]
            q = srt[j]
            q.src, q.lds, q.m, q.ids, q.n, q.ldd = L.ptr(s.sub), n, s.m, L.ptr(s.sub_ids), n, n
            q.dst, q.ids_sorted, q.perm = L.ptr(s.fsorted), L.ptr(s.ids_sorted), L.ptr(s.perm)
        stt = L.device_table(srt, self.dev)
        sst = torch.empty(P, dtype=torch.int32, device=self.dev)
        L.check(L.lib().sisso_sort_subspace_batched(L.ptr(stt), P, max(states[p].m for p in which), L.ptr(sst),
                                                    L.stream_handle(self.dev)), "sisso_sort_subspace_batched")
        recs = (L.L0Problem * P)()
        for j, p in enumerate(which):
            recs[j] = states[p].so_record(self.y[p], t, ws_of(p), sort=False)
        tbl = L.device_table(recs, self.dev)
        self._sort_hold = (stt, sst)
        self._l0_table = tbl                     # alive until the results are read
        self._l0_status = torch.empty(len(which), dtype=torch.int32, device=self.dev)
        if timings is not None:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
        m_max = max(states[p].m for p in which)
        n_max = max(self.n[p] for p in which)
        L.check(L.lib().sisso_l0_search_batched(L.ptr(tbl), len(which), t, m_max, n_max, singular_tol,
                                                L.ptr(self._l0_status), L.stream_handle(self.dev)),
                "sisso_l0_search_batched")
        if timings is not None:
            e1.record()
            timings.setdefault(f"l0_batched_D{t}", []).append((e0, e1))

    def results(self, which, states, lists, upd, keep, t: int) -> List[StepResult]:
        """StepResults of step t for every problem in `which`, in three copies."""
        small = torch.cat([torch.cat([states[p].tup[:t].double(), states[p].sse, states[p].coef[:t + 1],
                                      states[p].stats]) for p in which]).cpu().numpy()
        ids = torch.cat([torch.cat([states[p].ids_sorted[:states[p].m], states[p].sub_ids[:states[p].m],
                                    lists[p][0][:upd[p][2]]]) for p in which]).cpu().numpy()
        scs = torch.cat([lists[p][1][:upd[p][2]] for p in which]).cpu().numpy()
        st = self._l0_status.cpu().numpy()
        if np.any(st != 0):
            raise L.SissoError(f"sisso_l0_search_batched: entry status {st.tolist()}")
        sv = self._sort_hold[1].cpu().numpy()
        if np.any(sv != 0):
            raise L.SissoError(f"sisso_sort_subspace_batched: entry status {sv.tolist()}")
        out, o_s, o_i, o_c = [], 0, 0, 0
        w = 2 * t + 6
        for p in which:
            m, ct = states[p].m, upd[p][2]
            v = small[o_s:o_s + w]
            o_s += w
            srt, sub = ids[o_i:o_i + m], ids[o_i + m:o_i + 2 * m]
            lid = ids[o_i + 2 * m:o_i + 2 * m + ct]
            o_i += 2 * m + ct
            lsc = scs[o_c:o_c + ct]
            o_c += ct
            tp = v[:t].astype(np.int64)
            sse, coef, stt = v[t], v[t + 1:2 * t + 2], np.ascontiguousarray(v[2 * t + 2:2 * t + 6])
            L.check(L.lib().sisso_l0_outcome(stt.ctypes.data), f"sisso_l0_search_batched (problem {p})")
            best = srt[tp] if (tp >= 0).all() else np.full(t, -1)
            out.append(StepResult(t, lid, lsc, sub, best, coef, float(sse), float(stt[0]), float(stt[1]),
                                  int(stt[2]), int(stt[3]), keep[p], upd[p][1]))
        return out

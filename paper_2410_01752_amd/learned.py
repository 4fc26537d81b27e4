"""Learned proposal for the one-sided rung-3 slice: capture, training and
pruned screening, over the library's kernels.

* capture: exhaustive FP32 SIS of the slice's binary block gives the top
  candidates (the tail of |corr|) and exact scores of a uniform sample of ids
  give the bulk;
* training: sisso_mlp_forward -> sisso_mlp_backward -> sisso_adam_step on the
  device, on network inputs built by sisso_encode_operands and
  sisso_candidate_inputs;
* pruning: per residual the operand encodings and the network's first-layer
  parts (GEMMs), a threshold at the (1 - frac) quantile of the network score
  on a uniform sample of the block (sisso_mlp_score_ids + sisso_select_kth),
  then sisso_expand_score_pruned scores exactly only what passes.

This module marshals arguments and moves tensors; the arithmetic is in the
library.  Random ids and batch orders are drawn here with seeded numpy
generators and handed to the kernels as inputs.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

H, K_IN, E = L.MLP_HIDDEN, L.MLP_IN, L.ENC


def flatten_params(P: Dict[str, np.ndarray]) -> np.ndarray:
    """W1 | b1 | w2 | b2 as one FP32 vector (the library's layout)."""
    return np.concatenate([np.asarray(P["W1"], np.float64).reshape(-1), np.asarray(P["b1"]).reshape(-1),
                           np.asarray(P["w2"]).reshape(-1), np.asarray(P["b2"]).reshape(-1)]).astype(np.float32)


def unflatten_params(v: np.ndarray) -> Dict[str, np.ndarray]:
    v = np.asarray(v, dtype=np.float64)
    o = H * K_IN
    return {"W1": v[:o].reshape(H, K_IN), "b1": v[o:o + H], "w2": v[o + H:o + 2 * H], "b2": v[o + 2 * H:o + 2 * H + 1]}


# ------------------------------------------------------------------ per-engine

def encode(eng, r64: torch.Tensor) -> torch.Tensor:
    """Encodings of every stored column of eng against residual r64."""
    eng.prepare_residual(r64)
    pL = int(eng.space.pool[eng.levels])
    enc = torch.empty(pL * E, dtype=torch.float32, device=eng.dev)
    a = eng.score_args(1)
    L.check(L.lib().sisso_encode_operands(ctypes.byref(eng.space), ctypes.byref(a), 0, pL, L.ptr(enc),
                                          eng.stream()), "sisso_encode_operands")
    return enc.view(pL, E)


def inputs(eng, enc: torch.Tensor, ids: torch.Tensor) -> torch.Tensor:
    X = torch.empty(ids.numel() * K_IN, dtype=torch.float32, device=eng.dev)
    L.check(L.lib().sisso_candidate_inputs(ctypes.byref(eng.space), L.ptr(enc), L.ptr(ids), ids.numel(), L.ptr(X),
                                           eng.stream()), "sisso_candidate_inputs")
    return X.view(-1, K_IN)


def score_ids(eng, ids: torch.Tensor) -> torch.Tensor:
    """Exact FP32 scores of slice binary ids against the prepared residual."""
    out = torch.empty(ids.numel(), dtype=torch.float32, device=eng.dev)
    a = eng.score_args(1)
    L.check(L.lib().sisso_score_ids(ctypes.byref(eng.space), ctypes.byref(a), L.ptr(ids), ids.numel(), L.ptr(out),
                                    eng.stream()), "sisso_score_ids")
    return out


def sample_ids(eng, count: int, seed: int) -> np.ndarray:
    """Uniform random ids of the slice's binary block (seeded)."""
    rng = np.random.default_rng(seed)
    return rng.integers(eng.binary_base(), eng.total, size=count, dtype=np.int64)


def capture(eng, r64: torch.Tensor, top: int = 2048, n_sample: int = 1 << 17, seed: int = 0):
    """(ids, |corr|) training examples of one residual: the exhaustive top
    `top` of the binary block and the valid ones of a uniform sample."""
    bb = eng.binary_base()
    ids_t, sc_t, cnt = eng.screen(r64, top, None, begin=bb, precision="fp32")
    c = int(cnt.item())
    ids_t, sc_t = ids_t[:c].cpu().numpy(), sc_t[:c].cpu().numpy()
    sid = np.unique(sample_ids(eng, n_sample, seed))
    sid = np.setdiff1d(sid, ids_t)
    eng.prepare_residual(r64)
    ssc = score_ids(eng, torch.from_numpy(sid).to(eng.dev)).cpu().numpy()
    ok = ssc >= 0.0
    return np.concatenate([ids_t, sid[ok]]), np.concatenate([sc_t, ssc[ok]]).astype(np.float32)


def dataset(eng, r64: torch.Tensor, ids: np.ndarray, scores: np.ndarray):
    """Device tensors X (inputs), t = atanh(|corr|) and unit weights."""
    enc = encode(eng, r64)
    X = inputs(eng, enc, torch.from_numpy(np.ascontiguousarray(ids)).to(eng.dev))
    sc = torch.from_numpy(np.ascontiguousarray(scores, dtype=np.float32)).to(eng.dev)
    t = torch.empty_like(sc)
    L.check(L.lib().sisso_mlp_target(L.ptr(sc), sc.numel(), L.ptr(t), L.stream_handle(eng.dev)), "sisso_mlp_target")
    return X, t, torch.ones(len(ids), dtype=torch.float32, device=eng.dev)


# ------------------------------------------------------------------ training

@dataclass
class TrainLog:
    steps: int
    losses: List[float]
    ms: float


def train(X: torch.Tensor, t: torch.Tensor, w: torch.Tensor, params: np.ndarray, steps: int = 2000,
          batch: int = 4096, lr: float = 1e-3, seed: int = 0, decay_from: float = 0.75,
          log_every: int = 100) -> Tuple[np.ndarray, TrainLog]:
    """Adam on the weighted squared error; returns the FP32 parameters."""
    dev = X.device
    st = L.stream_handle(dev)
    lib = L.lib()
    P = torch.from_numpy(np.asarray(params, np.float32)).to(dev)
    G = torch.zeros_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    Z = torch.empty(batch * H, dtype=torch.float32, device=dev)
    s = torch.empty(batch, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = torch.empty(lib.sisso_mlp_workspace_size(batch), dtype=torch.uint8, device=dev)
    N = X.shape[0]
    rng = np.random.default_rng(seed)
    order = rng.permutation(N)
    pos = 0
    losses = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for step in range(1, steps + 1):
        if pos + batch > N:
            order = rng.permutation(N)
            pos = 0
        idx = torch.from_numpy(order[pos:pos + batch]).to(dev)
        pos += batch
        b = idx.numel()
        Xb, tb, wb = X.index_select(0, idx), t.index_select(0, idx), w.index_select(0, idx)
        L.check(lib.sisso_mlp_forward(L.ptr(P), L.ptr(Xb), b, L.ptr(Z), L.ptr(s), st), "sisso_mlp_forward")
        L.check(lib.sisso_mlp_backward(L.ptr(P), L.ptr(Xb), L.ptr(Z), L.ptr(s), L.ptr(tb), L.ptr(wb), b, L.ptr(G),
                                       L.ptr(loss), L.ptr(ws), ws.numel(), st), "sisso_mlp_backward")
        lr_t = lr if step <= decay_from * steps else lr * 0.1
        L.check(lib.sisso_adam_step(L.ptr(P), L.ptr(G), L.ptr(M), L.ptr(V), P.numel(), step, lr_t, 0.9, 0.999,
                                    1e-8, st), "sisso_adam_step")
        if log_every and (step % log_every == 0 or step == steps):
            losses.append(float(loss.item()))
    e1.record()
    torch.cuda.synchronize()
    return P.cpu().numpy(), TrainLog(steps, losses, e0.elapsed_time(e1))


# ------------------------------------------------------------------ pruning

class Pruner:
    """Pruned screening of one Engine's slice with trained parameters."""

    def __init__(self, eng, params: np.ndarray):
        self.eng = eng
        self.P = torch.from_numpy(np.asarray(params, np.float32)).to(eng.dev)
        self.tables = torch.empty(L.MLP_TABLES, dtype=torch.float32, device=eng.dev)
        L.check(L.lib().sisso_mlp_tables(L.ptr(self.P), L.ptr(self.tables), eng.stream()), "sisso_mlp_tables")
        s = eng.space
        self.ulo, self.uhi = int(s.pool[eng.levels - 1]), int(s.pool[eng.levels])
        self.Au = torch.empty((self.uhi - self.ulo) * H, dtype=torch.float32, device=eng.dev)
        self.Bv = torch.empty(self.ulo * H, dtype=torch.float32, device=eng.dev)
        self.tau = torch.zeros(1, dtype=torch.float32, device=eng.dev)
        self.kept = torch.zeros(1, dtype=torch.int64, device=eng.dev)
        self.enc: Optional[torch.Tensor] = None

    def prepare(self, r64: torch.Tensor):
        """Encodings and first-layer parts for residual r64."""
        eng, lib, st = self.eng, L.lib(), self.eng.stream()
        self._r64 = r64
        self.enc = encode(eng, r64)
        L.check(lib.sisso_mlp_parts(L.ptr(self.P), L.ptr(self.enc[self.ulo:]), self.uhi - self.ulo, 0,
                                    L.ptr(self.Au), st), "sisso_mlp_parts")
        L.check(lib.sisso_mlp_parts(L.ptr(self.P), L.ptr(self.enc), self.ulo, 1, L.ptr(self.Bv), st),
                "sisso_mlp_parts")

    def net_scores(self, ids: torch.Tensor) -> torch.Tensor:
        out = torch.empty(ids.numel(), dtype=torch.float32, device=self.eng.dev)
        L.check(L.lib().sisso_mlp_score_ids(ctypes.byref(self.eng.space), L.ptr(self.Au), L.ptr(self.Bv),
                                            L.ptr(self.tables), L.ptr(ids), ids.numel(), L.ptr(out),
                                            self.eng.stream()), "sisso_mlp_score_ids")
        return out

    def threshold(self, frac: float, n_sample: int = 1 << 20, seed: int = 0) -> torch.Tensor:
        """tau = the (frac * n_sample)-th largest network score of a uniform sample."""
        ids = torch.from_numpy(sample_ids(self.eng, n_sample, seed)).to(self.eng.dev)
        sc = self.net_scores(ids)
        q = max(1, int(round(frac * n_sample)))
        L.check(L.lib().sisso_select_kth(L.ptr(sc), n_sample, q, L.ptr(self.tau), self.eng.stream()),
                "sisso_select_kth")
        return self.tau

    def tail_recall(self, n_sample: int = 1 << 18, top: int = 64, seed: int = 1) -> Tuple[int, int]:
        """(n, passing): of the `top` best exactly scored ids of a uniform
        sample, how many pass the current threshold (needs prepare and a
        threshold).  passing / n estimates the recall of the pruned pass."""
        eng, lib, st = self.eng, L.lib(), self.eng.stream()
        ids = torch.from_numpy(sample_ids(eng, n_sample, seed)).to(eng.dev)
        eng.prepare_residual(self._r64)
        ex = score_ids(eng, ids)
        net = self.net_scores(ids)
        thr = torch.empty(1, dtype=torch.float32, device=eng.dev)
        L.check(lib.sisso_select_kth(L.ptr(ex), n_sample, top, L.ptr(thr), st), "sisso_select_kth")
        out = torch.zeros(2, dtype=torch.int32, device=eng.dev)
        L.check(lib.sisso_count_pass(L.ptr(ex), L.ptr(net), n_sample, L.ptr(thr), L.ptr(self.tau), L.ptr(out), st),
                "sisso_count_pass")
        o = out.cpu().numpy()
        return int(o[0]), int(o[1])

    def set_threshold(self, value: float):
        self.tau.fill_(value)

    def screen_binary(self, a, ws: torch.Tensor, begin: int, end: int):
        """Pruned screening of [begin, end) of the binary block into ws (args a)."""
        eng = self.eng
        self.kept.zero_()
        L.check(L.lib().sisso_expand_score_pruned(ctypes.byref(eng.space), ctypes.byref(a), L.ptr(self.Au),
                                                  L.ptr(self.Bv), L.ptr(self.tables), L.ptr(self.tau), begin, end,
                                                  L.ptr(ws), ws.numel(), L.ptr(self.kept), eng.stream()),
                "sisso_expand_score_pruned")
        return L.lib().sisso_expand_score_pruned_lists(ctypes.byref(eng.space), ctypes.byref(a), begin, end)


def recall_of(ref_ids: np.ndarray, ref_sc: np.ndarray, got_ids: np.ndarray, tol: float = 1e-6) -> float:
    """Top-K' recall of got against the exhaustive list ref (score desc); a
    reference member within tol of the cutoff counts as found (a tie)."""
    if len(ref_ids) == 0:
        return 1.0
    got = set(np.asarray(got_ids).tolist())
    cutoff = float(ref_sc[-1])
    found = sum(1 for i, s in zip(ref_ids.tolist(), ref_sc.tolist()) if i in got or s <= cutoff + tol)
    return found / len(ref_ids)

"""FP64 reference of the learned proposal for rung-3 screening (test
infrastructure only: imported by tests/, the smoke check and the benchmark's
CPU baseline, never by the product path).

The proposal ranks candidates op(u, v) of the one-sided rung-3 slice before
exact scoring, so that only a small fraction is scored exactly.  It is the
learned screening addition to SIS (Sec. 2.2); the paper itself scores every
candidate.  The network is a two-layer perceptron

    z = W1 x + b1,   h = relu(z),   s = w2 . h + b2

on the input x = [enc(u) | enc(v) | onehot(form) | 0-padding] (K_IN values),
fitted to t = atanh(min(|corr|, T_MAX)) of the candidate by weighted least
squares and trained with Adam.  The GPU computes the products x W1^T and the
weight gradient on BF16 matrix cores with FP32 accumulation; this reference
takes BF16-rounded inputs and weights and does everything else in FP64.

Operand encoding enc(x) (E_OP values; x is a pool feature: a base feature or
op(a[, b]) of lower-level features):
    [0, 14)   class of x's operator      (0 base feature, 1 + op code, 13 none)
    [14, 28)  class of x's left operand  (13 none for a base feature)
    [28, 42)  class of x's right operand (13 none for a base feature or a unary op)
    42  corr(x, r)             43  |corr(x, r)|
    44  corr(1/x, r)           45  corr(log|x|, r)       46  corr(x^2, r)
    47  |corr(1/x, r)|         48  |corr(log|x|, r)|
    49  clip(log10(sd/|mean|), -4, 4) / 4
    50  clip(skewness, -10, 10) / 10
    51  clip(log10|mean|, -6, 6) / 6
    52  clip(log10 sd, -6, 6) / 6
    53  1 if min(x) > 0            54  1 if x has a zero
    55  1
    [56, 64)  0
A correlation with a constant or undefined transform (zero in x for 1/x and
log|x|) is 0, and so is any statistic that is not finite (a column with an
overflowing value).  corr is Pearson's correlation; the population moments are
taken about the exact mean (two passes).
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

import numpy as np

E_OP = 64
N_CLASS = 14
K_IN = 144          # 2 * E_OP + 5 forms + 11 zeros
HIDDEN = 256
T_MAX = 0.999999
NONE_CLASS = 13


# ------------------------------------------------------------------ encoding

def _corr(f: np.ndarray, r: np.ndarray) -> float:
    """Pearson correlation, two-pass FP64; 0 when either side is constant."""
    fc = f - f.mean()
    rc = r - r.mean()
    sff = float(fc @ fc)
    srr = float(rc @ rc)
    if not (sff > 0.0 and srr > 0.0) or not np.isfinite(sff):
        return 0.0
    return float(fc @ rc) / math.sqrt(sff * srr)


def operand_stats(x: np.ndarray, r: np.ndarray) -> np.ndarray:
    """The 14 statistics of enc(x) (entries 42..55) for one FP64 column x."""
    x = np.asarray(x, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    n = x.size
    mean = x.mean()
    dev = x - mean
    sd = math.sqrt(float(dev @ dev) / n)
    has_zero = bool(np.any(x == 0.0))
    c1 = _corr(x, r)
    c2 = 0.0 if has_zero else _corr(1.0 / x, r)
    c3 = 0.0 if has_zero else _corr(np.log(np.abs(x)), r)
    c4 = _corr(x * x, r)
    skew = float(np.mean(dev ** 3)) / sd ** 3 if sd > 0.0 else 0.0
    am = abs(mean)
    cv = sd / am if am > 0.0 else 1e300
    out = np.zeros(14)
    out[0], out[1] = c1, abs(c1)
    out[2], out[3], out[4] = c2, c3, c4
    out[5], out[6] = abs(c2), abs(c3)
    out[7] = min(max(math.log10(cv) if cv > 0.0 else -4.0, -4.0), 4.0) / 4.0
    out[8] = min(max(skew, -10.0), 10.0) / 10.0
    out[9] = min(max(math.log10(am) if am > 0.0 else -6.0, -6.0), 6.0) / 6.0
    out[10] = min(max(math.log10(sd) if sd > 0.0 else -6.0, -6.0), 6.0) / 6.0
    out[11] = 1.0 if x.min() > 0.0 else 0.0
    out[12] = 1.0 if has_zero else 0.0
    out[13] = 1.0
    out[~np.isfinite(out)] = 0.0
    return out


def op_class(op: int) -> int:
    """Class of an operator code (-1 = base feature)."""
    return 0 if op < 0 else 1 + op


def tree_classes(space, fid: int) -> Tuple[int, int, int]:
    """(root, left, right) classes of pool feature fid of an oracle Space."""
    op, a, b = space.decode(int(fid))
    if op < 0:
        return 0, NONE_CLASS, NONE_CLASS
    la = op_class(space.decode(int(a))[0])
    lb = op_class(space.decode(int(b))[0]) if b >= 0 else NONE_CLASS
    return op_class(op), la, lb


def encode(classes: Tuple[int, int, int], stats: np.ndarray) -> np.ndarray:
    e = np.zeros(E_OP)
    for slot, c in enumerate(classes):
        e[slot * N_CLASS + c] = 1.0
    e[42:56] = stats
    return e


def candidate_input(enc_u: np.ndarray, enc_v: np.ndarray, form: int) -> np.ndarray:
    """Network input of candidate form `form` (0 add, 1 sub, 2 mul, 3 u/v, 4 v/u) of (u, v)."""
    x = np.zeros(K_IN)
    x[:E_OP] = enc_u
    x[E_OP:2 * E_OP] = enc_v
    x[2 * E_OP + form] = 1.0
    return x


def target(abs_corr: np.ndarray) -> np.ndarray:
    return np.arctanh(np.minimum(np.asarray(abs_corr, dtype=np.float64), T_MAX))


# ------------------------------------------------------------------ network

def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest BF16 (ties to even), returned as FP64.
    BF16 keeps the top 16 bits of an IEEE single."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    bias = ((u >> 16) & 1) + 0x7FFF
    u = ((u + bias) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(X: np.ndarray, P: Dict[str, np.ndarray], bf16: bool = True):
    """z, h, s for a batch X (B x K_IN) with BF16-rounded X and W1 (bf16=False:
    unrounded, the form the gradient is the exact derivative of)."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    Xb = rnd(X)
    W1 = rnd(P["W1"])
    z = Xb @ W1.T + P["b1"]
    h = np.maximum(z, 0.0)
    s = h @ P["w2"] + P["b2"][0]
    return z, h, s


def loss_and_grad(X: np.ndarray, t: np.ndarray, w: np.ndarray, P: Dict[str, np.ndarray], bf16: bool = True):
    """Weighted mean squared error sum w (s - t)^2 / sum w and its gradient
    (the rounding of X and W1 to BF16 is passed through unchanged)."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    z, h, s = forward(X, P, bf16)
    W = float(np.sum(w))
    e = s - t
    loss = float(np.sum(w * e * e)) / W
    ds = 2.0 * w * e / W
    g = {"w2": h.T @ ds, "b2": np.array([np.sum(ds)])}
    dz = np.outer(ds, P["w2"]) * (z > 0.0)
    g["W1"] = dz.T @ rnd(X)
    g["b1"] = dz.sum(axis=0)
    return loss, g, s


def adam_step(P, G, M, V, step: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (bias-corrected moments) of every parameter array."""
    out_p, out_m, out_v = {}, {}, {}
    for k in P:
        m = beta1 * M[k] + (1.0 - beta1) * G[k]
        v = beta2 * V[k] + (1.0 - beta2) * G[k] * G[k]
        mh = m / (1.0 - beta1 ** step)
        vh = v / (1.0 - beta2 ** step)
        out_p[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
        out_m[k], out_v[k] = m, v
    return out_p, out_m, out_v


def score_factorised(enc_u: np.ndarray, enc_v: np.ndarray, form: int, P: Dict[str, np.ndarray]) -> float:
    """Network score of one candidate from its operands (same value as
    forward on candidate_input; written out as the sum of the three parts)."""
    W1 = bf16_round(P["W1"])
    a = W1[:, :E_OP] @ bf16_round(enc_u)
    b = W1[:, E_OP:2 * E_OP] @ bf16_round(enc_v)
    c = W1[:, 2 * E_OP + form] + P["b1"]
    return float(np.maximum(a + b + c, 0.0) @ P["w2"] + P["b2"][0])

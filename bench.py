#!/usr/bin/env python3
"""Benchmark: one SISSO fit at rung 3 per step on one MI355X.

Workload (the rung-3 configuration): n = 2000 samples, d = 20 base features
LogNormal(0, 0.5), a planted two-term target from the one-sided rung-3 block
plus 1% noise; operators {+, -, *, /, x^2, sqrt, 1/x}; SIS space = pool levels
0..2 (2,652,785 stored columns) plus the rung-3 slice (13,664,493,515
candidates generated on the fly); SIS k = 200 per dimension; SO D = 1..3 over
C(600, 3) = 35,820,200 models at D = 3.

A step is the whole hot path for one fit: operand pools, and for t = 1..3
screening, top-k, FP64 subspace update and the l0 search.  Inputs are
resident in HBM before the timed region.  `value` is SIS candidates scored per
second of step time; SO tuples per second are reported beside it.

Screening forms: before the timed steps the binary rung-3 block is screened
once against y with the plain FP32 form, the BF16-MFMA form (band rescored in
FP32) and the learned form (a network trained here, on the GPU, on eight
smaller seeded rung-3 problems, keeps the top 1% for exact FP32 scoring);
their times, speedups over FP32 and top-K' recall against the FP32 form are
reported under "forms".  The timed steps use the fastest form whose recall
is >= 0.99 and whose whole fit (best tuple and RMSE for every D) reproduces a
plain FP32 fit run beside it; otherwise the plain FP32 form.

Batched problems: after the timed steps, the 64-problem cross-validation /
bootstrap batch (n = 100..2000, d = 12, rung 2, k = 50, D = 1..2) is fitted
with one persistent screening launch per step; its time and rates are
reported under "batched".

Prints one JSON line (see the fields below).  `--gpus N` with N > 1 exits:
the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_HBM_GBS = 8000.0
MI355X_FP32_NONPACKED_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FLOPS_PER_CAND_SAMPLE = 6               # generate + add + 2 FMA (sum, sum of squares, cross)
NET_FLOPS_PER_CAND = 4 * 256            # per hidden unit: two adds, max, FMA into the score
BATCH_FLOPS_PER_CAND_SAMPLE = 6


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration),
    or None when no summary for this kernel and workload exists."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    return d.get("hbm_bytes_per_launch")


def fit_once(p, form, keep0, band, params, args):
    """One whole fit with a screening form; best tuples and RMSE per D."""
    import torch
    from paper_2410_01752_amd.fit import Engine
    eng = Engine(p.X, p.y, p.unary, p.binary, p.rung, p.rect)
    if form == "learned":
        from paper_2410_01752_amd import learned as LN
        eng.set_pruner(LN.Pruner(eng, params), frac=args.learned_frac, n_sample=1 << 20, seed=3,
                       fallback=args.learned_fallback)
    res = eng.fit(p.k, p.dmax, keep0=keep0, precision=form, band=band)
    torch.cuda.synchronize()
    out = {"best_ids": [list(map(int, r.best_ids)) for r in res], "rmse": [r.rmse for r in res]}
    if form == "learned":
        out["tail_check"] = [list(x) for x in eng.learned_log]
    del eng
    torch.cuda.empty_cache()
    return out


def train_proposal(args, log):
    """Train the proposal network on the GPU (capture + Adam), seeded."""
    import torch
    from paper_2410_01752_amd import inputs as I
    from paper_2410_01752_amd import learned as LN
    from paper_2410_01752_amd.fit import Engine
    t0 = time.perf_counter()
    Xs, ts, ws = [], [], []
    seeds = list(range(501, 509))
    for s in seeds:
        q = I.config3(seed=s, n=2000, d=12)
        e = Engine(q.X, q.y, q.unary, q.binary, q.rung, q.rect)
        e.fit(q.k, 2)
        for ri, r in enumerate(e.residuals[:3]):
            ids, sc = LN.capture(e, r, top=2048, n_sample=1 << 17, seed=ri)
            X, t, w = LN.dataset(e, r, ids, sc)
            Xs.append(X); ts.append(t); ws.append(w)
        del e
        torch.cuda.empty_cache()
    X, t, w = torch.cat(Xs), torch.cat(ts), torch.cat(ws)
    del Xs, ts, ws
    cap_s = time.perf_counter() - t0
    params, tl = LN.train(X, t, w, LN.flatten_params(I.mlp_init(7)), steps=args.learned_steps, batch=4096,
                          lr=1e-3, seed=1, log_every=max(1, args.learned_steps // 6))
    info = {"data": f"seeded rung-3 problems {seeds[0]}-{seeds[-1]} (n=2000, d=12, LogNormal(0,0.5)), "
                    "residuals y, r_1 and r_2; exhaustive top 2048 + 2^17 uniform ids each",
            "examples": int(X.shape[0]), "steps": args.learned_steps, "batch": 4096, "capture_s": cap_s,
            "train_ms": tl.ms, "loss": tl.losses}
    log(f"proposal trained: {X.shape[0]} examples, loss {tl.losses[0]:.4f} -> {tl.losses[-1]:.4f}, "
        f"{tl.ms:.0f} ms")
    del X, t, w
    torch.cuda.empty_cache()
    return params, info


def learned_c5(params, args, log):
    """The learned form on its own workload: a held-out d = 30 rung-3 problem
    (seed 509, 1.51e11 candidates in the slice's binary block), one screening
    against y per form; top-K' recall and speedup against exhaustive FP32.
    The proposal is measured by itself here (no tail-check fallback)."""
    import torch
    from paper_2410_01752_amd import inputs as I
    from paper_2410_01752_amd import learned as LN
    from paper_2410_01752_amd.fit import Engine
    q = I.config5(seed=509)
    e = Engine(q.X, q.y, q.unary, q.binary, q.rung, q.rect)
    bb, keep = e.binary_base(), 2048

    def run(form, **kw):
        ev = {}
        ids, sc, cnt = e.screen(e.y, keep, None, begin=bb, precision=form, events=ev, **kw)
        torch.cuda.synchronize()
        c = int(cnt.item())
        return ids[:c].cpu().numpy(), sc[:c].cpu().numpy(), sum(a.elapsed_time(b) for a, b in ev["binary"])

    fi, fs, fms = run("fp32")
    log(f"C5 fp32 {fms:.0f} ms")
    out = {"workload": "held-out rung-3 problem: n=2000, d=30 LogNormal(0,0.5), seed 509; binary block of the "
                       "one-sided slice against y",
           "candidates": int(e.total - bb), "keep": keep, "fp32_ms": fms}
    for frac in (0.05, 0.01):
        e.set_pruner(LN.Pruner(e, params), frac=frac, n_sample=1 << 20, seed=3, min_recall=0.0)
        gi, gs, ms = run("learned")
        out[f"learned_{frac:g}"] = {"ms": ms, "recall": LN.recall_of(fi, fs, gi), "speedup_vs_fp32": fms / ms,
                                    "tail_check": list(e.learned_log[-1])}
        log(f"C5 learned {frac:g}: {ms:.0f} ms, recall {out[f'learned_{frac:g}']['recall']:.4f}")
    bi, bs, bms = run("bf16", band=min(4 * keep, 7168))
    out["bf16"] = {"ms": bms, "recall": LN.recall_of(fi, fs, bi), "speedup_vs_fp32": fms / bms}
    log(f"C5 bf16 {bms:.0f} ms, recall {out['bf16']['recall']:.4f}")
    del e
    torch.cuda.empty_cache()
    return out


def batched_fit(log, autotune: bool = True):
    """The 64-problem CV / bootstrap batch: one persistent screening launch per step."""
    import torch
    from paper_2410_01752_amd import inputs as I
    from paper_2410_01752_amd.batch import Batch
    ps = I.config4()
    grid, tuned = 0, None
    if autotune:
        from paper_2410_01752_amd import autotune as AT
        b0 = Batch([(q.X, q.y) for q in ps], ps[0].unary, ps[0].binary, 2)
        ch = AT.tune_batched(b0, keep=2 * ps[0].k)
        grid = ch.grid
        tuned = {"kernel": "k_score_batch", "grid": grid, "ms": ch.ms, "timings_ms": ch.timings}
        log(f"autotune batched: grid {grid}")
        del b0
        torch.cuda.empty_cache()

    def step(tm=None):
        b = Batch([(q.X, q.y) for q in ps], ps[0].unary, ps[0].binary, 2)
        res = b.fit(ps[0].k, ps[0].dmax, grid=grid, timings=tm)
        return b, res

    step()
    torch.cuda.synchronize()
    tm = {}
    t0 = time.perf_counter()
    b, res = step(tm)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sc = [a.elapsed_time(c) for a, c in tm.get("batch_screen", [])]
    tk = [a.elapsed_time(c) for a, c in tm.get("batch_topk", [])]
    total = b.total
    sum_n = sum(b.n)
    passes = len(sc)
    # roofline over the launches that screened every problem (one per t)
    full = [i for i, s in enumerate(tm.get("batch_screen_sum_n", [])) if s == sum_n]
    flops = BATCH_FLOPS_PER_CAND_SAMPLE * sum_n * total
    kern_ms = sum(sc[i] for i in full) / max(1, len(full))
    info = {"workload": "64 SISSO fits (8 datasets x 5 CV folds + 3 bootstraps), n=100..2000, d=12 "
                        "U(0.1,10), full operator set, rung 2 (482,031 candidates each), k=50, D=1..2",
            "problems": len(ps), "sum_n": sum_n, "ms_per_step": wall * 1e3,
            "screen_launches": passes, "screen_ms": sc, "topk_ms": tk,
            "screen_launch_sum_n": tm.get("batch_screen_sum_n", []),
            "screen_launch_problems": tm.get("batch_screen_problems", []),
            "candidates_per_s": sum(tm.get("batch_screen_problems", [])) * total / wall,
            "roofline": {"bound": "alu", "kernel": "k_score_batch", "achieved": flops / (kern_ms * 1e-3) / 1e12,
                         "peak": MI355X_FP32_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                         "frac": flops / (kern_ms * 1e-3) / 1e12 / MI355X_FP32_NONPACKED_TFLOPS,
                         "per_unit": f"{BATCH_FLOPS_PER_CAND_SAMPLE} flops per (candidate, sample), "
                                     f"{total} candidates x sum_n={sum_n} per launch"},
            "rmse_D2": [r[-1].rmse for r in res[:4]],
            "autotune": tuned}
    log(f"batched: {len(ps)} problems, {wall * 1e3:.1f} ms per step, screen {kern_ms:.2f} ms per launch")
    return info


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C3", choices=["C3", "C2", "C1"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--keep0", type=int, default=0,
                    help="screened-list length before duplicate removal (k + slack); 0 = 2k, "
                         "or 2048 for the rung-3 workload (no re-screening when duplicates crowd the list)")
    ap.add_argument("--learned-frac", type=float, default=0.01,
                    help="learned form: fraction of the binary block scored exactly")
    ap.add_argument("--learned-steps", type=int, default=3000, help="training steps of the proposal network")
    ap.add_argument("--no-learned", action="store_true", help="skip training and the learned form")
    ap.add_argument("--learned-fallback", default="bf16", choices=["fp32", "bf16"],
                    help="exhaustive form of a learned pass whose proposal fails the tail check")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 64-problem fit")
    ap.add_argument("--c5", action="store_true",
                    help="also screen a held-out d=30 problem with every form (learned at 5%% and 1%%); ~2 min")
    ap.add_argument("--precision", default="auto", choices=["auto", "fp32", "bf16", "learned"],
                    help="screening form of the rung-3 slice; auto = the fastest form whose recall against "
                         "the FP32 form is >= 0.99 and whose whole fit matches an FP32 fit, both measured here")
    ap.add_argument("--band", type=int, default=0,
                    help="BF16 form: candidates rescored in FP32 (0: 4 x K', at most 7168)")
    ap.add_argument("--no-forms", action="store_true", help="skip the BF16 vs FP32 recall check")
    ap.add_argument("--no-autotune", action="store_true", help="use the library's default launch shapes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference kernel for HBM counters)")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:                          # noqa: BLE001 - lscpu is optional
        pass
    return "unknown"


def cpu_baseline(p, budget_s: float, sub=None):
    """The FP64 oracle on bounded samples of the same workload: the binary
    rung-3 block for consecutive u operands (all v, all slots) on one thread,
    then the same rate from one single-threaded process per core (at most 16,
    the host share of one GPU), then the SO step on the fit's 600-column
    subspace at D = 3 (C(600, 3) tuples)."""
    from oracle import oracle as O
    sp = O.Space(p.X.shape[1], p.unary, p.binary, p.rung, p.rect)
    if p.rect:
        p1, p2 = sp.pool(1), sp.pool(2)
        base = p2 + len(p.unary) * (p2 - p1)
        per_u = p1 * sum(2 if b == "div" else 1 for b in p.binary)
    else:
        base, per_u = 0, 1000
    # calibrate on a small slice, then size the sample to the budget
    t0 = time.perf_counter()
    sp.score_range(p.X, p.y, base, base + per_u)
    dt = time.perf_counter() - t0
    n_u = max(1, int(budget_s / max(dt, 1e-6)) - 1)
    n_u = min(n_u, 400)
    t0 = time.perf_counter()
    sp.score_range(p.X, p.y, base + per_u, base + per_u * (1 + n_u))
    dt = time.perf_counter() - t0
    cands = per_u * n_u
    out = {"value": cands / dt, "unit": "candidates/s", "cores": 1, "kind": "oracle",
           "sample": f"{cands} candidates ({n_u} u operands x {per_u} (v, op) pairs of the "
                     f"binary rung-3 block) scored in FP64, one thread, {dt:.1f} s",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    # all cores: independent single-threaded processes on disjoint slices
    if p.rect and p.name == "C3":
        procs = max(1, min(os.cpu_count() or 1, 16))
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        per_proc = max(1, n_u // 2)
        start = base + per_u * (1 + n_u)
        t0 = time.perf_counter()
        workers = []
        for i in range(procs):
            b = start + i * per_proc * per_u
            workers.append(subprocess.Popen(
                [sys.executable, "-m", "oracle.slice_worker", str(p.seed), str(b), str(b + per_proc * per_u)],
                cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        done = 0
        for w in workers:
            o, _ = w.communicate()
            if w.returncode == 0:
                done += int(o.split()[0])
        wall = time.perf_counter() - t0
        out["all_core"] = {"value": done / wall, "unit": "candidates/s", "cores": procs,
                           "sample": f"{procs} single-threaded processes x {per_proc * per_u} candidates "
                                     f"(disjoint u ranges of the binary block), {wall:.1f} s wall including "
                                     f"each process's start-up"}
    if sub is not None:
        F, y, D = sub
        t0 = time.perf_counter()
        r = O.l0(F, y, D)
        dt = time.perf_counter() - t0
        out["so"] = {"value": r.n_tuples / dt, "unit": "tuples/s", "cores": 1,
                     "sample": f"oracle SO over the fit's {F.shape[1]}-column subspace at D = {D} "
                               f"({r.n_tuples} tuples, Gram + Gaussian elimination per tuple), {dt:.2f} s"}
    return out


MI355X_FP16_TFLOPS = 2500.0               # dense MFMA, FP16 and BF16 alike
CONTRACTIONS_PER_PAIR = 9            # algorithmic: (u v, u (v r), u^2 v^2) for u * v, u / v and v / u
EXECUTED_MFMA_GEMMS = 12             # the plain kernel: 12 centred contractions, one FP16 product each
MOMENT_CONTRACTIONS_PER_PAIR = 9     # moments pass: the residual-independent ones of the plain kernel's 12
READ_CONTRACTIONS_PER_PAIR = 3       # read pass: u (v r) for u * v, u / v and v / u
MOMENT_BYTES_PER_PAIR = 24           # six FP32 residual-independent moments per (u, v) pair
CONTRACTION_BYTES_PER_PAIR = 12      # three FP32 residual contractions per (u, v) pair


def recall_of(fi, fs, bi, tol=1e-6):
    """Tie-aware top-K' recall of a form against the FP32 form (a missing FP32
    member within tol of the cutoff ties with it and counts as found)."""
    got = set(bi.tolist())
    cutoff = fs[-1]
    found = sum(1 for i, sc in zip(fi.tolist(), fs.tolist()) if i in got or sc <= cutoff + tol)
    raw = sum(1 for i in fi.tolist() if i in got)
    return found / len(fi), raw / len(fi)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; run with --gpus 1"}))
        sys.exit(2)
    import torch
    from paper_2410_01752_amd import inputs as I
    from paper_2410_01752_amd.fit import Engine

    p = {"C3": I.config3, "C2": I.config2, "C1": I.config1}[args.workload]()
    dev = torch.device("cuda:0")
    n = p.X.shape[0]
    log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)
    log(f"workload {args.workload} n={n} d={p.X.shape[1]} k={p.k} D={p.dmax}")
    keep0 = args.keep0 or (2048 if p.rect else 2 * p.k)
    band = args.band or min(4 * keep0, 7168)

    if args.copy_calibration:
        # an elementwise kernel that reads 1 GiB and writes 1 GiB (a copy through
        # the shader engines, so that rocprofv3 counters see it as a kernel)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x 1 GiB elementwise copies")

    def ev_ms(tm, name):
        return [a.elapsed_time(b) for a, b in tm.get(name, [])]

    # ---- forms on the first residual (y): plain FP32, BF16 MFMA + band rescore, learned proposal
    forms = {}
    prec = args.precision
    learned_params = None
    if p.rect and not args.no_learned and prec in ("auto", "learned"):
        learned_params, forms["learned_training"] = train_proposal(args, log)
    if p.rect and not args.no_forms:
        from paper_2410_01752_amd import learned as LN
        eng = Engine(p.X, p.y, p.unary, p.binary, p.rung, p.rect)
        y64 = eng.y
        bb = eng.binary_base()

        def run(form, reps=1):
            for _ in range(reps):
                tm = {}
                ids, sc, cnt = eng.screen(y64, keep0, None, begin=bb, precision=form, band=band, events=tm)
                torch.cuda.synchronize()
            c = int(cnt.item())
            return ids[:c].cpu().numpy(), sc[:c].cpu().numpy(), tm

        fi, fs, tf = run("fp32")
        fp32_ms = sum(ev_ms(tf, "binary"))
        forms["fp32"] = {"binary_block_ms": fp32_ms, "k_score_rect_ms": fp32_ms, "recall": 1.0, "keep": keep0}
        log(f"forms: fp32 {fp32_ms:.1f} ms")
        if prec in ("auto", "bf16"):
            bi, bs, tb = run("bf16", reps=2)             # the first call prepares the BF16 operands
            rec, raw = recall_of(fi, fs, bi)
            bf16_ms = sum(ev_ms(tb, "binary"))
            forms["bf16"] = {"binary_block_ms": bf16_ms, "k_score_rect_bf16_ms": sum(ev_ms(tb, "bf16_screen")),
                             "operand_prep_ms": sum(ev_ms(tb, "bf16_residual")),
                             "band_rescore_ms": sum(ev_ms(tb, "bf16_rescore")), "band": band,
                             "recall": rec, "recall_raw": raw, "speedup_vs_fp32": fp32_ms / bf16_ms, "keep": keep0}
            log(f"forms: bf16 {bf16_ms:.1f} ms, recall {rec:.4f} (raw {raw:.4f})")
        if learned_params is not None:
            pr = LN.Pruner(eng, learned_params)
            eng.set_pruner(pr, frac=args.learned_frac, n_sample=1 << 20, seed=3, fallback=args.learned_fallback)
            li, ls, tl = run("learned", reps=2)
            rec, raw = recall_of(fi, fs, li)
            l_ms = sum(ev_ms(tl, "binary"))
            forms["learned"] = {"binary_block_ms": l_ms, "k_score_pruned_ms": sum(ev_ms(tl, "learned_screen")),
                                "encode_and_parts_ms": sum(ev_ms(tl, "learned_prepare")),
                                "threshold_ms": sum(ev_ms(tl, "learned_threshold")),
                                "budget_frac": args.learned_frac,
                                "kept_frac": int(pr.kept.item()) / max(1, eng.total - bb),
                                "recall": rec, "recall_raw": raw, "speedup_vs_fp32": fp32_ms / l_ms, "keep": keep0}
            log(f"forms: learned {l_ms:.1f} ms, recall {rec:.4f} (raw {raw:.4f})")
        del eng
        torch.cuda.empty_cache()
        if prec == "auto":
            # the fastest form whose recall on y is >= 0.99 AND whose whole fit
            # (every D) reproduces the plain FP32 fit: same best tuples, RMSE within 1e-6
            ok = sorted((v["binary_block_ms"], f) for f, v in forms.items()
                        if f in ("bf16", "learned") and v["recall"] >= 0.99)
            ref = fit_once(p, "fp32", keep0, band, learned_params, args)
            forms["fp32"]["fit"] = ref
            prec = "fp32"
            for _, f in ok:
                got = fit_once(p, f, keep0, band, learned_params, args)
                same = all(a == b for a, b in zip(got["best_ids"], ref["best_ids"])) and \
                    all(abs(a - b) <= 1e-6 * b for a, b in zip(got["rmse"], ref["rmse"]))
                forms[f]["fit"] = dict(got, matches_fp32=same)
                log(f"fit check {f}: {'matches' if same else 'differs from'} the FP32 fit")
                if same:
                    prec = f
                    break
    elif prec == "auto":
        prec = "fp32"
    if prec == "learned" and learned_params is None:
        learned_params, forms["learned_training"] = train_proposal(args, log)

    # ---- autotuned launch shape of the slice kernel for the chosen form
    tile, grid, col_grid, tuned = args.tile, args.grid, 0, None
    if p.rect and prec in ("fp32", "bf16") and not args.no_autotune and not (args.tile or args.grid):
        from paper_2410_01752_amd import autotune as AT
        eng = Engine(p.X, p.y, p.unary, p.binary, p.rung, p.rect)
        ch = AT.tune_engine(eng, form=prec, keep=keep0, band=band, sample_tiles=1024)
        tile, grid = ch.tile, ch.grid
        cc = AT.tune_columns(eng, keep=keep0)
        col_grid = cc.grid
        tuned = {"tile": tile, "grid": grid, "sample_ms": ch.ms, "timings_ms": ch.timings,
                 "columns": {"kernel": "k_score_columns", "col_grid": col_grid, "ms": cc.ms,
                             "timings_ms": cc.timings}}
        log(f"autotune {prec}: tile {tile} grid {grid}; stored columns: col_grid {col_grid}")
        del eng
        torch.cuda.empty_cache()

    def one_step(timings=None):
        eng = Engine(p.X, p.y, p.unary, p.binary, p.rung, p.rect)
        if prec == "learned":
            from paper_2410_01752_amd import learned as LN
            eng.set_pruner(LN.Pruner(eng, learned_params), frac=args.learned_frac, n_sample=1 << 20, seed=3,
                           fallback=args.learned_fallback)
        eng.col_grid = col_grid
        res = eng.fit(p.k, p.dmax, keep0=keep0, grid=grid, tile=tile, timings=timings,
                      precision=prec, band=band)
        return eng, res

    for w in range(args.warmup):
        one_step()
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")

    timings = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    eng = None
    for st in range(args.steps):
        eng = None                               # the previous step's device state is released first
        eng, res = one_step(timings)
        results.append(res)
        torch.cuda.synchronize()
        log(f"step {st + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3

    total = eng.total
    bb = eng.binary_base()
    n_bin = total - bb
    passes_per_step = len(ev_ms(timings, "pool")) / args.steps if ev_ms(timings, "pool") else \
        len(ev_ms(timings, "binary")) / args.steps
    cands_per_step = passes_per_step * total
    value = cands_per_step / (wall / args.steps)
    l0_ms = sum(sum(ev_ms(timings, f"l0_D{t}")) for t in range(1, p.dmax + 1)) / args.steps
    d3 = ev_ms(timings, f"l0_D{p.dmax}")
    so_ms_d3 = sum(d3) / max(1, len(d3))
    so_m = timings.get("so_m", [0])
    dmax_tuples = math.comb(so_m[p.dmax - 1] if len(so_m) >= p.dmax else p.k * p.dmax, p.dmax)
    pool_ms = ev_ms(timings, "pool")
    if n_bin > 0 and prec == "learned":
        ks = ev_ms(timings, "learned_screen")
        kernel_ms = sum(ks) / len(ks)
        kept = forms.get("learned", {}).get("kept_frac", args.learned_frac) * n_bin
        flops = NET_FLOPS_PER_CAND * n_bin + FLOPS_PER_CAND_SAMPLE * n * kept
        achieved = flops / (kernel_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "k_score_pruned", "achieved": achieved,
                "peak": MI355X_FP32_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / MI355X_FP32_NONPACKED_TFLOPS, "traffic": None,
                "avg_launch_ms": kernel_ms, "units_per_launch": n_bin,
                "per_unit": f"{NET_FLOPS_PER_CAND} network flops per candidate + {FLOPS_PER_CAND_SAMPLE} flops "
                            f"x n={n} per exactly scored candidate ({kept:.3g} per launch)"}
    elif n_bin > 0 and prec == "bf16":
        pairs = n_bin // eng.space.n_slots
        km = ev_ms(timings, "bf16_moments")
        kr = ev_ms(timings, "bf16_screen_read")
        if km:
            # a fit's first pass runs the moments pass (nine residual-independent
            # GEMMs per pair, the dominant kernel), every pass a read pass (three
            # residual GEMMs, then the scorer of the stored contractions)
            kernel_ms = sum(km) / len(km)
            flops = 2.0 * MOMENT_CONTRACTIONS_PER_PAIR * n * pairs
            achieved = flops / (kernel_ms * 1e-3) / 1e12
            roof = {"bound": "mfma", "kernel": "k_bf_moments", "achieved": achieved,
                    "peak": MI355X_FP16_TFLOPS, "unit": "TFLOP/s", "frac": achieved / MI355X_FP16_TFLOPS,
                    "traffic": measured_traffic("k_bf_moments", args.workload), "avg_launch_ms": kernel_ms,
                    "units_per_launch": pairs, "launches_per_step": len(km) / args.steps,
                    "per_unit": f"{MOMENT_CONTRACTIONS_PER_PAIR} residual-independent contractions x 2 flops x "
                                f"n={n} samples per (u, v) pair"}
            ki = ev_ms(timings, "bf16_images")
            if ki:
                roof["images"] = {"kernels": "k_bf16_u_image, k_bf16_vm_image", "avg_ms": sum(ki) / len(ki),
                                  "launches_per_step": len(ki) / args.steps}
        else:
            ks = ev_ms(timings, "bf16_screen")
            kernel_ms = sum(ks) / len(ks)
            flops = 2.0 * CONTRACTIONS_PER_PAIR * n * pairs
            achieved = flops / (kernel_ms * 1e-3) / 1e12
            executed = 2.0 * EXECUTED_MFMA_GEMMS * n * pairs / (kernel_ms * 1e-3) / 1e12
            roof = {"bound": "mfma", "kernel": "k_score_rect_bf16", "achieved": achieved,
                    "peak": MI355X_FP16_TFLOPS, "unit": "TFLOP/s", "frac": achieved / MI355X_FP16_TFLOPS,
                    "traffic": None, "avg_launch_ms": kernel_ms, "units_per_launch": pairs,
                    "per_unit": f"{CONTRACTIONS_PER_PAIR} contractions x 2 flops x n={n} samples per (u, v) pair",
                    "executed_mfma_tflops": executed, "executed_frac": executed / MI355X_FP16_TFLOPS,
                    "launches_per_step": len(ks) / args.steps}
        if kr:
            read_ms = sum(kr) / len(kr)
            rflops = 2.0 * READ_CONTRACTIONS_PER_PAIR * n * pairs
            roof["read_pass"] = {
                "kernels": "k_score_rect_bf16<read> (residual GEMMs), k_bf_score_stored (bound, then scores)",
                "avg_ms": read_ms, "launches_per_step": len(kr) / args.steps,
                "achieved": rflops / (read_ms * 1e-3) / 1e12, "unit": "TFLOP/s",
                "frac": rflops / (read_ms * 1e-3) / 1e12 / MI355X_FP16_TFLOPS,
                "per_unit": f"{READ_CONTRACTIONS_PER_PAIR} residual contractions x 2 flops x n={n} samples per "
                            f"(u, v) pair, plus {MOMENT_BYTES_PER_PAIR} bytes of stored moments and "
                            f"{CONTRACTION_BYTES_PER_PAIR} of contractions written and read"}
    elif n_bin > 0:
        kb = ev_ms(timings, "binary")
        kernel_ms = sum(kb) / len(kb)
        flops = FLOPS_PER_CAND_SAMPLE * n * n_bin
        achieved = flops / (kernel_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "k_score_rect", "achieved": achieved,
                "peak": MI355X_FP32_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / MI355X_FP32_NONPACKED_TFLOPS, "traffic": None,
                "avg_launch_ms": kernel_ms, "units_per_launch": n_bin,
                "per_unit": f"{FLOPS_PER_CAND_SAMPLE} flops x n={n} samples per candidate"}
    else:
        kernel_ms = sum(pool_ms) / max(1, len(pool_ms))
        byts = 4.0 * n * total
        achieved = byts / (kernel_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "k_score_columns", "achieved": achieved,
                "peak": MI355X_HBM_GBS, "unit": "GB/s", "frac": achieved / MI355X_HBM_GBS,
                "traffic": None, "avg_launch_ms": kernel_ms, "units_per_launch": total,
                "per_unit": f"4 bytes x n={n} samples per stored column"}
    roof["traffic"] = measured_traffic(roof["kernel"], args.workload)
    if roof["traffic"] is not None:
        roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    if "fp32" in forms and n_bin > 0:
        fms = forms["fp32"]["k_score_rect_ms"]
        forms["fp32"]["roofline_frac"] = FLOPS_PER_CAND_SAMPLE * n * n_bin / (fms * 1e-3) / 1e12 / \
            MI355X_FP32_NONPACKED_TFLOPS

    last = results[-1]
    out = {
        "metric": "SIS candidates scored/s + SO tuples/s at rung 3; learned/BF16 vs plain @99% recall",
        "value": value, "unit": "candidates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp16" if prec == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": {"C3": "rung-3 SISSO fit: n=2000, d=20 LogNormal(0,0.5), ops {+,-,*,/,^2,sqrt,1/x}, "
                                      "pool levels 0-2 + one-sided rung-3 slice (13,667,146,300 candidates), "
                                      "k=200, D=1..3, FP64 SO",
                                "C2": "rung-2 SISSO fit: n=500, d=10, full operator set, k=100, D=1..3",
                                "C1": "rung-2 SISSO fit: n=50, d=5, k=20, D=1..2"}[args.workload],
                   "n": n, "d": p.X.shape[1], "candidates_per_pass": total, "k": p.k, "D": p.dmax,
                   "screening_form": prec, "keep0": keep0, "band": band if prec == "bf16" else None,
                   "bf16_moments": (eng.bf16_moments is not None) if prec == "bf16" else None,
                   "learned_frac": args.learned_frac if prec == "learned" else None},
        "sis_passes_per_step": passes_per_step,
        "sis_candidates_per_step": cands_per_step,
        "so_tuples_per_s": dmax_tuples / (so_ms_d3 * 1e-3) if so_ms_d3 > 0 else None,
        "so_tuples_D3": dmax_tuples,
        "so_ms_per_step": l0_ms,
        "sis_pool_pass_ms": (sum(pool_ms) / len(pool_ms)) if pool_ms else None,
        "topk_ms": (sum(ev_ms(timings, "topk")) / len(ev_ms(timings, "topk"))) if ev_ms(timings, "topk") else None,
        "roofline": roof,
        "forms": forms,
        "autotune": tuned,
        "fit": {"rmse": [r.rmse for r in last], "best_ids": [list(map(int, r.best_ids)) for r in last],
                "keep": [r.keep for r in last]},
    }
    if not args.no_batched:
        out["batched"] = batched_fit(log, autotune=not args.no_autotune)
    if args.c5:
        if learned_params is None:
            learned_params, forms["learned_training"] = train_proposal(args, log)
        out["learned_c5"] = learned_c5(learned_params, args, log)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        sub = None
        if p.rect and len(last) == p.dmax:
            from oracle import oracle as O
            sp = O.Space(p.X.shape[1], p.unary, p.binary, p.rung, p.rect)
            F, ok = sp.eval(p.X, np.sort(last[-1].sub_ids))
            sub = (F, p.y, p.dmax)
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds, sub)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

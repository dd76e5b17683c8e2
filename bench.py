#!/usr/bin/env python3
"""Benchmark: uncompressed words/s analysed by word count (+ sort) on a
Sequitur-compressed synthetic corpus resident in HBM, on one MI355X.

One step = the whole path from the compressed grammar in device memory to
the final results: load (validation, in-degrees, level frontiers, top-down
weights), word count, sort. Inputs are generated and compressed on the host
before timing and copied to the GPU once.

Prints one JSON line (last line of stdout).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def describe(name: str) -> str:
    import synth
    s = synth.WORKLOADS[name]
    return (f"{name}: {s.files} file(s), {s.tokens} tokens, vocab {s.vocab} Zipf({s.zipf_s}), "
            f"{int(s.copy_frac * 100)}% span repeats of {s.span_min}-{s.span_max} tokens, Sequitur grammar "
            f"resident in HBM; step = load (validate, levels, weights) + word count + sort")


def cpu_baseline(g, tokens: int, budget_s: float) -> dict:
    """The oracle's sequential DAG-traversal word count on the host, repeated
    within a time budget on the full grammar."""
    import oracle
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.traverse_word_count(g)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 20:
            break
    per = el / reps
    return {"value": tokens / per, "unit": "words/s", "cores": 1, "kind": "oracle",
            "sample": f"whole grammar, {reps} run(s) of the sequential traversal word count, {per:.3f} s each"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="wc-100m")
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the workload (testing only)")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds for the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it"}))
        sys.exit(2)

    import numpy as np
    import synth
    t0 = time.time()
    c, g = synth.workload(args.workload, args.scale)
    T = len(c.tokens)
    log(f"corpus {args.workload} x{args.scale}: T={T} F={g.num_files} -> grammar R={g.num_rules} S={len(g.sym)} "
        f"({time.time() - t0:.1f}s)")
    del c

    import torch
    import paper_2106_06889_amd as gt
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ro = torch.from_numpy(g.rule_off).to(dev)
    sym = torch.from_numpy(g.sym).to(dev)
    fo = torch.from_numpy(g.file_off).to(dev)
    V = g.vocab
    R, S = g.num_rules, len(g.sym)
    arena = 64 * R + 8 * S + 64 * V + (64 << 20)
    ctx = gt.Context(arena, dev)
    counts = torch.empty(V, dtype=torch.int64, device=dev)
    ids = torch.empty(V, dtype=torch.int32, device=dev)
    scnt = torch.empty(V, dtype=torch.int64, device=dev)
    num = torch.empty(1, dtype=torch.int64, device=dev)
    lib = gt.lib()
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    def step(ev=None):
        G = ctx.load(ro, sym, fo, V, borrow=True)
        if ev is not None:
            ev[0].record(stream)
        gt.gtadoc._check(lib.gtadoc_word_count(G.handle, counts.data_ptr(), sp))
        if ev is not None:
            ev[1].record(stream)
        gt.gtadoc._check(lib.gtadoc_sort(G.handle, counts.data_ptr(), ids.data_ptr(), scnt.data_ptr(),
                                         num.data_ptr(), sp))
        G.free()

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    # sanity: exact against the grammar's own token count
    G = ctx.load(ro, sym, fo, V, borrow=True)
    st = G.stats
    G.free()
    assert st["tokens"] == T, (st["tokens"], T)
    total = int(gt.to_u64(counts).sum())
    assert total == T, (total, T)
    log(f"stats: {st}")

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_step = 1e3 * t_total / args.steps
    wc_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    log(f"{args.steps} steps in {t_total:.3f}s ({ms_step:.3f} ms/step); word-count call {wc_ms * 1e3:.1f} us")

    # algorithmic bytes of the word-count pass: symbols, rule offsets, weights, counts
    wc_bytes = 4 * S + 8 * (R + 1) + 8 * R + 8 * V
    achieved = wc_bytes / (wc_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "word count pass (gtadoc_word_count)", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes": wc_bytes}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cpu = cpu_baseline(g, T, args.cpu_budget)
        log(f"cpu baseline {cpu['value']:.3e} words/s")
    out = {
        "metric": "uncompressed words/s analysed (word count)",
        "value": T * args.steps / t_total,
        "unit": "words/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": describe(args.workload) if args.scale == 1.0 else f"{args.workload} x{args.scale}",
                   "tokens": T, "rules": R, "symbols": S, "depth": st["depth"], "files": g.num_files,
                   "vocab": V, "word_count_call_us": wc_ms * 1e3},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

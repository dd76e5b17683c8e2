#!/usr/bin/env python3
"""Benchmark of exact analytics on Sequitur-compressed synthetic corpora
resident in HBM, on one MI355X.

Default (`--query wc`): uncompressed words/s analysed by word count (+ sort).
One step = the whole path from the compressed grammar in device memory to the
final results: load (validation, in-degrees, level frontiers, top-down
weights), word count, sort. Other modes:
  --query sc     step = load + sequence count n = 2 and n = 3 (nested-repeat corpus)
  --query tv     step = load + term vector + inverted index (4,000 files)
  --query serve  256 resident grammars, Poisson query stream, continuous
                 batching vs one query per call (p50/p99 latency)
Inputs are generated and compressed on the host before timing and copied to
the GPU once. Prints one JSON line (last line of stdout).
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
DEFAULT_WORKLOAD = {"wc": "wc-100m", "sc": "seq-20m", "sc4": "seq4-20m", "tv": "tv-4000files",
                    "rii": "tv-4000files"}
SEQ_NS = {"sc": (2, 3), "sc4": (4,)}
METRIC = {"wc": "uncompressed words/s analysed (word count)",
          "sc": "uncompressed words/s analysed (sequence count, n = 2 and 3)",
          "sc4": "uncompressed words/s analysed (sequence count, n = 4)",
          "tv": "uncompressed words/s analysed (term vector + inverted index)",
          "rii": "uncompressed words/s analysed (term vector + ranked inverted index)"}
STEP = {"wc": "load (validate, in-degrees, weights by the dataflow walk) + word count + sort",
        "sc": "load (validate, in-degrees, levels and weights) + sequence count n=2 + sequence count n=3",
        "sc4": "load (validate, in-degrees, levels and weights) + sequence count n=4",
        "tv": "load (validate, in-degrees, levels and weights) + term vector + inverted index",
        "rii": "load (validate, in-degrees, levels and weights) + term vector + ranked inverted index"}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def describe(name: str, query: str) -> str:
    import synth
    s = synth.WORKLOADS[name]
    shape = (f"{s.motif_chains} nested motif chains of {s.motif_levels} levels" if s.kind == 1 else
             f"{int(s.copy_frac * 100)}% span repeats of {s.span_min}-{s.span_max} tokens"
             + (" from earlier files" if s.cross_file else ""))
    return (f"{name}: {s.files} file(s), {s.tokens if s.files == 1 else '~lognormal sizes'} tokens, vocab {s.vocab} "
            f"Zipf({s.zipf_s}), {shape}, Sequitur grammar resident in HBM; step = {STEP[query]}")


def host_info() -> dict:
    """Host CPUs the baseline ran on: usable cores, model name."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0))
    return {"nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def baseline_threads() -> int:
    usable = len(os.sched_getaffinity(0))
    try:
        return max(1, min(usable, int(os.environ.get("OMP_NUM_THREADS", usable))))
    except ValueError:
        return usable


def timed(fn, budget_s: float, max_reps: int = 20) -> tuple[float, int]:
    """Seconds per run of fn (repeated within the budget) and the runs made."""
    reps, t0 = 0, time.perf_counter()
    while True:
        fn()
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= max_reps:
            return el / reps, reps


def cpu_baseline(query: str, g, file_tokens, budget_s: float) -> dict:
    """The oracle timed on the host: the sequential DAG traversal on one core
    (the primary figure: the paper compares against sequential TADOC), the
    same traversal on all usable cores, and (word count) the brute force
    that decompresses then counts, on one core. Word count and sequence
    count run on the whole grammar, repeated within a time budget; the term
    vector over the leading files until the budget is spent."""
    import oracle
    import synth
    T = int(file_tokens.sum())
    threads = baseline_threads()
    variants = []
    if query in ("tv", "rii"):
        F = g.num_files

        def run_files(fn, budget, files_per_call):
            f, t0 = 0, time.perf_counter()
            while f < F and time.perf_counter() - t0 < budget:
                hi = min(F, f + files_per_call)
                off, word, cnt = fn(synth.Grammar(g.rule_off, g.sym, g.file_off[f:hi + 1], g.vocab))
                if query == "rii":
                    oracle.ranked_inverted_index(off, word, cnt, g.vocab)
                f = hi
            el = time.perf_counter() - t0
            return int(file_tokens[:f].sum()) / el, f, el
        what = "term vector" + (" + ranked inverted index of each chunk" if query == "rii" else "")
        chunk = max(1, F // 400)
        v1, f1, e1 = run_files(oracle.traverse_term_vector, budget_s, chunk)
        vp, fp, ep = run_files(lambda h: oracle.traverse_term_vector_parallel(h, threads), budget_s / 2,
                               chunk * threads)
        variants.append({"value": vp, "unit": "words/s", "cores": threads,
                         "sample": f"file-parallel top-down traversal {what} on {threads} threads, "
                                   f"first {fp} of {F} files in {ep:.1f} s"})
        return {"value": v1, "unit": "words/s", "cores": 1, "kind": "oracle",
                "sample": f"per-file top-down traversal {what}, first {f1} of {F} files in {e1:.1f} s",
                "variants": variants, "host": host_info()}
    if query == "wc":
        per, reps = timed(lambda: oracle.traverse_word_count(g), budget_s)
        what = "word count"
        pp, rp = timed(lambda: oracle.traverse_word_count_parallel(g, threads), budget_s / 3)
        variants.append({"value": T / pp, "unit": "words/s", "cores": threads,
                         "sample": f"whole grammar, {rp} run(s) of the traversal word count with the "
                                   f"accumulation on {threads} threads, {pp:.3f} s each"})
        pb, rb = timed(lambda: oracle.brute_word_count(g), budget_s / 3, max_reps=5)
        variants.append({"value": T / pb, "unit": "words/s", "cores": 1,
                         "sample": f"whole grammar, {rb} run(s) of decompress-then-count, {pb:.3f} s each"})
    else:
        per, reps = timed(lambda: [oracle.traverse_sequence_count(g, n) for n in SEQ_NS[query]], budget_s)
        what = "sequence count " + " and ".join(f"n={n}" for n in SEQ_NS[query])
    return {"value": T / per, "unit": "words/s", "cores": 1, "kind": "oracle",
            "sample": f"whole grammar, {reps} run(s) of the sequential traversal {what}, {per:.3f} s each",
            "variants": variants, "host": host_info()}


def measured_traffic(kernel: str | None, workload: str):
    """HBM bytes per launch of a kernel from a committed PMC summary
    (profiles/*_hbm_traffic.md), or None when there is none for this
    workload or the kernel's source has changed since the counters were
    taken."""
    import glob
    import hashlib
    if not kernel:
        return None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.md"))):
        for line in open(path):
            if not line.startswith("traffic-record: "):
                continue
            rec = json.loads(line[len("traffic-record: "):])
            if rec.get("kernel") != kernel or rec.get("workload") != workload or "sources" not in rec:
                continue
            h = hashlib.sha256()
            try:
                for src in rec["sources"]:
                    h.update(open(os.path.join(ROOT, src), "rb").read())
            except OSError:
                continue
            if h.hexdigest() == rec["sources_sha256"]:
                return int(rec["traffic_bytes_per_launch"])
    return None


def dist(ms: list) -> dict:
    """Median and 90th percentile of per-step device times (ms)."""
    import numpy as np
    a = np.asarray(ms, dtype=np.float64)
    return {"median": float(np.median(a)), "p90": float(np.percentile(a, 90)), "n": int(a.size)}


def roofline(name: str, nbytes: float, us: float) -> dict:
    achieved = nbytes / (us * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": int(nbytes),
            "avg_us": us}


def run_query(args):
    import numpy as np
    import synth
    t0 = time.time()
    c, g = synth.workload(args.workload, args.scale)
    T = len(c.tokens)
    file_tokens = np.diff(c.file_off)
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
    R, S, F = g.num_rules, len(g.sym), g.num_files
    root_syms = int(g.rule_off[1] - g.rule_off[0])
    q = args.query
    arena = 64 * R + 8 * S + 64 * V + (64 << 20)
    if q in SEQ_NS:
        # exact table (16 B per slot, slots < 2 (n-1) S + 2), results, sort scratch, head/tail/len
        arena += 256 * S + 48 * R
    if q in ("tv", "rii"):
        arena += 48 * T // 10 + 64 * S + 64 * R + 16 * V + (1 << 30)
    if q == "rii":
        arena += 8 * T // 3  # term frequencies of the ranked index, 8 B per (file, word) pair
    ctx = gt.Context(arena, dev)
    counts = torch.empty(V, dtype=torch.int64, device=dev)
    ids = torch.empty(V, dtype=torch.int32, device=dev)
    scnt = torch.empty(V, dtype=torch.int64, device=dev)
    num = torch.empty(1, dtype=torch.int64, device=dev)
    lib = gt.lib()
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    sizes = {}

    # the word count needs weights only; the other queries also need the
    # levels, which the load then builds with the level walk
    levels = q != "wc"

    # the word-count step calls the C ABI directly (no binding objects per
    # step: the load's read-back drains the stream, so host time between the
    # calls idles the GPU)
    import ctypes
    load_flags = gt.gtadoc.IN_DEVICE | gt.gtadoc.IN_BORROW | (gt.gtadoc.LOAD_LEVELS if levels else 0)
    load_args = (ctx.handle, ro.data_ptr(), R, sym.data_ptr(), S, fo.data_ptr(), F, V, load_flags, sp)

    def step():
        if q == "wc":
            h = ctypes.c_void_p()
            gt.gtadoc._check(lib.gtadoc_load_grammar(*load_args, ctypes.byref(h)))
            gt.gtadoc._check(lib.gtadoc_word_count(h, counts.data_ptr(), sp))
            gt.gtadoc._check(lib.gtadoc_sort(h, counts.data_ptr(), ids.data_ptr(), scnt.data_ptr(),
                                             num.data_ptr(), sp))
            gt.gtadoc._check(lib.gtadoc_free_grammar(h))
            return
        G = ctx.load(ro, sym, fo, V, borrow=True, levels=levels)
        if q in SEQ_NS:
            for n in SEQ_NS[q]:
                res = G.sequence_count(n)
                sizes[f"U{n}"] = res.length(0)
                res.free()
        else:
            tv = G.term_vector()
            sizes["nnz_tv"] = tv.length(1)
            ii = G.ranked_inverted_index_from(tv) if q == "rii" else G.inverted_index_from(tv)
            sizes["nnz_ii"] = ii.length(1)
            ii.free()
            tv.free()
        G.free()

    # launch shape of the load and the word-count chunk: the tuner's cache for
    # this GPU and size, else a greedy search (the paper's parameter
    # selection) on this grammar before anything is timed
    from paper_2106_06889_amd import autotune
    tune_key = f"{autotune.arch()}/{'load-levels' if levels else 'load-flow'}/{autotune.size_bucket(T)}"
    tuned = "defaults"
    if not args.no_tune:
        if autotune.apply(ctx, tune_key):
            tuned = "cache"
        else:
            res = autotune.tune_load(ctx, ro, sym, fo, V, reps=10, levels=levels)
            autotune.save(tune_key, res)
            tuned = "searched on this grammar before the timed region"
    tuned_params = {name: ctx.get_param(p) for p, name in autotune.NAMES.items()
                    if p in (autotune.LOAD_CANDIDATES if levels else autotune.FLOW_CANDIDATES)}
    log(f"load parameters ({tuned}): {tuned_params}")

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    # sanity: exact totals against the grammar's own token count
    G = ctx.load(ro, sym, fo, V, borrow=True, levels=levels)
    G.build_levels()  # the depth, for the record (built here when the load did not)
    st = G.stats
    if q == "wc":
        total = int(gt.to_u64(G.word_count()).sum())
        assert total == T, (total, T)
    elif q in SEQ_NS:
        lens = file_tokens
        for n in SEQ_NS[q]:
            res = G.sequence_count(n)
            tot = int(gt.to_u64(res.arrays[1]).sum())
            res.free()
            want = int(np.maximum(lens - n + 1, 0).sum())
            assert tot == want, (n, tot, want)
    else:
        res = G.term_vector()
        tot = int(gt.to_u64(res.arrays[2]).sum())
        res.free()
        assert tot == T, (tot, T)
    G.free()
    assert st["tokens"] == T, (st["tokens"], T)
    log(f"stats: {st}")

    def read_phases():
        out = {}
        for ph in gt.PHASES:
            ms, n = ctx.phase_time(ph, reset=True)
            if n:
                out[ph] = {"avg_us": 1e3 * ms / n, "count": n}
        return out

    def tv_total(ph):
        # the term vector pass = rule tables + per-file reduce, per call
        if "tv_tables" in ph and "tv_reduce" in ph:
            ph["term_vector"] = {"avg_us": ph["tv_tables"]["avg_us"] + ph["tv_reduce"]["avg_us"],
                                 "count": ph["tv_tables"]["count"]}
        return ph

    # phase run (not part of `value`): every phase timed, for the per-kernel
    # figures and the rooflines of the other kernels
    n_phase = max(3, min(args.steps, 10))
    ctx.set_param(gt.PARAM_TIMING, 1)
    read_phases()
    for _ in range(n_phase):
        step()
    torch.cuda.synchronize()
    phases = tv_total(read_phases())
    # algorithmic bytes of each timed kernel (what the method must move):
    #   level walk  : non-root bodies, rule offsets, weights written, level order written
    #   word count  : all bodies, rule offsets, weights, counts written
    #   seq windows : all bodies, rule offsets, weights, len, head+tail, the distinct (key, count) pairs
    #   tv tables   : non-root bodies, rule offsets, the per-rule tables written (8 B per entry)
    #   dataflow walk: non-root bodies, rule offsets, weights written
    wc_bytes = 4 * S + 8 * (R + 1) + 8 * R + 8 * V
    lv_bytes = 4 * (S - root_syms) + 8 * (R + 1) + 8 * R + 4 * R
    flow_bytes = 4 * (S - root_syms) + 8 * (R + 1) + 8 * R
    walk_kernel = "k_levels" if levels else "k_flow"
    cands = {"levels": ("level walk (k_levels)", lv_bytes) if levels else ("dataflow walk (k_flow)", flow_bytes),
             "word_count": ("word count pass (bucket scatter + reduce)", wc_bytes)}
    if q in SEQ_NS:
        ns = SEQ_NS[q]
        U = sum(sizes.get(f"U{n}", 0) for n in ns)
        cands["seq_windows"] = ("owned windows into the exact table (k_seq_windows)",
                                (len(ns) * (4 * S + 8 * (R + 1) + 16 * R) + 8 * R + 16 * R + 16 * U) / len(ns))
    if q in ("tv", "rii"):
        # the term vector pass (bottom-up tables + per-file reduce), per call
        cands["term_vector"] = ("term vector pass (rule tables + per-file reduce)",
                                4 * S + 8 * (R + 1) + 8 * (F + 1) + 12 * sizes.get("nnz_tv", 0))

    dom = max((p for p in cands if p in phases), key=lambda p: phases[p]["avg_us"] * phases[p]["count"])
    dom_phases = ("tv_tables", "tv_reduce") if dom == "term_vector" else (dom,)

    # timed region: K whole steps back to back (the `value`); HIP events only
    # around the dominant kernel (its roofline) and around every step (the
    # per-step device times), since every event pair leaves the GPU idle for
    # a few microseconds
    ctx.set_param(gt.PARAM_TIMING, gt.timing_mask(*dom_phases))
    read_phases()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]  # one per step boundary
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        step()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_step = 1e3 * t_total / args.steps
    phases_timed = tv_total(read_phases())
    warm_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    log(f"{args.steps} steps in {t_total:.3f}s ({ms_step:.3f} ms/step); {dom} {phases_timed[dom]['avg_us']:.1f} us; "
        f"phase run {phases}")
    ctx.set_param(gt.PARAM_TIMING, 1)

    # cold steps: a 1 GiB write before each evicts the 256 MB Infinity Cache
    # and the L2s, so the step reads the grammar from HBM (not timed in `value`)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    n_cold = max(5, min(args.steps, 10))

    def cold_times(fn):
        times = []
        for k in range(n_cold):
            flush.fill_(k & 0xff)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        return times

    read_phases()
    cold_ms = cold_times(step)
    phases_cold = tv_total(read_phases())
    # the query alone on a grammar loaded once (weights cached at load)
    query_only = None
    if q == "wc":
        Gq = ctx.load(ro, sym, fo, V, borrow=True)

        def query():
            gt.gtadoc._check(lib.gtadoc_word_count(Gq.handle, counts.data_ptr(), sp))
            gt.gtadoc._check(lib.gtadoc_sort(Gq.handle, counts.data_ptr(), ids.data_ptr(), scnt.data_ptr(),
                                             num.data_ptr(), sp))
        for _ in range(2):
            query()
        evq = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        for k in range(args.steps):
            evq[k][0].record(stream)
            query()
            evq[k][1].record(stream)
        torch.cuda.synchronize()
        qwarm = [a.elapsed_time(b) for a, b in evq]
        qcold = cold_times(query)
        Gq.free()
        query_only = {"what": "word count + sort on a grammar loaded once (weights cached at load)",
                      "warm_ms": dist(qwarm), "cold_ms": dist(qcold),
                      "words_per_s_warm_median": T / (dist(qwarm)["median"] * 1e-3)}
    ctx.set_param(gt.PARAM_TIMING, 0)
    # release the library's device objects before the interpreter shuts down
    ctx.close()
    del counts, ids, scnt, num, ro, sym, fo, flush
    torch.cuda.synchronize()

    roof = roofline(cands[dom][0], cands[dom][1], phases_timed[dom]["avg_us"])
    if args.scale == 1.0:
        roof["traffic"] = measured_traffic(walk_kernel if dom == "levels" else None, args.workload)
    others = {p: roofline(cands[p][0], cands[p][1], phases[p]["avg_us"]) for p in cands if p in phases and p != dom}
    # the same kernels in the cold steps (grammar read from HBM, not the Infinity Cache)
    roof_cold = {p: roofline(cands[p][0], cands[p][1], phases_cold[p]["avg_us"]) for p in cands if p in phases_cold}
    if q == "wc" and "word_count" in phases_cold:
        # the flat pass on rule-body bytes alone (4 S + 8 (R + 1))
        roof_cold["word_count_body_bytes"] = roofline("word count pass, rule-body bytes",
                                                      4 * S + 8 * (R + 1), phases_cold["word_count"]["avg_us"])

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cpu = cpu_baseline(q, g, file_tokens, args.cpu_budget)
        log(f"cpu baseline {cpu['value']:.3e} words/s")
    out = {
        "metric": METRIC[q],
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
        "config": {"workload": describe(args.workload, q) if args.scale == 1.0 else f"{args.workload} x{args.scale}",
                   "tokens": T, "rules": R, "symbols": S, "root_symbols": root_syms, "depth": st["depth"],
                   "files": F, "vocab": V, **sizes, "launch_params": tuned_params, "launch_params_from": tuned},
        "roofline": roof,
        "phases_us": {p: v["avg_us"] for p, v in phases.items()},
        "phases_from": f"{n_phase} steps with every phase timed, outside the timed region",
        "roofline_other": others,
        "step_device_ms": {"warm": dist(warm_ms), "cold": dist(cold_ms),
                           "cold_protocol": "1 GiB device write before each step"},
        "phases_cold_us": {p: v["avg_us"] for p, v in phases_cold.items()},
        "roofline_cold": roof_cold,
        "query_only": query_only,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# ------------------------------------------- traversal / baseline comparisons
def device_times(stream, fn, reps: int, cold: bool = False, flush=None) -> dict:
    """Median and p90 of the device time of fn (HIP events on `stream`),
    after two untimed runs; cold: a 1 GiB write before each run."""
    import torch
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    ms = []
    for k in range(reps):
        if cold:
            flush.fill_(k & 0xff)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return dist(ms)


def run_compare(args):
    """--query uncompressed: the compressed path beside analytics on the
    uncompressed text on the same GPU (the text resident in HBM, and
    decompression on the GPU followed by the same analytics), per query kind
    (Evaluation, Discussion: comparison with GPU-accelerated uncompressed
    analytics). --query tvsel: term vector by the bottom-up and the top-down
    traversal and the selector's choice (Evaluation, Optimization Analysis:
    top-down vs. bottom-up traversals)."""
    import numpy as np
    import synth
    t0 = time.time()
    c, g = synth.workload(args.workload, args.scale)
    T = len(c.tokens)
    file_tokens = np.diff(c.file_off)
    log(f"corpus {args.workload} x{args.scale}: T={T} F={g.num_files} -> grammar R={g.num_rules} S={len(g.sym)} "
        f"({time.time() - t0:.1f}s)")
    import torch
    import paper_2106_06889_amd as gt
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ro = torch.from_numpy(g.rule_off).to(dev)
    sym = torch.from_numpy(g.sym).to(dev)
    fo = torch.from_numpy(g.file_off).to(dev)
    text = torch.from_numpy(c.tokens).to(dev)
    text_off = torch.from_numpy(c.file_off).to(dev)
    text_ro = torch.tensor([0, T], dtype=torch.int64, device=dev)
    del c
    V, R, S, F = g.vocab, g.num_rules, len(g.sym), g.num_files
    ctx = gt.Context(96 * R + 72 * S + 80 * V + 64 * T + 8 * F * V + (4 << 30), dev)
    stream = torch.cuda.current_stream()
    flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    reps = args.steps
    counts = torch.empty(V, dtype=torch.int64, device=dev)
    ids = torch.empty(V, dtype=torch.int32, device=dev)
    scnt = torch.empty(V, dtype=torch.int64, device=dev)
    num = torch.empty(1, dtype=torch.int64, device=dev)
    lib = gt.lib()
    sp = stream.cuda_stream

    def query(G, kind):
        if kind == "wc":
            gt.gtadoc._check(lib.gtadoc_word_count(G.handle, counts.data_ptr(), sp))
            gt.gtadoc._check(lib.gtadoc_sort(G.handle, counts.data_ptr(), ids.data_ptr(), scnt.data_ptr(),
                                             num.data_ptr(), sp))
        elif kind == "tv":
            G.term_vector().free()
        else:
            G.sequence_count(2).free()

    out = {"metric": None, "unit": "words/s", "n_gpus": 1, "steps": reps, "warmup": 2, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": describe(args.workload, "wc") if args.scale == 1.0 else
                      f"{args.workload} x{args.scale}", "tokens": T, "rules": R, "symbols": S, "files": F,
                      "vocab": V}}
    if args.query == "uncompressed":
        kinds = ["tv"] if F > 1 else ["wc", "sc2"]
        rows = {}
        for kind in kinds:
            lv = kind != "wc"  # the term vector and the n-gram count also need the levels

            # compressed: load (weights, levels when needed) + query from the resident grammar
            def comp():
                G = ctx.load(ro, sym, fo, V, borrow=True, levels=lv)
                query(G, kind)
                G.free()

            # uncompressed, resident text: the same query kernels on a one-rule grammar of the tokens
            def plain():
                P = ctx.load(text_ro, text, text_off, V, borrow=True, levels=lv)
                query(P, kind)
                P.free()

            # decompression on the GPU, then the analytics on the text
            Gd = ctx.load(ro, sym, fo, V, borrow=True, levels=True)

            def dec_plain():
                tok, off = Gd.decompress()
                P = ctx.load(text_ro, tok, off, V, borrow=True, levels=lv)
                query(P, kind)
                P.free()
            r = {"compressed_ms": device_times(stream, comp, reps),
                 "uncompressed_resident_ms": device_times(stream, plain, reps),
                 "decompress_then_query_ms": device_times(stream, dec_plain, reps),
                 "compressed_cold_ms": device_times(stream, comp, max(3, reps // 2), True, flush),
                 "uncompressed_resident_cold_ms": device_times(stream, plain, max(3, reps // 2), True, flush)}
            Gd.free()
            r["speedup_vs_resident_text"] = r["uncompressed_resident_ms"]["median"] / r["compressed_ms"]["median"]
            r["speedup_vs_decompress"] = r["decompress_then_query_ms"]["median"] / r["compressed_ms"]["median"]
            rows[kind] = r
            log(f"{kind}: compressed {r['compressed_ms']['median']:.3f} ms, text {r['uncompressed_resident_ms']['median']:.3f}"
                f" ms, decompress+text {r['decompress_then_query_ms']['median']:.3f} ms")
        first = rows[kinds[0]]
        out.update({"metric": f"uncompressed words/s analysed ({'+'.join(kinds)}), compressed path vs GPU "
                              f"uncompressed baseline",
                    "value": T / (first["compressed_ms"]["median"] * 1e-3),
                    "ms_per_step": first["compressed_ms"]["median"], "comparison": rows,
                    "step": "compressed: load + query; uncompressed: load of the one-rule text grammar + the same "
                            "query; decompress: GPU decompression + that"})
    else:
        Gs = ctx.load(ro, sym, fo, V, borrow=True, levels=True)
        choice = {gt.TV_TOP_DOWN: "top-down", gt.TV_BOTTOM_UP: "bottom-up"}[Gs.tv_strategy()]
        rows = {}
        for name, strat in (("bottom-up", gt.TV_BOTTOM_UP), ("top-down", gt.TV_TOP_DOWN)):
            rows[name] = device_times(stream, lambda: Gs.term_vector(strat).free(), reps)
            log(f"term vector {name}: {rows[name]['median']:.3f} ms")
        Gs.free()
        best = min(rows, key=lambda k: rows[k]["median"])
        out.update({"metric": "uncompressed words/s analysed (term vector), bottom-up vs top-down traversal",
                    "value": T / (rows[choice]["median"] * 1e-3), "ms_per_step": rows[choice]["median"],
                    "traversals_ms": rows, "selector_choice": choice, "fastest": best,
                    "step": "term vector on a grammar loaded once"})
    ctx.close()
    del text, text_off, ro, sym, fo, flush
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ serving
def run_serve(args):
    import numpy as np
    import synth
    t0 = time.time()
    specs = synth.serving_specs(count=args.grammars, scale=args.scale)
    pairs = synth.serving_grammars(specs, workers=args.workers)
    totT = sum(t for _, t in pairs)
    log(f"{len(pairs)} grammars, sum T = {totT} ({time.time() - t0:.1f}s)")

    import torch
    import paper_2106_06889_amd as gt
    from paper_2106_06889_amd import serve
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    gbytes = sum(16 * len(g.sym) + 80 * g.num_rules + 16 * g.num_files for g, _ in pairs)
    biggest = max(t for _, t in pairs)
    arena = gbytes + 64 * biggest + 16 * sum(len(g.sym) for g, _ in pairs) // 4 + (2 << 30)
    ctx = gt.Context(arena, dev)
    loaded = [ctx.load(g.rule_off, g.sym, g.file_off, g.vocab) for g, _ in pairs]
    torch.cuda.synchronize()
    log(f"loaded; arena in use {ctx.usage()[0] / 2**30:.2f} GiB of {arena / 2**30:.2f}")
    # launch parameters of the batched word count: the tuner's cache for this
    # GPU and size, else a greedy search on a sample of the grammars (saved)
    from paper_2106_06889_amd import autotune
    key = f"{autotune.arch()}/batch_word_count/{autotune.size_bucket(totT // len(pairs))}"
    tuned = autotune.apply(ctx, key)
    if not tuned:
        res = autotune.tune_batch_word_count(ctx, loaded[:: max(1, len(loaded) // 32)], reps=3)
        autotune.save(key, res)
        tuned = autotune.apply(ctx, key)
    params = {name: ctx.get_param(p) for p, name in autotune.NAMES.items()}
    log(f"batched word count parameters ({'cache' if tuned else 'defaults'}): {params}")
    srv = serve.Server(ctx, loaded, max_batch=args.max_batch)
    t1 = time.time()
    srv.prepare()  # per-grammar query footprints (admission by memory)
    log(f"query footprints measured in {time.time() - t1:.1f}s")
    # warm up every query kind once on a few grammars
    srv.run(serve.poisson_trace(64, 0, len(loaded), seed=1), realtime=False)
    srv.run_plain(serve.poisson_trace(32, 0, len(loaded), seed=2), realtime=False)
    torch.cuda.synchronize()

    # closed-loop capacity of the served system: every query present at t = 0
    closed = serve.poisson_trace(args.queries, 0, len(loaded), seed=synth.SEED_BASE + 6)
    t1 = time.perf_counter()
    srv.run(closed, realtime=False)
    cap = args.queries / (time.perf_counter() - t1)
    t1 = time.perf_counter()
    srv.run_plain(closed, realtime=False)
    cap_plain = args.queries / (time.perf_counter() - t1)
    log(f"closed-loop capacity: served {cap:.1f} q/s, plain {cap_plain:.1f} q/s")
    loads = {}
    for frac in (0.70, 0.95):
        rate = frac * cap
        trace = serve.poisson_trace(args.queries, rate, len(loaded), seed=synth.SEED_BASE + 7)
        span = trace[-1].arrival
        ra, rb = srv.run(trace), srv.run_plain(trace)
        a, b = serve.percentiles(ra), serve.percentiles(rb)
        a["by_kind"] = {k: serve.percentiles([r for r in ra if r.kind == k]) for k in serve.KINDS}
        b["by_kind"] = {k: serve.percentiles([r for r in rb if r.kind == k]) for k in serve.KINDS}
        loads[f"{frac:.2f}C"] = {"rate_qps": rate, "trace_s": span, "served": a, "plain": b}
        log(f"lambda={frac:.2f}C ({rate:.0f} q/s): served p50 {a['p50_ms']:.2f} p99 {a['p99_ms']:.2f} ms; "
            f"plain p50 {b['p50_ms']:.2f} p99 {b['p99_ms']:.2f} ms")
    srv.close()
    for G in loaded:
        G.free()
    ctx.close()
    torch.cuda.synchronize()
    mean_T = totT / len(pairs)
    out = {
        "metric": "served queries/s at saturation (closed loop, mixed word count / term vector / bigram)",
        "value": cap, "unit": "queries/s", "n_gpus": 1, "steps": args.queries, "warmup": 96,
        "ms_per_step": 1e3 / cap, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{len(pairs)} resident grammars, sizes log-uniform 1e4-2e7 tokens x{args.scale}, "
                               f"sum T = {totT}; queries 50% word count, 30% term vector, 20% bigram count",
                   "queries_per_trace": args.queries, "batched_word_count_params": params,
                   "max_batch": args.max_batch, "plain_capacity_qps": cap_plain,
                   "served_words_per_s": cap * mean_T},
        "latency": loads,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--query", choices=("wc", "sc", "sc4", "tv", "rii", "serve", "uncompressed", "tvsel"),
                    default="wc")
    ap.add_argument("--workload", default=None)
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the workload (testing only)")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds for the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch parameters")
    ap.add_argument("--grammars", type=int, default=256, help="serve: resident grammars")
    ap.add_argument("--queries", type=int, default=20000, help="serve: queries per trace")
    ap.add_argument("--max-batch", type=int, default=64, help="serve: word counts per batch")
    ap.add_argument("--workers", type=int, default=16, help="serve: host processes generating grammars")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the multi-GPU path (sharding by symbol range or files) is not implemented"}))
        sys.exit(2)
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 5}), flush=True)
        return
    if args.query == "serve":
        run_serve(args)
        return
    if args.query in ("uncompressed", "tvsel"):
        args.workload = args.workload or {"uncompressed": "wc-100m", "tvsel": "tv-4files"}[args.query]
        run_compare(args)
        return
    args.workload = args.workload or DEFAULT_WORKLOAD[args.query]
    run_query(args)


if __name__ == "__main__":
    main()

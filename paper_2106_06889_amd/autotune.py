"""Autotuner for the library's launch parameters.

Following the paper's parameter selection (Section Fine-Grained Thread-Level
Execution Engine, parameter selection): take a sample of the input and set
the parameters greedily, one at a time, keeping the others fixed; without a
sample, fall back to defaults. Two groups of tunables, each searched
greedily on its own:
  * the batched word count: persistent scatter workgroups per CU and the
    reduce chunk (timed on a sample batch of grammars);
  * the load's level walk and the word count of one grammar: the bucketed
    mode threshold, the thread-group threshold for long rule bodies (the
    paper's "16 times the average elements per thread" rule), the width
    below which levels run on fewer workgroups and how many, the width below
    which one workgroup finishes, and the word-count reduce chunk (timed on a
    sample grammar: load, then word count).
Each candidate is timed with HIP events on the query stream. Results are
cached in a JSON file keyed by (GPU architecture, query kind, size bucket).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import gtadoc as gt

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

CANDIDATES = {
    gt.PARAM_BATCH_BLOCKS_PER_CU: [1, 2, 4, 8],
    gt.PARAM_WC_CHUNK: [8192, 16384, 32768, 65536],
}
DEFAULTS = {gt.PARAM_BATCH_BLOCKS_PER_CU: 4, gt.PARAM_WC_CHUNK: 16384}
NAMES = {gt.PARAM_BATCH_BLOCKS_PER_CU: "batch_blocks_per_cu", gt.PARAM_WC_CHUNK: "wc_chunk",
         gt.PARAM_LEVEL_WIDE: "level_wide", gt.PARAM_LEVEL_LONG_BODY: "level_long_body",
         gt.PARAM_LEVEL_MID_RULES: "level_mid_rules", gt.PARAM_LEVEL_MID_BLOCKS: "level_mid_blocks",
         gt.PARAM_LEVEL_TAIL_RULES: "level_tail_rules", gt.PARAM_FLOW_KEEP: "flow_keep",
         gt.PARAM_FLOW_GROUP: "flow_group", gt.PARAM_FLOW_CHUNK: "flow_chunk"}

# the load (level walk) and the single-grammar word count, in search order
LOAD_CANDIDATES = {
    gt.PARAM_LEVEL_WIDE: [0, 131072, 262144, 524288, 1 << 30],
    gt.PARAM_LEVEL_MID_RULES: [16384, 32768, 49152, 98304],
    gt.PARAM_LEVEL_MID_BLOCKS: [8, 16, 32, 64],
    gt.PARAM_LEVEL_TAIL_RULES: [256, 1024, 4096, 8192],
    gt.PARAM_LEVEL_LONG_BODY: [16, 32, 64, 128],
    gt.PARAM_WC_CHUNK: [8192, 16384, 32768, 65536],
}
LOAD_DEFAULTS = {gt.PARAM_LEVEL_WIDE: 262144, gt.PARAM_LEVEL_MID_RULES: 49152, gt.PARAM_LEVEL_MID_BLOCKS: 32,
                 gt.PARAM_LEVEL_TAIL_RULES: 1024, gt.PARAM_LEVEL_LONG_BODY: 32, gt.PARAM_WC_CHUNK: 16384}
# the load by the dataflow walk (no levels) and the word count
FLOW_CANDIDATES = {
    gt.PARAM_FLOW_CHUNK: [64, 128, 256, 512],
    gt.PARAM_FLOW_KEEP: [1024, 2048, 4096, 7168],
    gt.PARAM_WC_CHUNK: [8192, 16384, 32768, 65536],
}
FLOW_DEFAULTS = {gt.PARAM_FLOW_CHUNK: 128, gt.PARAM_FLOW_GROUP: 1024, gt.PARAM_FLOW_KEEP: 4096,
                 gt.PARAM_WC_CHUNK: 16384}


def arch() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def size_bucket(total_tokens: int) -> str:
    return f"2^{max(0, int(math.log2(max(total_tokens, 1))))}"


def _time(fn, reps: int) -> float:
    stream = torch.cuda.current_stream()
    fn()  # warm up (and capture, in graph mode)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def tune_batch_word_count(ctx: gt.Context, grammars, reps: int = 5, verbose: bool = False) -> dict:
    """Greedy per-parameter search for the batched word count on a sample
    batch of loaded grammars. Leaves the best values set on ctx."""
    outs = [torch.empty(g.vocab, dtype=torch.int64, device=ctx.device) for g in grammars]
    entries = sum(int(g.stats["word_syms"]) for g in grammars)
    plan = ctx.batch(len(grammars), entries)
    best = dict(DEFAULTS)
    for p, v in best.items():
        ctx.set_param(p, v)
    timings = {}
    for p, cands in CANDIDATES.items():
        scores = {}
        for v in cands:
            ctx.set_param(p, v)
            scores[v] = _time(lambda: plan.word_count(grammars, outs), reps)
            if verbose:
                print(f"[autotune] {NAMES[p]}={v}: {scores[v] * 1e3:.1f} us", flush=True)
        best[p] = min(scores, key=scores.get)
        ctx.set_param(p, best[p])
        timings[NAMES[p]] = {str(k): v for k, v in scores.items()}
    plan.close()
    return {"params": {NAMES[p]: v for p, v in best.items()}, "timings_ms": timings}


def greedy(ctx, candidates: dict, defaults: dict, run, reps: int, verbose: bool = False) -> dict:
    """Set each parameter in turn to its fastest candidate (timing `run`),
    the others fixed at their current best; leaves the best values set."""
    best = dict(defaults)
    for p, v in best.items():
        ctx.set_param(p, v)
    timings = {}
    for p, cands in candidates.items():
        scores = {}
        for v in cands:
            ctx.set_param(p, v)
            scores[v] = _time(run, reps)
            if verbose:
                print(f"[autotune] {NAMES[p]}={v}: {scores[v] * 1e3:.1f} us", flush=True)
        best[p] = min(scores, key=scores.get)
        ctx.set_param(p, best[p])
        timings[NAMES[p]] = {str(k): v for k, v in scores.items()}
    return {"params": {NAMES[p]: v for p, v in best.items()}, "timings_ms": timings}


def tune_load(ctx: gt.Context, rule_off, sym, file_off, vocab: int, reps: int = 3, verbose: bool = False,
              levels: bool = False) -> dict:
    """Greedy search of the weight walk's launch shape (the level walk with
    levels=True, else the dataflow walk) and the word-count chunk on a sample
    grammar (device tensors, loaded by borrowing): each candidate is timed
    over a load followed by a word count."""
    out = torch.empty(vocab, dtype=torch.int64, device=ctx.device)

    def run():
        G = ctx.load(rule_off, sym, file_off, vocab, borrow=True, levels=levels)
        G.word_count(out)
        G.free()
    if levels:
        return greedy(ctx, LOAD_CANDIDATES, LOAD_DEFAULTS, run, reps, verbose)
    return greedy(ctx, FLOW_CANDIDATES, FLOW_DEFAULTS, run, reps, verbose)


def load_cache() -> dict:
    if os.path.exists(CACHE_PATH):
        with open(CACHE_PATH) as f:
            return json.load(f)
    return {}


def save(key: str, result: dict, path: str = CACHE_PATH):
    cache = load_cache() if path == CACHE_PATH else {}
    cache[key] = result
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def apply(ctx: gt.Context, key: str) -> bool:
    """Set the cached parameters for `key` on ctx; False (defaults kept) when
    the key is not cached."""
    entry = load_cache().get(key)
    if not entry:
        return False
    by_name = {v: k for k, v in NAMES.items()}
    for name, value in entry["params"].items():
        ctx.set_param(by_name[name], int(value))
    return True

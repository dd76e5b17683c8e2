"""Autotuner for the library's launch parameters.

Following the paper's parameter selection (Section Fine-Grained Thread-Level
Execution Engine, parameter selection): take a sample of the input and set
the parameters greedily, one at a time, keeping the others fixed; without a
sample, fall back to defaults. Here the tunables are the persistent scatter
workgroups per CU of the batched word count and the reduce chunk; each
candidate is timed with HIP events on the query stream. Results are cached in
a JSON file keyed by (GPU architecture, query kind, size bucket).
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
DEFAULTS = {gt.PARAM_BATCH_BLOCKS_PER_CU: 4, gt.PARAM_WC_CHUNK: 32768}
NAMES = {gt.PARAM_BATCH_BLOCKS_PER_CU: "batch_blocks_per_cu", gt.PARAM_WC_CHUNK: "wc_chunk"}


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

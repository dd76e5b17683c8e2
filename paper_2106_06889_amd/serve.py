"""Serving loop over grammars resident in HBM.

Queries (word count, term vector, bigram count) arrive over time against any
of the resident grammars. `Server.run` is continuous batching: every step
admits what has arrived, launches all admitted word counts as one batch
(one launch sequence over many grammars, see gtadoc_batch_word_count), and
runs the admitted term-vector and bigram queries behind it; queries that
arrive while a step is on the GPU join the next step. Admission is by
memory: a step's word counts must fit the batch plan's entry scratch, and a
term-vector or bigram query is admitted only while the arena has room for
its estimated scratch. `Server.run_plain` is the baseline: first come first
served, one query per call, waiting for each to finish.

Latency = arrival time to the moment the host sees the query's result on the
device (its completion event, or the end of a synchronizing call).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import gtadoc as gt

KINDS = ("wc", "tv", "sc2")


@dataclass
class Query:
    qid: int
    kind: str         # "wc" | "tv" | "sc2"
    grammar: int      # index into the server's grammar list
    arrival: float    # seconds from the start of the trace


@dataclass
class Record:
    qid: int
    kind: str
    grammar: int
    arrival: float
    start: float = 0.0
    finish: float = 0.0
    result: object = None

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def poisson_trace(n: int, rate: float, num_grammars: int, seed: int, mix=(0.5, 0.3, 0.2)) -> list[Query]:
    """n queries with exponential inter-arrival times (rate per second),
    kinds drawn with probabilities `mix`, grammars uniform."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n) if rate > 0 else np.zeros(n)
    t = np.cumsum(gaps) - gaps[0]
    kinds = rng.choice(len(KINDS), size=n, p=np.asarray(mix) / sum(mix))
    gs = rng.integers(0, num_grammars, size=n)
    return [Query(i, KINDS[k], int(g), float(a)) for i, (k, g, a) in enumerate(zip(kinds, gs, t))]


def percentiles(records: list[Record]) -> dict:
    lat = np.array([r.latency for r in records]) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "n": len(lat)}


class Server:
    def __init__(self, ctx: gt.Context, grammars: list, max_batch: int = 64, max_entries: int | None = None,
                 keep_results: bool = False):
        self.ctx = ctx
        self.grammars = grammars
        self.max_batch = max_batch
        words = [int(g.stats["word_syms"]) for g in grammars]
        self.max_entries = max_entries or max(sum(sorted(words)[-max_batch:]), 1)
        self.plan = ctx.batch(max_batch, self.max_entries)
        self.keep = keep_results
        self.stream = torch.cuda.current_stream()
        self.outs = [torch.empty(g.vocab, dtype=torch.int64, device=ctx.device) for g in grammars]

    def close(self):
        self.plan.close()

    # ------------------------------------------------------------ one query
    def _estimate_bytes(self, q: Query) -> int:
        st = self.grammars[q.grammar].stats
        if q.kind == "sc2":
            cap = 1 << max(10, int(2 * st["symbols"] + 1).bit_length())
            return 16 * cap + 64 * st["symbols"]
        if q.kind == "tv":
            return 40 * st["tokens"] + 64 * st["rules"] + (1 << 20)
        return 0

    def _run_single(self, q: Query, rec: Record):
        G = self.grammars[q.grammar]
        if q.kind == "wc":
            out = torch.empty(G.vocab, dtype=torch.int64, device=self.ctx.device)
            G.word_count(out)
            torch.cuda.current_stream().synchronize()
            rec.result = gt.to_u64(out) if self.keep else None
        elif q.kind == "tv":
            res = G.term_vector()
            rec.result = tuple(a.cpu().numpy() for a in res.arrays) if self.keep else None
            res.free()
        else:
            res = G.sequence_count(2)
            rec.result = tuple(gt.to_u64(a) for a in res.arrays) if self.keep else None
            res.free()
        # the call returns with its last kernels still queued (the emit after
        # the size read-back, the key sort): the result is ready only once
        # the stream has passed them
        self.stream.synchronize()

    # --------------------------------------------------- continuous batching
    def run(self, queries: list[Query], realtime: bool = True) -> list[Record]:
        pending = sorted(queries, key=lambda q: q.arrival)
        recs = {q.qid: Record(q.qid, q.kind, q.grammar, q.arrival) for q in pending}
        queue: deque[Query] = deque()
        i, n = 0, len(pending)
        inflight = None  # (event, [queries], [outs])
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        while i < n or queue or inflight:
            now = clock()
            while i < n and (not realtime or pending[i].arrival <= now):
                queue.append(pending[i])
                i += 1
            if inflight and inflight[0].query():
                done = clock()
                for q, out in zip(inflight[1], inflight[2]):
                    recs[q.qid].finish = done
                    if self.keep:
                        recs[q.qid].result = gt.to_u64(out)
                inflight = None
            if inflight is None and queue:
                # admit: word counts into the batch (entry budget), others by arena headroom
                batch, entries, rest, others = [], 0, deque(), []
                free = self.ctx.usage()[2] - self.ctx.usage()[0]
                while queue:
                    q = queue.popleft()
                    G = self.grammars[q.grammar]
                    if q.kind == "wc":
                        w = int(G.stats["word_syms"])
                        dup = any(b.grammar == q.grammar for b in batch)  # one output per grammar per step
                        if len(batch) < self.max_batch and entries + w <= self.max_entries and not dup:
                            batch.append(q)
                            entries += w
                            continue
                    else:
                        need = self._estimate_bytes(q)
                        if need <= free and len(others) < 4:
                            others.append(q)
                            free -= need
                            continue
                    rest.append(q)
                queue = rest
                if not batch and not others and queue:
                    others.append(queue.popleft())  # too big for any step: run it alone
                start = clock()
                if batch:
                    outs = [self.outs[q.grammar] for q in batch]
                    self.plan.word_count([self.grammars[q.grammar] for q in batch], outs)
                    ev = torch.cuda.Event()
                    ev.record(self.stream)
                    for q in batch:
                        recs[q.qid].start = start
                    inflight = (ev, batch, outs)
                for q in others:  # queued behind the batch on the same stream
                    recs[q.qid].start = clock()
                    self._run_single(q, recs[q.qid])
                    recs[q.qid].finish = clock()
            elif inflight is None and i < n:
                # idle until the next arrival
                wait = pending[i].arrival - clock()
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        return [recs[q.qid] for q in queries]

    # -------------------------------------------------------- plain baseline
    def run_plain(self, queries: list[Query], realtime: bool = True) -> list[Record]:
        order = sorted(queries, key=lambda q: q.arrival)
        recs = {}
        t0 = time.perf_counter()
        for q in order:
            if realtime:
                while time.perf_counter() - t0 < q.arrival:
                    pass
            r = Record(q.qid, q.kind, q.grammar, q.arrival)
            r.start = time.perf_counter() - t0
            self._run_single(q, r)
            r.finish = time.perf_counter() - t0
            recs[q.qid] = r
        return [recs[q.qid] for q in queries]

"""Serving loop over grammars resident in HBM.

Queries (word count, term vector, bigram count) arrive over time against any
of the resident grammars. `Server.run` is continuous batching: every step
admits what has arrived and fits, and runs it as one mixed batch
(gtadoc_batch_submit: the word counts as one batched launch sequence, the
other queries on the plan's streams, overlapping on the device); two plans
alternate so the next step is admitted while the previous one runs, and
queries that arrive meanwhile join the next step. Admission is by memory: a
step's word counts must fit the plan's entry scratch, and a term-vector or
bigram query is admitted only while the arena's free bytes cover its
footprint as the library measures it (gtadoc_query_bytes). `Server.run_plain`
is the baseline: first come first served, one query per call, waiting for
each to finish.

Latency = arrival time to the moment the host sees the query's result on the
device (the step's completion event, or the end of a synchronizing call).
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
    """Continuous batching over resident grammars.

    Every step admits what has arrived and fits: word counts (at most
    max_batch, one per grammar per step, word symbols within the plan) and
    term-vector / bigram queries while the arena's free bytes cover their
    footprint (gtadoc_query_bytes, measured by the library per grammar and
    kind), at most max_other per step. A step of a single query calls its
    own entry point. The step is one mixed batch
    (gtadoc_batch_submit): the word counts as one batched launch sequence,
    the other queries on the plan's own streams, their kernels overlapping on
    the device. Two plans alternate, so a step is admitted and queued while
    the previous one is still on the GPU; queries that arrive meanwhile join
    the next step. The word counts of a step are submitted first and
    complete at their own event, so they do not wait for the step's term
    vectors and bigram counts."""

    def __init__(self, ctx: gt.Context, grammars: list, max_batch: int = 64, max_entries: int | None = None,
                 keep_results: bool = False, max_other: int = 8, plans: int = 2):
        self.ctx = ctx
        self.grammars = grammars
        self.max_batch = max_batch
        self.max_other = max_other
        words = [int(g.stats["word_syms"]) for g in grammars]
        self.max_entries = max_entries or max(sum(sorted(words)[-max_batch:]), 1)
        self.plans = [ctx.batch(max_batch, self.max_entries) for _ in range(max(1, plans))]
        self.keep = keep_results
        self.stream = torch.cuda.current_stream()
        # word-count outputs per (plan, grammar): two steps in flight never share one
        self.outs = [dict() for _ in self.plans]
        self._bytes = {}

    def close(self):
        for p in self.plans:
            p.close()

    # ------------------------------------------------------------ one query
    def query_bytes(self, q: Query) -> int:
        """Arena footprint of the query (the library's measured figure)."""
        key = (q.grammar, q.kind)
        if key not in self._bytes:
            G = self.grammars[q.grammar]
            if q.kind == "tv":
                self._bytes[key] = G.query_bytes(gt.QUERY_TERM_VECTOR)
            elif q.kind == "sc2":
                self._bytes[key] = G.query_bytes(gt.QUERY_SEQUENCE_COUNT, 2)
            else:
                self._bytes[key] = 0
        return self._bytes[key]

    def prepare(self):
        """Footprints of every (grammar, kind) and the grammars' head/tail
        buffers, before any trace runs (they are measured by running each
        query once)."""
        for i in range(len(self.grammars)):
            for k in ("tv", "sc2"):
                self.query_bytes(Query(-1, k, i, 0.0))
        torch.cuda.synchronize()

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

    def _finish(self, group, now: float, recs: dict):
        _, qs, got = group
        for q, r in zip(qs, got):
            rec = recs[q.qid]
            rec.finish = now
            if isinstance(r, Exception):
                rec.result = r
                continue
            if q.kind == "wc":
                rec.result = gt.to_u64(r) if self.keep else None
            else:
                if self.keep:
                    rec.result = (tuple(a.cpu().numpy() for a in r.arrays) if q.kind == "tv"
                                  else tuple(gt.to_u64(a) for a in r.arrays))
                r.free()

    # --------------------------------------------------- continuous batching
    def run(self, queries: list[Query], realtime: bool = True) -> list[Record]:
        pending = sorted(queries, key=lambda q: q.arrival)
        recs = {q.qid: Record(q.qid, q.kind, q.grammar, q.arrival) for q in pending}
        queue: deque[Query] = deque()
        i, n = 0, len(pending)
        inflight: deque = deque()  # steps, oldest first: lists of (event, queries, results) groups
        turn = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        while i < n or queue or inflight:
            now = clock()
            while i < n and (not realtime or pending[i].arrival <= now):
                queue.append(pending[i])
                i += 1
            while inflight:
                groups = inflight[0]
                for gr in [gr for gr in groups if gr[0].query()]:
                    self._finish(gr, clock(), recs)
                    groups.remove(gr)
                if groups:
                    break
                inflight.popleft()
            if queue and len(inflight) < len(self.plans):
                # admit: word counts into the batch, the others by arena headroom
                batch, entries, rest, others = [], 0, deque(), []
                in_use, _, cap = self.ctx.usage()
                free = cap - in_use
                seen = set()
                while queue:
                    q = queue.popleft()
                    G = self.grammars[q.grammar]
                    if q.kind == "wc":
                        w = int(G.stats["word_syms"])
                        if len(batch) < self.max_batch and entries + w <= self.max_entries and q.grammar not in seen:
                            batch.append(q)
                            seen.add(q.grammar)
                            entries += w
                            continue
                    else:
                        need = self.query_bytes(q)
                        if need <= free and len(others) < self.max_other:
                            others.append(q)
                            free -= need
                            continue
                    rest.append(q)
                queue = rest
                if not batch and not others:
                    if inflight:
                        continue  # wait for memory to come back
                    others.append(queue.popleft())  # too big for any step with others: alone
                start = clock()
                slot = turn % len(self.plans)
                outs = self.outs[slot]
                groups = []
                if len(batch) + len(others) == 1:
                    # a step of one query runs it by its own entry point, as
                    # the plain loop does: the batch machinery pays off only
                    # when several queries share a step
                    q = (batch + others)[0]
                    recs[q.qid].start = start
                    G = self.grammars[q.grammar]
                    try:
                        if q.kind == "wc":
                            if q.grammar not in outs:
                                outs[q.grammar] = torch.empty(G.vocab, dtype=torch.int64, device=self.ctx.device)
                            r = G.word_count(outs[q.grammar])
                        elif q.kind == "tv":
                            r = G.term_vector()
                        else:
                            r = G.sequence_count(2)
                    except gt.GtadocError as e:
                        r = e
                    ev = torch.cuda.Event()
                    ev.record(self.stream)
                    groups.append((ev, [q], [r]))
                    batch, others = [], []
                for qs in (batch, others):  # the word counts first, at their own event
                    if not qs:
                        continue
                    spec = []
                    for q in qs:
                        G = self.grammars[q.grammar]
                        if q.kind == "wc":
                            if q.grammar not in outs:
                                outs[q.grammar] = torch.empty(G.vocab, dtype=torch.int64, device=self.ctx.device)
                            spec.append({"grammar": G, "kind": gt.QUERY_WORD_COUNT, "counts": outs[q.grammar]})
                        elif q.kind == "tv":
                            spec.append({"grammar": G, "kind": gt.QUERY_TERM_VECTOR})
                        else:
                            spec.append({"grammar": G, "kind": gt.QUERY_SEQUENCE_COUNT, "n": 2})
                        recs[q.qid].start = start
                    got = self.plans[slot].submit(spec)
                    ev = torch.cuda.Event()
                    ev.record(self.stream)
                    groups.append((ev, qs, got))
                turn += 1
                inflight.append(groups)
            elif inflight:
                pass  # poll the oldest step's events again (a sleep would add its timer slack to the latency)
            elif i < n:
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

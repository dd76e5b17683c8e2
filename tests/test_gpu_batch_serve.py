"""GPU: batched word count over many grammars (eager and hipGraph replays),
the autotuner, and the serving loop (every result in the mixed, continuously
batched run equals its result alone and the oracle)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_2106_06889_amd as gt
    assert torch.cuda.is_available()
    ctx = gt.Context(2 << 30)
    grammars = []
    for seed in range(10):
        c = synth.random_corpus(300 + seed, 1 + seed % 4, 200 + 700 * seed, [4, 60, 900][seed % 3])
        grammars.append(synth.compress(c.tokens, c.file_off, c.vocab))
    grammars.append(synth.workload("wc-200k")[1])
    grammars.append(synth.Grammar(np.array([0, 0], np.int64), np.zeros(0, np.int32), np.array([0, 0], np.int64), 7))
    loaded = [ctx.load(g.rule_off, g.sym, g.file_off, g.vocab) for g in grammars]
    want = [oracle.traverse_word_count(g) for g in grammars]
    yield ctx, grammars, loaded, want
    for G in loaded:
        G.free()
    ctx.close()


def run_batch(ctx, plan, Gs):
    import torch
    outs = [torch.full((G.vocab,), -1, dtype=torch.int64, device=ctx.device) for G in Gs]
    plan.word_count(Gs, outs)
    torch.cuda.synchronize()
    return outs


def test_batch_matches_single_and_oracle(setup):
    import paper_2106_06889_amd as gt
    ctx, grammars, loaded, want = setup
    plan = ctx.batch(len(loaded), sum(G.stats["word_syms"] for G in loaded))
    outs = run_batch(ctx, plan, loaded)
    for G, o, w in zip(loaded, outs, want):
        assert np.array_equal(gt.to_u64(o), w)
        assert np.array_equal(gt.to_u64(G.word_count()), w)
    plan.close()


def test_batch_graph_replays(setup):
    import paper_2106_06889_amd as gt
    ctx, grammars, loaded, want = setup
    ctx.set_param(gt.PARAM_BATCH_GRAPH, 1)
    try:
        plan = ctx.batch(len(loaded), sum(G.stats["word_syms"] for G in loaded))
        batches = [list(range(len(loaded))), [3, 10, 1], list(range(len(loaded)))[::-1], [11, 0]]
        for rep in range(2):
            for idx in batches:
                outs = run_batch(ctx, plan, [loaded[i] for i in idx])
                for i, o in zip(idx, outs):
                    assert np.array_equal(gt.to_u64(o), want[i]), (rep, idx, i)
                # eager work between replays
                assert np.array_equal(gt.to_u64(loaded[idx[0]].word_count()), want[idx[0]])
        plan.close()
    finally:
        ctx.set_param(gt.PARAM_BATCH_GRAPH, 0)


def test_batch_limits(setup):
    import paper_2106_06889_amd as gt
    ctx, grammars, loaded, want = setup
    plan = ctx.batch(2, 10)
    import torch
    outs = [torch.empty(G.vocab, dtype=torch.int64, device=ctx.device) for G in loaded[:3]]
    with pytest.raises(gt.GtadocError) as e:
        plan.word_count(loaded[:3], outs)
    assert e.value.code == gt.ERR_INVALID_ARG
    with pytest.raises(gt.GtadocError):
        plan.word_count(loaded[10:11], outs[:1])  # more entries than the plan holds
    plan.close()


def test_autotune(setup, tmp_path):
    import paper_2106_06889_amd as gt
    from paper_2106_06889_amd import autotune
    ctx, grammars, loaded, want = setup
    res = autotune.tune_batch_word_count(ctx, loaded, reps=2)
    assert res["params"]["batch_blocks_per_cu"] in autotune.CANDIDATES[gt.PARAM_BATCH_BLOCKS_PER_CU]
    assert res["params"]["wc_chunk"] in autotune.CANDIDATES[gt.PARAM_WC_CHUNK]
    path = tmp_path / "cache.json"
    autotune.save("test-key", res, path=str(path))
    assert path.exists()
    # tuned parameters keep results exact
    plan = ctx.batch(len(loaded), sum(G.stats["word_syms"] for G in loaded))
    for G, o, w in zip(loaded, run_batch(ctx, plan, loaded), want):
        assert np.array_equal(gt.to_u64(o), w)
    plan.close()
    for p, v in autotune.DEFAULTS.items():
        ctx.set_param(p, v)


def _tv_np(res):
    import paper_2106_06889_amd as gt
    out = (res.arrays[0].cpu().numpy(), res.arrays[1].cpu().numpy().view(np.uint32), gt.to_u64(res.arrays[2]))
    res.free()
    return out


def test_mixed_batch_submit(setup):
    """Every query kind in one submit, several per grammar, each against the
    oracle, in two submits of the same plan with eager work between them."""
    import torch
    import paper_2106_06889_amd as gt
    ctx, grammars, loaded, want = setup
    plan = ctx.batch(len(loaded), sum(G.stats["word_syms"] for G in loaded))
    qs, expect = [], []
    for i, (g, G) in enumerate(zip(grammars, loaded)):
        out = torch.full((G.vocab,), -1, dtype=torch.int64, device=ctx.device)
        qs.append({"grammar": G, "kind": gt.QUERY_WORD_COUNT, "counts": out})
        expect.append(("wc", want[i]))
        if g.num_rules > 1 or len(g.sym):
            strat = [gt.TV_AUTO, gt.TV_BOTTOM_UP, gt.TV_TOP_DOWN][i % 3]
            qs.append({"grammar": G, "kind": gt.QUERY_TERM_VECTOR, "strategy": strat})
            expect.append(("tv", oracle.traverse_term_vector(g)))
            for n in (2, 3):
                if n == 3 and g.vocab > (1 << 21):
                    continue
                qs.append({"grammar": G, "kind": gt.QUERY_SEQUENCE_COUNT, "n": n})
                expect.append(("sc", oracle.traverse_sequence_count(g, n)))
            off, word, cnt = oracle.traverse_term_vector(g)
            qs.append({"grammar": G, "kind": gt.QUERY_INVERTED_INDEX})
            expect.append(("ii", oracle.inverted_index(off, word, g.vocab)))
            qs.append({"grammar": G, "kind": gt.QUERY_RANKED_INVERTED_INDEX})
            expect.append(("rii", oracle.ranked_inverted_index(off, word, cnt, g.vocab)))
    for rep in range(2):
        got = plan.submit(qs)
        torch.cuda.synchronize()
        for (kind, w), r in zip(expect, got):
            assert not isinstance(r, Exception), r
            if kind == "wc":
                assert np.array_equal(gt.to_u64(r), w)
            elif kind == "tv":
                assert all(np.array_equal(a, b) for a, b in zip(_tv_np(r), w))
            elif kind == "sc":
                k, c = gt.to_u64(r.arrays[0]), gt.to_u64(r.arrays[1])
                r.free()
                assert np.array_equal(k, w[0]) and np.array_equal(c, w[1])
            elif kind == "ii":
                a = (r.arrays[0].cpu().numpy(), r.arrays[1].cpu().numpy().view(np.uint32))
                r.free()
                assert np.array_equal(a[0], w[0]) and np.array_equal(a[1], w[1])
            else:
                assert all(np.array_equal(a, b) for a, b in zip(_tv_np(r), w))
        # eager work between submits
        assert np.array_equal(gt.to_u64(loaded[0].word_count()), want[0])
    plan.close()


def test_mixed_batch_errors(setup):
    """Malformed queries refuse the whole submit; a query that fails alone
    (4-grams over a vocabulary too large for 16-bit fields) reports its own
    status while the others complete."""
    import torch
    import paper_2106_06889_amd as gt
    ctx, grammars, loaded, want = setup
    plan = ctx.batch(2, sum(G.stats["word_syms"] for G in loaded))
    G = loaded[1]
    out = torch.empty(G.vocab, dtype=torch.int64, device=ctx.device)
    for bad in ({"grammar": G, "kind": 99}, {"grammar": G, "kind": gt.QUERY_SEQUENCE_COUNT, "n": 9},
                {"grammar": G, "kind": gt.QUERY_TERM_VECTOR, "strategy": 5}):
        with pytest.raises(gt.GtadocError) as e:
            plan.submit([{"grammar": G, "kind": gt.QUERY_WORD_COUNT, "counts": out}, bad])
        assert e.value.code == gt.ERR_INVALID_ARG
    with pytest.raises(gt.GtadocError):  # three word counts in a plan of two
        plan.submit([{"grammar": G, "kind": gt.QUERY_WORD_COUNT, "counts": out}] * 3)
    big = [i for i, g in enumerate(grammars) if g.vocab >= (1 << 16)]
    if not big:
        c = synth.random_corpus(77, 2, 300, 70000)
        g = synth.compress(c.tokens, c.file_off, c.vocab)
        Gb = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    else:
        Gb = loaded[big[0]]
    got = plan.submit([{"grammar": G, "kind": gt.QUERY_WORD_COUNT, "counts": out},
                       {"grammar": Gb, "kind": gt.QUERY_SEQUENCE_COUNT, "n": 4},
                       {"grammar": G, "kind": gt.QUERY_SEQUENCE_COUNT, "n": 2}])
    torch.cuda.synchronize()
    assert isinstance(got[1], gt.GtadocError) and got[1].code == gt.ERR_UNSUPPORTED
    assert np.array_equal(gt.to_u64(got[0]), want[1])
    wk, wc = oracle.traverse_sequence_count(grammars[1], 2)
    assert np.array_equal(gt.to_u64(got[2].arrays[0]), wk) and np.array_equal(gt.to_u64(got[2].arrays[1]), wc)
    got[2].free()
    if not big:
        Gb.free()
    plan.close()


def test_serving_isolation(setup):
    from paper_2106_06889_amd import serve
    ctx, grammars, loaded, want = setup
    srv = serve.Server(ctx, loaded, max_batch=8, keep_results=True)
    trace = serve.poisson_trace(60, rate=2000.0, num_grammars=len(loaded), seed=7)
    served = {r.qid: r for r in srv.run(trace)}
    alone = {r.qid: r for r in srv.run_plain(trace, realtime=False)}
    for q in trace:
        a, b = served[q.qid], alone[q.qid]
        assert a.finish >= a.arrival
        if q.kind == "wc":
            assert np.array_equal(a.result, b.result) and np.array_equal(a.result, want[q.grammar])
        else:
            assert len(a.result) == len(b.result)
            for x, y in zip(a.result, b.result):
                assert np.array_equal(x, y)
    st = serve.percentiles(list(served.values()))
    assert st["n"] == 60 and st["p99_ms"] >= st["p50_ms"]
    srv.close()


def test_edges_and_query_bytes(setup):
    """E (distinct parent-child pairs) against a count over the bodies, and
    the per-query arena figures: stable, nonzero where the query needs
    scratch, and covering what a run of the query holds."""
    import paper_2106_06889_amd as gt
    ctx, grammars, loaded, want = setup
    for g, G in zip(grammars, loaded):
        owner = np.repeat(np.arange(g.num_rules), np.diff(g.rule_off))
        ref = g.sym < 0
        pairs = set(zip(owner[ref].tolist(), (-g.sym[ref]).tolist()))
        assert G.edges() == len(pairs)
        if not len(g.sym):
            continue
        kinds = [(gt.QUERY_WORD_COUNT, 0, 0), (gt.QUERY_TERM_VECTOR, 0, gt.TV_BOTTOM_UP),
                 (gt.QUERY_TERM_VECTOR, 0, gt.TV_TOP_DOWN), (gt.QUERY_SEQUENCE_COUNT, 2, 0),
                 (gt.QUERY_INVERTED_INDEX, 0, 0)]
        for kind, n, strat in kinds:
            b = G.query_bytes(kind, n, strat)
            assert b > 0 and G.query_bytes(kind, n, strat) == b
            if kind == gt.QUERY_TERM_VECTOR:
                before = ctx.usage()[0]
                res = G.term_vector(strat)
                assert ctx.usage()[0] - before <= b  # the result is part of the peak
                res.free()
            if kind == gt.QUERY_WORD_COUNT:
                assert b >= 4 * G.stats["word_syms"]


def test_edges_golden():
    """E on the hand-worked grammars: E1 (R0 -> R1, R1 -> R2) = 2;
    E2 (R0 -> R1, R2; R1 -> R2) = 3."""
    import json
    import os
    import paper_2106_06889_amd as gt
    ctx = gt.Context(64 << 20)
    try:
        for name, want in (("e1_sequitur_abcdbc", 2), ("e2_two_files", 3)):
            d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", f"{name}.json")))
            gd = d["grammar"]
            G = ctx.load(np.array(gd["rule_off"], np.int64), np.array(gd["sym"], np.int32),
                         np.array(gd["file_off"], np.int64), d["vocab"])
            assert G.edges() == want
            G.free()
    finally:
        ctx.close()

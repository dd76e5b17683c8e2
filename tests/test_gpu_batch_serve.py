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

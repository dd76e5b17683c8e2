"""GPU parity at the full workload sizes (complete outputs against the
oracle's traversal, which is fast in C): word count + sort on the 100M-token
single-file corpus, bigram and trigram counts on the 20M-token nested-repeat
corpus."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2106_06889_amd as gt
    assert torch.cuda.is_available()
    c = gt.Context(6 << 30)
    yield c
    c.close()


@pytest.mark.timeout(300)
def test_wc_100m_full(ctx):
    import paper_2106_06889_amd as gt
    c, g = synth.workload("wc-100m")
    T = len(c.tokens)
    want = oracle.traverse_word_count(g)
    assert int(want.sum()) == T
    del c
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    assert G.stats["tokens"] == T
    got = gt.to_u64(G.word_count())
    assert np.array_equal(got, want)
    ids, cnt, num = G.sort()
    wid, wcnt = oracle.sort_counts(want)
    k = int(num.item())
    assert k == len(wid)
    assert np.array_equal(ids[:k].cpu().numpy().view(np.uint32), wid)
    assert np.array_equal(gt.to_u64(cnt[:k]), wcnt)
    G.free()


@pytest.mark.timeout(300)
def test_seq_20m_full(ctx):
    import paper_2106_06889_amd as gt
    c, g = synth.workload("seq-20m")
    T = len(c.tokens)
    del c
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    assert G.stats["depth"] >= 40
    for n in (2, 3):
        res = G.sequence_count(n)
        k, cnt = gt.to_u64(res.arrays[0]), gt.to_u64(res.arrays[1])
        res.free()
        wk, wc = oracle.traverse_sequence_count(g, n)
        assert np.array_equal(k, wk) and np.array_equal(cnt, wc), n
        assert int(cnt.sum()) == T - n + 1
    G.free()

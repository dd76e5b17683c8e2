"""GPU parity at the full workload sizes (complete outputs against the
oracle's traversal, which is fast in C): word count + sort on the 100M-token
single-file corpus, bigram and trigram counts on the 20M-token nested-repeat
corpus; term vector + inverted index + ranked inverted index on the
4,000-file corpus, and the term vector by both traversals on the 4-file
corpus (every file's row against the uncompressed text)."""
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
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab, levels=True)
    assert G.stats["depth"] >= 40
    for n in (2, 3):
        res = G.sequence_count(n)
        k, cnt = gt.to_u64(res.arrays[0]), gt.to_u64(res.arrays[1])
        res.free()
        wk, wc = oracle.traverse_sequence_count(g, n)
        assert np.array_equal(k, wk) and np.array_equal(cnt, wc), n
        assert int(cnt.sum()) == T - n + 1
    G.free()


@pytest.mark.timeout(900)
def test_tv_4000files_full(capsys):
    """Term vector + inverted index + ranked inverted index at the full
    4,000-file size, in the calls the benchmark times (term vector, then the
    indexes built from it). Every file's row is compared element by element
    with the oracle's brute-force term vector of the uncompressed text; both
    indexes with the oracle's indexes built from that reference term vector
    (not from the GPU's)."""
    import time
    import torch
    import paper_2106_06889_amd as gt
    with capsys.disabled():  # the generator reports its progress on stderr
        c, g = synth.workload("tv-4000files")
    F, T, V = g.num_files, len(c.tokens), g.vocab
    R, S = g.num_rules, len(g.sym)
    ctx = gt.Context(128 * R + 72 * S + 80 * V + 48 * T // 10 + (4 << 30))
    try:
        G = ctx.load(g.rule_off, g.sym, g.file_off, V)
        assert G.stats["tokens"] == T
        tv = G.term_vector()
        off = tv.arrays[0].cpu().numpy()
        word = tv.arrays[1].cpu().numpy().view(np.uint32)
        cnt = gt.to_u64(tv.arrays[2])
        ii = G.inverted_index_from(tv)
        ioff = ii.arrays[0].cpu().numpy()
        ifile = ii.arrays[1].cpu().numpy().view(np.uint32)
        ii.free()
        rii = G.ranked_inverted_index_from(tv)
        roff = rii.arrays[0].cpu().numpy()
        rfile = rii.arrays[1].cpu().numpy().view(np.uint32)
        rtf = gt.to_u64(rii.arrays[2])
        rii.free()
        tv.free()
        G.free()
    finally:
        ctx.close()
    torch.cuda.synchronize()
    t0 = time.time()
    w_off, w_word, w_cnt = oracle.tv_text(c.tokens, c.file_off, V)
    del c
    nnz = int(w_off[-1])
    print(f"oracle term vector of the text: {nnz} pairs in {time.time() - t0:.1f} s", flush=True)
    assert np.array_equal(off, w_off)
    assert np.array_equal(word[:nnz], w_word)
    assert np.array_equal(cnt[:nnz], w_cnt)
    del word, cnt
    i_off, i_file = oracle.inverted_index(w_off, w_word, V)
    assert np.array_equal(ioff, i_off)
    assert np.array_equal(ifile[:nnz], i_file)
    del ifile, i_file
    r_off, r_file, r_tf = oracle.ranked_inverted_index(w_off, w_word, w_cnt, V)
    assert np.array_equal(roff, r_off)
    assert np.array_equal(rfile[:nnz], r_file)
    assert np.array_equal(rtf[:nnz], r_tf)


@pytest.mark.timeout(300)
def test_seq4_20m_full(ctx):
    """4-gram counts on the 20M-token nested-repeat corpus with a vocabulary
    that fits 16-bit key fields (V = 60,000)."""
    import paper_2106_06889_amd as gt
    c, g = synth.workload("seq4-20m")
    T = len(c.tokens)
    del c
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    res = G.sequence_count(4)
    k, cnt = gt.to_u64(res.arrays[0]), gt.to_u64(res.arrays[1])
    res.free()
    G.free()
    wk, wc = oracle.traverse_sequence_count(g, 4)
    assert np.array_equal(k, wk) and np.array_equal(cnt, wc)
    assert int(cnt.sum()) == T - 3


@pytest.mark.timeout(600)
def test_seq_20m_fourgrams_wide_full(ctx):
    """4-gram counts of the 20M-token nested-repeat corpus with its own
    vocabulary of 200,000 words (too large for 16-bit key fields), through
    the wide keys, against the oracle's traversal."""
    import paper_2106_06889_amd as gt
    c, g = synth.workload("seq-20m")
    T = len(c.tokens)
    del c
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    res = G.sequence_count_wide(4)
    got = tuple(gt.to_u64(a) for a in res.arrays)
    res.free()
    G.free()
    want = oracle.traverse_sequence_count_wide(g, 4)
    assert all(np.array_equal(a, b) for a, b in zip(got, want))
    assert int(got[2].sum()) == T - 3


@pytest.mark.timeout(600)
def test_tv_4files_both_traversals_full(capsys):
    """Term vector of the 4-file 10^8-token corpus by the bottom-up and the
    top-down traversal and by the selector's choice (top-down here), in the
    calls the traversal-choice benchmark times: the grammar loaded from
    device tensors, one term-vector call per strategy. Every row against the
    oracle's brute-force term vector of the uncompressed text, and the
    inverted index of the selector's term vector against the oracle's."""
    import torch
    import paper_2106_06889_amd as gt
    with capsys.disabled():
        c, g = synth.workload("tv-4files")
    F, T, V = g.num_files, len(c.tokens), g.vocab
    R, S = g.num_rules, len(g.sym)
    assert F == 4
    w_off, w_word, w_cnt = oracle.tv_text(c.tokens, c.file_off, V)
    del c
    nnz = int(w_off[-1])
    dev = torch.device("cuda", 0)
    ro = torch.from_numpy(g.rule_off).to(dev)
    sym = torch.from_numpy(g.sym).to(dev)
    fo = torch.from_numpy(g.file_off).to(dev)
    ctx = gt.Context(128 * R + 72 * S + 80 * V + 48 * T // 10 + (4 << 30))
    try:
        G = ctx.load(ro, sym, fo, V, borrow=True)
        assert G.stats["tokens"] == T
        assert G.tv_strategy() == gt.TV_TOP_DOWN
        for strat in (gt.TV_BOTTOM_UP, gt.TV_TOP_DOWN, None):
            tv = G.term_vector() if strat is None else G.term_vector(strat)
            off = tv.arrays[0].cpu().numpy()
            assert np.array_equal(off, w_off), strat
            assert np.array_equal(tv.arrays[1][:nnz].cpu().numpy().view(np.uint32), w_word), strat
            assert np.array_equal(gt.to_u64(tv.arrays[2])[:nnz], w_cnt), strat
            if strat is None:
                ii = G.inverted_index_from(tv)
                i_off, i_file = oracle.inverted_index(w_off, w_word, V)
                assert np.array_equal(ii.arrays[0].cpu().numpy(), i_off)
                assert np.array_equal(ii.arrays[1][:nnz].cpu().numpy().view(np.uint32), i_file)
                ii.free()
            tv.free()
        G.free()
    finally:
        ctx.close()

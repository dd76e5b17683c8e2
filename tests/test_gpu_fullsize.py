"""GPU parity at the full workload sizes (complete outputs against the
oracle's traversal, which is fast in C): word count + sort on the 100M-token
single-file corpus, bigram and trigram counts on the 20M-token nested-repeat
corpus; term vector + inverted index + ranked inverted index on the
4,000-file corpus (sampled files against the uncompressed text, properties
on every file)."""
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


@pytest.mark.timeout(600)
def test_tv_4000files_full(capsys):
    """Term vector + inverted index at the full 4,000-file size, in the
    calls the benchmark times (term vector, then the index built from it).
    Every file: its counts sum to its token count and its words ascend; 40
    sampled files (the largest, the smallest, seeded others): exact against
    counting the uncompressed file directly; the index: exactly the
    transpose of the term vector's (file, word) pattern, files ascending."""
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
        word = tv.arrays[1].cpu().numpy().view(np.uint32).astype(np.int64)
        cnt = gt.to_u64(tv.arrays[2])
        ii = G.inverted_index_from(tv)
        ioff = ii.arrays[0].cpu().numpy()
        ifile = ii.arrays[1].cpu().numpy().view(np.uint32).astype(np.int64)
        ii.free()
        rii = G.ranked_inverted_index_from(tv)
        roff = rii.arrays[0].cpu().numpy()
        rfile = rii.arrays[1].cpu().numpy().view(np.uint32).astype(np.int64)
        rtf = gt.to_u64(rii.arrays[2])
        rii.free()
        tv.free()
        G.free()
    finally:
        ctx.close()
    torch.cuda.synchronize()
    nnz = int(off[-1])
    assert len(off) == F + 1 and off[0] == 0 and np.all(np.diff(off) >= 0)
    assert len(word) >= nnz and len(cnt) >= nnz
    word, cnt = word[:nnz], cnt[:nnz]
    assert np.all(cnt > 0) and np.all(word < V)
    # per file: counts sum to the file's length, words strictly ascending
    lens = np.diff(c.file_off)
    sums = np.zeros(F, np.uint64)
    nz = np.diff(off) > 0
    sums[nz] = np.add.reduceat(cnt, off[:-1][nz])
    assert np.array_equal(sums, lens.astype(np.uint64))
    file_of = np.repeat(np.arange(F), np.diff(off))
    same_file = file_of[1:] == file_of[:-1]
    assert np.all(np.diff(word)[same_file] > 0)
    # sampled files against direct counts of the uncompressed text
    rng = np.random.default_rng(2106)
    pick = set(rng.choice(F, 38, replace=False).tolist()) | {int(np.argmax(lens)), int(np.argmin(lens))}
    for f in sorted(pick):
        u, k = np.unique(c.tokens[c.file_off[f]:c.file_off[f + 1]], return_counts=True)
        a, b = off[f], off[f + 1]
        assert np.array_equal(word[a:b], u.astype(np.int64)), f
        assert np.array_equal(cnt[a:b], k.astype(np.uint64)), f
    # the index is the transpose of the (file, word) pattern
    order = np.lexsort((file_of, word))
    want_off = np.concatenate([[0], np.cumsum(np.bincount(word, minlength=V))])
    assert np.array_equal(ioff[:V + 1], want_off)
    assert np.array_equal(ifile[:nnz], file_of[order])
    # the ranked index: per word, term frequency desc, then file asc
    rorder = np.lexsort((file_of, -cnt.astype(np.int64), word))
    assert np.array_equal(roff[:V + 1], want_off)
    assert np.array_equal(rfile[:nnz], file_of[rorder])
    assert np.array_equal(rtf[:nnz], cnt[rorder])


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

"""The oracle and the Sequitur compressor against invariants, closed forms and
brute force, on many small irregular corpora (empty files, runs, repeats,
tiny vocabularies)."""
import numpy as np
import pytest

import oracle
import synth

CASES = [(s, files, mt, V) for s in range(8) for (files, mt, V) in ((1, 300, 3), (3, 400, 7), (5, 150, 50))]


def build(seed, files, max_tokens, vocab):
    c = synth.random_corpus(seed, files, max_tokens, vocab)
    return c, synth.compress(c.tokens, c.file_off, vocab)


@pytest.mark.parametrize("seed,files,max_tokens,vocab", CASES)
def test_sequitur_invariants(seed, files, max_tokens, vocab):
    c, g = build(seed, files, max_tokens, vocab)
    assert oracle.check_structure(g) == 0
    assert oracle.check_sequitur(g) == 0          # digram uniqueness, utility, length >= 2, acyclic
    tok, off = oracle.expand(g)                    # expansion == input, per file
    assert np.array_equal(tok, c.tokens) and np.array_equal(off, c.file_off)


@pytest.mark.parametrize("seed,files,max_tokens,vocab", CASES)
def test_traversal_equals_brute_force(seed, files, max_tokens, vocab):
    c, g = build(seed, files, max_tokens, vocab)
    T = len(c.tokens)
    wc = oracle.traverse_word_count(g)
    assert np.array_equal(wc, oracle.wc_text(c.tokens, vocab))
    assert int(wc.sum()) == T
    # weights: sum over rules of weight * (words in body) = T
    w = oracle.weights(g)
    words = np.add.reduceat((g.sym >= 0).astype(np.uint64), g.rule_off[:-1]) if len(g.sym) else np.zeros(0)
    words = np.where(np.diff(g.rule_off) > 0, words, 0)
    assert int((w * words.astype(np.uint64)).sum()) == T
    # term vector
    off, word, cnt = oracle.traverse_term_vector(g)
    boff, bword, bcnt = oracle.tv_text(c.tokens, c.file_off, vocab)
    assert np.array_equal(off, boff) and np.array_equal(word, bword) and np.array_equal(cnt, bcnt)
    for f in range(len(off) - 1):
        assert int(cnt[off[f]:off[f + 1]].sum()) == int(c.file_off[f + 1] - c.file_off[f])
        assert np.all(np.diff(word[off[f]:off[f + 1]].astype(np.int64)) > 0)
    tvsum = np.zeros(vocab, np.uint64)
    np.add.at(tvsum, word, cnt)
    assert np.array_equal(tvsum, wc)
    # inverted index is the transpose of the term vector
    ioff, ifile = oracle.inverted_index(off, word, vocab)
    pairs = sorted((int(wd), f) for f in range(len(off) - 1) for wd in word[off[f]:off[f + 1]])
    got = sorted((wd, int(fl)) for wd in range(vocab) for fl in ifile[ioff[wd]:ioff[wd + 1]])
    assert pairs == got
    # sequences, n = 1 reduces to the word count
    k1, c1 = oracle.traverse_sequence_count(g, 1)
    assert np.array_equal(k1, np.nonzero(wc)[0].astype(np.uint64)) and np.array_equal(c1, wc[wc > 0])
    for n in (2, 3, 4):
        k, cn = oracle.traverse_sequence_count(g, n)
        bk, bc = oracle.sc_text(c.tokens, c.file_off, n, vocab)
        assert np.array_equal(k, bk) and np.array_equal(cn, bc)
        sizes = np.diff(c.file_off)
        assert int(cn.sum()) == int(np.maximum(sizes - n + 1, 0).sum())
        assert np.all(k[1:] > k[:-1])  # strictly ascending (uint64 compare: n = 4 keys exceed 2^53)


@pytest.mark.parametrize("seed,files,max_tokens,vocab", CASES[:12])
def test_owned_windows_equal_eq1(seed, files, max_tokens, vocab):
    """Sequence support: per rule, the number of windows the rule itself must
    count equals wordSize + (l-1) * subRuleSize - (l-1) whenever every child
    expands to at least l-1 words (always so for Sequitur rules and l <= 3);
    the root obeys it per file span."""
    c, g = build(seed, files, max_tokens, vocab)
    lens = np.diff(g.rule_off)
    for n in (2, 3):
        own = oracle.owned_counts(g, n)
        for r in range(1, g.num_rules):
            body = g.sym[g.rule_off[r]:g.rule_off[r + 1]]
            words, subs = int((body >= 0).sum()), int((body < 0).sum())
            assert int(own[r]) == max(words + (n - 1) * subs - (n - 1), 0), (r, n)
        root_total = 0
        for f in range(g.num_files):
            body = g.sym[g.file_off[f]:g.file_off[f + 1]]
            if len(body) == 0:
                continue
            words, subs = int((body >= 0).sum()), int((body < 0).sum())
            # a span's bound counts windows; it cannot go below zero
            root_total += max(words + (n - 1) * subs - (n - 1), 0)
        assert int(own[0]) == root_total
        assert lens[0] >= 0
    # n = 4: Eq. upperLimit is only an upper bound once a child expands to
    # fewer than n - 1 = 3 words (Sequitur children have at least 2)
    own = oracle.owned_counts(g, 4)
    for r in range(1, g.num_rules):
        body = g.sym[g.rule_off[r]:g.rule_off[r + 1]]
        words, subs = int((body >= 0).sum()), int((body < 0).sum())
        assert int(own[r]) <= max(words + 3 * subs - 3, 0), r


def test_sort_order_is_total():
    wc = np.array([3, 0, 5, 3, 1, 5], np.uint64)
    ids, cnt = oracle.sort_counts(wc)
    assert ids.tolist() == [2, 5, 0, 3, 4] and cnt.tolist() == [5, 5, 3, 3, 1]


def test_structure_rejects_bad_grammars():
    V = 4
    ok = synth.Grammar(np.array([0, 2, 4], np.int64), np.array([-1, -1, 0, 1], np.int32), np.array([0, 2], np.int64), V)
    assert oracle.check_structure(ok) == 0
    bad_word = synth.Grammar(ok.rule_off, np.array([-1, -1, 0, 4], np.int32), ok.file_off, V)
    bad_ref = synth.Grammar(ok.rule_off, np.array([-1, -2, 0, 1], np.int32), ok.file_off, V)
    bad_span = synth.Grammar(ok.rule_off, ok.sym, np.array([0, 1], np.int64), V)
    for g in (bad_word, bad_ref, bad_span):
        assert oracle.check_structure(g) == oracle.OR_ERR_RANGE
    cyc = synth.Grammar(np.array([0, 1, 3], np.int64), np.array([-1, 0, -1], np.int32), np.array([0, 1], np.int64), V)
    with pytest.raises(RuntimeError):
        oracle.weights(cyc)


def test_workload_small_scale_end_to_end():
    """The wc-200k recipe: grammar valid, traversal == brute force."""
    c, g = synth.workload("wc-200k", scale=0.25)
    assert oracle.check_sequitur(g) == 0
    assert np.array_equal(oracle.traverse_word_count(g), oracle.wc_text(c.tokens, c.vocab))


def test_parallel_variants_equal_sequential():
    """The CPU-baseline variants on several host threads give the sequential
    oracle's results exactly (rule-range word count; file-parallel term
    vector), and both equal the brute force on the text."""
    for seed in range(3):
        c = synth.random_corpus(40 + seed, 1 + 3 * seed, 3000, 50)
        g = synth.compress(c.tokens, c.file_off, 50)
        want = oracle.wc_text(c.tokens, 50)
        for t in (1, 3, 8):
            assert np.array_equal(oracle.traverse_word_count_parallel(g, t), want)
        boff, bword, bcnt = oracle.tv_text(c.tokens, c.file_off, 50)
        for t in (1, 4):
            off, word, cnt = oracle.traverse_term_vector_parallel(g, t)
            assert np.array_equal(off, boff) and np.array_equal(word, bword) and np.array_equal(cnt, bcnt)

"""GPU parity: n-gram sequence count (n = 2, 3, and 4 where the vocabulary
fits 16-bit key fields) through the C ABI against the oracle (traversal and
brute force), bit-exact keys and counts."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2106_06889_amd as gt
    assert torch.cuda.is_available()
    c = gt.Context(3 << 30)
    yield c
    c.close()


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        d = json.load(f)
    g = synth.Grammar(np.array(d["grammar"]["rule_off"], np.int64), np.array(d["grammar"]["sym"], np.int32),
                      np.array(d["grammar"]["file_off"], np.int64), d["vocab"])
    return d, g


def gpu_sc(G, n):
    import paper_2106_06889_amd as gt
    res = G.sequence_count(n)
    k, c = gt.to_u64(res.arrays[0]), gt.to_u64(res.arrays[1])
    res.free()
    return k, c


def check(ctx, g, ns=None, brute=True):
    if ns is None:
        ns = (2, 3, 4) if g.vocab < (1 << 16) else (2, 3)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        for n in ns:
            k, c = gpu_sc(G, n)
            wk, wc = oracle.traverse_sequence_count(g, n)
            assert np.array_equal(k, wk) and np.array_equal(c, wc), n
            if brute:
                bk, bc = oracle.brute_sequence_count(g, n)
                assert np.array_equal(k, bk) and np.array_equal(c, bc)
            # a second call reuses the cached head/tail buffers
            k2, c2 = gpu_sc(G, n)
            assert np.array_equal(k, k2) and np.array_equal(c, c2)
    finally:
        G.free()


@pytest.mark.parametrize("name", ["e1_sequitur_abcdbc.json", "e2_two_files.json", "e3_head_tail.json"])
def test_golden(ctx, name):
    d, g = gold(name)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    for n, key in ((2, "bigrams"), (3, "trigrams"), (4, "fourgrams")):
        if key in d:
            k, c = gpu_sc(G, n)
            assert {int(a): int(b) for a, b in zip(k, c)} == {int(a): b for a, b in d[key].items()}
    G.free()


@pytest.mark.parametrize("seed", range(10))
def test_random_corpora(ctx, seed):
    c = synth.random_corpus(100 + seed, 1 + seed % 5, 2500, [2, 9, 300][seed % 3])
    check(ctx, synth.compress(c.tokens, c.file_off, c.vocab))


def test_non_sequitur_short_children(ctx):
    """Children that expand to a single word (allowed by the encoding, never
    made by Sequitur): windows span several pieces."""
    # R1 = [7], R2 = [R1 3], R3 = [R1]; root: f0 = R2 R3 R1 5, f1 = R3, f2 = (empty), f3 = 2 R1 R3 R2
    sym = np.array([-2, -3, -1, 5, -3, 2, -1, -3, -2, 7, -1, 3, -1], np.int32)
    g = synth.Grammar(np.array([0, 9, 10, 12, 13], np.int64), sym, np.array([0, 4, 5, 5, 9], np.int64), 8)
    assert oracle.check_structure(g) == 0
    check(ctx, g)


def test_seq_20m_recipe_scaled(ctx):
    c, g = synth.workload("seq-20m", scale=0.05)
    check(ctx, g, brute=False)
    k, cn = oracle.sc_text(c.tokens, c.file_off, 2, c.vocab)
    assert int(cn.sum()) == len(c.tokens) - 1


def test_multi_file_recipe_scaled(ctx):
    c, g = synth.workload("tv-4000files", scale=0.005)  # 20 files
    check(ctx, g, brute=False)


def test_argument_errors(ctx):
    import paper_2106_06889_amd as gt
    d, g = gold("e1_sequitur_abcdbc.json")
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    for n in (1, 5):
        with pytest.raises(gt.GtadocError) as e:
            G.sequence_count(n)
        assert e.value.code == gt.ERR_INVALID_ARG
    G.free()
    wide = synth.Grammar(g.rule_off, g.sym, g.file_off, 1 << 16)
    G = ctx.load(wide.rule_off, wide.sym, wide.file_off, wide.vocab)
    with pytest.raises(gt.GtadocError) as e:
        G.sequence_count(4)  # 16-bit key fields, and the all-ones key marks empty slots
    assert e.value.code == gt.ERR_UNSUPPORTED
    G.free()
    big = synth.Grammar(g.rule_off, g.sym, g.file_off, (1 << 21) + 1)
    G = ctx.load(big.rule_off, big.sym, big.file_off, big.vocab)
    with pytest.raises(gt.GtadocError) as e:
        G.sequence_count(3)
    assert e.value.code == gt.ERR_UNSUPPORTED
    k, c = gpu_sc(G, 2)  # bigrams still fine
    assert int(c.sum()) == 11
    G.free()


def test_fourgrams_single_file_recipe(ctx):
    """n = 4 on the 200K-token single-file recipe (V = 5,000): Sequitur
    children of 2 words, shorter than n - 1, hand windows on to the next
    pieces."""
    c, g = synth.workload("wc-200k")
    check(ctx, g, ns=(4,))
    k, cn = oracle.sc_text(c.tokens, c.file_off, 4, c.vocab)
    kk, cc = gpu_sc_of(ctx, g, 4)
    assert np.array_equal(kk, k) and np.array_equal(cc, cn)


def test_fourgrams_nested_recipe_scaled(ctx):
    c, g = synth.workload("seq4-20m", scale=0.05)
    check(ctx, g, ns=(4,), brute=False)
    assert int(gpu_sc_of(ctx, g, 4)[1].sum()) == len(c.tokens) - 3


def gpu_sc_of(ctx, g, n):
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        return gpu_sc(G, n)
    finally:
        G.free()


def gpu_wide(G, n):
    import paper_2106_06889_amd as gt
    res = G.sequence_count_wide(n)
    out = tuple(gt.to_u64(a) for a in res.arrays)
    res.free()
    return out


@pytest.mark.parametrize("seed", range(6))
def test_wide_keys_random_corpora(ctx, seed):
    """Wide keys for every n in 2..8 (as far as n * bits(V - 1) <= 126),
    bit-exact against the oracle's traversal and its brute force."""
    c = synth.random_corpus(700 + seed, 1 + seed % 4, 2500, [3, 40, 900, 70000, 5, 200][seed])
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        for n in range(2, 9):
            if n * oracle.wide_bits(c.vocab) > 126:
                continue
            got = gpu_wide(G, n)
            want = oracle.traverse_sequence_count_wide(g, n)
            assert all(np.array_equal(a, b) for a, b in zip(got, want)), n
            brute = oracle.sc_text_wide(c.tokens, c.file_off, n, c.vocab)
            assert all(np.array_equal(a, b) for a, b in zip(got, brute)), n
    finally:
        G.free()


def test_wide_keys_golden_fivegrams(ctx):
    d = json.load(open(os.path.join(GOLD, "e1_fivegrams.json")))
    tok = np.array(d["tokens"], np.int32)
    g = synth.compress(tok, np.array(d["file_off_text"], np.int64), d["vocab"])
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    hi, lo, cnt = gpu_wide(G, 5)
    G.free()
    assert oracle.unpack_wide(hi, lo, 5, d["vocab"]).tolist() == d["grams"]
    assert cnt.tolist() == d["counts"]


def test_wide_keys_errors(ctx):
    import paper_2106_06889_amd as gt
    c = synth.random_corpus(3, 2, 300, 1 << 30)
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        for n, code in ((1, gt.ERR_INVALID_ARG), (9, gt.ERR_INVALID_ARG), (5, gt.ERR_UNSUPPORTED)):
            with pytest.raises(gt.GtadocError) as e:
                G.sequence_count_wide(n)
            assert e.value.code == code, n
    finally:
        G.free()


@pytest.mark.timeout(300)
def test_wide_keys_seq_recipe(ctx):
    """The nested-repeat recipe (V = 200,000, so 4-grams do not fit 64-bit
    keys) at n = 4 and n = 7, scaled to 1/20."""
    c, g = synth.workload("seq-20m", scale=0.05)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        for n in (4, 7):
            got = gpu_wide(G, n)
            want = oracle.traverse_sequence_count_wide(g, n)
            assert all(np.array_equal(a, b) for a, b in zip(got, want)), n
            assert int(got[2].sum()) == len(c.tokens) - n + 1
    finally:
        G.free()

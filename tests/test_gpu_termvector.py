"""GPU parity: term vector and inverted index through the C ABI against the
oracle (per-file top-down traversal and brute force), bit-exact."""
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
    c = gt.Context(4 << 30)
    yield c
    c.close()


def gpu_tv(G, strategy=None):
    import paper_2106_06889_amd as gt
    res = G.term_vector(strategy)
    off = res.arrays[0].cpu().numpy()
    word = res.arrays[1].cpu().numpy().view(np.uint32)
    cnt = gt.to_u64(res.arrays[2])
    res.free()
    return off, word, cnt


def gpu_ii(G):
    res = G.inverted_index()
    off = res.arrays[0].cpu().numpy()
    files = res.arrays[1].cpu().numpy().view(np.uint32)
    res.free()
    return off, files


def gpu_rii(res):
    import paper_2106_06889_amd as gt
    out = (res.arrays[0].cpu().numpy(), res.arrays[1].cpu().numpy().view(np.uint32), gt.to_u64(res.arrays[2]))
    res.free()
    return out


def same_rii(got, want):
    return all(np.array_equal(a, b) for a, b in zip(got, want))


def check(ctx, g, brute=True):
    import paper_2106_06889_amd as gt
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        woff, wword, wcnt = oracle.traverse_term_vector(g)
        # both traversals, then the selector's choice
        for strategy in (gt.TV_BOTTOM_UP, gt.TV_TOP_DOWN, None):
            off, word, cnt = gpu_tv(G, strategy)
            assert np.array_equal(off, woff), strategy
            assert np.array_equal(word, wword), strategy
            assert np.array_equal(cnt, wcnt), strategy
        if brute:
            boff, bword, bcnt = oracle.brute_term_vector(g)
            assert np.array_equal(off, boff) and np.array_equal(word, bword) and np.array_equal(cnt, bcnt)
        ioff, ifile = gpu_ii(G)
        woff2, wfile = oracle.inverted_index(woff, wword, g.vocab)
        assert np.array_equal(ioff, woff2) and np.array_equal(ifile, wfile)
        # the same from a term vector result, without recomputing it
        tv = G.term_vector()
        ii = G.inverted_index_from(tv)
        assert np.array_equal(ii.arrays[0].cpu().numpy(), woff2)
        assert np.array_equal(ii.arrays[1].cpu().numpy().view(np.uint32), wfile)
        ii.free()
        # ranked: files by term frequency desc, then file asc
        want_r = oracle.ranked_inverted_index(woff, wword, wcnt, g.vocab)
        assert same_rii(gpu_rii(G.ranked_inverted_index_from(tv)), want_r)
        tv.free()
        assert same_rii(gpu_rii(G.ranked_inverted_index()), want_r)
    finally:
        G.free()


def test_golden_e2(ctx):
    with open(os.path.join(GOLD, "e2_two_files.json")) as f:
        d = json.load(f)
    g = synth.Grammar(np.array(d["grammar"]["rule_off"], np.int64), np.array(d["grammar"]["sym"], np.int32),
                      np.array(d["grammar"]["file_off"], np.int64), d["vocab"])
    import paper_2106_06889_amd as gt
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    for strategy in (gt.TV_BOTTOM_UP, gt.TV_TOP_DOWN, None):
        off, word, cnt = gpu_tv(G, strategy)
        assert off.tolist() == d["term_vector"]["off"]
        assert word.tolist() == d["term_vector"]["word"] and cnt.tolist() == d["term_vector"]["cnt"]
    ioff, ifile = gpu_ii(G)
    assert ioff.tolist() == d["inverted_index"]["off"] and ifile.tolist() == d["inverted_index"]["file"]
    G.free()


@pytest.mark.parametrize("seed", range(10))
def test_random_corpora(ctx, seed):
    c = synth.random_corpus(200 + seed, 1 + 2 * (seed % 5), 2500, [3, 11, 500][seed % 3])
    check(ctx, synth.compress(c.tokens, c.file_off, c.vocab))


def test_long_bodies_and_empty_files(ctx):
    """Bodies longer than the merge's register cursors, repeated children,
    empty files, an unreachable rule."""
    rng = np.random.default_rng(5)
    V = 40
    r1 = rng.integers(0, V, 5).astype(np.int32)                      # R1: 5 words
    r2 = np.concatenate([rng.integers(0, V, 30), [-1, -1, -1]]).astype(np.int32)  # R2: 33 symbols, R1 x3
    r3 = np.array([-2, 7, -1, -2], np.int32)                            # R3: R2 twice, R1
    r4 = np.array([1, 2, 3], np.int32)                                 # R4: unreachable
    f0 = np.array([-3, 5, -1], np.int32)
    f2 = np.concatenate([rng.integers(0, V, 25), [-2, -3, -1]]).astype(np.int32)
    root = np.concatenate([f0, f2])
    sym = np.concatenate([root, r1, r2, r3, r4])
    lens = [len(root), len(r1), len(r2), len(r3), len(r4)]
    rule_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    file_off = np.array([0, len(f0), len(f0), len(root), len(root)], np.int64)  # files 1 and 3 empty
    g = synth.Grammar(rule_off, sym, file_off, V)
    assert oracle.check_structure(g) == 0
    check(ctx, g)


def test_large_tables(ctx):
    """Merges spread over a workgroup: a rule whose children's tables hold
    thousands of words (more inputs than one wave merges), overlapping word
    ranges that span several 4096-id windows, repeated children, and a rule
    with more body symbols than the workgroup merge keeps cursors for."""
    rng = np.random.default_rng(11)
    V = 20000
    a = rng.permutation(V)[:3000].astype(np.int32)                   # R1: 3000 distinct words
    b = np.concatenate([a[1000:2500], rng.integers(0, V, 1500)]).astype(np.int32)  # R2: overlaps R1
    c = np.array([-1, -2, 7, -1, 19999, 0], np.int32)               # R3: R1 twice, R2, words
    d = rng.integers(0, V, 5000).astype(np.int32)                    # R4: 5000 symbols
    e = np.array([-3, -4, 5], np.int32)                              # R5
    root = np.array([-5, 3, -3, -4, -5, -1, -2, 12], np.int32)
    bodies = [root, a, b, c, d, e]
    rule_off = np.cumsum([0] + [len(x) for x in bodies]).astype(np.int64)
    g = synth.Grammar(rule_off, np.concatenate(bodies), np.array([0, 3, 3, 8], np.int64), V)
    check(ctx, g)


def test_tv_recipe_scaled(ctx):
    c, g = synth.workload("tv-4000files", scale=0.01)  # 40 files
    check(ctx, g, brute=False)


def test_wc_recipe_single_file(ctx):
    c, g = synth.workload("wc-200k")
    check(ctx, g)


def test_inverted_index_from_foreign_result(ctx):
    import paper_2106_06889_amd as gt
    c = synth.random_corpus(5, 3, 400, 30)
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    G, H = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab), ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        sc = G.sequence_count(2)
        with pytest.raises(gt.GtadocError) as e:
            G.inverted_index_from(sc)
        assert e.value.code == gt.ERR_INVALID_ARG
        with pytest.raises(gt.GtadocError) as e:
            G.ranked_inverted_index_from(sc)
        assert e.value.code == gt.ERR_INVALID_ARG
        tv = H.term_vector()
        with pytest.raises(gt.GtadocError) as e:
            G.inverted_index_from(tv)  # a term vector of another grammar
        assert e.value.code == gt.ERR_INVALID_ARG
        with pytest.raises(gt.GtadocError) as e:
            G.ranked_inverted_index_from(tv)
        assert e.value.code == gt.ERR_INVALID_ARG
        tv.free()
        sc.free()
    finally:
        G.free()
        H.free()


def test_golden_ranked_inverted_index(ctx):
    with open(os.path.join(GOLD, "e4_ranked_inverted_index.json")) as f:
        d = json.load(f)
    tokens = np.concatenate([np.asarray(x, np.int32) for x in d["files"]])
    file_off = np.concatenate([[0], np.cumsum([len(x) for x in d["files"]])]).astype(np.int64)
    g = synth.compress(tokens, file_off, d["vocab"])
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        off, file, tf = gpu_rii(G.ranked_inverted_index())
        want = d["ranked_inverted_index"]
        assert off.tolist() == want["off"] and file.tolist() == want["file"] and tf.tolist() == want["tf"]
    finally:
        G.free()


def test_ranked_ties_and_heavy_counts(ctx):
    """Many files with equal term frequencies (ties broken by file id) and a
    word whose frequency in one file needs more than 16 bits."""
    rng = np.random.default_rng(9)
    files = [np.array([1, 2, 1, 2, 3], np.int32) for _ in range(40)]
    files.append(np.full(70000, 4, np.int32))
    files.append(np.concatenate([np.full(65536, 4, np.int32), rng.integers(0, 6, 300).astype(np.int32)]))
    tokens = np.concatenate(files)
    file_off = np.concatenate([[0], np.cumsum([len(x) for x in files])]).astype(np.int64)
    g = synth.compress(tokens, file_off, 6)
    check(ctx, g, brute=False)


def test_few_large_files_recipe_scaled(ctx):
    """The few-large-files corpus (4 files) the top-down traversal is for."""
    import paper_2106_06889_amd as gt
    c, g = synth.workload("tv-4files", scale=0.01)
    assert g.num_files == 4
    check(ctx, g, brute=False)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    assert G.tv_strategy() == gt.TV_TOP_DOWN
    G.free()


def test_selector_and_strategy_errors(ctx):
    """The selector takes top-down for few files and bottom-up for many, or
    when the dense per-file counts would be too large; unknown strategies
    are refused."""
    import paper_2106_06889_amd as gt
    c = synth.random_corpus(7, 3, 500, 50)
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    assert G.tv_strategy() == gt.TV_TOP_DOWN
    with pytest.raises(gt.GtadocError) as e:
        G.term_vector(7)
    assert e.value.code == gt.ERR_INVALID_ARG
    G.free()
    c = synth.random_corpus(8, 40, 200, 50)
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    assert G.tv_strategy() == gt.TV_BOTTOM_UP
    G.free()
    G = ctx.load(g.rule_off, g.sym, g.file_off[::4], 1 << 24)  # 10 files x 2^24 ids x 8 B > 1 GiB
    assert G.tv_strategy() == gt.TV_BOTTOM_UP
    G.free()

"""GPU parity: decompression (gtadoc_decompress) and the analytics on the
uncompressed text it yields (the baseline of the paper's comparison with
GPU-accelerated uncompressed analytics), through the C ABI.

The decompressed tokens and file offsets must equal the generator's own text
(the definition the grammar was built from) and the oracle's expansion; the
word count, term vector and bigram count of the text, loaded back as a
one-rule grammar, must equal the oracle's definitions on that text."""
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
    c = gt.Context(6 << 30)
    yield c
    c.close()


def decompress(ctx, g):
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        tok, off = G.decompress()
        return tok.cpu().numpy(), off.cpu().numpy()
    finally:
        G.free()


def check_text(ctx, g, tokens, file_off):
    tok, off = decompress(ctx, g)
    assert np.array_equal(off, file_off)
    assert np.array_equal(tok, tokens)
    wtok, woff = oracle.expand(g)
    assert np.array_equal(tok, wtok) and np.array_equal(off, woff)


def plain_grammar(ctx, tokens_dev, file_off_dev, vocab):
    """The uncompressed text as a one-rule grammar (root = the tokens)."""
    import torch
    T = int(tokens_dev.numel())
    ro = torch.tensor([0, T], dtype=torch.int64, device=tokens_dev.device)
    return ctx.load(ro, tokens_dev, file_off_dev, vocab, borrow=True)


@pytest.mark.parametrize("name", ["e1_sequitur_abcdbc", "e2_two_files", "e3_head_tail"])
def test_golden(ctx, name):
    d = json.load(open(os.path.join(GOLD, f"{name}.json")))
    gd = d["grammar"]
    g = synth.Grammar(np.array(gd["rule_off"], np.int64), np.array(gd["sym"], np.int32),
                      np.array(gd["file_off"], np.int64), int(d["vocab"]))
    # the fixture's hand-written text
    check_text(ctx, g, np.array(d["tokens"], np.int32), np.array(d["file_off_text"], np.int64))


@pytest.mark.parametrize("seed", range(8))
def test_random_corpora(ctx, seed):
    """Uneven and empty files, runs, tiny vocabularies."""
    c = synth.random_corpus(100 + seed, 1 + seed % 5, 3000, [3, 40, 500][seed % 3])
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    check_text(ctx, g, c.tokens, c.file_off)


def test_hand_built_dag(ctx):
    """Not a Sequitur output: a one-symbol body, a rule used twice in one
    body, an unreachable rule, an empty file between two others."""
    # R1 = [R2 R2 a], R2 = [b], R3 = [c d] (unreachable); root: f0 = [R1 e], f1 = [], f2 = [R2 R1]
    rule_off = np.array([0, 4, 7, 8, 10], np.int64)
    sym = np.array([-1, 4, -2, -1, -2, -2, 0, 1, 2, 3], np.int32)
    file_off = np.array([0, 2, 2, 4], np.int64)
    g = synth.Grammar(rule_off, sym, file_off, 5)
    tokens = np.array([1, 1, 0, 4, 1, 1, 1, 0], np.int32)
    check_text(ctx, g, tokens, np.array([0, 4, 4, 8], np.int64))


@pytest.mark.parametrize("name,scale", [("wc-100m", 0.02), ("tv-4000files", 0.02), ("seq-20m", 0.05)])
def test_recipes_scaled(ctx, name, scale):
    c, g = synth.workload(name, scale)
    check_text(ctx, g, c.tokens, c.file_off)


def test_uncompressed_analytics_match_oracle(ctx):
    """Word count, term vector and bigram count on the decompressed text
    (one-rule grammar) against the oracle's definitions on the text."""
    import paper_2106_06889_amd as gt
    c, g = synth.workload("tv-4000files", 0.01)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    tok, off = G.decompress()
    P = plain_grammar(ctx, tok, off, g.vocab)
    try:
        assert P.stats["tokens"] == len(c.tokens) and P.build_levels() == 0
        assert np.array_equal(gt.to_u64(P.word_count()), oracle.wc_text(c.tokens, g.vocab))
        res = P.term_vector()
        got = (res.arrays[0].cpu().numpy(), res.arrays[1].cpu().numpy().view(np.uint32), gt.to_u64(res.arrays[2]))
        res.free()
        want = oracle.tv_text(c.tokens, c.file_off, g.vocab)
        assert all(np.array_equal(a, b) for a, b in zip(got, want))
        res = P.sequence_count(2)
        k, n = gt.to_u64(res.arrays[0]), gt.to_u64(res.arrays[1])
        res.free()
        wk, wn = oracle.sc_text(c.tokens, c.file_off, 2, g.vocab)
        assert np.array_equal(k, wk) and np.array_equal(n, wn)
    finally:
        P.free()
        G.free()


@pytest.mark.timeout(300)
def test_wc_100m_full(ctx):
    """The 10^8-token single-file corpus at full size, in the launch
    configuration the benchmark times: every token against the generator's
    text; word count of the text against the oracle."""
    import paper_2106_06889_amd as gt
    c, g = synth.workload("wc-100m")
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        tok, off = G.decompress()
        assert np.array_equal(off.cpu().numpy(), c.file_off)
        assert np.array_equal(tok.cpu().numpy(), c.tokens)
        P = plain_grammar(ctx, tok, off, g.vocab)
        assert np.array_equal(gt.to_u64(P.word_count()), oracle.wc_text(c.tokens, g.vocab))
        P.free()
    finally:
        G.free()

"""GPU parity: word count and sort through the C ABI against the oracle,
bit-exact (uint64 counts; the sort order is total, so unique)."""
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
    c = gt.Context(2 << 30)
    yield c
    c.close()


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        d = json.load(f)
    return synth.Grammar(np.array(d["grammar"]["rule_off"], np.int64), np.array(d["grammar"]["sym"], np.int32),
                         np.array(d["grammar"]["file_off"], np.int64), d["vocab"])


def check_wc_sort(ctx, g, expect_tokens=None):
    """Word count and sort against the oracle after both loads: the dataflow
    walk (levels built afterwards) and the level walk during the load; their
    figures agree. Returns the stats (depth included)."""
    import paper_2106_06889_amd as gt
    want = oracle.traverse_word_count(g)
    wid, wcnt = oracle.sort_counts(want)
    stats = []
    for levels in (False, True):
        G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab, levels=levels)
        try:
            assert (G.stats["depth"] == -1) != levels
            got = gt.to_u64(G.word_count())
            assert np.array_equal(got, want), levels
            assert G.stats["tokens"] == int(want.sum())
            if expect_tokens is not None:
                assert G.stats["tokens"] == expect_tokens
            ids, cnt, num = G.sort()
            k = int(num.item())
            assert k == len(wid)
            assert np.array_equal(ids[:k].cpu().numpy().view(np.uint32), wid)
            assert np.array_equal(gt.to_u64(cnt[:k]), wcnt)
            # sort from precomputed counts gives the same
            ids2, cnt2, num2 = G.sort(word_counts=G.word_count())
            assert int(num2.item()) == k and np.array_equal(ids2[:k].cpu().numpy(), ids[:k].cpu().numpy())
            G.build_levels()
            stats.append(G.stats)
        finally:
            G.free()
    assert stats[0] == stats[1]
    return stats[1]


@pytest.mark.parametrize("name", ["e1_sequitur_abcdbc.json", "e2_two_files.json", "e3_head_tail.json"])
def test_golden(ctx, name):
    g = gold(name)
    st = check_wc_sort(ctx, g)
    assert st["depth"] == {"e1_sequitur_abcdbc.json": 2, "e2_two_files.json": 2, "e3_head_tail.json": 1}[name]


def test_root_only_and_empty(ctx):
    tok = np.array([3, 1, 3, 0, 2, 3], np.int32)
    g = synth.Grammar(np.array([0, 6], np.int64), tok, np.array([0, 2, 2, 6], np.int64), 5)
    assert check_wc_sort(ctx, g)["depth"] == 0
    empty = synth.Grammar(np.array([0, 0], np.int64), np.zeros(0, np.int32), np.array([0, 0], np.int64), 3)
    check_wc_sort(ctx, empty, expect_tokens=0)


@pytest.mark.parametrize("seed", range(12))
def test_random_corpora(ctx, seed):
    c = synth.random_corpus(seed, 1 + seed % 4, 3000, [3, 20, 400][seed % 3])
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    check_wc_sort(ctx, g, expect_tokens=len(c.tokens))


def test_unreachable_rule_contributes_nothing(ctx):
    # rule 2 is never referenced; rule 3 only from rule 2
    g = synth.Grammar(np.array([0, 3, 5, 7, 9], np.int64), np.array([-1, 0, -1, 1, 2, -3, 0, 4, 4], np.int32),
                      np.array([0, 3], np.int64), 5)
    check_wc_sort(ctx, g)


def test_wc_200k_full(ctx):
    c, g = synth.workload("wc-200k")
    st = check_wc_sort(ctx, g, expect_tokens=len(c.tokens))
    assert np.array_equal(oracle.traverse_word_count(g), oracle.wc_text(c.tokens, c.vocab))
    assert st["rules"] == g.num_rules


def test_wc_100m_recipe_scaled(ctx):
    c, g = synth.workload("wc-100m", scale=0.03)
    check_wc_sort(ctx, g, expect_tokens=len(c.tokens))


@pytest.mark.parametrize("wide", [0, 1, 4096, 20000])
def test_level_walk_modes(ctx, wide):
    """The level walk's bucketed mode (levels of at least `wide` rules; 0 =
    never, 1 = every level) gives the same weights, levels and counts."""
    import paper_2106_06889_amd as gt
    cases = [synth.workload("wc-100m", scale=0.03), synth.workload("seq-20m", scale=0.02)]
    for seed in (3, 4, 5):
        c = synth.random_corpus(seed, 1 + seed % 3, 4000, [5, 60, 700][seed % 3])
        cases.append((c, synth.compress(c.tokens, c.file_off, c.vocab)))
    old = ctx.get_param(gt.PARAM_LEVEL_WIDE)
    ctx.set_param(gt.PARAM_LEVEL_WIDE, wide)
    try:
        for c, g in cases:
            st = check_wc_sort(ctx, g, expect_tokens=len(c.tokens))
            assert st["root_syms"] == int(g.rule_off[1])
            post = oracle.postorder(g)
            assert st["depth"] == longest_path_levels(g)
            assert len(post) == g.num_rules
    finally:
        ctx.set_param(gt.PARAM_LEVEL_WIDE, old)


def longest_path_levels(g):
    """Number of rule levels below the root: the longest root-to-rule path
    (rules only), by a pass over the oracle's postorder reversed."""
    post = oracle.postorder(g)
    depth = np.zeros(g.num_rules, np.int64)
    for r in post[::-1]:
        body = g.sym[g.rule_off[r]:g.rule_off[r + 1]]
        kids = -body[body < 0]
        if len(kids):
            np.maximum.at(depth, kids, depth[r] + 1)
    return int(depth.max())


def test_tile_boundaries(ctx):
    """Bodies that straddle many tile boundaries: a long non-root rule and a
    root longer than several tiles, with a ragged tail."""
    rng = np.random.default_rng(7)
    body1 = rng.integers(0, 50, size=9000).astype(np.int32)          # rule 1: > 2 tiles of words
    root = np.where(rng.random(13001) < 0.1, -1, rng.integers(0, 50, size=13001)).astype(np.int32)
    sym = np.concatenate([root, body1])
    g = synth.Grammar(np.array([0, len(root), len(sym)], np.int64), sym, np.array([0, 5000, len(root)], np.int64), 50)
    check_wc_sort(ctx, g)


def test_rejects_bad_grammars(ctx):
    import paper_2106_06889_amd as gt
    V = 4
    cases = {
        "word>=V": (np.array([0, 2, 4], np.int64), np.array([-1, -1, 0, 4], np.int32), np.array([0, 2], np.int64), gt.ERR_BAD_GRAMMAR),
        "ref>=R": (np.array([0, 2, 4], np.int64), np.array([-1, -3, 0, 1], np.int32), np.array([0, 2], np.int64), gt.ERR_BAD_GRAMMAR),
        "int32 min": (np.array([0, 2, 4], np.int64), np.array([-1, -2**31, 0, 1], np.int32), np.array([0, 2], np.int64), gt.ERR_BAD_GRAMMAR),
        "offsets": (np.array([0, 3, 2], np.int64), np.array([-1, -1, 0, 1], np.int32)[:2], np.array([0, 3], np.int64), gt.ERR_BAD_GRAMMAR),
        "empty body": (np.array([0, 2, 2], np.int64), np.array([0, 1], np.int32), np.array([0, 2], np.int64), gt.ERR_BAD_GRAMMAR),
        "spans": (np.array([0, 2, 4], np.int64), np.array([-1, -1, 0, 1], np.int32), np.array([0, 1], np.int64), gt.ERR_BAD_GRAMMAR),
        "cycle": (np.array([0, 1, 3, 5], np.int64), np.array([-1, 0, -2, -1, 1], np.int32), np.array([0, 1], np.int64), gt.ERR_CYCLE),
    }
    before = ctx.usage()[0]
    for name, (ro, sym, fo, code) in cases.items():
        for levels in (False, True):
            with pytest.raises(gt.GtadocError) as e:
                ctx.load(ro, sym, fo, V, levels=levels)
            assert e.value.code == code, (name, levels)
    assert ctx.usage()[0] == before  # nothing leaked


def test_arena_too_small():
    import paper_2106_06889_amd as gt
    small = gt.Context(1 << 16)
    c, g = synth.workload("wc-200k")
    with pytest.raises(gt.GtadocError) as e:
        small.load(g.rule_off, g.sym, g.file_off, g.vocab)
    assert e.value.code == gt.ERR_OOM
    small.close()


def test_device_and_borrowed_inputs(ctx):
    import torch
    import paper_2106_06889_amd as gt
    c, g = synth.workload("wc-200k", scale=0.5)
    want = oracle.traverse_word_count(g)
    dev = [torch.from_numpy(a).cuda() for a in (g.rule_off, g.sym, g.file_off)]
    for borrow in (False, True):
        G = ctx.load(*dev, g.vocab, borrow=borrow)
        assert np.array_equal(gt.to_u64(G.word_count()), want)
        G.free()


def test_vocabulary_beyond_bucket_table(ctx):
    """Vocabularies above 2^24 words take the direct-atomic word count path."""
    V = (1 << 24) + 5
    rng = np.random.default_rng(3)
    tok = rng.choice(np.array([0, 7, V - 1, 1 << 20, (1 << 24) + 1], np.int64), size=3000).astype(np.int32)
    g = synth.compress(tok, np.array([0, 1000, 3000], np.int64), V)
    check_wc_sort(ctx, g, expect_tokens=3000)


@pytest.mark.parametrize("keep,group,chunk", [(0, 1024, 128), (64, 512, 1), (4096, 1024, 7), (7168, 512, 4096),
                                              (1024, 512, 65535), (1024, 1024, 128)])
def test_dataflow_walk_shapes(ctx, keep, group, chunk):
    """The dataflow walk with rings that share everything beyond 0 or 64
    rules (many published chunks) or keep up to 7168, in workgroups of 512
    or 1024 threads, with level-1 chunks of 1 to 65535 rules: the same counts
    as the oracle on recipe-scaled corpora and random ones."""
    import paper_2106_06889_amd as gt
    cases = [synth.workload("wc-100m", scale=0.02), synth.workload("seq-20m", scale=0.02),
             synth.workload("tv-4000files", scale=0.005)]
    for seed in (6, 7):
        c = synth.random_corpus(seed, 2, 5000, [40, 900][seed % 2])
        cases.append((c, synth.compress(c.tokens, c.file_off, c.vocab)))
    old = ctx.get_param(gt.PARAM_FLOW_KEEP), ctx.get_param(gt.PARAM_FLOW_GROUP), ctx.get_param(gt.PARAM_FLOW_CHUNK)
    ctx.set_param(gt.PARAM_FLOW_KEEP, keep)
    ctx.set_param(gt.PARAM_FLOW_GROUP, group)
    ctx.set_param(gt.PARAM_FLOW_CHUNK, chunk)
    try:
        for c, g in cases:
            G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
            try:
                assert np.array_equal(gt.to_u64(G.word_count()), oracle.traverse_word_count(g))
                assert G.stats["tokens"] == len(c.tokens)
            finally:
                G.free()
    finally:
        ctx.set_param(gt.PARAM_FLOW_KEEP, old[0])
        ctx.set_param(gt.PARAM_FLOW_GROUP, old[1])
        ctx.set_param(gt.PARAM_FLOW_CHUNK, old[2])


def test_dataflow_ring_overflow(ctx):
    """One rule readies 20,000 sub-rules at once (each used only by it), far
    more than a workgroup's ring holds: the overflow goes to the shared queue
    as chunks of the readying waves. Also a second parent for half of them,
    so their last in-edge arrives from another rule."""
    import paper_2106_06889_amd as gt
    K, V = 20000, 11
    root = np.array([-1, 0, -1, -2], np.int32)        # rule 1 twice, rule 2 once
    body1 = -np.arange(3, 3 + K, dtype=np.int32)         # rules 3 .. K+2
    body2 = -np.arange(3, 3 + K, 2, dtype=np.int32)      # every other one again
    leaves = [np.array([r % V, (r * 7) % V], np.int32) for r in range(K)]
    bodies = [root, body1, body2] + leaves
    rule_off = np.cumsum([0] + [len(b) for b in bodies]).astype(np.int64)
    g = synth.Grammar(rule_off, np.concatenate(bodies), np.array([0, 4], np.int64), V)
    assert oracle.check_structure(g) == 0
    for group in (512, 1024):
        old = ctx.get_param(gt.PARAM_FLOW_GROUP)
        ctx.set_param(gt.PARAM_FLOW_GROUP, group)
        try:
            check_wc_sort(ctx, g)
        finally:
            ctx.set_param(gt.PARAM_FLOW_GROUP, old)


def test_deep_chain(ctx):
    """A chain of 5,000 rules under the root: one rule per level, a depth
    past the level offsets read back together with the load counters, so the
    longer read-back is taken; word count, sort, term vector, inverted index
    and bigram/trigram counts against the oracle."""
    import paper_2106_06889_amd as gt
    R, V = 5001, 7
    bodies = [np.array([-1, 3, -1, 4], np.int32)]  # root: rule 1 twice
    bodies += [np.array([-(r + 1), r % V], np.int32) for r in range(1, R - 1)]
    bodies.append(np.array([5, 6], np.int32))
    rule_off = np.cumsum([0] + [len(b) for b in bodies]).astype(np.int64)
    g = synth.Grammar(rule_off, np.concatenate(bodies), np.array([0, 2, 4], np.int64), V)
    assert oracle.check_structure(g) == 0
    st = check_wc_sort(ctx, g, expect_tokens=2 * R + 2)
    assert st["depth"] == R - 1
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        tv = G.term_vector()
        woff, wword, wcnt = oracle.traverse_term_vector(g)
        assert np.array_equal(tv.arrays[0].cpu().numpy(), woff)
        assert np.array_equal(tv.arrays[1].cpu().numpy().view(np.uint32), wword)
        assert np.array_equal(gt.to_u64(tv.arrays[2]), wcnt)
        ii = G.inverted_index_from(tv)
        ioff, ifile = oracle.inverted_index(woff, wword, g.vocab)
        assert np.array_equal(ii.arrays[0].cpu().numpy(), ioff)
        assert np.array_equal(ii.arrays[1].cpu().numpy().view(np.uint32), ifile)
        ii.free()
        tv.free()
        for n in (2, 3):
            res = G.sequence_count(n)
            wk, wc = oracle.traverse_sequence_count(g, n)
            assert np.array_equal(gt.to_u64(res.arrays[0]), wk), n
            assert np.array_equal(gt.to_u64(res.arrays[1]), wc), n
            res.free()
    finally:
        G.free()


def heavy_grammar():
    """One file: a few random words, a run of 3 * 2^21 copies of one word,
    a few more random words. Sequitur folds the run into doubling rules, so
    the innermost rule (the word twice) is used 3 * 2^20 times: its words
    take the heavy-weight path of the word-count scatter (a rule weight of
    2^20 or more does not fit the packed entry)."""
    rng = np.random.default_rng(77)
    run = np.full(3 << 21, 5, np.int32)
    tokens = np.concatenate([rng.integers(0, 40, 300, dtype=np.int32), run,
                             rng.integers(0, 40, 200, dtype=np.int32)])
    g = synth.compress(tokens, np.array([0, len(tokens)], np.int64), 40)
    return tokens, g


@pytest.mark.timeout(300)
def test_heavy_rule_weight(ctx):
    import torch
    import paper_2106_06889_amd as gt
    tokens, g = heavy_grammar()
    w = oracle.weights(g)
    assert int(w.max()) >= 1 << 20  # the case this test is for
    want = oracle.wc_text(tokens, g.vocab)
    assert np.array_equal(oracle.traverse_word_count(g), want)
    G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
    try:
        assert np.array_equal(gt.to_u64(G.word_count()), want)
        plan = ctx.batch(2, 2 * G.stats["word_syms"])
        try:
            outs = [torch.full((g.vocab,), -1, dtype=torch.int64, device=ctx.device) for _ in range(2)]
            plan.word_count([G, G], outs)
            torch.cuda.synchronize()
            for o in outs:
                assert np.array_equal(gt.to_u64(o), want)
        finally:
            plan.close()
    finally:
        G.free()


def test_timing_mask_and_order_across_streams(ctx):
    """A timing mask times only the phases it names; a call on another stream
    is ordered after the previous call's work (the sort on stream 2 reads the
    counts the word count on stream 1 writes)."""
    import torch
    import paper_2106_06889_amd as gt
    c = synth.random_corpus(29, 2, 60000, 3000)
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    want = oracle.traverse_word_count(g)
    wid, wcnt = oracle.sort_counts(want)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for ph in gt.PHASES:
        ctx.phase_time(ph, reset=True)
    ctx.set_param(gt.PARAM_TIMING, gt.timing_mask("levels", "sort"))
    try:
        assert ctx.get_param(gt.PARAM_TIMING) == gt.timing_mask("levels", "sort")
        G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab, stream=s1)
        out = torch.empty(g.vocab, dtype=torch.int64, device=ctx.device)
        torch.cuda.synchronize()
        for _ in range(3):
            G.word_count(out, stream=s1)
            ids, cnt, num = G.sort(out, stream=s2)
            s2.synchronize()
            k = int(num.item())
            assert k == len(wid)
            assert np.array_equal(ids[:k].cpu().numpy().view(np.uint32), wid)
            assert np.array_equal(gt.to_u64(cnt[:k]), wcnt)
        s1.synchronize()
        assert np.array_equal(gt.to_u64(out), want)
        counts = {ph: ctx.phase_time(ph, reset=True)[1] for ph in ("levels", "word_count", "sort", "load")}
        assert counts == {"levels": 1, "word_count": 0, "sort": 3, "load": 0}, counts
        G.free()
    finally:
        ctx.set_param(gt.PARAM_TIMING, 0)
    with pytest.raises(gt.GtadocError):
        ctx.set_param(gt.PARAM_TIMING, 2 << len(gt.PHASES))


def test_call_after_previous_stream_destroyed():
    """A call on a new stream after the previous call's stream was destroyed
    still runs (ordered by a device-wide wait) and is exact. Runs in a child
    process of its own, so a failure cannot take the test session down."""
    import subprocess
    import sys
    script = r"""
import ctypes, sys
import numpy as np, torch
sys.path.insert(0, %r)
import oracle, synth
import paper_2106_06889_amd as gt
hip = ctypes.CDLL("libamdhip64.so")
c = synth.random_corpus(31, 1, 20000, 500)
g = synth.compress(c.tokens, c.file_off, c.vocab)
want = oracle.traverse_word_count(g)
ctx = gt.Context(64 << 20)
lib = gt.lib()
s = ctypes.c_void_p()
assert hip.hipStreamCreate(ctypes.byref(s)) == 0
h = ctypes.c_void_p()
ro, sy, fo = np.ascontiguousarray(g.rule_off), np.ascontiguousarray(g.sym), np.ascontiguousarray(g.file_off)
gt.gtadoc._check(lib.gtadoc_load_grammar(ctx.handle, ro.ctypes.data, len(ro) - 1, sy.ctypes.data, len(sy),
                                         fo.ctypes.data, len(fo) - 1, g.vocab, gt.gtadoc.IN_HOST, s, ctypes.byref(h)))
out1 = torch.empty(g.vocab, dtype=torch.int64, device="cuda")
gt.gtadoc._check(lib.gtadoc_word_count(h, out1.data_ptr(), s))
assert hip.hipStreamSynchronize(s) == 0
assert hip.hipStreamDestroy(s) == 0
out2 = torch.empty(g.vocab, dtype=torch.int64, device="cuda")
gt.gtadoc._check(lib.gtadoc_word_count(h, out2.data_ptr(), torch.cuda.current_stream().cuda_stream))
torch.cuda.synchronize()
assert np.array_equal(gt.to_u64(out1), want) and np.array_equal(gt.to_u64(out2), want)
gt.gtadoc._check(lib.gtadoc_free_grammar(h))
ctx.close()
print("ok")
""" % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.returncode, r.stdout[-2000:], r.stderr[-2000:])

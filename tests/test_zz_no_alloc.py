"""The allocation-free word count (gtadoc_word_count_noalloc) against the
arena word count (gtadoc_word_count) through the C ABI: two calls in a row,
the second on a smaller grammar (the static scratch keeps the first call's
entries), bit-exact against each other and the oracle; the size limit is
refused before any work is queued."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _counts(G, fn):
    import torch
    out = torch.full((G.vocab,), -1, dtype=torch.int64, device=G.ctx.device)
    fn(out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


@pytest.mark.timeout(300)
def test_noalloc_matches_arena_word_count():
    import paper_2106_06889_amd as gt
    ctx = gt.Context(1 << 30)
    try:
        big = synth.workload("wc-200k")[1]
        c = synth.random_corpus(5, 3, 3000, 80)
        small = synth.compress(c.tokens, c.file_off, c.vocab)
        for g in (big, small):  # second call smaller than the first
            G = ctx.load(g.rule_off, g.sym, g.file_off, g.vocab)
            lib = gt.lib()
            want = oracle.traverse_word_count(g)
            a = _counts(G, lambda o: gt.gtadoc._check(lib.gtadoc_word_count(G.handle, o.data_ptr(), None)))
            b = _counts(G, lambda o: gt.gtadoc._check(lib.gtadoc_word_count_noalloc(G.handle, o.data_ptr(), None)))
            assert np.array_equal(a, want)
            assert np.array_equal(b, a)
            used_before = ctx.usage()[0]
            b2 = _counts(G, G.word_count_noalloc)
            assert np.array_equal(b2, a)
            assert ctx.usage()[0] == used_before  # no arena memory taken
            G.free()
    finally:
        ctx.close()


@pytest.mark.timeout(300)
def test_noalloc_refuses_beyond_static_scratch():
    import torch
    import paper_2106_06889_amd as gt
    n = (32 << 20) + 1  # one word symbol more than the static scratch holds
    rng = np.random.default_rng(3)
    sym = torch.from_numpy(rng.integers(0, 1000, n, dtype=np.int32)).cuda()
    ro = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    fo = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    ctx = gt.Context(512 << 20)
    try:
        G = ctx.load(ro, sym, fo, 1000, borrow=True)
        out = torch.full((1000,), 7, dtype=torch.int64, device="cuda")
        with pytest.raises(gt.GtadocError) as e:
            G.word_count_noalloc(out)
        assert e.value.code == gt.ERR_UNSUPPORTED
        torch.cuda.synchronize()
        assert bool((out == 7).all())  # outputs untouched
        got = gt.to_u64(G.word_count())
        assert np.array_equal(got, np.bincount(sym.cpu().numpy(), minlength=1000).astype(np.uint64))
        G.free()
    finally:
        ctx.close()

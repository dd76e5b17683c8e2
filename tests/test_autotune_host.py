"""Host-side logic of the autotuner (no GPU): the greedy per-parameter search
against a timing function with a known optimum, the JSON cache and the size
buckets."""
from paper_2106_06889_amd import autotune
from paper_2106_06889_amd import gtadoc as gt


class FakePlan:
    def word_count(self, grammars, outs):
        return outs

    def close(self):
        pass


class FakeCtx:
    device = "cpu"

    def __init__(self):
        self.params = {}

    def set_param(self, p, v):
        self.params[p] = v

    def batch(self, n, entries):
        return FakePlan()


class FakeGrammar:
    vocab = 4
    stats = {"word_syms": 10}


def test_greedy_search_finds_separable_optimum(monkeypatch):
    ctx = FakeCtx()
    best_blocks, best_chunk = 2, 16384

    def fake_time(fn, reps):
        fn()
        b = ctx.params[gt.PARAM_BATCH_BLOCKS_PER_CU]
        c = ctx.params[gt.PARAM_WC_CHUNK]
        return abs(b - best_blocks) + abs(c - best_chunk) / 8192.0 + 1.0

    monkeypatch.setattr(autotune, "_time", fake_time)
    res = autotune.tune_batch_word_count(ctx, [FakeGrammar(), FakeGrammar()], reps=1)
    assert res["params"] == {"batch_blocks_per_cu": best_blocks, "wc_chunk": best_chunk}
    assert ctx.params[gt.PARAM_BATCH_BLOCKS_PER_CU] == best_blocks
    assert ctx.params[gt.PARAM_WC_CHUNK] == best_chunk
    assert set(res["timings_ms"]["batch_blocks_per_cu"]) == {"1", "2", "4", "8"}


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = str(tmp_path / "cache.json")
    monkeypatch.setattr(autotune, "CACHE_PATH", path)
    key = "gfx950/wc/2^20"
    autotune.save(key, {"params": {"batch_blocks_per_cu": 8, "wc_chunk": 8192}, "timings_ms": {}}, path=path)
    ctx = FakeCtx()
    assert autotune.apply(ctx, key)
    assert ctx.params == {gt.PARAM_BATCH_BLOCKS_PER_CU: 8, gt.PARAM_WC_CHUNK: 8192}
    assert not autotune.apply(FakeCtx(), "gfx950/wc/2^30")


def test_size_bucket():
    assert autotune.size_bucket(0) == "2^0"
    assert autotune.size_bucket(1024) == "2^10"
    assert autotune.size_bucket(1500) == "2^10"
    assert autotune.size_bucket(2 ** 27) == "2^27"


def test_greedy_load_parameters(monkeypatch):
    """The level walk's launch shape and the word-count chunk: a timing
    function with a separable optimum inside the candidate lists is found
    one parameter at a time, and the best values are left set."""
    ctx = FakeCtx()
    target = {gt.PARAM_LEVEL_WIDE: 524288, gt.PARAM_LEVEL_MID_RULES: 16384, gt.PARAM_LEVEL_MID_BLOCKS: 64,
              gt.PARAM_LEVEL_TAIL_RULES: 4096, gt.PARAM_LEVEL_LONG_BODY: 64, gt.PARAM_WC_CHUNK: 8192}

    def fake_time(fn, reps):
        fn()
        return sum(abs(ctx.params[p] - v) / v for p, v in target.items())
    monkeypatch.setattr(autotune, "_time", fake_time)
    res = autotune.greedy(ctx, autotune.LOAD_CANDIDATES, autotune.LOAD_DEFAULTS, lambda: None, reps=1)
    for p, v in target.items():
        assert ctx.params[p] == v
        assert res["params"][autotune.NAMES[p]] == v

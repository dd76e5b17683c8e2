"""Seeded synthetic inputs: corpora shaped like the paper's workloads and
their Sequitur grammars.

This module holds no analytics arithmetic. It produces
  * token streams (Zipf words, repeated spans, many files, nested repeats), and
  * the compressed grammar that both the GPU library and the CPU oracle read
    (Background, "TADOC": dictionary-encoded words, a Sequitur grammar,
    unique splitters between files).

Grammar encoding (CSR, numpy arrays):
  rule_off int64[R+1]  body(r) = sym[rule_off[r]:rule_off[r+1]], r = 0 is the root
  sym      int32[S]    s >= 0 word id < vocab; s < 0 reference to rule -s
  file_off int64[F+1]  file f = root body [file_off[f], file_off[f+1])
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.cpp")
SEED_BASE = 2106068890


def build(force: bool = True) -> str:
    """Compile synth.cpp into libsynth.so (host code only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("files", ctypes.c_int32), ("tokens", ctypes.c_int64),
        ("lognorm_median", ctypes.c_double), ("lognorm_sigma", ctypes.c_double),
        ("file_min", ctypes.c_int64), ("file_max", ctypes.c_int64),
        ("vocab", ctypes.c_int32), ("zipf_s", ctypes.c_double),
        ("copy_frac", ctypes.c_double), ("span_min", ctypes.c_int32), ("span_max", ctypes.c_int32),
        ("cross_file", ctypes.c_int32),
        ("motif_chains", ctypes.c_int32), ("motif_levels", ctypes.c_int32),
        ("motif_min", ctypes.c_int32), ("motif_max", ctypes.c_int32),
        ("motif_ext_max", ctypes.c_int32), ("motif_min_inserts", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("normalize", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.synth_corpus_new.restype = vp
        lib.synth_corpus_new.argtypes = [ctypes.POINTER(_Params)]
        lib.synth_corpus_tokens.restype = i64
        lib.synth_corpus_tokens.argtypes = [vp]
        lib.synth_corpus_files.restype = i64
        lib.synth_corpus_files.argtypes = [vp]
        lib.synth_corpus_copy.argtypes = [vp, vp, vp]
        lib.synth_corpus_free.argtypes = [vp]
        lib.synth_sequitur.restype = vp
        lib.synth_sequitur.argtypes = [vp, vp, i64, i32]
        for f in ("synth_grammar_rules", "synth_grammar_syms", "synth_grammar_files"):
            getattr(lib, f).restype = i64
            getattr(lib, f).argtypes = [vp]
        lib.synth_grammar_copy.argtypes = [vp, vp, vp, vp]
        lib.synth_grammar_free.argtypes = [vp]
        _lib = lib
    return _lib


@dataclass(frozen=True)
class CorpusSpec:
    """Recipe of a seeded synthetic corpus."""
    name: str
    kind: int = 0                 # 0 span-copy text, 1 nested motif chains
    tokens: int = 200_000
    files: int = 1
    lognorm_median: float = 50_000.0
    lognorm_sigma: float = 1.32
    file_min: int = 256
    file_max: int = 5_000_000
    vocab: int = 5_000
    zipf_s: float = 1.1
    copy_frac: float = 0.30
    span_min: int = 8
    span_max: int = 64
    cross_file: int = 0
    motif_chains: int = 256
    motif_levels: int = 40
    motif_min: int = 4
    motif_max: int = 16
    motif_ext_max: int = 4
    motif_min_inserts: int = 2
    seed: int = SEED_BASE
    normalize: int = 0

    def scaled(self, factor: float, name: str | None = None) -> "CorpusSpec":
        """Same recipe at a fraction of the size: the tokens (single files and
        normalized file sets, which keep their number of files), else the
        number of files."""
        if self.files > 1 and self.normalize:
            return replace(self, name=name or f"{self.name}/x{factor:g}",
                           tokens=max(16 * self.files, int(round(self.tokens * factor))),
                           lognorm_median=self.lognorm_median * factor)
        if self.files > 1:
            return replace(self, name=name or f"{self.name}/x{factor:g}",
                           files=max(2, int(round(self.files * factor))))
        return replace(self, name=name or f"{self.name}/x{factor:g}",
                       tokens=max(16, int(round(self.tokens * factor))))


# The five workloads (sizes, vocabularies and repeat structure of the paper's
# evaluation: single large files, thousands of small files, nested repeats).
WORKLOADS = {
    "wc-200k": CorpusSpec("wc-200k", tokens=200_000, vocab=5_000, zipf_s=1.1, copy_frac=0.30,
                          span_min=8, span_max=64, seed=SEED_BASE + 1),
    "wc-100m": CorpusSpec("wc-100m", tokens=100_000_000, vocab=1_000_000, zipf_s=1.05, copy_frac=0.50,
                          span_min=16, span_max=512, seed=SEED_BASE + 2),
    "tv-4000files": CorpusSpec("tv-4000files", files=4000, lognorm_median=50_000.0, lognorm_sigma=1.32,
                               file_min=256, file_max=5_000_000, vocab=500_000, zipf_s=1.0,
                               copy_frac=0.40, span_min=8, span_max=256, cross_file=1,
                               seed=SEED_BASE + 3),
    # few large files (the top-down term vector's case): 4 files of about
    # 25M tokens each, the vocabulary and reuse of tv-4000files
    "tv-4files": CorpusSpec("tv-4files", tokens=100_000_000, files=4, lognorm_median=25_000_000.0,
                            lognorm_sigma=0.3, file_min=1, file_max=100_000_000, vocab=500_000, zipf_s=1.0,
                            copy_frac=0.40, span_min=8, span_max=256, cross_file=1, seed=SEED_BASE + 7,
                            normalize=1),
    "seq-20m": CorpusSpec("seq-20m", kind=1, tokens=20_000_000, vocab=200_000, zipf_s=1.1,
                          copy_frac=0.50, motif_chains=256, motif_levels=40, seed=SEED_BASE + 4),
    # the same shape with a vocabulary that fits 4-gram keys (16 bits per word)
    "seq4-20m": CorpusSpec("seq4-20m", kind=1, tokens=20_000_000, vocab=60_000, zipf_s=1.1,
                           copy_frac=0.50, motif_chains=256, motif_levels=40, seed=SEED_BASE + 6),
}


@dataclass
class Corpus:
    tokens: np.ndarray    # int32[T]
    file_off: np.ndarray  # int64[F+1]
    vocab: int


@dataclass
class Grammar:
    rule_off: np.ndarray  # int64[R+1]
    sym: np.ndarray       # int32[S]
    file_off: np.ndarray  # int64[F+1]
    vocab: int

    @property
    def num_rules(self) -> int:
        return len(self.rule_off) - 1

    @property
    def num_files(self) -> int:
        return len(self.file_off) - 1


def corpus(spec: CorpusSpec) -> Corpus:
    lib = _load()
    p = _Params()
    for name, _ in _Params._fields_:
        setattr(p, name, getattr(spec, name))
    h = lib.synth_corpus_new(ctypes.byref(p))
    if not h:
        raise RuntimeError(f"corpus generation failed for {spec.name}")
    try:
        T = lib.synth_corpus_tokens(h)
        F = lib.synth_corpus_files(h)
        tok = np.empty(T, dtype=np.int32)
        off = np.empty(F + 1, dtype=np.int64)
        lib.synth_corpus_copy(h, tok.ctypes.data, off.ctypes.data)
    finally:
        lib.synth_corpus_free(h)
    return Corpus(tok, off, spec.vocab)


def compress(tokens: np.ndarray, file_off: np.ndarray, vocab: int) -> Grammar:
    """Sequitur-compress the files tokens[file_off[f]:file_off[f+1]]."""
    lib = _load()
    tokens = np.ascontiguousarray(tokens, dtype=np.int32)
    file_off = np.ascontiguousarray(file_off, dtype=np.int64)
    F = len(file_off) - 1
    h = lib.synth_sequitur(tokens.ctypes.data if len(tokens) else None, file_off.ctypes.data, F, vocab)
    if not h:
        raise ValueError("sequitur: invalid input (token outside [0, vocab) or no files)")
    try:
        R = lib.synth_grammar_rules(h)
        S = lib.synth_grammar_syms(h)
        Fo = lib.synth_grammar_files(h)
        rule_off = np.empty(R + 1, dtype=np.int64)
        sym = np.empty(S, dtype=np.int32)
        foff = np.empty(Fo + 1, dtype=np.int64)
        lib.synth_grammar_copy(h, rule_off.ctypes.data, sym.ctypes.data, foff.ctypes.data)
    finally:
        lib.synth_grammar_free(h)
    return Grammar(rule_off, sym, foff, vocab)


def workload(name: str, scale: float = 1.0) -> tuple[Corpus, Grammar]:
    """Corpus and grammar of a named workload, optionally scaled down. With
    GTADOC_SYNTH_CACHE set to a directory, the pair is kept there (.npz,
    keyed by the recipe) and reused by later calls."""
    spec = WORKLOADS[name]
    if scale != 1.0:
        spec = spec.scaled(scale)
    cache = os.environ.get("GTADOC_SYNTH_CACHE")
    path = None
    if cache:
        import hashlib
        key = hashlib.sha256(repr(spec).encode()).hexdigest()[:16]
        path = os.path.join(cache, f"{name.replace('/', '_')}-{key}.npz")
        if os.path.exists(path):
            z = np.load(path)
            return (Corpus(z["tokens"], z["file_off"], int(z["vocab"])),
                    Grammar(z["rule_off"], z["sym"], z["g_file_off"], int(z["vocab"])))
    c = corpus(spec)
    g = compress(c.tokens, c.file_off, c.vocab)
    if path:
        os.makedirs(cache, exist_ok=True)
        tmp = path + ".tmp.npz"
        np.savez(tmp, tokens=c.tokens, file_off=c.file_off, vocab=c.vocab, rule_off=g.rule_off, sym=g.sym,
                 g_file_off=g.file_off)
        os.replace(tmp, path)
    return c, g


def random_corpus(seed: int, files: int, max_tokens: int, vocab: int, run_bias: float = 0.3) -> Corpus:
    """Small irregular corpora for property tests: uneven (possibly empty)
    files, tiny vocabularies, runs such as "a a a a" and repeated spans."""
    rng = np.random.default_rng(seed)
    toks, off = [], [0]
    for _ in range(files):
        n = int(rng.integers(0, max_tokens + 1))
        f = []
        while len(f) < n:
            r = rng.random()
            if r < run_bias:
                f.extend([int(rng.integers(0, vocab))] * int(rng.integers(2, 7)))
            elif r < run_bias + 0.3 and len(toks) + len(f) >= 2:
                src = toks + f
                L = int(rng.integers(2, min(12, len(src)) + 1))
                s = int(rng.integers(0, len(src) - L + 1))
                f.extend(src[s:s + L])
            else:
                f.append(int(rng.integers(0, vocab)))
        f = f[:n]
        toks.extend(f)
        off.append(len(toks))
    return Corpus(np.asarray(toks, dtype=np.int32), np.asarray(off, dtype=np.int64), vocab)


def serving_specs(count: int = 256, t_min: float = 1e4, t_max: float = 2e7, seed: int = SEED_BASE + 5,
                  scale: float = 1.0) -> list[CorpusSpec]:
    """The resident grammars of the serving workload: sizes log-uniform in
    [t_min, t_max] tokens (times `scale`), max(1, round(T/50,000)) files of
    lognormal sizes each, shared vocabulary 500,000 Zipf(1.0), 30% of each
    file copied from spans of 8-256 tokens of earlier files."""
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(count):
        T = int(round(np.exp(rng.uniform(np.log(t_min), np.log(t_max))) * scale))
        T = max(T, 64)
        F = max(1, int(round(T / 50_000)))
        specs.append(CorpusSpec(f"serve-{k}", tokens=T, files=F, lognorm_median=T / F, lognorm_sigma=1.32,
                                file_min=1, file_max=T, vocab=500_000, zipf_s=1.0, copy_frac=0.30,
                                span_min=8, span_max=256, cross_file=1, seed=seed * 1000 + k, normalize=1))
    return specs


def _build_one(spec: CorpusSpec):
    c = corpus(spec)
    g = compress(c.tokens, c.file_off, c.vocab)
    return g.rule_off, g.sym, g.file_off, g.vocab, len(c.tokens)


def serving_grammars(specs: list[CorpusSpec], workers: int = 8) -> list[tuple[Grammar, int]]:
    """Generate and compress the serving grammars in parallel processes;
    returns (grammar, tokens) pairs in spec order."""
    import multiprocessing as mp
    build()  # make sure the library exists before forking
    order = sorted(range(len(specs)), key=lambda i: -specs[i].tokens)  # biggest first
    out = [None] * len(specs)
    ctx = mp.get_context("fork")
    with ctx.Pool(processes=max(1, workers)) as pool:
        for i, res in zip(order, pool.imap(_build_one, [specs[i] for i in order])):
            ro, sym, fo, V, T = res
            out[i] = (Grammar(ro, sym, fo, V), T)
    return out

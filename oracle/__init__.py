"""CPU oracle for the analytics on Sequitur grammars -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package. The GPU library never imports, links or calls it, and the two
share no code.

Two independent routes to every result (see oracle.c):
  brute_*     expand the grammar back to text, then apply the plain definition;
  traverse_*  walk the rule DAG (weights top-down; head/tail buffers and owned
              windows for sequences; per-file top-down weights for term vectors).
Plus structural checks and the Sequitur properties of a grammar.

All results are exact integers in canonical (sorted) order:
  word_count      uint64[V]
  sort            (uint32 id[K], uint64 cnt[K]) by count desc, id asc
  term_vector     (int64 off[F+1], uint32 word[NNZ], uint64 cnt[NNZ]) per file, word asc
  inverted_index  (int64 off[V+1], uint32 file[NNZ]) per word, file asc
  ranked_inverted_index  (int64 off[V+1], uint32 file[NNZ], uint64 tf[NNZ]) per
                  word, tf desc, then file asc
  sequence_count  (uint64 key[U], uint64 cnt[U]) key asc; key packs the n-gram
                  (n=2: w0<<32|w1; n=3: w0<<42|w1<<21|w2; n=4: 16 bits per word)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OR_OK, OR_ERR_RANGE, OR_ERR_CYCLE, OR_ERR_NOMEM, OR_ERR_ARG = 0, -1, -2, -3, -4


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain C99, host only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None
_vp, _i64, _i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        sig = {
            "or_free": (None, [_vp]),
            "or_check_structure": (ctypes.c_int, [_vp, _i64, _vp, _i64, _vp, _i64, _i32]),
            "or_postorder": (_i64, [_vp, _i64, _vp, _vp]),
            "or_rule_len": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
            "or_expand": (_i64, [_vp, _i64, _vp, _vp, _i64, _vp, _vp]),
            "or_wc_text": (None, [_vp, _i64, _i32, _vp]),
            "or_sort": (_i64, [_vp, _i32, _vp, _vp]),
            "or_tv_text": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp, _vp]),
            "or_inverted_index": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp]),
            "or_sc_text": (_i64, [_vp, _vp, _i64, ctypes.c_int, _i32, _vp, _vp]),
            "or_weights": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
            "or_wc_traverse": (ctypes.c_int, [_vp, _i64, _vp, _i32, _vp]),
            "or_wc_traverse_par": (ctypes.c_int, [_vp, _i64, _vp, _i32, _vp, ctypes.c_int]),
            "or_tv_traverse": (ctypes.c_int, [_vp, _i64, _vp, _vp, _i64, _i32, _vp, _vp, _vp]),
            "or_head_tail": (ctypes.c_int, [_vp, _i64, _vp, _vp, ctypes.c_int, _vp, _vp]),
            "or_owned_counts": (ctypes.c_int, [_vp, _i64, _vp, _vp, _i64, ctypes.c_int, _vp]),
            "or_sc_traverse": (_i64, [_vp, _i64, _vp, _vp, _i64, ctypes.c_int, _i32, _vp, _vp]),
            "or_sc_text_wide": (_i64, [_vp, _vp, _i64, ctypes.c_int, _i32, _vp, _vp, _vp]),
            "or_sc_traverse_wide": (_i64, [_vp, _i64, _vp, _vp, _i64, ctypes.c_int, _i32, _vp, _vp, _vp]),
            "or_check_sequitur": (ctypes.c_int, [_vp, _i64, _vp, _vp, _i64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data if a.size else None


def _grammar(g):
    ro = np.ascontiguousarray(g.rule_off, dtype=np.int64)
    sym = np.ascontiguousarray(g.sym, dtype=np.int32)
    fo = np.ascontiguousarray(g.file_off, dtype=np.int64)
    return ro, sym, fo, len(ro) - 1, len(fo) - 1


def _take(ptr, n, dtype):
    """Copy n elements of a malloc'ed C array into numpy and free it."""
    lib = _load()
    out = np.empty(n, dtype=dtype)
    if n:
        ctypes.memmove(out.ctypes.data, ptr, n * out.itemsize)
    lib.or_free(ptr)
    return out


def _check(rc: int, what: str):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


# ---------------------------------------------------------------- structure
def check_structure(g) -> int:
    ro, sym, fo, R, F = _grammar(g)
    return _load().or_check_structure(_p(ro), R, _p(sym), len(sym), _p(fo), F, int(g.vocab))


def check_sequitur(g) -> int:
    """0 if digram uniqueness, rule utility, body length >= 2 and
    acyclic/reachable all hold; else bit flags 1, 2, 4, 8 of what fails."""
    ro, sym, fo, R, F = _grammar(g)
    return _check(_load().or_check_sequitur(_p(ro), R, _p(sym), _p(fo), F), "check_sequitur")


def postorder(g) -> np.ndarray:
    ro, sym, _, R, _ = _grammar(g)
    post = np.empty(R, dtype=np.int32)
    n = _check(_load().or_postorder(_p(ro), R, _p(sym), _p(post)), "postorder")
    return post[:n]


def rule_len(g) -> np.ndarray:
    ro, sym, _, R, _ = _grammar(g)
    ln = np.empty(R, dtype=np.uint64)
    _check(_load().or_rule_len(_p(ro), R, _p(sym), _p(ln)), "rule_len")
    return ln


def expand(g) -> tuple[np.ndarray, np.ndarray]:
    """Decompress: (tokens int32[T], file_off int64[F+1])."""
    ro, sym, fo, R, F = _grammar(g)
    ln = rule_len(g)
    T = 0
    for s in sym[fo[0]:fo[F]]:
        T += 1 if s >= 0 else int(ln[-s])
    tok = np.empty(T, dtype=np.int32)
    off = np.empty(F + 1, dtype=np.int64)
    n = _check(_load().or_expand(_p(ro), R, _p(sym), _p(fo), F, _p(tok), _p(off)), "expand")
    assert n == T
    return tok, off


# ------------------------------------------------- plain definitions on text
def wc_text(tokens: np.ndarray, vocab: int) -> np.ndarray:
    tokens = np.ascontiguousarray(tokens, dtype=np.int32)
    wc = np.empty(vocab, dtype=np.uint64)
    _load().or_wc_text(_p(tokens), len(tokens), vocab, _p(wc))
    return wc


def sort_counts(wc: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    wc = np.ascontiguousarray(wc, dtype=np.uint64)
    ids = np.empty(len(wc), dtype=np.uint32)
    cnt = np.empty(len(wc), dtype=np.uint64)
    k = _check(_load().or_sort(_p(wc), len(wc), _p(ids), _p(cnt)), "sort")
    return ids[:k], cnt[:k]


def tv_text(tokens: np.ndarray, file_off: np.ndarray, vocab: int):
    tokens = np.ascontiguousarray(tokens, dtype=np.int32)
    file_off = np.ascontiguousarray(file_off, dtype=np.int64)
    F = len(file_off) - 1
    po, pw, pc = _vp(), _vp(), _vp()
    _check(_load().or_tv_text(_p(tokens), _p(file_off), F, vocab, ctypes.byref(po), ctypes.byref(pw),
                              ctypes.byref(pc)), "tv_text")
    off = _take(po, F + 1, np.int64)
    nnz = int(off[-1])
    return off, _take(pw, nnz, np.uint32), _take(pc, nnz, np.uint64)


def inverted_index(tv_off: np.ndarray, tv_word: np.ndarray, vocab: int):
    tv_off = np.ascontiguousarray(tv_off, dtype=np.int64)
    tv_word = np.ascontiguousarray(tv_word, dtype=np.uint32)
    F = len(tv_off) - 1
    po, pf = _vp(), _vp()
    _check(_load().or_inverted_index(_p(tv_off), _p(tv_word), F, vocab, ctypes.byref(po), ctypes.byref(pf)),
           "inverted_index")
    off = _take(po, vocab + 1, np.int64)
    return off, _take(pf, int(off[-1]), np.uint32)


def ranked_inverted_index(tv_off: np.ndarray, tv_word: np.ndarray, tv_cnt: np.ndarray, vocab: int):
    """Ranked inverted index from a term vector (the paper lists it among the
    applications of its Implementation section without stating its order).
    Reading: for every word, the files that contain it, ordered by the word's
    occurrences in the file (term frequency) descending, ties by file id
    ascending. Returns (int64 off[V+1], uint32 file[NNZ], uint64 tf[NNZ]).
    A library sort is the one step: keys (word asc, tf desc, file asc)."""
    tv_off = np.asarray(tv_off, dtype=np.int64)
    word = np.asarray(tv_word, dtype=np.int64)
    tf = np.asarray(tv_cnt, dtype=np.uint64)
    file = np.repeat(np.arange(len(tv_off) - 1, dtype=np.int64), np.diff(tv_off))
    order = np.lexsort((file, -tf.astype(np.int64), word))
    off = np.zeros(vocab + 1, np.int64)
    np.cumsum(np.bincount(word, minlength=vocab), out=off[1:])
    return off, file[order].astype(np.uint32), tf[order]


def ranked_inverted_index_of(g):
    off, word, cnt = traverse_term_vector(g)
    return ranked_inverted_index(off, word, cnt, int(g.vocab))


def sc_text(tokens: np.ndarray, file_off: np.ndarray, n: int, vocab: int):
    tokens = np.ascontiguousarray(tokens, dtype=np.int32)
    file_off = np.ascontiguousarray(file_off, dtype=np.int64)
    pk, pc = _vp(), _vp()
    u = _check(_load().or_sc_text(_p(tokens), _p(file_off), len(file_off) - 1, n, vocab, ctypes.byref(pk),
                                  ctypes.byref(pc)), "sc_text")
    return _take(pk, u, np.uint64), _take(pc, u, np.uint64)


def wide_bits(vocab: int) -> int:
    """Bits per word of the wide keys: the bits of vocab - 1 (at least 1)."""
    return max(1, int(vocab - 1).bit_length())


def sc_text_wide(tokens: np.ndarray, file_off: np.ndarray, n: int, vocab: int):
    """Sequence count with wide keys (n <= 8, n * wide_bits(vocab) <= 126):
    ascending (hi uint64[U], lo uint64[U], count uint64[U]); the n-gram is the
    big-endian packing of its words, wide_bits(vocab) bits each, split into
    63-bit halves hi and lo."""
    tokens = np.ascontiguousarray(tokens, dtype=np.int32)
    file_off = np.ascontiguousarray(file_off, dtype=np.int64)
    ph, pl, pc = _vp(), _vp(), _vp()
    u = _check(_load().or_sc_text_wide(_p(tokens), _p(file_off), len(file_off) - 1, n, vocab, ctypes.byref(ph),
                                       ctypes.byref(pl), ctypes.byref(pc)), "sc_text_wide")
    return _take(ph, u, np.uint64), _take(pl, u, np.uint64), _take(pc, u, np.uint64)


def traverse_sequence_count_wide(g, n: int):
    """Sequence count with wide keys by traversal (head/tail buffers, owned
    windows weighted by rule weights); same layout as sc_text_wide."""
    ro, sym, fo, R, F = _grammar(g)
    ph, pl, pc = _vp(), _vp(), _vp()
    u = _check(_load().or_sc_traverse_wide(_p(ro), R, _p(sym), _p(fo), F, n, int(g.vocab), ctypes.byref(ph),
                                           ctypes.byref(pl), ctypes.byref(pc)), "sc_traverse_wide")
    return _take(ph, u, np.uint64), _take(pl, u, np.uint64), _take(pc, u, np.uint64)


def unpack_wide(hi: np.ndarray, lo: np.ndarray, n: int, vocab: int) -> np.ndarray:
    """The n-grams of wide keys as rows of word ids (int64[U, n])."""
    b = wide_bits(vocab)
    words = np.empty((len(hi), n), dtype=np.int64)
    h = hi.astype(object)
    l = lo.astype(object)
    v = [(int(a) << 63) | int(c) for a, c in zip(h, l)]
    mask = (1 << b) - 1
    for j in range(n):
        shift = b * (n - 1 - j)
        words[:, j] = [(x >> shift) & mask for x in v]
    return words


# --------------------------------------------------------- (A) brute force
def brute_word_count(g) -> np.ndarray:
    tok, _ = expand(g)
    return wc_text(tok, g.vocab)


def brute_term_vector(g):
    tok, off = expand(g)
    return tv_text(tok, off, g.vocab)


def brute_sequence_count(g, n: int):
    tok, off = expand(g)
    return sc_text(tok, off, n, g.vocab)


# ------------------------------------------------------------ (B) traversal
def weights(g) -> np.ndarray:
    ro, sym, _, R, _ = _grammar(g)
    w = np.empty(R, dtype=np.uint64)
    _check(_load().or_weights(_p(ro), R, _p(sym), _p(w)), "weights")
    return w


def traverse_word_count(g) -> np.ndarray:
    ro, sym, _, R, _ = _grammar(g)
    wc = np.empty(g.vocab, dtype=np.uint64)
    _check(_load().or_wc_traverse(_p(ro), R, _p(sym), int(g.vocab), _p(wc)), "wc_traverse")
    return wc


def traverse_word_count_parallel(g, threads: int) -> np.ndarray:
    """traverse_word_count with the accumulation on `threads` host threads
    (rule ranges, private count arrays); the same result."""
    ro, sym, _, R, _ = _grammar(g)
    wc = np.empty(g.vocab, dtype=np.uint64)
    _check(_load().or_wc_traverse_par(_p(ro), R, _p(sym), int(g.vocab), _p(wc), int(threads)), "wc_traverse_par")
    return wc


def traverse_term_vector_parallel(g, threads: int):
    """The per-file traversal term vector with files spread over `threads`
    host threads (the library call releases the interpreter lock), joined in
    file order: the same result as traverse_term_vector."""
    from concurrent.futures import ThreadPoolExecutor
    F = len(g.file_off) - 1
    cuts = np.linspace(0, F, min(F, 4 * threads) + 1).astype(np.int64)

    def part(k):
        sub = type(g)(g.rule_off, g.sym, g.file_off[cuts[k]:cuts[k + 1] + 1], g.vocab)
        return traverse_term_vector(sub)
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(part, range(len(cuts) - 1)))
    offs, words, cnts, base = [np.zeros(1, np.int64)], [], [], 0
    for off, word, cnt in parts:
        offs.append(off[1:] + base)
        base += int(off[-1])
        words.append(word)
        cnts.append(cnt)
    return np.concatenate(offs), np.concatenate(words), np.concatenate(cnts)


def traverse_term_vector(g):
    ro, sym, fo, R, F = _grammar(g)
    po, pw, pc = _vp(), _vp(), _vp()
    _check(_load().or_tv_traverse(_p(ro), R, _p(sym), _p(fo), F, int(g.vocab), ctypes.byref(po),
                                  ctypes.byref(pw), ctypes.byref(pc)), "tv_traverse")
    off = _take(po, F + 1, np.int64)
    nnz = int(off[-1])
    return off, _take(pw, nnz, np.uint32), _take(pc, nnz, np.uint64)


def head_tail(g, n: int):
    ro, sym, _, R, _ = _grammar(g)
    ln = rule_len(g)
    m = max(n - 1, 1)
    head = np.full((R, m), -1, dtype=np.int32)
    tail = np.full((R, m), -1, dtype=np.int32)
    _check(_load().or_head_tail(_p(ro), R, _p(sym), _p(ln), n, _p(head), _p(tail)), "head_tail")
    return head[:, :n - 1], tail[:, :n - 1], ln


def owned_counts(g, n: int) -> np.ndarray:
    ro, sym, fo, R, F = _grammar(g)
    own = np.empty(R, dtype=np.uint64)
    _check(_load().or_owned_counts(_p(ro), R, _p(sym), _p(fo), F, n, _p(own)), "owned_counts")
    return own


def traverse_sequence_count(g, n: int):
    ro, sym, fo, R, F = _grammar(g)
    pk, pc = _vp(), _vp()
    u = _check(_load().or_sc_traverse(_p(ro), R, _p(sym), _p(fo), F, n, int(g.vocab), ctypes.byref(pk),
                                      ctypes.byref(pc)), "sc_traverse")
    return _take(pk, u, np.uint64), _take(pc, u, np.uint64)


# ------------------------------------------------------------- conveniences
def word_count(g) -> np.ndarray:
    """Word count by traversal (cross-checked against brute force in the tests)."""
    return traverse_word_count(g)


def sort(g):
    return sort_counts(traverse_word_count(g))


def term_vector(g):
    return traverse_term_vector(g)


def inverted_index_of(g):
    off, word, _ = traverse_term_vector(g)
    return inverted_index(off, word, int(g.vocab))


def sequence_count(g, n: int):
    return traverse_sequence_count(g, n)


def pack(gram, n: int) -> int:
    """Key of an n-gram (same packing as the C code)."""
    if n == 1:
        return int(gram[0])
    if n == 2:
        return int(gram[0]) << 32 | int(gram[1])
    if n == 3:
        return int(gram[0]) << 42 | int(gram[1]) << 21 | int(gram[2])
    return int(gram[0]) << 48 | int(gram[1]) << 32 | int(gram[2]) << 16 | int(gram[3])

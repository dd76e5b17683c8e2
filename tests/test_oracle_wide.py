"""Pins of the oracle's sequence count with wide keys (n-grams packed into
two 63-bit halves, for n up to 8 or vocabularies whose n-grams exceed 64
bits): a hand-listed fixture, the plain definition by a library counter,
agreement of the text and traversal routes, the narrow keys where both
exist, and the closed-form total."""
import collections
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def counter_of(tokens, file_off, n):
    c = collections.Counter()
    for f in range(len(file_off) - 1):
        x = tokens[file_off[f]:file_off[f + 1]].tolist()
        for i in range(len(x) - n + 1):
            c[tuple(x[i:i + n])] += 1
    return c


def as_counter(hi, lo, cnt, n, vocab):
    rows = oracle.unpack_wide(hi, lo, n, vocab)
    return {tuple(int(v) for v in r): int(k) for r, k in zip(rows, cnt)}


def test_golden_e1_fivegrams():
    d = json.load(open(os.path.join(GOLD, "e1_fivegrams.json")))
    tok = np.array(d["tokens"], np.int32)
    off = np.array(d["file_off_text"], np.int64)
    hi, lo, cnt = oracle.sc_text_wide(tok, off, d["n"], d["vocab"])
    assert oracle.unpack_wide(hi, lo, d["n"], d["vocab"]).tolist() == d["grams"]
    assert cnt.tolist() == d["counts"]
    g = synth.compress(tok, off, d["vocab"])
    th, tl, tc = oracle.traverse_sequence_count_wide(g, d["n"])
    assert np.array_equal(th, hi) and np.array_equal(tl, lo) and np.array_equal(tc, cnt)


@pytest.mark.parametrize("seed", range(8))
def test_routes_agree_with_counter(seed):
    c = synth.random_corpus(900 + seed, 1 + seed % 4, 600, [3, 9, 300, 70000][seed % 4])
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    for n in range(2, 9):
        if n * oracle.wide_bits(c.vocab) > 126:
            continue
        hi, lo, cnt = oracle.sc_text_wide(c.tokens, c.file_off, n, c.vocab)
        th, tl, tc = oracle.traverse_sequence_count_wide(g, n)
        assert np.array_equal(th, hi) and np.array_equal(tl, lo) and np.array_equal(tc, cnt), n
        assert as_counter(hi, lo, cnt, n, c.vocab) == dict(counter_of(c.tokens, c.file_off, n))
        lens = np.diff(c.file_off)
        assert int(cnt.sum()) == int(np.maximum(lens - n + 1, 0).sum())
        # ascending (hi, lo) is lexicographic order of the n-grams
        rows = oracle.unpack_wide(hi, lo, n, c.vocab)
        assert [tuple(r) for r in rows.tolist()] == sorted(tuple(r) for r in rows.tolist())


def test_matches_narrow_keys():
    """Where the 64-bit keys exist (n <= 4), the wide keys name the same
    n-grams with the same counts."""
    c = synth.random_corpus(31, 3, 1500, 200)
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    for n, unpack in ((2, lambda k: [k >> 32, k & 0xffffffff]),
                      (3, lambda k: [k >> 42, (k >> 21) & 0x1fffff, k & 0x1fffff]),
                      (4, lambda k: [k >> 48, (k >> 32) & 0xffff, (k >> 16) & 0xffff, k & 0xffff])):
        k, cnt = oracle.traverse_sequence_count(g, n)
        narrow = {tuple(int(v) for v in unpack(int(x))): int(y) for x, y in zip(k, cnt)}
        hi, lo, wc = oracle.traverse_sequence_count_wide(g, n)
        assert as_counter(hi, lo, wc, n, c.vocab) == narrow


def test_refuses_out_of_range():
    tok = np.arange(20, dtype=np.int32)
    off = np.array([0, 20], np.int64)
    with pytest.raises(RuntimeError):
        oracle.sc_text_wide(tok, off, 9, 20)  # n > 8
    with pytest.raises(RuntimeError):
        oracle.sc_text_wide(tok, off, 5, 1 << 30)  # 5 x 30 bits > 126

"""The oracle against hand-worked examples (tests/golden/*.json, each citing
the passage it instantiates) and against textbook routines on root-only
grammars."""
import collections
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        d = json.load(f)
    g = synth.Grammar(np.array(d["grammar"]["rule_off"], np.int64), np.array(d["grammar"]["sym"], np.int32),
                      np.array(d["grammar"]["file_off"], np.int64), d["vocab"])
    return d, g


def as_dict(keys, cnts):
    return {int(k): int(c) for k, c in zip(keys, cnts)}


@pytest.mark.parametrize("name", ["e1_sequitur_abcdbc.json", "e2_two_files.json", "e3_head_tail.json"])
def test_expand_matches_text(name):
    d, g = load(name)
    assert oracle.check_structure(g) == 0
    tok, off = oracle.expand(g)
    assert tok.tolist() == d["tokens"]
    assert off.tolist() == d["file_off_text"]


def test_e1_sequitur_shape():
    d, g = load("e1_sequitur_abcdbc.json")
    got = synth.compress(np.array(d["tokens"], np.int32), np.array(d["file_off_text"]), d["vocab"])
    assert got.rule_off.tolist() == d["grammar"]["rule_off"]
    assert got.sym.tolist() == d["grammar"]["sym"]
    assert got.file_off.tolist() == d["grammar"]["file_off"]
    assert oracle.check_sequitur(got) == 0


@pytest.mark.parametrize("name", ["e1_sequitur_abcdbc.json", "e2_two_files.json"])
def test_weights_wc_sort(name):
    d, g = load(name)
    assert oracle.weights(g).tolist() == d["weights"]
    assert oracle.traverse_word_count(g).tolist() == d["word_count"]
    assert oracle.brute_word_count(g).tolist() == d["word_count"]
    ids, cnt = oracle.sort(g)
    assert ids.tolist() == d["sort"]["id"] and cnt.tolist() == d["sort"]["cnt"]


@pytest.mark.parametrize("name", ["e1_sequitur_abcdbc.json", "e2_two_files.json", "e3_head_tail.json"])
def test_sequences(name):
    d, g = load(name)
    for n, key in ((2, "bigrams"), (3, "trigrams"), (4, "fourgrams")):
        if key not in d:
            continue
        want = {int(k): v for k, v in d[key].items()}
        assert as_dict(*oracle.traverse_sequence_count(g, n)) == want
        assert as_dict(*oracle.brute_sequence_count(g, n)) == want


def test_owned_windows_e1_e3():
    d, g = load("e1_sequitur_abcdbc.json")
    assert oracle.owned_counts(g, 2).tolist() == d["owned_n2"]
    assert oracle.owned_counts(g, 3).tolist() == d["owned_n3"]
    d, g = load("e3_head_tail.json")
    assert oracle.owned_counts(g, 3).tolist() == d["owned_n3"]


def test_head_tail_e3():
    d, g = load("e3_head_tail.json")
    head, tail, _ = oracle.head_tail(g, 3)
    for r, h in d["head_n3"].items():
        assert head[int(r)].tolist() == h
    for r, t in d["tail_n3"].items():
        assert tail[int(r)].tolist() == t


def test_e2_term_vector_inverted_index():
    d, g = load("e2_two_files.json")
    for off, word, cnt in (oracle.traverse_term_vector(g), oracle.brute_term_vector(g)):
        assert off.tolist() == d["term_vector"]["off"]
        assert word.tolist() == d["term_vector"]["word"]
        assert cnt.tolist() == d["term_vector"]["cnt"]
    ioff, ifile = oracle.inverted_index_of(g)
    assert ioff.tolist() == d["inverted_index"]["off"] and ifile.tolist() == d["inverted_index"]["file"]


def test_e5_runs_sequitur():
    # a a a a -> R0 = R1 R1, R1 = a a ;  a a a a a -> R0 = R1 R1 a
    g = synth.compress(np.zeros(4, np.int32), np.array([0, 4]), 1)
    assert g.rule_off.tolist() == [0, 2, 4] and g.sym.tolist() == [-1, -1, 0, 0]
    g = synth.compress(np.zeros(5, np.int32), np.array([0, 5]), 1)
    assert g.rule_off.tolist() == [0, 3, 5] and g.sym.tolist() == [-1, -1, 0, 0, 0]
    assert oracle.check_sequitur(g) == 0
    assert oracle.traverse_word_count(g).tolist() == [5]
    k, c = oracle.traverse_sequence_count(g, 2)
    assert k.tolist() == [0] and c.tolist() == [4]
    k, c = oracle.traverse_sequence_count(g, 3)
    assert k.tolist() == [0] and c.tolist() == [3]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_e4_root_only_reduces_to_textbook(seed):
    """A grammar with no rules: word count is a bincount, sequence count is a
    sliding-window Counter, the term vector is per-file bincounts."""
    rng = np.random.default_rng(seed)
    V = 37
    sizes = rng.integers(0, 200, size=4)
    tok = rng.integers(0, V, size=int(sizes.sum())).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    g = synth.Grammar(np.array([0, len(tok)], np.int64), tok.copy(), off, V)
    assert oracle.traverse_word_count(g).tolist() == np.bincount(tok, minlength=V).tolist()
    toff, tw, tc = oracle.traverse_term_vector(g)
    for f in range(4):
        bc = np.bincount(tok[off[f]:off[f + 1]], minlength=V)
        nz = np.nonzero(bc)[0]
        assert tw[toff[f]:toff[f + 1]].tolist() == nz.tolist()
        assert tc[toff[f]:toff[f + 1]].tolist() == bc[nz].tolist()
    for n in (2, 3, 4):
        ctr = collections.Counter()
        for f in range(4):
            t = tok[off[f]:off[f + 1]].tolist()
            for i in range(len(t) - n + 1):
                ctr[oracle.pack(t[i:i + n], n)] += 1
        assert as_dict(*oracle.traverse_sequence_count(g, n)) == dict(ctr)


def _grammar_of_files(files, vocab):
    tokens = np.concatenate([np.asarray(f, np.int32) for f in files])
    file_off = np.concatenate([[0], np.cumsum([len(f) for f in files])]).astype(np.int64)
    return tokens, file_off, synth.compress(tokens, file_off, vocab)


def test_e4_ranked_inverted_index_hand_worked():
    with open(os.path.join(GOLD, "e4_ranked_inverted_index.json")) as f:
        d = json.load(f)
    _, _, g = _grammar_of_files(d["files"], d["vocab"])
    want = d["ranked_inverted_index"]
    for off, word, cnt in (oracle.traverse_term_vector(g), oracle.brute_term_vector(g)):
        roff, rfile, rtf = oracle.ranked_inverted_index(off, word, cnt, d["vocab"])
        assert roff.tolist() == want["off"] and rfile.tolist() == want["file"] and rtf.tolist() == want["tf"]
    roff, rfile, rtf = oracle.ranked_inverted_index_of(g)
    assert rfile.tolist() == want["file"]


@pytest.mark.parametrize("seed", range(6))
def test_ranked_inverted_index_by_counting(seed):
    """Against a pure-Python construction from the text (a counter per file,
    then each word's (file, tf) list sorted by tf desc, file asc), and the
    plain inverted index's file sets."""
    c = synth.random_corpus(300 + seed, 1 + 3 * (seed % 4), 1500, [5, 40, 300][seed % 3])
    g = synth.compress(c.tokens, c.file_off, c.vocab)
    roff, rfile, rtf = oracle.ranked_inverted_index_of(g)
    per_word = collections.defaultdict(list)
    for f in range(len(c.file_off) - 1):
        for w, k in collections.Counter(c.tokens[c.file_off[f]:c.file_off[f + 1]].tolist()).items():
            per_word[w].append((f, k))
    files, tfs, off = [], [], [0]
    for w in range(c.vocab):
        for f, k in sorted(per_word[w], key=lambda x: (-x[1], x[0])):
            files.append(f)
            tfs.append(k)
        off.append(len(files))
    assert roff.tolist() == off and rfile.tolist() == files and rtf.tolist() == tfs
    ioff, ifile = oracle.inverted_index_of(g)
    assert np.array_equal(ioff, roff)
    for w in range(c.vocab):
        assert sorted(rfile[roff[w]:roff[w + 1]].tolist()) == ifile[ioff[w]:ioff[w + 1]].tolist()
    assert np.array_equal(np.add.reduceat(rtf, roff[:-1][np.diff(roff) > 0]) if len(rtf) else rtf,
                          oracle.wc_text(c.tokens, c.vocab)[np.diff(roff) > 0])

"""Planted mistakes: each test compiles a copy of the oracle with one
plausible error (a dropped term, a wrong index or order, a transposed
operand) and checks that the pins used in this suite catch it. The original
oracle must pass the same pins."""
import importlib.util
import json
import multiprocessing
import os
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
GOLD = os.path.join(ROOT, "tests", "golden")

MUTANTS = {
    "weight_not_multiplied": ("if (sym[i] < 0) w[-sym[i]] += w[r];", "if (sym[i] < 0) w[-sym[i]] += 1;"),
    "wc_unweighted": ("if (sym[i] >= 0) wc[sym[i]] += w[r];", "if (sym[i] >= 0) wc[sym[i]] += 1;"),
    "tv_weight_overwritten": ("if (sym[i] < 0) wf[-sym[i]] += wf[r];", "if (sym[i] < 0) wf[-sym[i]] = wf[r];"),
    "tail_reversed": ("t[want - 1 - got++] = s;", "t[got++] = s;"),
    "child_head_from_tail": ("h[got++] = head[(size_t)(-s) * m + j];", "h[got++] = tail[(size_t)(-s) * m + j];"),
    "trigram_operands_swapped": ("(uint64_t)(uint32_t)g[1] << 21 | (uint32_t)g[2];",
                                 "(uint64_t)(uint32_t)g[2] << 21 | (uint32_t)g[1];"),
    "sort_ties_descending": ("return x < y ? -1 : (x > y);\n}\nint64_t or_sort",
                             "return x > y ? -1 : (x < y);\n}\nint64_t or_sort"),
    "windows_cross_files": ("for (int64_t i = file_off[f]; i + n <= file_off[f + 1]; ++i) keys[m++]",
                            "for (int64_t i = file_off[f]; i + n <= file_off[F] && i < file_off[f + 1]; ++i) keys[m++]"),
    "short_child_overlap_kept": ("for (int j = tn - (L - hn); j < tn; ++j)", "for (int j = 0; j < tn; ++j)"),
    "root_span_weight_dropped": ("if (sym[i] < 0) wf[-sym[i]] += 1;", "if (sym[i] < 0) wf[-sym[i]] = 1;"),
}


# Planted mistakes in the two grammar checkers, caught by the hand-built
# cases of tests/golden/checker_cases.json.
CHECKER_MUTANTS = {
    "overlap_exception_widened": ("d[i].rule == d[i + 1].rule && d[i + 1].pos == d[i].pos + 1 &&",
                                  "d[i].rule == d[i + 1].rule &&"),
    "three_occurrences_allowed": ("} else if (j - i > 2) {", "} else if (j - i > 3) {"),
    "root_pairs_across_files": ("    int64_t nspan = r == 0 ? F : 1;\n"
                                "    for (int64_t f = 0; f < nspan; ++f) {\n"
                                "      int64_t lo = r == 0 ? file_off[f] : rule_off[r];\n"
                                "      int64_t hi = r == 0 ? file_off[f + 1] : rule_off[r + 1];",
                                "    int64_t nspan = 1;\n"
                                "    for (int64_t f = 0; f < nspan; ++f) {\n"
                                "      int64_t lo = r == 0 ? file_off[f] : rule_off[r];\n"
                                "      int64_t hi = r == 0 ? file_off[F] : rule_off[r + 1];"),
    "utility_threshold_one": ("if (refs[r] < 2) flags |= 2;", "if (refs[r] < 1) flags |= 2;"),
    "short_body_threshold_one": ("rule_off[r + 1] - rule_off[r] < 2) flags |= 4;",
                                 "rule_off[r + 1] - rule_off[r] < 1) flags |= 4;"),
    "unreachable_not_flagged": ("if (n < 0 || n != R) flags |= 8;", "if (n < 0) flags |= 8;"),
    "structure_empty_body_allowed": ("    if (rule_off[r + 1] == rule_off[r]) return OR_ERR_RANGE; /* empty non-root body */\n",
                                     ""),
    "structure_offsets_unchecked": ("    if (rule_off[r + 1] < rule_off[r]) return OR_ERR_RANGE;\n", ""),
}


def checker_pins_hold(o) -> bool:
    """Every hand-built checker case gives its exact value."""
    with open(os.path.join(GOLD, "checker_cases.json")) as f:
        d = json.load(f)

    def gram(c):
        return synth.Grammar(np.array(c["rule_off"], np.int64), np.array(c["sym"], np.int32),
                             np.array(c["file_off"], np.int64), d["vocab"])
    try:
        for c in d["sequitur"]:
            if o.check_sequitur(gram(c)) != c["flags"]:
                return False
        for c in d["structure"]:
            if o.check_structure(gram(c)) != c["result"]:
                return False
    except (RuntimeError, IndexError, ValueError):
        return False
    return True


def load_variant(tmp_path, name, src_text):
    d = tmp_path / name
    d.mkdir()
    (d / "oracle.c").write_text(src_text)
    so = d / "liboracle.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-o", str(so), str(d / "oracle.c")])
    spec = importlib.util.spec_from_file_location(f"oracle_{name}", os.path.join(ROOT, "oracle", "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB_PATH = str(so)
    mod._lib = None
    return mod


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        d = json.load(f)
    g = synth.Grammar(np.array(d["grammar"]["rule_off"], np.int64), np.array(d["grammar"]["sym"], np.int32),
                      np.array(d["grammar"]["file_off"], np.int64), d["vocab"])
    return d, g


def pins_hold(o) -> bool:
    """A compact run of the suite's pins: golden values, brute force ==
    traversal, closed forms."""
    try:
        for name in ("e1_sequitur_abcdbc.json", "e2_two_files.json", "e3_head_tail.json"):
            d, g = gold(name)
            if "weights" in d and o.weights(g).tolist() != d["weights"]:
                return False
            if "word_count" in d and o.traverse_word_count(g).tolist() != d["word_count"]:
                return False
            if "sort" in d:
                ids, cnt = o.sort(g)
                if ids.tolist() != d["sort"]["id"] or cnt.tolist() != d["sort"]["cnt"]:
                    return False
            if "term_vector" in d:
                off, word, cnt = o.traverse_term_vector(g)
                if off.tolist() != d["term_vector"]["off"] or cnt.tolist() != d["term_vector"]["cnt"]:
                    return False
            for n, key in ((2, "bigrams"), (3, "trigrams")):
                if key in d:
                    want = {int(k): v for k, v in d[key].items()}
                    for fn in (o.traverse_sequence_count, o.brute_sequence_count):
                        k, c = fn(g, n)
                        if {int(a): int(b) for a, b in zip(k, c)} != want:
                            return False
            if "head_n3" in d:
                h, t, _ = o.head_tail(g, 3)
                if any(t[int(r)].tolist() != v for r, v in d["tail_n3"].items()):
                    return False
        for seed in range(4):
            c = synth.random_corpus(seed, 3, 300, 6)
            g = synth.compress(c.tokens, c.file_off, 6)
            wc = o.wc_text(c.tokens, 6)
            if not np.array_equal(o.traverse_word_count(g), wc):
                return False
            off, word, cnt = o.traverse_term_vector(g)
            boff, bword, bcnt = o.tv_text(c.tokens, c.file_off, 6)
            if not (np.array_equal(off, boff) and np.array_equal(cnt, bcnt)):
                return False
            for n in (2, 3):
                k, cn = o.traverse_sequence_count(g, n)
                bk, bc = o.sc_text(c.tokens, c.file_off, n, 6)
                if not (np.array_equal(k, bk) and np.array_equal(cn, bc)):
                    return False
                if int(bc.sum()) != int(np.maximum(np.diff(c.file_off) - n + 1, 0).sum()):
                    return False
    except (RuntimeError, IndexError, ValueError):
        return False
    return True


def _child(so_dir, name, which):
    import faulthandler
    faulthandler.disable()
    mod = importlib.util.module_from_spec(
        importlib.util.spec_from_file_location(f"oracle_{name}", os.path.join(ROOT, "oracle", "__init__.py")))
    mod.__spec__.loader.exec_module(mod)
    mod._LIB_PATH = os.path.join(so_dir, "liboracle.so")
    mod._lib = None
    ok = checker_pins_hold(mod) if which == "checker" else pins_hold(mod)
    os._exit(0 if ok else 1)


def run_pins(tmp_path, name, src_text, which="analytics") -> bool:
    """Pins of a variant, in a forked child: a variant that crashes (a planted
    out-of-bounds write, say) counts as caught."""
    load_variant(tmp_path, name, src_text)
    ctx = multiprocessing.get_context("fork")
    p = ctx.Process(target=_child, args=(str(tmp_path / name), name, which))
    p.start()
    p.join(120)
    if p.is_alive():
        p.kill()
        p.join()
        return False
    return p.exitcode == 0


def test_original_passes(tmp_path):
    with open(SRC) as f:
        src = f.read()
    assert run_pins(tmp_path, "original", src)
    assert run_pins(tmp_path, "original_checker", src, which="checker")


@pytest.mark.parametrize("mutant", sorted(CHECKER_MUTANTS))
def test_checker_mutant_is_caught(tmp_path, mutant):
    with open(SRC) as f:
        src = f.read()
    old, new = CHECKER_MUTANTS[mutant]
    assert src.count(old) == 1, f"mutation site for {mutant} not unique"
    assert not run_pins(tmp_path, mutant, src.replace(old, new), which="checker")


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, mutant):
    with open(SRC) as f:
        src = f.read()
    old, new = MUTANTS[mutant]
    assert src.count(old) == 1, f"mutation site for {mutant} not unique"
    assert not run_pins(tmp_path, mutant, src.replace(old, new))


def _ranked_variant(order_keys):
    """A copy of the ranked inverted index with another sort key list."""
    import oracle

    def ranked(tv_off, tv_word, tv_cnt, vocab):
        tv_off = np.asarray(tv_off, dtype=np.int64)
        word = np.asarray(tv_word, dtype=np.int64)
        tf = np.asarray(tv_cnt, dtype=np.uint64)
        file = np.repeat(np.arange(len(tv_off) - 1, dtype=np.int64), np.diff(tv_off))
        order = np.lexsort(order_keys(file, tf.astype(np.int64), word))
        off = np.zeros(vocab + 1, np.int64)
        np.cumsum(np.bincount(word, minlength=vocab), out=off[1:])
        return off, file[order].astype(np.uint32), tf[order]
    return ranked, oracle


RANKED_MUTANTS = {
    "tf_ascending": lambda f, t, w: (f, t, w),
    "ties_by_file_descending": lambda f, t, w: (-f, -t, w),
    "tf_before_word": lambda f, t, w: (f, w, -t),
}


@pytest.mark.parametrize("mutant", sorted(RANKED_MUTANTS))
def test_ranked_mutant_is_caught(mutant):
    """The hand-worked ranked inverted index fixture catches a wrong order."""
    with open(os.path.join(GOLD, "e4_ranked_inverted_index.json")) as fh:
        d = json.load(fh)
    tokens = np.concatenate([np.asarray(x, np.int32) for x in d["files"]])
    file_off = np.concatenate([[0], np.cumsum([len(x) for x in d["files"]])]).astype(np.int64)
    g = synth.compress(tokens, file_off, d["vocab"])
    ranked, oracle = _ranked_variant(RANKED_MUTANTS[mutant])
    off, word, cnt = oracle.traverse_term_vector(g)
    want = d["ranked_inverted_index"]
    good = oracle.ranked_inverted_index(off, word, cnt, d["vocab"])
    assert good[1].tolist() == want["file"] and good[2].tolist() == want["tf"]
    bad = ranked(off, word, cnt, d["vocab"])
    assert bad[1].tolist() != want["file"] or bad[2].tolist() != want["tf"]

"""Pins of the oracle's two grammar checkers against hand-built grammars
(tests/golden/checker_cases.json): one grammar per flag of the Sequitur
property check, the cases that must not be flagged (overlapping runs, a pair
straddling a file boundary), and one grammar per rejection of the structure
check, each asserting its exact value.

Paper: Background, TADOC (Sequitur's digram uniqueness and rule utility;
unique splitters between files; rules as nodes of a DAG)."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "checker_cases.json")
with open(GOLD) as _f:
    CASES = json.load(_f)


def grammar(case):
    return synth.Grammar(np.array(case["rule_off"], np.int64), np.array(case["sym"], np.int32),
                         np.array(case["file_off"], np.int64), CASES["vocab"])


@pytest.mark.parametrize("case", CASES["sequitur"], ids=lambda c: c["name"])
def test_sequitur_flags(case):
    g = grammar(case)
    assert oracle.check_structure(g) == 0, "the property cases are all valid encodings"
    assert oracle.check_sequitur(g) == case["flags"]


@pytest.mark.parametrize("case", CASES["structure"], ids=lambda c: c["name"])
def test_structure_result(case):
    assert oracle.check_structure(grammar(case)) == case["result"]


def test_every_flag_is_exercised_alone():
    """Each of the four flags is the whole result of at least one case, so a
    checker that drops one flag, or raises an unrelated one, fails."""
    alone = {c["flags"] for c in CASES["sequitur"]}
    assert {1, 2, 4, 8} <= alone and 0 in alone


def test_compressor_output_passes_and_mutated_output_fails():
    """The input compressor's grammars pass; the same grammar with one rule
    inlined at one of its uses (so the rule is used once) fails with flag 2."""
    c = synth.random_corpus(5, 2, 600, 8)
    g = synth.compress(c.tokens, c.file_off, 8)
    assert oracle.check_sequitur(g) == 0
    ro, sym = g.rule_off, g.sym
    refs = np.bincount(-sym[sym < 0], minlength=g.num_rules)
    r = int(np.flatnonzero(refs == 2)[0])
    at = int(np.flatnonzero(sym == -r)[0])
    body = sym[ro[r]:ro[r + 1]]
    new_sym = np.concatenate([sym[:at], body, sym[at + 1:]]).astype(np.int32)
    shift = np.where(np.arange(len(ro)) > np.searchsorted(ro, at, side="right") - 1, len(body) - 1, 0)
    new_ro = (ro + shift).astype(np.int64)
    owner = np.searchsorted(ro, at, side="right") - 1
    new_fo = g.file_off.copy()
    if owner == 0:
        new_fo = np.where(g.file_off > at, g.file_off + len(body) - 1, g.file_off).astype(np.int64)
    h = synth.Grammar(new_ro, new_sym, new_fo, g.vocab)
    assert oracle.check_structure(h) == 0
    assert np.array_equal(oracle.expand(h)[0], oracle.expand(g)[0])
    assert oracle.check_sequitur(h) & 2

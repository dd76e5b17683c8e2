"""The C-ABI library loads and exports every function include/gtadoc.h
declares (no compute: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gtadoc.h")
LIB = os.path.join(ROOT, "paper_2106_06889_amd", "libgtadoc.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gtadoc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared()
    for must in ("gtadoc_load_grammar", "gtadoc_word_count", "gtadoc_sort", "gtadoc_term_vector",
                 "gtadoc_inverted_index", "gtadoc_sequence_count"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgtadoc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2106_06889_amd import gtadoc
    assert sorted(gtadoc.EXPORTS) == declared()


def test_timing_mask_bits():
    """PARAM_TIMING masks: bit p + 1 per phase p; 1 stays 'every phase'."""
    import paper_2106_06889_amd as gt
    assert gt.timing_mask("levels") == 2
    assert gt.timing_mask("tv_tables", "tv_reduce") == (2 << gt.PHASES["tv_tables"]) | (2 << gt.PHASES["tv_reduce"])
    assert gt.timing_mask() == 0
    assert gt.timing_mask("sort", "sort") == 2 << gt.PHASES["sort"]
    assert all(gt.timing_mask(p) != 1 for p in gt.PHASES)

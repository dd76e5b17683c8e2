"""MI355X-native exact text analytics on Sequitur-compressed text (the
data-parallel hot path of G-TADOC, arXiv 2106.06889), behind the C ABI of
include/gtadoc.h. The HIP library is libgtadoc.so in this directory."""
from .gtadoc import (Batch, Context, PARAM_BATCH_BLOCKS_PER_CU, PARAM_BATCH_GRAPH, PARAM_LEVEL_WIDE, PARAM_TIMING, PARAM_WC_CHUNK, PHASES, Grammar, GtadocError, Result, Stats, lib, to_u64,  # noqa: F401
                     ERR_BAD_GRAMMAR, ERR_CYCLE, ERR_HIP, ERR_INVALID_ARG, ERR_OOM, ERR_OVERFLOW,
                     ERR_UNSUPPORTED, EXPORTS, HEADER, LIB_PATH, QUERY_INVERTED_INDEX,
                     QUERY_RANKED_INVERTED_INDEX, QUERY_SEQUENCE_COUNT, QUERY_TERM_VECTOR, QUERY_WORD_COUNT,
                     TV_AUTO, TV_BOTTOM_UP, TV_TOP_DOWN, PARAM_LEVEL_LONG_BODY, PARAM_LEVEL_MID_BLOCKS,
                     PARAM_LEVEL_MID_RULES, PARAM_LEVEL_TAIL_RULES, PARAM_FLOW_KEEP, PARAM_FLOW_GROUP, PARAM_FLOW_CHUNK,
                     LOAD_LEVELS, timing_mask)

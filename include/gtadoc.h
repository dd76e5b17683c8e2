/* gtadoc.h -- exact text analytics directly on Sequitur-compressed text,
 * on AMD Instinct MI355X (gfx950).
 *
 * The input is text compressed the TADOC way (Background, "TADOC"): words are
 * dictionary-encoded as integers and a context-free grammar, inferred by
 * Sequitur, represents the text; rules are nodes of a DAG whose root R0
 * spells the whole text, with unique splitters between files. The library
 * answers five analytics without decompressing (Section "Implementation",
 * the applications kept from the CompressDirect library): word count, sort,
 * term vector, inverted index and sequence count. Every result is an exact
 * integer; nothing is approximate.
 *
 * Conventions
 *  - Every function returns an int status: GTADOC_OK (0) or a negative
 *    GTADOC_ERR_*. No function throws. On error the caller's outputs are left
 *    untouched and gtadoc_last_error() returns a message (thread-local).
 *  - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *    Query calls are asynchronous on it unless stated otherwise.
 *  - Device memory comes from the caller: a context manages one caller-owned
 *    device buffer (the arena) from which the library sub-allocates grammars,
 *    scratch and variable-size results (the paper's self-maintained memory
 *    pool, Section "Data Structures"). The library never calls hipMalloc for
 *    them.
 *  - A context is driven by one host thread at a time. Calls on different
 *    streams are ordered by the context: a call on another stream than the
 *    previous call's waits for an event recorded after the previous call's
 *    work, so arena memory released by one call is never reused while
 *    another stream still reads it. A call on a caller-created stream
 *    records that event when it ends (the stream may be destroyed later);
 *    consecutive calls on the null stream record none (the next call on
 *    another stream records it on the null stream). gtadoc_ctx_destroy waits
 *    for the whole device.
 *
 * Grammar encoding (CSR, identical for host and device inputs):
 *   rule_off int64[num_rules + 1]  body(r) = sym[rule_off[r] .. rule_off[r+1]);
 *                                  rule 0 is the root; rule_off[0] = 0,
 *                                  rule_off[num_rules] = num_sym, non-decreasing
 *   sym      int32[num_sym]        s >= 0: a word id, s < vocab;
 *                                  s < 0: a reference to rule -s, 1 <= -s < num_rules
 *                                  (the root cannot be referenced)
 *   file_off int64[num_files + 1]  file f is the root body [file_off[f], file_off[f+1]):
 *                                  file_off[0] = 0, file_off[num_files] = length of
 *                                  the root body, non-decreasing (empty files allowed)
 *   Every rule other than the root must have a non-empty body and the rule
 *   graph must be acyclic. Rules that the root does not reach are allowed and
 *   contribute nothing.
 */
#ifndef GTADOC_H
#define GTADOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define GTADOC_OK 0
#define GTADOC_ERR_INVALID_ARG (-1)  /* null pointer, bad size, n out of range, vocab <= 0 */
#define GTADOC_ERR_BAD_GRAMMAR (-2)  /* offsets, ids or file spans violate the encoding above */
#define GTADOC_ERR_CYCLE (-3)        /* the rule graph has a cycle */
#define GTADOC_ERR_OOM (-4)          /* the arena cannot hold what the call needs */
#define GTADOC_ERR_UNSUPPORTED (-5)  /* e.g. n-gram keys that do not fit 64 bits */
#define GTADOC_ERR_OVERFLOW (-6)     /* an exact hash table could not place a key */
#define GTADOC_ERR_HIP (-7)          /* a HIP runtime call failed */

/* ---- load flags (exactly one of the first two, optionally BORROW) ---- */
#define GTADOC_IN_HOST 0x1u    /* inputs are host pointers; copied into the arena */
#define GTADOC_IN_DEVICE 0x2u  /* inputs are device pointers; copied into the arena */
#define GTADOC_IN_BORROW 0x4u  /* with IN_DEVICE: keep the caller's device arrays by
                                  reference instead of copying; they must stay alive
                                  and unchanged until gtadoc_free_grammar, and sym
                                  must be 16-byte aligned */
#define GTADOC_LOAD_LEVELS 0x8u /* build the level structure during the load (one
                                  level-synchronous walk gives levels and weights);
                                  without it the load computes the weights with the
                                  dataflow walk and the levels are built on first need */

typedef struct gtadoc_ctx_s* gtadoc_ctx;
typedef struct gtadoc_grammar_s* gtadoc_grammar;
typedef struct gtadoc_result_s* gtadoc_result;

/* Figures of a loaded grammar. */
typedef struct {
  int64_t tokens;      /* T: words of the decompressed text */
  int64_t symbols;     /* S: symbols over all rule bodies, root included */
  int64_t rules;       /* R, root included */
  int64_t files;       /* F */
  int64_t word_syms;   /* W: word symbols in all bodies */
  int64_t root_syms;   /* symbols in the root body */
  int64_t depth;       /* D: number of rule levels below the root (longest path);
                          -1 until the levels are built (GTADOC_LOAD_LEVELS,
                          gtadoc_build_levels, or a query that needs them) */
  int32_t vocab;       /* V */
  int32_t reserved;
  uint64_t arena_bytes; /* arena bytes the grammar holds */
} gtadoc_stats;

/* ---- context ---------------------------------------------------------- */

/* Create a context over a caller-owned device buffer `arena` of
 * `arena_bytes` bytes on the current HIP device (256-byte aligned). The
 * buffer must outlive the context. Errors: INVALID_ARG (null, too small or
 * misaligned), HIP. */
int gtadoc_ctx_create(void* arena, uint64_t arena_bytes, gtadoc_ctx* out);

/* Destroy a context. Grammars and results still alive in it become invalid.
 * Waits for the context's outstanding work. */
int gtadoc_ctx_destroy(gtadoc_ctx ctx);

/* Arena bytes in use now, the peak so far, and the capacity. */
int gtadoc_ctx_usage(gtadoc_ctx ctx, uint64_t* in_use, uint64_t* peak, uint64_t* capacity);

/* ---- grammars --------------------------------------------------------- */

/* Load a compressed text (encoding above) into the context and prepare it
 * for queries: validation, then the initialization phase of the paper
 * (Section "Overview", phases; Algorithm "Top-Down Traversal", mask
 * initialization and traversal): in-degrees of the rules and the top-down
 * rule weights (weight(root) = 1, weight(c) = sum over the occurrences of c
 * in body(p) of weight(p)), and with GTADOC_LOAD_LEVELS the level-by-level
 * topological frontiers of the rule DAG (level = longest path from the
 * root). Without the flag the weights come from a dataflow walk (a rule is
 * walked as soon as its last in-edge arrives, no level barriers), and the
 * levels, which the word count and sort do not use, are built by the first
 * call that needs them. Blocks until the load has finished on `stream` (it
 * reads back the validation status). Host inputs may be freed on return;
 * copied device inputs once the call has returned.
 * Errors: INVALID_ARG, BAD_GRAMMAR, CYCLE, OOM, HIP; UNSUPPORTED when a rule
 * occurs 2^40 or more times in the text or is referenced 2^24 or more times
 * by other rules (the load keeps a rule's weight and pending in-edges in one
 * 64-bit word). */
int gtadoc_load_grammar(gtadoc_ctx ctx, const int64_t* rule_off, int64_t num_rules, const int32_t* sym,
                        int64_t num_sym, const int64_t* file_off, int64_t num_files, int32_t vocab,
                        uint32_t flags, void* stream, gtadoc_grammar* out);

int gtadoc_grammar_stats(gtadoc_grammar g, gtadoc_stats* out);

/* Build the level structure of a grammar loaded without GTADOC_LOAD_LEVELS
 * (Algorithm "Top-Down Traversal", the rounds as levels): the in-degree pass
 * again into scratch, then the level walk; afterwards the stats carry the
 * depth. Does nothing when the levels exist. Term vectors, inverted indexes,
 * sequence counts, decompression, query footprints and mixed batches call
 * it themselves. Synchronizes `stream`. Errors: INVALID_ARG, OOM, HIP. */
int gtadoc_build_levels(gtadoc_grammar g, void* stream);

/* E: the number of distinct (parent, child) rule pairs of the DAG (root
 * included), counted on the first call and kept. Synchronizes `stream` on
 * the first call. Errors: INVALID_ARG, OOM, HIP. */
int gtadoc_grammar_edges(gtadoc_grammar g, int64_t* edges, void* stream);

/* Release a grammar's arena memory (after its queued work completes). */
int gtadoc_free_grammar(gtadoc_grammar g);

/* ---- queries ---------------------------------------------------------- */

/* Word count (Background, "TADOC", word-count walk-through; Algorithm
 * "Top-Down Traversal", reduce step): counts[w] = number of occurrences of
 * word w in all files, for w in [0, vocab). `counts` is a caller-owned
 * device array of vocab uint64, overwritten entirely. Asynchronous.
 * Errors: INVALID_ARG, OOM, HIP. */
int gtadoc_word_count(gtadoc_grammar g, uint64_t* counts, void* stream);

/* Word count without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation. Same result and arguments as gtadoc_word_count, but the
 * call's scratch (one 4-byte entry per word symbol of the bodies) is a
 * static device array of the library, 128 MiB per device, held from the
 * first context on that device until the process ends; no arena scratch is
 * taken and no hipMalloc, hipFree or allocating library routine is called.
 * Limit: grammars with at most 33,554,432 word symbols (stats.word_syms);
 * larger ones fail with UNSUPPORTED before any work is queued. Every call on
 * one device shares that array: calls that overlap on the same device (on
 * different streams, contexts or host threads without ordering between them)
 * race and give wrong counts; calls ordered on one stream or one context do
 * not. Asynchronous. Errors: INVALID_ARG, UNSUPPORTED, HIP. */
int gtadoc_word_count_noalloc(gtadoc_grammar g, uint64_t* counts, void* stream);

/* Decompression on the GPU (the baseline of Evaluation, Discussion,
 * "Comparison with GPU-accelerated uncompressed analytics": analytics on the
 * uncompressed text on the same GPU). Writes the text the grammar spells:
 * tokens[0..T) (caller-owned device int32, T = stats.tokens) holds the words
 * of file 0, then file 1, ...; file_off[0..F] (caller-owned device int64)
 * gets each file's start in tokens, file_off[F] = T. Expansion lengths of the
 * rules come first (children first), then the derivation tree is expanded
 * one depth at a time. Scratch from the arena: 8 B per rule, 8 B per root
 * symbol and 24 B per item of the widest depth (at most min(T, number of rule
 * occurrences in the derivation tree)). Waits once for the occurrence count,
 * then returns with the expansion queued on `stream`. The plain tokens can be
 * loaded back as a one-rule grammar (rule_off {0, T}, sym = tokens,
 * file_off) to run any query on the uncompressed text. Errors: INVALID_ARG,
 * OOM, HIP. */
int gtadoc_decompress(gtadoc_grammar g, int32_t* tokens, int64_t* file_off, void* stream);

/* Sort (an application of Section "Implementation"): the words with a
 * nonzero count, ordered by count descending, then word id ascending.
 * `word_counts` is a device array of vocab uint64 from gtadoc_word_count on
 * the same grammar, or NULL to compute it inside the call. Writes ids[0..K)
 * and counts[0..K) (caller-owned device arrays with room for vocab entries;
 * entries K..vocab are scratch on return) and K to the device int64 *num.
 * Asynchronous. Errors: INVALID_ARG, OOM, HIP. */
int gtadoc_sort(gtadoc_grammar g, const uint64_t* word_counts, uint32_t* ids, uint64_t* counts, int64_t* num,
                void* stream);

/* Term vector (an application of Section "Implementation"; bottom-up
 * traversal of Section "Fine-Grained Thread-Level Execution Engine"): for
 * every file, the (word, count) pairs with count > 0, word ascending.
 * Result arrays: [0] int64 off[F+1], [1] uint32 word[NNZ], [2] uint64 count[NNZ],
 * file f owning [off[f], off[f+1]). Synchronizes `stream` (sizes are data
 * dependent). Errors: INVALID_ARG, OOM, HIP. */
int gtadoc_term_vector(gtadoc_grammar g, gtadoc_result* out, void* stream);

/* Term vector with an explicit traversal (Section "Fine-Grained Thread-Level
 * Execution Engine": both traversals exist and a selector picks one;
 * Evaluation, Optimization Analysis, "Top-down vs. bottom-up traversals"):
 *  GTADOC_TV_BOTTOM_UP: per-rule word tables built children first, then one
 *    reduce over the files' root spans (suits many small files);
 *  GTADOC_TV_TOP_DOWN: per-file rule weights pushed from the root down, 8
 *    files at a time, then one word-count pass per file (suits few files);
 *    needs 8 B per (file, vocabulary id) of scratch for the dense counts;
 *  GTADOC_TV_AUTO: the selector's choice (gtadoc_term_vector_strategy).
 * Same result layout and errors as gtadoc_term_vector (+ INVALID_ARG for an
 * unknown strategy). */
#define GTADOC_TV_AUTO 0
#define GTADOC_TV_BOTTOM_UP 1
#define GTADOC_TV_TOP_DOWN 2
int gtadoc_term_vector_ex(gtadoc_grammar g, int strategy, gtadoc_result* out, void* stream);

/* The traversal GTADOC_TV_AUTO takes for this grammar: top-down when the
 * grammar has at most 16 files and their dense counts (8 B per file and
 * vocabulary id) fit in 1 GiB, else bottom-up. Errors: INVALID_ARG. */
int gtadoc_term_vector_strategy(gtadoc_grammar g, int* strategy);

/* Inverted index (an application of Section "Implementation"): for every
 * word, the ascending list of files that contain it. Result arrays:
 * [0] int64 off[V+1], [1] uint32 file[NNZ]. Synchronizes `stream`.
 * Errors: INVALID_ARG, OOM, HIP. */
int gtadoc_inverted_index(gtadoc_grammar g, gtadoc_result* out, void* stream);

/* Inverted index from a term vector result `term_vector` of the same grammar
 * (from gtadoc_term_vector on g, not yet freed): the same output as
 * gtadoc_inverted_index without recomputing the term vector. Synchronizes
 * `stream`. Errors: INVALID_ARG (null, or a result that is not a term vector
 * of g), OOM, HIP. */
int gtadoc_inverted_index_from_tv(gtadoc_grammar g, gtadoc_result term_vector, gtadoc_result* out, void* stream);

/* Ranked inverted index (Section "Implementation": one of the six
 * applications behind the CompressDirect interfaces; the paper names it
 * without stating its order).
 * Read here as: for every word, the files that contain it ordered by term
 * frequency descending, ties by file ascending. Result arrays: [0] int64
 * off[V+1], [1] uint32 file[NNZ], [2] uint64 tf[NNZ] (occurrences of the
 * word in that file). Synchronizes `stream`. Errors: INVALID_ARG, OOM, HIP. */
int gtadoc_ranked_inverted_index(gtadoc_grammar g, gtadoc_result* out, void* stream);

/* The ranked inverted index from a term vector result of the same grammar
 * (as gtadoc_inverted_index_from_tv). Errors: INVALID_ARG (null, or a result
 * that is not a term vector of g), OOM, HIP. */
int gtadoc_ranked_inverted_index_from_tv(gtadoc_grammar g, gtadoc_result term_vector, gtadoc_result* out,
                                         void* stream);

/* Sequence count (Section "Sequence Support"): occurrences of every run of n
 * consecutive words inside one file (runs never cross files), n in {2, 3, 4}.
 * Result arrays: [0] uint64 key[U] ascending, [1] uint64 count[U], where the
 * key packs the n-gram (w0, .., w(n-1)) as w0<<32|w1 for n = 2,
 * w0<<42|w1<<21|w2 for n = 3 and w0<<48|w1<<32|w2<<16|w3 for n = 4
 * (ascending keys = lexicographic order). Synchronizes `stream`. Errors:
 * INVALID_ARG (n), UNSUPPORTED (n = 3 with vocab > 2^21, n = 4 with vocab
 * >= 2^16), OVERFLOW, OOM, HIP. */
int gtadoc_sequence_count(gtadoc_grammar g, int n, gtadoc_result* out, void* stream);

/* Sequence count for any length n in 2..8 with wide keys (Section "Sequence
 * Support": sequences of a general length; head and tail buffers of up to 7
 * words per rule). The n-gram's words, b = bits of (vocab - 1) each, are
 * packed big-endian into a number of n * b <= 126 bits, split into the upper
 * and lower 63 bits (hi, lo), so ascending (hi, lo) is lexicographic n-gram
 * order. Result arrays: [0] uint64 hi[U], [1] uint64 lo[U], [2] uint64
 * count[U], ascending (hi, lo). Synchronizes `stream`. Errors: INVALID_ARG
 * (n outside 2..8), UNSUPPORTED (n * b > 126), OOM, OVERFLOW, HIP. */
int gtadoc_sequence_count_wide(gtadoc_grammar g, int n, gtadoc_result* out, void* stream);

/* ---- tunables (read by the autotuner; per context) ---------------------- */
#define GTADOC_PARAM_WC_CHUNK 1          /* word-count reduce: entries per work item (>= 1024) */
#define GTADOC_PARAM_BATCH_BLOCKS_PER_CU 2  /* batched word count: persistent scatter workgroups per CU */
#define GTADOC_PARAM_BATCH_GRAPH 3       /* 1: replay a batch's launch sequence from a captured hipGraph */

#define GTADOC_PARAM_TIMING 4          /* 1: record HIP events around the main kernels of every call;
                                          other values: a mask, bit (p + 1) times phase p only (each
                                          event pair leaves the GPU idle for a few microseconds) */
#define GTADOC_PARAM_LEVEL_WIDE 5      /* load: levels of at least this many rules accumulate weights and
                                          in-edges by bucket instead of atomics (0: never; default 262144) */
#define GTADOC_PARAM_LEVEL_LONG_BODY 6  /* load: rule bodies longer than this are walked by a whole
                                          wave (the thread-group threshold for long rules); default 32 */
#define GTADOC_PARAM_LEVEL_MID_RULES 7  /* load: levels narrower than this run on MID_BLOCKS workgroups */
#define GTADOC_PARAM_LEVEL_MID_BLOCKS 8 /* load: workgroups of the narrower levels (1..256); default 32 */
#define GTADOC_PARAM_LEVEL_TAIL_RULES 9 /* load: levels narrower than this run on one workgroup; default 1024 */
#define GTADOC_PARAM_FLOW_KEEP 10       /* load, dataflow walk: ready rules a workgroup keeps in its ring at
                                          the end of a round, per 1024 threads; the rest go to the shared
                                          queue (0..7168; default 4096) */
#define GTADOC_PARAM_FLOW_GROUP 11      /* load, dataflow walk: threads per workgroup, 512 (two per CU) or
                                          1024 (default) */
#define GTADOC_PARAM_FLOW_CHUNK 12      /* load, dataflow walk: rules per chunk of level 1 in its queue
                                          (1..65535; default 128) */

/* Set / get a tunable. Errors: INVALID_ARG (unknown parameter or value). */
int gtadoc_ctx_set_param(gtadoc_ctx ctx, int param, int64_t value);
int gtadoc_ctx_get_param(gtadoc_ctx ctx, int param, int64_t* value);

/* ---- kernel timing (GTADOC_PARAM_TIMING) ------------------------------------
 * With timing on, every call records a pair of HIP events on its stream
 * around each of the phases below; gtadoc_ctx_phase_time waits for the
 * recorded events and returns the summed device time (ms) and the number of
 * timed occurrences, optionally resetting them. */
#define GTADOC_PHASE_LEVELS 0       /* load: the weight walk (the level walk or the dataflow walk), one
                                       kernel; also the level walk of gtadoc_build_levels */
#define GTADOC_PHASE_WORD_COUNT 1   /* word count: bucket scatter + on-chip reduce */
#define GTADOC_PHASE_SORT 2         /* sort: compaction + radix passes */
#define GTADOC_PHASE_SEQ_WINDOWS 3  /* sequence count: owned windows into the exact hash table, one kernel */
#define GTADOC_PHASE_TV_TABLES 4    /* term vector: bottom-up rule tables */
#define GTADOC_PHASE_TV_REDUCE 5    /* term vector: per-file scatter + reduce */
#define GTADOC_PHASE_LOAD 6         /* load: all device work after validation (degrees, levels, weights) */
#define GTADOC_PHASE_DECOMPRESS 7   /* decompression: rule lengths, root positions, depth-by-depth expansion */
#define GTADOC_PHASE_TV_TOPDOWN 8   /* term vector, top-down: per-file weights and per-file word-count passes */
#define GTADOC_NUM_PHASES 9
int gtadoc_ctx_phase_time(gtadoc_ctx ctx, int phase, double* total_ms, int64_t* count, int reset);

/* ---- batched queries ------------------------------------------------------
 * Many grammars of uneven size in one launch sequence: persistent kernels
 * with a fixed grid walk a flattened list of work items (each grammar's
 * blocks and chunks) described in device memory. The sequence is identical
 * for every batch, so with GTADOC_PARAM_BATCH_GRAPH it is captured once into
 * a hipGraph and replayed; only the descriptors change. */
typedef struct gtadoc_batch_s* gtadoc_batch;

/* A batch plan on ctx for up to max_items grammars whose word symbols total
 * at most max_entries; its scratch is taken from the arena now. Errors:
 * INVALID_ARG, OOM, HIP. */
int gtadoc_batch_create(gtadoc_ctx ctx, int max_items, uint64_t max_entries, gtadoc_batch* out);

/* Word count of gs[i] into counts[i] (device arrays of vocab_i uint64), for
 * i < n, asynchronous on `stream`. Waits for the plan's previous batch
 * before reusing its descriptors. Every grammar must belong to the plan's
 * context and use the bucketed word count (vocab <= 2^24).
 * Errors: INVALID_ARG (n, sizes, foreign grammar), UNSUPPORTED, HIP. */
int gtadoc_batch_word_count(gtadoc_batch b, const gtadoc_grammar* gs, uint64_t* const* counts, int n, void* stream);

int gtadoc_batch_destroy(gtadoc_batch b);

/* A query of a mixed batch (gtadoc_batch_submit). */
#define GTADOC_QUERY_WORD_COUNT 1      /* counts: caller-owned device array of vocab uint64 */
#define GTADOC_QUERY_TERM_VECTOR 2     /* result as gtadoc_term_vector_ex(strategy) */
#define GTADOC_QUERY_SEQUENCE_COUNT 3  /* result as gtadoc_sequence_count(n) */
#define GTADOC_QUERY_INVERTED_INDEX 4  /* result as gtadoc_inverted_index */
#define GTADOC_QUERY_RANKED_INVERTED_INDEX 5
typedef struct {
  gtadoc_grammar grammar; /* in: a grammar of the plan's context */
  int32_t kind;           /* in: GTADOC_QUERY_* */
  int32_t n;              /* in: n-gram length (SEQUENCE_COUNT) */
  uint64_t* counts;       /* in: output of WORD_COUNT */
  gtadoc_result result;   /* out: result of the other kinds (NULL on error); free with gtadoc_result_free */
  int32_t status;         /* out: GTADOC_OK or the query's error code */
  int32_t strategy;       /* in: TERM_VECTOR traversal (GTADOC_TV_*; 0 = the selector) */
} gtadoc_query;

/* Run a mixed batch: word counts, term vectors, sequence counts and
 * (ranked) inverted indexes of any grammars of the plan's context. The word
 * counts (at most the plan's max_items, word symbols within max_entries) run
 * as one batched persistent launch sequence on `stream`, like
 * gtadoc_batch_word_count; each other query runs on one of the plan's own
 * streams (four, default priority; sequence counts of one grammar share a
 * stream), all of them ordered after the context's earlier work, so their
 * kernels overlap on the device with each other and with the word counts.
 * Grammars loaded without levels get them first (gtadoc_build_levels, once
 * per grammar, synchronizing `stream`) when a query other than a word count
 * needs them. The call returns once every query is queued (variable-size
 * results synchronize their own stream for their sizes); all of the batch's work is
 * complete when `stream` passes the point of return. Each query's status is
 * written to q[i].status (OOM, UNSUPPORTED, ... for that query alone).
 * Errors of the call itself: INVALID_ARG (a malformed query: null or foreign
 * grammar, unknown kind, bad n or strategy, missing counts; too many word
 * counts for the plan; nothing is queued then), HIP. */
int gtadoc_batch_submit(gtadoc_batch b, gtadoc_query* q, int nq, void* stream);

/* Arena bytes a query of this kind on g takes at its peak (scratch plus its
 * result; for WORD_COUNT the scratch alone, the counts being the caller's):
 * the admission figure of a server that keeps grammars resident. Allocation
 * sizes depend only on the grammar and the query, so the first call for a
 * (kind, n, strategy) runs the query once on `stream`, measures the arena's
 * peak above its level before the query, frees the result and keeps the
 * figure (the call synchronizes `stream`); later calls return it at once.
 * Sequence count's head/tail buffers, built on first use and kept with the
 * grammar, are not part of the figure. n: SEQUENCE_COUNT only; strategy:
 * TERM_VECTOR only (GTADOC_TV_*). Errors: INVALID_ARG, UNSUPPORTED, OOM (the
 * arena cannot hold the query now), HIP. */
int gtadoc_query_bytes(gtadoc_grammar g, int kind, int n, int strategy, uint64_t* bytes, void* stream);

/* Array `index` of a result: device pointer (inside the arena), element
 * count and element size in bytes. The result's sizes are final when the
 * producing call returns. Errors: INVALID_ARG. */
int gtadoc_result_array(gtadoc_result res, int index, void** dptr, int64_t* length, int* elem_bytes);

/* Release a result's arena memory. */
int gtadoc_result_free(gtadoc_result res);

/* Message of the last error on this host thread ("" if none). */
const char* gtadoc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GTADOC_H */

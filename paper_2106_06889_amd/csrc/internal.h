// internal.h -- shared declarations of the gtadoc library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/gtadoc.h"

namespace gt {

// ---------------------------------------------------------------------------
// Launch geometry
// ---------------------------------------------------------------------------
// Position-parallel passes over the rule bodies work on tiles of kTileSyms
// consecutive symbols, one 256-thread workgroup per tile, 16 consecutive
// symbols per thread (four 16-byte loads).
constexpr int kTileSyms = 4096;
constexpr int kTileThreads = 256;
constexpr int kPerThread = kTileSyms / kTileThreads;
// LDS slots for a tile's rule offsets: at most kTileSyms + 2 rules overlap a tile.
constexpr int kTileRuleSlots = kTileSyms + 4;
// Passes that keep per-block tables (histograms, bucket cursors) walk
// kSubTiles consecutive tiles per workgroup: blocks of kBlockSyms symbols.
// Three tiles keep the word-count scatter's LDS (rule offsets + the block's
// staged entries) under half of a CU's 160 KB, so two 1024-thread
// workgroups share a CU.
constexpr int kSubTiles = 3;
constexpr int kBlockSyms = kTileSyms * kSubTiles;
// Word count by buckets of consecutive word ids: a bucket's counters
// (kWcBucket x uint64) fit in LDS. Entries pack (weight << kWcBits | local id).
constexpr int kWcBits = 12;
constexpr int kWcBucket = 1 << kWcBits;
constexpr int kWcMaxBuckets = 4096;  // vocabularies up to 2^24 words use buckets
// In-degrees the same way: buckets of 4096 consecutive rule ids, one uint16
// entry per rule reference (low 12 bits of the child id, bit 15 = the
// reference sits in the root).
constexpr int kRcBits = 12;
constexpr int kRcBucket = 1 << kRcBits;
constexpr int kRcMaxBuckets = 4096;  // grammars up to 2^24 rules
constexpr uint16_t kRcRootFlag = 0x8000;
// Per-block runs of a bucket are ordered XCD by XCD (workgroups are dispatched
// to the 8 XCDs round-robin), so neighbouring runs are written through the
// same L2. A table row holds nslot = 8 * ceil(nblk / 8) slots.
constexpr int kXcds = 8;
__host__ __device__ inline int64_t xcd_slot(int64_t blk, int64_t nslot) {
  return (blk % kXcds) * (nslot / kXcds) + blk / kXcds;
}

// During the load every rule's weight and its pending in-edges (references
// from non-root bodies not yet applied) share one 64-bit word,
// weight << kPendBits | pending, so that one atomic adds a parent's weight
// and retires its in-edge, and its return value tells whether that was the
// last one. The load unpacks the words into plain weights at the end.
constexpr int kPendBits = 24;
constexpr uint64_t kPendMask = (1ull << kPendBits) - 1;
constexpr int kWeightBits = 64 - kPendBits;

// Bits of the validation status word.
enum : uint32_t {
  ST_BAD_OFFSETS = 1u,   // rule_off not monotone / not [0, S]
  ST_EMPTY_BODY = 2u,    // a non-root rule has an empty body
  ST_BAD_FILES = 4u,     // file spans do not tile the root body
  ST_BAD_WORD = 8u,      // word id >= vocab
  ST_BAD_REF = 16u,      // rule reference outside [1, R)
  ST_PACK = 32u,         // a weight >= 2^40 or an in-degree >= 2^24 (beyond the packed load word)
  ST_FLOW = 64u,         // the dataflow walk ran out of queue room or waited past its bound (internal)
};
// A load may queue its later passes before the host has read the layout
// checks; these passes then leave at once when one of these bits is set
// (the offsets cannot be trusted for indexing).
constexpr uint32_t kBadLayout = ST_BAD_OFFSETS | ST_EMPTY_BODY | ST_BAD_FILES;

// Device view of a loaded grammar and its initialization-phase products.
struct DevGrammar {
  const int64_t* rule_off;   // [R+1]
  const int32_t* sym;        // [S]
  const int64_t* file_off;   // [F+1]
  int64_t R, S, F;
  int32_t V;
  int64_t ntiles;            // ceil(S / kTileSyms)
  const int32_t* tile_rule;  // [ntiles+1]: rule holding the first symbol of each tile; [ntiles] = R-1
  uint64_t* w;               // [R] top-down weights, w[0] = 1 (packed with pending in-edges during the load)
  int32_t* level_rule;       // [R-1] rules grouped by level (level 1 first)
  int32_t* level_off;        // [D+2] level d occupies level_rule[level_off[d] .. level_off[d+1]), d >= 1
  int64_t nblk;              // ceil(S / kBlockSyms)
  int64_t nslot;             // kXcds * ceil(nblk / kXcds): slots per bucket row
  int32_t wc_nb;             // word buckets (0: vocabulary too large, word count uses direct atomics)
  uint32_t* wc_off;          // [wc_nb * nslot] bucket-major exclusive offsets of word entries
  int32_t rc_nb;             // rule buckets for in-degrees (0: too many rules, direct atomics)
  uint32_t* rc_off;          // [rc_nb * nslot] bucket-major exclusive offsets of reference entries
  int64_t span_file = -1;    // word-count pass: -1 = every root word has weight 1; f = only file f's root words
};

// Load-phase scalars written by the kernels and read back once.
struct LoadCounters {
  uint32_t status;       // ST_* bits
  int32_t depth;         // number of levels
  int32_t placed;        // rules placed in levels (R-1 unless there is a cycle)
  int32_t pad;
  uint64_t tokens;       // T
  uint64_t word_syms;    // W
  uint64_t root_words;   // words directly in the root body
  int64_t frontier0;     // rules of level 1
  int64_t wc_entries;    // word entries counted into wc_off (= W)
  int64_t rc_entries;    // reference entries counted into rc_off (= S - W)
  int64_t root_syms;     // length of the root body
  int64_t wide_entries;  // references from non-root bodies (capacity of the wide-level entries)
};

// Buffers of the bucketed mode of the level walk (wide levels): the
// references of every non-root body, grouped by the referenced rule's bucket
// (bucket = id mod nbk, slot = id / nbk, nbk a power of two); bucket b owns
// [off[b], off[b+1]) of ew/ec, filled level after level (cur[b] = end of what
// is written, seg_lo[b] = end of what is reduced). ew == nullptr disables the
// mode.
constexpr int kWideBucket = 4096;  // most slots per bucket (LDS table of the reduce)
constexpr int kWideMaxBuckets = 16384;
struct WideBufs {
  uint64_t* ew;      // weight of the referencing rule
  uint16_t* ec;      // slot of the referenced rule in its bucket
  uint32_t* cur;     // [nbk]
  uint32_t* seg_lo;  // [nbk]
  int32_t nbk;       // power of two, nbk * kWideBucket >= R
  int32_t nbk_bits;  // log2(nbk)
  int32_t slots;     // ceil(R / nbk) <= kWideBucket
  int32_t min_rules;  // levels with at least this many rules use the bucketed mode
};

// ---------------------------------------------------------------------------
// Kernel launchers (each returns the launch status)
// ---------------------------------------------------------------------------
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

// load phase
hipError_t launch_check_rules(const int64_t* rule_off, int64_t R, int64_t S, int32_t* tile_rule, int64_t ntiles,
                              LoadCounters* lc, hipStream_t s);
// both checks plus zero fills of up to 6 ranges (in 32-bit words) in one
// launch (lc zero before it)
struct ZeroRanges {
  uint32_t* p[6];
  int64_t n[6];
  int count;
  void add(void* ptr, int64_t words) {
    if (ptr && words > 0) p[count] = static_cast<uint32_t*>(ptr), n[count] = words, ++count;
  }
};
hipError_t launch_load_prologue(const int64_t* rule_off, int64_t R, int64_t S, const int64_t* file_off, int64_t F,
                                int32_t* tile_rule, int64_t ntiles, LoadCounters* lc, const ZeroRanges& z,
                                hipStream_t s);
hipError_t launch_check_files(const int64_t* file_off, int64_t F, const int64_t* rule_off, LoadCounters* lc,
                              hipStream_t s);
hipError_t launch_scan_symbols(const DevGrammar& g, LoadCounters* lc, hipStream_t s);
// in-degrees and initial weights (packed in g.w) from the reference entries
// (after the offsets are scanned)
hipError_t launch_in_degrees(const DevGrammar& g, uint16_t* entries, const int64_t* n, LoadCounters* lc, hipStream_t s,
                             bool w_zeroed = false);
struct FlowState;
// level 1 (rules no rule references) by compaction into g.level_rule in
// rule-id order (and, when qw is given, their weights into qw and the
// dataflow walk's counters into fs), then the level walk
hipError_t launch_level_frontier(const DevGrammar& g, LoadCounters* lc, uint32_t* scratch, hipStream_t s,
                                 uint64_t* qw = nullptr, FlowState* fs = nullptr);
hipError_t prepare_level_walk(const DevGrammar& g, LoadCounters* lc, uint32_t* scratch, const WideBufs& wide,
                              hipStream_t s);
// Launch shape of the level walk (context parameters, tunable):
//  long_body   bodies longer than this are walked by a whole wave (the
//              paper's thread-group threshold for long rules);
//  mid_rules   levels narrower than this run on the first mid_blocks
//              workgroups only (a cheaper barrier);
//  tail_rules  levels narrower than this run on workgroup 0 alone.
//  flow_keep   the dataflow walk keeps at most this many ready rules in a
//              workgroup's ring at the end of a round and shares the rest
//              (per 1024 threads);
//  flow_group  threads per workgroup of the dataflow walk (512: two
//              workgroups per CU, or 1024);
//  flow_chunk  rules per level-1 chunk of the dataflow walk's queue.
struct LevelParams {
  int32_t long_body = 32;
  int32_t mid_rules = 48 * 1024;
  int32_t mid_blocks = 32;
  int32_t tail_rules = 1024;
  int32_t flow_keep = 4096;
  int32_t flow_group = 1024;
  int32_t flow_chunk = 128;
};
hipError_t launch_level_walk(const DevGrammar& g, int32_t* level_cnt, LoadCounters* lc, uint32_t* scratch,
                             const WideBufs& wide, const LevelParams& params, int device, hipStream_t s);
// after the walk: g.w[r] = weight of r (the pending fields are zero)
hipError_t launch_unpack_weights(const DevGrammar& g, hipStream_t s);

// Dataflow walk (weights without levels): the global queue of ready rules
// (level 1 first, with their weights) and the descriptors of the chunks
// published into it; counters in FlowState. Waiting workgroups poll `live`
// and working ones take tickets and queue space, so the groups of counters
// sit on separate 256-byte lines: atomics on one line are served one after
// the other, and polls would otherwise queue the working side's atomics.
struct FlowState {
  alignas(256) int64_t live;  // rules queued anywhere or being walked
  alignas(256) uint32_t ticket;  // next chunk ticket
  uint32_t space;              // queue entries reserved (level 1 first)
  uint32_t nspill;             // chunks published beyond level 1
  alignas(256) uint32_t idle;  // workgroups waiting for work
  alignas(256) int64_t n1;     // rules of level 1
};
struct FlowBufs {
  int32_t* qc;     // [qcap] rules (level_rule)
  uint64_t* qw;    // [qcap] their final weights
  uint64_t* desc;  // [ndesc] published chunks: start << 16 | count, 0 = not yet
  uint32_t qcap, ndesc;
};
// The walk, after launch_level_frontier has queued level 1. placed and
// tokens are added to lc (zero before); fs (beyond what the frontier set)
// and fb.desc must be zero; g.w holds packed words on entry and unpacks like
// after the level walk.
hipError_t launch_flow_walk(const DevGrammar& g, LoadCounters* lc, FlowState* fs, const FlowBufs& fb,
                            const LevelParams& lp, int device, hipStream_t s);

// word count and sort
hipError_t launch_word_count(const DevGrammar& g, uint64_t* counts, hipStream_t s);   // direct atomics
hipError_t launch_word_count_buckets(const DevGrammar& g, uint64_t* counts, uint32_t* entries, int64_t W,
                                     int64_t chunk, hipStream_t s);
// batched word count: descriptors in device memory
constexpr int kBatchMax = 1024;
struct BatchItem {
  DevGrammar g;
  uint64_t* out;       // [V] counts
  uint32_t* entries;   // [W] scratch
  int64_t W;
};
struct BatchDesc {
  int32_t n;
  int32_t pad;
  int64_t chunk;                       // reduce chunk (entries per work item)
  int64_t fill_base[kBatchMax + 1];    // prefix of ceil(V / 4096) per grammar
  int64_t scatter_base[kBatchMax + 1]; // prefix of nblk
  int64_t reduce_base[kBatchMax + 1];  // prefix of ceil(W / chunk)
  BatchItem items[kBatchMax];
};
hipError_t launch_word_count_batch(const BatchDesc* d, int grid_scatter, int grid_reduce, int max_nb, hipStream_t s);
hipError_t launch_scan_offsets(uint32_t* a, int64_t n, int64_t* total, uint32_t* sums, hipStream_t s);
// both arrays (either may be empty) in three launches; sums needs
// scan2_scratch_entries(na, nb)
hipError_t launch_scan_offsets2(uint32_t* a, int64_t na, int64_t* ta, uint32_t* b, int64_t nb, int64_t* tb,
                                uint32_t* sums, hipStream_t s);
int64_t scan2_scratch_entries(int64_t na, int64_t nb);
int64_t scan_scratch_entries(int64_t n);
struct SortScratch {
  uint64_t* key[2];
  uint32_t* val[2];
  uint32_t* hist;       // [word_sort_hist_entries(V)]
};
int64_t sort_scratch_hist_entries(int64_t n);
int64_t word_sort_hist_entries(int64_t V);
// The bits of a 64-bit key that can differ between keys: nseg (1..4) ranges
// [lo[i], lo[i] + len[i]), ascending and disjoint; every other bit is the
// same in all keys.
struct KeyBits {
  int nseg;
  int lo[4], len[4];
};
int64_t key_sort_hist_entries(int64_t n);
// Stable ascending LSD sort of n < 2^32 (key, value) pairs on the bits kb
// names: input (k0, v0), scratch (k1, v1), result in (kout, vout), which may
// not alias the input or the scratch; hist holds key_sort_hist_entries(n).
hipError_t launch_sort_key_bits(uint64_t* k0, uint64_t* v0, uint64_t* k1, uint64_t* v1, int64_t n,
                                const KeyBits& kb, uint32_t* hist, uint64_t* kout, uint64_t* vout, hipStream_t s);

// term vector / inverted index
struct TvFiles {
  const int64_t* unit_off;  // [F+1] first kTileSyms-unit of every file
  int64_t nunits;
  int32_t nb;               // word buckets
  uint32_t* table;          // [nb * nunits] counts, then offsets
  const uint64_t* toff;     // rule table offsets in the pool
  const uint32_t* tsize;    // rule table sizes
  const uint32_t* pw;       // pool: words
  const uint32_t* pc;       // pool: counts
};
hipError_t launch_tv_bounds(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* len,
                            uint64_t* bound, hipStream_t s);
// per level: rules sorted into thread / small-wave / wave / workgroup merges
// (lists: 4 x level width, counters: 4 (depth + 2))
hipError_t launch_tv_tables(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, const uint64_t* toff,
                            uint32_t* tsize, uint32_t* pw, uint32_t* pc, int32_t* lists, int32_t* counts,
                            hipStream_t s);
hipError_t launch_tv_units(const DevGrammar& g, int64_t* units, hipStream_t s);
hipError_t launch_tv_count(const DevGrammar& g, const TvFiles& t, hipStream_t s);
hipError_t launch_tv_scatter(const DevGrammar& g, const TvFiles& t, uint64_t* entries, hipStream_t s);
hipError_t launch_tv_reduce(const DevGrammar& g, const TvFiles& t, uint64_t* entries, int64_t E, uint32_t* nnz,
                            int32_t* lists, int32_t* counts, hipStream_t s);
hipError_t launch_tv_emit(const DevGrammar& g, const TvFiles& t, const uint64_t* entries, int64_t E,
                          const uint32_t* nnz, const uint32_t* noff, uint32_t* out_word, uint64_t* out_cnt,
                          int64_t* out_off, hipStream_t s);
// Inverted index from a term vector (file-major, words ascending per file).
// With tv_cnt set, the ranked index: per word by term frequency descending,
// then file ascending, term frequencies in tf_out.
hipError_t launch_ii(const int64_t* tv_off, int64_t F, const uint32_t* tv_word, const uint64_t* tv_cnt, int64_t nnz,
                     int32_t V, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint64_t* kout,
                     uint32_t* file_out, const int64_t* num, uint32_t* hist, int64_t* ii_off, uint64_t* tf_out,
                     hipStream_t s);
hipError_t launch_scan_u64_ext(uint64_t* a, int64_t n, int64_t* total, uint64_t* sums, hipStream_t s);
hipError_t launch_scan_u32_ext(uint32_t* a, int64_t n, int64_t* total, uint32_t* sums, hipStream_t s);

// term vector by the top-down traversal: kTdGroup files at a time, each rule
// holding one uint64 weight per file of the group
constexpr int kTdGroup = 8;
hipError_t launch_td_root(const DevGrammar& g, int64_t f0, int32_t nf, uint64_t* w, hipStream_t s);
hipError_t launch_td_levels(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* w,
                            hipStream_t s);
hipError_t launch_td_column(const uint64_t* w, int64_t R, int f, uint64_t* out, hipStream_t s);
hipError_t launch_td_compact_count(const uint64_t* dense, int64_t n, uint32_t* blk, hipStream_t s);
hipError_t launch_td_compact_write(const uint64_t* dense, int64_t n, int32_t V, const uint32_t* blk_off, uint32_t* word,
                                   uint64_t* cnt, hipStream_t s);
hipError_t launch_td_row_off(const uint64_t* dense, int64_t F, int32_t V, int64_t* off, hipStream_t s);

// distinct (parent, child) rule pairs: per non-root rule its distinct
// sub-rules, plus the distinct sub-rules of the root (flags[R] scratch)
hipError_t launch_count_edges(const DevGrammar& g, int64_t root_syms, uint8_t* flags, unsigned long long* out,
                              hipStream_t s);

// decompression (text of the grammar on the device)
hipError_t launch_rule_lengths(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* len,
                               hipStream_t s);
hipError_t launch_sum_u64(const uint64_t* a, int64_t n, unsigned long long* out, hipStream_t s);
hipError_t launch_root_positions(const DevGrammar& g, const uint64_t* len, uint64_t* pos, int64_t nroot, uint64_t T,
                                 int64_t* file_out, uint64_t* sums, hipStream_t s);
hipError_t launch_expand_root(const DevGrammar& g, const uint64_t* pos, int64_t nroot, int32_t* tokens,
                              int32_t* out_rule, int64_t* out_off, unsigned long long* out_n, hipStream_t s);
hipError_t launch_expand_depth(const DevGrammar& g, const uint64_t* len, const int32_t* in_rule, const int64_t* in_off,
                               const unsigned long long* in_n, int64_t cap, int32_t* tokens, int32_t* out_rule,
                               int64_t* out_off, unsigned long long* out_n, hipStream_t s);

// sequence count with wide keys (any n <= 8; key = (hi, lo) 63-bit halves)
hipError_t launch_headtail_wide(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* len,
                                int32_t* head, int32_t* tail, hipStream_t s);
hipError_t launch_seq_windows_wide(const DevGrammar& g, int n, const uint64_t* len, const int32_t* head,
                                   const int32_t* tail, int b, uint64_t* table, uint64_t cap, uint32_t* overflow,
                                   hipStream_t s);
hipError_t launch_wocc_count(const uint64_t* table, int64_t cap, uint32_t* cnt, int64_t* total, uint32_t* sums,
                             hipStream_t s);
hipError_t launch_wide_sort(const uint64_t* table, int64_t cap, const uint32_t* off, const int64_t* num, int64_t U,
                            uint64_t lo_mask, uint64_t hi_mask, uint64_t* const* k, uint32_t* const* v,
                            uint32_t* hist, uint64_t* out_hi, uint64_t* out_lo, uint64_t* out_cnt, hipStream_t s);

// sequence count
hipError_t launch_headtail(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* len,
                           int32_t* head, int32_t* tail, hipStream_t s);
// the exact table interleaves key and count: 2 * cap uint64
hipError_t launch_seq_windows(const DevGrammar& g, int n, const uint64_t* len, const int32_t* head,
                              const int32_t* tail, uint64_t* table, uint64_t cap, uint32_t* overflow, hipStream_t s);
hipError_t launch_occ_count(const uint64_t* table, int64_t cap, uint32_t* cnt, int64_t* total, uint32_t* sums,
                            hipStream_t s);
hipError_t launch_occ_write(const uint64_t* table, int64_t cap, const uint32_t* off, uint64_t* okey, uint64_t* oval,
                            hipStream_t s);
hipError_t launch_sort_by_count(const uint64_t* counts, int32_t V, int key_bits, SortScratch& sc, uint32_t* ids_out,
                                uint64_t* cnt_out, int64_t* num_out, hipStream_t s);

}  // namespace gt

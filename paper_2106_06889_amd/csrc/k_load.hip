// k_load.hip -- initialization phase of a grammar on the GPU, up to the
// level walk: validation of offsets, ids and file spans, the tile table of
// the position-parallel passes, and the rule in-degrees and initial weights
// (frequencies in the root) by bucketed accumulation.
//
// Paper: Section "Overview" (initialization phase, then graph traversal);
// Algorithm "Top-Down Traversal", mask initialization (in-edges that do not
// come from the root; initial weights from the root). The level walk itself
// is in k_levels.hip.
#include "device.h"
#include "radix.h"

namespace gt {

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

static int fill_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_u64<<<fill_blocks(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_i32<<<fill_blocks(n), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

// Rule offsets: rule_off[0] = 0, rule_off[R] = S, non-decreasing, non-root
// bodies non-empty. Also records, for every tile whose first symbol lies in
// a non-root body, that body's rule (root tiles: k_root_tiles).
__global__ void k_check_rules(const int64_t* rule_off, int64_t R, int64_t S, int32_t* tile_rule, int64_t ntiles,
                              LoadCounters* lc) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r == 0) tile_rule[ntiles] = (int32_t)(R - 1);
  if (r >= R) return;
  const int64_t lo = rule_off[r], hi = rule_off[r + 1];
  uint32_t bad = 0;
  if (lo < 0 || hi > S || lo > hi) bad |= ST_BAD_OFFSETS;
  if (r == 0 && lo != 0) bad |= ST_BAD_OFFSETS;
  if (r == R - 1 && hi != S) bad |= ST_BAD_OFFSETS;
  if (r > 0 && hi == lo) bad |= ST_EMPTY_BODY;
  if (bad) {
    atomicOr(&lc->status, bad);
    return;
  }
  if (r == 0) {
    lc->root_syms = hi;
    return;
  }
  for (int64_t k = (lo + kTileSyms - 1) / kTileSyms; k * kTileSyms < hi; ++k) tile_rule[k] = (int32_t)r;
}

__global__ void k_root_tiles(const int64_t* rule_off, int32_t* tile_rule, int64_t ntiles) {
  const int64_t root_end = rule_off[1];
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ntiles; k += (int64_t)gridDim.x * blockDim.x)
    if (k * kTileSyms < root_end) tile_rule[k] = 0;
}

hipError_t launch_check_rules(const int64_t* rule_off, int64_t R, int64_t S, int32_t* tile_rule, int64_t ntiles,
                              LoadCounters* lc, hipStream_t s) {
  k_check_rules<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(rule_off, R, S, tile_rule, ntiles, lc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ntiles == 0) return e;
  k_root_tiles<<<fill_blocks(ntiles), 256, 0, s>>>(rule_off, tile_rule, ntiles);
  return hipGetLastError();
}

// The same checks in one launch, with the zero fills the dataflow load
// needs (one launch instead of eight keeps the GPU from waiting for the
// host at the start of a load): rule offsets and the tile table
// (k_check_rules, k_root_tiles), file spans (k_check_files), and zeros over
// the word counts of `z` (the offset histograms, the packed words, the
// walk's counters and chunk descriptors). lc must be zero before the launch.
__global__ __launch_bounds__(256) void k_load_prologue(const int64_t* rule_off, int64_t R, int64_t S,
                                                       const int64_t* file_off, int64_t F, int32_t* tile_rule,
                                                       int64_t ntiles, LoadCounters* lc, ZeroRanges z) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  uint32_t bad = 0;
  for (int64_t r = tid; r < R; r += nth) {
    const int64_t lo = rule_off[r], hi = rule_off[r + 1];
    uint32_t b = 0;
    if (lo < 0 || hi > S || lo > hi) b |= ST_BAD_OFFSETS;
    if (r == 0 && lo != 0) b |= ST_BAD_OFFSETS;
    if (r == R - 1 && hi != S) b |= ST_BAD_OFFSETS;
    if (r > 0 && hi == lo) b |= ST_EMPTY_BODY;
    bad |= b;
    if (b) continue;
    if (r == 0) {
      lc->root_syms = hi;
      continue;
    }
    for (int64_t k = (lo + kTileSyms - 1) / kTileSyms; k * kTileSyms < hi; ++k) tile_rule[k] = (int32_t)r;
  }
  const int64_t root_end = rule_off[1];
  for (int64_t k = tid; k < ntiles; k += nth)
    if (k * kTileSyms < root_end) tile_rule[k] = 0;
  if (tid == 0) tile_rule[ntiles] = (int32_t)(R - 1);
  for (int64_t f = tid; f < F; f += nth) {
    const int64_t a = file_off[f], b = file_off[f + 1];
    if (a > b || (f == 0 && a != 0) || (f == F - 1 && b != root_end)) bad |= ST_BAD_FILES;
  }
  for (int r = 0; r < z.count; ++r)
    for (int64_t i = tid; i < z.n[r]; i += nth) z.p[r][i] = 0;
  if (bad) atomicOr(&lc->status, bad);
}

hipError_t launch_load_prologue(const int64_t* rule_off, int64_t R, int64_t S, const int64_t* file_off, int64_t F,
                                int32_t* tile_rule, int64_t ntiles, LoadCounters* lc, const ZeroRanges& z,
                                hipStream_t s) {
  int64_t n = R > ntiles ? R : ntiles;
  if (F > n) n = F;
  for (int r = 0; r < z.count; ++r) n = z.n[r] > n ? z.n[r] : n;
  k_load_prologue<<<fill_blocks(n), 256, 0, s>>>(rule_off, R, S, file_off, F, tile_rule, ntiles, lc, z);
  return hipGetLastError();
}

// File spans tile the root body: file_off[0] = 0, non-decreasing,
// file_off[F] = length of the root body.
__global__ void k_check_files(const int64_t* file_off, int64_t F, const int64_t* rule_off, LoadCounters* lc) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= F) return;
  const int64_t a = file_off[f], b = file_off[f + 1];
  bool bad = a > b;
  if (f == 0 && a != 0) bad = true;
  if (f == F - 1 && b != rule_off[1]) bad = true;
  if (bad) atomicOr(&lc->status, (uint32_t)ST_BAD_FILES);
}

hipError_t launch_check_files(const int64_t* file_off, int64_t F, const int64_t* rule_off, LoadCounters* lc,
                              hipStream_t s) {
  k_check_files<<<(unsigned)((F + 255) / 256), 256, 0, s>>>(file_off, F, rule_off, lc);
  return hipGetLastError();
}

// Position-parallel scan of every body: symbol ranges and word totals, plus
// two per-block histograms that fix where later passes place their entries:
// word symbols per word bucket (wc_off) and rule references per rule bucket
// (rc_off). Each workgroup walks kSubTiles tiles. Dynamic LDS: the tile's
// rule offsets, then the two histograms. 1024 threads, 4 symbols (one
// 16-byte load) each per tile: four times the loads in flight of 256
// threads x 16, for the same tile table.
constexpr int kScanThreads = 1024;
constexpr int kScanPerThread = kTileSyms / kScanThreads;

__device__ __forceinline__ void load4(const DevGrammar& g, const Tile& t, int32_t q0, int32_t (&v)[kScanPerThread]) {
  if (q0 + kScanPerThread <= t.len) {
    const v4i32 x4 = __builtin_nontemporal_load(reinterpret_cast<const v4i32*>(g.sym + t.a + q0));
    v[0] = x4.x, v[1] = x4.y, v[2] = x4.z, v[3] = x4.w;
  } else {
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) v[k] = q0 + k < t.len ? g.sym[t.a + q0 + k] : 0;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_symbols(DevGrammar g, LoadCounters* lc) {
  // a plain load: the layout bits were set by earlier kernels, and a
  // device-scope load would queue behind the other blocks' counter atomics
  // on this line
  if (lc->status & kBadLayout) return;
  extern __shared__ int32_t lds_scan[];
  int32_t* roff = lds_scan;
  uint32_t* whist = reinterpret_cast<uint32_t*>(lds_scan + kTileRuleSlots);
  uint32_t* rhist = whist + g.wc_nb;
  const int wnb = g.wc_nb, rnb = g.rc_nb;
  for (int b = threadIdx.x; b < wnb + rnb; b += blockDim.x) whist[b] = 0;
  uint32_t bad = 0;
  uint64_t words = 0, root_words = 0;
  for (int sub = 0; sub < kSubTiles; ++sub) {
    const int64_t tile = (int64_t)blockIdx.x * kSubTiles + sub;
    if (tile >= g.ntiles) break;  // uniform for the block
    const Tile t = tile_begin(g, tile, roff);
    const int32_t q0 = threadIdx.x * kScanPerThread;
    if (q0 < t.len) {
      int32_t v[kScanPerThread];
      load4(g, t, q0, v);
      int32_t j = tile_find(roff, t.nr, q0);
      int32_t next = roff[j + 1];
#pragma unroll
      for (int k = 0; k < kScanPerThread; ++k) {
        const int32_t q = q0 + k;
        if (q >= t.len) continue;
        while (q >= next) next = roff[++j + 1];
        const int32_t r = t.r0 + j;
        const int32_t s = v[k];
        if (s >= 0) {
          if (s >= g.V) {
            bad |= ST_BAD_WORD;
          } else {
            ++words;
            root_words += (r == 0);
            if (wnb) atomicAdd(&whist[s >> kWcBits], 1u);
          }
        } else {
          const int64_t c = -(int64_t)s;
          if (c >= g.R) bad |= ST_BAD_REF;
          else if (rnb) atomicAdd(&rhist[c >> kRcBits], 1u);
          else if (r == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&g.w[c]), 1ull << kPendBits);
          else if ((atomicAdd(reinterpret_cast<unsigned long long*>(&g.w[c]), 1ull) & kPendMask) == kPendMask)
            bad |= ST_PACK;
        }
      }
    }
    __syncthreads();  // roff is rewritten by the next tile
  }
  const int64_t slot = xcd_slot(blockIdx.x, g.nslot);
  for (int b = threadIdx.x; b < wnb; b += blockDim.x) g.wc_off[(int64_t)b * g.nslot + slot] = whist[b];
  for (int b = threadIdx.x; b < rnb; b += blockDim.x) g.rc_off[(int64_t)b * g.nslot + slot] = rhist[b];
  // block totals, one atomic per block (per-wave atomics on one address serialize)
  __shared__ uint64_t wsum[2][kScanThreads / 64];
  words = wave_sum_u64(words);
  root_words = wave_sum_u64(root_words);
  if (lane_id() == 0) wsum[0][threadIdx.x >> 6] = words, wsum[1][threadIdx.x >> 6] = root_words;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t a = 0, b = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) a += wsum[0][w], b += wsum[1][w];
    if (a) atomicAdd(reinterpret_cast<unsigned long long*>(&lc->word_syms), (unsigned long long)a);
    if (b) atomicAdd(reinterpret_cast<unsigned long long*>(&lc->root_words), (unsigned long long)b);
  }
  if (bad) atomicOr(&lc->status, bad);
}

hipError_t launch_scan_symbols(const DevGrammar& g, LoadCounters* lc, hipStream_t s) {
  if (g.ntiles == 0) return hipSuccess;
  const size_t shmem = sizeof(int32_t) * (kTileRuleSlots + g.wc_nb + g.rc_nb);
  k_scan_symbols<<<(unsigned)g.nblk, kScanThreads, shmem, s>>>(g, lc);
  return hipGetLastError();
}

// In-degree scatter: one uint16 entry per rule reference into the bucket of
// its child, at the block's cursor (offsets from the scan above).
__global__ __launch_bounds__(kScanThreads) void k_ref_scatter(DevGrammar g, uint16_t* entries, const LoadCounters* lc) {
  if (lc->status & kBadLayout) return;
  extern __shared__ int32_t lds_ref[];
  int32_t* roff = lds_ref;
  uint32_t* cursor = reinterpret_cast<uint32_t*>(lds_ref + kTileRuleSlots);
  const int64_t slot = xcd_slot(blockIdx.x, g.nslot);
  for (int b = threadIdx.x; b < g.rc_nb; b += blockDim.x) cursor[b] = g.rc_off[(int64_t)b * g.nslot + slot];
  for (int sub = 0; sub < kSubTiles; ++sub) {
    const int64_t tile = (int64_t)blockIdx.x * kSubTiles + sub;
    if (tile >= g.ntiles) break;  // uniform for the block
    const Tile t = tile_begin(g, tile, roff);
    const int32_t q0 = threadIdx.x * kScanPerThread;
    if (q0 < t.len) {
      int32_t v[kScanPerThread];
      load4(g, t, q0, v);
      int32_t j = tile_find(roff, t.nr, q0);
      int32_t next = roff[j + 1];
#pragma unroll
      for (int k = 0; k < kScanPerThread; ++k) {
        const int32_t q = q0 + k;
        if (q >= t.len) continue;
        while (q >= next) next = roff[++j + 1];
        const int32_t s = v[k];
        const int64_t c64 = -(int64_t)s;
        if (s < 0 && c64 < g.R) {  // out-of-range ids were not counted; the grammar is rejected
          const uint32_t c = (uint32_t)c64;
          const uint32_t at = atomicAdd(&cursor[c >> kRcBits], 1u);
          entries[at] = (uint16_t)((c & (kRcBucket - 1)) | (t.r0 + j == 0 ? kRcRootFlag : 0));
        }
      }
    }
    __syncthreads();
  }
}

// In-degree reduce over fixed chunks of the entry array (bucket sizes are
// very uneven: preorder numbering gives the most used rules small ids).
// Occurrences in the root add to the initial weight (frequency in the root),
// the others to the count of pending in-edges; per bucket segment both are
// summed in LDS and added to the zeroed packed words with one coalesced
// atomic per rule (a field overflow sets ST_PACK). The
// most common key of each wave step is merged with one ballot first (every
// entry counts 1), which takes the bulk of the same-address LDS updates.
constexpr int kRcThreads = 1024;
constexpr int64_t kRcChunk = 32 * kRcThreads;

__global__ __launch_bounds__(kRcThreads) void k_ref_reduce(DevGrammar g, const uint16_t* entries, const int64_t* total,
                                                           LoadCounters* lc) {
  __shared__ uint32_t in_root[kRcBucket];
  __shared__ uint32_t in_rules[kRcBucket];
  __shared__ int first_bucket;
  if (blockIdx.x == 0 && threadIdx.x == 0) g.w[0] = 1;  // the root's weight (never packed: no in-edges)
  const int64_t n = *total;
  const int64_t c_lo = (int64_t)blockIdx.x * kRcChunk;
  if (c_lo >= n) return;  // uniform for the block
  const int64_t c_hi = c_lo + kRcChunk < n ? c_lo + kRcChunk : n;
  for (int i = threadIdx.x; i < kRcBucket; i += blockDim.x) in_root[i] = 0, in_rules[i] = 0;
  if (threadIdx.x == 0) {
    int lo = 0, hi = g.rc_nb - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((int64_t)g.rc_off[(int64_t)mid * g.nslot] <= c_lo) lo = mid;
      else hi = mid - 1;
    }
    first_bucket = lo;
  }
  __syncthreads();
  for (int b = first_bucket; b < g.rc_nb; ++b) {
    const int64_t b_lo = g.rc_off[(int64_t)b * g.nslot];
    const int64_t b_hi = (b + 1 < g.rc_nb) ? (int64_t)g.rc_off[(int64_t)(b + 1) * g.nslot] : n;
    if (b_lo >= c_hi) break;
    const int64_t lo = b_lo > c_lo ? b_lo : c_lo, hi = b_hi < c_hi ? b_hi : c_hi;
    for (int64_t i0 = lo; i0 < hi; i0 += blockDim.x) {  // uniform trip count: whole waves step together
      const int64_t i = i0 + threadIdx.x;
      const bool valid = i < hi;
      const uint32_t key = valid ? entries[i] : 0xffffffffu;
      const uint32_t key0 = __builtin_amdgcn_readfirstlane(key);
      const uint64_t same = __ballot(valid && key == key0);
      uint32_t add = 1;
      if (key == key0) add = (lane_id() == __ffsll((unsigned long long)same) - 1) ? (uint32_t)__popcll(same) : 0u;
      if (valid && add)
        atomicAdd((key & kRcRootFlag) ? &in_root[key & (kRcBucket - 1)] : &in_rules[key & (kRcBucket - 1)], add);
    }
    __syncthreads();
    const int64_t base = (int64_t)b * kRcBucket;
    for (int i = threadIdx.x; i < kRcBucket; i += blockDim.x) {
      const int64_t c = base + i;
      const uint32_t r = in_root[i], p = in_rules[i];
      in_root[i] = 0, in_rules[i] = 0;
      if (c >= g.R || (r | p) == 0) continue;
      const uint64_t old = atomicAdd(reinterpret_cast<unsigned long long*>(&g.w[c]),
                                     ((unsigned long long)r << kPendBits) + p);
      if ((old & kPendMask) + p > kPendMask || (old >> kPendBits) + r >= (1ull << kWeightBits))
        atomicOr(&lc->status, (uint32_t)ST_PACK);
    }
    __syncthreads();
  }
}

hipError_t launch_in_degrees(const DevGrammar& g, uint16_t* entries, const int64_t* n, LoadCounters* lc, hipStream_t s,
                             bool w_zeroed) {
  if (g.rc_nb == 0) return hipSuccess;  // counted with direct atomics by the scan
  if (!w_zeroed) {
    const hipError_t e0 = launch_fill_u64(g.w, g.R, 0, s);
    if (e0 != hipSuccess) return e0;
  }
  if (g.ntiles > 0) {
    const size_t shmem = sizeof(int32_t) * (kTileRuleSlots + g.rc_nb);
    k_ref_scatter<<<(unsigned)g.nblk, kScanThreads, shmem, s>>>(g, entries, lc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // at most S entries; chunks past the actual count exit at once
  const int64_t chunks = (g.S + kRcChunk - 1) / kRcChunk;
  if (chunks > 0) {
    k_ref_reduce<<<(unsigned)chunks, kRcThreads, 0, s>>>(g, entries, n, lc);  // also sets the root's weight
    return hipGetLastError();
  }
  k_fill_u64<<<1, 64, 0, s>>>(g.w, 1, 1);  // the root's weight (never packed: the root has no in-edges)
  return hipGetLastError();
}

// Unpacking after the level walk: every placed rule's pending field is zero,
// so its weight is the word shifted down (the root keeps its weight 1).
__global__ __launch_bounds__(256) void k_unpack_weights(uint64_t* w, int64_t R) {
  for (int64_t r = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x)
    w[r] >>= kPendBits;
}

hipError_t launch_unpack_weights(const DevGrammar& g, hipStream_t s) {
  if (g.R <= 1) return hipSuccess;
  const int64_t want = (g.R + 255) / 256;
  k_unpack_weights<<<(unsigned)(want < 8192 ? want : 8192), 256, 0, s>>>(g.w, g.R);
  return hipGetLastError();
}

// Scan of the word-bucket offsets (bucket-major), for the host.
hipError_t launch_scan_offsets(uint32_t* a, int64_t n, int64_t* total, uint32_t* sums, hipStream_t s) {
  return launch_scan_u32(a, n, total, sums, s);
}

// Both offset histograms of the load scanned in three launches instead of
// six: chunk sums of a (blocks [0, ca)) and b (blocks [ca, ca + cb)), one
// workgroup scanning each half of the sums from zero (totals to *ta, *tb),
// then every chunk rewritten with its offset.
struct Scan2 {
  uint32_t* a;
  int64_t na;
  uint32_t* b;
  int64_t nb;
  int64_t ca, cb;  // chunks of kRadixTile elements
};

__device__ __forceinline__ void scan2_chunk(const Scan2& q, uint32_t*& arr, int64_t& n, int64_t& chunk) {
  if ((int64_t)blockIdx.x < q.ca) arr = q.a, n = q.na, chunk = blockIdx.x;
  else arr = q.b, n = q.nb, chunk = blockIdx.x - q.ca;
}

// A chunk of kRadixTile entries is read as element i0 + k * 256 + thread
// (k < 16): the lanes of a wave read consecutive words.
__global__ __launch_bounds__(256) void k_scan2_sums(Scan2 q, uint32_t* sums) {
  uint32_t* arr;
  int64_t n, chunk;
  scan2_chunk(q, arr, n, chunk);
  const int64_t i0 = chunk * kRadixTile + threadIdx.x;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (i0 + k * 256 < n) c += arr[i0 + k * 256];
  __shared__ uint32_t lds[4];
  uint32_t total;
  block_exclusive_scan_256(c, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of a[0..n) in place by the whole (1024-thread) workgroup.
__device__ __forceinline__ void block_scan_inplace(uint32_t* a, int64_t n, int64_t* total, uint64_t* wsum) {
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = threadIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  uint64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += a[i];
  uint64_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o);
    if (lane_id() >= o) x += y;
  }
  if (lane_id() == 63) wsum[threadIdx.x >> 6] = x;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < (int)(threadIdx.x >> 6)) base += wsum[w];
    tot += wsum[w];
  }
  uint64_t run = base + x - s;
  for (int64_t i = lo; i < hi; ++i) {
    const uint32_t c = a[i];
    a[i] = (uint32_t)run;
    run += c;
  }
  if (threadIdx.x == 0 && total) *total = (int64_t)tot;
  __syncthreads();  // wsum is reused
}

__global__ __launch_bounds__(1024) void k_scan2_mid(uint32_t* sums, int64_t ca, int64_t cb, int64_t* ta, int64_t* tb) {
  __shared__ uint64_t wsum[16];
  block_scan_inplace(sums, ca, ta, wsum);
  block_scan_inplace(sums + ca, cb, tb, wsum);
}

// Element order within the chunk is (step k, wave, lane): each wave scans
// its 64 values of every step, then one wave scans the 64 (step, wave)
// totals, which places every value at its element-order prefix.
__global__ __launch_bounds__(256) void k_scan2_apply(Scan2 q, const uint32_t* sums) {
  uint32_t* arr;
  int64_t n, chunk;
  scan2_chunk(q, arr, n, chunk);
  const int64_t i0 = chunk * kRadixTile + threadIdx.x;
  const int wave = threadIdx.x >> 6, lane = lane_id();
  __shared__ uint32_t start[16][4];  // per (step, wave): total, then exclusive prefix
  uint32_t v[16], ex[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = (i0 + k * 256 < n) ? arr[i0 + k * 256] : 0u;
    uint32_t x = v[k];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    ex[k] = x - v[k];
    if (lane == 63) start[k][wave] = x;
  }
  __syncthreads();
  if (wave == 0) {
    const uint32_t t = start[lane >> 2][lane & 3];
    uint32_t x = t;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    start[lane >> 2][lane & 3] = sums[blockIdx.x] + x - t;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (i0 + k * 256 < n) arr[i0 + k * 256] = start[k][wave] + ex[k];
}

hipError_t launch_scan_offsets2(uint32_t* a, int64_t na, int64_t* ta, uint32_t* b, int64_t nb, int64_t* tb,
                                uint32_t* sums, hipStream_t s) {
  Scan2 q{a, na, b, nb, (na + kRadixTile - 1) / kRadixTile, (nb + kRadixTile - 1) / kRadixTile};
  if (q.ca + q.cb == 0) return hipSuccess;
  k_scan2_sums<<<(unsigned)(q.ca + q.cb), 256, 0, s>>>(q, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scan2_mid<<<1, 1024, 0, s>>>(sums, q.ca, q.cb, ta, tb);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scan2_apply<<<(unsigned)(q.ca + q.cb), 256, 0, s>>>(q, sums);
  return hipGetLastError();
}
int64_t scan2_scratch_entries(int64_t na, int64_t nb) {
  return (na + kRadixTile - 1) / kRadixTile + (nb + kRadixTile - 1) / kRadixTile + 1;
}
int64_t scan_scratch_entries(int64_t n) { return scan_sums_entries(n); }

}  // namespace gt

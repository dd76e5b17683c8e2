// k_seq.hip -- sequence count: occurrences of every run of n consecutive
// words (n = 2, 3, 4) inside one file, without decompressing.
//
// Paper: Section "Data Structures", head and tail structures (each rule keeps
// the first and last words of its expansion so that its parents can count
// the sequences that cross into it); Section "Sequence Support"
// (initialization phase fills head and tail buffers children first; graph
// traversal phase counts every rule's sequences into a shared hash table;
// the memory bound of the per-rule table, Eq. "upperLimit").
//
// Every length-n window of a file lies inside the expansion of exactly one
// deepest rule occurrence; that rule "owns" it. A rule's owned windows are
// the windows of its body that are not inside one child's expansion, and a
// window counts weight(rule) times. Here they are enumerated position by
// position: the piece at body position q (a word, or a child's expansion)
// starts the windows whose first word is among its last n-1 words and that
// run past its end; their remaining words come from the heads of the next
// pieces. Per rule this gives wordSize + (n-1) x subRuleSize - (n-1)
// windows whenever every child expands to at least n-1 words; for n = 4 a
// child of 2 words hands the window on to the pieces after it, and the
// count is below that bound.
//
// Differences from the paper's design: head/tail buffers are filled level by
// level from the deepest level (one launch per level) instead of a host loop
// that retries rules whose children are not ready; the shared table is
// lock-free open addressing (64-bit CAS on the key, 64-bit atomic add on the
// count) instead of per-entry locks with relaunch on contention; the result
// is compacted and radix-sorted by key.
#include "device.h"
#include "radix.h"

namespace gt {

constexpr uint64_t kEmptyKey = ~0ull;  // never a valid packed n-gram

// head[4r ..] = first min(len, kHT) words of exp(r), tail[4r ..] = last
// min(len, kHT) words in text order (unused entries -1; rows padded to 16
// bytes so a row is one vector load); len[r] = words in exp(r). kHT = 3
// serves every n <= 4. The rule's children (deeper levels) are done.
constexpr int kHT = 3;
constexpr int kHTRow = 4;

// The rule's length sums its pieces (a word, or a child's length) with the
// loads of 8 pieces in flight at a time; its first kHT words come from its
// first kHT pieces and its last kHT words from its last kHT pieces (every
// piece is at least one word), loaded together, so a rule costs a few
// dependent memory round trips instead of two per piece.
__device__ __forceinline__ void headtail_rule(const DevGrammar& g, int32_t r, uint64_t* len, int32_t* head,
                                              int32_t* tail) {
  constexpr int kBatch = 8;
  const int64_t a = g.rule_off[r], b = g.rule_off[r + 1];
  const int64_t np = b - a;
  int32_t fs[kHT], ls[kHT];  // first pieces in order; last pieces from the end
  v4i32 fr[kHT], lr[kHT];    // their head / tail rows (children only)
  uint64_t fl[kHT], ll[kHT];
#pragma unroll
  for (int k = 0; k < kHT; ++k) {
    fs[k] = k < np ? g.sym[a + k] : 0;
    ls[k] = k < np ? g.sym[b - 1 - k] : 0;
  }
#pragma unroll
  for (int k = 0; k < kHT; ++k) {
    fl[k] = 1, ll[k] = 1;
    if (k < np && fs[k] < 0) {
      const int64_t c = -(int64_t)fs[k];
      fl[k] = len[c];
      fr[k] = *reinterpret_cast<const v4i32*>(head + kHTRow * c);
    }
    if (k < np && ls[k] < 0) {
      const int64_t c = -(int64_t)ls[k];
      ll[k] = len[c];
      lr[k] = *reinterpret_cast<const v4i32*>(tail + kHTRow * c);
    }
  }
  uint64_t L = 0;
  for (int64_t q0 = a; q0 < b; q0 += kBatch) {
    int32_t sv[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) sv[k] = q0 + k < b ? g.sym[q0 + k] : 0;
    uint64_t lc[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) lc[k] = q0 + k >= b ? 0 : (sv[k] >= 0 ? 1 : len[-(int64_t)sv[k]]);
#pragma unroll
    for (int k = 0; k < kBatch; ++k) L += lc[k];
  }
  int32_t h[kHT] = {-1, -1, -1};
  int hc = 0;
#pragma unroll
  for (int k = 0; k < kHT; ++k) {
    if (k >= np) break;
    if (fs[k] >= 0) {
      if (hc < kHT) h[hc++] = fs[k];
    } else {
      const int take = fl[k] < kHT ? (int)fl[k] : kHT;
      const int32_t row[4] = {fr[k].x, fr[k].y, fr[k].z, fr[k].w};
      for (int j = 0; j < take && hc < kHT; ++j) h[hc++] = row[j];
    }
  }
  int32_t tr[kHT] = {-1, -1, -1};  // collected from the right: tr[0] is the last word
  int tc = 0;
#pragma unroll
  for (int k = 0; k < kHT; ++k) {
    if (k >= np) break;
    if (ls[k] >= 0) {
      if (tc < kHT) tr[tc++] = ls[k];
    } else {
      const int take = ll[k] < kHT ? (int)ll[k] : kHT;
      const int32_t row[4] = {lr[k].x, lr[k].y, lr[k].z, lr[k].w};
      for (int j = take - 1; j >= 0 && tc < kHT; --j) tr[tc++] = row[j];
    }
  }
  len[r] = L;
  v4i32 hv, tv;
  hv.x = h[0], hv.y = h[1], hv.z = h[2], hv.w = -1;
  tv.x = tc > 0 ? tr[tc - 1] : -1;
  tv.y = tc > 1 ? tr[tc - 2] : -1;
  tv.z = tc > 2 ? tr[tc - 3] : -1;
  tv.w = -1;
  *reinterpret_cast<v4i32*>(head + kHTRow * (int64_t)r) = hv;
  *reinterpret_cast<v4i32*>(tail + kHTRow * (int64_t)r) = tv;
}

// One level, a thread per rule.
__global__ void k_headtail_level(DevGrammar g, const int32_t* rules, int32_t n, uint64_t* len, int32_t* head,
                                 int32_t* tail) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) headtail_rule(g, rules[i], len, head, tail);
}

// A run of narrow levels, deepest (d_hi) first, in one workgroup: a
// workgroup barrier between levels instead of a launch per level (deep
// grammars end in long chains of levels of a few rules each).
constexpr int kHeadtailNarrowThreads = 1024;
__global__ __launch_bounds__(kHeadtailNarrowThreads) void k_headtail_narrow(DevGrammar g, int32_t d_lo, int32_t d_hi,
                                                                            uint64_t* len, int32_t* head,
                                                                            int32_t* tail) {
  for (int32_t d = d_hi; d >= d_lo; --d) {
    const int32_t lo = g.level_off[d], hi = g.level_off[d + 1];
    for (int32_t i = lo + (int32_t)threadIdx.x; i < hi; i += kHeadtailNarrowThreads)
      headtail_rule(g, g.level_rule[i], len, head, tail);
    __syncthreads();  // the next level reads what this one wrote
  }
}

hipError_t launch_headtail(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* len,
                           int32_t* head, int32_t* tail, hipStream_t s) {
  for (int32_t d = depth; d >= 1;) {
    const int32_t lo = level_off_host[d], hi = level_off_host[d + 1];
    if (hi - lo <= kHeadtailNarrowThreads) {
      int32_t d_lo = d;  // the run of narrow levels from d upwards
      while (d_lo > 1 && level_off_host[d_lo] - level_off_host[d_lo - 1] <= kHeadtailNarrowThreads) --d_lo;
      if (d_lo < d) {
        k_headtail_narrow<<<1, kHeadtailNarrowThreads, 0, s>>>(g, d_lo, d, len, head, tail);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        d = d_lo - 1;
        continue;
      }
    }
    if (hi > lo) {
      k_headtail_level<<<(unsigned)((hi - lo + 255) / 256), 256, 0, s>>>(g, g.level_rule + lo, hi - lo, len, head,
                                                                         tail);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    --d;
  }
  return hipSuccess;
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

// Lock-free insert-or-add: the first thread to CAS an empty slot owns it for
// that key; every occurrence then adds its weight to the slot's count.
// The table interleaves key and count: slot h is table[2h] (key) and
// table[2h + 1] (count), one cache line for both.
__device__ __forceinline__ void table_add(uint64_t* table, uint64_t mask, uint64_t key, uint64_t w,
                                          uint32_t* overflow) {
  uint64_t h = mix64(key) & mask;
  for (uint64_t p = 0; p <= mask; ++p) {
    uint64_t k = __hip_atomic_load(&table[2 * h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k == kEmptyKey) {
      k = atomicCAS(reinterpret_cast<unsigned long long*>(&table[2 * h]), (unsigned long long)kEmptyKey,
                    (unsigned long long)key);
      if (k == kEmptyKey) k = key;
    }
    if (k == key) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&table[2 * h + 1]), (unsigned long long)w);
      return;
    }
    h = (h + 1) & mask;
  }
  atomicOr(overflow, 1u);
}

__device__ __forceinline__ uint64_t pack_gram(const int32_t* x, int n) {
  if (n == 2) return (uint64_t)(uint32_t)x[0] << 32 | (uint32_t)x[1];
  if (n == 3) return (uint64_t)(uint32_t)x[0] << 42 | (uint64_t)(uint32_t)x[1] << 21 | (uint32_t)x[2];
  return (uint64_t)(uint32_t)x[0] << 48 | (uint64_t)(uint32_t)x[1] << 32 | (uint64_t)(uint32_t)x[2] << 16 |
         (uint32_t)x[3];
}

// Words of the piece at body position q: a word, or the first (head) / last
// (tail) min(len, m) words of a child's expansion, m = n - 1 <= kHT.
struct Piece {
  int32_t w[kHT];
  int cnt;
};

// A buffer row is loaded (one 16-byte load) without waiting for len[c],
// then the piece's words are picked in registers.
__device__ __forceinline__ int32_t pick3(const int32_t (&raw)[kHT], int i) {
  return i == 0 ? raw[0] : (i == 1 ? raw[1] : raw[2]);
}

__device__ __forceinline__ Piece piece_head(const uint64_t* len, const int32_t* head, int32_t s, int m) {
  Piece p;
  if (s >= 0) {
    p.w[0] = s, p.cnt = 1;
  } else {
    const int64_t c = -(int64_t)s;
    const v4i32 row = *reinterpret_cast<const v4i32*>(head + kHTRow * c);
    p.w[0] = row.x, p.w[1] = row.y, p.w[2] = row.z;
    const uint64_t lc = len[c];
    p.cnt = lc < (uint64_t)m ? (int)lc : m;
  }
  return p;
}

__device__ __forceinline__ Piece piece_tail(const uint64_t* len, const int32_t* tail, int32_t s, int m) {
  Piece p;
  if (s >= 0) {
    p.w[0] = s, p.cnt = 1;
  } else {
    const int64_t c = -(int64_t)s;
    const v4i32 row = *reinterpret_cast<const v4i32*>(tail + kHTRow * c);
    const int32_t raw[kHT] = {row.x, row.y, row.z};
    const uint64_t lc = len[c];
    const int k = lc < (uint64_t)kHT ? (int)lc : kHT;  // tail entries held
    p.cnt = lc < (uint64_t)m ? (int)lc : m;
#pragma unroll
    for (int x = 0; x < kHT; ++x) p.w[x] = pick3(raw, k - p.cnt + x);  // used for x < cnt only
  }
  return p;
}

// Two-level exact table: every workgroup first merges its windows in an LDS
// open-addressing table (key -> weight sum); a key that finds no slot within
// kSeqProbes probes goes straight to the global table, and at the end the
// LDS slots are flushed to the global table, one insert-or-add per distinct
// key of the tile instead of one per window.
constexpr int kSeqSlots = 2048;
constexpr int kSeqProbes = 8;

struct SeqLds {
  int32_t roff[kTileRuleSlots];
  uint64_t key[kSeqSlots];
  uint64_t val[kSeqSlots];
};

__device__ __forceinline__ void seq_add(SeqLds& L, uint64_t* table, uint64_t mask, uint64_t key,
                                        uint64_t w, uint32_t* overflow) {
  const uint32_t h = (uint32_t)(mix64(key) >> 40) & (kSeqSlots - 1);
#pragma unroll
  for (int p = 0; p < kSeqProbes; ++p) {
    const uint32_t slot = (h + p) & (kSeqSlots - 1);
    uint64_t k = __hip_atomic_load(&L.key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == kEmptyKey)
      k = atomicCAS(reinterpret_cast<unsigned long long*>(&L.key[slot]), (unsigned long long)kEmptyKey,
                    (unsigned long long)key);
    if (k == kEmptyKey || k == key) {
      atomicAdd(reinterpret_cast<unsigned long long*>(&L.val[slot]), (unsigned long long)w);
      return;
    }
  }
  table_add(table, mask, key, w, overflow);
}

// Owned windows, position-parallel over the tiles of all bodies. The root is
// split at file boundaries: windows never cross files.
template <int n>
__global__ __launch_bounds__(kTileThreads) void k_seq_windows(DevGrammar g, const uint64_t* len, const int32_t* head,
                                                              const int32_t* tail, uint64_t* table, uint64_t mask,
                                                              uint32_t* overflow) {
  __shared__ SeqLds L;
  for (int x = threadIdx.x; x < kSeqSlots; x += blockDim.x) L.key[x] = kEmptyKey, L.val[x] = 0;
  const Tile t = tile_begin(g, blockIdx.x, L.roff);  // (synchronizes)
  const int32_t q0 = threadIdx.x * kPerThread;
  if (q0 < t.len) {
    int32_t v[kPerThread];
    tile_load_syms(g, t, q0, v);
    int32_t j = tile_find(L.roff, t.nr, q0);
    int32_t next = L.roff[j + 1];
    int64_t f = -1, f_end = 0;  // file span of the current root position
    for (int k = 0; k < kPerThread; ++k) {
      const int32_t qt = q0 + k;
      if (qt >= t.len) break;
      while (qt >= next) next = L.roff[++j + 1];
      const int32_t r = t.r0 + j;
      const int64_t q = t.a + qt;
      int64_t end;
      uint64_t wt;
      if (r == 0) {
        if (q >= f_end) {  // locate the file span holding q (binary search on file_off)
          int64_t lo = 0, hi = g.F - 1;
          while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (g.file_off[mid] <= q) lo = mid;
            else hi = mid - 1;
          }
          f = lo;
          f_end = g.file_off[f + 1];
        }
        end = f_end;
        wt = 1;
      } else {
        end = g.rule_off[r + 1];
        wt = g.w[r];
      }
      if (wt == 0) continue;
      const Piece st = piece_tail(len, tail, v[k], n - 1);
      const int starts = st.cnt < n - 1 ? st.cnt : n - 1;
      // words after the piece: heads of the next pieces, at most n-1 of them
      int32_t ahead[n - 1];
      int na = 0;
      for (int64_t q2 = q + 1; q2 < end && na < n - 1; ++q2) {
        const int32_t kk = k + (int32_t)(q2 - q);
        const Piece p = piece_head(len, head, (kk < kPerThread && q0 + kk < t.len) ? v[kk] : g.sym[q2], n - 1);
        for (int x = 0; x < p.cnt && na < n - 1; ++x) ahead[na++] = p.w[x];
      }
      for (int s0 = st.cnt - starts; s0 < st.cnt; ++s0) {
        int32_t win[n];
        int wn = 0;
        for (int x = s0; x < st.cnt && wn < n; ++x) win[wn++] = st.w[x];
        for (int x = 0; x < na && wn < n; ++x) win[wn++] = ahead[x];
        if (wn == n) seq_add(L, table, mask, pack_gram(win, n), wt, overflow);
      }
    }
  }
  __syncthreads();
  for (int x = threadIdx.x; x < kSeqSlots; x += blockDim.x)
    if (L.key[x] != kEmptyKey) table_add(table, mask, L.key[x], L.val[x], overflow);
}

__global__ void k_fill_table(uint64_t* table, int64_t cap) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
    table[2 * i] = kEmptyKey;
    table[2 * i + 1] = 0;
  }
}

hipError_t launch_seq_windows(const DevGrammar& g, int n, const uint64_t* len, const int32_t* head,
                              const int32_t* tail, uint64_t* table, uint64_t cap, uint32_t* overflow, hipStream_t s) {
  const int64_t fb = (int64_t)((cap + 255) / 256);
  k_fill_table<<<(unsigned)(fb < 8192 ? fb : 8192), 256, 0, s>>>(table, (int64_t)cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.ntiles == 0) return e;
  const unsigned grid = (unsigned)g.ntiles;
  if (n == 2) k_seq_windows<2><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, table, cap - 1, overflow);
  else if (n == 3) k_seq_windows<3><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, table, cap - 1, overflow);
  else k_seq_windows<4><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, table, cap - 1, overflow);
  return hipGetLastError();
}

// Compaction of the occupied slots (any order: a radix sort follows). Slot
// i0 + k * 256 + thread for k < 16: the lanes of a wave read consecutive
// slots, one line per 8 lanes.
__global__ __launch_bounds__(256) void k_occ_count(const uint64_t* table, int64_t cap, uint32_t* cnt) {
  const int64_t i0 = (int64_t)blockIdx.x * kRadixTile + threadIdx.x;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < cap && __builtin_nontemporal_load(table + 2 * i) != kEmptyKey) ++c;
  }
  __shared__ uint32_t lds[4];
  uint32_t total;
  block_exclusive_scan_256(c, lds, &total);
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// The block's output is ordered by (step k, wave, lane), so the occupied
// lanes of one wave step write consecutive positions.
typedef uint64_t v2u64 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void k_occ_write(const uint64_t* table, int64_t cap, const uint32_t* off,
                                                   uint64_t* okey, uint64_t* oval) {
  const int64_t i0 = (int64_t)blockIdx.x * kRadixTile + threadIdx.x;
  const int wave = threadIdx.x >> 6, lane = lane_id();
  __shared__ uint32_t start[16][4];  // per (step, wave): count, then first output position
  v2u64 kv[16];
  uint64_t occ[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t i = i0 + k * 256;
    kv[k] = i < cap ? __builtin_nontemporal_load(reinterpret_cast<const v2u64*>(table) + i) : v2u64{kEmptyKey, 0};
    occ[k] = __ballot(kv[k].x != kEmptyKey);
    if (lane == 0) start[k][wave] = (uint32_t)__popcll(occ[k]);
  }
  __syncthreads();
  if (wave == 0) {  // exclusive scan of the 64 counts in (k, wave) order
    const uint32_t v = start[lane >> 2][lane & 3];
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    start[lane >> 2][lane & 3] = off[blockIdx.x] + x - v;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (kv[k].x != kEmptyKey) {
      const uint32_t pos = start[k][wave] + (uint32_t)__popcll(occ[k] & lanes_below());
      okey[pos] = kv[k].x;
      oval[pos] = kv[k].y;
    }
}

hipError_t launch_occ_count(const uint64_t* table, int64_t cap, uint32_t* cnt, int64_t* total, uint32_t* sums,
                            hipStream_t s) {
  const int64_t nb = (cap + kRadixTile - 1) / kRadixTile;
  k_occ_count<<<(unsigned)nb, 256, 0, s>>>(table, cap, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scan_u32(cnt, nb, total, sums, s);
}

hipError_t launch_occ_write(const uint64_t* table, int64_t cap, const uint32_t* off, uint64_t* okey, uint64_t* oval,
                            hipStream_t s) {
  const int64_t nb = (cap + kRadixTile - 1) / kRadixTile;
  k_occ_write<<<(unsigned)nb, 256, 0, s>>>(table, cap, off, okey, oval);
  return hipGetLastError();
}


}  // namespace gt

// k_seq_wide.hip -- sequence count for any n up to 8 with wide keys: n-grams
// whose packed form needs more than 64 bits (long n, or vocabularies too
// large for 16-bit fields at n = 4).
//
// Paper: Section "Sequence Support" (sequences of a general length: head and
// tail buffers of the first and last words of every rule, filled children
// first, let a parent count the sequences that cross into its children;
// every rule counts its own sequences into a shared table). The windows a
// rule owns are enumerated as in k_seq.hip; here the buffers hold up to 7
// words (rows of 8) and the key is the big-endian packing of the n words,
// b = bits(vocab - 1) each, into at most 126 bits, kept as two 63-bit halves
// (hi, lo) so that ascending (hi, lo) is lexicographic n-gram order.
//
// The exact table has 128-bit keys, but the GPU's atomics are 64-bit: a slot
// is claimed by a CAS of hi into its first word; the claimer then stores lo
// into the second; a thread that finds its hi in a slot waits until the
// slot's lo is written (each word is written once, so a relaxed load that
// sees a written value sees the final one) and compares it. Because both
// halves have a zero top bit, all-ones marks an unwritten word. The claim and
// the wait are two consecutive branch regions, so in a wave the claiming lane
// always stores before any lane of the same wave waits.
#include "device.h"
#include "radix.h"

namespace gt {

constexpr int kWHT = 7;       // head/tail words kept per rule (n - 1 <= 7)
constexpr int kWRow = 8;      // row stride (32 bytes)
constexpr uint64_t kWEmpty = ~0ull;

// Length with the loads of 8 pieces in flight at a time; the first (last)
// kWHT words come from the first (last) kWHT pieces, loaded together.
__device__ __forceinline__ void headtail_wide_rule(const DevGrammar& g, int32_t r, uint64_t* len, int32_t* head,
                                                   int32_t* tail) {
  constexpr int kBatch = 8;
  const int64_t a = g.rule_off[r], b = g.rule_off[r + 1];
  const int64_t np = b - a;
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
  int32_t h[kWRow];
  for (int x = 0; x < kWRow; ++x) h[x] = -1;
  int hc = 0;
  {
    int32_t ps[kWHT];
    uint64_t pl[kWHT];
#pragma unroll
    for (int k = 0; k < kWHT; ++k) ps[k] = k < np ? g.sym[a + k] : 0;
#pragma unroll
    for (int k = 0; k < kWHT; ++k) pl[k] = k < np && ps[k] < 0 ? len[-(int64_t)ps[k]] : 1;
    for (int k = 0; k < kWHT && k < np && hc < kWHT; ++k) {
      if (ps[k] >= 0) {
        h[hc++] = ps[k];
      } else {
        const int64_t c = -(int64_t)ps[k];
        const int take = pl[k] < kWHT ? (int)pl[k] : kWHT;
        for (int j = 0; j < take && hc < kWHT; ++j) h[hc++] = head[kWRow * c + j];
      }
    }
  }
  int32_t tr[kWHT];  // collected from the right: tr[0] is the last word
  int tc = 0;
  {
    int32_t ps[kWHT];
    uint64_t pl[kWHT];
#pragma unroll
    for (int k = 0; k < kWHT; ++k) ps[k] = k < np ? g.sym[b - 1 - k] : 0;
#pragma unroll
    for (int k = 0; k < kWHT; ++k) pl[k] = k < np && ps[k] < 0 ? len[-(int64_t)ps[k]] : 1;
    for (int k = 0; k < kWHT && k < np && tc < kWHT; ++k) {
      if (ps[k] >= 0) {
        tr[tc++] = ps[k];
      } else {
        const int64_t c = -(int64_t)ps[k];
        const int take = pl[k] < kWHT ? (int)pl[k] : kWHT;
        for (int j = take - 1; j >= 0 && tc < kWHT; --j) tr[tc++] = tail[kWRow * c + j];
      }
    }
  }
  len[r] = L;
  int32_t* hr = head + kWRow * (int64_t)r;
  int32_t* trow = tail + kWRow * (int64_t)r;
  for (int x = 0; x < kWRow; ++x) {
    hr[x] = h[x];
    trow[x] = x < tc ? tr[tc - 1 - x] : -1;
  }
}

// One level, a thread per rule; its children (deeper levels) are done.
__global__ void k_headtail_wide_level(DevGrammar g, const int32_t* rules, int32_t n, uint64_t* len, int32_t* head,
                                      int32_t* tail) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) headtail_wide_rule(g, rules[i], len, head, tail);
}

// A run of narrow levels, deepest (d_hi) first, in one workgroup with a
// workgroup barrier between levels instead of a launch per level.
constexpr int kWideNarrowThreads = 1024;
__global__ __launch_bounds__(kWideNarrowThreads) void k_headtail_wide_narrow(DevGrammar g, int32_t d_lo, int32_t d_hi,
                                                                             uint64_t* len, int32_t* head,
                                                                             int32_t* tail) {
  for (int32_t d = d_hi; d >= d_lo; --d) {
    const int32_t lo = g.level_off[d], hi = g.level_off[d + 1];
    for (int32_t i = lo + (int32_t)threadIdx.x; i < hi; i += kWideNarrowThreads)
      headtail_wide_rule(g, g.level_rule[i], len, head, tail);
    __syncthreads();  // the next level reads what this one wrote
  }
}

hipError_t launch_headtail_wide(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* len,
                                int32_t* head, int32_t* tail, hipStream_t s) {
  for (int32_t d = depth; d >= 1;) {
    const int32_t lo = level_off_host[d], hi = level_off_host[d + 1];
    if (hi - lo <= kWideNarrowThreads) {
      int32_t d_lo = d;  // the run of narrow levels from d upwards
      while (d_lo > 1 && level_off_host[d_lo] - level_off_host[d_lo - 1] <= kWideNarrowThreads) --d_lo;
      if (d_lo < d) {
        k_headtail_wide_narrow<<<1, kWideNarrowThreads, 0, s>>>(g, d_lo, d, len, head, tail);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        d = d_lo - 1;
        continue;
      }
    }
    if (hi > lo) {
      k_headtail_wide_level<<<(unsigned)((hi - lo + 255) / 256), 256, 0, s>>>(g, g.level_rule + lo, hi - lo, len,
                                                                             head, tail);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    --d;
  }
  return hipSuccess;
}

__device__ __forceinline__ uint64_t mix64w(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

// Insert-or-add of a 128-bit key; slot h is table[4h .. 4h+3] = hi, lo, count, unused.
__device__ __forceinline__ void wide_add(uint64_t* table, uint64_t mask, uint64_t hi, uint64_t lo, uint64_t w,
                                         uint32_t* overflow) {
  uint64_t h = mix64w(hi * 0x9E3779B97F4A7C15ull ^ lo) & mask;
  for (uint64_t p = 0; p <= mask; ++p) {
    uint64_t* sl = table + 4 * h;
    uint64_t k = __hip_atomic_load(&sl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool mine = false;
    if (k == kWEmpty) {
      k = atomicCAS(reinterpret_cast<unsigned long long*>(&sl[0]), (unsigned long long)kWEmpty, (unsigned long long)hi);
      mine = k == kWEmpty;
      if (mine) k = hi;
    }
    if (mine) __hip_atomic_store(&sl[1], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k == hi) {
      uint64_t l;
      while ((l = __hip_atomic_load(&sl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == kWEmpty)
        __builtin_amdgcn_s_sleep(1);
      if (l == lo) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&sl[2]), (unsigned long long)w);
        return;
      }
    }
    h = (h + 1) & mask;
  }
  atomicOr(overflow, 1u);
}

// The first (head) or last (tail) min(len, m) words of the piece at a body
// position: a word, or a child's buffer row.
struct WPiece {
  int32_t w[kWHT];
  int cnt;
};

__device__ __forceinline__ WPiece wpiece_head(const uint64_t* len, const int32_t* head, int32_t s, int m) {
  WPiece p;
  if (s >= 0) {
    p.w[0] = s, p.cnt = 1;
    return p;
  }
  const int64_t c = -(int64_t)s;
  const uint64_t lc = len[c];
  p.cnt = lc < (uint64_t)m ? (int)lc : m;
  for (int x = 0; x < kWHT; ++x) p.w[x] = x < p.cnt ? head[kWRow * c + x] : -1;
  return p;
}

__device__ __forceinline__ WPiece wpiece_tail(const uint64_t* len, const int32_t* tail, int32_t s, int m) {
  WPiece p;
  if (s >= 0) {
    p.w[0] = s, p.cnt = 1;
    return p;
  }
  const int64_t c = -(int64_t)s;
  const uint64_t lc = len[c];
  const int k = lc < (uint64_t)kWHT ? (int)lc : kWHT;  // tail entries held
  p.cnt = lc < (uint64_t)m ? (int)lc : m;
  for (int x = 0; x < kWHT; ++x) p.w[x] = x < p.cnt ? tail[kWRow * c + k - p.cnt + x] : -1;
  return p;
}

__device__ __forceinline__ void pack_wide_key(const int32_t* win, int n, int b, uint64_t* hi, uint64_t* lo) {
  const uint64_t m63 = (1ull << 63) - 1;
  uint64_t h = 0, l = 0;
  for (int i = 0; i < n; ++i) {
    h = ((h << b) | (l >> (63 - b))) & m63;
    l = ((l << b) | (uint32_t)win[i]) & m63;
  }
  *hi = h, *lo = l;
}

// Owned windows, one thread per body position (tiles of all bodies, root
// split at file boundaries), straight into the global table.
template <int n>
__global__ __launch_bounds__(kTileThreads) void k_seq_windows_wide(DevGrammar g, const uint64_t* len,
                                                                   const int32_t* head, const int32_t* tail, int b,
                                                                   uint64_t* table, uint64_t mask, uint32_t* overflow) {
  __shared__ int32_t roff[kTileRuleSlots];
  const Tile t = tile_begin(g, blockIdx.x, roff);
  const int32_t q0 = threadIdx.x * kPerThread;
  if (q0 >= t.len) return;
  int32_t j = tile_find(roff, t.nr, q0);
  int32_t next = roff[j + 1];
  int64_t f_end = 0;
  for (int k = 0; k < kPerThread; ++k) {
    const int32_t qt = q0 + k;
    if (qt >= t.len) break;
    while (qt >= next) next = roff[++j + 1];
    const int32_t r = t.r0 + j;
    const int64_t q = t.a + qt;
    int64_t end;
    uint64_t wt;
    if (r == 0) {
      if (q >= f_end) {  // the file span holding q (binary search on file_off)
        int64_t lo = 0, hi = g.F - 1;
        while (lo < hi) {
          const int64_t mid = (lo + hi + 1) >> 1;
          if (g.file_off[mid] <= q) lo = mid;
          else hi = mid - 1;
        }
        f_end = g.file_off[lo + 1];
      }
      end = f_end;
      wt = 1;
    } else {
      end = g.rule_off[r + 1];
      wt = g.w[r];
    }
    if (wt == 0) continue;
    const WPiece st = wpiece_tail(len, tail, g.sym[q], n - 1);
    const int starts = st.cnt < n - 1 ? st.cnt : n - 1;
    int32_t ahead[n - 1];
    int na = 0;
    for (int64_t q2 = q + 1; q2 < end && na < n - 1; ++q2) {
      const WPiece p = wpiece_head(len, head, g.sym[q2], n - 1);
      for (int x = 0; x < p.cnt && na < n - 1; ++x) ahead[na++] = p.w[x];
    }
    for (int s0 = st.cnt - starts; s0 < st.cnt; ++s0) {
      int32_t win[n];
      int wn = 0;
      for (int x = s0; x < st.cnt && wn < n; ++x) win[wn++] = st.w[x];
      for (int x = 0; x < na && wn < n; ++x) win[wn++] = ahead[x];
      if (wn == n) {
        uint64_t hk, lk;
        pack_wide_key(win, n, b, &hk, &lk);
        wide_add(table, mask, hk, lk, wt, overflow);
      }
    }
  }
}

__global__ void k_fill_wide(uint64_t* table, int64_t cap) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
    table[4 * i] = kWEmpty;
    table[4 * i + 1] = kWEmpty;
    table[4 * i + 2] = 0;
    table[4 * i + 3] = 0;
  }
}

hipError_t launch_seq_windows_wide(const DevGrammar& g, int n, const uint64_t* len, const int32_t* head,
                                   const int32_t* tail, int b, uint64_t* table, uint64_t cap, uint32_t* overflow,
                                   hipStream_t s) {
  const int64_t fb = (int64_t)((cap + 255) / 256);
  k_fill_wide<<<(unsigned)(fb < 8192 ? fb : 8192), 256, 0, s>>>(table, (int64_t)cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.ntiles == 0) return e;
  const unsigned grid = (unsigned)g.ntiles;
  const uint64_t mask = cap - 1;
  switch (n) {
    case 2: k_seq_windows_wide<2><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, b, table, mask, overflow); break;
    case 3: k_seq_windows_wide<3><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, b, table, mask, overflow); break;
    case 4: k_seq_windows_wide<4><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, b, table, mask, overflow); break;
    case 5: k_seq_windows_wide<5><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, b, table, mask, overflow); break;
    case 6: k_seq_windows_wide<6><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, b, table, mask, overflow); break;
    case 7: k_seq_windows_wide<7><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, b, table, mask, overflow); break;
    default: k_seq_windows_wide<8><<<grid, kTileThreads, 0, s>>>(g, len, head, tail, b, table, mask, overflow); break;
  }
  return hipGetLastError();
}

// Occupied slots: a count per 4096-slot block, then the (lo, slot) pairs of
// the occupied slots at their compacted positions (slot order).
__global__ __launch_bounds__(256) void k_wocc_count(const uint64_t* table, int64_t cap, uint32_t* cnt) {
  const int64_t i0 = (int64_t)blockIdx.x * kRadixTile + threadIdx.x;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < cap && table[4 * i] != kWEmpty) ++c;
  }
  __shared__ uint32_t lds[4];
  uint32_t total;
  block_exclusive_scan_256(c, lds, &total);
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_wocc_write(const uint64_t* table, int64_t cap, const uint32_t* off,
                                                    uint64_t* key, uint32_t* slot) {
  const int64_t i0 = (int64_t)blockIdx.x * kRadixTile + threadIdx.x;
  bool occ[16];
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t i = i0 + k * 256;
    occ[k] = i < cap && table[4 * i] != kWEmpty;
    c += occ[k];
  }
  __shared__ uint32_t lds[4];
  uint32_t total;
  uint32_t pos = off[blockIdx.x] + block_exclusive_scan_256(c, lds, &total);
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (occ[k]) {
      const int64_t i = i0 + k * 256;
      key[pos] = table[4 * i + 1];  // lo first: the least significant sort key
      slot[pos] = (uint32_t)i;
      ++pos;
    }
}

// key[i] = hi of slot[i] (the second sort key), after the sort by lo.
__global__ __launch_bounds__(256) void k_wgather_hi(const uint64_t* table, const uint32_t* slot, const int64_t* num,
                                                    uint64_t* key) {
  const int64_t U = *num;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < U; i += (int64_t)gridDim.x * blockDim.x)
    key[i] = table[4 * (int64_t)slot[i]];
}

// The result in (hi, lo) order from the final slot permutation.
__global__ __launch_bounds__(256) void k_wgather_out(const uint64_t* table, const uint32_t* slot, const int64_t* num,
                                                     uint64_t* hi, uint64_t* lo, uint64_t* cnt) {
  const int64_t U = *num;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < U; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t* sl = table + 4 * (int64_t)slot[i];
    hi[i] = sl[0];
    lo[i] = sl[1];
    cnt[i] = sl[2];
  }
}

hipError_t launch_wocc_count(const uint64_t* table, int64_t cap, uint32_t* cnt, int64_t* total, uint32_t* sums,
                             hipStream_t s) {
  const int64_t nb = (cap + kRadixTile - 1) / kRadixTile;
  k_wocc_count<<<(unsigned)nb, 256, 0, s>>>(table, cap, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scan_u32(cnt, nb, total, sums, s);
}

// Sorts the occupied slots by (hi, lo): a stable radix sort of (lo, slot) by
// lo, then of (hi, slot) by hi, then gathers the result. The radix sort uses
// its input and scratch arrays as ping-pong buffers, so every sort writes to
// an array that is neither: k[0..2], v[0..2] hold U entries each.
hipError_t launch_wide_sort(const uint64_t* table, int64_t cap, const uint32_t* off, const int64_t* num, int64_t U,
                            uint64_t lo_mask, uint64_t hi_mask, uint64_t* const* k, uint32_t* const* v,
                            uint32_t* hist, uint64_t* out_hi, uint64_t* out_lo, uint64_t* out_cnt, hipStream_t s) {
  const int64_t nb = (cap + kRadixTile - 1) / kRadixTile;
  k_wocc_write<<<(unsigned)nb, 256, 0, s>>>(table, cap, off, k[0], v[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = radix_sort_pairs_bytes<uint32_t>(k[0], v[0], k[1], v[1], num, U, lo_mask, false, hist, k[2], v[2], s);
  if (e != hipSuccess) return e;
  const int64_t gb = (U + 255) / 256;
  const unsigned grid = (unsigned)(gb < 4096 ? (gb > 0 ? gb : 1) : 4096);
  k_wgather_hi<<<grid, 256, 0, s>>>(table, v[2], num, k[0]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = radix_sort_pairs_bytes<uint32_t>(k[0], v[2], k[1], v[1], num, U, hi_mask, false, hist, k[2], v[0], s);
  if (e != hipSuccess) return e;
  k_wgather_out<<<grid, 256, 0, s>>>(table, v[0], num, out_hi, out_lo, out_cnt);
  return hipGetLastError();
}

}  // namespace gt

// k_tv.hip -- term vector and inverted index by bottom-up traversal.
//
// Paper: Section "Fine-Grained Thread-Level Execution Engine", bottom-up
// traversal (Algorithm "Bottom-Up Traversal"): a light bottom-up pass bounds
// every rule's local table (own words plus its children's bounds), the
// tables are allocated from the memory pool at those bounds (Section "Data
// Structures", memory pool), a second bottom-up pass fills each rule's table
// from its own words and its children's tables, and the result is reduced
// from the root's words and the tables of the root's children (the
// "level-2 nodes"), file by file since the root holds the file information.
//
// MI355X design:
//  - Bounds and tables are built level by level from the deepest level (one
//    launch per level; a rule's children are all deeper). The bound pass is a
//    bump allocation: one exclusive scan of the bounds gives every table its
//    offset in the pool. A table is the rule's word counts sorted by word,
//    produced by a merge of the children's sorted tables and its own words.
//  - The per-file reduce avoids global atomics: every file's inputs (its root
//    words, and one entry per table entry of each root child) are grouped by
//    (file, word bucket of 4096 ids) at offsets fixed by a counting pass, and
//    each group is summed in a dense LDS table whose nonzero slots come out in
//    word order -- the term vector rows are sorted without a sort.
//  - The inverted index is the stable transpose: a radix sort of the term
//    vector's (word, file) pairs by word keeps files ascending.
#include "device.h"
#include "radix.h"

namespace gt {

// Expansion length and table bound of the rules of one level (children done):
// len(r) = words of exp(r); bound(r) = min(len(r), V, own words + sum of the
// children's bounds), an upper bound on the distinct words of exp(r).
__global__ void k_tv_bound_level(DevGrammar g, const int32_t* rules, int32_t n, uint64_t* len, uint64_t* bound) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t r = rules[i];
  uint64_t L = 0, B = 0;
  const int64_t a = g.rule_off[r], b = g.rule_off[r + 1];
  for (int64_t q0 = a; q0 < b; q0 += 8) {  // 8 symbols, then their children's figures, in flight together
    int32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = q0 + k < b ? g.sym[q0 + k] : 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (q0 + k >= b) continue;
      if (v[k] >= 0) {
        ++L, ++B;
      } else {
        L += len[-v[k]];
        B += bound[-v[k]];
      }
    }
  }
  if (B > L) B = L;
  if (B > (uint64_t)g.V) B = (uint64_t)g.V;
  len[r] = L;
  bound[r] = B;
}

hipError_t launch_tv_bounds(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* len,
                            uint64_t* bound, hipStream_t s) {
  for (int32_t d = depth; d >= 1; --d) {
    const int32_t lo = level_off_host[d], hi = level_off_host[d + 1];
    if (hi <= lo) continue;
    k_tv_bound_level<<<(unsigned)((hi - lo + 255) / 256), 256, 0, s>>>(g, g.level_rule + lo, hi - lo, len, bound);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Table of rule r = the merge of its pieces (own words, each counting 1, and
// the sorted tables of its children, once per occurrence), in word order.
// The merge of one rule is spread over a wave or a workgroup, never one
// thread: a serial merge costs one dependent load per output entry, which is
// milliseconds for the large tables near the top of the DAG. Per level, a
// classification pass counts each rule's merge inputs n_in (own words plus
// its children's table sizes) and sorts the rules into three lists:
//  - n_in <= kTvThreadMax (most rules): one thread gathers the inputs into
//    registers and sorts them with a fixed compare-exchange network;
//  - n_in <= kTvWaveMax: one wave per rule gathers the inputs into LDS
//    (a 2 KB buffer per wave up to kTvWaveSmall inputs, 16 KB above),
//    bitonic-sorts them by word, and writes one entry per distinct word with
//    the summed count;
//  - larger: one workgroup per rule walks the word space in windows of 4096
//    ids; each piece keeps a cursor, the window's inputs of every piece are
//    summed in a dense LDS table, and its nonzero slots come out in order.
constexpr int kTvThreadMax = 16;   // inputs merged by one thread in registers
constexpr int kTvWaveSmall = 256;  // inputs merged by one wave with a small LDS buffer
constexpr int kTvWaveMax = 2048;   // inputs merged by one wave with a large LDS buffer
constexpr int kTvBigThreads = 1024;
constexpr int kTvBigPieces = 4096;  // body symbols the workgroup merge keeps cursors for

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t first_at_least(const uint32_t* w, uint32_t lo, uint32_t hi, uint32_t x) {
  while (lo < hi) {  // first index in [lo, hi) with w[i] >= x
    const uint32_t mid = (lo + hi) >> 1;
    if (w[mid] >= x) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_tv_classify(DevGrammar g, const int32_t* rules, int32_t n,
                                                     const uint32_t* tsize, int32_t* list_thread, int32_t* list_small,
                                                     int32_t* list_wave, int32_t* list_big, int32_t* counts) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < n;
  const int32_t r = live ? rules[i] : 0;
  const int64_t a = live ? g.rule_off[r] : 0, b = live ? g.rule_off[r + 1] : 0;
  uint64_t n_in = 0;
  for (int64_t q0 = a; q0 < b; q0 += 8) {
    int32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = q0 + k < b ? g.sym[q0 + k] : 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (q0 + k < b) n_in += v[k] >= 0 ? 1u : tsize[-v[k]];
  }
  // one counter atomic per wave and list (a per-thread atomic on one address
  // serializes millions of them)
  const int tier = n_in <= (uint64_t)kTvThreadMax ? 0 : n_in <= (uint64_t)kTvWaveSmall ? 1
                   : n_in <= (uint64_t)kTvWaveMax ? 2 : 3;
  // appends aggregated per workgroup: one global atomic per workgroup and
  // list (per wave they still made ~60K same-address atomics on a 4M-rule level)
  __shared__ int32_t wcnt[4], wbase[4];
  if (threadIdx.x < 4) wcnt[threadIdx.x] = 0;
  __syncthreads();
  int32_t my = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const uint64_t mask = __ballot(live && tier == t);
    if (mask) {
      const int leader = __ffsll((unsigned long long)mask) - 1;
      int32_t base = 0;
      if (lane_id() == leader) base = atomicAdd(&wcnt[t], (int32_t)__popcll(mask));
      base = __shfl(base, leader);
      if (live && tier == t) my = base + (int32_t)__popcll(mask & lanes_below());
    }
  }
  __syncthreads();
  if (threadIdx.x < 4) wbase[threadIdx.x] = wcnt[threadIdx.x] ? atomicAdd(&counts[threadIdx.x], wcnt[threadIdx.x]) : 0;
  __syncthreads();
  if (live) {
    const int32_t at = wbase[tier] + my;
    if (tier == 0) list_thread[at] = r;
    else if (tier == 1) list_small[at] = r;
    else if (tier == 2) list_wave[at] = r;
    else list_big[at] = r;
  }
}

// One thread per rule with at most kTvThreadMax inputs: the inputs (word <<
// 32 | count) are gathered into a register array (each insert a fixed loop
// of selects, so the array is never indexed dynamically), sorted by a
// bitonic network over the 16 slots, and the runs of equal words summed.
__device__ __forceinline__ void reg_insert(uint64_t (&e)[kTvThreadMax], int at, uint64_t x) {
#pragma unroll
  for (int i = 0; i < kTvThreadMax; ++i)
    if (i == at) e[i] = x;
}

__global__ __launch_bounds__(256) void k_tv_merge_thread(DevGrammar g, const int32_t* list, const int32_t* count,
                                                         const uint64_t* toff, uint32_t* tsize, uint32_t* pw,
                                                         uint32_t* pc) {
  const int32_t nr = *count;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nr; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = list[j];
    const int64_t a = g.rule_off[r], b = g.rule_off[r + 1];
    uint64_t e[kTvThreadMax];
#pragma unroll
    for (int i = 0; i < kTvThreadMax; ++i) e[i] = ~0ull;
    int n = 0;
    for (int64_t q = a; q < b; ++q) {
      const int32_t s = g.sym[q];
      if (s >= 0) {
        reg_insert(e, n++, ((uint64_t)(uint32_t)s << 32) | 1u);
      } else {
        const uint32_t t = tsize[-s];
        const uint64_t o = toff[-s];
        for (uint32_t x = 0; x < t && n < kTvThreadMax; ++x) reg_insert(e, n++, ((uint64_t)pw[o + x] << 32) | pc[o + x]);
      }
    }
#pragma unroll
    for (int k = 2; k <= kTvThreadMax; k <<= 1) {
#pragma unroll
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
#pragma unroll
        for (int i = 0; i < kTvThreadMax; ++i) {
          const int l = i ^ jj;
          if (l > i) {
            const uint64_t u = e[i], v = e[l];
            const bool swap = ((i & k) == 0) ? (u > v) : (u < v);
            e[i] = swap ? v : u;
            e[l] = swap ? u : v;
          }
        }
      }
    }
    const uint64_t out = toff[r];
    uint32_t m = 0, run_w = 0xffffffffu, run_c = 0;
#pragma unroll
    for (int i = 0; i < kTvThreadMax; ++i) {
      const uint32_t wd = (uint32_t)(e[i] >> 32), c = (uint32_t)e[i];
      if (i < n) {
        if (wd != run_w) {
          if (run_c) pw[out + m] = run_w, pc[out + m] = run_c, ++m;
          run_w = wd, run_c = c;
        } else {
          run_c += c;
        }
      }
    }
    if (run_c) pw[out + m] = run_w, pc[out + m] = run_c, ++m;
    tsize[r] = m;
  }
}

template <int kMax, int kWaves>
__global__ __launch_bounds__(64 * kWaves) void k_tv_merge_wave(DevGrammar g, const int32_t* list, const int32_t* count,
                                                               const uint64_t* toff, uint32_t* tsize, uint32_t* pw,
                                                               uint32_t* pc) {
  constexpr int kTvWaveWaves = kWaves;
  __shared__ uint64_t buf[kWaves][kMax];  // (word << 32 | count) per input
  const int wave = threadIdx.x >> 6, lane = lane_id();
  uint64_t* e = buf[wave];
  const int32_t nr = *count;
  for (int64_t j = (int64_t)blockIdx.x * kTvWaveWaves + wave; j < nr; j += (int64_t)gridDim.x * kTvWaveWaves) {
    const int32_t r = list[j];
    const int64_t a = g.rule_off[r], b = g.rule_off[r + 1];
    // gather: 64 pieces at a time, their sizes and sources loaded by the lanes
    uint32_t n = 0;
    for (int64_t q0 = a; q0 < b; q0 += 64) {
      const int64_t q = q0 + lane;
      const int32_t s = q < b ? g.sym[q] : 0;
      const uint32_t size = q >= b ? 0u : (s >= 0 ? 1u : tsize[-s]);
      const uint64_t src = (q < b && s < 0) ? toff[-s] : 0;
      uint32_t incl = size;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
      }
      const uint32_t at = n + incl - size;
      const int np = (int)(b - q0 < 64 ? b - q0 : 64);
      for (int pp = 0; pp < np; ++pp) {
        const int32_t sp = __shfl(s, pp);
        const uint32_t tp = __shfl(size, pp), ap = __shfl(at, pp);
        const uint64_t op = __shfl(src, pp);
        if (sp >= 0) {
          if (lane == 0) e[ap] = ((uint64_t)(uint32_t)sp << 32) | 1u;
        } else {
          for (uint32_t x = lane; x < tp; x += 64) e[ap + x] = ((uint64_t)pw[op + x] << 32) | pc[op + x];
        }
      }
      n += __shfl(incl, 63);
    }
    uint32_t P = 1;
    while (P < n) P <<= 1;
    for (uint32_t x = n + lane; x < P; x += 64) e[x] = ~0ull;
    wave_lds_sync();
    // bitonic sort, ascending
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
        for (uint32_t x = lane; x < P; x += 64) {
          const uint32_t l = x ^ jj;
          if (l > x) {
            const uint64_t u = e[x], v = e[l];
            if ((u > v) == ((x & k) == 0)) e[x] = v, e[l] = u;
          }
        }
        wave_lds_sync();
      }
    }
    // one output entry per distinct word: lanes take consecutive chunks
    const uint32_t C = (n + 63) / 64;
    const uint32_t c0 = lane * C < n ? lane * C : n, c1 = c0 + C < n ? c0 + C : n;
    uint32_t h = 0;
    for (uint32_t x = c0; x < c1; ++x) h += x == 0 || (e[x] >> 32) != (e[x - 1] >> 32);
    uint32_t incl = h;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    uint32_t o = incl - h;
    const uint64_t out = toff[r];
    for (uint32_t x = c0; x < c1; ++x) {
      const uint32_t wd = (uint32_t)(e[x] >> 32);
      if (x == 0 || wd != (uint32_t)(e[x - 1] >> 32)) {
        uint32_t sum = 0;
        for (uint32_t y = x; y < n && (uint32_t)(e[y] >> 32) == wd; ++y) sum += (uint32_t)e[y];
        pw[out + o] = wd;
        pc[out + o] = sum;
        ++o;
      }
    }
    if (lane == 63) tsize[r] = incl;
    wave_lds_sync();  // the next rule reuses the buffer
  }
}

// Exclusive scan over a 1024-thread workgroup (16 waves); *total gets the sum.
__device__ __forceinline__ uint32_t block_scan_1024(uint32_t v, uint32_t* lds16, uint32_t* total) {
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane_id() >= o) x += y;
  }
  if (lane_id() == 63) lds16[threadIdx.x >> 6] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    const uint32_t c = lds16[w];
    if (w < (int)(threadIdx.x >> 6)) base += c;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__device__ __forceinline__ uint32_t block_min_1024(uint32_t v, uint32_t* lds16) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t y = __shfl_xor(v, o);
    v = y < v ? y : v;
  }
  if (lane_id() == 0) lds16[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t m = 0xffffffffu;
#pragma unroll
  for (int w = 0; w < 16; ++w) m = lds16[w] < m ? lds16[w] : m;
  __syncthreads();
  return m;
}

// Serial merge by binary search (rules with more than kTvBigPieces body
// symbols; never produced by Sequitur in practice, kept for completeness).
__device__ void tv_merge_serial(const DevGrammar& g, int32_t r, const uint64_t* toff, uint32_t* tsize, uint32_t* pw,
                                uint32_t* pc) {
  const int64_t a = g.rule_off[r], k = g.rule_off[r + 1] - a;
  const uint64_t out = toff[r];
  uint32_t m = 0;
  uint32_t next = 0;  // smallest word not yet emitted
  while (true) {
    uint32_t best = 0xffffffffu;
    for (int64_t j = 0; j < k; ++j) {
      const int32_t s = g.sym[a + j];
      if (s >= 0) {
        if ((uint32_t)s >= next && (uint32_t)s < best) best = (uint32_t)s;
      } else {
        const uint32_t t = tsize[-s];
        const uint32_t x = first_at_least(pw + toff[-s], 0, t, next);
        if (x < t && pw[toff[-s] + x] < best) best = pw[toff[-s] + x];
      }
    }
    if (best == 0xffffffffu) break;
    uint32_t cnt = 0;
    for (int64_t j = 0; j < k; ++j) {
      const int32_t s = g.sym[a + j];
      if (s >= 0) {
        cnt += (uint32_t)s == best;
      } else {
        const uint32_t t = tsize[-s];
        const uint32_t x = first_at_least(pw + toff[-s], 0, t, best);
        if (x < t && pw[toff[-s] + x] == best) cnt += pc[toff[-s] + x];
      }
    }
    pw[out + m] = best;
    pc[out + m] = cnt;
    ++m;
    next = best + 1;
  }
  tsize[r] = m;
}

__global__ __launch_bounds__(kTvBigThreads) void k_tv_merge_big(DevGrammar g, const int32_t* list,
                                                                const int32_t* count, const uint64_t* toff,
                                                                uint32_t* tsize, uint32_t* pw, uint32_t* pc) {
  __shared__ uint32_t cnt[kWcBucket];
  __shared__ uint32_t cur[kTvBigPieces], endp[kTvBigPieces], pref[kTvBigPieces];
  __shared__ uint32_t red[16];
  const int32_t nr = *count;
  for (int32_t j = blockIdx.x; j < nr; j += gridDim.x) {
    const int32_t r = list[j];
    const int64_t a = g.rule_off[r];
    const int32_t k = (int32_t)(g.rule_off[r + 1] - a);
    if (k > kTvBigPieces) {
      if (threadIdx.x == 0) tv_merge_serial(g, r, toff, tsize, pw, pc);
      __syncthreads();
      continue;
    }
    const uint64_t out = toff[r];
    for (int p = threadIdx.x; p < k; p += blockDim.x) cur[p] = 0;
    for (int x = threadIdx.x; x < kWcBucket; x += blockDim.x) cnt[x] = 0;
    __syncthreads();
    uint32_t m = 0;
    while (true) {
      // the window is the 4096-id bucket of the smallest pending word
      uint32_t lmin = 0xffffffffu;
      for (int p = threadIdx.x; p < k; p += blockDim.x) {
        const int32_t s = g.sym[a + p];
        uint32_t wd = 0xffffffffu;
        if (s >= 0) {
          if (cur[p] == 0) wd = (uint32_t)s;
        } else if (cur[p] < tsize[-s]) {
          wd = pw[toff[-s] + cur[p]];
        }
        lmin = wd < lmin ? wd : lmin;
      }
      const uint32_t w0 = block_min_1024(lmin, red);
      if (w0 == 0xffffffffu) break;
      const uint32_t wb = w0 & ~(uint32_t)(kWcBucket - 1);
      const uint64_t w1 = (uint64_t)wb + kWcBucket;
      // every piece's inputs inside the window, and their offsets (4 pieces per thread)
      uint32_t mine[4], tot4 = 0;
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int p = threadIdx.x * 4 + x;
        uint32_t c = 0;
        if (p < k) {
          const int32_t s = g.sym[a + p];
          uint32_t e;
          if (s >= 0) {
            e = (cur[p] == 0 && (uint64_t)s < w1) ? 1u : cur[p];
          } else {
            const uint32_t t = tsize[-s];
            e = w1 > 0xffffffffull ? t : first_at_least(pw + toff[-s], cur[p], t, (uint32_t)w1);
          }
          endp[p] = e;
          c = e - cur[p];
        }
        mine[x] = c;
        tot4 += c;
      }
      uint32_t total;
      uint32_t base = block_scan_1024(tot4, red, &total);
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int p = threadIdx.x * 4 + x;
        if (p < k) pref[p] = base;
        base += mine[x];
      }
      __syncthreads();
      for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
        int lo = 0, hi = k - 1;  // last piece with pref <= e
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (pref[mid] <= e) lo = mid;
          else hi = mid - 1;
        }
        const int32_t s = g.sym[a + lo];
        if (s >= 0) {
          atomicAdd(&cnt[(uint32_t)s - wb], 1u);
        } else {
          const uint64_t at = toff[-s] + cur[lo] + (e - pref[lo]);
          atomicAdd(&cnt[pw[at] - wb], pc[at]);
        }
      }
      __syncthreads();
      // the window's nonzero slots, in word order (4 consecutive slots per thread)
      uint32_t c4[4], nz = 0;
#pragma unroll
      for (int x = 0; x < 4; ++x) c4[x] = cnt[threadIdx.x * 4 + x], nz += c4[x] != 0;
      uint32_t nz_total;
      uint32_t pos = m + block_scan_1024(nz, red, &nz_total);
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        if (c4[x]) {
          pw[out + pos] = wb + threadIdx.x * 4 + x;
          pc[out + pos] = c4[x];
          ++pos;
          cnt[threadIdx.x * 4 + x] = 0;
        }
      }
      m += nz_total;
      for (int p = threadIdx.x; p < k; p += blockDim.x) cur[p] = endp[p];
      __syncthreads();
    }
    if (threadIdx.x == 0) tsize[r] = m;
    __syncthreads();
  }
}

hipError_t launch_tv_tables(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, const uint64_t* toff,
                            uint32_t* tsize, uint32_t* pw, uint32_t* pc, int32_t* lists, int32_t* counts,
                            hipStream_t s) {
  hipError_t e = launch_fill_i32(counts, 4 * ((int64_t)depth + 2), 0, s);
  if (e != hipSuccess) return e;
  for (int32_t d = depth; d >= 1; --d) {
    const int32_t lo = level_off_host[d], hi = level_off_host[d + 1];
    if (hi <= lo) continue;
    const int32_t n = hi - lo;
    int32_t* c = counts + 4 * d;
    int32_t* list_thread = lists;
    int32_t* list_small = lists + n;
    int32_t* list_wave = lists + 2 * (int64_t)n;
    int32_t* list_big = lists + 3 * (int64_t)n;
    k_tv_classify<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, g.level_rule + lo, n, tsize, list_thread, list_small,
                                                               list_wave, list_big, c);
    const int32_t g0 = (n + 255) / 256;
    k_tv_merge_thread<<<(unsigned)(g0 < 4096 ? g0 : 4096), 256, 0, s>>>(g, list_thread, c + 0, toff, tsize, pw, pc);
    const int32_t g1 = (n + 15) / 16;
    k_tv_merge_wave<kTvWaveSmall, 16><<<(unsigned)(g1 < 4096 ? g1 : 4096), 1024, 0, s>>>(g, list_small, c + 1, toff,
                                                                                           tsize, pw, pc);
    const int32_t g2 = (n + 3) / 4;
    k_tv_merge_wave<kTvWaveMax, 4><<<(unsigned)(g2 < 4096 ? g2 : 4096), 256, 0, s>>>(g, list_wave, c + 2, toff, tsize,
                                                                                       pw, pc);
    k_tv_merge_big<<<(unsigned)(n < 1024 ? n : 1024), kTvBigThreads, 0, s>>>(g, list_big, c + 3, toff, tsize, pw, pc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Per-file reduce. A file span is cut into units of kTileSyms root symbols;
// unit_off[f] = first unit of file f (exclusive scan of the unit counts). The
// count table has one slot per (file, bucket, unit), laid out file by file,
// bucket-major inside a file: slot(f, b, u) = nb * unit_off[f] + b * n_f +
// (u - unit_off[f]), so one scan of the table makes every (file, bucket)
// group contiguous.
// ---------------------------------------------------------------------------
__global__ void k_tv_unit_counts(DevGrammar g, int64_t* units) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f < g.F) units[f] = (g.file_off[f + 1] - g.file_off[f] + kTileSyms - 1) / kTileSyms;
}

__device__ __forceinline__ int64_t file_of_unit(const int64_t* unit_off, int64_t F, int64_t u) {
  int64_t lo = 0, hi = F - 1;  // last f with unit_off[f] <= u (files with units)
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (unit_off[mid] <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Pass 1 (count) and pass 2 (scatter) walk the same inputs of one unit: its
// root words (count 1) and every entry of the table of each referenced
// child. The unit's inputs are numbered by an exclusive scan of the symbols'
// input counts, and the workgroup's threads take them in turn (a binary
// search in LDS finds the symbol of input e), so a child with a huge table
// is spread over the whole workgroup instead of one thread.
template <bool kScatter>
__global__ __launch_bounds__(256) void k_tv_group(DevGrammar g, TvFiles t, uint64_t* entries) {
  extern __shared__ uint32_t lds_tv[];  // per-bucket counts (pass 1) or cursors (pass 2)
  __shared__ uint32_t pre[kTileSyms];   // exclusive prefix of the symbols' input counts
  __shared__ int32_t syms[kTileSyms];
  __shared__ uint32_t part[4];
  __shared__ int64_t sh_f;
  const int64_t u = blockIdx.x;
  if (threadIdx.x == 0) sh_f = file_of_unit(t.unit_off, g.F, u);
  __syncthreads();
  const int64_t f = sh_f;
  const int64_t n_f = t.unit_off[f + 1] - t.unit_off[f];
  const int64_t k = u - t.unit_off[f];
  const int64_t slot0 = (int64_t)t.nb * t.unit_off[f] + k;
  for (int b = threadIdx.x; b < t.nb; b += blockDim.x) lds_tv[b] = kScatter ? t.table[slot0 + b * n_f] : 0u;
  const int64_t fs = g.file_off[f] + k * kTileSyms, fe0 = g.file_off[f + 1];
  const int32_t len = (int32_t)(fs + kTileSyms < fe0 ? kTileSyms : fe0 - fs);
  // input counts of this thread's 16 symbols, then their offsets
  uint32_t c[kPerThread], mine = 0;
#pragma unroll
  for (int x = 0; x < kPerThread; ++x) {
    const int32_t j = threadIdx.x * kPerThread + x;
    int32_t sv = 0;
    c[x] = 0;
    if (j < len) {
      sv = g.sym[fs + j];
      c[x] = sv >= 0 ? 1u : t.tsize[-sv];
      syms[j] = sv;
    }
    mine += c[x];
  }
  uint32_t total;
  uint32_t base = block_exclusive_scan_256(mine, part, &total);
#pragma unroll
  for (int x = 0; x < kPerThread; ++x) {
    const int32_t j = threadIdx.x * kPerThread + x;
    if (j < len) pre[j] = base;
    base += c[x];
  }
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
    int32_t lo = 0, hi = len - 1;  // last symbol with pre <= e (every symbol has >= 1 input)
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int32_t sv = syms[lo];
    uint32_t wd, cn;
    if (sv >= 0) {
      wd = (uint32_t)sv, cn = 1;
    } else {
      const uint64_t at = t.toff[-sv] + (e - pre[lo]);
      wd = t.pw[at], cn = t.pc[at];
    }
    const uint32_t at = atomicAdd(&lds_tv[wd >> kWcBits], 1u);
    if (kScatter) entries[at] = ((uint64_t)cn << kWcBits) | (uint64_t)(wd & (kWcBucket - 1));
  }
  if (!kScatter) {
    __syncthreads();
    for (int b = threadIdx.x; b < t.nb; b += blockDim.x) t.table[slot0 + b * n_f] = lds_tv[b];
  }
}

hipError_t launch_tv_count(const DevGrammar& g, const TvFiles& t, hipStream_t s) {
  if (t.nunits == 0) return hipSuccess;
  k_tv_group<false><<<(unsigned)t.nunits, 256, sizeof(uint32_t) * t.nb, s>>>(g, t, nullptr);
  return hipGetLastError();
}
hipError_t launch_tv_scatter(const DevGrammar& g, const TvFiles& t, uint64_t* entries, hipStream_t s) {
  if (t.nunits == 0) return hipSuccess;
  k_tv_group<true><<<(unsigned)t.nunits, 256, sizeof(uint32_t) * t.nb, s>>>(g, t, entries);
  return hipGetLastError();
}
hipError_t launch_tv_units(const DevGrammar& g, int64_t* units, hipStream_t s) {
  k_tv_unit_counts<<<(unsigned)((g.F + 255) / 256), 256, 0, s>>>(g, units);
  return hipGetLastError();
}

// Start of group s = (file f, bucket b) in the scanned table (E past the end).
__device__ __forceinline__ int64_t group_start(const DevGrammar& g, const TvFiles& t, int64_t s, int64_t E) {
  const int64_t nb = t.nb;
  const int64_t f = s / nb, b = s % nb;
  if (f >= g.F) return E;
  const int64_t n_f = t.unit_off[f + 1] - t.unit_off[f];
  const int64_t slot = nb * t.unit_off[f] + b * n_f;
  return slot < nb * t.nunits ? (int64_t)t.table[slot] : E;
}

// Pass 3: sum each group (file f, word bucket b); the distinct words come
// out in word order, written back over the group's own entries as (word <<
// 32 | count), and their number to nnz[group]. A dense 4096-slot LDS table
// per group costs F x V slot visits whatever the group sizes (most groups
// hold a few hundred entries), so groups are merged by size:
//  - up to kTvGroupSmall entries: one wave per group sorts them in LDS
//    (bitonic, by low word id) and sums the runs of equal words;
//  - larger: one workgroup per group, dense LDS table.
// (A middle class sorting up to 2048 entries per wave was measured slower
// than the dense table.) The wave pass hands the larger groups on in a list,
// one atomic per workgroup.
constexpr int kTvThreads = 1024;
constexpr int kTvGroupSmall = 256;

template <int kMax, int kWaves, bool kFromList>
__global__ __launch_bounds__(64 * kWaves) void k_tv_group_merge(DevGrammar g, TvFiles t, uint64_t* entries, int64_t E,
                                                                uint32_t* nnz, const int32_t* list, const int32_t* count,
                                                                int32_t* next_list, int32_t* next_count) {
  __shared__ uint64_t buf[kWaves][kMax];
  __shared__ int32_t handed[kWaves][64];  // groups for the next size class, gathered per wave
  __shared__ int32_t handed_n[kWaves], handed_base;
  const int wave = threadIdx.x >> 6, lane = lane_id();
  uint64_t* e = buf[wave];
  int32_t nh = 0;  // this wave's handed groups (uniform in the wave)
  const int64_t ngroups = kFromList ? (int64_t)*count : g.F * (int64_t)t.nb;
  for (int64_t j = (int64_t)blockIdx.x * kWaves + wave; j < ngroups; j += (int64_t)gridDim.x * kWaves) {
    const int64_t grp = kFromList ? (int64_t)list[j] : j;
    const int64_t lo = group_start(g, t, grp, E), hi = group_start(g, t, grp + 1, E);
    const uint32_t n = (uint32_t)(hi - lo);
    if (n > (uint32_t)kMax) {  // uniform for the wave: hand the group on
      if (nh == 64) {  // buffer full: flush it with one atomic
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(next_count, 64);
        base = __shfl(base, 0);
        next_list[base + lane] = handed[wave][lane];
        wave_lds_sync();
        nh = 0;
      }
      if (lane == 0) handed[wave][nh] = (int32_t)grp;
      ++nh;
      wave_lds_sync();
      continue;
    }
    if (n == 0) continue;  // nnz stays 0
    // (low id << 32 | count), sorted by low id, so equal words are adjacent
    uint32_t P = 1;
    while (P < n) P <<= 1;
    for (uint32_t x = lane; x < P; x += 64) {
      if (x < n) {
        const uint64_t v = entries[lo + x];
        e[x] = ((v & (kWcBucket - 1)) << 32) | (v >> kWcBits);
      } else {
        e[x] = ~0ull;
      }
    }
    wave_lds_sync();
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
        for (uint32_t x = lane; x < P; x += 64) {
          const uint32_t l = x ^ jj;
          if (l > x) {
            const uint64_t u = e[x], v = e[l];
            if ((u > v) == ((x & k) == 0)) e[x] = v, e[l] = u;
          }
        }
        wave_lds_sync();
      }
    }
    const uint32_t C = (n + 63) / 64;
    const uint32_t c0 = lane * C < n ? lane * C : n, c1 = c0 + C < n ? c0 + C : n;
    uint32_t h = 0;
    for (uint32_t x = c0; x < c1; ++x) h += x == 0 || (e[x] >> 32) != (e[x - 1] >> 32);
    uint32_t incl = h;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    uint32_t o = incl - h;
    const uint64_t wbase = (uint64_t)(grp % t.nb) * kWcBucket;
    for (uint32_t x = c0; x < c1; ++x) {
      const uint32_t low = (uint32_t)(e[x] >> 32);
      if (x == 0 || low != (uint32_t)(e[x - 1] >> 32)) {
        uint32_t sum = 0;
        for (uint32_t y = x; y < n && (uint32_t)(e[y] >> 32) == low; ++y) sum += (uint32_t)e[y];
        entries[lo + o] = ((wbase + low) << 32) | sum;
        ++o;
      }
    }
    if (lane == 63) nnz[grp] = incl;
    wave_lds_sync();  // the next group reuses the buffer
  }
  // the handed groups of the whole workgroup, with one atomic
  if (lane == 0) handed_n[wave] = nh;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t tot = 0;
    for (int w = 0; w < kWaves; ++w) tot += handed_n[w];
    handed_base = tot ? atomicAdd(next_count, tot) : 0;
  }
  __syncthreads();
  int32_t off = handed_base;
  for (int w = 0; w < wave; ++w) off += handed_n[w];
  if (lane < nh) next_list[off + lane] = handed[wave][lane];
}

// Groups too large for a wave: one workgroup each, dense LDS table.
__global__ __launch_bounds__(kTvThreads) void k_tv_group_dense(DevGrammar g, TvFiles t, uint64_t* entries, int64_t E,
                                                               uint32_t* nnz, const int32_t* list,
                                                               const int32_t* count) {
  __shared__ uint32_t cnt[kWcBucket];
  __shared__ uint32_t wsum[kTvThreads / 64];
  for (int i = threadIdx.x; i < kWcBucket; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const int32_t ng = *count;
  for (int32_t j = blockIdx.x; j < ng; j += gridDim.x) {
    const int64_t s = list[j];
    const int64_t lo = group_start(g, t, s, E), hi = group_start(g, t, s + 1, E);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const uint64_t e = entries[i];
      atomicAdd(&cnt[e & (kWcBucket - 1)], (uint32_t)(e >> kWcBits));
    }
    __syncthreads();
    // compact the nonzero slots in word order: 4 consecutive slots per thread
    uint32_t c4[4], nz = 0;
#pragma unroll
    for (int x = 0; x < 4; ++x) c4[x] = cnt[threadIdx.x * 4 + x], nz += c4[x] != 0;
    uint32_t incl = nz;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane_id() >= o) incl += y;
    }
    if (lane_id() == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (int w = 0; w < kTvThreads / 64; ++w) {
      if (w < (int)(threadIdx.x >> 6)) base += wsum[w];
      total += wsum[w];
    }
    uint32_t pos = base + incl - nz;
    const uint64_t b = (uint64_t)(s % t.nb) * kWcBucket;
#pragma unroll
    for (int x = 0; x < 4; ++x)
      if (c4[x]) entries[lo + pos++] = ((b + threadIdx.x * 4 + x) << 32) | c4[x];
    if (threadIdx.x == 0) nnz[s] = total;
#pragma unroll
    for (int x = 0; x < 4; ++x) cnt[threadIdx.x * 4 + x] = 0;
    __syncthreads();
  }
}

// lists: F * nb group ids; counts: 1 counter.
hipError_t launch_tv_reduce(const DevGrammar& g, const TvFiles& t, uint64_t* entries, int64_t E, uint32_t* nnz,
                            int32_t* lists, int32_t* counts, hipStream_t s) {
  const int64_t ngroups = g.F * (int64_t)t.nb;
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(nnz), ngroups, 0, s);
  if (e == hipSuccess) e = launch_fill_i32(counts, 1, 0, s);
  if (e != hipSuccess || ngroups == 0) return e;
  int32_t* l1 = lists;
  const int64_t g0 = (ngroups + 15) / 16;
  k_tv_group_merge<kTvGroupSmall, 16, false><<<(unsigned)(g0 < 4096 ? g0 : 4096), 1024, 0, s>>>(
      g, t, entries, E, nnz, nullptr, nullptr, l1, counts + 0);
  k_tv_group_dense<<<(unsigned)(ngroups < 2048 ? ngroups : 2048), kTvThreads, 0, s>>>(g, t, entries, E, nnz, l1,
                                                                                   counts + 0);
  return hipGetLastError();
}

// Pass 4: groups to the final CSR. noff = exclusive scan of nnz (group order
// = file order, word order); one workgroup per group copies its pairs.
__global__ __launch_bounds__(256) void k_tv_emit(DevGrammar g, TvFiles t, const uint64_t* entries, int64_t E,
                                                 const uint32_t* nnz, const uint32_t* noff, uint32_t* out_word,
                                                 uint64_t* out_cnt, int64_t* out_off) {
  const int64_t s = blockIdx.x;
  const int64_t lo = group_start(g, t, s, E);
  const uint32_t n = nnz[s], o = noff[s];
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const uint64_t e = entries[lo + i];
    out_word[o + i] = (uint32_t)(e >> 32);
    out_cnt[o + i] = e & 0xffffffffull;
  }
  if (threadIdx.x == 0 && s % t.nb == 0) out_off[s / t.nb] = o;
}

hipError_t launch_tv_emit(const DevGrammar& g, const TvFiles& t, const uint64_t* entries, int64_t E,
                          const uint32_t* nnz, const uint32_t* noff, uint32_t* out_word, uint64_t* out_cnt,
                          int64_t* out_off, hipStream_t s) {
  const int64_t ngroups = g.F * (int64_t)t.nb;
  if (ngroups == 0) return hipSuccess;
  k_tv_emit<<<(unsigned)ngroups, 256, 0, s>>>(g, t, entries, E, nnz, noff, out_word, out_cnt, out_off);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inverted index: stable radix sort of (word, file) by word, then the word
// offsets from the run boundaries.
// ---------------------------------------------------------------------------
// (word, file) pairs of the term vector. A workgroup takes 4096 consecutive
// entries: the files of its first and last entry are found once (binary
// search on tv_off), and each entry searches only that range (nearly always
// one file), instead of a full search per entry.
// One (key, file) pair per term-vector entry, in the term vector's
// file-major order. key = word, or for the ranked index (tv_cnt given)
// word << 32 | (2^32 - 1 - tf), so that one ascending stable sort orders by
// word, then term frequency descending, then file (the input order).
__global__ __launch_bounds__(256) void k_ii_pairs(const int64_t* tv_off, int64_t F, const uint32_t* tv_word,
                                                  const uint64_t* tv_cnt, int64_t nnz, uint64_t* key, uint32_t* file) {
  __shared__ int64_t frange[2];
  const int64_t c0 = (int64_t)blockIdx.x * 4096;
  const int64_t c1 = c0 + 4096 < nnz ? c0 + 4096 : nnz;
  if (threadIdx.x < 2) {
    const int64_t i = threadIdx.x == 0 ? c0 : c1 - 1;
    int64_t lo = 0, hi = F - 1;  // file f with tv_off[f] <= i < tv_off[f+1] (the last such f)
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (tv_off[mid] <= i) lo = mid;
      else hi = mid - 1;
    }
    frange[threadIdx.x] = lo;
  }
  __syncthreads();
  const int64_t flo = frange[0], fhi = frange[1];
  for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
    int64_t lo = flo, hi = fhi;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (tv_off[mid] <= i) lo = mid;
      else hi = mid - 1;
    }
    key[i] = tv_cnt ? (uint64_t)tv_word[i] << 32 | (0xffffffffull - tv_cnt[i]) : (uint64_t)tv_word[i];
    file[i] = (uint32_t)lo;
  }
}

__global__ void k_ii_offsets(const uint64_t* key, int shift, int64_t nnz, int32_t V, int64_t* off) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > nnz) return;
  // words w in (word[i-1], word[i]] start at i; past the end, up to V
  const int64_t prev = i == 0 ? -1 : (int64_t)(key[i - 1] >> shift);
  const int64_t cur = i == nnz ? (int64_t)V : (int64_t)(key[i] >> shift);
  for (int64_t w = prev + 1; w <= cur; ++w) off[w] = i;
}

// Term frequencies of the ranked index, back from the sorted keys.
__global__ void k_rii_tf(const uint64_t* key, int64_t nnz, uint64_t* tf) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nnz) tf[i] = 0xffffffffull - (key[i] & 0xffffffffull);
}

hipError_t launch_ii(const int64_t* tv_off, int64_t F, const uint32_t* tv_word, const uint64_t* tv_cnt, int64_t nnz,
                     int32_t V, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint64_t* kout,
                     uint32_t* file_out, const int64_t* num, uint32_t* hist, int64_t* ii_off, uint64_t* tf_out,
                     hipStream_t s) {
  const int shift = tv_cnt ? 32 : 0;
  if (nnz > 0) {
    k_ii_pairs<<<(unsigned)((nnz + 4095) / 4096), 256, 0, s>>>(tv_off, F, tv_word, tv_cnt, nnz, k0, v0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int b = 1;
    while (b < 32 && (1ll << b) < (int64_t)V) ++b;
    // word bytes, and for the ranked index the four frequency bytes below them
    e = radix_sort_pairs<uint32_t>(k0, v0, k1, v1, num, nnz, tv_cnt ? 0 : shift, shift + b, false, hist, kout,
                                   file_out, s);
    if (e != hipSuccess) return e;
    if (tv_cnt) {
      k_rii_tf<<<(unsigned)((nnz + 255) / 256), 256, 0, s>>>(kout, nnz, tf_out);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  k_ii_offsets<<<(unsigned)((nnz + 1 + 255) / 256), 256, 0, s>>>(kout, shift, nnz, V, ii_off);
  return hipGetLastError();
}

hipError_t launch_scan_u64_ext(uint64_t* a, int64_t n, int64_t* total, uint64_t* sums, hipStream_t s) {
  return launch_scan_u64(a, n, total, sums, s);
}
hipError_t launch_scan_u32_ext(uint32_t* a, int64_t n, int64_t* total, uint32_t* sums, hipStream_t s) {
  return launch_scan_u32(a, n, total, sums, s);
}

}  // namespace gt

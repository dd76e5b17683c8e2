// k_levels.hip -- level-by-level topological frontiers and top-down rule
// weights of a loaded grammar (the initialization phase's traversal).
//
// Paper: Algorithm "Top-Down Traversal" (mask initialization from the
// in-edges that do not come from the root, initial weights = frequencies in
// the root, then rounds in which every ready rule adds frequency x weight to
// its sub-rules and a sub-rule becomes ready when all its in-edges have
// arrived).
//
// Differences from the paper's design (same results): the rounds are not
// relaunched from the host until a stop flag stays set. One cooperative
// launch walks the levels with a grid barrier between them (narrow levels
// finish on a single workgroup), and each level's ready rules are compacted
// into a frontier list (gathered per workgroup in LDS, one global atomic per
// workgroup and level), so a round touches only the rules of that level
// rather than scanning every rule's mask. Bodies are walked by one thread
// (short) or one wave (long), and the widest levels can accumulate by
// bucket instead of atomics. In-degrees count occurrences (a rule used twice
// by the same parent waits for both), which gives the same levels and
// weights. A rule's weight and its pending in-edges share one 64-bit word
// (weight << kPendBits | pending) during the walk: one atomic adds a
// parent's weight and retires the in-edge, and its return value tells the
// last parent that the rule is ready.
#include "device.h"
#include "radix.h"

namespace gt {

// Level 1 = the rules with no pending in-edge (used only by the root, or not
// at all), compacted in rule-id order: a count per block of kRadixTile
// rules, an exclusive scan, then every block writes its rules at its offset.
// Rule i0 + k * 256 + thread (k < 16) of a block: the lanes of a wave read
// consecutive words, and the output keeps rule-id order by ranking the
// rules of each (step k, wave) with a ballot.
__global__ __launch_bounds__(256) void k_zero_count(const uint64_t* pw, int64_t R, uint32_t* cnt) {
  const int64_t i0 = (int64_t)blockIdx.x * kRadixTile + threadIdx.x;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t r = i0 + k * 256;
    if (r >= 1 && r < R && (pw[r] & kPendMask) == 0) ++c;
  }
  __shared__ uint32_t lds[4];
  uint32_t total;
  block_exclusive_scan_256(c, lds, &total);
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_zero_write(const uint64_t* pw, int64_t R, const uint32_t* off,
                                                    int32_t* out, uint64_t* qw, FlowState* fs, const int64_t* n1p) {
  if (fs && blockIdx.x == 0 && threadIdx.x == 0) {
    // the dataflow walk's queue starts with level 1 in rule-id order (low ids,
    // the rules Sequitur made first, tend to head the deepest subtrees, so
    // they start first)
    const int64_t n1 = *n1p;
    fs->n1 = n1;
    fs->live = n1;
    fs->space = (uint32_t)n1;
    fs->ticket = 0;
    fs->nspill = 0;
  }
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t i0 = (int64_t)blockIdx.x * kRadixTile + threadIdx.x;
  __shared__ uint32_t start[16][4];  // per (step, wave): count, then first output position
  uint64_t w[16];
  uint64_t zm[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t r = i0 + k * 256;
    w[k] = r < R ? pw[r] : 1u;
    zm[k] = __ballot(r >= 1 && r < R && (w[k] & kPendMask) == 0);
    if (lane == 0) start[k][wave] = (uint32_t)__popcll(zm[k]);
  }
  __syncthreads();
  if (wave == 0) {  // exclusive scan of the 64 counts in (k, wave) order = rule-id order
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
    if ((zm[k] >> lane) & 1) {
      const uint32_t pos = start[k][wave] + (uint32_t)__popcll(zm[k] & lanes_below());
      if (qw) qw[pos] = w[k] >> kPendBits;
      out[pos] = (int32_t)(i0 + k * 256);
    }
}

// The level walk (one cooperative launch, one 1024-thread workgroup per CU).
// Level d is level_rule[lo, hi). Every rule p of the level adds its (final)
// weight to each sub-rule occurrence and retires one pending in-edge of it;
// a sub-rule whose last in-edge retires joins level d+1.
//  - Contributions to the same sub-rule are first merged per workgroup in an
//    LDS hash table (sub-rule -> weight sum, edge count) and applied with one
//    pair of global atomics per table entry at the end of the level, so a
//    sub-rule used by thousands of parents does not serialize thousands of
//    atomics on one address. When the probe sequence is full the occurrence
//    goes straight to global memory.
//  - New members of level d+1 are gathered per workgroup in LDS and appended
//    with one global atomic per workgroup, after hi; the count of level d+1
//    lives in level_cnt[d+1] and is stable once the grid barrier has passed.
// The same walk sums weight x (words in body) over the non-root rules.
constexpr int kLevelThreads = 1024;
constexpr int kLevelList = 8192;
constexpr int kAggBits = 12;
constexpr int kAggSlots = 1 << kAggBits;
constexpr int kAggProbes = 8;
constexpr int kLongList = 4 * kLevelThreads;   // rules per workgroup and sub-round of a level

struct LevelLds {
  int32_t list[kLevelList];
  union {
    struct {  // atomic mode: merge table
      int32_t key[kAggSlots];
      uint64_t wsum[kAggSlots];
      uint32_t cnt[kAggSlots];
    } agg;
    struct {  // bucketed mode, reduce: dense sums of one bucket
      uint64_t wsum[kWideBucket];
      uint32_t cnt[kWideBucket];
    } dense;
    uint32_t hist[kWideMaxBuckets];  // bucketed mode, scatter: per-bucket counts, then write cursors
  } u;
  int32_t longs[kLongList];  // rules with long bodies, walked by whole waves
  int32_t list_n, list_base, list_total, nlong;
  uint32_t seg[2];
  uint64_t part[kLevelThreads / 64];
};

// Append c (where `ready`) to the workgroup's list of level d+1; lanes past
// the LDS capacity append directly to the global level list.
__device__ __forceinline__ void level_append(bool ready, int32_t c, LevelLds& L, DevGrammar& g, int32_t* level_cnt,
                                             int32_t d, int32_t hi) {
  const uint64_t mask = __ballot(ready);
  if (!mask) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  const int32_t n = (int32_t)__popcll(mask);
  int32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(&L.list_n, n);
  base = __shfl(base, leader);
  const int32_t at = base + (int32_t)__popcll(mask & lanes_below());
  const bool spill = ready && at >= kLevelList;
  if (ready && !spill) L.list[at] = c;
  if (base + n > kLevelList) {
    const int32_t slot = wave_append(spill, &level_cnt[d + 1]);
    if (spill) g.level_rule[hi + slot] = c;
  }
}

__device__ __forceinline__ bool agg_add(LevelLds& L, int32_t c, uint64_t w) {
  const uint32_t h = ((uint32_t)c * 2654435761u) >> (32 - kAggBits);
#pragma unroll
  for (int p = 0; p < kAggProbes; ++p) {
    const uint32_t slot = (h + p) & (kAggSlots - 1);
    int32_t k = __hip_atomic_load(&L.u.agg.key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == -1) k = atomicCAS(&L.u.agg.key[slot], -1, c);
    if (k == -1 || k == c) {
      if (w) atomicAdd(reinterpret_cast<unsigned long long*>(&L.u.agg.wsum[slot]), (unsigned long long)w);
      atomicAdd(&L.u.agg.cnt[slot], 1u);
      return true;
    }
  }
  return false;
}

// Barrier among the first `nblocks` workgroups of the launch (all of them,
// or the subset that walks the narrower levels; the others have left): a
// counter and a generation word in device memory, zero at launch, touched by
// one thread per workgroup. The block barrier orders the workgroup's writes
// before thread 0's arrival; the arrival is an acquire-release RMW at agent
// scope (it publishes the workgroup's writes, and the last arriver acquires
// everyone's), the last arriver resets the counter and bumps the generation
// with a release RMW, and the others poll the generation with relaxed loads
// (an acquire per poll would invalidate the caches under the working
// workgroups) and acquire once it has moved. Measured on MI355X with 1024
// threads per workgroup: 11 us for 256 workgroups, 2.4 us for 32, against
// 32 us and 5 us for the cooperative-groups grid barrier.
__device__ __forceinline__ void group_barrier(uint32_t* bar, uint32_t nblocks, uint32_t& gen) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t a = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (a == nblocks - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) __builtin_amdgcn_s_sleep(1);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  ++gen;
  __syncthreads();
}


// The workgroup's list of level d+1 goes after hi with one global atomic.
__device__ __forceinline__ void level_list_out(DevGrammar& g, int32_t* level_cnt, LevelLds& L, int32_t d, int32_t hi) {
  __syncthreads();
  const int32_t n_local = L.list_n < kLevelList ? L.list_n : kLevelList;
  if (threadIdx.x == 0) {
    L.list_base = n_local ? atomicAdd(&level_cnt[d + 1], n_local) : 0;
    // the level's size when this workgroup is the only one appending (its
    // spills, if any, were counted before this add)
    L.list_total = n_local ? L.list_base + n_local : 0;
  }
  __syncthreads();
  for (int32_t k = threadIdx.x; k < n_local; k += blockDim.x) g.level_rule[hi + L.list_base + k] = L.list[k];
  if (threadIdx.x == 0) L.list_n = 0;
}

// Walks the bodies of the rules level_rule[lo, hi) shared by `nthreads`
// threads (this one is `tid`), calling op.begin(weight of p), op.sym(s) for
// each body symbol and op.end() per rule. Short bodies are walked by one thread with 8
// symbols loaded at a time; bodies longer than lp.long_body are queued in LDS
// and walked by a whole wave, lanes across the body, so one long rule never
// holds a wave for hundreds of dependent loads. A level is taken in
// sub-rounds of at most kLongList rules per workgroup, so the queue never
// overflows.
template <class Op>
__device__ __forceinline__ void walk_bodies(const DevGrammar& g, LevelLds& L, int32_t lo, int32_t hi, int64_t tid,
                                            int64_t nthreads, int32_t long_body, Op& op) {
  const int64_t span = (int64_t)(kLongList / kLevelThreads) * nthreads;
  for (int64_t base = lo; base < hi; base += span) {
    const int64_t end = base + span < hi ? base + span : hi;
    for (int64_t i = base + tid; i < end; i += nthreads) {
      const int32_t p = g.level_rule[i];
      const int64_t a = g.rule_off[p], e = g.rule_off[p + 1];
      const uint64_t wp = g.w[p] >> kPendBits;  // final (no pending in-edge); issued with the offsets
      if (e - a > long_body) {
        L.longs[atomicAdd(&L.nlong, 1)] = p;
        continue;
      }
      op.begin(wp);
      for (int64_t q0 = a; q0 < e; q0 += 8) {
        int32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = q0 + k < e ? g.sym[q0 + k] : 0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (q0 + k < e) op.sym(v[k]);
      }
      op.end();
    }
    __syncthreads();
    const int nl = L.nlong;
    for (int j = threadIdx.x >> 6; j < nl; j += kLevelThreads >> 6) {
      const int32_t p = L.longs[j];
      const int64_t e = g.rule_off[p + 1];
      op.begin(g.w[p] >> kPendBits);
      int64_t q = g.rule_off[p] + lane_id();
      int32_t cur = q < e ? g.sym[q] : 0;
      for (; q < e; q += 64) {
        const int32_t nxt = q + 64 < e ? g.sym[q + 64] : 0;  // next load in flight while this one is used
        op.sym(cur);
        cur = nxt;
      }
      op.end();
    }
    __syncthreads();
    if (threadIdx.x == 0) L.nlong = 0;
    __syncthreads();
  }
}

// Per-symbol work of the atomic mode: the referencing rule's weight goes to
// the sub-rule (merged in LDS when possible) and one of its in-edges
// retires; a sub-rule whose last in-edge retires joins level d+1.
// Adds weight dw and retires dn in-edges of rule c (one packed atomic);
// true when these were its last pending in-edges. A weight carried past the
// packed field sets ST_PACK.
__device__ __forceinline__ bool retire(uint64_t* w, int32_t c, uint64_t dw, uint32_t dn, uint32_t* status) {
  const uint64_t old = atomicAdd(reinterpret_cast<unsigned long long*>(&w[c]),
                                 (unsigned long long)((dw << kPendBits) - dn));
  if ((old >> kPendBits) + dw >= (1ull << kWeightBits)) atomicOr(status, (uint32_t)ST_PACK);
  return (old & kPendMask) == dn;
}

struct AtomicOp {
  DevGrammar& g;
  uint32_t* status;
  int32_t* level_cnt;
  LevelLds& L;
  int32_t d, hi;
  uint64_t& tokens;
  uint64_t wp = 0, words = 0;
  __device__ void begin(uint64_t w) { wp = w, words = 0; }
  __device__ void sym(int32_t s) {
    bool ready = false;
    int32_t c = 0;
    if (s >= 0) {
      ++words;
    } else if (-(int64_t)s < g.R) {
      // out-of-range ids are reported by the scan and never touched here
      c = (int32_t)(-(int64_t)s);
      if (!agg_add(L, c, wp)) ready = retire(g.w, c, wp, 1u, status);
    }
    level_append(ready, c, L, g, level_cnt, d, hi);
  }
  __device__ void end() { tokens += wp * words; }
};

// One level in the atomic mode: rules level_rule[lo, hi) processed by
// `nthreads` threads (this one is `tid`); new members of level d+1 are
// appended after hi.
__device__ __forceinline__ void level_round(DevGrammar& g, const LevelParams& lp, uint32_t* status, int32_t* level_cnt,
                                            LevelLds& L, int32_t lo, int32_t hi, int32_t d, int64_t tid,
                                            int64_t nthreads, uint64_t& tokens) {
  AtomicOp op{g, status, level_cnt, L, d, hi, tokens};
  walk_bodies(g, L, lo, hi, tid, nthreads, lp.long_body, op);
  // apply the merged contributions: all of the thread's atomics are issued
  // before any result is used, so their round trips overlap
  constexpr int kPer = kAggSlots / kLevelThreads;
  int32_t cs[kPer];
  bool ready[kPer];
#pragma unroll
  for (int x = 0; x < kPer; ++x) {
    const int slot = (int)threadIdx.x + x * kLevelThreads;
    cs[x] = L.u.agg.key[slot];
    ready[x] = false;
    if (cs[x] >= 0) {
      ready[x] = retire(g.w, cs[x], L.u.agg.wsum[slot], L.u.agg.cnt[slot], status);
      L.u.agg.key[slot] = -1;
      L.u.agg.wsum[slot] = 0;
      L.u.agg.cnt[slot] = 0;
    }
  }
#pragma unroll
  for (int x = 0; x < kPer; ++x) level_append(ready[x], cs[x], L, g, level_cnt, d, hi);
  level_list_out(g, level_cnt, L, d, hi);
}

// Empty merge table (its LDS is shared with the bucketed mode).
__device__ __forceinline__ void agg_reset(LevelLds& L) {
  for (int i = threadIdx.x; i < kAggSlots; i += blockDim.x) L.u.agg.key[i] = -1, L.u.agg.wsum[i] = 0, L.u.agg.cnt[i] = 0;
  __syncthreads();
}

// Bucketed mode, first half of a wide level: every reference in the bodies
// of level_rule[lo, hi) becomes an entry (weight of the referencing rule,
// slot of the referenced rule in its bucket) in its bucket's region. The
// workgroup counts its references per bucket in LDS, reserves each bucket's
// share with one global atomic, then writes its entries. Buckets interleave
// the rule ids (bucket = id mod nbk, slot = id / nbk, nbk a power of two):
// rules referenced most often tend to have nearby ids (Sequitur numbers rules
// by first use), and interleaving spreads them over all buckets, so the
// per-bucket reduce is balanced (on the 10^8-token corpus the largest bucket
// of the widest level holds 3x the mean instead of 40x).
struct CountOp {  // bucketed mode, first pass: references per bucket, tokens
  const DevGrammar& g;
  LevelLds& L;
  uint64_t& tokens;
  uint32_t mask;  // nbk - 1
  uint64_t wp = 0, words = 0;
  __device__ void begin(uint64_t w) { wp = w, words = 0; }
  __device__ void sym(int32_t s) {
    if (s >= 0) ++words;
    else if (-(int64_t)s < g.R) atomicAdd(&L.u.hist[(uint32_t)(-(int64_t)s) & mask], 1u);
  }
  __device__ void end() { tokens += wp * words; }
};

struct WriteOp {  // bucketed mode, second pass: one entry per reference
  const DevGrammar& g;
  const WideBufs& wb;
  LevelLds& L;
  uint64_t wp = 0;
  __device__ void begin(uint64_t w) { wp = w; }
  __device__ void sym(int32_t s) {
    if (s < 0 && -(int64_t)s < g.R) {
      const uint32_t c = (uint32_t)(-(int64_t)s);
      const uint32_t at = atomicAdd(&L.u.hist[c & (uint32_t)(wb.nbk - 1)], 1u);
      wb.ew[at] = wp;
      wb.ec[at] = (uint16_t)(c >> wb.nbk_bits);
    }
  }
  __device__ void end() {}
};

__device__ __forceinline__ void wide_scatter(DevGrammar& g, const LevelParams& lp, const WideBufs& wb, LevelLds& L,
                                             int32_t lo, int32_t hi, int64_t tid, int64_t nthreads, uint64_t& tokens) {
  for (int k = threadIdx.x; k < wb.nbk; k += blockDim.x) L.u.hist[k] = 0;
  __syncthreads();
  CountOp count{g, L, tokens, (uint32_t)(wb.nbk - 1)};
  walk_bodies(g, L, lo, hi, tid, nthreads, lp.long_body, count);
  for (int k = threadIdx.x; k < wb.nbk; k += blockDim.x) {
    const uint32_t h = L.u.hist[k];
    if (h) L.u.hist[k] = atomicAdd(&wb.cur[k], h);
  }
  __syncthreads();
  WriteOp write{g, wb, L};
  walk_bodies(g, L, lo, hi, tid, nthreads, lp.long_body, write);
}

// Bucketed mode, second half: each bucket's new entries are summed in a
// dense LDS table (one slot per rule of the bucket) by the one workgroup that
// owns the bucket, which then applies weight and retired in-edges to every
// referenced rule with plain read-modify-writes (no other workgroup touches
// the bucket's rules) and lists the rules whose last in-edge retired.
__device__ __forceinline__ void wide_reduce(DevGrammar& g, uint32_t* status, int32_t* level_cnt, const WideBufs& wb,
                                            LevelLds& L, int32_t d, int32_t hi) {
  for (int32_t b = blockIdx.x; b < wb.nbk; b += gridDim.x) {
    if (threadIdx.x == 0) L.seg[0] = wb.seg_lo[b], L.seg[1] = wb.cur[b];
    __syncthreads();
    const uint32_t s0 = L.seg[0], s1 = L.seg[1];
    if (s0 != s1) {
      for (int k = threadIdx.x; k < wb.slots; k += blockDim.x) L.u.dense.wsum[k] = 0, L.u.dense.cnt[k] = 0;
      __syncthreads();
      for (uint32_t e = s0 + threadIdx.x; e < s1; e += blockDim.x) {
        const uint32_t k = wb.ec[e];
        const uint64_t wv = wb.ew[e];
        if (wv) atomicAdd(reinterpret_cast<unsigned long long*>(&L.u.dense.wsum[k]), (unsigned long long)wv);
        atomicAdd(&L.u.dense.cnt[k], 1u);
      }
      __syncthreads();
      for (int k0 = 0; k0 < wb.slots; k0 += kLevelThreads) {  // uniform trip count: level_append is wave-collective
        const int k = k0 + (int)threadIdx.x;
        const uint32_t n = k < wb.slots ? L.u.dense.cnt[k] : 0u;
        const int32_t c = (int32_t)(((uint32_t)k << wb.nbk_bits) | (uint32_t)b);
        bool ready = false;
        if (n) {
          const uint64_t old = g.w[c], dw = L.u.dense.wsum[k];
          const uint64_t now = old + ((dw << kPendBits) - n);
          if ((old >> kPendBits) + dw >= (1ull << kWeightBits)) atomicOr(status, (uint32_t)ST_PACK);
          g.w[c] = now;
          ready = (now & kPendMask) == 0;
        }
        level_append(ready, c, L, g, level_cnt, d, hi);
      }
      if (threadIdx.x == 0) wb.seg_lo[b] = s1;
    }
    __syncthreads();
  }
  level_list_out(g, level_cnt, L, d, hi);
}

// Levels narrower than this finish on workgroup 0 alone (block barriers
// instead of grid barriers); the other workgroups leave.

__global__ __launch_bounds__(kLevelThreads) void k_levels(DevGrammar g, int32_t* level_cnt, LoadCounters* lc,
                                                          WideBufs wb, LevelParams lp, uint32_t* bar) {
  uint32_t* status = &lc->status;
  __shared__ LevelLds L;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  int32_t lo = 0;
  int32_t hi = (int32_t)__hip_atomic_load(&lc->frontier0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int32_t d = 1;
  uint64_t tokens = 0;
  if (threadIdx.x == 0) L.list_n = 0, L.nlong = 0;
  agg_reset(L);
  bool agg_clean = true;
  uint32_t gen = 0;  // barrier generation (the barrier words are zero at launch)
  // wide levels: the whole grid, a grid barrier between levels
  const bool shrink = gridDim.x > (unsigned)lp.mid_blocks;
  while (lo < hi && (hi - lo >= (shrink ? lp.mid_rules : lp.tail_rules) || gridDim.x == 1)) {
    if (wb.ew && hi - lo >= wb.min_rules) {
      wide_scatter(g, lp, wb, L, lo, hi, tid, nthreads, tokens);
      group_barrier(bar, gridDim.x, gen);
      wide_reduce(g, status, level_cnt, wb, L, d, hi);
      agg_clean = false;
    } else {
      if (!agg_clean) agg_reset(L), agg_clean = true;
      level_round(g, lp, status, level_cnt, L, lo, hi, d, tid, nthreads, tokens);
    }
    group_barrier(bar, gridDim.x, gen);
    const int32_t next = __hip_atomic_load(&level_cnt[d + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) {
      g.level_off[d] = lo;
      g.level_off[d + 1] = hi;
    }
    lo = hi;
    hi += next;
    ++d;
  }
  // mid levels: the first lp.mid_blocks workgroups, the others leave
  if (shrink && blockIdx.x < (unsigned)lp.mid_blocks) {
    if (!agg_clean) agg_reset(L), agg_clean = true;
    const int64_t mtid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t mthreads = (int64_t)lp.mid_blocks * blockDim.x;
    while (lo < hi && hi - lo >= lp.tail_rules) {
      level_round(g, lp, status, level_cnt, L, lo, hi, d, mtid, mthreads, tokens);
      group_barrier(bar, (uint32_t)lp.mid_blocks, gen);
      const int32_t next = __hip_atomic_load(&level_cnt[d + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (mtid == 0) {
        g.level_off[d] = lo;
        g.level_off[d + 1] = hi;
      }
      lo = hi;
      hi += next;
      ++d;
    }
  }
  // narrow levels: workgroup 0 alone
  if (blockIdx.x == 0) {
    if (!agg_clean) agg_reset(L);
    while (lo < hi) {
      // one workgroup: the block barriers inside the round order its global
      // writes (level list, weights, pending counts) for the next round
      level_round(g, lp, status, level_cnt, L, lo, hi, d, threadIdx.x, blockDim.x, tokens);
      __syncthreads();
      const int32_t next = L.list_total;
      if (threadIdx.x == 0) {
        g.level_off[d] = lo;
        g.level_off[d + 1] = hi;
      }
      __syncthreads();
      lo = hi;
      hi += next;
      ++d;
    }
  }
  // block sum of the token contributions, one atomic per block
  tokens = wave_sum_u64(tokens);
  if (lane_id() == 0) L.part[threadIdx.x >> 6] = tokens;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t sum = 0;
    for (int w = 0; w < kLevelThreads / 64; ++w) sum += L.part[w];
    if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(&lc->tokens), (unsigned long long)sum);
  }
  if (tid == 0) {
    lc->depth = d - 1;
    lc->placed = hi;
  }
}

hipError_t launch_level_frontier(const DevGrammar& g, LoadCounters* lc, uint32_t* scratch, hipStream_t s,
                                 uint64_t* qw, FlowState* fs) {
  // level 1 by compaction (scratch: per-block counts, then the scan's block sums)
  const int64_t nb = (g.R + kRadixTile - 1) / kRadixTile;
  k_zero_count<<<(unsigned)nb, 256, 0, s>>>(g.w, g.R, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_u32(scratch, nb, &lc->frontier0, scratch + nb, s);
  if (e != hipSuccess) return e;
  k_zero_write<<<(unsigned)(nb > 0 ? nb : 1), 256, 0, s>>>(g.w, g.R, scratch, g.level_rule, qw, fs, &lc->frontier0);
  return hipGetLastError();
}

// Capacity of every bucket of the bucketed mode: the pending in-edges of its
// rules (bucket = id mod nbk). Each block sums a range of kCapRules rules
// into an LDS table by bucket, then adds it to the (zeroed) capacities.
constexpr int kCapRules = 65536;
__global__ __launch_bounds__(1024) void k_wide_caps(const uint64_t* pw, int64_t R, uint32_t* cap, int nbk) {
  __shared__ uint32_t h[kWideMaxBuckets];
  for (int k = threadIdx.x; k < nbk; k += blockDim.x) h[k] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kCapRules;
  for (int k = threadIdx.x; k < kCapRules; k += blockDim.x) {
    const int64_t c = base + k;
    const uint32_t p = c < R ? (uint32_t)(pw[c] & kPendMask) : 0u;
    if (p) atomicAdd(&h[c & (nbk - 1)], p);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nbk; k += blockDim.x)
    if (h[k]) atomicAdd(&cap[k], h[k]);
}

// The barrier words of the shrinking phase: 2 words after the frontier scan's scratch.
static uint32_t* level_barrier_words(const DevGrammar& g, uint32_t* scratch) {
  const int64_t nb = (g.R + kRadixTile - 1) / kRadixTile;
  return scratch + nb + scan_sums_entries(nb);
}

hipError_t prepare_level_walk(const DevGrammar& g, LoadCounters* lc, uint32_t* scratch, const WideBufs& wide,
                              hipStream_t s) {
  const WideBufs& wb = wide;
  if (wb.ew) {
    // bucket regions: exclusive scan of the capacities; both cursors start there
    hipError_t e0 = launch_fill_i32(reinterpret_cast<int32_t*>(wb.cur), wb.nbk, 0, s);
    if (e0 != hipSuccess) return e0;
    k_wide_caps<<<(unsigned)((g.R + kCapRules - 1) / kCapRules), 1024, 0, s>>>(g.w, g.R, wb.cur, wb.nbk);
    e0 = hipGetLastError();
    if (e0 == hipSuccess) e0 = launch_scan_u32(wb.cur, wb.nbk, &lc->wide_entries, scratch, s);
    if (e0 == hipSuccess)
      e0 = hipMemcpyAsync(wb.seg_lo, wb.cur, sizeof(uint32_t) * wb.nbk, hipMemcpyDeviceToDevice, s);
    if (e0 != hipSuccess) return e0;
  }
  return launch_fill_i32(reinterpret_cast<int32_t*>(level_barrier_words(g, scratch)), 2, 0, s);
}

hipError_t launch_level_walk(const DevGrammar& g, int32_t* level_cnt, LoadCounters* lc, uint32_t* scratch,
                             const WideBufs& wide, const LevelParams& params, int device, hipStream_t s) {
  WideBufs wb = wide;
  int per_cu = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_levels), kLevelThreads, 0);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int64_t want = (g.R + kLevelThreads - 1) / kLevelThreads;
  const int64_t cap = cus;  // one workgroup per CU: few participants in every grid barrier
  const unsigned grid = (unsigned)(want < 1 ? 1 : (want < cap ? want : cap));
  DevGrammar gg = g;
  uint32_t* bar = level_barrier_words(g, scratch);
  LevelParams lp = params;
  if (lp.mid_blocks < 1) lp.mid_blocks = 1;
  if (lp.tail_rules < 1) lp.tail_rules = 1;
  void* args[] = {&gg, &level_cnt, &lc, &wb, &lp, &bar};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_levels), dim3(grid), dim3(kLevelThreads), args, 0,
                                    s);
}

}  // namespace gt

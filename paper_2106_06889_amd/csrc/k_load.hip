// k_load.hip -- initialization phase of a grammar on the GPU: validation, the
// tile table of the position-parallel passes, rule in-degrees, level-by-level
// topological frontiers and top-down rule weights.
//
// Paper: Section "Overview" (initialization phase, then graph traversal);
// Algorithm "Top-Down Traversal" (mask initialization from the in-edges that
// do not come from the root, initial weights = frequencies in the root, then
// rounds in which every ready rule adds frequency x weight to its sub-rules
// and a sub-rule becomes ready when all its in-edges have arrived).
//
// Differences from the paper's design (same results): the rounds are not
// relaunched from the host until a stop flag stays set. One cooperative
// launch walks the levels with a grid barrier between them, and each level's
// ready rules are compacted into a frontier list (wave ballot + one atomic per
// wave), so a round touches only the rules of that level rather than scanning
// every rule's mask. In-degrees count occurrences (a rule used twice by the
// same parent waits for both), which gives the same levels and weights.
#include <hip/hip_cooperative_groups.h>

#include "device.h"

namespace cg = cooperative_groups;

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
  if (r == 0) return;
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

// Position-parallel scan of every body: symbol ranges, word totals, and the
// in-edges of the top-down traversal. An occurrence of c in the root adds 1
// to c's initial weight (its frequency in the root); an occurrence in any
// other body adds 1 to c's count of pending in-edges.
__global__ __launch_bounds__(kTileThreads) void k_scan_symbols(DevGrammar g, int32_t* pend, LoadCounters* lc) {
  __shared__ int32_t roff[kTileRuleSlots];
  const Tile t = tile_begin(g, blockIdx.x, roff);
  const int32_t q0 = threadIdx.x * kPerThread;
  int32_t v[kPerThread];
  tile_load_syms(g, t, q0, v);
  uint32_t bad = 0;
  uint64_t words = 0, root_words = 0;
  if (q0 < t.len) {
    int32_t j = tile_find(roff, t.nr, q0);
    int32_t next = roff[j + 1];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int32_t q = q0 + k;
      if (q >= t.len) break;
      while (q >= next) next = roff[++j + 1];
      const int32_t r = t.r0 + j;
      const int32_t s = v[k];
      if (s >= 0) {
        if (s >= g.V) {
          bad |= ST_BAD_WORD;
        } else {
          ++words;
          root_words += (r == 0);
        }
      } else {
        const int64_t c = -(int64_t)s;
        if (c >= g.R) bad |= ST_BAD_REF;
        else if (r == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&g.w[c]), 1ull);
        else atomicAdd(&pend[c], 1);
      }
    }
  }
  words = wave_sum_u64(words);
  root_words = wave_sum_u64(root_words);
  if (lane_id() == 0) {
    if (words) atomicAdd(reinterpret_cast<unsigned long long*>(&lc->word_syms), (unsigned long long)words);
    if (root_words) atomicAdd(reinterpret_cast<unsigned long long*>(&lc->root_words), (unsigned long long)root_words);
  }
  if (bad) atomicOr(&lc->status, bad);
}

hipError_t launch_scan_symbols(const DevGrammar& g, int32_t* pend, LoadCounters* lc, hipStream_t s) {
  if (g.ntiles == 0) return hipSuccess;
  k_scan_symbols<<<(unsigned)g.ntiles, kTileThreads, 0, s>>>(g, pend, lc);
  return hipGetLastError();
}

// Level 1: the rules with no pending in-edge (used only by the root, or not
// at all). Also sets the root's weight to 1.
__global__ void k_frontier0(DevGrammar g, const int32_t* pend, int32_t* level_cnt) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c == 0) g.w[0] = 1;
  const bool ready = c >= 1 && c < g.R && pend[c] == 0;
  const int32_t slot = wave_append(ready, &level_cnt[1]);
  if (ready) g.level_rule[slot] = (int32_t)c;
}

// The level walk (one cooperative launch). Level d is level_rule[lo, hi).
// Every rule p of the level adds its (final) weight to each sub-rule
// occurrence and retires one pending in-edge of it; a sub-rule whose last
// in-edge retires joins level d+1, appended after hi. Counts of level d+1
// go to level_cnt[d+1], so they are stable once the grid barrier has passed.
// The same walk sums weight x (words in body) over the non-root rules, the
// number of words they contribute to the text.
__global__ __launch_bounds__(256) void k_levels(DevGrammar g, int32_t* pend, int32_t* level_cnt, LoadCounters* lc) {
  cg::grid_group grid = cg::this_grid();
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  int32_t lo = 0;
  int32_t hi = __hip_atomic_load(&level_cnt[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int32_t d = 1;
  uint64_t tokens = 0;
  while (lo < hi) {
    for (int64_t i = lo + tid; i < hi; i += nthreads) {
      const int32_t p = g.level_rule[i];
      const uint64_t wp = g.w[p];
      const int64_t e = g.rule_off[p + 1];
      uint64_t words = 0;
      for (int64_t q = g.rule_off[p]; q < e; ++q) {
        const int32_t s = g.sym[q];
        bool ready = false;
        int32_t c = 0;
        if (s >= 0) {
          ++words;
        } else {
          c = -s;
          if (c < g.R) {  // out-of-range ids are reported by the scan; never touched here
            if (wp) atomicAdd(reinterpret_cast<unsigned long long*>(&g.w[c]), (unsigned long long)wp);
            ready = atomicSub(&pend[c], 1) == 1;
          }
        }
        const int32_t slot = wave_append(ready, &level_cnt[d + 1]);
        if (ready) g.level_rule[hi + slot] = c;
      }
      tokens += wp * words;
    }
    grid.sync();
    const int32_t next = __hip_atomic_load(&level_cnt[d + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) {
      g.level_off[d] = lo;
      g.level_off[d + 1] = hi;
    }
    lo = hi;
    hi += next;
    ++d;
  }
  // block sum of the token contributions, one atomic per block
  __shared__ uint64_t part[4];
  tokens = wave_sum_u64(tokens);
  if (lane_id() == 0) part[threadIdx.x >> 6] = tokens;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t sum = part[0] + part[1] + part[2] + part[3];
    if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(&lc->tokens), (unsigned long long)sum);
  }
  if (tid == 0) {
    lc->depth = d - 1;
    lc->placed = hi;
  }
}

hipError_t launch_levels(const DevGrammar& g, int32_t* pend, int32_t* level_cnt, LoadCounters* lc, int device,
                         hipStream_t s) {
  k_frontier0<<<(unsigned)((g.R + 255) / 256), 256, 0, s>>>(g, pend, level_cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int per_cu = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_levels), 256, 0);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  int64_t want = (g.R + 255) / 256;
  int64_t cap = (int64_t)per_cu * cus;
  if (cap > 4 * (int64_t)cus) cap = 4 * (int64_t)cus;  // enough waves for the widest level
  const unsigned grid = (unsigned)(want < 1 ? 1 : (want < cap ? want : cap));
  DevGrammar gg = g;
  void* args[] = {&gg, &pend, &level_cnt, &lc};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_levels), dim3(grid), dim3(256), args, 0, s);
}

}  // namespace gt

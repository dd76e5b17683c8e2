// device.h -- device-side helpers shared by the kernels (wave64 primitives and
// the tile machinery of the position-parallel passes).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace gt {

__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

// Append the active lanes whose `want` is set to a list whose length lives in
// *counter: one atomic per wave, slots in lane order. Returns the slot of the
// calling lane (meaningful only where want is true).
__device__ __forceinline__ int32_t wave_append(bool want, int32_t* counter) {
  const uint64_t mask = __ballot(want);
  if (mask == 0) return 0;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  int32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, (int32_t)__popcll(mask));
  base = __shfl(base, leader);
  return base + (int32_t)__popcll(mask & lanes_below());
}

// Sum of a value over the active lanes of the wave, returned to all of them.
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One tile of a position-parallel pass: symbols [a, a + len) and the rules
// r0 .. r0+nr-1 that overlap them. roff (LDS) holds the rule boundaries
// relative to a, clamped to [0, kTileSyms]: rule r0+j covers tile positions
// [roff[j], roff[j+1]).
typedef int32_t v4i32 __attribute__((ext_vector_type(4)));

struct Tile {
  int64_t a;
  int32_t len;
  int32_t r0;
  int32_t nr;
};

__device__ __forceinline__ Tile tile_begin(const DevGrammar& g, int64_t tile, int32_t* roff) {
  Tile t;
  t.a = tile * (int64_t)kTileSyms;
  const int64_t rem = g.S - t.a;
  t.len = (int32_t)(rem < kTileSyms ? rem : kTileSyms);
  t.r0 = g.tile_rule[tile];
  const int32_t r1 = g.tile_rule[tile + 1];
  t.nr = r1 - t.r0 + 1;
  for (int j = threadIdx.x; j <= t.nr; j += blockDim.x) {
    int64_t o = g.rule_off[t.r0 + j] - t.a;
    o = o < 0 ? 0 : (o > kTileSyms ? kTileSyms : o);
    roff[j] = (int32_t)o;
  }
  __syncthreads();
  return t;
}

// Index j of the rule holding tile position q: the largest j with roff[j] <= q
// (empty rules are skipped because the next boundary equals theirs).
__device__ __forceinline__ int32_t tile_find(const int32_t* roff, int32_t nr, int32_t q) {
  int32_t lo = 0, hi = nr - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (roff[mid] <= q) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The kPerThread consecutive symbols of the calling thread, from global
// memory. Positions past the tile's end read as 0 and must be masked by the
// caller (q < t.len).
__device__ __forceinline__ void tile_load_syms(const DevGrammar& g, const Tile& t, int32_t q0, int32_t (&v)[kPerThread]) {
  const int32_t* p = g.sym + t.a + q0;
  if (q0 + kPerThread <= t.len) {
    const v4i32* p4 = reinterpret_cast<const v4i32*>(p);
#pragma unroll
    for (int k = 0; k < kPerThread / 4; ++k) {
      const v4i32 x = __builtin_nontemporal_load(p4 + k);
      v[4 * k + 0] = x.x;
      v[4 * k + 1] = x.y;
      v[4 * k + 2] = x.z;
      v[4 * k + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) v[k] = (q0 + k < t.len) ? p[k] : 0;
  }
}

}  // namespace gt

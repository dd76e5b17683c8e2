// k_wordcount.hip -- word count by one position-parallel pass over all rule
// bodies.
//
// Paper: Background, "TADOC" (word-count walk-through: every rule's local
// word frequencies reach the root scaled by how often the rule is used);
// Algorithm "Top-Down Traversal", reduce step (the words of every rule,
// multiplied by the rule's accumulated weight, merged into the global table).
//
// The paper gives each rule a thread and the long root a thread group. Here
// the bodies of all rules, root included, are cut into fixed tiles of
// consecutive symbols, so the work is balanced whatever the rule lengths, and
// the symbols stream through with 16-byte loads. counts[w] += weight(rule) for
// every word symbol w of the rule's body.
#include "device.h"

namespace gt {

__global__ __launch_bounds__(kTileThreads) void k_word_count(DevGrammar g, uint64_t* counts) {
  __shared__ int32_t roff[kTileRuleSlots];
  const Tile t = tile_begin(g, blockIdx.x, roff);
  const int32_t q0 = threadIdx.x * kPerThread;
  if (q0 >= t.len) return;
  int32_t v[kPerThread];
  tile_load_syms(g, t, q0, v);
  int32_t j = tile_find(roff, t.nr, q0);
  int32_t next = roff[j + 1];
  uint64_t wr = g.w[t.r0 + j];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int32_t q = q0 + k;
    if (q >= t.len) break;
    if (q >= next) {
      while (q >= next) next = roff[++j + 1];
      wr = g.w[t.r0 + j];
    }
    const int32_t s = v[k];
    if (s >= 0 && wr != 0) atomicAdd(reinterpret_cast<unsigned long long*>(&counts[s]), (unsigned long long)wr);
  }
}

hipError_t launch_word_count(const DevGrammar& g, uint64_t* counts, hipStream_t s) {
  hipError_t e = launch_fill_u64(counts, g.V, 0, s);
  if (e != hipSuccess || g.ntiles == 0) return e;
  k_word_count<<<(unsigned)g.ntiles, kTileThreads, 0, s>>>(g, counts);
  return hipGetLastError();
}

}  // namespace gt

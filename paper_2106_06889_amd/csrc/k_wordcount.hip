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
//
// Global atomics on the count array would serialize on frequent words, so
// the sums are formed on chip instead: a scatter pass writes one packed entry
// (weight << 12 | low 12 bits of the word id) per word symbol into the
// bucket of its word id (4096 ids per bucket), at offsets fixed by the
// per-block bucket histogram taken at load; a reduce pass then sums the
// entries in dense LDS tables and adds the sums to the counts with
// coalesced atomics. k_word_count (direct atomics) remains for vocabularies
// too large for the bucket table.
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

// Scatter: one workgroup per block of kSubTiles tiles. LDS holds the block's
// write cursor per bucket, starting at its offset from the load-time scan.
__global__ __launch_bounds__(kTileThreads) void k_wc_scatter(DevGrammar g, uint64_t* entries) {
  extern __shared__ int32_t lds_wc[];
  int32_t* roff = lds_wc;
  uint32_t* cursor = reinterpret_cast<uint32_t*>(lds_wc + kTileRuleSlots);
  const int64_t slot = xcd_slot(blockIdx.x, g.nslot);
  for (int b = threadIdx.x; b < g.wc_nb; b += blockDim.x) cursor[b] = g.wc_off[(int64_t)b * g.nslot + slot];
  for (int sub = 0; sub < kSubTiles; ++sub) {
    const int64_t tile = (int64_t)blockIdx.x * kSubTiles + sub;
    if (tile >= g.ntiles) break;  // uniform for the block
    const Tile t = tile_begin(g, tile, roff);
    const int32_t q0 = threadIdx.x * kPerThread;
    if (q0 < t.len) {
      int32_t v[kPerThread];
      tile_load_syms(g, t, q0, v);
      int32_t j = tile_find(roff, t.nr, q0);
      int32_t next = roff[j + 1];
      uint64_t wr = g.w[t.r0 + j];
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        const int32_t q = q0 + k;
        if (q >= t.len) continue;
        if (q >= next) {
          while (q >= next) next = roff[++j + 1];
          wr = g.w[t.r0 + j];
        }
        const int32_t s = v[k];
        if (s >= 0) {
          const uint32_t at = atomicAdd(&cursor[s >> kWcBits], 1u);
          entries[at] = (wr << kWcBits) | (uint64_t)(s & (kWcBucket - 1));
        }
      }
    }
    __syncthreads();  // roff is rewritten by the next tile
  }
}

// Reduce: the entry array is cut into chunks of kWcChunk entries (bucket
// sizes follow the word frequencies, so whole buckets per workgroup would
// leave a few workgroups with most of the work). A workgroup sums each
// bucket segment of its chunk in LDS -- kWcCopies copies of the bucket's
// table, wave w using copy w % kWcCopies, so one frequent word's adds spread
// over several addresses -- then adds the nonzero sums to the (zeroed) count
// array with coalesced global atomics.
constexpr int kWcCopies = 4;
constexpr int kWcThreads = 1024;
constexpr int64_t kWcChunk = 32 * kWcThreads;

// First bucket whose range [start(b), start(b+1)) holds entry i; start(b) =
// off[b * nslot], start(nb) = n.
__device__ __forceinline__ int bucket_of(const uint32_t* off, int64_t nslot, int nb, int64_t n, int64_t i) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)off[(int64_t)mid * nslot] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kWcThreads) void k_wc_reduce(DevGrammar g, const uint64_t* entries, int64_t W,
                                                          uint64_t* counts) {
  __shared__ uint64_t acc[kWcCopies][kWcBucket];
  __shared__ int first_bucket;
  for (int i = threadIdx.x; i < kWcCopies * kWcBucket; i += blockDim.x) (&acc[0][0])[i] = 0;
  const int64_t c_lo = (int64_t)blockIdx.x * kWcChunk;
  const int64_t c_hi = c_lo + kWcChunk < W ? c_lo + kWcChunk : W;
  if (threadIdx.x == 0) first_bucket = bucket_of(g.wc_off, g.nslot, g.wc_nb, W, c_lo);
  __syncthreads();
  uint64_t* mine = acc[(threadIdx.x >> 6) % kWcCopies];
  for (int b = first_bucket; b < g.wc_nb; ++b) {
    const int64_t b_lo = g.wc_off[(int64_t)b * g.nslot];
    const int64_t b_hi = (b + 1 < g.wc_nb) ? (int64_t)g.wc_off[(int64_t)(b + 1) * g.nslot] : W;
    if (b_lo >= c_hi) break;
    const int64_t lo = b_lo > c_lo ? b_lo : c_lo, hi = b_hi < c_hi ? b_hi : c_hi;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const uint64_t e = __builtin_nontemporal_load(entries + i);
      atomicAdd(reinterpret_cast<unsigned long long*>(&mine[e & (kWcBucket - 1)]), (unsigned long long)(e >> kWcBits));
    }
    __syncthreads();
    const int64_t base = (int64_t)b * kWcBucket;
    for (int i = threadIdx.x; i < kWcBucket; i += blockDim.x) {
      uint64_t sum = 0;
#pragma unroll
      for (int c = 0; c < kWcCopies; ++c) sum += acc[c][i], acc[c][i] = 0;
      if (sum && base + i < g.V) atomicAdd(reinterpret_cast<unsigned long long*>(&counts[base + i]), (unsigned long long)sum);
    }
    __syncthreads();
  }
}

hipError_t launch_word_count_buckets(const DevGrammar& g, uint64_t* counts, uint64_t* entries, int64_t W,
                                     hipStream_t s) {
  hipError_t e = launch_fill_u64(counts, g.V, 0, s);
  if (e != hipSuccess) return e;
  if (g.ntiles == 0 || W == 0) return hipSuccess;
  const size_t shmem = sizeof(int32_t) * (kTileRuleSlots + g.wc_nb);
  k_wc_scatter<<<(unsigned)g.nblk, kTileThreads, shmem, s>>>(g, entries);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_wc_reduce<<<(unsigned)((W + kWcChunk - 1) / kWcChunk), kWcThreads, 0, s>>>(g, entries, W, counts);
  return hipGetLastError();
}

hipError_t launch_word_count(const DevGrammar& g, uint64_t* counts, hipStream_t s) {
  hipError_t e = launch_fill_u64(counts, g.V, 0, s);
  if (e != hipSuccess || g.ntiles == 0) return e;
  k_word_count<<<(unsigned)g.ntiles, kTileThreads, 0, s>>>(g, counts);
  return hipGetLastError();
}

}  // namespace gt

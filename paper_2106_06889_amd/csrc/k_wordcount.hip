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

// Scatter of block `blk` (kSubTiles tiles of kTileSyms symbols, walked one
// after the other by kWcScatterThreads threads, 4 symbols each). Entries are
// 32-bit: weight << 12 | low 12 bits of the word id, for weights below 2^20;
// a word of a heavier rule (rare: a rule used a million times) adds its
// weight to the count directly and leaves a zero-weight entry. The block's
// entries are staged in LDS grouped by bucket (local offsets from the
// block's bucket counts, known from the load-time histogram), then every
// bucket run is copied to its global position by consecutive lanes, so the
// writes are whole lines instead of one 8-byte store per word.
constexpr int kWcScatterThreads = 1024;
constexpr int kWcSymsPerThread = kTileSyms / kWcScatterThreads;  // 4: one 16-byte load
constexpr uint64_t kWcMaxWeight = 1ull << (32 - kWcBits);

struct WcScatterLds {
  int32_t roff[kTileRuleSlots];
  uint32_t stage[kBlockSyms];
  uint16_t chunk_bucket[kBlockSyms / 64];  // bucket of entry 64k of the staged run
};

// Dynamic LDS after WcScatterLds: cur[nb], lstart[nb], gstart[nb] (uint32).
// kSpan: only the root words inside file g.span_file's span count (weight 1),
// the other root words get weight 0 (the top-down term vector's pass for one
// file); without it every root word has weight 1.
template <bool kSpan>
__device__ __forceinline__ void wc_scatter_block(const DevGrammar& g, int64_t blk, uint32_t* entries, uint64_t* counts,
                                                 WcScatterLds& L, uint32_t* dyn, int64_t W) {
  const int nb = g.wc_nb;
  uint32_t* cur = dyn;
  uint32_t* lstart = dyn + nb;
  uint32_t* gstart = dyn + 2 * nb;
  __shared__ uint32_t red[16];
  const int64_t slot = xcd_slot(blk, g.nslot);
  // the block's bucket counts: differences of consecutive offsets (next slot, or next bucket row)
  uint32_t mine[4], tot4 = 0;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int b = threadIdx.x * 4 + x;
    uint32_t c = 0;
    if (b < nb) {
      const int64_t at = (int64_t)b * g.nslot + slot;
      const uint32_t o = g.wc_off[at];
      const int64_t nxt = slot + 1 < g.nslot ? (int64_t)g.wc_off[at + 1]
                                             : (b + 1 < nb ? (int64_t)g.wc_off[(int64_t)(b + 1) * g.nslot] : W);
      c = (uint32_t)(nxt - o);
      gstart[b] = o;
    }
    mine[x] = c;
    tot4 += c;
  }
  // exclusive scan of the counts over the 1024 threads (16 waves)
  uint32_t x_incl = tot4;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x_incl, o);
    if (lane_id() >= o) x_incl += y;
  }
  if (lane_id() == 63) red[threadIdx.x >> 6] = x_incl;
  __syncthreads();
  uint32_t base = 0, n_block = 0;
#pragma unroll
  for (int w = 0; w < kWcScatterThreads / 64; ++w) {
    if (w < (int)(threadIdx.x >> 6)) base += red[w];
    n_block += red[w];
  }
  base += x_incl - tot4;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int b = threadIdx.x * 4 + x;
    if (b < nb) lstart[b] = base, cur[b] = base;
    base += mine[x];
  }
  int64_t span_lo = 0, span_hi = 0;
  if (kSpan) span_lo = g.file_off[g.span_file], span_hi = g.file_off[g.span_file + 1];
  __syncthreads();
  for (int sub = 0; sub < kSubTiles; ++sub) {
    const int64_t tile = blk * kSubTiles + sub;
    if (tile >= g.ntiles) break;  // uniform for the block
    const Tile t = tile_begin(g, tile, L.roff);
    const int32_t q0 = threadIdx.x * kWcSymsPerThread;
    if (q0 < t.len) {
      int32_t v[kWcSymsPerThread];
      if (q0 + kWcSymsPerThread <= t.len) {
        const v4i32 x4 = __builtin_nontemporal_load(reinterpret_cast<const v4i32*>(g.sym + t.a + q0));
        v[0] = x4.x, v[1] = x4.y, v[2] = x4.z, v[3] = x4.w;
      } else {
#pragma unroll
        for (int k = 0; k < kWcSymsPerThread; ++k) v[k] = q0 + k < t.len ? g.sym[t.a + q0 + k] : 0;
      }
      int32_t j = tile_find(L.roff, t.nr, q0);
      int32_t next = L.roff[j + 1];
      uint64_t wr = g.w[t.r0 + j];
#pragma unroll
      for (int k = 0; k < kWcSymsPerThread; ++k) {
        const int32_t q = q0 + k;
        if (q >= t.len) continue;
        if (q >= next) {
          while (q >= next) next = L.roff[++j + 1];
          wr = g.w[t.r0 + j];
        }
        const int32_t s = v[k];
        if (s >= 0) {
          uint64_t we = wr;
          if (kSpan && t.r0 + j == 0) {
            const int64_t qa = t.a + q;
            we = qa >= span_lo && qa < span_hi ? 1ull : 0ull;
          }
          const uint32_t at = atomicAdd(&cur[s >> kWcBits], 1u);
          const bool light = we < kWcMaxWeight;
          L.stage[at] = (light ? (uint32_t)(we << kWcBits) : 0u) | (uint32_t)(s & (kWcBucket - 1));
          if (!light) atomicAdd(reinterpret_cast<unsigned long long*>(&counts[s]), (unsigned long long)we);
        }
      }
    }
    __syncthreads();  // roff is rewritten by the next tile
  }
  // copy out: the run of bucket b goes to gstart[b] .. ; lanes take consecutive entries.
  // The bucket of entry e is found from the bucket of its 64-entry chunk's
  // first entry, stepping over the few bucket starts inside the chunk
  // (empty buckets share the next start).
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const uint32_t s0 = lstart[b], s1 = b + 1 < nb ? lstart[b + 1] : n_block;
    for (uint32_t k = (s0 + 63) >> 6; (k << 6) < s1; ++k) L.chunk_bucket[k] = (uint16_t)b;
  }
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < n_block; e += blockDim.x) {
    int b = L.chunk_bucket[e >> 6];
    while (b + 1 < nb && lstart[b + 1] <= e) ++b;
    entries[gstart[b] + (e - lstart[b])] = L.stage[e];
  }
  __syncthreads();  // LDS is reused by the next block of a persistent grid
}

template <bool kSpan>
__global__ __launch_bounds__(kWcScatterThreads) void k_wc_scatter(DevGrammar g, uint32_t* entries, uint64_t* counts,
                                                                  int64_t W) {
  __shared__ WcScatterLds L;
  extern __shared__ uint32_t lds_wc[];
  wc_scatter_block<kSpan>(g, blockIdx.x, entries, counts, L, lds_wc, W);
}

// Reduce: the entry array is cut into chunks (bucket sizes follow the word
// frequencies, so whole buckets per workgroup would leave a few workgroups
// with most of the work). A workgroup sums each bucket segment of its chunk
// in LDS -- kWcCopies copies of the bucket's table, wave w using copy
// w % kWcCopies -- then adds the nonzero sums to the (zeroed) count array
// with coalesced global atomics. One copy: spreading a frequent word's adds
// over four copies (128 KB of LDS, one workgroup per CU) took 176 us for the
// pass on the 10^8-token corpus, one copy (32 KB, two workgroups per CU)
// 162 us; same-address LDS conflicts cost less than the lost occupancy.
constexpr int kWcCopies = 1;
constexpr int kWcThreads = 1024;

// First bucket whose range [start(b), start(b+1)) holds entry i; start(b) =
// off[b * nslot].
__device__ __forceinline__ int bucket_of(const uint32_t* off, int64_t nslot, int nb, int64_t i) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)off[(int64_t)mid * nslot] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct WcReduceLds {
  uint64_t acc[kWcCopies][kWcBucket];
  int first_bucket;
};

__device__ __forceinline__ void wc_reduce_chunk(const DevGrammar& g, const uint32_t* entries, int64_t W,
                                                uint64_t* counts, int64_t chunk_idx, int64_t chunk, WcReduceLds& L) {
  const int64_t c_lo = chunk_idx * chunk;
  const int64_t c_hi = c_lo + chunk < W ? c_lo + chunk : W;
  if (threadIdx.x == 0) L.first_bucket = bucket_of(g.wc_off, g.nslot, g.wc_nb, c_lo);
  __syncthreads();
  uint64_t* mine = L.acc[(threadIdx.x >> 6) % kWcCopies];
  for (int b = L.first_bucket; b < g.wc_nb; ++b) {
    const int64_t b_lo = g.wc_off[(int64_t)b * g.nslot];
    const int64_t b_hi = (b + 1 < g.wc_nb) ? (int64_t)g.wc_off[(int64_t)(b + 1) * g.nslot] : W;
    if (b_lo >= c_hi) break;
    const int64_t lo = b_lo > c_lo ? b_lo : c_lo, hi = b_hi < c_hi ? b_hi : c_hi;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const uint32_t e = __builtin_nontemporal_load(entries + i);
      if (e >> kWcBits)
        atomicAdd(reinterpret_cast<unsigned long long*>(&mine[e & (kWcBucket - 1)]), (unsigned long long)(e >> kWcBits));
    }
    __syncthreads();
    const int64_t base = (int64_t)b * kWcBucket;
    for (int i = threadIdx.x; i < kWcBucket; i += blockDim.x) {
      uint64_t sum = 0;
#pragma unroll
      for (int c = 0; c < kWcCopies; ++c) sum += L.acc[c][i], L.acc[c][i] = 0;
      if (sum && base + i < g.V)
        atomicAdd(reinterpret_cast<unsigned long long*>(&counts[base + i]), (unsigned long long)sum);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kWcThreads) void k_wc_reduce(DevGrammar g, const uint32_t* entries, int64_t W,
                                                          uint64_t* counts, int64_t chunk) {
  __shared__ WcReduceLds L;
  for (int i = threadIdx.x; i < kWcCopies * kWcBucket; i += blockDim.x) (&L.acc[0][0])[i] = 0;
  __syncthreads();
  wc_reduce_chunk(g, entries, W, counts, blockIdx.x, chunk, L);
}

hipError_t launch_word_count_buckets(const DevGrammar& g, uint64_t* counts, uint32_t* entries, int64_t W,
                                     int64_t chunk, hipStream_t s) {
  hipError_t e = launch_fill_u64(counts, g.V, 0, s);
  if (e != hipSuccess) return e;
  if (g.ntiles == 0 || W == 0) return hipSuccess;
  if (g.span_file >= 0)
    k_wc_scatter<true><<<(unsigned)g.nblk, kWcScatterThreads, sizeof(uint32_t) * 3 * g.wc_nb, s>>>(g, entries, counts, W);
  else
    k_wc_scatter<false><<<(unsigned)g.nblk, kWcScatterThreads, sizeof(uint32_t) * 3 * g.wc_nb, s>>>(g, entries, counts, W);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_wc_reduce<<<(unsigned)((W + chunk - 1) / chunk), kWcThreads, 0, s>>>(g, entries, W, counts, chunk);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched word count over many grammars: persistent kernels with a fixed grid
// walk a flattened list of work items (item k of grammar i = its k-th block,
// chunk or fill range) described in device memory. The launch sequence is the
// same for every batch -- only the descriptors change -- so it can be
// captured once in a hipGraph and replayed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int batch_item_owner(const int64_t* base, int n, int64_t it) {
  int lo = 0, hi = n - 1;  // last i with base[i] <= it
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= it) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_wcb_fill(const BatchDesc* d) {
  const int n = d->n;
  const int64_t total = d->fill_base[n];
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int i = batch_item_owner(d->fill_base, n, it);
    const BatchItem& b = d->items[i];
    const int64_t lo = (it - d->fill_base[i]) * kWcBucket;
    for (int64_t x = lo + threadIdx.x; x < lo + kWcBucket && x < b.g.V; x += blockDim.x) b.out[x] = 0;
  }
}

__global__ __launch_bounds__(kWcScatterThreads) void k_wcb_scatter(const BatchDesc* d) {
  __shared__ WcScatterLds L;
  extern __shared__ uint32_t lds_wcb[];
  const int n = d->n;
  const int64_t total = d->scatter_base[n];
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int i = batch_item_owner(d->scatter_base, n, it);
    const BatchItem& b = d->items[i];
    wc_scatter_block<false>(b.g, it - d->scatter_base[i], b.entries, b.out, L, lds_wcb, b.W);
  }
}

__global__ __launch_bounds__(kWcThreads) void k_wcb_reduce(const BatchDesc* d) {
  __shared__ WcReduceLds L;
  for (int i = threadIdx.x; i < kWcCopies * kWcBucket; i += blockDim.x) (&L.acc[0][0])[i] = 0;
  __syncthreads();
  const int n = d->n;
  const int64_t total = d->reduce_base[n];
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int i = batch_item_owner(d->reduce_base, n, it);
    const BatchItem& b = d->items[i];
    wc_reduce_chunk(b.g, b.entries, b.W, b.out, it - d->reduce_base[i], d->chunk, L);
    __syncthreads();
  }
}

hipError_t launch_word_count_batch(const BatchDesc* d, int grid_scatter, int grid_reduce, int max_nb, hipStream_t s) {
  k_wcb_fill<<<grid_scatter, 256, 0, s>>>(d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_wcb_scatter<<<grid_scatter, kWcScatterThreads, sizeof(uint32_t) * 3 * max_nb, s>>>(d);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_wcb_reduce<<<grid_reduce, kWcThreads, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_word_count(const DevGrammar& g, uint64_t* counts, hipStream_t s) {
  hipError_t e = launch_fill_u64(counts, g.V, 0, s);
  if (e != hipSuccess || g.ntiles == 0) return e;
  k_word_count<<<(unsigned)g.ntiles, kTileThreads, 0, s>>>(g, counts);
  return hipGetLastError();
}

}  // namespace gt

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
  for (int64_t q = g.rule_off[r]; q < g.rule_off[r + 1]; ++q) {
    const int32_t s = g.sym[q];
    if (s >= 0) {
      ++L, ++B;
    } else {
      L += len[-s];
      B += bound[-s];
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

// Table of rule r = merge of its pieces (own words, each counting 1, and the
// sorted tables of its children, once per occurrence), emitted in word order.
// Short bodies keep one cursor per piece in registers; long bodies locate
// each piece's next word by binary search.
constexpr int kTvCursors = 16;

__device__ __forceinline__ uint32_t first_above(const uint32_t* w, uint32_t n, int64_t x) {
  uint32_t lo = 0, hi = n;  // first index with w[i] > x
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((int64_t)w[mid] > x) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

__global__ void k_tv_merge_level(DevGrammar g, const int32_t* rules, int32_t n, const uint64_t* toff, uint32_t* tsize,
                                 uint32_t* pw, uint32_t* pc) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t r = rules[i];
  const int64_t a = g.rule_off[r];
  const int64_t k = g.rule_off[r + 1] - a;
  const uint64_t out = toff[r];
  uint32_t m = 0;
  if (k <= kTvCursors) {
    int32_t sj[kTvCursors];
    uint32_t cur[kTvCursors], lim[kTvCursors];
    uint64_t base[kTvCursors];
#pragma unroll
    for (int j = 0; j < kTvCursors; ++j) {
      sj[j] = j < k ? g.sym[a + j] : 0;
      cur[j] = 0;
      if (j < k && sj[j] < 0) {
        lim[j] = tsize[-sj[j]];
        base[j] = toff[-sj[j]];
      } else {
        lim[j] = (j < k) ? 1u : 0u;  // a word piece holds one entry
        base[j] = 0;
      }
    }
    while (true) {
      uint32_t best = 0xffffffffu;
#pragma unroll
      for (int j = 0; j < kTvCursors; ++j) {
        if (cur[j] < lim[j]) {
          const uint32_t wd = sj[j] >= 0 ? (uint32_t)sj[j] : pw[base[j] + cur[j]];
          best = wd < best ? wd : best;
        }
      }
      if (best == 0xffffffffu) break;
      uint32_t cnt = 0;
#pragma unroll
      for (int j = 0; j < kTvCursors; ++j) {
        if (cur[j] < lim[j]) {
          if (sj[j] >= 0) {
            if ((uint32_t)sj[j] == best) ++cnt, ++cur[j];
          } else if (pw[base[j] + cur[j]] == best) {
            cnt += pc[base[j] + cur[j]];
            ++cur[j];
          }
        }
      }
      pw[out + m] = best;
      pc[out + m] = cnt;
      ++m;
    }
  } else {
    int64_t last = -1;
    while (true) {
      uint32_t best = 0xffffffffu;
      for (int64_t j = 0; j < k; ++j) {
        const int32_t s = g.sym[a + j];
        if (s >= 0) {
          if ((int64_t)s > last && (uint32_t)s < best) best = (uint32_t)s;
        } else {
          const uint32_t* w = pw + toff[-s];
          const uint32_t t = tsize[-s];
          const uint32_t x = first_above(w, t, last);
          if (x < t && w[x] < best) best = w[x];
        }
      }
      if (best == 0xffffffffu) break;
      uint32_t cnt = 0;
      for (int64_t j = 0; j < k; ++j) {
        const int32_t s = g.sym[a + j];
        if (s >= 0) {
          cnt += (uint32_t)s == best;
        } else {
          const uint32_t* w = pw + toff[-s];
          const uint32_t t = tsize[-s];
          const uint32_t x = first_above(w, t, last);
          if (x < t && w[x] == best) cnt += pc[toff[-s] + x];
        }
      }
      pw[out + m] = best;
      pc[out + m] = cnt;
      ++m;
      last = best;
    }
  }
  tsize[r] = m;
}

hipError_t launch_tv_tables(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, const uint64_t* toff,
                            uint32_t* tsize, uint32_t* pw, uint32_t* pc, hipStream_t s) {
  for (int32_t d = depth; d >= 1; --d) {
    const int32_t lo = level_off_host[d], hi = level_off_host[d + 1];
    if (hi <= lo) continue;
    k_tv_merge_level<<<(unsigned)((hi - lo + 63) / 64), 64, 0, s>>>(g, g.level_rule + lo, hi - lo, toff, tsize, pw, pc);
    hipError_t e = hipGetLastError();
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

// Pass 1 (count) and pass 2 (scatter) walk the same inputs of one unit.
template <bool kScatter>
__global__ __launch_bounds__(256) void k_tv_group(DevGrammar g, TvFiles t, uint64_t* entries) {
  extern __shared__ uint32_t lds_tv[];  // per-bucket counts (pass 1) or cursors (pass 2)
  __shared__ int64_t sh_f;
  const int64_t u = blockIdx.x;
  if (threadIdx.x == 0) sh_f = file_of_unit(t.unit_off, g.F, u);
  __syncthreads();
  const int64_t f = sh_f;
  const int64_t n_f = t.unit_off[f + 1] - t.unit_off[f];
  const int64_t k = u - t.unit_off[f];
  const int64_t slot0 = (int64_t)t.nb * t.unit_off[f] + k;
  for (int b = threadIdx.x; b < t.nb; b += blockDim.x) lds_tv[b] = kScatter ? t.table[slot0 + b * n_f] : 0u;
  __syncthreads();
  const int64_t fs = g.file_off[f] + k * kTileSyms, fe0 = g.file_off[f + 1];
  const int64_t fe = fs + kTileSyms < fe0 ? fs + kTileSyms : fe0;
  for (int64_t q = fs + threadIdx.x * kPerThread, qe = q + kPerThread; q < qe && q < fe; ++q) {
    const int32_t s = g.sym[q];
    if (s >= 0) {
      const uint32_t at = atomicAdd(&lds_tv[s >> kWcBits], 1u);
      if (kScatter) entries[at] = (1ull << kWcBits) | (uint64_t)(s & (kWcBucket - 1));
    } else {
      const uint64_t o = t.toff[-s];
      const uint32_t n = t.tsize[-s];
      for (uint32_t e = 0; e < n; ++e) {
        const uint32_t wd = t.pw[o + e];
        const uint32_t at = atomicAdd(&lds_tv[wd >> kWcBits], 1u);
        if (kScatter) entries[at] = ((uint64_t)t.pc[o + e] << kWcBits) | (uint64_t)(wd & (kWcBucket - 1));
      }
    }
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

// Pass 3: sum each group in a dense LDS table; the nonzero slots are written
// back over the group's own entries in word order, packed (word << 32 |
// count), and their number to nnz[group]. Workgroup j takes the groups that
// start in [j * kTvChunk, (j+1) * kTvChunk) of the entry array.
constexpr int kTvThreads = 1024;
constexpr int64_t kTvChunk = 16 * kTvThreads;

__global__ __launch_bounds__(kTvThreads) void k_tv_reduce(DevGrammar g, TvFiles t, uint64_t* entries, int64_t E,
                                                          uint32_t* nnz) {
  __shared__ uint32_t cnt[kWcBucket];
  __shared__ int64_t first_group;
  __shared__ uint32_t wsum[kTvThreads / 64];
  const int64_t ngroups = g.F * (int64_t)t.nb;
  const int64_t c_lo = (int64_t)blockIdx.x * kTvChunk, c_hi = c_lo + kTvChunk;
  if (threadIdx.x == 0) {
    int64_t lo = 0, hi = ngroups;  // first group starting at or after c_lo
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (group_start(g, t, mid, E) < c_lo) lo = mid + 1;
      else hi = mid;
    }
    first_group = lo;
  }
  for (int i = threadIdx.x; i < kWcBucket; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  for (int64_t s = first_group; s < ngroups; ++s) {
    const int64_t lo = group_start(g, t, s, E);
    if (lo >= c_hi) break;  // empty groups past the end keep nnz = 0
    const int64_t hi = group_start(g, t, s + 1, E);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const uint64_t e = entries[i];
      atomicAdd(&cnt[e & (kWcBucket - 1)], (uint32_t)(e >> kWcBits));
    }
    __syncthreads();
    // compact the nonzero slots in word order: 4 consecutive slots per thread
    uint32_t c4[4], nz = 0;
#pragma unroll
    for (int x = 0; x < 4; ++x) c4[x] = cnt[threadIdx.x * 4 + x], nz += c4[x] != 0;
    // block exclusive scan of nz (16 waves)
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

hipError_t launch_tv_reduce(const DevGrammar& g, const TvFiles& t, uint64_t* entries, int64_t E, uint32_t* nnz,
                            hipStream_t s) {
  const int64_t blocks = E > 0 ? (E + kTvChunk - 1) / kTvChunk : 1;
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(nnz), g.F * (int64_t)t.nb, 0, s);
  if (e != hipSuccess) return e;
  k_tv_reduce<<<(unsigned)blocks, kTvThreads, 0, s>>>(g, t, entries, E, nnz);
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
__global__ void k_ii_pairs(const int64_t* tv_off, int64_t F, const uint32_t* tv_word, int64_t nnz, uint64_t* key,
                           uint32_t* file) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  int64_t lo = 0, hi = F - 1;  // file f with tv_off[f] <= i < tv_off[f+1]
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (tv_off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  key[i] = tv_word[i];
  file[i] = (uint32_t)lo;
}

__global__ void k_ii_offsets(const uint64_t* key, int64_t nnz, int32_t V, int64_t* off) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > nnz) return;
  // words w in (key[i-1], key[i]] start at i; past the end, up to V
  const int64_t prev = i == 0 ? -1 : (int64_t)key[i - 1];
  const int64_t cur = i == nnz ? (int64_t)V : (int64_t)key[i];
  for (int64_t w = prev + 1; w <= cur; ++w) off[w] = i;
}

hipError_t launch_ii(const int64_t* tv_off, int64_t F, const uint32_t* tv_word, int64_t nnz, int32_t V,
                     uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint64_t* kout, uint32_t* file_out,
                     const int64_t* num, uint32_t* hist, int64_t* ii_off, hipStream_t s) {
  if (nnz > 0) {
    k_ii_pairs<<<(unsigned)((nnz + 255) / 256), 256, 0, s>>>(tv_off, F, tv_word, nnz, k0, v0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int b = 1;
    while (b < 32 && (1ll << b) < (int64_t)V) ++b;
    e = radix_sort_pairs<uint32_t>(k0, v0, k1, v1, num, nnz, 0, b, false, hist, kout, file_out, s);
    if (e != hipSuccess) return e;
  }
  k_ii_offsets<<<(unsigned)((nnz + 1 + 255) / 256), 256, 0, s>>>(kout, nnz, V, ii_off);
  return hipGetLastError();
}

hipError_t launch_scan_u64_ext(uint64_t* a, int64_t n, int64_t* total, uint64_t* sums, hipStream_t s) {
  return launch_scan_u64(a, n, total, sums, s);
}
hipError_t launch_scan_u32_ext(uint32_t* a, int64_t n, int64_t* total, uint32_t* sums, hipStream_t s) {
  return launch_scan_u32(a, n, total, sums, s);
}

}  // namespace gt

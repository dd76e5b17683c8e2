// k_tv_topdown.hip -- term vector by the top-down traversal with per-file
// rule weights, for grammars with few files.
//
// Paper: Section "Fine-Grained Thread-Level Execution Engine" (both
// traversals are built and a selector picks one per input and task);
// Evaluation, Optimization Analysis, "Top-down vs. bottom-up traversals":
// with few files, every rule carries a small buffer of file information
// (how often the rule occurs in each file) that flows from the root to the
// leaves, and the per-file word counts come out of one pass over the bodies;
// with many small files that buffer and its transmission dominate and the
// bottom-up traversal wins.
//
// Here files are taken kTdGroup at a time. For a group, every rule holds
// kTdGroup uint64 weights, w_f(r) = occurrences of r in the expansion of file
// f: the root's references add 1 to the referenced rule's weight of the file
// the reference sits in; then level by level (the load's levels, from the
// root down) every rule adds its weights to each sub-rule occurrence. The
// per-file counts tv[f][x] = sum over rules r of w_f(r) * (occurrences of
// word x in body(r)), plus the words of the file's root span, are the
// library's word-count pass run with weight column f (the root weight of a
// file is 1 inside its span and 0 elsewhere). The dense per-file counts are
// compacted into the term vector rows (words ascending).
#include "device.h"
#include "radix.h"

namespace gt {

// Root references of files [f0, f0 + nf): w[c * kTdGroup + (f - f0)] += 1.
// One thread per root symbol; references to the same (rule, file) inside a
// workgroup are merged in an LDS table first (frequent sub-rules would
// otherwise serialize on one global address).
constexpr int kTdRootSlots = 4096;
__global__ __launch_bounds__(256) void k_td_root(DevGrammar g, int64_t f0, int32_t nf, uint64_t* w) {
  __shared__ int64_t key[kTdRootSlots];
  __shared__ uint32_t cnt[kTdRootSlots];
  __shared__ int64_t span[kTdGroup + 1];
  for (int k = threadIdx.x; k < kTdRootSlots; k += blockDim.x) key[k] = -1, cnt[k] = 0;
  if (threadIdx.x <= nf) span[threadIdx.x] = g.file_off[f0 + threadIdx.x];
  __syncthreads();
  const int64_t lo = span[0], hi = span[nf];
  const int64_t per_block = (int64_t)blockDim.x * 16;
  for (int64_t b0 = lo + (int64_t)blockIdx.x * per_block; b0 < hi; b0 += (int64_t)gridDim.x * per_block) {
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
      const int64_t q = b0 + (int64_t)k * blockDim.x + threadIdx.x;
      if (q >= hi) break;
      const int32_t s = g.sym[q];
      if (s >= 0 || -(int64_t)s >= g.R) continue;
      int32_t f = 0;
      while (f + 1 < nf && span[f + 1] <= q) ++f;
      const int64_t kk = (int64_t)(-s) * kTdGroup + f;
      const uint32_t h = (uint32_t)(((uint64_t)kk * 0x9E3779B97F4A7C15ull) >> 52);
      bool done = false;
      for (int p = 0; p < 8 && !done; ++p) {
        const uint32_t slot = (h + p) & (kTdRootSlots - 1);
        int64_t cur = __hip_atomic_load(&key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == -1) {
          const unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(&key[slot]),
                                                    ~0ull, (unsigned long long)kk);
          cur = prev == ~0ull ? kk : (int64_t)prev;
        }
        if (cur == kk) {
          atomicAdd(&cnt[slot], 1u);
          done = true;
        }
      }
      if (!done) atomicAdd(reinterpret_cast<unsigned long long*>(&w[kk]), 1ull);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kTdRootSlots; k += blockDim.x)
    if (cnt[k]) atomicAdd(reinterpret_cast<unsigned long long*>(&w[key[k]]), (unsigned long long)cnt[k]);
}

// One level, root side first: every rule p of the level adds its kTdGroup
// weights to each sub-rule occurrence (zero weights are skipped, so a rule
// that occurs in one file of the group costs one atomic per reference).
__global__ __launch_bounds__(256) void k_td_level(DevGrammar g, const int32_t* rules, int32_t n, uint64_t* w) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t p = rules[i];
  uint64_t wp[kTdGroup];
  bool any = false;
#pragma unroll
  for (int f = 0; f < kTdGroup; ++f) {
    wp[f] = w[(int64_t)p * kTdGroup + f];
    any |= wp[f] != 0;
  }
  if (!any) return;
  const int64_t a = g.rule_off[p], b = g.rule_off[p + 1];
  for (int64_t q = a; q < b; ++q) {
    const int32_t s = g.sym[q];
    if (s >= 0 || -(int64_t)s >= g.R) continue;
    uint64_t* wc = w + (int64_t)(-s) * kTdGroup;
#pragma unroll
    for (int f = 0; f < kTdGroup; ++f)
      if (wp[f]) atomicAdd(reinterpret_cast<unsigned long long*>(&wc[f]), (unsigned long long)wp[f]);
  }
}

// Weight column f of the group: out[r] = w[r * kTdGroup + f]; the root gets 1.
__global__ __launch_bounds__(256) void k_td_column(const uint64_t* w, int64_t R, int f, uint64_t* out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= R) return;
  out[r] = r == 0 ? 1ull : w[r * kTdGroup + f];
}

// Nonzero entries per 4096-entry block of the dense per-file counts, then
// (word, count) of each at its compacted position; row f of the dense matrix
// starts at f * V, so the compacted order is file-major, words ascending.
__global__ __launch_bounds__(256) void k_td_nz_count(const uint64_t* dense, int64_t n, uint32_t* blk_cnt) {
  const int64_t i0 = blockIdx.x * (int64_t)kRadixTile + threadIdx.x * 16;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (i0 + k < n && dense[i0 + k] != 0) ++c;
  __shared__ uint32_t lds[4];
  uint32_t total;
  block_exclusive_scan_256(c, lds, &total);
  if (threadIdx.x == 0) blk_cnt[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_td_nz_write(const uint64_t* dense, int64_t n, int32_t V, const uint32_t* blk_off,
                                                     uint32_t* word, uint64_t* cnt) {
  const int64_t i0 = blockIdx.x * (int64_t)kRadixTile + threadIdx.x * 16;
  uint64_t c[16];
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    c[k] = (i0 + k < n) ? dense[i0 + k] : 0;
    m += c[k] != 0;
  }
  __shared__ uint32_t lds[4];
  uint32_t total;
  uint32_t pos = blk_off[blockIdx.x] + block_exclusive_scan_256(m, lds, &total);
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (c[k] != 0) {
      word[pos] = (uint32_t)((i0 + k) % V);
      cnt[pos] = c[k];
      ++pos;
    }
}

// Row sizes: off[f] = nonzero entries of row f (V entries of the dense
// matrix), one workgroup per row; an exclusive scan over off[0..F] (with
// off[F] = 0) turns them into row offsets.
__global__ __launch_bounds__(256) void k_td_row_off(const uint64_t* dense, int64_t F, int32_t V, int64_t* off) {
  __shared__ uint32_t part[4];
  const int64_t f = blockIdx.x;
  if (f >= F) return;
  uint32_t c = 0;
  for (int64_t x = threadIdx.x; x < V; x += blockDim.x) c += dense[f * (int64_t)V + x] != 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
  if (lane_id() == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) off[f] = (int64_t)(part[0] + part[1] + part[2] + part[3]);
}

hipError_t launch_td_root(const DevGrammar& g, int64_t f0, int32_t nf, uint64_t* w, hipStream_t s) {
  // the span is read on the device: a fixed grid strides over it
  k_td_root<<<2048, 256, 0, s>>>(g, f0, nf, w);
  return hipGetLastError();
}

hipError_t launch_td_levels(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* w,
                            hipStream_t s) {
  for (int32_t d = 1; d <= depth; ++d) {
    const int32_t lo = level_off_host[d], hi = level_off_host[d + 1];
    if (hi <= lo) continue;
    k_td_level<<<(unsigned)((hi - lo + 255) / 256), 256, 0, s>>>(g, g.level_rule + lo, hi - lo, w);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_td_column(const uint64_t* w, int64_t R, int f, uint64_t* out, hipStream_t s) {
  k_td_column<<<(unsigned)((R + 255) / 256), 256, 0, s>>>(w, R, f, out);
  return hipGetLastError();
}

hipError_t launch_td_compact_count(const uint64_t* dense, int64_t n, uint32_t* blk, hipStream_t s) {
  const int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  k_td_nz_count<<<(unsigned)nb, 256, 0, s>>>(dense, n, blk);
  return hipGetLastError();
}

hipError_t launch_td_compact_write(const uint64_t* dense, int64_t n, int32_t V, const uint32_t* blk_off, uint32_t* word,
                                   uint64_t* cnt, hipStream_t s) {
  const int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  k_td_nz_write<<<(unsigned)nb, 256, 0, s>>>(dense, n, V, blk_off, word, cnt);
  return hipGetLastError();
}

hipError_t launch_td_row_off(const uint64_t* dense, int64_t F, int32_t V, int64_t* off, hipStream_t s) {
  k_td_row_off<<<(unsigned)F, 256, 0, s>>>(dense, F, V, off);
  return hipGetLastError();
}

}  // namespace gt

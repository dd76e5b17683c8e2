// k_expand.hip -- decompression of a loaded grammar on the GPU: the token
// sequence of every file, written to a caller-owned array.
//
// Paper: Evaluation, Discussion ("Comparison with GPU-accelerated
// uncompressed analytics"): the method is compared with analytics that run
// on the uncompressed text on the same GPU. This is the decompression half
// of that comparison (the analytics on the plain tokens reuse the library's
// query kernels on a grammar that is one root body of words); the text is
// the expansion of the root (Background, "TADOC": the root spells the files,
// a rule stands for the expansion of its body).
//
// Steps: the expansion length of every rule, children first (one launch per
// level from the deepest); the output position of every root symbol by an
// exclusive scan of their lengths; then the derivation tree is walked one
// depth at a time. An item (rule, output offset) writes the words of the
// rule's body at their positions and emits one item per sub-rule occurrence
// for the next depth. Items of one depth cover disjoint output ranges, so a
// depth never holds more items than there are tokens.
#include "device.h"
#include "radix.h"

namespace gt {

// len[r] = expansion length of rule r, for the rules of one level (their
// children, at deeper levels, are done).
__global__ __launch_bounds__(256) void k_len_level(DevGrammar g, const int32_t* rules, int32_t n, uint64_t* len) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t r = rules[i];
  const int64_t a = g.rule_off[r], b = g.rule_off[r + 1];
  uint64_t L = 0;
  for (int64_t q0 = a; q0 < b; q0 += 8) {  // 8 symbols (and then their children's lengths) in flight together
    int32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = q0 + k < b ? g.sym[q0 + k] : 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (q0 + k >= b) continue;
      L += v[k] >= 0 ? 1ull : len[-v[k]];
    }
  }
  len[r] = L;
}

// Length of every root symbol (1 for a word, len of a rule), to be scanned
// into output positions.
__global__ __launch_bounds__(256) void k_root_lens(DevGrammar g, const uint64_t* len, uint64_t* pos, int64_t n) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int32_t s = g.sym[q];
  pos[q] = s >= 0 ? 1ull : len[-s];
}

// Output offsets of the files: the position of each file's first root symbol.
__global__ __launch_bounds__(256) void k_file_out(DevGrammar g, const uint64_t* pos, int64_t nroot, uint64_t T,
                                                  int64_t* file_out) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f > g.F) return;
  const int64_t q = g.file_off[f];
  file_out[f] = q < nroot ? (int64_t)pos[q] : (int64_t)T;
}

// Items of the next depth are appended per block: one global atomic per
// block, each thread's items at its exclusive offset.
__device__ __forceinline__ int64_t block_reserve(uint32_t n, unsigned long long* counter, uint32_t* lds,
                                                 uint64_t* base_lds) {
  uint32_t total;
  const uint32_t mine = block_exclusive_scan_256(n, lds, &total);
  if (threadIdx.x == 0) *base_lds = total ? atomicAdd(counter, (unsigned long long)total) : 0ull;
  __syncthreads();
  const int64_t at = (int64_t)*base_lds + mine;
  __syncthreads();
  return at;
}

// Depth 0: the root body, one thread per symbol. Words go to their output
// positions, rule references become items.
__global__ __launch_bounds__(256) void k_expand_root(DevGrammar g, const uint64_t* pos, int64_t nroot, int32_t* tokens,
                                                     int32_t* out_rule, int64_t* out_off, unsigned long long* out_n) {
  __shared__ uint32_t lds[4];
  __shared__ uint64_t base;
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < nroot; b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = b0 + threadIdx.x;
    int32_t s = 0;
    uint64_t p = 0;
    if (q < nroot) {
      s = g.sym[q];
      p = pos[q];
      if (s >= 0) tokens[p] = s;
    }
    const bool ref = q < nroot && s < 0;
    const int64_t at = block_reserve(ref ? 1u : 0u, out_n, lds, &base);
    if (ref) {
      out_rule[at] = -s;
      out_off[at] = (int64_t)p;
    }
  }
}

// One depth of the derivation tree: each item (rule r at output offset o)
// writes the words of body(r) and emits an item per sub-rule occurrence.
// The body is walked twice (count, then write), so the block reserves its
// items with one atomic.
__global__ __launch_bounds__(256) void k_expand_depth(DevGrammar g, const uint64_t* len, const int32_t* in_rule,
                                                      const int64_t* in_off, const unsigned long long* in_n,
                                                      int32_t* tokens, int32_t* out_rule, int64_t* out_off,
                                                      unsigned long long* out_n) {
  __shared__ uint32_t lds[4];
  __shared__ uint64_t base;
  const int64_t n = (int64_t)*in_n;
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < n; b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = b0 + threadIdx.x;
    int64_t a = 0, e = 0, o = 0;
    uint32_t refs = 0;
    if (i < n) {
      const int32_t r = in_rule[i];
      o = in_off[i];
      a = g.rule_off[r];
      e = g.rule_off[r + 1];
      for (int64_t q = a; q < e; ++q) refs += g.sym[q] < 0;
    }
    int64_t at = block_reserve(refs, out_n, lds, &base);
    for (int64_t q = a; q < e; ++q) {
      const int32_t s = g.sym[q];
      if (s >= 0) {
        tokens[o++] = s;
      } else {
        out_rule[at] = -s;
        out_off[at] = o;
        ++at;
        o += (int64_t)len[-s];
      }
    }
  }
}

hipError_t launch_rule_lengths(const DevGrammar& g, const int32_t* level_off_host, int32_t depth, uint64_t* len,
                               hipStream_t s) {
  for (int32_t d = depth; d >= 1; --d) {
    const int32_t lo = level_off_host[d], hi = level_off_host[d + 1];
    if (hi <= lo) continue;
    k_len_level<<<(unsigned)((hi - lo + 255) / 256), 256, 0, s>>>(g, g.level_rule + lo, hi - lo, len);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Sum of n uint64 values into *out (zeroed by the caller).
__global__ __launch_bounds__(256) void k_sum_u64(const uint64_t* a, int64_t n, unsigned long long* out) {
  uint64_t v = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) v += a[i];
  v = wave_sum_u64(v);
  if (lane_id() == 0 && v) atomicAdd(out, (unsigned long long)v);
}

hipError_t launch_sum_u64(const uint64_t* a, int64_t n, unsigned long long* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  k_sum_u64<<<(unsigned)(want < 1024 ? want : 1024), 256, 0, s>>>(a, n, out);
  return hipGetLastError();
}

// Distinct sub-rules of every non-root rule (a reference counts when the
// same rule does not occur earlier in the body; bodies are short, so the
// quadratic scan is cheap), summed into *out.
__global__ __launch_bounds__(256) void k_edges_rules(DevGrammar g, unsigned long long* out) {
  const int64_t r = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  uint64_t e = 0;
  if (r < g.R) {
    const int64_t a = g.rule_off[r], b = g.rule_off[r + 1];
    for (int64_t q = a; q < b; ++q) {
      const int32_t s = g.sym[q];
      if (s >= 0) continue;
      bool first = true;
      for (int64_t p = a; p < q && first; ++p) first = g.sym[p] != s;
      e += first;
    }
  }
  e = wave_sum_u64(e);
  if (lane_id() == 0 && e) atomicAdd(out, (unsigned long long)e);
}

// Sub-rules of the root: a flag per referenced rule (plain stores of 1),
// then the flags are counted.
__global__ __launch_bounds__(256) void k_edges_root_flags(DevGrammar g, int64_t nroot, uint8_t* flags) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nroot; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = g.sym[q];
    if (s < 0) flags[-s] = 1;
  }
}

__global__ __launch_bounds__(256) void k_edges_root_count(const uint8_t* flags, int64_t R, unsigned long long* out) {
  uint64_t e = 0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x)
    e += flags[r];
  e = wave_sum_u64(e);
  if (lane_id() == 0 && e) atomicAdd(out, (unsigned long long)e);
}

hipError_t launch_count_edges(const DevGrammar& g, int64_t root_syms, uint8_t* flags, unsigned long long* out,
                              hipStream_t s) {
  hipError_t e = launch_fill_u64(reinterpret_cast<uint64_t*>(out), 1, 0, s);
  if (e != hipSuccess) return e;
  e = launch_fill_i32(reinterpret_cast<int32_t*>(flags), (g.R + 3) / 4, 0, s);  // the block is 256-byte rounded
  if (e != hipSuccess) return e;
  if (g.R > 1) {
    k_edges_rules<<<(unsigned)((g.R - 1 + 255) / 256), 256, 0, s>>>(g, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int64_t want = (root_syms + 255) / 256;
  if (root_syms > 0) {
    k_edges_root_flags<<<(unsigned)(want < 4096 ? want : 4096), 256, 0, s>>>(g, root_syms, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int64_t wr = (g.R + 255) / 256;
  k_edges_root_count<<<(unsigned)(wr < 4096 ? wr : 4096), 256, 0, s>>>(flags, g.R, out);
  return hipGetLastError();
}

hipError_t launch_root_positions(const DevGrammar& g, const uint64_t* len, uint64_t* pos, int64_t nroot, uint64_t T,
                                 int64_t* file_out, uint64_t* sums, hipStream_t s) {
  if (nroot > 0) {
    k_root_lens<<<(unsigned)((nroot + 255) / 256), 256, 0, s>>>(g, len, pos, nroot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan_u64(pos, nroot, nullptr, sums, s);
    if (e != hipSuccess) return e;
  }
  k_file_out<<<(unsigned)((g.F + 1 + 255) / 256), 256, 0, s>>>(g, pos, nroot, T, file_out);
  return hipGetLastError();
}

hipError_t launch_expand_root(const DevGrammar& g, const uint64_t* pos, int64_t nroot, int32_t* tokens,
                              int32_t* out_rule, int64_t* out_off, unsigned long long* out_n, hipStream_t s) {
  if (nroot == 0) return hipSuccess;
  const int64_t want = (nroot + 255) / 256;
  k_expand_root<<<(unsigned)(want < 8192 ? want : 8192), 256, 0, s>>>(g, pos, nroot, tokens, out_rule, out_off, out_n);
  return hipGetLastError();
}

hipError_t launch_expand_depth(const DevGrammar& g, const uint64_t* len, const int32_t* in_rule, const int64_t* in_off,
                               const unsigned long long* in_n, int64_t cap, int32_t* tokens, int32_t* out_rule,
                               int64_t* out_off, unsigned long long* out_n, hipStream_t s) {
  const int64_t want = (cap + 255) / 256;
  k_expand_depth<<<(unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192), 256, 0, s>>>(
      g, len, in_rule, in_off, in_n, tokens, out_rule, out_off, out_n);
  return hipGetLastError();
}

}  // namespace gt

// radix.h -- stable LSD radix sort of (uint64 key, value) pairs on the GPU,
// and the block/grid scans it uses. Header-only templates; the kernels are
// instantiated by the translation units that use them.
#pragma once

#include "device.h"

namespace gt {

constexpr int kRadixTile = 4096;  // keys per workgroup (256 threads x 16)

// Exclusive scan of one value per thread over a 256-thread block. `lds`
// holds 4 entries. Returns the exclusive prefix; *total gets the block sum.
__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t v, uint32_t* lds, uint32_t* total) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t c = lds[w];
    if (w < wave) base += c;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// Exclusive scan of a[0..n) in place by one 1024-thread block; the total goes
// to *total (int64) if non-null.
static __global__ __attribute__((unused)) __launch_bounds__(1024) void k_scan_u32(uint32_t* a, int64_t n, int64_t* total) {
  __shared__ uint64_t wsum[16];
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = threadIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  uint64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += a[i];
  // inclusive scan of s over the block
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint64_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) base += wsum[w];
    tot += wsum[w];
  }
  uint64_t run = base + x - s;
  for (int64_t i = lo; i < hi; ++i) {
    const uint32_t c = a[i];
    a[i] = (uint32_t)run;
    run += c;
  }
  if (threadIdx.x == 0 && total) *total = (int64_t)tot;
}

// Multi-block exclusive scan of u32 values (sums must fit 32 bits): block
// sums of 4096-element chunks, one small scan of those, then every chunk
// scanned in place with its offset. `sums` needs scan_sums_entries(n).
inline int64_t scan_sums_entries(int64_t n) { return (n + kRadixTile - 1) / kRadixTile + 1; }

static __global__ __attribute__((unused)) __launch_bounds__(256) void k_scan_sums(const uint32_t* a, int64_t n, uint32_t* sums) {
  const int64_t i0 = blockIdx.x * (int64_t)kRadixTile + threadIdx.x * 16;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (i0 + k < n) c += a[i0 + k];
  __shared__ uint32_t lds[4];
  uint32_t total;
  block_exclusive_scan_256(c, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

static __global__ __attribute__((unused)) __launch_bounds__(256) void k_scan_apply(uint32_t* a, int64_t n, const uint32_t* sums) {
  const int64_t i0 = blockIdx.x * (int64_t)kRadixTile + threadIdx.x * 16;
  uint32_t v[16], c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = (i0 + k < n) ? a[i0 + k] : 0u;
    c += v[k];
  }
  __shared__ uint32_t lds[4];
  uint32_t total;
  uint32_t run = sums[blockIdx.x] + block_exclusive_scan_256(c, lds, &total);
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (i0 + k < n) {
      a[i0 + k] = run;
      run += v[k];
    }
}

inline hipError_t launch_scan_u32(uint32_t* a, int64_t n, int64_t* total, uint32_t* sums, hipStream_t s) {
  const int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  if (nb <= 1) {
    k_scan_u32<<<1, 1024, 0, s>>>(a, n, total);
    return hipGetLastError();
  }
  k_scan_sums<<<(unsigned)nb, 256, 0, s>>>(a, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scan_u32<<<1, 1024, 0, s>>>(sums, nb, total);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scan_apply<<<(unsigned)nb, 256, 0, s>>>(a, n, sums);
  return hipGetLastError();
}

// 64-bit exclusive scan (same three phases) for offsets that may pass 2^32.
static __global__ __attribute__((unused)) __launch_bounds__(1024) void k_scan_u64_single(uint64_t* a, int64_t n,
                                                                                        int64_t* total) {
  __shared__ uint64_t wsum[16];
  const int64_t per = (n + 1023) / 1024;
  const int64_t lo = threadIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  uint64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += a[i];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint64_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) base += wsum[w];
    tot += wsum[w];
  }
  uint64_t run = base + x - s;
  for (int64_t i = lo; i < hi; ++i) {
    const uint64_t c = a[i];
    a[i] = run;
    run += c;
  }
  if (threadIdx.x == 0 && total) *total = (int64_t)tot;
}

__device__ __forceinline__ uint64_t block_exclusive_scan_256_u64(uint64_t v, uint64_t* lds, uint64_t* total) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  uint64_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint64_t c = lds[w];
    if (w < wave) base += c;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

static __global__ __attribute__((unused)) __launch_bounds__(256) void k_scan_sums_u64(const uint64_t* a, int64_t n,
                                                                                      uint64_t* sums) {
  const int64_t i0 = blockIdx.x * (int64_t)kRadixTile + threadIdx.x * 16;
  uint64_t c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (i0 + k < n) c += a[i0 + k];
  __shared__ uint64_t lds[4];
  uint64_t total;
  block_exclusive_scan_256_u64(c, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

static __global__ __attribute__((unused)) __launch_bounds__(256) void k_scan_apply_u64(uint64_t* a, int64_t n,
                                                                                       const uint64_t* sums) {
  const int64_t i0 = blockIdx.x * (int64_t)kRadixTile + threadIdx.x * 16;
  uint64_t v[16], c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = (i0 + k < n) ? a[i0 + k] : 0ull;
    c += v[k];
  }
  __shared__ uint64_t lds[4];
  uint64_t total;
  uint64_t run = sums[blockIdx.x] + block_exclusive_scan_256_u64(c, lds, &total);
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (i0 + k < n) {
      a[i0 + k] = run;
      run += v[k];
    }
}

// In-place exclusive scan of uint64 values; `sums` needs scan_sums_entries(n).
inline hipError_t launch_scan_u64(uint64_t* a, int64_t n, int64_t* total, uint64_t* sums, hipStream_t s) {
  const int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  if (nb <= 1) {
    k_scan_u64_single<<<1, 1024, 0, s>>>(a, n, total);
    return hipGetLastError();
  }
  k_scan_sums_u64<<<(unsigned)nb, 256, 0, s>>>(a, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scan_u64_single<<<1, 1024, 0, s>>>(sums, nb, total);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scan_apply_u64<<<(unsigned)nb, 256, 0, s>>>(a, n, sums);
  return hipGetLastError();
}

__device__ __forceinline__ uint32_t radix_digit(uint64_t k, int shift, bool desc) {
  return (uint32_t)(((desc ? ~k : k) >> shift) & 0xffu);
}

// Digit histogram of every tile: hist[d * nb + b] (digit-major, so that one
// exclusive scan gives every tile's output offset per digit).
static __global__ __attribute__((unused)) __launch_bounds__(256) void k_radix_hist(const uint64_t* key, const int64_t* num, int shift, bool desc,
                                                    uint32_t* hist, int nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = *num;
  const int64_t t0 = blockIdx.x * (int64_t)kRadixTile;
  if (t0 < n) {
    for (int k = threadIdx.x; k < kRadixTile; k += 256) {
      const int64_t i = t0 + k;
      if (i < n) atomicAdd(&h[radix_digit(key[i], shift, desc)], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one digit pass. Wave w of a tile owns tile elements
// [w*1024, (w+1)*1024) in 16 steps of 64; a lane's rank among equal digits
// in a step comes from 8 ballots, and per-wave digit counters in LDS carry
// the ranks across steps; waves are then ordered by a prefix over the
// per-wave counts.
template <typename V>
__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t* kin, const V* vin, uint64_t* kout, V* vout,
                                                       const int64_t* num, int shift, bool desc, const uint32_t* hist,
                                                       int nb) {
  __shared__ uint32_t wcnt[4][256];
  __shared__ uint32_t base[4][256];
  const int64_t n = *num;
  const int64_t t0 = blockIdx.x * (int64_t)kRadixTile;
  if (t0 >= n) return;  // uniform for the block
  const int wave = threadIdx.x >> 6, lane = lane_id();
  for (int i = threadIdx.x; i < 4 * 256; i += 256) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  uint64_t key[16];
  V val[16];
  uint32_t rank[16];
  uint32_t dig[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int64_t idx = t0 + wave * 1024 + j * 64 + lane;
    const bool valid = idx < n;
    const uint64_t k = valid ? kin[idx] : 0;
    const uint32_t d = radix_digit(k, shift, desc);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t before = wcnt[wave][d];
    const uint32_t r = (uint32_t)__popcll(peers & lanes_below());
    __builtin_amdgcn_wave_barrier();
    if (valid && r == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    key[j] = k;
    val[j] = valid ? vin[idx] : V(0);
    rank[j] = valid ? before + r : 0xffffffffu;
    dig[j] = d;
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t acc = hist[(int64_t)d * nb + blockIdx.x];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      base[w][d] = acc;
      acc += wcnt[w][d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (rank[j] == 0xffffffffu) continue;
    const uint32_t pos = base[wave][dig[j]] + rank[j];
    kout[pos] = key[j];
    vout[pos] = val[j];
  }
}

inline int64_t radix_hist_entries(int64_t cap) {
  const int64_t nb = (cap + kRadixTile - 1) / kRadixTile;
  return 256 * (nb > 0 ? nb : 1) + scan_sums_entries(256 * (nb > 0 ? nb : 1));
}

// Sort (key, val) pairs stably by the key bytes set in byte_mask (bit i =
// byte i; bytes outside the mask must be equal in all keys), ascending or
// descending (desc). n = *num (device) <= cap. The input is (k0, v0); (k1, v1)
// is scratch of the same size; the result lands in (kout, vout). hist needs
// radix_hist_entries(cap) entries. At least one byte must be set.
template <typename V>
hipError_t radix_sort_pairs_bytes(uint64_t* k0, V* v0, uint64_t* k1, V* v1, const int64_t* num, int64_t cap,
                                  uint64_t byte_mask, bool desc, uint32_t* hist, uint64_t* kout, V* vout,
                                  hipStream_t s) {
  const int nb = (int)((cap + kRadixTile - 1) / kRadixTile);
  if (nb == 0) return hipSuccess;
  int shifts[8], npass = 0;
  for (int b = 0; b < 8; ++b)
    if (byte_mask >> b & 1) shifts[npass++] = 8 * b;
  if (npass == 0) shifts[npass++] = 0;
  const uint64_t* ksrc = k0;
  const V* vsrc = v0;
  for (int p = 0; p < npass; ++p) {
    const int shift = shifts[p];
    uint64_t* kdst = (p == npass - 1) ? kout : ((p & 1) == 0 ? k1 : k0);
    V* vdst = (p == npass - 1) ? vout : ((p & 1) == 0 ? v1 : v0);
    k_radix_hist<<<nb, 256, 0, s>>>(ksrc, num, shift, desc, hist, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan_u32(hist, (int64_t)256 * nb, nullptr, hist + (int64_t)256 * nb, s);
    if (e != hipSuccess) return e;
    k_radix_scatter<V><<<nb, 256, 0, s>>>(ksrc, vsrc, kdst, vdst, num, shift, desc, hist, nb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ksrc = kdst;
    vsrc = vdst;
  }
  return hipSuccess;
}

// The same over the bits [bit_lo, bit_hi), rounded out to whole bytes.
template <typename V>
hipError_t radix_sort_pairs(uint64_t* k0, V* v0, uint64_t* k1, V* v1, const int64_t* num, int64_t cap, int bit_lo,
                            int bit_hi, bool desc, uint32_t* hist, uint64_t* kout, V* vout, hipStream_t s) {
  uint64_t mask = 0;
  for (int b = bit_lo / 8; b * 8 < bit_hi && b < 8; ++b) mask |= 1ull << b;
  return radix_sort_pairs_bytes<V>(k0, v0, k1, v1, num, cap, mask, desc, hist, kout, vout, s);
}

}  // namespace gt

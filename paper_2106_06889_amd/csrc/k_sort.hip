// k_sort.hip -- "sort": the words with a nonzero count, by count descending
// then word id ascending (an application the paper keeps from CompressDirect,
// Section "Implementation").
//
// Stable compaction of the nonzero counts (ids stay ascending), then a
// stable least-significant-digit radix sort on the count with 8-bit digits,
// only over the bytes that the largest possible count (the token total)
// needs. Ranks inside a tile come from wave64 ballots over the digit bits,
// so equal digits keep their input order and ties stay in id order.
#include "device.h"
#include "radix.h"

namespace gt {

// Nonzero counts per 4096-id block.
__global__ __launch_bounds__(256) void k_nz_count(const uint64_t* counts, int32_t V, uint32_t* blk_cnt) {
  const int64_t i0 = blockIdx.x * (int64_t)kRadixTile + threadIdx.x * 16;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (i0 + k < V && counts[i0 + k] != 0) ++c;
  __shared__ uint32_t lds[4];
  uint32_t total;
  block_exclusive_scan_256(c, lds, &total);
  if (threadIdx.x == 0) blk_cnt[blockIdx.x] = total;
}

// Write (count, id) of the nonzero entries at their compacted positions.
__global__ __launch_bounds__(256) void k_nz_write(const uint64_t* counts, int32_t V, const uint32_t* blk_off,
                                                  uint64_t* key, uint32_t* val) {
  const int64_t i0 = blockIdx.x * (int64_t)kRadixTile + threadIdx.x * 16;
  uint64_t c[16];
  uint32_t n = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    c[k] = (i0 + k < V) ? counts[i0 + k] : 0;
    n += c[k] != 0;
  }
  __shared__ uint32_t lds[4];
  uint32_t total;
  uint32_t pos = blk_off[blockIdx.x] + block_exclusive_scan_256(n, lds, &total);
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (c[k] != 0) {
      key[pos] = c[k];
      val[pos] = (uint32_t)(i0 + k);
      ++pos;
    }
}

int64_t sort_scratch_hist_entries(int64_t n) { return radix_hist_entries(n); }

hipError_t launch_sort_by_count(const uint64_t* counts, int32_t V, int key_bytes, SortScratch& sc, uint32_t* ids_out,
                                uint64_t* cnt_out, int64_t* num_out, hipStream_t s) {
  const int nb = (int)((V + kRadixTile - 1) / kRadixTile);
  uint32_t* blk = sc.hist;  // reused: block counts, then digit histograms
  k_nz_count<<<nb, 256, 0, s>>>(counts, V, blk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_u32(blk, nb, sc.num, blk + nb, s);  // exclusive offsets; total K -> *sc.num
  if (e != hipSuccess) return e;
  k_nz_write<<<nb, 256, 0, s>>>(counts, V, blk, sc.key[0], sc.val[0]);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = radix_sort_pairs<uint32_t>(sc.key[0], sc.val[0], sc.key[1], sc.val[1], sc.num, V, 0, 8 * key_bytes,
                                 /*descending=*/true, sc.hist, cnt_out, ids_out, s);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(num_out, sc.num, sizeof(int64_t), hipMemcpyDeviceToDevice, s);
}

}  // namespace gt

// k_sort.hip -- "sort": the words with a nonzero count, by count descending
// then word id ascending (an application the paper keeps from CompressDirect,
// Section "Implementation").
//
// A stable least-significant-digit radix sort of all V (count, id) pairs on
// the count, over the bits that the largest possible count (the token total)
// needs, in as few passes of at most 9-bit digits as cover them (3 passes
// for 27 bits). The first pass reads the counts directly (ids are the
// positions, so ties start in id order) and counts the zeros; zero counts
// sort last, and K = V - zeros. A pass is three launches: per-tile digit
// histograms (digit-major), a scan of each digit's column over the tiles
// (one workgroup per digit, which also leaves the digit's total), and the
// stable scatter, which turns the digit totals into digit starts itself.
// Tiles are 4096 keys (1024 threads x 4); within a tile every wave owns 256
// consecutive keys, ranks equal digits by ballots over the digit bits and
// keeps running counts per digit in LDS, and waves are ordered by a prefix
// over their counts.
//
// The same passes sort the packed n-gram keys of the sequence count
// ascending (launch_sort_key_bits): their digits are taken from the bits
// that word ids can occupy only (36 bits for bigrams over a 2*10^5-word
// vocabulary, 4 passes instead of one per occupied byte), with the counts as
// 64-bit values.
#include "device.h"
#include "radix.h"

namespace gt {

constexpr int kWsThreads = 1024;
constexpr int kWsPer = 4;
constexpr int kWsTile = kWsThreads * kWsPer;
constexpr int kWsWaves = kWsThreads / 64;
constexpr int kWsMaxBits = 9;
constexpr int kWsMaxDigits = 1 << kWsMaxBits;
constexpr int kWsColThreads = 256;

// Digit of a count for a descending sort: dbits bits of ~count at shift.
struct CountDigit {
  int shift, dbits;
  __device__ __forceinline__ uint32_t operator()(uint64_t count) const {
    return (uint32_t)((~count >> shift) & ((1u << dbits) - 1u));
  }
};

// Digit of a key for an ascending sort over chosen bits: up to four bit
// ranges of the key, [s[i], s[i] + l[i]), joined low to high.
struct BitsDigit {
  int dbits;
  uint8_t s[4], l[4];
  __device__ __forceinline__ uint32_t operator()(uint64_t k) const {
    uint32_t d = 0;
    int at = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (l[i]) d |= (uint32_t)((k >> s[i]) & ((1ull << l[i]) - 1u)) << at;
      at += l[i];
    }
    return d;
  }
};

// Lanes of the wave whose digit equals this lane's (among `valid` lanes).
__device__ __forceinline__ uint64_t ws_peers(bool valid, uint32_t d, int dbits) {
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < dbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Digit histogram of every tile: hist[d * nb + tile]. The first pass reads
// the counts and also writes the tile's number of zero counts.
template <bool kFirst, class Dig>
__global__ __launch_bounds__(kWsThreads) void k_ws_hist(const uint64_t* keys, int64_t V, Dig dig, uint32_t* hist,
                                                        int nb, uint32_t* zeros) {
  __shared__ uint32_t h[kWsMaxDigits];
  __shared__ uint32_t zs[kWsWaves];
  const int dbits = dig.dbits;
  const int nd = 1 << dbits;
  for (int d = threadIdx.x; d < nd; d += kWsThreads) h[d] = 0;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int64_t base = (int64_t)blockIdx.x * kWsTile + (int64_t)wave * (kWsPer * 64);
  uint32_t z = 0;
#pragma unroll
  for (int j = 0; j < kWsPer; ++j) {
    const int64_t idx = base + j * 64 + lane;
    const bool valid = idx < V;
    const uint64_t k = valid ? keys[idx] : 0;
    if (kFirst) z += valid && k == 0;
    const uint32_t d = dig(k);
    const uint64_t peers = ws_peers(valid, d, dbits);
    // one LDS add per distinct digit of the step (Zipf-hot digits would
    // otherwise serialize on one address)
    if (valid && (peers & lanes_below()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
  }
  if (kFirst) {
    for (int o = 32; o >= 1; o >>= 1) z += __shfl_xor(z, o);
    if (lane == 0) zs[wave] = z;
  }
  __syncthreads();
  for (int d = threadIdx.x; d < nd; d += kWsThreads) hist[(int64_t)d * nb + blockIdx.x] = h[d];
  if (kFirst && threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kWsWaves; ++w) t += zs[w];
    zeros[blockIdx.x] = t;
  }
}

// Column scan: workgroup d scans hist[d * nb .. d * nb + nb) (exclusive, in
// place) and writes the digit's total to tot[d]. With `zeros`, workgroup 0
// also writes *num = V - (zero counts over the tiles).
__global__ __launch_bounds__(kWsColThreads) void k_ws_colscan(uint32_t* hist, int nb, uint32_t* tot,
                                                              const uint32_t* zeros, int64_t V, int64_t* num) {
  __shared__ uint32_t part[kWsColThreads / 64];
  uint32_t* col = hist + (int64_t)blockIdx.x * nb;
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kWsColThreads) {
    const int b = b0 + (int)threadIdx.x;
    const uint32_t v = b < nb ? col[b] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan_256(v, part, &total);
    if (b < nb) col[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
  if (zeros && blockIdx.x == 0) {
    uint32_t z = 0;
    for (int b = threadIdx.x; b < nb; b += kWsColThreads) z += zeros[b];
    uint32_t total;
    block_exclusive_scan_256(z, part, &total);
    if (threadIdx.x == 0) *num = V - (int64_t)total;
  }
}

// Stable scatter of one pass. The first pass of the count sort takes the
// counts as keys and the positions as values.
template <bool kFirst, class Dig, typename VT>
__global__ __launch_bounds__(kWsThreads) void k_ws_scatter(const uint64_t* kin, const VT* vin, uint64_t* kout,
                                                           VT* vout, int64_t V, Dig dig, const uint32_t* hist,
                                                           const uint32_t* tot, int nb) {
  __shared__ uint32_t wcnt[kWsWaves][kWsMaxDigits];
  __shared__ uint32_t base[kWsWaves][kWsMaxDigits];
  __shared__ uint32_t dstart[kWsMaxDigits];
  __shared__ uint32_t part[kWsWaves];
  const int dbits = dig.dbits;
  const int nd = 1 << dbits;
  const int wave = threadIdx.x >> 6, lane = lane_id();
  // digit starts: exclusive scan of the digit totals (nd <= 512 <= threads)
  {
    const uint32_t v = (int)threadIdx.x < nd ? tot[threadIdx.x] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) part[wave] = x;
    for (int d = lane; d < nd; d += 64) wcnt[wave][d] = 0;
    __syncthreads();
    uint32_t off = x - v;
    for (int w = 0; w < wave; ++w) off += part[w];
    if ((int)threadIdx.x < nd) dstart[threadIdx.x] = off;
  }
  const int64_t t0 = (int64_t)blockIdx.x * kWsTile + (int64_t)wave * (kWsPer * 64);
  uint64_t key[kWsPer];
  VT val[kWsPer];
  uint32_t rank[kWsPer], dgt[kWsPer];
#pragma unroll
  for (int j = 0; j < kWsPer; ++j) {
    const int64_t idx = t0 + j * 64 + lane;
    const bool valid = idx < V;
    const uint64_t k = valid ? kin[idx] : 0;
    const uint32_t d = dig(k);
    const uint64_t peers = ws_peers(valid, d, dbits);
    const uint32_t before = wcnt[wave][d];
    const uint32_t r = (uint32_t)__popcll(peers & lanes_below());
    __builtin_amdgcn_wave_barrier();
    if (valid && r == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    key[j] = k;
    val[j] = valid ? (kFirst ? (VT)idx : vin[idx]) : VT(0);
    rank[j] = valid ? before + r : 0xffffffffu;
    dgt[j] = d;
  }
  __syncthreads();
  for (int d = threadIdx.x; d < nd; d += kWsThreads) {
    uint32_t acc = dstart[d] + hist[(int64_t)d * nb + blockIdx.x];
    for (int w = 0; w < kWsWaves; ++w) {
      base[w][d] = acc;
      acc += wcnt[w][d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kWsPer; ++j) {
    if (rank[j] == 0xffffffffu) continue;
    const uint32_t pos = base[wave][dgt[j]] + rank[j];
    kout[pos] = key[j];
    vout[pos] = val[j];
  }
}

int64_t sort_scratch_hist_entries(int64_t n) { return radix_hist_entries(n); }

int64_t word_sort_hist_entries(int64_t V) {
  const int64_t nb = (V + kWsTile - 1) / kWsTile;
  return (int64_t)kWsMaxDigits * (nb > 0 ? nb : 1) + (nb > 0 ? nb : 1) + kWsMaxDigits;
}

hipError_t launch_sort_by_count(const uint64_t* counts, int32_t V, int key_bits, SortScratch& sc, uint32_t* ids_out,
                                uint64_t* cnt_out, int64_t* num_out, hipStream_t s) {
  const int nb = (int)((V + kWsTile - 1) / kWsTile);
  if (nb == 0) return launch_fill_i32(reinterpret_cast<int32_t*>(num_out), 2, 0, s);
  const int bits = key_bits < 1 ? 1 : (key_bits > 64 ? 64 : key_bits);
  const int npass = (bits + kWsMaxBits - 1) / kWsMaxBits;
  const int dbits = (bits + npass - 1) / npass;
  uint32_t* hist = sc.hist;
  uint32_t* zeros = sc.hist + (int64_t)kWsMaxDigits * nb;
  uint32_t* tot = zeros + nb;
  const uint64_t* kin = counts;
  const uint32_t* vin = nullptr;
  for (int p = 0; p < npass; ++p) {
    const int shift = p * dbits;
    const bool last = p == npass - 1;
    uint64_t* kdst = last ? cnt_out : sc.key[p & 1];
    uint32_t* vdst = last ? ids_out : sc.val[p & 1];
    const CountDigit dig{shift, dbits};
    if (p == 0) k_ws_hist<true><<<nb, kWsThreads, 0, s>>>(kin, V, dig, hist, nb, zeros);
    else k_ws_hist<false><<<nb, kWsThreads, 0, s>>>(kin, V, dig, hist, nb, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ws_colscan<<<1 << dbits, kWsColThreads, 0, s>>>(hist, nb, tot, p == 0 ? zeros : nullptr, V, num_out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (p == 0) k_ws_scatter<true><<<nb, kWsThreads, 0, s>>>(kin, vin, kdst, vdst, V, dig, hist, tot, nb);
    else k_ws_scatter<false><<<nb, kWsThreads, 0, s>>>(kin, vin, kdst, vdst, V, dig, hist, tot, nb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    kin = kdst;
    vin = vdst;
  }
  return hipSuccess;
}

int64_t key_sort_hist_entries(int64_t n) { return word_sort_hist_entries(n); }

hipError_t launch_sort_key_bits(uint64_t* k0, uint64_t* v0, uint64_t* k1, uint64_t* v1, int64_t n,
                                const KeyBits& kb, uint32_t* hist, uint64_t* kout, uint64_t* vout, hipStream_t s) {
  const int nb = (int)((n + kWsTile - 1) / kWsTile);
  if (nb == 0) return hipSuccess;
  int total = 0;
  for (int i = 0; i < kb.nseg; ++i) total += kb.len[i];
  if (kb.nseg < 1 || kb.nseg > 4 || total < 1 || total > 64 || n >= (1ll << 32)) return hipErrorInvalidValue;
  const int npass = (total + kWsMaxBits - 1) / kWsMaxBits;
  const int dbits = (total + npass - 1) / npass;
  uint32_t* tot = hist + (int64_t)kWsMaxDigits * nb + nb;
  const uint64_t* kin = k0;
  const uint64_t* vin = v0;
  int seg = 0, used = 0;  // next significant bit: bit `used` of segment `seg`
  for (int p = 0; p < npass; ++p) {
    BitsDigit dig{};
    int want = dbits, parts = 0;
    while (want > 0 && seg < kb.nseg) {
      const int take = kb.len[seg] - used < want ? kb.len[seg] - used : want;
      if (parts == 4) return hipErrorInvalidValue;
      dig.s[parts] = (uint8_t)(kb.lo[seg] + used);
      dig.l[parts] = (uint8_t)take;
      ++parts;
      want -= take;
      used += take;
      if (used == kb.len[seg]) ++seg, used = 0;
    }
    dig.dbits = dbits - want;
    const bool last = p == npass - 1;
    uint64_t* kdst = last ? kout : ((p & 1) == 0 ? k1 : k0);
    uint64_t* vdst = last ? vout : ((p & 1) == 0 ? v1 : v0);
    k_ws_hist<false><<<nb, kWsThreads, 0, s>>>(kin, n, dig, hist, nb, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ws_colscan<<<1 << dig.dbits, kWsColThreads, 0, s>>>(hist, nb, tot, nullptr, n, nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ws_scatter<false><<<nb, kWsThreads, 0, s>>>(kin, vin, kdst, vdst, n, dig, hist, tot, nb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    kin = kdst;
    vin = vdst;
  }
  return hipSuccess;
}

}  // namespace gt

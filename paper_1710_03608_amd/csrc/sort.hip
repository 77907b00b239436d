// Stable LSD radix sort of 64-bit keys with a 32-bit payload (8-bit digits).
//
// Per digit pass: a histogram kernel counts digits per 2048-key tile, a spine
// kernel turns the digit-major (digit, tile) counts into exclusive offsets
// (one workgroup per digit), and a scatter kernel ranks keys inside each
// tile with wave ballots (stable: earlier keys of a digit get lower ranks),
// orders the tile by digit in LDS and writes it out from there, so the keys
// of one digit leave a tile as one contiguous run.  Integer work only, so
// results are exact and independent of scheduling.
#include "kernels.h"

namespace ctd {

namespace {
constexpr int kSortBlock = 256;                 // 4 waves
constexpr int kSortItems = 8;                   // keys per lane
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kRadix = 256;
constexpr int kWavesPerBlock = kSortBlock / kWave;
constexpr int kWaveSpan = kWave * kSortItems;   // keys per wave per tile

__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                           int64_t n_max, const int32_t* d_n,
                                                           int shift, uint32_t* __restrict__ hist,
                                                           int nblocks) {
  __shared__ uint32_t cnt[kRadix];
  const int64_t n = d_n ? (int64_t)*d_n : n_max;
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base < n) {
#pragma unroll 4
    for (int i = 0; i < kSortItems; ++i) {
      const int64_t e = base + (int64_t)i * kSortBlock + threadIdx.x;
      if (e < n) atomicAdd(&cnt[(uint32_t)(keys[e] >> shift) & 0xFFu], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// One workgroup per digit: exclusive scan of that digit's per-tile counts,
// digit total into dtot[digit].
__global__ __launch_bounds__(kSortBlock) void k_radix_spine(uint32_t* __restrict__ hist,
                                                            uint32_t* __restrict__ dtot,
                                                            int nblocks) {
  __shared__ uint32_t tmp[kWavesPerBlock + 1];
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nblocks; b0 += kSortBlock) {
    const int b = b0 + threadIdx.x;
    const uint32_t v = b < nblocks ? row[b] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t, kSortBlock>(v, tmp, &tot);
    if (b < nblocks) row[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
    uint64_t* __restrict__ okeys, uint32_t* __restrict__ ovals, int64_t n_max,
    const int32_t* d_n, int shift, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ dtot, int nblocks) {
  __shared__ uint32_t gofs[kRadix];
  __shared__ uint32_t lofs[kRadix];
  __shared__ uint32_t wcnt[kWavesPerBlock][kRadix];
  __shared__ uint32_t wpre[kWavesPerBlock][kRadix];
  __shared__ uint32_t tmp[kWavesPerBlock + 1];
  __shared__ uint64_t sk[kSortTile];   // the tile ordered by digit (stable)
  __shared__ uint32_t sv[kSortTile];
  const int64_t n = d_n ? (int64_t)*d_n : n_max;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= n) return;  // uniform for the whole block

  const uint32_t t = dtot[threadIdx.x];
  uint32_t tot;
  const uint32_t ex = block_excl_scan<uint32_t, kSortBlock>(t, tmp, &tot);
  gofs[threadIdx.x] = ex + hist[(int64_t)threadIdx.x * nblocks + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();

  const int w = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
  uint64_t k[kSortItems];
  uint32_t v[kSortItems];
  uint32_t rk[kSortItems];
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t e = base + (int64_t)w * kWaveSpan + (int64_t)it * kWave + lane;
    const bool valid = e < n;
    const uint64_t key = valid ? keys[e] : 0ull;
    const uint32_t val = valid ? vals[e] : 0u;
    const uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bm = __ballot(bit);
      peers &= bit ? bm : ~bm;
    }
    // Same-wave LDS operations complete in issue order, so every lane reads the
    // count before the group's lowest lane advances it.
    const uint32_t prior = wcnt[w][d];
    if (valid && (peers & lt) == 0ull) wcnt[w][d] = prior + (uint32_t)__popcll(peers);
    rk[it] = prior + (uint32_t)__popcll(peers & lt);
    k[it] = key;
    v[it] = val;
  }
  __syncthreads();
  uint32_t run = 0;   // the tile's count of digit threadIdx.x
#pragma unroll
  for (int w2 = 0; w2 < kWavesPerBlock; ++w2) {
    const uint32_t c = wcnt[w2][threadIdx.x];
    wpre[w2][threadIdx.x] = run;
    run += c;
  }
  uint32_t tile_tot;
  lofs[threadIdx.x] = block_excl_scan<uint32_t, kSortBlock>(run, tmp, &tile_tot);
  __syncthreads();
  // a key's place in the tile ordered by digit is its place among the
  // tile's keys of that digit after the tile's keys of smaller digits; the
  // ordered tile is then written out with neighbouring threads on
  // neighbouring places, so each digit's run of the output is written whole
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t e = base + (int64_t)w * kWaveSpan + (int64_t)it * kWave + lane;
    if (e < n) {
      const uint32_t d = (uint32_t)(k[it] >> shift) & 0xFFu;
      const uint32_t lp = lofs[d] + wpre[w][d] + rk[it];
      sk[lp] = k[it];
      sv[lp] = v[it];
    }
  }
  __syncthreads();
  const int m = (int)min<int64_t>(kSortTile, n - base);
  for (int j = threadIdx.x; j < m; j += kSortBlock) {
    const uint64_t key = sk[j];
    const uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
    const uint32_t pos = gofs[d] + ((uint32_t)j - lofs[d]);
    okeys[pos] = key;
    ovals[pos] = sv[j];
  }
}
}  // namespace

size_t radix_sort_hist_elems(int64_t n_max) {
  const int64_t nb = n_max > 0 ? (n_max + kSortTile - 1) / kSortTile : 1;
  return (size_t)(kRadix * nb + kRadix);
}

bool radix_sort(hipStream_t st, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                uint32_t* vals_alt, int64_t n_max, const int32_t* d_n, int nbits,
                uint32_t* hist_ws) {
  if (n_max <= 0 || nbits <= 0) return false;
  const int nblocks = div_up(n_max, kSortTile);
  uint32_t* hist = hist_ws;
  uint32_t* dtot = hist_ws + (size_t)kRadix * nblocks;
  bool alt = false;
  for (int shift = 0; shift < nbits; shift += 8) {
    const uint64_t* ki = alt ? keys_alt : keys;
    const uint32_t* vi = alt ? vals_alt : vals;
    uint64_t* ko = alt ? keys : keys_alt;
    uint32_t* vo = alt ? vals : vals_alt;
    hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(kSortBlock), 0, st, ki, n_max, d_n,
                       shift, hist, nblocks);
    hipLaunchKernelGGL(k_radix_spine, dim3(kRadix), dim3(kSortBlock), 0, st, hist, dtot,
                       nblocks);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kSortBlock), 0, st, ki, vi, ko, vo,
                       n_max, d_n, shift, hist, dtot, nblocks);
    alt = !alt;
  }
  return alt;
}

}  // namespace ctd

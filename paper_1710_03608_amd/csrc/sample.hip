// Weighted sampling with replacement from the column distribution P(i) and
// unique selection of the drawn fibers (Algorithms 1 and 2).
//
// Draw j: r = Philox4x32-10(counter (j, j>>32, step, tensor), key (seed,
// seed>>32)) read as a 128-bit integer, target t = floor(r * W / 2^128)
// computed exactly with 64-bit high/low products, drawn fiber = the fiber
// holding the first nonzero whose inclusive weight prefix exceeds t.
#include "kernels.h"

namespace ctd {

namespace {
constexpr int kDrawBlock = 256;
constexpr int kUniqBlock = 1024;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies by fixed odd multipliers, XOR of the high halves with
// the other counter words and the round key, and a word permutation; the key
// advances by two Weyl constants between rounds.
__device__ inline void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
}

// floor(r * W / 2^128) for a 128-bit r = (hi, lo) and W < 2^62.
__device__ inline uint64_t scale_target(uint64_t lo, uint64_t hi, uint64_t W) {
  const uint64_t a_hi = __umul64hi(lo, W);
  const uint64_t b_lo = hi * W;
  const uint64_t b_hi = __umul64hi(hi, W);
  const uint64_t mid = a_hi + b_lo;
  return b_hi + (mid < a_hi ? 1ull : 0ull);
}

// first index e in [0, n) with a[e] > t (n if none)
template <typename T>
__device__ inline int64_t upper_bound_dev(const T* a, int64_t n, T t) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] > t)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

__global__ __launch_bounds__(kDrawBlock) void k_draws(const uint64_t* __restrict__ qpref,
                                                      const int32_t* __restrict__ fptr,
                                                      const uint64_t* __restrict__ fid,
                                                      int64_t nnz, int64_t s, uint64_t seed,
                                                      uint32_t step, uint32_t tensor,
                                                      int32_t* __restrict__ draw_fi,
                                                      uint64_t* __restrict__ draw_fid,
                                                      DevScalars* sc) {
  const int64_t j = (int64_t)blockIdx.x * kDrawBlock + threadIdx.x;
  if (j >= s) return;
  if (sc->status != 0 || sc->W == 0) {
    draw_fi[j] = 0;
    draw_fid[j] = 0;
    return;
  }
  uint32_t c0 = (uint32_t)j, c1 = (uint32_t)((uint64_t)j >> 32), c2 = step, c3 = tensor;
  philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t lo = (uint64_t)c0 | ((uint64_t)c1 << 32);
  const uint64_t hi = (uint64_t)c2 | ((uint64_t)c3 << 32);
  const uint64_t W = sc->W;
  const uint64_t t = scale_target(lo, hi, W);
  const int64_t e = upper_bound_dev<uint64_t>(qpref, nnz, t);
  const int32_t n_f = sc->n_f;
  const int64_t f = upper_bound_dev<int32_t>(fptr, n_f, (int32_t)e) - 1;
  draw_fi[j] = (int32_t)f;
  draw_fid[j] = fid[f];
}

__global__ __launch_bounds__(kDrawBlock) void k_locate_given(const uint64_t* __restrict__ fid,
                                                             int64_t s,
                                                             const uint64_t* __restrict__ draw_fid,
                                                             int32_t* __restrict__ draw_fi,
                                                             DevScalars* sc) {
  const int64_t j = (int64_t)blockIdx.x * kDrawBlock + threadIdx.x;
  if (j >= s) return;
  const int32_t n_f = sc->n_f;
  const uint64_t x = draw_fid[j];
  int64_t lo = 0, hi = n_f;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (fid[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo >= n_f || fid[lo] != x) {
    latch_status(sc, CTD_ERR_INVALID_ARG);
    lo = 0;
  }
  draw_fi[j] = (int32_t)lo;
}

// Single workgroup: bitonic sort of the s draws in LDS, then unique positions,
// multiplicities, probabilities and merge scales.
__global__ __launch_bounds__(kUniqBlock) void k_unique(
    const int32_t* __restrict__ draw_fi, int64_t s, const uint64_t* __restrict__ qpref,
    const int32_t* __restrict__ fptr, const uint64_t* __restrict__ fid,
    int32_t* __restrict__ uniq_fi, uint64_t* __restrict__ uniq_fid, int32_t* __restrict__ counts,
    double* __restrict__ prob, double* __restrict__ scale, DevScalars* sc) {
  __shared__ int32_t a[CTD_MAX_DRAWS];
  __shared__ int32_t pos[CTD_MAX_DRAWS + 1];
  __shared__ uint32_t tmp[kUniqBlock / kWave + 1];
  if (sc->status != 0 || sc->W == 0 || sc->n_f == 0) {
    if (threadIdx.x == 0) sc->s_unique = 0;
    return;
  }
  int P = 1;
  while (P < s) P <<= 1;
  for (int i = threadIdx.x; i < P; i += kUniqBlock) a[i] = i < s ? draw_fi[i] : 0x7FFFFFFF;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += kUniqBlock) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int32_t x = a[i], y = a[ixj];
          const bool up = (i & k) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // unique starts, contiguous chunk per thread
  constexpr int kPer = CTD_MAX_DRAWS / kUniqBlock;
  const int b = threadIdx.x * kPer;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int e = b + i;
    if (e < s && (e == 0 || a[e] != a[e - 1])) ++c;
  }
  uint32_t tot;
  uint32_t ex = block_excl_scan<uint32_t, kUniqBlock>(c, tmp, &tot);
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int e = b + i;
    if (e < s && (e == 0 || a[e] != a[e - 1])) pos[ex++] = e;
  }
  if (threadIdx.x == 0) {
    pos[tot] = (int32_t)s;
    sc->s_unique = (int32_t)tot;
  }
  __syncthreads();
  const uint64_t W = sc->W;
  for (int k = threadIdx.x; k < (int)tot; k += kUniqBlock) {
    const int32_t f = a[pos[k]];
    const int32_t n = pos[k + 1] - pos[k];
    const int32_t e0 = fptr[f], e1 = fptr[f + 1];
    const uint64_t w = qpref[e1 - 1] - (e0 > 0 ? qpref[e0 - 1] : 0ull);
    const double p = (double)w / (double)W;
    uniq_fi[k] = f;
    uniq_fid[k] = fid[f];
    counts[k] = n;
    prob[k] = p;
    scale[k] = sqrt((double)n / ((double)s * p));
  }
}
}  // namespace

void launch_draws(hipStream_t st, const uint64_t* qpref, const int32_t* fptr,
                  const uint64_t* fid, int64_t nnz, int64_t s, uint64_t seed, uint32_t step,
                  uint32_t tensor, int32_t* draw_fi, uint64_t* draw_fid, DevScalars* sc) {
  hipLaunchKernelGGL(k_draws, dim3(div_up(s, kDrawBlock)), dim3(kDrawBlock), 0, st, qpref, fptr,
                     fid, nnz, s, seed, step, tensor, draw_fi, draw_fid, sc);
}

void launch_locate_given(hipStream_t st, const uint64_t* fid, int64_t s,
                         const uint64_t* draw_fid, int32_t* draw_fi, DevScalars* sc) {
  hipLaunchKernelGGL(k_locate_given, dim3(div_up(s, kDrawBlock)), dim3(kDrawBlock), 0, st, fid,
                     s, draw_fid, draw_fi, sc);
}

void launch_unique(hipStream_t st, const int32_t* draw_fi, int64_t s, const uint64_t* qpref,
                   const int32_t* fptr, const uint64_t* fid, int32_t* uniq_fi,
                   uint64_t* uniq_fid, int32_t* counts, double* prob, double* scale,
                   DevScalars* sc) {
  hipLaunchKernelGGL(k_unique, dim3(1), dim3(kUniqBlock), 0, st, draw_fi, s, qpref, fptr, fid,
                     uniq_fi, uniq_fid, counts, prob, scale, sc);
}

}  // namespace ctd

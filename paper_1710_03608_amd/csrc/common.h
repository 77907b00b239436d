// Shared device-side definitions of the CTD library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/ctd.h"

namespace ctd {

constexpr int kWave = 64;

// Scalars produced on the device and read back only by ctd_get_result /
// ctd_sync, so a whole decomposition runs without host round trips.
// Fibers with more than kLongFiber nonzeros are gathered by a workgroup of
// kLongWaves waves per column slice of the projection (at most kProjSlices
// slices, one per XCD) or per column chunk of C's columns.
constexpr int kLongFiber = 64;
constexpr int kLongWaves = 8;
constexpr int kProjSlices = 8;
// Hot rows of the projection of a large input: at most kHotMax rows, counted
// over every kHotSample-th fiber of 2 .. kLongFiber nonzeros and each holding
// at least kHotMinCount nonzeros of that sample, for inputs of more than
// kHotMinNnz nonzeros over at most kHotMaxRows rows (an LDS histogram in
// each of kHotParts workgroups).
constexpr int kHotMax = 64;
constexpr int kHotSample = 8;
constexpr int kHotMinCount = 64;
constexpr int64_t kHotMinNnz = int64_t(1) << 18;
constexpr int kHotMaxRows = 16384;
constexpr int kHotParts = 256;

struct DevScalars {
  uint64_t W;            // total integer sampling weight of the last input
  uint64_t vmax2_bits;   // bit pattern of the largest squared value (positive doubles order like u64)
  double norm2;          // ||X||_F^2 of the last input (tensor or slice)
  double err2;           // ||X - P X||_F^2 of the last input
  double total_norm2;    // all data decomposed so far (CTD-S tensor plus CTD-D slices)
  double total_err2;     // ||X - X~||_F^2 over all data so far
  int64_t n_cols_total;  // CTD-D: columns of C held
  int32_t status;        // first device-detected error (ctd_status), 0 if none
  int32_t sigma;         // weight quantization exponent
  int32_t n_f;           // non-empty fibers of the last input
  int32_t s_unique;      // s' of the last call
  int32_t s_tilde;       // fibers accepted by the last call
  int32_t n_accept_total;// accepted fibers held in R
  int32_t allow_empty;   // CTD-D: an all-zero slice is not an error
  int32_t base_accept;   // fibers kept before the current call
  int32_t wacc_base;     // CTD-D: fibers kept before the current batch of slices
  int32_t n_long;        // fibers listed for the workgroup-per-chunk gather
  int32_t blk_na;        // fibers kept by the current candidate block
  int32_t blk_reorth;    // the block's first Cholesky-QR pass left it non-orthonormal
  int32_t n_cold;        // fibers listed for the gather over their cold rows
};
__device__ inline void latch_status(DevScalars* sc, int code) {
  atomicCAS(&sc->status, 0, code);
}

__device__ inline int lane_id() { return __lane_id(); }

typedef double dbl4 __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4f64 on gfx950: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; the 16 x 16 result D[i][j] sits in lane j + 16 (i % 4)
// at component i / 4 (lane l holds D[l / 16 + 4 r][l % 16], r = 0..3).
__device__ inline dbl4 mfma16(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Inclusive scan across the 64 lanes of a wave.
template <typename T>
__device__ inline T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  return v;
}

// Exclusive scan across a whole block of BLOCK threads.  `tmp` must hold
// BLOCK/64 elements of LDS.  Returns the exclusive prefix; *total gets the
// block sum.  Contains barriers: every thread of the block must call it.
template <typename T, int BLOCK>
__device__ inline T block_excl_scan(T v, T* tmp, T* total) {
  constexpr int NW = BLOCK / kWave;
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  T inc = wave_incl_scan(v);
  if (lane == kWave - 1) tmp[w] = inc;
  __syncthreads();
  if (w == 0) {
    T x = lane < NW ? tmp[lane] : T(0);
    T xi = wave_incl_scan(x);
    if (lane < NW) tmp[lane] = xi - x;
    if (lane == NW - 1) tmp[NW] = xi;
  }
  __syncthreads();
  T res = tmp[w] + inc - v;
  *total = tmp[NW];
  __syncthreads();
  return res;
}

// Deterministic block sum (fixed reduction tree).
template <typename T, int BLOCK>
__device__ inline T block_sum(T v, T* tmp) {
  constexpr int NW = BLOCK / kWave;
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  v = wave_sum(v);
  if (lane == 0) tmp[w] = v;
  __syncthreads();
  T r = T(0);
  if (threadIdx.x == 0) {
    for (int i = 0; i < NW; ++i) r += tmp[i];
    tmp[0] = r;
  }
  __syncthreads();
  r = tmp[0];
  __syncthreads();
  return r;
}

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace ctd

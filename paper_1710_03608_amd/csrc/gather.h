// Row gathers along the nonzeros of a fiber: z = sum_e v_e A[r_e, c0 : c0 + w]
// for a dense row-major A (the basis Q for the residual, the kept fibers R for
// columns of C).  Fibers of up to kLongFiber nonzeros are done by one wave;
// longer ones are listed and split over the kLongWaves waves of a workgroup,
// one workgroup per column chunk, so that a heavy fiber (a hot destination
// under a Zipf law) does not serialize a whole launch.
#pragma once
#include "common.h"

namespace ctd {


__device__ inline int32_t read_lane(int32_t v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}
template <typename T>
__device__ inline T read_lane(T v, int lane) {
  static_assert(sizeof(T) == 8 || sizeof(T) == 4, "float or double");
  if constexpr (sizeof(T) == 8) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
  } else {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
  }
}

// VEC consecutive elements of a row (32 B per lane: two 16 B loads).
template <typename T, int VEC>
__device__ inline void load_seg(const T* p, T (&x)[VEC]) {
#pragma unroll
  for (int k = 0; k < VEC; k += 16 / sizeof(T)) {
    if constexpr (sizeof(T) == 8) {
      const double2 u = *(const double2*)(p + k);
      x[k] = u.x;
      x[k + 1] = u.y;
    } else {
      const float4 u = *(const float4*)(p + k);
      x[k] = u.x;
      x[k + 1] = u.y;
      x[k + 2] = u.z;
      x[k + 3] = u.w;
    }
  }
}

// Nonzeros e = eb + 0 .. n - 1 (n <= 64) of a fiber, their (row, value) held
// one per lane in (rr, vv): acc0 += sum v_e A[r_e][ca ..], acc1 likewise at
// cb.  qa / qb point at row 0, column ca / cb (valid when ina / inb).  Two
// nonzeros times two segments are in flight per iteration.
template <typename T, int VEC>
__device__ inline void gather_batch(int32_t rr, T vv, int n, const T* qa, const T* qb, bool ina,
                                    bool inb, int64_t ld, T (&acc0)[VEC], T (&acc1)[VEC]) {
  int k = 0;
  for (; k + 1 < n; k += 2) {
    const int64_t r0 = read_lane(rr, k), r1 = read_lane(rr, k + 1);
    const T v0 = read_lane(vv, k), v1 = read_lane(vv, k + 1);
    T x0[VEC], x1[VEC], y0[VEC], y1[VEC];
    if (ina) {
      load_seg<T, VEC>(qa + r0 * ld, x0);
      load_seg<T, VEC>(qa + r1 * ld, x1);
    }
    if (inb) {
      load_seg<T, VEC>(qb + r0 * ld, y0);
      load_seg<T, VEC>(qb + r1 * ld, y1);
    }
    if (ina) {
#pragma unroll
      for (int j = 0; j < VEC; ++j) acc0[j] += v0 * x0[j] + v1 * x1[j];
    }
    if (inb) {
#pragma unroll
      for (int j = 0; j < VEC; ++j) acc1[j] += v0 * y0[j] + v1 * y1[j];
    }
  }
  if (k < n) {
    const int64_t r0 = read_lane(rr, k);
    const T v0 = read_lane(vv, k);
    T x0[VEC], y0[VEC];
    if (ina) load_seg<T, VEC>(qa + r0 * ld, x0);
    if (inb) load_seg<T, VEC>(qb + r0 * ld, y0);
    if (ina) {
#pragma unroll
      for (int j = 0; j < VEC; ++j) acc0[j] += v0 * x0[j];
    }
    if (inb) {
#pragma unroll
      for (int j = 0; j < VEC; ++j) acc1[j] += v0 * y0[j];
    }
  }
}

// One chunk of a long fiber by a workgroup of kLongWaves waves: wave wv
// takes nonzeros in interleaved batches of 64; the partial segments are added
// in LDS in wave order and wave 0 returns the chunk's z (lane l: columns
// c + VEC l ..) in `z`.  Every thread of the workgroup must call it.
template <typename T, int VEC>
__device__ inline void wg_gather_chunk(const int32_t* __restrict__ row, const T* __restrict__ vals,
                                       int32_t e0, int32_t e1, const T* q, bool in, int64_t ld,
                                       double* red /* [kLongWaves][VEC * kWave] */,
                                       double (&z)[VEC]) {
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  T acc[VEC], dummy[VEC];
#pragma unroll
  for (int j = 0; j < VEC; ++j) acc[j] = dummy[j] = T(0);
  for (int32_t eb = e0 + wv * kWave; eb < e1; eb += kLongWaves * kWave) {
    const int n = min(kWave, e1 - eb);
    const int32_t rr = lane < n ? row[eb + lane] : 0;
    const T vv = lane < n ? vals[eb + lane] : T(0);
    gather_batch<T, VEC>(rr, vv, n, q, q, in, false, ld, acc, dummy);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < VEC; ++j) red[(size_t)wv * VEC * kWave + lane * VEC + j] = (double)acc[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < VEC; ++j) {
    double s = 0.0;
    if (wv == 0) {
      for (int w = 0; w < kLongWaves; ++w) s += red[(size_t)w * VEC * kWave + lane * VEC + j];
    }
    z[j] = s;
  }
}

}  // namespace ctd

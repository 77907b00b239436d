// Projection of X_(alpha) onto span(R) over all nonzeros and the Frobenius
// residual (the final step of Algorithm 1, Eq. 14).
//
// With Q = R L^{-T} orthonormal, X~ = R U C_(alpha) = Q Q^T X_(alpha), so
// ||X - X~||_F^2 = sum_f (||x_f||^2 - ||Q^T x_f||^2) over the non-empty
// fibers f.  A kept fiber lies in span(R) and contributes exactly 0, so it is
// skipped.  A fiber with one nonzero v at row r has ||Q^T x_f||^2 = v^2
// ||Q_r||^2 (precomputed row leverage), so only fibers with two or more
// nonzeros run the sparse-times-dense product z_f = sum_e v_e Q[r_e, :]: one
// wave per fiber, 64 lanes across the columns of Q, the fiber's (row, value)
// pairs read as wave-uniform scalars, z kept in registers and reduced to
// ||z_f||^2 without ever being written.  Per-fiber residuals land in a
// fiber-indexed array and are summed by a fixed reduction tree, so the
// result is bit-identical from run to run.
#include "kernels.h"

namespace ctd {

namespace {
constexpr int kBlock = 256;
constexpr int kRedBlock = 1024;
constexpr int kRedItems = 8;

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

// VEC consecutive elements of a row of Q (32 B per lane: two 16 B loads).
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

// Residual of every fiber.  A wave takes 64 consecutive fibers, one per
// lane.  Fibers with one nonzero v at row r are done lane-parallel from the
// row leverage: ||Q^T x||^2 = v^2 ||Q_r||^2.  The wave then walks the others
// one at a time: z_f = sum_e v_e Q[r_e, :], lane l holding columns
// VEC l .. VEC l + VEC of each 64 VEC-column chunk.  The fiber's (row, value)
// pairs are loaded once per 64 nonzeros into lanes and broadcast with
// readlane, so the inner loop only issues row gathers: two nonzeros times two
// column chunks (8 KB per wave) in flight per iteration.  Column chunks of z
// are squared and summed as they complete; z is never written.  Kept fibers
// lie in span(Q) and get 0.
template <typename T, int VEC>
__global__ __launch_bounds__(kBlock) void k_proj_multi(ProjectArgs a, const DevScalars* sc) {
  constexpr int kCols = VEC * kWave;
  if (sc->status != 0) return;
  const int64_t n_f = sc->n_f;
  const int64_t ncols = *a.d_ncols;
  const int lane = lane_id();
  const T* Qb = sizeof(T) == 8 ? (const T*)a.Q : (const T*)a.Qf;
  const T* vals = sizeof(T) == 8 ? (const T*)a.val : (const T*)a.val32;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  for (int64_t fb = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave * kWave; fb < n_f;
       fb += nwaves * kWave) {
    const int64_t fl = fb + lane;
    bool multi = false;
    if (fl < n_f) {
      const int32_t s0 = a.fptr[fl], s1 = a.fptr[fl + 1];
      const bool kept = a.fiber_mark && a.fiber_mark[fl];
      if (kept) {
        a.resid[fl] = 0.0;
      } else if (s1 - s0 == 1) {
        const double v = a.val[s0];
        const double x2 = v * v;
        const double z2 = x2 * a.lev[a.row[s0]];
        a.resid[fl] = x2 - z2;
      } else {
        multi = true;
      }
    }
    uint64_t todo = __ballot(multi);
    while (todo) {
      const int i = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int64_t f = fb + i;
      const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
      double x2 = 0.0, z2 = 0.0;
      for (int64_t c0 = 0; c0 < ncols; c0 += 2 * kCols) {
        const int64_t ca = c0 + (int64_t)VEC * lane, cb = ca + kCols;
        const bool ina = ca < ncols, inb = cb < ncols;
        const T* qa = Qb + (ina ? ca : 0);
        const T* qb = Qb + (inb ? cb : 0);
        T acc0[VEC], acc1[VEC];
  #pragma unroll
        for (int k = 0; k < VEC; ++k) acc0[k] = acc1[k] = T(0);
        for (int32_t eb = e0; eb < e1; eb += kWave) {
          const int nb = min(kWave, e1 - eb);
          const int32_t rr = lane < nb ? a.row[eb + lane] : 0;
          const T vv = lane < nb ? vals[eb + lane] : T(0);
          if (c0 == 0 && lane < nb) x2 += a.val[eb + lane] * a.val[eb + lane];
          int k = 0;
          for (; k + 1 < nb; k += 2) {
            const int64_t r0 = read_lane(rr, k), r1 = read_lane(rr, k + 1);
            const T v0 = read_lane(vv, k), v1 = read_lane(vv, k + 1);
            T x0[VEC], x1[VEC], y0[VEC], y1[VEC];
            if (ina) {
              load_seg<T, VEC>(qa + r0 * a.ldq, x0);
              load_seg<T, VEC>(qa + r1 * a.ldq, x1);
            }
            if (inb) {
              load_seg<T, VEC>(qb + r0 * a.ldq, y0);
              load_seg<T, VEC>(qb + r1 * a.ldq, y1);
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
          if (k < nb) {
            const int64_t r0 = read_lane(rr, k);
            const T v0 = read_lane(vv, k);
            T x0[VEC], y0[VEC];
            if (ina) load_seg<T, VEC>(qa + r0 * a.ldq, x0);
            if (inb) load_seg<T, VEC>(qb + r0 * a.ldq, y0);
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
  #pragma unroll
        for (int j = 0; j < VEC; ++j) {
          const double d0 = (double)acc0[j], d1 = (double)acc1[j];
          z2 += (ca + j < ncols) ? d0 * d0 : 0.0;
          z2 += (cb + j < ncols) ? d1 * d1 : 0.0;
        }
      }
      x2 = wave_sum(x2);
      z2 = wave_sum(z2);
      if (lane == 0) a.resid[f] = x2 - z2;
    }
  }
}

__global__ __launch_bounds__(kRedBlock) void k_reduce_partial(const double* __restrict__ x,
                                                              double* __restrict__ partial,
                                                              const DevScalars* sc) {
  __shared__ double tmp[kRedBlock / kWave + 1];
  const int64_t n = sc->status == 0 ? sc->n_f : 0;
  const int64_t base = (int64_t)blockIdx.x * kRedBlock * kRedItems + (int64_t)threadIdx.x * kRedItems;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kRedItems; ++i)
    if (base + i < n) s += x[base + i];
  s = block_sum<double, kRedBlock>(s, tmp);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedBlock) void k_reduce_final(const double* __restrict__ partial,
                                                            int nparts, DevScalars* sc) {
  __shared__ double tmp[kRedBlock / kWave + 1];
  const int64_t n = sc->status == 0 ? sc->n_f : 0;
  const int used = (int)((n + kRedBlock * kRedItems - 1) / (kRedBlock * kRedItems));
  double s = 0.0;
  for (int i = threadIdx.x; i < used && i < nparts; i += kRedBlock) s += partial[i];
  s = block_sum<double, kRedBlock>(s, tmp);
  if (threadIdx.x == 0) sc->err2 = s;
}

}  // namespace

void launch_project(hipStream_t st, const ProjectArgs& a, int64_t nnz_max, DevScalars* sc,
                    hipEvent_t ev0, hipEvent_t ev1) {
  const int gm = std::max(1, std::min(4096, div_up(nnz_max, kBlock)));
  if (ev0) (void)hipEventRecord(ev0, st);
  if (a.mixed)
    hipLaunchKernelGGL((k_proj_multi<float, 8>), dim3(gm), dim3(kBlock), 0, st, a, sc);
  else
    hipLaunchKernelGGL((k_proj_multi<double, 4>), dim3(gm), dim3(kBlock), 0, st, a, sc);
  if (ev1) (void)hipEventRecord(ev1, st);
  const int np = std::max(1, div_up(nnz_max, kRedBlock * kRedItems));
  hipLaunchKernelGGL(k_reduce_partial, dim3(np), dim3(kRedBlock), 0, st, a.resid, a.partial, sc);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedBlock), 0, st, a.partial, np, sc);
}

}  // namespace ctd

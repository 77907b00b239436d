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

__global__ __launch_bounds__(kBlock) void k_proj_single(ProjectArgs a, const DevScalars* sc,
                                                        int32_t* n_multi) {
  const int64_t n_f = sc->status == 0 ? sc->n_f : 0;
  const int lane = lane_id();
  for (int64_t f0 = (int64_t)blockIdx.x * kBlock; f0 < n_f; f0 += (int64_t)gridDim.x * kBlock) {
    const int64_t f = f0 + threadIdx.x;
    bool multi = false;
    if (f < n_f) {
      const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
      if (e1 - e0 == 1) {
        const double v = a.val[e0];
        const double x2 = v * v;
        const double z2 = x2 * a.lev[a.row[e0]];
        a.resid[f] = (a.fiber_mark && a.fiber_mark[f]) ? 0.0 : x2 - z2;
      } else {
        multi = true;
      }
    }
    const uint64_t m = __ballot(multi);
    int32_t base = 0;
    if (lane == 0 && m) base = atomicAdd(n_multi, (int32_t)__popcll(m));
    base = __shfl(base, 0, kWave);
    if (multi) {
      const uint64_t lt = lane == 0 ? 0ull : ((~0ull) >> (kWave - lane));
      a.multi[base + __popcll(m & lt)] = (int32_t)f;
    }
  }
}

// One wave per fiber with >= 2 nonzeros.  T = value type of Q, VEC columns per lane.
template <typename T, int VEC>
__global__ __launch_bounds__(kBlock) void k_proj_multi(ProjectArgs a, const DevScalars* sc,
                                                       const int32_t* n_multi) {
  constexpr int kCols = VEC * kWave;
  const int64_t nm = sc->status == 0 ? *n_multi : 0;
  const int64_t ncols = *a.d_ncols;
  const int lane = lane_id();
  const T* Qb = nullptr;
  if constexpr (sizeof(T) == 8)
    Qb = (const T*)a.Q;
  else
    Qb = (const T*)a.Qf;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  for (int64_t w = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave; w < nm; w += nwaves) {
    const int32_t f = a.multi[w];
    const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
    double x2 = 0.0;
    for (int32_t e = e0; e < e1; ++e) {
      const double v = a.val[e];
      x2 += v * v;
    }
    double z2 = 0.0;
    for (int64_t c0 = 0; c0 < ncols; c0 += kCols) {
      const int64_t c = c0 + (int64_t)VEC * lane;
      const bool active = c < ncols;
      T acc[VEC];
#pragma unroll
      for (int k = 0; k < VEC; ++k) acc[k] = T(0);
      if (active) {
        int32_t e = e0;
        for (; e + 1 < e1; e += 2) {
          const int32_t r0 = a.row[e], r1 = a.row[e + 1];
          T v0, v1;
          if constexpr (sizeof(T) == 8) {
            v0 = a.val[e];
            v1 = a.val[e + 1];
          } else {
            v0 = a.val32[e];
            v1 = a.val32[e + 1];
          }
          const T* q0 = Qb + (int64_t)r0 * a.ldq + c;
          const T* q1 = Qb + (int64_t)r1 * a.ldq + c;
          T x0[VEC], x1[VEC];
#pragma unroll
          for (int k = 0; k < VEC; k += 16 / sizeof(T)) {
            if constexpr (sizeof(T) == 8) {
              const double2 u0 = *(const double2*)(q0 + k);
              const double2 u1 = *(const double2*)(q1 + k);
              x0[k] = u0.x; x0[k + 1] = u0.y;
              x1[k] = u1.x; x1[k + 1] = u1.y;
            } else {
              const float4 u0 = *(const float4*)(q0 + k);
              const float4 u1 = *(const float4*)(q1 + k);
              x0[k] = u0.x; x0[k + 1] = u0.y; x0[k + 2] = u0.z; x0[k + 3] = u0.w;
              x1[k] = u1.x; x1[k + 1] = u1.y; x1[k + 2] = u1.z; x1[k + 3] = u1.w;
            }
          }
#pragma unroll
          for (int k = 0; k < VEC; ++k) acc[k] += v0 * x0[k];
#pragma unroll
          for (int k = 0; k < VEC; ++k) acc[k] += v1 * x1[k];
        }
        if (e < e1) {
          const int32_t r0 = a.row[e];
          T v0;
          if constexpr (sizeof(T) == 8)
            v0 = a.val[e];
          else
            v0 = a.val32[e];
          const T* q0 = Qb + (int64_t)r0 * a.ldq + c;
#pragma unroll
          for (int k = 0; k < VEC; k += 16 / sizeof(T)) {
            if constexpr (sizeof(T) == 8) {
              const double2 u0 = *(const double2*)(q0 + k);
              acc[k] += v0 * u0.x;
              acc[k + 1] += v0 * u0.y;
            } else {
              const float4 u0 = *(const float4*)(q0 + k);
              acc[k] += v0 * u0.x;
              acc[k + 1] += v0 * u0.y;
              acc[k + 2] += v0 * u0.z;
              acc[k + 3] += v0 * u0.w;
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const double d = (double)acc[k];
        z2 += (c + k < ncols) ? d * d : 0.0;
      }
    }
    z2 = wave_sum(z2);
    if (lane == 0) a.resid[f] = (a.fiber_mark && a.fiber_mark[f]) ? 0.0 : x2 - z2;
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

__global__ void k_zero_i32(int32_t* p) { *p = 0; }
}  // namespace

void launch_project(hipStream_t st, const ProjectArgs& a, int64_t nnz_max, DevScalars* sc,
                    hipEvent_t ev0, hipEvent_t ev1) {
  int32_t* n_multi = &sc->n_multi;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, n_multi);
  const int gs = std::max(1, std::min(8192, div_up(nnz_max, kBlock)));
  hipLaunchKernelGGL(k_proj_single, dim3(gs), dim3(kBlock), 0, st, a, sc, n_multi);
  const int gm = std::max(1, std::min(4096, div_up(nnz_max / 2 * kWave, kBlock)));
  if (ev0) (void)hipEventRecord(ev0, st);
  if (a.mixed)
    hipLaunchKernelGGL((k_proj_multi<float, 8>), dim3(gm), dim3(kBlock), 0, st, a, sc, n_multi);
  else
    hipLaunchKernelGGL((k_proj_multi<double, 4>), dim3(gm), dim3(kBlock), 0, st, a, sc, n_multi);
  if (ev1) (void)hipEventRecord(ev1, st);
  const int np = std::max(1, div_up(nnz_max, kRedBlock * kRedItems));
  hipLaunchKernelGGL(k_reduce_partial, dim3(np), dim3(kRedBlock), 0, st, a.resid, a.partial, sc);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedBlock), 0, st, a.partial, np, sc);
}

}  // namespace ctd

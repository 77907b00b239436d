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
#include "gather.h"
#include "kernels.h"

namespace ctd {

namespace {
constexpr int kBlock = 256;
constexpr int kRedBlock = 1024;
constexpr int kRedItems = 8;

// Residual of every fiber.  A wave takes fpw consecutive fibers, one per
// lane (64 for a large input; a few for a small one such as a time slice, so
// that its few fibers still spread over many waves).  Kept fibers lie in span(Q) and get 0.  Fibers with one nonzero v at
// row r are done lane-parallel from the row leverage: ||Q^T x||^2 =
// v^2 ||Q_r||^2.  Fibers of more than kLongFiber nonzeros are listed for
// k_proj_long.  The wave walks the rest one at a time: z_f = sum_e v_e
// Q[r_e, :], lane l holding columns VEC l .. VEC l + VEC of each 64 VEC-column
// chunk, the fiber's (row, value) pairs loaded once into lanes and
// broadcast, two nonzeros times two chunks of row gathers in flight.  Column
// chunks of z are squared and summed as they complete; z is never written.
template <typename T, int VEC>
__global__ __launch_bounds__(kBlock) void k_proj_multi(ProjectArgs a, DevScalars* sc, int fpw) {
  constexpr int kCols = VEC * kWave;
  if (sc->status != 0) return;
  const int64_t n_f = sc->n_f;
  const int64_t ncols = *a.d_ncols;
  const int lane = lane_id();
  const T* Qb = sizeof(T) == 8 ? (const T*)a.Q : (const T*)a.Qf;
  const T* vals = sizeof(T) == 8 ? (const T*)a.val : (const T*)a.val32;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  const uint64_t lt = lane == 0 ? 0ull : ((~0ull) >> (kWave - lane));
  for (int64_t fb = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave * fpw; fb < n_f;
       fb += nwaves * fpw) {
    const int64_t fl = fb + lane;
    bool multi = false, lng = false;
    if (lane < fpw && fl < n_f) {
      const int32_t s0 = a.fptr[fl], s1 = a.fptr[fl + 1];
      const bool kept = a.fiber_mark && a.fiber_mark[fl];
      if (kept) {
        a.resid[fl] = 0.0;
      } else if (s1 - s0 == 1) {
        const double v = a.val[s0];
        const double x2 = v * v;
        const double z2 = x2 * a.lev[a.row[s0]];
        a.resid[fl] = x2 - z2;
      } else if (s1 - s0 > kLongFiber) {
        lng = true;
      } else {
        multi = true;
      }
    }
    const uint64_t ml = __ballot(lng);
    if (ml) {
      int32_t base = 0;
      if (lane == 0) base = atomicAdd(&sc->n_long, (int32_t)__popcll(ml));
      base = __shfl(base, 0, kWave);
      if (lng) a.long_list[base + __popcll(ml & lt)] = (int32_t)fl;
    }
    uint64_t todo = __ballot(multi);
    while (todo) {
      const int i = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int64_t f = fb + i;
      const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
      const int n = e1 - e0;
      const int32_t rr = lane < n ? a.row[e0 + lane] : 0;
      const T vv = lane < n ? vals[e0 + lane] : T(0);
      const double v64 = lane < n ? a.val[e0 + lane] : 0.0;
      double z2 = 0.0;
      for (int64_t c0 = 0; c0 < ncols; c0 += 2 * kCols) {
        const int64_t ca = c0 + (int64_t)VEC * lane, cb = ca + kCols;
        const bool ina = ca < ncols, inb = cb < ncols;
        T acc0[VEC], acc1[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) acc0[k] = acc1[k] = T(0);
        gather_batch<T, VEC>(rr, vv, n, Qb + (ina ? ca : 0), Qb + (inb ? cb : 0), ina, inb,
                             a.ldq, acc0, acc1);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
          const double d0 = (double)acc0[j], d1 = (double)acc1[j];
          z2 += (ca + j < ncols) ? d0 * d0 : 0.0;
          z2 += (cb + j < ncols) ? d1 * d1 : 0.0;
        }
      }
      const double x2 = wave_sum(v64 * v64);
      z2 = wave_sum(z2);
      if (lane == 0) a.resid[f] = x2 - z2;
    }
  }
}

// Long fibers: workgroup (chunk, i) forms z of listed fiber i over one
// column chunk with all its waves and stores ||z_chunk||^2.
template <typename T, int VEC>
__global__ __launch_bounds__(kLongWaves * kWave) void k_proj_long(ProjectArgs a,
                                                                  const DevScalars* sc) {
  constexpr int kCols = VEC * kWave;
  __shared__ double red[kLongWaves * VEC * kWave];
  if (sc->status != 0) return;
  const int64_t n_long = sc->n_long;
  const int64_t ncols = *a.d_ncols;
  const int64_t c0 = (int64_t)blockIdx.x * kCols;
  if (c0 >= ncols) return;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const T* Qb = sizeof(T) == 8 ? (const T*)a.Q : (const T*)a.Qf;
  const T* vals = sizeof(T) == 8 ? (const T*)a.val : (const T*)a.val32;
  const int64_t c = c0 + (int64_t)VEC * lane;
  const bool in = c < ncols;
  for (int64_t i = blockIdx.y; i < n_long; i += gridDim.y) {
    const int32_t f = a.long_list[i];
    double z[VEC];
    wg_gather_chunk<T, VEC>(a.row, vals, a.fptr[f], a.fptr[f + 1], Qb + (in ? c : 0), in,
                            a.ldq, red, z);
    if (wv == 0) {
      double z2 = 0.0;
#pragma unroll
      for (int j = 0; j < VEC; ++j) z2 += (c + j < ncols) ? z[j] * z[j] : 0.0;
      z2 = wave_sum(z2);
      if (lane == 0) a.long_part[i * a.long_ld + blockIdx.x] = z2;
    }
  }
}

// resid of listed fiber i = ||x_f||^2 - sum over chunks (in chunk order); one wave each.
__global__ __launch_bounds__(kBlock) void k_proj_long_fin(ProjectArgs a, const DevScalars* sc,
                                                          int chunk_cols) {
  if (sc->status != 0) return;
  const int64_t n_long = sc->n_long;
  const int64_t ncols = *a.d_ncols;
  const int64_t nch = (ncols + chunk_cols - 1) / chunk_cols;
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  for (int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave; i < n_long; i += nwaves) {
    const int32_t f = a.long_list[i];
    const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
    double x2 = 0.0;
    for (int32_t e = e0 + lane; e < e1; e += kWave) x2 += a.val[e] * a.val[e];
    x2 = wave_sum(x2);
    if (lane == 0) {
      double z2 = 0.0;
      for (int64_t ch = 0; ch < nch; ++ch) z2 += a.long_part[i * a.long_ld + ch];
      a.resid[f] = x2 - z2;
    }
  }
}

__global__ void k_zero_long(DevScalars* sc) { sc->n_long = 0; }

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
  // fibers per wave: few for a small input (a time slice has a few thousand
  // fibers, which must still spread over many waves), 64 for a large one;
  // the autotuner picks among the candidates per input-size bucket
  static const int kFpw[] = {2, 8, kWave};
  constexpr int kNFpw = 3;
  const int prec = a.mixed ? 1 : 0, bucket = tune_bucket(nnz_max);
  int choice = tune_get(TUNE_PROJ_FPW, prec, bucket, kNFpw);
  std::vector<hipEvent_t> tev;
  const bool measure = choice < 0 && tune_begin(TUNE_PROJ_FPW, prec, bucket, kNFpw, &tev);
  if (choice < 0) choice = nnz_max <= (int64_t(1) << 18) ? 0 : 2;
  auto multi = [&](int fpw) {
    hipLaunchKernelGGL(k_zero_long, dim3(1), dim3(1), 0, st, sc);
    const int64_t waves = (std::max<int64_t>(nnz_max, 1) + fpw - 1) / fpw;
    const int gm = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (waves + 3) / 4));
    if (a.mixed)
      hipLaunchKernelGGL((k_proj_multi<float, 8>), dim3(gm), dim3(kBlock), 0, st, a, sc, fpw);
    else
      hipLaunchKernelGGL((k_proj_multi<double, 4>), dim3(gm), dim3(kBlock), 0, st, a, sc, fpw);
  };
  const int64_t max_long = nnz_max / (kLongFiber + 1) + 1;
  const int gy = (int)std::max<int64_t>(1, std::min<int64_t>(1024, max_long));
  const int cols = a.mixed ? 8 * kWave : 4 * kWave;
  const int nch = (int)std::max<int64_t>(1, div_up(a.ncols_max, cols));
  if (ev0) (void)hipEventRecord(ev0, st);
  if (measure) {
    // every candidate once, timed; the last run's residuals and long-fiber
    // list are the ones used (all runs write the same values)
    for (int c = 0; c < kNFpw; ++c) {
      (void)hipEventRecord(tev[2 * c], st);
      multi(kFpw[c]);
      (void)hipEventRecord(tev[2 * c + 1], st);
    }
  } else {
    multi(kFpw[choice]);
  }
  if (a.mixed)
    hipLaunchKernelGGL((k_proj_long<float, 8>), dim3(nch, gy), dim3(kLongWaves * kWave), 0, st, a,
                       sc);
  else
    hipLaunchKernelGGL((k_proj_long<double, 4>), dim3(nch, gy), dim3(kLongWaves * kWave), 0, st, a,
                       sc);
  hipLaunchKernelGGL(k_proj_long_fin, dim3(std::max(1, std::min(1024, (int)div_up(max_long * kWave, kBlock)))),
                     dim3(kBlock), 0, st, a, sc, cols);
  if (ev1) (void)hipEventRecord(ev1, st);
  const int np = std::max(1, div_up(nnz_max, kRedBlock * kRedItems));
  hipLaunchKernelGGL(k_reduce_partial, dim3(np), dim3(kRedBlock), 0, st, a.resid, a.partial, sc);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedBlock), 0, st, a.partial, np, sc);
}

}  // namespace ctd

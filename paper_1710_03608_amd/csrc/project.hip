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
//
// ||Q^T x_f||^2 is a sum over the columns of Q, so it splits over column
// slices.  The launches are sliced S ways (S in 1, 2, 4, 8) with the slice as
// the fastest grid dimension: workgroups go to the eight XCDs in turn, so each
// XCD gathers from one slice of Q only, and its L2 holds that slice's rows
// (1/S of a row each) instead of whole rows.  Each slice's ||z||^2 is stored
// per fiber and the slices are added in slice order.
#include "gather.h"
#include "kernels.h"

namespace ctd {

namespace {
constexpr int kBlock = 256;
constexpr int kRedBlock = 1024;
constexpr int kRedItems = 8;
constexpr int kLongBatch = 16;   // nonzeros per wave and step in k_proj_long

// z += sum_e v_e A[r_e, c .. c + VEC) over the n (<= 64) nonzeros whose
// (row, value) are held one per lane in (rr, vv), four rows in flight.
template <typename T, int VEC>
__device__ inline void gather_seg(int32_t rr, T vv, int n, const T* q, bool in, int64_t ld,
                                  T (&acc)[VEC]) {
  int k = 0;
  for (; k + 3 < n; k += 4) {
    const int64_t r0 = read_lane(rr, k), r1 = read_lane(rr, k + 1);
    const int64_t r2 = read_lane(rr, k + 2), r3 = read_lane(rr, k + 3);
    const T v0 = read_lane(vv, k), v1 = read_lane(vv, k + 1);
    const T v2 = read_lane(vv, k + 2), v3 = read_lane(vv, k + 3);
    if (in) {
      T x0[VEC], x1[VEC], x2[VEC], x3[VEC];
      load_seg<T, VEC>(q + r0 * ld, x0);
      load_seg<T, VEC>(q + r1 * ld, x1);
      load_seg<T, VEC>(q + r2 * ld, x2);
      load_seg<T, VEC>(q + r3 * ld, x3);
#pragma unroll
      for (int j = 0; j < VEC; ++j) acc[j] += (v0 * x0[j] + v1 * x1[j]) + (v2 * x2[j] + v3 * x3[j]);
    }
  }
  for (; k < n; ++k) {
    const int64_t r0 = read_lane(rr, k);
    const T v0 = read_lane(vv, k);
    if (in) {
      T x0[VEC];
      load_seg<T, VEC>(q + r0 * ld, x0);
#pragma unroll
      for (int j = 0; j < VEC; ++j) acc[j] += v0 * x0[j];
    }
  }
}

// Columns [lo, hi) of slice `slice` of S: a width of ceil(ncols / S) rounded
// up to VEC, so every lane's VEC-element load starts inside the row.
template <int VEC>
__device__ inline void slice_cols(int64_t ncols, int S, int slice, int64_t& lo, int64_t& hi) {
  const int64_t w = ((ncols + S - 1) / S + VEC - 1) / VEC * VEC;
  lo = min(ncols, (int64_t)slice * w);
  hi = min(ncols, lo + w);
}

// Residual of every fiber, column slice blockIdx.x of gridDim.x.  A wave
// takes fpw consecutive fibers, one per lane (64 for a large input; a few for
// a small one such as a time slice, so that its few fibers still spread over
// many waves).  Slice 0 also does the fibers that need no gather: kept fibers
// lie in span(Q) and get 0, a fiber with one nonzero v at row r gets v^2 -
// v^2 ||Q_r||^2 from the row leverage, and fibers of more than kLongFiber
// nonzeros are listed for k_proj_long.  For the rest the wave walks the fibers
// one at a time: z_f = sum_e v_e Q[r_e, lo:hi], lane l holding columns
// lo + VEC l .. of each VEC * 64-column chunk of the slice, the fiber's
// (row, value) pairs loaded once into lanes and broadcast.  With one slice the
// wave writes resid[f] = ||x_f||^2 - ||z_f||^2 itself; with several, the
// slice's ||z||^2 goes to zpart[slice][f], slice 0 puts ||x_f||^2 into
// resid[f] and k_proj_multi_fin subtracts the slices.
// kSliced: gridDim.x column slices (partials to zpart) rather than whole rows.
template <typename T, int VEC, bool kSliced>
__global__ __launch_bounds__(kBlock) void k_proj_multi(ProjectArgs a, DevScalars* sc, int fpw) {
  constexpr int kCols = VEC * kWave;
  if (sc->status != 0) return;
  const int64_t n_f = sc->n_f;
  const int slice = blockIdx.x;
  int64_t lo, hi;
  slice_cols<VEC>(*a.d_ncols, gridDim.x, slice, lo, hi);
  const int lane = lane_id();
  const T* Qb = sizeof(T) == 8 ? (const T*)a.Q : (const T*)a.Qf;
  const T* vals = sizeof(T) == 8 ? (const T*)a.val : (const T*)a.val32;
  double* zp = a.zpart + (int64_t)slice * a.zpart_ld;
  const int64_t nwaves = (int64_t)gridDim.y * (kBlock / kWave);
  const uint64_t lt = lane == 0 ? 0ull : ((~0ull) >> (kWave - lane));
  for (int64_t fb = ((int64_t)blockIdx.y * kBlock + threadIdx.x) / kWave * fpw; fb < n_f;
       fb += nwaves * fpw) {
    const int64_t fl = fb + lane;
    bool multi = false, lng = false;
    if (lane < fpw && fl < n_f) {
      const int32_t s0 = a.fptr[fl], s1 = a.fptr[fl + 1];
      const bool kept = a.fiber_mark && a.fiber_mark[fl];
      if (kept) {
        if (slice == 0) a.resid[fl] = 0.0;
      } else if (s1 - s0 == 1) {
        if (slice == 0) {
          const double v = a.val[s0];
          const double x2 = v * v;
          a.resid[fl] = x2 - x2 * a.lev[a.row[s0]];
        }
      } else if (s1 - s0 > kLongFiber) {
        lng = true;
      } else {
        multi = true;
      }
    }
    if (slice == 0) {
      const uint64_t ml = __ballot(lng);
      if (ml) {
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(&sc->n_long, (int32_t)__popcll(ml));
        base = __shfl(base, 0, kWave);
        if (lng) a.long_list[base + __popcll(ml & lt)] = (int32_t)fl;
      }
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
      double z2 = 0.0;
      if (!kSliced || hi - lo > kCols) {
        // whole rows or a wide slice: two chunks times two nonzeros in flight
        for (int64_t c0 = lo; c0 < hi; c0 += 2 * kCols) {
          const int64_t ca = c0 + (int64_t)VEC * lane, cb = ca + kCols;
          const bool ina = ca < hi, inb = cb < hi;
          T acc0[VEC], acc1[VEC];
#pragma unroll
          for (int k = 0; k < VEC; ++k) acc0[k] = acc1[k] = T(0);
          gather_batch<T, VEC>(rr, vv, n, Qb + (ina ? ca : 0), Qb + (inb ? cb : 0), ina, inb,
                               a.ldq, acc0, acc1);
#pragma unroll
          for (int j = 0; j < VEC; ++j) {
            const double d0 = (double)acc0[j], d1 = (double)acc1[j];
            z2 += (ca + j < hi) ? d0 * d0 : 0.0;
            z2 += (cb + j < hi) ? d1 * d1 : 0.0;
          }
        }
      } else if constexpr (kSliced) {
        // one chunk: four nonzeros in flight
        const int64_t ca = lo + (int64_t)VEC * lane;
        const bool in = ca < hi;
        T acc[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) acc[k] = T(0);
        gather_seg<T, VEC>(rr, vv, n, Qb + (in ? ca : 0), in, a.ldq, acc);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
          const double d = (double)acc[j];
          z2 += (ca + j < hi) ? d * d : 0.0;
        }
      }
      z2 = wave_sum(z2);
      if (!kSliced) {
        const double v64 = lane < n ? a.val[e0 + lane] : 0.0;
        const double x2 = wave_sum(v64 * v64);
        if (lane == 0) a.resid[f] = x2 - z2;
      } else {
        if (lane == 0) zp[f] = z2;
        if (slice == 0) {
          const double v64 = lane < n ? a.val[e0 + lane] : 0.0;
          const double x2 = wave_sum(v64 * v64);
          if (lane == 0) a.resid[f] = x2;
        }
      }
    }
  }
}

// resid[f] = ||x_f||^2 - sum over the S slices (in slice order) for every
// fiber of 2 .. kLongFiber nonzeros that is not kept; one thread per fiber.
__global__ __launch_bounds__(kBlock) void k_proj_multi_fin(ProjectArgs a, const DevScalars* sc,
                                                           int S) {
  if (sc->status != 0) return;
  const int64_t n_f = sc->n_f;
  for (int64_t f = (int64_t)blockIdx.x * kBlock + threadIdx.x; f < n_f;
       f += (int64_t)gridDim.x * kBlock) {
    const int32_t n = a.fptr[f + 1] - a.fptr[f];
    if (n < 2 || n > kLongFiber || (a.fiber_mark && a.fiber_mark[f])) continue;
    double z2 = 0.0;
    for (int sl = 0; sl < S; ++sl) z2 += a.zpart[(int64_t)sl * a.zpart_ld + f];
    a.resid[f] -= z2;
  }
}

// Long fibers: workgroup (slice, i) forms z of listed fiber i over column
// slice blockIdx.x with all its waves (wave wv takes the nonzeros in
// interleaved batches of kLongBatch, so that a fiber of a few hundred
// nonzeros still keeps all eight waves busy; the waves' partial z are added
// in LDS in wave order) and stores the slice's ||z||^2.
template <typename T, int VEC>
__global__ __launch_bounds__(kLongWaves * kWave) void k_proj_long(ProjectArgs a,
                                                                  const DevScalars* sc) {
  constexpr int kCols = VEC * kWave;
  __shared__ double red[kLongWaves * VEC * kWave];
  if (sc->status != 0) return;
  const int64_t n_long = sc->n_long;
  int64_t lo, hi;
  slice_cols<VEC>(*a.d_ncols, gridDim.x, blockIdx.x, lo, hi);
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const T* Qb = sizeof(T) == 8 ? (const T*)a.Q : (const T*)a.Qf;
  const T* vals = sizeof(T) == 8 ? (const T*)a.val : (const T*)a.val32;
  for (int64_t i = blockIdx.y; i < n_long; i += gridDim.y) {
    const int32_t f = a.long_list[i];
    const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
    double z2 = 0.0;
    for (int64_t c0 = lo; c0 < hi; c0 += kCols) {
      const int64_t c = c0 + (int64_t)VEC * lane;
      const bool in = c < hi;
      T acc[VEC];
#pragma unroll
      for (int j = 0; j < VEC; ++j) acc[j] = T(0);
      for (int32_t eb = e0 + wv * kLongBatch; eb < e1; eb += kLongWaves * kLongBatch) {
        const int n = min(kLongBatch, e1 - eb);
        const int32_t rr = lane < n ? a.row[eb + lane] : 0;
        const T vv = lane < n ? vals[eb + lane] : T(0);
        gather_seg<T, VEC>(rr, vv, n, Qb + (in ? c : 0), in, a.ldq, acc);
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < VEC; ++j) red[(size_t)wv * VEC * kWave + lane * VEC + j] = (double)acc[j];
      __syncthreads();
      if (wv == 0) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
          double zs = 0.0;
          for (int w = 0; w < kLongWaves; ++w) zs += red[(size_t)w * VEC * kWave + lane * VEC + j];
          z2 += (c + j < hi) ? zs * zs : 0.0;
        }
      }
    }
    if (wv == 0) {
      z2 = wave_sum(z2);
      if (lane == 0) a.long_part[i * a.long_ld + blockIdx.x] = z2;
    }
  }
}

// resid of listed fiber i = ||x_f||^2 - sum over the S slices (in slice
// order); one wave each.
__global__ __launch_bounds__(kBlock) void k_proj_long_fin(ProjectArgs a, const DevScalars* sc,
                                                          int S) {
  if (sc->status != 0) return;
  const int64_t n_long = sc->n_long;
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
      for (int sl = 0; sl < S; ++sl) z2 += a.long_part[i * a.long_ld + sl];
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

// Column slices of a launch: the largest power of two up to kProjSlices (one
// per XCD) that leaves each slice at least three quarters of a chunk of
// `chunk` columns.
static int proj_slices(int64_t ncols_max, int chunk) {
  int S = 1;
  while (S < kProjSlices && 4 * ncols_max >= (int64_t)(2 * S) * 3 * chunk) S *= 2;
  return S;
}

void launch_project(hipStream_t st, const ProjectArgs& a, int64_t nnz_max, DevScalars* sc,
                    hipEvent_t ev0, hipEvent_t ev1) {
  // Fibers of up to kLongFiber nonzeros.  Column slices: each XCD's L2 then
  // caches a smaller part of every row and a small input gets more waves, but
  // every fiber's bookkeeping is repeated per slice.  A small input (a time
  // slice) takes the most slices; a large one two in float64 and whole rows
  // in float32, where the rows are half as long.  The slice count is fixed
  // by this rule rather than measured, because the sum over slices rounds
  // differently: the autotuner's candidates, the fibers per wave (few for a
  // small input, whose few thousand fibers must still spread over many
  // waves; 64 for a large one), all give bit-identical results.
  static const int kFpw[] = {2, 8, kWave};
  constexpr int kNCand = 3;
  const bool small = nnz_max <= (int64_t(1) << 18);
  const int prec = a.mixed ? 1 : 0, bucket = tune_bucket(nnz_max);
  int choice = tune_get(TUNE_PROJ_FPW, prec, bucket, kNCand);
  std::vector<hipEvent_t> tev;
  const bool measure = choice < 0 && tune_begin(TUNE_PROJ_FPW, prec, bucket, kNCand, &tev);
  if (choice < 0) choice = small ? 0 : 2;
  const int s_max = proj_slices(a.ncols_max, 4 * kWave);
  const int S = small ? s_max : std::min(a.mixed ? 1 : 2, s_max);
  auto multi = [&](int c) {
    const int fpw = kFpw[c];
    hipLaunchKernelGGL(k_zero_long, dim3(1), dim3(1), 0, st, sc);
    const int64_t waves = (std::max<int64_t>(nnz_max, 1) + fpw - 1) / fpw;
    const int gm = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (waves + 3) / 4));
    const dim3 grid(S, gm);
    if (S > 1 && a.mixed)
      hipLaunchKernelGGL((k_proj_multi<float, 4, true>), grid, dim3(kBlock), 0, st, a, sc, fpw);
    else if (S > 1)
      hipLaunchKernelGGL((k_proj_multi<double, 4, true>), grid, dim3(kBlock), 0, st, a, sc, fpw);
    else if (a.mixed)
      hipLaunchKernelGGL((k_proj_multi<float, 8, false>), grid, dim3(kBlock), 0, st, a, sc, fpw);
    else
      hipLaunchKernelGGL((k_proj_multi<double, 4, false>), grid, dim3(kBlock), 0, st, a, sc, fpw);
  };
  const int64_t max_long = nnz_max / (kLongFiber + 1) + 1;
  const int gy = (int)std::max<int64_t>(1, std::min<int64_t>(1024, max_long));
  if (ev0) (void)hipEventRecord(ev0, st);
  if (measure) {
    // every candidate once, timed; the last run's residuals, slice partials
    // and long-fiber list are the ones used (all runs write the same values)
    for (int c = 0; c < kNCand; ++c) {
      (void)hipEventRecord(tev[2 * c], st);
      multi(c);
      (void)hipEventRecord(tev[2 * c + 1], st);
    }
    tune_recorded(TUNE_PROJ_FPW, prec, bucket);
  } else {
    multi(choice);
  }
  if (S > 1)
    hipLaunchKernelGGL(k_proj_multi_fin,
                       dim3((int)std::max<int64_t>(1, std::min<int64_t>(4096, div_up(nnz_max, kBlock)))),
                       dim3(kBlock), 0, st, a, sc, S);
  const int s_long = proj_slices(a.ncols_max, (a.mixed ? 8 : 4) * kWave);
  if (a.mixed)
    hipLaunchKernelGGL((k_proj_long<float, 8>), dim3(s_long, gy), dim3(kLongWaves * kWave), 0, st,
                       a, sc);
  else
    hipLaunchKernelGGL((k_proj_long<double, 4>), dim3(s_long, gy), dim3(kLongWaves * kWave), 0, st,
                       a, sc);
  hipLaunchKernelGGL(k_proj_long_fin, dim3(std::max(1, std::min(1024, (int)div_up(max_long * kWave, kBlock)))),
                     dim3(kBlock), 0, st, a, sc, s_long);
  if (ev1) (void)hipEventRecord(ev1, st);
  const int np = std::max(1, div_up(nnz_max, kRedBlock * kRedItems));
  hipLaunchKernelGGL(k_reduce_partial, dim3(np), dim3(kRedBlock), 0, st, a.resid, a.partial, sc);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedBlock), 0, st, a.partial, np, sc);
}

}  // namespace ctd

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
//
// Hot rows (large inputs).  Under the skewed source distribution of traffic
// data a few rows of X_(alpha) hold a large share of the nonzeros of the
// multi-nonzero fibers, and each of those nonzeros gathers a whole row of Q.
// For a set H of at most kHotMax such rows, G = Q Q_H^T (n_rows x |H|) is
// formed once on the MFMAs.  A fiber's z = z_H + z_C then splits over its hot
// and cold nonzeros, and with t_e = sum over hot e' of v_e' G[r_e][h(e')],
//   ||z||^2 = sum_{e hot} v_e t_e + 2 sum_{c cold} v_c t_c + ||z_C||^2,
// so a hot nonzero costs one table lookup per hot nonzero of its fiber
// instead of a row gather.  ||z_C||^2 is v^2 ||Q_r||^2 for one cold nonzero
// and a gather over the cold rows only for two or more.  H is the set of rows
// whose nonzero count clears a threshold picked from the counts alone, so it
// is the same on every run.
#include "gather.h"
#include "kernels.h"

namespace ctd {

namespace {
constexpr int kBlock = 256;
constexpr int kRedBlock = 1024;
constexpr int kRedItems = 8;
constexpr int kLongBatch = 16;   // nonzeros per wave and step in k_proj_long
constexpr int kColdSlices = 4;   // column slices of k_proj_cold
constexpr int kHotGroup = 32;    // GH entries per lane in flight in k_proj_long_fin_hot
constexpr int kFinWaves = 2;     // waves per long fiber in k_proj_long_fin_hot
constexpr int kSmallFiber = 16;  // k_proj_multi_hot: fibers up to this size go four to a wave
static_assert(kHotMax % kHotGroup == 0, "whole groups of GH entries");

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

// Lane l gets lane s(l) of v, where s(l) is the l-th set bit of m (lanes
// l >= popcount(m) get some lane of v).  Used to pack the lanes of a mask
// into lanes 0, 1, ...
__device__ inline int packed_source(uint64_t m, int l) {
  int need = l, pos = 0;
#pragma unroll
  for (int w = 32; w > 0; w >>= 1) {
    const int low = __popcll(m & ((1ull << w) - 1));
    if (need >= low) {
      need -= low;
      m >>= w;
      pos += w;
    }
  }
  return pos;
}

// hot_id[r] = 0 for every row (it holds the counts until k_hot_select).
__global__ __launch_bounds__(kBlock) void k_hot_clear(ProjectArgs a) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r < a.n_rows) a.hot_id[r] = 0;
}

// Row counts over the nonzeros of every kHotSample-th fiber, among those with
// 2 .. kLongFiber nonzeros that are not kept (the fibers k_proj_multi
// gathers), into hot_id: workgroup p counts sampled fibers p * 1024 + t, ...
// into an LDS histogram and adds its nonzero bins with integer atomics (so
// the totals do not depend on their order).
__global__ __launch_bounds__(1024) void k_hot_count(ProjectArgs a, const DevScalars* sc) {
  __shared__ int32_t h[kHotMaxRows];
  const int n_rows = (int)a.n_rows;
  for (int r = threadIdx.x; r < n_rows; r += 1024) h[r] = 0;
  __syncthreads();
  const int64_t n_f = sc->status == 0 ? sc->n_f : 0;
  for (int64_t f = ((int64_t)blockIdx.x * 1024 + threadIdx.x) * kHotSample; f < n_f;
       f += (int64_t)gridDim.x * 1024 * kHotSample) {
    const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
    if (e1 - e0 < 2 || e1 - e0 > kLongFiber || (a.fiber_mark && a.fiber_mark[f])) continue;
    for (int32_t e = e0; e < e1; ++e) atomicAdd(&h[a.row[e]], 1);
  }
  __syncthreads();
  for (int r = threadIdx.x; r < n_rows; r += 1024)
    if (h[r] != 0) atomicAdd(&a.hot_id[r], h[r]);
}

// Count class of c >= 1: eight classes per power of two (the three bits
// below the leading one), non-decreasing in c.
__device__ inline int hot_class(int32_t c) {
  const int lead = 31 - __clz(c);
  const int frac = lead >= 3 ? (c >> (lead - 3)) & 7 : (c << (3 - lead)) & 7;
  return lead * 8 + frac;
}

// Picks H: the rows of the highest count classes such that at most kHotMax
// rows are taken and each has at least kHotMinCount nonzeros (a class is
// taken whole or not at all, so ties never split).  Hot rows are numbered in
// row order: hot_id[r] = index or -1, hot_meta[0 .. |H|) = rows, and
// hot_meta[kHotMax] = |H|.  One workgroup; thread t owns rows
// t * per .. t * per + per - 1.
__global__ __launch_bounds__(1024) void k_hot_select(ProjectArgs a, const DevScalars* sc) {
  constexpr int kPer = kHotMaxRows / 1024;
  __shared__ int32_t bins[256];
  __shared__ int32_t wsum[1024 / kWave];
  __shared__ int32_t thr;
  const int n_rows = sc->status == 0 ? (int)a.n_rows : 0;
  const int t = threadIdx.x;
  const int per = (n_rows + 1023) / 1024;
  int32_t c[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int r = t * per + i;
    c[i] = (i < per && r < n_rows) ? a.hot_id[r] : 0;
  }
  if (t < 256) bins[t] = 0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kPer; ++i)
    if (c[i] >= kHotMinCount) atomicAdd(&bins[hot_class(c[i])], 1);
  __syncthreads();
  if (t == 0) {
    int taken = 0, b_lo = 256;
    for (int b = 255; b >= hot_class(kHotMinCount); --b) {
      if (taken + bins[b] > kHotMax) break;
      taken += bins[b];
      b_lo = b;
    }
    thr = b_lo;
  }
  __syncthreads();
  const int b_lo = thr;
  int mine = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) mine += (c[i] >= kHotMinCount && hot_class(c[i]) >= b_lo) ? 1 : 0;
  // exclusive scan of `mine` over the workgroup, in thread order
  const int lane = lane_id(), w = t / kWave;
  int incl = mine;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int y = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += y;
  }
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  int base = incl - mine;
  for (int v = 0; v < w; ++v) base += wsum[v];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int r = t * per + i;
    if (i < per && r < n_rows) {
      const bool hot = c[i] >= kHotMinCount && hot_class(c[i]) >= b_lo;
      a.hot_id[r] = hot ? base : -1;
      if (hot) a.hot_meta[base++] = r;
    }
  }
  if (t == 1023) {
    int total = 0;
    for (int v = 0; v < 1024 / kWave; ++v) total += wsum[v];
    a.hot_meta[kHotMax] = total;
  }
}

// GH[r][a] = Q_r . Q_{hot_meta[a]} for a < |H| (0 for the rest) over the
// columns of Q, on float64 MFMAs.  One workgroup of four waves per 32 rows;
// wave w computes rows 16 (w / 2) .. + 16 and hot rows 32 (w % 2) .. + 32.
// Chunks of kHotK columns are staged through LDS, the next chunk's loads in
// registers while the current one is in the MFMAs.
constexpr int kHotK = 32;
__global__ __launch_bounds__(kBlock) void k_hot_gram(ProjectArgs a, const DevScalars* sc) {
  constexpr int kR = 32;
  __shared__ double As[kR][kHotK + 1];
  __shared__ double Bs[kHotK][kHotMax + 1];
  if (sc->status != 0) return;
  const int n_hot = a.hot_meta[kHotMax];
  if (n_hot == 0) return;
  const int64_t n_rows = a.n_rows, ldq = a.ldq, k = *a.d_ncols;
  const double* __restrict__ Q = a.Q;
  const int64_t r0 = (int64_t)blockIdx.x * kR;
  const int t = threadIdx.x, w = t / kWave, l = lane_id();
  const int rb = (w / 2) * 16, cb = (w % 2) * 32;
  // rows of Q_H this thread loads: hot index j = idx / kHotK
  int64_t hrow[kHotMax * kHotK / kBlock];
#pragma unroll
  for (int u = 0; u < kHotMax * kHotK / kBlock; ++u) {
    const int j = (u * kBlock + t) / kHotK;
    hrow[u] = j < n_hot ? (int64_t)a.hot_meta[j] : -1;
  }
  const int64_t nch = (k + kHotK - 1) / kHotK;
  double ra[kR * kHotK / kBlock], rb_[kHotMax * kHotK / kBlock];
  auto load = [&](int64_t ch) {
    const int64_t c0 = ch * kHotK;
#pragma unroll
    for (int u = 0; u < kR * kHotK / kBlock; ++u) {
      const int idx = u * kBlock + t, r = idx / kHotK, c = idx % kHotK;
      ra[u] = (ch < nch && c0 + c < k && r0 + r < n_rows) ? Q[(r0 + r) * ldq + c0 + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kHotMax * kHotK / kBlock; ++u) {
      const int c = (u * kBlock + t) % kHotK;
      rb_[u] = (ch < nch && c0 + c < k && hrow[u] >= 0) ? Q[hrow[u] * ldq + c0 + c] : 0.0;
    }
  };
  dbl4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  const bool active = cb < n_hot;
  load(0);
  for (int64_t ch = 0; ch < nch; ++ch) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kR * kHotK / kBlock; ++u) {
      const int idx = u * kBlock + t;
      As[idx / kHotK][idx % kHotK] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < kHotMax * kHotK / kBlock; ++u) {
      const int idx = u * kBlock + t;
      Bs[idx % kHotK][idx / kHotK] = rb_[u];
    }
    __syncthreads();
    load(ch + 1);
    if (active) {
#pragma unroll
      for (int ks = 0; ks < kHotK / 4; ++ks) {
        const double av = As[rb + l % 16][ks * 4 + l / 16];
        acc0 = mfma16(av, Bs[ks * 4 + l / 16][cb + l % 16], acc0);
        acc1 = mfma16(av, Bs[ks * 4 + l / 16][cb + 16 + l % 16], acc1);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t row = r0 + rb + l / 16 + 4 * q;
    if (row < n_rows) {
      a.GH[row * kHotMax + cb + l % 16] = acc0[q];
      a.GH[row * kHotMax + cb + 16 + l % 16] = acc1[q];
    }
  }
}

// This lane's share of ||z_C||^2 = ||sum over the cold lanes c of v_c Q[r_c, :]||^2
// (whole rows of hi columns), the cold lanes (mask mc) packed into lanes
// 0 .. |mc| - 1 first.
template <typename T, int VEC>
__device__ inline double cold_rows_z2(uint64_t mc, int32_t rr, T vv, const T* Qb, int64_t ldq,
                                      int64_t hi) {
  constexpr int kCols = VEC * kWave;
  const int lane = lane_id();
  const int nc = __popcll(mc);
  const int src = packed_source(mc, lane);
  const int32_t rc = __shfl(rr, src, kWave);
  const T vc = __shfl(vv, src, kWave);
  double z2 = 0.0;
  for (int64_t c0 = 0; c0 < hi; c0 += 2 * kCols) {
    const int64_t ca = c0 + (int64_t)VEC * lane, cb = ca + kCols;
    const bool ina = ca < hi, inb = cb < hi;
    T acc0[VEC], acc1[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) acc0[j] = acc1[j] = T(0);
    gather_batch<T, VEC>(rc, vc, nc, Qb + (ina ? ca : 0), Qb + (inb ? cb : 0), ina, inb, ldq, acc0,
                         acc1);
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
      const double d0 = (double)acc0[j], d1 = (double)acc1[j];
      z2 += (ca + j < hi) ? d0 * d0 : 0.0;
      z2 += (cb + j < hi) ? d1 * d1 : 0.0;
    }
  }
  return z2;
}

// The fibers of k_proj_multi with the hot-row split.  Per fiber, the hot
// nonzeros' part of ||z||^2 comes from lookups into GH (hot lanes packed,
// four lookups in flight) and the cold part from the row leverage when the
// fiber has one cold nonzero.  With two or more cold nonzeros, kInline
// gathers ||z_C||^2 over the packed cold lanes here, whole rows at a time;
// otherwise the fiber gets resid[f] = ||x_f||^2 - (hot part) and is listed
// for k_proj_cold, which subtracts ||z_C||^2 in column slices.  Fibers of up
// to kSmallFiber nonzeros take their hot part four at a time, one per 16-lane
// group, so that the wave's memory round trips serve four fibers; longer
// ones take the whole wave.  Every other fiber is handled as in k_proj_multi.
template <typename T, int VEC, bool kInline>
__global__ __launch_bounds__(kBlock) void k_proj_multi_hot(ProjectArgs a, DevScalars* sc, int fpw) {
  constexpr int kG = kSmallFiber;
  if (sc->status != 0) return;
  const int64_t n_f = sc->n_f;
  const int64_t hi = *a.d_ncols;
  const T* Qb = sizeof(T) == 8 ? (const T*)a.Q : (const T*)a.Qf;
  const T* vals = sizeof(T) == 8 ? (const T*)a.val : (const T*)a.val32;
  const int lane = lane_id();
  const int grp = lane / kG, sub = lane % kG;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  const uint64_t lt = lane == 0 ? 0ull : ((~0ull) >> (kWave - lane));
  for (int64_t fb = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave * fpw; fb < n_f;
       fb += nwaves * fpw) {
    const int64_t fl = fb + lane;
    bool multi = false, lng = false;
    int32_t s0 = 0, len = 0;
    if (lane < fpw && fl < n_f) {
      s0 = a.fptr[fl];
      len = a.fptr[fl + 1] - s0;
      const bool kept = a.fiber_mark && a.fiber_mark[fl];
      if (kept) {
        a.resid[fl] = 0.0;
      } else if (len == 1) {
        const double v = a.val[s0];
        const double x2 = v * v;
        a.resid[fl] = x2 - x2 * a.lev[a.row[s0]];
      } else if (len > kLongFiber) {
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
    uint64_t small = __ballot(multi && len <= kG), todo = __ballot(multi && len > kG);
    uint64_t cold = 0, inl = 0;
    double keep = 0.0;   // lane i: ||x_f||^2 - (hot part) of fiber fb + i, gathered below
    while (small) {
      int ig[kWave / kG];
#pragma unroll
      for (int g = 0; g < kWave / kG; ++g) {
        ig[g] = small ? __builtin_ctzll(small) : -1;
        small &= small - 1;
      }
      int my = ig[0];
#pragma unroll
      for (int g = 1; g < kWave / kG; ++g) my = grp == g ? ig[g] : my;
      // (the shuffles run on every lane: a lane that sits out a shuffle
      // gives 0 to the lanes reading it)
      const int from = my < 0 ? 0 : my;
      const int32_t e0 = __shfl(s0, from, kWave);
      const int32_t n_from = __shfl(len, from, kWave);
      const int n = my < 0 ? 0 : n_from;
      const bool in_f = sub < n;
      const int32_t rr = in_f ? a.row[e0 + sub] : 0;
      const double v64 = in_f ? a.val[e0 + sub] : 0.0;
      const int32_t hid = in_f ? a.hot_id[rr] : -1;
      const bool hot = hid >= 0;
      const uint64_t mh = __ballot(hot), mc = __ballot(in_f && !hot);
      const uint64_t gm = (1ull << kG) - 1;
      const int nh = __popcll((mh >> (grp * kG)) & gm), nc = __popcll((mc >> (grp * kG)) & gm);
      int nh_max = 0;
#pragma unroll
      for (int g = 0; g < kWave / kG; ++g) nh_max = max(nh_max, __popcll((mh >> (g * kG)) & gm));
      double t = 0.0;
      if (nh_max > 0) {
        const int pos = packed_source((mh >> (grp * kG)) & gm, sub) % kG;
        const int32_t hp = __shfl(hid, grp * kG + pos, kWave);
        const double vp = __shfl(v64, grp * kG + pos, kWave);
        const double* g = a.GH + (int64_t)rr * kHotMax;
        for (int k = 0; k < nh_max; k += 4) {
          int h[4];
          double w[4], x[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            h[j] = __shfl(hp, grp * kG + k + j, kWave);
            w[j] = __shfl(vp, grp * kG + k + j, kWave);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) x[j] = (in_f && k + j < nh) ? g[h[j]] : 0.0;
          if (in_f) {
#pragma unroll
            for (int j = 0; j < 4; ++j) w[j] = k + j < nh ? w[j] : 0.0;
            t += (w[0] * x[0] + w[1] * x[1]) + (w[2] * x[2] + w[3] * x[3]);
          }
        }
      }
      double part = hot ? v64 * t : 2.0 * v64 * t;
      if (nc == 1 && in_f && !hot) part += v64 * v64 * a.lev[rr];
      double x2 = v64 * v64;
#pragma unroll
      for (int off = kG / 2; off > 0; off >>= 1) {
        part += __shfl_xor(part, off, kWave);
        x2 += __shfl_xor(x2, off, kWave);
      }
      const double rest = x2 - part;
      const uint64_t need = __ballot(sub == 0 && my >= 0 && nc >= 2);
      if (kInline) {
#pragma unroll
        for (int g = 0; g < kWave / kG; ++g) {
          const double r = __shfl(rest, g * kG, kWave);
          if (((need >> (g * kG)) & 1) && lane == ig[g]) keep = r;
        }
      }
      if (sub == 0 && my >= 0 && !(kInline && nc >= 2)) a.resid[fb + my] = rest;
#pragma unroll
      for (int g = 0; g < kWave / kG; ++g)
        if ((need >> (g * kG)) & 1) {
          if (kInline)
            inl |= 1ull << ig[g];
          else
            cold |= 1ull << ig[g];
        }
    }
    if (kInline) {
      // the small fibers with two or more cold nonzeros: their cold rows
      while (inl) {
        const int i = __builtin_ctzll(inl);
        inl &= inl - 1;
        const int32_t e0 = a.fptr[fb + i];
        const int n = a.fptr[fb + i + 1] - e0;
        const bool in_f = lane < n;
        const int32_t rr = in_f ? a.row[e0 + lane] : 0;
        const T vv = in_f ? vals[e0 + lane] : T(0);
        const uint64_t mc = __ballot(in_f && a.hot_id[rr] < 0);
        const double z2 = wave_sum(cold_rows_z2<T, VEC>(mc, rr, vv, Qb, a.ldq, hi));
        if (lane == 0) a.resid[fb + i] = read_lane(keep, i) - z2;
      }
    }
    while (todo) {
      const int i = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int64_t f = fb + i;
      const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
      const int n = e1 - e0;
      const bool in_f = lane < n;
      const int32_t rr = in_f ? a.row[e0 + lane] : 0;
      const double v64 = in_f ? a.val[e0 + lane] : 0.0;
      const int32_t hid = in_f ? a.hot_id[rr] : -1;
      const bool hot = hid >= 0;
      const uint64_t mh = __ballot(hot), mc = __ballot(in_f && !hot);
      const int nh = __popcll(mh), nc = __popcll(mc);
      // t = sum over the hot nonzeros e' of v_e' GH[r_lane][h(e')]
      double t = 0.0;
      if (nh > 0) {
        const int src = packed_source(mh, lane);
        const int32_t hp = __shfl(hid, src, kWave);
        const double vp = __shfl(v64, src, kWave);
        const double* g = a.GH + (int64_t)rr * kHotMax;
        int k = 0;
        for (; k + 3 < nh; k += 4) {
          const int h0 = read_lane(hp, k), h1 = read_lane(hp, k + 1);
          const int h2 = read_lane(hp, k + 2), h3 = read_lane(hp, k + 3);
          const double w0 = read_lane(vp, k), w1 = read_lane(vp, k + 1);
          const double w2 = read_lane(vp, k + 2), w3 = read_lane(vp, k + 3);
          if (in_f) t += (w0 * g[h0] + w1 * g[h1]) + (w2 * g[h2] + w3 * g[h3]);
        }
        for (; k < nh; ++k) {
          const int h0 = read_lane(hp, k);
          const double w0 = read_lane(vp, k);
          if (in_f) t += w0 * g[h0];
        }
      }
      double part = hot ? v64 * t : 2.0 * v64 * t;
      if (nc == 1 && in_f && !hot) part += v64 * v64 * a.lev[rr];
      if (nc >= 2 && !kInline) cold |= 1ull << i;
      if (nc >= 2 && kInline) {
        const T vv = in_f ? vals[e0 + lane] : T(0);
        part += cold_rows_z2<T, VEC>(mc, rr, vv, Qb, a.ldq, hi);
      }
      const double z2 = wave_sum(part);
      const double x2 = wave_sum(v64 * v64);
      if (lane == 0) a.resid[f] = x2 - z2;
    }
    if (cold) {
      int32_t base = 0;
      if (lane == 0) base = atomicAdd(&sc->n_cold, (int32_t)__popcll(cold));
      base = __shfl(base, 0, kWave);
      if ((cold >> lane) & 1) a.cold_list[base + __popcll(cold & lt)] = (int32_t)(fb + lane);
    }
  }
}

// ||z_C||^2 of listed fiber i over column slice blockIdx.x of gridDim.x, into
// zpart[slice][i]: one wave per fiber, its cold (row, value) pairs packed
// into lanes 0 .. n_cold - 1 and gathered as in k_proj_multi.
template <typename T, int VEC>
__global__ __launch_bounds__(kBlock) void k_proj_cold(ProjectArgs a, const DevScalars* sc) {
  constexpr int kCols = VEC * kWave;
  if (sc->status != 0) return;
  const int64_t n_cold = sc->n_cold;
  const int slice = blockIdx.x;
  int64_t lo, hi;
  slice_cols<VEC>(*a.d_ncols, gridDim.x, slice, lo, hi);
  const int lane = lane_id();
  const T* Qb = sizeof(T) == 8 ? (const T*)a.Q : (const T*)a.Qf;
  const T* vals = sizeof(T) == 8 ? (const T*)a.val : (const T*)a.val32;
  double* zp = a.zpart + (int64_t)slice * a.zpart_ld;
  const int64_t nwaves = (int64_t)gridDim.y * (kBlock / kWave);
  for (int64_t i = ((int64_t)blockIdx.y * kBlock + threadIdx.x) / kWave; i < n_cold; i += nwaves) {
    const int32_t f = a.cold_list[i];
    const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
    const int n = e1 - e0;
    const bool in_f = lane < n;
    const int32_t rr = in_f ? a.row[e0 + lane] : 0;
    const T vv = in_f ? vals[e0 + lane] : T(0);
    const bool cold = in_f && a.hot_id[rr] < 0;
    const uint64_t mc = __ballot(cold);
    const int nc = __popcll(mc);
    const int src = packed_source(mc, lane);
    const int32_t rc = __shfl(rr, src, kWave);
    const T vc = __shfl(vv, src, kWave);
    double z2 = 0.0;
    if (hi - lo > kCols) {
      for (int64_t c0 = lo; c0 < hi; c0 += 2 * kCols) {
        const int64_t ca = c0 + (int64_t)VEC * lane, cb = ca + kCols;
        const bool ina = ca < hi, inb = cb < hi;
        T acc0[VEC], acc1[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) acc0[k] = acc1[k] = T(0);
        gather_batch<T, VEC>(rc, vc, nc, Qb + (ina ? ca : 0), Qb + (inb ? cb : 0), ina, inb, a.ldq,
                             acc0, acc1);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
          const double d0 = (double)acc0[j], d1 = (double)acc1[j];
          z2 += (ca + j < hi) ? d0 * d0 : 0.0;
          z2 += (cb + j < hi) ? d1 * d1 : 0.0;
        }
      }
    } else {
      const int64_t ca = lo + (int64_t)VEC * lane;
      const bool in = ca < hi;
      T acc[VEC];
#pragma unroll
      for (int k = 0; k < VEC; ++k) acc[k] = T(0);
      gather_seg<T, VEC>(rc, vc, nc, Qb + (in ? ca : 0), in, a.ldq, acc);
#pragma unroll
      for (int j = 0; j < VEC; ++j) {
        const double d = (double)acc[j];
        z2 += (ca + j < hi) ? d * d : 0.0;
      }
    }
    z2 = wave_sum(z2);
    if (lane == 0) zp[i] = z2;
  }
}

// resid[f] -= sum over the S slices (in slice order) of listed fiber i.
__global__ __launch_bounds__(kBlock) void k_proj_cold_fin(ProjectArgs a, const DevScalars* sc,
                                                          int S) {
  if (sc->status != 0) return;
  const int64_t n_cold = sc->n_cold;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_cold;
       i += (int64_t)gridDim.x * kBlock) {
    double z2 = 0.0;
    for (int sl = 0; sl < S; ++sl) z2 += a.zpart[(int64_t)sl * a.zpart_ld + i];
    a.resid[a.cold_list[i]] -= z2;
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
// in LDS in wave order) and stores the slice's ||z||^2.  With the hot-row
// split (hot set) only the cold nonzeros of each batch are gathered (packed
// into the batch's first lanes), so the result is the slice's ||z_C||^2.
template <typename T, int VEC>
__global__ __launch_bounds__(kLongWaves * kWave) void k_proj_long(ProjectArgs a,
                                                                  const DevScalars* sc, bool hot) {
  constexpr int kCols = VEC * kWave;
  __shared__ double red[kLongWaves * VEC * kWave];
  if (sc->status != 0) return;
  const int64_t n_long = sc->n_long;
  int64_t lo, hi;
  slice_cols<VEC>(*a.d_ncols, gridDim.x, blockIdx.x, lo, hi);
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const T* Qb = sizeof(T) == 8 ? (const T*)a.Q : (const T*)a.Qf;
  const T* vals = sizeof(T) == 8 ? (const T*)a.val : (const T*)a.val32;
  // with the hot split about half of a batch is gathered: take twice as many
  const int batch = hot ? 2 * kLongBatch : kLongBatch;
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
      for (int32_t eb = e0 + wv * batch; eb < e1; eb += kLongWaves * batch) {
        const int n = min(batch, e1 - eb);
        int32_t rr = lane < n ? a.row[eb + lane] : 0;
        T vv = lane < n ? vals[eb + lane] : T(0);
        int nc = n;
        if (hot) {
          const uint64_t mc = __ballot(lane < n && a.hot_id[rr] < 0);
          nc = __popcll(mc);
          const int src = packed_source(mc, lane);
          rr = __shfl(rr, src, kWave);
          vv = __shfl(vv, src, kWave);
        }
        gather_seg<T, VEC>(rr, vv, nc, Qb + (in ? c : 0), in, a.ldq, acc);
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

// k_proj_long_fin with the hot-row split, one workgroup of kFinWaves waves
// per listed fiber (the slices hold ||z_C||^2).  The fiber's hot values are
// placed at their hot index in LDS (a fiber holds each row at most once, so
// at most kHotMax hot nonzeros land on distinct slots); then every nonzero e
// gets t_e = sum over the fiber's hot h of c_h GH[r_e][h], and the hot part
// sum_{e hot} v_e t_e + 2 sum_{e cold} v_e t_e is added to the slices.  The
// waves take the nonzeros in interleaved chunks of 64 and their sums are
// added in wave order.
__global__ __launch_bounds__(kFinWaves * kWave) void k_proj_long_fin_hot(ProjectArgs a,
                                                                          const DevScalars* sc,
                                                                          int S) {
  __shared__ double cv[kHotMax];
  __shared__ int32_t on[kHotMax];
  __shared__ double red[2][kFinWaves];
  if (sc->status != 0) return;
  const int64_t n_long = sc->n_long;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  for (int64_t i = blockIdx.x; i < n_long; i += gridDim.x) {
    const int32_t f = a.long_list[i];
    const int32_t e0 = a.fptr[f], e1 = a.fptr[f + 1];
    if (threadIdx.x < kHotMax) {
      on[threadIdx.x] = 0;
      cv[threadIdx.x] = 0.0;
    }
    __syncthreads();
    double x2 = 0.0;
    for (int32_t eb = e0 + wv * kWave; eb < e1; eb += kFinWaves * kWave) {
      const bool in = eb + lane < e1;
      const double v = in ? a.val[eb + lane] : 0.0;
      x2 += v * v;
      const int32_t hid = in ? a.hot_id[a.row[eb + lane]] : -1;
      if (hid >= 0) {
        cv[hid] = v;
        on[hid] = 1;
      }
    }
    __syncthreads();
    const bool any = __ballot(on[lane] != 0) != 0;
    double part = 0.0;
    if (any) {
      // t_e = GH[r_e] . c over the hot indices in use, c dense in LDS (0 where
      // the fiber has no nonzero; GH is 0 past the hot count), the row read
      // as 16-byte vectors, kHotGroup entries in flight
      const int n_hot = a.hot_meta[kHotMax];
      for (int32_t eb = e0 + wv * kWave; eb < e1; eb += kFinWaves * kWave) {
        const bool in = eb + lane < e1;
        const int32_t rr = in ? a.row[eb + lane] : 0;
        const double v = in ? a.val[eb + lane] : 0.0;
        const bool is_hot = in && a.hot_id[rr] >= 0;
        const double2* g = (const double2*)(a.GH + (int64_t)rr * kHotMax);
        double t = 0.0;
        for (int h0 = 0; h0 < n_hot; h0 += kHotGroup) {
          double2 x[kHotGroup / 2];
#pragma unroll
          for (int u = 0; u < kHotGroup / 2; ++u) x[u] = in ? g[h0 / 2 + u] : double2{0.0, 0.0};
#pragma unroll
          for (int u = 0; u < kHotGroup / 2; ++u)
            t += x[u].x * cv[h0 + 2 * u] + x[u].y * cv[h0 + 2 * u + 1];
        }
        part += is_hot ? v * t : 2.0 * v * t;
      }
    }
    x2 = wave_sum(x2);
    part = wave_sum(part);
    if (lane == 0) {
      red[0][wv] = x2;
      red[1][wv] = part;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double xs = 0.0, z2 = 0.0;
      for (int w = 0; w < kFinWaves; ++w) {
        xs += red[0][w];
        z2 += red[1][w];
      }
      for (int sl = 0; sl < S; ++sl) z2 += a.long_part[i * a.long_ld + sl];
      a.resid[f] = xs - z2;
    }
    __syncthreads();
  }
}

__global__ void k_zero_long(DevScalars* sc) {
  sc->n_long = 0;
  sc->n_cold = 0;
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
  int choice = tune_get(st, TUNE_PROJ_FPW, prec, bucket, kNCand);
  std::vector<hipEvent_t> tev;
  const bool measure = choice < 0 && tune_begin(st, TUNE_PROJ_FPW, prec, bucket, kNCand, &tev);
  if (choice < 0) choice = small ? 0 : 2;
  // Hot rows for a large input over few enough rows (whole rows: the hot
  // split leaves too few gathers to gain from column slices).
  const bool hot = a.GH && !small && a.n_rows > 0 && a.n_rows <= kHotMaxRows;
  const int s_max = proj_slices(a.ncols_max, 4 * kWave);
  const int S = hot ? 1 : small ? s_max : std::min(a.mixed ? 1 : 2, s_max);
  auto multi = [&](int c) {
    const int fpw = kFpw[c];
    hipLaunchKernelGGL(k_zero_long, dim3(1), dim3(1), 0, st, sc);
    const int64_t waves = (std::max<int64_t>(nnz_max, 1) + fpw - 1) / fpw;
    const int gm = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (waves + 3) / 4));
    const dim3 grid(S, gm);
    if (hot && a.mixed)
      hipLaunchKernelGGL((k_proj_multi_hot<float, 8, true>), dim3(gm), dim3(kBlock), 0, st, a, sc,
                         fpw);
    else if (hot)
      hipLaunchKernelGGL((k_proj_multi_hot<double, 4, false>), dim3(gm), dim3(kBlock), 0, st, a, sc,
                         fpw);
    else if (S > 1 && a.mixed)
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
  if (hot) {
    const int n_rows = (int)a.n_rows;
    hipLaunchKernelGGL(k_hot_clear, dim3(div_up(n_rows, kBlock)), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_hot_count, dim3(kHotParts), dim3(1024), 0, st, a, sc);
    hipLaunchKernelGGL(k_hot_select, dim3(1), dim3(1024), 0, st, a, sc);
    hipLaunchKernelGGL(k_hot_gram, dim3(div_up(n_rows, 32)), dim3(kBlock), 0, st, a, sc);
  }
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
  if (hot && !a.mixed) {
    // float64: the listed fibers' cold rows in kColdSlices column slices
    // (float32 rows are half as long and are gathered whole, inline)
    const dim3 grid(kColdSlices,
                    (int)std::max<int64_t>(1, std::min<int64_t>(4096, div_up(nnz_max / 2 + 1, 4))));
    hipLaunchKernelGGL((k_proj_cold<double, 4>), grid, dim3(kBlock), 0, st, a, sc);
    hipLaunchKernelGGL(k_proj_cold_fin,
                       dim3(std::max(1, std::min(4096, div_up(nnz_max / 2 + 1, kBlock)))),
                       dim3(kBlock), 0, st, a, sc, kColdSlices);
  }
  if (S > 1)
    hipLaunchKernelGGL(k_proj_multi_fin,
                       dim3((int)std::max<int64_t>(1, std::min<int64_t>(4096, div_up(nnz_max, kBlock)))),
                       dim3(kBlock), 0, st, a, sc, S);
  const int s_long = proj_slices(a.ncols_max, (a.mixed ? 8 : 4) * kWave);
  if (a.mixed)
    hipLaunchKernelGGL((k_proj_long<float, 8>), dim3(s_long, gy), dim3(kLongWaves * kWave), 0, st,
                       a, sc, hot);
  else
    hipLaunchKernelGGL((k_proj_long<double, 4>), dim3(s_long, gy), dim3(kLongWaves * kWave), 0, st,
                       a, sc, hot);
  if (hot)
    hipLaunchKernelGGL(k_proj_long_fin_hot,
                       dim3((int)std::max<int64_t>(1, std::min<int64_t>(8192, max_long))),
                       dim3(kFinWaves * kWave), 0, st, a, sc, s_long);
  else
    hipLaunchKernelGGL(k_proj_long_fin,
                       dim3(std::max(1, std::min(1024, (int)div_up(max_long * kWave, kBlock)))),
                       dim3(kBlock), 0, st, a, sc, s_long);
  if (ev1) (void)hipEventRecord(ev1, st);
  const int np = std::max(1, div_up(nnz_max, kRedBlock * kRedItems));
  hipLaunchKernelGGL(k_reduce_partial, dim3(np), dim3(kRedBlock), 0, st, a.resid, a.partial, sc);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedBlock), 0, st, a.partial, np, sc);
}

}  // namespace ctd

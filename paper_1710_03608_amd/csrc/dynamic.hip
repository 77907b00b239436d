// CTD-D (Section 3.2, Algorithm 2) and the core tensor C of CTD-S
// (the final step of Algorithm 1).
//
// State kept between slices (all device memory):
//   Rs  n_rows x capD  the kept fibers (the paper's R), row-major
//   Q   n_rows x capD  orthonormal basis of span(R)
//   Xt  capD x capD    upper triangular M with Q = R M, so U = (R^T R)^{-1} = M M^T
//   C   capD x capN    C_(alpha) = R^T X_(alpha), column-major, one column per
//                      non-empty fiber seen so far (tensor then slices)
// One slice dX with d draws:
//   1. fibers, weights, draws (Philox counter word = step t), unique
//      candidates: the same kernels as CTD-S (the sampling steps of Algorithm 2);
//   2. the candidates are tested against R^(t) and each other and the kept
//      ones extend R, Q and M: the same block filter as CTD-S, started from
//      the d~_t columns already held (the independence loop of Algorithm 2);
//   3. C (the core update of Algorithm 2, Eq. 13): rows for the kept fibers over the earlier
//      columns are ((dR^T R^(t)) U^(t)) C^(t), parenthesized from the left as
//      the paper prescribes; with w = Q^(t)T x the row vector dR^T R^(t) U^(t)
//      equals (M^(t) w)^T, so one pass over C^(t) applies them; the new
//      columns are R^(t+1)T dX;
//   4. error: earlier columns keep their reconstruction (span(R) only grows),
//      so ||X^(t+1) - X~^(t+1)||^2 = E^(t) + ||dX - P_{t+1} dX||^2, the slice
//      term computed by the CTD-S projection kernels with the grown Q.
#include <string.h>

#include <string>
#include <vector>

#include "gather.h"
#include "state.h"

namespace ctd {

namespace {
constexpr int kBlock = 256;

// Clear the per-call scalars.  With keep_stream the stream totals, the basis
// size, the column count and the batch base stay in place: they are neither
// read nor written here.  (A copy-then-restore would read fields through the
// scalar cache and overwrite the same bytes with vector stores; the two are
// not ordered, so the restore could pick up the zeros.)
__global__ void k_reset(DevScalars* sc, bool keep_stream) {
  if (threadIdx.x != 0) return;
  sc->W = 0;
  sc->vmax2_bits = 0;
  sc->norm2 = 0.0;
  sc->err2 = 0.0;
  sc->status = 0;
  sc->sigma = 0;
  sc->n_f = 0;
  sc->s_unique = 0;
  sc->s_tilde = 0;
  sc->base_accept = 0;
  sc->n_long = 0;
  sc->blk_na = 0;
  sc->blk_reorth = 0;
  sc->allow_empty = keep_stream ? 1 : 0;
  if (!keep_stream) {
    sc->total_norm2 = 0.0;
    sc->total_err2 = 0.0;
    sc->n_cols_total = 0;
    sc->n_accept_total = 0;
    sc->wacc_base = 0;
  }
}

__global__ void k_static_totals(DevScalars* sc) {
  sc->total_norm2 = sc->norm2;
  sc->total_err2 = sc->err2;
  sc->n_accept_total = sc->s_tilde;
  sc->n_cols_total = sc->n_f;
}

// Columns of R^T X: out[(col0 + f) * ldo + k] = sum_e v_e A[r_e][k] for
// k < ncols and every fiber f < n_f.  A wave takes fpw consecutive fibers
// (64 for a large input; a few for a small one such as a time slice, so that
// its few fibers still spread over many waves) and walks those of up to
// kLongFiber nonzeros (rows and values loaded once into lanes and broadcast,
// two nonzeros times two 256-column chunks in flight) over the columns
// [cspan y, cspan (y + 1)) of y = blockIdx.y; longer ones are listed (by the
// y = 0 workgroups) for k_spmm_long.
template <typename TO>
__global__ __launch_bounds__(kBlock) void k_spmm_cols(const int32_t* __restrict__ fptr,
                                                      const int32_t* __restrict__ row,
                                                      const double* __restrict__ val,
                                                      DevScalars* sc,
                                                      const double* __restrict__ A, int64_t lda,
                                                      const int32_t* d_ncols,
                                                      TO* __restrict__ out, int64_t ldo,
                                                      const int64_t* d_col0,
                                                      int32_t* __restrict__ long_list, int fpw,
                                                      int64_t cspan) {
  constexpr int VEC = 4, kCols = VEC * kWave;
  const int64_t n_f = sc->status == 0 ? sc->n_f : 0;
  const int64_t ncols = *d_ncols;
  const int64_t col0 = d_col0 ? *d_col0 : 0;
  const int64_t c_beg = (int64_t)blockIdx.y * cspan;
  if (c_beg >= ncols) return;
  const int64_t c_end = min(ncols, c_beg + cspan);
  const int lane = lane_id();
  const uint64_t lt = lane == 0 ? 0ull : ((~0ull) >> (kWave - lane));
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  for (int64_t fb = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave * fpw; fb < n_f;
       fb += nwaves * fpw) {
    const int64_t fl = fb + lane;
    int32_t len = 0;
    if (lane < fpw && fl < n_f) len = fptr[fl + 1] - fptr[fl];
    const bool lng = len > kLongFiber;
    const uint64_t ml = __ballot(lng);
    if (ml && blockIdx.y == 0) {
      int32_t base = 0;
      if (lane == 0) base = atomicAdd(&sc->n_long, (int32_t)__popcll(ml));
      base = __shfl(base, 0, kWave);
      if (lng) long_list[base + __popcll(ml & lt)] = (int32_t)fl;
    }
    uint64_t todo = __ballot(len > 0 && !lng);
    while (todo) {
      const int i = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int64_t f = fb + i;
      const int32_t e0 = fptr[f];
      const int n = fptr[f + 1] - e0;
      const int32_t rr = lane < n ? row[e0 + lane] : 0;
      const double vv = lane < n ? val[e0 + lane] : 0.0;
      TO* o = out + (col0 + f) * ldo;
      for (int64_t c0 = c_beg; c0 < c_end; c0 += 2 * kCols) {
        const int64_t ca = c0 + (int64_t)VEC * lane, cb = ca + kCols;
        const bool ina = ca < c_end, inb = cb < c_end;
        double acc0[VEC], acc1[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) acc0[k] = acc1[k] = 0.0;
        gather_batch<double, VEC>(rr, vv, n, A + (ina ? ca : 0), A + (inb ? cb : 0), ina, inb,
                                  lda, acc0, acc1);
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          if (ca + k < c_end) o[ca + k] = (TO)acc0[k];
          if (cb + k < c_end) o[cb + k] = (TO)acc1[k];
        }
      }
    }
  }
}

// Listed long fibers: workgroup (chunk, i) writes one 256-column chunk of
// fiber i's column.
template <typename TO>
__global__ __launch_bounds__(kLongWaves * kWave) void k_spmm_long(
    const int32_t* __restrict__ fptr, const int32_t* __restrict__ row,
    const double* __restrict__ val, const DevScalars* sc, const double* __restrict__ A,
    int64_t lda, const int32_t* d_ncols, TO* __restrict__ out, int64_t ldo,
    const int64_t* d_col0, const int32_t* __restrict__ long_list) {
  constexpr int VEC = 4, kCols = VEC * kWave;
  __shared__ double red[kLongWaves * VEC * kWave];
  if (sc->status != 0) return;
  const int64_t n_long = sc->n_long;
  const int64_t ncols = *d_ncols;
  const int64_t col0 = d_col0 ? *d_col0 : 0;
  const int64_t c0 = (int64_t)blockIdx.x * kCols;
  if (c0 >= ncols) return;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int64_t c = c0 + (int64_t)VEC * lane;
  const bool in = c < ncols;
  for (int64_t i = blockIdx.y; i < n_long; i += gridDim.y) {
    const int32_t f = long_list[i];
    double z[VEC];
    wg_gather_chunk<double, VEC>(row, val, fptr[f], fptr[f + 1], A + (in ? c : 0), in, lda, red,
                                 z);
    if (wv == 0) {
      TO* o = out + (col0 + f) * ldo;
#pragma unroll
      for (int k = 0; k < VEC; ++k)
        if (c + k < ncols) o[c + k] = (TO)z[k];
    }
  }
}

__global__ void k_zero_long(DevScalars* sc) { sc->n_long = 0; }

// Batch bookkeeping.  info[2 b], info[2 b + 1]: fibers kept and columns held
// when slice b of the batch starts (b = B: when the batch ends).
__global__ void k_batch_mark(const DevScalars* sc, int64_t* info, int b) {
  info[2 * b] = sc->n_accept_total;
  info[2 * b + 1] = sc->n_cols_total;
}
__global__ void k_batch_begin(DevScalars* sc) { sc->wacc_base = sc->n_accept_total; }

// Range of cross pass p (Eq. 13 over a batch of B slices): the fibers kept by
// the batch that were not yet held when the columns were added get their rows
// ((dR^T R) U) C over those columns, with R, U truncated to the rank K the
// columns were created with.  Pass 0: columns held before the batch, K = the
// rank at the batch start (one pass over C^(t) for all B slices, since
// P_{t+b} P_t = P_t).  Pass b + 1: the columns of slice b, K = the rank after
// slice b, rows of the fibers kept by later slices.  rng = {K, a_lo, na, c_lo,
// c_hi}: rows a_lo .. a_lo + na of the batch's Wacc, C rows K .. K + na.
__global__ void k_cross_setup(const int64_t* info, int B, const DevScalars* sc, int64_t* rng) {
  const int p = threadIdx.x;
  if (p >= B) return;
  const int64_t base = info[0], total = info[2 * B] - base;
  int64_t K, c_lo, c_hi;
  if (p == 0) {
    K = info[0];
    c_lo = 0;
    c_hi = info[1];
  } else {
    const int b = p - 1;
    K = info[2 * (b + 1)];
    c_lo = info[2 * b + 1];
    c_hi = info[2 * (b + 1) + 1];
  }
  const int64_t a_lo = K - base;
  int64_t* r = rng + 5 * p;
  r[0] = K;
  r[1] = a_lo;
  r[2] = sc->status == 0 ? total - a_lo : 0;
  r[3] = c_lo;
  r[4] = c_hi;
}

// Rows of ((dR^T R) U): Y[a][c] = sum_{c <= j < K} M[c][j] Wacc[a_lo + a][j]
// for c < K (with w = Q^T x the row x^T R U equals (M w)^T); one wave per c,
// pass p = blockIdx.y writing Y + p * ystride.
__global__ __launch_bounds__(kBlock) void k_cross_rows(const double* __restrict__ M, int64_t ldm,
                                                       const double* __restrict__ Wacc,
                                                       int64_t ldw, double* __restrict__ Yall,
                                                       int64_t ldy, int64_t ystride,
                                                       const int64_t* rng_all) {
  const int64_t* rng = rng_all + 5 * blockIdx.y;
  double* Y = Yall + blockIdx.y * ystride;
  const int64_t K = rng[0], a_lo = rng[1], na = rng[2];
  const int lane = lane_id();
  const int64_t c = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (c >= K || na <= 0) return;
  const double* mr = M + c * ldm;
  for (int64_t a = 0; a < na; ++a) {
    const double* w = Wacc + (a_lo + a) * ldw;
    double s = 0.0;
    for (int64_t j = c + lane; j < K; j += kWave) s += mr[j] * w[j];
    s = wave_sum(s);
    if (lane == 0) Y[a * ldy + c] = s;
  }
}

// Cross term: C[d + a][f] = sum_{k<d} Y[a][k] C[k][f] for f in [c_lo, c_hi)
// (d = K of the pass; pass 0 reads all of C^(t): the HBM-bound step).  Pass
// p = blockIdx.y.  A product of the 16 RT new rows with C, on f64 MFMAs: wave
// w of a workgroup owns the 16 CT columns 16 CT w .. + 16 CT (CT 16-column
// tiles) against all RT row tiles.  The reduction runs in chunks of 16 rows
// of C; lane (i, g) = (l % 16, l / 16) reads C[k0 + 4 g .. + 4][f] of its
// column as one 32-byte vector (C is column-major), and MFMA t multiplies
// element t with Y[a][k0 + 4 g + t], so the four MFMAs of a chunk cover its 16
// rows in a fixed permutation.  The 16 RT x 16 Y chunk is shared through LDS
// (double-buffered, one barrier per chunk); the next chunk of C is in flight
// in registers while the current one is in the MFMAs.  C is read once per
// 16 RT new rows.  NW waves a workgroup (the Y chunk needs 4 x 16 RT
// threads).  With RT = 4 two column tiles per wave (CT = 2) leave room for
// three waves per SIMD instead of one: more of C in flight per CU.
constexpr int kCrossCols = 256;

template <int RT, int NW = 4, int CT = 2>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(CT < 4 ? 3 : 1)))
void k_cross_term(double* __restrict__ C, int64_t ldc,
                                                           const double* __restrict__ Yall,
                                                           int64_t ldy, int64_t ystride,
                                                           const int64_t* rng_all) {
  constexpr int kRows = 16 * RT;
  __shared__ dbl4 Ys[2][kRows][5];   // [buf][row a][g]: Y[a][k0 + 4 g .. + 4], padded
  const int64_t* rng = rng_all + 5 * blockIdx.y;
  const double* Y = Yall + blockIdx.y * ystride;
  const int64_t d = rng[0], na = rng[2], ncols = rng[4];
  static_assert(64 * NW >= 4 * 16 * RT, "the Y chunk needs 4 threads per row");
  const int64_t f0 = rng[3] + (int64_t)blockIdx.x * (16 * CT * NW);
  if (na <= 0 || f0 >= ncols) return;
  const int t = threadIdx.x, w = t / kWave, l = lane_id(), i = l % 16, g = l / 16;
  const int64_t nch = (d + 15) / 16;
  const double* cp[CT];
  bool cin[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int64_t f = f0 + 16 * CT * w + 16 * ct + i;
    cin[ct] = f < ncols;
    cp[ct] = C + (cin[ct] ? f : f0) * ldc + 4 * g;
  }
  const int yr = t / 4, yg = t % 4;   // this thread's 4 values of the Y chunk
  // zero the elements of a 4-vector at rows k .. k + 3 that lie at or past d
  auto mask4 = [&](dbl4 v, int64_t k) -> dbl4 {
    v[0] = k < d ? v[0] : 0.0;
    v[1] = k + 1 < d ? v[1] : 0.0;
    v[2] = k + 2 < d ? v[2] : 0.0;
    v[3] = k + 3 < d ? v[3] : 0.0;
    return v;
  };
  for (int64_t a0 = 0; a0 < na; a0 += kRows) {
    const int nr = (int)min<int64_t>(kRows, na - a0);
    const bool yin = yr < nr;
    const double* yrow = Y + (a0 + (yin ? yr : 0)) * ldy + 4 * yg;
    dbl4 acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = dbl4{0, 0, 0, 0};
    dbl4 cf[CT], yv;
    auto load = [&](int64_t ch) {
      const int64_t k = ch * 16 + 4 * g;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        cf[ct] = (ch < nch && cin[ct] && k < d) ? *(const dbl4*)(cp[ct] + ch * 16) : dbl4{0, 0, 0, 0};
        cf[ct] = mask4(cf[ct], k);
      }
      const int64_t ky = ch * 16 + 4 * yg;
      yv = (ch < nch && yin && ky < d) ? *(const dbl4*)(yrow + ch * 16) : dbl4{0, 0, 0, 0};
      yv = mask4(yv, ky);
    };
    load(0);
    int buf = 0;
    for (int64_t ch = 0; ch < nch; ++ch) {
      if (yr < kRows) Ys[buf][yr][yg] = yv;
      dbl4 cc[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) cc[ct] = cf[ct];
      __syncthreads();
      load(ch + 1);
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const double a = Ys[buf][rt * 16 + i][g][tt];
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = mfma16(a, cc[ct][tt], acc[rt][ct]);
        }
      buf ^= 1;
    }
    // lane (i, g) holds D[g + 4 r][i] of tile (rt, ct): new row rt * 16 + g + 4 r, column ct * 16 + i
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      if (!cin[ct]) continue;
      double* col = C + (f0 + 16 * CT * w + 16 * ct + i) * ldc + d + a0;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = rt * 16 + g + 4 * r;
          if (a < nr) col[a] = acc[rt][ct][r];
        }
    }
    __syncthreads();   // the next row block reuses Ys
  }
}

// k_cross_term for at most 16 new rows (one row tile) without LDS: lane
// (i, g) needs exactly Y[a0 + i][k0 + 4 g .. + 4] for its MFMAs, so it reads
// that 32-byte vector itself (Y is small and stays in L2) and the waves run
// with no barrier between chunks.  The MFMAs see the same operands in the same
// order as when the chunk was staged through LDS, so the values are the same.
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3)))
void k_cross_term_direct(double* __restrict__ C, int64_t ldc, const double* __restrict__ Yall,
                         int64_t ldy, int64_t ystride, const int64_t* rng_all) {
  const int64_t* rng = rng_all + 5 * blockIdx.y;
  const double* Y = Yall + blockIdx.y * ystride;
  const int64_t d = rng[0], na = rng[2], ncols = rng[4];
  const int64_t f0 = rng[3] + (int64_t)blockIdx.x * (64 * NW);
  if (na <= 0 || f0 >= ncols) return;
  const int w = threadIdx.x / kWave, l = lane_id(), i = l % 16, g = l / 16;
  const int64_t nch = (d + 15) / 16;
  const double* cp[4];
  bool cin[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int64_t f = f0 + 64 * w + 16 * ct + i;
    cin[ct] = f < ncols;
    cp[ct] = C + (cin[ct] ? f : f0) * ldc + 4 * g;
  }
  auto mask4 = [&](dbl4 v, int64_t k) -> dbl4 {
    v[0] = k < d ? v[0] : 0.0;
    v[1] = k + 1 < d ? v[1] : 0.0;
    v[2] = k + 2 < d ? v[2] : 0.0;
    v[3] = k + 3 < d ? v[3] : 0.0;
    return v;
  };
  for (int64_t a0 = 0; a0 < na; a0 += 16) {
    const int nr = (int)min<int64_t>(16, na - a0);
    const bool yin = i < nr;
    const double* yrow = Y + (a0 + (yin ? i : 0)) * ldy + 4 * g;
    dbl4 acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = dbl4{0, 0, 0, 0};
    dbl4 cf[4], yv;
    auto load = [&](int64_t ch) {
      const int64_t k = ch * 16 + 4 * g;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        cf[ct] = (ch < nch && cin[ct] && k < d) ? *(const dbl4*)(cp[ct] + ch * 16) : dbl4{0, 0, 0, 0};
        cf[ct] = mask4(cf[ct], k);
      }
      yv = (ch < nch && yin && k < d) ? *(const dbl4*)(yrow + ch * 16) : dbl4{0, 0, 0, 0};
      yv = mask4(yv, k);
    };
    load(0);
    for (int64_t ch = 0; ch < nch; ++ch) {
      dbl4 cc[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) cc[ct] = cf[ct];
      const dbl4 ya = yv;
      load(ch + 1);
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma16(ya[tt], cc[ct][tt], acc[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      if (!cin[ct]) continue;
      double* col = C + (f0 + 64 * w + 16 * ct + i) * ldc + d + a0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = g + 4 * r;
        if (a < nr) col[a] = acc[ct][r];
      }
    }
  }
}

// The same product for a mixed-precision handle, whose C is held in float32:
// float32 MFMAs (v_mfma_f32_16x16x4f32) with float32 accumulation, Y rounded to
// float32 as it is staged.  The reduction runs in chunks of 32 rows so that a
// lane still reads 32 bytes of its column (8 consecutive rows, k0 + 8 g ..),
// and MFMA t (t < 8) takes element t of them.  Lane l holds D[4 (l / 16) +
// r][l % 16] of a 16 x 16 float32 tile.  NW waves a workgroup, as above.
template <int RT, int NW = 4>
__global__ __launch_bounds__(64 * NW) void k_cross_term32(float* __restrict__ C, int64_t ldc,
                                                             const double* __restrict__ Yall,
                                                             int64_t ldy, int64_t ystride,
                                                             const int64_t* rng_all) {
  typedef float flt4 __attribute__((ext_vector_type(4)));
  typedef float flt8 __attribute__((ext_vector_type(8)));
  constexpr int kRows = 16 * RT;
  __shared__ flt8 Ys[2][kRows][5];   // [buf][row a][g]: Y[a][k0 + 8 g .. + 8], padded
  const int64_t* rng = rng_all + 5 * blockIdx.y;
  const double* Y = Yall + blockIdx.y * ystride;
  const int64_t d = rng[0], na = rng[2], ncols = rng[4];
  static_assert(64 * NW >= 4 * 16 * RT, "the Y chunk needs 4 threads per row");
  const int64_t f0 = rng[3] + (int64_t)blockIdx.x * (64 * NW);
  if (na <= 0 || f0 >= ncols) return;
  const int t = threadIdx.x, w = t / kWave, l = lane_id(), i = l % 16, g = l / 16;
  const int64_t nch = (d + 31) / 32;
  const float* cp[4];
  bool cin[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int64_t f = f0 + 64 * w + 16 * ct + i;
    cin[ct] = f < ncols;
    cp[ct] = C + (cin[ct] ? f : f0) * ldc + 8 * g;
  }
  const int yr = t / 4, yg = t % 4;
  auto mask8 = [&](flt8 v, int64_t k) -> flt8 {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = k + e < d ? v[e] : 0.0f;
    return v;
  };
  for (int64_t a0 = 0; a0 < na; a0 += kRows) {
    const int nr = (int)min<int64_t>(kRows, na - a0);
    const bool yin = yr < nr;
    const double* yrow = Y + (a0 + (yin ? yr : 0)) * ldy + 8 * yg;
    flt4 acc[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = flt4{0, 0, 0, 0};
    flt8 cf[4], yv;
    auto load = [&](int64_t ch) {
      const int64_t k = ch * 32 + 8 * g;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        cf[ct] = (ch < nch && cin[ct] && k < d) ? *(const flt8*)(cp[ct] + ch * 32)
                                                 : flt8{0, 0, 0, 0, 0, 0, 0, 0};
        cf[ct] = mask8(cf[ct], k);
      }
      const int64_t ky = ch * 32 + 8 * yg;
      dbl4 ya = {0, 0, 0, 0}, yb = {0, 0, 0, 0};
      if (ch < nch && yin && ky < d) {
        ya = *(const dbl4*)(yrow + ch * 32);
        yb = *(const dbl4*)(yrow + ch * 32 + 4);
      }
      yv = mask8(flt8{(float)ya[0], (float)ya[1], (float)ya[2], (float)ya[3],
                      (float)yb[0], (float)yb[1], (float)yb[2], (float)yb[3]}, ky);
    };
    load(0);
    int buf = 0;
    for (int64_t ch = 0; ch < nch; ++ch) {
      if (yr < kRows) Ys[buf][yr][yg] = yv;
      flt8 cc[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) cc[ct] = cf[ct];
      __syncthreads();
      load(ch + 1);
#pragma unroll
      for (int tt = 0; tt < 8; ++tt)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const float a = Ys[buf][rt * 16 + i][g][tt];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, cc[ct][tt], acc[rt][ct], 0, 0, 0);
        }
      buf ^= 1;
    }
    // lane (i, g) holds D[4 g + r][i] of tile (rt, ct): new row rt * 16 + 4 g + r, column ct * 16 + i
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      if (!cin[ct]) continue;
      float* col = C + (f0 + 64 * w + 16 * ct + i) * ldc + d + a0;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = rt * 16 + 4 * g + r;
          if (a < nr) col[a] = acc[rt][ct][r];
        }
    }
    __syncthreads();   // the next row block reuses Ys
  }
}

// The float32 product for more than 16 new rows (batches of slices), which
// the float32 MFMA rate bounds, on bfloat16 MFMAs (v_mfma_f32_16x16x32_bf16,
// float32 accumulation).  Each float32 operand is split into three bfloat16
// parts x ~ hi + mid + lo (each the rounded remainder of the ones before it;
// the remainders are exact in float32, and the three parts carry x to about
// 2^-24 relative).  Of the nine partial products the six of relative size
// 2^-16 or more (mid mid, lo hi, hi lo, mid hi, hi mid, hi hi, added in that
// order) are taken, so a product keeps about float32 accuracy; the six 16 x
// 16 x 32 MFMAs of a 32-row chunk take about 3/8 of the cycles of the eight
// 16 x 16 x 4 float32 MFMAs they replace.  The splitting costs vector-ALU work
// per element of C, so for the few new rows of a single slice, where HBM
// bounds the pass, the float32 form above stays.  A chunk is 32 rows of C:
// lane (i, g) reads rows k0 + 8 g .. + 8 of its column (32 bytes) as the B
// operand as laid out (no permutation); Y is rounded to float32 and split as
// it is staged in LDS.  Lane l holds D[4 (l / 16) + r][l % 16] of a 16 x 16
// float32 tile.  Each column tile of C is split just before its MFMAs (so the
// next tile's split overlaps them and one tile's parts are live at a time:
// two waves per SIMD); PF chunks of C and Y are in flight per wave.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
struct Split3 {
  bf8 hi, mid, lo;
};
__device__ inline Split3 split3(const float* x) {
  Split3 s;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 h = (__bf16)x[j];
    const float r1 = x[j] - (float)h;
    const __bf16 m = (__bf16)r1;
    const float r2 = r1 - (float)m;
    s.hi[j] = h;
    s.mid[j] = m;
    s.lo[j] = (__bf16)r2;
  }
  return s;
}
template <int RT, int PF>
__global__ __launch_bounds__(kCrossCols) __attribute__((amdgpu_waves_per_eu(2)))
void k_cross_term_bf3(float* __restrict__ C, int64_t ldc,
                                                             const double* __restrict__ Yall,
                                                             int64_t ldy, int64_t ystride,
                                                             const int64_t* rng_all) {
  typedef float flt4 __attribute__((ext_vector_type(4)));
  typedef float flt8 __attribute__((ext_vector_type(8)));
  constexpr int kRows = 16 * RT;
  __shared__ Split3 Ys[2][kRows][5];   // [buf][row a][g]: Y[a][k0 + 8 g .. + 8] split, padded
  const int64_t* rng = rng_all + 5 * blockIdx.y;
  const double* Y = Yall + blockIdx.y * ystride;
  const int64_t d = rng[0], na = rng[2], ncols = rng[4];
  const int64_t f0 = rng[3] + (int64_t)blockIdx.x * kCrossCols;
  if (na <= 0 || f0 >= ncols) return;
  const int t = threadIdx.x, w = t / kWave, l = lane_id(), i = l % 16, g = l / 16;
  const int64_t nch = (d + 31) / 32;
  const float* cp[4];
  bool cin[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int64_t f = f0 + 64 * w + 16 * ct + i;
    cin[ct] = f < ncols;
    cp[ct] = C + (cin[ct] ? f : f0) * ldc + 8 * g;
  }
  const int yr = t / 4, yg = t % 4;
  auto mask8 = [&](flt8 v, int64_t k) -> flt8 {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = k + e < d ? v[e] : 0.0f;
    return v;
  };
  for (int64_t a0 = 0; a0 < na; a0 += kRows) {
    const int nr = (int)min<int64_t>(kRows, na - a0);
    const bool yin = yr < nr;
    const double* yrow = Y + (a0 + (yin ? yr : 0)) * ldy + 8 * yg;
    flt4 acc[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = flt4{0, 0, 0, 0};
    // PF chunks of C (and of Y) in flight: slot u holds chunk ch0 + u
    flt8 cf[PF][4], yv[PF];
    auto load = [&](int64_t ch, flt8 (&cfs)[4], flt8& yvs) {
      const int64_t k = ch * 32 + 8 * g;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        cfs[ct] = (ch < nch && cin[ct] && k < d) ? *(const flt8*)(cp[ct] + ch * 32)
                                                  : flt8{0, 0, 0, 0, 0, 0, 0, 0};
        cfs[ct] = mask8(cfs[ct], k);
      }
      const int64_t ky = ch * 32 + 8 * yg;
      dbl4 ya = {0, 0, 0, 0}, yb = {0, 0, 0, 0};
      if (ch < nch && yin && ky < d) {
        ya = *(const dbl4*)(yrow + ch * 32);
        yb = *(const dbl4*)(yrow + ch * 32 + 4);
      }
      yvs = mask8(flt8{(float)ya[0], (float)ya[1], (float)ya[2], (float)ya[3],
                       (float)yb[0], (float)yb[1], (float)yb[2], (float)yb[3]}, ky);
    };
#pragma unroll
    for (int u = 0; u < PF; ++u) load(u, cf[u], yv[u]);
    int buf = 0;
    for (int64_t ch0 = 0; ch0 < nch; ch0 += PF) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int64_t ch = ch0 + u;
        if (ch >= nch) break;
        if (yr < kRows) {
          float yf[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) yf[e] = yv[u][e];
          Ys[buf][yr][yg] = split3(yf);
        }
        __syncthreads();
        Split3 ya[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) ya[rt] = Ys[buf][rt * 16 + i][g];
        // each column tile is split just before its MFMAs, so the split of the
        // next tile overlaps them; the slot is refilled once all are split
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          float cf8[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) cf8[e] = cf[u][ct][e];
          const Split3 cs = split3(cf8);
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            flt4 c = acc[rt][ct];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[rt].mid, cs.mid, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[rt].lo, cs.hi, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[rt].hi, cs.lo, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[rt].mid, cs.hi, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[rt].hi, cs.mid, c, 0, 0, 0);
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[rt].hi, cs.hi, c, 0, 0, 0);
          }
        }
        load(ch + PF, cf[u], yv[u]);
        buf ^= 1;
      }
    }
    // lane (i, g) holds D[4 g + r][i] of tile (rt, ct): new row rt * 16 + 4 g + r, column ct * 16 + i
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      if (!cin[ct]) continue;
      float* col = C + (f0 + 64 * w + 16 * ct + i) * ldc + d + a0;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = rt * 16 + 4 * g + r;
          if (a < nr) col[a] = acc[rt][ct][r];
        }
    }
    __syncthreads();   // the next row block reuses Ys
  }
}

// dst[f * ldd + k] = (float)src[f * lds + k] for k < rows, f < cols (a
// column-major float64 block converted to float32).
__global__ __launch_bounds__(kBlock) void k_cols_to_f32(const double* __restrict__ src,
                                                        int64_t lds, float* __restrict__ dst,
                                                        int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t f = t / rows, k = t % rows;
    dst[f * ldd + k] = (float)src[f * lds + k];
  }
}

__global__ void k_append_ids(const uint64_t* __restrict__ src, const int32_t* d_count,
                             uint64_t* __restrict__ dst, const int32_t* d_off32,
                             const int64_t* d_off64, uint64_t add) {
  const int64_t n = *d_count;
  const int64_t off = d_off32 ? (int64_t)*d_off32 : *d_off64;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[off + i] = src[i] + add;
}

__global__ void k_finish_slice(DevScalars* sc) {
  sc->total_norm2 += sc->norm2;
  sc->total_err2 += sc->err2;
  sc->n_cols_total += sc->n_f;
}

int grid_for(int64_t work, int per = kBlock);

// C columns R^T X for the fibers of the current input (short and long paths).
template <typename TO>
void launch_cols(hipStream_t st, const StaticBufs& b, int64_t nnz_max, DevScalars* sc,
                 const double* A, int64_t lda, const int32_t* d_ncols, int64_t ncols_max,
                 TO* out, int64_t ldo, const int64_t* d_col0) {
  // fibers per wave and column span: a small input (a time slice) has few
  // fibers, which must still spread over many waves (two per wave, columns
  // split over blockIdx.y in spans of 512); a large one takes 64 per wave
  // over all columns.  The autotuner picks among the candidates per
  // input-size bucket (all write the same values).
  static const int kFpw[] = {2, 8, kWave};
  constexpr int kNCand = 3;
  const int bucket = tune_bucket(nnz_max), prec = sizeof(TO) == 4 ? 1 : 0;
  int choice = tune_get(st, TUNE_COLS_FPW, prec, bucket, kNCand);
  std::vector<hipEvent_t> tev;
  const bool measure = choice < 0 && tune_begin(st, TUNE_COLS_FPW, prec, bucket, kNCand, &tev);
  if (choice < 0) choice = nnz_max <= (int64_t(1) << 18) ? 0 : 2;
  auto cols = [&](int c) {
    const int fpw = kFpw[c];
    const int64_t cspan = fpw < kWave ? 2 * 4 * kWave : std::max<int64_t>(ncols_max, 1);
    const int ny = (int)std::max<int64_t>(1, (ncols_max + cspan - 1) / cspan);
    const int64_t waves = (std::max<int64_t>(nnz_max, 1) + fpw - 1) / fpw;
    const int gm = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (waves + 3) / 4));
    hipLaunchKernelGGL(k_zero_long, dim3(1), dim3(1), 0, st, sc);
    hipLaunchKernelGGL(k_spmm_cols<TO>, dim3(gm, ny), dim3(kBlock), 0, st, b.fptr, b.row, b.val, sc,
                       A, lda, d_ncols, out, ldo, d_col0, b.long_list, fpw, cspan);
  };
  if (measure) {
    for (int c = 0; c < kNCand; ++c) {
      (void)hipEventRecord(tev[2 * c], st);
      cols(c);
      (void)hipEventRecord(tev[2 * c + 1], st);
    }
    tune_recorded(TUNE_COLS_FPW, prec, bucket);
  } else {
    cols(choice);
  }
  const int64_t max_long = nnz_max / (kLongFiber + 1) + 1;
  const int gy = (int)std::max<int64_t>(1, std::min<int64_t>(1024, max_long));
  const int nch = (int)std::max<int64_t>(1, (ncols_max + 4 * kWave - 1) / (4 * kWave));
  hipLaunchKernelGGL(k_spmm_long<TO>, dim3(nch, gy), dim3(kLongWaves * kWave), 0, st, b.fptr,
                     b.row, b.val, sc, A, lda, d_ncols, out, ldo, d_col0, b.long_list);
}

int grid_for(int64_t work, int per) {
  return std::max(1, std::min(8192, div_up(std::max<int64_t>(work, 1), per)));
}

#define HIP_CHECK(h, expr)                                                            \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess)                                                             \
      return fail(h, CTD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// (Re)allocate the CTD-D state with the given capacities, keeping contents.
ctd_status dyn_reserve(ctd_handle* h, int64_t capD, int64_t capN) {
  DynState& S = h->dyn;
  const int64_t n_rows = h->n_rows;
  const bool mixed = h->opt.precision == CTD_PREC_MIXED;
  capD = std::min<int64_t>(round8(capD), round8(n_rows));
  if (capD <= S.capD && capN <= S.capN) return CTD_OK;
  capD = std::max(capD, S.capD);
  capN = std::max(capN, S.capN);
  HIP_CHECK(h, hipStreamSynchronize(h->stream));
  DynState N = S;
  N.capD = capD;
  N.capN = capN;
  N.rows = n_rows;
  N.mixed = mixed;
  auto alloc = [&](void** p, size_t bytes) -> bool {
    if (dev_alloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return true;
  };
  bool ok = true;
  ok = ok && alloc((void**)&N.Rs, n_rows * capD * 8);
  ok = ok && alloc((void**)&N.Q, n_rows * capD * 8);
  if (mixed) ok = ok && alloc((void**)&N.Qf, n_rows * capD * 4);
  ok = ok && alloc((void**)&N.Xt, capD * capD * 8);
  N.C = nullptr;
  N.Cf = nullptr;
  if (mixed)
    ok = ok && alloc((void**)&N.Cf, (size_t)capD * capN * 4);
  else
    ok = ok && alloc((void**)&N.C, (size_t)capD * capN * 8);
  ok = ok && alloc((void**)&N.acc_fid, capD * 8);
  ok = ok && alloc((void**)&N.col_fid, capN * 8);
  if (!S.lev) ok = ok && alloc((void**)&N.lev, n_rows * 8);
  if (!ok) {
    (void)hipFree(N.Rs);
    (void)hipFree(N.Q);
    if (mixed) (void)hipFree(N.Qf);
    (void)hipFree(N.Xt);
    if (N.C) (void)hipFree(N.C);
    if (N.Cf) (void)hipFree(N.Cf);
    (void)hipFree(N.acc_fid);
    (void)hipFree(N.col_fid);
    if (!S.lev) (void)hipFree(N.lev);
    return fail(h, CTD_ERR_OOM, "CTD-D state allocation failed");
  }
  if (S.capD && (S.d_tilde > 0 || S.n_cols > 0)) {
    const int64_t dr = S.d_tilde, nc = S.n_cols;
    HIP_CHECK(h, hipMemcpy2DAsync(N.Rs, capD * 8, S.Rs, S.capD * 8, dr * 8, n_rows,
                                  hipMemcpyDeviceToDevice, h->stream));
    HIP_CHECK(h, hipMemcpy2DAsync(N.Q, capD * 8, S.Q, S.capD * 8, dr * 8, n_rows,
                                  hipMemcpyDeviceToDevice, h->stream));
    if (mixed)
      HIP_CHECK(h, hipMemcpy2DAsync(N.Qf, capD * 4, S.Qf, S.capD * 4, dr * 4, n_rows,
                                    hipMemcpyDeviceToDevice, h->stream));
    HIP_CHECK(h, hipMemcpy2DAsync(N.Xt, capD * 8, S.Xt, S.capD * 8, dr * 8, dr,
                                  hipMemcpyDeviceToDevice, h->stream));
    if (nc > 0 && !mixed)
      HIP_CHECK(h, hipMemcpy2DAsync(N.C, capD * 8, S.C, S.capD * 8, dr * 8, nc,
                                    hipMemcpyDeviceToDevice, h->stream));
    if (nc > 0 && mixed)
      HIP_CHECK(h, hipMemcpy2DAsync(N.Cf, capD * 4, S.Cf, S.capD * 4, dr * 4, nc,
                                    hipMemcpyDeviceToDevice, h->stream));
    HIP_CHECK(h, hipMemcpyAsync(N.acc_fid, S.acc_fid, dr * 8, hipMemcpyDeviceToDevice, h->stream));
    if (nc > 0)
      HIP_CHECK(h, hipMemcpyAsync(N.col_fid, S.col_fid, nc * 8, hipMemcpyDeviceToDevice, h->stream));
  }
  if (S.capD) {
    HIP_CHECK(h, hipStreamSynchronize(h->stream));
    (void)hipFree(S.Rs);
    (void)hipFree(S.Q);
    if (S.Qf) (void)hipFree(S.Qf);
    (void)hipFree(S.Xt);
    if (S.C) (void)hipFree(S.C);
    if (S.Cf) (void)hipFree(S.Cf);
    (void)hipFree(S.acc_fid);
    (void)hipFree(S.col_fid);
  }
  S = N;
  return CTD_OK;
}

// The handle's cross stream and its fork and join events, created at first
// use (default priority); false if they cannot be created.
bool cross_stream(ctd_handle* h) {
  if (!h->xstream && hipStreamCreateWithFlags(&h->xstream, hipStreamNonBlocking) != hipSuccess) {
    h->xstream = nullptr;
    (void)hipGetLastError();
    return false;
  }
  if (!h->xfork && hipEventCreateWithFlags(&h->xfork, hipEventDisableTiming) != hipSuccess) {
    h->xfork = nullptr;
    (void)hipGetLastError();
    return false;
  }
  if (!h->xjoin && hipEventCreateWithFlags(&h->xjoin, hipEventDisableTiming) != hipSuccess) {
    h->xjoin = nullptr;
    (void)hipGetLastError();
    return false;
  }
  return true;
}

ctd_status dyn_sync_sizes(ctd_handle* h) {
  DevScalars sc{};
  HIP_CHECK(h, hipStreamSynchronize(h->stream));
  HIP_CHECK(h, hipMemcpy(&sc, h->d_sc, sizeof(sc), hipMemcpyDeviceToHost));
  if (sc.status != 0) return fail(h, (ctd_status)sc.status, "device reported an error");
  h->dyn.d_tilde = sc.n_accept_total;
  h->dyn.n_cols = sc.n_cols_total;
  h->dyn.d_ub = sc.n_accept_total;
  h->dyn.n_cols_ub = sc.n_cols_total;
  return CTD_OK;
}

}  // namespace

ctd_status dyn_resize(ctd_handle* h, int64_t capD, int64_t capN) { return dyn_reserve(h, capD, capN); }

void launch_reset_scalars(hipStream_t st, DevScalars* sc, bool keep_stream) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, st, sc, keep_stream);
}

void launch_static_totals(hipStream_t st, DevScalars* sc) {
  hipLaunchKernelGGL(k_static_totals, dim3(1), dim3(1), 0, st, sc);
}

// C = R_S^T X_(alpha) for CTD-S (column-major, ld = b.ld).
void launch_core_static(hipStream_t st, StaticBufs& b, int64_t n_rows, int64_t nnz_max,
                        DevScalars* sc) {
  (void)n_rows;
  launch_cols<double>(st, b, nnz_max, sc, b.Rs, b.ld, &sc->s_tilde, b.ld, b.C, b.ld, nullptr);
}

ctd_status dyn_begin(ctd_handle* h, const ctd_coo* X) {
  const FiberLayout& lay = h->layout;
  if (lay.mode == lay.order - 1) return CTD_OK;  // no time mode left for CTD-D
  StaticBufs& b = h->sb;
  DevScalars sc{};
  HIP_CHECK(h, hipStreamSynchronize(h->stream));
  HIP_CHECK(h, hipMemcpy(&sc, h->d_sc, sizeof(sc), hipMemcpyDeviceToHost));
  if (sc.status != 0) return fail(h, (ctd_status)sc.status, "device reported an error");
  const int64_t st = sc.s_tilde, nf = sc.n_f;
  DynState& S = h->dyn;
  // a new stream: the buffers of an earlier stream on this handle are reused
  // when they fit (same I_alpha and precision, enough capacity); nothing is
  // copied from them
  const bool mixed_now = h->opt.precision == CTD_PREC_MIXED;
  if (S.capD && (S.rows != h->n_rows || S.mixed != mixed_now)) {
    HIP_CHECK(h, hipStreamSynchronize(h->stream));
    dyn_free(h);
  }
  S.d_tilde = S.d_ub = 0;
  S.n_cols = S.n_cols_ub = 0;
  S.T = 0;
  const int64_t capD = std::max<int64_t>(2 * h->s + 256, st + 64);
  const int64_t capN = 2 * nf + (1 << 16);
  ctd_status rc = dyn_reserve(h, capD, capN);
  if (rc != CTD_OK) return rc;
  const bool mixed = h->opt.precision == CTD_PREC_MIXED;
  const int64_t n_rows = h->n_rows;
  HIP_CHECK(h, hipMemcpy2DAsync(S.Rs, S.capD * 8, b.Rs, b.ld * 8, st * 8, n_rows,
                                hipMemcpyDeviceToDevice, h->stream));
  HIP_CHECK(h, hipMemcpy2DAsync(S.Q, S.capD * 8, b.Q, b.ld * 8, st * 8, n_rows,
                                hipMemcpyDeviceToDevice, h->stream));
  if (mixed)
    HIP_CHECK(h, hipMemcpy2DAsync(S.Qf, S.capD * 4, b.Qf, b.ld * 4, st * 4, n_rows,
                                  hipMemcpyDeviceToDevice, h->stream));
  HIP_CHECK(h, hipMemcpy2DAsync(S.Xt, S.capD * 8, b.M, b.ld * 8, st * 8, st,
                                hipMemcpyDeviceToDevice, h->stream));
  if (mixed)
    hipLaunchKernelGGL(k_cols_to_f32, dim3(grid_for(st * nf)), dim3(kBlock), 0, h->stream, b.C,
                       b.ld, S.Cf, S.capD, st, nf);
  else
    HIP_CHECK(h, hipMemcpy2DAsync(S.C, S.capD * 8, b.C, b.ld * 8, st * 8, nf,
                                  hipMemcpyDeviceToDevice, h->stream));
  HIP_CHECK(h, hipMemcpyAsync(S.lev, b.lev, n_rows * 8, hipMemcpyDeviceToDevice, h->stream));
  HIP_CHECK(h, hipMemcpyAsync(S.acc_fid, b.acc_fid, st * 8, hipMemcpyDeviceToDevice, h->stream));
  HIP_CHECK(h, hipMemcpyAsync(S.col_fid, b.fid, nf * 8, hipMemcpyDeviceToDevice, h->stream));
  S.d_tilde = S.d_ub = st;
  S.n_cols = S.n_cols_ub = nf;
  S.T = lay.dims[lay.order - 1];
  int64_t dN = 1;
  for (int m = 0; m < lay.order - 1; ++m)
    if (m != lay.mode) dN *= lay.dims[m];
  S.dN = dN;
  h->dyn_ready = true;
  (void)X;
  return CTD_OK;
}

void dyn_free(ctd_handle* h) {
  DynState& S = h->dyn;
  if (S.Rs) (void)hipFree(S.Rs);
  if (S.Q) (void)hipFree(S.Q);
  if (S.Qf) (void)hipFree(S.Qf);
  if (S.Xt) (void)hipFree(S.Xt);
  if (S.C) (void)hipFree(S.C);
  if (S.Cf) (void)hipFree(S.Cf);
  if (S.lev) (void)hipFree(S.lev);
  if (S.acc_fid) (void)hipFree(S.acc_fid);
  if (S.col_fid) (void)hipFree(S.col_fid);
  if (S.ws) (void)hipFree(S.ws);
  S = DynState{};
  h->dyn_ready = false;
}

// Whether the CTD-D C is held in float32 (mixed-precision handle).
static bool mixed_c(const DynState& S) { return S.Cf != nullptr; }

void fill_result(ctd_handle* h, const DevScalars& sc, ctd_result* out) {
  const StaticBufs& b = h->sb;
  if (h->opt.profile) {
    auto span = [&](int a, int c) -> float {
      float ms = 0.f;
      if (h->ev_used[a] && h->ev_used[c]) (void)hipEventElapsedTime(&ms, h->ev[a], h->ev[c]);
      return ms;
    };
    out->stage_ms[CTD_STAGE_SORT] = span(MARK_START, MARK_SORTED);
    out->stage_ms[CTD_STAGE_SAMPLE] = span(MARK_SORTED, MARK_SAMPLED);
    out->stage_ms[CTD_STAGE_PANEL] = span(MARK_SAMPLED, MARK_PANEL);
    out->stage_ms[CTD_STAGE_BASIS] = span(MARK_PANEL, MARK_BASIS);
    out->stage_ms[CTD_STAGE_PROJECT] = span(MARK_PROJ0, MARK_PROJECTED);
    out->stage_ms[CTD_STAGE_SPMM] = span(MARK_SPMM0, MARK_SPMM1);
    out->stage_ms[CTD_STAGE_CORE] =
        h->last_was_update ? span(MARK_CROSS0, MARK_CORE) : span(MARK_PROJECTED, MARK_CORE);
    out->stage_ms[CTD_STAGE_TOTAL] = span(MARK_START, MARK_END);
  }
  out->s = h->s;
  out->s_unique = sc.s_unique;
  out->n_f = sc.n_f;
  out->n_rows = h->n_rows;
  out->step = h->step;
  out->weight_total = sc.W;
  out->norm2 = sc.total_norm2;
  out->err2 = sc.total_err2;
  out->rel_err = sc.total_norm2 > 0 ? sc.total_err2 / sc.total_norm2 : 0.0;
  out->slice_err2 = sc.err2;
  out->status = sc.status;
  out->draws = b.draw_fid;
  out->unique = b.uniq_fid;
  out->counts = b.counts;
  out->prob = b.prob;
  out->scale = b.scale;
  out->fiber_ids = b.fid;
  out->fiber_resid = h->opt.want_fiber_stats ? b.resid : nullptr;
  if (h->last_was_update && h->dyn_ready) {
    const DynState& S = h->dyn;
    out->s_tilde = sc.n_accept_total;
    out->accepted = S.acc_fid;
    out->Q = S.Q;
    out->ldq = S.capD;
    out->Linv_t = S.Xt;
    out->ldx = S.capD;
    out->R = S.Rs;
    out->ldr = S.capD;
    out->C = mixed_c(S) ? (const void*)S.Cf : (const void*)S.C;
    out->C_dtype = mixed_c(S) ? CTD_F32 : CTD_F64;
    out->ldc = S.capD;
    out->n_cols = sc.n_cols_total;
    out->col_ids = S.col_fid;
  } else {
    out->s_tilde = sc.s_tilde;
    out->accepted = b.acc_fid;
    out->Q = b.Q;
    out->ldq = b.ld;
    out->Linv_t = b.M;
    out->ldx = b.ld;
    out->R = b.Rs;
    out->ldr = b.ld;
    out->C = h->opt.want_C ? b.C : nullptr;
    out->C_dtype = CTD_F64;
    out->ldc = b.ld;
    out->n_cols = sc.n_f;
    out->col_ids = b.fid;
  }
}

}  // namespace ctd

using namespace ctd;

extern "C" ctd_status ctd_update_batched(ctd_handle* h, const ctd_coo* slices, int32_t B,
                                         int64_t d) {
  if (!h) return CTD_ERR_INVALID_ARG;
  h->last_error.clear();
  (void)hipGetLastError();
  if (h->failed) return fail(h, CTD_ERR_STATE, "handle is in a failed state; call ctd_decompose");
  if (!h->dyn_ready)
    return fail(h, CTD_ERR_STATE, "ctd_update needs a prior ctd_decompose with want_C on a non-time mode");
  if (B < 1 || B > CTD_MAX_BATCH || !slices)
    return fail(h, CTD_ERR_INVALID_ARG, "B must be in [1, CTD_MAX_BATCH]");
  const FiberLayout& full = h->layout;
  std::vector<FiberLayout> lays(B);
  int64_t nnz_max = 0, nnz_sum = 0;
  for (int b = 0; b < B; ++b) {
    const ctd_coo* slice = &slices[b];
    if (slice->order != full.order) return fail(h, CTD_ERR_STATE, "slice order differs from the stream's");
    for (int m = 0; m < full.order - 1; ++m)
      if (slice->dims[m] != full.dims[m]) return fail(h, CTD_ERR_STATE, "slice dims differ from the stream's");
    if (slice->dims[full.order - 1] != 1) return fail(h, CTD_ERR_STATE, "slice time dim must be 1");
    uint64_t ncols = 0;
    ctd_status rc = check_coo(h, slice, full.mode, &lays[b], &ncols);
    if (rc != CTD_OK) return rc;
    if (d < 1 || (uint64_t)d > ncols) return fail(h, CTD_ERR_INVALID_ARG, "d must be in [1, dN_alpha]");
    nnz_max = std::max<int64_t>(nnz_max, slice->nnz);
    nnz_sum += slice->nnz;
  }
  if (d > CTD_MAX_DRAWS) return fail(h, CTD_ERR_CAPACITY, "d above CTD_MAX_DRAWS");
  ctd_status rc = CTD_OK;
  hipStream_t st = h->stream;
  DynState& S = h->dyn;
  const int64_t n_rows = h->n_rows;
  const bool mixed = h->opt.precision == CTD_PREC_MIXED;
  DevScalars* sc = h->d_sc;
  // capacities (host upper bounds; exact sizes only at a sync)
  const int64_t need_d = std::min<int64_t>(n_rows, S.d_ub + (int64_t)B * d);
  const int64_t need_n = S.n_cols_ub + nnz_sum;
  if (need_d > S.capD || need_n > S.capN) {
    rc = dyn_sync_sizes(h);
    if (rc != CTD_OK) return rc;
    const int64_t nd = std::min<int64_t>(n_rows, S.d_tilde + (int64_t)B * d);
    const int64_t nn = S.n_cols + nnz_sum;
    if (nd > S.capD || nn > S.capN) {
      rc = dyn_reserve(h, nd > S.capD ? std::max(nd, 2 * S.capD) : S.capD,
                       nn > S.capN ? std::max(nn, 2 * S.capN) : S.capN);
      if (rc != CTD_OK) return rc;
    }
  }
  StaticBufs& b = h->sb;
  rc = plan_static(h, nnz_max, d, n_rows, mixed, false, false, S.capD, &b);
  if (rc != CTD_OK) return rc;
  // workspace: block-filter scratch, W rows of the batch's kept fibers, cross
  // rows, slice records and pass ranges
  const int64_t kept_max = std::min<int64_t>(n_rows, (int64_t)B * d);
  const size_t ws_doubles = basis_scratch_doubles(n_rows, S.capD, 2) +
                            (size_t)(1 + B) * kept_max * S.capD + (size_t)2 * (B + 1) +
                            (size_t)5 * B + 64;
  if (ws_doubles * 8 > S.ws_bytes) {
    if (S.ws) {
      HIP_CHECK(h, hipStreamSynchronize(st));
      (void)hipFree(S.ws);
      S.ws = nullptr;
    }
    if (dev_alloc(&S.ws, ws_doubles * 8) != hipSuccess) {
      (void)hipGetLastError();
      S.ws_bytes = 0;
      return fail(h, CTD_ERR_OOM, "CTD-D workspace allocation failed");
    }
    S.ws_bytes = ws_doubles * 8;
  }
  double* scratch = (double*)S.ws;
  double* Wacc = scratch + basis_scratch_doubles(n_rows, S.capD, 2);
  double* Y = Wacc + (size_t)kept_max * S.capD;
  int64_t* info = (int64_t*)(Y + (size_t)B * kept_max * S.capD);   // Y: one block per pass
  int64_t* rng = info + 2 * (B + 1);

  for (bool& u : h->ev_used) u = false;
  // C rows of the batch's kept fibers (Eq. 13): pass 0 over the columns held
  // before the batch, pass b + 1 over the columns of slice b
  auto cross_stage = [&](hipStream_t cs) {
    mark_on(h, MARK_CROSS0, cs);
    {
      // columns of the widest pass: those held before the batch, or a slice's
      int64_t cols_max = S.n_cols_ub;
      for (int p = 1; p < B; ++p) cols_max = std::max<int64_t>(cols_max, slices[p - 1].nnz);
      auto tiles_of = [&](int cols) { return (cols_max + cols - 1) / cols; };
      const int64_t ystride = kept_max * S.capD;
      hipLaunchKernelGGL(k_cross_setup, dim3(1), dim3(CTD_MAX_BATCH), 0, cs, info, B, sc, rng);
      hipLaunchKernelGGL(k_cross_rows, dim3(grid_for(S.capD * kWave), B), dim3(kBlock), 0, cs, S.Xt,
                         S.capD, Wacc, S.capD, Y, S.capD, ystride, rng);
      if (cols_max > 0 && kept_max > 16) {
        if (S.Cf)
          hipLaunchKernelGGL((k_cross_term_bf3<4, 1>), dim3(tiles_of(kCrossCols), B), dim3(kCrossCols),
                             0, cs, S.Cf, S.capD, Y, S.capD, ystride, rng);
        else
          hipLaunchKernelGGL((k_cross_term<4, 4, 2>), dim3(tiles_of(128), B), dim3(kCrossCols), 0, cs,
                             S.C, S.capD, Y, S.capD, ystride, rng);
      } else if (cols_max > 0) {
        // at most 16 new rows: waves per workgroup (2, 4 or 8) chosen by the
        // autotuner per bucket of the column count (every choice writes the same
        // values; a measuring call runs all three, each reading rows < d only)
        constexpr int kNCand = 3;
        const int prec = S.Cf ? 1 : 0, bucket = tune_bucket(cols_max);
        int choice = tune_get(cs, TUNE_CROSS_NW, prec, bucket, kNCand);
        std::vector<hipEvent_t> tev;
        const bool measure = choice < 0 && tune_begin(cs, TUNE_CROSS_NW, prec, bucket, kNCand, &tev);
        if (choice < 0) choice = 1;
        auto cross = [&](int c) {
          const int nw = 2 << c;
          const dim3 grid((unsigned)tiles_of(64 * nw), B);
          if (S.Cf) {
            if (nw == 2)
              hipLaunchKernelGGL((k_cross_term32<1, 2>), grid, dim3(128), 0, cs, S.Cf, S.capD, Y, S.capD,
                                 ystride, rng);
            else if (nw == 4)
              hipLaunchKernelGGL((k_cross_term32<1, 4>), grid, dim3(256), 0, cs, S.Cf, S.capD, Y, S.capD,
                                 ystride, rng);
            else
              hipLaunchKernelGGL((k_cross_term32<1, 8>), grid, dim3(512), 0, cs, S.Cf, S.capD, Y, S.capD,
                                 ystride, rng);
          } else {
            if (nw == 2)
              hipLaunchKernelGGL((k_cross_term_direct<2>), grid, dim3(128), 0, cs, S.C, S.capD, Y, S.capD,
                                 ystride, rng);
            else if (nw == 4)
              hipLaunchKernelGGL((k_cross_term_direct<4>), grid, dim3(256), 0, cs, S.C, S.capD, Y, S.capD,
                                 ystride, rng);
            else
              hipLaunchKernelGGL((k_cross_term_direct<8>), grid, dim3(512), 0, cs, S.C, S.capD, Y, S.capD,
                                 ystride, rng);
          }
        };
        if (measure) {
          for (int c = 0; c < kNCand; ++c) {
            (void)hipEventRecord(tev[2 * c], cs);
            cross(c);
            (void)hipEventRecord(tev[2 * c + 1], cs);
          }
          tune_recorded(TUNE_CROSS_NW, prec, bucket);
        } else {
          cross(choice);
        }
      }
    }
    mark_on(h, MARK_CORE, cs);
  };
  // A one-slice update's cross term needs only the rank after the slice's
  // filter: it runs on the handle's cross stream beside the slice's own
  // columns and residual (which write other parts of C and read neither Y
  // nor the ranges), and the handle's stream waits for it before the call
  // ends.
  const bool early_cross = B == 1 && cross_stream(h);
  bool cross_forked = false;
  mark(h, MARK_START);
  int64_t d_ub = S.d_ub;
  for (int bi = 0; bi < B; ++bi) {
    const ctd_coo* slice = &slices[bi];
    const int64_t nnz = slice->nnz;
    const uint32_t step = (uint32_t)(h->step + 1 + bi);
    launch_reset_scalars(st, sc, true);
    if (bi == 0) hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(1), 0, st, sc);
    hipLaunchKernelGGL(k_batch_mark, dim3(1), dim3(1), 0, st, sc, info, bi);
    const uint64_t t_off = (uint64_t)(S.T + bi) * (uint64_t)S.dN;
    const int64_t d_next = std::min<int64_t>(n_rows, d_ub + d);
    if (nnz > 0) {
      rc = enqueue_input(h, slice, lays[bi], d, h->seed, step, nullptr, b, 0u);
      if (rc != CTD_OK) return rc;
      // candidates against R^(t) and each other; kept ones extend R, Q, M
      launch_panel(st, b.uniq_fi, d, b.fptr, b.row, b.val, n_rows, b.P, b.ld, sc);
      mark(h, MARK_PANEL);
      BasisArgs ba{};
      ba.P = b.P;
      ba.ldp = b.ld;
      ba.n_rows = n_rows;
      ba.s_max = d;
      ba.k0_max = d_ub;
      ba.uniq_fi = b.uniq_fi;
      ba.uniq_fid = b.uniq_fid;
      ba.fptr = b.fptr;
      ba.row = b.row;
      ba.val = b.val;
      ba.Q = S.Q;
      ba.ldq = S.capD;
      ba.Qf = mixed ? S.Qf : nullptr;
      ba.R = S.Rs;
      ba.ldr = S.capD;
      ba.M = S.Xt;
      ba.ldm = S.capD;
      ba.lev = S.lev;
      ba.lev_accumulate = true;
      ba.eps2 = h->opt.eps * h->opt.eps;
      ba.accept = b.accept;
      ba.acc_fid = S.acc_fid;
      ba.acc_fi_local = nullptr;
      ba.fiber_mark = b.fiber_mark;
      ba.id_offset = t_off;
      ba.Wacc = Wacc;
      ba.ldwa = S.capD;
      ba.scratch = scratch;
      ba.cap = S.capD;
      ba.w2_sets = 2;
      rc = ensure_bdev(h, 1);
      if (rc != CTD_OK) return rc;
      launch_basis(st, &ba, &sc, 1, h->bdev, basis_side(h));
      mark(h, MARK_BASIS);
      if (early_cross) {
        hipLaunchKernelGGL(k_batch_mark, dim3(1), dim3(1), 0, st, sc, info, 1);
        HIP_CHECK(h, hipEventRecord(h->xfork, st));
        HIP_CHECK(h, hipStreamWaitEvent(h->xstream, h->xfork, 0));
        cross_stage(h->xstream);
        HIP_CHECK(h, hipEventRecord(h->xjoin, h->xstream));
        cross_forked = true;
      }
      // the slice's own columns R^(t+1)T dX (rows held after its filter)
      if (mixed)
        launch_cols<float>(st, b, nnz, sc, S.Rs, S.capD, &sc->n_accept_total, d_next, S.Cf, S.capD,
                           &sc->n_cols_total);
      else
        launch_cols<double>(st, b, nnz, sc, S.Rs, S.capD, &sc->n_accept_total, d_next, S.C,
                            S.capD, &sc->n_cols_total);
      hipLaunchKernelGGL(k_append_ids, dim3(grid_for(nnz)), dim3(kBlock), 0, st, b.fid, &sc->n_f,
                         S.col_fid, nullptr, &sc->n_cols_total, t_off);
      // slice residual against the grown basis
      ProjectArgs pa = project_args(h, b, S.Q, S.Qf, S.capD, S.lev, &sc->n_accept_total, d_next,
                                    S.rows);
      if (h->opt.profile) {
        mark(h, MARK_PROJ0);
        mark(h, MARK_SPMM0);
        mark(h, MARK_SPMM1);
      }
      launch_project(st, pa, nnz, sc, h->opt.profile ? h->ev[MARK_SPMM0] : nullptr,
                     h->opt.profile ? h->ev[MARK_SPMM1] : nullptr);
      mark(h, MARK_PROJECTED);
    }
    hipLaunchKernelGGL(k_finish_slice, dim3(1), dim3(1), 0, st, sc);
    d_ub = d_next;
  }
  if (cross_forked) {
    HIP_CHECK(h, hipStreamWaitEvent(st, h->xjoin, 0));
  } else {
    hipLaunchKernelGGL(k_batch_mark, dim3(1), dim3(1), 0, st, sc, info, B);
    cross_stage(st);
  }
  mark(h, MARK_END);
  HIP_CHECK(h, hipGetLastError());
  h->s = d;
  h->step += B;
  h->last_was_update = true;
  S.T += B;
  S.d_ub = d_ub;
  S.n_cols_ub += nnz_sum;
  h->nnz_seen += nnz_sum;
  return CTD_OK;
}

extern "C" ctd_status ctd_update(ctd_handle* h, const ctd_coo* slice, int64_t d) {
  if (!h) return CTD_ERR_INVALID_ARG;
  if (!slice) return fail(h, CTD_ERR_STATE, "null slice");
  return ctd_update_batched(h, slice, 1, d);
}

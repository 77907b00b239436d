// Independence filter and orthonormal basis, block by block (the
// independence loops of Algorithms 1 and 2).
//
// Candidates are visited in order in blocks of 64.  For a block B, with the
// fibers kept so far spanned by the orthonormal columns of Q (k of them):
//   W = Q^T X_B                       sparse: the fibers' rows of Q
//   Y = X_B - Q W^T,  W2 = Q^T Y,
//   Y <- Y - Q W2^T,  W <- W + W2     block Gram-Schmidt applied twice, so Y
//                                     is orthogonal to Q to working accuracy
//   G = Y^T Y in double-double        its Schur complements are the squared
//                                     residual norms ||res||^2 of the test
//   Cholesky of G in candidate order (double-double), dropping a candidate
//   whose pivot is <= eps^2 ||x||^2 (the skip rule), with L^{-1} formed in
//   place.
// The kept residuals Y_A become the next columns of Q as Y_A L^{-T}, followed
// by a second Cholesky-QR pass when the first leaves them non-orthonormal.
// With Q = R M (M upper triangular, so U = (R^T R)^{-1} = M M^T) the new
// columns of M are M[:k, new] = -M W_A^T T and M[new, new] = T, T being the
// product of the inverse transposed Cholesky factors.  Sizes are read on the
// device, so one block is a fixed sequence of launches.
//
// For few inputs the projection of block b + 1 runs on a second stream, in
// two panels: both passes against the columns final once block b - 1 has
// finished (while block b decides), then both passes against block b's new
// columns (as soon as they are final, while M and the book-keeping finish).
// Each panel is Gram-Schmidt applied twice against an orthonormal set, so the
// residual ends orthogonal to both panels to working accuracy, as with the
// two passes over all columns at once (the second panel's coefficients
// Q_new^T Y equal Q_new^T x to working accuracy and are exactly what is
// subtracted).  Consecutive blocks use two sets of W, g and Y.
#include <algorithm>
#include <vector>

#include "kernels.h"

namespace ctd {

namespace {
constexpr int kB = 64;        // candidates per block
constexpr int kTakeParts = 256;   // workgroups of k_blk_take: partial Grams of the new columns
constexpr int kBlock = 256;
constexpr int kSplitWMax = 128; // row splits of W2 = Q^T Y (at most)
constexpr int kW2Grid = 512;    // workgroups aimed at for W2 = Q^T Y (two per CU)
constexpr int kFewInputs = 4;   // inputs per launch up to which single-input tunings apply
constexpr int kSplitDD = 256;   // row splits of the double-double Gram (at most)


// One input's arguments and scratch, in device memory: every kernel below
// serves a set of independent inputs at once, input blockIdx.z reading entry
// blockIdx.z of the array, so a block step of many inputs is one sequence of
// launches.  Grids are sized for the largest input; workgroups beyond an
// input's own sizes return at once.
struct BasisDev {
  BasisArgs a;
  DevScalars* sc;
  double* W;        // 2 x 64 x cap: Q^T x rows of the candidates (even, odd steps)
  double* W2p[2];   // w2_splits x 64 x 64 T partial coefficients (even, odd steps)
  double* W2[2];    // 64 x cap second-pass coefficients (even, odd steps; one set
                    // serves both when the passes of consecutive steps never overlap)
  double* part;     // ntake x 64 x 64 partial Grams of the new columns
  double* part_hi;  // nsplit_dd x 64 x 64 partial double-double Grams
  double* part_lo;
  double* Glo;
  double* G;
  double* Tcur;
  double* Tacc;
  double* g;        // 2 x 64 squared candidate norms (even, odd steps)
  double* Ybuf;     // 2 x n_rows x 64 block residuals (even, odd steps)
  double* Zp;       // newm_splits(kmax) x kmax x 64 partials of Z = M W_A^T
  int64_t* kcut;    // 2: columns of Q the early first pass of a step covers
  int32_t* pos;     // 64 kept positions
  int32_t nsplit_dd, ntake;
  int32_t pad;
};
static_assert(sizeof(BasisDev) % 8 == 0, "BasisDev is copied as 64-bit words");


// Double-double arithmetic (a value is hi + lo with |lo| <= ulp(hi)/2): the
// error-free transforms of Knuth (two_sum) and Dekker/FMA (two_prod).  FMA
// contraction is switched off inside them: fusing a product into the sum
// that follows it would break the exactness the transforms rely on.
__device__ inline void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ inline void quick_two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  e = b - (s - a);
}
__device__ inline void two_prod(double a, double b, double& p, double& e) {
#pragma clang fp contract(off)
  p = a * b;
  e = fma(a, b, -p);
}
// (ah, al) -= (bh, bl) * (ch, cl)
__device__ inline void dd_fnma(double& ah, double& al, double bh, double bl, double ch, double cl) {
#pragma clang fp contract(off)
  double p, pe;
  two_prod(bh, ch, p, pe);
  pe = fma(bh, cl, pe);
  pe = fma(bl, ch, pe);
  double s, se;
  two_sum(ah, -p, s, se);
  se += al - pe;
  quick_two_sum(s, se, ah, al);
}
// (rh, rl) = 1 / sqrt(ah + al) for ah > 0: one Newton step in double-double
// from the double estimate r0, r = r0 + r0 (1 - a r0^2) / 2, with a r0^2
// formed exactly enough that 1 - a r0^2 is accurate to about u^2.
__device__ inline void dd_rsqrt(double ah, double al, double& rh, double& rl) {
#pragma clang fp contract(off)
  const double r0 = rsqrt(ah);
  double t, te, p, pe;
  two_prod(r0, r0, t, te);
  two_prod(ah, t, p, pe);
  pe = fma(ah, te, pe);
  pe = fma(al, t, pe);
  const double e = (1.0 - p) - pe;
  quick_two_sum(r0, r0 * e * 0.5, rh, rl);
}

// Steps alternate between two sets of the per-step buffers W, g and Ybuf, so
// that the first projection pass of step b0 + 64 can run while step b0 is
// still deciding (see launch_basis).
__device__ inline int64_t blk_par(int64_t b0) { return (b0 / kB) & 1; }
__device__ inline double* w_of(const BasisDev& d, int64_t b0) {
  return d.W + blk_par(b0) * kB * d.a.cap;
}
__device__ inline double* g_of(const BasisDev& d, int64_t b0) { return d.g + blk_par(b0) * kB; }
__device__ inline double* y_of(const BasisDev& d, int64_t b0) {
  return d.Ybuf + blk_par(b0) * kB * d.a.n_rows;
}

// Column ranges of a projection: the whole of [0, k) at once, or split into
// an early panel [0, kcut) (run ahead on a second stream against the columns
// already final) and the late panel [kcut, k) (the previous step's new
// columns, at most 64, projected out of the early residual).
enum Range : int { kAll = 0, kEarly = 1, kLate = 2 };

__device__ inline int64_t blk_count(const DevScalars* sc, int64_t b0) {
  const int64_t sp = sc->status == 0 ? sc->s_unique : 0;
  return b0 < sp ? min((int64_t)kB, sp - b0) : 0;
}
// Candidates of the block that need work: none once the kept fibers span all
// n_rows rows, since every later residual is then zero and every later
// candidate is skipped.
__device__ inline int64_t blk_work(const DevScalars* sc, int64_t b0, int64_t n_rows) {
  return sc->n_accept_total >= n_rows ? 0 : blk_count(sc, b0);
}

// The late part runs on the second stream too, as soon as the previous
// step's new columns are final, while that step still finishes: its range is
// [kcut, kcut + na) with na that step's kept count (read before the next
// decisions overwrite it), and whether the step has work follows from the
// range's end, the k the step starts with.
__device__ inline int64_t late_end(const BasisDev& d, int64_t b0) {
  return d.kcut[blk_par(b0)] + d.sc->blk_na;
}
__device__ inline int64_t late_work(const BasisDev& d, int64_t b0) {
  return late_end(d, b0) >= d.a.n_rows ? 0 : blk_count(d.sc, b0);
}
// Columns [lo, hi) of a range and the candidates of the step it serves.
struct ColRange {
  int64_t lo, hi, nb;
};
__device__ inline ColRange col_range(const BasisDev& d, int64_t b0, int range) {
  const DevScalars* sc = d.sc;
  const int64_t kc = d.kcut[blk_par(b0)];
  if (range == kEarly) return {0, kc, kc >= d.a.n_rows ? 0 : blk_count(sc, b0)};
  if (range == kLate) return {kc, late_end(d, b0), late_work(d, b0)};
  return {0, (int64_t)sc->n_accept_total, blk_work(sc, b0, d.a.n_rows)};
}

// W[j][c] = sum_e v_e Q[r_e][c] for c in the first pass's range (all of
// [0, k), or the early part [0, kcut)), and g[j] = ||x_{b0+j}||^2.
// Workgroup (chunk, j) covers columns 128 chunk .. + 128 of candidate j (two
// per lane); its eight waves take the fiber's nonzeros in interleaved groups
// of 16 (sixteen row gathers in flight per wave) and their partial rows are
// added in LDS in wave order.  Chunk 0 also forms the squared norm.
constexpr int kWWaves = 8;
constexpr int kWCols = 2 * kWave;
__global__ __launch_bounds__(kWWaves * kWave) void k_blk_w(const BasisDev* __restrict__ bd,
                                                            int64_t b0, int range) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ Q = d.a.Q;
  const int64_t ldq = d.a.ldq, ldw = d.a.cap;
  const int32_t* __restrict__ uniq_fi = d.a.uniq_fi;
  const int32_t* __restrict__ fptr = d.a.fptr;
  const int32_t* __restrict__ row = d.a.row;
  const double* __restrict__ val = d.a.val;
  double* __restrict__ W = w_of(d, b0);
  double* __restrict__ g = g_of(d, b0);
  constexpr int kU = 16;
  __shared__ double part[kWWaves][kWCols];
  __shared__ double gpart[kWWaves];
  const ColRange cr = col_range(d, b0, range);   // kAll or kEarly: lo = 0
  const int64_t nb = cr.nb, k = cr.hi;
  const int j = blockIdx.y;
  const int64_t cbase = (int64_t)blockIdx.x * kWCols;
  if (j >= nb || (blockIdx.x > 0 && cbase >= k)) return;
  const int wv = threadIdx.x / kWave, l = lane_id();
  const int64_t c = cbase + 2 * l;
  const bool active = c < k;   // ldq is even, so the 16 B load at c stays in the row
  const double* Qc = Q + (active ? c : 0);
  const int32_t f = uniq_fi[b0 + j];
  const int32_t e0 = fptr[f], e1 = fptr[f + 1];
  double a0 = 0.0, a1 = 0.0, gs = 0.0;
  for (int32_t eb = e0 + wv * kU; eb < e1; eb += kWWaves * kU) {
    const int n = min(kU, e1 - eb);
    int32_t r[kU];
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      r[u] = u < n ? row[eb + u] : 0;
      v[u] = u < n ? val[eb + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) gs += v[u] * v[u];
    if (active) {
      double2 q[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        q[u] = u < n ? *(const double2*)(Qc + (int64_t)r[u] * ldq) : make_double2(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        a0 += v[u] * q[u].x;
        a1 += v[u] * q[u].y;
      }
    }
  }
  part[wv][2 * l] = a0;
  part[wv][2 * l + 1] = a1;
  if (l == 0) gpart[wv] = gs;
  __syncthreads();
  if (wv == 0) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int w = 0; w < kWWaves; ++w) {
      s0 += part[w][2 * l];
      s1 += part[w][2 * l + 1];
    }
    if (c < k) W[(int64_t)j * ldw + c] = s0;
    if (c + 1 < k) W[(int64_t)j * ldw + c + 1] = s1;
    if (blockIdx.x == 0 && l == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWWaves; ++w) t += gpart[w];
      g[j] = t;
    }
  }
}

// Dense f64 MFMA kernels below run 512 threads as two groups of four waves
// that split the reduction dimension between them (chunks alternate), with
// the next chunk's global loads in registers while the current one is in
// MFMAs; the two partial tiles are combined through LDS at the end.
constexpr int kGemm = 512;
constexpr int kGK = 32;       // reduction chunk

// Y[r][j] = P[r][b0 + j] - sum_c Q[r][c] W[j][c] for every candidate j of
// the block (residuals against span(Q)), into Ybuf (n_rows x 64), over the
// columns of the range: all of [0, k) or the early panel [0, kcut) (kAll,
// kEarly); the late panel subtracts the rest, Ybuf[r][j] -= sum_{kcut <= c <
// k} Q[r][c] W[j][c].  With second set, the second pass over the range,
// Ybuf[r][j] -= sum_c Q[r][c] W2[j][c].  One workgroup per 32 rows; wave w of
// a group computes rows 16 (w / 2) .. + 16 and candidates 32 (w % 2) .. + 32
// with two f64 MFMA accumulators.
__global__ __launch_bounds__(kGemm) void k_blk_form_y(const BasisDev* __restrict__ bd, int64_t b0,
                                                      int range, int second) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ P = d.a.P;
  const double* __restrict__ Q = d.a.Q;
  const bool subtract = second || range == kLate;
  const double* __restrict__ W = second ? d.W2[blk_par(b0)] : w_of(d, b0);
  const int64_t ldp = d.a.ldp, n_rows = d.a.n_rows, ldq = d.a.ldq, ldw = d.a.cap;
  double* __restrict__ Ybuf = y_of(d, b0);
  constexpr int kR = 32;
  __shared__ double As[2][kR][kGK + 1];   // Q tile [row][c]
  __shared__ double Bs[2][kGK][kB + 1];   // W^T tile [c][j]
  const ColRange cr = col_range(d, b0, range);
  const int64_t nb = cr.nb;
  if (nb == 0) return;
  const int64_t klo = cr.lo, k = cr.hi;
  if (subtract && klo >= k) return;
  const int64_t r0 = (int64_t)blockIdx.x * kR;
  if (r0 >= n_rows) return;
  const int grp = threadIdx.x / kBlock, t = threadIdx.x % kBlock;
  const int w = t / kWave, l = lane_id();
  const int rb = (w / 2) * 16, cb = (w % 2) * 32;
  const int64_t nch = (k - klo + kGK - 1) / kGK;
  const int64_t iters = (nch + 1) / 2;
  double ra[kR * kGK / kBlock], rw[kB * kGK / kBlock];
  auto load = [&](int64_t ch) {
    const int64_t c0 = klo + ch * kGK;
#pragma unroll
    for (int u = 0; u < kR * kGK / kBlock; ++u) {
      const int idx = u * kBlock + t, r = idx / kGK, c = idx % kGK;
      ra[u] = (ch < nch && c0 + c < k && r0 + r < n_rows) ? Q[(r0 + r) * ldq + c0 + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kB * kGK / kBlock; ++u) {
      const int idx = u * kBlock + t, j = idx / kGK, c = idx % kGK;
      rw[u] = (ch < nch && c0 + c < k && j < nb) ? W[(int64_t)j * ldw + c0 + c] : 0.0;
    }
  };
  dbl4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  load(grp);
  for (int64_t it = 0; it < iters; ++it) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kR * kGK / kBlock; ++u) {
      const int idx = u * kBlock + t;
      As[grp][idx / kGK][idx % kGK] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < kB * kGK / kBlock; ++u) {
      const int idx = u * kBlock + t;
      Bs[grp][idx % kGK][idx / kGK] = rw[u];
    }
    __syncthreads();
    load(grp + 2 * (it + 1));
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      const double a = As[grp][rb + l % 16][ks * 4 + l / 16];
      const double b0v = Bs[grp][ks * 4 + l / 16][cb + l % 16];
      const double b1v = Bs[grp][ks * 4 + l / 16][cb + 16 + l % 16];
      acc0 = mfma16(a, b0v, acc0);
      acc1 = mfma16(a, b1v, acc1);
    }
  }
  // combine the two groups: group 1 parks its tile in LDS
  double(*red)[kB + 1] = Bs[0];   // 32 x 65 doubles
  __syncthreads();
  if (grp == 1) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[rb + l / 16 + 4 * r][cb + l % 16] = acc0[r];
      red[rb + l / 16 + 4 * r][cb + 16 + l % 16] = acc1[r];
    }
  }
  __syncthreads();
  if (grp == 1) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = rb + l / 16 + 4 * r;
    const int64_t row = r0 + rr;
    if (row >= n_rows) continue;
    const int j0 = cb + l % 16, j1 = cb + 16 + l % 16;
    const double s0 = acc0[r] + red[rr][j0], s1 = acc1[r] + red[rr][j1];
    if (subtract) {
      if (j0 < nb) Ybuf[row * kB + j0] -= s0;
      if (j1 < nb) Ybuf[row * kB + j1] -= s1;
    } else {
      Ybuf[row * kB + j0] = j0 < nb ? P[row * ldp + b0 + j0] - s0 : 0.0;
      Ybuf[row * kB + j1] = j1 < nb ? P[row * ldp + b0 + j1] - s1 : 0.0;
    }
  }
}

// Row splits of W2 = Q^T Y at a block step whose Q spans T tiles of 64
// columns, for nz inputs in the launch: at most kW2Grid workgroups in all
// (one round of two resident workgroups per CU: a second round for a few more
// costs more than the larger splits), each split at least 64 rows, at most
// kSplitWMax splits.  A step's own T is the launch's bound capped by the
// input's column capacity.
__host__ __device__ inline int w2_splits(int64_t n_rows, int64_t T, int nz) {
  int64_t by_rows = (n_rows + 63) / 64;
  if (by_rows > kSplitWMax) by_rows = kSplitWMax;
  int64_t want = kW2Grid / ((T > 0 ? T : 1) * (nz > 0 ? nz : 1));
  if (want > by_rows) want = by_rows;
  return want > 0 ? (int)want : 1;
}
// Columns an input can hold: at most its capacity and at most n_rows (kept
// fibers are linearly independent).
__host__ __device__ inline int64_t kmax_of(const BasisArgs& a) {
  return a.cap < a.n_rows ? a.cap : a.n_rows;
}
__device__ inline int64_t w2_tiles(const BasisDev& d, int64_t t_launch) {
  const int64_t tc = (kmax_of(d.a) + kB - 1) / kB;
  return t_launch < tc ? t_launch : tc;
}

// Projection coefficients Wp[j][c] = sum_r Q[r][c] Y[r][j] for the columns c
// of the range, partial over w2_splits row ranges: workgroup (ct, s) covers c
// in [lo + 64 ct, lo + 64 ct + 64) and writes W2p[s][j][c - lo] (row length
// 64 T); wave w of a group computes c rows 16 w .. + 16 against all 64 j with
// four f64 MFMA tiles.  Over all columns or the early panel these are the
// second pass's coefficients; over the late panel (the previous step's new
// columns, at most 64, T = 1) first the late panel's first-pass coefficients
// (those columns are orthogonal to the early panel, so Q_new^T Y equals
// Q_new^T x to working accuracy, and it is exactly what the late pass
// subtracts), then its second pass.
__global__ __launch_bounds__(kGemm) void k_blk_w2_part(const BasisDev* __restrict__ bd,
                                                       int64_t b0, int64_t t_launch, int range) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ Q = d.a.Q;
  const double* __restrict__ Y = y_of(d, b0);
  double* __restrict__ W2p = d.W2p[blk_par(b0)];
  const int64_t ldq = d.a.ldq, n_rows = d.a.n_rows;
  const int64_t T = range == kLate ? 1 : w2_tiles(d, t_launch), ldp = T * kB;
  const int nsplit = w2_splits(n_rows, T, gridDim.z);
  __shared__ double Qs[2][kGK][kB + 1];   // [r][c]
  __shared__ double Ys[2][kGK][kB + 1];   // [r][j]
  const ColRange cr = col_range(d, b0, range);
  const int64_t nb = cr.nb, k = cr.hi;
  const int64_t cw = cr.lo;   // first column held
  const int64_t c0 = cw + (int64_t)blockIdx.x * kB;
  if (nb == 0 || c0 >= k || (int)blockIdx.y >= nsplit) return;
  const int64_t chunk = (n_rows + nsplit - 1) / nsplit;
  const int64_t r0 = blockIdx.y * chunk, r1 = min(n_rows, r0 + chunk);
  const int grp = threadIdx.x / kBlock, t = threadIdx.x % kBlock;
  const int w = t / kWave, l = lane_id();
  const int64_t nch = (r1 - r0 + kGK - 1) / kGK;
  const int64_t iters = (nch + 1) / 2;
  double rq[kGK * kB / kBlock], ry[kGK * kB / kBlock];
  auto load = [&](int64_t ch) {
    const int64_t rr = r0 + ch * kGK;
#pragma unroll
    for (int u = 0; u < kGK * kB / kBlock; ++u) {
      const int idx = u * kBlock + t, r = idx / kB, c = idx % kB;
      const bool rin = ch < nch && rr + r < r1;
      rq[u] = (rin && c0 + c < k) ? Q[(rr + r) * ldq + c0 + c] : 0.0;
      ry[u] = (rin && c < nb) ? Y[(rr + r) * kB + c] : 0.0;
    }
  };
  dbl4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  load(grp);
  for (int64_t it = 0; it < iters; ++it) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kGK * kB / kBlock; ++u) {
      const int idx = u * kBlock + t;
      Qs[grp][idx / kB][idx % kB] = rq[u];
      Ys[grp][idx / kB][idx % kB] = ry[u];
    }
    __syncthreads();
    load(grp + 2 * (it + 1));
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      const double a = Qs[grp][ks * 4 + l / 16][w * 16 + l % 16];   // A = Q^T: A[c][r] = Q[r][c]
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = mfma16(a, Ys[grp][ks * 4 + l / 16][q * 16 + l % 16], acc[q]);
    }
  }
  double(*red)[kB + 1] = Qs[0];   // reuse Qs (2 x 32 x 65 doubles) as a 64 x 65 tile
  __syncthreads();
  if (grp == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[w * 16 + l / 16 + 4 * r][q * 16 + l % 16] = acc[q][r];
  }
  __syncthreads();
  if (grp == 1) return;
  double* p = W2p + (int64_t)blockIdx.y * kB * ldp;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cc = w * 16 + l / 16 + 4 * r;
      const int64_t c = c0 + cc;
      const int j = q * 16 + l % 16;
      if (c < k) p[(int64_t)j * ldp + c - cw] = acc[q][r] + red[cc][j];
    }
}

// s = sum_s W2p[s][j][c] (fixed order) for column lo + c of the range: with
// second set W2[j][lo + c] = s and W[j][lo + c] += s (second-pass
// coefficients), else W[j][lo + c] = s (the late panel's first pass).  A
// workgroup takes 32 consecutive entries per pass, each summed by kW2Ways
// threads over every kW2Ways-th partial (all loads in flight together), and
// the ways are added in order.
constexpr int kW2Ways = 8, kW2Per = kBlock / kW2Ways;
__global__ __launch_bounds__(kBlock) void k_blk_w2_sum(const BasisDev* __restrict__ bd,
                                                       int64_t b0, int64_t t_launch, int range,
                                                       int second) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ W2p = d.W2p[blk_par(b0)];
  double* __restrict__ W2 = d.W2[blk_par(b0)];
  double* __restrict__ W = w_of(d, b0);
  const int64_t ldw = d.a.cap;
  const int64_t T = range == kLate ? 1 : w2_tiles(d, t_launch), ldp = T * kB;
  const int nsplit = w2_splits(d.a.n_rows, T, gridDim.z);
  const ColRange cr = col_range(d, b0, range);
  const int64_t nb = cr.nb;
  const int64_t cw = cr.lo;          // first column
  const int64_t k = cr.hi - cw;      // columns
  const int64_t total = k > 0 ? nb * k : 0;
  __shared__ double sh[kBlock];
  const int e = threadIdx.x % kW2Per, q = threadIdx.x / kW2Per;
  constexpr int kIt = kSplitWMax / kW2Ways;
  for (int64_t t0 = (int64_t)blockIdx.x * kW2Per; t0 < total; t0 += (int64_t)gridDim.x * kW2Per) {
    const int64_t t = t0 + e;
    const int64_t j = t / k, c = t % k;
    double s = 0.0;
    if (t < total) {
      double v[kIt];
#pragma unroll
      for (int u = 0; u < kIt; ++u) {
        const int p = q + u * kW2Ways;
        v[u] = p < nsplit ? W2p[((int64_t)p * kB + j) * ldp + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kIt; ++u) s += v[u];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    if (q == 0 && t < total) {
      for (int w = 1; w < kW2Ways; ++w) s += sh[w * kW2Per + e];
      if (second) {
        W2[j * ldw + cw + c] = s;
        W[j * ldw + cw + c] += s;
      } else {
        W[j * ldw + cw + c] = s;
      }
    }
    __syncthreads();
  }
}

// Double-double Gram of the block buffer, partial over kSplitDD row ranges:
// (hi, lo)[s][i][j] = sum_{r in range s} Y[r][i] Y[r][j], each product split
// exactly by an FMA and accumulated with two_sum.  The independence decisions
// need the block Gram to about u^2: rounding it to float64 alone moves the
// Schur complement of an exactly dependent candidate to ~u * cond^2 ||x||^2,
// which can reach eps^2 ||x||^2.
// NG groups of kBlock threads take every NG-th row of each 64-row tile and
// their sums are added in group order: four groups (four waves per SIMD) when
// few inputs share the launch and nothing runs beside it; one when many inputs
// fill the GPU by themselves, or when the side streams' projection GEMMs hold
// CUs (a 256-thread workgroup with 33 KB of LDS fits beside one of theirs, a
// 1024-thread one with 66 KB waits for CUs to drain: 11.48 -> 11.25 ms per
// decomposition of the 5M-nonzero tensor).
template <int NG>
__global__ __launch_bounds__(kBlock * NG) void k_blk_gram_dd(const BasisDev* __restrict__ bd,
                                                             int64_t b0) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ Y = y_of(d, b0);
  double* __restrict__ part_hi = d.part_hi;
  double* __restrict__ part_lo = d.part_lo;
  const int64_t n_rows = d.a.n_rows;
  const int nsplit = d.nsplit_dd;
  const DevScalars* sc = d.sc;
  __shared__ double Ys[kB][kB + 1];   // [row][col]
  const int64_t width = blk_work(sc, b0, n_rows);
  if (width == 0 || (int)blockIdx.x >= nsplit) return;
  const int64_t chunk = (n_rows + nsplit - 1) / nsplit;
  const int64_t k0 = blockIdx.x * chunk;
  const int64_t k1 = min(n_rows, k0 + chunk);
  const int grp = threadIdx.x / kBlock, tl = threadIdx.x % kBlock;
  const int ty = tl / 16, tx = tl % 16;
  double hi[4][4] = {}, lo[4][4] = {};
  for (int64_t kk0 = k0; kk0 < k1; kk0 += kB) {
    __syncthreads();
    constexpr int kLd = kB * kB / (kBlock * NG);
    double v[kLd];
#pragma unroll
    for (int u = 0; u < kLd; ++u) {
      const int t = u * kBlock * NG + threadIdx.x, kk = t / kB, i = t % kB;
      v[u] = (kk0 + kk < k1 && i < width) ? Y[(kk0 + kk) * kB + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLd; ++u) {
      const int t = u * kBlock * NG + threadIdx.x;
      Ys[t / kB][t % kB] = v[u];
    }
    __syncthreads();
    const int kn = (int)min((int64_t)kB, k1 - kk0);
    for (int kk = grp; kk < kn; kk += NG) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = Ys[kk][ty * 4 + u];
        y[u] = Ys[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double p, pe, s2, se;
          two_prod(x[u], y[v], p, pe);
          two_sum(hi[u][v], p, s2, se);
          hi[u][v] = s2;
          lo[u][v] += se + pe;
        }
    }
  }
  // groups 1, 2, 3 in turn park their sums in LDS and group 0 adds them
  double(*Yl)[kB + 1] = Ys;   // hi parked in Ys, lo in Yl2
  __shared__ double Yl2[kB][kB + 1];
  for (int g = 1; g < NG; ++g) {
    __syncthreads();
    if (grp == g) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Yl[ty * 4 + u][tx * 4 + v] = hi[u][v];
          Yl2[ty * 4 + u][tx * 4 + v] = lo[u][v];
        }
    }
    __syncthreads();
    if (grp == 0) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double s2, se;
          two_sum(hi[u][v], Yl[ty * 4 + u][tx * 4 + v], s2, se);
          hi[u][v] = s2;
          lo[u][v] += se + Yl2[ty * 4 + u][tx * 4 + v];
        }
    }
  }
  if (grp != 0) return;
  const int64_t off = (int64_t)blockIdx.x * kB * kB;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int t = (ty * 4 + u) * kB + tx * 4 + v;
      double h, l;
      quick_two_sum(hi[u][v], lo[u][v], h, l);
      part_hi[off + t] = h;
      part_lo[off + t] = l;
    }
}

// G = sum over the kSplitDD partial Grams in double-double: a workgroup takes
// kBlock / kSumWays consecutive elements, kSumWays threads per element each
// summing every kSumWays-th partial (neighbouring lanes read neighbouring
// elements), and the kSumWays sums are added in a fixed order.
constexpr int kSumWays = 16;
__global__ __launch_bounds__(kBlock) void k_blk_sum_dd(const BasisDev* __restrict__ bd,
                                                       int64_t b0) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ part_hi = d.part_hi;
  const double* __restrict__ part_lo = d.part_lo;
  double* __restrict__ G_hi = d.G;
  double* __restrict__ G_lo = d.Glo;
  const int nsplit = d.nsplit_dd;
  const DevScalars* sc = d.sc;
  __shared__ double sh[kBlock], sl[kBlock];
  if (blk_work(sc, b0, d.a.n_rows) == 0) return;
  constexpr int kPer = kBlock / kSumWays;
  const int e = threadIdx.x % kPer, q = threadIdx.x / kPer;
  const int t = blockIdx.x * kPer + e;
  double h = 0.0, l = 0.0;
  if (t < kB * kB) {
    // loads first (all in flight), then the compensated sum in order of p
    constexpr int kIt = kSplitDD / kSumWays;
    double vh[kIt], vl[kIt];
#pragma unroll
    for (int i = 0; i < kIt; ++i) {
      const int p = q + i * kSumWays;
      vh[i] = p < nsplit ? part_hi[(int64_t)p * kB * kB + t] : 0.0;
      vl[i] = p < nsplit ? part_lo[(int64_t)p * kB * kB + t] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kIt; ++i) {
      if (q + i * kSumWays >= nsplit) break;
      double s2, er;
      two_sum(h, vh[i], s2, er);
      h = s2;
      l += er + vl[i];
    }
  }
  sh[threadIdx.x] = h;
  sl[threadIdx.x] = l;
  __syncthreads();
  if (q == 0 && t < kB * kB) {
    for (int j = 1; j < kSumWays; ++j) {
      double s2, er;
      two_sum(h, sh[j * kPer + e], s2, er);
      h = s2;
      l += er + sl[j * kPer + e];
    }
    quick_two_sum(h, l, G_hi[t], G_lo[t]);
  }
}

// G[i][j] = sum_s part[s][i][j] in a fixed order (deterministic).
__global__ __launch_bounds__(kBlock) void k_blk_sum_parts(const BasisDev* __restrict__ bd) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ part = d.part;
  double* __restrict__ G = d.G;
  const int nparts = d.ntake;
  const DevScalars* sc = d.sc;
  __shared__ double sh[kBlock];
  if (sc->blk_na == 0) return;
  constexpr int kPer = kBlock / kSumWays;
  const int e = threadIdx.x % kPer, q = threadIdx.x / kPer;
  const int t = blockIdx.x * kPer + e;
  double s = 0.0;
  if (t < kB * kB) {
    constexpr int kIt = kTakeParts / kSumWays;
    double v[kIt];
#pragma unroll
    for (int i = 0; i < kIt; ++i) {
      const int p = q + i * kSumWays;
      v[i] = p < nparts ? part[(int64_t)p * kB * kB + t] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kIt; ++i) s += v[i];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  if (q == 0 && t < kB * kB) {
    for (int j = 1; j < kSumWays; ++j) s += sh[j * kPer + e];
    G[t] = s;
  }
}

// The 64 x 64 factorizations run in one workgroup of kChol threads: a
// right-looking Cholesky that builds L^{-1} in the same sweep, the matrix held
// in registers (kSlots columns per wave, one row per lane).
constexpr int kChol = 1024;
constexpr int kSlots = kB / (kChol / kWave);   // columns held per wave
typedef double LdsMat[kB][kB + 1];

// (ah, al) *= (bh, bl)
__device__ inline void dd_mul(double& ah, double& al, double bh, double bl) {
#pragma clang fp contract(off)
  double p, pe;
  two_prod(ah, bh, p, pe);
  pe = fma(ah, bl, pe);
  pe = fma(al, bh, pe);
  quick_two_sum(p, pe, ah, al);
}

// Cholesky of the leading n x n block of A (lower triangle, A[i][c] for
// c <= i, zeros above; double-double when Al != nullptr) in candidate order,
// producing X = L^{-1} in place of A.  Lane i of wave w holds row i of
// columns w + 16 q (q < 4) in registers, so whether a held column is left of,
// at or right of the step's column is the same for the whole wave.  Step j
// (right-looking): column j of A below the diagonal, row j of X left of it and
// the pivot decision with 1 / L[j][j] arrive through LDS from the end of step
// j - 1; each lane scales what it needs itself (L[i][j] = A[i][j] / L[j][j],
// and per held column L[c][j] or X[j][c] = X'[j][c] / L[j][j]), so each step
// needs a single barrier.  Columns right of j take the Schur update A[i][c] -=
// L[i][j] L[c][j] (i >= c), columns at or left of it the elimination X[i][c]
// -= L[i][j] X[j][c]; entry (i, j) turns from A into X at step j.  The owners
// of column j + 1, row j + 1 and entry (j + 1, j + 1) then publish them into
// the other half of the double-buffered exchange arrays (ch, cl, xrow:
// 2 x 64; piv: 2 x 4).  With drop set, candidate j is kept iff its pivot
// exceeds eps2 * gs[j] and fewer than `room` are kept so far; a dropped
// candidate gets an identity row and a zero column in X, so X restricted to
// the kept set is the inverse of the kept factor.  X goes to LDS; returns the
// kept mask (same in every thread).
template <bool kDD>
__device__ uint64_t wg_chol_inv(const LdsMat& Ah, const LdsMat* Al, LdsMat& X, double* ch,
                                double* cl, double* xrow, double* piv, const double* gs, int n,
                                bool drop, double eps2, int64_t room) {
  constexpr int kWaves = kChol / kWave;
  const int i = threadIdx.x % kWave, w = threadIdx.x / kWave;
  double ah[kSlots], al[kSlots];
#pragma unroll
  for (int q = 0; q < kSlots; ++q) {
    ah[q] = Ah[i][w + kWaves * q];
    al[q] = kDD ? (*Al)[i][w + kWaves * q] : 0.0;
  }
  // The owner of diagonal entry (j, j) decides candidate j and publishes
  // {keep, 1 / L[j][j] (hi, lo)}.
  auto publish = [&](double dh, double dl, int j, int kept, double* pv) {
    const bool keep = !drop || (((dh - eps2 * gs[j]) + dl > 0.0) && kept < room);
    double rh = 0.0, rl = 0.0;
    if (keep) {
      if (kDD)
        dd_rsqrt(dh, dl, rh, rl);
      else
        rh = 1.0 / sqrt(fmax(dh, 1e-300));
    }
    pv[0] = keep ? 1.0 : 0.0;
    pv[1] = rh;
    pv[2] = rl;
  };
  if (n > 0 && w == 0) {   // column 0 is slot 0 of wave 0
    if (i > 0 && i < n) {
      ch[i] = ah[0];
      cl[i] = al[0];
    }
    if (i == 0) publish(ah[0], al[0], 0, 0, piv);
  }
  __syncthreads();
  uint64_t mask = 0;
  int kept = 0;
  for (int j = 0; j < n; ++j) {
    const int pb = (j & 1) * kB, nb = kB - pb;
    const double* pv = piv + (j & 1) * 4;
    const bool keep = pv[0] != 0.0;
    if (keep) {
      const double rh = pv[1], rl = pv[2];
      double lih = 0.0, lil = 0.0;   // L[i][j]
      if (i > j && i < n) {
        lih = ch[pb + i];
        lil = cl[pb + i];
        if (kDD)
          dd_mul(lih, lil, rh, rl);
        else
          lih *= rh;
      }
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        const int c = w + kWaves * q;
        if (c >= n) continue;
        if (c > j) {                     // Schur update of A, rows i >= c
          if (i >= c && i < n) {
            double lch = ch[pb + c], lcl = cl[pb + c];   // L[c][j]
            if (kDD) {
              dd_mul(lch, lcl, rh, rl);
              dd_fnma(ah[q], al[q], lih, lil, lch, lcl);
            } else {
              ah[q] -= lih * (lch * rh);
            }
          }
        } else if (c == j) {
          if (i == j)
            ah[q] = rh;                  // X[j][j]
          else if (i > j && i < n)
            ah[q] = -lih * rh;           // X[i][j] = -L[i][j] X[j][j]
        } else {
          const double xr = xrow[pb + c] * rh;   // X[j][c]
          if (i == j)
            ah[q] = xr;
          else if (i > j && i < n)
            ah[q] -= lih * xr;           // X[i][c] -= L[i][j] X[j][c]
        }
      }
      ++kept;
      mask |= 1ull << j;
    } else {
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        const int c = w + kWaves * q;
        if ((c == j && i >= j) || (c < j && i == j)) ah[q] = (i == c) ? 1.0 : 0.0;
      }
    }
    const int j1 = j + 1;
    if (j1 < n) {
#pragma unroll
      for (int q = 0; q < kSlots; ++q) {
        const int c = w + kWaves * q;
        if (c == j1) {
          if (i > j1 && i < n) {
            ch[nb + i] = ah[q];
            cl[nb + i] = al[q];
          } else if (i == j1) {
            publish(ah[q], al[q], j1, kept, piv + (j1 & 1) * 4);
          }
        } else if (c < j1 && i == j1) {
          xrow[nb + c] = ah[q];
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kSlots; ++q) X[i][w + kWaves * q] = ah[q];
  __syncthreads();
  return mask;
}

// The value of lane `src` (wave-uniform) in every lane.
__device__ inline double bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// Double-double Cholesky with drop of the leading n x n block of (Ah, Al)
// (lower triangle, kChol threads), blocked by panels of kPanel columns, with
// a one-panel lookahead.  For panel p: first waves 0 .. kPanel - 1 subtract
// panel p - 1's rank-kPanel product from panel p's columns (wave w: column
// c0 + w); then wave 0 factors panel p on its own (lane i holds row i of the
// panel's columns; the pivot and L[c][j] come from their lanes by readlane,
// so a panel's steps need no barrier) while the other waves subtract panel
// p - 1's product from the columns past panel p (wave w: columns c0 + kPanel
// + w - 1 + 15 q, lane i: row i).  Every entry still takes the panels'
// products in panel order, as without the lookahead.  Candidate j is kept iff
// its Schur pivot exceeds eps2 * gs[j] and fewer than `room` are kept so far;
// a dropped candidate's column of L is zero.  L replaces (Ah, Al) in place;
// returns the kept mask (same in every thread).
constexpr int kPanel = 8;
// A[i][c] -= sum_{j in the panel at p0} L[i][j] L[c][j] for i >= c
__device__ inline void panel_update(LdsMat& Ah, LdsMat& Al, int i, int c, int p0) {
  double ah = Ah[i][c], al = Al[i][c];
#pragma unroll
  for (int jj = 0; jj < kPanel; ++jj)
    dd_fnma(ah, al, Ah[i][p0 + jj], Al[i][p0 + jj], Ah[c][p0 + jj], Al[c][p0 + jj]);
  Ah[i][c] = ah;
  Al[i][c] = al;
}
__device__ uint64_t wg_chol_drop_blocked(LdsMat& Ah, LdsMat& Al, const double* gs, int n,
                                         double eps2, int64_t room, uint64_t* s_mask) {
  constexpr int kWaves = kChol / kWave;
  static_assert(kPanel <= kWaves, "one wave per column of the next panel");
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), i = lane_id();
  uint64_t mask = 0;   // wave 0's
  int kept = 0;
  for (int c0 = 0; c0 < n; c0 += kPanel) {
    const int p0 = c0 - kPanel;   // the previous panel
    if (c0 > 0) {
      // panel p - 1's product on panel p's columns
      const int c = c0 + w;
      if (w < kPanel && c < n && i >= c && i < n) panel_update(Ah, Al, i, c, p0);
      __syncthreads();
    }
    if (w == 0) {
      double h[kPanel], l[kPanel];
#pragma unroll
      for (int cc = 0; cc < kPanel; ++cc) {
        const int c = c0 + cc;
        const bool in = c < n && i >= c && i < n;
        h[cc] = in ? Ah[i][c] : 0.0;
        l[cc] = in ? Al[i][c] : 0.0;
      }
#pragma unroll
      for (int jj = 0; jj < kPanel; ++jj) {
        const int j = c0 + jj;
        if (j >= n) break;
        const double dh = bcast(h[jj], j), dl = bcast(l[jj], j);
        // the same in every lane: taken as a scalar branch
        const bool keep =
            __builtin_amdgcn_readfirstlane((((dh - eps2 * gs[j]) + dl > 0.0) && kept < room) ? 1 : 0);
        if (keep) {
          double rh, rl;
          dd_rsqrt(dh, dl, rh, rl);
          if (i >= j && i < n) dd_mul(h[jj], l[jj], rh, rl);   // L[i][j], L[j][j] = sqrt(pivot)
#pragma unroll
          for (int cc = jj + 1; cc < kPanel; ++cc) {
            const int c = c0 + cc;
            const double lch = bcast(h[jj], c), lcl = bcast(l[jj], c);   // L[c][j]
            if (c < n && i >= c && i < n) dd_fnma(h[cc], l[cc], h[jj], l[jj], lch, lcl);
          }
          ++kept;
          mask |= 1ull << j;
        } else {
          h[jj] = 0.0;
          l[jj] = 0.0;
        }
      }
#pragma unroll
      for (int cc = 0; cc < kPanel; ++cc) {
        const int c = c0 + cc;
        if (c < n && i < n) {
          Ah[i][c] = h[cc];
          Al[i][c] = l[cc];
        }
      }
    } else if (c0 > 0 && i < n) {
      // panel p - 1's product on the columns past panel p
      for (int c = c0 + kPanel + w - 1; c < n; c += kWaves - 1)
        if (i >= c) panel_update(Ah, Al, i, c, p0);
    }
    __syncthreads();
  }
  // the last panel's product is not needed: no column follows it
  if (threadIdx.x == 0) *s_mask = mask;
  __syncthreads();
  return *s_mask;
}

// X = L^{-1} in float64 for the factor of wg_chol_drop_blocked, a dropped
// candidate (and each row past n) taking a unit row and column so that X
// restricted to the kept set is the inverse of the kept factor.  Ld (the
// float64 L, built here) and X are kB x kB; wave w solves L x = e_c for its
// columns c = w + 16 q by forward substitution, lane i holding row i, x_m
// reaching the other lanes by readlane: no barrier inside the solve.  Lane
// m's entry is final once step m has read it, so X is written after the solve.
__device__ void wg_lower_inverse(const LdsMat& Ah, LdsMat& Ld, LdsMat& X, uint64_t mask, int n) {
  constexpr int kWaves = kChol / kWave;
  const int tid = threadIdx.x, i = lane_id();
  const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
  for (int e = tid; e < kB * kB; e += kChol) {
    const int r = e / kB, c = e % kB;
    const bool kr = r < n && ((mask >> r) & 1ull), kc = c < n && ((mask >> c) & 1ull);
    double v = 0.0;
    if (r == c)
      v = kr ? Ah[r][c] : 1.0;
    else if (c < r && kr && kc)
      v = Ah[r][c];
    Ld[r][c] = v;
  }
  __syncthreads();
  const double inv_d = 1.0 / Ld[i][i];
  double acc[kSlots];   // the wave's four columns advance together (independent chains)
#pragma unroll
  for (int q = 0; q < kSlots; ++q) acc[q] = i == w + kWaves * q ? 1.0 : 0.0;
#pragma unroll 2
  for (int m = w; m < kB; ++m) {
    const double lim = Ld[i][m];
#pragma unroll
    for (int q = 0; q < kSlots; ++q) {
      const int c = w + kWaves * q;
      if (m >= c) {
        const double xm = bcast(acc[q] * inv_d, m);
        if (i > m) acc[q] = fma(-lim, xm, acc[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kSlots; ++q) {
    const int c = w + kWaves * q;
    X[i][c] = i >= c ? acc[q] * inv_d : 0.0;   // X[m][c] = x_m, the value lane m gave
  }
  __syncthreads();
}

// The block's residual Gram G (double-double): Cholesky with column drop in
// candidate order (pivot vs eps^2 ||x||^2); kept positions compacted into
// pos[0..na), na into sc->blk_na; Tacc = L_A^{-T} over the kept rows/columns
// (first Cholesky-QR pass of the kept residuals).
__global__ __launch_bounds__(kChol) void k_blk_decide(const BasisDev* __restrict__ bd, int64_t b0) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ G = d.G;
  const double* __restrict__ Glo = d.Glo;
  const double* __restrict__ g = g_of(d, b0);
  const double eps2 = d.a.eps2;
  const int64_t n_rows = d.a.n_rows;
  int32_t* __restrict__ pos = d.pos;
  int32_t* __restrict__ accept_all = d.a.accept;
  double* __restrict__ Tacc = d.Tacc;
  DevScalars* sc = d.sc;
  __shared__ LdsMat Ah, Al, X;
  __shared__ double gs[kB];
  __shared__ int32_t ps[kB];
  __shared__ uint64_t s_mask;
  const int64_t nb_all = blk_count(sc, b0);
  const int64_t nb = blk_work(sc, b0, n_rows);
  const int tid = threadIdx.x;
  if (nb == 0) {
    if (tid == 0) sc->blk_na = 0;
    if (accept_all)
      for (int t = tid; t < nb_all; t += kChol) accept_all[b0 + t] = 0;
    return;
  }
  const int64_t room = n_rows - (int64_t)sc->n_accept_total;   // at most n_rows independent fibers
  for (int e = tid; e < kB * kB; e += kChol) {
    const int i = e / kB, c = e % kB;
    const bool in = i < nb && c <= i;
    Ah[i][c] = in ? G[e] : 0.0;
    Al[i][c] = in ? Glo[e] : 0.0;
  }
  if (tid < kB) gs[tid] = tid < nb ? g[tid] : 0.0;
  __syncthreads();
  const uint64_t m = wg_chol_drop_blocked(Ah, Al, gs, (int)nb, eps2, room, &s_mask);
  wg_lower_inverse(Ah, Al, X, m, (int)nb);   // Al is free once L is formed: it holds L in float64
  const int na = (int)__popcll(m);
  if (tid < kB) {
    const bool my_keep = (m >> tid) & 1ull;
    if (my_keep) {
      const uint64_t lt = tid == 0 ? 0ull : ((~0ull) >> (kWave - tid));
      const int slot = (int)__popcll(m & lt);
      pos[slot] = tid;
      ps[slot] = tid;
    }
    if (tid < nb && accept_all) accept_all[b0 + tid] = my_keep ? 1 : 0;
  }
  if (tid == 0) sc->blk_na = na;
  __syncthreads();   // ps
  // Tacc[a][b] = L_A^{-1}[b][a] = L^{-1}[ps[b]][ps[a]]
  for (int e = tid; e < kB * kB; e += kChol) {
    const int a = e / kB, bb = e % kB;
    Tacc[e] = (a < na && bb < na) ? X[ps[bb]][ps[a]] : 0.0;
  }
}

// Second Cholesky-QR pass of the kept block, taken only when needed: if the
// Gram of the first-pass columns is within kOrthTol of the identity they are
// orthonormal to working accuracy and Tacc stays as it is (blk_reorth = 0).
// Otherwise Cholesky (no drop) of that Gram, Tcur = L^{-T}, Tacc <- Tacc Tcur.
constexpr double kOrthTol = 1e-12;
__global__ __launch_bounds__(kChol) void k_blk_cholinv(const BasisDev* __restrict__ bd) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ G = d.G;
  double* __restrict__ Tcur = d.Tcur;
  double* __restrict__ Tacc = d.Tacc;
  DevScalars* sc = d.sc;
  __shared__ LdsMat L, X, Ta;
  __shared__ double ch[2 * kB], cl[2 * kB], xrow[2 * kB], piv[8];
  __shared__ int any_off;
  const int na = sc->blk_na;
  const int tid = threadIdx.x;
  if (na == 0) return;
  if (tid == 0) any_off = 0;
  __syncthreads();
  bool off = false;
  for (int e = tid; e < kB * kB; e += kChol) {
    const int i = e / kB, c = e % kB;
    if (i < na && c < na) off = off || fabs(G[e] - (i == c ? 1.0 : 0.0)) > kOrthTol;
  }
  if (off) any_off = 1;
  __syncthreads();
  if (!any_off) {
    if (tid == 0) sc->blk_reorth = 0;
    return;
  }
  if (tid == 0) sc->blk_reorth = 1;
  for (int e = tid; e < kB * kB; e += kChol) {
    const int i = e / kB, c = e % kB;
    L[i][c] = (i < na && c <= i) ? G[e] : 0.0;
    Ta[i][c] = Tacc[e];
  }
  __syncthreads();
  wg_chol_inv<false>(L, nullptr, X, ch, cl, xrow, piv, nullptr, na, false, 0.0, kB);
  for (int e = tid; e < kB * kB; e += kChol) {
    const int i = e / kB, bcol = e % kB;
    const bool live = i < na && bcol < na;
    Tcur[e] = live ? X[bcol][i] : 0.0;
    double acc = 0.0;
    for (int c = i; c <= bcol; ++c) acc += Ta[i][c] * X[bcol][c];   // Tacc upper, Tcur[c][bcol] = X[bcol][c]
    Tacc[e] = live ? acc : 0.0;
  }
}

// Kept residuals times the first-pass factor: Q[r][k + a] = sum_{a' <= a}
// Ybuf[r][pos[a']] T[a'][a]; R[r][k + a] = P[r][b0 + pos[a]].  A workgroup
// walks 64-row tiles with a stride of the grid.  Per tile, wave w forms rows
// 16 w .. + 16 of the new columns with f64 MFMAs (A gathered from the Y tile
// through pos, B = T; T is zero past the kept count), and after a barrier the
// Gram of the tile's new rows (wave w: Gram rows 16 w .. + 16) accumulates;
// the sum over its tiles goes to part[blockIdx.x] for the orthogonality
// check of the block.
__global__ __launch_bounds__(kBlock) void k_blk_take(const BasisDev* __restrict__ bd, int64_t b0) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ Ybuf = y_of(d, b0);
  const double* __restrict__ P = d.a.P;
  const int32_t* __restrict__ pos = d.pos;
  const double* __restrict__ T = d.Tacc;
  double* __restrict__ Q = d.a.Q;
  double* __restrict__ R = d.a.R;
  double* __restrict__ part = d.part;
  const int64_t ldp = d.a.ldp, n_rows = d.a.n_rows, ldq = d.a.ldq, ldr = d.a.ldr;
  const int ntake = d.ntake;
  const DevScalars* sc = d.sc;
  __shared__ double Ts[kB][kB + 1];
  __shared__ double Ys[kB][kB + 1];   // Ybuf rows, then the new Q rows
  __shared__ int32_t ps[kB];
  const int na = sc->blk_na;
  if (na == 0 || (int)blockIdx.x >= ntake) return;
  const int64_t k = sc->n_accept_total;
  constexpr int kLd = kB * kB / kBlock;   // tile elements per thread
  {
    double v[kLd];
#pragma unroll
    for (int u = 0; u < kLd; ++u) v[u] = T[u * kBlock + threadIdx.x];
#pragma unroll
    for (int u = 0; u < kLd; ++u) Ts[(u * kBlock + threadIdx.x) / kB][threadIdx.x % kB] = v[u];
  }
  if (threadIdx.x < kB) ps[threadIdx.x] = threadIdx.x < na ? pos[threadIdx.x] : 0;
  const int rl = threadIdx.x / 4;
  const int a_lo = (threadIdx.x % 4) * 16;
  const int w = threadIdx.x / kWave, l = lane_id();
  dbl4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  for (int64_t r0 = (int64_t)blockIdx.x * kB; r0 < n_rows; r0 += (int64_t)ntake * kB) {
    double v[kLd];
#pragma unroll
    for (int u = 0; u < kLd; ++u) {
      const int64_t rr = r0 + (u * kBlock + threadIdx.x) / kB;
      v[u] = rr < n_rows ? Ybuf[rr * kB + threadIdx.x % kB] : 0.0;
    }
    __syncthreads();   // previous tile's Gram reads of Ys done (and Ts, ps written)
#pragma unroll
    for (int u = 0; u < kLd; ++u) Ys[(u * kBlock + threadIdx.x) / kB][threadIdx.x % kB] = v[u];
    __syncthreads();
    // new columns of rows 16 w .. + 16: lane (i, g) holds row 16 w + g + 4 x, column 16 ct + i
    dbl4 qo[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    const int nks = (na + 3) / 4;
    for (int ks = 0; ks < nks; ++ks) {
      const int ap = ks * 4 + l / 16;
      const double av = Ys[w * 16 + l % 16][ps[ap]];   // A[i][a'] = Y[row][pos[a']]
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) qo[ct] = mfma16(av, Ts[ap][ct * 16 + l % 16], qo[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int64_t r = r0 + w * 16 + l / 16 + 4 * x;
        const int a = ct * 16 + l % 16;
        if (r < n_rows && a < na) Q[r * ldq + k + a] = qo[ct][x];
      }
    if (R) {
      const int64_t r = r0 + rl;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int a = a_lo + u;
        if (r < n_rows && a < na) R[r * ldr + k + a] = P[r * ldp + b0 + ps[a]];
      }
    }
    __syncthreads();   // all reads of Ys done
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int x = 0; x < 4; ++x) Ys[w * 16 + l / 16 + 4 * x][ct * 16 + l % 16] = qo[ct][x];
    __syncthreads();
    // acc[i][j] += sum_r Qn[r][i] Qn[r][j] over this tile
#pragma unroll
    for (int ks = 0; ks < kB / 4; ++ks) {
      const double av = Ys[ks * 4 + l / 16][w * 16 + l % 16];   // A[i][r] = Qn[r][i]
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) acc[qq] = mfma16(av, Ys[ks * 4 + l / 16][qq * 16 + l % 16], acc[qq]);
    }
  }
  double* pp = part + (int64_t)blockIdx.x * kB * kB;
#pragma unroll
  for (int qq = 0; qq < 4; ++qq)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) pp[(w * 16 + l / 16 + 4 * rr) * kB + qq * 16 + l % 16] = acc[qq][rr];
}

// Q[r][k + a] <- sum_{a' <= a} Q[r][k + a'] T[a'][a]; rows staged in LDS.
__global__ __launch_bounds__(kBlock) void k_blk_apply(const BasisDev* __restrict__ bd) {
  const BasisDev& d = bd[blockIdx.z];
  double* __restrict__ Q = d.a.Q;
  const double* __restrict__ T = d.Tcur;
  const int64_t ldq = d.a.ldq, n_rows = d.a.n_rows;
  const DevScalars* sc = d.sc;
  __shared__ double Ts[kB][kB + 1];
  __shared__ double Ys[kB][kB + 1];
  const int na = sc->blk_na;
  if (na == 0 || !sc->blk_reorth) return;
  const int64_t k = sc->n_accept_total;
  const int64_t r0 = (int64_t)blockIdx.x * kB;
  if (r0 >= n_rows) return;
  for (int t = threadIdx.x; t < kB * kB; t += kBlock) {
    Ts[t / kB][t % kB] = T[t];
    const int64_t rr = r0 + t / kB;
    const int c = t % kB;
    Ys[t / kB][c] = (rr < n_rows && c < na) ? Q[rr * ldq + k + c] : 0.0;
  }
  __syncthreads();
  const int rl = threadIdx.x / 4;
  const int64_t r = r0 + rl;
  const int a_lo = (threadIdx.x % 4) * 16;
  if (r >= n_rows || a_lo >= na) return;
  double out[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) out[u] = 0.0;
  for (int ap = 0; ap < na; ++ap) {
    const double y = Ys[rl][ap];
#pragma unroll
    for (int u = 0; u < 16; ++u) out[u] += y * Ts[ap][a_lo + u];
  }
  double* q = Q + r * ldq + k;
#pragma unroll
  for (int u = 0; u < 16; ++u)
    if (a_lo + u < na) q[a_lo + u] = out[u];
}

// New columns of M (Q = R M) for the block's kept fibers:
//   M[c][k + a] = -sum_{b <= a} Z[c][b] T[b][a],  Z = M W_A^T  (c < k),
//   M[k + b][k + a] = T[b][a] (b <= a), M[k + b][c] = 0 below the diagonal,
// W_A the W rows of the kept candidates and T = L1^{-T} (L2^{-T}).
//
// k_blk_newm_part: Z over the upper triangle of M, split over j: workgroup
// (x, js) covers rows 32 x .. + 32 and j in [jw js, jw js + jw) from j = 32 x
// on, with f64 MFMAs (two groups of four waves alternating the 32-wide j
// chunks), and writes its 32 x 64 partial to Zp[js] (workgroups whose j range
// lies left of their rows write nothing).  jw is at least 128 and gives at
// most 16 splits of the block step's bound on k.
constexpr int kNewmJMin = 128, kNewmSplits = 16;
inline int64_t newm_jw(int64_t k1) {
  return std::max<int64_t>(kNewmJMin, div_up(div_up(k1, kNewmSplits), 32) * 32);
}
inline int64_t newm_splits(int64_t cap) {
  return std::min<int64_t>(kNewmSplits, div_up(cap, kNewmJMin));
}
__global__ __launch_bounds__(kGemm) void k_blk_newm_part(const BasisDev* __restrict__ bd, int64_t b0,
                                                         int64_t jw) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ M = d.a.M;
  const double* __restrict__ W = w_of(d, b0);
  const int32_t* __restrict__ pos = d.pos;
  double* __restrict__ Zp = d.Zp;
  const int64_t ldm = d.a.ldm, ldw = d.a.cap;
  const DevScalars* sc = d.sc;
  constexpr int kR = 32;
  __shared__ double As[2][kR][kGK + 1];   // M tile [grp][row][j]
  __shared__ double Bs[2][kGK][kB + 1];   // W_A^T tile [grp][j][a]
  __shared__ int32_t ps[kB];
  const int64_t k = sc->n_accept_total;
  const int na = sc->blk_na;
  if (na == 0 || sc->status != 0) return;
  const int64_t r0 = (int64_t)blockIdx.x * kR;
  const int64_t js = blockIdx.y;
  const int64_t jlo = max(r0, js * jw), jhi = min(k, (js + 1) * jw);
  if (r0 >= k || jlo >= jhi) return;
  if (threadIdx.x < kB) ps[threadIdx.x] = threadIdx.x < na ? pos[threadIdx.x] : 0;
  __syncthreads();
  const int grp = threadIdx.x / kBlock, t = threadIdx.x % kBlock;
  const int w = t / kWave, l = lane_id();
  const int rb = (w / 2) * 16, cb = (w % 2) * 32;
  const int64_t nch = (jhi - jlo + kGK - 1) / kGK;
  const int64_t iters = (nch + 1) / 2;
  double ra[kR * kGK / kBlock], rw[kB * kGK / kBlock];
  auto load = [&](int64_t ch) {
    const int64_t j0 = jlo + ch * kGK;
#pragma unroll
    for (int u = 0; u < kR * kGK / kBlock; ++u) {
      const int idx = u * kBlock + t, r = idx / kGK, jj = idx % kGK;
      ra[u] = (ch < nch && j0 + jj < jhi && r0 + r < k) ? M[(r0 + r) * ldm + j0 + jj] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kB * kGK / kBlock; ++u) {
      const int idx = u * kBlock + t, a = idx / kGK, jj = idx % kGK;
      rw[u] = (ch < nch && j0 + jj < jhi && a < na) ? W[(int64_t)ps[a] * ldw + j0 + jj] : 0.0;
    }
  };
  dbl4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  load(grp);
  for (int64_t it = 0; it < iters; ++it) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kR * kGK / kBlock; ++u) {
      const int idx = u * kBlock + t;
      As[grp][idx / kGK][idx % kGK] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < kB * kGK / kBlock; ++u) {
      const int idx = u * kBlock + t;
      Bs[grp][idx % kGK][idx / kGK] = rw[u];
    }
    __syncthreads();
    load(grp + 2 * (it + 1));
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      const double av = As[grp][rb + l % 16][ks * 4 + l / 16];
      const double b0v = Bs[grp][ks * 4 + l / 16][cb + l % 16];
      const double b1v = Bs[grp][ks * 4 + l / 16][cb + 16 + l % 16];
      acc0 = mfma16(av, b0v, acc0);
      acc1 = mfma16(av, b1v, acc1);
    }
  }
  // combine the two groups and write the partial tile
  double(*red)[kB + 1] = Bs[0];   // 32 x 65 doubles
  __syncthreads();
  if (grp == 1) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[rb + l / 16 + 4 * r][cb + l % 16] = acc0[r];
      red[rb + l / 16 + 4 * r][cb + 16 + l % 16] = acc1[r];
    }
  }
  __syncthreads();
  if (grp == 1) return;
  double* zp = Zp + js * kmax_of(d.a) * kB;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = rb + l / 16 + 4 * r;
    if (r0 + rr >= k) continue;
    zp[(r0 + rr) * kB + cb + l % 16] = acc0[r] + red[rr][cb + l % 16];
    zp[(r0 + rr) * kB + cb + 16 + l % 16] = acc1[r] + red[rr][cb + 16 + l % 16];
  }
}

// k_blk_newm_fin: the diagonal block and the zero rows (grid-stride over all
// workgroups), then workgroup x sums the partials of rows 32 x .. + 32 in
// order of js and multiplies by T on f64 MFMAs.
__global__ __launch_bounds__(kGemm) void k_blk_newm_fin(const BasisDev* __restrict__ bd, int64_t jw) {
  const BasisDev& d = bd[blockIdx.z];
  double* __restrict__ M = d.a.M;
  const double* __restrict__ Zp = d.Zp;
  const double* __restrict__ T = d.Tacc;
  const int64_t ldm = d.a.ldm;
  const DevScalars* sc = d.sc;
  constexpr int kR = 32;
  __shared__ double Zs[kR][kB + 1];
  __shared__ double Ts[kB][kB + 1];
  const int64_t k = sc->n_accept_total;
  const int na = sc->blk_na;
  if (na == 0 || sc->status != 0) return;
  {
    const int64_t tot = (int64_t)na * (k + na);
    for (int64_t t = (int64_t)blockIdx.x * kGemm + threadIdx.x; t < tot;
         t += (int64_t)gridDim.x * kGemm) {
      const int64_t b = t / (k + na), c = t % (k + na);
      double v = 0.0;
      if (c >= k) {
        const int64_t a = c - k;
        v = b <= a ? T[b * kB + a] : 0.0;
      }
      M[(k + b) * ldm + c] = v;
    }
  }
  const int64_t r0 = (int64_t)blockIdx.x * kR;
  if (r0 >= k) return;
  const int64_t js0 = r0 / jw, js1 = (k + jw - 1) / jw;
  const int64_t zs = kmax_of(d.a) * kB;   // one split's partials
  // every partial's load issued before the sums, which run in order of js
  static_assert(kR * kB % kGemm == 0, "whole tile per pass");
#pragma unroll
  for (int u = 0; u < kR * kB / kGemm; ++u) {
    const int e = u * kGemm + threadIdx.x, r = e / kB, a = e % kB;
    double zv[kNewmSplits];
#pragma unroll
    for (int q = 0; q < kNewmSplits; ++q)
      zv[q] = (r0 + r < k && js0 + q < js1) ? Zp[(js0 + q) * zs + (r0 + r) * kB + a] : 0.0;
    double z = 0.0;
#pragma unroll
    for (int q = 0; q < kNewmSplits; ++q) z += zv[q];
    Zs[r][a] = z;
  }
  for (int e = threadIdx.x; e < kB * kB; e += kGemm) {
    const int b = e / kB, a = e % kB;
    Ts[b][a] = (b <= a && a < na) ? T[e] : 0.0;
  }
  __syncthreads();
  // -Z T on f64 MFMAs: wave w forms the 16 x 16 tile (w / 4, w % 4)
  static_assert(kGemm / kWave == (kR / 16) * (kB / 16), "one output tile per wave");
  const int w = threadIdx.x / kWave, l = lane_id();
  const int rt = (w / 4) * 16, ct = (w % 4) * 16;
  dbl4 acc = {0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < kB / 4; ++ks)
    acc = mfma16(Zs[rt + l % 16][ks * 4 + l / 16], Ts[ks * 4 + l / 16][ct + l % 16], acc);
  const int a = ct + l % 16;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t c = r0 + rt + l / 16 + 4 * r;
    if (c < k && a < na) M[c * ldm + k + a] = -acc[r];
  }
}

// Book-keeping of one block: ids and marks of the kept fibers, saved W rows,
// and k += na.
__global__ void k_blk_finish(const BasisDev* __restrict__ bd, int64_t b0) {
  const BasisDev& d = bd[blockIdx.z];
  const int32_t* __restrict__ pos = d.pos;
  const int32_t* __restrict__ uniq_fi = d.a.uniq_fi;
  const uint64_t* __restrict__ uniq_fid = d.a.uniq_fid;
  const uint64_t id_offset = d.a.id_offset;
  uint64_t* __restrict__ acc_fid = d.a.acc_fid;
  int32_t* __restrict__ acc_fi_local = d.a.acc_fi_local;
  uint8_t* __restrict__ fiber_mark = d.a.fiber_mark;
  const double* __restrict__ W = w_of(d, b0);
  double* __restrict__ Wacc = d.a.Wacc;
  const int64_t ldw = d.a.cap, ldwa = d.a.ldwa;
  DevScalars* sc = d.sc;
  const int64_t k = sc->n_accept_total;
  const int na = sc->blk_na;
  const int64_t base = k - sc->wacc_base;     // row of the first new fiber in Wacc
  for (int a = threadIdx.x; a < na; a += blockDim.x) {
    const int64_t b = b0 + pos[a];
    acc_fid[k + a] = uniq_fid[b] + id_offset;
    if (acc_fi_local) acc_fi_local[base + a] = uniq_fi[b];
    if (fiber_mark) fiber_mark[uniq_fi[b]] = 1;
  }
  if (Wacc)
    for (int64_t t = threadIdx.x; t < (int64_t)na * k; t += blockDim.x) {
      const int64_t a = t / k, c = t % k;
      Wacc[(base + a) * ldwa + c] = W[(int64_t)pos[a] * ldw + c];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    sc->n_accept_total = (int32_t)(k + na);
    sc->s_tilde += na;
    d.kcut[blk_par(b0)] = k + na;   // the early first pass of step b0 + 128
  }
}

__global__ void k_begin_basis(const BasisDev* __restrict__ bd) {
  const BasisDev& d = bd[blockIdx.z];
  DevScalars* sc = d.sc;
  sc->base_accept = sc->n_accept_total;   // kept before this call
  sc->s_tilde = 0;
  d.kcut[0] = sc->n_accept_total;
  d.kcut[1] = sc->n_accept_total;   // the early first pass of step 64
}

// lev[i] = sum_{c in [c0, k)} Q[i][c]^2 (+= when accumulating); Qf copy of those columns.
__global__ __launch_bounds__(kBlock) void k_lev(const BasisDev* __restrict__ bd) {
  const BasisDev& d = bd[blockIdx.z];
  const double* __restrict__ Q = d.a.Q;
  float* __restrict__ Qf = d.a.Qf;
  double* __restrict__ lev = d.a.lev;
  const bool from_base = d.a.lev_accumulate;
  const int64_t ldq = d.a.ldq, n_rows = d.a.n_rows;
  const DevScalars* sc = d.sc;
  const int64_t k = sc->n_accept_total;
  const int64_t c0 = from_base ? sc->base_accept : 0;
  const int lane = lane_id();
  const int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (r >= n_rows) return;
  const double* q = Q + r * ldq;
  double s = 0.0;
  for (int64_t c = c0 + lane; c < k; c += kWave) {
    const double v = q[c];
    s += v * v;
    if (Qf) Qf[r * ldq + c] = (float)v;
  }
  s = wave_sum(s);
  if (lane == 0) lev[r] = (from_base ? lev[r] : 0.0) + s;
}

struct Splits {
  int dd, take;
};
// Row splits of one input: enough rows per split that small inputs do not
// write (and sum) mostly empty partials.
Splits splits_for(int64_t n_rows) {
  Splits sp;
  sp.dd = (int)std::max<int64_t>(1, std::min<int64_t>(kSplitDD, div_up(n_rows, 32)));
  sp.take = (int)std::max<int64_t>(1, std::min<int64_t>(kTakeParts, div_up(n_rows, kB)));
  return sp;
}

// Up to kPutPack entries of the argument array, passed by value.
constexpr int kPutPack = 8;
struct BasisPack {
  BasisDev d[kPutPack];
};
__global__ void k_put_dev(BasisDev* __restrict__ out, BasisPack pk, int n) {
  constexpr int kWords = sizeof(BasisDev) / 8;
  const uint64_t* src = (const uint64_t*)pk.d;
  uint64_t* dst = (uint64_t*)out;
  for (int t = threadIdx.x; t < n * kWords; t += blockDim.x) dst[t] = src[t];
}
}  // namespace

// Room for the W2 partials at any block step of an input.
size_t w2p_doubles(int64_t n_rows, int64_t cap) {
  size_t w2p = 0;
  for (int64_t T = 1; T <= div_up(std::min(cap, n_rows), kB); ++T)
    w2p = std::max(w2p, (size_t)w2_splits(n_rows, T, 1) * kB * kB * T);
  return w2p;
}

size_t basis_scratch_doubles(int64_t n_rows, int64_t cap, int w2_sets) {
  const Splits sp = splits_for(n_rows);
  return (size_t)2 * kB * cap                       // W (two sets)
         + (w2_sets > 1 ? 2 : 1) * (w2p_doubles(n_rows, cap) + (size_t)kB * cap)   // W2p, W2
         + (size_t)sp.take * kB * kB                // part
         + (size_t)sp.dd * kB * kB * 2 + (size_t)kB * kB   // part_hi/lo, G_lo
         + (size_t)kB * kB * 3                      // G, Tcur, Tacc
         + 2 * kB                                   // g (two sets)
         + (size_t)2 * kB * n_rows                  // Ybuf (two sets)
         + 2                                        // kcut
         + (size_t)newm_splits(std::min(cap, n_rows)) * std::min(cap, n_rows) * kB   // Zp
         + 64;                                      // pos
}

size_t basis_dev_bytes(int count) { return (size_t)std::max(count, 1) * sizeof(BasisDev); }

// Orders later work on `waiter` after the work enqueued so far on `signaler`
// (event record and wait); if either call fails, waits for `signaler` on the
// host instead, which orders the same work.
static void order_after(hipStream_t waiter, hipStream_t signaler, hipEvent_t ev) {
  if (hipEventRecord(ev, signaler) == hipSuccess && hipStreamWaitEvent(waiter, ev, 0) == hipSuccess)
    return;
  (void)hipGetLastError();
  (void)hipStreamSynchronize(signaler);
}

void launch_basis(hipStream_t st, const BasisArgs* args, DevScalars* const* scs, int count,
                  void* dev, BasisSide* side) {
  if (count <= 0) return;
  // inputs in order of decreasing candidate bound, so the inputs still
  // working at a block step are a prefix of the array
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return args[x].s_max > args[y].s_max; });
  std::vector<BasisDev> hd(count);
  for (int i = 0; i < count; ++i) {
    const BasisArgs& a = args[order[i]];
    const Splits sp = splits_for(a.n_rows);
    BasisDev& d = hd[i];
    d = BasisDev{};
    d.a = a;
    d.sc = scs[order[i]];
    d.W = a.scratch;
    d.W2p[0] = d.W + (size_t)2 * kB * a.cap;
    d.W2[0] = d.W2p[0] + w2p_doubles(a.n_rows, a.cap);
    double* after = d.W2[0] + (size_t)kB * a.cap;
    if (a.w2_sets > 1) {
      d.W2p[1] = after;
      d.W2[1] = d.W2p[1] + w2p_doubles(a.n_rows, a.cap);
      after = d.W2[1] + (size_t)kB * a.cap;
    } else {
      d.W2p[1] = d.W2p[0];
      d.W2[1] = d.W2[0];
    }
    d.part = after;
    d.part_hi = d.part + (size_t)sp.take * kB * kB;
    d.part_lo = d.part_hi + (size_t)sp.dd * kB * kB;
    d.Glo = d.part_lo + (size_t)sp.dd * kB * kB;
    d.G = d.Glo + kB * kB;
    d.Tcur = d.G + kB * kB;
    d.Tacc = d.Tcur + kB * kB;
    d.g = d.Tacc + kB * kB;
    d.Ybuf = d.g + 2 * kB;
    d.kcut = (int64_t*)(d.Ybuf + (size_t)2 * kB * a.n_rows);
    d.Zp = (double*)(d.kcut + 2);
    d.pos = (int32_t*)(d.Zp + (size_t)newm_splits(kmax_of(a)) * kmax_of(a) * kB);
    d.nsplit_dd = sp.dd;
    d.ntake = sp.take;
  }
  BasisDev* dd = (BasisDev*)dev;
  for (int i0 = 0; i0 < count; i0 += kPutPack) {
    BasisPack pk;
    const int n = std::min(kPutPack, count - i0);
    for (int u = 0; u < n; ++u) pk.d[u] = hd[i0 + u];
    hipLaunchKernelGGL(k_put_dev, dim3(1), dim3(256), 0, st, dd + i0, pk, n);
  }
  const int sums = kB * kB * kSumWays / kBlock;
  constexpr int kMaxZ = 65535;
  // the side stream fills CUs that single-workgroup steps leave idle: with
  // many inputs in a launch those steps fill the GPU by themselves
  const bool ahead = side && side->st[0] && count <= kFewInputs;
  // steps of either parity on a stream of their own when every input holds two
  // sets of the W2 buffers: the late panel of step b + 1 then overlaps the
  // early panel of step b + 2
  bool two = ahead && side->st[1];
  for (int i = 0; i < count; ++i) two = two && args[i].w2_sets > 1;
  auto sst = [&](int64_t bx) { return side->st[two ? (int)((bx / kB) & 1) : 0]; };
  for (int z0 = 0; z0 < count; z0 += kMaxZ) {
    const int nz_all = std::min(kMaxZ, count - z0);
    const BasisDev* bd = dd + z0;
    int64_t rows_all = 1;
    for (int i = z0; i < z0 + nz_all; ++i) rows_all = std::max(rows_all, hd[i].a.n_rows);
    // inputs with candidates left at b0 (a prefix), and host bounds over them
    // of the columns held at the start of the step (k <= min(n_rows, k0 + b0))
    // and of the row splits
    struct Bounds {
      int nz = 0, dd_max = 1, take_max = 1;
      int64_t rows = 1, kub = 0;
    };
    auto bounds = [&](int64_t b0) {
      Bounds r;
      while (r.nz < nz_all && hd[z0 + r.nz].a.s_max > b0) {
        const BasisDev& d = hd[z0 + r.nz];
        r.rows = std::max(r.rows, d.a.n_rows);
        r.kub = std::max(r.kub, std::min(std::min(d.a.n_rows, d.a.k0_max + b0), d.a.cap));
        r.dd_max = std::max(r.dd_max, d.nsplit_dd);
        r.take_max = std::max(r.take_max, d.ntake);
        ++r.nz;
      }
      return r;
    };
    const dim3 wthreads(kWWaves * kWave);
    hipLaunchKernelGGL(k_begin_basis, dim3(1, 1, nz_all), dim3(1), 0, st, bd);
    const int64_t s_all = hd[z0].a.s_max;
    // W2 = Q^T Y over the columns of `range` (host bound kb), partial over row
    // splits then summed, and Y -= Q W2^T: one projection pass of step bx
    auto coef_pass = [&](hipStream_t s, int64_t bx, const Bounds& nx, int64_t kb, int range,
                         int second) {
      const int64_t tl = range == kLate ? 1 : div_up(kb, kB);
      int w = 1;
      for (int i = z0; i < z0 + nx.nz; ++i)
        w = std::max(w, w2_splits(hd[i].a.n_rows,
                                  range == kLate ? 1 : std::min<int64_t>(tl, div_up(kmax_of(hd[i].a), kB)),
                                  nx.nz));
      // (workgroups loop over their entries: with many inputs a few per input suffice)
      const int sum_grid = std::max(1, std::min({4096, div_up((int64_t)kB * kb, kW2Per),
                                                 std::max(8, 65536 / nx.nz)}));
      hipLaunchKernelGGL(k_blk_w2_part, dim3(range == kLate ? 1 : tl, w, nx.nz), dim3(kGemm), 0, s,
                         bd, bx, tl, range);
      hipLaunchKernelGGL(k_blk_w2_sum, dim3(sum_grid, 1, nx.nz), dim3(kBlock), 0, s, bd, bx, tl,
                         range, second);
      hipLaunchKernelGGL(k_blk_form_y, dim3(div_up(nx.rows, 32), 1, nx.nz), dim3(kGemm), 0, s, bd,
                         bx, range, second);
    };
    // both passes of step bx against the columns [0, kb) of range kAll or
    // kEarly: the sparse coefficients Q^T x, Y = P - Q W^T, then the second pass
    auto project = [&](hipStream_t s, int64_t bx, const Bounds& nx, int64_t kb, int range) {
      hipLaunchKernelGGL(k_blk_w, dim3(div_up(kb, kWCols), kB, nx.nz), wthreads, 0, s, bd, bx,
                         range);
      hipLaunchKernelGGL(k_blk_form_y, dim3(div_up(nx.rows, 32), 1, nx.nz), dim3(kGemm), 0, s, bd,
                         bx, range, 0);
      coef_pass(s, bx, nx, kb, range, 1);
    };
    // With the side stream, step bx's early panel (the columns held once step
    // bx - 2 finished, host bound kb) runs there as soon as that step's
    // book-keeping is done, and its late panel (step bx - 1's new columns)
    // once those are final; step bx then waits for done[bx's parity].
    // The W2 partials and sums are shared by the two streams' passes, so the
    // first early panel starts after step 0's own passes.
    bool done_ok[2] = {true, true};
    for (int64_t b0 = 0; b0 < s_all; b0 += kB) {
      const Bounds bn = bounds(b0);
      const int nz = bn.nz;
      const int64_t k1 = std::max<int64_t>(bn.kub, 1);
      const int rows4 = div_up(bn.rows, kB);
      const int par = (int)((b0 / kB) & 1);
      if (ahead && b0 > 0) {
        // both panels ran on the side; a failed record or wait falls back to the host
        if (!done_ok[par] || hipStreamWaitEvent(st, side->done[par], 0) != hipSuccess) {
          (void)hipGetLastError();
          (void)hipStreamSynchronize(sst(b0));
        }
      } else {
        // block classical Gram-Schmidt against all of Q, twice
        project(st, b0, bn, k1, kAll);
        if (ahead && b0 == 0 && s_all > kB) {
          order_after(sst(kB), st, side->start);
          project(sst(kB), kB, bounds(kB), std::max<int64_t>(bn.kub, 1), kEarly);
        }
      }
      if (nz <= kFewInputs && !ahead)
        hipLaunchKernelGGL(k_blk_gram_dd<4>, dim3(bn.dd_max, 1, nz), dim3(kBlock * 4), 0, st, bd, b0);
      else
        hipLaunchKernelGGL(k_blk_gram_dd<1>, dim3(bn.dd_max, 1, nz), dim3(kBlock), 0, st, bd, b0);
      hipLaunchKernelGGL(k_blk_sum_dd, dim3(sums, 1, nz), dim3(kBlock), 0, st, bd, b0);
      hipLaunchKernelGGL(k_blk_decide, dim3(1, 1, nz), dim3(kChol), 0, st, bd, b0);
      hipLaunchKernelGGL(k_blk_take, dim3(bn.take_max, 1, nz), dim3(kBlock), 0, st, bd, b0);
      hipLaunchKernelGGL(k_blk_sum_parts, dim3(sums, 1, nz), dim3(kBlock), 0, st, bd);
      hipLaunchKernelGGL(k_blk_cholinv, dim3(1, 1, nz), dim3(kChol), 0, st, bd);
      hipLaunchKernelGGL(k_blk_apply, dim3(rows4, 1, nz), dim3(kBlock), 0, st, bd);
      // the late panel of the next step: this step's new columns are final
      // here, and M's new columns and the book-keeping follow on st
      if (ahead && b0 + kB < s_all) {
        const Bounds nx = bounds(b0 + kB);
        hipStream_t s1 = sst(b0 + kB);
        order_after(s1, st, side->mid);
        coef_pass(s1, b0 + kB, nx, kB, kLate, 0);
        coef_pass(s1, b0 + kB, nx, kB, kLate, 1);
        done_ok[1 - par] = hipEventRecord(side->done[1 - par], s1) == hipSuccess;
        if (!done_ok[1 - par]) (void)hipGetLastError();
      }
      // M's new columns: split over j for few inputs, whole for many
      const int64_t jw = nz <= kFewInputs ? newm_jw(k1) : std::max<int64_t>(k1, kNewmJMin);
      hipLaunchKernelGGL(k_blk_newm_part, dim3(div_up(k1, 32), div_up(k1, jw), nz), dim3(kGemm), 0,
                         st, bd, b0, jw);
      hipLaunchKernelGGL(k_blk_newm_fin, dim3(div_up(k1, 32), 1, nz), dim3(kGemm), 0, st, bd, jw);
      hipLaunchKernelGGL(k_blk_finish, dim3(1, 1, nz), dim3(256), 0, st, bd, b0);
      // the early panel of the step after next, against the columns held
      // now: its W, g and Ybuf set (this step's) is free once finish has run
      if (ahead && b0 + 2 * kB < s_all) {
        order_after(sst(b0 + 2 * kB), st, side->start);
        project(sst(b0 + 2 * kB), b0 + 2 * kB, bounds(b0 + 2 * kB),
                std::max<int64_t>(bounds(b0 + kB).kub, 1), kEarly);
      }
    }
    hipLaunchKernelGGL(k_lev, dim3(div_up(rows_all * kWave, kBlock), 1, nz_all), dim3(kBlock), 0, st,
                       bd);
  }
}

bool basis_side_init(BasisSide* side) {
  *side = BasisSide{};
  // the events order work between two streams of one device: a device-scope
  // release suffices (no system-scope cache writeback at each record)
  const unsigned fl = hipEventDisableTiming | hipEventReleaseToDevice;
  bool ok = hipStreamCreateWithFlags(&side->st[0], hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&side->st[1], hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&side->start, fl) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&side->mid, fl) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&side->done[0], fl) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&side->done[1], fl) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    basis_side_free(side);
  }
  return ok;
}

void basis_side_free(BasisSide* side) {
  for (hipStream_t& x : side->st)
    if (x) (void)hipStreamDestroy(x);
  if (side->start) (void)hipEventDestroy(side->start);
  if (side->mid) (void)hipEventDestroy(side->mid);
  for (hipEvent_t& e : side->done)
    if (e) (void)hipEventDestroy(e);
  *side = BasisSide{};
}

}  // namespace ctd

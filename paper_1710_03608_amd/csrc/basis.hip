// Independence filter and orthonormal basis, block by block (Algorithm 1
// lines 5-15; Algorithm 2 lines 5-16).
//
// Candidates are visited in order in blocks of 64.  For a block B with the
// kept set so far spanned by the orthonormal columns of Q (k of them):
//   W = Q^T X_B                 (sparse fibers times dense Q)
//   M = X_B^T X_B - W W^T       (Gram of the residuals X_B - Q W: its
//                                Schur complements are the squared residual
//                                norms ||res||^2 of Algorithm 1 line 7)
//   Cholesky of M in candidate order, dropping a candidate whose pivot is
//   <= eps^2 ||x||^2 (line 8); the pivots are accurate to about u ||x||^2
//   because Q is orthonormal, whatever the conditioning of R.
// The kept candidates' residuals Y = X_A - Q W_A are formed explicitly and
// orthonormalized by two Cholesky-QR passes (Y <- Y L1^{-T}, Y <- Y L2^{-T});
// they become the next columns of Q.  With Q = R M (M upper triangular, so
// U = (R^T R)^{-1} = M M^T) the new columns of M are
//   M[:k, new] = -M W_A^T T,  M[new, new] = T,  T = L1^{-T} L2^{-T}.
// One block is ~12 small launches; sizes are read on the device.
#include "kernels.h"

namespace ctd {

namespace {
constexpr int kB = 64;        // candidates per block
constexpr int kSplit = 16;    // K-splits of the long 64 x 64 products
constexpr int kBlock = 256;

__device__ inline int64_t blk_count(const DevScalars* sc, int64_t b0) {
  const int64_t sp = sc->status == 0 ? sc->s_unique : 0;
  return b0 < sp ? min((int64_t)kB, sp - b0) : 0;
}

// Gb[j][c] = x_{b0+j} . x_{b0+c} (c <= j) through the dense panel; one wave per candidate.
__global__ __launch_bounds__(kBlock) void k_blk_gram(const double* __restrict__ P, int64_t ldp,
                                                     const int32_t* __restrict__ uniq_fi,
                                                     const int32_t* __restrict__ fptr,
                                                     const int32_t* __restrict__ row,
                                                     const double* __restrict__ val, int64_t b0,
                                                     double* __restrict__ Gb,
                                                     const DevScalars* sc) {
  const int64_t nb = blk_count(sc, b0);
  const int j = (blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int lane = lane_id();
  if (j >= nb) return;
  const int32_t f = uniq_fi[b0 + j];
  const int32_t e0 = fptr[f], e1 = fptr[f + 1];
  double acc = 0.0;
  const bool active = lane < nb;
  for (int32_t e = e0; e < e1; ++e) {
    const double v = val[e];
    if (active) acc += v * P[(int64_t)row[e] * ldp + b0 + lane];
  }
  Gb[j * kB + lane] = (lane <= j && active) ? acc : 0.0;
}

// W[j][c] = sum_e v_e Q[r_e][c] for c < k; one wave per (candidate, 256 columns).
__global__ __launch_bounds__(kBlock) void k_blk_w(const double* __restrict__ Q, int64_t ldq,
                                                  const int32_t* __restrict__ uniq_fi,
                                                  const int32_t* __restrict__ fptr,
                                                  const int32_t* __restrict__ row,
                                                  const double* __restrict__ val, int64_t b0,
                                                  double* __restrict__ W, int64_t ldw, int nchunk,
                                                  const DevScalars* sc) {
  const int64_t nb = blk_count(sc, b0);
  const int64_t k = sc->n_accept_total;
  const int64_t wid = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int j = (int)(wid / nchunk);
  const int64_t c = (wid % nchunk) * 4 * kWave + 4 * lane_id();
  if (j >= nb || c >= k) return;
  const int32_t f = uniq_fi[b0 + j];
  const int32_t e0 = fptr[f], e1 = fptr[f + 1];
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int32_t e = e0; e < e1; ++e) {
    const double v = val[e];
    const double* q = Q + (int64_t)row[e] * ldq + c;
    const double2 x = *(const double2*)q;
    const double2 y = *(const double2*)(q + 2);
    a0 += v * x.x;
    a1 += v * x.y;
    a2 += v * y.x;
    a3 += v * y.y;
  }
  double* w = W + (int64_t)j * ldw + c;
  const double a[4] = {a0, a1, a2, a3};
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (c + u < k) w[u] = a[u];
}

// 64 x 64 Gram of the columns of Y, partial over split row ranges:
//   part[s][i][j] = sum_{r in range s} Y[r][col0 + i] Y[r][col0 + j]
// mode 0: Y = the block buffer (col0 = 0, width = candidates of the block)
// mode 1: Y = Q[:, k : k + na]   (the kept block after its first pass)
__global__ __launch_bounds__(kBlock) void k_blk_gram_part(const double* __restrict__ A, int64_t lda,
                                                          int64_t K, int mode, int64_t b0,
                                                          double* __restrict__ part,
                                                          const DevScalars* sc) {
  __shared__ double As[kB][kB + 1];   // [kk][i]
  const int64_t col0 = mode == 0 ? 0 : (int64_t)sc->n_accept_total;
  const int64_t width = mode == 0 ? blk_count(sc, b0) : (int64_t)sc->blk_na;
  if (width == 0) return;  // nothing downstream reads part for an empty block
  const int64_t chunk = ((K + kSplit - 1) / kSplit + kB - 1) / kB * kB;
  const int64_t k0 = blockIdx.x * chunk;
  const int64_t k1 = min(K, k0 + chunk);
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  double acc[4][4] = {};
  for (int64_t kk0 = k0; kk0 < k1; kk0 += kB) {
    __syncthreads();
    for (int t = threadIdx.x; t < kB * kB; t += kBlock) {
      const int kk = t / kB, i = t % kB;
      double v = 0.0;
      if (kk0 + kk < k1 && i < width) v = A[(kk0 + kk) * lda + col0 + i];
      As[kk][i] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kB; ++kk) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = As[kk][ty * 4 + u];
        y[u] = As[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += x[u] * y[v];
    }
  }
  double* p = part + (int64_t)blockIdx.x * kB * kB;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) p[(ty * 4 + u) * kB + tx * 4 + v] = acc[u][v];
}

// One wave: M = sum_s part[s], the Gram of the block's residuals against Q;
// Cholesky with column drop in candidate order (pivot vs eps^2 ||x||^2, with
// ||x||^2 from Gb's diagonal); kept positions compacted into pos[0..na), na
// into sc->blk_na; Tacc = L_A^{-T} for the kept rows/columns (first
// Cholesky-QR pass of the kept residuals).
__global__ __launch_bounds__(kWave) void k_blk_decide(const double* __restrict__ Gb,
                                                      const double* __restrict__ part, double eps2,
                                                      int64_t b0, int64_t n_rows,
                                                      int32_t* __restrict__ pos,
                                                      int32_t* __restrict__ accept_all,
                                                      double* __restrict__ Tacc,
                                                      DevScalars* sc) {
  __shared__ double T[kB][kB + 1];
  __shared__ double Xs[kB][kB + 1];
  __shared__ double g[kB];
  __shared__ int32_t ps[kB];
  const int64_t nb = blk_count(sc, b0);
  const int i = threadIdx.x;
  if (nb == 0) {
    if (i == 0) sc->blk_na = 0;
    return;
  }
  const int64_t k_now = sc->n_accept_total;
  int kept = 0;
  for (int j = 0; j < kB; ++j) {
    double m = 0.0;
    if (i < nb && j <= i)
      for (int s = 0; s < kSplit; ++s) m += part[(int64_t)s * kB * kB + i * kB + j];
    T[i][j] = m;
  }
  g[i] = i < nb ? Gb[i * kB + i] : 0.0;
  __syncthreads();
  bool my_keep = false;
  for (int j = 0; j < nb; ++j) {
    const double d = T[j][j];
    // at most n_rows fibers can be independent
    const bool keep = d > eps2 * g[j] && k_now + kept < n_rows;
    kept += keep ? 1 : 0;
    __syncthreads();
    if (keep) {
      const double l = sqrt(d);
      if (i >= j) T[i][j] = (i == j) ? l : T[i][j] / l;
      __syncthreads();
      if (i > j && i < nb) {
        const double lij = T[i][j];
        for (int c = j + 1; c <= i; ++c) T[i][c] -= lij * T[c][j];
      }
    } else {
      if (i >= j) T[i][j] = 0.0;
    }
    if (i == j) my_keep = keep;
    __syncthreads();
  }
  const uint64_t m = __ballot(my_keep && i < nb);
  const int na = (int)__popcll(m);
  if (my_keep && i < nb) {
    const uint64_t lt = i == 0 ? 0ull : ((~0ull) >> (kWave - i));
    const int slot = (int)__popcll(m & lt);
    pos[slot] = i;
    ps[slot] = i;
  }
  if (i < nb && accept_all) accept_all[b0 + i] = my_keep ? 1 : 0;
  if (i == 0) sc->blk_na = na;
  __syncthreads();
  // lane c: column c of L_A^{-1}, L_A[a][a'] = T[ps[a]][ps[a']]
  const int c = i;
  for (int r = 0; r < kB; ++r) Xs[r][c] = 0.0;
  if (c < na) {
    Xs[c][c] = 1.0 / T[ps[c]][ps[c]];
    for (int r = c + 1; r < na; ++r) {
      double x = 0.0;
      for (int j = c; j < r; ++j) x += T[ps[r]][ps[j]] * Xs[j][c];
      Xs[r][c] = -x / T[ps[r]][ps[r]];
    }
  }
  __syncthreads();
  for (int bcol = 0; bcol < kB; ++bcol) Tacc[i * kB + bcol] = (i < na && bcol < na) ? Xs[bcol][i] : 0.0;
}

// Y[i][j] = P[i][b0 + j] - sum_{c<k} Q[i][c] W[j][c] for every candidate j of
// the block (residuals against span(Q)), into Ybuf (n_rows x 64).  One
// workgroup per 64 rows.
__global__ __launch_bounds__(kBlock) void k_blk_form_y(const double* __restrict__ P, int64_t ldp,
                                                       int64_t n_rows, const double* __restrict__ Q,
                                                       int64_t ldq, const double* __restrict__ W,
                                                       int64_t ldw, int64_t b0,
                                                       double* __restrict__ Ybuf,
                                                       const DevScalars* sc) {
  __shared__ double Qs[kB][kB + 1];   // [c][row]
  __shared__ double Ws[kB][kB + 1];   // [c][j]
  const int64_t nb = blk_count(sc, b0);
  if (nb == 0) return;
  const int64_t k = sc->n_accept_total;
  const int64_t r0 = (int64_t)blockIdx.x * kB;
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  double acc[4][4] = {};
  for (int64_t c0 = 0; c0 < k; c0 += kB) {
    __syncthreads();
    for (int t = threadIdx.x; t < kB * kB; t += kBlock) {
      const int a = t / kB, c = t % kB;
      const bool cin = c0 + c < k;
      Qs[c][a] = (cin && r0 + a < n_rows) ? Q[(r0 + a) * ldq + c0 + c] : 0.0;
      Ws[c][a] = (cin && a < nb) ? W[(int64_t)a * ldw + c0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < kB; ++c) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = Qs[c][ty * 4 + u];
        y[u] = Ws[c][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += x[u] * y[v];
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = r0 + ty * 4 + u;
    if (r >= n_rows) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = tx * 4 + v;
      Ybuf[r * kB + j] = j < nb ? P[r * ldp + b0 + j] - acc[u][v] : 0.0;
    }
  }
}

// Kept residuals times the first-pass factor: Q[r][k + a] = sum_{a' <= a}
// Ybuf[r][pos[a']] T[a'][a]; R[r][k + a] = P[r][b0 + pos[a]].  Thread per row.
__global__ __launch_bounds__(kBlock) void k_blk_take(const double* __restrict__ Ybuf,
                                                     const double* __restrict__ P, int64_t ldp,
                                                     int64_t n_rows, const int32_t* __restrict__ pos,
                                                     const double* __restrict__ T, int64_t b0,
                                                     double* __restrict__ Q, int64_t ldq,
                                                     double* __restrict__ R, int64_t ldr,
                                                     const DevScalars* sc) {
  __shared__ double Ts[kB][kB + 1];
  __shared__ int32_t ps[kB];
  const int na = sc->blk_na;
  if (na == 0) return;
  const int64_t k = sc->n_accept_total;
  for (int t = threadIdx.x; t < kB * kB; t += kBlock) Ts[t / kB][t % kB] = T[t];
  if (threadIdx.x < kB) ps[threadIdx.x] = threadIdx.x < na ? pos[threadIdx.x] : 0;
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n_rows) return;
  double y[kB];
#pragma unroll
  for (int a = 0; a < kB; ++a) y[a] = a < na ? Ybuf[r * kB + ps[a]] : 0.0;
  double* q = Q + r * ldq + k;
#pragma unroll
  for (int a = 0; a < kB; ++a) {
    double s = 0.0;
#pragma unroll
    for (int ap = 0; ap <= a; ++ap) s += y[ap] * Ts[ap][a];
    if (a < na) {
      q[a] = s;
      if (R) R[r * ldr + k + a] = P[r * ldp + b0 + ps[a]];
    }
  }
}

// One wave: G = sum_s part[s] (na x na), Cholesky (no drop), Tcur = L^{-T}
// (upper), Tacc <- Tacc Tcur (second Cholesky-QR pass).
__global__ __launch_bounds__(kWave) void k_blk_cholinv(const double* __restrict__ part,
                                                       double* __restrict__ Tcur,
                                                       double* __restrict__ Tacc, int pass,
                                                       const DevScalars* sc) {
  __shared__ double Lm[kB][kB + 1];
  __shared__ double Xs[kB][kB + 1];
  const int na = sc->blk_na;
  const int i = threadIdx.x;
  if (na == 0) return;
  for (int j = 0; j < kB; ++j) {
    double m = 0.0;
    if (i < na && j < na)
      for (int s = 0; s < kSplit; ++s) m += part[(int64_t)s * kB * kB + i * kB + j];
    Lm[i][j] = (i < na && j < na) ? m : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < kB; ++j) {
    const double d = Lm[j][j];
    const double l = sqrt(fmax(d, 1e-300));
    __syncthreads();
    if (i > j) Lm[i][j] = Lm[i][j] / l;
    if (i == j) Lm[j][j] = l;
    __syncthreads();
    if (i > j) {
      const double lij = Lm[i][j];
      for (int c = j + 1; c <= i; ++c) Lm[i][c] -= lij * Lm[c][j];
    }
    __syncthreads();
  }
  // lane c: column c of L^{-1}
  const int c = i;
  for (int r = 0; r < kB; ++r) Xs[r][c] = 0.0;
  Xs[c][c] = 1.0 / Lm[c][c];
  for (int r = c + 1; r < kB; ++r) {
    double x = 0.0;
    for (int j = c; j < r; ++j) x += Lm[r][j] * Xs[j][c];
    Xs[r][c] = -x / Lm[r][r];
  }
  __syncthreads();
  // T = (L^{-1})^T: T[a][b] = Xs[b][a]
  if (pass == 0) {
    for (int b = 0; b < kB; ++b) Tacc[i * kB + b] = Xs[b][i];
  } else {
    for (int b = 0; b < kB; ++b) Tcur[i * kB + b] = Xs[b][i];
    __syncthreads();
    // Tacc <- Tacc Tcur (row i)
    double rowv[kB];
    for (int b = 0; b < kB; ++b) rowv[b] = Tacc[i * kB + b];
    for (int b = 0; b < kB; ++b) {
      double s = 0.0;
      for (int a = 0; a <= b; ++a) s += rowv[a] * Xs[b][a];
      Tacc[i * kB + b] = s;
    }
  }
}

// Q[i][k + a] <- sum_{a' <= a} Q[i][k + a'] T[a'][a]  (thread per row, in place).
__global__ __launch_bounds__(kBlock) void k_blk_apply(double* __restrict__ Q, int64_t ldq,
                                                      int64_t n_rows, const double* __restrict__ T,
                                                      const DevScalars* sc) {
  __shared__ double Ts[kB][kB + 1];
  const int na = sc->blk_na;
  if (na == 0) return;
  const int64_t k = sc->n_accept_total;
  for (int t = threadIdx.x; t < kB * kB; t += kBlock) Ts[t / kB][t % kB] = T[t];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n_rows) return;
  double* q = Q + r * ldq + k;
  double y[kB];
#pragma unroll
  for (int a = 0; a < kB; ++a) y[a] = a < na ? q[a] : 0.0;
#pragma unroll
  for (int a = kB - 1; a >= 0; --a) {
    double s = 0.0;
#pragma unroll
    for (int ap = 0; ap <= a; ++ap) s += y[ap] * Ts[ap][a];
    if (a < na) q[a] = s;
  }
}

// Z[a][c] = sum_{c <= j < k} M[c][j] W[pos[a]][j] for c < k; one wave per row c.
__global__ __launch_bounds__(kBlock) void k_blk_cross(const double* __restrict__ M, int64_t ldm,
                                                      const double* __restrict__ W, int64_t ldw,
                                                      const int32_t* __restrict__ pos,
                                                      double* __restrict__ Z, int64_t ldz,
                                                      const DevScalars* sc) {
  const int64_t k = sc->n_accept_total;
  const int na = sc->blk_na;
  const int lane = lane_id();
  const int64_t c = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (c >= k || na == 0) return;
  const double* mr = M + c * ldm;
  for (int a = 0; a < na; ++a) {
    const double* w = W + (int64_t)pos[a] * ldw;
    double s = 0.0;
    for (int64_t j = c + lane; j < k; j += kWave) s += mr[j] * w[j];
    s = wave_sum(s);
    if (lane == 0) Z[(int64_t)a * ldz + c] = s;
  }
}

// New columns of M: M[c][k + a] = -sum_{a' <= a} Z[a'][c] T[a'][a] (c < k),
// M[k + a'][k + a] = T[a'][a] (a' <= a), M[k + a'][c] = 0 below the diagonal.
__global__ void k_blk_extend_m(double* __restrict__ M, int64_t ldm, const double* __restrict__ Z,
                               int64_t ldz, const double* __restrict__ T, const DevScalars* sc) {
  const int64_t k = sc->n_accept_total;
  const int64_t na = sc->blk_na;
  if (na == 0) return;
  const int64_t rows = k + na;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < rows * na;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / na, a = t % na;
    double v;
    if (c < k) {
      double s = 0.0;
      for (int64_t ap = 0; ap <= a; ++ap) s += Z[ap * ldz + c] * T[ap * kB + a];
      v = -s;
    } else {
      const int64_t ap = c - k;
      v = ap <= a ? T[ap * kB + a] : 0.0;
    }
    M[c * ldm + k + a] = v;
  }
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < na * k;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ap = t / k, c = t % k;
    M[(k + ap) * ldm + c] = 0.0;
  }
}

// Book-keeping of one block: ids and marks of the kept fibers, saved W rows,
// and k += na.
__global__ void k_blk_finish(const int32_t* __restrict__ pos, int64_t b0,
                             const int32_t* __restrict__ uniq_fi,
                             const uint64_t* __restrict__ uniq_fid, uint64_t id_offset,
                             uint64_t* __restrict__ acc_fid, int32_t* __restrict__ acc_fi_local,
                             uint8_t* __restrict__ fiber_mark, const double* __restrict__ W,
                             int64_t ldw, double* __restrict__ Wacc, int64_t ldwa,
                             DevScalars* sc) {
  const int64_t k = sc->n_accept_total;
  const int na = sc->blk_na;
  const int64_t base = k - sc->base_accept;   // kept so far in this call
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
  }
}

__global__ void k_begin_basis(DevScalars* sc) {
  sc->base_accept = sc->n_accept_total;   // kept before this call
  sc->s_tilde = 0;
}

// lev[i] = sum_{c in [c0, k)} Q[i][c]^2 (+= when accumulate); Qf copy of those columns.
__global__ __launch_bounds__(kBlock) void k_lev(const double* __restrict__ Q, int64_t ldq,
                                                int64_t n_rows, float* __restrict__ Qf,
                                                double* __restrict__ lev, bool from_base,
                                                const DevScalars* sc) {
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
}  // namespace

size_t basis_scratch_doubles(int64_t n_rows, int64_t cap) {
  return (size_t)kB * cap            // W
         + (size_t)kSplit * kB * kB  // part
         + (size_t)kB * kB * 3       // Gb, Tcur, Tacc
         + (size_t)kB * cap          // Z
         + (size_t)kB * n_rows       // Ybuf
         + 64;                       // pos
}

void launch_basis(hipStream_t st, const BasisArgs& a, DevScalars* sc) {
  double* W = a.scratch;
  double* part = W + (size_t)kB * a.cap;
  double* Gb = part + (size_t)kSplit * kB * kB;
  double* Tcur = Gb + kB * kB;
  double* Tacc = Tcur + kB * kB;
  double* Z = Tacc + kB * kB;
  double* Ybuf = Z + (size_t)kB * a.cap;
  int32_t* pos = (int32_t*)(Ybuf + (size_t)kB * a.n_rows);
  const int nchunk = div_up(a.cap, 4 * kWave);
  const int rows_tiles = div_up(a.n_rows, kB);
  hipLaunchKernelGGL(k_begin_basis, dim3(1), dim3(1), 0, st, sc);
  for (int64_t b0 = 0; b0 < a.s_max; b0 += kB) {
    hipLaunchKernelGGL(k_blk_gram, dim3(kB * kWave / kBlock), dim3(kBlock), 0, st, a.P, a.ldp,
                       a.uniq_fi, a.fptr, a.row, a.val, b0, Gb, sc);
    hipLaunchKernelGGL(k_blk_w, dim3(div_up((int64_t)kB * nchunk * kWave, kBlock)), dim3(kBlock), 0,
                       st, a.Q, a.ldq, a.uniq_fi, a.fptr, a.row, a.val, b0, W, a.cap, nchunk, sc);
    hipLaunchKernelGGL(k_blk_form_y, dim3(rows_tiles), dim3(kBlock), 0, st, a.P, a.ldp, a.n_rows,
                       a.Q, a.ldq, W, a.cap, b0, Ybuf, sc);
    hipLaunchKernelGGL(k_blk_gram_part, dim3(kSplit), dim3(kBlock), 0, st, Ybuf, (int64_t)kB,
                       a.n_rows, 0, b0, part, sc);
    hipLaunchKernelGGL(k_blk_decide, dim3(1), dim3(kWave), 0, st, Gb, part, a.eps2, b0, a.n_rows,
                       pos, a.accept, Tacc, sc);
    hipLaunchKernelGGL(k_blk_take, dim3(div_up(a.n_rows, kBlock)), dim3(kBlock), 0, st, Ybuf, a.P,
                       a.ldp, a.n_rows, pos, Tacc, b0, a.Q, a.ldq, a.R, a.ldr, sc);
    hipLaunchKernelGGL(k_blk_gram_part, dim3(kSplit), dim3(kBlock), 0, st, a.Q, a.ldq, a.n_rows,
                       1, b0, part, sc);
    hipLaunchKernelGGL(k_blk_cholinv, dim3(1), dim3(kWave), 0, st, part, Tcur, Tacc, 1, sc);
    hipLaunchKernelGGL(k_blk_apply, dim3(div_up(a.n_rows, kBlock)), dim3(kBlock), 0, st, a.Q,
                       a.ldq, a.n_rows, Tcur, sc);
    hipLaunchKernelGGL(k_blk_cross, dim3(div_up(a.cap * kWave, kBlock)), dim3(kBlock), 0, st, a.M,
                       a.ldm, W, a.cap, pos, Z, a.cap, sc);
    hipLaunchKernelGGL(k_blk_extend_m, dim3(std::max(1, std::min(4096, div_up((a.cap + kB) * kB, 256)))),
                       dim3(256), 0, st, a.M, a.ldm, Z, a.cap, Tacc, sc);
    hipLaunchKernelGGL(k_blk_finish, dim3(1), dim3(256), 0, st, pos, b0, a.uniq_fi, a.uniq_fid,
                       a.id_offset, a.acc_fid, a.acc_fi_local, a.fiber_mark, W, a.cap, a.Wacc,
                       a.ldwa, sc);
  }
  hipLaunchKernelGGL(k_lev, dim3(div_up(a.n_rows * kWave, kBlock)), dim3(kBlock), 0, st, a.Q, a.ldq,
                     a.n_rows, a.Qf, a.lev, a.lev_accumulate, sc);
}

}  // namespace ctd

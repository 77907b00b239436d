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
constexpr int kSplit = 64;    // row splits of the 64 x 64 Gram products
constexpr int kBlock = 256;

__device__ inline int64_t blk_count(const DevScalars* sc, int64_t b0) {
  const int64_t sp = sc->status == 0 ? sc->s_unique : 0;
  return b0 < sp ? min((int64_t)kB, sp - b0) : 0;
}

// g[j] = ||x_{b0+j}||^2; one wave per candidate.
__global__ __launch_bounds__(kBlock) void k_blk_norms(const int32_t* __restrict__ uniq_fi,
                                                      const int32_t* __restrict__ fptr,
                                                      const double* __restrict__ val, int64_t b0,
                                                      double* __restrict__ g,
                                                      const DevScalars* sc) {
  const int64_t nb = blk_count(sc, b0);
  const int j = (blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (j >= nb) return;
  const int32_t f = uniq_fi[b0 + j];
  const int32_t e0 = fptr[f], e1 = fptr[f + 1];
  double s = 0.0;
  for (int32_t e = e0 + lane_id(); e < e1; e += kWave) s += val[e] * val[e];
  s = wave_sum(s);
  if (lane_id() == 0) g[j] = s;
}

// W[j][c] = sum_e v_e Q[r_e][c] for c < k; one wave per (candidate, 128
// columns), eight nonzeros in flight per iteration.
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
  const int64_t c = (wid % nchunk) * 2 * kWave + 2 * lane_id();
  if (j >= nb || (wid % nchunk) * 2 * kWave >= k) return;
  const bool active = c < k;
  const int32_t f = uniq_fi[b0 + j];
  const int32_t e0 = fptr[f], e1 = fptr[f + 1];
  double a0 = 0.0, a1 = 0.0;
  int32_t e = e0;
  for (; e + 8 <= e1; e += 8) {
    int32_t r[8];
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      r[u] = row[e + u];
      v[u] = val[e + u];
    }
    double2 q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      q[u] = active ? *(const double2*)(Q + (int64_t)r[u] * ldq + c) : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a0 += v[u] * q[u].x;
      a1 += v[u] * q[u].y;
    }
  }
  for (; e < e1; ++e) {
    const double v = val[e];
    if (active) {
      const double2 q = *(const double2*)(Q + (int64_t)row[e] * ldq + c);
      a0 += v * q.x;
      a1 += v * q.y;
    }
  }
  if (active) {
    double* w = W + (int64_t)j * ldw + c;
    w[0] = a0;
    if (c + 1 < k) w[1] = a1;
  }
}

// Y[r][j] = P[r][b0 + j] - sum_{c<k} Q[r][c] W[j][c] for every candidate j of
// the block (residuals against span(Q)), into Ybuf (n_rows x 64).  One
// workgroup per 32 rows; each thread owns 2 rows x 4 candidates.
__global__ __launch_bounds__(kBlock) void k_blk_form_y(const double* __restrict__ P, int64_t ldp,
                                                       int64_t n_rows, const double* __restrict__ Q,
                                                       int64_t ldq, const double* __restrict__ W,
                                                       int64_t ldw, int64_t b0,
                                                       double* __restrict__ Ybuf,
                                                       const DevScalars* sc) {
  constexpr int kR = 32;
  constexpr int kK = 32;
  __shared__ double Qs[kK][kR + 1];   // [c][row]
  __shared__ double Ws[kK][kB + 1];   // [c][j]
  const int64_t nb = blk_count(sc, b0);
  if (nb == 0) return;
  const int64_t k = sc->n_accept_total;
  const int64_t r0 = (int64_t)blockIdx.x * kR;
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  double acc[2][4] = {};
  for (int64_t c0 = 0; c0 < k; c0 += kK) {
    __syncthreads();
    for (int t = threadIdx.x; t < kK * kR; t += kBlock) {
      const int a = t / kK, c = t % kK;
      Qs[c][a] = (c0 + c < k && r0 + a < n_rows) ? Q[(r0 + a) * ldq + c0 + c] : 0.0;
    }
    for (int t = threadIdx.x; t < kK * kB; t += kBlock) {
      const int a = t / kK, c = t % kK;
      Ws[c][a] = (c0 + c < k && a < nb) ? W[(int64_t)a * ldw + c0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < kK; ++c) {
      const double x0 = Qs[c][ty * 2], x1 = Qs[c][ty * 2 + 1];
      double y[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) y[v] = Ws[c][tx * 4 + v];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[0][v] += x0 * y[v];
        acc[1][v] += x1 * y[v];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int64_t r = r0 + ty * 2 + u;
    if (r >= n_rows) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = tx * 4 + v;
      Ybuf[r * kB + j] = j < nb ? P[r * ldp + b0 + j] - acc[u][v] : 0.0;
    }
  }
}

// 64 x 64 Gram of the columns of Y, partial over kSplit row ranges:
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
  const int64_t chunk = (K + kSplit - 1) / kSplit;
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
    const int kn = (int)min((int64_t)kB, k1 - kk0);
    for (int kk = 0; kk < kn; ++kk) {
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

// G[i][j] = sum_s part[s][i][j] in a fixed order (deterministic).
__global__ __launch_bounds__(kBlock) void k_blk_sum_parts(const double* __restrict__ part,
                                                          double* __restrict__ G, int mode,
                                                          int64_t b0, const DevScalars* sc) {
  const int64_t width = mode == 0 ? blk_count(sc, b0) : (int64_t)sc->blk_na;
  if (width == 0) return;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= kB * kB) return;
  double s = 0.0;
  for (int p = 0; p < kSplit; ++p) s += part[(int64_t)p * kB * kB + t];
  G[t] = s;
}

// Lane c of one wave: column c of L^{-1} for the na x na lower factor in Lm
// (identity-padded), written transposed into Tout: Tout[c][r] = L^{-1}[r][c].
__device__ inline void wave_tri_inverse_t(double (*Lm)[kB + 1], double (*Xs)[kB + 1], int na,
                                          double* __restrict__ Tout) {
  const int c = threadIdx.x;
  for (int r = 0; r < kB; ++r) Xs[r][c] = 0.0;
  if (c < na) {
    Xs[c][c] = 1.0 / Lm[c][c];
    for (int r = c + 1; r < na; ++r) {
      double x = 0.0;
      for (int j = c; j < r; ++j) x += Lm[r][j] * Xs[j][c];
      Xs[r][c] = -x / Lm[r][r];
    }
  }
  __syncthreads();
  for (int b = 0; b < kB; ++b) Tout[c * kB + b] = (c < na && b < na) ? Xs[b][c] : 0.0;
}

// One wave: the block's residual Gram G; Cholesky with column drop in
// candidate order (pivot vs eps^2 ||x||^2); kept positions compacted into
// pos[0..na), na into sc->blk_na; Tacc = L_A^{-T} over the kept rows/columns
// (first Cholesky-QR pass of the kept residuals).
__global__ __launch_bounds__(kWave) void k_blk_decide(const double* __restrict__ G,
                                                      const double* __restrict__ g, double eps2,
                                                      int64_t b0, int64_t n_rows,
                                                      int32_t* __restrict__ pos,
                                                      int32_t* __restrict__ accept_all,
                                                      double* __restrict__ Tacc,
                                                      DevScalars* sc) {
  __shared__ double T[kB][kB + 1];
  __shared__ double Xs[kB][kB + 1];
  __shared__ int32_t ps[kB];
  const int64_t nb = blk_count(sc, b0);
  const int i = threadIdx.x;
  if (nb == 0) {
    if (i == 0) sc->blk_na = 0;
    return;
  }
  const int64_t k_now = sc->n_accept_total;
  for (int j = 0; j < kB; ++j) T[j][i] = (i < nb && j < nb && i <= j) ? G[j * kB + i] : 0.0;
  const double gi = i < nb ? g[i] : 0.0;
  __syncthreads();
  int kept = 0;
  bool my_keep = false;
  for (int j = 0; j < nb; ++j) {
    const double d = T[j][j];
    const double gj = __shfl(gi, j, kWave);
    // at most n_rows fibers can be independent
    const bool keep = d > eps2 * gj && k_now + kept < n_rows;
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
  // compact L_A into Xs (reused as the factor), then invert
  for (int r = 0; r < kB; ++r)
    Xs[r][i] = (r < na && i < na) ? (i <= r ? T[ps[r]][ps[i]] : 0.0) : (r == i ? 1.0 : 0.0);
  __syncthreads();
  wave_tri_inverse_t(Xs, T, na, Tacc);
}

// One wave: Cholesky (no drop) of the kept block's Gram after its first pass,
// Tcur = L^{-T}, Tacc <- Tacc Tcur.
__global__ __launch_bounds__(kWave) void k_blk_cholinv(const double* __restrict__ G,
                                                       double* __restrict__ Tcur,
                                                       double* __restrict__ Tacc,
                                                       const DevScalars* sc) {
  __shared__ double Lm[kB][kB + 1];
  __shared__ double Xs[kB][kB + 1];
  const int na = sc->blk_na;
  const int i = threadIdx.x;
  if (na == 0) return;
  for (int j = 0; j < kB; ++j)
    Lm[j][i] = (i < na && j < na) ? G[j * kB + i] : (i == j ? 1.0 : 0.0);
  __syncthreads();
  for (int j = 0; j < na; ++j) {
    const double l = sqrt(fmax(Lm[j][j], 1e-300));
    __syncthreads();
    if (i >= j) Lm[i][j] = (i == j) ? l : Lm[i][j] / l;
    __syncthreads();
    if (i > j && i < na) {
      const double lij = Lm[i][j];
      for (int c = j + 1; c <= i; ++c) Lm[i][c] -= lij * Lm[c][j];
    }
    __syncthreads();
  }
  wave_tri_inverse_t(Lm, Xs, na, Tcur);
  __syncthreads();
  // Tacc <- Tacc Tcur: stage Tacc in Lm, Tcur is Xs^T
  for (int b = 0; b < kB; ++b) Lm[i][b] = Tacc[i * kB + b];
  __syncthreads();
  for (int b = 0; b < kB; ++b) {
    double s = 0.0;
    for (int a = 0; a <= b; ++a) s += Lm[i][a] * Xs[b][a];
    Tacc[i * kB + b] = (i < na && b < na) ? s : 0.0;
  }
}

// Kept residuals times the first-pass factor: Q[r][k + a] = sum_{a' <= a}
// Ybuf[r][pos[a']] T[a'][a]; R[r][k + a] = P[r][b0 + pos[a]].  Four threads
// per row, 16 output columns each.
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
  const int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 4;
  const int q4 = threadIdx.x % 4;
  if (r >= n_rows) return;
  const int a_lo = q4 * 16;
  if (a_lo >= na) return;
  const int a_hi = min(na, a_lo + 16);
  double out[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) out[u] = 0.0;
  for (int ap = 0; ap < a_hi; ++ap) {
    const double y = Ybuf[r * kB + ps[ap]];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (ap <= a_lo + u) out[u] += y * Ts[ap][a_lo + u];
  }
  double* q = Q + r * ldq + k;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int a = a_lo + u;
    if (a < a_hi) {
      q[a] = out[u];
      if (R) R[r * ldr + k + a] = P[r * ldp + b0 + ps[a]];
    }
  }
}

// Q[r][k + a] <- sum_{a' <= a} Q[r][k + a'] T[a'][a]; four threads per row.
__global__ __launch_bounds__(kBlock) void k_blk_apply(double* __restrict__ Q, int64_t ldq,
                                                      int64_t n_rows, const double* __restrict__ T,
                                                      const DevScalars* sc) {
  __shared__ double Ts[kB][kB + 1];
  const int na = sc->blk_na;
  if (na == 0) return;
  const int64_t k = sc->n_accept_total;
  for (int t = threadIdx.x; t < kB * kB; t += kBlock) Ts[t / kB][t % kB] = T[t];
  __syncthreads();
  const int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 4;
  const int q4 = threadIdx.x % 4;
  const bool live = r < n_rows && q4 * 16 < na;
  double* q = Q + r * ldq + k;
  const int a_lo = q4 * 16;
  const int a_hi = min(na, a_lo + 16);
  double out[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) out[u] = 0.0;
  if (live) {
    for (int ap = 0; ap < a_hi; ++ap) {
      const double y = q[ap];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (ap <= a_lo + u) out[u] += y * Ts[ap][a_lo + u];
    }
  }
  // all four threads of a row read the row before any writes it
  __syncthreads();
  if (live) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (a_lo + u < a_hi) q[a_lo + u] = out[u];
  }
}

// Z[a][c] = sum_{c <= j < k} M[c][j] W[pos[a]][j] for c < k; one workgroup
// per 64 rows of M, 4 x 4 outputs per thread.
__global__ __launch_bounds__(kBlock) void k_blk_cross(const double* __restrict__ M, int64_t ldm,
                                                      const double* __restrict__ W, int64_t ldw,
                                                      const int32_t* __restrict__ pos,
                                                      double* __restrict__ Z, int64_t ldz,
                                                      const DevScalars* sc) {
  __shared__ double Ms[kB][kB + 1];   // [j][c]
  __shared__ double Wsh[kB][kB + 1];  // [j][a]
  __shared__ int32_t ps[kB];
  const int64_t k = sc->n_accept_total;
  const int na = sc->blk_na;
  const int64_t c0 = (int64_t)blockIdx.x * kB;
  if (c0 >= k || na == 0) return;
  if (threadIdx.x < kB) ps[threadIdx.x] = threadIdx.x < na ? pos[threadIdx.x] : 0;
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  double acc[4][4] = {};
  for (int64_t j0 = c0; j0 < k; j0 += kB) {
    __syncthreads();
    for (int t = threadIdx.x; t < kB * kB; t += kBlock) {
      const int a = t / kB, jj = t % kB;
      const bool jin = j0 + jj < k;
      Ms[jj][a] = (jin && c0 + a < k) ? M[(c0 + a) * ldm + j0 + jj] : 0.0;
      Wsh[jj][a] = (jin && a < na) ? W[(int64_t)ps[a] * ldw + j0 + jj] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int jj = 0; jj < kB; ++jj) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = Ms[jj][ty * 4 + u];
        y[u] = Wsh[jj][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += x[u] * y[v];
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t c = c0 + ty * 4 + u;
    if (c >= k) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = tx * 4 + v;
      if (a < na) Z[(int64_t)a * ldz + c] = acc[u][v];
    }
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

// lev[i] = sum_{c in [c0, k)} Q[i][c]^2 (+= when accumulating); Qf copy of those columns.
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
         + (size_t)kB * kB * 3       // G, Tcur, Tacc
         + kB                        // g
         + (size_t)kB * cap          // Z
         + (size_t)kB * n_rows       // Ybuf
         + 64;                       // pos
}

void launch_basis(hipStream_t st, const BasisArgs& a, DevScalars* sc) {
  double* W = a.scratch;
  double* part = W + (size_t)kB * a.cap;
  double* G = part + (size_t)kSplit * kB * kB;
  double* Tcur = G + kB * kB;
  double* Tacc = Tcur + kB * kB;
  double* g = Tacc + kB * kB;
  double* Z = g + kB;
  double* Ybuf = Z + (size_t)kB * a.cap;
  int32_t* pos = (int32_t*)(Ybuf + (size_t)kB * a.n_rows);
  const int nchunk = div_up(a.cap, 2 * kWave);
  const int rows_tiles32 = div_up(a.n_rows, 32);
  const int rows4 = div_up(a.n_rows * 4, kBlock);
  const int cross_tiles = div_up(a.cap, kB);
  const int ext_grid = std::max(1, std::min(4096, div_up((a.cap + kB) * kB, 256)));
  hipLaunchKernelGGL(k_begin_basis, dim3(1), dim3(1), 0, st, sc);
  for (int64_t b0 = 0; b0 < a.s_max; b0 += kB) {
    hipLaunchKernelGGL(k_blk_norms, dim3(kB * kWave / kBlock), dim3(kBlock), 0, st, a.uniq_fi,
                       a.fptr, a.val, b0, g, sc);
    hipLaunchKernelGGL(k_blk_w, dim3(div_up((int64_t)kB * nchunk * kWave, kBlock)), dim3(kBlock), 0,
                       st, a.Q, a.ldq, a.uniq_fi, a.fptr, a.row, a.val, b0, W, a.cap, nchunk, sc);
    hipLaunchKernelGGL(k_blk_form_y, dim3(rows_tiles32), dim3(kBlock), 0, st, a.P, a.ldp, a.n_rows,
                       a.Q, a.ldq, W, a.cap, b0, Ybuf, sc);
    hipLaunchKernelGGL(k_blk_gram_part, dim3(kSplit), dim3(kBlock), 0, st, Ybuf, (int64_t)kB,
                       a.n_rows, 0, b0, part, sc);
    hipLaunchKernelGGL(k_blk_sum_parts, dim3(kB * kB / kBlock), dim3(kBlock), 0, st, part, G, 0, b0,
                       sc);
    hipLaunchKernelGGL(k_blk_decide, dim3(1), dim3(kWave), 0, st, G, g, a.eps2, b0, a.n_rows, pos,
                       a.accept, Tacc, sc);
    hipLaunchKernelGGL(k_blk_take, dim3(rows4), dim3(kBlock), 0, st, Ybuf, a.P, a.ldp, a.n_rows,
                       pos, Tacc, b0, a.Q, a.ldq, a.R, a.ldr, sc);
    hipLaunchKernelGGL(k_blk_gram_part, dim3(kSplit), dim3(kBlock), 0, st, a.Q, a.ldq, a.n_rows,
                       1, b0, part, sc);
    hipLaunchKernelGGL(k_blk_sum_parts, dim3(kB * kB / kBlock), dim3(kBlock), 0, st, part, G, 1, b0,
                       sc);
    hipLaunchKernelGGL(k_blk_cholinv, dim3(1), dim3(kWave), 0, st, G, Tcur, Tacc, sc);
    hipLaunchKernelGGL(k_blk_apply, dim3(rows4), dim3(kBlock), 0, st, a.Q, a.ldq, a.n_rows, Tcur,
                       sc);
    hipLaunchKernelGGL(k_blk_cross, dim3(cross_tiles), dim3(kBlock), 0, st, a.M, a.ldm, W, a.cap,
                       pos, Z, a.cap, sc);
    hipLaunchKernelGGL(k_blk_extend_m, dim3(ext_grid), dim3(256), 0, st, a.M, a.ldm, Z, a.cap, Tacc,
                       sc);
    hipLaunchKernelGGL(k_blk_finish, dim3(1), dim3(256), 0, st, pos, b0, a.uniq_fi, a.uniq_fid,
                       a.id_offset, a.acc_fid, a.acc_fi_local, a.fiber_mark, W, a.cap, a.Wacc,
                       a.ldwa, sc);
  }
  hipLaunchKernelGGL(k_lev, dim3(div_up(a.n_rows * kWave, kBlock)), dim3(kBlock), 0, st, a.Q, a.ldq,
                     a.n_rows, a.Qf, a.lev, a.lev_accumulate, sc);
}

}  // namespace ctd

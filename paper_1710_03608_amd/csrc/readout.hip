// Attack candidates read off R (the online detection of the paper's
// application section, Section 5): the kept fibers are actual fibers, so each
// names its coordinates in the other modes.  Kept fibers with the same
// coordinate in the grouping mode (the destination host of a source x
// destination x time traffic tensor decomposed along the source mode) stand
// for one activity, represented by the earliest kept one; representatives
// whose norm ||x_f|| is above the representatives' mean are the candidates.
//
// The norms are column norms of the dense R on the device (one thread per
// kept fiber, rows summed in order); grouping and selection run on the host
// over the s~ kept fibers, which is O(s~) work after an O(I_alpha s~) pass.
//
// The memory usage of the factors (Eq. 15) counts nonzeros of R and C on the
// device; U = (R^T R)^{-1} is block diagonal over the groups of kept fibers
// linked by shared rows, so its nonzeros are counted from R's pattern on the
// host (union-find over the rows).
#include <math.h>

#include <algorithm>

#include <string>
#include <unordered_map>
#include <vector>

#include "state.h"

namespace ctd {
namespace {

constexpr int kBlock = 256;

// norm[a] = ||R[:, a]|| for a < s~ (R row-major, ldr per row)
__global__ __launch_bounds__(kBlock) void k_col_norms(const double* __restrict__ R, int64_t ldr,
                                                      int64_t n_rows, int64_t cols,
                                                      double* __restrict__ norm) {
  const int64_t a = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (a >= cols) return;
  double s = 0.0;
  for (int64_t r = 0; r < n_rows; ++r) {
    const double v = R[r * ldr + a];
    s += v * v;
  }
  norm[a] = sqrt(s);
}

#define RO_HIP(h, expr)                                                                 \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(h, CTD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

// Nonzero entries of an outer x inner strided block (element (o, i) at
// p[o * ld + i]), added into *count.
__global__ void k_zero2(unsigned long long* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_count_nz(const T* __restrict__ p, int64_t outer,
                                                     int64_t inner, int64_t ld,
                                                     unsigned long long* count) {
  __shared__ unsigned long long part[kBlock / kWave];
  unsigned long long c = 0;
  const int64_t total = outer * inner;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * kBlock) {
    const int64_t o = t / inner, i = t % inner;
    c += p[o * ld + i] != T(0) ? 1ull : 0ull;
  }
  for (int off = kWave / 2; off > 0; off /= 2) c += __shfl_down(c, off, kWave);
  if (lane_id() == 0) part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < kBlock / kWave; ++w) s += part[w];
    atomicAdd(count, s);
  }
}

int64_t find_root(std::vector<int64_t>& parent, int64_t a) {
  while (parent[a] != a) {
    parent[a] = parent[parent[a]];
    a = parent[a];
  }
  return a;
}

// Coordinate in mode m of a fiber id (column-major over the non-alpha modes);
// the last of those modes is not reduced modulo its length (a stream's time
// index grows past it).
uint64_t coordinate(const FiberLayout& lay, uint64_t fid, int m) {
  int last = -1;
  for (int q = 0; q < lay.order; ++q)
    if (q != lay.mode) last = q;
  const uint64_t v = fid / (uint64_t)lay.stride[m];
  return m == last ? v : v % (uint64_t)lay.dims[m];
}

}  // namespace
}  // namespace ctd

using namespace ctd;

extern "C" ctd_status ctd_attack_candidates(ctd_handle* h, int32_t group_mode, uint64_t* fids,
                                            double* norms, int64_t cap, int64_t* n_out,
                                            int64_t* n_groups) {
  if (!h) return CTD_ERR_INVALID_ARG;
  h->last_error.clear();
  if (!n_out || !n_groups || cap < 0 || (cap > 0 && (!fids || !norms)))
    return fail(h, CTD_ERR_INVALID_ARG, "n_out and n_groups are required; fids and norms when cap > 0");
  if (!h->has_static) return fail(h, CTD_ERR_STATE, "no decomposition held");
  const FiberLayout& lay = h->layout;
  if (group_mode < 0 || group_mode >= lay.order || group_mode == lay.mode)
    return fail(h, CTD_ERR_INVALID_ARG, "group_mode must be a mode other than the decomposition mode");
  RO_HIP(h, hipStreamSynchronize(h->stream));
  DevScalars sc{};
  RO_HIP(h, hipMemcpy(&sc, h->d_sc, sizeof(sc), hipMemcpyDeviceToHost));
  if (sc.status != 0) return fail(h, (ctd_status)sc.status, "device reported an error");
  ctd_result res{};
  fill_result(h, sc, &res);
  if (!res.R) return fail(h, CTD_ERR_STATE, "the dense R is not held");
  const int64_t k = res.s_tilde;
  *n_out = 0;
  *n_groups = 0;
  if (k <= 0) return CTD_OK;
  double* d_norm = nullptr;
  RO_HIP(h, dev_alloc(&d_norm, (size_t)k * sizeof(double)));
  hipLaunchKernelGGL(k_col_norms, dim3((unsigned)((k + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     h->stream, res.R, res.ldr, h->n_rows, k, d_norm);
  std::vector<double> nrm(k);
  std::vector<uint64_t> acc(k);
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemcpy(nrm.data(), d_norm, (size_t)k * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(acc.data(), res.accepted, (size_t)k * 8, hipMemcpyDeviceToHost);
  (void)hipFree(d_norm);
  if (e != hipSuccess) return fail(h, CTD_ERR_HIP, std::string("readout copy: ") + hipGetErrorString(e));
  // representatives: the earliest kept fiber of each group, in order
  std::unordered_map<uint64_t, int64_t> first;
  std::vector<int64_t> reps;
  for (int64_t a = 0; a < k; ++a) {
    if (first.emplace(coordinate(lay, acc[a], group_mode), a).second) reps.push_back(a);
  }
  // mean norm of the representatives, summed in order
  double sum = 0.0;
  for (int64_t a : reps) sum += nrm[a];
  const double mean = sum / (double)reps.size();
  int64_t n = 0;
  for (int64_t a : reps) {
    if (nrm[a] > mean) {
      if (n < cap) {
        fids[n] = acc[a];
        norms[n] = nrm[a];
      }
      ++n;
    }
  }
  *n_out = n;
  *n_groups = (int64_t)reps.size();
  return CTD_OK;
}

extern "C" ctd_status ctd_memory_usage(ctd_handle* h, ctd_memory* out) {
  if (!h) return CTD_ERR_INVALID_ARG;
  h->last_error.clear();
  if (!out) return fail(h, CTD_ERR_INVALID_ARG, "out is NULL");
  if (!h->has_static) return fail(h, CTD_ERR_STATE, "no decomposition held");
  RO_HIP(h, hipStreamSynchronize(h->stream));
  DevScalars sc{};
  RO_HIP(h, hipMemcpy(&sc, h->d_sc, sizeof(sc), hipMemcpyDeviceToHost));
  if (sc.status != 0) return fail(h, (ctd_status)sc.status, "device reported an error");
  ctd_result res{};
  fill_result(h, sc, &res);
  if (!res.C) return fail(h, CTD_ERR_STATE, "C is not held (create the handle with want_C)");
  if (!res.R) return fail(h, CTD_ERR_STATE, "the dense R is not held");
  const int64_t k = res.s_tilde, n_rows = h->n_rows;
  *out = ctd_memory{};
  out->nnz_X = h->nnz_seen;
  unsigned long long* d_cnt = nullptr;
  RO_HIP(h, dev_alloc(&d_cnt, 2 * sizeof(unsigned long long)));
  hipLaunchKernelGGL(k_zero2, dim3(1), dim3(64), 0, h->stream, d_cnt);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && k > 0) {
    hipLaunchKernelGGL(k_count_nz<double>, dim3(1024), dim3(kBlock), 0, h->stream, res.R, n_rows,
                       k, res.ldr, d_cnt);
    if (res.C_dtype == CTD_F32)
      hipLaunchKernelGGL(k_count_nz<float>, dim3(1024), dim3(kBlock), 0, h->stream,
                         (const float*)res.C, res.n_cols, k, res.ldc, d_cnt + 1);
    else
      hipLaunchKernelGGL(k_count_nz<double>, dim3(1024), dim3(kBlock), 0, h->stream,
                         (const double*)res.C, res.n_cols, k, res.ldc, d_cnt + 1);
    e = hipGetLastError();
  }
  unsigned long long cnt[2] = {0, 0};
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemcpy(cnt, d_cnt, sizeof(cnt), hipMemcpyDeviceToHost);
  // rows of R for the structure of U (host copy of the k kept columns)
  std::vector<double> Rh;
  if (e == hipSuccess && k > 0) {
    Rh.resize((size_t)n_rows * k);
    e = hipMemcpy2D(Rh.data(), (size_t)k * 8, res.R, (size_t)res.ldr * 8, (size_t)k * 8,
                    (size_t)n_rows, hipMemcpyDeviceToHost);
  }
  (void)hipFree(d_cnt);
  if (e != hipSuccess) return fail(h, CTD_ERR_HIP, std::string("memory usage: ") + hipGetErrorString(e));
  out->nnz_R = (int64_t)cnt[0];
  out->nnz_C = (int64_t)cnt[1];
  // kept fibers sharing a row belong to one diagonal block of U
  std::vector<int64_t> parent(k);
  for (int64_t a = 0; a < k; ++a) parent[a] = a;
  for (int64_t r = 0; r < n_rows; ++r) {
    int64_t prev = -1;
    for (int64_t a = 0; a < k; ++a) {
      if (Rh[(size_t)r * k + a] == 0.0) continue;
      if (prev >= 0) {
        const int64_t x = find_root(parent, prev), y = find_root(parent, a);
        if (x != y) parent[std::max(x, y)] = std::min(x, y);
      }
      prev = a;
    }
  }
  std::vector<int64_t> size(k, 0);
  for (int64_t a = 0; a < k; ++a) ++size[find_root(parent, a)];
  int64_t nu = 0;
  for (int64_t a = 0; a < k; ++a) nu += size[a] * size[a];
  out->nnz_U = nu;
  out->usage = out->nnz_X > 0
                   ? (double)(out->nnz_C + out->nnz_U + out->nnz_R) / (double)out->nnz_X
                   : 0.0;
  return CTD_OK;
}

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
#include <math.h>

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
  RO_HIP(h, hipMalloc(&d_norm, (size_t)k * sizeof(double)));
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

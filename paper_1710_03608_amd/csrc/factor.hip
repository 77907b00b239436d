// Candidate panel (Algorithm 1: R is initialized with and extended by actual
// fibers of X).  The s' unique candidate fibers are scattered into a dense
// row-major n_rows x s' panel, zero elsewhere, so that block Gram products and
// residual vectors of the independence filter read them with coalesced rows.
#include "kernels.h"

namespace ctd {

namespace {
__global__ void k_fill_panel(double* __restrict__ P, int64_t n_rows, int64_t ldp,
                             const DevScalars* sc) {
  const int64_t cols = sc->s_unique;
  const int64_t total = n_rows * ldp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i % ldp < cols) P[i] = 0.0;
  }
}

__global__ void k_scatter_panel(const int32_t* __restrict__ uniq_fi, const int32_t* __restrict__ fptr,
                                const int32_t* __restrict__ row, const double* __restrict__ val,
                                double* __restrict__ P, int64_t ldp, const DevScalars* sc) {
  const int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (b >= sc->s_unique) return;
  const int32_t f = uniq_fi[b];
  const int32_t e0 = fptr[f], e1 = fptr[f + 1];
  for (int32_t e = e0 + lane_id(); e < e1; e += kWave) P[(int64_t)row[e] * ldp + b] = val[e];
}

}  // namespace

void launch_panel(hipStream_t st, const int32_t* uniq_fi, int64_t s_max, const int32_t* fptr,
                  const int32_t* row, const double* val, int64_t n_rows, double* P, int64_t ldp,
                  DevScalars* sc) {
  hipLaunchKernelGGL(k_fill_panel, dim3(2048), dim3(256), 0, st, P, n_rows, ldp, sc);
  hipLaunchKernelGGL(k_scatter_panel, dim3(div_up(s_max * kWave, 256)), dim3(256), 0, st,
                     uniq_fi, fptr, row, val, P, ldp, sc);
}

}  // namespace ctd

// The factor C_(alpha) = R^T X_(alpha) of Algorithm 1 as a sparse matrix
// (the sparse output whose nonzeros Eq. 15 counts).  R's columns are actual
// fibers, so C[a][f] is nonzero only where kept fiber a and fiber f share a
// row: an SpGEMM with 2 sum_i deg_R(i) deg_X(i) flops.
//
// R is held dense (I_alpha x s~, row-major); its rows become lists of
// (a, R[i][a]) in increasing a (one wave per row, ballot prefix).  Each
// non-empty fiber f is one wave with a dense accumulator of s~ doubles in LDS:
// for its nonzeros (i, v) in fiber order, lanes add v R[i][a] over row i's
// list (the a of one list are distinct, so lanes never collide, and the
// additions to one entry follow the fiber's order: deterministic).  A first
// pass counts the nonzero entries per column, an exclusive scan gives the
// column pointers, and a second pass, which repeats the same additions,
// writes the entries in increasing a.
#include <mutex>
#include <string>

#include "state.h"

namespace ctd {
namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 16;                    // per thread of a scan block
constexpr int kScanTile = kBlock * kScanItems;    // elements per scan block
constexpr int64_t kMaxLdsDoubles = 8192;          // 64 KiB of accumulators per workgroup

// cnt[i] = #{a < k : R[i][a] != 0}; one wave per row
__global__ __launch_bounds__(kBlock) void k_r_rowcount(const double* __restrict__ R, int64_t ldr,
                                                       int64_t n_rows, int64_t k,
                                                       int64_t* __restrict__ cnt) {
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (i >= n_rows) return;
  const int lane = lane_id();
  int64_t c = 0;
  for (int64_t a = lane; a < k; a += kWave) c += R[i * ldr + a] != 0.0 ? 1 : 0;
  c = wave_sum(c);
  if (lane == 0) cnt[i] = c;
}

// the lists: rcol/rval[rptr[i] ..] = (a, R[i][a]) for the nonzero R[i][a], a increasing
__global__ __launch_bounds__(kBlock) void k_r_rowfill(const double* __restrict__ R, int64_t ldr,
                                                      int64_t n_rows, int64_t k,
                                                      const int64_t* __restrict__ rptr,
                                                      int32_t* __restrict__ rcol,
                                                      double* __restrict__ rval) {
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  if (i >= n_rows) return;
  const int lane = lane_id();
  const uint64_t lt = lane == 0 ? 0ull : ((~0ull) >> (kWave - lane));
  int64_t p = rptr[i];
  for (int64_t a0 = 0; a0 < k; a0 += kWave) {
    const int64_t a = a0 + lane;
    const double v = a < k ? R[i * ldr + a] : 0.0;
    const uint64_t m = __ballot(v != 0.0);
    if (v != 0.0) {
      const int64_t q = p + __popcll(m & lt);
      rcol[q] = (int32_t)a;
      rval[q] = v;
    }
    p += __popcll(m);
  }
}

// Fiber f's column of C into the wave's accumulator acc[0 .. k).
__device__ inline void accumulate_column(double* acc, int64_t k, int32_t e0, int32_t e1,
                                         const int32_t* __restrict__ row,
                                         const double* __restrict__ val,
                                         const int64_t* __restrict__ rptr,
                                         const int32_t* __restrict__ rcol,
                                         const double* __restrict__ rval) {
  const int lane = lane_id();
  for (int64_t a = lane; a < k; a += kWave) acc[a] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int32_t e = e0; e < e1; ++e) {
    const int32_t i = row[e];
    const double v = val[e];
    const int64_t p1 = rptr[i + 1];
    for (int64_t p = rptr[i] + lane; p < p1; p += kWave) acc[rcol[p]] += v * rval[p];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// One wave per non-empty fiber; kWrite = false: colptr[f] = nonzero entries of
// column f; kWrite = true: the entries at colptr[f] in increasing a.
template <bool kWrite>
__global__ __launch_bounds__(kBlock) void k_c_columns(const int32_t* __restrict__ fptr,
                                                      const int32_t* __restrict__ row,
                                                      const double* __restrict__ val,
                                                      const DevScalars* sc, int64_t k,
                                                      const int64_t* __restrict__ rptr,
                                                      const int32_t* __restrict__ rcol,
                                                      const double* __restrict__ rval,
                                                      int64_t* __restrict__ colptr,
                                                      int32_t* __restrict__ row_idx,
                                                      double* __restrict__ vals) {
  extern __shared__ double lds[];
  const int waves = blockDim.x / kWave;
  const int w = threadIdx.x / kWave, lane = lane_id();
  double* acc = lds + (int64_t)w * k;
  const int64_t n_f = sc->n_f;
  const uint64_t lt = lane == 0 ? 0ull : ((~0ull) >> (kWave - lane));
  for (int64_t f = (int64_t)blockIdx.x * waves + w; f < n_f; f += (int64_t)gridDim.x * waves) {
    accumulate_column(acc, k, fptr[f], fptr[f + 1], row, val, rptr, rcol, rval);
    if (!kWrite) {
      int64_t c = 0;
      for (int64_t a = lane; a < k; a += kWave) c += acc[a] != 0.0 ? 1 : 0;
      c = wave_sum(c);
      if (lane == 0) colptr[f] = c;
    } else {
      int64_t p = colptr[f];
      for (int64_t a0 = 0; a0 < k; a0 += kWave) {
        const int64_t a = a0 + lane;
        const double v = a < k ? acc[a] : 0.0;
        const uint64_t m = __ballot(v != 0.0);
        if (v != 0.0) {
          const int64_t q = p + __popcll(m & lt);
          row_idx[q] = (int32_t)a;
          vals[q] = v;
        }
        p += __popcll(m);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();   // the accumulator is cleared for the next fiber
  }
}

// Exclusive scan of x[0 .. n) in place, x[n] = total (x holds n + 1 entries):
// block sums, a scan of the block sums in one workgroup, then each block's
// elements with its offset.
__global__ __launch_bounds__(kBlock) void k_scan_sums(const int64_t* __restrict__ x, int64_t n,
                                                      int64_t* __restrict__ part) {
  __shared__ int64_t tmp[kBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < kScanItems; ++u)
    if (base + u < n) s += x[base + u];
  s = block_sum<int64_t, kBlock>(s, tmp);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_scan_parts(int64_t* __restrict__ part, int64_t nparts) {
  __shared__ int64_t tmp[kBlock / kWave + 1];
  int64_t tot = 0;
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nparts; b0 += kBlock) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t v = b < nparts ? part[b] : 0;
    const int64_t ex = block_excl_scan<int64_t, kBlock>(v, tmp, &tot);
    if (b < nparts) part[b] = carry + ex;
    carry += tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(int64_t* __restrict__ x, int64_t n,
                                                       const int64_t* __restrict__ part,
                                                       int64_t nparts) {
  __shared__ int64_t tmp[kBlock / kWave + 1];
  int64_t tot = 0;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < kScanItems; ++u) {
    v[u] = base + u < n ? x[base + u] : 0;
    s += v[u];
  }
  int64_t run = part[blockIdx.x] + block_excl_scan<int64_t, kBlock>(s, tmp, &tot);
#pragma unroll
  for (int u = 0; u < kScanItems; ++u) {
    if (base + u < n) x[base + u] = run;
    run += v[u];
  }
  if (blockIdx.x == nparts - 1 && threadIdx.x == kBlock - 1) x[n] = run;
}

}  // namespace

// x[0 .. n] as above; part holds div_up(n, kScanTile) entries (at least one).
static void scan_excl(hipStream_t st, int64_t* x, int64_t n, int64_t* part) {
  const int64_t nparts = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nparts), dim3(kBlock), 0, st, x, n, part);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kBlock), 0, st, part, nparts);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nparts), dim3(kBlock), 0, st, x, n, part, nparts);
}

}  // namespace ctd

using namespace ctd;

#define SC_HIP(expr)                                                            \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess) {                                                     \
      rc = fail(h, CTD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
      goto done;                                                                \
    }                                                                           \
  } while (0)

namespace {

// Scratch of ctd_sparse_core_noalloc: one array per GPU, resident until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host the name is a stand-in, not a device address): the device address of
// each GPU's copy is looked up once with hipGetSymbolAddress and kept.
__device__ __align__(256) unsigned char scratch[CTD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch (the GPU of the handle's stream).
ctd_status scratch_address(ctd_handle* h, void** out) {
  hipDevice_t dev = 0;
  hipError_t e = hipStreamGetDevice(h->stream, &dev);
  if (e != hipSuccess) return fail(h, CTD_ERR_HIP, std::string("hipStreamGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(h, CTD_ERR_CAPACITY, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) return fail(h, CTD_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess)
      return fail(h, CTD_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(h, CTD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CTD_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace of one sparse-core call: R's row pointers, the scan's block sums
// and R's row lists.  `base` null: each buffer is allocated (and freed by
// release); otherwise they are carved from `base`, `cap` bytes long.
struct CoreWs {
  char* base = nullptr;
  size_t cap = 0;
  bool owned = false;
  int64_t* rptr = nullptr;
  int64_t* part = nullptr;
  int32_t* rcol = nullptr;
  double* rval = nullptr;
  size_t head = 0;       // bytes of rptr and part in the carved layout

  hipError_t front(int64_t n_rows, int64_t nparts) {
    if (!base) {
      owned = true;
      hipError_t e = dev_alloc(&rptr, (size_t)(n_rows + 1) * sizeof(int64_t));
      if (e != hipSuccess) return e;
      return dev_alloc(&part, (size_t)nparts * sizeof(int64_t));
    }
    rptr = (int64_t*)base;
    part = (int64_t*)(base + align256((size_t)(n_rows + 1) * sizeof(int64_t)));
    head = align256((size_t)(n_rows + 1) * sizeof(int64_t)) + align256((size_t)nparts * sizeof(int64_t));
    return hipSuccess;
  }
  static size_t front_bytes(int64_t n_rows, int64_t nparts) {
    return align256((size_t)(n_rows + 1) * sizeof(int64_t)) + align256((size_t)nparts * sizeof(int64_t));
  }
  size_t lists_bytes(int64_t nnz_r) const {
    const size_t n = (size_t)std::max<int64_t>(nnz_r, 1);
    return align256(n * sizeof(double)) + align256(n * sizeof(int32_t));
  }
  hipError_t lists(int64_t nnz_r) {
    const size_t n = (size_t)std::max<int64_t>(nnz_r, 1);
    if (owned) {
      hipError_t e = dev_alloc(&rcol, n * sizeof(int32_t));
      if (e != hipSuccess) return e;
      return dev_alloc(&rval, n * sizeof(double));
    }
    rval = (double*)(base + head);
    rcol = (int32_t*)(base + head + align256(n * sizeof(double)));
    return hipSuccess;
  }
  void release() {
    if (!owned) return;
    if (rptr) (void)hipFree(rptr);
    if (part) (void)hipFree(part);
    if (rcol) (void)hipFree(rcol);
    if (rval) (void)hipFree(rval);
  }
};

ctd_status sparse_core_impl(ctd_handle* h, int64_t* col_ptr, int32_t* row_idx, double* vals,
                            int64_t cap, int64_t* nnz_out, char* ws_base, size_t ws_cap);

}  // namespace

extern "C" ctd_status ctd_sparse_core(ctd_handle* h, int64_t* col_ptr, int32_t* row_idx, double* vals,
                                   int64_t cap, int64_t* nnz_out) {
  return sparse_core_impl(h, col_ptr, row_idx, vals, cap, nnz_out, nullptr, 0);
}

extern "C" ctd_status ctd_sparse_core_noalloc(ctd_handle* h, int64_t* col_ptr, int32_t* row_idx,
                                           double* vals, int64_t cap, int64_t* nnz_out) {
  if (!h) return CTD_ERR_INVALID_ARG;
  void* p = nullptr;
  const ctd_status st = scratch_address(h, &p);
  if (st != CTD_OK) return st;
  return sparse_core_impl(h, col_ptr, row_idx, vals, cap, nnz_out, (char*)p, CTD_NOALLOC_SCRATCH_BYTES);
}

namespace {

ctd_status sparse_core_impl(ctd_handle* h, int64_t* col_ptr, int32_t* row_idx, double* vals,
                            int64_t cap, int64_t* nnz_out, char* ws_base, size_t ws_cap) {
  if (!h) return CTD_ERR_INVALID_ARG;
  h->last_error.clear();
  if (!col_ptr || !nnz_out || cap < 0 || (cap > 0 && (!row_idx || !vals)))
    return fail(h, CTD_ERR_INVALID_ARG, "col_ptr and nnz_out are required; row_idx and vals when cap > 0");
  if (!h->has_static || h->last_was_update)
    return fail(h, CTD_ERR_STATE, "needs the CTD-S decomposition of the last ctd_decompose");
  {
    const hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, CTD_ERR_HIP, std::string("sync: ") + hipGetErrorString(e));
  }
  DevScalars sc{};
  if (hipMemcpy(&sc, h->d_sc, sizeof(sc), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(h, CTD_ERR_HIP, "reading the device scalars failed");
  if (sc.status != 0) return fail(h, (ctd_status)sc.status, "device reported an error");
  ctd_result res{};
  fill_result(h, sc, &res);
  if (!res.R) return fail(h, CTD_ERR_STATE, "the dense R is not held");
  const int64_t k = res.s_tilde, n_rows = h->n_rows, n_f = sc.n_f;
  if (k > kMaxLdsDoubles)
    return fail(h, CTD_ERR_CAPACITY, "sparse C needs s~ <= " + std::to_string(kMaxLdsDoubles));
  *nnz_out = 0;
  const StaticBufs& b = h->sb;
  hipStream_t st = h->stream;
  ctd_status rc = CTD_OK;
  CoreWs ws;
  ws.base = ws_base;
  ws.cap = ws_cap;
  int64_t nnz_r = 0, nnz_c = 0;
  const int64_t nparts = std::max<int64_t>(
      1, (std::max(n_rows, n_f) + kScanTile - 1) / kScanTile);
  if (ws_base && CoreWs::front_bytes(n_rows, nparts) + ws.lists_bytes(0) > ws_cap)
    return fail(h, CTD_ERR_CAPACITY, "the workspace for " + std::to_string(n_rows) + " rows exceeds the " +
                                         std::to_string(ws_cap) + "-byte scratch");
  const int waves = (int)std::max<int64_t>(1, std::min<int64_t>(4, kMaxLdsDoubles / std::max<int64_t>(k, 1)));
  const size_t lds = (size_t)waves * std::max<int64_t>(k, 1) * sizeof(double);
  const unsigned grid_rows = (unsigned)std::max<int64_t>(1, (n_rows * kWave + kBlock - 1) / kBlock);
  const unsigned grid_f = (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, (n_f + waves - 1) / waves));
  SC_HIP(ws.front(n_rows, nparts));
  // R's rows as lists
  hipLaunchKernelGGL(k_r_rowcount, dim3(grid_rows), dim3(kBlock), 0, st, res.R, res.ldr, n_rows, k,
                     ws.rptr);
  scan_excl(st, ws.rptr, n_rows, ws.part);
  SC_HIP(hipMemcpyAsync(&nnz_r, ws.rptr + n_rows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SC_HIP(hipStreamSynchronize(st));
  if (ws_base && ws.head + ws.lists_bytes(nnz_r) > ws_cap) {
    rc = fail(h, CTD_ERR_CAPACITY, "R's " + std::to_string(nnz_r) + " nonzeros exceed the " +
                                       std::to_string(ws_cap) + "-byte scratch");
    goto done;
  }
  SC_HIP(ws.lists(nnz_r));
  hipLaunchKernelGGL(k_r_rowfill, dim3(grid_rows), dim3(kBlock), 0, st, res.R, res.ldr, n_rows, k,
                     ws.rptr, ws.rcol, ws.rval);
  // counts per column, pointers, total
  hipLaunchKernelGGL((k_c_columns<false>), dim3(grid_f), dim3(waves * kWave), lds, st, b.fptr, b.row,
                     b.val, h->d_sc, k, ws.rptr, ws.rcol, ws.rval, col_ptr, nullptr, nullptr);
  scan_excl(st, col_ptr, n_f, ws.part);
  SC_HIP(hipMemcpyAsync(&nnz_c, col_ptr + n_f, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  SC_HIP(hipStreamSynchronize(st));
  *nnz_out = nnz_c;
  if (nnz_c > cap) {
    rc = fail(h, CTD_ERR_CAPACITY, "sparse C has " + std::to_string(nnz_c) + " entries, cap is " +
                                       std::to_string(cap));
    goto done;
  }
  hipLaunchKernelGGL((k_c_columns<true>), dim3(grid_f), dim3(waves * kWave), lds, st, b.fptr, b.row,
                     b.val, h->d_sc, k, ws.rptr, ws.rcol, ws.rval, col_ptr, row_idx, vals);
  SC_HIP(hipGetLastError());
  SC_HIP(hipStreamSynchronize(st));
done:
  ws.release();
  return rc;
}

}  // namespace

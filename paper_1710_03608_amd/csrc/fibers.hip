// Fiber keying and fiber-major layout (matricization, Section 2.1), squared
// norms and integer sampling weights (the column distribution of Algorithm 1).
//
// Each nonzero gets the 64-bit key (fiber id << rbits | row), where the
// fiber id is its column in X_(alpha) (column-major over the other modes)
// and row its mode-alpha index.  After the radix sort, equal fiber ids are
// contiguous with rows ascending: the CSF-like layout (fptr, fid, row, val)
// every later step streams.  The same pass forms the integer weight
// q_e = floor(v_e^2 * 2^sigma), with sigma = 62 - ceil(log2 nnz) - E and
// E the binary exponent bounding the largest v^2, and the inclusive prefix
// of q over nonzeros: the fiber distribution's cumulative weights are the
// prefix values at fiber ends, so sampling searches this array directly.
#include "kernels.h"

namespace ctd {

namespace {
constexpr int kKeyBlock = 256;
constexpr int kSegBlock = 1024;
constexpr int kSegItems = 8;
constexpr int kSegTile = kSegBlock * kSegItems;

__device__ inline double load_val(const void* val, int dtype, int64_t e) {
  return dtype == CTD_F32 ? (double)((const float*)val)[e] : ((const double*)val)[e];
}

__device__ inline uint64_t quantize(double v, int sigma) {
  const double v2 = v * v;
  return (uint64_t)ldexp(v2, sigma);
}

__global__ __launch_bounds__(kKeyBlock) void k_build_keys(FiberLayout lay,
                                                          const int32_t* __restrict__ idx,
                                                          const void* __restrict__ val, int dtype,
                                                          int64_t nnz, uint64_t* __restrict__ keys,
                                                          uint32_t* __restrict__ perm,
                                                          DevScalars* sc) {
  __shared__ uint64_t wmax[kKeyBlock / kWave];
  uint64_t v2bits = 0;
  bool oob_any = false, nan_any = false;
  for (int64_t e = (int64_t)blockIdx.x * kKeyBlock + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * kKeyBlock) {
    uint64_t fid = 0;
    uint64_t row = 0;
    bool oob = false;
    for (int m = 0; m < lay.order; ++m) {
      const int32_t i = idx[(int64_t)m * nnz + e];
      if (i < 0 || (int64_t)i >= lay.dims[m]) oob = true;
      if (m == lay.mode)
        row = (uint64_t)(uint32_t)i;
      else
        fid += (uint64_t)(uint32_t)i * (uint64_t)lay.stride[m];
    }
    const double v = load_val(val, dtype, e);
    if (oob) {
      oob_any = true;
      fid = 0;
      row = 0;
    }
    const bool fin = isfinite(v);
    nan_any |= !fin;
    keys[e] = (fid << lay.rbits) | row;
    perm[e] = (uint32_t)e;
    const uint64_t b = (uint64_t)__double_as_longlong(fin ? v * v : 0.0);
    v2bits = b > v2bits ? b : v2bits;   // positive doubles order like their bit patterns
  }
  if (oob_any) latch_status(sc, CTD_ERR_INDEX_OOB);
  if (nan_any) latch_status(sc, CTD_ERR_NONFINITE);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v2bits, off, kWave);
    v2bits = o > v2bits ? o : v2bits;
  }
  if (lane_id() == 0) wmax[threadIdx.x / kWave] = v2bits;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t m = 0;
    for (int w = 0; w < kKeyBlock / kWave; ++w) m = wmax[w] > m ? wmax[w] : m;
    if (m) atomicMax((unsigned long long*)&sc->vmax2_bits, (unsigned long long)m);
  }
}

__global__ void k_sigma(int64_t nnz, DevScalars* sc) {
  const double vmax2 = __longlong_as_double((long long)sc->vmax2_bits);
  int e = 0;
  if (nnz == 0 || !(vmax2 > 0.0)) {
    if (!sc->allow_empty) latch_status(sc, CTD_ERR_EMPTY);
    sc->sigma = 0;
    return;
  }
  frexp(vmax2, &e);  // vmax2 < 2^e
  const int lbits = nnz > 1 ? 64 - __clzll((long long)(nnz - 1)) : 0;
  sc->sigma = 62 - lbits - e;
}

__global__ __launch_bounds__(kSegBlock) void k_seg_reduce(SegmentBuffers b, int64_t nnz, int rbits,
                                                          DevScalars* sc) {
  __shared__ uint64_t tq[kSegBlock / kWave + 1];
  __shared__ uint32_t tc[kSegBlock / kWave + 1];
  __shared__ double tv[kSegBlock / kWave + 1];
  const int sigma = sc->sigma;
  const uint64_t rmask = rbits ? ((~0ull) >> (64 - rbits)) : 0ull;
  // only the tile's totals are needed here, so its elements are taken in
  // strided order (neighbouring lanes on neighbouring elements)
  const int64_t tile = (int64_t)blockIdx.x * kSegTile;
  uint32_t cnt = 0;
  uint64_t qs = 0;
  double v2s = 0.0;
  bool dup = false;
#pragma unroll
  for (int i = 0; i < kSegItems; ++i) {
    const int64_t e = tile + (int64_t)i * kSegBlock + threadIdx.x;
    if (e < nnz) {
      const uint64_t key = b.keys[e];
      const uint64_t prev = e > 0 ? b.keys[e - 1] : ~0ull;
      const bool start = (e == 0) || ((key >> rbits) != (prev >> rbits));
      dup |= (e > 0) && (key == prev);
      const double v = load_val(b.val_in, b.val_dtype, b.perm[e]);
      b.val[e] = v;
      if (b.val32) b.val32[e] = (float)v;
      b.row[e] = (int32_t)(key & rmask);
      cnt += start ? 1u : 0u;
      qs += quantize(v, sigma);
      v2s += v * v;
    }
  }
  if (dup) latch_status(sc, CTD_ERR_DUPLICATE);
  uint32_t ctot;
  block_excl_scan<uint32_t, kSegBlock>(cnt, tc, &ctot);
  uint64_t qtot;
  block_excl_scan<uint64_t, kSegBlock>(qs, tq, &qtot);
  const double vtot = block_sum<double, kSegBlock>(v2s, tv);
  if (threadIdx.x == 0) {
    b.blk_cnt[blockIdx.x] = ctot;
    b.blk_q[blockIdx.x] = qtot;
    b.blk_v2[blockIdx.x] = vtot;
  }
}

__global__ __launch_bounds__(kSegBlock) void k_seg_spine(SegmentBuffers b, int nblocks,
                                                         int64_t nnz, DevScalars* sc) {
  __shared__ uint64_t tq[kSegBlock / kWave + 1];
  __shared__ uint32_t tc[kSegBlock / kWave + 1];
  __shared__ double tv[kSegBlock / kWave + 1];
  uint32_t ccarry = 0;
  uint64_t qcarry = 0;
  double vsum = 0.0;
  for (int b0 = 0; b0 < nblocks; b0 += kSegBlock) {
    const int i = b0 + threadIdx.x;
    const uint32_t c = i < nblocks ? b.blk_cnt[i] : 0u;
    const uint64_t q = i < nblocks ? b.blk_q[i] : 0ull;
    const double v = i < nblocks ? b.blk_v2[i] : 0.0;
    uint32_t ct;
    uint64_t qt;
    const uint32_t ce = block_excl_scan<uint32_t, kSegBlock>(c, tc, &ct);
    const uint64_t qe = block_excl_scan<uint64_t, kSegBlock>(q, tq, &qt);
    const double vt = block_sum<double, kSegBlock>(v, tv);
    if (i < nblocks) {
      b.blk_cnt[i] = ccarry + ce;
      b.blk_q[i] = qcarry + qe;
    }
    ccarry += ct;
    qcarry += qt;
    vsum += vt;
  }
  if (threadIdx.x == 0) {
    sc->n_f = (int32_t)ccarry;
    sc->W = qcarry;
    sc->norm2 = vsum;
    b.fptr[ccarry] = (int32_t)nnz;
    if ((nnz == 0 || qcarry == 0) && !sc->allow_empty) latch_status(sc, CTD_ERR_EMPTY);
  }
}

__global__ __launch_bounds__(kSegBlock) void k_seg_scan(SegmentBuffers b, int64_t nnz, int rbits,
                                                        DevScalars* sc) {
  __shared__ uint64_t tq[kSegBlock / kWave + 1];
  __shared__ uint32_t tc[kSegBlock / kWave + 1];
  const int sigma = sc->sigma;
  const int64_t base = (int64_t)blockIdx.x * kSegTile + (int64_t)threadIdx.x * kSegItems;
  uint64_t q[kSegItems];
  uint64_t fids[kSegItems];
  bool st[kSegItems];
  uint32_t cnt = 0;
  uint64_t qs = 0;
  uint64_t prev = base > 0 && base < nnz ? b.keys[base - 1] : ~0ull;
#pragma unroll
  for (int i = 0; i < kSegItems; ++i) {
    const int64_t e = base + i;
    q[i] = 0;
    st[i] = false;
    fids[i] = 0;
    if (e < nnz) {
      const uint64_t key = b.keys[e];
      fids[i] = key >> rbits;
      st[i] = (e == 0) || (fids[i] != (prev >> rbits));
      prev = key;
      q[i] = quantize(b.val[e], sigma);
      cnt += st[i] ? 1u : 0u;
      qs += q[i];
    }
  }
  uint32_t ct;
  uint64_t qt;
  uint32_t cex = block_excl_scan<uint32_t, kSegBlock>(cnt, tc, &ct) + b.blk_cnt[blockIdx.x];
  uint64_t qex = block_excl_scan<uint64_t, kSegBlock>(qs, tq, &qt) + b.blk_q[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kSegItems; ++i) {
    const int64_t e = base + i;
    if (e < nnz) {
      qex += q[i];
      b.qpref[e] = qex;
      if (st[i]) {
        b.fptr[cex] = (int32_t)e;
        b.fid[cex] = fids[i];
        ++cex;
      }
    }
  }
}
}  // namespace

void launch_build_keys(hipStream_t st, const FiberLayout& lay, const int32_t* idx,
                       const void* val, int val_dtype, int64_t nnz, uint64_t* keys,
                       uint32_t* perm, DevScalars* sc) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_build_keys, dim3(std::min(1024, div_up(nnz, kKeyBlock))), dim3(kKeyBlock),
                       0, st, lay, idx, val, val_dtype, nnz, keys, perm, sc);
  hipLaunchKernelGGL(k_sigma, dim3(1), dim3(1), 0, st, nnz, sc);
}

size_t segment_blocks(int64_t nnz) { return (size_t)(nnz > 0 ? div_up(nnz, kSegTile) : 1); }

void launch_segment(hipStream_t st, const SegmentBuffers& b, int64_t nnz, int rbits,
                    DevScalars* sc) {
  const int nb = (int)segment_blocks(nnz);
  if (nnz > 0)
    hipLaunchKernelGGL(k_seg_reduce, dim3(nb), dim3(kSegBlock), 0, st, b, nnz, rbits, sc);
  hipLaunchKernelGGL(k_seg_spine, dim3(1), dim3(kSegBlock), 0, st, b, nnz > 0 ? nb : 0, nnz, sc);
  if (nnz > 0)
    hipLaunchKernelGGL(k_seg_scan, dim3(nb), dim3(kSegBlock), 0, st, b, nnz, rbits, sc);
}

}  // namespace ctd

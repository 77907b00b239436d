// C ABI of the CTD library: argument checks, workspace, and the order in
// which the kernels of one CTD-S decomposition (Algorithm 1) or one CTD-D
// step (Algorithm 2) are enqueued.  Nothing here synchronizes except
// ctd_sync / ctd_get_result; sizes known only on the device are bounded on
// the host (s' <= s, s~ <= min(s', I_alpha), n_f <= nnz).
#include <string.h>

#include <string>
#include <vector>

#include "kernels.h"
#include "state.h"

using namespace ctd;

namespace ctd {

void Arena::reset() { off = 0; }

void* Arena::take(size_t bytes) {
  const size_t a = (off + 255) & ~size_t(255);
  off = a + ((bytes + 255) & ~size_t(255));
  return (void*)a;  // offset, rebased in commit()
}

}  // namespace ctd

namespace ctd {
void mark(ctd_handle* h, int i) { mark_on(h, i, h->stream); }

void mark_on(ctd_handle* h, int i, hipStream_t st) {
  if (!h->opt.profile) return;
  if (!h->ev[i]) (void)hipEventCreate(&h->ev[i]);
  (void)hipEventRecord(h->ev[i], st);
  h->ev_used[i] = true;
}

int bits_for(uint64_t n) {  // ceil(log2(n)) for n >= 1
  return n <= 1 ? 0 : 64 - __builtin_clzll(n - 1);
}
// Host-side argument errors leave the handle usable; runtime, allocation and
// device-detected errors put it into the failed state.
ctd_status fail(ctd_handle* h, ctd_status st, const std::string& msg) {
  if (h) {
    h->last_error = msg;
    if (st == CTD_ERR_HIP || st == CTD_ERR_OOM || st == CTD_ERR_INDEX_OOB ||
        st == CTD_ERR_DUPLICATE || st == CTD_ERR_NONFINITE || st == CTD_ERR_EMPTY)
      h->failed = true;
  }
  return st;
}
}  // namespace ctd

namespace {

#define HIP_TRY(h, expr)                                                         \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess)                                                        \
      return fail(h, CTD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)


}  // namespace

namespace ctd {
// Zeroes n 64-bit words (a kernel rather than hipMemsetAsync, whose graph
// nodes are unreliable on replay).
__global__ void k_zero_words(uint64_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_fill_u8(uint8_t* p, int64_t n_max, const DevScalars* sc) {
  const int64_t n = std::min<int64_t>(n_max, sc->n_f);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

ctd_status check_coo(ctd_handle* h, const ctd_coo* X, int32_t mode, FiberLayout* lay,
                     uint64_t* n_cols_total) {
  if (!X) return fail(h, CTD_ERR_INVALID_ARG, "tensor is NULL");
  if (X->order < 2 || X->order > CTD_MAX_ORDER)
    return fail(h, CTD_ERR_INVALID_ARG, "order must be in [2, 8]");
  if (!X->dims) return fail(h, CTD_ERR_INVALID_ARG, "dims is NULL");
  if (mode < 0 || mode >= X->order) return fail(h, CTD_ERR_INVALID_ARG, "mode out of range");
  if (X->nnz < 0 || X->nnz >= (int64_t)INT32_MAX)
    return fail(h, CTD_ERR_INVALID_ARG, "nnz must be in [0, 2^31 - 1)");
  if (X->nnz > 0 && (!X->idx || !X->val))
    return fail(h, CTD_ERR_INVALID_ARG, "idx/val is NULL");
  if (X->val_dtype != CTD_F64 && X->val_dtype != CTD_F32)
    return fail(h, CTD_ERR_INVALID_ARG, "val_dtype must be CTD_F64 or CTD_F32");
  unsigned __int128 total = 1;
  uint64_t ncols = 1;
  lay->order = X->order;
  lay->mode = mode;
  for (int m = 0; m < X->order; ++m) {
    const int64_t d = X->dims[m];
    if (d < 1 || d > (int64_t)INT32_MAX)
      return fail(h, CTD_ERR_INVALID_ARG, "dims must be in [1, 2^31 - 1]");
    total *= (unsigned __int128)d;
    if (total >= ((unsigned __int128)1 << 62))
      return fail(h, CTD_ERR_INVALID_ARG, "product of dims must stay below 2^62");
    lay->dims[m] = d;
  }
  for (int m = 0; m < X->order; ++m) {
    if (m == mode) {
      lay->stride[m] = 0;
      continue;
    }
    lay->stride[m] = (int64_t)ncols;
    ncols *= (uint64_t)X->dims[m];
  }
  lay->n_rows = X->dims[mode];
  lay->rbits = bits_for((uint64_t)X->dims[mode]);
  *n_cols_total = ncols;
  return CTD_OK;
}

// Leading dimensions of Q, R and M are multiples of 8, so a lane's 32-byte
// row segment (4 float64 or 8 float32 columns) never crosses a row end.
int64_t round8(int64_t x) { return (x + 7) & ~int64_t(7); }

namespace {
struct PlanItem {
  void** p;
  size_t bytes;
};
// The workspace of one CTD-S call (or one CTD-D slice), as a list of buffers.
void static_items(int64_t nnz, int64_t s, int64_t n_rows, bool mixed, bool want_C, bool want_R,
                  int64_t max_cols, int w2_sets, StaticBufs* b, std::vector<PlanItem>& items) {
  const int64_t n = std::max<int64_t>(nnz, 1);
  const int64_t ld = round8(s);
  const int64_t nb = (int64_t)segment_blocks(nnz);
  auto add = [&](void* pp, size_t bytes) { items.push_back({(void**)pp, bytes}); };
  add(&b->keys, 2 * n * 8);
  add(&b->perm, 2 * n * 4);
  add(&b->hist, radix_sort_hist_elems(n) * 4);
  add(&b->row, n * 4);
  add(&b->val, n * 8);
  add(&b->val32, mixed ? n * 4 : 4);
  add(&b->qpref, n * 8);
  add(&b->fptr, (n + 1) * 4);
  add(&b->fid, n * 8);
  add(&b->blk_cnt, (nb + 1) * 4);
  add(&b->blk_q, (nb + 1) * 8);
  add(&b->blk_v2, (nb + 1) * 8);
  add(&b->draw_fi, s * 4);
  add(&b->draw_fid, s * 8);
  add(&b->uniq_fi, s * 4);
  add(&b->uniq_fid, s * 8);
  add(&b->counts, s * 4);
  add(&b->prob, s * 8);
  add(&b->scale, s * 8);
  add(&b->P, n_rows * ld * 8);
  add(&b->accept, s * 4);
  add(&b->acc_fid, s * 8);
  add(&b->M, s * ld * 8);
  add(&b->scratch, basis_scratch_doubles(n_rows, ld, w2_sets) * 8);
  add(&b->Q, n_rows * ld * 8);
  add(&b->Qf, mixed ? n_rows * ld * 4 : 4);
  add(&b->lev, n_rows * 8);
  add(&b->fiber_mark, n);
  add(&b->resid, n * 8);
  const int64_t n_long = n / (kLongFiber + 1) + 1;
  const int64_t long_ld = kProjSlices;
  add(&b->long_list, n_long * 4);
  add(&b->long_part, n_long * long_ld * 8);
  add(&b->zpart, (size_t)kProjSlices * n * 8);
  add(&b->partial, ((n + 8191) / 8192 + 1) * 8);
  b->hot_id = b->hot_meta = nullptr;
  b->GH = nullptr;
  b->cold_list = nullptr;
  if (nnz > kHotMinNnz && n_rows <= kHotMaxRows) {
    add(&b->hot_id, n_rows * 4);
    add(&b->hot_meta, (kHotMax + 1) * 4);
    add(&b->GH, n_rows * kHotMax * 8);
    add(&b->cold_list, (n / 2 + 1) * 4);
  }
  add(&b->Rs, want_R ? n_rows * ld * 8 : 8);
  add(&b->C, want_C ? (size_t)ld * n * 8 : 8);
}
}  // namespace

size_t static_bytes(int64_t nnz, int64_t s, int64_t n_rows, bool mixed, bool want_C, bool want_R,
                    int64_t max_cols) {
  StaticBufs tmp{};
  std::vector<PlanItem> items;
  static_items(nnz, s, n_rows, mixed, want_C, want_R, max_cols, 1, &tmp, items);
  Arena A;
  for (auto& it : items) (void)A.take(it.bytes);
  return A.off;
}

// Plan the workspace of one CTD-S call (or one CTD-D slice) and bind pointers.
ctd_status plan_static(ctd_handle* h, int64_t nnz, int64_t s, int64_t n_rows, bool mixed,
                       bool want_C, bool want_R, int64_t max_cols, StaticBufs* b) {
  Arena& A = h->arena;
  A.reset();
  const int64_t ld = round8(s);
  const int64_t long_ld = kProjSlices;
  std::vector<PlanItem> items;
  static_items(nnz, s, n_rows, mixed, want_C, want_R, max_cols, h->w2_sets, b, items);
  std::vector<size_t> offs;
  for (auto& it : items) offs.push_back((size_t)A.take(it.bytes));
  if (A.off > A.cap) {
    if (A.base) {
      (void)hipStreamSynchronize(h->stream);
      (void)hipFree(A.base);
      A.base = nullptr;
      A.cap = 0;
    }
    void* p = nullptr;
    if (dev_alloc(&p, A.off) != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, CTD_ERR_OOM, "workspace allocation of " + std::to_string(A.off) + " bytes failed");
    }
    A.base = (char*)p;
    A.cap = A.off;
  }
  for (size_t i = 0; i < items.size(); ++i) *items[i].p = (void*)(A.base + offs[i]);
  b->ld = ld;
  b->s_max = s;
  b->long_ld = long_ld;
  b->zpart_ld = std::max<int64_t>(nnz, 1);
  return CTD_OK;
}

}  // namespace ctd

namespace ctd {

// A0-A3 on one COO input: keys, fiber-major layout, weights, draws (sampled
// with Philox counter word `step`, or given) and the unique candidates.
ctd_status enqueue_input(ctd_handle* h, const ctd_coo* X, const FiberLayout& lay, int64_t s,
                         uint64_t seed, uint32_t step, const uint64_t* given, StaticBufs& b,
                         uint32_t tensor) {
  hipStream_t st = h->stream;
  const bool mixed = h->opt.precision == CTD_PREC_MIXED;
  const int64_t nnz = X->nnz;
  DevScalars* sc = h->d_sc;
  // A0: keys and fiber-major order
  launch_build_keys(st, lay, X->idx, X->val, X->val_dtype, nnz, b.keys, b.perm, sc);
  uint64_t n_cols = 1;
  for (int m = 0; m < lay.order; ++m)
    if (m != lay.mode) n_cols *= (uint64_t)lay.dims[m];
  const int nbits = lay.rbits + bits_for(n_cols);
  const int64_t n1 = std::max<int64_t>(nnz, 1);
  const bool alt = radix_sort(st, b.keys, b.perm, b.keys + n1, b.perm + n1, nnz, nullptr, nbits,
                              b.hist);
  mark(h, MARK_SORTED);
  SegmentBuffers sb{};
  sb.keys = alt ? b.keys + n1 : b.keys;
  sb.perm = alt ? b.perm + n1 : b.perm;
  sb.val_in = X->val;
  sb.val_dtype = X->val_dtype;
  sb.row = b.row;
  sb.val = b.val;
  sb.val32 = mixed ? b.val32 : nullptr;
  sb.qpref = b.qpref;
  sb.fptr = b.fptr;
  sb.fid = b.fid;
  sb.blk_cnt = b.blk_cnt;
  sb.blk_q = b.blk_q;
  sb.blk_v2 = b.blk_v2;
  // A1: weights, norms; A2: prefix
  launch_segment(st, sb, nnz, lay.rbits, sc);
  hipLaunchKernelGGL(k_fill_u8, dim3(std::max(1, std::min(4096, div_up(nnz, 256)))), dim3(256), 0,
                     st, b.fiber_mark, n1, sc);
  // A2: draws
  if (given) {
    HIP_TRY(h, hipMemcpyAsync(b.draw_fid, given, s * 8, hipMemcpyHostToDevice, st));
    launch_locate_given(st, b.fid, s, b.draw_fid, b.draw_fi, sc);
  } else {
    launch_draws(st, b.qpref, b.fptr, b.fid, nnz, s, seed, step, tensor, b.draw_fi, b.draw_fid, sc);
  }
  // A3: unique
  launch_unique(st, b.draw_fi, s, b.qpref, b.fptr, b.fid, b.uniq_fi, b.uniq_fid, b.counts, b.prob,
                b.scale, sc);
  mark(h, MARK_SAMPLED);
  return CTD_OK;
}

int key_bits(const FiberLayout& lay) {
  uint64_t n_cols = 1;
  for (int m = 0; m < lay.order; ++m)
    if (m != lay.mode) n_cols *= (uint64_t)lay.dims[m];
  return lay.rbits + bits_for(n_cols);
}

ProjectArgs project_args(ctd_handle* h, StaticBufs& b, const double* Q, const float* Qf,
                         int64_t ldq, const double* lev, const int32_t* d_ncols, int64_t ncols_max,
                         int64_t n_rows) {
  const bool mixed = h->opt.precision == CTD_PREC_MIXED;
  ProjectArgs pa{};
  pa.fptr = b.fptr;
  pa.row = b.row;
  pa.val = b.val;
  pa.val32 = mixed ? b.val32 : nullptr;
  pa.Q = Q;
  pa.Qf = mixed ? Qf : nullptr;
  pa.ldq = ldq;
  pa.lev = lev;
  pa.fiber_mark = b.fiber_mark;
  pa.d_ncols = d_ncols;
  pa.ncols_max = ncols_max;
  pa.resid = b.resid;
  pa.long_list = b.long_list;
  pa.long_part = b.long_part;
  pa.long_ld = b.long_ld;
  pa.zpart = b.zpart;
  pa.zpart_ld = b.zpart_ld;
  pa.partial = b.partial;
  pa.mixed = mixed;
  pa.n_rows = n_rows;
  pa.hot_id = b.hot_id;
  pa.hot_meta = b.hot_meta;
  pa.GH = b.GH;
  pa.cold_list = b.cold_list;
  return pa;
}

}  // namespace ctd

namespace ctd {

// Device array of basis arguments for up to `count` inputs.
BasisSide* basis_side(ctd_handle* h) {
  if (h->side_state == 0) h->side_state = basis_side_init(&h->side) ? 1 : -1;
  return h->side_state > 0 ? &h->side : nullptr;
}

ctd_status ensure_bdev(ctd_handle* h, int count) {
  if (h->bdev && h->bdev_cap >= count) return CTD_OK;
  if (h->bdev) {
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    (void)hipFree(h->bdev);
    h->bdev = nullptr;
    h->bdev_cap = 0;
  }
  if (dev_alloc(&h->bdev, basis_dev_bytes(count)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, CTD_ERR_OOM, "basis argument array allocation failed");
  }
  h->bdev_cap = count;
  return CTD_OK;
}

// CTD-S up to the basis: workspace, A0-A3 (draws either sampled with Philox
// counter word `tensor`, or given) and the candidate panel (A4); *ba receives
// the arguments of the basis construction.
ctd_status static_front(ctd_handle* h, const ctd_coo* X, const FiberLayout& lay, int64_t s,
                        uint64_t seed, const uint64_t* given, uint32_t tensor, BasisArgs* ba) {
  hipStream_t st = h->stream;
  const bool mixed = h->opt.precision == CTD_PREC_MIXED;
  const bool want_C = h->opt.want_C != 0;
  const int64_t nnz = X->nnz;
  const int64_t n_rows = lay.n_rows;
  StaticBufs& b = h->sb;
  ctd_status rc = plan_static(h, nnz, s, n_rows, mixed, want_C, h->keep_R, round8(s), &b);
  if (rc != CTD_OK) return rc;
  DevScalars* sc = h->d_sc;
  for (bool& u : h->ev_used) u = false;
  mark(h, MARK_START);
  launch_reset_scalars(st, sc, false);
  rc = enqueue_input(h, X, lay, s, seed, 0u, given, b, tensor);
  if (rc != CTD_OK) return rc;
  // A4: candidate panel
  launch_panel(st, b.uniq_fi, s, b.fptr, b.row, b.val, n_rows, b.P, b.ld, sc);
  mark(h, MARK_PANEL);
  // A5-A7: independence filter and orthonormal basis, block by block
  *ba = BasisArgs{};
  ba->P = b.P;
  ba->ldp = b.ld;
  ba->n_rows = n_rows;
  ba->s_max = s;
  ba->k0_max = 0;
  ba->uniq_fi = b.uniq_fi;
  ba->uniq_fid = b.uniq_fid;
  ba->fptr = b.fptr;
  ba->row = b.row;
  ba->val = b.val;
  ba->Q = b.Q;
  ba->ldq = b.ld;
  ba->Qf = mixed ? b.Qf : nullptr;
  ba->R = h->keep_R ? b.Rs : nullptr;
  ba->ldr = b.ld;
  ba->M = b.M;
  ba->ldm = b.ld;
  ba->lev = b.lev;
  ba->lev_accumulate = false;
  ba->eps2 = h->opt.eps * h->opt.eps;
  ba->accept = b.accept;
  ba->acc_fid = b.acc_fid;
  ba->acc_fi_local = nullptr;
  ba->fiber_mark = b.fiber_mark;
  ba->id_offset = 0;
  ba->Wacc = nullptr;
  ba->ldwa = 0;
  ba->scratch = b.scratch;
  ba->cap = b.ld;
  ba->w2_sets = h->w2_sets;
  return CTD_OK;
}

// CTD-S after the basis: A8 projection and residual, C when asked for, totals.
ctd_status static_back(ctd_handle* h, const ctd_coo* X, const FiberLayout& lay, int64_t s) {
  hipStream_t st = h->stream;
  const int64_t nnz = X->nnz;
  const int64_t n_rows = lay.n_rows;
  StaticBufs& b = h->sb;
  DevScalars* sc = h->d_sc;
  // s~ <= min(s, I_alpha): the bound sets the projection's column slices
  ProjectArgs pa = project_args(h, b, b.Q, b.Qf, b.ld, b.lev, &sc->s_tilde, std::min(s, n_rows),
                                n_rows);
  if (h->opt.profile) {
    mark(h, MARK_PROJ0);
    mark(h, MARK_SPMM0);
    mark(h, MARK_SPMM1);
  }
  launch_project(st, pa, nnz, sc, h->opt.profile ? h->ev[MARK_SPMM0] : nullptr,
                 h->opt.profile ? h->ev[MARK_SPMM1] : nullptr);
  mark(h, MARK_PROJECTED);
  if (h->opt.want_C) launch_core_static(st, b, n_rows, nnz, sc);
  mark(h, MARK_CORE);
  launch_static_totals(st, sc);
  mark(h, MARK_END);
  HIP_TRY(h, hipGetLastError());
  h->s = s;
  h->n_rows = n_rows;
  h->nnz_seen = nnz;
  h->step = 0;
  h->has_static = true;
  h->last_was_update = false;
  h->mode = lay.mode;
  h->layout = lay;
  return CTD_OK;
}

// Enqueue CTD-S on `lay`/`X`; draws either sampled (given == nullptr, Philox
// counter word `tensor`) or given.
ctd_status run_static(ctd_handle* h, const ctd_coo* X, const FiberLayout& lay, int64_t s,
                      uint64_t seed, const uint64_t* given, uint32_t tensor) {
  BasisArgs ba{};
  ctd_status rc = static_front(h, X, lay, s, seed, given, tensor, &ba);
  if (rc != CTD_OK) return rc;
  rc = ensure_bdev(h, 1);
  if (rc != CTD_OK) return rc;
  DevScalars* sc = h->d_sc;
  launch_basis(h->stream, &ba, &sc, 1, h->bdev, basis_side(h));
  mark(h, MARK_BASIS);
  return static_back(h, X, lay, s);
}

}  // namespace ctd

namespace {
// Message of the last failed ctd_create on this thread (there is no handle to hold it).
thread_local std::string g_create_error;
}  // namespace

extern "C" {

ctd_status ctd_create(ctd_handle** out, const ctd_options* opt, void* hip_stream) {
  g_create_error.clear();
  if (!out) return CTD_ERR_INVALID_ARG;
  ctd_handle* h = new ctd_handle();
  h->stream = (hipStream_t)hip_stream;
  h->opt.precision = CTD_PREC_FP64;
  h->opt.eps = 1e-6;
  h->opt.want_C = 0;
  h->opt.want_fiber_stats = 0;
  if (opt) {
    if (opt->precision != CTD_PREC_FP64 && opt->precision != CTD_PREC_MIXED) {
      delete h;
      return CTD_ERR_INVALID_ARG;
    }
    if (!(opt->eps >= 0.0) || opt->eps >= 1.0) {
      delete h;
      return CTD_ERR_INVALID_ARG;
    }
    h->opt = *opt;
  }
  const hipError_t e = dev_alloc(&h->d_sc, sizeof(DevScalars));
  if (e != hipSuccess) {
    g_create_error = std::string("hipMalloc of the device scalars: ") + hipGetErrorName(e) + ": " +
                     hipGetErrorString(e);
    (void)hipGetLastError();
    delete h;
    return CTD_ERR_OOM;
  }
  static_assert(sizeof(DevScalars) % 8 == 0, "DevScalars is zeroed as 64-bit words");
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, h->stream, (uint64_t*)h->d_sc,
                     (int64_t)(sizeof(DevScalars) / 8));
  (void)hipGetLastError();
  *out = h;
  return CTD_OK;
}

ctd_status ctd_decompose(ctd_handle* h, const ctd_coo* X, int32_t mode, int64_t s, uint64_t seed) {
  if (!h) return CTD_ERR_INVALID_ARG;
  h->last_error.clear();
  (void)hipGetLastError();
  FiberLayout lay{};
  uint64_t ncols = 0;
  ctd_status rc = check_coo(h, X, mode, &lay, &ncols);
  if (rc != CTD_OK) return rc;
  if (s < 1 || (uint64_t)s > ncols)
    return fail(h, CTD_ERR_INVALID_ARG, "sample size must be in [1, N_alpha]");
  if (s > CTD_MAX_DRAWS)
    return fail(h, CTD_ERR_CAPACITY, "sample size above CTD_MAX_DRAWS");
  if (X->nnz == 0) return fail(h, CTD_ERR_EMPTY, "tensor has no nonzeros");
  h->failed = false;
  h->has_static = false;
  h->dyn_ready = false;
  h->seed = seed;
  rc = run_static(h, X, lay, s, seed, nullptr, 0u);
  if (rc == CTD_OK && h->opt.want_C) rc = dyn_begin(h, X);
  return rc;
}

ctd_status ctd_decompose_given(ctd_handle* h, const ctd_coo* X, int32_t mode,
                               const uint64_t* draws, int64_t s) {
  if (!h) return CTD_ERR_INVALID_ARG;
  h->last_error.clear();
  (void)hipGetLastError();
  FiberLayout lay{};
  uint64_t ncols = 0;
  ctd_status rc = check_coo(h, X, mode, &lay, &ncols);
  if (rc != CTD_OK) return rc;
  if (!draws || s < 1) return fail(h, CTD_ERR_INVALID_ARG, "draws must be a non-empty host array");
  if (s > CTD_MAX_DRAWS) return fail(h, CTD_ERR_CAPACITY, "sample size above CTD_MAX_DRAWS");
  for (int64_t j = 0; j < s; ++j)
    if (draws[j] >= ncols) return fail(h, CTD_ERR_INVALID_ARG, "draw outside [0, N_alpha)");
  if (X->nnz == 0) return fail(h, CTD_ERR_EMPTY, "tensor has no nonzeros");
  h->failed = false;
  h->has_static = false;
  h->dyn_ready = false;
  h->given.assign(draws, draws + s);
  h->seed = 0;
  rc = run_static(h, X, lay, s, 0, h->given.data(), 0u);
  if (rc == CTD_OK && h->opt.want_C) rc = dyn_begin(h, X);
  return rc;
}

ctd_status ctd_sync(ctd_handle* h) {
  if (!h) return CTD_ERR_INVALID_ARG;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  DevScalars sc{};
  HIP_TRY(h, hipMemcpy(&sc, h->d_sc, sizeof(sc), hipMemcpyDeviceToHost));
  if (sc.status != 0) {
    h->failed = true;
    if (h->last_error.empty()) h->last_error = "device reported status " + std::to_string(sc.status);
    return (ctd_status)sc.status;
  }
  return CTD_OK;
}

ctd_status ctd_get_result(ctd_handle* h, ctd_result* out) {
  if (!h || !out) return CTD_ERR_INVALID_ARG;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  DevScalars sc{};
  HIP_TRY(h, hipMemcpy(&sc, h->d_sc, sizeof(sc), hipMemcpyDeviceToHost));
  memset(out, 0, sizeof(*out));
  fill_result(h, sc, out);
  if (sc.status != 0) {
    h->failed = true;
    return (ctd_status)sc.status;
  }
  return CTD_OK;
}

const char* ctd_last_error(const ctd_handle* h) {
  if (h) return h->last_error.c_str();
  return g_create_error.empty() ? "null handle" : g_create_error.c_str();
}

void ctd_destroy(ctd_handle* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  if (h->xstream) (void)hipStreamSynchronize(h->xstream);
  if (h->batch) {
    ctd::BatchState* B = h->batch;
    for (hipStream_t st : B->pool) (void)hipStreamSynchronize(st);
    for (ctd_handle* sub : B->subs) ctd_destroy(sub);   // their streams belong to the pool
    for (hipEvent_t e : B->done) (void)hipEventDestroy(e);
    if (B->start) (void)hipEventDestroy(B->start);
    if (B->based) (void)hipEventDestroy(B->based);
    for (hipStream_t st : B->pool) (void)hipStreamDestroy(st);
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->cap) {
      (void)hipStreamSynchronize(B->cap);
      (void)hipStreamDestroy(B->cap);
    }
    if (B->fork) (void)hipEventDestroy(B->fork);
    if (B->join) (void)hipEventDestroy(B->join);
    ctd::batch_free_storage(B);
    delete B;
  }
  for (hipEvent_t& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  dyn_free(h);
  if (h->bdev) (void)hipFree(h->bdev);
  if (h->side_state > 0) basis_side_free(&h->side);
  if (h->xstream) (void)hipStreamDestroy(h->xstream);
  if (h->xfork) (void)hipEventDestroy(h->xfork);
  if (h->xjoin) (void)hipEventDestroy(h->xjoin);
  if (h->arena.base) (void)hipFree(h->arena.base);
  if (h->d_sc) (void)hipFree(h->d_sc);
  delete h;
}

}  // extern "C"

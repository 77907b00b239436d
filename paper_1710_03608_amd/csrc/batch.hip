// Many independent tensors in one call (the batched execution form): every
// tensor gets the CTD-S path of Algorithm 1, its draws using Philox counter
// word tensor = b.  Tensors are spread over kBatchStreams sub-handles, each
// with a stream of its own (default priority), so the small per-block
// kernels of different tensors overlap on the GPU.  The caller's stream is
// joined with events at entry and exit.  After each tensor its scalars and
// index arrays are copied (on the tensor's stream) into storage owned by the
// batch, so a sub-handle's workspace can take the next tensor at once.
#include <string>
#include <vector>

#include "state.h"

namespace ctd {

namespace {
constexpr int kBatchStreams = 8;

#define BATCH_HIP(h, expr)                                                              \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(h, CTD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

ctd_status new_sub(ctd_handle* h, ctd_handle** out) {
  ctd_handle* sub = new ctd_handle();
  sub->opt = h->opt;
  sub->opt.want_C = 0;
  sub->opt.profile = 0;
  if (hipStreamCreateWithFlags(&sub->stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    delete sub;
    return fail(h, CTD_ERR_HIP, "stream creation for a batch failed");
  }
  sub->own_stream = true;
  if (hipMalloc(&sub->d_sc, sizeof(DevScalars)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamDestroy(sub->stream);
    delete sub;
    return fail(h, CTD_ERR_OOM, "batch scalar allocation failed");
  }
  (void)hipMemsetAsync(sub->d_sc, 0, sizeof(DevScalars), sub->stream);
  *out = sub;
  return CTD_OK;
}

ctd_status sync_all(ctd_handle* h) {
  BATCH_HIP(h, hipStreamSynchronize(h->stream));
  if (h->batch)
    for (ctd_handle* sub : h->batch->subs) BATCH_HIP(h, hipStreamSynchronize(sub->stream));
  return CTD_OK;
}
}  // namespace

void batch_free_storage(BatchState* B) {
  if (B->scal) (void)hipFree(B->scal);
  if (B->draws) (void)hipFree(B->draws);
  if (B->unique) (void)hipFree(B->unique);
  if (B->accepted) (void)hipFree(B->accepted);
  if (B->counts) (void)hipFree(B->counts);
  if (B->prob) (void)hipFree(B->prob);
  if (B->scale) (void)hipFree(B->scale);
  B->scal = nullptr;
  B->draws = B->unique = B->accepted = nullptr;
  B->counts = nullptr;
  B->prob = B->scale = nullptr;
  B->cap_t = B->cap_s = 0;
}

}  // namespace ctd

using namespace ctd;

extern "C" ctd_status ctd_decompose_batched(ctd_handle* h, const ctd_coo* Xs, int32_t nb,
                                            int32_t mode, const int64_t* s, uint64_t seed) {
  if (!h) return CTD_ERR_INVALID_ARG;
  h->last_error.clear();
  (void)hipGetLastError();
  if (nb < 1 || nb > CTD_MAX_TENSORS || !Xs || !s)
    return fail(h, CTD_ERR_INVALID_ARG, "B must be in [1, CTD_MAX_TENSORS] with tensors and sizes");
  std::vector<FiberLayout> lays(nb);
  int64_t total_s = 0;
  for (int b = 0; b < nb; ++b) {
    uint64_t ncols = 0;
    ctd_status rc = check_coo(h, &Xs[b], mode, &lays[b], &ncols);
    if (rc != CTD_OK) return rc;
    if (s[b] < 1 || (uint64_t)s[b] > ncols)
      return fail(h, CTD_ERR_INVALID_ARG, "tensor " + std::to_string(b) + ": sample size must be in [1, N_alpha]");
    if (s[b] > CTD_MAX_DRAWS)
      return fail(h, CTD_ERR_CAPACITY, "tensor " + std::to_string(b) + ": sample size above CTD_MAX_DRAWS");
    if (Xs[b].nnz == 0) return fail(h, CTD_ERR_EMPTY, "tensor " + std::to_string(b) + " has no nonzeros");
    total_s += s[b];
  }
  if (!h->batch) h->batch = new BatchState();
  BatchState& B = *h->batch;
  const int K = std::min(kBatchStreams, (int)nb);
  while ((int)B.subs.size() < K) {
    ctd_handle* sub = nullptr;
    ctd_status rc = new_sub(h, &sub);
    if (rc != CTD_OK) return rc;
    B.subs.push_back(sub);
    hipEvent_t e = nullptr;
    BATCH_HIP(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    B.done.push_back(e);
  }
  for (ctd_handle* sub : B.subs) {
    if (sub->opt.precision != h->opt.precision || sub->opt.eps != h->opt.eps) {
      BATCH_HIP(h, hipStreamSynchronize(sub->stream));
      sub->opt.precision = h->opt.precision;
      sub->opt.eps = h->opt.eps;
    }
  }
  if (!B.start) BATCH_HIP(h, hipEventCreateWithFlags(&B.start, hipEventDisableTiming));
  // per-tensor result storage
  if ((size_t)nb > B.cap_t || (size_t)total_s > B.cap_s) {
    ctd_status rc = sync_all(h);
    if (rc != CTD_OK) return rc;
    batch_free_storage(&B);
    const size_t nt = (size_t)nb, ns = (size_t)std::max<int64_t>(total_s, 1);
    bool ok = hipMalloc(&B.scal, nt * sizeof(DevScalars)) == hipSuccess &&
              hipMalloc(&B.draws, ns * 8) == hipSuccess &&
              hipMalloc(&B.unique, ns * 8) == hipSuccess &&
              hipMalloc(&B.accepted, ns * 8) == hipSuccess &&
              hipMalloc(&B.counts, ns * 4) == hipSuccess &&
              hipMalloc(&B.prob, ns * 8) == hipSuccess &&
              hipMalloc(&B.scale, ns * 8) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      batch_free_storage(&B);
      return fail(h, CTD_ERR_OOM, "batch result storage allocation failed");
    }
    B.cap_t = nt;
    B.cap_s = ns;
  }
  B.B = nb;
  B.s.assign(s, s + nb);
  B.off.resize(nb);
  B.rows.resize(nb);
  int64_t o = 0;
  for (int b = 0; b < nb; ++b) {
    B.off[b] = o;
    B.rows[b] = lays[b].n_rows;
    o += s[b];
  }
  B.host_valid = false;
  // tensors start after the caller's earlier work on its stream
  BATCH_HIP(h, hipEventRecord(B.start, h->stream));
  for (int k = 0; k < K; ++k) BATCH_HIP(h, hipStreamWaitEvent(B.subs[k]->stream, B.start, 0));
  for (int b = 0; b < nb; ++b) {
    ctd_handle* sub = B.subs[b % K];
    sub->failed = false;
    ctd_status rc = run_static(sub, &Xs[b], lays[b], s[b], seed, nullptr, (uint32_t)b);
    if (rc != CTD_OK)
      return fail(h, rc, "tensor " + std::to_string(b) + ": " + sub->last_error);
    const StaticBufs& sb = sub->sb;
    hipStream_t st = sub->stream;
    const size_t n = (size_t)s[b], off = (size_t)B.off[b];
    BATCH_HIP(h, hipMemcpyAsync(B.scal + b, sub->d_sc, sizeof(DevScalars), hipMemcpyDeviceToDevice, st));
    BATCH_HIP(h, hipMemcpyAsync(B.draws + off, sb.draw_fid, n * 8, hipMemcpyDeviceToDevice, st));
    BATCH_HIP(h, hipMemcpyAsync(B.unique + off, sb.uniq_fid, n * 8, hipMemcpyDeviceToDevice, st));
    BATCH_HIP(h, hipMemcpyAsync(B.accepted + off, sb.acc_fid, n * 8, hipMemcpyDeviceToDevice, st));
    BATCH_HIP(h, hipMemcpyAsync(B.counts + off, sb.counts, n * 4, hipMemcpyDeviceToDevice, st));
    BATCH_HIP(h, hipMemcpyAsync(B.prob + off, sb.prob, n * 8, hipMemcpyDeviceToDevice, st));
    BATCH_HIP(h, hipMemcpyAsync(B.scale + off, sb.scale, n * 8, hipMemcpyDeviceToDevice, st));
  }
  // the caller's stream continues after every tensor
  for (int k = 0; k < K; ++k) {
    BATCH_HIP(h, hipEventRecord(B.done[k], B.subs[k]->stream));
    BATCH_HIP(h, hipStreamWaitEvent(h->stream, B.done[k], 0));
  }
  return CTD_OK;
}

extern "C" ctd_status ctd_get_batch_result(ctd_handle* h, int32_t b, ctd_result* out) {
  if (!h) return CTD_ERR_INVALID_ARG;
  if (!out) return fail(h, CTD_ERR_INVALID_ARG, "null result");
  if (!h->batch || h->batch->B == 0) return fail(h, CTD_ERR_STATE, "no batched decomposition held");
  BatchState& B = *h->batch;
  if (b < 0 || b >= B.B) return fail(h, CTD_ERR_INVALID_ARG, "tensor index out of range");
  BATCH_HIP(h, hipStreamSynchronize(h->stream));
  if (!B.host_valid) {
    B.host.resize(B.B);
    BATCH_HIP(h, hipMemcpy(B.host.data(), B.scal, (size_t)B.B * sizeof(DevScalars),
                           hipMemcpyDeviceToHost));
    B.host_valid = true;
  }
  const DevScalars& sc = B.host[b];
  *out = ctd_result{};
  out->s = B.s[b];
  out->s_unique = sc.s_unique;
  out->s_tilde = sc.s_tilde;
  out->n_f = sc.n_f;
  out->n_rows = B.rows[b];
  out->step = 0;
  out->weight_total = sc.W;
  out->norm2 = sc.norm2;
  out->err2 = sc.err2;
  out->rel_err = sc.norm2 > 0 ? sc.err2 / sc.norm2 : 0.0;
  out->slice_err2 = 0.0;
  out->status = sc.status;
  const size_t off = (size_t)B.off[b];
  out->draws = B.draws + off;
  out->unique = B.unique + off;
  out->counts = B.counts + off;
  out->prob = B.prob + off;
  out->scale = B.scale + off;
  out->accepted = B.accepted + off;
  return sc.status ? (ctd_status)sc.status : CTD_OK;
}

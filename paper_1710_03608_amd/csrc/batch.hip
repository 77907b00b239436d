// Many independent tensors in one call (the batched execution form): every
// tensor gets the CTD-S path of Algorithm 1, its draws using Philox counter
// word tensor = b.  Tensors go in groups that fit a device-memory budget, one
// sub-handle (own workspace and scalars) per tensor of a group.  The
// per-tensor stages before and after the basis (keys, sort, weights, draws,
// unique, panel; projection and residual) run on a pool of kBatchStreams
// streams (default priority); the independence filter and basis of the whole
// group, the long sequential part, is one sequence of launches whose grids
// span all tensors of the group.  The caller's stream is joined with events
// at entry and exit.  After each tensor its scalars and index arrays are
// copied into storage owned by the batch.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "state.h"

namespace ctd {

namespace {
constexpr int kBatchStreams = 8;
constexpr int kMaxGroup = 4096;                      // tensors per group
// workspace budget per group: under half of the 288 GB of HBM, so that a
// group of hundreds of mid-sized tensors is one sequence of launches
constexpr size_t kGroupBytes = size_t(128) << 30;

#define BATCH_HIP(h, expr)                                                              \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(h, CTD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

ctd_status new_sub(ctd_handle* h, ctd_handle** out) {
  ctd_handle* sub = new ctd_handle();
  sub->opt = h->opt;
  sub->keep_R = false;
  sub->w2_sets = 1;
  if (dev_alloc(&sub->d_sc, sizeof(DevScalars)) != hipSuccess) {
    (void)hipGetLastError();
    delete sub;
    return fail(h, CTD_ERR_OOM, "batch scalar allocation failed");
  }
  *out = sub;
  return CTD_OK;
}

ctd_status sync_all(ctd_handle* h) {
  BATCH_HIP(h, hipStreamSynchronize(h->stream));
  if (h->batch)
    for (hipStream_t st : h->batch->pool) BATCH_HIP(h, hipStreamSynchronize(st));
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

namespace {
// Everything a batched call's launches depend on: the options, mode and seed,
// and per tensor its shape, nonzero count, sample size and input pointers.
std::vector<uint64_t> batch_signature(const ctd_handle* h, const ctd_coo* Xs, int32_t nb,
                                      int32_t mode, const int64_t* s, uint64_t seed) {
  std::vector<uint64_t> g;
  uint64_t eps_bits = 0;
  static_assert(sizeof(eps_bits) == sizeof(h->opt.eps), "eps is a double");
  memcpy(&eps_bits, &h->opt.eps, sizeof(eps_bits));
  g.insert(g.end(), {(uint64_t)nb, (uint64_t)(uint32_t)mode, seed, (uint64_t)h->opt.precision, eps_bits,
                     (uint64_t)h->opt.want_C, (uint64_t)h->opt.want_fiber_stats,
                     (uint64_t)h->opt.profile});
  for (int b = 0; b < nb; ++b) {
    const ctd_coo& X = Xs[b];
    g.insert(g.end(), {(uint64_t)X.order, (uint64_t)X.nnz, (uint64_t)(uintptr_t)X.idx,
                       (uint64_t)(uintptr_t)X.val, (uint64_t)X.val_dtype, (uint64_t)s[b]});
    for (int m = 0; m < X.order; ++m) g.push_back((uint64_t)X.dims[m]);
  }
  return g;
}

void drop_graph(BatchState& B) {
  if (B.exec) (void)hipGraphExecDestroy(B.exec);
  B.exec = nullptr;
  B.graph_sig.clear();
}

ctd_status batched_body(ctd_handle* h, const ctd_coo* Xs, int32_t nb, int32_t mode,
                        const int64_t* s, uint64_t seed, const std::vector<FiberLayout>& lays,
                        int64_t total_s);
}  // namespace

// Host checks, then the launches of the call, or the replay of a graph of
// them: a call with the same signature as the call before it is captured
// (its work then runs as a graph launch), and later calls with that
// signature replay the graph.  Capture and replay run on a stream of the
// batch state that forks from the caller's stream and joins it again, so the
// caller's stream is never captured itself (the legacy default stream cannot
// be).  Between calls nothing the launches read on the host changes: with
// the same sizes no workspace is reallocated, and the autotuner's choices
// were settled by the earlier calls.  Any failure of capture, instantiation
// or launch falls back to direct launches on the caller's stream.

// Replays B.exec on B.cap between a fork from and a join to the caller's stream.
bool replay(BatchState& B, hipStream_t user) {
  return hipEventRecord(B.fork, user) == hipSuccess &&
         hipStreamWaitEvent(B.cap, B.fork, 0) == hipSuccess &&
         hipGraphLaunch(B.exec, B.cap) == hipSuccess &&
         hipEventRecord(B.join, B.cap) == hipSuccess &&
         hipStreamWaitEvent(user, B.join, 0) == hipSuccess;
}

// The stream and events a capture uses, created at the first capture.
bool capture_objects(BatchState& B) {
  if (!B.cap && hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking) != hipSuccess) {
    B.cap = nullptr;
    return false;
  }
  if (!B.fork && hipEventCreateWithFlags(&B.fork, hipEventDisableTiming) != hipSuccess) {
    B.fork = nullptr;
    return false;
  }
  if (!B.join && hipEventCreateWithFlags(&B.join, hipEventDisableTiming) != hipSuccess) {
    B.join = nullptr;
    return false;
  }
  return true;
}
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
  std::vector<uint64_t> sig = batch_signature(h, Xs, nb, mode, s, seed);
  if (B.exec && sig == B.graph_sig) {
    if (replay(B, h->stream)) {
      B.host_valid = false;
      ++B.graph_launches;
      return CTD_OK;
    }
    (void)hipGetLastError();
    (void)hipStreamSynchronize(B.cap);
    drop_graph(B);
  }
  drop_graph(B);
  const char* off = getenv("CTD_NO_GRAPH");
  const bool capture = sig == B.last_sig && !(off && *off && *off != '0');
  B.last_sig = sig;
  if (!capture || !capture_objects(B)) {
    (void)hipGetLastError();
    return batched_body(h, Xs, nb, mode, s, seed, lays, total_s);
  }
  hipStream_t user = h->stream;
  if (hipEventRecord(B.fork, user) != hipSuccess || hipStreamWaitEvent(B.cap, B.fork, 0) != hipSuccess ||
      hipStreamBeginCapture(B.cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    return batched_body(h, Xs, nb, mode, s, seed, lays, total_s);
  }
  h->stream = B.cap;
  ctd_status rc = batched_body(h, Xs, nb, mode, s, seed, lays, total_s);
  h->stream = user;
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(B.cap, &g);
  hipGraphExec_t x = nullptr;
  bool ok = rc == CTD_OK && ec == hipSuccess && g &&
            hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (ok) {
    B.exec = x;
    B.graph_sig = sig;
    if (replay(B, user)) {
      ++B.graph_launches;
      return CTD_OK;
    }
    B.exec = nullptr;
    B.graph_sig.clear();
  }
  // nothing of the captured work ran: run it directly
  (void)hipGetLastError();
  if (x) (void)hipGraphExecDestroy(x);
  B.last_sig.clear();
  h->last_error.clear();
  return batched_body(h, Xs, nb, mode, s, seed, lays, total_s);
}

namespace {
ctd_status batched_body(ctd_handle* h, const ctd_coo* Xs, int32_t nb, int32_t mode,
                        const int64_t* s, uint64_t seed, const std::vector<FiberLayout>& lays,
                        int64_t total_s) {
  BatchState& B = *h->batch;
  while ((int)B.pool.size() < kBatchStreams) {
    hipStream_t st = nullptr;
    BATCH_HIP(h, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    B.pool.push_back(st);
    hipEvent_t e = nullptr;
    BATCH_HIP(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    B.done.push_back(e);
  }
  if (!B.start) BATCH_HIP(h, hipEventCreateWithFlags(&B.start, hipEventDisableTiming));
  if (!B.based) BATCH_HIP(h, hipEventCreateWithFlags(&B.based, hipEventDisableTiming));
  const int K = kBatchStreams;
  // per-tensor result storage
  if ((size_t)nb > B.cap_t || (size_t)total_s > B.cap_s) {
    ctd_status rc = sync_all(h);
    if (rc != CTD_OK) return rc;
    batch_free_storage(&B);
    const size_t nt = (size_t)nb, ns = (size_t)std::max<int64_t>(total_s, 1);
    bool ok = dev_alloc(&B.scal, nt * sizeof(DevScalars)) == hipSuccess &&
              dev_alloc(&B.draws, ns * 8) == hipSuccess &&
              dev_alloc(&B.unique, ns * 8) == hipSuccess &&
              dev_alloc(&B.accepted, ns * 8) == hipSuccess &&
              dev_alloc(&B.counts, ns * 4) == hipSuccess &&
              dev_alloc(&B.prob, ns * 8) == hipSuccess &&
              dev_alloc(&B.scale, ns * 8) == hipSuccess;
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
  const bool mixed = h->opt.precision == CTD_PREC_MIXED;
  // tensors start after the caller's earlier work on its stream
  BATCH_HIP(h, hipEventRecord(B.start, h->stream));
  for (int k = 0; k < K; ++k) BATCH_HIP(h, hipStreamWaitEvent(B.pool[k], B.start, 0));
  std::vector<BasisArgs> args;
  std::vector<DevScalars*> scs;
  for (int g0 = 0; g0 < nb;) {
    // the group: consecutive tensors within the workspace budget
    int g1 = g0;
    size_t bytes = 0;
    while (g1 < nb && g1 - g0 < kMaxGroup) {
      const size_t t = static_bytes(Xs[g1].nnz, s[g1], lays[g1].n_rows, mixed, false, false,
                                    round8(s[g1]));
      if (g1 > g0 && bytes + t > kGroupBytes) break;
      bytes += t;
      ++g1;
    }
    const int n = g1 - g0;
    while ((int)B.subs.size() < n) {
      ctd_handle* sub = nullptr;
      ctd_status rc = new_sub(h, &sub);
      if (rc != CTD_OK) return rc;
      sub->stream = B.pool[B.subs.size() % K];
      B.subs.push_back(sub);
    }
    args.assign(n, BasisArgs{});
    scs.assign(n, nullptr);
    for (int i = 0; i < n; ++i) {
      const int b = g0 + i;
      ctd_handle* sub = B.subs[i];   // always on stream pool[i % K]
      sub->opt = h->opt;
      sub->opt.want_C = 0;
      sub->opt.profile = 0;
      sub->failed = false;
      ctd_status rc = static_front(sub, &Xs[b], lays[b], s[b], seed, nullptr, (uint32_t)b, &args[i]);
      if (rc != CTD_OK)
        return fail(h, rc, "tensor " + std::to_string(b) + ": " + sub->last_error);
      scs[i] = sub->d_sc;
    }
    // the group's basis on the caller's stream, after every tensor's panel
    for (int k = 0; k < K; ++k) {
      BATCH_HIP(h, hipEventRecord(B.done[k], B.pool[k]));
      BATCH_HIP(h, hipStreamWaitEvent(h->stream, B.done[k], 0));
    }
    ctd_status rc = ensure_bdev(h, n);
    if (rc != CTD_OK) return rc;
    launch_basis(h->stream, args.data(), scs.data(), n, h->bdev, basis_side(h));
    BATCH_HIP(h, hipGetLastError());
    BATCH_HIP(h, hipEventRecord(B.based, h->stream));
    for (int k = 0; k < K; ++k) BATCH_HIP(h, hipStreamWaitEvent(B.pool[k], B.based, 0));
    for (int i = 0; i < n; ++i) {
      const int b = g0 + i;
      ctd_handle* sub = B.subs[i];
      rc = static_back(sub, &Xs[b], lays[b], s[b]);
      if (rc != CTD_OK)
        return fail(h, rc, "tensor " + std::to_string(b) + ": " + sub->last_error);
      const StaticBufs& sb = sub->sb;
      hipStream_t st = sub->stream;
      const size_t ns = (size_t)s[b], off = (size_t)B.off[b];
      BATCH_HIP(h, hipMemcpyAsync(B.scal + b, sub->d_sc, sizeof(DevScalars), hipMemcpyDeviceToDevice, st));
      BATCH_HIP(h, hipMemcpyAsync(B.draws + off, sb.draw_fid, ns * 8, hipMemcpyDeviceToDevice, st));
      BATCH_HIP(h, hipMemcpyAsync(B.unique + off, sb.uniq_fid, ns * 8, hipMemcpyDeviceToDevice, st));
      BATCH_HIP(h, hipMemcpyAsync(B.accepted + off, sb.acc_fid, ns * 8, hipMemcpyDeviceToDevice, st));
      BATCH_HIP(h, hipMemcpyAsync(B.counts + off, sb.counts, ns * 4, hipMemcpyDeviceToDevice, st));
      BATCH_HIP(h, hipMemcpyAsync(B.prob + off, sb.prob, ns * 8, hipMemcpyDeviceToDevice, st));
      BATCH_HIP(h, hipMemcpyAsync(B.scale + off, sb.scale, ns * 8, hipMemcpyDeviceToDevice, st));
    }
    g0 = g1;
  }
  // the caller's stream continues after every tensor
  for (int k = 0; k < K; ++k) {
    BATCH_HIP(h, hipEventRecord(B.done[k], B.pool[k]));
    BATCH_HIP(h, hipStreamWaitEvent(h->stream, B.done[k], 0));
  }
  return CTD_OK;
}

}  // namespace

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

extern "C" int64_t ctd_batch_graph_launches(const ctd_handle* h) {
  return h && h->batch ? h->batch->graph_launches : 0;
}

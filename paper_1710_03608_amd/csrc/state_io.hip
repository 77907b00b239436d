// Checkpoint and resume of a CTD-D stream.  Algorithm 2 carries R, U and C
// (and the stream's error and norm) from one time step to the next; the
// library holds them as R (kept fibers), the orthonormal Q = R M with its
// upper-triangular M (U = M M^T), the row leverages ||Q_i||^2, C and the fiber
// ids of R's and C's columns.  ctd_save_state copies all of it, with the
// handle's host-side sizes and bounds, into a caller's host buffer;
// ctd_load_state puts it back into a handle, so the stream continues with
// the same launches and the same bits as if it had never stopped.
//
// Buffer layout (native byte order, version 1): the header below, then the
// arrays, each starting at a multiple of 64 bytes:
//   R, Q   [n_rows x d] float64 row-major (d = kept fibers)
//   Qf     [n_rows x d] float32 row-major (mixed-precision handles only)
//   M      [d x d] float64 row-major (upper triangle meaningful)
//   lev    [n_rows] float64
//   acc    [d] uint64 kept fiber ids, col [n_cols] uint64 column fiber ids
//   C      [n_cols x d] column-major, float64 (float32 for mixed handles)
#include <string.h>

#include <string>

#include "state.h"

using namespace ctd;

namespace {

constexpr char kMagic[8] = {'C', 'T', 'D', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t kVersion = 1;

struct StateHeader {
  char magic[8];
  uint32_t version;
  uint32_t header_bytes;
  uint32_t layout_bytes;
  uint32_t scalars_bytes;
  uint64_t total_bytes;
  int32_t precision;
  int32_t mode;
  double eps;
  FiberLayout layout;
  uint64_t seed;
  int64_t n_rows, step, nnz_seen;
  int64_t capD, capN, d_tilde, n_cols, d_ub, n_cols_ub, T, dN;
  DevScalars sc;
};

size_t up64(size_t x) { return (x + 63) & ~size_t(63); }

struct Sections {
  size_t R, Q, Qf, M, lev, acc, col, C, total;
};

Sections sections(int64_t n_rows, int64_t d, int64_t n_cols, bool mixed) {
  Sections s{};
  size_t o = up64(sizeof(StateHeader));
  s.R = o;   o = up64(o + (size_t)n_rows * d * 8);
  s.Q = o;   o = up64(o + (size_t)n_rows * d * 8);
  s.Qf = o;  o = up64(o + (mixed ? (size_t)n_rows * d * 4 : 0));
  s.M = o;   o = up64(o + (size_t)d * d * 8);
  s.lev = o; o = up64(o + (size_t)n_rows * 8);
  s.acc = o; o = up64(o + (size_t)d * 8);
  s.col = o; o = up64(o + (size_t)n_cols * 8);
  s.C = o;   o = up64(o + (size_t)n_cols * d * (mixed ? 4 : 8));
  s.total = o;
  return s;
}

#define IO_HIP(h, expr)                                                               \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess)                                                             \
      return fail(h, CTD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

}  // namespace

extern "C" ctd_status ctd_save_state(ctd_handle* h, void* host_buf, size_t* bytes) {
  if (!h || !bytes) return CTD_ERR_INVALID_ARG;
  h->last_error.clear();
  if (h->failed) return fail(h, CTD_ERR_STATE, "handle is in a failed state");
  if (!h->dyn_ready) return fail(h, CTD_ERR_STATE, "no CTD-D stream held (ctd_decompose with want_C on a non-time mode)");
  IO_HIP(h, hipStreamSynchronize(h->stream));
  DevScalars sc{};
  IO_HIP(h, hipMemcpy(&sc, h->d_sc, sizeof(sc), hipMemcpyDeviceToHost));
  if (sc.status != 0) return fail(h, (ctd_status)sc.status, "device reported an error");
  const DynState& S = h->dyn;
  const int64_t d = sc.n_accept_total, nc = sc.n_cols_total, n_rows = h->n_rows;
  const bool mixed = S.Cf != nullptr;
  const Sections sec = sections(n_rows, d, nc, mixed);
  const size_t cap = *bytes;
  *bytes = sec.total;
  if (!host_buf) return CTD_OK;
  if (cap < sec.total)
    return fail(h, CTD_ERR_CAPACITY, "state needs " + std::to_string(sec.total) + " bytes");
  char* out = (char*)host_buf;
  StateHeader hd;
  memset(&hd, 0, sizeof(hd));
  memcpy(hd.magic, kMagic, sizeof(kMagic));
  hd.version = kVersion;
  hd.header_bytes = sizeof(StateHeader);
  hd.layout_bytes = sizeof(FiberLayout);
  hd.scalars_bytes = sizeof(DevScalars);
  hd.total_bytes = sec.total;
  hd.precision = h->opt.precision;
  hd.mode = h->mode;
  hd.eps = h->opt.eps;
  hd.layout = h->layout;
  hd.seed = h->seed;
  hd.n_rows = n_rows;
  hd.step = h->step;
  hd.nnz_seen = h->nnz_seen;
  hd.capD = S.capD;
  hd.capN = S.capN;
  hd.d_tilde = d;
  hd.n_cols = nc;
  hd.d_ub = S.d_ub;
  hd.n_cols_ub = S.n_cols_ub;
  hd.T = S.T;
  hd.dN = S.dN;
  hd.sc = sc;
  memset(out, 0, up64(sizeof(StateHeader)));
  memcpy(out, &hd, sizeof(hd));
  hipStream_t st = h->stream;
  if (d > 0) {
    IO_HIP(h, hipMemcpy2DAsync(out + sec.R, d * 8, S.Rs, S.capD * 8, d * 8, n_rows,
                               hipMemcpyDeviceToHost, st));
    IO_HIP(h, hipMemcpy2DAsync(out + sec.Q, d * 8, S.Q, S.capD * 8, d * 8, n_rows,
                               hipMemcpyDeviceToHost, st));
    if (mixed)
      IO_HIP(h, hipMemcpy2DAsync(out + sec.Qf, d * 4, S.Qf, S.capD * 4, d * 4, n_rows,
                                 hipMemcpyDeviceToHost, st));
    IO_HIP(h, hipMemcpy2DAsync(out + sec.M, d * 8, S.Xt, S.capD * 8, d * 8, d,
                               hipMemcpyDeviceToHost, st));
    IO_HIP(h, hipMemcpyAsync(out + sec.acc, S.acc_fid, d * 8, hipMemcpyDeviceToHost, st));
  }
  IO_HIP(h, hipMemcpyAsync(out + sec.lev, S.lev, n_rows * 8, hipMemcpyDeviceToHost, st));
  if (nc > 0) {
    IO_HIP(h, hipMemcpyAsync(out + sec.col, S.col_fid, nc * 8, hipMemcpyDeviceToHost, st));
    if (d > 0) {
      const size_t es = mixed ? 4 : 8;
      IO_HIP(h, hipMemcpy2DAsync(out + sec.C, d * es, mixed ? (const void*)S.Cf : (const void*)S.C,
                                 S.capD * es, d * es, nc, hipMemcpyDeviceToHost, st));
    }
  }
  IO_HIP(h, hipStreamSynchronize(st));
  return CTD_OK;
}

extern "C" ctd_status ctd_load_state(ctd_handle* h, const void* host_buf, size_t bytes) {
  if (!h || !host_buf) return CTD_ERR_INVALID_ARG;
  h->last_error.clear();
  (void)hipGetLastError();
  if (bytes < sizeof(StateHeader)) return fail(h, CTD_ERR_INVALID_ARG, "buffer shorter than a state header");
  StateHeader hd;
  memcpy(&hd, host_buf, sizeof(hd));
  if (memcmp(hd.magic, kMagic, sizeof(kMagic)) != 0 || hd.version != kVersion ||
      hd.header_bytes != sizeof(StateHeader) || hd.layout_bytes != sizeof(FiberLayout) ||
      hd.scalars_bytes != sizeof(DevScalars))
    return fail(h, CTD_ERR_INVALID_ARG, "not a state written by this library version");
  const bool mixed = hd.precision == CTD_PREC_MIXED;
  if (hd.n_rows < 1 || hd.d_tilde < 0 || hd.d_tilde > hd.capD || hd.capD > ((hd.n_rows + 7) & ~int64_t(7)) ||
      hd.n_cols < 0 || hd.n_cols > hd.capN || hd.d_ub < hd.d_tilde || hd.n_cols_ub < hd.n_cols ||
      hd.layout.order < 2 || hd.layout.order > CTD_MAX_ORDER || hd.mode != hd.layout.mode ||
      hd.mode < 0 || hd.mode >= hd.layout.order - 1 || hd.layout.n_rows != hd.n_rows ||
      hd.sc.n_accept_total != hd.d_tilde || hd.sc.n_cols_total != hd.n_cols)
    return fail(h, CTD_ERR_INVALID_ARG, "inconsistent state header");
  const Sections sec = sections(hd.n_rows, hd.d_tilde, hd.n_cols, mixed);
  if (hd.total_bytes != sec.total || bytes < sec.total)
    return fail(h, CTD_ERR_INVALID_ARG, "state buffer is truncated");
  if (hd.precision != h->opt.precision || hd.eps != h->opt.eps || !h->opt.want_C)
    return fail(h, CTD_ERR_STATE, "the handle's precision and eps must equal the saved ones, and want_C be set");
  IO_HIP(h, hipStreamSynchronize(h->stream));
  // the handle's previous stream (if any) is dropped
  dyn_free(h);
  h->has_static = false;
  h->last_was_update = false;
  h->failed = false;
  h->layout = hd.layout;
  h->mode = hd.mode;
  h->n_rows = hd.n_rows;
  h->seed = hd.seed;
  h->step = hd.step;
  h->nnz_seen = hd.nnz_seen;
  h->s = 0;
  ctd_status rc = dyn_resize(h, hd.capD, hd.capN);
  if (rc != CTD_OK) return rc;
  DynState& S = h->dyn;
  if (S.capD != hd.capD || S.capN != hd.capN) {
    dyn_free(h);
    return fail(h, CTD_ERR_STATE, "capacities differ from the saved ones");
  }
  const char* in = (const char*)host_buf;
  const int64_t d = hd.d_tilde, nc = hd.n_cols, n_rows = hd.n_rows;
  hipStream_t st = h->stream;
  if (d > 0) {
    IO_HIP(h, hipMemcpy2DAsync(S.Rs, S.capD * 8, in + sec.R, d * 8, d * 8, n_rows,
                               hipMemcpyHostToDevice, st));
    IO_HIP(h, hipMemcpy2DAsync(S.Q, S.capD * 8, in + sec.Q, d * 8, d * 8, n_rows,
                               hipMemcpyHostToDevice, st));
    if (mixed)
      IO_HIP(h, hipMemcpy2DAsync(S.Qf, S.capD * 4, in + sec.Qf, d * 4, d * 4, n_rows,
                                 hipMemcpyHostToDevice, st));
    IO_HIP(h, hipMemcpy2DAsync(S.Xt, S.capD * 8, in + sec.M, d * 8, d * 8, d,
                               hipMemcpyHostToDevice, st));
    IO_HIP(h, hipMemcpyAsync(S.acc_fid, in + sec.acc, d * 8, hipMemcpyHostToDevice, st));
  }
  IO_HIP(h, hipMemcpyAsync(S.lev, in + sec.lev, n_rows * 8, hipMemcpyHostToDevice, st));
  if (nc > 0) {
    IO_HIP(h, hipMemcpyAsync(S.col_fid, in + sec.col, nc * 8, hipMemcpyHostToDevice, st));
    if (d > 0) {
      const size_t es = mixed ? 4 : 8;
      IO_HIP(h, hipMemcpy2DAsync(mixed ? (void*)S.Cf : (void*)S.C, S.capD * es, in + sec.C, d * es,
                                 d * es, nc, hipMemcpyHostToDevice, st));
    }
  }
  // the stream's totals carry over; the last call's per-input fields do not
  DevScalars sc = hd.sc;
  sc.W = 0;
  sc.vmax2_bits = 0;
  sc.norm2 = 0.0;
  sc.err2 = 0.0;
  sc.status = 0;
  sc.sigma = 0;
  sc.n_f = 0;
  sc.s_unique = 0;
  sc.s_tilde = 0;
  sc.base_accept = 0;
  sc.n_long = 0;
  sc.blk_na = 0;
  sc.blk_reorth = 0;
  sc.allow_empty = 1;
  IO_HIP(h, hipMemcpyAsync(h->d_sc, &sc, sizeof(sc), hipMemcpyHostToDevice, st));
  IO_HIP(h, hipStreamSynchronize(st));
  S.d_tilde = d;
  S.n_cols = nc;
  S.d_ub = hd.d_ub;
  S.n_cols_ub = hd.n_cols_ub;
  S.T = hd.T;
  S.dN = hd.dN;
  h->dyn_ready = true;
  h->has_static = true;
  h->last_was_update = true;
  for (bool& u : h->ev_used) u = false;
  return CTD_OK;
}

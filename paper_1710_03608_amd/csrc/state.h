// Host-side handle of the CTD library.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "kernels.h"

namespace ctd {

// Bump allocator over one device buffer; `take` returns offsets that are
// rebased onto `base` once the total is known.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  void reset();
  void* take(size_t bytes);
};

// Workspace of one CTD-S call (all device pointers into the arena).
struct StaticBufs {
  uint64_t* keys;
  uint32_t* perm;
  uint32_t* hist;
  int32_t* row;
  double* val;
  float* val32;
  uint64_t* qpref;
  int32_t* fptr;
  uint64_t* fid;
  uint32_t* blk_cnt;
  uint64_t* blk_q;
  double* blk_v2;
  int32_t* draw_fi;
  uint64_t* draw_fid;
  int32_t* uniq_fi;
  uint64_t* uniq_fid;
  int32_t* counts;
  double* prob;
  double* scale;
  double* P;
  int32_t* accept;
  uint64_t* acc_fid;
  double* M;
  double* scratch;
  double* Q;
  float* Qf;
  double* lev;
  uint8_t* fiber_mark;
  double* resid;
  int32_t* long_list;
  double* long_part;
  int64_t long_ld;
  double* zpart;
  int64_t zpart_ld;
  double* partial;
  int32_t* hot_id;     // hot-row projection (null when not planned)
  int32_t* hot_meta;
  double* GH;
  int32_t* cold_list;
  double* Rs;
  double* C;
  int64_t ld;
  int64_t s_max;
};

// CTD-D state: factors of step t, kept on the device between calls.
struct DynState {
  int64_t capD = 0;        // row capacity of C / column capacity of R, Q, Xt
  int64_t capN = 0;        // column capacity of C
  int64_t d_tilde = 0;     // accepted fibers held (host copy, updated at sync points)
  int64_t n_cols = 0;      // columns of C held (non-empty fibers seen)
  int64_t d_ub = 0;        // host upper bound of d_tilde between syncs
  int64_t n_cols_ub = 0;   // host upper bound of n_cols between syncs
  int64_t T = 0;           // time steps held
  int64_t dN = 0;          // columns per time step (N_alpha of a slice)
  int64_t rows = 0;        // I_alpha the buffers were allocated for
  bool mixed = false;      // whether Qf is held
  double* Rs = nullptr;    // n_rows x capD row-major: kept fibers
  double* Q = nullptr;     // n_rows x capD row-major: orthonormal basis
  float* Qf = nullptr;     // mixed precision copy of Q
  double* Xt = nullptr;    // capD x capD row-major upper M with Q = R M
  double* lev = nullptr;   // n_rows: ||Q_i||^2
  double* C = nullptr;     // capD x capN column-major (float64 handles)
  float* Cf = nullptr;     // the same in float32 (mixed handles; C stays null)
  uint64_t* acc_fid = nullptr;  // capD kept fiber ids
  uint64_t* col_fid = nullptr;  // capN fiber ids of C's columns
  void* ws = nullptr;      // per-slice workspace
  size_t ws_bytes = 0;
};

// Many independent tensors in one call: tensors go in groups, one sub-handle
// (own workspace) per tensor of a group; their per-tensor stages run on a
// pool of streams and the basis of the whole group in one launch sequence;
// per-tensor results are copied into batch storage.
struct BatchState {
  std::vector<hipStream_t> pool;
  std::vector<hipEvent_t> done;    // one per pool stream
  std::vector<ctd_handle*> subs;   // one per tensor slot of a group
  hipEvent_t start = nullptr;
  hipEvent_t based = nullptr;
  int32_t B = 0;
  std::vector<int64_t> s, off, rows;
  DevScalars* scal = nullptr;      // [B] scalars of each tensor
  size_t cap_t = 0;
  uint64_t* draws = nullptr;       // per tensor at off[b]: s[b] entries each
  uint64_t* unique = nullptr;
  uint64_t* accepted = nullptr;
  int32_t* counts = nullptr;
  double* prob = nullptr;
  double* scale = nullptr;
  size_t cap_s = 0;
  std::vector<DevScalars> host;
  bool host_valid = false;
  // A repeated call with the same inputs and sizes replays a captured graph
  // of its launches (see ctd_decompose_batched).
  std::vector<uint64_t> last_sig;  // the previous call's signature
  std::vector<uint64_t> graph_sig; // the signature exec was captured for
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;       // the stream captured and replayed on
  hipEvent_t fork = nullptr;       // caller's stream -> cap
  hipEvent_t join = nullptr;       // cap -> caller's stream
  int64_t graph_launches = 0;      // calls that ran as a graph launch
};

}  // namespace ctd

struct ctd_handle {
  hipStream_t stream = nullptr;
  hipEvent_t ev[12] = {};   // profiling marks (MARK_COUNT)
  bool ev_used[12] = {};
  ctd_options opt{};
  ctd::DevScalars* d_sc = nullptr;
  ctd::Arena arena;
  ctd::StaticBufs sb{};
  ctd::DynState dyn;
  ctd::FiberLayout layout{};
  std::vector<uint64_t> given;
  std::string last_error;
  int64_t s = 0;
  uint64_t seed = 0;
  int64_t n_rows = 0;
  int64_t step = 0;
  int32_t mode = 0;
  bool failed = false;
  bool has_static = false;
  bool dyn_ready = false;
  bool last_was_update = false;
  bool keep_R = true;               // keep the dense kept fibers R (not needed inside a batch)
  int w2_sets = 2;                  // basis W2 buffer sets (1 inside a batch: no side streams)
  int64_t nnz_seen = 0;             // nonzeros of all input held (CTD-D: initial plus slices)
  void* bdev = nullptr;             // device array of basis arguments
  int bdev_cap = 0;
  ctd::BasisSide side{};            // side stream of the basis (created at first use)
  int side_state = 0;               // 0 not yet tried, 1 held, -1 unavailable
  // CTD-D cross term of a one-slice update, beside the slice's own columns
  // and residual (created at first use; default priority)
  hipStream_t xstream = nullptr;
  hipEvent_t xfork = nullptr, xjoin = nullptr;
  ctd::BatchState* batch = nullptr;
};

namespace ctd {
// Profiling marks (no-ops unless the handle profiles): mark(h, i) records
// event i on the handle's stream.  Stage times are differences of marks.
enum { MARK_START = 0, MARK_SORTED = 1, MARK_SAMPLED = 2, MARK_PANEL = 3, MARK_BASIS = 4,
       MARK_SPMM0 = 5, MARK_SPMM1 = 6, MARK_PROJECTED = 7, MARK_CORE = 8, MARK_END = 9,
       MARK_PROJ0 = 10, MARK_CROSS0 = 11, MARK_COUNT = 12 };
void mark(ctd_handle* h, int i);
void mark_on(ctd_handle* h, int i, hipStream_t st);
int bits_for(uint64_t n);
int64_t round8(int64_t x);
ctd_status fail(ctd_handle* h, ctd_status st, const std::string& msg);
ctd_status check_coo(ctd_handle* h, const ctd_coo* X, int32_t mode, FiberLayout* lay,
                     uint64_t* n_cols_total);
// The handle's basis side stream, created on first use; null if unavailable
// (the basis then runs on the handle's stream alone).
BasisSide* basis_side(ctd_handle* h);
ctd_status plan_static(ctd_handle* h, int64_t nnz, int64_t s, int64_t n_rows, bool mixed,
                       bool want_C, bool want_R, int64_t max_cols, StaticBufs* b);
ctd_status enqueue_input(ctd_handle* h, const ctd_coo* X, const FiberLayout& lay, int64_t s,
                         uint64_t seed, uint32_t step, const uint64_t* given, StaticBufs& b,
                         uint32_t tensor);
ctd_status run_static(ctd_handle* h, const ctd_coo* X, const FiberLayout& lay, int64_t s,
                      uint64_t seed, const uint64_t* given, uint32_t tensor);
ctd_status static_front(ctd_handle* h, const ctd_coo* X, const FiberLayout& lay, int64_t s,
                        uint64_t seed, const uint64_t* given, uint32_t tensor, BasisArgs* ba);
ctd_status static_back(ctd_handle* h, const ctd_coo* X, const FiberLayout& lay, int64_t s);
ctd_status ensure_bdev(ctd_handle* h, int count);
size_t static_bytes(int64_t nnz, int64_t s, int64_t n_rows, bool mixed, bool want_C, bool want_R,
                    int64_t max_cols);
int key_bits(const FiberLayout& lay);
ProjectArgs project_args(ctd_handle* h, StaticBufs& b, const double* Q, const float* Qf,
                         int64_t ldq, const double* lev, const int32_t* d_ncols, int64_t ncols_max,
                         int64_t n_rows);
void launch_reset_scalars(hipStream_t st, DevScalars* sc, bool keep_stream);
void launch_static_totals(hipStream_t st, DevScalars* sc);
void launch_core_static(hipStream_t st, StaticBufs& b, int64_t n_rows, int64_t nnz_max,
                        DevScalars* sc);
ctd_status dyn_begin(ctd_handle* h, const ctd_coo* X);
// (Re)allocate the CTD-D state with at least these capacities, keeping what it holds.
ctd_status dyn_resize(ctd_handle* h, int64_t capD, int64_t capN);
void dyn_free(ctd_handle* h);
void fill_result(ctd_handle* h, const DevScalars& sc, ctd_result* out);
void batch_free_storage(BatchState* B);
}  // namespace ctd

// Host-side launch wrappers of the CTD kernels.  Every wrapper enqueues on
// `st` and never synchronizes.  Sizes that are known only on the device are
// passed as pointers into DevScalars; host arguments give upper bounds.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "common.h"

namespace ctd {

// ---- tune.hip --------------------------------------------------------------
// Every device allocation of the library goes through dev_alloc.  With the
// environment variable CTD_FAIL_ALLOC set to k, the k-th allocation after the
// value was last set or changed fails with hipErrorOutOfMemory without calling
// the runtime (fault injection for the error paths; later ones succeed).
hipError_t dev_alloc_raw(void** p, size_t bytes);
template <typename T>
inline hipError_t dev_alloc(T** p, size_t bytes) {
  return dev_alloc_raw((void**)p, bytes);
}

// Per-process choice among bit-identical kernel variants (fibers per wave of
// the projection and of C's columns, waves per workgroup of the CTD-D cross
// term for at most 16 new rows), by shape bucket
// (tune_bucket(n) = ceil(log2 n)).  tune_get returns the chosen variant or -1
// (undecided; a finished measurement is resolved here).  tune_begin returns
// true, with 2 events per candidate, when the caller should time every
// candidate now (event 2c before candidate c, 2c + 1 after it), and then
// tune_recorded once every record is enqueued: until then no other thread
// reads the events.  While st is being captured into a graph no measurement
// starts (its event records would become graph nodes that outlive the
// events) and none is resolved (querying an event invalidates the capture):
// tune_get then returns only a choice already made.  The table is shared by
// the threads of a process.
enum { TUNE_PROJ_FPW = 0, TUNE_COLS_FPW = 1, TUNE_CROSS_NW = 2 };
int tune_bucket(int64_t n);
int tune_get(hipStream_t st, int knob, int prec, int bucket, int ncand);
bool tune_begin(hipStream_t st, int knob, int prec, int bucket, int ncand,
                std::vector<hipEvent_t>* evs);
void tune_recorded(int knob, int prec, int bucket);

// ---- sort.hip --------------------------------------------------------------
// Stable LSD radix sort of (key, payload) pairs on the low `nbits` bits of the
// keys.  The element count is *d_n if d_n != nullptr, else n_max.  Returns
// true if the sorted data ended in the *_alt buffers.
size_t radix_sort_hist_elems(int64_t n_max);
bool radix_sort(hipStream_t st, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                uint32_t* vals_alt, int64_t n_max, const int32_t* d_n, int nbits,
                uint32_t* hist_ws);

// ---- fibers.hip ------------------------------------------------------------
struct FiberLayout {
  int order;
  int mode;
  int rbits;              // bits of the row (mode-alpha) index
  int64_t n_rows;         // I_alpha
  int64_t dims[CTD_MAX_ORDER];
  int64_t stride[CTD_MAX_ORDER];  // fiber-id stride of each mode (0 for alpha)
};

// A0: validate, build keys (fid << rbits | row) and the identity payload, track
// max v^2.  val_dtype selects float64/float32 input.
void launch_build_keys(hipStream_t st, const FiberLayout& lay, const int32_t* idx,
                       const void* val, int val_dtype, int64_t nnz, uint64_t* keys,
                       uint32_t* perm, DevScalars* sc);
// A0/A1/A2: segment the sorted keys into fibers, gather values, quantized
// weights, inclusive weight prefix, ||X||^2.
struct SegmentBuffers {
  const uint64_t* keys;   // sorted
  const uint32_t* perm;   // sorted payload (original positions)
  const void* val_in;
  int val_dtype;
  int32_t* row;           // [nnz] out
  double* val;            // [nnz] out (float64 copy in fiber order)
  float* val32;           // [nnz] out (float32 copy) or nullptr
  uint64_t* qpref;        // [nnz] out inclusive prefix of quantized weights
  int32_t* fptr;          // [nnz+1] out fiber starts
  uint64_t* fid;          // [nnz] out fiber ids
  uint32_t* blk_cnt;      // workspace [nblocks+1]
  uint64_t* blk_q;        // workspace [nblocks+1]
  double* blk_v2;         // workspace [nblocks]
};
size_t segment_blocks(int64_t nnz);
void launch_segment(hipStream_t st, const SegmentBuffers& b, int64_t nnz, int rbits,
                    DevScalars* sc);

// ---- sample.hip ------------------------------------------------------------
// A2: s Philox draws -> fiber index and fiber id per draw.
void launch_draws(hipStream_t st, const uint64_t* qpref, const int32_t* fptr,
                  const uint64_t* fid, int64_t nnz, int64_t s, uint64_t seed, uint32_t step,
                  uint32_t tensor, int32_t* draw_fi, uint64_t* draw_fid, DevScalars* sc);
// Given draws (fiber ids, device) -> fiber index per draw (binary search).
void launch_locate_given(hipStream_t st, const uint64_t* fid, int64_t s,
                         const uint64_t* draw_fid, int32_t* draw_fi, DevScalars* sc);
// A3: sort the s draws, unique, multiplicities, probabilities, merge scales.
void launch_unique(hipStream_t st, const int32_t* draw_fi, int64_t s, const uint64_t* qpref,
                   const int32_t* fptr, const uint64_t* fid, int32_t* uniq_fi,
                   uint64_t* uniq_fid, int32_t* counts, double* prob, double* scale,
                   DevScalars* sc);

// ---- factor.hip ------------------------------------------------------------
// A4: dense row-major panel P (n_rows x ldp) of the s' candidate fibers.
void launch_panel(hipStream_t st, const int32_t* uniq_fi, int64_t s_max, const int32_t* fptr,
                  const int32_t* row, const double* val, int64_t n_rows, double* P, int64_t ldp,
                  DevScalars* sc);

// ---- basis.hip -------------------------------------------------------------
// A5-A7: independence filter over the s' candidates in blocks of 64, growing
// an orthonormal basis Q of span(R), R itself and M (Q = R M, U = M M^T).
// Starts from the sc->n_accept_total columns already held (0 for CTD-S).
struct BasisArgs {
  const double* P;           // candidate panel, n_rows x ldp
  int64_t ldp;
  int64_t n_rows;
  int64_t s_max;             // host bound of s'
  int64_t k0_max;            // host bound of the basis columns held before this call
  const int32_t* uniq_fi;    // candidate fiber positions (ascending)
  const uint64_t* uniq_fid;  // candidate fiber ids
  const int32_t* fptr;
  const int32_t* row;
  const double* val;
  double* Q;                 // n_rows x ldq
  int64_t ldq;
  float* Qf;                 // optional float copy of Q (same ld)
  double* R;                 // n_rows x ldr kept fibers (optional)
  int64_t ldr;
  double* M;                 // ldm x ldm upper triangular
  int64_t ldm;
  double* lev;               // n_rows: ||Q_i||^2
  bool lev_accumulate;       // add the new columns only
  double eps2;
  int32_t* accept;           // optional [s'] 0/1 per candidate
  uint64_t* acc_fid;         // kept fiber ids, indexed by global column
  int32_t* acc_fi_local;     // optional: kept fiber positions, indexed within this call
  uint8_t* fiber_mark;       // optional: 1 for kept fibers of this input
  uint64_t id_offset;        // added to fiber ids written to acc_fid
  double* Wacc;              // optional: Q^T x rows of the kept fibers (this call)
  int64_t ldwa;
  double* scratch;           // basis_scratch_doubles(n_rows, cap, w2_sets)
  int64_t cap;               // column capacity of Q, M, W (>= final k + 64)
  int w2_sets;               // 2: room for the side streams of a single input
};
size_t basis_scratch_doubles(int64_t n_rows, int64_t cap, int w2_sets);
// Device bytes of the argument array for `count` inputs.
size_t basis_dev_bytes(int count);
// Two more streams (default priority, non-blocking), one per block parity,
// and events: the projection passes of each block step run there ahead of
// the step, against the columns of Q already final.  Owned by the caller.
struct BasisSide {
  hipStream_t st[2] = {nullptr, nullptr};
  hipEvent_t start = nullptr, mid = nullptr;
  hipEvent_t done[2] = {nullptr, nullptr};
};
// Creates the streams and events on the current device; false (and nothing
// held) if any creation fails.
bool basis_side_init(BasisSide* side);
void basis_side_free(BasisSide* side);
// The basis of `count` independent inputs (args[i] with scalars scs[i]) in one
// sequence of launches on st; dev holds basis_dev_bytes(count) device bytes
// that stay untouched by others until the launches have run.  With a side
// (may be null), part of each step runs on the side streams, joined back to
// st by events before the step's results are used: the work as a whole is
// ordered on st like a single-stream launch sequence.
void launch_basis(hipStream_t st, const BasisArgs* args, DevScalars* const* scs, int count,
                  void* dev, BasisSide* side);

// ---- project.hip -----------------------------------------------------------
// A8: per-fiber residual ||x_f||^2 - ||Q^T x_f||^2 (0 for marked fibers) and
// its deterministic sum into sc->err2.
struct ProjectArgs {
  const int32_t* fptr;
  const int32_t* row;
  const double* val;
  const float* val32;      // mixed precision
  const double* Q;
  const float* Qf;         // mixed precision
  int64_t ldq;
  const double* lev;
  const uint8_t* fiber_mark;
  const int32_t* d_ncols;  // device count of columns of Q
  int64_t ncols_max;
  double* resid;           // [n_f] out
  int32_t* long_list;      // [nnz / (kLongFiber + 1) + 1] workspace: long fibers
  double* long_part;       // [long_list size x long_ld] per-slice ||z||^2 of long fibers
  int64_t long_ld;         // column slices held per long fiber (>= kProjSlices)
  double* zpart;           // [kProjSlices x zpart_ld] per-slice ||z||^2 of the other fibers
  int64_t zpart_ld;        // >= number of fibers
  double* partial;         // workspace
  bool mixed;
  int64_t n_rows;          // rows of Q
  // hot-row path (null when the input is too small or has too many rows)
  int32_t* hot_id;         // [n_rows] hot index of each row, -1 when cold
  int32_t* hot_meta;       // [kHotMax + 1] hot rows in row order, then their count
  double* GH;              // [n_rows x kHotMax] GH[r][a] = Q_r . Q_{hot row a}
  int32_t* cold_list;      // [nnz / 2 + 1] fibers with two or more cold nonzeros
};
// ev0/ev1 (optional) are recorded right before and after the multi-nonzero SpMM kernel.
void launch_project(hipStream_t st, const ProjectArgs& a, int64_t nnz_max, DevScalars* sc,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

}  // namespace ctd

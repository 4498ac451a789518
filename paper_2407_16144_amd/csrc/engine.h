// Host-side solver engine: device storage for a set of LPs ("instances"),
// preprocessing, power iteration, and the chunked iteration loop.  A single
// LP is an engine holding one instance; the batched and serving front ends
// hold many.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "halp.h"
#include "halp_types.h"

namespace halp {

struct Problem {  // one input LP; pointers are host or device memory
  int64_t n = 0, m_eq = 0, m_ineq = 0;
  const int32_t* rp = nullptr;
  const int32_t* ci = nullptr;
  const double* val = nullptr;
  const double* c = nullptr;
  const double* rhs = nullptr;
  const double* lb = nullptr;
  const double* ub = nullptr;
};

struct Options {
  int method = 1;  // 0 rHPDHG, 1 r2HPDHG, 2 restarted average PDHG (the comparison method)
  double avg_beta_sufficient = 0.2;  // average PDHG: KKT decay that restarts by itself
  double avg_beta_necessary = 0.8;   // ... that restarts when the last check made no progress
  int precision = 0;  // 0 fp64, 1 fp32
  int ruiz_iters = 10;
  double pc_alpha = 1.0;
  int check_every = 64;
  double restart_beta = 0.36787944117144233;
  double artificial_restart = 0.36;
  double step_safety = 0.9;
  int power_max_iters = 1000;
  int power_min_iters = 20;
  double power_rtol = 1e-4;
  double eps_infeas = 1e-8;
  int primal_weight = 1;
  uint64_t seed = 0;
  double eta = 0.0;
  double omega0 = 0.0;
  int chunk = 64;
  int use_graph = 1;
  int profile = 0;  // > 0: time every profile-th chunk's kernels with HIP events
  int64_t slice_min_bytes = 2 << 20;  // most bytes of the gathered vector per column slice (< 0: never slice)
  double polish_tol = 1e-3;  // fp32: solve to this tolerance in fp32, then polish in fp64
  int polish_weight = 1;     // FP64 phase's primal weight: 0 initial, 1 the FP32 phase's last, 2 by how it ended
  // bytes of vectors and matrix tiles the step kernels keep in the last-level
  // (Infinity) cache; tiles beyond it are read with non-temporal loads (< 0: all cached)
  int64_t cache_budget_bytes = 208ll << 20;
  // FP32 phase before an FP64 polish: an LP leaves it after this many checks
  // without a 10% drop of its best KKT error (its FP32 floor), 0: never
  int64_t stall_checks = 200;
  int xcd_pin = 1;                 // with many LPs, run each LP's blocks on one XCD
  int tile_rows = kMaxRows;        // rows per plain workgroup tile (<= 256)
  int slice_entries = kSliceNB;    // entries per slice tile: 256, 512 or 1024
  int slice_rows = kSliceRows;     // rows per sliced row group (<= 256)
  int slice_sort = 1;              // sliced / large products: sorted groups, LDS-atomic row sums
  int plain_sort = 1;              // other products: column-sorted blocks, LDS-atomic row sums
  int sort_rows = kSortRows;       // most rows per sorted group (plain sorted blocks: at most kSortRowsPlain)
  int group_threads = 0;           // threads per workgroup of the sorted-group slice kernels: 256, 512, 1024; 0: by size
  int group_batched = 1;           // 1: a thread's gathers issued together; 0: one gather per LDS add
  int group_blocks = kMinGroupBlocks;  // fewest workgroups a sorted-group product is cut into
  int restart_mode = 0;            // 0 adaptive, 1 fixed frequency, 2 none
  int64_t fixed_restart_len = 0;   // k* of the fixed-frequency rule
  int verbose = 0;
};

// Kernel durations summed over the steps timed with HIP events; a slice
// kernel runs only where a product is column-sliced (else its sum stays 0).
struct KernelTimes {
  double primal_slice_ms = 0.0, primal_ms = 0.0, dual_slice_ms = 0.0, dual_ms = 0.0;
  double event_pair_ms = 0.0;  // two events recorded back to back: included in every figure above
  double nnz = 0.0, n = 0.0, m = 0.0;  // entries, variables and rows of the LPs in the timed steps (sums)
  int64_t launches = 0;        // timed steps
};

struct Result {
  int status = 0;
  int64_t iters = 0, restarts = 0, checks = 0;
  double kkt = 0, rel_p = 0, rel_d = 0, rel_gap = 0, pobj = 0, dobj = 0, resid = 0;
  double omega = 0, eta = 0, sigma_hat = 0;
  int power_iters = 0, ray = 0;
  double seconds = 0;
  int64_t active_changes = 0, ident_iters = 0;
};

class Error : public std::runtime_error {
 public:
  Error(int code, const std::string& msg) : std::runtime_error(msg), code(code) {}
  int code;
};

class EngineBase {
 public:
  virtual ~EngineBase() = default;
  // add LPs (validated, preprocessed, iterates initialised); returns slot ids.
  // partial: admit the longest prefix that fits instead of failing.
  virtual std::vector<int> add(const std::vector<Problem>& probs, bool on_device, bool partial = false) = 0;
  // tolerance and iteration limit of the next solve; stall_checks > 0 also
  // ends an LP (ITER_LIMIT) after that many checks without a 10% drop of its
  // best KKT error (a low-precision phase that has reached its floor)
  virtual void set_params(const std::vector<int>& ids, double tol, int64_t max_iter,
                          int64_t stall_checks = 0) = 0;
  // run until every listed slot has terminated (or the time limit)
  virtual void run(double time_limit_s) = 0;
  // advance all live slots by `chunks` chunks; returns slots that finished since last call
  virtual std::vector<int> advance(int chunks) = 0;
  virtual void remove(const std::vector<int>& ids) = 0;
  virtual Result result(int id) = 0;
  virtual void solution(int id, double* x, double* y, bool to_device) = 0;
  virtual void certificate(int id, double* ray, bool to_device) = 0;
  virtual int64_t n_of(int id) const = 0;
  virtual int64_t m_of(int id) const = 0;
  virtual int live() const = 0;
  virtual hipStream_t stream() const = 0;
  // bytes of device storage an LP of this size needs (admission control)
  virtual int64_t footprint(int64_t n, int64_t m, int64_t nnz) const = 0;
  // fits: room for the LP now; fits_empty: room once no LP is live
  virtual bool fits(int64_t n, int64_t m, int64_t nnz) const = 0;
  virtual bool fits_empty(int64_t n, int64_t m, int64_t nnz) const = 0;
  virtual KernelTimes kernel_times() const = 0;
  // last check candidate T(z) in the scaled space, as float64 device arrays
  virtual void export_point(int id, double* x, double* y, double* omega) = 0;
  // start the next solve of `id` from (x, y) (scaled, float64 device arrays)
  // with primal weight omega (omega <= 0: the LP's initial weight
  // ||c~|| / ||q~||): iterate and anchor both set to the point
  virtual void import_point(int id, const double* x, const double* y, double omega) = 0;
  // the scaled K (transpose false) or K^T of `id` as stored, CSR with row
  // pointers from 0 and column indices relative to the LP, FP64 values, into
  // host arrays; only while that product is stored in row order (no column
  // slices, no column-sorted blocks or groups), else Error(-4)
  virtual void stored_matrix(int id, bool transpose, int32_t* rp, int32_t* ci, double* val) = 0;
  // smaller column-sorted blocks for the LPs still running (by the statuses
  // of the last advance) when few of them share the launches
  virtual void refine_layouts() = 0;
};

// Size of the static device workspace of the allocation-free entry point.
constexpr int64_t kWorkspaceBytes = LP_STATIC_WORKSPACE_BYTES;

// While a WorkspaceScope is alive on a thread, every device buffer that an
// engine created on that thread allocates comes from the static workspace of
// the current device (no hipMalloc), cleared to zero on `stream`; engines
// created in the scope must be destroyed before it ends.  Scopes do not nest.
class WorkspaceScope {
 public:
  explicit WorkspaceScope(hipStream_t stream);
  ~WorkspaceScope();
  WorkspaceScope(const WorkspaceScope&) = delete;
  WorkspaceScope& operator=(const WorkspaceScope&) = delete;
  size_t peak() const;  // most bytes in use at once so far
};

// Host-side validation of a host-memory LP (throws Error(-1, ...)); needs no GPU.
void validate_host_problem(const Problem& p);
// Device int64 row pointers narrowed into int32 (dst, count entries) on
// `stream`; returns nonzero when an entry is negative or above 2^31 - 1.
int narrow_row_ptr(const int64_t* src, int32_t* dst, int64_t count, hipStream_t stream);

// capacity: sizes of the three spaces and the slot count (0 = grow to fit)
std::unique_ptr<EngineBase> make_engine(const Options& opt, hipStream_t stream, int64_t cap_m,
                                        int64_t cap_n, int64_t cap_nnz, int max_slots);

}  // namespace halp

// Shared host/device types of the HIP solver.
//
// Vectors of every live LP sit in three "spaces": m-space (constraint rows),
// n-space (variables) and nnz-space (matrix entries).  An instance owns the
// contiguous ranges [row0, row0 + m + 1), [col0, col0 + n + 1) and
// [nz0, nz0 + nnz); the extra position closes its CSR row pointers.  Column
// indices of K and of the explicit transpose K^T are stored as global space
// positions, so the sparse kernels never translate indices.
#pragma once
#include <stdint.h>

namespace halp {

constexpr int kThreads = 256;        // threads per workgroup (4 wave64)
constexpr int kMaxRows = 256;        // rows per "stream" block (one epilogue row per thread)
constexpr int kNS = 8;               // partial-sum slots per block
constexpr int kNAcc = 12;            // sums kept from a check step for the following eval step

// Entries per stream block: plain blocks (whole rows) and the slice blocks of
// column-sliced matrices (measured on MI355X: random gathers, not HBM
// bandwidth, bound these products, and smaller tiles keep more independent
// gathers in flight).  Rows longer than a tile get a block of their own.
constexpr int kPlainNB = 1024;
constexpr int kSliceNB = 512;    // default entries per slice tile (also 256 and 1024 compiled)
constexpr int kSliceRows = 128;  // default rows per sliced row group
template <class T> struct Tile { static constexpr int NB = kPlainNB; };

enum Mode : int { M_SKIP = 0, M_NORMAL = 1, M_CHECK = 2, M_EVAL = 3, M_RESID = 4 };
enum Phase : int { PH_NORMAL = 0, PH_EVAL = 1, PH_RESID = 2 };
enum BlkKind : int { BK_STREAM = 0, BK_LONG = 1, BK_PAD = 2, BK_SORTED = 3 };

// Column slices of a sliced matrix: one per XCD, so that consecutive
// workgroups (dispatched round-robin over the XCDs) gather from a slice of the
// vector small enough to stay in that XCD's L2.
constexpr int kSlices = 8;
constexpr int kPinMinLPs = 16;   // schedules with at least this many LPs pin each LP to one XCD
enum Status : int { ST_RUNNING = 0, ST_OPTIMAL = 1, ST_PRIMAL_INFEAS = 2, ST_DUAL_INFEAS = 3,
                    ST_ITER_LIMIT = 4, ST_TIME_LIMIT = 5, ST_NUMERICAL = 6 };

// One workgroup's share of a CSR matrix: rows [r0, r1) (space positions) and
// the entries [p0, p0 + pn).  A plain block covers whole rows; the blocks of
// a sliced row group (nsl = kSlices) cover the same rows, block `slice`
// holding only the entries whose column falls in that slice, with its own
// row pointers at brp[rp_off].  gid numbers row groups (partial sums and
// arrival counters); meta packs kind | nsl << 8 | slice << 16, and kBlkNT
// marks a block whose entries are read with non-temporal loads (they are not
// meant to stay in the last-level cache: see the cache budget of Options).
struct Blk {
  int32_t r0, r1, inst, meta;
  int32_t gid, rp_off, p0, pn;
};

__host__ __device__ inline int blk_kind(const Blk& b) { return b.meta & 0xff; }
__host__ __device__ inline int blk_nsl(const Blk& b) { return (b.meta >> 8) & 0xff; }
__host__ __device__ inline int blk_slice(const Blk& b) { return (b.meta >> 16) & 0xff; }
constexpr int32_t kBlkNT = 1 << 24;
__host__ __device__ inline bool blk_nt(const Blk& b) { return (b.meta & kBlkNT) != 0; }
// kBlkPart marks a step-kernel block whose row sums are the nsl slice
// partial sums a slice kernel wrote (sliced or sorted-group products).
constexpr int32_t kBlkPart = 1 << 30;
__host__ __device__ inline bool blk_part(const Blk& b) { return (b.meta & kBlkPart) != 0; }

// Column-sorted row groups (a product stored as "sorted groups": K when its
// gathered vector is larger than Options::slice_min_bytes, and either
// product when its matrix is large enough for groups of more rows than a
// plain sorted block): the rows are cut into groups, each group's entries
// into nsl column slices (1, 2, 4 or 8; with 8 each slice's gathers stay in
// one XCD's L2), and the entries of one (group, slice) block are ordered by
// column, each column index stored as (column - first column of the slice)
// << rb | (row - b.r0), with rb in meta bits 25..29 and the slice's first
// column (a space position) in rp_off.  The slice kernel adds a block's
// products into LDS row sums (at most kSortRows rows per group) and writes
// them as the group's slice-`slice` partial sums; the step kernel adds the
// nsl partials of a row in slice order.  A block holds at most kSortEntries
// entries.
constexpr int kSortRows = 16384;
constexpr int kSortEntries = 1 << 18;
// Sorted-group products are cut into at least this many workgroups (about
// one per CU); the engine gives each group as many rows as that allows.
constexpr int kMinGroupBlocks = 240;
constexpr int kCUs = 256;        // compute units of an MI355X
// A plain block of the step kernels may be column-sorted too (kind
// BK_SORTED, same packing, rp_off = the LP's first column): at most
// kSortRowsPlain rows (its row sums share the step kernel's LDS with the
// plain tile), rows of at most kPlainNB entries.
constexpr int kSortRowsPlain = 2048;
__host__ __device__ inline int blk_rowbits(const Blk& b) { return (b.meta >> 25) & 31; }
__host__ __device__ inline int32_t blk_meta(int kind, int nsl, int slice) {
  return kind | (nsl << 8) | (slice << 16);
}

// Check-step sums (stored in InstState::acc between the check and eval steps).
enum AccSlot : int {
  A_DX2 = 0, A_AX2, A_POBJ, A_CD1, A_CD2,       // from the primal kernel
  A_DY2, A_AY2, A_DOBJQ, A_QY1, A_QY2,          // from the dual kernel
  A_ACTX, A_ACTY,                               // activity changes (primal, dual)
};

struct alignas(16) InstState {
  // layout and constants
  int64_t row0, col0, nz0;
  int32_t m, m_eq, n, reflect;
  int32_t C, primal_weight;
  int32_t pb0, pb1, db0, db1;        // this instance's row groups (gids) in the primal / dual schedules
  double tol, eps_inf, beta, artificial, eta, qnorm, cnorm;
  int64_t max_iter;
  // dynamic state
  int32_t status, phase;
  int64_t kbase, tbase, nrest, checks;
  int64_t next_check;                // global step index of the next check step
  double omega, tau, sigma, r0;
  double acc[kNAcc];
  // last check
  double kkt, rel_p, rel_d, rel_gap, pobj, dobj, resid;
  int64_t iters;
  int32_t ray, pad0;
  // stall rule (a low-precision phase ends when its KKT error stops falling):
  // best error so far, the check that set it, and the allowed checks without
  // a 10% improvement (0: off)
  double best_kkt;
  int64_t best_check, stall_checks;
  // restart rule: 0 adaptive (eq. (adaptive-restart) + artificial), 1 fixed
  // frequency (eq. (fixed-restart), k >= fixed_len), 2 none
  int64_t fixed_len;
  int32_t restart_mode, avg;         // avg = 1: restarted average PDHG (plain T steps, average candidate)
  // average PDHG's KKT-based restart: error at the epoch's start and at its
  // previous check, and the sufficient / necessary decay factors
  double kkt_anchor, kkt_prev, avg_b1, avg_b2;
  // two-stage diagnostics: variables / inequality rows whose activity (at a
  // bound; dual at zero) changed between the last two checks, and the
  // iteration count at the last check where any changed
  int64_t act_changes, ident_iters;
  // power iteration
  double pw_scale, pw_prev, sigma_hat;
  int32_t pw_iter, pw_done;
};

}  // namespace halp

// Host-side engine of the HIP solver.  This translation unit also holds the
// kernels (included below), so every launch resolves inside one code object.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"
#include "kernels.hip"
#include "layout_kernels.hip"

namespace halp {

#define HIPCHECK(expr)                                                                       \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw Error(-3, std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// first-fit allocator over one space
class RangeAlloc {
 public:
  explicit RangeAlloc(int64_t cap = 0) : cap_(cap) {
    if (cap > 0) free_[0] = cap;
  }
  int64_t alloc(int64_t len) {
    if (len <= 0) return 0;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        const int64_t at = it->first, rest = it->second - len;
        free_.erase(it);
        if (rest > 0) free_[at + len] = rest;
        return at;
      }
    }
    return -1;
  }
  void release(int64_t at, int64_t len) {
    if (len <= 0) return;
    auto it = free_.emplace(at, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  bool can(int64_t len) const {
    if (len <= 0) return true;
    for (auto& kv : free_)
      if (kv.second >= len) return true;
    return false;
  }

 private:
  int64_t cap_;
  std::map<int64_t, int64_t> free_;
};

// ---------------------------------------------------------------------------
// device memory
//
// Every buffer of an engine comes from dalloc.  Normally that is hipMalloc;
// inside a WorkspaceScope (the allocation-free entry point) the buffers are
// carved out of `scratch`, a static device array, by a stack allocator: a
// freed block is reclaimed once every block above it is freed too (the
// engine frees its temporaries in the reverse order of their allocation).
// Carved blocks are cleared to zero on the workspace's stream, as fresh
// device memory would be.
// ---------------------------------------------------------------------------

static __device__ __align__(256) char scratch[kWorkspaceBytes];

struct Workspace {
  char* base = nullptr;    // this device's copy of `scratch` (from hipGetSymbolAddress)
  size_t used = 0, peak = 0;
  hipStream_t stream = nullptr;
  std::vector<std::pair<size_t, bool>> blocks;  // (offset, freed) in allocation order
};
static thread_local Workspace* t_ws = nullptr;

// Address of this device's copy of `scratch`; looked up once per device with
// that device current (the array's host-side name is not a device address).
static char* scratch_base(int device) {
  static std::mutex mu;
  static std::map<int, char*> base;
  std::lock_guard<std::mutex> lk(mu);
  auto it = base.find(device);
  if (it != base.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    throw Error(-3, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
  base[device] = (char*)p;
  return (char*)p;
}

static void* ws_alloc(size_t bytes) {
  Workspace& w = *t_ws;
  const size_t b = (bytes + 255) & ~size_t(255);
  if (w.used + b > (size_t)kWorkspaceBytes)
    throw Error(-2, "static workspace exhausted: " + std::to_string(w.used + b) + " bytes needed of " +
                        std::to_string((long long)kWorkspaceBytes));
  char* p = w.base + w.used;
  w.blocks.push_back({w.used, false});
  w.used += b;
  w.peak = std::max(w.peak, w.used);
  const hipError_t e = hipMemsetAsync(p, 0, b, w.stream);
  if (e != hipSuccess) throw Error(-3, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  return p;
}

static bool ws_free(void* p) {
  Workspace* w = t_ws;
  if (!w || (char*)p < w->base || (char*)p >= w->base + kWorkspaceBytes) return false;
  const size_t off = (size_t)((char*)p - w->base);
  for (auto& bl : w->blocks)
    if (bl.first == off) bl.second = true;
  while (!w->blocks.empty() && w->blocks.back().second) {
    w->used = w->blocks.back().first;
    w->blocks.pop_back();
  }
  return true;
}

template <class P>
static void dalloc(P** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  if (t_ws) {
    *p = (P*)ws_alloc(sizeof(P) * (size_t)count);
    return;
  }
  hipError_t e = hipMalloc((void**)p, sizeof(P) * (size_t)count);
  if (e != hipSuccess) throw Error(-2, std::string("device allocation failed: ") + hipGetErrorString(e));
}

template <class P>
static void dfree(P*& p) {
  if (p && !ws_free((void*)p)) (void)hipFree((void*)p);
  p = nullptr;
}

WorkspaceScope::WorkspaceScope(hipStream_t stream) {
  if (t_ws) throw Error(-4, "nested use of the static workspace");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) throw Error(-3, "hipGetDevice failed");
  std::unique_ptr<Workspace> w(new Workspace());
  w->base = scratch_base(dev);
  w->stream = stream;
  t_ws = w.release();
}

WorkspaceScope::~WorkspaceScope() {
  delete t_ws;
  t_ws = nullptr;
}

size_t WorkspaceScope::peak() const { return t_ws ? t_ws->peak : 0; }

}  // namespace halp

#include "radix_sort.hip"

namespace halp {

// Workgroup schedule of one LP's rows: consecutive rows are packed into
// "stream" blocks of at most NB entries and kMaxRows rows; a row with more
// than NB entries gets a "long" block.  Every LP gets at least one block so
// that its controller always runs.  gid counts blocks from 0 (offset when the
// schedules of all LPs are concatenated).
static void build_blocks(const int32_t* rp, int64_t nrows, int64_t base, int inst, int NB, int max_rows,
                         std::vector<Blk>& out) {
  const size_t first = out.size();
  int64_t start = 0, acc = 0;
  auto emit = [&](int64_t a, int64_t b, int kind) {
    Blk k;
    k.r0 = (int32_t)(base + a);
    k.r1 = (int32_t)(base + b);
    k.inst = inst;
    k.meta = blk_meta(kind, 1, 0);
    k.gid = (int32_t)(out.size() - first);
    k.rp_off = 0;
    k.p0 = rp[a];
    k.pn = rp[b] - rp[a];
    out.push_back(k);
  };
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t len = (int64_t)rp[r + 1] - rp[r];
    if (len > NB) {
      if (r > start) emit(start, r, BK_STREAM);
      emit(r, r + 1, BK_LONG);
      start = r + 1;
      acc = 0;
      continue;
    }
    if (acc + len > NB || (r - start) >= max_rows) {
      if (r > start) emit(start, r, BK_STREAM);
      start = r;
      acc = 0;
    }
    acc += len;
  }
  if (nrows > start) emit(start, nrows, BK_STREAM);
  if (out.size() == first) emit(0, 0, BK_STREAM);
}

// Column-sliced schedule of one LP's rows.  cnt[r * kSlices + s] counts row
// r's entries in column slice s.  Rows are grouped (at most max_rows rows)
// so that every slice of a group holds at most NB entries (a row with more
// gets a group of its own and "long" slice blocks).  Each group has kSlices
// slice blocks in `sl` whose entries are stored group-major, then
// slice-major, then row-major starting at entry position nz0.  `grp` gets
// epilogue blocks (nsl = kSlices, kMaxRows rows each) that add up the
// slice partial sums.  Row pointers of slice blocks go to brp (positions from brp_base);
// dst[r * kSlices + s] receives the first position of row r's slice s.
static void build_sliced(const int32_t* cnt, int64_t nrows, int64_t base, int inst, int NB, int max_rows,
                         int64_t nz0,
                         int64_t brp_base, std::vector<Blk>& grp, std::vector<Blk>& sl,
                         std::vector<int32_t>& brp, std::vector<int32_t>& dst) {
  std::vector<std::pair<int64_t, int64_t>> groups;
  int64_t start = 0;
  int64_t acc[kSlices] = {0};
  auto flush = [&](int64_t e) {
    if (e > start) groups.emplace_back(start, e);
    start = e;
    for (int q = 0; q < kSlices; ++q) acc[q] = 0;
  };
  for (int64_t r = 0; r < nrows; ++r) {
    const int32_t* c = cnt + r * kSlices;
    bool big = false, over = (r - start) >= max_rows;
    for (int q = 0; q < kSlices; ++q) {
      big |= c[q] > NB;
      over |= acc[q] + c[q] > NB;
    }
    if (big) {
      flush(r);
      groups.emplace_back(r, r + 1);
      start = r + 1;
      continue;
    }
    if (over) flush(r);
    for (int q = 0; q < kSlices; ++q) acc[q] += c[q];
  }
  flush(nrows);
  if (groups.empty()) groups.emplace_back(0, 0);
  dst.assign(nrows * kSlices, 0);
  int64_t pos = nz0;
  // epilogue blocks: kMaxRows consecutive rows each, independent of the groups
  for (int64_t a = 0; a < std::max<int64_t>(nrows, 1); a += kMaxRows) {
    Blk ep;
    ep.r0 = (int32_t)(base + a);
    ep.r1 = (int32_t)(base + std::min<int64_t>(a + kMaxRows, nrows));
    ep.inst = inst;
    ep.meta = blk_meta(BK_STREAM, kSlices, 0) | kBlkPart;
    ep.gid = (int32_t)grp.size();
    ep.rp_off = 0;
    ep.p0 = 0;
    ep.pn = 0;
    grp.push_back(ep);
  }
  for (size_t g = 0; g < groups.size(); ++g) {
    const int64_t a = groups[g].first, e = groups[g].second;
    Blk ep;
    ep.r0 = (int32_t)(base + a);
    ep.r1 = (int32_t)(base + e);
    ep.inst = inst;
    ep.gid = (int32_t)g;
    for (int q = 0; q < kSlices; ++q) {
      Blk k = ep;
      k.rp_off = (int32_t)(brp_base + (int64_t)brp.size());
      k.p0 = (int32_t)pos;
      int64_t mx = 0;
      for (int64_t r = a; r < e; ++r) {
        brp.push_back((int32_t)pos);
        dst[r * kSlices + q] = (int32_t)pos;
        pos += cnt[r * kSlices + q];
        mx = std::max<int64_t>(mx, cnt[r * kSlices + q]);
      }
      brp.push_back((int32_t)pos);
      k.pn = (int32_t)(pos - k.p0);
      k.meta = blk_meta((e - a == 1 && mx > NB) ? BK_LONG : BK_STREAM, kSlices, q);
      sl.push_back(k);
    }
  }
}

// Blocks per product of a column-sorted LP: at least kMinSortedBlocks (rows
// down to kMaxRows) in engines of many LPs, whose products share each
// launch; for an LP among few, enough that the engine's products have about
// kTailBlocks workgroups (rows down to kMinSortedRows), since its blocks are
// most of what the launch has (measured on MI355X, LPs of 12.8k and 18.6k
// rows alone: 21.4 and 36.8 us per iteration with 256-row blocks, 13.0 and
// 17.5 us with 128-row blocks; in a batch of 512 such LPs 64-row blocks
// everywhere cost 7% over the default).  Engines re-block their running LPs
// as LPs finish (refine_layouts).
constexpr int64_t kMinSortedBlocks = 64;
constexpr int64_t kMinSortedRows = 64;
// the products of an engine with few LPs keep at least this many
// workgroups in all: blocks are sized for the LPs that share the launches
constexpr int64_t kTailBlocks = 768;

// Blocks per product (at least) and smallest row cap of the column-sorted
// blocks of an LP that shares the launches with `live` LPs in all.
static void plain_shape(int64_t live, int64_t* min_blocks, int64_t* min_rows) {
  live = std::max<int64_t>(live, 1);
  if (live * kMinSortedBlocks >= kTailBlocks) {
    *min_blocks = kMinSortedBlocks;
    *min_rows = kMaxRows;
  } else {
    *min_blocks = (kTailBlocks + live - 1) / live;
    *min_rows = kMinSortedRows;
  }
}

struct Slot {
  bool used = false;
  int64_t n = 0, m = 0, m_eq = 0, nnz = 0;
  int64_t row0 = 0, col0 = 0, nz0 = 0;
  std::vector<Blk> bP, bD;  // one block per row group (inst field = slot id, gid local)
  std::vector<Blk> bPS, bDS;  // slice blocks of sliced groups (empty when not sliced)
  int64_t brpP0 = 0, brpPn = 0, brpD0 = 0, brpDn = 0;  // ranges in the brp spaces
  int rowsP = 0, rowsD = 0;  // rows of the largest sorted group of K^T / K (0: not grouped)
  int64_t plainP = 0, plainD = 0;  // row cap of K^T's / K's column-sorted plain blocks (0: none)
  bool watched = false;
  bool reported = false;
};

template <class T>
class Engine final : public EngineBase {
 public:
  Engine(const Options& opt, hipStream_t s, int64_t cap_m, int64_t cap_n, int64_t cap_nnz, int slots)
      : opt_(opt), stream_(s), MS_(cap_m), NS_(cap_n), NZ_(cap_nnz), nslots_(slots),
        am_(cap_m), an_(cap_n), az_(cap_nnz), abK_(2 * kSlices * cap_m), abKT_(2 * kSlices * cap_n),
        slots_(slots) {
    try {
      allocate();
    } catch (...) {
      release_all();
      throw;
    }
  }
  ~Engine() override {
    if (stream_) (void)hipStreamSynchronize(stream_);
    for (hipEvent_t e : pev_) (void)hipEventDestroy(e);
    release_all();
  }

  hipStream_t stream() const override { return stream_; }
  int64_t n_of(int id) const override { return slots_.at(id).n; }
  int64_t m_of(int id) const override { return slots_.at(id).m; }
  int live() const override {
    int c = 0;
    for (auto& s : slots_) c += s.used;
    return c;
  }

  int64_t footprint(int64_t n, int64_t m, int64_t nnz) const override {
    // as allocate() sizes the spaces: per row K_rp, three FP64 and ten (twelve
    // with sorted blocks) compute-type vectors, the activity byte and the
    // slice row pointers; per variable the same for K^T's side
    const int64_t s = sizeof(T);
    const int64_t brp = opt_.slice_min_bytes >= 0 ? 2 * kSlices * 4 : 0;
    const int64_t ev = opt_.plain_sort ? 2 * s : 0;
    const int64_t per_row = 4 + 3 * 8 + 10 * s + ev + 1 + brp, per_col = 4 + 5 * 8 + 11 * s + ev + 1 + brp;
    const int64_t per_nz = 8 + 16 + (sizeof(T) == 8 ? 0 : 2 * s);
    return per_row * (m + 1) + per_col * (n + 1) + per_nz * nnz;
  }
  KernelTimes kernel_times() const override { return ktimes_; }
  bool fits(int64_t n, int64_t m, int64_t nnz) const override {
    int free_slots = 0;
    for (auto& s : slots_) free_slots += !s.used;
    return free_slots > 0 && am_.can(m + 1) && an_.can(n + 1) && az_.can(nnz);
  }
  bool fits_empty(int64_t n, int64_t m, int64_t nnz) const override {
    return nslots_ > 0 && m + 1 <= MS_ && n + 1 <= NS_ && nnz <= NZ_;
  }

  std::vector<int> add(const std::vector<Problem>& probs, bool on_device, bool partial) override;
  void set_params(const std::vector<int>& ids, double tol, int64_t max_iter,
                  int64_t stall_checks = 0) override;
  void run(double time_limit_s) override;
  std::vector<int> advance(int chunks) override;
  void remove(const std::vector<int>& ids) override;
  Result result(int id) override;
  void solution(int id, double* x, double* y, bool to_device) override;
  void certificate(int id, double* ray, bool to_device) override;
  void export_point(int id, double* x, double* y, double* omega) override;
  void stored_matrix(int id, bool transpose, int32_t* rp, int32_t* ci, double* val) override;
  void refine_layouts() override {
    HIPCHECK(hipStreamSynchronize(stream_));
    reblock_for(h_status[0]);
  }
  void import_point(int id, const double* x, const double* y, double omega) override;

 private:
  void allocate();
  void release_all();
  void rebuild_schedules();
  void pin_to_xcds(std::vector<Blk>& v, const std::vector<std::pair<int, int>>& ranges) const;
  void launch_slices(bool dual, const IterArgs<T>& A, int step);
  template <bool DUAL>
  void launch_group(unsigned g, int tpb, size_t lds, const IterArgs<T>& A, int step);
  int ldsP_ = 0, ldsD_ = 0;  // rows of the largest sorted group in the current schedules
  int tpbP_ = 256, tpbD_ = 256;  // threads per workgroup of the sorted-group kernels
  void mark_streaming(const std::vector<int>& live, std::vector<Blk>& P, std::vector<Blk>& PS,
                      std::vector<Blk>& DS, std::vector<Blk>& D) const;
  int scheduled_ = 0;          // LPs in the current schedules
  bool compacted_ = false;     // current schedules leave finished LPs out
  const int* finished_ = nullptr;  // status words used to leave finished LPs out (compaction)
  void launch_chunk();
  void collect_times();
  void transpose_group(int64_t z0, int64_t nnz, int64_t c0, int64_t c1, const std::vector<Blk>& bD);
  void preprocess(const std::vector<int>& ids, const std::vector<Blk>& nP, const std::vector<Blk>& nD,
                  const std::vector<int4>& nr);
  void slice_matrix(int id, bool dual);
  void group_sorted(int id, bool dual, int nsl, int64_t rows);
  bool group_shape(int64_t nrows, int64_t width, int nsl_min, int* nsl, int64_t* rows) const;
  int group_lds_rows(bool dual) const;
  void sort_blocks(int id, bool dual, int64_t min_blocks, int64_t min_rows, bool reblock);
  void reblock_for(const int* status);
  int64_t plain_rows(int64_t nrows, int64_t width, int64_t min_blocks, int64_t min_rows) const;
  IterArgs<T> args() const;
  void pull_states();

  Options opt_;
  hipStream_t stream_;
  int64_t MS_, NS_, NZ_;
  int nslots_;
  RangeAlloc am_, an_, az_, abK_, abKT_;
  std::vector<Slot> slots_;
  int64_t g_next_ = 0;  // index of the next step to launch

  // nnz-space
  int32_t *K_ci = nullptr, *KT_ci = nullptr;
  double *K_v64 = nullptr, *KT_v64 = nullptr;
  T *K_v = nullptr, *KT_v = nullptr;
  // m-space
  int32_t* K_rp = nullptr;
  double *q_o = nullptr, *Dr = nullptr, *fm = nullptr;
  T *q = nullptr, *y = nullptr, *y0 = nullptr, *yT = nullptr, *dy = nullptr, *kxbar = nullptr,
    *kxp = nullptr, *cy1 = nullptr, *cy2 = nullptr, *ys = nullptr;
  // n-space
  int32_t* KT_rp = nullptr;
  double *c_o = nullptr, *l_o = nullptr, *u_o = nullptr, *Dc = nullptr, *fn = nullptr;
  T *c = nullptr, *l = nullptr, *u = nullptr, *x = nullptr, *x0 = nullptr, *xbar = nullptr,
    *xT = nullptr, *ktyp = nullptr, *cx1 = nullptr, *cx2 = nullptr, *xs = nullptr;
  // column-sliced layout
  int32_t *brpK = nullptr, *brpKT = nullptr;
  T *spartD = nullptr, *spartP = nullptr;
  T *kt1_ = nullptr, *kt2_ = nullptr, *kx1_ = nullptr, *kx2_ = nullptr;  // sorted blocks' eval products
  uint8_t *actx = nullptr, *acty = nullptr;  // activity at the last check (two-stage diagnostics)
  Blk *d_schedPS = nullptr, *d_schedDS = nullptr;
  int* d_live_ = nullptr;       // slot ids of the LPs in the current schedules (control kernel)
  int64_t cap_live_ = 0;
  int64_t capPS_ = 0, capDS_ = 0, nPS_ = 0, nDS_ = 0;
  // control
  InstState* d_st = nullptr;
  int* d_status = nullptr;
  int* d_cnt = nullptr;
  int64_t* d_gbase = nullptr;
  Blk *d_schedP = nullptr, *d_schedD = nullptr;
  int64_t capP_ = 0, capD_ = 0, nP_ = 0, nD_ = 0;
  double *partP = nullptr, *partD = nullptr;
  int* h_status[2] = {nullptr, nullptr};
  hipEvent_t ev_[2] = {nullptr, nullptr};
  bool ws_ = false;  // buffers come from the static workspace (no events, no pinned memory)
  bool sched_dirty_ = true;
  hipGraphExec_t gexec_ = nullptr;
  hipGraph_t graph_ = nullptr;
  std::vector<InstState> h_st_;
  int64_t chunk_count_ = 0;
  std::vector<hipEvent_t> pev_;  // 6 events per step of one chunk, reused by each timed chunk
  bool pev_pending_ = false;     // pev_ holds a timed chunk not yet added to ktimes_
  bool pev_slices_[2] = {false, false};  // the timed chunk launched primal / dual slice kernels
  double pev_size_[3] = {0, 0, 0};       // nnz, n, m of the LPs in the timed chunk's schedules
  double sched_size_[3] = {0, 0, 0};     // the same for the current schedules
  KernelTimes ktimes_;
};

template <class T>
void Engine<T>::allocate() {
  dalloc(&K_ci, NZ_);
  dalloc(&KT_ci, NZ_);
  dalloc(&K_v64, NZ_);
  dalloc(&KT_v64, NZ_);
  if (sizeof(T) == 8) {
    K_v = (T*)K_v64;
    KT_v = (T*)KT_v64;
  } else {
    dalloc(&K_v, NZ_);
    dalloc(&KT_v, NZ_);
  }
  dalloc(&K_rp, MS_);
  dalloc(&q_o, MS_);
  dalloc(&Dr, MS_);
  dalloc(&fm, MS_);
  for (T** p : {&q, &y, &y0, &yT, &dy, &kxbar, &kxp, &cy1, &cy2, &ys}) dalloc(p, MS_);
  dalloc(&KT_rp, NS_);
  for (double** p : {&c_o, &l_o, &u_o, &Dc, &fn}) dalloc(p, NS_);
  for (T** p : {&c, &l, &u, &x, &x0, &xbar, &xT, &ktyp, &cx1, &cx2, &xs}) dalloc(p, NS_);
  dalloc(&actx, NS_);
  dalloc(&acty, MS_);
  if (opt_.plain_sort) {
    dalloc(&kx1_, MS_);
    dalloc(&kx2_, MS_);
    dalloc(&kt1_, NS_);
    dalloc(&kt2_, NS_);
  }
  // row pointers of row-major slice tiles: only where products may be sliced
  const bool may_slice = opt_.slice_min_bytes >= 0;
  dalloc(&brpK, may_slice ? 2 * kSlices * MS_ : 1);
  dalloc(&brpKT, may_slice ? 2 * kSlices * NS_ : 1);
  dalloc(&d_st, nslots_);
  dalloc(&d_status, nslots_);
  dalloc(&d_cnt, nslots_);
  dalloc(&d_gbase, 1);
  HIPCHECK(hipMemsetAsync(d_cnt, 0, sizeof(int) * nslots_, stream_));
  HIPCHECK(hipMemsetAsync(d_status, 0, sizeof(int) * nslots_, stream_));
  HIPCHECK(hipMemsetAsync(d_st, 0, sizeof(InstState) * nslots_, stream_));
  // a zeroed state reads as running: park every slot until an LP is added
  set_limit_status_kernel<<<nblk(nslots_), 256, 0, stream_>>>(d_st, d_status, nslots_, ST_ITER_LIMIT);
  HIPCHECK(hipGetLastError());
  const int64_t gb = -(int64_t)opt_.chunk;
  HIPCHECK(hipMemcpyAsync(d_gbase, &gb, sizeof(int64_t), hipMemcpyHostToDevice, stream_));
  ws_ = t_ws != nullptr;
  for (int i = 0; i < 2; ++i) {
    if (ws_) {
      // static workspace: ordinary host memory, status reads synchronise the stream
      h_status[i] = new int[nslots_];
    } else {
      HIPCHECK(hipHostMalloc((void**)&h_status[i], sizeof(int) * nslots_, hipHostMallocDefault));
      HIPCHECK(hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming));
    }
    std::memset(h_status[i], 0, sizeof(int) * nslots_);
  }
  h_st_.resize(nslots_);
  // sorted groups keep up to kSortRows row sums in dynamic LDS
  const int lds_max = (int)(sizeof(double) * kSortRows);
  for (const void* f : {(const void*)sorted_group_step<T, true, 256, true>, (const void*)sorted_group_step<T, true, 256, false>,
                        (const void*)sorted_group_step<T, true, 512, true>, (const void*)sorted_group_step<T, true, 512, false>,
                        (const void*)sorted_group_step<T, true, 1024, true>, (const void*)sorted_group_step<T, true, 1024, false>,
                        (const void*)sorted_group_step<T, false, 256, true>, (const void*)sorted_group_step<T, false, 256, false>,
                        (const void*)sorted_group_step<T, false, 512, true>, (const void*)sorted_group_step<T, false, 512, false>,
                        (const void*)sorted_group_step<T, false, 1024, true>,
                        (const void*)sorted_group_step<T, false, 1024, false>})
    HIPCHECK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max));
  HIPCHECK(hipStreamSynchronize(stream_));
}

template <class T>
void Engine<T>::release_all() {
  if (gexec_) (void)hipGraphExecDestroy(gexec_);
  if (graph_) (void)hipGraphDestroy(graph_);
  gexec_ = nullptr;
  graph_ = nullptr;
  dfree(K_ci);
  dfree(KT_ci);
  if (sizeof(T) != 8) {
    dfree(K_v);
    dfree(KT_v);
  }
  dfree(K_v64);
  dfree(KT_v64);
  dfree(K_rp);
  dfree(q_o);
  dfree(Dr);
  dfree(fm);
  for (T** p : {&q, &y, &y0, &yT, &dy, &kxbar, &kxp, &cy1, &cy2, &ys}) dfree(*p);
  dfree(KT_rp);
  for (double** p : {&c_o, &l_o, &u_o, &Dc, &fn}) dfree(*p);
  for (T** p : {&c, &l, &u, &x, &x0, &xbar, &xT, &ktyp, &cx1, &cx2, &xs}) dfree(*p);
  dfree(actx);
  dfree(acty);
  dfree(brpK);
  dfree(brpKT);
  dfree(spartD);
  dfree(kt1_);
  dfree(kt2_);
  dfree(kx1_);
  dfree(kx2_);
  dfree(spartP);
  dfree(d_schedPS);
  dfree(d_schedDS);
  dfree(d_live_);
  dfree(d_st);
  dfree(d_status);
  dfree(d_cnt);
  dfree(d_gbase);
  dfree(d_schedP);
  dfree(d_schedD);
  dfree(partP);
  dfree(partD);
  for (int i = 0; i < 2; ++i) {
    if (h_status[i]) {
      if (ws_) delete[] h_status[i];
      else (void)hipHostFree(h_status[i]);
    }
    h_status[i] = nullptr;
    if (ev_[i]) (void)hipEventDestroy(ev_[i]);
    ev_[i] = nullptr;
  }
}

template <class T>
IterArgs<T> Engine<T>::args() const {
  IterArgs<T> A;
  A.K_rp = K_rp;
  A.K_ci = K_ci;
  A.K_v = K_v;
  A.KT_rp = KT_rp;
  A.KT_ci = KT_ci;
  A.KT_v = KT_v;
  A.brpK = brpK;
  A.brpKT = brpKT;
  A.spartD = spartD;
  A.spartP = spartP;
  A.kt1 = kt1_;
  A.kt2 = kt2_;
  A.kx1 = kx1_;
  A.kx2 = kx2_;
  A.MS = MS_;
  A.NS = NS_;
  A.c = c;
  A.l = l;
  A.u = u;
  A.Dc = Dc;
  A.x = x;
  A.x0 = x0;
  A.xbar = xbar;
  A.xT = xT;
  A.ktyp = ktyp;
  A.cx1 = cx1;
  A.cx2 = cx2;
  A.xs = xs;
  A.actx = actx;
  A.q = q;
  A.Dr = Dr;
  A.y = y;
  A.y0 = y0;
  A.yT = yT;
  A.dy = dy;
  A.kxbar = kxbar;
  A.kxp = kxp;
  A.cy1 = cy1;
  A.cy2 = cy2;
  A.ys = ys;
  A.acty = acty;
  A.st = d_st;
  A.gbase = d_gbase;
  A.cnt = d_cnt;
  A.status_out = d_status;
  A.partP = partP;
  A.partD = partD;
  A.schedP = d_schedP;
  A.schedD = d_schedD;
  A.schedPS = d_schedPS;
  A.schedDS = d_schedDS;
  return A;
}

// ---------------------------------------------------------------------------
// input validation and canonical CSR on the host
// ---------------------------------------------------------------------------

struct HostCSR {
  std::vector<int32_t> rp, ci;
  std::vector<double> val;
};

static void validate_host(const Problem& p, HostCSR& canon, bool& use_canon) {
  const int64_t m = p.m_eq + p.m_ineq, n = p.n;
  if (n < 1 || p.m_eq < 0 || p.m_ineq < 0) throw Error(-1, "sizes must satisfy n >= 1, m_eq >= 0, m_ineq >= 0");
  if (!p.rp || (m > 0 && (!p.c || !p.rhs)) || !p.c || !p.lb || !p.ub)
    throw Error(-1, "null input pointer");
  if (p.rp[0] != 0) throw Error(-1, "row_ptr[0] must be 0");
  for (int64_t i = 0; i < m; ++i)
    if (p.rp[i + 1] < p.rp[i]) throw Error(-1, "row_ptr must be non-decreasing");
  const int64_t nnz = p.rp[m];
  if (nnz > 0 && (!p.ci || !p.val)) throw Error(-1, "null column or value array");
  bool sorted = true;
  for (int64_t i = 0; i < m; ++i) {
    for (int64_t e = p.rp[i]; e < p.rp[i + 1]; ++e) {
      const int64_t cidx = p.ci[e];
      if (cidx < 0 || cidx >= n) throw Error(-1, "column index out of range");
      if (!std::isfinite(p.val[e])) throw Error(-1, "non-finite matrix value");
      if (e > p.rp[i] && cidx <= p.ci[e - 1]) sorted = false;
    }
  }
  for (int64_t i = 0; i < m; ++i)
    if (!std::isfinite(p.rhs[i])) throw Error(-1, "non-finite right-hand side");
  for (int64_t j = 0; j < n; ++j) {
    if (!std::isfinite(p.c[j])) throw Error(-1, "non-finite objective");
    const double a = p.lb[j], b = p.ub[j];
    if (std::isnan(a) || std::isnan(b) || a > b || a == INFINITY || b == -INFINITY)
      throw Error(-1, "invalid bounds (NaN, lb > ub, lb = +inf or ub = -inf)");
  }
  use_canon = !sorted;
  if (sorted) return;
  // sort each row by column and sum duplicate entries
  canon.rp.assign(m + 1, 0);
  canon.ci.clear();
  canon.val.clear();
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < m; ++i) {
    row.clear();
    for (int64_t e = p.rp[i]; e < p.rp[i + 1]; ++e) row.emplace_back(p.ci[e], p.val[e]);
    std::stable_sort(row.begin(), row.end(),
                     [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                       return a.first < b.first;
                     });
    for (size_t k = 0; k < row.size(); ++k) {
      if (k > 0 && row[k].first == canon.ci.back()) {
        canon.val.back() += row[k].second;
      } else {
        canon.ci.push_back(row[k].first);
        canon.val.push_back(row[k].second);
      }
    }
    canon.rp[i + 1] = (int32_t)canon.ci.size();
  }
}

void validate_host_problem(const Problem& p) {
  HostCSR canon;
  bool uc = false;
  validate_host(p, canon, uc);
}

// ---------------------------------------------------------------------------
// add LPs
// ---------------------------------------------------------------------------

template <class T>
void Engine<T>::transpose_group(int64_t z0, int64_t nnz, int64_t c0, int64_t c1,
                                const std::vector<Blk>& bD) {
  if (nnz > 0) {
    Blk* d_b = nullptr;
    int32_t *rowid = nullptr, *vin = nullptr, *vout = nullptr;
    uint32_t *keys = nullptr, *kout = nullptr;
    dalloc(&d_b, (int64_t)bD.size());
    dalloc(&rowid, nnz);
    dalloc(&keys, nnz);
    dalloc(&kout, nnz);
    dalloc(&vin, nnz);
    dalloc(&vout, nnz);
    HIPCHECK(hipMemcpyAsync(d_b, bD.data(), sizeof(Blk) * bD.size(), hipMemcpyHostToDevice, stream_));
    row_ids_kernel<<<(unsigned)bD.size(), kThreads, 0, stream_>>>(d_b, K_rp, z0, rowid);
    iota_kernel<<<nblk(nnz), 256, 0, stream_>>>(vin, nnz);
    // keys: columns relative to the LP's first column; a stable sort keeps
    // each column's entries in row order
    shift_copy_kernel<<<nblk(nnz), 256, 0, stream_>>>((int32_t*)keys, K_ci + z0, nnz, -c0);
    HIPCHECK(hipGetLastError());
    std::vector<int> shifts;
    radix_shifts(shifts, 0, bits_for(c1 - c0));
    radix_sort_pairs<uint32_t>(keys, vin, kout, vout, nnz, shifts, stream_);
    transpose_gather_kernel<double><<<nblk(nnz), 256, 0, stream_>>>(vout, rowid, K_v64, z0, nnz, KT_ci,
                                                                     KT_v64);
    transpose_rowptr_kernel<<<nblk(c1 - c0 + 1), 256, 0, stream_>>>(kout, nnz, z0, c0, c1, KT_rp);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(stream_));
    dfree(vout);
    dfree(vin);
    dfree(kout);
    dfree(keys);
    dfree(rowid);
    dfree(d_b);
  } else {
    std::vector<int32_t> h(c1 - c0 + 1, (int32_t)z0);
    HIPCHECK(hipMemcpyAsync(KT_rp + c0, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice,
                            stream_));
    HIPCHECK(hipStreamSynchronize(stream_));
  }
}

template <class T>
std::vector<int> Engine<T>::add(const std::vector<Problem>& probs_in, bool on_device, bool partial) {
  std::vector<Problem> probs(probs_in);
  constexpr int NB = Tile<T>::NB;
  std::vector<int> ids;
  HIPCHECK(hipStreamSynchronize(stream_));
  // 1. validate and reserve
  std::vector<HostCSR> canon(probs.size());
  std::vector<char> use_canon(probs.size(), 0);
  for (size_t k = 0; k < probs.size(); ++k) {
    const Problem& p = probs[k];
    if (!on_device) {
      bool uc = false;
      validate_host(p, canon[k], uc);
      use_canon[k] = uc;
    } else {
      if (p.n < 1 || p.m_eq < 0 || p.m_ineq < 0) throw Error(-1, "sizes must satisfy n >= 1, m >= 0");
      const int64_t m = p.m_eq + p.m_ineq;
      int32_t ends[2] = {0, 0};
      HIPCHECK(hipMemcpy(&ends[0], p.rp, sizeof(int32_t), hipMemcpyDeviceToHost));
      HIPCHECK(hipMemcpy(&ends[1], p.rp + m, sizeof(int32_t), hipMemcpyDeviceToHost));
      if (ends[0] != 0 || ends[1] < 0) throw Error(-1, "row_ptr must start at 0 and end at nnz >= 0");
      int* d_flags = nullptr;
      dalloc(&d_flags, 1);
      HIPCHECK(hipMemsetAsync(d_flags, 0, sizeof(int), stream_));
      if (m > 0) {
        validate_rowptr_kernel<<<nblk(m), 256, 0, stream_>>>(p.rp, m, ends[1], d_flags);
        if (ends[1] > 0)
          validate_entries_kernel<<<nblk(ends[1]), 256, 0, stream_>>>(p.rp, p.ci, p.val, m, p.n, ends[1], d_flags);
      }
      validate_vectors_kernel<<<nblk(std::max<int64_t>(m, p.n)), 256, 0, stream_>>>(p.c, p.rhs, p.lb, p.ub,
                                                                                     m, p.n, d_flags);
      int flags = 0;
      HIPCHECK(hipMemcpyAsync(&flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, stream_));
      HIPCHECK(hipStreamSynchronize(stream_));
      dfree(d_flags);
      if (flags & 1) throw Error(-1, "row_ptr must be non-decreasing from 0 to nnz");
      if (flags & 2) throw Error(-1, "device CSR needs in-range, strictly increasing column indices per row");
      if (flags & 4) throw Error(-1, "non-finite matrix value");
      if (flags & 8) throw Error(-1, "non-finite objective or right-hand side");
      if (flags & 16) throw Error(-1, "invalid bounds (NaN, lb > ub, lb = +inf or ub = -inf)");
    }
  }
  std::vector<int64_t> nnzs(probs.size());
  for (size_t k = 0; k < probs.size(); ++k) {
    const Problem& p = probs[k];
    const int64_t m = p.m_eq + p.m_ineq;
    if (use_canon[k]) {
      nnzs[k] = canon[k].rp[m];
    } else if (!on_device) {
      nnzs[k] = p.rp[m];
    } else {
      int32_t e = 0;
      HIPCHECK(hipMemcpy(&e, p.rp + m, sizeof(int32_t), hipMemcpyDeviceToHost));
      nnzs[k] = e;
    }
  }
  std::vector<int> fresh;
  try {
    for (size_t k = 0; k < probs.size(); ++k) {
      const Problem& p = probs[k];
      const int64_t m = p.m_eq + p.m_ineq;
      int id = -1;
      for (int s = 0; s < nslots_; ++s)
        if (!slots_[s].used) {
          id = s;
          break;
        }
      if (id < 0) {
        if (partial) break;
        throw Error(-2, "no free LP slot");
      }
      const int64_t r0 = am_.alloc(m + 1);
      const int64_t c0 = r0 < 0 ? -1 : an_.alloc(p.n + 1);
      const int64_t z0 = c0 < 0 ? -1 : az_.alloc(nnzs[k]);
      if (r0 < 0 || c0 < 0 || z0 < 0) {
        if (r0 >= 0) am_.release(r0, m + 1);
        if (c0 >= 0) an_.release(c0, p.n + 1);
        if (partial) break;
        throw Error(-2, "not enough device memory reserved for this LP");
      }
      if (z0 + nnzs[k] > INT32_MAX) throw Error(-1, "more than 2^31 stored entries");
      Slot& S = slots_[id];
      S = Slot();
      S.used = true;
      S.n = p.n;
      S.m = m;
      S.m_eq = p.m_eq;
      S.nnz = nnzs[k];
      S.row0 = r0;
      S.col0 = c0;
      S.nz0 = z0;
      ids.push_back(id);
      fresh.push_back(id);
    }
  } catch (...) {
    for (int id : fresh) {
      Slot& S = slots_[id];
      am_.release(S.row0, S.m + 1);
      an_.release(S.col0, S.n + 1);
      az_.release(S.nz0, S.nnz);
      S = Slot();
    }
    throw;
  }

  if (ids.size() < probs.size()) {
    probs.resize(ids.size());
    canon.resize(ids.size());
    use_canon.resize(ids.size());
    nnzs.resize(ids.size());
  }
  if (ids.empty()) return ids;
  // 2. upload (K values in FP64, row pointers / columns shifted to space positions)
  std::vector<std::vector<int32_t>> host_rp(probs.size());
  for (size_t k = 0; k < probs.size(); ++k) {
    const Problem& p = probs[k];
    Slot& S = slots_[ids[k]];
    const int64_t m = S.m, n = S.n, nnz = S.nnz;
    const auto kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const int32_t* rp_src = use_canon[k] ? canon[k].rp.data() : p.rp;
    const int32_t* ci_src = use_canon[k] ? canon[k].ci.data() : p.ci;
    const double* v_src = use_canon[k] ? canon[k].val.data() : p.val;
    host_rp[k].resize(m + 1);
    if (!on_device) {
      for (int64_t i = 0; i <= m; ++i) host_rp[k][i] = (int32_t)(rp_src[i] + S.nz0);
      HIPCHECK(hipMemcpyAsync(K_rp + S.row0, host_rp[k].data(), sizeof(int32_t) * (m + 1),
                              hipMemcpyHostToDevice, stream_));
      std::vector<int32_t> cs(nnz);
      for (int64_t e = 0; e < nnz; ++e) cs[e] = (int32_t)(ci_src[e] + S.col0);
      if (nnz) {
        HIPCHECK(hipMemcpyAsync(K_ci + S.nz0, cs.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, stream_));
        HIPCHECK(hipMemcpyAsync(K_v64 + S.nz0, v_src, sizeof(double) * nnz, hipMemcpyHostToDevice, stream_));
      }
      HIPCHECK(hipStreamSynchronize(stream_));
    } else {
      shift_copy_kernel<<<nblk(m + 1), 256, 0, stream_>>>(K_rp + S.row0, p.rp, m + 1, S.nz0);
      if (nnz) {
        shift_copy_kernel<<<nblk(nnz), 256, 0, stream_>>>(K_ci + S.nz0, p.ci, nnz, S.col0);
        HIPCHECK(hipMemcpyAsync(K_v64 + S.nz0, p.val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, stream_));
      }
      HIPCHECK(hipMemcpyAsync(host_rp[k].data(), K_rp + S.row0, sizeof(int32_t) * (m + 1),
                              hipMemcpyDeviceToHost, stream_));
    }
    if (m) HIPCHECK(hipMemcpyAsync(q_o + S.row0, p.rhs, sizeof(double) * m, kind, stream_));
    HIPCHECK(hipMemcpyAsync(c_o + S.col0, p.c, sizeof(double) * n, kind, stream_));
    HIPCHECK(hipMemcpyAsync(l_o + S.col0, p.lb, sizeof(double) * n, kind, stream_));
    HIPCHECK(hipMemcpyAsync(u_o + S.col0, p.ub, sizeof(double) * n, kind, stream_));
    fill_kernel<<<nblk(m + 1), 256, 0, stream_>>>(Dr + S.row0, m + 1, 1.0);
    fill_kernel<<<nblk(n + 1), 256, 0, stream_>>>(Dc + S.col0, n + 1, 1.0);
  }
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(stream_));

  // 3. dual schedules, transpose, primal schedules
  for (size_t k = 0; k < probs.size(); ++k) {
    Slot& S = slots_[ids[k]];
    build_blocks(host_rp[k].data(), S.m, S.row0, ids[k], NB, opt_.tile_rows, S.bD);
    // host_rp holds space positions; build_blocks only uses differences
  }
  // contiguous groups transpose together
  size_t k = 0;
  while (k < probs.size()) {
    size_t e = k + 1;
    while (e < probs.size()) {
      const Slot& A = slots_[ids[e - 1]];
      const Slot& B = slots_[ids[e]];
      if (B.row0 != A.row0 + A.m + 1 || B.col0 != A.col0 + A.n + 1 || B.nz0 != A.nz0 + A.nnz) break;
      ++e;
    }
    const Slot& F = slots_[ids[k]];
    const Slot& L = slots_[ids[e - 1]];
    std::vector<Blk> bD;
    for (size_t t = k; t < e; ++t) bD.insert(bD.end(), slots_[ids[t]].bD.begin(), slots_[ids[t]].bD.end());
    transpose_group(F.nz0, L.nz0 + L.nnz - F.nz0, F.col0, L.col0 + L.n, bD);
    k = e;
  }
  for (size_t t = 0; t < probs.size(); ++t) {
    Slot& S = slots_[ids[t]];
    std::vector<int32_t> krp(S.n + 1);
    HIPCHECK(hipMemcpy(krp.data(), KT_rp + S.col0, sizeof(int32_t) * (S.n + 1), hipMemcpyDeviceToHost));
    build_blocks(krp.data(), S.n, S.col0, ids[t], NB, opt_.tile_rows, S.bP);
  }

  // 4. temporary schedules of the new LPs, preprocessing, power iteration
  std::vector<Blk> nP, nD;
  std::vector<int4> nr;
  for (int id : ids) {
    const Slot& S = slots_[id];
    int4 r;
    r.x = (int)nP.size();
    nP.insert(nP.end(), S.bP.begin(), S.bP.end());
    r.y = (int)nP.size();
    r.z = (int)nD.size();
    nD.insert(nD.end(), S.bD.begin(), S.bD.end());
    r.w = (int)nD.size();
    nr.push_back(r);
  }
  compacted_ = false;
  preprocess(ids, nP, nD, nr);
  // Layout of each product.  A product whose gathered vector would not stay
  // in one XCD's L2 is column-sliced (8 slices): in sorted groups by default,
  // in row-major slice tiles with slice_sort = 0.  With sorted layouts on, a
  // product large enough for sorted groups of more rows than a plain sorted
  // block holds is stored in sorted groups of 1 or 2 slices (larger groups:
  // more entries share each cache line of the gathered vector).  The other
  // products get column-sorted plain blocks (plain_sort) or plain tiles.
  const int64_t live_after = live();
  for (int id : ids) {
    const Slot& S = slots_[id];
    for (const bool dual : {true, false}) {
      const int64_t nrows = dual ? S.m : S.n, width = dual ? S.n : S.m;
      // fewest slices that keep each slice of the gathered vector within
      // slice_min_bytes (1: the product need not be sliced)
      int nsl_min = 1;
      if (opt_.slice_min_bytes >= 0 && S.nnz > 0)
        while (nsl_min < kSlices && width * (int64_t)sizeof(T) > opt_.slice_min_bytes * nsl_min) nsl_min *= 2;
      const bool slice = nsl_min > 1;
      int nsl = 0;
      int64_t rows = 0;
      if (slice && !opt_.slice_sort) {
        slice_matrix(id, dual);
      } else if (S.nnz > 0 && opt_.slice_sort && (slice || opt_.plain_sort) &&
                 group_shape(nrows, width, nsl_min, &nsl, &rows) &&
                 (slice || rows > std::min<int64_t>(opt_.sort_rows, kSortRowsPlain))) {
        group_sorted(id, dual, nsl, rows);
      } else if (opt_.plain_sort) {
        int64_t minb = 0, minr = 0;
        plain_shape(live_after, &minb, &minr);
        sort_blocks(id, dual, minb, minr, false);
      }
    }
  }
  sched_dirty_ = true;
  for (int id : ids) slots_[id].watched = true;
  return ids;
}

template <class T>
void Engine<T>::preprocess(const std::vector<int>& ids, const std::vector<Blk>& nP,
                           const std::vector<Blk>& nD, const std::vector<int4>& nr) {
  const int ni = (int)ids.size();
  Blk *d_nP = nullptr, *d_nD = nullptr;
  int* d_ids = nullptr;
  int4* d_nr = nullptr;
  double* d_pp = nullptr;
  double* d_norms = nullptr;
  int* d_active = nullptr;
  InstState* d_src = nullptr;
  auto cleanup = [&]() {
    dfree(d_nP);
    dfree(d_nD);
    dfree(d_ids);
    dfree(d_nr);
    dfree(d_pp);
    dfree(d_norms);
    dfree(d_active);
    dfree(d_src);
  };
  try {
    dalloc(&d_nP, (int64_t)nP.size());
    dalloc(&d_nD, (int64_t)nD.size());
    dalloc(&d_ids, ni);
    dalloc(&d_nr, ni);
    dalloc(&d_pp, (int64_t)nP.size() * kNS);
    dalloc(&d_norms, 2 * ni);
    dalloc(&d_active, 1);
    dalloc(&d_src, ni);
    HIPCHECK(hipMemcpyAsync(d_nP, nP.data(), sizeof(Blk) * nP.size(), hipMemcpyHostToDevice, stream_));
    HIPCHECK(hipMemcpyAsync(d_nD, nD.data(), sizeof(Blk) * nD.size(), hipMemcpyHostToDevice, stream_));
    HIPCHECK(hipMemcpyAsync(d_ids, ids.data(), sizeof(int) * ni, hipMemcpyHostToDevice, stream_));
    HIPCHECK(hipMemcpyAsync(d_nr, nr.data(), sizeof(int4) * ni, hipMemcpyHostToDevice, stream_));
    const unsigned gP = (unsigned)nP.size(), gD = (unsigned)nD.size();

    // scaling (Ruiz infinity-norm passes, then Pock-Chambolle)
    for (int it = 0; it < opt_.ruiz_iters; ++it) {
      row_factor_kernel<<<gD, kThreads, 0, stream_>>>(d_nD, K_rp, K_v64, 0, 1.0, fm, Dr);
      row_factor_kernel<<<gP, kThreads, 0, stream_>>>(d_nP, KT_rp, KT_v64, 0, 1.0, fn, Dc);
      scale_values_kernel<<<gD, kThreads, 0, stream_>>>(d_nD, K_rp, K_ci, K_v64, fm, fn, 0);
      scale_values_kernel<<<gP, kThreads, 0, stream_>>>(d_nP, KT_rp, KT_ci, KT_v64, fm, fn, 1);
    }
    if (opt_.pc_alpha > 0.0) {
      row_factor_kernel<<<gD, kThreads, 0, stream_>>>(d_nD, K_rp, K_v64, 1, 2.0 - opt_.pc_alpha, fm, Dr);
      row_factor_kernel<<<gP, kThreads, 0, stream_>>>(d_nP, KT_rp, KT_v64, 1, opt_.pc_alpha, fn, Dc);
      scale_values_kernel<<<gD, kThreads, 0, stream_>>>(d_nD, K_rp, K_ci, K_v64, fm, fn, 0);
      scale_values_kernel<<<gP, kThreads, 0, stream_>>>(d_nP, KT_rp, KT_ci, KT_v64, fm, fn, 1);
    }
    scale_primal_kernel<T><<<gP, kThreads, 0, stream_>>>(d_nP, Dc, c_o, l_o, u_o, c, l, u);
    scale_dual_kernel<T><<<gD, kThreads, 0, stream_>>>(d_nD, Dr, q_o, q);

    // layout constants for the norm and power kernels
    std::vector<InstState> src(ni);
    for (int k = 0; k < ni; ++k) {
      const Slot& S = slots_[ids[k]];
      InstState& s = src[k];
      std::memset(&s, 0, sizeof(InstState));
      s.row0 = S.row0;
      s.col0 = S.col0;
      s.nz0 = S.nz0;
      s.m = (int32_t)S.m;
      s.m_eq = (int32_t)S.m_eq;
      s.n = (int32_t)S.n;
      s.status = ST_ITER_LIMIT;  // parked until set_params
      s.pw_done = opt_.eta > 0.0 ? 1 : 0;
    }
    HIPCHECK(hipMemcpyAsync(d_src, src.data(), sizeof(InstState) * ni, hipMemcpyHostToDevice, stream_));
    write_states_kernel<<<nblk(ni), 256, 0, stream_>>>(d_st, d_status, d_cnt, d_ids, d_src, ni);
    inst_norms_kernel<<<ni, kThreads, 0, stream_>>>(d_st, d_ids, q_o, c_o, Dr, Dc, d_norms);

    // power iteration on K~^T K~ (u in fm, w in fn)
    int piters = 0;
    if (opt_.eta <= 0.0) {
      pw_start_kernel<<<gP, kThreads, 0, stream_>>>(d_nP, d_st, opt_.seed, fn, d_pp);
      HIPCHECK(hipMemsetAsync(d_active, 0, sizeof(int), stream_));
      pw_control_kernel<<<ni, kThreads, 0, stream_>>>(d_st, d_ids, d_nr, d_pp, 1, opt_.power_min_iters,
                                                      opt_.power_max_iters, opt_.power_rtol, d_active);
      int active = 1;
      while (active > 0 && piters < opt_.power_max_iters) {
        const int batch = 8;
        for (int b = 0; b < batch && piters < opt_.power_max_iters; ++b, ++piters) {
          pw_forward_kernel<<<gD, kThreads, 0, stream_>>>(d_nD, d_st, K_rp, K_ci, K_v64, fn, fm);
          pw_backward_kernel<<<gP, kThreads, 0, stream_>>>(d_nP, d_st, KT_rp, KT_ci, KT_v64, fm, fn, d_pp);
          HIPCHECK(hipMemsetAsync(d_active, 0, sizeof(int), stream_));
          pw_control_kernel<<<ni, kThreads, 0, stream_>>>(d_st, d_ids, d_nr, d_pp, 0, opt_.power_min_iters,
                                                          opt_.power_max_iters, opt_.power_rtol, d_active);
        }
        HIPCHECK(hipMemcpyAsync(&active, d_active, sizeof(int), hipMemcpyDeviceToHost, stream_));
        HIPCHECK(hipStreamSynchronize(stream_));
      }
    }
    if (sizeof(T) != 8) {
      for (int id : ids) {
        const Slot& S = slots_[id];
        if (S.nnz) {
          cast_kernel<T><<<nblk(S.nnz), 256, 0, stream_>>>(K_v64 + S.nz0, K_v + S.nz0, S.nnz);
          cast_kernel<T><<<nblk(S.nnz), 256, 0, stream_>>>(KT_v64 + S.nz0, KT_v + S.nz0, S.nnz);
        }
      }
    }
    init_primal_kernel<T><<<gP, kThreads, 0, stream_>>>(d_nP, l, u, x, x0, actx);
    init_dual_kernel<T><<<gD, kThreads, 0, stream_>>>(d_nD, y, y0, acty);
    HIPCHECK(hipGetLastError());

    // step size and primal weight, then park the LPs until set_params
    std::vector<double> norms(2 * ni);
    HIPCHECK(hipMemcpyAsync(norms.data(), d_norms, sizeof(double) * 2 * ni, hipMemcpyDeviceToHost, stream_));
    std::vector<InstState> cur(ni);
    for (int k = 0; k < ni; ++k)
      HIPCHECK(hipMemcpyAsync(&cur[k], d_st + ids[k], sizeof(InstState), hipMemcpyDeviceToHost, stream_));
    HIPCHECK(hipStreamSynchronize(stream_));
    for (int k = 0; k < ni; ++k) {
      InstState& s = cur[k];
      const double sh = s.sigma_hat;
      double eta;
      if (opt_.eta > 0.0) {
        eta = opt_.eta;
        s.sigma_hat = NAN;
      } else {
        eta = sh > 0.0 ? opt_.step_safety / sh : opt_.step_safety;
      }
      const double nq = norms[2 * k], nc = norms[2 * k + 1];
      double omega = 1.0;
      if (opt_.omega0 > 0.0) omega = opt_.omega0;
      else if (opt_.primal_weight && nc > 1e-10 && nq > 1e-10) omega = nc / nq;
      s.eta = eta;
      s.omega = omega;
      s.tau = eta / omega;
      s.sigma = eta * omega;
      s.reflect = opt_.method == 1;
      s.avg = opt_.method == 2;
      s.avg_b1 = opt_.avg_beta_sufficient;
      s.avg_b2 = opt_.avg_beta_necessary;
      s.kkt_anchor = NAN;
      s.kkt_prev = INFINITY;
      s.act_changes = 0;
      s.ident_iters = 0;
      s.C = opt_.check_every;
      s.primal_weight = opt_.primal_weight;
      s.beta = opt_.restart_beta;
      s.artificial = opt_.artificial_restart;
      s.restart_mode = opt_.restart_mode;
      s.fixed_len = opt_.fixed_restart_len;
      s.eps_inf = opt_.eps_infeas;
      s.r0 = NAN;
      s.status = ST_ITER_LIMIT;  // parked
      s.phase = PH_NORMAL;
      s.nrest = 0;
      s.checks = 0;
      s.ray = 0;
      s.iters = 0;
      s.kkt = NAN;
      s.best_kkt = INFINITY;
      s.best_check = 0;
      s.stall_checks = 0;
      h_st_[ids[k]] = s;
    }
    HIPCHECK(hipMemcpyAsync(d_src, cur.data(), sizeof(InstState) * ni, hipMemcpyHostToDevice, stream_));
    write_states_kernel<<<nblk(ni), 256, 0, stream_>>>(d_st, d_status, d_cnt, d_ids, d_src, ni);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(stream_));
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

// Reorders one LP's K (dual = true; slices over its variables) or K^T
// (slices over its constraints) into the column-sliced layout.
template <class T>
void Engine<T>::slice_matrix(int id, bool dual) {
  const int NB = opt_.slice_entries;
  Slot& S = slots_[id];
  const int64_t nrows = dual ? S.m : S.n;
  const int64_t r0 = dual ? S.row0 : S.col0;
  const int64_t c0 = dual ? S.col0 : S.row0;
  const int64_t len = dual ? S.n : S.m;
  const int32_t* rp = dual ? K_rp : KT_rp;
  int32_t* ci = dual ? K_ci : KT_ci;
  T* val = dual ? K_v : KT_v;
  double* v64 = dual ? K_v64 : KT_v64;
  if (nrows == 0 || S.nnz == 0) return;
  int32_t* d_cnt = nullptr;
  dalloc(&d_cnt, nrows * kSlices);
  slice_count_kernel<<<nblk(nrows), 256, 0, stream_>>>(rp, ci, r0, nrows, c0, len, kSlices, d_cnt);
  std::vector<int32_t> cnt(nrows * kSlices);
  HIPCHECK(hipMemcpyAsync(cnt.data(), d_cnt, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost, stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  std::vector<Blk> grp, sl;
  std::vector<int32_t> brp, dst;
  RangeAlloc& ab = dual ? abK_ : abKT_;
  // reserve the worst case first, then return what is unused
  const int64_t cap = kSlices * (2 * nrows + 1);
  const int64_t at = ab.alloc(cap);
  if (at < 0) {
    dfree(d_cnt);
    throw Error(-2, "no room for sliced row pointers");
  }
  build_sliced(cnt.data(), nrows, r0, id, NB, opt_.slice_rows, S.nz0, at, grp, sl, brp, dst);
  if ((int64_t)brp.size() > cap) throw Error(-3, "sliced row pointer overflow");
  ab.release(at + (int64_t)brp.size(), cap - (int64_t)brp.size());
  int32_t* brp_d = dual ? brpK : brpKT;
  HIPCHECK(hipMemcpyAsync(brp_d + at, brp.data(), sizeof(int32_t) * brp.size(), hipMemcpyHostToDevice, stream_));
  int32_t* d_dst = nullptr;
  int32_t* ci2 = nullptr;
  T* v2 = nullptr;
  double* v642 = nullptr;
  dalloc(&d_dst, nrows * kSlices);
  dalloc(&ci2, S.nnz);
  dalloc(&v2, S.nnz);
  if (sizeof(T) != 8) dalloc(&v642, S.nnz);
  HIPCHECK(hipMemcpyAsync(d_dst, dst.data(), sizeof(int32_t) * dst.size(), hipMemcpyHostToDevice, stream_));
  // the scatter writes positions nz0..nz0+nnz; shift the temporaries by -nz0
  slice_scatter_kernel<T><<<nblk(nrows), 256, 0, stream_>>>(rp, ci, val, v64, r0, nrows, c0, len, d_dst,
                                                            ci2 - S.nz0, v2 - S.nz0,
                                                            v642 ? v642 - S.nz0 : nullptr);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(ci + S.nz0, ci2, sizeof(int32_t) * S.nnz, hipMemcpyDeviceToDevice, stream_));
  HIPCHECK(hipMemcpyAsync(val + S.nz0, v2, sizeof(T) * S.nnz, hipMemcpyDeviceToDevice, stream_));
  if (v642) HIPCHECK(hipMemcpyAsync(v64 + S.nz0, v642, sizeof(double) * S.nnz, hipMemcpyDeviceToDevice, stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  dfree(d_cnt);
  dfree(d_dst);
  dfree(ci2);
  dfree(v2);
  dfree(v642);
  if (dual) {
    S.bD = grp;
    S.bDS = sl;
    S.brpD0 = at;
    S.brpDn = (int64_t)brp.size();
  } else {
    S.bP = grp;
    S.bPS = sl;
    S.brpP0 = at;
    S.brpPn = (int64_t)brp.size();
  }
  // slice partial sums live in space-sized buffers, allocated on first use
  if (dual && !spartD) dalloc(&spartD, 3 * kSlices * MS_);
  if (!dual && !spartP) dalloc(&spartP, 3 * kSlices * NS_);
}


// Row cap of the column-sorted plain blocks of a product of nrows rows over
// `width` columns (the packed index holds the column and the row in the
// block in 32 bits).
template <class T>
int64_t Engine<T>::plain_rows(int64_t nrows, int64_t width, int64_t min_blocks, int64_t min_rows) const {
  int cb = 0;
  while (((int64_t)1 << cb) < width) ++cb;
  const int64_t rows =
      std::min<int64_t>(std::min<int64_t>(opt_.sort_rows, kSortRowsPlain), (int64_t)1 << (32 - std::min(cb, 31)));
  return std::min<int64_t>(rows, std::max<int64_t>(min_rows, (nrows + min_blocks - 1) / min_blocks));
}

// Smaller column-sorted blocks for the LPs still running (status) when few
// are left (plain_shape for their number), so that the launches keep the
// CUs busy.  Products in sorted groups, column slices or plain tiles keep
// their layout.
template <class T>
void Engine<T>::reblock_for(const int* status) {
  std::vector<int> run;
  for (int s = 0; s < nslots_; ++s)
    if (slots_[s].used && status[s] == ST_RUNNING) run.push_back(s);
  if (run.empty()) return;
  int64_t minb = 0, minr = 0;
  plain_shape((int64_t)run.size(), &minb, &minr);
  bool changed = false;
  for (int s : run) {
    for (int d = 0; d < 2; ++d) {
      const bool dual = d == 1;
      const Slot& S = slots_[s];
      const int64_t cur = dual ? S.plainD : S.plainP;
      if (cur == 0) continue;
      if (plain_rows(dual ? S.m : S.n, dual ? S.n : S.m, minb, minr) < cur) {
        sort_blocks(s, dual, minb, minr, true);
        changed = true;
      }
    }
  }
  if (changed) sched_dirty_ = true;
}

// Column-sorted blocks of one LP's K (dual = true) or K^T, for a product
// that is not column-sliced: rows longer than a plain tile keep a long
// block; the other rows go to blocks of at most min(sort_rows,
// kSortRowsPlain, max(min_rows, rows / min_blocks)) rows and kSortEntries
// entries whose entries are put in column order, each column index packed
// with the entry's row in the block (see blk_rowbits).  Built on the device:
// a 64-bit key per entry (block index, packed key) and one stable radix
// sort.  From the row-major input (reblock false), or re-blocking a product
// already in column-sorted blocks into smaller ones (reblock true: each
// entry's row and column are read back from its packed key).
template <class T>
void Engine<T>::sort_blocks(int id, bool dual, int64_t min_blocks, int64_t min_rows, bool reblock) {
  Slot& S = slots_[id];
  const int64_t nrows = dual ? S.m : S.n;
  const int64_t base = dual ? S.row0 : S.col0;
  const int64_t c0 = dual ? S.col0 : S.row0;
  const int64_t width = dual ? S.n : S.m;
  const int32_t* rpd = dual ? K_rp : KT_rp;
  int32_t* ci = dual ? K_ci : KT_ci;
  T* val = dual ? K_v : KT_v;
  double* v64 = dual ? K_v64 : KT_v64;
  if (nrows == 0 || S.nnz == 0) return;
  int cb = 0;
  while (((int64_t)1 << cb) < width) ++cb;
  if (cb >= 32) return;
  const int64_t rows = plain_rows(nrows, width, min_blocks, min_rows);
  int rb = 0;
  while (((int64_t)1 << rb) < rows) ++rb;
  std::vector<int32_t> rp(nrows + 1);
  HIPCHECK(hipMemcpy(rp.data(), rpd + base, sizeof(int32_t) * (nrows + 1), hipMemcpyDeviceToHost));
  std::vector<Blk> out, sorted;
  auto emit = [&](int64_t a, int64_t e, int kind) {
    Blk k;
    k.r0 = (int32_t)(base + a);
    k.r1 = (int32_t)(base + e);
    k.inst = id;
    k.meta = blk_meta(kind, 1, 0) | (kind == BK_SORTED ? (rb << 25) : 0);
    k.gid = (int32_t)out.size();
    k.rp_off = kind == BK_SORTED ? (int32_t)c0 : 0;
    k.p0 = rp[a];
    k.pn = rp[e] - rp[a];
    out.push_back(k);
    if (kind == BK_SORTED) {
      sorted.push_back(k);
    }
  };
  int64_t start = 0, acc = 0;
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t len = (int64_t)rp[r + 1] - rp[r];
    if (len > kPlainNB) {
      if (r > start) emit(start, r, BK_SORTED);
      emit(r, r + 1, BK_LONG);
      start = r + 1;
      acc = 0;
      continue;
    }
    if ((r - start) >= rows || acc + len > kSortEntries) {
      if (r > start) emit(start, r, BK_SORTED);
      start = r;
      acc = 0;
    }
    acc += len;
  }
  if (nrows > start) emit(start, nrows, BK_SORTED);
  if (!sorted.empty()) {
    // one stable sort of the LP's entries by (block, key): the entries of
    // BK_SORTED blocks end in column order, all others where they were
    const int64_t nnz = S.nnz;
    const int nseg = (int)sorted.size();
    const int nall = (int)out.size();
    Blk *d_all = nullptr, *d_blk = nullptr;
    int32_t *src_in = nullptr, *src_out = nullptr;
    uint64_t *key_in = nullptr, *key_out = nullptr;
    T* v_tmp = nullptr;
    double* v64_tmp = nullptr;
    dalloc(&d_all, nall);
    dalloc(&d_blk, nseg);
    dalloc(&key_in, nnz);
    dalloc(&key_out, nnz);
    dalloc(&src_in, nnz);
    dalloc(&src_out, nnz);
    dalloc(&v_tmp, nnz);
    if (sizeof(T) != 8) dalloc(&v64_tmp, nnz);
    HIPCHECK(hipMemcpyAsync(d_all, out.data(), sizeof(Blk) * nall, hipMemcpyHostToDevice, stream_));
    HIPCHECK(hipMemcpyAsync(d_blk, sorted.data(), sizeof(Blk) * nseg, hipMemcpyHostToDevice, stream_));
    HIPCHECK(hipMemcpyAsync(v_tmp, val + S.nz0, sizeof(T) * nnz, hipMemcpyDeviceToDevice, stream_));
    if (v64_tmp)
      HIPCHECK(hipMemcpyAsync(v64_tmp, v64 + S.nz0, sizeof(double) * nnz, hipMemcpyDeviceToDevice, stream_));
    Blk* d_old = nullptr;
    int2* d_where = nullptr;
    if (!reblock) {
      block_keys_kernel<<<(unsigned)nall, kThreads, 0, stream_>>>(d_all, rpd, ci, S.nz0, key_in, src_in);
    } else {
      // each row's new block and its row in that block
      const std::vector<Blk>& old_blocks = dual ? S.bD : S.bP;
      std::vector<int2> where(nrows);
      for (int bi = 0; bi < nall; ++bi)
        for (int32_t r = out[bi].r0; r < out[bi].r1; ++r) where[r - base] = make_int2(bi, r - out[bi].r0);
      dalloc(&d_old, (int64_t)old_blocks.size());
      dalloc(&d_where, nrows);
      HIPCHECK(hipMemcpyAsync(d_old, old_blocks.data(), sizeof(Blk) * old_blocks.size(), hipMemcpyHostToDevice,
                              stream_));
      HIPCHECK(hipMemcpyAsync(d_where, where.data(), sizeof(int2) * nrows, hipMemcpyHostToDevice, stream_));
      reblock_keys_kernel<<<(unsigned)old_blocks.size(), kThreads, 0, stream_>>>(d_old, d_where, base, rb, ci,
                                                                                   S.nz0, key_in, src_in);
    }
    HIPCHECK(hipGetLastError());
    // low word: packed keys below 2^(cb + rb) in sorted blocks, entry
    // indices below 2^bits_for(longest block) elsewhere
    int32_t longest = 0;
    for (const Blk& b : out) longest = std::max(longest, b.pn);
    std::vector<int> shifts;
    radix_shifts(shifts, 0, std::min(32, std::max(cb + rb, bits_for(longest))));
    radix_shifts(shifts, 32, 32 + bits_for(nall - 1));
    radix_sort_pairs<uint64_t>(key_in, src_in, key_out, src_out, nnz, shifts, stream_);
    sorted_block_gather_kernel<T><<<(unsigned)nseg, kThreads, 0, stream_>>>(d_blk, S.nz0, key_out, src_out, val,
                                                                           v64, ci, v_tmp, v64_tmp);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(val + S.nz0, v_tmp, sizeof(T) * nnz, hipMemcpyDeviceToDevice, stream_));
    if (v64_tmp)
      HIPCHECK(hipMemcpyAsync(v64 + S.nz0, v64_tmp, sizeof(double) * nnz, hipMemcpyDeviceToDevice, stream_));
    HIPCHECK(hipStreamSynchronize(stream_));
    dfree(d_where);
    dfree(d_old);
    dfree(v64_tmp);
    dfree(v_tmp);
    dfree(src_out);
    dfree(src_in);
    dfree(key_out);
    dfree(key_in);
    dfree(d_blk);
    dfree(d_all);
  }
  (dual ? S.plainD : S.plainP) = sorted.empty() ? 0 : rows;
  if (dual) S.bD = out;
  else S.bP = out;
}

// Shape of a sorted-group layout for a product of nrows rows over `width`
// columns: the slice count, from nsl_min (the fewest that keep a slice of
// the gathered vector within slice_min_bytes) up to 8 for a product that
// must be sliced, else 1 or 2, and the rows per group, the largest that
// leaves at least group_blocks workgroups per product, fits the packed
// column index (row bits + column bits of a slice <= 32), Options::sort_rows
// and kSortRows.  More slices allow larger groups of a product with few
// rows; the slice count with the larger groups wins (a tie goes to fewer
// slices: fewer partial sums).  False when no shape fits.
template <class T>
bool Engine<T>::group_shape(int64_t nrows, int64_t width, int nsl_min, int* nsl, int64_t* rows) const {
  int best_s = 0;
  int64_t best_r = 0;
  for (int q = nsl_min; q <= (nsl_min == 1 ? 2 : kSlices); q *= 2) {
    const int64_t w = (width + q - 1) / q + 1;
    int cb = 0;
    while (((int64_t)1 << cb) < w) ++cb;
    if (cb >= 31) continue;
    int64_t r = std::min<int64_t>(std::min<int64_t>(opt_.sort_rows, kSortRows), (int64_t)1 << (32 - cb));
    while (r > kMaxRows && ((nrows + r - 1) / r) * q < opt_.group_blocks) r /= 2;
    if (r > best_r) {
      best_r = r;
      best_s = q;
    }
  }
  *nsl = best_s;
  *rows = best_r;
  return best_s > 0;
}

// Rows of the largest sorted group among the live LPs' K (dual) or K^T
// products: the slice kernel's dynamic LDS holds that many row sums.
template <class T>
int Engine<T>::group_lds_rows(bool dual) const {
  int r = 0;
  for (const Slot& sl : slots_)
    if (sl.used) r = std::max(r, dual ? sl.rowsD : sl.rowsP);
  return r;
}

// Sorted groups of one LP's K (dual = true; gathers over its variables) or
// K^T (gathers over its constraints): rows cut into groups of at most `rows`
// rows and kSortEntries entries per slice, each group's entries into nsl
// column slices, the entries of each (group, slice) block in column order,
// each column index packed with the entry's row in the group (see
// blk_rowbits).  Built on the device: per-slice counts of every row, keys in
// row-major block order, a radix sort by (block, key) (keys are unique in a
// block, so the order is fixed), a gather of the values.
template <class T>
void Engine<T>::group_sorted(int id, bool dual, int nsl, int64_t rows) {
  Slot& S = slots_[id];
  const int64_t nrows = dual ? S.m : S.n, r0 = dual ? S.row0 : S.col0, c0 = dual ? S.col0 : S.row0;
  const int64_t len = dual ? S.n : S.m;
  const int32_t* rp = dual ? K_rp : KT_rp;
  int32_t* ci = dual ? K_ci : KT_ci;
  T* val = dual ? K_v : KT_v;
  double* v64 = dual ? K_v64 : KT_v64;
  if (nrows == 0 || S.nnz == 0) return;
  if (nsl < 1 || nsl > kSlices || kSlices % nsl != 0) throw Error(-3, "bad slice count");
  int rb = 0;
  while (((int64_t)1 << rb) < rows) ++rb;
  int32_t* d_cnt = nullptr;
  dalloc(&d_cnt, nrows * nsl);
  slice_count_kernel<<<nblk(nrows), 256, 0, stream_>>>(rp, ci, r0, nrows, c0, len, nsl, d_cnt);
  std::vector<int32_t> cnt(nrows * nsl);
  HIPCHECK(hipMemcpyAsync(cnt.data(), d_cnt, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost, stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  dfree(d_cnt);
  // groups
  std::vector<std::pair<int64_t, int64_t>> groups;
  int64_t start = 0;
  int64_t acc[kSlices] = {0};
  for (int64_t r = 0; r < nrows; ++r) {
    const int32_t* c = cnt.data() + r * nsl;
    bool over = (r - start) >= rows;
    for (int q = 0; q < nsl; ++q) over |= acc[q] + c[q] > kSortEntries;
    if (over && r > start) {
      groups.emplace_back(start, r);
      start = r;
      for (int q = 0; q < nsl; ++q) acc[q] = 0;
    }
    for (int q = 0; q < nsl; ++q) acc[q] += c[q];
  }
  groups.emplace_back(start, nrows);
  // step-kernel blocks (kMaxRows rows each, row sums from the partials),
  // slice blocks, row-major positions and the row of each row in its group
  std::vector<Blk> grp, sl;
  for (int64_t a = 0; a < nrows; a += kMaxRows) {
    Blk ep;
    ep.r0 = (int32_t)(r0 + a);
    ep.r1 = (int32_t)(r0 + std::min<int64_t>(a + kMaxRows, nrows));
    ep.inst = id;
    ep.meta = blk_meta(BK_STREAM, nsl, 0) | kBlkPart;
    ep.gid = (int32_t)grp.size();
    ep.rp_off = 0;
    ep.p0 = 0;
    ep.pn = 0;
    grp.push_back(ep);
  }
  std::vector<int32_t> dst(nrows * nsl), rloc(nrows), off;
  int64_t pos = S.nz0, maxrows = 0;
  for (size_t g = 0; g < groups.size(); ++g) {
    const int64_t a = groups[g].first, e = groups[g].second;
    maxrows = std::max(maxrows, e - a);
    for (int64_t r = a; r < e; ++r) rloc[r] = (int32_t)(r - a);
    for (int q = 0; q < nsl; ++q) {
      Blk k;
      k.r0 = (int32_t)(r0 + a);
      k.r1 = (int32_t)(r0 + e);
      k.inst = id;
      k.gid = (int32_t)g;
      k.rp_off = (int32_t)(c0 + (q * len + nsl - 1) / nsl);
      k.p0 = (int32_t)pos;
      off.push_back((int32_t)(pos - S.nz0));
      for (int64_t r = a; r < e; ++r) {
        dst[r * nsl + q] = (int32_t)pos;
        pos += cnt[r * nsl + q];
      }
      k.pn = (int32_t)(pos - k.p0);
      k.meta = blk_meta(BK_STREAM, nsl, q) | (rb << 25);
      sl.push_back(k);
    }
  }
  off.push_back((int32_t)(pos - S.nz0));
  if (pos != S.nz0 + S.nnz) throw Error(-3, "sorted group layout does not cover the matrix");
  const int64_t nnz = S.nnz;
  const int nseg = (int)sl.size();
  int32_t *d_dst = nullptr, *d_rloc = nullptr, *d_off = nullptr, *src_in = nullptr, *src_out = nullptr;
  uint32_t* key32 = nullptr;
  uint64_t *key_in = nullptr, *key_out = nullptr;
  T* v2 = nullptr;
  double* v642 = nullptr;
  dalloc(&d_dst, nrows * nsl);
  dalloc(&d_rloc, nrows);
  dalloc(&d_off, (int64_t)off.size());
  dalloc(&key32, nnz);
  dalloc(&key_in, nnz);
  dalloc(&key_out, nnz);
  dalloc(&src_in, nnz);
  dalloc(&src_out, nnz);
  dalloc(&v2, nnz);
  if (sizeof(T) != 8) dalloc(&v642, nnz);
  HIPCHECK(hipMemcpyAsync(d_dst, dst.data(), sizeof(int32_t) * dst.size(), hipMemcpyHostToDevice, stream_));
  HIPCHECK(hipMemcpyAsync(d_rloc, rloc.data(), sizeof(int32_t) * rloc.size(), hipMemcpyHostToDevice, stream_));
  HIPCHECK(hipMemcpyAsync(d_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, stream_));
  // positions run from nz0: shift the temporaries by -nz0
  slice_keys_kernel<<<nblk(nrows), 256, 0, stream_>>>(rp, ci, r0, nrows, c0, len, nsl, d_dst, d_rloc, rb,
                                                      key32 - S.nz0, src_in - S.nz0);
  segment_keys_kernel<<<(unsigned)nseg, kThreads, 0, stream_>>>(d_off, key32, key_in);
  HIPCHECK(hipGetLastError());
  // one stable sort by (block, packed key): keys are unique within a block,
  // so each block ends in column order
  std::vector<int> shifts;
  radix_shifts(shifts, 0, std::min(32, bits_for((len + nsl - 1) / nsl) + rb));
  radix_shifts(shifts, 32, 32 + bits_for(nseg - 1));
  radix_sort_pairs<uint64_t>(key_in, src_in, key_out, src_out, nnz, shifts, stream_);
  sorted_gather_kernel<T><<<nblk(nnz), 256, 0, stream_>>>(key_out, src_out, val, v64, nnz, ci + S.nz0, v2, v642);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(val + S.nz0, v2, sizeof(T) * nnz, hipMemcpyDeviceToDevice, stream_));
  if (v642) HIPCHECK(hipMemcpyAsync(v64 + S.nz0, v642, sizeof(double) * nnz, hipMemcpyDeviceToDevice, stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  dfree(v642);
  dfree(v2);
  dfree(src_out);
  dfree(src_in);
  dfree(key_out);
  dfree(key_in);
  dfree(key32);
  dfree(d_off);
  dfree(d_rloc);
  dfree(d_dst);
  if (dual) {
    S.bD = grp;
    S.bDS = sl;
    S.brpD0 = 0;
    S.brpDn = 0;
    S.rowsD = (int)maxrows;
    if (!spartD) dalloc(&spartD, 3 * kSlices * MS_);
  } else {
    S.bP = grp;
    S.bPS = sl;
    S.brpP0 = 0;
    S.brpPn = 0;
    S.rowsP = (int)maxrows;
    if (!spartP) dalloc(&spartP, 3 * kSlices * NS_);
  }
}

template <class T>
void Engine<T>::set_params(const std::vector<int>& ids, double tol, int64_t max_iter, int64_t stall_checks) {
  HIPCHECK(hipStreamSynchronize(stream_));
  const int ni = (int)ids.size();
  if (ni == 0) return;
  std::vector<InstState> cur(ni);
  for (int k = 0; k < ni; ++k)
    HIPCHECK(hipMemcpyAsync(&cur[k], d_st + ids[k], sizeof(InstState), hipMemcpyDeviceToHost, stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  for (int k = 0; k < ni; ++k) {
    InstState& s = cur[k];
    s.tol = tol;
    s.max_iter = max_iter;
    s.stall_checks = stall_checks;
    s.best_kkt = INFINITY;
    s.best_check = s.checks;
    if (s.status != ST_RUNNING) {
      // (re)start from the last candidate as a fresh epoch is not supported
      // for finished LPs; a parked LP starts here
      if (s.checks == 0) {
        s.status = ST_RUNNING;
        s.phase = PH_NORMAL;
        s.kbase = g_next_;
        s.tbase = g_next_;
        s.next_check = g_next_ + s.C;
      }
    }
    slots_[ids[k]].watched = true;
    slots_[ids[k]].reported = false;
  }
  InstState* d_src = nullptr;
  int* d_ids = nullptr;
  dalloc(&d_src, ni);
  dalloc(&d_ids, ni);
  HIPCHECK(hipMemcpyAsync(d_src, cur.data(), sizeof(InstState) * ni, hipMemcpyHostToDevice, stream_));
  HIPCHECK(hipMemcpyAsync(d_ids, ids.data(), sizeof(int) * ni, hipMemcpyHostToDevice, stream_));
  write_states_kernel<<<nblk(ni), 256, 0, stream_>>>(d_st, d_status, d_cnt, d_ids, d_src, ni);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(stream_));
  dfree(d_src);
  dfree(d_ids);
  for (int k = 0; k < ni; ++k) h_status[0][ids[k]] = h_status[1][ids[k]] = cur[k].status;
}

// Many LPs in one schedule: each LP's blocks go to one XCD.  Workgroups are
// dispatched round-robin over the 8 XCDs, so schedule position p runs on XCD
// p % 8; LPs are assigned to 8 lanes (largest first, to the lane with the
// fewest blocks) and lane q fills positions q, q + 8, ... (padded with no-op
// blocks).  Each XCD's L2 then caches only the gathered vectors of its own
// LPs instead of every running LP's.
template <class T>
void Engine<T>::pin_to_xcds(std::vector<Blk>& v, const std::vector<std::pair<int, int>>& ranges) const {
  std::vector<int> order(ranges.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return ranges[a].second - ranges[a].first > ranges[b].second - ranges[b].first;
  });
  std::vector<std::vector<Blk>> lane(kSlices);
  for (int i : order) {
    int q = 0;
    for (int k = 1; k < kSlices; ++k)
      if (lane[k].size() < lane[q].size()) q = k;
    for (int p = ranges[i].first; p < ranges[i].second; ++p) lane[q].push_back(v[p]);
  }
  size_t len = 0;
  for (auto& l : lane) len = std::max(len, l.size());
  Blk pad{};
  pad.meta = blk_meta(BK_PAD, 1, 0);
  std::vector<Blk> out;
  out.reserve(len * kSlices);
  for (size_t r = 0; r < len; ++r)
    for (int q = 0; q < kSlices; ++q) out.push_back(r < lane[q].size() ? lane[q][r] : pad);
  v.swap(out);
}

// The vectors of a step and the matrix tiles read before the cache budget is
// used up are read normally and stay in the last-level cache from one step to
// the next; the remaining tiles are streamed with non-temporal loads, so that
// they do not evict what fits.  (A matrix pair larger than the cache read
// round-robin would otherwise evict every line before its next use.)
template <class T>
void Engine<T>::mark_streaming(const std::vector<int>& live, std::vector<Blk>& P, std::vector<Blk>& PS,
                               std::vector<Blk>& DS, std::vector<Blk>& D) const {
  const int64_t budget = opt_.cache_budget_bytes;
  int64_t used = 0;
  for (int s : live) {
    const Slot& sl = slots_[s];
    // n-space: c, l, u, x, x0, xbar; m-space: q, y, y0; row pointers; slice partial sums
    used += (int64_t)sizeof(T) * (6 * sl.n + 3 * sl.m) + 4 * (sl.n + sl.m);
    if (!sl.bDS.empty()) used += (int64_t)(sizeof(T) + 4) * kSlices * sl.m;
    if (!sl.bPS.empty()) used += (int64_t)(sizeof(T) + 4) * kSlices * sl.n;
  }
  auto mark = [&](std::vector<Blk>& v) {
    for (Blk& k : v) {
      k.meta &= ~kBlkNT;
      if (blk_kind(k) == BK_PAD) continue;
      const int64_t bytes = (int64_t)k.pn * (int64_t)(sizeof(T) + 4);
      if (budget >= 0 && used + bytes > budget) k.meta |= kBlkNT;
      else used += bytes;
    }
  };
  mark(P);
  mark(PS);
  mark(DS);
  mark(D);
}

template <class T>
void Engine<T>::rebuild_schedules() {
  std::vector<Blk> P, D, PS, DS;
  std::vector<int> live;
  std::vector<int4> rg;
  auto append = [](std::vector<Blk>& dst, const std::vector<Blk>& src, int32_t goff) {
    for (Blk k : src) {
      k.gid += goff;
      dst.push_back(k);
    }
  };
  for (int s = 0; s < nslots_; ++s) {
    const Slot& sl = slots_[s];
    if (!sl.used) continue;
    if (finished_ && finished_[s] != ST_RUNNING) continue;  // done: its blocks would only exit
    int4 r;
    r.x = (int)P.size();
    append(PS, sl.bPS, r.x);
    append(P, sl.bP, r.x);
    r.y = (int)P.size();
    r.z = (int)D.size();
    append(DS, sl.bDS, r.z);
    append(D, sl.bD, r.z);
    r.w = (int)D.size();
    live.push_back(s);
    rg.push_back(r);
  }
  for (double& v : sched_size_) v = 0.0;
  for (int s : live) {
    sched_size_[0] += (double)slots_[s].nnz;
    sched_size_[1] += (double)slots_[s].n;
    sched_size_[2] += (double)slots_[s].m;
  }
  if (opt_.xcd_pin && (int)live.size() >= kPinMinLPs) {
    std::vector<std::pair<int, int>> rp, rd;
    for (const int4& r : rg) {
      rp.push_back({r.x, r.y});
      rd.push_back({r.z, r.w});
    }
    pin_to_xcds(P, rp);
    pin_to_xcds(D, rd);
  }
  ldsP_ = ldsD_ = 0;
  for (int s2 : live) {
    ldsP_ = std::max(ldsP_, slots_[s2].rowsP);
    ldsD_ = std::max(ldsD_, slots_[s2].rowsD);
  }
  // threads per sorted-group workgroup: the configured count, or enough for
  // about eight waves per CU over the product's workgroups (measured: the
  // products are bound by cache-line gathers, so large groups with few
  // workgroups need wide ones)
  auto pick = [&](size_t nb) {
    if (opt_.group_threads > 0) return opt_.group_threads;
    const int64_t t = (int64_t)kCUs * 8 * 64 / std::max<int64_t>(1, (int64_t)nb);
    return t >= 1024 ? 1024 : t >= 512 ? 512 : 256;
  };
  tpbP_ = pick(PS.size());
  tpbD_ = pick(DS.size());
  mark_streaming(live, P, PS, DS, D);
  HIPCHECK(hipStreamSynchronize(stream_));
  auto upload = [&](std::vector<Blk>& v, Blk*& d, int64_t& cap, int64_t& n, double** part) {
    if ((int64_t)v.size() > cap) {
      dfree(d);
      if (part) dfree(*part);
      cap = std::max<int64_t>((int64_t)v.size(), 2 * cap);
      dalloc(&d, cap);
      if (part) dalloc(part, cap * kNS);
    }
    n = (int64_t)v.size();
    if (n) HIPCHECK(hipMemcpyAsync(d, v.data(), sizeof(Blk) * n, hipMemcpyHostToDevice, stream_));
  };
  scheduled_ = (int)live.size();
  if ((int64_t)live.size() > cap_live_) {
    dfree(d_live_);
    cap_live_ = std::max<int64_t>((int64_t)live.size(), 2 * cap_live_);
    dalloc(&d_live_, cap_live_);
  }
  if (!live.empty())
    HIPCHECK(hipMemcpyAsync(d_live_, live.data(), sizeof(int) * live.size(), hipMemcpyHostToDevice, stream_));
  upload(P, d_schedP, capP_, nP_, &partP);
  upload(D, d_schedD, capD_, nD_, &partD);
  upload(PS, d_schedPS, capPS_, nPS_, nullptr);
  upload(DS, d_schedDS, capDS_, nDS_, nullptr);
  if (!live.empty()) {
    int* d_ids = nullptr;
    int4* d_rg = nullptr;
    dalloc(&d_ids, (int64_t)live.size());
    dalloc(&d_rg, (int64_t)live.size());
    HIPCHECK(hipMemcpyAsync(d_ids, live.data(), sizeof(int) * live.size(), hipMemcpyHostToDevice, stream_));
    HIPCHECK(hipMemcpyAsync(d_rg, rg.data(), sizeof(int4) * rg.size(), hipMemcpyHostToDevice, stream_));
    set_ranges_kernel<<<nblk((int64_t)live.size()), 256, 0, stream_>>>(d_st, d_ids, d_rg, (int)live.size());
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(stream_));
    dfree(d_ids);
    dfree(d_rg);
  }
  if (gexec_) {
    (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
  }
  if (graph_) {
    (void)hipGraphDestroy(graph_);
    graph_ = nullptr;
  }
  sched_dirty_ = false;
}

// The sorted-group slice kernel in the configured shape (threads per
// workgroup, gather order), its dynamic LDS raised to what the groups need.
template <class T>
template <bool DUAL>
void Engine<T>::launch_group(unsigned g, int tpb, size_t lds, const IterArgs<T>& A, int step) {
  auto go = [&](auto kern, int t) { kern<<<g, t, lds, stream_>>>(A, step); };
  const bool b = opt_.group_batched != 0;
  switch (tpb) {
    case 512:
      if (b) go(sorted_group_step<T, DUAL, 512, true>, 512);
      else go(sorted_group_step<T, DUAL, 512, false>, 512);
      break;
    case 1024:
      if (b) go(sorted_group_step<T, DUAL, 1024, true>, 1024);
      else go(sorted_group_step<T, DUAL, 1024, false>, 1024);
      break;
    default:
      if (b) go(sorted_group_step<T, DUAL, 256, true>, 256);
      else go(sorted_group_step<T, DUAL, 256, false>, 256);
      break;
  }
}

template <class T>
void Engine<T>::launch_slices(bool dual, const IterArgs<T>& A, int step) {
  const unsigned g = (unsigned)(dual ? nDS_ : nPS_);
  if (opt_.slice_sort) {
    const size_t lds = sizeof(double) * (size_t)std::max(1, dual ? ldsD_ : ldsP_);
    if (dual) launch_group<true>(g, dual ? tpbD_ : tpbP_, lds, A, step);
    else launch_group<false>(g, dual ? tpbD_ : tpbP_, lds, A, step);
    return;
  }
  switch (opt_.slice_entries) {
    case 256:
      if (dual) dual_slice_step<T, 256><<<g, kThreads, 0, stream_>>>(A, step);
      else primal_slice_step<T, 256><<<g, kThreads, 0, stream_>>>(A, step);
      break;
    case 1024:
      if (dual) dual_slice_step<T, 1024><<<g, kThreads, 0, stream_>>>(A, step);
      else primal_slice_step<T, 1024><<<g, kThreads, 0, stream_>>>(A, step);
      break;
    default:
      if (dual) dual_slice_step<T, 512><<<g, kThreads, 0, stream_>>>(A, step);
      else primal_slice_step<T, 512><<<g, kThreads, 0, stream_>>>(A, step);
      break;
  }
}

template <class T>
void Engine<T>::launch_chunk() {
  if (sched_dirty_ && !compacted_) rebuild_schedules();
  if (nP_ == 0 || nD_ == 0) return;
  const IterArgs<T> A = args();
  const int CH = opt_.chunk;
  const bool prof = opt_.profile > 0 && (chunk_count_ % opt_.profile) == 0;
  ++chunk_count_;
  if (prof) {
    collect_times();  // the previous timed chunk (long finished) frees the event pool
    if ((int)pev_.size() != 6 * CH) {
      for (hipEvent_t e : pev_) (void)hipEventDestroy(e);
      pev_.assign(6 * CH, nullptr);
      for (auto& e : pev_) HIPCHECK(hipEventCreate(&e));
    }
  }
  auto enqueue = [&](bool timed) {
    tick_kernel<<<1, 1, 0, stream_>>>(d_gbase, (int64_t)CH);
    for (int i = 0; i < CH; ++i) {
      hipEvent_t* e = timed ? &pev_[6 * i] : nullptr;
      if (timed) HIPCHECK(hipEventRecord(e[0], stream_));
      if (nPS_) launch_slices(false, A, i);
      if (timed) HIPCHECK(hipEventRecord(e[1], stream_));
      primal_step<T><<<(unsigned)nP_, kThreads, 0, stream_>>>(A, i);
      if (timed) HIPCHECK(hipEventRecord(e[2], stream_));
      if (nDS_) launch_slices(true, A, i);
      if (timed) HIPCHECK(hipEventRecord(e[3], stream_));
      dual_step<T><<<(unsigned)nD_, kThreads, 0, stream_>>>(A, i);
      if (timed) {
        HIPCHECK(hipEventRecord(e[4], stream_));
        HIPCHECK(hipEventRecord(e[5], stream_));  // empty pair: the events' own cost
      }
      control_kernel<<<(unsigned)scheduled_, kThreads, 0, stream_>>>(d_st, d_live_, partP, partD, d_gbase, i,
                                                                     d_status);
    }
  };
  if (prof) {
    enqueue(true);
    HIPCHECK(hipGetLastError());
    pev_pending_ = true;
    pev_slices_[0] = nPS_ > 0;
    pev_slices_[1] = nDS_ > 0;
    for (int q = 0; q < 3; ++q) pev_size_[q] = sched_size_[q];
  } else if (opt_.use_graph) {
    if (!gexec_) {
      HIPCHECK(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
      enqueue(false);
      HIPCHECK(hipStreamEndCapture(stream_, &graph_));
      HIPCHECK(hipGraphInstantiate(&gexec_, graph_, nullptr, nullptr, 0));
    }
    HIPCHECK(hipGraphLaunch(gexec_, stream_));
  } else {
    enqueue(false);
    HIPCHECK(hipGetLastError());
  }
  g_next_ += CH;
}

template <class T>
void Engine<T>::collect_times() {
  if (!pev_pending_) return;
  HIPCHECK(hipEventSynchronize(pev_.back()));
  for (size_t k = 0; k + 5 < pev_.size(); k += 6) {
    float d[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    for (int q = 0; q < 5; ++q) HIPCHECK(hipEventElapsedTime(&d[q], pev_[k + q], pev_[k + q + 1]));
    // an event pair around a kernel that was not launched measures only the
    // events' own overhead: count it as no time
    if (pev_slices_[0]) ktimes_.primal_slice_ms += d[0];
    ktimes_.primal_ms += d[1];
    if (pev_slices_[1]) ktimes_.dual_slice_ms += d[2];
    ktimes_.dual_ms += d[3];
    ktimes_.event_pair_ms += d[4];
    ktimes_.nnz += pev_size_[0];
    ktimes_.n += pev_size_[1];
    ktimes_.m += pev_size_[2];
    ktimes_.launches += 1;
  }
  pev_pending_ = false;
}

template <class T>
void Engine<T>::run(double time_limit_s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (sched_dirty_) {
    compacted_ = false;
    rebuild_schedules();
  }
  auto all_done = [&](const int* h) {
    for (int s = 0; s < nslots_; ++s)
      if (slots_[s].used && slots_[s].watched && h[s] == ST_RUNNING) return false;
    return true;
  };
  if (all_done(h_status[0]) && all_done(h_status[1])) {
    HIPCHECK(hipStreamSynchronize(stream_));
    HIPCHECK(hipMemcpy(h_status[0], d_status, sizeof(int) * nslots_, hipMemcpyDeviceToHost));
    if (all_done(h_status[0])) return;
  }
  int64_t j = 0;
  bool limit_set = false;
  double next_print = (double)opt_.verbose;
  while (true) {
    launch_chunk();
    HIPCHECK(hipMemcpyAsync(h_status[j & 1], d_status, sizeof(int) * nslots_, hipMemcpyDeviceToHost, stream_));
    if (ev_[j & 1]) HIPCHECK(hipEventRecord(ev_[j & 1], stream_));
    else HIPCHECK(hipStreamSynchronize(stream_));
    if (j >= 1) {
      if (ev_[(j - 1) & 1]) HIPCHECK(hipEventSynchronize(ev_[(j - 1) & 1]));
      if (all_done(h_status[(j - 1) & 1])) break;
      // leave finished LPs out of the schedules once half of them are done
      int running = 0;
      for (int s = 0; s < nslots_; ++s) running += slots_[s].used && h_status[(j - 1) & 1][s] == ST_RUNNING;
      if (scheduled_ > 1 && 2 * running <= scheduled_) {
        HIPCHECK(hipStreamSynchronize(stream_));
        HIPCHECK(hipMemcpy(h_status[0], d_status, sizeof(int) * nslots_, hipMemcpyDeviceToHost));
        std::memcpy(h_status[1], h_status[0], sizeof(int) * nslots_);
        finished_ = h_status[0];
        reblock_for(h_status[0]);
        rebuild_schedules();
        finished_ = nullptr;
        sched_dirty_ = true;  // the next add / remove / solve rebuilds the full schedules
        compacted_ = true;
      }
    }
    ++j;
    if (opt_.verbose > 0) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (el >= next_print) {
        next_print = el + (double)opt_.verbose;
        int first = -1, running = 0, watched = 0;
        for (int s = 0; s < nslots_; ++s) {
          if (!slots_[s].used || !slots_[s].watched) continue;
          ++watched;
          if (h_status[(j - 1) & 1][s] == ST_RUNNING) {
            ++running;
            if (first < 0) first = s;
          }
        }
        if (first >= 0) {
          InstState st;
          HIPCHECK(hipMemcpy(&st, d_st + first, sizeof(InstState), hipMemcpyDeviceToHost));
          fprintf(stderr, "[halp] %.1fs step %lld: %d/%d LPs running; LP %d: iters %lld restarts %lld kkt %.3e "
                  "(p %.2e d %.2e gap %.2e) omega %.3e\n", el, (long long)g_next_, running, watched, first,
                  (long long)st.iters, (long long)st.nrest, st.kkt, st.rel_p, st.rel_d, st.rel_gap, st.omega);
          fflush(stderr);
        }
      }
    }
    if (!limit_set && time_limit_s >= 0.0) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (el > time_limit_s) {
        set_limit_status_kernel<<<nblk(nslots_), 256, 0, stream_>>>(d_st, d_status, nslots_, ST_TIME_LIMIT);
        limit_set = true;
      }
    }
  }
  HIPCHECK(hipStreamSynchronize(stream_));
  HIPCHECK(hipMemcpy(h_status[0], d_status, sizeof(int) * nslots_, hipMemcpyDeviceToHost));
  std::memcpy(h_status[1], h_status[0], sizeof(int) * nslots_);
  collect_times();
}

template <class T>
std::vector<int> Engine<T>::advance(int chunks) {
  for (int i = 0; i < chunks; ++i) launch_chunk();
  HIPCHECK(hipMemcpyAsync(h_status[0], d_status, sizeof(int) * nslots_, hipMemcpyDeviceToHost, stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  collect_times();
  std::vector<int> done;
  for (int s = 0; s < nslots_; ++s) {
    if (slots_[s].used && slots_[s].watched && !slots_[s].reported && h_status[0][s] != ST_RUNNING) {
      slots_[s].reported = true;
      done.push_back(s);
    }
  }
  return done;
}

template <class T>
void Engine<T>::remove(const std::vector<int>& ids) {
  HIPCHECK(hipStreamSynchronize(stream_));
  for (int id : ids) {
    Slot& S = slots_.at(id);
    if (!S.used) continue;
    am_.release(S.row0, S.m + 1);
    an_.release(S.col0, S.n + 1);
    az_.release(S.nz0, S.nnz);
    abK_.release(S.brpD0, S.brpDn);
    abKT_.release(S.brpP0, S.brpPn);
    S = Slot();
    h_status[0][id] = h_status[1][id] = 0;
  }
  sched_dirty_ = true;
  compacted_ = false;
}

template <class T>
Result Engine<T>::result(int id) {
  if (id < 0 || id >= nslots_ || !slots_[id].used) throw Error(-1, "invalid LP id");
  InstState s;
  HIPCHECK(hipStreamSynchronize(stream_));
  HIPCHECK(hipMemcpy(&s, d_st + id, sizeof(InstState), hipMemcpyDeviceToHost));
  Result r;
  r.status = s.status;
  if (s.checks == 0 && s.status == ST_ITER_LIMIT) r.status = 0;  // parked, never run
  r.iters = s.iters;
  r.restarts = s.nrest;
  r.checks = s.checks;
  r.kkt = s.kkt;
  r.rel_p = s.rel_p;
  r.rel_d = s.rel_d;
  r.rel_gap = s.rel_gap;
  r.pobj = s.pobj;
  r.dobj = s.dobj;
  r.resid = s.resid;
  r.omega = s.omega;
  r.eta = s.eta;
  r.sigma_hat = s.sigma_hat;
  r.power_iters = s.pw_iter;
  r.ray = s.ray;
  r.active_changes = s.act_changes;
  r.ident_iters = s.ident_iters;
  return r;
}

template <class T>
void Engine<T>::solution(int id, double* xo, double* yo, bool to_device) {
  if (id < 0 || id >= nslots_ || !slots_[id].used) throw Error(-1, "invalid LP id");
  const Slot& S = slots_[id];
  double* tmp = nullptr;
  dalloc(&tmp, S.n + S.m);
  unscale_kernel<T><<<nblk(S.n), 256, 0, stream_>>>(xT, Dc, S.col0, S.n, tmp);
  if (S.m) unscale_kernel<T><<<nblk(S.m), 256, 0, stream_>>>(yT, Dr, S.row0, S.m, tmp + S.n);
  HIPCHECK(hipGetLastError());
  const auto kind = to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (xo) HIPCHECK(hipMemcpyAsync(xo, tmp, sizeof(double) * S.n, kind, stream_));
  if (yo && S.m) HIPCHECK(hipMemcpyAsync(yo, tmp + S.n, sizeof(double) * S.m, kind, stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  dfree(tmp);
}

template <class T>
void Engine<T>::certificate(int id, double* ray, bool to_device) {
  if (id < 0 || id >= nslots_ || !slots_[id].used) throw Error(-1, "invalid LP id");
  const Slot& S = slots_[id];
  InstState s;
  HIPCHECK(hipStreamSynchronize(stream_));
  HIPCHECK(hipMemcpy(&s, d_st + id, sizeof(InstState), hipMemcpyDeviceToHost));
  if (s.status != ST_PRIMAL_INFEAS && s.status != ST_DUAL_INFEAS)
    throw Error(-4, "no certificate: the LP was not found infeasible");
  const bool primal = s.status == ST_PRIMAL_INFEAS;
  const int64_t len = primal ? S.m : S.n;
  double* tmp = nullptr;
  dalloc(&tmp, len);
  if (primal)
    unscale_kernel<T><<<nblk(len), 256, 0, stream_>>>(s.ray == 1 ? cy1 : cy2, Dr, S.row0, len, tmp);
  else
    unscale_kernel<T><<<nblk(len), 256, 0, stream_>>>(s.ray == 1 ? cx1 : cx2, Dc, S.col0, len, tmp);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(ray, tmp, sizeof(double) * len, to_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  dfree(tmp);
}

template <class T>
void Engine<T>::export_point(int id, double* xo, double* yo, double* omega) {
  if (id < 0 || id >= nslots_ || !slots_[id].used) throw Error(-1, "invalid LP id");
  const Slot& S = slots_[id];
  copy_state_kernel<T><<<nblk(S.n), 256, 0, stream_>>>(xT, xo, S.col0, S.n);
  if (S.m) copy_state_kernel<T><<<nblk(S.m), 256, 0, stream_>>>(yT, yo, S.row0, S.m);
  HIPCHECK(hipGetLastError());
  InstState st;
  HIPCHECK(hipMemcpyAsync(&st, d_st + id, sizeof(InstState), hipMemcpyDeviceToHost, stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  *omega = st.omega;
}

template <class T>
void Engine<T>::import_point(int id, const double* xi, const double* yi, double omega) {
  if (id < 0 || id >= nslots_ || !slots_[id].used) throw Error(-1, "invalid LP id");
  const Slot& S = slots_[id];
  load_point_kernel<T><<<nblk(S.n), 256, 0, stream_>>>(xi, x, x0, S.col0, S.n);
  if (S.m) load_point_kernel<T><<<nblk(S.m), 256, 0, stream_>>>(yi, y, y0, S.row0, S.m);
  HIPCHECK(hipGetLastError());
  InstState st;
  HIPCHECK(hipMemcpyAsync(&st, d_st + id, sizeof(InstState), hipMemcpyDeviceToHost, stream_));
  HIPCHECK(hipStreamSynchronize(stream_));
  if (omega > 0.0 && std::isfinite(omega)) {  // else keep the LP's initial primal weight
    st.omega = omega;
    st.tau = st.eta / omega;
    st.sigma = st.eta * omega;
  }
  InstState* d_src = nullptr;
  int* d_ids = nullptr;
  dalloc(&d_src, 1);
  dalloc(&d_ids, 1);
  HIPCHECK(hipMemcpyAsync(d_src, &st, sizeof(InstState), hipMemcpyHostToDevice, stream_));
  HIPCHECK(hipMemcpyAsync(d_ids, &id, sizeof(int), hipMemcpyHostToDevice, stream_));
  write_states_kernel<<<1, 256, 0, stream_>>>(d_st, d_status, d_cnt, d_ids, d_src, 1);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(stream_));
  dfree(d_src);
  dfree(d_ids);
}

template <class T>
void Engine<T>::stored_matrix(int id, bool transpose, int32_t* rp, int32_t* ci, double* val) {
  if (id < 0 || id >= nslots_ || !slots_[id].used) throw Error(-1, "invalid LP id");
  const Slot& S = slots_[id];
  const std::vector<Blk>& blocks = transpose ? S.bP : S.bD;
  const std::vector<Blk>& slices = transpose ? S.bPS : S.bDS;
  bool row_order = slices.empty();
  for (const Blk& b : blocks) row_order &= blk_kind(b) != BK_SORTED && !blk_part(b);
  if (!row_order) throw Error(-4, "the product is not stored in row order (column slices or sorted layout)");
  const int64_t rows = transpose ? S.n : S.m, r0 = transpose ? S.col0 : S.row0;
  const int64_t c0 = transpose ? S.row0 : S.col0;
  HIPCHECK(hipStreamSynchronize(stream_));
  HIPCHECK(hipMemcpy(rp, (transpose ? KT_rp : K_rp) + r0, sizeof(int32_t) * (rows + 1), hipMemcpyDeviceToHost));
  if (S.nnz > 0) {
    HIPCHECK(hipMemcpy(ci, (transpose ? KT_ci : K_ci) + S.nz0, sizeof(int32_t) * S.nnz, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(val, (transpose ? KT_v64 : K_v64) + S.nz0, sizeof(double) * S.nnz,
                       hipMemcpyDeviceToHost));
  }
  for (int64_t r = 0; r <= rows; ++r) rp[r] -= (int32_t)S.nz0;
  for (int64_t e = 0; e < S.nnz; ++e) ci[e] -= (int32_t)c0;
}

int narrow_row_ptr(const int64_t* src, int32_t* dst, int64_t count, hipStream_t stream) {
  if (count <= 0) return 0;
  int* d_bad = nullptr;
  dalloc(&d_bad, 1);
  HIPCHECK(hipMemsetAsync(d_bad, 0, sizeof(int), stream));
  narrow_row_ptr_kernel<<<nblk(count), 256, 0, stream>>>(src, dst, count, d_bad);
  HIPCHECK(hipGetLastError());
  int bad = 0;
  HIPCHECK(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIPCHECK(hipStreamSynchronize(stream));
  dfree(d_bad);
  return bad;
}

std::unique_ptr<EngineBase> make_engine(const Options& opt, hipStream_t stream, int64_t cap_m, int64_t cap_n,
                                        int64_t cap_nnz, int max_slots) {
  if (opt.precision == 1)
    return std::unique_ptr<EngineBase>(new Engine<float>(opt, stream, cap_m, cap_n, cap_nnz, max_slots));
  return std::unique_ptr<EngineBase>(new Engine<double>(opt, stream, cap_m, cap_n, cap_nnz, max_slots));
}

}  // namespace halp

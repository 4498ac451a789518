// C ABI over the solver engine (see include/halp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/halp.h"
#include "engine.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

template <class F>
int guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const halp::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(LP_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(LP_ERR_DEVICE, e.what());
  }
}

halp::Options to_opts(const lp_options* o) {
  halp::Options r;
  if (!o) return r;
  r.method = o->method;
  r.precision = o->precision;
  r.ruiz_iters = o->ruiz_iters;
  r.pc_alpha = o->pc_alpha;
  r.check_every = o->check_every;
  r.restart_beta = o->restart_beta;
  r.artificial_restart = o->artificial_restart;
  r.step_safety = o->step_safety;
  r.power_max_iters = o->power_max_iters;
  r.power_min_iters = o->power_min_iters;
  r.power_rtol = o->power_rtol;
  r.eps_infeas = o->eps_infeas;
  r.primal_weight = o->primal_weight;
  r.seed = o->seed;
  r.eta = o->eta;
  r.omega0 = o->omega0;
  r.chunk = o->chunk;
  r.use_graph = o->use_graph;
  r.profile = o->profile;
  r.slice_min_bytes = o->slice_min_bytes;
  r.polish_tol = o->polish_tol;
  r.verbose = o->verbose;
  r.cache_budget_bytes = o->cache_budget_bytes;
  r.stall_checks = o->stall_checks;
  r.restart_mode = o->restart_mode;
  r.fixed_restart_len = o->fixed_restart_len;
  r.xcd_pin = o->xcd_pin;
  r.tile_rows = o->tile_rows;
  r.slice_entries = o->slice_entries;
  r.slice_rows = o->slice_rows;
  r.slice_sort = o->slice_sort;
  r.sort_rows = o->sort_rows;
  r.plain_sort = o->plain_sort;
  r.group_threads = o->group_threads;
  r.group_batched = o->group_batched;
  r.group_blocks = o->group_blocks;
  r.polish_weight = o->polish_weight;
  return r;
}

void check_opts(const halp::Options& o) {
  if (o.restart_mode < 0 || o.restart_mode > 2) throw halp::Error(LP_ERR_INVALID, "restart_mode must be 0, 1 or 2");
  if (o.tile_rows < 1 || o.tile_rows > halp::kMaxRows || o.slice_rows < 1 || o.slice_rows > halp::kMaxRows)
    throw halp::Error(LP_ERR_INVALID, "tile_rows and slice_rows must be in 1..256");
  if (o.slice_entries != 256 && o.slice_entries != 512 && o.slice_entries != 1024)
    throw halp::Error(LP_ERR_INVALID, "slice_entries must be 256, 512 or 1024");
  if (o.slice_sort < 0 || o.slice_sort > 1) throw halp::Error(LP_ERR_INVALID, "slice_sort must be 0 or 1");
  if (o.plain_sort < 0 || o.plain_sort > 1) throw halp::Error(LP_ERR_INVALID, "plain_sort must be 0 or 1");
  if (o.sort_rows < 1 || o.sort_rows > halp::kSortRows)
    throw halp::Error(LP_ERR_INVALID, "sort_rows must be in 1..16384");
  if (o.group_threads != 0 && o.group_threads != 256 && o.group_threads != 512 && o.group_threads != 1024)
    throw halp::Error(LP_ERR_INVALID, "group_threads must be 0, 256, 512 or 1024");
  if (o.group_batched < 0 || o.group_batched > 1) throw halp::Error(LP_ERR_INVALID, "group_batched must be 0 or 1");
  if (o.group_blocks < 0) throw halp::Error(LP_ERR_INVALID, "group_blocks must be >= 0");
  if (o.polish_weight < 0 || o.polish_weight > 2) throw halp::Error(LP_ERR_INVALID, "polish_weight must be 0, 1 or 2");
  if (o.restart_mode == 1 && o.fixed_restart_len < 1)
    throw halp::Error(LP_ERR_INVALID, "fixed restarts need fixed_restart_len >= 1");
  if (o.method < 0 || o.method > 2) throw halp::Error(LP_ERR_INVALID, "method must be 0, 1 or 2");
  if (o.precision != 0 && o.precision != 1) throw halp::Error(LP_ERR_INVALID, "precision must be 0 or 1");
  if (o.check_every < 1 || o.chunk < 1 || o.chunk > 4096)
    throw halp::Error(LP_ERR_INVALID, "check_every >= 1 and 1 <= chunk <= 4096 required");
  if (o.ruiz_iters < 0 || o.power_max_iters < 1 || o.power_min_iters < 1)
    throw halp::Error(LP_ERR_INVALID, "bad iteration counts");
  if (!(o.step_safety > 0.0) || !(o.restart_beta > 0.0) || !(o.eps_infeas > 0.0))
    throw halp::Error(LP_ERR_INVALID, "step_safety, restart_beta and eps_infeas must be positive");
}

lp_result to_result(const halp::Result& r, double seconds) {
  lp_result o;
  std::memset(&o, 0, sizeof(o));
  o.status = r.status;
  o.ray = r.ray;
  o.iters = r.iters;
  o.restarts = r.restarts;
  o.checks = r.checks;
  o.pobj = r.pobj;
  o.dobj = r.dobj;
  o.rel_kkt = r.kkt;
  o.rel_primal = r.rel_p;
  o.rel_dual = r.rel_d;
  o.rel_gap = r.rel_gap;
  o.omega = r.omega;
  o.eta = r.eta;
  o.sigma_hat = r.sigma_hat;
  o.power_iters = r.power_iters;
  o.seconds = seconds;
  o.active_changes = r.active_changes;
  o.ident_iters = r.ident_iters;
  return o;
}

halp::Problem to_problem(const lp_problem& p) {
  halp::Problem q;
  q.n = p.n;
  q.m_eq = p.m_eq;
  q.m_ineq = p.m_ineq;
  q.rp = p.row_ptr;
  q.ci = p.col_idx;
  q.val = p.val;
  q.c = p.c;
  q.rhs = p.rhs;
  q.lb = p.lb;
  q.ub = p.ub;
  return q;
}

int64_t read_nnz(const lp_problem& p, bool on_device) {
  if (!p.row_ptr) throw halp::Error(LP_ERR_INVALID, "null row_ptr");
  if (p.m_eq < 0 || p.m_ineq < 0 || p.n < 1)
    throw halp::Error(LP_ERR_INVALID, "sizes must satisfy n >= 1, m_eq >= 0, m_ineq >= 0");
  const int64_t m = p.m_eq + p.m_ineq;
  if (m > INT32_MAX - 2 || p.n > INT32_MAX - 2) throw halp::Error(LP_ERR_INVALID, "dimension too large");
  int32_t e = 0;
  if (on_device) {
    if (hipMemcpy(&e, p.row_ptr + m, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
      throw halp::Error(LP_ERR_DEVICE, "cannot read row_ptr[m] from device");
  } else {
    e = p.row_ptr[m];
  }
  if (e < 0) throw halp::Error(LP_ERR_INVALID, "row_ptr[m] must be >= 0");
  return e;
}

struct StreamHolder {
  hipStream_t s = nullptr;
  bool own = false;
  void init(void* user) {
    if (user) {
      s = (hipStream_t)user;
    } else {
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        throw halp::Error(LP_ERR_DEVICE, "hipStreamCreate failed");
      own = true;
    }
  }
  ~StreamHolder() {
    if (own && s) (void)hipStreamDestroy(s);
  }
};

void hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) throw halp::Error(LP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Copy of an LP's inputs kept by FP32 handles for the FP64 polish phase
// (host vectors for host inputs, device buffers for device inputs).
struct RawLP {
  bool on_device = false;
  int64_t n = 0, m_eq = 0, m_ineq = 0, nnz = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> val, c, rhs, lb, ub;
  void* dmem = nullptr;
  lp_problem view{};
  void capture(const lp_problem& p, int64_t nz, bool dev, hipStream_t s) {
    on_device = dev;
    n = p.n;
    m_eq = p.m_eq;
    m_ineq = p.m_ineq;
    nnz = nz;
    const int64_t m = m_eq + m_ineq;
    if (!dev) {
      rp.assign(p.row_ptr, p.row_ptr + m + 1);
      if (nz) {
        ci.assign(p.col_idx, p.col_idx + nz);
        val.assign(p.val, p.val + nz);
      }
      c.assign(p.c, p.c + n);
      lb.assign(p.lb, p.lb + n);
      ub.assign(p.ub, p.ub + n);
      if (m) rhs.assign(p.rhs, p.rhs + m);
      view = lp_problem{n, m_eq, m_ineq, rp.data(), ci.data(), val.data(), c.data(), rhs.data(),
                        lb.data(), ub.data()};
      return;
    }
    const size_t bytes = 4 * (m + 1) + 12 * nz + 8 * (3 * n + m) + 64;
    if (hipMalloc(&dmem, bytes) != hipSuccess) throw halp::Error(LP_ERR_OOM, "device allocation failed");
    char* q = (char*)dmem;
    auto take = [&](size_t b) {
      char* r = q;
      q += (b + 7) & ~size_t(7);
      return (void*)r;
    };
    int32_t* drp = (int32_t*)take(4 * (m + 1));
    int32_t* dci = (int32_t*)take(4 * nz);
    double* dval = (double*)take(8 * nz);
    double* dc = (double*)take(8 * n);
    double* drhs = (double*)take(8 * m);
    double* dlb = (double*)take(8 * n);
    double* dub = (double*)take(8 * n);
    auto cp = [&](void* d, const void* src, size_t b) {
      if (b && hipMemcpyAsync(d, src, b, hipMemcpyDeviceToDevice, s) != hipSuccess)
        throw halp::Error(LP_ERR_DEVICE, "device copy failed");
    };
    cp(drp, p.row_ptr, 4 * (m + 1));
    cp(dci, p.col_idx, 4 * nz);
    cp(dval, p.val, 8 * nz);
    cp(dc, p.c, 8 * n);
    cp(drhs, p.rhs, 8 * m);
    cp(dlb, p.lb, 8 * n);
    cp(dub, p.ub, 8 * n);
    view = lp_problem{n, m_eq, m_ineq, drp, dci, dval, dc, drhs, dlb, dub};
  }
  ~RawLP() {
    if (dmem) (void)hipFree(dmem);
  }
};

namespace {

// FP64 continuation of LPs that an FP32 engine solved to the polish
// tolerance (or left at its precision floor: stall rule, iteration limit).
// Each continues from its FP32 candidate T(z) in the same scaled space (both
// engines compute the scaling and the step size in FP64 from the same inputs)
// with the FP32 primal weight, as a fresh epoch, for the iterations left.
struct Polish {
  std::unique_ptr<halp::EngineBase> eng;
  std::vector<int> id;                // per LP of the FP32 engine: FP64 id, or -1
  std::vector<halp::Result> first;    // the FP32 phase's result of each polished LP
};

// Iterations the FP32 phase of a polished solve may take: a tenth of the
// request's budget (at least 1), so that an LP whose FP32 trajectory
// converges slowly without stalling still leaves the FP64 phase most of it.
int64_t fp32_budget(int64_t max_iter) { return std::max<int64_t>(1, max_iter / 10); }

// Primal weight the FP64 phase starts with (import_point: <= 0 means the
// LP's initial weight ||c~|| / ||q~||).  1 (default): the FP32 phase's last
// weight, which keeps the balance of primal and dual progress the FP32
// trajectory found, so the continuation ends near where an FP64 solve would.
// 0: the initial weight, far larger than the settled one on many LPs: the
// continuation then mostly corrects the dual side, reaches the tolerance in
// fewer iterations and keeps much of the FP32 candidate's objective error
// (the relative KKT error does not bound it).  2: the initial weight when
// the FP32 phase reached polish_tol, else the last one.
double polish_omega(const halp::Options& o, const halp::Result& first, double omega) {
  if (o.polish_weight == 0) return 0.0;
  if (o.polish_weight == 1) return omega;
  return first.status == LP_OPTIMAL ? 0.0 : omega;
}

bool polish_wanted(const halp::Result& r, int64_t max_iter) {
  const bool go = r.status == LP_OPTIMAL || r.status == LP_ITER_LIMIT || r.status == LP_NUMERICAL;
  return go && r.iters < max_iter;
}

void run_polish(Polish& P, const halp::Options& opt, hipStream_t stream, halp::EngineBase& src,
                const std::vector<int>& src_ids, const std::vector<const RawLP*>& raw, double tol,
                int64_t max_iter, double left_s) {
  const int count = (int)src_ids.size();
  P.id.assign(count, -1);
  P.first.assign(count, halp::Result());
  std::vector<int> which;
  int64_t ms = 0, ns = 0, zs = 0, buf_len = 1;
  for (int i = 0; i < count; ++i) {
    const halp::Result r = src.result(src_ids[i]);
    if (!polish_wanted(r, max_iter)) continue;
    which.push_back(i);
    P.first[i] = r;
    const lp_problem& p = raw[i]->view;
    ms += p.m_eq + p.m_ineq + 1;
    ns += p.n + 1;
    zs += raw[i]->nnz;
    buf_len = std::max<int64_t>(buf_len, p.n + p.m_eq + p.m_ineq + 1);
  }
  if (which.empty() || (left_s >= 0.0 && left_s <= 0.0)) return;
  halp::Options o64 = opt;
  o64.precision = 0;
  P.eng = halp::make_engine(o64, stream, ms, ns, zs, (int)which.size());
  std::vector<halp::Problem> probs;
  for (int i : which) probs.push_back(to_problem(raw[i]->view));
  const std::vector<int> ids = P.eng->add(probs, raw[which[0]]->on_device);
  double* buf = nullptr;
  if (hipMalloc((void**)&buf, sizeof(double) * buf_len) != hipSuccess)
    throw halp::Error(LP_ERR_OOM, "device allocation failed");
  try {
    for (size_t k = 0; k < which.size(); ++k) {
      const int i = which[k];
      const lp_problem& p = raw[i]->view;
      double omega = 1.0;
      src.export_point(src_ids[i], buf, buf + p.n, &omega);
      P.eng->import_point(ids[k], buf, buf + p.n, polish_omega(opt, P.first[i], omega));
      P.id[i] = ids[k];
      P.eng->set_params({ids[k]}, tol, max_iter - P.first[i].iters);
    }
  } catch (...) {
    (void)hipFree(buf);
    throw;
  }
  (void)hipFree(buf);
  P.eng->run(left_s);
}

// Engine and id holding LP i's final iterate: the FP64 continuation when it
// was polished, else the FP32 engine.
halp::EngineBase& final_engine(const Polish& P, int i, halp::EngineBase& src, int src_id, int* id) {
  if (P.eng && i < (int)P.id.size() && P.id[i] >= 0) {
    *id = P.id[i];
    return *P.eng;
  }
  *id = src_id;
  return src;
}

// Result of LP i: the FP64 continuation's (iterations and restarts of both
// phases added) when it was polished, else the FP32 phase's.
lp_result polish_result(const Polish& P, int i, halp::EngineBase& src, int src_id, double seconds) {
  if (P.eng && i < (int)P.id.size() && P.id[i] >= 0) {
    lp_result o = to_result(P.eng->result(P.id[i]), seconds);
    o.polish_iters = o.iters;
    o.ident_iters = o.ident_iters > 0 ? o.ident_iters + P.first[i].iters : P.first[i].ident_iters;
    o.iters += P.first[i].iters;
    o.restarts += P.first[i].restarts;
    o.checks += P.first[i].checks;
    return o;
  }
  return to_result(src.result(src_id), seconds);
}

}  // namespace

struct lp_solver {
  StreamHolder stream;
  halp::Options opt;
  std::unique_ptr<halp::EngineBase> eng;
  int id = -1;
  bool solved = false;
  double seconds = 0.0;
  // FP32 mode: inputs kept for the FP64 polish, and the polish stage
  std::unique_ptr<RawLP> raw;
  Polish polish;
};

struct lp_batch {
  StreamHolder stream;
  halp::Options opt;
  std::unique_ptr<halp::EngineBase> eng;
  std::vector<int> ids;
  double seconds = 0.0;
  std::vector<std::unique_ptr<RawLP>> raw;  // FP32 mode: inputs kept for the FP64 polish
  Polish polish;
};

extern "C" {

void lp_default_options(lp_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  halp::Options d;
  o->method = d.method;
  o->precision = d.precision;
  o->ruiz_iters = d.ruiz_iters;
  o->pc_alpha = d.pc_alpha;
  o->check_every = d.check_every;
  o->restart_beta = d.restart_beta;
  o->artificial_restart = d.artificial_restart;
  o->step_safety = d.step_safety;
  o->power_max_iters = d.power_max_iters;
  o->power_min_iters = d.power_min_iters;
  o->power_rtol = d.power_rtol;
  o->eps_infeas = d.eps_infeas;
  o->primal_weight = d.primal_weight;
  o->seed = d.seed;
  o->eta = d.eta;
  o->omega0 = d.omega0;
  o->chunk = d.chunk;
  o->use_graph = d.use_graph;
  o->profile = d.profile;
  o->slice_min_bytes = d.slice_min_bytes;
  o->polish_tol = d.polish_tol;
  o->verbose = d.verbose;
  o->cache_budget_bytes = d.cache_budget_bytes;
  o->stall_checks = d.stall_checks;
  o->restart_mode = d.restart_mode;
  o->fixed_restart_len = d.fixed_restart_len;
  o->xcd_pin = d.xcd_pin;
  o->tile_rows = d.tile_rows;
  o->slice_entries = d.slice_entries;
  o->slice_rows = d.slice_rows;
  o->slice_sort = d.slice_sort;
  o->sort_rows = d.sort_rows;
  o->plain_sort = d.plain_sort;
  o->group_threads = d.group_threads;
  o->group_batched = d.group_batched;
  o->group_blocks = d.group_blocks;
  o->polish_weight = d.polish_weight;
}

const char* lp_last_error(void) { return g_err.c_str(); }

int lp_create(lp_solver** out, int64_t n, int64_t m_eq, int64_t m_ineq, const int32_t* row_ptr,
              const int32_t* col_idx, const double* val, const double* c, const double* rhs, const double* lb,
              const double* ub, int inputs_on_device, void* stream, const lp_options* opt) {
  return guarded([&]() -> int {
    if (!out) return fail(LP_ERR_INVALID, "null output handle");
    *out = nullptr;
    lp_problem p{n, m_eq, m_ineq, row_ptr, col_idx, val, c, rhs, lb, ub};
    const halp::Options o = to_opts(opt);
    check_opts(o);
    const int64_t nnz = read_nnz(p, inputs_on_device != 0);
    if (!inputs_on_device) halp::validate_host_problem(to_problem(p));
    std::unique_ptr<lp_solver> s(new lp_solver());
    s->stream.init(stream);
    s->opt = o;
    s->eng = halp::make_engine(o, s->stream.s, m_eq + m_ineq + 1, n + 1, nnz, 1);
    s->id = s->eng->add({to_problem(p)}, inputs_on_device != 0)[0];
    if (o.precision == 1 && o.polish_tol > 0.0) {
      s->raw.reset(new RawLP());
      s->raw->capture(p, nnz, inputs_on_device != 0, s->stream.s);
    }
    *out = s.release();
    return LP_OK;
  });
}

int lp_create64(lp_solver** out, int64_t n, int64_t m_eq, int64_t m_ineq, const int64_t* row_ptr,
                const int32_t* col_idx, const double* val, const double* c, const double* rhs, const double* lb,
                const double* ub, int inputs_on_device, void* stream, const lp_options* opt) {
  return guarded([&]() -> int {
    if (!out) return fail(LP_ERR_INVALID, "null output handle");
    *out = nullptr;
    if (!row_ptr) return fail(LP_ERR_INVALID, "null row_ptr");
    if (m_eq < 0 || m_ineq < 0) return fail(LP_ERR_INVALID, "sizes must satisfy n >= 1, m >= 0");
    const int64_t m = m_eq + m_ineq;
    if (!inputs_on_device) {
      std::vector<int32_t> rp(m + 1);
      for (int64_t i = 0; i <= m; ++i) {
        if (row_ptr[i] < 0 || row_ptr[i] > (int64_t)INT32_MAX)
          return fail(LP_ERR_INVALID, "row_ptr entry outside [0, 2^31 - 1] (at most 2^31 - 1 stored entries)");
        rp[i] = (int32_t)row_ptr[i];
      }
      return lp_create(out, n, m_eq, m_ineq, rp.data(), col_idx, val, c, rhs, lb, ub, 0, stream, opt);
    }
    int32_t* rp = nullptr;
    if (hipMalloc((void**)&rp, sizeof(int32_t) * (m + 1)) != hipSuccess)
      return fail(LP_ERR_OOM, "device allocation failed");
    int rc = LP_OK;
    try {
      if (halp::narrow_row_ptr(row_ptr, rp, m + 1, (hipStream_t)stream))
        rc = fail(LP_ERR_INVALID, "row_ptr entry outside [0, 2^31 - 1] (at most 2^31 - 1 stored entries)");
      else
        rc = lp_create(out, n, m_eq, m_ineq, rp, col_idx, val, c, rhs, lb, ub, 1, stream, opt);
      // lp_create copies its inputs on the handle's stream: wait for it
      if (rc == LP_OK) hip_ok(hipStreamSynchronize((*out)->stream.s), "stream synchronize");
    } catch (...) {
      (void)hipFree(rp);
      throw;
    }
    (void)hipFree(rp);
    return rc;
  });
}

int lp_solve(lp_solver* s, double tol, int64_t max_iter, double time_limit_s) {
  return guarded([&]() -> int {
    if (!s) return fail(LP_ERR_INVALID, "null handle");
    if (s->solved) return fail(LP_ERR_STATE, "this handle has already solved its LP");
    if (!(tol >= 0.0) || max_iter < 1) return fail(LP_ERR_INVALID, "need tol >= 0 and max_iter >= 1");
    const double t0 = now_s();
    const bool polish = s->raw && tol < s->opt.polish_tol;
    s->eng->set_params({s->id}, polish ? s->opt.polish_tol : tol, polish ? fp32_budget(max_iter) : max_iter,
                       polish ? s->opt.stall_checks : 0);
    s->eng->run(time_limit_s);
    if (polish) {
      const double left = time_limit_s < 0 ? -1.0 : time_limit_s - (now_s() - t0);
      run_polish(s->polish, s->opt, s->stream.s, *s->eng, {s->id}, {s->raw.get()}, tol, max_iter, left);
    }
    s->seconds = now_s() - t0;
    s->solved = true;
    return LP_OK;
  });
}

int lp_status(const lp_solver* s, lp_result* out) {
  return guarded([&]() -> int {
    if (!s || !out) return fail(LP_ERR_INVALID, "null argument");
    *out = polish_result(s->polish, 0, *s->eng, s->id, s->seconds);
    return LP_OK;
  });
}

int lp_get_solution(const lp_solver* s, double* x, double* y, int to_device) {
  return guarded([&]() -> int {
    if (!s) return fail(LP_ERR_INVALID, "null handle");
    if (!s->solved) return fail(LP_ERR_STATE, "solve first");
    int id = -1;
    final_engine(s->polish, 0, *s->eng, s->id, &id).solution(id, x, y, to_device != 0);
    return LP_OK;
  });
}

int lp_get_certificate(const lp_solver* s, double* ray, int to_device) {
  return guarded([&]() -> int {
    if (!s || !ray) return fail(LP_ERR_INVALID, "null argument");
    if (!s->solved) return fail(LP_ERR_STATE, "solve first");
    int id = -1;
    final_engine(s->polish, 0, *s->eng, s->id, &id).certificate(id, ray, to_device != 0);
    return LP_OK;
  });
}

int lp_kernel_times(const lp_solver* s, lp_kernel_timing* out) {
  return guarded([&]() -> int {
    if (!s || !out) return fail(LP_ERR_INVALID, "null argument");
    const halp::KernelTimes t = s->eng->kernel_times();
    out->primal_slice_ms = t.primal_slice_ms;
    out->primal_ms = t.primal_ms;
    out->dual_slice_ms = t.dual_slice_ms;
    out->dual_ms = t.dual_ms;
    out->event_pair_ms = t.event_pair_ms;
    out->nnz = t.nnz;
    out->n = t.n;
    out->m = t.m;
    out->steps = t.launches;
    return LP_OK;
  });
}

int lp_get_scaled_matrix(const lp_solver* s, int transpose, int32_t* row_ptr, int32_t* col_idx, double* val) {
  return guarded([&]() -> int {
    if (!s || !row_ptr || !col_idx || !val || (transpose != 0 && transpose != 1))
      return fail(LP_ERR_INVALID, "bad argument");
    s->eng->stored_matrix(s->id, transpose != 0, row_ptr, col_idx, val);
    return LP_OK;
  });
}

void lp_destroy(lp_solver* s) {
  try {
    delete s;
  } catch (...) {
  }
}

// ------------------------------------------------------------------ no allocation

int lp_solve_static(int64_t n, int64_t m_eq, int64_t m_ineq, const int32_t* row_ptr, const int32_t* col_idx,
                    const double* val, const double* c, const double* rhs, const double* lb, const double* ub,
                    void* stream, const lp_options* opt, double tol, int64_t max_iter, double time_limit_s,
                    double* x, double* y, lp_result* out) {
  static std::mutex mu;  // one workspace per GPU: calls of this process take turns
  return guarded([&]() -> int {
    if (!out) return fail(LP_ERR_INVALID, "null result");
    if (!(tol >= 0.0) || max_iter < 1) return fail(LP_ERR_INVALID, "need tol >= 0 and max_iter >= 1");
    halp::Options o = to_opts(opt);
    check_opts(o);
    if (o.precision != 0) return fail(LP_ERR_INVALID, "lp_solve_static solves in FP64 only");
    o.use_graph = 0;
    o.profile = 0;
    lp_problem p{n, m_eq, m_ineq, row_ptr, col_idx, val, c, rhs, lb, ub};
    const int64_t nnz = read_nnz(p, true);
    const int64_t m = m_eq + m_ineq;
    // K and K^T (indices and FP64 values) alone need 24 bytes per entry
    const int64_t floor_bytes = 24 * nnz + 8 * (m + n);
    if (floor_bytes > halp::kWorkspaceBytes)
      return fail(LP_ERR_OOM, "LP too large for the static workspace: at least " + std::to_string(floor_bytes) +
                                  " bytes needed of " + std::to_string((long long)halp::kWorkspaceBytes));
    std::lock_guard<std::mutex> lk(mu);
    hipStream_t st = (hipStream_t)stream;
    const double t0 = now_s();
    halp::WorkspaceScope ws(st);
    {
      std::unique_ptr<halp::EngineBase> eng = halp::make_engine(o, st, m + 1, n + 1, nnz, 1);
      const int id = eng->add({to_problem(p)}, true)[0];
      eng->set_params({id}, tol, max_iter, 0);
      eng->run(time_limit_s);
      const halp::Result r = eng->result(id);
      if (x || y) eng->solution(id, x, y, true);
      *out = to_result(r, now_s() - t0);
    }
    hip_ok(hipStreamSynchronize(st), "hipStreamSynchronize");
    return LP_OK;
  });
}

// ------------------------------------------------------------------ batch

int lp_batch_create(lp_batch** out, int count, const lp_problem* problems, int inputs_on_device, void* stream,
                    const lp_options* opt) {
  return guarded([&]() -> int {
    if (!out || (count > 0 && !problems) || count < 1) return fail(LP_ERR_INVALID, "need count >= 1 problems");
    *out = nullptr;
    const halp::Options o = to_opts(opt);
    check_opts(o);
    int64_t ms = 0, ns = 0, zs = 0;
    std::vector<halp::Problem> ps;
    for (int i = 0; i < count; ++i) {
      const int64_t nnz = read_nnz(problems[i], inputs_on_device != 0);
      if (!inputs_on_device) halp::validate_host_problem(to_problem(problems[i]));
      ms += problems[i].m_eq + problems[i].m_ineq + 1;
      ns += problems[i].n + 1;
      zs += nnz;
      ps.push_back(to_problem(problems[i]));
    }
    if (zs > INT32_MAX) return fail(LP_ERR_INVALID, "batch holds more than 2^31 - 1 entries");
    std::unique_ptr<lp_batch> b(new lp_batch());
    b->stream.init(stream);
    b->opt = o;
    b->eng = halp::make_engine(o, b->stream.s, ms, ns, zs, count);
    b->ids = b->eng->add(ps, inputs_on_device != 0);
    if (o.precision == 1 && o.polish_tol > 0.0) {
      for (int i = 0; i < count; ++i) {
        b->raw.emplace_back(new RawLP());
        b->raw.back()->capture(problems[i], read_nnz(problems[i], inputs_on_device != 0), inputs_on_device != 0,
                               b->stream.s);
      }
    }
    *out = b.release();
    return LP_OK;
  });
}

int lp_batch_solve(lp_batch* b, double tol, int64_t max_iter, double time_limit_s) {
  return guarded([&]() -> int {
    if (!b) return fail(LP_ERR_INVALID, "null handle");
    if (!(tol >= 0.0) || max_iter < 1) return fail(LP_ERR_INVALID, "need tol >= 0 and max_iter >= 1");
    const double t0 = now_s();
    const bool polish = !b->raw.empty() && tol < b->opt.polish_tol;
    b->eng->set_params(b->ids, polish ? b->opt.polish_tol : tol, polish ? fp32_budget(max_iter) : max_iter,
                       polish ? b->opt.stall_checks : 0);
    b->eng->run(time_limit_s);
    if (polish) {
      std::vector<const RawLP*> raw;
      for (auto& r : b->raw) raw.push_back(r.get());
      const double left = time_limit_s < 0 ? -1.0 : time_limit_s - (now_s() - t0);
      run_polish(b->polish, b->opt, b->stream.s, *b->eng, b->ids, raw, tol, max_iter, left);
    }
    b->seconds = now_s() - t0;
    return LP_OK;
  });
}

int lp_batch_status(const lp_batch* b, int index, lp_result* out) {
  return guarded([&]() -> int {
    if (!b || !out || index < 0 || index >= (int)b->ids.size()) return fail(LP_ERR_INVALID, "bad argument");
    *out = polish_result(b->polish, index, *b->eng, b->ids[index], b->seconds);
    return LP_OK;
  });
}

int lp_batch_get_solution(const lp_batch* b, int index, double* x, double* y, int to_device) {
  return guarded([&]() -> int {
    if (!b || index < 0 || index >= (int)b->ids.size()) return fail(LP_ERR_INVALID, "bad argument");
    int id = -1;
    final_engine(b->polish, index, *b->eng, b->ids[index], &id).solution(id, x, y, to_device != 0);
    return LP_OK;
  });
}

int lp_batch_get_certificate(const lp_batch* b, int index, double* ray, int to_device) {
  return guarded([&]() -> int {
    if (!b || !ray || index < 0 || index >= (int)b->ids.size()) return fail(LP_ERR_INVALID, "bad argument");
    int id = -1;
    final_engine(b->polish, index, *b->eng, b->ids[index], &id).certificate(id, ray, to_device != 0);
    return LP_OK;
  });
}

int lp_batch_kernel_times(const lp_batch* b, lp_kernel_timing* out) {
  return guarded([&]() -> int {
    if (!b || !out) return fail(LP_ERR_INVALID, "null argument");
    const halp::KernelTimes t = b->eng->kernel_times();
    out->primal_slice_ms = t.primal_slice_ms;
    out->primal_ms = t.primal_ms;
    out->dual_slice_ms = t.dual_slice_ms;
    out->dual_ms = t.dual_ms;
    out->event_pair_ms = t.event_pair_ms;
    out->nnz = t.nnz;
    out->n = t.n;
    out->m = t.m;
    out->steps = t.launches;
    return LP_OK;
  });
}

void lp_batch_destroy(lp_batch* b) {
  try {
    delete b;
  } catch (...) {
  }
}

}  // extern "C"

// ------------------------------------------------------------------ serving

namespace {

struct Request {
  int64_t ticket = 0;
  int64_t n = 0, m_eq = 0, m_ineq = 0, nnz = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> val, c, rhs, lb, ub;
  double tol = 1e-4;
  int64_t max_iter = 1;
  double t_arrival = 0.0;
  int slot = -1;
  bool done = false;
  lp_result res{};
  double t_done = 0.0;
  std::vector<double> x, y;
  std::vector<double> ray;  // certificate of an infeasible request (m or n entries)
  // FP32 server with polish: the FP32 phase's candidate (scaled) and result,
  // and the slot of the FP64 phase
  std::vector<double> px, py;
  double pomega = 1.0;
  halp::Result first;
  int slot64 = -1;
};

halp::Problem request_problem(const Request& r) {
  halp::Problem q;
  q.n = r.n;
  q.m_eq = r.m_eq;
  q.m_ineq = r.m_ineq;
  q.rp = r.rp.data();
  q.ci = r.ci.data();
  q.val = r.val.data();
  q.c = r.c.data();
  q.rhs = r.rhs.data();
  q.lb = r.lb.data();
  q.ub = r.ub.data();
  return q;
}

// engine capacities for a memory budget: the budget is split over the three
// spaces for a reference mix of n = 4 m and nnz = 36 m (the batched sizes)
// Capacities of one server engine from its share of the budget: three
// quarters for the persistent storage of live LPs (per row, per variable and
// per stored entry as the engine allocates them; `staging`: plus the FP64
// phase's staging of one candidate, 8 bytes per row and variable), one
// quarter for the transient buffers of an admission (transpose and layout
// sorts, about kAdmitBytesPerEntry per stored entry of the LPs admitted in
// one step).  Servers never column-slice a product, so no slice partial
// sums are allocated.
constexpr int64_t kAdmitBytesPerEntry = 48;

bool server_caps(int64_t share, int precision, bool staging, int64_t* cap_m, int64_t* cap_n, int64_t* cap_nz,
                 int64_t* admit_nz) {
  const int64_t sz = precision == 1 ? 4 : 8;
  // as the engine allocates them without slice row pointers (see footprint())
  const int64_t per_row = 4 + 24 + 12 * sz + 1 + (staging ? 8 : 0);
  const int64_t per_col = 4 + 40 + 13 * sz + 1 + (staging ? 8 : 0);
  const int64_t per_nz = 24 + (precision == 1 ? 8 : 0);
  const int64_t unit = per_row + 4 * per_col + 36 * per_nz;
  const int64_t u = (share / 4 * 3) / unit;
  if (u < 16) return false;
  *cap_m = u;
  *cap_n = 4 * u;
  *cap_nz = std::min<int64_t>(36 * u, INT32_MAX - 1);
  *admit_nz = std::max<int64_t>(1, (share / 4) / kAdmitBytesPerEntry);
  return true;
}

}  // namespace

struct lp_server {
  StreamHolder stream;
  halp::Options opt;
  std::unique_ptr<halp::EngineBase> eng;
  int64_t budget = 0;
  int max_slots = 0;
  int64_t next_ticket = 1;
  std::deque<int64_t> queue;
  std::map<int64_t, Request> reqs;
  std::map<int, int64_t> slot_ticket;
  // FP32 servers: the FP64 polish phase (its own engine, queue and slots)
  std::unique_ptr<halp::EngineBase> eng64;
  std::deque<int64_t> queue64;
  std::map<int, int64_t> slot_ticket64;
  double* dbuf = nullptr;  // device staging of candidates between the phases
  int64_t dbuf_len = 0;
  int64_t admit_nz = 0, admit_nz64 = 0;  // stored entries one admission may add to each engine
  // live LPs of each engine when its layouts were last sized: once half of
  // them have retired the rest are re-blocked for fewer LPs per launch
  int refine_live = 0, refine_live64 = 0;
  double t0 = 0.0;
  double clock() const { return now_s() - t0; }
  ~lp_server() {
    if (dbuf) (void)hipFree(dbuf);
  }
  // the staging buffer is allocated with the server, sized for the largest
  // LP the FP64 engine can hold
  double* staging(int64_t len) {
    if (len > dbuf_len) throw halp::Error(LP_ERR_STATE, "staging buffer too small");
    return dbuf;
  }
};

extern "C" {

int lp_server_create(lp_server** out, int64_t budget, int max_slots, void* stream, const lp_options* opt) {
  return guarded([&]() -> int {
    if (!out || budget <= 0 || max_slots < 1) return fail(LP_ERR_INVALID, "need budget > 0 and max_slots >= 1");
    *out = nullptr;
    const halp::Options o = to_opts(opt);
    check_opts(o);
    std::unique_ptr<lp_server> s(new lp_server());
    s->stream.init(stream);
    s->opt = o;
    // FP32 servers split the budget between the FP32 engine and the FP64
    // polish engine; served LPs are never column-sliced (no partial-sum
    // buffers that an admission would have to allocate)
    s->opt.slice_min_bytes = -1;
    const bool two = o.precision == 1 && o.polish_tol > 0.0;
    const int64_t share = two ? budget / 2 : budget;
    int64_t cm = 0, cn = 0, cz = 0;
    if (!server_caps(share, o.precision, false, &cm, &cn, &cz, &s->admit_nz))
      return fail(LP_ERR_INVALID, "budget too small");
    s->budget = budget;
    s->max_slots = max_slots;
    s->eng = halp::make_engine(s->opt, s->stream.s, cm + max_slots, cn + max_slots, cz, max_slots);
    if (two) {
      halp::Options o64 = s->opt;
      o64.precision = 0;
      if (!server_caps(share, 0, true, &cm, &cn, &cz, &s->admit_nz64))
        return fail(LP_ERR_INVALID, "budget too small");
      s->eng64 = halp::make_engine(o64, s->stream.s, cm + max_slots, cn + max_slots, cz, max_slots);
      s->dbuf_len = cm + cn + 2 * max_slots;
      if (hipMalloc((void**)&s->dbuf, sizeof(double) * s->dbuf_len) != hipSuccess)
        return fail(LP_ERR_OOM, "device allocation failed");
    }
    s->t0 = now_s();
    *out = s.release();
    return LP_OK;
  });
}

int lp_server_submit(lp_server* s, const lp_problem* p, double tol, int64_t max_iter, double t_arrival,
                     int64_t* ticket) {
  return guarded([&]() -> int {
    if (!s || !p || !ticket) return fail(LP_ERR_INVALID, "null argument");
    if (!(tol >= 0.0) || max_iter < 1) return fail(LP_ERR_INVALID, "need tol >= 0 and max_iter >= 1");
    const int64_t nnz = read_nnz(*p, false);
    const int64_t m = p->m_eq + p->m_ineq;
    Request r;
    r.ticket = s->next_ticket++;
    r.n = p->n;
    r.m_eq = p->m_eq;
    r.m_ineq = p->m_ineq;
    r.nnz = nnz;
    r.rp.assign(p->row_ptr, p->row_ptr + m + 1);
    if (nnz) {
      if (!p->col_idx || !p->val) return fail(LP_ERR_INVALID, "null column or value array");
      r.ci.assign(p->col_idx, p->col_idx + nnz);
      r.val.assign(p->val, p->val + nnz);
    }
    if (!p->c || !p->lb || !p->ub || (m && !p->rhs)) return fail(LP_ERR_INVALID, "null vector");
    r.c.assign(p->c, p->c + p->n);
    r.lb.assign(p->lb, p->lb + p->n);
    r.ub.assign(p->ub, p->ub + p->n);
    if (m) r.rhs.assign(p->rhs, p->rhs + m);
    halp::validate_host_problem(to_problem(*p));
    r.tol = tol;
    r.max_iter = max_iter;
    r.t_arrival = t_arrival;
    // refused at once if it would not fit even an idle server (it would
    // otherwise block the head of the queue for good)
    if (!s->eng->fits_empty(r.n, m, nnz) || nnz > s->admit_nz)
      return fail(LP_ERR_INVALID, "LP is larger than the server's reserved memory");
    if (s->eng64 && tol < s->opt.polish_tol && (!s->eng64->fits_empty(r.n, m, nnz) || nnz > s->admit_nz64))
      return fail(LP_ERR_INVALID, "LP is larger than the server's reserved memory (FP64 phase)");
    *ticket = r.ticket;
    s->queue.push_back(r.ticket);
    s->reqs.emplace(r.ticket, std::move(r));
    return LP_OK;
  });
}

}  // extern "C"

namespace {

void finish_request(lp_server* s, Request& r, halp::EngineBase& eng, int slot, const lp_result& res, double tnow) {
  r.res = res;
  r.x.resize(r.n);
  r.y.resize(r.m_eq + r.m_ineq);
  eng.solution(slot, r.x.data(), r.y.empty() ? nullptr : r.y.data(), false);
  if (res.status == LP_PRIMAL_INFEASIBLE || res.status == LP_DUAL_INFEASIBLE) {
    r.ray.resize(res.status == LP_PRIMAL_INFEASIBLE ? r.m_eq + r.m_ineq : r.n);
    if (!r.ray.empty()) eng.certificate(slot, r.ray.data(), false);
  }
  r.t_done = tnow;
  r.done = true;
  r.slot = r.slot64 = -1;
  eng.remove({slot});
  // drop the input copy and the staged candidate
  std::vector<int32_t>().swap(r.rp);
  std::vector<int32_t>().swap(r.ci);
  std::vector<double>().swap(r.val);
  std::vector<double>().swap(r.px);
  std::vector<double>().swap(r.py);
}

// admits the longest prefix of `queue` that fits `eng` (preprocessed
// together), at most admit_nz stored entries at a time (the transient
// buffers of an admission are sized by them)
std::vector<std::pair<int64_t, int>> admit(lp_server* s, halp::EngineBase& eng, std::deque<int64_t>& queue,
                                           int64_t admit_nz) {
  std::vector<std::pair<int64_t, int>> out;
  if (queue.empty() || eng.live() >= s->max_slots) return out;
  std::vector<halp::Problem> ps;
  int64_t nz = 0;
  for (int64_t t : queue) {
    if ((int)ps.size() >= s->max_slots - eng.live()) break;
    const Request& r = s->reqs.at(t);
    if (!ps.empty() && nz + r.nnz > admit_nz) break;
    nz += r.nnz;
    ps.push_back(request_problem(r));
  }
  std::vector<int> ids = eng.add(ps, false, true);
  for (size_t k = 0; k < ids.size(); ++k) {
    out.push_back({queue.front(), ids[k]});
    queue.pop_front();
  }
  return out;
}

}  // namespace

extern "C" {

int lp_server_step(lp_server* s, int chunks, int* n_done) {
  return guarded([&]() -> int {
    if (!s || chunks < 0) return fail(LP_ERR_INVALID, "bad argument");
    // admission to the first (or only) phase
    {
      std::map<std::tuple<double, int64_t, int64_t>, std::vector<int>> by_params;
      for (auto& [t, id] : admit(s, *s->eng, s->queue, s->admit_nz)) {
        Request& r = s->reqs.at(t);
        const bool polish = s->eng64 && r.tol < s->opt.polish_tol;
        by_params[{polish ? s->opt.polish_tol : r.tol, polish ? fp32_budget(r.max_iter) : r.max_iter,
                   polish ? s->opt.stall_checks : 0}].push_back(id);
        r.slot = id;
        s->slot_ticket[id] = t;
      }
      for (auto& kv : by_params)
        s->eng->set_params(kv.second, std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first));
    }
    // admission to the FP64 polish phase, from the FP32 candidates
    if (s->eng64) {
      for (auto& [t, id] : admit(s, *s->eng64, s->queue64, s->admit_nz64)) {
        Request& r = s->reqs.at(t);
        double* buf = s->staging(r.n + r.m_eq + r.m_ineq + 1);
        hip_ok(hipMemcpy(buf, r.px.data(), sizeof(double) * r.n, hipMemcpyHostToDevice), "staging copy");
        if (!r.py.empty())
          hip_ok(hipMemcpy(buf + r.n, r.py.data(), sizeof(double) * r.py.size(), hipMemcpyHostToDevice),
                 "staging copy");
        s->eng64->import_point(id, buf, buf + r.n, polish_omega(s->opt, r.first, r.pomega));
        s->eng64->set_params({id}, r.tol, r.max_iter - r.first.iters);
        r.slot64 = id;
        s->slot_ticket64[id] = t;
      }
    }
    s->refine_live = std::max(s->refine_live, s->eng->live());
    if (s->eng64) s->refine_live64 = std::max(s->refine_live64, s->eng64->live());
    int nd = 0;
    if (s->eng->live() > 0 && chunks > 0) {
      std::vector<int> done = s->eng->advance(chunks);
      const double tnow = s->clock();
      for (int slot : done) {
        const int64_t t = s->slot_ticket.at(slot);
        Request& r = s->reqs.at(t);
        s->slot_ticket.erase(slot);
        const halp::Result res = s->eng->result(slot);
        if (s->eng64 && r.tol < s->opt.polish_tol && polish_wanted(res, r.max_iter)) {
          // stage the FP32 candidate on the host and queue the FP64 phase
          double* buf = s->staging(r.n + r.m_eq + r.m_ineq + 1);
          s->eng->export_point(slot, buf, buf + r.n, &r.pomega);
          r.px.resize(r.n);
          r.py.resize(r.m_eq + r.m_ineq);
          hip_ok(hipMemcpy(r.px.data(), buf, sizeof(double) * r.n, hipMemcpyDeviceToHost), "staging copy");
          if (!r.py.empty())
            hip_ok(hipMemcpy(r.py.data(), buf + r.n, sizeof(double) * r.py.size(), hipMemcpyDeviceToHost),
                   "staging copy");
          r.first = res;
          r.slot = -1;
          s->eng->remove({slot});
          s->queue64.push_back(t);
          continue;
        }
        finish_request(s, r, *s->eng, slot, to_result(res, 0.0), tnow);
        ++nd;
      }
    }
    if (s->eng64 && s->eng64->live() > 0 && chunks > 0) {
      std::vector<int> done = s->eng64->advance(chunks);
      const double tnow = s->clock();
      for (int slot : done) {
        const int64_t t = s->slot_ticket64.at(slot);
        Request& r = s->reqs.at(t);
        s->slot_ticket64.erase(slot);
        lp_result o = to_result(s->eng64->result(slot), 0.0);
        o.polish_iters = o.iters;
        o.ident_iters = o.ident_iters > 0 ? o.ident_iters + r.first.iters : r.first.ident_iters;
        o.iters += r.first.iters;
        o.restarts += r.first.restarts;
        o.checks += r.first.checks;
        finish_request(s, r, *s->eng64, slot, o, tnow);
        ++nd;
      }
    }
    auto refine = [](halp::EngineBase& e, int& at) {
      const int live = e.live();
      if (live > 0 && 2 * live <= at) {
        e.refine_layouts();
        at = live;
      } else if (live == 0) {
        at = 0;
      }
    };
    refine(*s->eng, s->refine_live);
    if (s->eng64) refine(*s->eng64, s->refine_live64);
    if (n_done) *n_done = nd;
    return LP_OK;
  });
}

int lp_server_poll(lp_server* s, int64_t ticket, int* done, lp_result* out, double* t_done) {
  return guarded([&]() -> int {
    if (!s || !done) return fail(LP_ERR_INVALID, "null argument");
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(LP_ERR_INVALID, "unknown ticket");
    *done = it->second.done ? 1 : 0;
    if (it->second.done) {
      if (out) *out = it->second.res;
      if (t_done) *t_done = it->second.t_done;
    }
    return LP_OK;
  });
}

int lp_server_get_solution(lp_server* s, int64_t ticket, double* x, double* y) {
  return guarded([&]() -> int {
    if (!s) return fail(LP_ERR_INVALID, "null handle");
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(LP_ERR_INVALID, "unknown ticket");
    if (!it->second.done) return fail(LP_ERR_STATE, "ticket not finished");
    if (x) std::memcpy(x, it->second.x.data(), sizeof(double) * it->second.x.size());
    if (y && !it->second.y.empty()) std::memcpy(y, it->second.y.data(), sizeof(double) * it->second.y.size());
    return LP_OK;
  });
}

int lp_server_get_certificate(lp_server* s, int64_t ticket, double* ray) {
  return guarded([&]() -> int {
    if (!s || !ray) return fail(LP_ERR_INVALID, "null argument");
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(LP_ERR_INVALID, "unknown ticket");
    if (!it->second.done) return fail(LP_ERR_STATE, "ticket not finished");
    const int st = it->second.res.status;
    if (st != LP_PRIMAL_INFEASIBLE && st != LP_DUAL_INFEASIBLE)
      return fail(LP_ERR_STATE, "no certificate: the request was not found infeasible");
    if (!it->second.ray.empty())
      std::memcpy(ray, it->second.ray.data(), sizeof(double) * it->second.ray.size());
    return LP_OK;
  });
}

int lp_server_release(lp_server* s, int64_t ticket) {
  return guarded([&]() -> int {
    if (!s) return fail(LP_ERR_INVALID, "null handle");
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(LP_ERR_INVALID, "unknown ticket");
    if (!it->second.done) return fail(LP_ERR_STATE, "ticket not finished");
    s->reqs.erase(it);
    return LP_OK;
  });
}

int lp_server_clock(const lp_server* s, double* now) {
  return guarded([&]() -> int {
    if (!s || !now) return fail(LP_ERR_INVALID, "null argument");
    *now = s->clock();
    return LP_OK;
  });
}

int lp_server_info(const lp_server* s, int* queued, int* live, int64_t* bytes) {
  return guarded([&]() -> int {
    if (!s) return fail(LP_ERR_INVALID, "null handle");
    if (queued) *queued = (int)(s->queue.size() + s->queue64.size());
    if (live) *live = s->eng->live() + (s->eng64 ? s->eng64->live() : 0);
    if (bytes) {
      int64_t b = 0;
      for (auto& kv : s->slot_ticket) {
        const Request& r = s->reqs.at(kv.second);
        b += s->eng->footprint(r.n, r.m_eq + r.m_ineq, r.nnz);
      }
      for (auto& kv : s->slot_ticket64) {
        const Request& r = s->reqs.at(kv.second);
        b += s->eng64->footprint(r.n, r.m_eq + r.m_ineq, r.nnz);
      }
      *bytes = b;
    }
    return LP_OK;
  });
}

void lp_server_destroy(lp_server* s) {
  try {
    delete s;
  } catch (...) {
  }
}

}  // extern "C"

/* Host-side checks of the C ABI, built together with the library's sources
 * with host AddressSanitizer and UndefinedBehaviorSanitizer (device code is
 * not instrumented) by tests/test_abi_sanitized.py.  Every case here is
 * rejected or handled before any GPU work, so the program runs on a machine
 * without a GPU: malformed LPs and options, NULL handles and arguments for
 * every entry point, a randomised sweep of malformed CSR input, and host
 * canonicalisation (unsorted and duplicate column indices) of valid input,
 * which then stops at the first HIP call when no GPU is present.  Prints
 * "abi checks passed" and exits 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "halp.h"

static int failures = 0;

#define EXPECT(cond, ...)                      \
  do {                                         \
    if (!(cond)) {                             \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      fprintf(stderr, __VA_ARGS__);            \
      fprintf(stderr, " [%s]\n", lp_last_error()); \
      ++failures;                              \
    }                                          \
  } while (0)

/* A small valid LP: 2 equality + 1 inequality rows, 4 variables. */
typedef struct {
  int64_t n, m_eq, m_ineq;
  int32_t rp[4];
  int32_t ci[7];
  double val[7], c[4], rhs[3], lb[4], ub[4];
} Tiny;

static void tiny(Tiny* t) {
  static const int32_t rp[4] = {0, 2, 5, 7};
  static const int32_t ci[7] = {0, 2, 1, 2, 3, 0, 3};
  static const double val[7] = {1.0, -2.0, 0.5, 1.5, 3.0, 2.0, -1.0};
  t->n = 4;
  t->m_eq = 2;
  t->m_ineq = 1;
  memcpy(t->rp, rp, sizeof rp);
  memcpy(t->ci, ci, sizeof ci);
  memcpy(t->val, val, sizeof val);
  for (int j = 0; j < 4; ++j) {
    t->c[j] = 1.0 + j;
    t->lb[j] = 0.0;
    t->ub[j] = 10.0;
  }
  t->rhs[0] = 1.0;
  t->rhs[1] = 2.0;
  t->rhs[2] = -1.0;
}

static int create(const Tiny* t, const lp_options* opt, lp_solver** h) {
  *h = NULL;
  return lp_create(h, t->n, t->m_eq, t->m_ineq, t->rp, t->ci, t->val, t->c, t->rhs, t->lb, t->ub, 0, NULL, opt);
}

static void expect_invalid(const Tiny* t, const lp_options* opt, const char* what) {
  lp_solver* h = (lp_solver*)0x1;
  const int rc = create(t, opt, &h);
  EXPECT(rc == LP_ERR_INVALID, "%s: rc %d", what, rc);
  EXPECT(h == NULL, "%s: handle set on failure", what);
  if (rc == LP_OK) lp_destroy(h);
}

static void malformed_lps(void) {
  Tiny t;
  tiny(&t); t.n = 0; expect_invalid(&t, NULL, "n = 0");
  tiny(&t); t.m_eq = -1; expect_invalid(&t, NULL, "negative m_eq");
  tiny(&t); t.m_ineq = -2; expect_invalid(&t, NULL, "negative m_ineq");
  tiny(&t); t.rp[0] = 1; expect_invalid(&t, NULL, "row_ptr[0] != 0");
  tiny(&t); t.rp[2] = 1; expect_invalid(&t, NULL, "decreasing row_ptr");
  tiny(&t); t.ci[3] = 4; expect_invalid(&t, NULL, "column = n");
  tiny(&t); t.ci[0] = -1; expect_invalid(&t, NULL, "negative column");
  tiny(&t); t.val[4] = NAN; expect_invalid(&t, NULL, "NaN value");
  tiny(&t); t.val[6] = INFINITY; expect_invalid(&t, NULL, "infinite value");
  tiny(&t); t.c[1] = -INFINITY; expect_invalid(&t, NULL, "infinite objective");
  tiny(&t); t.rhs[2] = NAN; expect_invalid(&t, NULL, "NaN rhs");
  tiny(&t); t.lb[0] = 11.0; expect_invalid(&t, NULL, "lb > ub");
  tiny(&t); t.lb[3] = INFINITY; expect_invalid(&t, NULL, "lb = +inf");
  tiny(&t); t.ub[2] = -INFINITY; t.lb[2] = -INFINITY; expect_invalid(&t, NULL, "ub = -inf");
  tiny(&t); t.ub[1] = NAN; expect_invalid(&t, NULL, "NaN bound");
  {
    lp_solver* h = NULL;
    tiny(&t);
    EXPECT(lp_create(NULL, t.n, t.m_eq, t.m_ineq, t.rp, t.ci, t.val, t.c, t.rhs, t.lb, t.ub, 0, NULL, NULL) ==
               LP_ERR_INVALID, "NULL out");
    EXPECT(lp_create(&h, t.n, t.m_eq, t.m_ineq, NULL, t.ci, t.val, t.c, t.rhs, t.lb, t.ub, 0, NULL, NULL) ==
               LP_ERR_INVALID, "NULL row_ptr");
    EXPECT(lp_create(&h, t.n, t.m_eq, t.m_ineq, t.rp, NULL, t.val, t.c, t.rhs, t.lb, t.ub, 0, NULL, NULL) ==
               LP_ERR_INVALID, "NULL col_idx");
    EXPECT(lp_create(&h, t.n, t.m_eq, t.m_ineq, t.rp, t.ci, t.val, NULL, t.rhs, t.lb, t.ub, 0, NULL, NULL) ==
               LP_ERR_INVALID, "NULL c");
    EXPECT(lp_create(&h, t.n, t.m_eq, t.m_ineq, t.rp, t.ci, t.val, t.c, NULL, t.lb, t.ub, 0, NULL, NULL) ==
               LP_ERR_INVALID, "NULL rhs");
    EXPECT(lp_create(&h, t.n, t.m_eq, t.m_ineq, t.rp, t.ci, t.val, t.c, t.rhs, t.lb, NULL, 0, NULL, NULL) ==
               LP_ERR_INVALID, "NULL ub");
  }
}

static void row_ptr64(void) {
  Tiny t;
  tiny(&t);
  int64_t rp[4] = {0, 2, 5, 7};
  lp_solver* h = (lp_solver*)0x1;
  EXPECT(lp_create64(NULL, t.n, t.m_eq, t.m_ineq, rp, t.ci, t.val, t.c, t.rhs, t.lb, t.ub, 0, NULL, NULL) ==
             LP_ERR_INVALID, "lp_create64(NULL out)");
  EXPECT(lp_create64(&h, t.n, t.m_eq, t.m_ineq, NULL, t.ci, t.val, t.c, t.rhs, t.lb, t.ub, 0, NULL, NULL) ==
             LP_ERR_INVALID, "lp_create64(NULL row_ptr)");
  rp[2] = (int64_t)1 << 33;
  EXPECT(lp_create64(&h, t.n, t.m_eq, t.m_ineq, rp, t.ci, t.val, t.c, t.rhs, t.lb, t.ub, 0, NULL, NULL) ==
             LP_ERR_INVALID, "lp_create64(row_ptr above 2^31 - 1)");
  rp[2] = -5;
  EXPECT(lp_create64(&h, t.n, t.m_eq, t.m_ineq, rp, t.ci, t.val, t.c, t.rhs, t.lb, t.ub, 0, NULL, NULL) ==
             LP_ERR_INVALID, "lp_create64(negative row_ptr)");
  rp[2] = 5;
  t.ci[1] = 9;
  EXPECT(lp_create64(&h, t.n, t.m_eq, t.m_ineq, rp, t.ci, t.val, t.c, t.rhs, t.lb, t.ub, 0, NULL, NULL) ==
             LP_ERR_INVALID, "lp_create64(column out of range)");
  EXPECT(h == NULL, "lp_create64: handle set on failure");
}

static void invalid_options(void) {
  Tiny t;
  tiny(&t);
  lp_options o;
#define BAD(field, value)               \
  do {                                  \
    lp_default_options(&o);             \
    o.field = value;                    \
    expect_invalid(&t, &o, #field " = " #value); \
  } while (0)
  BAD(method, 3);
  BAD(method, -1);
  BAD(precision, 2);
  BAD(check_every, 0);
  BAD(step_safety, 0.0);
  BAD(step_safety, NAN);
  BAD(restart_mode, 3);
  BAD(tile_rows, 0);
  BAD(tile_rows, 257);
  BAD(slice_rows, 300);
  BAD(slice_entries, 700);
  BAD(slice_sort, 2);
  BAD(sort_rows, 0);
  BAD(sort_rows, 16385);
  BAD(plain_sort, -1);
  BAD(group_threads, 300);
  BAD(group_batched, 2);
  BAD(group_blocks, -1);
  BAD(polish_weight, 3);
#undef BAD
}

static void null_handles(void) {
  lp_result r;
  lp_kernel_timing kt;
  double x[4], y[3];
  int32_t rp[5], ci[8];
  double v[8];
  EXPECT(lp_solve(NULL, 1e-4, 10, -1.0) == LP_ERR_INVALID, "lp_solve(NULL)");
  EXPECT(lp_status(NULL, &r) == LP_ERR_INVALID, "lp_status(NULL)");
  EXPECT(lp_get_solution(NULL, x, y, 0) == LP_ERR_INVALID, "lp_get_solution(NULL)");
  EXPECT(lp_get_certificate(NULL, x, 0) == LP_ERR_INVALID, "lp_get_certificate(NULL)");
  EXPECT(lp_kernel_times(NULL, &kt) == LP_ERR_INVALID, "lp_kernel_times(NULL)");
  EXPECT(lp_get_scaled_matrix(NULL, 0, rp, ci, v) == LP_ERR_INVALID, "lp_get_scaled_matrix(NULL)");
  lp_destroy(NULL);

  lp_batch* b = (lp_batch*)0x1;
  EXPECT(lp_batch_create(&b, 0, NULL, 0, NULL, NULL) == LP_ERR_INVALID, "lp_batch_create(count 0)");
  EXPECT(lp_batch_create(NULL, 1, NULL, 0, NULL, NULL) == LP_ERR_INVALID, "lp_batch_create(NULL)");
  EXPECT(lp_batch_solve(NULL, 1e-4, 10, -1.0) == LP_ERR_INVALID, "lp_batch_solve(NULL)");
  EXPECT(lp_batch_status(NULL, 0, &r) == LP_ERR_INVALID, "lp_batch_status(NULL)");
  EXPECT(lp_batch_get_solution(NULL, 0, x, y, 0) == LP_ERR_INVALID, "lp_batch_get_solution(NULL)");
  EXPECT(lp_batch_get_certificate(NULL, 0, x, 0) == LP_ERR_INVALID, "lp_batch_get_certificate(NULL)");
  EXPECT(lp_batch_kernel_times(NULL, &kt) == LP_ERR_INVALID, "lp_batch_kernel_times(NULL)");
  lp_batch_destroy(NULL);

  lp_server* s = (lp_server*)0x1;
  int done = 0, q = 0, live = 0;
  int64_t bytes = 0, ticket = 0;
  double t = 0.0;
  EXPECT(lp_server_create(&s, 0, 4, NULL, NULL) == LP_ERR_INVALID, "lp_server_create(budget 0)");
  EXPECT(lp_server_create(&s, 1 << 30, 0, NULL, NULL) == LP_ERR_INVALID, "lp_server_create(0 slots)");
  EXPECT(lp_server_create(NULL, 1 << 30, 4, NULL, NULL) == LP_ERR_INVALID, "lp_server_create(NULL)");
  EXPECT(lp_server_submit(NULL, NULL, 1e-4, 10, 0.0, &ticket) == LP_ERR_INVALID, "lp_server_submit(NULL)");
  EXPECT(lp_server_step(NULL, 1, &done) == LP_ERR_INVALID, "lp_server_step(NULL)");
  EXPECT(lp_server_poll(NULL, 1, &done, &r, &t) == LP_ERR_INVALID, "lp_server_poll(NULL)");
  EXPECT(lp_server_get_solution(NULL, 1, x, y) == LP_ERR_INVALID, "lp_server_get_solution(NULL)");
  EXPECT(lp_server_get_certificate(NULL, 1, x) == LP_ERR_INVALID, "lp_server_get_certificate(NULL)");
  EXPECT(lp_server_release(NULL, 1) == LP_ERR_INVALID, "lp_server_release(NULL)");
  EXPECT(lp_server_clock(NULL, &t) == LP_ERR_INVALID, "lp_server_clock(NULL)");
  EXPECT(lp_server_info(NULL, &q, &live, &bytes) == LP_ERR_INVALID, "lp_server_info(NULL)");
  lp_server_destroy(NULL);

  Tiny tn;
  tiny(&tn);
  lp_options o;
  lp_default_options(&o);
  o.precision = 1;
  EXPECT(lp_solve_static(tn.n, tn.m_eq, tn.m_ineq, tn.rp, tn.ci, tn.val, tn.c, tn.rhs, tn.lb, tn.ub, NULL, &o,
                         1e-4, 10, -1.0, NULL, NULL, &r) == LP_ERR_INVALID, "lp_solve_static(FP32)");
  EXPECT(lp_solve_static(tn.n, tn.m_eq, tn.m_ineq, tn.rp, tn.ci, tn.val, tn.c, tn.rhs, tn.lb, tn.ub, NULL, NULL,
                         1e-4, 10, -1.0, NULL, NULL, NULL) == LP_ERR_INVALID, "lp_solve_static(NULL out)");
  EXPECT(lp_last_error() != NULL && lp_last_error()[0] != '\0', "empty error message");
}

/* Random CSR of m rows over n columns with one planted defect; every case
 * must be rejected, whatever the defect's position. */
static uint64_t rng_state = 0x2407161440ull;
static uint64_t next_u64(void) {
  /* SplitMix64 (Steele, Lea and Flood, 2014) */
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

static void random_malformed(int rounds) {
  for (int k = 0; k < rounds; ++k) {
    const int64_t m = 1 + (int64_t)(next_u64() % 60), n = 1 + (int64_t)(next_u64() % 80);
    int32_t* rp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m + 1));
    rp[0] = 0;
    for (int64_t i = 0; i < m; ++i) rp[i + 1] = rp[i] + (int32_t)(next_u64() % 6);
    const int64_t nnz = rp[m];
    int32_t* ci = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double* val = (double*)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    double* lb = (double*)malloc(sizeof(double) * (size_t)n);
    double* ub = (double*)malloc(sizeof(double) * (size_t)n);
    double* rhs = (double*)malloc(sizeof(double) * (size_t)m);
    for (int64_t e = 0; e < nnz; ++e) {
      ci[e] = (int32_t)(next_u64() % (uint64_t)n);
      val[e] = 1.0 + (double)(next_u64() % 100);
    }
    for (int64_t j = 0; j < n; ++j) {
      c[j] = (double)(next_u64() % 7) - 3.0;
      lb[j] = 0.0;
      ub[j] = (next_u64() & 1) ? INFINITY : 5.0;
    }
    for (int64_t i = 0; i < m; ++i) rhs[i] = (double)(next_u64() % 9);
    const int kind = (int)(next_u64() % 6);
    const char* what = "";
    if (kind == 0 && nnz > 0) {
      ci[next_u64() % (uint64_t)nnz] = (int32_t)n;
      what = "column = n";
    } else if (kind == 1 && nnz > 0) {
      val[next_u64() % (uint64_t)nnz] = NAN;
      what = "NaN value";
    } else if (kind == 2) {
      rhs[next_u64() % (uint64_t)m] = INFINITY;
      what = "infinite rhs";
    } else if (kind == 3) {
      const int64_t j = (int64_t)(next_u64() % (uint64_t)n);
      lb[j] = 6.0;
      ub[j] = 5.0;
      what = "lb > ub";
    } else if (kind == 4 && m > 1) {
      const int64_t i = 1 + (int64_t)(next_u64() % (uint64_t)(m - 1));
      rp[i] = rp[i + 1] + 1;
      what = "decreasing row_ptr";
    } else {
      c[next_u64() % (uint64_t)n] = NAN;
      what = "NaN objective";
    }
    lp_solver* h = NULL;
    const int64_t m_eq = (int64_t)(next_u64() % (uint64_t)(m + 1));
    const int rc = lp_create(&h, n, m_eq, m - m_eq, rp, ci, val, c, rhs, lb, ub, 0, NULL, NULL);
    EXPECT(rc == LP_ERR_INVALID, "random case %d (%s): rc %d", k, what, rc);
    if (rc == LP_OK) lp_destroy(h);
    free(rp);
    free(ci);
    free(val);
    free(c);
    free(lb);
    free(ub);
    free(rhs);
  }
}

/* Valid input with unsorted and duplicate column indices: the host
 * canonicalisation runs, then the call either succeeds (a GPU is present)
 * or stops at the first HIP call (LP_ERR_DEVICE). */
static void canonicalisation(void) {
  Tiny t;
  tiny(&t);
  const int32_t ci[7] = {2, 0, 3, 2, 2, 3, 0};
  memcpy(t.ci, ci, sizeof ci);
  lp_solver* h = NULL;
  const int rc = create(&t, NULL, &h);
  EXPECT(rc == LP_OK || rc == LP_ERR_DEVICE, "canonicalisation: rc %d", rc);
  if (rc == LP_OK) lp_destroy(h);
}

int main(void) {
  lp_options o;
  lp_default_options(&o);
  EXPECT(o.method == 1 && o.precision == 0, "defaults");
  malformed_lps();
  row_ptr64();
  invalid_options();
  null_handles();
  random_malformed(2000);
  canonicalisation();
  if (failures) {
    fprintf(stderr, "%d abi checks failed\n", failures);
    return 1;
  }
  printf("abi checks passed\n");
  return 0;
}

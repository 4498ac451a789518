// Device kernels of the restarted Halpern PDHG solver (gfx950 / CDNA4).
//
// One solver step is two launches over fixed workgroup schedules:
//   primal_step : y-gather SpMV over the rows of the explicit K^T, fused with
//                 the primal PDHG step, box projection and Halpern blend;
//   dual_step   : xbar-gather SpMV over the rows of K, fused with the dual
//                 step, cone projection and Halpern blend; the last workgroup
//                 of each LP (arrival counter) reduces that LP's block partial
//                 sums in a fixed order and runs its restart / termination
//                 controller on the device.
// The path is bandwidth bound (about 2 flop per 12 bytes of matrix), so there
// is no MFMA: the work is coalesced entry loads, gathers, LDS staging and
// wave64 shuffle reductions.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "halp_types.h"
#include "kernels.h"

namespace halp {

// ---------------------------------------------------------------------------
// reductions (fixed order: results do not depend on scheduling)
// ---------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of kNS per-thread values over the block; result valid in s_out[0..kNS).
__device__ __forceinline__ void block_sum_ns(double (&v)[kNS], double (*s_red)[kNS], double* s_out) {
#pragma unroll
  for (int s = 0; s < kNS; ++s) v[s] = wave_sum(v[s]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < kNS; ++s) s_red[wave][s] = v[s];
  }
  __syncthreads();
  if (threadIdx.x < kNS) {
    double a = s_red[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) a += s_red[w][threadIdx.x];
    s_out[threadIdx.x] = a;
  }
  __syncthreads();
}

template <class T>
__device__ __forceinline__ T block_sum1(T v, double (*s_red)[kNS]) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s_red[wave][0] = (double)v;
  __syncthreads();
  T a = (T)s_red[0][0];
#pragma unroll
  for (int w = 1; w < kThreads / 64; ++w) a += (T)s_red[w][0];
  __syncthreads();
  return a;
}

// Fixed-order sum of nb rows of kNS partials; all threads call, result in s_out.
__device__ void sum_partials(const double* part, int nb, double (*s_red)[kNS], double* s_out) {
  double v[kNS];
#pragma unroll
  for (int s = 0; s < kNS; ++s) v[s] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) {
#pragma unroll
    for (int s = 0; s < kNS; ++s) v[s] += part[(int64_t)b * kNS + s];
  }
  block_sum_ns(v, s_red, s_out);
}

__device__ __forceinline__ int group_size(int nrows) {
  // largest power of two G <= 64 with nrows * G <= kThreads (at least 1)
  int g = 64;
  while (g > 1 && g * nrows > kThreads) g >>= 1;
  return g;
}

// Workgroup barrier that orders LDS only: outstanding global loads (prefetched
// epilogue operands) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// block SpMV: row sums of NV gathered vectors for the rows of one block.
// rp points at the block's row pointers (rp[0..nrows], entry positions);
// the entry range [b.p0, b.p0 + b.pn) comes with the descriptor, so entry
// loads start without waiting for the row pointers.
// Stream blocks (<= NB entries, <= kMaxRows rows): entries are loaded once,
// coalesced, into registers; per gathered vector the products go to LDS and
// groups of G lanes reduce each row.  Long blocks (one row): strided loop
// with four accumulators and a block reduction.
// Result: s_rsum[a][r - b.r0].
// ---------------------------------------------------------------------------

template <class T, int NB = kPlainNB>
struct TileRegs {
  static constexpr int EPT = NB / kThreads;
  int cidx[EPT];
  T v[EPT];
  T p[EPT];      // products with a gathered vector
  int rpv = 0;   // row pointer t of the block (relative to p0), t = thread
  int rpv2 = 0;  // row pointer kThreads (thread 0, blocks of kThreads rows)
};

// Products with the step's usual gathered vector, issued before the LP
// state is read (the state only decides whether they are used).
template <class T, int NB>
__device__ __forceinline__ void spec_products(const Blk& b, const T* __restrict__ src, TileRegs<T, NB>& R) {
  if (blk_kind(b) != BK_STREAM) return;
#pragma unroll
  for (int k = 0; k < TileRegs<T, NB>::EPT; ++k) {
    const int e = (int)threadIdx.x + k * kThreads;
    if (e < b.pn) R.p[k] = R.v[k] * src[R.cidx[k]];
  }
}

// Loads a stream block's entries (coalesced) and row pointers into
// registers; independent of the step mode, so callers issue it before
// reading the LP state.  rp points at the block's first row pointer.
template <bool NT, class V>
__device__ __forceinline__ V ld_entry(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NT, class T, int NB>
__device__ __forceinline__ void load_tile_as(const Blk& b, const int32_t* __restrict__ rp,
                                             const int32_t* __restrict__ ci, const T* __restrict__ val,
                                             TileRegs<T, NB>& R) {
  const int t = threadIdx.x;
  const int nrows = b.r1 - b.r0;
#pragma unroll
  for (int k = 0; k < TileRegs<T, NB>::EPT; ++k) {
    const int e = t + k * kThreads;
    if (e < b.pn) {
      R.cidx[k] = ld_entry<NT>(ci + b.p0 + e);
      R.v[k] = ld_entry<NT>(val + b.p0 + e);
    }
  }
  if (t <= nrows) R.rpv = rp[t] - b.p0;
  if (nrows == kThreads && t == 0) R.rpv2 = rp[kThreads] - b.p0;
}

// Loads a stream block's entries (coalesced) and row pointers into
// registers; independent of the step mode, so callers issue it before
// reading the LP state.  rp points at the block's first row pointer.
template <class T, int NB>
__device__ __forceinline__ void load_tile(const Blk& b, const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ ci, const T* __restrict__ val,
                                          TileRegs<T, NB>& R) {
  if (blk_kind(b) != BK_STREAM) return;
  if (blk_nt(b)) load_tile_as<true, T, NB>(b, rp, ci, val, R);
  else load_tile_as<false, T, NB>(b, rp, ci, val, R);
}

// Strided partial sums of one long row (entries [p0, p0 + pn)).
template <bool NT, class T>
__device__ __forceinline__ T long_row_sum(int p0, int pn, const int32_t* __restrict__ ci,
                                          const T* __restrict__ val, const T* __restrict__ src) {
  T acc0 = (T)0, acc1 = (T)0;
  int e = threadIdx.x;
  for (; e + kThreads < pn; e += 2 * kThreads) {
    const int c0 = ld_entry<NT>(ci + p0 + e), c1 = ld_entry<NT>(ci + p0 + e + kThreads);
    const T v0 = ld_entry<NT>(val + p0 + e), v1 = ld_entry<NT>(val + p0 + e + kThreads);
    acc0 += v0 * src[c0];
    acc1 += v1 * src[c1];
  }
  if (e < pn) acc0 += ld_entry<NT>(val + p0 + e) * src[ld_entry<NT>(ci + p0 + e)];
  return acc0 + acc1;
}

// One gathered vector: row sums into out[r - b.r0] (LDS).
template <class T, int NB>
__device__ void block_spmv1(const Blk& b, const int32_t* __restrict__ ci,
                            const T* __restrict__ val, const TileRegs<T, NB>& R, const T* __restrict__ src,
                            T* s_prod, T* out, int* s_rp, double (*s_red)[kNS], T scale = (T)1,
                            bool have_products = false) {
  const int tid = threadIdx.x;
  const int nrows = b.r1 - b.r0;
  const int p0 = b.p0, pn = b.pn;
  if (blk_kind(b) == BK_LONG) {
    T t = wave_sum(blk_nt(b) ? long_row_sum<true>(p0, pn, ci, val, src) : long_row_sum<false>(p0, pn, ci, val, src));
    if ((tid & 63) == 0) s_red[tid >> 6][0] = (double)t;
    lds_barrier();
    if (tid == 0) {
      T u = (T)s_red[0][0];
#pragma unroll
      for (int w = 1; w < kThreads / 64; ++w) u += (T)s_red[w][0];
      out[0] = u * scale;
    }
    lds_barrier();
    return;
  }
  constexpr int EPT = TileRegs<T, NB>::EPT;
  if (tid <= nrows) s_rp[tid] = R.rpv;
  if (nrows == kThreads && tid == 0) s_rp[kThreads] = R.rpv2;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = tid + k * kThreads;
    if (e < pn) s_prod[e] = have_products ? R.p[k] : R.v[k] * src[R.cidx[k]];
  }
  lds_barrier();
  const int G = group_size(nrows);
  const int lane = tid & (G - 1);
  const int rpb = kThreads / G;  // rows per pass
  for (int base = 0; base < nrows; base += rpb) {
    const int r = base + tid / G;
    T acc = (T)0;
    if (r < nrows) {
      const int q1 = s_rp[r + 1];
      for (int q = s_rp[r] + lane; q < q1; q += G) acc += s_prod[q];
    }
    for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0 && r < nrows) out[r] = acc * scale;
  }
  lds_barrier();
}

// NV gathered vectors, one after the other over the same register tile
template <class T, int NV, int NB>
__device__ __forceinline__ void block_spmv_regs(const Blk& b,
                                                const int32_t* __restrict__ ci, const T* __restrict__ val,
                                                const TileRegs<T, NB>& R, const T* __restrict__ s0,
                                                const T* __restrict__ s1, const T* __restrict__ s2, T* s_prod,
                                                T (*s_rsum)[kMaxRows], int* s_rp, double (*s_red)[kNS],
                                                T scale0 = (T)1) {
  block_spmv1<T, NB>(b, ci, val, R, s0, s_prod, s_rsum[0], s_rp, s_red, scale0);
  if constexpr (NV > 1) block_spmv1<T, NB>(b, ci, val, R, s1, s_prod, s_rsum[1], s_rp, s_red);
  if constexpr (NV > 2) block_spmv1<T, NB>(b, ci, val, R, s2, s_prod, s_rsum[2], s_rp, s_red);
}

template <class T, int NV>
__device__ __forceinline__ void block_spmv(const Blk& b, const int32_t* __restrict__ rp,
                                           const int32_t* __restrict__ ci, const T* __restrict__ val,
                                           const T* __restrict__ s0, const T* __restrict__ s1,
                                           const T* __restrict__ s2, T* s_prod, T (*s_rsum)[kMaxRows],
                                           int* s_rp, double (*s_red)[kNS], T scale0 = (T)1) {
  TileRegs<T, kPlainNB> R;
  load_tile<T, kPlainNB>(b, rp, ci, val, R);
  block_spmv_regs<T, NV, kPlainNB>(b, ci, val, R, s0, s1, s2, s_prod, s_rsum, s_rp, s_red, scale0);
}

// Row sums of a row group whose products a slice kernel computed: the
// blk_nsl(b) partial sums per row, added in slice order.
template <class T, int NV>
__device__ __forceinline__ void gather_slices(const Blk& b, const T* __restrict__ spart, int64_t space,
                                              T (*s_rsum)[kMaxRows]) {
  const int nrows = b.r1 - b.r0;
  const int nsl = blk_nsl(b);
  const int t = threadIdx.x;
  if (t < nrows) {
    // one vector at a time: its partial loads in flight together, but not
    // the NV * nsl of all vectors (they would set the register budget of the
    // whole step kernel)
#pragma unroll 1
    for (int a = 0; a < NV; ++a) {
      T part[kSlices];
#pragma unroll
      for (int q = 0; q < kSlices; ++q)
        part[q] = q < nsl ? spart[(int64_t)(a * kSlices + q) * space + b.r0 + t] : (T)0;
      T acc = part[0];
#pragma unroll
      for (int q = 1; q < kSlices; ++q)
        if (q < nsl) acc += part[q];
      s_rsum[a][t] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// step modes
// ---------------------------------------------------------------------------

// Mode of step g for one LP.  Checks fall at inner counters k = C, 2C, ...
// of an epoch (k = g - kbase); the controller keeps the step index of the
// next one in next_check.
__device__ __forceinline__ int step_mode(const InstState& S, int64_t g) {
  if (S.status != ST_RUNNING) return M_SKIP;
  if (S.phase == PH_EVAL) return M_EVAL;
  if (S.phase == PH_RESID) return M_RESID;
  if (g < S.kbase) return M_SKIP;
  if (g == S.next_check) return M_CHECK;
  return M_NORMAL;
}

template <class T>
__device__ __forceinline__ T clampT(T v, T lo, T hi) {
  return fmin(fmax(v, lo), hi);
}

// projection of a direction onto the recession cone of [l, u]
template <class T>
__device__ __forceinline__ T rec_proj(T d, bool lf, bool uf) {
  return (lf && uf) ? (T)0 : lf ? fmax(d, (T)0) : uf ? fmin(d, (T)0) : d;
}

// ---------------------------------------------------------------------------
// primal step (rows of K^T = variables)
// ---------------------------------------------------------------------------

// Row sums of one column-sorted block (a plain BK_SORTED block) for the
// gathered vector src, accumulated in FP64 LDS words whatever the compute
// type (products in the compute type; on gfx950 ds_add_f64 measured 1.8x
// faster than ds_add_f32 on these scattered adds):
// consecutive entries gather nearby elements of the slice, so the rows of
// the group share the cache lines of their gathers.  Products go to the LDS
// row sums s_row by atomic adds, so the order of the additions within a row
// is not fixed (the last bits of a sum can differ from run to run).
// U: entries in flight per thread (measured on the large LP: 8 for the
// slice groups of K, 4 for the blocks of K^T, whose step kernel also holds
// the epilogue's registers)
template <class T, bool NT, int U>
__device__ __forceinline__ void sorted_rows_sum(const Blk& b, const uint32_t* __restrict__ w,
                                                const T* __restrict__ val, const T* __restrict__ src,
                                                double* s_row) {
  const int rb = blk_rowbits(b);
  const uint32_t rmask = (1u << rb) - 1u;
  const T* srcb = src + b.rp_off;
  for (int e0 = threadIdx.x; e0 < b.pn; e0 += kThreads * U) {
    uint32_t k[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kThreads;
      if (e < b.pn) {
        k[u] = ld_entry<NT>(w + b.p0 + e);
        v[u] = ld_entry<NT>(val + b.p0 + e);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kThreads;
      if (e < b.pn) atomicAdd(&s_row[k[u] & rmask], (double)(v[u] * srcb[k[u] >> rb]));
    }
  }
}

// One variable's part of a primal step (rows of K^T): j is its space
// position, kty its row sum (K^T y, or K^T yT at an eval step, where g1 and
// g2 are K^T cy1 and K^T cy2; at a residual step the caller passes T(z) as
// xo and x0j and K^T yT as kty).  Adds the check / eval / residual terms of
// the variable to ps.
template <class T>
__device__ __forceinline__ void primal_row(const IterArgs<T>& A, const InstState& S, int mode, int64_t g,
                                           int64_t j, T cj, T lj, T uj, T xo, T x0j, T kty, T g1, T g2,
                                           double (&ps)[kNS]) {
  const bool resid = (mode == M_RESID);
  const bool lf = isfinite(lj), uf = isfinite(uj);
  if (mode == M_EVAL) {
    const T g0 = kty;
    A.ktyp[j] = g0;
    const double dc = A.Dc[j];
    const double r = (double)cj - (double)g0;
    const double lam = (lf && uf) ? r : lf ? fmax(r, 0.0) : uf ? fmin(r, 0.0) : 0.0;
    const double rd = (r - lam) / dc;
    ps[0] += rd * rd;
    ps[1] += (lf ? (double)lj * fmax(lam, 0.0) : 0.0) - (uf ? (double)uj * fmax(-lam, 0.0) : 0.0);
#pragma unroll
    for (int a = 1; a <= 2; ++a) {
      const double gg = (double)(a == 1 ? g1 : g2);
      double sv = 0.0, vv = 0.0;
      if (gg > 0.0) {
        if (uf) sv = (double)uj * gg; else vv = gg / dc;
      } else if (gg < 0.0) {
        if (lf) sv = (double)lj * gg; else vv = -gg / dc;
      }
      ps[2 * a] += sv;
      ps[2 * a + 1] += vv * vv;
    }
    return;
  }
  const T tau = (T)S.tau;
  const T xp = clampT<T>(xo - tau * (cj - kty), lj, uj);
  const T xb = (T)2 * xp - xo;
  const int64_t k = g - S.kbase;
  T xn, xc = xp;  // next iterate; check candidate (T(z), or the epoch average)
  if (S.avg) {
    // plain PDHG step; running sum of z^{n,0..k+1} (restarted at k = 0)
    const T xsum = (k == 0 ? xo : A.xs[j]) + xp;
    A.xs[j] = xsum;
    xn = xp;
    if (mode == M_CHECK) xc = xsum / (T)(k + 2);
  } else {
    const double w = (double)(k + 1) / (double)(k + 2);
    const T xh = S.reflect ? xb : xp;
    xn = (T)w * xh + (T)(1.0 - w) * x0j;
  }
  A.xbar[j] = xb;
  A.x[j] = xn;
  if (resid) {
    A.x0[j] = xo;
    const double d = (double)xo - (double)xp;
    ps[0] += d * d;
  } else if (mode == M_CHECK) {
    A.xT[j] = xc;
    const double d = (double)xo - (double)xp;
    const double ad = (double)xc - (double)x0j;
    const T d1 = rec_proj<T>(xp - xo, lf, uf);
    const T d2 = rec_proj<T>(xo - x0j, lf, uf);
    A.cx1[j] = d1;
    A.cx2[j] = d2;
    ps[0] += d * d;
    ps[1] += ad * ad;
    ps[2] += (double)cj * (double)xc;
    ps[3] += (double)cj * (double)d1;
    ps[4] += (double)cj * (double)d2;
    const uint8_t act = (lf && xp == lj) ? 1 : (uf && xp == uj) ? 2 : 0;
    const uint8_t was = A.actx[j];
    A.actx[j] = act;
    ps[5] += (was != 255 && was != act) ? 1.0 : 0.0;
  }
}

// Row sums of a column-sorted block (BK_SORTED) for the gathered vector src,
// left in s_row[0 .. nrows).
template <class T>
__device__ __forceinline__ void sorted_pass(const Blk& b, const int32_t* __restrict__ ci,
                                            const T* __restrict__ val, const T* __restrict__ src, double* s_row) {
  const int nrows = b.r1 - b.r0;
  for (int r = threadIdx.x; r < nrows; r += kThreads) s_row[r] = 0.0;
  lds_barrier();
  const uint32_t* w = reinterpret_cast<const uint32_t*>(ci);
  if (blk_nt(b)) sorted_rows_sum<T, true, 4>(b, w, val, src, s_row);
  else sorted_rows_sum<T, false, 4>(b, w, val, src, s_row);
  lds_barrier();
}

// The same, stored to out[b.r0 + r] by the thread that later reads it back
// (row r is handled by thread r mod kThreads in every loop over a block).
template <class T>
__device__ __forceinline__ void sorted_pass_to(const Blk& b, const int32_t* __restrict__ ci,
                                               const T* __restrict__ val, const T* __restrict__ src, double* s_row,
                                               T* out) {
  sorted_pass<T>(b, ci, val, src, s_row);
  const int nrows = b.r1 - b.r0;
  for (int r = threadIdx.x; r < nrows; r += kThreads) out[(int64_t)b.r0 + r] = (T)s_row[r];
  lds_barrier();
}

// A primal step over a column-sorted block of K^T rows (up to kSortRowsPlain
// variables): the products with y (yT, cy1, cy2 at an eval step) are added
// into LDS row sums, then each thread takes the epilogue of every
// kThreads-th variable.
template <class T>
__device__ void primal_sorted(const IterArgs<T>& A, const Blk& b, int step, double* s_row,
                              double (*s_red)[kNS], double* s_out) {
  const InstState& S = A.st[b.inst];
  const int64_t g = *A.gbase + step;
  const int mode = step_mode(S, g);
  if (mode == M_SKIP) return;
  const bool resid = (mode == M_RESID);
  const int nrows = b.r1 - b.r0;
  if (mode == M_EVAL) {
    sorted_pass_to<T>(b, A.KT_ci, A.KT_v, A.cy1, s_row, A.kt1);
    sorted_pass_to<T>(b, A.KT_ci, A.KT_v, A.cy2, s_row, A.kt2);
    sorted_pass<T>(b, A.KT_ci, A.KT_v, A.yT, s_row);
  } else if (!resid) {
    sorted_pass<T>(b, A.KT_ci, A.KT_v, A.y, s_row);
  }
  double ps[kNS];
#pragma unroll
  for (int s = 0; s < kNS; ++s) ps[s] = 0.0;
  for (int r = threadIdx.x; r < nrows; r += kThreads) {
    const int64_t j = (int64_t)b.r0 + r;
    const T cj = A.c[j], lj = A.l[j], uj = A.u[j];
    T xo, x0j, kty, g1 = 0, g2 = 0;
    if (resid) {
      xo = A.xT[j];
      x0j = xo;
      kty = A.ktyp[j];
    } else {
      xo = A.x[j];
      x0j = A.x0[j];
      kty = (T)s_row[r];
      if (mode == M_EVAL) {
        g1 = A.kt1[j];
        g2 = A.kt2[j];
      }
    }
    primal_row<T>(A, S, mode, g, j, cj, lj, uj, xo, x0j, kty, g1, g2, ps);
  }
  if (mode != M_NORMAL) {
    block_sum_ns(ps, s_red, s_out);
    if (threadIdx.x < kNS) A.partP[(int64_t)b.gid * kNS + threadIdx.x] = s_out[threadIdx.x];
  }
}

// LDS of a step kernel: the plain tile's products, row sums and row
// pointers, or the row sums of a column-sorted block (never both).
template <class T>
union StepSmem {
  struct {
    T prod[Tile<T>::NB];
    T rsum[3][kMaxRows];
    int rp[kMaxRows + 1];
  } p;
  double rows[kSortRowsPlain];
};

template <class T>
__global__ __launch_bounds__(kThreads) void primal_step(IterArgs<T> A, int step) {
  __shared__ StepSmem<T> sm;
  __shared__ double s_red[kThreads / 64][kNS];
  __shared__ double s_out[kNS];
  T* s_prod = sm.p.prod;
  T (*s_rsum)[kMaxRows] = sm.p.rsum;
  int* s_rp = sm.p.rp;

  const Blk b = A.schedP[blockIdx.x];
  if (blk_kind(b) == BK_PAD) return;
  if (blk_kind(b) == BK_SORTED) {
    primal_sorted<T>(A, b, step, sm.rows, s_red, s_out);
    return;
  }
  const int nrows = b.r1 - b.r0;
  const int t = threadIdx.x;
  const bool own = t < nrows;
  const int64_t j = (int64_t)b.r0 + (own ? t : 0);
  // entries and epilogue operands are loaded before the LP state is read,
  // so their latency overlaps the state loads (none depends on the mode)
  TileRegs<T, kPlainNB> R;
  load_tile<T, kPlainNB>(b, A.KT_rp + b.r0, A.KT_ci, A.KT_v, R);
  spec_products<T, kPlainNB>(b, A.y, R);
  T cj = 0, lj = 0, uj = 0, xo = 0, x0j = 0, kty = 0;
  if (own) {
    cj = A.c[j];
    lj = A.l[j];
    uj = A.u[j];
    xo = A.x[j];
    x0j = A.x0[j];
  }
  const InstState& S = A.st[b.inst];
  const int64_t g = *A.gbase + step;
  const int mode = step_mode(S, g);
  if (mode == M_SKIP) return;
  const bool resid = (mode == M_RESID);
  if (resid && own) {
    xo = A.xT[j];
    x0j = xo;
    kty = A.ktyp[j];
  }
  if (blk_part(b)) {
    if (mode == M_EVAL) gather_slices<T, 3>(b, A.spartP, A.NS, s_rsum);
    else if (!resid) gather_slices<T, 1>(b, A.spartP, A.NS, s_rsum);
  } else if (mode == M_EVAL) {
    block_spmv_regs<T, 3, kPlainNB>(b, A.KT_ci, A.KT_v, R, A.yT, A.cy1, A.cy2, s_prod, s_rsum, s_rp, s_red);
  } else if (!resid) {
    block_spmv1<T, kPlainNB>(b, A.KT_ci, A.KT_v, R, A.y, s_prod, s_rsum[0], s_rp, s_red, (T)1, true);
  }

  double ps[kNS];
#pragma unroll
  for (int s = 0; s < kNS; ++s) ps[s] = 0.0;
  if (own) {
    const bool eval = (mode == M_EVAL);
    primal_row<T>(A, S, mode, g, j, cj, lj, uj, xo, x0j, resid ? kty : s_rsum[0][t],
                  eval ? s_rsum[1][t] : (T)0, eval ? s_rsum[2][t] : (T)0, ps);
  }
  if (mode != M_NORMAL) {
    block_sum_ns(ps, s_red, s_out);
    if (t < kNS) A.partP[(int64_t)b.gid * kNS + t] = s_out[t];
  }
}

// Partial row sums of one column slice of a sliced row group (written to
// spart for the step kernel of the same step to add up).  dual = 1: rows of
// K gathering xbar (or xT, cx1, cx2 at an eval step); dual = 0: rows of K^T
// gathering y (or yT, cy1, cy2).
template <class T, bool dual, int NB>
__device__ __forceinline__ void slice_body(const IterArgs<T>& A, int step) {
  __shared__ T s_prod[NB];
  __shared__ T s_rsum[3][kMaxRows];
  __shared__ int s_rp[kMaxRows + 1];
  __shared__ double s_red[kThreads / 64][kNS];
  const Blk b = (dual ? A.schedDS : A.schedPS)[blockIdx.x];
  if (blk_kind(b) == BK_PAD) return;
  const int32_t* rp = (dual ? A.brpK : A.brpKT) + b.rp_off;
  const int32_t* ci = dual ? A.K_ci : A.KT_ci;
  const T* val = dual ? A.K_v : A.KT_v;
  TileRegs<T, NB> R;
  load_tile<T, NB>(b, rp, ci, val, R);
  const T* src = dual ? A.xbar : A.y;
  spec_products<T, NB>(b, src, R);
  const InstState& S = A.st[b.inst];
  const int64_t g = *A.gbase + step;
  const int mode = step_mode(S, g);
  if (mode == M_SKIP || (!dual && mode == M_RESID)) return;
  T* spart = dual ? A.spartD : A.spartP;
  const int64_t space = dual ? A.MS : A.NS;
  const int nv = mode == M_EVAL ? 3 : 1;
  if (mode == M_EVAL) {
    if (dual) block_spmv_regs<T, 3, NB>(b, ci, val, R, A.xT, A.cx1, A.cx2, s_prod, s_rsum, s_rp, s_red);
    else block_spmv_regs<T, 3, NB>(b, ci, val, R, A.yT, A.cy1, A.cy2, s_prod, s_rsum, s_rp, s_red);
  } else {
    block_spmv1<T, NB>(b, ci, val, R, src, s_prod, s_rsum[0], s_rp, s_red, (T)1, true);
  }
  const int nrows = b.r1 - b.r0;
  const int sl = blk_slice(b);
  for (int r = threadIdx.x; r < nrows; r += kThreads)
    for (int a = 0; a < nv; ++a) spart[(int64_t)(a * kSlices + sl) * space + b.r0 + r] = s_rsum[a][r];
}

// NB: entries per slice tile (kSliceTiles lists the compiled sizes; the
// engine picks one per solver, and the tuner in the Python package times them)
template <class T, int NB>
__global__ __launch_bounds__(kThreads) void primal_slice_step(IterArgs<T> A, int step) {
  slice_body<T, false, NB>(A, step);
}

template <class T, int NB>
__global__ __launch_bounds__(kThreads) void dual_slice_step(IterArgs<T> A, int step) {
  slice_body<T, true, NB>(A, step);
}

// Row sums of one (group, slice) block of a sorted-group product, TPB
// threads, U entries in flight per thread.  BATCHED: per batch the U entry
// loads, then the U gathers, then the U LDS adds, with no branch between
// them (the gathers of a thread in flight together); otherwise each gather
// is guarded by its own bounds test (a gather waits for the previous add).
// Both orders of the additions within a row depend on wave timing.
template <class T, int TPB, int U, bool BATCHED, bool NT>
__device__ __forceinline__ void group_rows_sum(const Blk& b, const uint32_t* __restrict__ w,
                                               const T* __restrict__ val, const T* __restrict__ src,
                                               double* s_row) {
  const int rb = blk_rowbits(b);
  const uint32_t rmask = (1u << rb) - 1u;
  const T* srcb = src + b.rp_off;
  const uint32_t* kp = w + b.p0;
  const T* vp = val + b.p0;
  const int pn = b.pn;
  int e0 = threadIdx.x;
  if constexpr (BATCHED) {
    const int full = pn - pn % (TPB * U);
    for (; e0 < full; e0 += TPB * U) {
      uint32_t k[U];
      T v[U], g[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        k[u] = ld_entry<NT>(kp + e0 + u * TPB);
        v[u] = ld_entry<NT>(vp + e0 + u * TPB);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) g[u] = srcb[k[u] >> rb];
#pragma unroll
      for (int u = 0; u < U; ++u) atomicAdd(&s_row[k[u] & rmask], (double)(v[u] * g[u]));
    }
    if (e0 < pn) {
      // last partial batch: positions past the block read its first entry
      // (a valid index) and add nothing
      uint32_t k[U];
      T v[U], g[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * TPB;
        const int ec = e < pn ? e : 0;
        k[u] = ld_entry<NT>(kp + ec);
        v[u] = ld_entry<NT>(vp + ec);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) g[u] = srcb[k[u] >> rb];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e0 + u * TPB < pn) atomicAdd(&s_row[k[u] & rmask], (double)(v[u] * g[u]));
    }
  } else {
    for (; e0 < pn; e0 += TPB * U) {
      uint32_t k[U];
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * TPB;
        if (e < pn) {
          k[u] = ld_entry<NT>(kp + e);
          v[u] = ld_entry<NT>(vp + e);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * TPB;
        if (e < pn) atomicAdd(&s_row[k[u] & rmask], (double)(v[u] * srcb[k[u] >> rb]));
      }
    }
  }
}

// Partial row sums of one column slice of a sorted row group (written to the
// slice-partial buffer for the step kernel of the same step to add up).
// DUAL: a group of K's rows gathering xbar (xT, cx1 and cx2 one after the
// other at an eval step) into spartD; otherwise a group of K^T's rows
// gathering y (yT, cy1, cy2) into spartP.  The group's row sums sit in
// dynamic LDS (FP64 words for the rows of the largest group of the schedule).
template <class T, bool DUAL, int TPB, bool BATCHED>
__global__ __launch_bounds__(TPB) void sorted_group_step(IterArgs<T> A, int step) {
  extern __shared__ __align__(16) unsigned char group_lds[];
  double* s_row = reinterpret_cast<double*>(group_lds);
  const Blk b = (DUAL ? A.schedDS : A.schedPS)[blockIdx.x];
  if (blk_kind(b) == BK_PAD) return;
  const InstState& S = A.st[b.inst];
  const int64_t g = *A.gbase + step;
  const int mode = step_mode(S, g);
  if (mode == M_SKIP || (!DUAL && mode == M_RESID)) return;
  const int nrows = b.r1 - b.r0;
  const int sl = blk_slice(b);
  const int nv = mode == M_EVAL ? 3 : 1;
  const uint32_t* w = reinterpret_cast<const uint32_t*>(DUAL ? A.K_ci : A.KT_ci);
  const T* val = DUAL ? A.K_v : A.KT_v;
  T* spart = DUAL ? A.spartD : A.spartP;
  const int64_t space = DUAL ? A.MS : A.NS;
  for (int a = 0; a < nv; ++a) {
    const T* src = DUAL ? (mode != M_EVAL ? A.xbar : a == 0 ? A.xT : a == 1 ? A.cx1 : A.cx2)
                        : (mode != M_EVAL ? A.y : a == 0 ? A.yT : a == 1 ? A.cy1 : A.cy2);
    for (int r = threadIdx.x; r < nrows; r += TPB) s_row[r] = 0.0;
    lds_barrier();
    if (blk_nt(b)) group_rows_sum<T, TPB, 4, BATCHED, true>(b, w, val, src, s_row);
    else group_rows_sum<T, TPB, 4, BATCHED, false>(b, w, val, src, s_row);
    lds_barrier();
    for (int r = threadIdx.x; r < nrows; r += TPB)
      spart[(int64_t)(a * kSlices + sl) * space + b.r0 + r] = (T)s_row[r];
    lds_barrier();
  }
}

// ---------------------------------------------------------------------------
// controller: runs once per LP per check / eval / residual step
// ---------------------------------------------------------------------------

__device__ void controller(InstState& S, const double* sp, const double* sd, int mode, int64_t g,
                           int* status_out, int inst) {
  if (mode == M_CHECK) {
    S.acc[A_DX2] = sp[0];
    S.acc[A_AX2] = sp[1];
    S.acc[A_POBJ] = sp[2];
    S.acc[A_CD1] = sp[3];
    S.acc[A_CD2] = sp[4];
    S.acc[A_DY2] = sd[0];
    S.acc[A_AY2] = sd[1];
    S.acc[A_DOBJQ] = sd[2];
    S.acc[A_QY1] = sd[3];
    S.acc[A_QY2] = sd[4];
    S.acc[A_ACTX] = sp[5];
    S.acc[A_ACTY] = sd[5];
    S.phase = PH_EVAL;
    return;
  }
  if (mode == M_RESID) {
    const double v = sp[0] / S.tau + sd[0] / S.sigma + 2.0 * sd[1];
    S.r0 = sqrt(fmax(v, 0.0));
    S.phase = PH_NORMAL;
    return;
  }
  // eval step: the check candidate is T(z^{n,k}) from the previous step
  const int64_t t = g - S.tbase;          // evaluations of T so far
  const int64_t k = (g - 1) - S.kbase;    // inner counter of the check step
  S.tbase += 1;
  S.checks += 1;
  const double vres = S.acc[A_DX2] / S.tau + S.acc[A_DY2] / S.sigma + 2.0 * sd[1];
  const double res = sqrt(fmax(vres, 0.0));
  const double rel_p = sqrt(sd[0]) / (1.0 + S.qnorm);
  const double rel_d = sqrt(sp[0]) / (1.0 + S.cnorm);
  const double pobj = S.acc[A_POBJ];
  const double dobj = S.acc[A_DOBJQ] + sp[1];
  const double gap = fabs(pobj - dobj) / (1.0 + fabs(pobj) + fabs(dobj));
  const double kkt = fmax(rel_p, fmax(rel_d, gap));
  S.kkt = kkt;
  S.rel_p = rel_p;
  S.rel_d = rel_d;
  S.rel_gap = gap;
  S.pobj = pobj;
  S.dobj = dobj;
  S.resid = res;
  S.iters = t;
  S.act_changes = (int64_t)(S.acc[A_ACTX] + S.acc[A_ACTY]);
  if (S.act_changes > 0) S.ident_iters = t;
  int st = ST_RUNNING;
  // a NaN or Inf in any reduction (fmax would pass over a NaN part)
  if (!isfinite(kkt) || !isfinite(vres) || !isfinite(rel_p) || !isfinite(rel_d) || !isfinite(gap)) {
    st = ST_NUMERICAL;
  } else if (kkt <= S.tol) {
    st = ST_OPTIMAL;
  } else {
    const double m1 = S.acc[A_QY1] - sp[2];
    const double m2 = S.acc[A_QY2] - sp[4];
    if (m1 > 0.0 && sqrt(sp[3]) <= S.eps_inf * m1) {
      st = ST_PRIMAL_INFEAS;
      S.ray = 1;
    } else if (m2 > 0.0 && sqrt(sp[5]) <= S.eps_inf * m2) {
      st = ST_PRIMAL_INFEAS;
      S.ray = 2;
    } else {
      const double c1 = S.acc[A_CD1], c2 = S.acc[A_CD2];
      if (c1 < 0.0 && sqrt(sd[2]) + sqrt(sd[3]) <= S.eps_inf * fabs(c1)) {
        st = ST_DUAL_INFEAS;
        S.ray = 1;
      } else if (c2 < 0.0 && sqrt(sd[4]) + sqrt(sd[5]) <= S.eps_inf * fabs(c2)) {
        st = ST_DUAL_INFEAS;
        S.ray = 2;
      }
    }
    if (st == ST_RUNNING && t >= S.max_iter) st = ST_ITER_LIMIT;
    if (!(kkt >= 0.9 * S.best_kkt)) {
      S.best_kkt = kkt;
      S.best_check = S.checks;
    }
    if (st == ST_RUNNING && S.stall_checks > 0 && S.checks - S.best_check >= S.stall_checks) st = ST_ITER_LIMIT;
  }
  if (st != ST_RUNNING) {
    S.status = st;
    S.phase = PH_NORMAL;
    status_out[inst] = st;
    return;
  }
  bool restart = false;
  const bool artificial = S.artificial > 0.0 && (double)k >= S.artificial * (double)t;
  if (S.restart_mode == 0 && S.avg)
    restart = (S.nrest == 0) || (kkt <= S.avg_b1 * S.kkt_anchor) ||
              (kkt <= S.avg_b2 * S.kkt_anchor && kkt > S.kkt_prev) || artificial;
  else if (S.restart_mode == 0)
    restart = (S.nrest == 0) || (res <= S.beta * S.r0) || artificial;
  else if (S.restart_mode == 1)
    restart = k >= S.fixed_len;
  S.kkt_prev = kkt;
  if (restart) {
    S.kkt_anchor = kkt;
    S.kkt_prev = INFINITY;
  }
  if (restart) {
    const double dX = sqrt(S.acc[A_AX2]), dY = sqrt(S.acc[A_AY2]);
    if (S.primal_weight && dX > 1e-10 && dY > 1e-10 && isfinite(dX) && isfinite(dY))
      S.omega = exp(0.5 * log(dY / dX) + 0.5 * log(S.omega));
    S.tau = S.eta / S.omega;
    S.sigma = S.eta * S.omega;
    S.nrest += 1;
    S.phase = PH_RESID;
    S.kbase = g + 1;
    S.next_check = g + 1 + S.C;
  } else {
    S.phase = PH_NORMAL;
    S.kbase += 1;
    S.next_check = g + S.C;
  }
}

// ---------------------------------------------------------------------------
// dual step (rows of K = constraints) + per-LP controller
// ---------------------------------------------------------------------------

// One constraint's part of a dual step (rows of K): i is its space
// position, s0 its row sum (K xbar, or K xT at an eval step, where a1 and a2
// are K cx1 and K cx2; at a residual step the caller passes T(z) as yo and
// y0i and the saved K x+ as kxpi).  Adds the check / eval / residual terms
// of the row to ps.
template <class T>
__device__ __forceinline__ void dual_row(const IterArgs<T>& A, const InstState& S, int mode, int64_t g,
                                         int64_t i, T qi, T yo, T y0i, T kxpi, T s0, T a1, T a2,
                                         double (&ps)[kNS]) {
  const bool resid = (mode == M_RESID);
  const bool ineq = (i - S.row0) >= S.m_eq;
  if (mode == M_EVAL) {
    A.kxp[i] = s0;
    const double dr = A.Dr[i];
    double r = ((double)s0 - (double)qi) / dr;
    if (ineq) r = fmin(r, 0.0);
    ps[0] += r * r;
    ps[1] += (double)A.dy[i] * ((double)s0 - (double)A.kxbar[i]);
#pragma unroll
    for (int a = 1; a <= 2; ++a) {
      const double av = (double)(a == 1 ? a1 : a2) / dr;
      if (ineq) {
        const double mv = fmin(av, 0.0);
        ps[2 * a + 1] += mv * mv;
      } else {
        ps[2 * a] += av * av;
      }
    }
    return;
  }
  const T sigma = (T)S.sigma;
  T yp = yo + sigma * (qi - s0);
  if (ineq) yp = fmax(yp, (T)0);
  const T yb = (T)2 * yp - yo;
  const int64_t k = g - S.kbase;
  T yc = yp;  // check candidate
  if (S.avg) {
    const T ysum = (k == 0 ? yo : A.ys[i]) + yp;
    A.ys[i] = ysum;
    A.y[i] = yp;
    if (mode == M_CHECK) yc = ysum / (T)(k + 2);
  } else {
    const double w = (double)(k + 1) / (double)(k + 2);
    const T yh = S.reflect ? yb : yp;
    A.y[i] = (T)w * yh + (T)(1.0 - w) * y0i;
  }
  if (resid) {
    A.y0[i] = yo;
    const double d = (double)yo - (double)yp;
    ps[0] += d * d;
    ps[1] += d * (0.5 * ((double)kxpi - (double)s0));
  } else if (mode == M_CHECK) {
    A.yT[i] = yc;
    const T dyv = yo - yp;
    A.dy[i] = dyv;
    A.kxbar[i] = s0;
    T e1 = yp - yo, e2 = yo - y0i;
    if (ineq) {
      e1 = fmax(e1, (T)0);
      e2 = fmax(e2, (T)0);
    }
    A.cy1[i] = e1;
    A.cy2[i] = e2;
    const double ad = (double)yc - (double)y0i;
    ps[0] += (double)dyv * (double)dyv;
    ps[1] += ad * ad;
    ps[2] += (double)qi * (double)yc;
    ps[3] += (double)qi * (double)e1;
    ps[4] += (double)qi * (double)e2;
    const uint8_t act = (ineq && yp == (T)0) ? 1 : 0;
    const uint8_t was = A.acty[i];
    A.acty[i] = act;
    ps[5] += (was != 255 && was != act) ? 1.0 : 0.0;
  }
}

// A dual step over a column-sorted block of K rows (up to kSortRowsPlain
// constraints): products with xbar (xT, cx1, cx2 at an eval step) added into
// LDS row sums, then each thread takes the epilogue of every kThreads-th row.
template <class T>
__device__ void dual_sorted(const IterArgs<T>& A, const Blk& b, int step, double* s_row, double (*s_red)[kNS],
                            double* s_out) {
  const InstState& S = A.st[b.inst];
  const int64_t g = *A.gbase + step;
  const int mode = step_mode(S, g);
  if (mode == M_SKIP) return;
  const bool resid = (mode == M_RESID);
  const int nrows = b.r1 - b.r0;
  if (mode == M_EVAL) {
    sorted_pass_to<T>(b, A.K_ci, A.K_v, A.cx1, s_row, A.kx1);
    sorted_pass_to<T>(b, A.K_ci, A.K_v, A.cx2, s_row, A.kx2);
    sorted_pass<T>(b, A.K_ci, A.K_v, A.xT, s_row);
  } else {
    sorted_pass<T>(b, A.K_ci, A.K_v, A.xbar, s_row);
  }
  double ps[kNS];
#pragma unroll
  for (int s = 0; s < kNS; ++s) ps[s] = 0.0;
  for (int r = threadIdx.x; r < nrows; r += kThreads) {
    const int64_t i = (int64_t)b.r0 + r;
    const T qi = A.q[i];
    T yo, y0i, kxpi = 0, a1 = 0, a2 = 0;
    if (resid) {
      yo = A.yT[i];
      y0i = yo;
      kxpi = A.kxp[i];
    } else {
      yo = A.y[i];
      y0i = A.y0[i];
    }
    if (mode == M_EVAL) {
      a1 = A.kx1[i];
      a2 = A.kx2[i];
    }
    dual_row<T>(A, S, mode, g, i, qi, yo, y0i, kxpi, (T)s_row[r], a1, a2, ps);
  }
  if (mode != M_NORMAL) {
    block_sum_ns(ps, s_red, s_out);
    if (threadIdx.x < kNS) A.partD[(int64_t)b.gid * kNS + threadIdx.x] = s_out[threadIdx.x];
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void dual_step(IterArgs<T> A, int step) {
  __shared__ StepSmem<T> sm;
  __shared__ double s_red[kThreads / 64][kNS];
  __shared__ double s_out[kNS];
  T* s_prod = sm.p.prod;
  T (*s_rsum)[kMaxRows] = sm.p.rsum;
  int* s_rp = sm.p.rp;

  const Blk b = A.schedD[blockIdx.x];
  if (blk_kind(b) == BK_PAD) return;
  if (blk_kind(b) == BK_SORTED) {
    dual_sorted<T>(A, b, step, sm.rows, s_red, s_out);
    return;
  }
  const int nrows = b.r1 - b.r0;
  const int t = threadIdx.x;
  const bool own = t < nrows;
  const int64_t i = (int64_t)b.r0 + (own ? t : 0);
  // entries and epilogue operands are loaded before the LP state is read
  TileRegs<T, kPlainNB> R;
  load_tile<T, kPlainNB>(b, A.K_rp + b.r0, A.K_ci, A.K_v, R);
  spec_products<T, kPlainNB>(b, A.xbar, R);
  T qi = 0, yo = 0, y0i = 0, kxpi = 0;
  if (own) {
    qi = A.q[i];
    yo = A.y[i];
    y0i = A.y0[i];
  }
  const InstState& S = A.st[b.inst];
  const int64_t g = *A.gbase + step;
  const int mode = step_mode(S, g);
  if (mode == M_SKIP) return;
  const bool resid = (mode == M_RESID);
  if (resid && own) {
    yo = A.yT[i];
    y0i = yo;
    kxpi = A.kxp[i];
  }
  if (blk_part(b)) {
    if (mode == M_EVAL) gather_slices<T, 3>(b, A.spartD, A.MS, s_rsum);
    else gather_slices<T, 1>(b, A.spartD, A.MS, s_rsum);
  } else if (mode == M_EVAL) {
    block_spmv_regs<T, 3, kPlainNB>(b, A.K_ci, A.K_v, R, A.xT, A.cx1, A.cx2, s_prod, s_rsum, s_rp, s_red);
  } else {
    block_spmv1<T, kPlainNB>(b, A.K_ci, A.K_v, R, A.xbar, s_prod, s_rsum[0], s_rp, s_red, (T)1, true);
  }

  double ps[kNS];
#pragma unroll
  for (int s = 0; s < kNS; ++s) ps[s] = 0.0;
  if (own) {
    const bool eval = (mode == M_EVAL);
    dual_row<T>(A, S, mode, g, i, qi, yo, y0i, kxpi, s_rsum[0][t], eval ? s_rsum[1][t] : (T)0,
                eval ? s_rsum[2][t] : (T)0, ps);
  }
  if (mode == M_NORMAL) return;

  block_sum_ns(ps, s_red, s_out);
  if (t < kNS) A.partD[(int64_t)b.gid * kNS + t] = s_out[t];
}

// Per-LP control after a step (one workgroup per LP slot): at check, eval
// and residual steps, the fixed-order sums of the step kernels' per-workgroup
// partial sums, then the controller.  A kernel of its own, so that the
// partial sums of every XCD are visible without device-scope fences inside
// the step kernels (each of which would write back the XCD's L2).
__global__ __launch_bounds__(kThreads) void control_kernel(InstState* st, const int* ids, const double* partP,
                                                           const double* partD, const int64_t* gbase,
                                                           int step, int* status_out) {
  __shared__ double s_red[kThreads / 64][kNS];
  __shared__ double s_sum[2][kNS];
  const int inst = ids[blockIdx.x];  // the LPs in the current schedules
  InstState& S = st[inst];
  const int64_t g = *gbase + step;
  const int mode = step_mode(S, g);
  if (mode == M_SKIP || mode == M_NORMAL) return;
  sum_partials(partP + (int64_t)S.pb0 * kNS, S.pb1 - S.pb0, s_red, s_sum[0]);
  sum_partials(partD + (int64_t)S.db0 * kNS, S.db1 - S.db0, s_red, s_sum[1]);
  if (threadIdx.x == 0) controller(S, s_sum[0], s_sum[1], mode, g, status_out, inst);
}

__global__ void tick_kernel(int64_t* gbase, int64_t add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *gbase += add;
}

// ---------------------------------------------------------------------------
// preprocessing: Ruiz / Pock-Chambolle factors and value scaling
// ---------------------------------------------------------------------------

// f[r] = sqrt(max_j |v_rj|) (op 0) or sqrt(sum_j |v_rj|) (op 1), 1 if zero;
// D[r] /= f[r].
__global__ __launch_bounds__(kThreads) void row_factor_kernel(const Blk* sched, const int32_t* rp,
                                                              const double* val, int op, double expo,
                                                              double* f, double* D) {
  __shared__ double s_red[kThreads / 64][kNS];
  const Blk b = sched[blockIdx.x];
  const int tid = threadIdx.x;
  const int nrows = b.r1 - b.r0;
  if (blk_kind(b) == BK_LONG) {
    const int p0 = rp[b.r0], p1 = rp[b.r0 + 1];
    double a = 0.0;
    for (int e = p0 + tid; e < p1; e += kThreads) {
      double v = fabs(val[e]);
      if (op == 1 && expo != 1.0) v = pow(v, expo);
      a = op == 0 ? fmax(a, v) : a + v;
    }
    // block reduce (max or sum) through LDS in fixed order
    __syncthreads();
    if (op == 0) {
      for (int off = 32; off > 0; off >>= 1) a = fmax(a, __shfl_xor(a, off, 64));
    } else {
      a = wave_sum(a);
    }
    if ((tid & 63) == 0) s_red[tid >> 6][0] = a;
    __syncthreads();
    if (tid == 0) {
      double r = s_red[0][0];
      for (int w = 1; w < kThreads / 64; ++w) r = op == 0 ? fmax(r, s_red[w][0]) : r + s_red[w][0];
      double fr = sqrt(r);
      if (!(fr > 0.0)) fr = 1.0;
      f[b.r0] = fr;
      D[b.r0] /= fr;
    }
    return;
  }
  const int G = group_size(nrows);
  const int lane = tid & (G - 1);
  for (int base = 0; base < nrows; base += kThreads / G) {
    const int r = base + tid / G;
    double a = 0.0;
    if (r < nrows) {
      const int p1 = rp[b.r0 + r + 1];
      for (int e = rp[b.r0 + r] + lane; e < p1; e += G) {
        double v = fabs(val[e]);
        if (op == 1 && expo != 1.0) v = pow(v, expo);
        a = op == 0 ? fmax(a, v) : a + v;
      }
    }
    for (int off = G >> 1; off > 0; off >>= 1) {
      const double o = __shfl_xor(a, off, 64);
      a = op == 0 ? fmax(a, o) : a + o;
    }
    if (lane == 0 && r < nrows) {
      double fr = sqrt(a);
      if (!(fr > 0.0)) fr = 1.0;
      f[b.r0 + r] = fr;
      D[b.r0 + r] /= fr;
    }
  }
}

// v_e <- v_e / fm[m-index] / fn[n-index]; for K the row is the m-index,
// for K^T the row is the n-index.  Same operation order for both, so K~ and
// (K~)^T hold bit-identical values.
__global__ __launch_bounds__(kThreads) void scale_values_kernel(const Blk* sched, const int32_t* rp,
                                                                const int32_t* ci, double* val,
                                                                const double* fm, const double* fn,
                                                                int transposed) {
  const Blk b = sched[blockIdx.x];
  const int nrows = b.r1 - b.r0;
  const int tid = threadIdx.x;
  const int G = (blk_kind(b) == BK_LONG) ? kThreads : group_size(nrows);
  const int lane = tid & (G - 1);
  for (int base = 0; base < nrows; base += kThreads / G) {
    const int r = base + tid / G;
    if (r >= nrows) continue;
    const int row = b.r0 + r;
    const int p1 = rp[row + 1];
    for (int e = rp[row] + lane; e < p1; e += G) {
      const int c = ci[e];
      const double a = transposed ? fm[c] : fm[row];
      const double d = transposed ? fn[row] : fn[c];
      val[e] = val[e] / a / d;
    }
  }
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <class T>
__global__ void cast_kernel(const double* src, T* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

// per-LP unscaled norms ||q|| and ||c|| (one block per LP, fixed order)
// per-LP norms: ||q||, ||c|| (unscaled) and ||D_r q||, ||D_c c|| (scaled),
// one block per LP, fixed order; the scaled pair goes to out[2 * block + {0,1}]
__global__ __launch_bounds__(kThreads) void inst_norms_kernel(InstState* st, const int* ids,
                                                              const double* q, const double* c,
                                                              const double* Dr, const double* Dc,
                                                              double* out) {
  __shared__ double s_red[kThreads / 64][kNS];
  __shared__ double s_out[kNS];
  InstState& S = st[ids[blockIdx.x]];
  double v[kNS];
  for (int s = 0; s < kNS; ++s) v[s] = 0.0;
  for (int64_t i = threadIdx.x; i < S.m; i += kThreads) {
    const double a = q[S.row0 + i];
    const double b = Dr[S.row0 + i] * a;
    v[0] += a * a;
    v[2] += b * b;
  }
  for (int64_t j = threadIdx.x; j < S.n; j += kThreads) {
    const double a = c[S.col0 + j];
    const double b = Dc[S.col0 + j] * a;
    v[1] += a * a;
    v[3] += b * b;
  }
  block_sum_ns(v, s_red, s_out);
  if (threadIdx.x == 0) {
    S.qnorm = sqrt(s_out[0]);
    S.cnorm = sqrt(s_out[1]);
    out[2 * blockIdx.x] = sqrt(s_out[2]);
    out[2 * blockIdx.x + 1] = sqrt(s_out[3]);
  }
}

// scaled vectors over the rows of the given schedules
template <class T>
__global__ __launch_bounds__(kThreads) void scale_primal_kernel(const Blk* schedP, const double* Dc,
                                                                const double* c, const double* l,
                                                                const double* u, T* cs, T* ls, T* us) {
  const Blk b = schedP[blockIdx.x];
  if ((int)threadIdx.x < b.r1 - b.r0) {
    const int64_t j = (int64_t)b.r0 + threadIdx.x;
    cs[j] = (T)(Dc[j] * c[j]);
    ls[j] = (T)(l[j] / Dc[j]);
    us[j] = (T)(u[j] / Dc[j]);
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void scale_dual_kernel(const Blk* schedD, const double* Dr,
                                                              const double* q, T* qs) {
  const Blk b = schedD[blockIdx.x];
  if ((int)threadIdx.x < b.r1 - b.r0) {
    const int64_t i = (int64_t)b.r0 + threadIdx.x;
    qs[i] = (T)(Dr[i] * q[i]);
  }
}

// write the host-prepared states of new LPs and clear their status words
__global__ void write_states_kernel(InstState* st, int* status_out, int* cnt, const int* ids,
                                    const InstState* src, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    st[ids[i]] = src[i];
    status_out[ids[i]] = src[i].status;
    cnt[ids[i]] = 0;
  }
}

// schedule ranges of live LPs after a schedule rebuild
__global__ void set_ranges_kernel(InstState* st, const int* ids, const int4* ranges, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    InstState& S = st[ids[i]];
    const int4 r = ranges[i];
    S.pb0 = r.x;
    S.pb1 = r.y;
    S.db0 = r.z;
    S.db1 = r.w;
  }
}

// ---------------------------------------------------------------------------
// power iteration on K~^T K~ (per LP)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// w = SplitMix64 uniform [-1, 1) start vector over each LP's variables, and
// the block partial of sum w^2
__global__ __launch_bounds__(kThreads) void pw_start_kernel(const Blk* schedP, const InstState* st,
                                                            uint64_t seed, double* w, double* partP) {
  __shared__ double s_red[kThreads / 64][kNS];
  __shared__ double s_out[kNS];
  const Blk b = schedP[blockIdx.x];
  const InstState& S = st[b.inst];
  double v[kNS];
  for (int s = 0; s < kNS; ++s) v[s] = 0.0;
  const int nrows = b.r1 - b.r0;
  if ((int)threadIdx.x < nrows) {
    const int64_t j = (int64_t)b.r0 + threadIdx.x;
    const uint64_t z = splitmix64_at(seed, (uint64_t)(j - S.col0));
    const double u = (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    w[j] = u;
    v[0] = u * u;
  }
  block_sum_ns(v, s_red, s_out);
  if (threadIdx.x < kNS) partP[(int64_t)blockIdx.x * kNS + threadIdx.x] = s_out[threadIdx.x];
}

// u = pw_scale * K~ w over the rows of K (dual schedule)
__global__ __launch_bounds__(kThreads) void pw_forward_kernel(const Blk* schedD, const InstState* st,
                                                              const int32_t* rp, const int32_t* ci,
                                                              const double* val, const double* w,
                                                              double* u) {
  __shared__ double s_prod[Tile<double>::NB];
  __shared__ double s_rsum[3][kMaxRows];
  __shared__ int s_rp[kMaxRows + 1];
  __shared__ double s_red[kThreads / 64][kNS];
  const Blk b = schedD[blockIdx.x];
  const InstState& S = st[b.inst];
  if (S.pw_done) return;
  block_spmv<double, 1>(b, rp + b.r0, ci, val, w, w, w, s_prod, s_rsum, s_rp, s_red, S.pw_scale);
  const int nrows = b.r1 - b.r0;
  if ((int)threadIdx.x < nrows) u[(int64_t)b.r0 + threadIdx.x] = s_rsum[0][threadIdx.x];
}

// w = K~^T u over the rows of K^T (primal schedule), with the partial sum w^2
__global__ __launch_bounds__(kThreads) void pw_backward_kernel(const Blk* schedP, const InstState* st,
                                                               const int32_t* rp, const int32_t* ci,
                                                               const double* val, const double* u,
                                                               double* w, double* partP) {
  __shared__ double s_prod[Tile<double>::NB];
  __shared__ double s_rsum[3][kMaxRows];
  __shared__ int s_rp[kMaxRows + 1];
  __shared__ double s_red[kThreads / 64][kNS];
  __shared__ double s_out[kNS];
  const Blk b = schedP[blockIdx.x];
  const InstState& S = st[b.inst];
  if (S.pw_done) return;
  block_spmv<double, 1>(b, rp + b.r0, ci, val, u, u, u, s_prod, s_rsum, s_rp, s_red);
  double v[kNS];
  for (int s = 0; s < kNS; ++s) v[s] = 0.0;
  const int nrows = b.r1 - b.r0;
  if ((int)threadIdx.x < nrows) {
    const double a = s_rsum[0][threadIdx.x];
    w[(int64_t)b.r0 + threadIdx.x] = a;
    v[0] = a * a;
  }
  block_sum_ns(v, s_red, s_out);
  if (threadIdx.x < kNS) partP[(int64_t)blockIdx.x * kNS + threadIdx.x] = s_out[threadIdx.x];
}

// one block per LP: ||w|| from the partials, estimate sqrt(||w||), stop rule
__global__ __launch_bounds__(kThreads) void pw_control_kernel(InstState* st, const int* ids,
                                                              const int4* ranges, const double* partP,
                                                              int start, int min_iters, int max_iters,
                                                              double rtol, int* active) {
  __shared__ double s_red[kThreads / 64][kNS];
  __shared__ double s_sum[kNS];
  InstState& S = st[ids[blockIdx.x]];
  if (S.pw_done) return;
  const int4 rg = ranges[blockIdx.x];
  sum_partials(partP + (int64_t)rg.x * kNS, rg.y - rg.x, s_red, s_sum);
  if (threadIdx.x != 0) return;
  const double nw = sqrt(s_sum[0]);
  if (start) {
    S.pw_scale = nw > 0.0 ? 1.0 / nw : 0.0;
    S.pw_iter = 0;
    S.pw_prev = -1.0;
    S.sigma_hat = 0.0;
    if (!(nw > 0.0)) S.pw_done = 1;
    else atomicAdd(active, 1);
    return;
  }
  S.pw_iter += 1;
  if (!(nw > 0.0)) {
    S.sigma_hat = 0.0;
    S.pw_done = 1;
    return;
  }
  const double s = sqrt(nw);
  S.sigma_hat = s;
  S.pw_scale = 1.0 / nw;
  if ((S.pw_prev >= 0.0 && S.pw_iter >= min_iters && fabs(s - S.pw_prev) <= rtol * s) ||
      S.pw_iter >= max_iters) {
    S.pw_done = 1;
    return;
  }
  S.pw_prev = s;
  atomicAdd(active, 1);
}

// ---------------------------------------------------------------------------
// iterate initialisation, results, validation
// ---------------------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(kThreads) void init_primal_kernel(const Blk* schedP, const T* l, const T* u,
                                                               T* x, T* x0, uint8_t* actx) {
  const Blk b = schedP[blockIdx.x];
  const int nrows = b.r1 - b.r0;
  if ((int)threadIdx.x < nrows) {
    const int64_t j = (int64_t)b.r0 + threadIdx.x;
    const T v = clampT<T>((T)0, l[j], u[j]);
    x[j] = v;
    x0[j] = v;
    actx[j] = 255;
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void init_dual_kernel(const Blk* schedD, T* y, T* y0, uint8_t* acty) {
  const Blk b = schedD[blockIdx.x];
  const int nrows = b.r1 - b.r0;
  if ((int)threadIdx.x < nrows) {
    const int64_t i = (int64_t)b.r0 + threadIdx.x;
    y[i] = (T)0;
    y0[i] = (T)0;
    acty[i] = 255;
  }
}

template <class T>
__global__ void unscale_kernel(const T* v, const double* D, int64_t off, int64_t n, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = D[off + i] * (double)v[off + i];
}

template <class T>
__global__ void load_point_kernel(const double* src, T* v, T* v0, int64_t off, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    v[off + i] = (T)src[i];
    v0[off + i] = (T)src[i];
  }
}

template <class T>
__global__ void copy_state_kernel(const T* src, double* dst, int64_t off, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[off + i];
}

__global__ void set_limit_status_kernel(InstState* st, int* status_out, int ninst, int code) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst && st[i].status == ST_RUNNING) {
    st[i].status = code;
    status_out[i] = code;
  }
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------

template __global__ void primal_step<double>(IterArgs<double>, int);
template __global__ void primal_step<float>(IterArgs<float>, int);
template __global__ void dual_step<double>(IterArgs<double>, int);
template __global__ void dual_step<float>(IterArgs<float>, int);
template __global__ void primal_slice_step<double, 256>(IterArgs<double>, int);
template __global__ void primal_slice_step<double, 512>(IterArgs<double>, int);
template __global__ void primal_slice_step<double, 1024>(IterArgs<double>, int);
template __global__ void primal_slice_step<float, 256>(IterArgs<float>, int);
template __global__ void primal_slice_step<float, 512>(IterArgs<float>, int);
template __global__ void primal_slice_step<float, 1024>(IterArgs<float>, int);
template __global__ void dual_slice_step<double, 256>(IterArgs<double>, int);
template __global__ void dual_slice_step<double, 512>(IterArgs<double>, int);
template __global__ void dual_slice_step<double, 1024>(IterArgs<double>, int);
template __global__ void dual_slice_step<float, 256>(IterArgs<float>, int);
template __global__ void dual_slice_step<float, 512>(IterArgs<float>, int);
template __global__ void dual_slice_step<float, 1024>(IterArgs<float>, int);
template __global__ void cast_kernel<float>(const double*, float*, int64_t);
template __global__ void scale_primal_kernel<double>(const Blk*, const double*, const double*,
                                                     const double*, const double*, double*, double*,
                                                     double*);
template __global__ void scale_primal_kernel<float>(const Blk*, const double*, const double*,
                                                    const double*, const double*, float*, float*, float*);
template __global__ void scale_dual_kernel<double>(const Blk*, const double*, const double*, double*);
template __global__ void scale_dual_kernel<float>(const Blk*, const double*, const double*, float*);
template __global__ void init_primal_kernel<double>(const Blk*, const double*, const double*, double*,
                                                    double*, uint8_t*);
template __global__ void init_primal_kernel<float>(const Blk*, const float*, const float*, float*, float*,
                                                   uint8_t*);
template __global__ void init_dual_kernel<double>(const Blk*, double*, double*, uint8_t*);
template __global__ void init_dual_kernel<float>(const Blk*, float*, float*, uint8_t*);
template __global__ void unscale_kernel<double>(const double*, const double*, int64_t, int64_t, double*);
template __global__ void unscale_kernel<float>(const float*, const double*, int64_t, int64_t, double*);
template __global__ void load_point_kernel<double>(const double*, double*, double*, int64_t, int64_t);
template __global__ void load_point_kernel<float>(const double*, float*, float*, int64_t, int64_t);
template __global__ void copy_state_kernel<double>(const double*, double*, int64_t, int64_t);
template __global__ void copy_state_kernel<float>(const float*, double*, int64_t, int64_t);

}  // namespace halp

// Kernels of lp_create (and of an engine that re-blocks its last LPs) that
// never run in a solver step: validation of device-resident input, the
// explicit transpose K^T, column slicing, the sort keys of column-sorted
// blocks and groups and the gathers that apply a sorted permutation.
// Included by engine.hip after kernels.hip (shared types from halp_types.h).

namespace halp {

// dst = src narrowed to int32 (row pointers given as int64); *bad = 1 when an
// entry is negative or above 2^31 - 1 (that entry is written as 0)
__global__ void narrow_row_ptr_kernel(const int64_t* src, int32_t* dst, int64_t n, int* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t v = src[i];
  if (v < 0 || v > (int64_t)INT32_MAX) {
    atomicOr(bad, 1);
    dst[i] = 0;
  } else {
    dst[i] = (int32_t)v;
  }
}

// flags: 1 bad row pointers, 2 column out of range or not increasing, 4 non-finite value
__global__ void validate_rowptr_kernel(const int32_t* rp, int64_t m, int64_t nnz, int* flags) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0 && (rp[0] != 0 || rp[m] != nnz)) atomicOr(flags, 1);
  if (r >= m) return;
  if (rp[r + 1] < rp[r] || rp[r] < 0 || rp[r + 1] > nnz) atomicOr(flags, 1);
}

// One thread per entry: column in range and strictly above the previous
// entry's unless the entry starts its row (found by a binary search of the
// row pointers: the last row whose start is at or before it), finite value.
// The search stays within rp[0..m] whatever the row pointers hold; invalid
// row pointers are flagged by validate_rowptr_kernel.
__global__ void validate_entries_kernel(const int32_t* rp, const int32_t* ci, const double* val, int64_t m,
                                        int64_t n, int64_t nnz, int* flags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int64_t c = ci[e];
  if (c < 0 || c >= n) atomicOr(flags, 2);
  if (!isfinite(val[e])) atomicOr(flags, 4);
  if (e == 0) return;
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if ((int64_t)rp[mid] <= e) lo = mid; else hi = mid - 1;
  }
  if ((int64_t)rp[lo] != e && c <= (int64_t)ci[e - 1]) atomicOr(flags, 2);
}

// flags: 8 non-finite c or rhs, 16 bad bounds
__global__ void validate_vectors_kernel(const double* c, const double* rhs, const double* lb,
                                        const double* ub, int64_t m, int64_t n, int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m && !isfinite(rhs[i])) atomicOr(flags, 8);
  if (i < n) {
    if (!isfinite(c[i])) atomicOr(flags, 8);
    const double a = lb[i], b = ub[i];
    if (isnan(a) || isnan(b) || a > b || a == INFINITY || b == -INFINITY) atomicOr(flags, 16);
  }
}

__global__ void shift_copy_kernel(int32_t* dst, const int32_t* src, int64_t n, int64_t add) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (int32_t)(src[i] + add);
}

__global__ void iota_kernel(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// rowid[e - z0] = row, for every entry of the rows in the dual schedule
__global__ __launch_bounds__(kThreads) void row_ids_kernel(const Blk* sched, const int32_t* rp,
                                                           int64_t z0, int32_t* rowid) {
  const Blk b = sched[blockIdx.x];
  const int nrows = b.r1 - b.r0;
  const int G = (blk_kind(b) == BK_LONG) ? kThreads : group_size(nrows);
  const int lane = threadIdx.x & (G - 1);
  for (int base = 0; base < nrows; base += kThreads / G) {
    const int r = base + threadIdx.x / G;
    if (r >= nrows) continue;
    const int row = b.r0 + r;
    const int p1 = rp[row + 1];
    for (int e = rp[row] + lane; e < p1; e += G) rowid[e - z0] = row;
  }
}

// cnt[(r - r0) * kSlices + s] = entries of row r whose column lies in slice s
// of the gathered range [c0, c0 + len)
__global__ void slice_count_kernel(const int32_t* rp, const int32_t* ci, int64_t r0, int64_t nrows,
                                   int64_t c0, int64_t len, int nsl, int32_t* cnt) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int32_t c[kSlices];
  for (int q = 0; q < kSlices; ++q) c[q] = 0;
  for (int32_t e = rp[r0 + r]; e < rp[r0 + r + 1]; ++e) {
    const int q = (int)(((int64_t)(ci[e] - c0) * nsl) / len);
    c[q] += 1;
  }
  for (int q = 0; q < nsl; ++q) cnt[r * nsl + q] = c[q];
}

// Scatter row r's entries to their slice-major positions: dst[(r - r0) *
// kSlices + s] is the first position of row r's slice-s entries.
template <class V>
__global__ void slice_scatter_kernel(const int32_t* rp, const int32_t* ci, const V* val, const double* v64,
                                     int64_t r0, int64_t nrows, int64_t c0, int64_t len, const int32_t* dst,
                                     int32_t* ci_out, V* val_out, double* v64_out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int32_t d[kSlices];
  for (int q = 0; q < kSlices; ++q) d[q] = dst[r * kSlices + q];
  for (int32_t e = rp[r0 + r]; e < rp[r0 + r + 1]; ++e) {
    const int q = (int)(((int64_t)(ci[e] - c0) * kSlices) / len);
    const int32_t p = d[q]++;
    ci_out[p] = ci[e];
    val_out[p] = val[e];
    if (v64_out) v64_out[p] = v64[e];
  }
}

// Sorted slicing, step 1: row r's entries go to their row-major positions
// in the sorted groups (dst as for slice_scatter_kernel), each with its sort
// key (column - first column of its slice) << rb | (r - first row of the
// group) and the position it came from.
__global__ void slice_keys_kernel(const int32_t* rp, const int32_t* ci, int64_t r0, int64_t nrows, int64_t c0,
                                  int64_t len, int nsl, const int32_t* dst, const int32_t* rloc, int rb,
                                  uint32_t* key_out, int32_t* src_out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int32_t d[kSlices];
  for (int q = 0; q < nsl; ++q) d[q] = dst[r * nsl + q];
  for (int32_t e = rp[r0 + r]; e < rp[r0 + r + 1]; ++e) {
    const int64_t c = ci[e] - c0;
    const int q = (int)((c * nsl) / len);
    const int64_t first = (q * len + nsl - 1) / nsl;
    const int32_t p = d[q]++;
    key_out[p] = ((uint32_t)(c - first) << rb) | (uint32_t)rloc[r];
    src_out[p] = e;
  }
}

// Column-sorting of plain blocks, step 1: for every entry of every block of
// one LP's schedule (blocks in position order, covering its entries), a
// 64-bit sort key with the block's index in the high word and, in the low
// word, (column - b.rp_off) << rb | (row - b.r0) for a BK_SORTED block, the
// entry's index in the block for any other (so that it stays in place), and
// the entry's position.  Positions are relative to nz0 in the key arrays.
__global__ __launch_bounds__(kThreads) void block_keys_kernel(const Blk* blks, const int32_t* rp,
                                                              const int32_t* ci, int64_t nz0, uint64_t* key,
                                                              int32_t* src) {
  const Blk b = blks[blockIdx.x];
  const uint64_t hi = (uint64_t)blockIdx.x << 32;
  if (blk_kind(b) == BK_SORTED) {
    // one thread per entry; its row is the last of the block's rows that
    // starts at or before it (empty rows share the next row's start)
    const int rb = blk_rowbits(b);
    const int nrows = b.r1 - b.r0;
    for (int k = threadIdx.x; k < b.pn; k += kThreads) {
      const int32_t e = b.p0 + k;
      int lo = 0, up = nrows - 1;
      while (lo < up) {
        const int mid = (lo + up + 1) >> 1;
        if (rp[b.r0 + mid] <= e) lo = mid; else up = mid - 1;
      }
      key[e - nz0] = hi | (((uint32_t)(ci[e] - b.rp_off) << rb) | (uint32_t)lo);
      src[e - nz0] = e;
    }
  } else {
    for (int e = threadIdx.x; e < b.pn; e += kThreads) {
      const int64_t p = (int64_t)b.p0 + e;
      key[p - nz0] = hi | (uint32_t)e;
      src[p - nz0] = (int32_t)p;
    }
  }
}

// Re-blocking of a product stored in column-sorted blocks: every entry of
// the old blocks `old` (which cover the LP's entries) gets the key of its
// place in the new blocks, where[row - base] = (new block index, row in that
// block).  BK_SORTED entries read their row and column back from the packed
// key (the column relative to b.rp_off, which the new blocks share); BK_LONG
// entries (rows that stay long) keep their order.
__global__ __launch_bounds__(kThreads) void reblock_keys_kernel(const Blk* old, const int2* where, int64_t base,
                                                                int rb_new, const int32_t* ci, int64_t nz0,
                                                                uint64_t* key, int32_t* src) {
  const Blk b = old[blockIdx.x];
  if (blk_kind(b) == BK_SORTED) {
    const int rb = blk_rowbits(b);
    const uint32_t rmask = (1u << rb) - 1u;
    for (int e = threadIdx.x; e < b.pn; e += kThreads) {
      const int64_t p = (int64_t)b.p0 + e;
      const uint32_t w = (uint32_t)ci[p];
      const int2 t = where[b.r0 + (int64_t)(w & rmask) - base];
      key[p - nz0] = ((uint64_t)(uint32_t)t.x << 32) | (((w >> rb) << rb_new) | (uint32_t)t.y);
      src[p - nz0] = (int32_t)p;
    }
  } else {
    const uint64_t hi = (uint64_t)(uint32_t)where[b.r0 - base].x << 32;
    for (int e = threadIdx.x; e < b.pn; e += kThreads) {
      const int64_t p = (int64_t)b.p0 + e;
      key[p - nz0] = hi | (uint32_t)e;
      src[p - nz0] = (int32_t)p;
    }
  }
}

// Step 2 (after the keys are sorted): the entries of every BK_SORTED block
// take the low words of the sorted keys as packed column indices and the
// values of the entries they came from (values staged in v_tmp / v64_tmp,
// relative to nz0).
template <class V>
__global__ __launch_bounds__(kThreads) void sorted_block_gather_kernel(const Blk* blks, int64_t nz0,
                                                                       const uint64_t* key, const int32_t* src,
                                                                       const V* val, const double* v64,
                                                                       int32_t* ci_out, V* v_tmp,
                                                                       double* v64_tmp) {
  const Blk b = blks[blockIdx.x];
  for (int e = threadIdx.x; e < b.pn; e += kThreads) {
    const int64_t p = (int64_t)b.p0 + e;
    const int64_t rel = p - nz0;
    const int32_t from = src[rel];
    ci_out[p] = (int32_t)(uint32_t)key[rel];
    v_tmp[rel] = val[from];
    if (v64_tmp) v64_tmp[rel] = v64[from];
  }
}

// Sorted groups: the key of every entry gets its (group, slice) block's
// index in the high word; block s holds positions [off[s], off[s + 1]).
__global__ __launch_bounds__(kThreads) void segment_keys_kernel(const int32_t* off, const uint32_t* k32,
                                                                uint64_t* k64) {
  const int s = blockIdx.x;
  const uint64_t hi = (uint64_t)s << 32;
  for (int64_t p = off[s] + threadIdx.x; p < off[s + 1]; p += kThreads) k64[p] = hi | k32[p];
}

// Sorted slicing, step 2 (after the keys are sorted within each block):
// entry p takes the sorted key as its packed column index and the value of
// the entry it came from.
template <class V>
__global__ void sorted_gather_kernel(const uint64_t* key, const int32_t* src, const V* val, const double* v64,
                                     int64_t nnz, int32_t* ci_out, V* val_out, double* v64_out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int32_t e = src[p];
  ci_out[p] = (int32_t)(uint32_t)key[p];
  val_out[p] = val[e];
  if (v64_out) v64_out[p] = v64[e];
}

template <class V>
__global__ void transpose_gather_kernel(const int32_t* perm, const int32_t* rowid, const V* val,
                                        int64_t z0, int64_t nnz, int32_t* kt_ci, V* kt_val) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int32_t e = perm[p];
  kt_ci[z0 + p] = rowid[e];
  kt_val[z0 + p] = val[z0 + e];
}

// kt_rp[j] = z0 + #{sorted keys < j - c0} for space positions j in [c0, c1]
// (keys: columns relative to c0)
__global__ void transpose_rowptr_kernel(const uint32_t* keys, int64_t nnz, int64_t z0, int64_t c0,
                                        int64_t c1, int32_t* kt_rp) {
  const int64_t j = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > c1) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] + c0 < j) lo = mid + 1; else hi = mid;
  }
  kt_rp[j] = (int32_t)(z0 + lo);
}

template __global__ void sorted_block_gather_kernel<double>(const Blk*, int64_t, const uint64_t*,
                                                            const int32_t*, const double*, const double*,
                                                            int32_t*, double*, double*);
template __global__ void sorted_block_gather_kernel<float>(const Blk*, int64_t, const uint64_t*,
                                                           const int32_t*, const float*, const double*,
                                                           int32_t*, float*, double*);
template __global__ void sorted_gather_kernel<double>(const uint64_t*, const int32_t*, const double*,
                                                      const double*, int64_t, int32_t*, double*, double*);
template __global__ void sorted_gather_kernel<float>(const uint64_t*, const int32_t*, const float*,
                                                     const double*, int64_t, int32_t*, float*, double*);
template __global__ void slice_scatter_kernel<double>(const int32_t*, const int32_t*, const double*,
                                                      const double*, int64_t, int64_t, int64_t, int64_t,
                                                      const int32_t*, int32_t*, double*, double*);
template __global__ void slice_scatter_kernel<float>(const int32_t*, const int32_t*, const float*,
                                                     const double*, int64_t, int64_t, int64_t, int64_t,
                                                     const int32_t*, int32_t*, float*, double*);
template __global__ void transpose_gather_kernel<double>(const int32_t*, const int32_t*, const double*,
                                                         int64_t, int64_t, int32_t*, double*);

}  // namespace halp

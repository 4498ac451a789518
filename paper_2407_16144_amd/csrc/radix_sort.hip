// Stable least-significant-digit radix sort of (key, value) pairs, used by
// the layout builders: the explicit transpose K^T (key: column), the
// column-sorted plain blocks and the sorted groups (key: block or segment
// index in the high word, packed column/row key in the low word).
//
// Each pass is a counting sort by one 8-bit digit of the key:
//   1. radix_hist_kernel: per tile of kRadixTile consecutive items, the count
//      of each digit (LDS histogram), written digit-major: counts[d * ntiles + t];
//   2. an exclusive scan of that table gives every (digit, tile) pair the
//      first output position of its items (all smaller digits, then the same
//      digit in earlier tiles);
//   3. radix_scatter_kernel: each tile walks its items in index order, 256 at
//      a time, ranks each item among the items of the same digit before it
//      (wave ballots over the digit's bits, then per-wave counts in LDS) and
//      writes it to base[digit] + rank.
// Equal digits keep their input order in every pass, so the sort is stable
// and its result does not depend on timing.  Included by engine.hip (uses
// dalloc / dfree / HIPCHECK / nblk defined there).

namespace halp {

constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixThreads = 256;  // one thread per bin in the per-tile tables
constexpr int kRadixWaves = kRadixThreads / 64;
constexpr int kRadixItems = 16;     // items per thread and tile
constexpr int kRadixTile = kRadixThreads * kRadixItems;
constexpr int kScanItems = 16;
constexpr int kScanTile = kRadixThreads * kScanItems;
static_assert(kRadixThreads == kRadixBins, "one thread per digit");

template <class K>
__device__ inline uint32_t radix_digit(K key, int shift) {
  return (uint32_t)(key >> shift) & (uint32_t)(kRadixBins - 1);
}

// counts[d * ntiles + tile] = items of the tile whose digit at `shift` is d
template <class K>
__global__ __launch_bounds__(kRadixThreads) void radix_hist_kernel(const K* keys, int64_t n, int shift,
                                                                   int64_t ntiles, uint32_t* counts) {
  __shared__ uint32_t h[kRadixBins];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
  for (int r = 0; r < kRadixItems; ++r) {
    const int64_t i = t0 + (int64_t)r * kRadixThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[radix_digit(keys[i], shift)], 1u);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan within tiles of kScanTile values: out[i] = sum of the
// tile's values before i; sums[tile] = the tile's total (if sums != null).
__global__ __launch_bounds__(kRadixThreads) void scan_tile_kernel(const uint32_t* in, uint32_t* out, int64_t n,
                                                                  uint32_t* sums) {
  __shared__ uint32_t s[kRadixThreads];
  const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t t = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = i0 + k < n ? in[i0 + k] : 0u;
    t += v[k];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < kRadixThreads; off <<= 1) {
    const uint32_t add = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - t;
  for (int k = 0; k < kScanItems; ++k) {
    if (i0 + k < n) out[i0 + k] = run;
    run += v[k];
  }
  if (sums && threadIdx.x == kRadixThreads - 1) sums[blockIdx.x] = s[threadIdx.x];
}

// out[i] += offs[i / kScanTile]: the scanned tile totals of the level above
__global__ void scan_add_kernel(uint32_t* out, int64_t n, const uint32_t* offs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i / kScanTile];
}

// One stable counting-sort pass: items of tile `blockIdx.x` go to
// offs[d * ntiles + tile] + (rank among the tile's earlier items of digit d).
template <class K>
__global__ __launch_bounds__(kRadixThreads) void radix_scatter_kernel(const K* kin, const int32_t* vin, K* kout,
                                                                      int32_t* vout, int64_t n, int shift,
                                                                      int64_t ntiles, const uint32_t* offs) {
  __shared__ uint32_t base[kRadixBins];
  __shared__ uint32_t wcnt[kRadixWaves][kRadixBins];
  base[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  for (int w = 0; w < kRadixWaves; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
  for (int r = 0; r < kRadixItems; ++r) {
    const int64_t i = t0 + (int64_t)r * kRadixThreads + threadIdx.x;
    const bool ok = i < n;
    const K k = ok ? kin[i] : K(0);
    const int32_t v = ok ? vin[i] : 0;
    const uint32_t d = radix_digit(k, shift);
    // lanes of this wave holding a valid item with the same digit
    uint64_t same = __ballot(ok);
    for (int b = 0; b < kRadixBits; ++b) {
      const uint32_t bit = (d >> b) & 1u;
      const uint64_t set = __ballot(bit);
      same &= bit ? set : ~set;
    }
    const uint32_t rank = (uint32_t)__popcll(same & below);
    if (ok && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
    __syncthreads();
    if (ok) {
      uint32_t pos = base[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int w = 0; w < kRadixWaves; ++w) {
      tot += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0;
    }
    base[threadIdx.x] += tot;
    __syncthreads();
  }
}

// Digit shifts that cover key bits [lo, hi): lo, lo + 8, ... (the top pass
// may read bits above hi, which must be zero).
static void radix_shifts(std::vector<int>& shifts, int lo, int hi) {
  for (int s = lo; s < hi; s += kRadixBits) shifts.push_back(s);
}

// Number of bits needed to hold the values 0 .. v (v >= 0).
static int bits_for(int64_t v) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) <= v) ++b;
  return b;
}

// Sorts the n pairs (kin, vin) by the digits at `shifts` (least significant
// first) into (kout, vout), stably.  kin / vin are read only; kout / vout
// must not overlap them.  Temporaries come from dalloc and are freed (in
// reverse order) after the stream has finished the sort.
template <class K>
static void radix_sort_pairs(const K* kin, const int32_t* vin, K* kout, int32_t* vout, int64_t n,
                             const std::vector<int>& shifts, hipStream_t stream) {
  if (n <= 0) return;
  if (n > (int64_t)INT32_MAX) throw Error(-3, "radix sort: more than 2^31 - 1 items");
  const int np = (int)shifts.size();
  if (np == 0) {
    HIPCHECK(hipMemcpyAsync(kout, kin, sizeof(K) * n, hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipMemcpyAsync(vout, vin, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipStreamSynchronize(stream));
    return;
  }
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  // scan levels: len[0] counts, len[l] tile totals of level l - 1
  std::vector<int64_t> len{ntiles * kRadixBins};
  while (len.back() > kScanTile) len.push_back((len.back() + kScanTile - 1) / kScanTile);
  const int L = (int)len.size();
  uint32_t *counts = nullptr, *offs = nullptr;
  dalloc(&counts, len[0]);
  dalloc(&offs, len[0]);
  std::vector<uint32_t*> sums(L, nullptr), scanned(L, nullptr);
  for (int l = 1; l < L; ++l) {
    dalloc(&sums[l], len[l]);
    dalloc(&scanned[l], len[l]);
  }
  scanned[0] = offs;
  K* kalt = nullptr;
  int32_t* valt = nullptr;
  if (np > 1) {
    dalloc(&kalt, n);
    dalloc(&valt, n);
  }
  const K* ks = kin;
  const int32_t* vs = vin;
  for (int j = 0; j < np; ++j) {
    // the last pass writes (kout, vout); the others alternate with (kalt, valt)
    const bool to_out = ((np - 1 - j) & 1) == 0;
    K* kd = to_out ? kout : kalt;
    int32_t* vd = to_out ? vout : valt;
    radix_hist_kernel<K><<<(unsigned)ntiles, kRadixThreads, 0, stream>>>(ks, n, shifts[j], ntiles, counts);
    const uint32_t* src = counts;
    for (int l = 0; l < L; ++l) {
      const unsigned tiles = (unsigned)((len[l] + kScanTile - 1) / kScanTile);
      scan_tile_kernel<<<tiles, kRadixThreads, 0, stream>>>(src, scanned[l], len[l], l + 1 < L ? sums[l + 1] : nullptr);
      if (l + 1 < L) src = sums[l + 1];
    }
    for (int l = L - 1; l >= 1; --l)
      scan_add_kernel<<<nblk(len[l - 1]), 256, 0, stream>>>(scanned[l - 1], len[l - 1], scanned[l]);
    radix_scatter_kernel<K><<<(unsigned)ntiles, kRadixThreads, 0, stream>>>(ks, vs, kd, vd, n, shifts[j], ntiles,
                                                                           offs);
    HIPCHECK(hipGetLastError());
    ks = kd;
    vs = vd;
  }
  HIPCHECK(hipStreamSynchronize(stream));
  dfree(valt);
  dfree(kalt);
  for (int l = L - 1; l >= 1; --l) {
    dfree(scanned[l]);
    dfree(sums[l]);
  }
  dfree(offs);
  dfree(counts);
}

}  // namespace halp

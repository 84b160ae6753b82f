// Setup primitives: scans, deterministic grouping and transposes, symbolic unions.
//
// Every output here is independent of thread scheduling: atomics only count or claim
// slots, and each group/row is put into ascending order afterwards, so two runs of a
// setup give bitwise-identical hierarchies.
#include "common.h"

namespace amgf {

// ======================================================================================
// exclusive scan (int32 data, int64 carries)
// ======================================================================================
constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = SCAN_T * SCAN_ITEMS;

__device__ __forceinline__ long long block_excl_scan(long long v, long long* wsum,
                                                     long long* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  long long inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    long long t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long acc = 0;
    for (int w = 0; w < SCAN_T / 64; ++w) {
      long long t = wsum[w];
      wsum[w] = acc;
      acc += t;
    }
    *total = acc;
  }
  __syncthreads();
  return inc - v + wsum[wid];
}

__global__ void k_scan_sums(const int* __restrict__ in, int n, long long* __restrict__ sums) {
  __shared__ long long wsum[SCAN_T / 64];
  __shared__ long long tot;
  const int64_t base = int64_t(blockIdx.x) * SCAN_CHUNK + int64_t(threadIdx.x) * SCAN_ITEMS;
  long long s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) s += in[base + i];
  block_excl_scan(s, wsum, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block: exclusive scan of the per-chunk sums in place
__global__ void k_scan_sums_single(long long* sums, int nb, int* flag) {
  __shared__ long long wsum[SCAN_T / 64];
  __shared__ long long tot;
  const int per = (nb + SCAN_T - 1) / SCAN_T;
  const int lo = threadIdx.x * per;
  long long s = 0;
  for (int i = 0; i < per; ++i)
    if (lo + i < nb) s += sums[lo + i];
  long long off = block_excl_scan(s, wsum, &tot);
  for (int i = 0; i < per; ++i)
    if (lo + i < nb) {
      long long t = sums[lo + i];
      sums[lo + i] = off;
      off += t;
    }
  if (threadIdx.x == 0) {
    sums[nb] = tot;
    if (tot > 0x7fffffffLL) atomicOr(flag, 1);
  }
}

__global__ void k_scan_final(const int* __restrict__ in, int* __restrict__ out, int n,
                             const long long* __restrict__ sums) {
  __shared__ long long wsum[SCAN_T / 64];
  __shared__ long long tot;
  const int64_t base = int64_t(blockIdx.x) * SCAN_CHUNK + int64_t(threadIdx.x) * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  long long s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  long long off = block_excl_scan(s, wsum, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) {
      out[base + i] = int(off);
      off += v[i];
    }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = int(sums[gridDim.x]);
}

int scan_exclusive(Ctx& c, const int* in, int* out, int n, bool want_total) {
  if (n == 0) {
    AMGF_HIP(hipMemsetAsync(out, 0, sizeof(int), c.s));
    return 0;
  }
  const int nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
  DBuf<long long> sums(nb + 1);
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(SCAN_T), 0, c.s, in, n, sums.p);
  hipLaunchKernelGGL(k_scan_sums_single, dim3(1), dim3(SCAN_T), 0, c.s, sums.p, nb, c.flag.p);
  hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(SCAN_T), 0, c.s, in, out, n, sums.p);
  AMGF_LAUNCH_CHECK();
  if (!want_total) return -1;
  int total = d2h_scalar(out + n, c.s);
  int fl = d2h_scalar(c.flag.p, c.s);
  AMGF_REQUIRE(fl == 0, AMGF_ENOMEM, "scan total exceeds int32");
  return total;
}

// ======================================================================================
// row expansion
// ======================================================================================
__global__ void k_expand_rows(const int* __restrict__ rowptr, int nrows, int* __restrict__ rows) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) rows[k] = r;
}

void expand_rows(Ctx& c, const int* rowptr, int nrows, int* rows) {
  if (nrows == 0) return;
  hipLaunchKernelGGL(k_expand_rows, dim3(grid_for(nrows, 256)), dim3(256), 0, c.s, rowptr,
                     nrows, rows);
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// deterministic group-by-key
// ======================================================================================
__global__ void k_count_keys(const int* __restrict__ keys, int n, int* __restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && keys[i] >= 0) atomicAdd(&counts[keys[i]], 1);
}
__global__ void k_fill_keys(const int* __restrict__ keys, int n, const int* __restrict__ off,
                            int* __restrict__ cursor, int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || keys[i] < 0) return;
  const int k = keys[i];
  perm[off[k] + atomicAdd(&cursor[k], 1)] = i;
}
constexpr int SMALL_SEGMENT = 2048;

// one wavefront per segment: rank sort of distinct values (ascending); segments longer
// than SMALL_SEGMENT are left to k_bitonic_segments
__global__ void k_segment_sort(const int* __restrict__ off, int nseg, const int* __restrict__ in,
                               int* __restrict__ out) {
  const int seg = blockIdx.x;
  if (seg >= nseg) return;
  const int a = off[seg], b = off[seg + 1];
  if (b - a > SMALL_SEGMENT) return;
  for (int j = a + threadIdx.x; j < b; j += blockDim.x) {
    const int v = in[j];
    int rank = 0;
    for (int i = a; i < b; ++i) rank += in[i] < v;
    out[a + rank] = v;
  }
}

__global__ void k_max_segment(const int* __restrict__ off, int nseg, int* __restrict__ mx) {
  const int seg = blockIdx.x * blockDim.x + threadIdx.x;
  if (seg < nseg) atomicMax(mx, off[seg + 1] - off[seg]);
}

int max_segment_length(Ctx& c, const int* off, int nseg) {
  DBuf<int> mx(1);
  AMGF_HIP(hipMemsetAsync(mx.p, 0, sizeof(int), c.s));
  if (nseg > 0)
    hipLaunchKernelGGL(k_max_segment, dim3(grid_for(nseg, 256)), dim3(256), 0, c.s, off, nseg,
                       mx.p);
  AMGF_LAUNCH_CHECK();
  return d2h_scalar(mx.p, c.s);
}

// one 1024-thread workgroup per long segment: bitonic sort in a padded scratch region
__global__ void __launch_bounds__(1024) k_bitonic_segments(const int* __restrict__ list,
                                                           const int* __restrict__ off,
                                                           const int64_t* __restrict__ soff,
                                                           const int* __restrict__ in,
                                                           int* __restrict__ out,
                                                           int* __restrict__ scratch) {
  const int seg = list[blockIdx.x];
  const int a = off[seg], s = off[seg + 1] - a;
  int P = 1;
  while (P < s) P <<= 1;
  int* buf = scratch + soff[blockIdx.x];
  for (int i = threadIdx.x; i < P; i += 1024) buf[i] = i < s ? in[a + i] : 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += 1024) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int x = buf[i], y = buf[ixj];
          if (((i & k) == 0) ? (x > y) : (x < y)) {
            buf[i] = y;
            buf[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < s; i += 1024) out[a + i] = buf[i];
}

void group_by_key(Ctx& c, const int* keys, int n, int nkeys, DBuf<int>& offsets,
                  DBuf<int>& perm, bool sorted) {
  offsets.alloc(size_t(nkeys) + 1);
  DBuf<int> counts(std::max(nkeys, 1));
  AMGF_HIP(hipMemsetAsync(counts.p, 0, counts.bytes(), c.s));
  if (n > 0)
    hipLaunchKernelGGL(k_count_keys, dim3(grid_for(n, 256)), dim3(256), 0, c.s, keys, n,
                       counts.p);
  const int total = scan_exclusive(c, counts.p, offsets.p, nkeys);
  perm.alloc(std::max(total, 1));
  if (total == 0) return;
  AMGF_HIP(hipMemsetAsync(counts.p, 0, counts.bytes(), c.s));
  if (!sorted) {
    // members of each key in arrival order (callers that only iterate over them)
    hipLaunchKernelGGL(k_fill_keys, dim3(grid_for(n, 256)), dim3(256), 0, c.s, keys, n,
                       offsets.p, counts.p, perm.p);
    AMGF_LAUNCH_CHECK();
    return;
  }
  DBuf<int> tmp(total);
  hipLaunchKernelGGL(k_fill_keys, dim3(grid_for(n, 256)), dim3(256), 0, c.s, keys, n,
                     offsets.p, counts.p, tmp.p);
  hipLaunchKernelGGL(k_segment_sort, dim3(nkeys), dim3(64), 0, c.s, offsets.p, nkeys, tmp.p,
                     perm.p);
  AMGF_LAUNCH_CHECK();
  DBuf<int> mx(1);
  AMGF_HIP(hipMemsetAsync(mx.p, 0, sizeof(int), c.s));
  hipLaunchKernelGGL(k_max_segment, dim3(grid_for(nkeys, 256)), dim3(256), 0, c.s, offsets.p,
                     nkeys, mx.p);
  if (d2h_scalar(mx.p, c.s) <= SMALL_SEGMENT) return;
  // long segments: list them on the host and bitonic-sort each in one workgroup
  std::vector<int> off = d2h(offsets.p, size_t(nkeys) + 1, c.s);
  std::vector<int> big;
  std::vector<int64_t> soff(1, 0);
  for (int k = 0; k < nkeys; ++k) {
    const int s = off[k + 1] - off[k];
    if (s > SMALL_SEGMENT) {
      int P = 1;
      while (P < s) P <<= 1;
      big.push_back(k);
      soff.push_back(soff.back() + P);
    }
  }
  DBuf<int> dlist(big.size()), scratch(soff.back());
  DBuf<int64_t> dsoff(soff.size());
  AMGF_HIP(hipMemcpyAsync(dlist.p, big.data(), sizeof(int) * big.size(), hipMemcpyHostToDevice,
                          c.s));
  AMGF_HIP(hipMemcpyAsync(dsoff.p, soff.data(), sizeof(int64_t) * soff.size(),
                          hipMemcpyHostToDevice, c.s));
  hipLaunchKernelGGL(k_bitonic_segments, dim3(big.size()), dim3(1024), 0, c.s, dlist.p, offsets.p,
                     dsoff.p, tmp.p, perm.p, scratch.p);
  AMGF_LAUNCH_CHECK();
  AMGF_HIP(hipStreamSynchronize(c.s));
}

// ======================================================================================
// BSR transpose
// ======================================================================================
// One thread per value of the transpose: consecutive threads write consecutive values,
// and the threads of one output block read the br*bc values of one source block, so both
// sides coalesce (a thread per block read its source block one scattered value at a time).
__global__ void k_transpose_fill(int64_t nnzb, const int* __restrict__ perm,
                                 const int* __restrict__ rows, const double* __restrict__ val,
                                 int br, int bc, int* __restrict__ tcol,
                                 double* __restrict__ tval) {
  const int bs = br * bc;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nnzb * bs) return;
  const int64_t k = e / bs;
  const int w = int(e - k * bs);
  const int src = perm[k];
  // value (q, p) of the bc x br transposed block is value (p, q) of the source block
  const int q = w / br, p = w - q * br;
  tval[e] = val[int64_t(src) * bs + p * bc + q];
  if (w == 0) tcol[k] = rows[src];
}

void bsr_transpose(Ctx& c, const BSR& A, BSR& T) {
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.br = A.bc;
  T.bc = A.br;
  T.nnzb = A.nnzb;
  DBuf<int> rows(std::max<int64_t>(A.nnzb, 1));
  expand_rows(c, A.rowptr.p, A.nrows, rows.p);
  DBuf<int> perm;
  group_by_key(c, A.col.p, int(A.nnzb), A.ncols, T.rowptr, perm);
  T.col.alloc(std::max<int64_t>(A.nnzb, 1));
  T.val.alloc(std::max<int64_t>(A.nnzb, 1) * A.bsz());
  if (A.nnzb)
    hipLaunchKernelGGL(k_transpose_fill, dim3(grid_for(A.nnzb * int64_t(A.bsz()), 256)),
                       dim3(256), 0, c.s, A.nnzb, perm.p, rows.p, A.val.p, A.br, A.bc,
                       T.col.p, T.val.p);
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// symbolic union (one wavefront per output row, LDS hash set)
// ======================================================================================
// The hash table of a launch has TS slots per row (a power of two at least twice the
// largest candidate count of any row, at most HS); rows with up to 512 slots share a
// 256-thread workgroup four at a time, larger tables get one wavefront per workgroup.
constexpr int HS = 2048;                 // largest hash table per row
constexpr int HS_MAX_UNIQUE = 1536;      // capacity before the row is rejected

__device__ __forceinline__ void hs_insert(int* table, int* list, int* cnt, int key,
                                          bool fill, int* flag, unsigned mask, int cap) {
  unsigned h = (unsigned(key) * 2654435761u) & mask;
  for (unsigned probe = 0; probe <= mask; ++probe) {
    const int old = atomicCAS(&table[h], -1, key);
    if (old == -1) {
      const int pos = atomicAdd(cnt, 1);
      if (pos < cap) {
        if (fill) list[pos] = key;
      } else {
        atomicOr(flag, 2);
      }
      return;
    }
    if (old == key) return;
    h = (h + 1) & mask;
  }
  atomicOr(flag, 2);
}

__global__ void k_max_int(const int* __restrict__ v, int n, int* __restrict__ mx) {
  int m = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    m = max(m, v[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(mx, m);
}

// largest entry of a non-negative int array (0 when empty); waits for the result
static int max_value(Ctx& c, const int* v, int n) {
  DBuf<int> mx(1);
  AMGF_HIP(hipMemsetAsync(mx.p, 0, sizeof(int), c.s));
  if (n > 0)
    hipLaunchKernelGGL(k_max_int, dim3(std::min<unsigned>(grid_for(n, 256), 1024)), dim3(256), 0,
                       c.s, v, n, mx.p);
  AMGF_LAUNCH_CHECK();
  return d2h_scalar(mx.p, c.s);
}

// candidate count of each row (an upper bound of its union size)
__global__ void k_union_bound(int nrows, const int* __restrict__ rp1,
                              const int* __restrict__ col1, const int* __restrict__ rp2,
                              const int* __restrict__ row_mask, int* __restrict__ bound) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int b = 0;
  if (!row_mask || row_mask[r])
    for (int t = rp1[r]; t < rp1[r + 1]; ++t) b += rp2 ? rp2[col1[t] + 1] - rp2[col1[t]] : 1;
  bound[r] = b;
}

__global__ void __launch_bounds__(256) k_union(int nrows, int ts, int cap,
                                               const int* __restrict__ rp1,
                                               const int* __restrict__ col1,
                                               const int* __restrict__ rp2,
                                               const int* __restrict__ col2,
                                               const int* __restrict__ map, int exclude_diag,
                                               const int* __restrict__ row_mask, int fill,
                                               int* __restrict__ counts,
                                               const int* __restrict__ rowptr,
                                               int* __restrict__ outcol, int* flag) {
  extern __shared__ int lds[];
  __shared__ int cnts[4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * (blockDim.x >> 6) + wv;
  int* table = lds + wv * (ts + cap);
  int* list = table + ts;
  int* cnt = &cnts[wv];
  if (r >= nrows) return;
  if ((row_mask && !row_mask[r]) || rp1[r] == rp1[r + 1]) {
    if (fill != 1 && lane == 0) counts[r] = 0;
    return;
  }
  const unsigned mask = unsigned(ts) - 1;
  for (int i = lane; i < ts; i += 64) table[i] = -1;
  if (lane == 0) *cnt = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (int t = rp1[r] + lane; t < rp1[r + 1]; t += 64) {
    const int mid = col1[t];
    if (rp2) {
      for (int u = rp2[mid]; u < rp2[mid + 1]; ++u) {
        int cand = col2[u];
        if (map) cand = map[cand];
        if (cand < 0 || (exclude_diag && cand == r)) continue;
        hs_insert(table, list, cnt, cand, fill, flag, mask, cap);
      }
    } else {
      int cand = map ? map[mid] : mid;
      if (cand < 0 || (exclude_diag && cand == r)) continue;
      hs_insert(table, list, cnt, cand, fill, flag, mask, cap);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  const int n = min(*cnt, cap);
  if (!fill) {
    if (lane == 0) counts[r] = n;
    return;
  }
  if (fill == 2 && lane == 0) counts[r] = n;     // sorted list at rowptr[r] = bound offset
  const int base = rowptr[r];
  for (int j = lane; j < n; j += 64) {
    const int v = list[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) rank += list[i] < v;
    outcol[base + rank] = v;
  }
}

// rows' sorted lists from their bound-sized slots (tmp at boff) to the compact pattern
__global__ void __launch_bounds__(256) k_union_compact(int nrows, const int* __restrict__ boff,
                                                       const int* __restrict__ tmp,
                                                       const int* __restrict__ rowptr,
                                                       int* __restrict__ col) {
  const int r = int((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 5);
  const int l = threadIdx.x & 31;
  if (r >= nrows) return;
  const int n = rowptr[r + 1] - rowptr[r];
  for (int j = l; j < n; j += 32) col[rowptr[r] + j] = tmp[boff[r] + j];
}

__global__ void k_sum_i64(const int* __restrict__ v, int n, unsigned long long* __restrict__ s) {
  unsigned long long a = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    a += unsigned(v[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(s, a);
}

// sum of a non-negative int array in 64 bits; waits for the result
static int64_t sum_i64(Ctx& c, const int* v, int n) {
  DBuf<unsigned long long> t(1);
  AMGF_HIP(hipMemsetAsync(t.p, 0, sizeof(unsigned long long), c.s));
  if (n > 0)
    hipLaunchKernelGGL(k_sum_i64, dim3(std::min<unsigned>(grid_for(n, 256), 1024)), dim3(256), 0,
                       c.s, v, n, t.p);
  AMGF_LAUNCH_CHECK();
  return int64_t(d2h_scalar(t.p, c.s));
}

// above this many candidate slots in all, the lists are hashed twice (count, then fill)
// instead of once into bound-sized slots
constexpr int64_t UNION_ONE_PASS_MAX = int64_t(1) << 30;

void union_symbolic(Ctx& c, int nrows, int ncols, const int* rp1, const int* col1,
                    const int* rp2, const int* col2, const int* map, bool exclude_diag,
                    const int* row_mask, BSR& C) {
  C.nrows = nrows;
  C.ncols = ncols;
  DBuf<int> counts(std::max(nrows, 1));
  C.rowptr.alloc(size_t(nrows) + 1);
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  if (nrows == 0) {
    C.nnzb = scan_exclusive(c, counts.p, C.rowptr.p, 0);
    C.col.alloc(1);
    return;
  }
  // table size from the largest candidate count
  hipLaunchKernelGGL(k_union_bound, dim3(grid_for(nrows, 256)), dim3(256), 0, c.s, nrows, rp1,
                     col1, rp2, row_mask, counts.p);
  AMGF_LAUNCH_CHECK();
  const int maxb = max_value(c, counts.p, nrows);
  int ts = 64;
  while (ts < 2 * maxb && ts < HS) ts <<= 1;
  const int cap = std::min(HS_MAX_UNIQUE, ts);
  const int wpg = ts <= 512 ? 4 : 1;                    // rows (wavefronts) per workgroup
  const size_t lds = size_t(wpg) * (ts + cap) * sizeof(int);
  const dim3 g((nrows + wpg - 1) / wpg), b(64 * wpg);
  // one hashing pass: each row's sorted list goes to a slot of its bound's size, then the
  // lists are packed; candidate bounds at most `cap` each keep the slots within the bound
  const int64_t total_bound = sum_i64(c, counts.p, nrows);
  if (total_bound <= UNION_ONE_PASS_MAX) {
    DBuf<int> boff(size_t(nrows) + 1);
    scan_exclusive(c, counts.p, boff.p, nrows, false);
    DBuf<int> tmp(std::max<int64_t>(total_bound, 1));
    hipLaunchKernelGGL(k_union, g, b, lds, c.s, nrows, ts, cap, rp1, col1, rp2, col2, map,
                       int(exclude_diag), row_mask, 2, counts.p, boff.p, tmp.p, c.flag.p);
    AMGF_LAUNCH_CHECK();
    int fl = d2h_scalar(c.flag.p, c.s);
    AMGF_REQUIRE(fl == 0, AMGF_ENOMEM, "symbolic product row exceeds the union capacity");
    C.nnzb = scan_exclusive(c, counts.p, C.rowptr.p, nrows);
    C.col.alloc(std::max<int64_t>(C.nnzb, 1));
    if (C.nnzb)
      hipLaunchKernelGGL(k_union_compact, dim3(grid_for(int64_t(nrows) * 32, 256)), dim3(256), 0,
                         c.s, nrows, boff.p, tmp.p, C.rowptr.p, C.col.p);
    AMGF_LAUNCH_CHECK();
    return;
  }
  hipLaunchKernelGGL(k_union, g, b, lds, c.s, nrows, ts, cap, rp1, col1, rp2, col2, map,
                     int(exclude_diag), row_mask, 0, counts.p, nullptr, nullptr, c.flag.p);
  AMGF_LAUNCH_CHECK();
  int fl = d2h_scalar(c.flag.p, c.s);
  AMGF_REQUIRE(fl == 0, AMGF_ENOMEM, "symbolic product row exceeds the union capacity");
  C.nnzb = scan_exclusive(c, counts.p, C.rowptr.p, nrows);
  C.col.alloc(std::max<int64_t>(C.nnzb, 1));
  if (C.nnzb)
    hipLaunchKernelGGL(k_union, g, b, lds, c.s, nrows, ts, cap, rp1, col1, rp2, col2, map,
                       int(exclude_diag), row_mask, 1, nullptr, C.rowptr.p, C.col.p, c.flag.p);
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// C = A + B (pattern union, exact values)
// ======================================================================================
__global__ void k_merge_count(int nrows, const int* __restrict__ ra, const int* __restrict__ ca,
                              const int* __restrict__ rb, const int* __restrict__ cb,
                              int* __restrict__ counts) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int i = ra[r], ie = ra[r + 1], j = rb[r], je = rb[r + 1], n = 0;
  while (i < ie || j < je) {
    if (j >= je || (i < ie && ca[i] < cb[j])) ++i;
    else if (i >= ie || cb[j] < ca[i]) ++j;
    else { ++i; ++j; }
    ++n;
  }
  counts[r] = n;
}

constexpr int MERGE_LDS = 256;   // column ids of A's and of B's row a wavefront stages

// one wavefront per row: rows without entries of B are copied block-parallel (the
// common case); for rows with both, the column lists go to LDS, lane 0 merges them there
// into (entry of A, entry of B) pairs and the wavefront then writes the blocks; rows longer
// than the staging are merged by lane 0 from memory
__global__ void __launch_bounds__(256) k_merge_fill(int nrows, int bsz, const int* __restrict__ ra,
                                                    const int* __restrict__ ca,
                                                    const double* __restrict__ va,
                                                    const int* __restrict__ rb,
                                                    const int* __restrict__ cb,
                                                    const double* __restrict__ vb,
                                                    const int* __restrict__ rc,
                                                    int* __restrict__ cc,
                                                    double* __restrict__ vc) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= nrows) return;
  const int i0 = ra[r], ie = ra[r + 1], j0 = rb[r], je = rb[r + 1], o0 = rc[r];
  if (j0 == je) {
    for (int k = lane; k < ie - i0; k += 64) cc[o0 + k] = ca[i0 + k];
    const int64_t nv = int64_t(ie - i0) * bsz;
    for (int64_t e = lane; e < nv; e += 64) vc[int64_t(o0) * bsz + e] = va[int64_t(i0) * bsz + e];
    return;
  }
  const int na = ie - i0, nb = je - j0;
  if (na <= MERGE_LDS && nb <= MERGE_LDS) {
    __shared__ int sa[4][MERGE_LDS], sb[4][MERGE_LDS];
    __shared__ int2 pair[4][2 * MERGE_LDS];
    const int wv = threadIdx.x >> 6;
    for (int k = lane; k < na; k += 64) sa[wv][k] = ca[i0 + k];
    for (int k = lane; k < nb; k += 64) sb[wv][k] = cb[j0 + k];
    wave_lds_sync();
    if (lane == 0) {
      int i = 0, j = 0, o = 0;
      while (i < na || j < nb) {
        if (j >= nb || (i < na && sa[wv][i] < sb[wv][j])) pair[wv][o] = make_int2(i++, -1);
        else if (i >= na || sb[wv][j] < sa[wv][i]) pair[wv][o] = make_int2(-1, j++);
        else pair[wv][o] = make_int2(i++, j++);
        ++o;
      }
    }
    wave_lds_sync();
    const int no = rc[r + 1] - o0;
    for (int k = lane; k < no; k += 64) {
      const int2 pr = pair[wv][k];
      cc[o0 + k] = pr.x >= 0 ? sa[wv][pr.x] : sb[wv][pr.y];
    }
    for (int64_t e = lane; e < int64_t(no) * bsz; e += 64) {
      const int k = int(e / bsz), q = int(e % bsz);
      const int2 pr = pair[wv][k];
      double v;
      if (pr.x >= 0 && pr.y >= 0)
        v = add_rn(va[int64_t(i0 + pr.x) * bsz + q], vb[int64_t(j0 + pr.y) * bsz + q]);
      else if (pr.x >= 0)
        v = va[int64_t(i0 + pr.x) * bsz + q];
      else
        v = vb[int64_t(j0 + pr.y) * bsz + q];
      vc[int64_t(o0) * bsz + e] = v;
    }
    return;
  }
  if (lane != 0) return;
  int i = i0, j = j0, o = o0;
  while (i < ie || j < je) {
    double* d = vc + int64_t(o) * bsz;
    if (j >= je || (i < ie && ca[i] < cb[j])) {
      cc[o] = ca[i];
      for (int e = 0; e < bsz; ++e) d[e] = va[int64_t(i) * bsz + e];
      ++i;
    } else if (i >= ie || cb[j] < ca[i]) {
      cc[o] = cb[j];
      for (int e = 0; e < bsz; ++e) d[e] = vb[int64_t(j) * bsz + e];
      ++j;
    } else {
      cc[o] = ca[i];
      for (int e = 0; e < bsz; ++e)
        d[e] = add_rn(va[int64_t(i) * bsz + e], vb[int64_t(j) * bsz + e]);
      ++i;
      ++j;
    }
    ++o;
  }
}

void bsr_add(Ctx& c, const BSR& A, const BSR& B, BSR& C) {
  AMGF_REQUIRE(A.nrows == B.nrows && A.br == B.br && A.bc == B.bc, AMGF_EINVAL,
               "bsr_add shape mismatch");
  C.nrows = A.nrows;
  C.ncols = A.ncols;
  C.br = A.br;
  C.bc = A.bc;
  DBuf<int> counts(std::max(A.nrows, 1));
  C.rowptr.alloc(size_t(A.nrows) + 1);
  if (A.nrows)
    hipLaunchKernelGGL(k_merge_count, dim3(grid_for(A.nrows, 256)), dim3(256), 0, c.s,
                       A.nrows, A.rowptr.p, A.col.p, B.rowptr.p, B.col.p, counts.p);
  C.nnzb = scan_exclusive(c, counts.p, C.rowptr.p, A.nrows);
  C.col.alloc(std::max<int64_t>(C.nnzb, 1));
  C.val.alloc(std::max<int64_t>(C.nnzb, 1) * C.bsz());
  if (A.nrows)
    hipLaunchKernelGGL(k_merge_fill, dim3(grid_for(A.nrows, 4)), dim3(256), 0, c.s,
                       A.nrows, int(A.bsz()), A.rowptr.p, A.col.p, A.val.p, B.rowptr.p,
                       B.col.p, B.val.p, C.rowptr.p, C.col.p, C.val.p);
  AMGF_LAUNCH_CHECK();
}

}  // namespace amgf

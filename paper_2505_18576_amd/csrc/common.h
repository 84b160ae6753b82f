// Shared declarations of the AMGF HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/amgf.h"

namespace amgf {

// ------------------------------------------------------------------------------------
// errors: thrown inside the library, converted to amgf_status at the C boundary
// ------------------------------------------------------------------------------------
struct Error : std::runtime_error {
  amgf_status status;
  Error(amgf_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define AMGF_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::amgf::Error(e_ == hipErrorOutOfMemory ? AMGF_ENOMEM : AMGF_EDEVICE,      \
                          std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define AMGF_REQUIRE(cond, status, msg)                                                \
  do {                                                                                 \
    if (!(cond)) throw ::amgf::Error(status, msg);                                     \
  } while (0)

#define AMGF_LAUNCH_CHECK() AMGF_HIP(hipGetLastError())

// ------------------------------------------------------------------------------------
// device buffers (owned by the handle)
// ------------------------------------------------------------------------------------
// Where device buffers come from: hipMalloc, or the caller's amgf_allocator that the
// running entry point installed (AllocScope).  A buffer gives its memory back to the source
// it came from, with the stream it was allocated on.
struct AllocSrc {
  amgf_allocator a{};
  hipStream_t s = nullptr;
};
inline thread_local const AllocSrc* g_alloc = nullptr;
struct AllocScope {
  const AllocSrc* prev;
  explicit AllocScope(const AllocSrc* a) : prev(g_alloc) { g_alloc = a; }
  ~AllocScope() { g_alloc = prev; }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
};

// Set while the allocation-free entry point runs: a device allocation there is a library
// bug, reported as an error instead of being made.
inline thread_local bool g_no_alloc = false;
struct NoAllocScope {
  bool prev;
  NoAllocScope() : prev(g_no_alloc) { g_no_alloc = true; }
  ~NoAllocScope() { g_no_alloc = prev; }
  NoAllocScope(const NoAllocScope&) = delete;
  NoAllocScope& operator=(const NoAllocScope&) = delete;
};

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  amgf_allocator src{};          // null alloc: the block came from hipMalloc
  hipStream_t src_s = nullptr;
  DBuf() = default;
  explicit DBuf(size_t count) { alloc(count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), src(o.src), src_s(o.src_s) {
    o.p = nullptr;
    o.n = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      src = o.src;
      src_s = o.src_s;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (!count) return;
    if (g_no_alloc)
      throw Error(AMGF_EDEVICE, "internal: device allocation in the allocation-free entry point");
    const size_t bytes = count * sizeof(T);
    if (g_alloc && g_alloc->a.alloc) {
      void* q = g_alloc->a.alloc(bytes, g_alloc->s, g_alloc->a.ctx);
      if (!q) throw Error(AMGF_ENOMEM, "amgf_allocator.alloc returned NULL");
      src = g_alloc->a;
      src_s = g_alloc->s;
      p = static_cast<T*>(q);
      n = count;
      if (reinterpret_cast<uintptr_t>(q) % 256) {
        release();
        throw Error(AMGF_EINVAL, "amgf_allocator.alloc returned a block not 256-byte aligned");
      }
      return;
    }
    AMGF_HIP(hipMalloc(&p, bytes));
    n = count;
  }
  void release() {
    if (p) {
      if (src.alloc)
        src.free(p, src_s, src.ctx);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
    src = amgf_allocator{};
    src_s = nullptr;
  }
  size_t bytes() const { return n * sizeof(T); }
  operator T*() const { return p; }
};

// Block-row sparse matrix with br x bc row-major blocks and ascending columns.
// FP16 entries of a transfer block that one lane loads together (chunked FP16 copy)
constexpr int fp16_group(int n) { return n % 4 == 0 ? 4 : (n % 2 == 0 ? 2 : 1); }

struct BSR {
  int nrows = 0, ncols = 0, br = 0, bc = 0;
  int64_t nnzb = 0;
  DBuf<int> rowptr, col;
  DBuf<double> val;
  DBuf<float> val32;       // FP32 copy used by the mixed-precision V-cycle
  // FP16 copy (transfer operators of the mixed V-cycle).  Chunked (valh_chunked) where
  // the transfer kernel gives a block row a whole wavefront: chunks of 64 blocks, entry e
  // of block j at valh[64 N (j / 64) + 64 G (e / G) + G (j % 64) + e % G], N = br * bc
  // entries per block, G = fp16_group(N), so the lanes, which read consecutive blocks, read
  // one contiguous stretch per load (nnzb rounded up to whole chunks); otherwise row-major
  // blocks like val (lanes of short rows read a few blocks each)
  DBuf<_Float16> valh;
  bool valh_chunked = false;
  // Sliced-ELL copy of a 3x3 matrix for the apply phase (built by bsr_build_sell):
  // slices of 64 block rows, each padded to its longest row.  Slot j of slice s holds
  // the column ids at sell_col[sell_off[s] + 64 j + i] and entry (p,q) of row i's block
  // at sell_val[9 (sell_off[s] + 64 j) + 64 (3p+q) + i]; padding has value 0.
  DBuf<int> sell_off, sell_col;
  DBuf<int16_t> sell_dcol;  // column id - row as int16, when every stored block fits
  DBuf<double> sell_val;
  DBuf<float> sell_val32;
  // BF16 copy (round to nearest even): per slot, entries (0,1) (2,3) (4,5) (6,7) of the
  // 64 rows as 4 x 64 packed pairs (uint32), then entry 8 as 64 uint16: 1152 bytes
  DBuf<uint16_t> sell_val16;
  // Packed copy of a square matrix (bsr_build_packed): row i's blocks padded with zero
  // blocks to a multiple of 16 from block offset pk_off[i], column ids pk_col[pk_off[i] + k]
  // (padding: i), entry e = b*p+q of block k at
  // pk_val[b*b*pk_off[i] + ((e / G) * nbp_i + k) * G + e % G], G the entries in 16 bytes
  // when b*b is a multiple of it, else 1
  DBuf<int> pk_off, pk_col;
  DBuf<double> pk_val;
  DBuf<float> pk_val32;
  size_t bsz() const { return size_t(br) * bc; }
};

// per-stream context passed to every host helper
struct Ctx {
  hipStream_t s = nullptr;
  DBuf<int> flag;          // device error/capacity flag
  DBuf<double> dot;        // partial sums of the deterministic dot products
};

// ------------------------------------------------------------------------------------
// small host helpers
// ------------------------------------------------------------------------------------
template <class T>
inline T d2h_scalar(const T* dptr, hipStream_t s) {
  T v;
  AMGF_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
  AMGF_HIP(hipStreamSynchronize(s));
  return v;
}
template <class T>
inline std::vector<T> d2h(const T* dptr, size_t n, hipStream_t s) {
  std::vector<T> v(n);
  if (n) {
    AMGF_HIP(hipMemcpyAsync(v.data(), dptr, n * sizeof(T), hipMemcpyDeviceToHost, s));
    AMGF_HIP(hipStreamSynchronize(s));
  }
  return v;
}
inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return unsigned(g < 1 ? 1 : g);
}

// ------------------------------------------------------------------------------------
// device helpers
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// Separately rounded FP64 multiply and add.  Contraction into FMA is switched off in
// these bodies (the HIP intrinsics of the same name are plain operators that the
// compiler may fuse), so results match a reference that rounds every operation.
__device__ __forceinline__ double mul_rn(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ double add_rn(double a, double b) {
#pragma clang fp contract(off)
  return a + b;
}

// Load of data a kernel streams through once (matrix values and column ids): marked
// non-temporal, so it does not displace the vectors the kernel gathers again and again
// (at C5 the level-0 FP32 SpMV went from 0.80 to 0.71 ms per launch).  Only for loads
// whose cache lines one wave instruction consumes whole (lane-contiguous layouts): the
// line is not kept, so a later instruction reading the rest of it goes back to HBM (the
// row-per-lane-group BSR kernels ran 2.5x slower with it).
template <class T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// LDS written by some lanes of a wavefront, then read by others of the same wavefront
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
template <class T>
__device__ __forceinline__ T group_sum(T v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}

// ------------------------------------------------------------------------------------
// primitives (primitives.hip)
// ------------------------------------------------------------------------------------
// out[0..n] = exclusive scan of in[0..n-1]; out[n] = total.  Returns the total.
int scan_exclusive(Ctx& c, const int* in, int* out, int n, bool want_total = true);
// longest segment off[s+1] - off[s] of nseg segments (0 when none); waits for the result
int max_segment_length(Ctx& c, const int* off, int nseg);
// rows[k] = block row of block k, for a CSR rowptr of nrows rows
void expand_rows(Ctx& c, const int* rowptr, int nrows, int* rows);
// Deterministic grouping: for keys[i] in [0, nkeys) (negative keys skipped),
// offsets[nkeys+1] and perm[] listing the indices i of each key in ascending order.
void group_by_key(Ctx& c, const int* keys, int n, int nkeys, DBuf<int>& offsets,
                  DBuf<int>& perm, bool sorted = true);
// Transpose a BSR matrix (blocks transposed too).  Deterministic.
void bsr_transpose(Ctx& c, const BSR& A, BSR& T);
// Symbolic union: row r of C collects map(col2[u]) for u in rows col1[t] of the inner
// CSR, t in row r of the outer CSR (inner == nullptr: map(col1[t]) directly).
// Negative mapped ids are skipped; exclude_diag drops id == r; row_mask (optional)
// selects the rows that get entries.  Produces C.rowptr / C.col (sorted).
void union_symbolic(Ctx& c, int nrows, int ncols, const int* rp1, const int* col1,
                    const int* rp2, const int* col2, const int* map, bool exclude_diag,
                    const int* row_mask, BSR& C);
// C = A + B pattern union (sorted merge) and exact values (A + B where both exist).
void bsr_add(Ctx& c, const BSR& A, const BSR& B, BSR& C);

}  // namespace amgf

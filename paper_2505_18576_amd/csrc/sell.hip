// Sliced-ELL copies of the level-0 stiffness and their SpMV kernels (FP64, FP32 and
// BF16 values): the V-cycle's smoothing steps and the CG operator spend most of the
// solve here.
#include <climits>

#include "apply.h"

namespace amgf {

// ======================================================================================
// Sliced-ELL SpMV for 3x3 blocks: one wave per slice of 64 block rows, lane i owns row
// 64 s + i.  For every slot the wave reads 64 column ids, 9 x 64 values (contiguous) and
// the three x entries of each column; neighbouring rows of a structured mesh have
// neighbouring columns, so the x reads coalesce too.  No cross-lane reduction.  SHORT:
// the column ids are 16-bit offsets from the row (128 B per slot instead of 256 B), used
// when every stored block lies within 32767 block columns of its row.
// ======================================================================================
template <bool SHORT>
__device__ __forceinline__ int64_t sell_col3(const int* __restrict__ cp,
                                             const int16_t* __restrict__ dp, int r, int j) {
  if constexpr (SHORT) return (int64_t(r) + ld_stream(&dp[j * 64])) * 3;
  else return int64_t(ld_stream(&cp[j * 64])) * 3;
}

template <class T, int MODE, bool SHORT>
__global__ void __launch_bounds__(256) k_sell3(int nrows, const int* __restrict__ off,
                                               const int* __restrict__ scol,
                                               const int16_t* __restrict__ sdcol,
                                               const T* __restrict__ sval,
                                               const T* __restrict__ x, T* __restrict__ y,
                                               const T* __restrict__ b,
                                               const T* __restrict__ w, T* __restrict__ xo) {
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int i = threadIdx.x & 63;
  if (int64_t(s) * 64 >= nrows) return;
  const int o0 = off[s];
  const int len = (off[s + 1] - o0) >> 6;
  const int* cp = SHORT ? nullptr : scol + o0 + i;
  const int16_t* dp = SHORT ? sdcol + o0 + i : nullptr;
  const int rr = s * 64 + i;
  const T* vp = sval + int64_t(o0) * 9 + i;
  T a0 = T(0), a1 = T(0), a2 = T(0);
  // FP64 blocks take two more iterations in flight: 1.56 -> 1.50 ms at 114M blocks,
  // while FP32 is unchanged by it
  constexpr int UNROLL = sizeof(T) == 8 ? 6 : 3;
#pragma unroll UNROLL
  for (int j = 0; j < len; ++j) {
    const int64_t cc = sell_col3<SHORT>(cp, dp, rr, j);
    T x0, x1, x2;
    if (MODE == SPMV_PRE) {
      x0 = w[cc] * b[cc];
      x1 = w[cc + 1] * b[cc + 1];
      x2 = w[cc + 2] * b[cc + 2];
    } else {
      x0 = x[cc];
      x1 = x[cc + 1];
      x2 = x[cc + 2];
    }
    const T* v = vp + int64_t(j) * 576;
    a0 += ld_stream(v) * x0 + ld_stream(v + 64) * x1 + ld_stream(v + 128) * x2;
    a1 += ld_stream(v + 192) * x0 + ld_stream(v + 256) * x1 + ld_stream(v + 320) * x2;
    a2 += ld_stream(v + 384) * x0 + ld_stream(v + 448) * x1 + ld_stream(v + 512) * x2;
  }
  const int r = s * 64 + i;
  if (r >= nrows) return;
  const T ax[3] = {a0, a1, a2};
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int64_t k = int64_t(r) * 3 + p;
    if (MODE == SPMV_Y) y[k] = ax[p];
    else if (MODE == SPMV_ADD) y[k] += ax[p];
    else if (MODE == SPMV_PRE) {
      const T bk = b[k];
      xo[k] = w[k] * bk;
      y[k] = bk - ax[p];
    } else if (MODE == SPMV_POST) {
      xo[k] = x[k] + w[k] * (b[k] - ax[p]);
    } else {
      y[k] = b[k] - ax[p];
    }
  }
}

__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xFFFF0000u); }

template <int MODE, bool SHORT>
__global__ void __launch_bounds__(256) k_sell3_bf16(int nrows, const int* __restrict__ off,
                                                    const int* __restrict__ scol,
                                                    const int16_t* __restrict__ sdcol,
                                                    const uint16_t* __restrict__ sval,
                                                    const float* __restrict__ x,
                                                    float* __restrict__ y,
                                                    const float* __restrict__ b,
                                                    const float* __restrict__ w,
                                                    float* __restrict__ xo) {
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int i = threadIdx.x & 63;
  if (int64_t(s) * 64 >= nrows) return;
  const int o0 = off[s];
  const int len = (off[s + 1] - o0) >> 6;
  const int* cp = SHORT ? nullptr : scol + o0 + i;
  const int16_t* dp = SHORT ? sdcol + o0 + i : nullptr;
  const int rr = s * 64 + i;
  const uint16_t* vs = sval + int64_t(o0) * 9;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll 3
  for (int j = 0; j < len; ++j) {
    const int64_t cc = sell_col3<SHORT>(cp, dp, rr, j);
    float x0, x1, x2;
    if (MODE == SPMV_PRE) {
      x0 = w[cc] * b[cc];
      x1 = w[cc + 1] * b[cc + 1];
      x2 = w[cc + 2] * b[cc + 2];
    } else {
      x0 = x[cc];
      x1 = x[cc + 1];
      x2 = x[cc + 2];
    }
    const uint16_t* slot = vs + int64_t(j) * 576;
    const uint32_t* pr = reinterpret_cast<const uint32_t*>(slot) + i;
    const uint32_t e01 = ld_stream(pr), e23 = ld_stream(pr + 64), e45 = ld_stream(pr + 128),
                   e67 = ld_stream(pr + 192);
    const float e8 = __uint_as_float(uint32_t(ld_stream(slot + 512 + i)) << 16);
    a0 += bf16_lo(e01) * x0 + bf16_hi(e01) * x1 + bf16_lo(e23) * x2;
    a1 += bf16_hi(e23) * x0 + bf16_lo(e45) * x1 + bf16_hi(e45) * x2;
    a2 += bf16_lo(e67) * x0 + bf16_hi(e67) * x1 + e8 * x2;
  }
  const int r = s * 64 + i;
  if (r >= nrows) return;
  const float ax[3] = {a0, a1, a2};
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const int64_t k = int64_t(r) * 3 + p;
    if (MODE == SPMV_Y) y[k] = ax[p];
    else if (MODE == SPMV_ADD) y[k] += ax[p];
    else if (MODE == SPMV_PRE) {
      const float bk = b[k];
      xo[k] = w[k] * bk;
      y[k] = bk - ax[p];
    } else if (MODE == SPMV_POST) {
      xo[k] = x[k] + w[k] * (b[k] - ax[p]);
    } else {
      y[k] = b[k] - ax[p];
    }
  }
}

// FP64 -> BF16 with one rounding to nearest even: truncate to FP32, mark inexactness in
// the last bit (round to odd, 16 spare bits), then round the FP32 bits to BF16.
__device__ __forceinline__ uint16_t bf16_rne(double v) {
  float f = __double2float_rz(v);
  uint32_t u = __float_as_uint(f);
  if (double(f) != v) u |= 1u;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

__global__ void k_sell_len(int nrows, int nslices, const int* __restrict__ rp,
                           int* __restrict__ len) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nslices) return;
  if (s == nslices) { len[s] = 0; return; }
  int m = 0;
  const int r1 = min(nrows, (s + 1) * 64);
  for (int r = s * 64; r < r1; ++r) m = max(m, rp[r + 1] - rp[r]);
  len[s] = m * 64;
}

// One workgroup per slice.  Eight slots at a time: the 64 rows' runs of 8 blocks are read
// in BSR order (each run is contiguous) into LDS, then written slot by slot in the sliced
// layout, so both the reads and the writes are coalesced.
constexpr int FILL_SLOTS = 8;
__global__ void __launch_bounds__(256) k_sell_fill(int nrows, const int* __restrict__ rp,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const int* __restrict__ off,
                                                   int* __restrict__ scol,
                                                   double* __restrict__ sv,
                                                   float* __restrict__ sv32,
                                                   uint16_t* __restrict__ sv16) {
  __shared__ double stage[FILL_SLOTS][9][65];
  __shared__ int cstage[FILL_SLOTS][64];
  __shared__ int rpo[65];
  const int s = blockIdx.x, tid = threadIdx.x;
  const int r0 = s * 64;
  for (int t = tid; t <= 64; t += 256) rpo[t] = rp[min(r0 + t, nrows)];
  __syncthreads();
  const int o0 = off[s], len = (off[s + 1] - o0) >> 6;
  for (int j0 = 0; j0 < len; j0 += FILL_SLOTS) {
    for (int e = tid; e < 64 * FILL_SLOTS * 9; e += 256) {
      const int i = e / (FILL_SLOTS * 9), rem = e % (FILL_SLOTS * 9);
      const int jj = rem / 9, q = rem % 9, j = j0 + jj;
      const int rl = rpo[i + 1] - rpo[i];
      stage[jj][q][i] = j < rl ? val[int64_t(rpo[i] + j) * 9 + q] : 0.0;
    }
    for (int e = tid; e < 64 * FILL_SLOTS; e += 256) {
      const int i = e / FILL_SLOTS, jj = e % FILL_SLOTS, j = j0 + jj;
      const int rl = rpo[i + 1] - rpo[i];
      cstage[jj][i] = j < rl ? col[rpo[i] + j] : min(r0 + i, nrows - 1);
    }
    __syncthreads();
    const int nslot = min(FILL_SLOTS, len - j0);
    for (int e = tid; e < nslot * 64; e += 256) {
      const int jj = e >> 6, i = e & 63;
      scol[int64_t(o0) + int64_t(j0 + jj) * 64 + i] = cstage[jj][i];
    }
    for (int e = tid; e < nslot * 576; e += 256) {
      const int jj = e / 576, pos = e % 576;
      const int64_t base = (int64_t(o0) + int64_t(j0 + jj) * 64) * 9;
      const int q = pos >> 6, i = pos & 63;
      const double v = stage[jj][q][i];
      if (sv) sv[base + pos] = v;
      if (sv32) sv32[base + pos] = float(v);
      if (sv16) {
        // pairs (2q, 2q+1) packed in uint32 q of the slot, entry 8 after the pairs
        const int qq = pos < 512 ? 2 * (pos >> 7) + (pos & 1) : 8;
        const int ii = pos < 512 ? (pos & 127) >> 1 : pos - 512;
        sv16[base + pos] = bf16_rne(stage[jj][qq][ii]);
      }
    }
    __syncthreads();
  }
}

// 16-bit column offsets from the row; flag bit 1 when one does not fit
__global__ void __launch_bounds__(64) k_sell_delta(const int* __restrict__ off,
                                                   const int* __restrict__ scol,
                                                   int16_t* __restrict__ dcol,
                                                   int* __restrict__ flag) {
  const int s = blockIdx.x, i = threadIdx.x;
  const int o0 = off[s], len = (off[s + 1] - o0) >> 6;
  const int r = s * 64 + i;
  bool bad = false;
  for (int j = 0; j < len; ++j) {
    const int d = scol[o0 + j * 64 + i] - r;
    bad = bad || d < -32768 || d > 32767;
    dcol[o0 + j * 64 + i] = int16_t(bad ? 0 : d);
  }
  if (bad) atomicOr(flag, 1);
}

void bsr_build_sell(Ctx& c, BSR& A, bool fp64, bool fp32, bool bf16) {
  AMGF_REQUIRE(A.br == 3 && A.bc == 3, AMGF_EINVAL, "sliced ELL needs 3x3 blocks");
  if (A.nrows == 0) return;
  const int ns = (A.nrows + 63) / 64;
  DBuf<int> len(ns + 1);
  hipLaunchKernelGGL(k_sell_len, dim3(grid_for(ns + 1, 256)), dim3(256), 0, c.s, A.nrows, ns,
                     A.rowptr.p, len.p);
  AMGF_LAUNCH_CHECK();
  A.sell_off.alloc(ns + 2);
  const int total = scan_exclusive(c, len.p, A.sell_off.p, ns + 1);
  A.sell_col.alloc(size_t(total));
  if (fp64) A.sell_val.alloc(size_t(total) * 9);
  if (fp32) A.sell_val32.alloc(size_t(total) * 9);
  if (bf16) A.sell_val16.alloc(size_t(total) * 9);
  hipLaunchKernelGGL(k_sell_fill, dim3(ns), dim3(256), 0, c.s, A.nrows, A.rowptr.p, A.col.p,
                     A.val.p, A.sell_off.p, A.sell_col.p, A.sell_val.p, A.sell_val32.p,
                     A.sell_val16.p);
  AMGF_LAUNCH_CHECK();
  // 16-bit offsets when the bandwidth allows (2 bytes less per stored block)
  A.sell_dcol.alloc(size_t(total));
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  hipLaunchKernelGGL(k_sell_delta, dim3(ns), dim3(64), 0, c.s, A.sell_off.p, A.sell_col.p,
                     A.sell_dcol.p, c.flag.p);
  AMGF_LAUNCH_CHECK();
  if (d2h_scalar(c.flag.p, c.s) != 0) A.sell_dcol.release();
}

template <class T>
void sell3_spmv(Ctx& c, int mode, const BSR& A, const T* sval, const T* x, T* y, const T* b,
                const T* w, T* xo) {
  const int ns = (A.nrows + 63) / 64;
  const dim3 g((ns + 3) / 4), blk(256);
  switch (mode) {
#define AMGF_MODE(MD)                                                                        \
  case MD:                                                                                   \
    if (A.sell_dcol.p)                                                                       \
      hipLaunchKernelGGL((k_sell3<T, MD, true>), g, blk, 0, c.s, A.nrows, A.sell_off.p,      \
                         A.sell_col.p, A.sell_dcol.p, sval, x, y, b, w, xo);                 \
    else                                                                                     \
      hipLaunchKernelGGL((k_sell3<T, MD, false>), g, blk, 0, c.s, A.nrows, A.sell_off.p,     \
                         A.sell_col.p, A.sell_dcol.p, sval, x, y, b, w, xo);                 \
    break;
    AMGF_MODE(SPMV_Y)
    AMGF_MODE(SPMV_ADD)
    AMGF_MODE(SPMV_PRE)
    AMGF_MODE(SPMV_POST)
    AMGF_MODE(SPMV_RES)
#undef AMGF_MODE
    default:
      throw Error(AMGF_EINVAL, "spmv mode");
  }
  AMGF_LAUNCH_CHECK();
}

template void sell3_spmv<double>(Ctx&, int, const BSR&, const double*, const double*, double*,
                                 const double*, const double*, double*);
template void sell3_spmv<float>(Ctx&, int, const BSR&, const float*, const float*, float*,
                                const float*, const float*, float*);

void sell_spmv_bf16(Ctx& c, int mode, const BSR& A, const float* x, float* y, const float* b,
                    const float* w, float* xo) {
  AMGF_REQUIRE(A.sell_val16.p, AMGF_EINVAL, "no BF16 sliced copy");
  if (A.nrows == 0) return;
  const int ns = (A.nrows + 63) / 64;
  const dim3 g((ns + 3) / 4), blk(256);
  switch (mode) {
#define AMGF_MODE(MD)                                                                        \
  case MD:                                                                                   \
    if (A.sell_dcol.p)                                                                       \
      hipLaunchKernelGGL((k_sell3_bf16<MD, true>), g, blk, 0, c.s, A.nrows, A.sell_off.p,    \
                         A.sell_col.p, A.sell_dcol.p, A.sell_val16.p, x, y, b, w, xo);       \
    else                                                                                     \
      hipLaunchKernelGGL((k_sell3_bf16<MD, false>), g, blk, 0, c.s, A.nrows, A.sell_off.p,   \
                         A.sell_col.p, A.sell_dcol.p, A.sell_val16.p, x, y, b, w, xo);       \
    break;
    AMGF_MODE(SPMV_Y)
    AMGF_MODE(SPMV_ADD)
    AMGF_MODE(SPMV_PRE)
    AMGF_MODE(SPMV_POST)
    AMGF_MODE(SPMV_RES)
#undef AMGF_MODE
    default:
      throw Error(AMGF_EINVAL, "spmv mode");
  }
  AMGF_LAUNCH_CHECK();
}

}  // namespace amgf

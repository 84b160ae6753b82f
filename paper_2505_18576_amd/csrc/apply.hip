// Apply-phase kernels: the V-cycle, the filter correction and the CG loop are built
// from these.  All are memory-bound; reductions are two-stage with a fixed
// assignment of elements to lanes, so results do not depend on scheduling.
#include <type_traits>

#include "apply.h"

namespace amgf {

// ======================================================================================
// BSR SpMV with fused smoother modes
// ======================================================================================
// one block's N values widened to T, value by value (FP32 and FP64 copies: block j at
// N j)
template <int N, class T, class TV>
__device__ __forceinline__ void load_block(const TV* __restrict__ v, T* out) {
#pragma unroll
  for (int k = 0; k < N; ++k) out[k] = T(v[k]);
}

// block j of a row-major FP16 copy widened to T, two values per load (N even: the block
// starts on a 4-byte boundary)
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
template <int N, class T>
__device__ __forceinline__ void load_block_h(const _Float16* __restrict__ v, T* out) {
  if constexpr (N % 2 == 0) {
    const half2v* v2 = reinterpret_cast<const half2v*>(v);
#pragma unroll
    for (int k = 0; k < N / 2; ++k) {
      const half2v h = v2[k];
      out[2 * k] = T(h.x);
      out[2 * k + 1] = T(h.y);
    }
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = T(v[k]);
  }
}

// block j of a chunked FP16 copy (BSR::valh) widened to T: N / G loads of G values, each
// reading the same G entries of the chunk's 64 blocks side by side
template <int N, class T>
__device__ __forceinline__ void load_block_chunked(const _Float16* __restrict__ val, int64_t j,
                                                   T* out) {
  constexpr int G = fp16_group(N);
  typedef _Float16 hG __attribute__((ext_vector_type(G)));
  const hG* base = reinterpret_cast<const hG*>(val + (j >> 6) * (64 * N)) + (j & 63);
#pragma unroll
  for (int g = 0; g < N / G; ++g) {
    const hG h = base[64 * g];
#pragma unroll
    for (int u = 0; u < G; ++u) out[g * G + u] = T(h[u]);
  }
}

// G lanes cooperate on one block row; lane l takes blocks l, l+G, ...; the BR partial
// row sums are reduced across the G lanes and lane p < BR writes output p.  Values of type
// TV (T, or FP16 for the transfer operators) are widened to T.
template <int BR, int BC, int G, class T, int MODE, class TV = T>
__global__ void __launch_bounds__(256) k_bsr(int nrows, const int* __restrict__ rp,
                                             const int* __restrict__ col,
                                             const TV* __restrict__ val, const T* __restrict__ x,
                                             T* __restrict__ y, const T* __restrict__ b,
                                             const T* __restrict__ w, T* __restrict__ xo) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = gid / G, l = gid % G;
  if (r >= nrows) return;
  T acc[BR];
#pragma unroll
  for (int p = 0; p < BR; ++p) acc[p] = T(0);
  const int j1 = rp[r + 1];
  for (int j = rp[r] + l; j < j1; j += G) {
    const int cc = col[j];
    T xv[BC];
#pragma unroll
    for (int q = 0; q < BC; ++q) {
      const int64_t ix = int64_t(cc) * BC + q;
      xv[q] = (MODE == SPMV_PRE) ? w[ix] * b[ix] : x[ix];
    }
    T v[BR * BC];
    if constexpr (std::is_same_v<TV, _Float16> && G == 64)
      load_block_chunked<BR * BC>(val, j, v);
    else if constexpr (std::is_same_v<TV, _Float16>)
      load_block_h<BR * BC>(val + int64_t(j) * (BR * BC), v);
    else
      load_block<BR * BC>(val + int64_t(j) * (BR * BC), v);
#pragma unroll
    for (int p = 0; p < BR; ++p)
#pragma unroll
      for (int q = 0; q < BC; ++q) acc[p] += v[p * BC + q] * xv[q];
  }
#pragma unroll
  for (int p = 0; p < BR; ++p) acc[p] = group_sum(acc[p], G);
  if (l >= BR) return;
  T ax = T(0);
#pragma unroll
  for (int p = 0; p < BR; ++p)
    if (l == p) ax = acc[p];
  const int64_t i = int64_t(r) * BR + l;
  if (MODE == SPMV_Y) y[i] = ax;
  else if (MODE == SPMV_YW) {
    y[i] = ax;
    xo[i] = w[i] * ax;
  } else if (MODE == SPMV_ADD) y[i] += ax;
  else if (MODE == SPMV_PRE) {
    const T xi = w[i] * b[i];
    xo[i] = xi;
    y[i] = b[i] - ax;
  } else if (MODE == SPMV_POST) {
    xo[i] = x[i] + w[i] * (b[i] - ax);
  } else {
    y[i] = b[i] - ax;
  }
}

// y[i] = b[i] - (A x)[i] on the listed block rows only (FP64 arithmetic, 3x3 blocks; x
// FP64 or FP32, widened exactly)
template <class TX>
__global__ void __launch_bounds__(256) k_bsr_res_rows(int nlist, const int* __restrict__ rows,
                                                      const int* __restrict__ rp,
                                                      const int* __restrict__ col,
                                                      const double* __restrict__ val,
                                                      const TX* __restrict__ x,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ y) {
  constexpr int G = 8;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int li = gid / G, l = gid % G;
  if (li >= nlist) return;
  const int r = rows[li];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int j = rp[r] + l; j < rp[r + 1]; j += G) {
    const int cc = col[j];
    const double* v = val + int64_t(j) * 9;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[p] += v[p * 3 + q] * double(x[int64_t(cc) * 3 + q]);
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) acc[p] = group_sum(acc[p], G);
  if (l >= 3) return;
  double ax = l == 0 ? acc[0] : (l == 1 ? acc[1] : acc[2]);
  const int64_t i = int64_t(r) * 3 + l;
  y[i] = b[i] - ax;
}

template <class TX>
void bsr_res_rows(Ctx& c, const BSR& A, const int* rows, int nlist, const TX* x,
                  const double* b, double* y) {
  if (nlist == 0) return;
  hipLaunchKernelGGL(k_bsr_res_rows<TX>, dim3(grid_for(int64_t(nlist) * 8, 256)), dim3(256), 0,
                     c.s, nlist, rows, A.rowptr.p, A.col.p, A.val.p, x, b, y);
  AMGF_LAUNCH_CHECK();
}
template void bsr_res_rows<double>(Ctx&, const BSR&, const int*, int, const double*,
                                   const double*, double*);
template void bsr_res_rows<float>(Ctx&, const BSR&, const int*, int, const float*,
                                  const double*, double*);

template <int BR, int BC, int G, class T>
static void launch_bsr(Ctx& c, int mode, const BSR& A, const T* val, const T* x, T* y,
                       const T* b, const T* w, T* xo) {
  const int64_t threads = int64_t(A.nrows) * G;
  const dim3 g(grid_for(threads, 256)), blk(256);
  switch (mode) {
#define AMGF_MODE(MD)                                                                        \
  case MD:                                                                                   \
    hipLaunchKernelGGL((k_bsr<BR, BC, G, T, MD>), g, blk, 0, c.s, A.nrows, A.rowptr.p,       \
                       A.col.p, val, x, y, b, w, xo);                                        \
    break;
    AMGF_MODE(SPMV_Y)
    AMGF_MODE(SPMV_ADD)
    AMGF_MODE(SPMV_PRE)
    AMGF_MODE(SPMV_POST)
    AMGF_MODE(SPMV_RES)
    AMGF_MODE(SPMV_YW)
#undef AMGF_MODE
    default:
      throw Error(AMGF_EINVAL, "spmv mode");
  }
  AMGF_LAUNCH_CHECK();
}

// y = A x, y += A x or y = A x with xo = w.y, FP16 values (the mixed V-cycle's restriction
// and prolongation)
template <int BR, int BC, int G>
static void launch_bsr_h(Ctx& c, int mode, const BSR& A, const float* x, float* y,
                         const float* w, float* xo) {
  const int64_t threads = int64_t(A.nrows) * G;
  const dim3 g(grid_for(threads, 256)), blk(256);
  if (mode == SPMV_Y)
    hipLaunchKernelGGL((k_bsr<BR, BC, G, float, SPMV_Y, _Float16>), g, blk, 0, c.s, A.nrows,
                       A.rowptr.p, A.col.p, A.valh.p, x, y, nullptr, nullptr, nullptr);
  else if (mode == SPMV_YW)
    hipLaunchKernelGGL((k_bsr<BR, BC, G, float, SPMV_YW, _Float16>), g, blk, 0, c.s, A.nrows,
                       A.rowptr.p, A.col.p, A.valh.p, x, y, nullptr, w, xo);
  else if (mode == SPMV_ADD)
    hipLaunchKernelGGL((k_bsr<BR, BC, G, float, SPMV_ADD, _Float16>), g, blk, 0, c.s, A.nrows,
                       A.rowptr.p, A.col.p, A.valh.p, x, y, nullptr, nullptr, nullptr);
  else
    throw Error(AMGF_EINVAL, "FP16 spmv mode");
  AMGF_LAUNCH_CHECK();
}

// lanes per block row of the FP16 transfer kernel for this operator's shape and density
int transfer_lanes(const BSR& A) {
  if (A.br == 6 && A.bc == 3) return 64;
  if (A.br == 6 && A.bc == 6) return A.nrows > 0 && double(A.nnzb) / A.nrows > 24 ? 64 : 16;
  return 8;
}

void transfer_spmv(Ctx& c, int mode, const BSR& A, const float* x, float* y, const float* w,
                   float* xo) {
  if (A.nrows == 0) return;
  if (!A.valh.p) return bsr_spmv<float>(c, mode, A, A.val32.p, x, y, nullptr, w, xo);
  const double avg = double(A.nnzb) / A.nrows;
  AMGF_REQUIRE(A.valh_chunked == (transfer_lanes(A) == 64), AMGF_EDEVICE,
               "FP16 copy laid out for another launch");
  if (A.br == 3 && A.bc == 3) return launch_bsr_h<3, 3, 8>(c, mode, A, x, y, w, xo);
  if (A.br == 3 && A.bc == 6) return launch_bsr_h<3, 6, 8>(c, mode, A, x, y, w, xo);
  if (A.br == 6 && A.bc == 3) return launch_bsr_h<6, 3, 64>(c, mode, A, x, y, w, xo);
  if (A.br == 6 && A.bc == 6) {
    if (avg > 24) return launch_bsr_h<6, 6, 64>(c, mode, A, x, y, w, xo);
    return launch_bsr_h<6, 6, 16>(c, mode, A, x, y, w, xo);
  }
  throw Error(AMGF_EINVAL, "FP16 spmv block size");
}

// FP64 -> FP16 with one rounding to nearest even (truncate to FP32, mark inexactness in the
// last bit, then the hardware's nearest-even FP32 -> FP16) into the chunked layout of
// BSR::valh (nb blocks of N entries); flag bit 1 on a non-finite result (a value beyond the
// FP16 range)
__global__ void k_d2h_chunked(const double* __restrict__ a, _Float16* __restrict__ b,
                              int64_t nb, int N, int G, int* __restrict__ flag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nb * N) return;
  const int64_t j = i / N;
  const int e = int(i % N);
  const double v = a[i];
  float f = __double2float_rz(v);
  if (double(f) != v) f = __uint_as_float(__float_as_uint(f) | 1u);
  const _Float16 h = _Float16(f);
  b[(j >> 6) * (64 * N) + (e / G) * (64 * G) + (j & 63) * G + e % G] = h;
  if (!__builtin_isfinite(float(h))) atomicOr(flag, 1);
}
__global__ void k_d2h(const double* __restrict__ a, _Float16* __restrict__ b, int64_t n,
                      int* __restrict__ flag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = a[i];
  float f = __double2float_rz(v);
  if (double(f) != v) f = __uint_as_float(__float_as_uint(f) | 1u);
  const _Float16 h = _Float16(f);
  b[i] = h;
  if (!__builtin_isfinite(float(h))) atomicOr(flag, 1);
}
void cast_d2h_transfer(Ctx& c, BSR& A, int* flag) {
  const int N = int(A.bsz());
  A.valh_chunked = transfer_lanes(A) == 64;
  if (A.valh_chunked) {
    A.valh.alloc(size_t((std::max<int64_t>(A.nnzb, 1) + 63) / 64 * 64) * N);
    cast_d2h_chunked(c, A.val.p, A.valh.p, A.nnzb, N, flag);
    return;
  }
  A.valh.alloc(size_t(std::max<int64_t>(A.nnzb, 1)) * N);
  if (A.nnzb)
    hipLaunchKernelGGL(k_d2h, dim3(grid_for(A.nnzb * N, 256)), dim3(256), 0, c.s, A.val.p,
                       A.valh.p, A.nnzb * N, flag);
  AMGF_LAUNCH_CHECK();
}
void cast_d2h_chunked(Ctx& c, const double* a, _Float16* b, int64_t nb, int N, int* flag) {
  if (nb)
    hipLaunchKernelGGL(k_d2h_chunked, dim3(grid_for(nb * N, 256)), dim3(256), 0, c.s, a, b, nb,
                       N, fp16_group(N), flag);
  AMGF_LAUNCH_CHECK();
}

template <int B, class TV, class T>
static void launch_packed(Ctx& c, int mode, const BSR& A, const TV* pv, const T* x, T* y,
                          const T* b, const T* w, T* xo);

template <class T>
void bsr_spmv(Ctx& c, int mode, const BSR& A, const T* val, const T* x, T* y, const T* b,
              const T* w, T* xo) {
  if (A.nrows == 0) return;
  const double avg = A.nrows ? double(A.nnzb) / A.nrows : 0.0;
  const bool plain_modes = mode != SPMV_YW;           // the copies below serve modes 0..4
  if (plain_modes && A.br == 3 && A.bc == 3 && A.sell_col.p) {
    // the sliced copy stands in for the BSR values of the same precision
    const T* sv = nullptr;
    if constexpr (sizeof(T) == 8) {
      if (val == A.val.p) sv = A.sell_val.p;
    } else {
      sv = A.sell_val32.p;     // level matrices keep no FP32 BSR values once sliced
    }
    if (sv) return sell3_spmv<T>(c, mode, A, sv, x, y, b, w, xo);
  }
  if (plain_modes && A.br == A.bc && (A.br == 6 || A.br == 3) && A.pk_off.p) {
    // the packed copy stands in for the BSR values of the same precision
#define AMGF_PK(TV, vp)                                                                      \
  return A.br == 6 ? launch_packed<6, TV, T>(c, mode, A, vp, x, y, b, w, xo)                \
                   : launch_packed<3, TV, T>(c, mode, A, vp, x, y, b, w, xo)
    if constexpr (sizeof(T) == 8) {
      if (val == A.val.p && A.pk_val.p) AMGF_PK(double, A.pk_val.p);
    } else {
      if (val == A.val32.p && A.pk_val32.p) AMGF_PK(float, A.pk_val32.p);
      // a matrix kept in FP64 only (a smoothing matrix that holds the contact term)
      if (val == nullptr && !A.val32.p && A.pk_val.p) AMGF_PK(double, A.pk_val.p);
    }
#undef AMGF_PK
  }
  if (A.br == 3 && A.bc == 3) return launch_bsr<3, 3, 8, T>(c, mode, A, val, x, y, b, w, xo);
  if (A.br == 3 && A.bc == 6) return launch_bsr<3, 6, 8, T>(c, mode, A, val, x, y, b, w, xo);
  if (A.br == 6 && A.bc == 3) return launch_bsr<6, 3, 64, T>(c, mode, A, val, x, y, b, w, xo);
  if (A.br == 6 && A.bc == 6) {
    if (avg > 24) return launch_bsr<6, 6, 64, T>(c, mode, A, val, x, y, b, w, xo);
    return launch_bsr<6, 6, 16, T>(c, mode, A, val, x, y, b, w, xo);
  }
  throw Error(AMGF_EINVAL, "spmv block size");
}
template void bsr_spmv<double>(Ctx&, int, const BSR&, const double*, const double*, double*,
                               const double*, const double*, double*);
template void bsr_spmv<float>(Ctx&, int, const BSR&, const float*, const float*, float*,
                              const float*, const float*, float*);

// ======================================================================================
// contact term  J^T D J x  (always FP64)
// ======================================================================================
// Level-0 contact rows are short (a constraint touches about five nodes, a node a few
// constraints): CT_G lanes per row, eight rows per wavefront.
constexpr int CT_G = 8;

// t_k = D_k (J x)_k: CT_G lanes per constraint row, over the row's blocks.
template <int B, class TX>
__global__ void __launch_bounds__(256) k_contact_t(int m, const int* __restrict__ rp,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ D,
                                                   const TX* __restrict__ x,
                                                   double* __restrict__ t) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = gid / CT_G, lane = gid % CT_G;
  if (k >= m) return;
  double s = 0.0;
  for (int u = rp[k] + lane; u < rp[k + 1]; u += CT_G) {
    const int64_t base = int64_t(col[u]) * B;
#pragma unroll
    for (int q = 0; q < B; ++q) s += val[int64_t(u) * B + q] * double(x[base + q]);
  }
  s = group_sum(s, CT_G);
  if (lane == 0) t[k] = D[k] * s;
}

// y_a (op)= (J^T t)_a over the listed node rows: G lanes per row (CT_G for the short rows
// of the fine interface, a wavefront where a coarse node meets hundreds of constraints).
template <int B, class TY, int MODE, int G>
__global__ void __launch_bounds__(256) k_contact_y(int nrows, const int* __restrict__ rows,
                                                   const int* __restrict__ rp,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ t,
                                                   TY* __restrict__ y,
                                                   const TY* __restrict__ w) {
  static_assert(B <= G, "one lane per output component");
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid / G, lane = gid % G;
  if (i >= nrows) return;
  const int a = rows[i];
  double acc[B];
#pragma unroll
  for (int p = 0; p < B; ++p) acc[p] = 0.0;
  for (int k = rp[a] + lane; k < rp[a + 1]; k += G) {
    const double tk = t[col[k]];
#pragma unroll
    for (int p = 0; p < B; ++p) acc[p] += val[int64_t(k) * B + p] * tk;
  }
#pragma unroll
  for (int p = 0; p < B; ++p) acc[p] = group_sum(acc[p], G);
  if (lane >= B) return;
  double v = 0.0;
#pragma unroll
  for (int p = 0; p < B; ++p)
    if (lane == p) v = acc[p];
  const int64_t ix = int64_t(a) * B + lane;
  if (MODE == CT_SUB_RES) y[ix] = TY(double(y[ix]) - v);
  else if (MODE == CT_SUB_W) y[ix] = TY(double(y[ix]) - double(w[ix]) * v);
  else y[ix] = TY(double(y[ix]) + v);
}

template <int B, int G, class TY>
static void launch_contact_y(Ctx& c, int mode, const BSR& JT, const int* crows, int ncrows,
                             const double* t, TY* y, const TY* w) {
  const dim3 gn(grid_for(int64_t(ncrows) * G, 256)), blk(256);
  if (mode == CT_SUB_RES)
    hipLaunchKernelGGL((k_contact_y<B, TY, CT_SUB_RES, G>), gn, blk, 0, c.s, ncrows, crows,
                       JT.rowptr.p, JT.col.p, JT.val.p, t, y, w);
  else if (mode == CT_SUB_W)
    hipLaunchKernelGGL((k_contact_y<B, TY, CT_SUB_W, G>), gn, blk, 0, c.s, ncrows, crows,
                       JT.rowptr.p, JT.col.p, JT.val.p, t, y, w);
  else
    hipLaunchKernelGGL((k_contact_y<B, TY, CT_ADD, G>), gn, blk, 0, c.s, ncrows, crows,
                       JT.rowptr.p, JT.col.p, JT.val.p, t, y, w);
}

template <class TX, class TY>
void contact_apply(Ctx& c, int mode, const BSR& J, const BSR& JT, const int* crows, int ncrows,
                   const double* D, const TX* x, double* t, TY* y, const TY* w) {
  if (J.nrows == 0 || J.nnzb == 0 || ncrows == 0) return;
  const int m = J.nrows;
  const dim3 gm(grid_for(int64_t(m) * CT_G, 256)), blk(256);
  // a wavefront per J^T row once the rows average more constraints than a wavefront has lanes
  const bool wide = JT.nnzb > int64_t(64) * ncrows;
  if (J.bc == 3) {
    hipLaunchKernelGGL((k_contact_t<3, TX>), gm, blk, 0, c.s, m, J.rowptr.p, J.col.p, J.val.p,
                       D, x, t);
    if (wide) launch_contact_y<3, 64>(c, mode, JT, crows, ncrows, t, y, w);
    else launch_contact_y<3, CT_G>(c, mode, JT, crows, ncrows, t, y, w);
  } else {
    hipLaunchKernelGGL((k_contact_t<6, TX>), gm, blk, 0, c.s, m, J.rowptr.p, J.col.p, J.val.p,
                       D, x, t);
    if (wide) launch_contact_y<6, 64>(c, mode, JT, crows, ncrows, t, y, w);
    else launch_contact_y<6, CT_G>(c, mode, JT, crows, ncrows, t, y, w);
  }
  AMGF_LAUNCH_CHECK();
}
template void contact_apply<double, double>(Ctx&, int, const BSR&, const BSR&, const int*, int,
                                            const double*, const double*, double*, double*,
                                            const double*);
template void contact_apply<float, float>(Ctx&, int, const BSR&, const BSR&, const int*, int,
                                          const double*, const float*, double*, float*,
                                          const float*);
template void contact_apply<double, float>(Ctx&, int, const BSR&, const BSR&, const int*, int,
                                           const double*, const double*, double*, float*,
                                           const float*);
template void contact_apply<float, double>(Ctx&, int, const BSR&, const BSR&, const int*, int,
                                           const double*, const float*, double*, double*,
                                           const double*);

// ======================================================================================
// packed copy of a square matrix (BSR::pk_*): rows padded to PACK_PAD blocks, entry-major
// ======================================================================================
constexpr int PACK_PAD = 16;   // blocks: 128-byte aligned entry stripes

__global__ void k_pack_count(int nrows, const int* __restrict__ rp, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  cnt[i] = (rp[i + 1] - rp[i] + PACK_PAD - 1) / PACK_PAD * PACK_PAD;
}

// Entries of one block that a lane loads together in the packed copy (16 bytes when the
// block's entry count allows it): entry e of block k of a row with nbp padded blocks sits at
// ((e / G) * nbp + k) * G + e % G, so each load instruction of a wavefront reads a
// contiguous stretch of 16-byte groups.
template <int B, class TV>
constexpr int pack_group() {
  return (B * B) % int(16 / sizeof(TV)) == 0 ? int(16 / sizeof(TV)) : 1;
}

// one wavefront per row, a lane per (padded) block
template <int B, class TV>
__global__ void __launch_bounds__(256) k_pack_fill(int nrows, const int* __restrict__ rp,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const int* __restrict__ off,
                                                   int* __restrict__ pcol,
                                                   TV* __restrict__ pval) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nrows) return;
  const int r0 = rp[i], nb = rp[i + 1] - r0;
  const int o0 = off[i], nbp = off[i + 1] - o0;
  constexpr int G = pack_group<B, TV>();
  TV* pv = pval + int64_t(o0) * B * B;
  for (int k = lane; k < nbp; k += 64) {
    if (k < nb) {
      pcol[o0 + k] = col[r0 + k];
      const double* v = val + int64_t(r0 + k) * B * B;
#pragma unroll
      for (int e = 0; e < B * B; ++e) pv[(int64_t(e / G) * nbp + k) * G + e % G] = TV(v[e]);
    } else {
      pcol[o0 + k] = i;
#pragma unroll
      for (int e = 0; e < B * B; ++e) pv[(int64_t(e / G) * nbp + k) * G + e % G] = TV(0);
    }
  }
}

// the packed copy of a whole square B x B matrix (a coarse level's smoothing matrix)
void bsr_build_packed(Ctx& c, BSR& A, bool fp64, bool fp32) {
  AMGF_REQUIRE(A.br == A.bc && A.nrows == A.ncols && (A.br == 6 || A.br == 3), AMGF_EINVAL,
               "packed copy needs a square matrix of 3x3 or 6x6 blocks");
  const int n = A.nrows, B = A.br;
  DBuf<int> cnt(std::max(n, 1));
  A.pk_off.alloc(size_t(n) + 1);
  if (n)
    hipLaunchKernelGGL(k_pack_count, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, A.rowptr.p,
                       cnt.p);
  const int total = scan_exclusive(c, cnt.p, A.pk_off.p, n);
  A.pk_col.alloc(std::max(total, 1));
  const size_t nv = std::max<size_t>(size_t(total) * B * B, 1);
  A.pk_val = DBuf<double>();
  A.pk_val32 = DBuf<float>();
  if (fp64) A.pk_val.alloc(nv);
  if (fp32) A.pk_val32.alloc(nv);
  if (n && total) {
    const dim3 g(grid_for(n, 4)), blk(256);
#define AMGF_PF(BB, TV, dst)                                                                 \
  hipLaunchKernelGGL((k_pack_fill<BB, TV>), g, blk, 0, c.s, n, A.rowptr.p, A.col.p, A.val.p,  \
                     A.pk_off.p, A.pk_col.p, dst)
    if (B == 6) {
      if (fp64) AMGF_PF(6, double, A.pk_val.p);
      if (fp32) AMGF_PF(6, float, A.pk_val32.p);
    } else {
      if (fp64) AMGF_PF(3, double, A.pk_val.p);
      if (fp32) AMGF_PF(3, float, A.pk_val32.p);
    }
#undef AMGF_PF
  }
  AMGF_LAUNCH_CHECK();
}

// y (op)= A x over every row through the packed copy: one wavefront per row, a lane per
// block, two 64-block stretches in flight; products accumulate in T per lane, then over the
// wavefront.  Modes and epilogue as k_bsr.  FP64 values with FP32 vectors (a level whose
// smoothing matrix holds the contact term) accumulate and form the residual in FP64.
template <int B, class TV, class T, int MODE>
__global__ void __launch_bounds__(256) k_packed_spmv(int nrows, const int* __restrict__ off,
                                                     const int* __restrict__ pcol,
                                                     const TV* __restrict__ pval,
                                                     const T* __restrict__ x, T* __restrict__ y,
                                                     const T* __restrict__ b,
                                                     const T* __restrict__ w,
                                                     T* __restrict__ xo) {
  using Acc = std::conditional_t<sizeof(TV) == 8, double, T>;
  constexpr int G = pack_group<B, TV>();
  typedef TV TVG __attribute__((ext_vector_type(G)));
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= nrows) return;
  const int o0 = off[r], nbp = off[r + 1] - o0;
  const TVG* pv = reinterpret_cast<const TVG*>(pval + int64_t(o0) * B * B);
  Acc acc[B];
#pragma unroll
  for (int p = 0; p < B; ++p) acc[p] = Acc(0);
#pragma unroll 2
  for (int k = lane; k < nbp; k += 64) {
    const int64_t base = int64_t(pcol[o0 + k]) * B;
    Acc xq[B];
#pragma unroll
    for (int q = 0; q < B; ++q)
      xq[q] = Acc((MODE == SPMV_PRE) ? w[base + q] * b[base + q] : x[base + q]);
    TV a[B * B];
#pragma unroll
    for (int g = 0; g < B * B / G; ++g) {
      const TVG v = pv[int64_t(g) * nbp + k];
#pragma unroll
      for (int u = 0; u < G; ++u) a[g * G + u] = v[u];
    }
#pragma unroll
    for (int p = 0; p < B; ++p)
#pragma unroll
      for (int q = 0; q < B; ++q) acc[p] += Acc(a[B * p + q]) * xq[q];
  }
#pragma unroll
  for (int p = 0; p < B; ++p) acc[p] = wave_sum(acc[p]);
  if (lane >= B) return;
  Acc ax = Acc(0);
#pragma unroll
  for (int p = 0; p < B; ++p)
    if (lane == p) ax = acc[p];
  const int64_t i = int64_t(r) * B + lane;
  if (MODE == SPMV_Y) y[i] = T(ax);
  else if (MODE == SPMV_ADD) y[i] = T(Acc(y[i]) + ax);
  else if (MODE == SPMV_PRE) {
    const T xi = w[i] * b[i];
    xo[i] = xi;
    y[i] = T(Acc(b[i]) - ax);
  } else if (MODE == SPMV_POST) {
    xo[i] = T(Acc(x[i]) + Acc(w[i]) * (Acc(b[i]) - ax));
  } else {
    y[i] = T(Acc(b[i]) - ax);
  }
}

template <int B, class TV, class T>
static void launch_packed(Ctx& c, int mode, const BSR& A, const TV* pv, const T* x, T* y,
                          const T* b, const T* w, T* xo) {
  const dim3 g(grid_for(A.nrows, 4)), blk(256);
  switch (mode) {
#define AMGF_MODE(MD)                                                                        \
  case MD:                                                                                   \
    hipLaunchKernelGGL((k_packed_spmv<B, TV, T, MD>), g, blk, 0, c.s, A.nrows, A.pk_off.p,   \
                       A.pk_col.p, pv, x, y, b, w, xo);                                      \
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

// nonempty rows of a CSR (compact list)
__global__ void k_nonempty_flag(int n, const int* __restrict__ rp, int* __restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = rp[i + 1] > rp[i];
}
__global__ void k_compact_index(int n, const int* __restrict__ f, const int* __restrict__ pos,
                                int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && f[i]) out[pos[i]] = i;
}
int nonempty_rows(Ctx& c, const int* rp, int n, DBuf<int>& rows) {
  DBuf<int> f(std::max(n, 1)), pos(size_t(n) + 1);
  if (n) hipLaunchKernelGGL(k_nonempty_flag, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, rp, f.p);
  const int cnt = scan_exclusive(c, f.p, pos.p, n);
  rows.alloc(std::max(cnt, 1));
  if (n && cnt)
    hipLaunchKernelGGL(k_compact_index, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, f.p, pos.p,
                       rows.p);
  AMGF_LAUNCH_CHECK();
  return cnt;
}

// ======================================================================================
// elementwise
// ======================================================================================
#define AMGF_ELEMWISE(name, params, body)                                                    \
  __global__ void name params {                                                              \
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;                        \
    if (i < n) { body; }                                                                     \
  }

AMGF_ELEMWISE(k_d2f, (const double* __restrict__ a, float* __restrict__ b, int64_t n),
              b[i] = float(a[i]))
AMGF_ELEMWISE(k_f2d, (const float* __restrict__ a, double* __restrict__ b, int64_t n),
              b[i] = double(a[i]))
// b = float(a) and the first smoothing iterate x = w.b of a V-cycle from zero
AMGF_ELEMWISE(k_d2f_w, (const double* __restrict__ a, const float* __restrict__ w,
                        float* __restrict__ b, float* __restrict__ x, int64_t n),
              const float bi = float(a[i]);
              b[i] = bi;
              x[i] = w[i] * bi)
AMGF_ELEMWISE(k_add_to_f, (const float* __restrict__ a, float* __restrict__ y, int64_t n),
              y[i] += a[i])
AMGF_ELEMWISE(k_wmul_f, (const float* __restrict__ w, const float* __restrict__ b,
                         float* __restrict__ x, int64_t n),
              x[i] = w[i] * b[i])
// FP64: b = a and x = w.b (level 0 of a V-cycle from zero), or x = w.b alone
AMGF_ELEMWISE(k_copy_w, (const double* __restrict__ a, const double* __restrict__ w,
                         double* __restrict__ b, double* __restrict__ x, int64_t n),
              const double bi = a[i];
              b[i] = bi;
              x[i] = w[i] * bi)
AMGF_ELEMWISE(k_wmul_d, (const double* __restrict__ w, const double* __restrict__ b,
                         double* __restrict__ x, int64_t n),
              x[i] = w[i] * b[i])
AMGF_ELEMWISE(k_copy, (const double* __restrict__ a, double* __restrict__ b, int64_t n),
              b[i] = a[i])
AMGF_ELEMWISE(k_axpby, (int64_t n, double al, const double* __restrict__ x, double be,
                        double* __restrict__ y),
              y[i] = al * x[i] + be * y[i])
AMGF_ELEMWISE(k_scale, (int64_t n, double s, double* __restrict__ x), x[i] *= s)
AMGF_ELEMWISE(k_add_f, (int64_t n, const double* __restrict__ a, const float* __restrict__ f,
                        double* __restrict__ z),
              z[i] = a[i] + double(f[i]))
AMGF_ELEMWISE(k_scale_div, (int64_t n, double* __restrict__ y, const double* __restrict__ d,
                            const unsigned char* __restrict__ dec),
              y[i] = (dec && dec[i]) ? 0.0 : y[i] / d[i])
AMGF_ELEMWISE(k_weights, (int64_t n, const double* __restrict__ d,
                          const double* __restrict__ th, double* __restrict__ w),
              w[i] = (th ? th[i] : 1.0) / d[i])
AMGF_ELEMWISE(k_xr, (int64_t n, double al, const double* __restrict__ p,
                     const double* __restrict__ q, double* __restrict__ x,
                     double* __restrict__ r),
              x[i] += al * p[i];
              r[i] -= al * q[i])
// alpha = rz / (p.q) with p.q read from device memory (no host round trip)
AMGF_ELEMWISE(k_xr_dev, (int64_t n, double rz, const double* __restrict__ pq,
                         const double* __restrict__ p, const double* __restrict__ q,
                         double* __restrict__ x, double* __restrict__ r),
              const double al = rz / pq[0];
              x[i] += al * p[i];
              r[i] -= al * q[i])
// the same, and the mixed V-cycle's first two level-0 vectors from the new residual:
// b = float(r), x = w.b (what the V-cycle would otherwise form in a pass of its own)
AMGF_ELEMWISE(k_xr_dev_f, (int64_t n, double rz, const double* __restrict__ pq,
                           const double* __restrict__ p, const double* __restrict__ q,
                           double* __restrict__ x, double* __restrict__ r,
                           const float* __restrict__ w, float* __restrict__ fb,
                           float* __restrict__ fx),
              const double al = rz / pq[0];
              x[i] += al * p[i];
              const double ri = r[i] - al * q[i];
              r[i] = ri;
              const float bi = float(ri);
              fb[i] = bi;
              fx[i] = w[i] * bi)
AMGF_ELEMWISE(k_pupd, (int64_t n, double be, const double* __restrict__ z, double* __restrict__ p),
              p[i] = z[i] + be * p[i])
// beta = (r.z - r.z_old) / rz with both dots read from device memory, then p = z + beta p
AMGF_ELEMWISE(k_pupd_dev, (int64_t n, double rz, const double* __restrict__ s,
                           const double* __restrict__ z, double* __restrict__ p),
              const double be = (s[0] - s[1]) / rz;
              p[i] = z[i] + be * p[i])
AMGF_ELEMWISE(k_power_start, (int64_t n, double* __restrict__ x,
                              const unsigned char* __restrict__ dec),
              x[i] = (dec && dec[i]) ? 0.0
                                     : double(fmix32(uint32_t(i))) * 0x1p-32 - 0.5)

__global__ void k_gather(const double* __restrict__ x, const int* __restrict__ idx, int n,
                         double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[idx[i]];
}
__global__ void k_scatter_add(const double* __restrict__ w, const int* __restrict__ idx, int n,
                              double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[idx[i]] += w[i];
}
// on the listed DOFs: z[k] = double(f[k]) + w[i], then f[k] = float(z[k])
__global__ void k_corr_at(float* f, const double* __restrict__ w, const int* __restrict__ idx,
                          int n, double* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t k = idx[i];
  const double v = double(f[k]) + w[i];
  z[k] = v;
  f[k] = float(v);
}
// z = double(a) + double(b), and z[k] = u[k] + double(b[k]) on the listed DOFs
AMGF_ELEMWISE(k_add_ff, (int64_t n, const float* __restrict__ a, const float* __restrict__ b,
                         double* __restrict__ z),
              z[i] = double(a[i]) + double(b[i]))
__global__ void k_add_at(const double* __restrict__ u, const float* __restrict__ b,
                         const int* __restrict__ idx, int n, double* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t k = idx[i];
  z[k] = u[k] + double(b[k]);
}
__global__ void k_check(const double* __restrict__ v, int64_t n, int pos, int* flag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = v[i];
  if (!isfinite(x)) atomicOr(flag, 1);
  if (pos == 1 && !(x > 0.0)) atomicOr(flag, 2);
  if (pos == 2 && !(x >= 0.0)) atomicOr(flag, 2);
}

// Chebyshev smoother steps (elementwise):
//   start: r = w.src; d = r * inv_theta; x = d (x_zero) or x + d
//   step:  r -= w.t;  d = c1 d + c2 r;    x += d
template <class T>
__global__ void k_cheb_start(int64_t n, const T* __restrict__ src, const T* __restrict__ w,
                             T* __restrict__ r, T* __restrict__ d, T* __restrict__ x,
                             T inv_theta, int x_zero) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T ri = w[i] * src[i];
  const T di = ri * inv_theta;
  r[i] = ri;
  d[i] = di;
  x[i] = x_zero ? di : x[i] + di;
}
template <class T>
__global__ void k_cheb_step(int64_t n, const T* __restrict__ t, const T* __restrict__ w,
                            T* __restrict__ r, T* __restrict__ d, T* __restrict__ x, T c1,
                            T c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T ri = r[i] - w[i] * t[i];
  const T di = c1 * d[i] + c2 * ri;
  r[i] = ri;
  d[i] = di;
  x[i] += di;
}

#define AMGF_L1D(n) dim3(grid_for((n), 256)), dim3(256), 0, c.s
template <class T>
void cheb_start(Ctx& c, int64_t n, const T* src, const T* w, T* r, T* d, T* x, double inv_theta,
                bool x_zero) {
  if (n) hipLaunchKernelGGL(k_cheb_start<T>, AMGF_L1D(n), n, src, w, r, d, x, T(inv_theta),
                            int(x_zero));
}
template <class T>
void cheb_step(Ctx& c, int64_t n, const T* t, const T* w, T* r, T* d, T* x, double c1,
               double c2) {
  if (n) hipLaunchKernelGGL(k_cheb_step<T>, AMGF_L1D(n), n, t, w, r, d, x, T(c1), T(c2));
}
template void cheb_start<double>(Ctx&, int64_t, const double*, const double*, double*, double*,
                                 double*, double, bool);
template void cheb_start<float>(Ctx&, int64_t, const float*, const float*, float*, float*,
                                float*, double, bool);
template void cheb_step<double>(Ctx&, int64_t, const double*, const double*, double*, double*,
                                double*, double, double);
template void cheb_step<float>(Ctx&, int64_t, const float*, const float*, float*, float*, float*,
                               double, double);
void cast_d2f(Ctx& c, const double* a, float* b, int64_t n) {
  if (n) hipLaunchKernelGGL(k_d2f, AMGF_L1D(n), a, b, n);
}
void cast_d2f_w(Ctx& c, const double* a, const float* w, float* b, float* x, int64_t n) {
  if (n) hipLaunchKernelGGL(k_d2f_w, AMGF_L1D(n), a, w, b, x, n);
}
void add_to_f32(Ctx& c, int64_t n, const float* a, float* y) {
  if (n) hipLaunchKernelGGL(k_add_to_f, AMGF_L1D(n), a, y, n);
}
void wmul_f32(Ctx& c, int64_t n, const float* w, const float* b, float* x) {
  if (n) hipLaunchKernelGGL(k_wmul_f, AMGF_L1D(n), w, b, x, n);
}
void copy_w(Ctx& c, const double* a, const double* w, double* b, double* x, int64_t n) {
  if (n) hipLaunchKernelGGL(k_copy_w, AMGF_L1D(n), a, w, b, x, n);
}
void wmul_f64(Ctx& c, int64_t n, const double* w, const double* b, double* x) {
  if (n) hipLaunchKernelGGL(k_wmul_d, AMGF_L1D(n), w, b, x, n);
}
void cast_f2d(Ctx& c, const float* a, double* b, int64_t n) {
  if (n) hipLaunchKernelGGL(k_f2d, AMGF_L1D(n), a, b, n);
}
void vcopy(Ctx& c, const double* a, double* b, int64_t n) {
  if (n) hipLaunchKernelGGL(k_copy, AMGF_L1D(n), a, b, n);
}
void axpby(Ctx& c, int64_t n, double alpha, const double* x, double beta, double* y) {
  if (n) hipLaunchKernelGGL(k_axpby, AMGF_L1D(n), n, alpha, x, beta, y);
}
void add_f32(Ctx& c, int64_t n, const double* a, const float* f, double* z) {
  if (n) hipLaunchKernelGGL(k_add_f, AMGF_L1D(n), n, a, f, z);
}
// x = y * (1 / sqrt(s[0])), the norm read from device memory (power iteration step)
AMGF_ELEMWISE(k_normalize_dev, (int64_t n, const double* __restrict__ s,
                                const double* __restrict__ y, double* __restrict__ x),
              x[i] = y[i] * (1.0 / sqrt(s[0])))
void normalize_dev(Ctx& c, int64_t n, const double* s, const double* y, double* x) {
  if (n) hipLaunchKernelGGL(k_normalize_dev, AMGF_L1D(n), n, s, y, x);
}
void vscale(Ctx& c, int64_t n, double s, double* x) {
  if (n) hipLaunchKernelGGL(k_scale, AMGF_L1D(n), n, s, x);
}
void gather(Ctx& c, const double* x, const int* idx, int n, double* y) {
  if (n) hipLaunchKernelGGL(k_gather, AMGF_L1D(n), x, idx, n, y);
}
void scatter_add(Ctx& c, const double* w, const int* idx, int n, double* y) {
  if (n) hipLaunchKernelGGL(k_scatter_add, AMGF_L1D(n), w, idx, n, y);
}
void correct_at(Ctx& c, float* f, const double* w, const int* idx, int n, double* z) {
  if (n) hipLaunchKernelGGL(k_corr_at, AMGF_L1D(n), f, w, idx, n, z);
}
void add_ff(Ctx& c, int64_t n, const float* a, const float* b, double* z) {
  if (n) hipLaunchKernelGGL(k_add_ff, AMGF_L1D(n), n, a, b, z);
}
void add_at(Ctx& c, const double* u, const float* b, const int* idx, int n, double* z) {
  if (n) hipLaunchKernelGGL(k_add_at, AMGF_L1D(n), u, b, idx, n, z);
}
void scale_div_zero(Ctx& c, int64_t n, double* y, const double* d, const unsigned char* dec) {
  if (n) hipLaunchKernelGGL(k_scale_div, AMGF_L1D(n), n, y, d, dec);
}
void fill_power_start(Ctx& c, int64_t n, double* x, const unsigned char* dec) {
  if (n) hipLaunchKernelGGL(k_power_start, AMGF_L1D(n), n, x, dec);
}
void weights_from_l1(Ctx& c, int64_t n, const double* d, const double* theta, double* w) {
  if (n) hipLaunchKernelGGL(k_weights, AMGF_L1D(n), n, d, theta, w);
}
void pcg_update_xr(Ctx& c, int64_t n, double alpha, const double* p, const double* q, double* x,
                   double* r) {
  if (n) hipLaunchKernelGGL(k_xr, AMGF_L1D(n), n, alpha, p, q, x, r);
}
void pcg_update_xr_dev(Ctx& c, int64_t n, double rz, const double* pq, const double* p,
                       const double* q, double* x, double* r) {
  if (n) hipLaunchKernelGGL(k_xr_dev, AMGF_L1D(n), n, rz, pq, p, q, x, r);
}
void pcg_update_xr_dev_f(Ctx& c, int64_t n, double rz, const double* pq, const double* p,
                         const double* q, double* x, double* r, const float* w, float* fb,
                         float* fx) {
  if (n) hipLaunchKernelGGL(k_xr_dev_f, AMGF_L1D(n), n, rz, pq, p, q, x, r, w, fb, fx);
}
void pcg_update_p(Ctx& c, int64_t n, double beta, const double* z, double* p) {
  if (n) hipLaunchKernelGGL(k_pupd, AMGF_L1D(n), n, beta, z, p);
}
void pcg_update_p_dev(Ctx& c, int64_t n, double rz, const double* s, const double* z,
                      double* p) {
  if (n) hipLaunchKernelGGL(k_pupd_dev, AMGF_L1D(n), n, rz, s, z, p);
}
void check_values(Ctx& c, const double* v, int64_t n, bool require_positive, int* flag) {
  if (n) hipLaunchKernelGGL(k_check, AMGF_L1D(n), v, n, int(require_positive), flag);
  AMGF_LAUNCH_CHECK();
}
void check_nonnegative(Ctx& c, const double* v, int64_t n, int* flag) {
  if (n) hipLaunchKernelGGL(k_check, AMGF_L1D(n), v, n, 2, flag);
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// deterministic dots: fixed grid, per-block partials, single-block final sum
// ======================================================================================
struct DotArgs {
  const double* x[DOT_MAX];
  const double* y[DOT_MAX];
};

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < int(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

template <int ND>
__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, DotArgs a,
                                                     double* __restrict__ part) {
  constexpr int U = 4;   // elements per thread whose loads go out together (order kept)
  __shared__ double sh[4];
  double acc[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) acc[d] = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i0 < n; i0 += U * stride) {
    double xv[U][ND], yv[U][ND];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t i = i0 + k * stride;
      const int64_t ic = i < n ? i : n - 1;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        xv[k][d] = a.x[d][ic];
        yv[k][d] = a.y[d][ic];
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (i0 + k * stride >= n) break;
#pragma unroll
      for (int d = 0; d < ND; ++d) acc[d] += xv[k][d] * yv[k][d];
    }
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double s = block_sum(acc[d], sh);
    if (threadIdx.x == 0) part[d * DOT_BLOCKS + blockIdx.x] = s;
  }
}
static void launch_dot_partial(Ctx& c, int64_t n, int nd, const DotArgs& a, double* part) {
  switch (nd) {
    case 1: hipLaunchKernelGGL(k_dot_partial<1>, dim3(DOT_BLOCKS), dim3(256), 0, c.s, n, a, part); break;
    case 2: hipLaunchKernelGGL(k_dot_partial<2>, dim3(DOT_BLOCKS), dim3(256), 0, c.s, n, a, part); break;
    case 3: hipLaunchKernelGGL(k_dot_partial<3>, dim3(DOT_BLOCKS), dim3(256), 0, c.s, n, a, part); break;
    default: hipLaunchKernelGGL(k_dot_partial<4>, dim3(DOT_BLOCKS), dim3(256), 0, c.s, n, a, part);
  }
}
__global__ void __launch_bounds__(256) k_dot_final(int nd, const double* __restrict__ part,
                                                   double* __restrict__ out) {
  __shared__ double sh[4];
  for (int d = 0; d < nd; ++d) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < DOT_BLOCKS; i += blockDim.x) acc += part[d * DOT_BLOCKS + i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[d] = s;
  }
}

// z = a + b (FP32 values widened) except on the DOFs set in mask (one bit each), where
// z = u + b; with the CG products r.z and r.zo as partial sums in the layout, element order
// and per-thread order of k_dot_partial (same grid), so k_dot_final gives bitwise the sums
// dots_device would give over the finished z
__global__ void __launch_bounds__(256) k_add_ff_dots(int64_t n, const float* __restrict__ a,
                                                     const float* __restrict__ b,
                                                     const double* __restrict__ u,
                                                     const uint32_t* __restrict__ mask,
                                                     const double* __restrict__ r,
                                                     const double* __restrict__ zo,
                                                     double* __restrict__ z,
                                                     double* __restrict__ part) {
  constexpr int U = 4;   // elements per thread whose loads go out together
  __shared__ double sh[4];
  double acc0 = 0.0, acc1 = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i0 < n; i0 += U * stride) {
    float av[U], bv[U];
    double rv[U], ov[U];
    uint32_t mv[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t i = i0 + k * stride;
      const int64_t ic = i < n ? i : n - 1;
      av[k] = a[ic];
      bv[k] = b[ic];
      rv[k] = r[ic];
      ov[k] = zo[ic];
      mv[k] = mask[ic >> 5];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t i = i0 + k * stride;
      if (i >= n) break;
      const bool on = (mv[k] >> (i & 31)) & 1u;
      const double zi = (on ? u[i] : double(av[k])) + double(bv[k]);
      z[i] = zi;
      acc0 += rv[k] * zi;
      acc1 += rv[k] * ov[k];
    }
  }
  const double s0 = block_sum(acc0, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s0;
  const double s1 = block_sum(acc1, sh);
  if (threadIdx.x == 0) part[DOT_BLOCKS + blockIdx.x] = s1;
}

__global__ void k_set_bits(const int* __restrict__ idx, int n, uint32_t* __restrict__ mask) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = idx[k];
  atomicOr(&mask[i >> 5], 1u << (i & 31));
}

// the partial sums (DOT_SCRATCH doubles): the caller's buffer, else the context's own
static double* dot_partials(Ctx& c, double* part) {
  if (part) return part;
  if (c.dot.n == 0) c.dot.alloc(DOT_SCRATCH);
  return c.dot.p;
}

void dots_device(Ctx& c, int64_t n, int nd, const double* const* xs, const double* const* ys,
                 double* out_dev, double* part) {
  AMGF_REQUIRE(nd >= 1 && nd <= DOT_MAX, AMGF_EINVAL, "dots count");
  double* pp = dot_partials(c, part);
  DotArgs a{};
  for (int d = 0; d < nd; ++d) {
    a.x[d] = xs[d];
    a.y[d] = ys[d];
  }
  launch_dot_partial(c, n, nd, a, pp);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, c.s, nd, pp, out_dev);
  AMGF_LAUNCH_CHECK();
}

void add_ff_dots(Ctx& c, int64_t n, const float* a, const float* b, const double* u,
                 const uint32_t* mask, const double* r, const double* zo, double* z,
                 double* out_dev, double* part) {
  double* pp = dot_partials(c, part);
  hipLaunchKernelGGL(k_add_ff_dots, dim3(DOT_BLOCKS), dim3(256), 0, c.s, n, a, b, u, mask, r,
                     zo, z, pp);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, c.s, 2, pp, out_dev);
  AMGF_LAUNCH_CHECK();
}

void bit_mask(Ctx& c, const int* idx, int n, int64_t nbits, DBuf<uint32_t>& mask) {
  const size_t words = size_t((nbits + 31) / 32);
  if (mask.n != std::max<size_t>(words, 1)) mask.alloc(std::max<size_t>(words, 1));
  AMGF_HIP(hipMemsetAsync(mask.p, 0, mask.bytes(), c.s));
  if (n) hipLaunchKernelGGL(k_set_bits, dim3(grid_for(n, 256)), dim3(256), 0, c.s, idx, n, mask.p);
  AMGF_LAUNCH_CHECK();
}

void dots(Ctx& c, int64_t n, int nd, const double* const* xs, const double* const* ys,
          double* out_host, double* part) {
  AMGF_REQUIRE(nd >= 1 && nd <= DOT_MAX, AMGF_EINVAL, "dots count");
  double* pp = dot_partials(c, part);
  DotArgs a{};
  for (int d = 0; d < nd; ++d) {
    a.x[d] = xs[d];
    a.y[d] = ys[d];
  }
  launch_dot_partial(c, n, nd, a, pp);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, c.s, nd, pp, pp + DOT_MAX * DOT_BLOCKS);
  AMGF_LAUNCH_CHECK();
  AMGF_HIP(hipMemcpyAsync(out_host, pp + DOT_MAX * DOT_BLOCKS, nd * sizeof(double),
                          hipMemcpyDeviceToHost, c.s));
  AMGF_HIP(hipStreamSynchronize(c.s));
}

}  // namespace amgf

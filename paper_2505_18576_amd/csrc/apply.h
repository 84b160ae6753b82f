// Apply-phase kernels (apply.hip): SpMV with fused smoother modes, contact term,
// transfers, vector updates and deterministic reductions.
#pragma once
#include "common.h"

namespace amgf {

enum SpmvMode {
  SPMV_Y = 0,     // y = A x
  SPMV_ADD = 1,   // y += A x
  SPMV_PRE = 2,   // xo = w.b ; y = b - A (w.b)          (first smoothing step from 0)
  SPMV_POST = 3,  // xo = x + w.(b - A x)                (Jacobi step, new buffer)
  SPMV_RES = 4,   // y = b - A x
  SPMV_YW = 5     // y = A x ; xo = w.y  (restriction into a level whose cycle starts at w.b;
                  // BSR kernels only)
};

// y/xo per mode; val is T-typed (double or float) and the vectors are T too.
template <class T>
void bsr_spmv(Ctx& c, int mode, const BSR& A, const T* val, const T* x, T* y, const T* b,
              const T* w, T* xo);

// y = A x (SPMV_Y), y += A x (SPMV_ADD) or y = A x with xo = w.y (SPMV_YW) in FP32 with the
// FP16 values A.valh, or with the FP32 values A.val32 when A has no FP16 copy (restriction
// and prolongation of the mixed V-cycle)
void transfer_spmv(Ctx& c, int mode, const BSR& A, const float* x, float* y,
                   const float* w = nullptr, float* xo = nullptr);
// b = FP16(a) in the chunked layout of BSR::valh (a: nb blocks of N entries; b holds nb
// rounded up to a multiple of 64 blocks), one rounding to nearest even; *flag |= 1 when a
// value overflows FP16
void cast_d2h_chunked(Ctx& c, const double* a, _Float16* b, int64_t nb, int N, int* flag);
// A.valh = FP16(A.val) in the layout the FP16 transfer kernel for A reads (chunked when it
// gives a block row a whole wavefront, row-major blocks otherwise; allocated here)
void cast_d2h_transfer(Ctx& c, BSR& A, int* flag);
// lanes per block row of the FP16 transfer kernel for A's shape and density
int transfer_lanes(const BSR& A);

// Build the sliced-ELL copy (FP64 values when fp64, FP32 values when fp32) of a 3x3
// BSR matrix; bsr_spmv then reads it in place of the BSR arrays.
void bsr_build_sell(Ctx& c, BSR& A, bool fp64, bool fp32, bool bf16 = false);
// SpMV modes on a sliced copy with T values (the dispatch of bsr_spmv uses it)
template <class T>
void sell3_spmv(Ctx& c, int mode, const BSR& A, const T* sval, const T* x, T* y, const T* b,
                const T* w, T* xo);
// SpMV modes on the BF16 sliced copy, FP32 vectors and FP32 accumulation
void sell_spmv_bf16(Ctx& c, int mode, const BSR& A, const float* x, float* y, const float* b,
                    const float* w, float* xo);

// contact term of a level over its contact node rows (crows, ncrows):
// t = D.(J x) then, per mode,
//   CT_SUB_RES:  y -= J^T t          (residual update)
//   CT_SUB_W:    y -= w.(J^T t)      (Jacobi step correction)
//   CT_ADD:      y += J^T t          (operator apply)
enum ContactMode { CT_SUB_RES = 0, CT_SUB_W = 1, CT_ADD = 2 };
template <class TX, class TY>
void contact_apply(Ctx& c, int mode, const BSR& J, const BSR& JT, const int* crows, int ncrows,
                   const double* D, const TX* x, double* t, TY* y, const TY* w);
// packed copy of a square matrix (BSR::pk_*) with FP64 and/or FP32 values; bsr_spmv then
// applies the matrix through it when it is handed the matrix's own values
void bsr_build_packed(Ctx& c, BSR& A, bool fp64, bool fp32);
// indices of the nonempty rows of a CSR pattern
int nonempty_rows(Ctx& c, const int* rp, int n, DBuf<int>& rows);
// y = b - A x on the listed block rows only (FP64, 3x3 blocks)
template <class TX>
void bsr_res_rows(Ctx& c, const BSR& A, const int* rows, int nlist, const TX* x,
                  const double* b, double* y);

// Chebyshev smoother steps: start r = w.src, d = r/theta, x = d or x + d;
// step r -= w.t, d = c1 d + c2 r, x += d
template <class T>
void cheb_start(Ctx& c, int64_t n, const T* src, const T* w, T* r, T* d, T* x, double inv_theta,
                bool x_zero);
template <class T>
void cheb_step(Ctx& c, int64_t n, const T* t, const T* w, T* r, T* d, T* x, double c1,
               double c2);

// elementwise helpers
void cast_d2f(Ctx& c, const double* a, float* b, int64_t n);
void cast_f2d(Ctx& c, const float* a, double* b, int64_t n);
// b = float(a), x = w.b (FP32 product of the rounded b)
void cast_d2f_w(Ctx& c, const double* a, const float* w, float* b, float* x, int64_t n);
void wmul_f32(Ctx& c, int64_t n, const float* w, const float* b, float* x);   // x = w.b
void add_to_f32(Ctx& c, int64_t n, const float* a, float* y);                    // y += a
void copy_w(Ctx& c, const double* a, const double* w, double* b, double* x, int64_t n);  // b = a, x = w.a
void wmul_f64(Ctx& c, int64_t n, const double* w, const double* b, double* x);  // x = w.b
void vcopy(Ctx& c, const double* a, double* b, int64_t n);
void add_f32(Ctx& c, int64_t n, const double* a, const float* f, double* z);  // z = a + f
void axpby(Ctx& c, int64_t n, double alpha, const double* x, double beta, double* y);  // y = a x + b y
void gather(Ctx& c, const double* x, const int* idx, int n, double* y);               // y = x[idx]
void scatter_add(Ctx& c, const double* w, const int* idx, int n, double* y);          // y[idx] += w
// on the n DOFs idx[i]: z = double(f) + w[i], then f = float(z)   (the filter correction)
void correct_at(Ctx& c, float* f, const double* w, const int* idx, int n, double* z);
void add_ff(Ctx& c, int64_t n, const float* a, const float* b, double* z);  // z = a + b
// z[idx] = u[idx] + b[idx] on the n listed DOFs
void add_at(Ctx& c, const double* u, const float* b, const int* idx, int n, double* z);
void scale_div_zero(Ctx& c, int64_t n, double* y, const double* d, const unsigned char* dec);
void fill_power_start(Ctx& c, int64_t n, double* x, const unsigned char* dec);
void weights_from_l1(Ctx& c, int64_t n, const double* d, const double* theta, double* w);
void vscale(Ctx& c, int64_t n, double s, double* x);

// deterministic dot products: out[i] = sum_k x_i[k] y_i[k] (host results), at most DOT_MAX
// at once over a fixed grid of DOT_BLOCKS partial sums.  `part`: DOT_SCRATCH device doubles
// for the partial sums, or nullptr for the context's own buffer (allocated on first use).
constexpr int DOT_BLOCKS = 1024;
constexpr int DOT_MAX = 4;
constexpr size_t DOT_SCRATCH = size_t(DOT_MAX) * DOT_BLOCKS + DOT_MAX;
void dots(Ctx& c, int64_t n, int nd, const double* const* xs, const double* const* ys,
          double* out_host, double* part = nullptr);

// the same sums left in device memory (out_dev[0 .. nd-1]), stream-ordered, no wait
void dots_device(Ctx& c, int64_t n, int nd, const double* const* xs, const double* const* ys,
                 double* out_dev, double* part = nullptr);

// The end of the mixed AMGF step fused with the CG dot products: z = a + b (FP32 halves
// widened), z = u + b on the DOFs set in mask; out_dev[0] = r.z, out_dev[1] = r.zo, bitwise
// what dots_device gives over the finished z (same partition and order)
void add_ff_dots(Ctx& c, int64_t n, const float* a, const float* b, const double* u,
                 const uint32_t* mask, const double* r, const double* zo, double* z,
                 double* out_dev, double* part = nullptr);
// mask = one bit per index below nbits, set for idx[0 .. n-1] (allocated here when its size
// differs)
void bit_mask(Ctx& c, const int* idx, int n, int64_t nbits, DBuf<uint32_t>& mask);

// x = y / sqrt(s[0]) with s in device memory
void normalize_dev(Ctx& c, int64_t n, const double* s, const double* y, double* x);

// PCG updates
void pcg_update_xr(Ctx& c, int64_t n, double alpha, const double* p, const double* q, double* x,
                   double* r);
// x += a p, r -= a q with a = rz / pq[0] (pq in device memory)
void pcg_update_xr_dev(Ctx& c, int64_t n, double rz, const double* pq, const double* p,
                       const double* q, double* x, double* r);
// the same, also writing fb = float(r) and fx = w.fb (the mixed V-cycle's level-0 input
// and first smoothing iterate)
void pcg_update_xr_dev_f(Ctx& c, int64_t n, double rz, const double* pq, const double* p,
                         const double* q, double* x, double* r, const float* w, float* fb,
                         float* fx);
void pcg_update_p(Ctx& c, int64_t n, double beta, const double* z, double* p);
// p = z + beta p with beta = (s[0] - s[1]) / rz, s = {r.z, r.z_old} in device memory
void pcg_update_p_dev(Ctx& c, int64_t n, double rz, const double* s, const double* z,
                      double* p);

// input validation: flag bit 1 non-finite, bit 2 non-positive
void check_values(Ctx& c, const double* v, int64_t n, bool require_positive, int* flag);
// bit 1 non-finite, bit 2 negative
void check_nonnegative(Ctx& c, const double* v, int64_t n, int* flag);

}  // namespace amgf

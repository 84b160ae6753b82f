// Dense FP64 SPD factorisation used for the coarsest level and the filter A_w.
//
// A = L L^T together with Linv = L^{-1} by recursive halving (all products are large
// MFMA GEMMs; 64x64 leaves are factored in LDS by one wavefront), so that each later
// solve x = Linv^T (Linv b) is two bandwidth-bound matrix-vector products instead of a
// sequence of dependent triangular steps.
#include "dense.h"

namespace amgf {

constexpr int NB = 64;

// ---------------------------------------------------------------- tiled DGEMM on MFMA
// C[M x N] = beta C + alpha A[M x K] op(B);  op(B) = B^T (B is N x K) or B (K x N).
// A 256-thread workgroup owns a 64x64 tile of C; each wavefront owns a 32x32 quarter as
// 2x2 tiles of v_mfma_f64_16x16x4f64 (operand lane l: A[l%16][l/16], B[l/16][l%16];
// result lane l, register r: D[4r + l/16][l%16]).  K advances in steps of 16 staged in
// LDS.  lower_only skips tiles strictly above the diagonal.
typedef double v4d __attribute__((ext_vector_type(4)));

template <bool TB>
__global__ void __launch_bounds__(256) k_dgemm(int M, int N, int K, double alpha,
                                               const double* __restrict__ A, int lda,
                                               const double* __restrict__ B, int ldb,
                                               double beta, double* __restrict__ C, int ldc,
                                               int lower_only) {
  const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
  if (lower_only && bn > bm + 63) return;
  __shared__ double As[64][17];     // [row][k]
  __shared__ double Bs[16][65];     // [k][col]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;   // wave quarter of the tile
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;            // 0..1023
      const int kk = e & 15, rr = e >> 4;     // A: 64 rows x 16 k, contiguous along k
      const int gr = bm + rr, gk = k0 + kk;
      As[rr][kk] = (gr < M && gk < K) ? A[int64_t(gr) * lda + gk] : 0.0;
      if (TB) {
        const int gc = bn + rr;
        Bs[kk][rr] = (gc < N && gk < K) ? B[int64_t(gc) * ldb + gk] : 0.0;
      } else {
        const int kb = e >> 6, cc = e & 63;   // B: 16 k x 64 cols, contiguous along cols
        const int gkb = k0 + kb, gc = bn + cc;
        Bs[kb][cc] = (gkb < K && gc < N) ? B[int64_t(gkb) * ldb + gc] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kq = ks * 4 + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = As[wr + a * 16 + (lane & 15)][kq];
#pragma unroll
      for (int b = 0; b < 2; ++b) bf[b] = Bs[kq][wc + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bm + wr + a * 16 + 4 * r + (lane >> 4);
        const int col = bn + wc + b * 16 + (lane & 15);
        if (row < M && col < N) {
          double* cp = C + int64_t(row) * ldc + col;
          *cp = alpha * acc[a][b][r] + (beta == 0.0 ? 0.0 : beta * *cp);
        }
      }
}

// Same product with a 32x32 tile per 64-lane workgroup (2x2 MFMA tiles per wavefront):
// four times as many workgroups, for products too small to fill the chip with 64x64.
template <bool TB>
__global__ void __launch_bounds__(64) k_dgemm32(int M, int N, int K, double alpha,
                                                const double* __restrict__ A, int lda,
                                                const double* __restrict__ B, int ldb,
                                                double beta, double* __restrict__ C, int ldc,
                                                int lower_only) {
  const int bm = blockIdx.y * 32, bn = blockIdx.x * 32;
  if (lower_only && bn > bm + 31) return;
  __shared__ double As[32][17];
  __shared__ double Bs[16][33];
  const int lane = threadIdx.x;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = lane + 64 * t;            // 0..511
      const int kk = e & 15, rr = e >> 4;     // 32 rows x 16 k
      const int gr = bm + rr, gk = k0 + kk;
      As[rr][kk] = (gr < M && gk < K) ? A[int64_t(gr) * lda + gk] : 0.0;
      if (TB) {
        const int gc = bn + rr;
        Bs[kk][rr] = (gc < N && gk < K) ? B[int64_t(gc) * ldb + gk] : 0.0;
      } else {
        const int kb = e >> 5, cc = e & 31;
        const int gkb = k0 + kb, gc = bn + cc;
        Bs[kb][cc] = (gkb < K && gc < N) ? B[int64_t(gkb) * ldb + gc] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kq = ks * 4 + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = As[a * 16 + (lane & 15)][kq];
#pragma unroll
      for (int b = 0; b < 2; ++b) bf[b] = Bs[kq][b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bm + a * 16 + 4 * r + (lane >> 4);
        const int col = bn + b * 16 + (lane & 15);
        if (row < M && col < N) {
          double* cp = C + int64_t(row) * ldc + col;
          *cp = alpha * acc[a][b][r] + (beta == 0.0 ? 0.0 : beta * *cp);
        }
      }
}

void dgemm(Ctx& c, bool transB, int M, int N, int K, double alpha, const double* A, int lda,
           const double* B, int ldb, double beta, double* C, int ldc, bool lower_only) {
  if (M <= 0 || N <= 0) return;
  if (int64_t((M + 63) / 64) * ((N + 63) / 64) < 512) {
    const dim3 g((N + 31) / 32, (M + 31) / 32);
    if (transB)
      hipLaunchKernelGGL(k_dgemm32<true>, g, dim3(64), 0, c.s, M, N, K, alpha, A, lda, B, ldb,
                         beta, C, ldc, int(lower_only));
    else
      hipLaunchKernelGGL(k_dgemm32<false>, g, dim3(64), 0, c.s, M, N, K, alpha, A, lda, B, ldb,
                         beta, C, ldc, int(lower_only));
    AMGF_LAUNCH_CHECK();
    return;
  }
  const dim3 g((N + 63) / 64, (M + 63) / 64);
  if (transB)
    hipLaunchKernelGGL(k_dgemm<true>, g, dim3(256), 0, c.s, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc, int(lower_only));
  else
    hipLaunchKernelGGL(k_dgemm<false>, g, dim3(256), 0, c.s, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc, int(lower_only));
  AMGF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- recursive factorisation
// Leaf (n <= 64): one wavefront; lane t keeps row t of the tile in registers (a tile
// smaller than 64 is padded with the identity).  Step j broadcasts column j through
// LDS and every lane updates its row; then lane t forms column t of L^{-1} by forward
// substitution against L rows read (as broadcasts) from LDS.  Writes L (zero upper)
// and L^{-1}.
__global__ void __launch_bounds__(64) k_chol_leaf(double* A, double* Li, int ld, int n,
                                                  int* info) {
  __shared__ double colj[NB];
  __shared__ double Ls[NB][NB + 1];
  const int t = threadIdx.x;
  // coalesced load of the tile (identity padding beyond n)
  for (int i = 0; i < NB; ++i)
    Ls[i][t] = (i < n && t < n) ? A[int64_t(i) * ld + t] : (i == t ? 1.0 : 0.0);
  __syncthreads();
  double row[NB];
#pragma unroll
  for (int l = 0; l < NB; ++l) row[l] = Ls[t][l];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    colj[t] = row[j];
    __syncthreads();
    const double p = colj[j];
    if (t == 0 && !(p > 0.0)) atomicOr(info, 1);
    const double dj = sqrt(p > 0.0 ? p : 1.0);
    const double lj = (t > j) ? row[j] / dj : dj;
    if (t >= j) row[j] = lj;
    __syncthreads();
    colj[t] = lj;
    __syncthreads();
    if (t > j) {
#pragma unroll
      for (int l = j + 1; l < NB; ++l)
        if (l <= t) row[l] -= lj * colj[l];
    }
    __syncthreads();
  }
#pragma unroll
  for (int l = 0; l < NB; ++l) Ls[t][l] = (l <= t) ? row[l] : 0.0;
  __syncthreads();
  for (int i = 0; i < n; ++i)
    if (t < n) A[int64_t(i) * ld + t] = Ls[i][t];
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double s = (i == t) ? 1.0 : 0.0;
#pragma unroll
    for (int l = 0; l < i; ++l) s -= Ls[i][l] * x[l];
    x[i] = (i >= t) ? s / Ls[i][i] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) Ls[i][t] = x[i];     // column t of L^{-1}
  __syncthreads();
  for (int i = 0; i < n; ++i)
    if (t < n) Li[int64_t(i) * ld + t] = Ls[i][t];
}

__global__ void k_copy2d(int rows, int cols, const double* __restrict__ S, int lds,
                         double* __restrict__ D, int ldd) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(rows) * cols) return;
  const int i = int(e / cols), j = int(e % cols);
  D[int64_t(i) * ldd + j] = S[int64_t(i) * lds + j];
}

// [A11 . ; A21 A22] = L L^T with Linv = L^{-1}, both in place in row-major n x n blocks of
// leading dimension ld:  L11 = chol(A11); L21 = A21 L11^{-T}; L22 = chol(A22 - L21 L21^T);
// Linv21 = -Linv22 (L21 Linv11).  Every product is one large GEMM.
static void chol_inv_rec(Ctx& c, double* A, double* Li, int n, int ld, double* T) {
  if (n <= NB) {
    hipLaunchKernelGGL(k_chol_leaf, dim3(1), dim3(64), 0, c.s, A, Li, ld, n, c.flag.p);
    AMGF_LAUNCH_CHECK();
    return;
  }
  const int n1 = ((n / 2 + NB - 1) / NB) * NB, n2 = n - n1;
  double* A21 = A + int64_t(n1) * ld;
  double* A22 = A21 + n1;
  double* Li21 = Li + int64_t(n1) * ld;
  double* Li22 = Li21 + n1;
  chol_inv_rec(c, A, Li, n1, ld, T);
  dgemm(c, true, n2, n1, n1, 1.0, A21, ld, Li, ld, 0.0, T, n1, false);       // L21
  hipLaunchKernelGGL(k_copy2d, dim3(grid_for(int64_t(n2) * n1, 256)), dim3(256), 0, c.s, n2,
                     n1, T, n1, A21, ld);
  dgemm(c, true, n2, n2, n1, -1.0, A21, ld, A21, ld, 1.0, A22, ld, true);     // A22 -= L21 L21^T
  chol_inv_rec(c, A22, Li22, n2, ld, T);
  dgemm(c, false, n2, n1, n1, 1.0, A21, ld, Li, ld, 0.0, T, n1, false);      // L21 Linv11
  dgemm(c, false, n2, n1, n2, -1.0, Li22, ld, T, n1, 0.0, Li21, ld, false);  // Linv21
}

void dense_cholesky_inverse(Ctx& c, double* A, int n, DBuf<double>& Linv) {
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  Linv.alloc(size_t(n) * n);
  AMGF_HIP(hipMemsetAsync(Linv.p, 0, Linv.bytes(), c.s));
  DBuf<double> T(size_t(n) * ((n + 1) / 2 + NB));
  chol_inv_rec(c, A, Linv.p, n, n, T.p);
  AMGF_REQUIRE(d2h_scalar(c.flag.p, c.s) == 0, AMGF_ENOTSPD,
               "dense Cholesky: non-positive pivot (matrix not SPD)");
}

// ---------------------------------------------------------------- solves
// y = Linv x  (one wavefront per row, lower triangle only)
__global__ void k_trmv_lower(int n, const double* __restrict__ L, const double* __restrict__ x,
                             double* __restrict__ y) {
  const int r = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  const double* row = L + int64_t(r) * n;
  double s = 0.0;
  for (int j = lane; j <= r; j += 64) s += row[j] * x[j];
  s = wave_sum(s);
  if (lane == 0) y[r] = s;
}
// z = Linv^T y  (thread per column, rows j..n-1)
__global__ void k_trmv_lower_t(int n, const double* __restrict__ L, const double* __restrict__ y,
                               double* __restrict__ z) {
  const int cidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (cidx >= n) return;
  double s = 0.0;
  for (int i = cidx; i < n; ++i) s += L[int64_t(i) * n + cidx] * y[i];
  z[cidx] = s;
}

void dense_solve(Ctx& c, const double* Linv, int n, const double* b, double* x, double* tmp) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_trmv_lower, dim3((n + 3) / 4), dim3(256), 0, c.s, n, Linv, b, tmp);
  hipLaunchKernelGGL(k_trmv_lower_t, dim3(grid_for(n, 128)), dim3(128), 0, c.s, n, Linv, tmp,
                     x);
  AMGF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- dense gathers
// BSR (b x b) -> dense n x n (all block rows/cols)
__global__ void k_bsr_to_dense(int nrows, int b, const int* __restrict__ rp,
                               const int* __restrict__ col, const double* __restrict__ val,
                               double* __restrict__ Dn, int ld) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  for (int k = rp[r]; k < rp[r + 1]; ++k)
    for (int p = 0; p < b; ++p)
      for (int q = 0; q < b; ++q)
        Dn[int64_t(r * b + p) * ld + col[k] * b + q] = val[int64_t(k) * b * b + p * b + q];
}

void bsr_to_dense(Ctx& c, const BSR& A, double* Dn) {
  const int n = A.nrows * A.br;
  AMGF_HIP(hipMemsetAsync(Dn, 0, size_t(n) * n * sizeof(double), c.s));
  hipLaunchKernelGGL(k_bsr_to_dense, dim3(grid_for(A.nrows, 128)), dim3(128), 0, c.s, A.nrows,
                     A.br, A.rowptr.p, A.col.p, A.val.p, Dn, n);
  AMGF_LAUNCH_CHECK();
}

// A_w = S[I_c, I_c] for a 3x3-block S; pos[dof] = index in I_c or -1
__global__ void k_gather_aw(int nc, const int* __restrict__ ic, const int* __restrict__ pos,
                            const int* __restrict__ rp, const int* __restrict__ col,
                            const double* __restrict__ val, double* __restrict__ Aw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const int dof = ic[i], a = dof / 3, p = dof % 3;
  for (int k = rp[a]; k < rp[a + 1]; ++k)
    for (int q = 0; q < 3; ++q) {
      const int j = pos[3 * col[k] + q];
      if (j >= 0) Aw[int64_t(i) * nc + j] = val[int64_t(k) * 9 + p * 3 + q];
    }
}


__global__ void k_pos_map(int nc, const int* __restrict__ ic, int* __restrict__ pos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc) pos[ic[i]] = i;
}

// sparse A_w = S[I_c, I_c] (scalar CSR, columns ascending) for refinement residuals
__global__ void k_aw_csr(int nc, int fill, const int* __restrict__ ic, const int* __restrict__ pos,
                         const int* __restrict__ rp, const int* __restrict__ col,
                         const double* __restrict__ val, int* __restrict__ cnt,
                         const int* __restrict__ orp, int* __restrict__ ocol,
                         double* __restrict__ oval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const int dof = ic[i], a = dof / 3, p = dof % 3;
  int o = fill ? orp[i] : 0;
  for (int k = rp[a]; k < rp[a + 1]; ++k)
    for (int q = 0; q < 3; ++q) {
      const int j = pos[3 * col[k] + q];
      if (j < 0) continue;
      if (fill) {
        ocol[o] = j;
        oval[o] = val[int64_t(k) * 9 + p * 3 + q];
      }
      ++o;
    }
  if (!fill) cnt[i] = o;
}

void filter_csr(Ctx& c, const BSR& S, const int* Ic, int nc, DBuf<int>& rp, DBuf<int>& col,
                DBuf<double>& val) {
  const int n = S.nrows * 3;
  DBuf<int> pos(std::max(n, 1)), cnt(std::max(nc, 1));
  AMGF_HIP(hipMemsetAsync(pos.p, 0xff, pos.bytes(), c.s));
  hipLaunchKernelGGL(k_pos_map, dim3(grid_for(nc, 256)), dim3(256), 0, c.s, nc, Ic, pos.p);
  hipLaunchKernelGGL(k_aw_csr, dim3(grid_for(nc, 128)), dim3(128), 0, c.s, nc, 0, Ic, pos.p,
                     S.rowptr.p, S.col.p, S.val.p, cnt.p, nullptr, nullptr, nullptr);
  rp.alloc(size_t(nc) + 1);
  const int nnz = scan_exclusive(c, cnt.p, rp.p, nc);
  col.alloc(std::max(nnz, 1));
  val.alloc(std::max(nnz, 1));
  hipLaunchKernelGGL(k_aw_csr, dim3(grid_for(nc, 128)), dim3(128), 0, c.s, nc, 1, Ic, pos.p,
                     S.rowptr.p, S.col.p, S.val.p, nullptr, rp.p, col.p, val.p);
  AMGF_LAUNCH_CHECK();
}

// res = r - A w for a scalar CSR A (one thread per row)
__global__ void k_csr_residual(int n, const int* __restrict__ rp, const int* __restrict__ col,
                               const double* __restrict__ val, const double* __restrict__ w,
                               const double* __restrict__ r, double* __restrict__ res) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * w[col[k]];
  res[i] = r[i] - s;
}

void csr_residual(Ctx& c, int n, const int* rp, const int* col, const double* val,
                  const double* w, const double* r, double* res) {
  if (n) hipLaunchKernelGGL(k_csr_residual, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, rp, col,
                            val, w, r, res);
  AMGF_LAUNCH_CHECK();
}

// square BSR (b x b) -> scalar CSR
__global__ void k_bsr_csr(int nrows, int b, const int* __restrict__ rp, const int* __restrict__ col,
                          const double* __restrict__ val, int* __restrict__ orp,
                          int* __restrict__ ocol, double* __restrict__ oval) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int len = (rp[r + 1] - rp[r]) * b;
  for (int p = 0; p < b; ++p) {
    const int row = r * b + p;
    int o = rp[r] * b * b + p * len;
    if (r == nrows - 1 && p == b - 1) orp[row + 1] = o + len;
    orp[row] = o;
    for (int k = rp[r]; k < rp[r + 1]; ++k)
      for (int q = 0; q < b; ++q) {
        ocol[o] = col[k] * b + q;
        oval[o] = val[int64_t(k) * b * b + p * b + q];
        ++o;
      }
  }
}

void bsr_to_csr(Ctx& c, const BSR& A, DBuf<int>& rp, DBuf<int>& col, DBuf<double>& val) {
  const int64_t nnz = A.nnzb * A.br * A.bc;
  rp.alloc(size_t(A.nrows) * A.br + 1);
  col.alloc(std::max<int64_t>(nnz, 1));
  val.alloc(std::max<int64_t>(nnz, 1));
  hipLaunchKernelGGL(k_bsr_csr, dim3(grid_for(A.nrows, 128)), dim3(128), 0, c.s, A.nrows, A.br,
                     A.rowptr.p, A.col.p, A.val.p, rp.p, col.p, val.p);
  AMGF_LAUNCH_CHECK();
}

void gather_filter_matrix(Ctx& c, const BSR& S, const int* Ic, int nc, double* Aw) {
  const int n = S.nrows * 3;
  DBuf<int> pos(std::max(n, 1));
  AMGF_HIP(hipMemsetAsync(pos.p, 0xff, pos.bytes(), c.s));
  AMGF_HIP(hipMemsetAsync(Aw, 0, size_t(nc) * nc * sizeof(double), c.s));
  hipLaunchKernelGGL(k_pos_map, dim3(grid_for(nc, 256)), dim3(256), 0, c.s, nc, Ic, pos.p);
  hipLaunchKernelGGL(k_gather_aw, dim3(grid_for(nc, 128)), dim3(128), 0, c.s, nc, Ic, pos.p,
                     S.rowptr.p, S.col.p, S.val.p, Aw);
  AMGF_LAUNCH_CHECK();
}

}  // namespace amgf

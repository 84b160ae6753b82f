// Dense FP64 SPD factorisation used for the coarsest level and the filter A_w.
//
// A = L L^T by a right-looking blocked Cholesky (64-wide panels, tiled DGEMM trailing
// update), then Linv = L^{-1} by block rows, so that each later solve
// x = Linv^T (Linv b) is two bandwidth-bound matrix-vector products instead of a
// sequence of dependent triangular steps.
#include "dense.h"

namespace amgf {

constexpr int NB = 64;

// ---------------------------------------------------------------- unblocked panel
__global__ void __launch_bounds__(256) k_potf2(double* A, int lda, int k0, int kb, int* info) {
  __shared__ double L[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < kb * kb; e += 256) {
    const int i = e / kb, j = e % kb;
    L[i][j] = A[int64_t(k0 + i) * lda + k0 + j];
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (tid == 0) {
      const double p = L[j][j];
      if (!(p > 0.0)) atomicOr(info, 1);
      L[j][j] = sqrt(p > 0.0 ? p : 1.0);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < kb; i += 256) L[i][j] /= L[j][j];
    __syncthreads();
    const int m = kb - j - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) L[i][l] -= L[i][j] * L[l][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < kb * kb; e += 256) {
    const int i = e / kb, j = e % kb;
    A[int64_t(k0 + i) * lda + k0 + j] = (j <= i) ? L[i][j] : 0.0;
  }
}

// rows below the panel: X L_kk^T = A_ik (forward substitution per row)
__global__ void __launch_bounds__(256) k_trsm_panel(double* A, int lda, int n, int k0, int kb) {
  __shared__ double L[NB][NB + 1];
  for (int e = threadIdx.x; e < kb * kb; e += 256) {
    const int i = e / kb, j = e % kb;
    L[i][j] = A[int64_t(k0 + i) * lda + k0 + j];
  }
  __syncthreads();
  const int r = k0 + kb + blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  double* row = A + int64_t(r) * lda + k0;
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = (j < kb) ? row[j] : 0.0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < kb) {
      double s = x[j];
#pragma unroll
      for (int l = 0; l < j; ++l) s -= x[l] * L[j][l];
      x[j] = s / L[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < kb) row[j] = x[j];
}

// ---------------------------------------------------------------- tiled DGEMM
// C[M x N] = beta C + alpha A[M x K] op(B);  op(B) = B^T (B is N x K) or B (K x N).
// 64x64 tiles, 256 threads, 4x4 outputs per thread.  lower_only skips tiles strictly
// above the diagonal (row-block origin offset by diag_off).
template <bool TB>
__global__ void __launch_bounds__(256) k_dgemm(int M, int N, int K, double alpha,
                                               const double* __restrict__ A, int lda,
                                               const double* __restrict__ B, int ldb,
                                               double beta, double* __restrict__ C, int ldc,
                                               int lower_only) {
  const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
  if (lower_only && bn > bm + 63) return;
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = threadIdx.x + 256 * t;     // 0..1023
      const int kk = e & 15, rr = e >> 4;      // rr 0..63
      const int gr = bm + rr, gk = k0 + kk;
      As[kk][rr] = (gr < M && gk < K) ? A[int64_t(gr) * lda + gk] : 0.0;
      const int gc = bn + rr;
      double bv = 0.0;
      if (TB) {
        if (gc < N && gk < K) bv = B[int64_t(gc) * ldb + gk];
      } else {
        const int kk2 = e >> 6, cc = e & 63;   // coalesced along N for B (K x N)
        const int gk2 = k0 + kk2, gc2 = bn + cc;
        if (gk2 < K && gc2 < N) bv = B[int64_t(gk2) * ldb + gc2];
        Bs[kk2][cc] = bv;
        continue;
      }
      Bs[kk][rr] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = bm + ty + 16 * i;
    if (r >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cidx = bn + tx + 16 * j;
      if (cidx >= N) continue;
      double* cp = C + int64_t(r) * ldc + cidx;
      *cp = alpha * acc[i][j] + (beta == 0.0 ? 0.0 : beta * *cp);
    }
  }
}

void dgemm(Ctx& c, bool transB, int M, int N, int K, double alpha, const double* A, int lda,
           const double* B, int ldb, double beta, double* C, int ldc, bool lower_only) {
  if (M <= 0 || N <= 0) return;
  const dim3 g((N + 63) / 64, (M + 63) / 64);
  if (transB)
    hipLaunchKernelGGL(k_dgemm<true>, g, dim3(256), 0, c.s, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc, int(lower_only));
  else
    hipLaunchKernelGGL(k_dgemm<false>, g, dim3(256), 0, c.s, M, N, K, alpha, A, lda, B, ldb,
                       beta, C, ldc, int(lower_only));
  AMGF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- inverse of a diagonal block
// X = L_ii^{-1} (lower triangular), one column per thread.
__global__ void __launch_bounds__(64) k_trtri_diag(const double* L, int lda, int k0, int kb,
                                                   double* X, int ldx) {
  __shared__ double Ls[NB][NB + 1];
  for (int e = threadIdx.x; e < kb * kb; e += 64) {
    const int i = e / kb, j = e % kb;
    Ls[i][j] = L[int64_t(k0 + i) * lda + k0 + j];
  }
  __syncthreads();
  const int cidx = threadIdx.x;
  if (cidx >= kb) return;
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = 0.0;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i < kb && i >= cidx) {
      double s = (i == cidx) ? 1.0 : 0.0;
#pragma unroll
      for (int l = 0; l < i; ++l) s -= Ls[i][l] * x[l];
      x[i] = s / Ls[i][i];
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < kb) X[int64_t(k0 + i) * ldx + k0 + cidx] = x[i];
}

void dense_cholesky_inverse(Ctx& c, double* A, int n, DBuf<double>& Linv) {
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = std::min(NB, n - k0);
    hipLaunchKernelGGL(k_potf2, dim3(1), dim3(256), 0, c.s, A, n, k0, kb, c.flag.p);
    const int rest = n - k0 - kb;
    if (rest > 0) {
      hipLaunchKernelGGL(k_trsm_panel, dim3((rest + 255) / 256), dim3(256), 0, c.s, A, n, n, k0,
                         kb);
      // trailing lower update: A22 -= L21 L21^T
      double* A21 = A + int64_t(k0 + kb) * n + k0;
      double* A22 = A + int64_t(k0 + kb) * n + k0 + kb;
      dgemm(c, true, rest, rest, kb, -1.0, A21, n, A21, n, 1.0, A22, n, true);
    }
    AMGF_LAUNCH_CHECK();
  }
  AMGF_REQUIRE(d2h_scalar(c.flag.p, c.s) == 0, AMGF_ENOTSPD,
               "dense Cholesky: non-positive pivot (matrix not SPD)");
  // Linv by block rows: Linv_ii = inv(L_ii); Linv[i, :i] = -Linv_ii (L[i, :i] Linv[:i, :i])
  Linv.alloc(size_t(n) * n);
  AMGF_HIP(hipMemsetAsync(Linv.p, 0, Linv.bytes(), c.s));
  DBuf<double> T(size_t(NB) * n);
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = std::min(NB, n - k0);
    hipLaunchKernelGGL(k_trtri_diag, dim3(1), dim3(64), 0, c.s, A, n, k0, kb, Linv.p, n);
    AMGF_LAUNCH_CHECK();
    if (k0 > 0) {
      dgemm(c, false, kb, k0, k0, 1.0, A + int64_t(k0) * n, n, Linv.p, n, 0.0, T.p, k0, false);
      dgemm(c, false, kb, k0, kb, -1.0, Linv.p + int64_t(k0) * n + k0, n, T.p, k0, 0.0,
            Linv.p + int64_t(k0) * n, n, false);
    }
  }
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

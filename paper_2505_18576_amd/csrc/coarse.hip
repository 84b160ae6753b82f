// Dense inverse of the coarsest operator (see coarse.h).
//
// Sweep of pivot k on a symmetric matrix with d = A_kk (Goodnight's sweep operator):
//   A_ij -= A_ik A_kj / d (i, j != k),  A_ik /= d,  A_kj /= d,  A_kk = -1/d;
// after sweeping every k the array holds -A^{-1}.  The sweep keeps the matrix symmetric,
// so only the upper triangle is updated (and mirrored at the end).  Step k reads column k
// of the current matrix from a separate vector, so the threads of one step never read what
// another writes; the threads holding column (or row) k+1 write it for the next step into
// the other vector.
#include "coarse.h"

namespace amgf {

namespace {

__global__ void k_bsr_to_dense(int nrows, int b, const int* __restrict__ rp,
                               const int* __restrict__ col, const double* __restrict__ val,
                               int n, double* __restrict__ X) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;       // scalar row
  if (r >= nrows * b) return;
  const int a = r / b, p = r - a * b;
  for (int e = rp[a]; e < rp[a + 1]; ++e)
    for (int q = 0; q < b; ++q)
      X[int64_t(r) * n + int64_t(col[e]) * b + q] = val[(int64_t(e) * b + p) * b + q];
}

__global__ void k_column(int n, const double* __restrict__ X, int k, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = X[int64_t(i) * n + k];
}

// one step on the upper triangle (j >= i) in 16 x 16 tiles; tiles below the diagonal exit
__global__ void __launch_bounds__(256) k_sweep(int n, double* __restrict__ X, int k,
                                               const double* __restrict__ v,
                                               double* __restrict__ vnext,
                                               int* __restrict__ flag) {
  if (blockIdx.y > blockIdx.x) return;
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  if (i >= n || j >= n || j < i) return;
  const int64_t t = int64_t(i) * n + j;
  const double d = v[k];
  double x;
  if (i == k && j == k) {
    if (!(d > 0.0)) atomicOr(flag, 4);
    x = -1.0 / d;
  } else if (i == k) {
    x = v[j] / d;
  } else if (j == k) {
    x = v[i] / d;
  } else {
    x = X[t] - v[i] * (v[j] / d);
  }
  X[t] = x;
  // column k + 1 of the symmetric matrix for the next step
  if (j == k + 1) vnext[i] = x;
  else if (i == k + 1) vnext[j] = x;
}

// lower triangle from the upper one
__global__ void k_mirror(int n, double* __restrict__ X) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * n) return;
  const int i = int(t / n), j = int(t - int64_t(i) * n);
  if (j < i) X[t] = X[int64_t(j) * n + i];
}

// y_i = -sum_j X_ij b_j, one wavefront per row
__global__ void __launch_bounds__(256) k_neg_gemv(int n, const double* __restrict__ X,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ y) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const double* row = X + int64_t(i) * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += row[j] * b[j];
  s = wave_sum(s);
  if (lane == 0) y[i] = -s;
}

}  // namespace

void DenseInverse::setup(Ctx& c, const BSR& A) {
  AMGF_REQUIRE(A.br == A.bc && A.nrows == A.ncols, AMGF_EINVAL, "square BSR expected");
  n = A.nrows * A.br;
  X.alloc(size_t(n) * n);
  if (!n) return;
  AMGF_HIP(hipMemsetAsync(X.p, 0, X.bytes(), c.s));
  hipLaunchKernelGGL(k_bsr_to_dense, dim3(grid_for(n, 256)), dim3(256), 0, c.s, A.nrows, A.br,
                     A.rowptr.p, A.col.p, A.val.p, n, X.p);
  AMGF_LAUNCH_CHECK();
  DBuf<double> v0(n), v1(n);
  hipLaunchKernelGGL(k_column, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, X.p, 0, v0.p);
  AMGF_LAUNCH_CHECK();
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  const unsigned nt = unsigned((n + 15) / 16);
  for (int k = 0; k < n; ++k) {
    const double* v = (k & 1) ? v1.p : v0.p;
    double* vn = (k & 1) ? v0.p : v1.p;
    hipLaunchKernelGGL(k_sweep, dim3(nt, nt), dim3(256), 0, c.s, n, X.p, k, v, vn, c.flag.p);
  }
  hipLaunchKernelGGL(k_mirror, dim3(grid_for(int64_t(n) * n, 256)), dim3(256), 0, c.s, n, X.p);
  AMGF_LAUNCH_CHECK();
  AMGF_REQUIRE(d2h_scalar(c.flag.p, c.s) == 0, AMGF_ENOTSPD,
               "coarsest operator is not positive definite");
}

void DenseInverse::solve(Ctx& c, const double* b, double* x) const {
  if (!n) return;
  hipLaunchKernelGGL(k_neg_gemv, dim3(grid_for(n, 4)), dim3(256), 0, c.s, n, X.p, b, x);
  AMGF_LAUNCH_CHECK();
}

}  // namespace amgf

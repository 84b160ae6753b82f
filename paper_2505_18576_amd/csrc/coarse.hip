// Dense inverse of the coarsest operator (see coarse.h).
//
// Sweep of pivot k on a symmetric matrix with d = A_kk (Goodnight's sweep operator):
//   A_ij -= A_ik A_kj / d (i, j != k),  A_ik /= d,  A_kj /= d,  A_kk = -1/d;
// after sweeping every k the array holds -A^{-1}.  Sweeping the pivots of a block K one by
// one equals the block sweep with P = A_KK:
//   A_ij -= A_iK P^{-1} A_Kj,  A_iK <- A_iK P^{-1},  A_Kj <- P^{-1} A_Kj,  A_KK <- -P^{-1},
// so the pivots are taken SWEEP_B at a time: one workgroup sweeps the small block P in LDS,
// then the rows of K are copied (V = A_K.) and multiplied (W = P^{-1} V), then every entry
// is updated from V and W, which no thread of that step writes.  The sweep keeps the matrix
// symmetric, so only the upper triangle is updated (and mirrored at the end).
#include "coarse.h"

#include <algorithm>

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

constexpr int SWEEP_B = 32;
static_assert(SWEEP_B % 4 == 0, "four wavefronts share a sweep block's rows");

// entry (i, j) of the symmetric matrix held in the upper triangle
__device__ __forceinline__ double sym_at(const double* X, int n, int i, int j) {
  return i <= j ? X[int64_t(i) * n + j] : X[int64_t(j) * n + i];
}

// Pi = P^{-1} for P = A_KK (K = k0 .. k0+kb-1) by the scalar sweep in LDS; flag bit 4 on a
// pivot that is not positive
__global__ void __launch_bounds__(256) k_sweep_pivot(int n, const double* __restrict__ X,
                                                     int k0, int kb, double* __restrict__ Pi,
                                                     int* __restrict__ flag) {
  __shared__ double P[SWEEP_B][SWEEP_B + 1];
  __shared__ double col[SWEEP_B];
  const int tid = threadIdx.x;
  for (int e = tid; e < kb * kb; e += 256) P[e / kb][e % kb] = sym_at(X, n, k0 + e / kb,
                                                                        k0 + e % kb);
  __syncthreads();
  for (int s = 0; s < kb; ++s) {
    if (tid < kb) col[tid] = P[tid][s];
    __syncthreads();
    const double d = col[s];
    if (tid == 0 && !(d > 0.0)) atomicOr(flag, 4);
    for (int e = tid; e < kb * kb; e += 256) {
      const int p = e / kb, q = e % kb;
      double x;
      if (p == s && q == s) x = -1.0 / d;
      else if (p == s) x = col[q] / d;
      else if (q == s) x = col[p] / d;
      else x = P[p][q] - col[p] * (col[q] / d);
      P[p][q] = x;
    }
    __syncthreads();
  }
  for (int e = tid; e < kb * kb; e += 256) Pi[e] = -P[e / kb][e % kb];
}

// V = A_K. (rows of the block, from the upper triangle) and W = Pi V for 64 columns per
// workgroup: the four wavefronts read 8 rows of V each into LDS, then each forms 8 rows of W
__global__ void __launch_bounds__(256) k_sweep_rows(int n, const double* __restrict__ X,
                                                    int k0, int kb,
                                                    const double* __restrict__ Pi,
                                                    double* __restrict__ V,
                                                    double* __restrict__ W) {
  __shared__ double vs[SWEEP_B][64];
  const int jj = threadIdx.x & 63, q0 = (threadIdx.x >> 6) * (SWEEP_B / 4);
  const int j = blockIdx.x * 64 + jj;
#pragma unroll
  for (int q = q0; q < q0 + SWEEP_B / 4; ++q) {
    const double v = (q < kb && j < n) ? sym_at(X, n, k0 + q, j) : 0.0;
    vs[q][jj] = v;
    if (q < kb && j < n) V[int64_t(q) * n + j] = v;
  }
  __syncthreads();
  if (j >= n) return;
  for (int p = q0; p < q0 + SWEEP_B / 4 && p < kb; ++p) {
    double w = 0.0;
#pragma unroll
    for (int q = 0; q < SWEEP_B; ++q)
      if (q < kb) w += Pi[p * kb + q] * vs[q][jj];
    W[int64_t(p) * n + j] = w;
  }
}

// one block step on the upper triangle (j >= i) in 16 x 16 tiles, the tile's rows of V and
// columns of W staged in LDS; tiles below the diagonal exit
__global__ void __launch_bounds__(256) k_sweep_update(int n, double* __restrict__ X, int k0,
                                                      int kb, const double* __restrict__ Pi,
                                                      const double* __restrict__ V,
                                                      const double* __restrict__ W) {
  if (blockIdx.y > blockIdx.x) return;
  __shared__ double vt[SWEEP_B][16], wt[SWEEP_B][16];
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  for (int e = threadIdx.x; e < SWEEP_B * 16; e += 256) {
    const int p = e >> 4, c = e & 15;
    vt[p][c] = (p < kb && i0 + c < n) ? V[int64_t(p) * n + i0 + c] : 0.0;
    wt[p][c] = (p < kb && j0 + c < n) ? W[int64_t(p) * n + j0 + c] : 0.0;
  }
  __syncthreads();
  const int i = i0 + ti, j = j0 + tj;
  if (i >= n || j >= n || j < i) return;
  const bool iK = i >= k0 && i < k0 + kb, jK = j >= k0 && j < k0 + kb;
  const int64_t t = int64_t(i) * n + j;
  double x;
  if (iK && jK) {
    x = -Pi[(i - k0) * kb + (j - k0)];
  } else if (iK) {
    x = wt[i - k0][tj];
  } else if (jK) {
    x = W[int64_t(j - k0) * n + i];
  } else {
    double acc = 0.0;
    for (int p = 0; p < kb; ++p) acc += vt[p][ti] * wt[p][tj];
    x = X[t] - acc;
  }
  X[t] = x;
}

// lower triangle from the upper one
__global__ void k_mirror(int n, double* __restrict__ X) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * n) return;
  const int i = int(t / n), j = int(t - int64_t(i) * n);
  if (j < i) X[t] = X[int64_t(j) * n + i];
}

// y_i = -sum_j X_ij b_j, one wavefront per row (FP64 sums; b and y FP64, or FP32 widened
// exactly and rounded once)
template <class TB>
__global__ void __launch_bounds__(256) k_neg_gemv(int n, const double* __restrict__ X,
                                                  const TB* __restrict__ b,
                                                  TB* __restrict__ y) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const double* row = X + int64_t(i) * n;
  double s = 0.0;
  // unrolled so that several loads of the row are in flight (the sum keeps its order)
#pragma unroll 8
  for (int j = lane; j < n; j += 64) s += row[j] * double(b[j]);
  s = wave_sum(s);
  if (lane == 0) y[i] = TB(-s);
}

}  // namespace

bool DenseInverse::setup(Ctx& c, const BSR& A) {
  AMGF_REQUIRE(A.br == A.bc && A.nrows == A.ncols, AMGF_EINVAL, "square BSR expected");
  n = A.nrows * A.br;
  X.alloc(size_t(n) * n);
  if (!n) return true;
  AMGF_HIP(hipMemsetAsync(X.p, 0, X.bytes(), c.s));
  hipLaunchKernelGGL(k_bsr_to_dense, dim3(grid_for(n, 256)), dim3(256), 0, c.s, A.nrows, A.br,
                     A.rowptr.p, A.col.p, A.val.p, n, X.p);
  AMGF_LAUNCH_CHECK();
  DBuf<double> Pi(SWEEP_B * SWEEP_B), V(size_t(SWEEP_B) * n), W(size_t(SWEEP_B) * n);
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  const unsigned nt = unsigned((n + 15) / 16);
  for (int k0 = 0; k0 < n; k0 += SWEEP_B) {
    const int kb = std::min(SWEEP_B, n - k0);
    hipLaunchKernelGGL(k_sweep_pivot, dim3(1), dim3(256), 0, c.s, n, X.p, k0, kb, Pi.p,
                       c.flag.p);
    hipLaunchKernelGGL(k_sweep_rows, dim3(grid_for(n, 64)), dim3(256), 0, c.s, n, X.p, k0, kb,
                       Pi.p, V.p, W.p);
    hipLaunchKernelGGL(k_sweep_update, dim3(nt, nt), dim3(256), 0, c.s, n, X.p, k0, kb, Pi.p,
                       V.p, W.p);
  }
  AMGF_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_mirror, dim3(grid_for(int64_t(n) * n, 256)), dim3(256), 0, c.s, n, X.p);
  AMGF_LAUNCH_CHECK();
  return d2h_scalar(c.flag.p, c.s) == 0;
}

void DenseInverse::solve(Ctx& c, const double* b, double* x) const {
  if (!n) return;
  hipLaunchKernelGGL(k_neg_gemv<double>, dim3(grid_for(n, 4)), dim3(256), 0, c.s, n, X.p, b,
                     x);
  AMGF_LAUNCH_CHECK();
}

void DenseInverse::solve_f32(Ctx& c, const float* b, float* x) const {
  if (!n) return;
  hipLaunchKernelGGL(k_neg_gemv<float>, dim3(grid_for(n, 4)), dim3(256), 0, c.s, n, X.p, b,
                     x);
  AMGF_LAUNCH_CHECK();
}

}  // namespace amgf

// Scalar CSR views used by the direct solvers: A_w = S[I_c, I_c] of the filter and the
// coarsest level's operator.
#include "csr.h"

namespace amgf {

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

}  // namespace amgf

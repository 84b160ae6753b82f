// Dense FP64 factorisation helpers (dense.hip).
#pragma once
#include "common.h"

namespace amgf {

void dgemm(Ctx& c, bool transB, int M, int N, int K, double alpha, const double* A, int lda,
           const double* B, int ldb, double beta, double* C, int ldc, bool lower_only);
// A (n x n row-major, overwritten by L) -> Linv = L^{-1}; throws ENOTSPD on a bad pivot
void dense_cholesky_inverse(Ctx& c, double* A, int n, DBuf<double>& Linv);
// x = Linv^T (Linv b); tmp has n entries
void dense_solve(Ctx& c, const double* Linv, int n, const double* b, double* x, double* tmp);
void bsr_to_dense(Ctx& c, const BSR& A, double* Dn);
void gather_filter_matrix(Ctx& c, const BSR& S, const int* Ic, int nc, double* Aw);
// A_w = S[I_c, I_c] as scalar CSR (for refinement residuals)
void filter_csr(Ctx& c, const BSR& S, const int* Ic, int nc, DBuf<int>& rp, DBuf<int>& col,
                DBuf<double>& val);
// square BSR -> scalar CSR (rows ordered block row by block row)
void bsr_to_csr(Ctx& c, const BSR& A, DBuf<int>& rp, DBuf<int>& col, DBuf<double>& val);
// res = r - A w (scalar CSR)
void csr_residual(Ctx& c, int n, const int* rp, const int* col, const double* val,
                  const double* w, const double* r, double* res);

}  // namespace amgf

// Scalar CSR helpers (csr.hip).
#pragma once
#include "common.h"

namespace amgf {

// A_w = S[I_c, I_c] (3x3-block S, I_c ascending DOF indices) as scalar CSR
void filter_csr(Ctx& c, const BSR& S, const int* Ic, int nc, DBuf<int>& rp, DBuf<int>& col,
                DBuf<double>& val);
// square BSR -> scalar CSR (rows ordered block row by block row, columns ascending)
void bsr_to_csr(Ctx& c, const BSR& A, DBuf<int>& rp, DBuf<int>& col, DBuf<double>& val);

}  // namespace amgf

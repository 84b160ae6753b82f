// Block-tridiagonal (level-set ordered) FP64 Cholesky solver (btd.hip).
#pragma once
#include "common.h"

namespace amgf {

struct BTDSolver {
  int n = 0, nb = 0;                  // unknowns, diagonal blocks
  std::vector<int> hoff;              // host block offsets (nb + 1)
  std::vector<int64_t> hmoff, hgoff, hhoff;
  DBuf<int> perm, rowblk, boff;       // permuted position -> original index
  DBuf<int64_t> moff;
  DBuf<double> Linv, LinvT, G, H;
  mutable DBuf<double> work;
  // A: scalar CSR (n x n, symmetric pattern, SPD); target: minimum block size
  void setup(Ctx& c, int n, const int* rp, const int* col, const double* val, int target);
  // x = A^{-1} r
  void solve(Ctx& c, const double* r, double* x) const;
  int64_t stored_doubles() const;
};

}  // namespace amgf

// Dense inverse of a small SPD matrix for the coarsest level of the V-cycle (coarse.hip).
#pragma once
#include "common.h"

namespace amgf {

// X = A^{-1} (n x n FP64, row-major) by the in-place sweep (Gauss-Jordan without pivoting,
// which an SPD matrix never needs: every pivot is a Schur complement of A).  A solve is then
// one matrix-vector product instead of a chain of triangular-solve launches.
struct DenseInverse {
  int n = 0;
  DBuf<double> X;                // -A^{-1} after the sweep (the product negates it back)
  // A: square BSR (FP64).  Returns false when a pivot is not positive (rounding can decide
  // the sign of a pivot when A is extremely ill-conditioned); the caller then factors A by
  // another method.
  bool setup(Ctx& c, const BSR& A);
  // x = A^{-1} b (b, x: n FP64, may not alias)
  void solve(Ctx& c, const double* b, double* x) const;
  // the same for FP32 vectors: b widened exactly, the product in FP64, x rounded once
  // (bitwise the FP64 solve between the two casts)
  void solve_f32(Ctx& c, const float* b, float* x) const;
};

}  // namespace amgf

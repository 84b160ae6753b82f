// Nested-dissection multifrontal FP64 Cholesky (multifrontal.hip): the direct solver of
// the filter matrix A_w = S[I_c, I_c] (Sec. 5.1) and of the coarsest AMG level.
#pragma once
#include "common.h"

namespace amgf {

struct MFSolver {
  int n = 0, bs = 1, nn = 0;          // unknowns, unknowns per graph node, graph nodes
  int ntree = 0, ndepth = 0;          // supernodes (tree nodes), tree depth
  std::vector<int> tree_off;          // supernodes of depth d: [tree_off[d], tree_off[d+1])
  std::vector<int> h_s, h_S, h_b, h_T;   // per supernode (host): separator DOFs, padded,
                                         // boundary DOFs, 64-row tiles of the front
  std::vector<int> wl_fwd_off, wl_bwd_off;  // per depth: range of its solve work lists
  std::vector<int> ks_fwd, ks_bwd;          // per depth: column split of its solve kernels
  DBuf<int> wl_fwd, wl_bwd;                 // (supernode, row block) pairs of the solve
  std::vector<int> fp_max;                  // per depth: largest front (padded rows)
  // device: ordering and symbolic structure
  DBuf<int> snode, sep_rank, soff, sperm;   // supernode of each node; members (ascending)
  DBuf<int> tdepth, child0, child1;
  DBuf<int> bnd_off, bnd, bnd_pos;          // boundary nodes (ascending) and their
                                            // positions in the parent front
  DBuf<int> fs, fS, fb, fT;
  DBuf<int64_t> mo, vo;                     // offsets of solve matrices and vectors
  // per supernode, M = [X; G] (Fp x S: X = L11^{-1}, G = L21 X, rows padded to tiles)
  // and its transpose
  DBuf<double> M, MT;
  mutable DBuf<double> fa, fv;              // front right-hand sides and results
  // A: scalar CSR (n x n, SPD, symmetric pattern); unknowns bs*v .. bs*v+bs-1 form node v
  // and share one sparsity pattern.
  void setup(Ctx& c, int n, int bs, const int* rp, const int* col, const double* val);
  // x = A^{-1} r
  void solve(Ctx& c, const double* r, double* x) const;
  int64_t stored_doubles() const;
};

}  // namespace amgf

// Nested-dissection multifrontal FP64 Cholesky (multifrontal.hip): the direct solver of
// the filter matrix A_w = S[I_c, I_c] (Sec. 5.1) and of the coarsest AMG level.
#pragma once
#include "common.h"

namespace amgf {

// One workgroup of a solve kernel: its front's data and its row block, one entry per
// workgroup (built at setup), so a workgroup reads everything it needs in one load.
struct MFWork {
  int blk;    // row block of the front
  int S;      // padded separator DOFs: the columns of X and the first row of G
  int b;      // boundary DOFs
  int s;      // separator DOFs
  int nch;    // children: their update vectors wait in the slot arrays (0 for a leaf)
  int roff;   // tree-order position of the separator's first DOF
  int vo;     // offset of the front in the per-front vectors and slot arrays
  int uoff;   // slot-array position of the parent's front that takes the update vector
  int boff;   // offset of the front's boundary node list
  int mo;     // offset of the front's solve matrix, in 64 x 64 tiles
};

struct MFSolver {
  int n = 0, bs = 1, nn = 0;          // unknowns, unknowns per graph node, graph nodes
  int ntree = 0, ndepth = 0;          // supernodes (tree nodes), tree depth
  int tv = 0;                         // sum of the padded front sizes
  std::vector<int> tree_off;          // supernodes of depth d: [tree_off[d], tree_off[d+1])
  std::vector<int> h_s, h_S, h_b, h_T;   // per supernode (host): separator DOFs, padded,
                                         // boundary DOFs, 64-row tiles of the front
  std::vector<int> wl_fwd_off, wl_bwd_off;  // per depth: range of its solve work lists
  std::vector<int> ks_fwd, ks_bwd;          // per depth: column split of its solve kernels
  DBuf<MFWork> wl_fwd, wl_bwd;              // solve work lists
  // device: ordering and symbolic structure
  DBuf<int> snode, sep_rank, soff, sperm;   // supernode of each node; members (ascending)
  DBuf<int> tdepth, child0, child1;
  DBuf<int> bnd_off, bnd, bnd_pos;          // boundary nodes (ascending) and their
                                            // positions in the parent front
  DBuf<int> bnd_tp;                         // boundary nodes as tree-order node positions
  DBuf<int> tdof;                           // tree order: DOF of each position
  DBuf<int> fs, fS, fb, fT;
  DBuf<int64_t> mo, vo;                     // offsets of solve matrices and vectors
  // per supernode, M = [X; G] (Fp x S: X = L11^{-1}, G = L21 X, rows padded to tiles)
  // and its transpose
  DBuf<double> M, MT;
  // forward results y = X f_s per front; two slot arrays (child 0, child 1) per front that
  // hold the children's update vectors at the front's positions (zero elsewhere, set at
  // setup); tree-order copies of the right-hand side and solution for solve()
  mutable DBuf<double> fv, us, rt, xt;
  // A: scalar CSR (n x n, SPD, symmetric pattern); unknowns bs*v .. bs*v+bs-1 form node v
  // and share one sparsity pattern.
  void setup(Ctx& c, int n, int bs, const int* rp, const int* col, const double* val);
  // x = A^{-1} r
  void solve(Ctx& c, const double* r, double* x) const;
  // the same with r and x in tree order: position q holds unknown tdof[q] (the members of
  // each supernode together, supernodes in the order of the tree)
  void solve_tree(Ctx& c, const double* r, double* x) const;
  // out[q] = idx[tdof[q]]: an index array over the unknowns, put in tree order
  void tree_index(Ctx& c, const int* idx, int* out) const;
  int64_t stored_doubles() const;
};

}  // namespace amgf

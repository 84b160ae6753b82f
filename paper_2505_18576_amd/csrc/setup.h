// Declarations of the hierarchy-setup helpers (setup.hip).
#pragma once
#include "common.h"

namespace amgf {

// aggregation graph (CSR, no self loops) with per-edge weights
struct Graph {
  int n = 0;
  int64_t nnz = 0;
  DBuf<int> rowptr, col;
  DBuf<double> w;
};

__global__ void k_fill_ones(double* w, int64_t n);
__global__ void k_nonneg_mask(int n, const int* __restrict__ a, int* __restrict__ m);
__global__ void k_diag_pos(int nrows, const int* __restrict__ rp, const int* __restrict__ col,
                           int* __restrict__ dpos);

void j_to_node_blocks(Ctx& c, int m, int n_nodes, const int* rp, const int* col,
                      const double* val, BSR& J);
void contact_operator(Ctx& c, const BSR& J, const BSR& JT, const double* D, BSR& C);
void strength_graph(Ctx& c, const BSR& A, double theta, Graph& G);
void decoupled_dofs(Ctx& c, const BSR& A, DBuf<unsigned char>& dec);
int mis2_aggregate(Ctx& c, const Graph& G, int level, DBuf<int>& agg, DBuf<int>& root_flag,
                   int* rounds_out);
void coarse_graph(Ctx& c, const Graph& G, const int* agg, int n_agg, const int* moff,
                  const int* members, Graph& Gc);
// P_t and R of every aggregate for nc near-null vectors (level 0: 6 rigid-body modes from
// coords, or 3 translations; coarser levels: the rows of the previous R, br == nc)
void tentative_prolongator(Ctx& c, int br, int nc, int n_nodes, int n_agg, const int* moff,
                           const int* members, bool level0, const double* coords,
                           const unsigned char* dec, const double* Rprev, double qr_tol,
                           DBuf<double>& Pt, DBuf<double>& R, DBuf<unsigned char>& dead);
void smooth_prolongator(Ctx& c, const BSR& A, const int* agg, int n_agg, int nc,
                        const double* Pt, const double* d, double omega, BSR& P);
void spgemm(Ctx& c, const BSR& A, const BSR& B, BSR& C);
void dead_identity(Ctx& c, BSR& Kc, const unsigned char* dead);
// Bound-constraint barrier diagonal on a 3x3 stiffness: K_aa(q,q) = K0 + E (E may be null,
// restoring K0).  The first call records the original diagonal entries K0 in k0.
void bound_diagonal(Ctx& c, BSR& K, const double* E, DBuf<double>& k0);
void l1_norms(Ctx& c, const BSR& A, DBuf<double>& d);
int filter_space_from_J(Ctx& c, const BSR& J, int n_nodes, DBuf<int>& Ic);

}  // namespace amgf

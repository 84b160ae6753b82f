// AMG hierarchy setup kernels: Schur operator, strength, MIS-2 aggregation,
// tentative and smoothed prolongators, Galerkin products.
//
// The level-0 operator and strength test are computed with separately rounded
// multiplies and adds (no contraction) in a fixed order, so they are bitwise
// reproducible; aggregation decisions on later levels are integer-only.
#include "setup.h"

#include <climits>

namespace amgf {

// ======================================================================================
// J (scalar CSR m x n) -> node blocks (1 x 3)
// ======================================================================================
__global__ void k_jnode_count(int m, const int* __restrict__ rp, const int* __restrict__ col,
                             int* __restrict__ counts) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  int n = 0, last = -1;
  for (int t = rp[k]; t < rp[k + 1]; ++t) {
    const int nd = col[t] / 3;
    if (nd != last) { ++n; last = nd; }
  }
  counts[k] = n;
}
__global__ void k_jnode_fill(int m, const int* __restrict__ rp, const int* __restrict__ col,
                            const double* __restrict__ val, const int* __restrict__ brp,
                            int* __restrict__ bcol, double* __restrict__ bval) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  int o = brp[k] - 1, last = -1;
  for (int t = rp[k]; t < rp[k + 1]; ++t) {
    const int nd = col[t] / 3;
    if (nd != last) {
      ++o;
      last = nd;
      bcol[o] = nd;
      bval[3 * int64_t(o)] = 0.0;
      bval[3 * int64_t(o) + 1] = 0.0;
      bval[3 * int64_t(o) + 2] = 0.0;
    }
    bval[3 * int64_t(o) + col[t] % 3] = val[t];
  }
}

void j_to_node_blocks(Ctx& c, int m, int n_nodes, const int* rp, const int* col,
                      const double* val, BSR& J) {
  J.nrows = m;
  J.ncols = n_nodes;
  J.br = 1;
  J.bc = 3;
  J.rowptr.alloc(size_t(m) + 1);
  DBuf<int> counts(std::max(m, 1));
  if (m)
    hipLaunchKernelGGL(k_jnode_count, dim3(grid_for(m, 256)), dim3(256), 0, c.s, m, rp, col,
                       counts.p);
  J.nnzb = scan_exclusive(c, counts.p, J.rowptr.p, m);
  J.col.alloc(std::max<int64_t>(J.nnzb, 1));
  J.val.alloc(std::max<int64_t>(J.nnzb, 1) * 3);
  if (m)
    hipLaunchKernelGGL(k_jnode_fill, dim3(grid_for(m, 256)), dim3(256), 0, c.s, m, rp, col,
                       val, J.rowptr.p, J.col.p, J.val.p);
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// contact term C = J^T diag(D) J with a fixed rounding order
// ======================================================================================
__device__ __forceinline__ int lower_bound_i(const int* a, int lo, int hi, int key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Output-stationary: one wavefront per row a, one lane per output block (a, b).  The
// lane sums over the constraint rows k of JT row a in ascending order:
//   C_ab(p, q) = C_ab(p, q) + D_k * (J_ka[p] * J_kb[q])   (each operation rounded)
// so every entry has a fixed summation order independent of scheduling.
template <int B>
__global__ void __launch_bounds__(256) k_contact_numeric(
    int nn, const int* __restrict__ jtrp, const int* __restrict__ jtcol,
    const double* __restrict__ jtval, const int* __restrict__ jrp, const int* __restrict__ jcol,
    const double* __restrict__ jval, const double* __restrict__ D, const int* __restrict__ crp,
    const int* __restrict__ ccol, double* __restrict__ cval) {
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (a >= nn) return;
  const int t0 = jtrp[a], t1 = jtrp[a + 1];
  for (int s = crp[a] + lane; s < crp[a + 1]; s += 64) {
    const int b = ccol[s];
    double acc[B * B];
#pragma unroll
    for (int e = 0; e < B * B; ++e) acc[e] = 0.0;
    for (int t = t0; t < t1; ++t) {
      const int k = jtcol[t];
      const int u = lower_bound_i(jcol, jrp[k], jrp[k + 1], b);
      if (u >= jrp[k + 1] || jcol[u] != b) continue;
      const double Dk = D[k];
#pragma unroll
      for (int p = 0; p < B; ++p) {
        const double ja = jtval[int64_t(t) * B + p];
#pragma unroll
        for (int q = 0; q < B; ++q)
          acc[p * B + q] = add_rn(acc[p * B + q], mul_rn(Dk, mul_rn(ja, jval[int64_t(u) * B + q])));
      }
    }
    double* C = cval + int64_t(s) * B * B;
#pragma unroll
    for (int e = 0; e < B * B; ++e) C[e] = acc[e];
  }
}

void contact_operator(Ctx& c, const BSR& J, const BSR& JT, const double* D, BSR& C) {
  const int nn = J.ncols, b = J.bc;
  union_symbolic(c, nn, nn, JT.rowptr.p, JT.col.p, J.rowptr.p, J.col.p, nullptr, false,
                 nullptr, C);
  C.br = C.bc = b;
  C.val.alloc(std::max<int64_t>(C.nnzb, 1) * b * b);
  if (nn && C.nnzb) {
    const dim3 g(grid_for(nn, 4)), blk(256);
    if (b == 3)
      hipLaunchKernelGGL(k_contact_numeric<3>, g, blk, 0, c.s, nn, JT.rowptr.p, JT.col.p,
                         JT.val.p, J.rowptr.p, J.col.p, J.val.p, D, C.rowptr.p, C.col.p, C.val.p);
    else
      hipLaunchKernelGGL(k_contact_numeric<6>, g, blk, 0, c.s, nn, JT.rowptr.p, JT.col.p,
                         JT.val.p, J.rowptr.p, J.col.p, J.val.p, D, C.rowptr.p, C.col.p, C.val.p);
  }
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// level-0 strength of connection and decoupled DOFs
// ======================================================================================
__global__ void k_block_nu(int64_t nnzb, int bsz, const double* __restrict__ val,
                           double* __restrict__ nu) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nnzb) return;
  double acc = 0.0;
  for (int e = 0; e < bsz; ++e) {
    const double v = val[k * bsz + e];
    acc = add_rn(acc, mul_rn(v, v));
  }
  nu[k] = acc;
}

__global__ void k_diag_pos(int nrows, const int* __restrict__ rp, const int* __restrict__ col,
                           int* __restrict__ dpos) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int s = lower_bound_i(col, rp[r], rp[r + 1], r);
  dpos[r] = (s < rp[r + 1] && col[s] == r) ? s : -1;
}

__global__ void k_strong(int64_t nnzb, const int* __restrict__ rows, const int* __restrict__ rp,
                         const int* __restrict__ col, const double* __restrict__ nu,
                         const int* __restrict__ dpos, double theta4, int* __restrict__ strong,
                         int* flag) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nnzb) return;
  const int a = rows[k], b = col[k];
  if (a == b) { strong[k] = 0; return; }
  const int t = lower_bound_i(col, rp[b], rp[b + 1], a);
  if (t >= rp[b + 1] || col[t] != a || dpos[a] < 0 || dpos[b] < 0) {
    atomicOr(flag, 4);
    strong[k] = 0;
    return;
  }
  const double naa = nu[dpos[a]], nbb = nu[dpos[b]];
  const double lhs = mul_rn(nu[k], nu[k]);
  const double rhs = mul_rn(theta4, mul_rn(naa, nbb));
  const double lhs_t = mul_rn(nu[t], nu[t]);
  const double rhs_t = mul_rn(theta4, mul_rn(nbb, naa));
  strong[k] = (lhs >= rhs) && (lhs_t >= rhs_t);
}

__global__ void k_count_flags(int nrows, const int* __restrict__ rp, const int* __restrict__ f,
                              int* __restrict__ counts) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int n = 0;
  for (int k = rp[r]; k < rp[r + 1]; ++k) n += f[k];
  counts[r] = n;
}
// 32 lanes per row, a lane per entry (coalesced): the strong entries keep their order, each
// at the row's start plus the number of strong entries before it (ballot prefix count)
__global__ void __launch_bounds__(256) k_compact_graph(int nrows, const int* __restrict__ rp,
                                                       const int* __restrict__ col,
                                                       const int* __restrict__ f,
                                                       const double* __restrict__ nu,
                                                       const int* __restrict__ grp,
                                                       int* __restrict__ gcol,
                                                       double* __restrict__ gw) {
  const int r = int((int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 5);
  const int l = threadIdx.x & 31, half = (threadIdx.x >> 5) & 1;
  if (r >= nrows) return;
  const int k1 = rp[r + 1];
  int o = grp[r];
  for (int base = rp[r]; base < k1; base += 32) {
    const int k = base + l;
    const bool st = k < k1 && f[k];
    const unsigned m = unsigned(__ballot(st) >> (32 * half));
    if (st) {
      const int pos = o + __popc(m & ((1u << l) - 1u));
      gcol[pos] = col[k];
      gw[pos] = nu[k];
    }
    o += __popc(m);
  }
}

void strength_graph(Ctx& c, const BSR& A, double theta, Graph& G) {
  const int n = A.nrows;
  const int64_t nz = A.nnzb;
  DBuf<double> nu(std::max<int64_t>(nz, 1));
  DBuf<int> rows(std::max<int64_t>(nz, 1)), dpos(std::max(n, 1)),
      strong(std::max<int64_t>(nz, 1)), counts(std::max(n, 1));
  expand_rows(c, A.rowptr.p, n, rows.p);
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  hipLaunchKernelGGL(k_block_nu, dim3(grid_for(nz, 256)), dim3(256), 0, c.s, nz, int(A.bsz()),
                     A.val.p, nu.p);
  hipLaunchKernelGGL(k_diag_pos, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, A.rowptr.p,
                     A.col.p, dpos.p);
  const double t2 = theta * theta;
  const double t4 = t2 * t2;
  hipLaunchKernelGGL(k_strong, dim3(grid_for(nz, 256)), dim3(256), 0, c.s, nz, rows.p,
                     A.rowptr.p, A.col.p, nu.p, dpos.p, t4, strong.p, c.flag.p);
  hipLaunchKernelGGL(k_count_flags, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, A.rowptr.p,
                     strong.p, counts.p);
  AMGF_LAUNCH_CHECK();
  AMGF_REQUIRE(d2h_scalar(c.flag.p, c.s) == 0, AMGF_EINVAL,
               "operator pattern is not symmetric or lacks a diagonal block");
  G.n = n;
  G.rowptr.alloc(size_t(n) + 1);
  G.nnz = scan_exclusive(c, counts.p, G.rowptr.p, n);
  G.col.alloc(std::max<int64_t>(G.nnz, 1));
  G.w.alloc(std::max<int64_t>(G.nnz, 1));
  hipLaunchKernelGGL(k_compact_graph, dim3(grid_for(int64_t(n) * 32, 256)), dim3(256), 0, c.s, n,
                     A.rowptr.p, A.col.p, strong.p, nu.p, G.rowptr.p, G.col.p, G.w.p);
  AMGF_LAUNCH_CHECK();
}

// DOF i of node a is decoupled when every off-diagonal entry of its row is 0.
// G lanes per block row read its B x B blocks entry by entry (coalesced); each lane keeps
// a bit per row p of the block row that has an off-diagonal nonzero, OR-reduced over the
// group.
template <int B, int G>
__global__ void __launch_bounds__(256) k_decoupled(int n, const int* __restrict__ rp,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   unsigned char* __restrict__ dec) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = t / G, g = t % G;
  unsigned mask = 0;
  if (a < n) {
    const int k0 = rp[a], ne = (rp[a + 1] - k0) * B * B;
    const double* v = val + int64_t(k0) * B * B;
    for (int e = g; e < ne; e += G) {
      if (v[e] == 0.0) continue;
      const int kb = e / (B * B), rem = e - kb * B * B;
      const int p = rem / B, q = rem - p * B;
      if (col[k0 + kb] != a || p != q) mask |= 1u << p;
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) mask |= __shfl_xor(mask, o);
  if (a < n && g < B) dec[int64_t(a) * B + g] = (mask >> g) & 1u ? 0 : 1;
}

void decoupled_dofs(Ctx& c, const BSR& A, DBuf<unsigned char>& dec) {
  dec.alloc(size_t(A.nrows) * A.br);
  AMGF_REQUIRE(A.br == 3 || A.br == 6, AMGF_EINVAL, "block size");
  if (A.br == 3)
    hipLaunchKernelGGL((k_decoupled<3, 16>), dim3(grid_for(int64_t(A.nrows) * 16, 256)),
                       dim3(256), 0, c.s,
                       A.nrows, A.rowptr.p, A.col.p, A.val.p, dec.p);
  else
    hipLaunchKernelGGL((k_decoupled<6, 16>), dim3(grid_for(int64_t(A.nrows) * 16, 256)),
                       dim3(256), 0, c.s,
                       A.nrows, A.rowptr.p, A.col.p, A.val.p, dec.p);
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// MIS-2 by parallel rounds
// ======================================================================================
// state: 0 undecided, 1 root, 2 out.  code(v) = ~0 for roots, the priority key
// (fmix32(v) << 32 | v) for undecided nodes, 0 otherwise.  A round takes the maximum
// code over the distance-2 ball: a ball holding a root excludes v, a ball whose
// maximum is v's own key makes v a root.  This yields the set the sequential greedy
// pass (descending keys) produces.
__device__ __forceinline__ unsigned long long mis_code(int v, unsigned char st) {
  if (st == 1) return ~0ull;
  if (st == 0) return (static_cast<unsigned long long>(fmix32(uint32_t(v))) << 32) | uint32_t(v);
  return 0ull;
}

__global__ void k_mis_init(int n, const int* __restrict__ rp, unsigned char* __restrict__ st) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) st[v] = (rp[v + 1] > rp[v]) ? 0 : 2;
}
// ball 1: MIS_G lanes per node share its neighbour list (coalesced column reads) and combine
// their maxima by shuffles within the group
constexpr int MIS_G = 8;
__device__ __forceinline__ unsigned long long group_max_u64(unsigned long long m) {
#pragma unroll
  for (int o = MIS_G / 2; o > 0; o >>= 1) {
    const unsigned long long x = __shfl_xor(m, o, MIS_G);
    m = x > m ? x : m;
  }
  return m;
}
__global__ void k_mis_ball1(int n, const int* __restrict__ rp, const int* __restrict__ col,
                            const unsigned char* __restrict__ st,
                            unsigned long long* __restrict__ m1) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int v = int(t / MIS_G), l = int(t % MIS_G);
  if (v >= n) return;
  unsigned long long m = l == 0 ? mis_code(v, st[v]) : 0ull;
  for (int k = rp[v] + l; k < rp[v + 1]; k += MIS_G) {
    const int u = col[k];
    const unsigned long long cu = mis_code(u, st[u]);
    m = cu > m ? cu : m;
  }
  m = group_max_u64(m);
  if (l == 0) m1[v] = m;
}
// thread per node: most nodes are decided after a few rounds and leave at once
__global__ void k_mis_ball2(int n, const int* __restrict__ rp, const int* __restrict__ col,
                            const unsigned long long* __restrict__ m1,
                            unsigned char* __restrict__ st, int* __restrict__ undecided) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || st[v] != 0) return;
  unsigned long long m = m1[v];
  for (int k = rp[v]; k < rp[v + 1]; ++k) m = m1[col[k]] > m ? m1[col[k]] : m;
  if (m == ~0ull) st[v] = 2;
  else if (m == mis_code(v, 0)) st[v] = 1;
  else atomicAdd(undecided, 1);
}

// ======================================================================================
// aggregation
// ======================================================================================
__global__ void k_root_flags(int n, const unsigned char* __restrict__ st, int* __restrict__ f) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) f[v] = st[v] == 1;
}
__global__ void k_agg_phase1(int n, const int* __restrict__ rp, const int* __restrict__ col,
                             const int* __restrict__ isroot, const int* __restrict__ rid,
                             int* __restrict__ p1, int* flag) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (isroot[v]) { p1[v] = rid[v]; return; }
  int a = -1;
  for (int k = rp[v]; k < rp[v + 1]; ++k) {
    const int u = col[k];
    if (isroot[u]) {
      if (a >= 0) atomicOr(flag, 8);
      a = rid[u];
    }
  }
  p1[v] = a;
}
// Phase 2 from phase-1 state only.  Level 0: the neighbour with the largest edge weight;
// later levels: the aggregate holding most neighbours; ties -> smallest aggregate id.
__global__ void k_agg_phase2(int n, int level, const int* __restrict__ rp,
                             const int* __restrict__ col, const double* __restrict__ w,
                             const int* __restrict__ p1, int* __restrict__ agg, int* flag) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int own = p1[v];
  if (own >= 0 || rp[v + 1] == rp[v]) { agg[v] = own; return; }
  int best = -1;
  if (level == 0) {
    double bw = 0.0;
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int J = p1[col[k]];
      if (J < 0) continue;
      if (best < 0 || w[k] > bw || (w[k] == bw && J < best)) { bw = w[k]; best = J; }
    }
  } else {
    int bc = 0;
    for (int k = rp[v]; k < rp[v + 1]; ++k) {
      const int J = p1[col[k]];
      if (J < 0) continue;
      int cnt = 0;
      for (int k2 = rp[v]; k2 < rp[v + 1]; ++k2) cnt += p1[col[k2]] == J;
      if (best < 0 || cnt > bc || (cnt == bc && J < best)) { bc = cnt; best = J; }
    }
  }
  if (best < 0) atomicOr(flag, 16);
  agg[v] = best;
}

int mis2_aggregate(Ctx& c, const Graph& G, int level, DBuf<int>& agg, DBuf<int>& root_flag,
                   int* rounds_out) {
  const int n = G.n;
  DBuf<unsigned char> st(std::max(n, 1));
  DBuf<unsigned long long> m1(std::max(n, 1));
  DBuf<int> und(1);
  hipLaunchKernelGGL(k_mis_init, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, G.rowptr.p,
                     st.p);
  int rounds = 0;
  for (;;) {
    AMGF_HIP(hipMemsetAsync(und.p, 0, sizeof(int), c.s));
    hipLaunchKernelGGL(k_mis_ball1, dim3(grid_for(int64_t(n) * MIS_G, 256)), dim3(256), 0, c.s,
                       n, G.rowptr.p, G.col.p, st.p, m1.p);
    hipLaunchKernelGGL(k_mis_ball2, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, G.rowptr.p,
                       G.col.p, m1.p, st.p, und.p);
    AMGF_LAUNCH_CHECK();
    ++rounds;
    if (d2h_scalar(und.p, c.s) == 0) break;
    AMGF_REQUIRE(rounds < 10000, AMGF_EDEVICE, "MIS-2 did not terminate");
  }
  if (rounds_out) *rounds_out = rounds;
  root_flag.alloc(std::max(n, 1));
  DBuf<int> rid(size_t(n) + 1), p1(std::max(n, 1));
  hipLaunchKernelGGL(k_root_flags, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, st.p,
                     root_flag.p);
  const int n_agg = scan_exclusive(c, root_flag.p, rid.p, n);
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  hipLaunchKernelGGL(k_agg_phase1, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, G.rowptr.p,
                     G.col.p, root_flag.p, rid.p, p1.p, c.flag.p);
  agg.alloc(std::max(n, 1));
  hipLaunchKernelGGL(k_agg_phase2, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, level,
                     G.rowptr.p, G.col.p, G.w.p, p1.p, agg.p, c.flag.p);
  AMGF_LAUNCH_CHECK();
  AMGF_REQUIRE(d2h_scalar(c.flag.p, c.s) == 0, AMGF_EDEVICE,
               "aggregation invariant violated (MIS-2 not maximal or not independent)");
  return n_agg;
}

// aggregate adjacency graph of the next level
void coarse_graph(Ctx& c, const Graph& G, const int* agg, int n_agg, const int* moff,
                  const int* members, Graph& Gc) {
  BSR tmp;
  union_symbolic(c, n_agg, n_agg, moff, members, G.rowptr.p, G.col.p, agg, true, nullptr, tmp);
  Gc.n = n_agg;
  Gc.nnz = tmp.nnzb;
  Gc.rowptr = std::move(tmp.rowptr);
  Gc.col = std::move(tmp.col);
  Gc.w.alloc(std::max<int64_t>(Gc.nnz, 1));
  hipLaunchKernelGGL(k_fill_ones, dim3(grid_for(std::max<int64_t>(Gc.nnz, 1), 256)), dim3(256),
                     0, c.s, Gc.w.p, std::max<int64_t>(Gc.nnz, 1));
  AMGF_LAUNCH_CHECK();
}

__global__ void k_fill_ones(double* w, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) w[i] = 1.0;
}

// ======================================================================================
// tentative prolongator: per-aggregate Gram-Schmidt QR of the near-null space
// ======================================================================================
// One 64-lane workgroup per aggregate; lane l owns rows l, l+64, ... of the aggregate's
// (BR * k) x NC near-null matrix, which is built in place in the P_t storage and
// orthonormalised there (two projection passes per column, dead columns zeroed).  Level 0
// builds the near-null vectors (NC = 6: rigid-body modes about the aggregate centroid;
// NC = 3: translations), coarser levels take the rows of the previous QR's R.
template <int BR, int NC>
__global__ void __launch_bounds__(64) k_tentative_mem(int n_agg, const int* __restrict__ off,
                                                  const int* __restrict__ members,
                                                  int level0,
                                                  const double* __restrict__ coords,
                                                  const unsigned char* __restrict__ dec,
                                                  const double* __restrict__ Rprev,
                                                  double qr_tol, double* __restrict__ Pt,
                                                  double* __restrict__ Rout,
                                                  unsigned char* __restrict__ dead) {
  const int J = blockIdx.x;
  if (J >= n_agg) return;
  const int lane = threadIdx.x;
  const int a0 = off[J], k = off[J + 1] - a0;
  const int rows = BR * k;
  __shared__ double cen[3];
  if (level0 && NC == 6) {
    if (lane == 0) {
      double cx = 0.0, cy = 0.0, cz = 0.0;
      for (int i = 0; i < k; ++i) {
        const int v = members[a0 + i];
        cx = cx + coords[3 * int64_t(v)];
        cy = cy + coords[3 * int64_t(v) + 1];
        cz = cz + coords[3 * int64_t(v) + 2];
      }
      cen[0] = cx / k;
      cen[1] = cy / k;
      cen[2] = cz / k;
    }
    __syncthreads();
  }
  // build
  for (int idx = lane; idx < rows; idx += 64) {
    const int v = members[a0 + idx / BR], p = idx % BR;
    double* row = Pt + (int64_t(v) * BR + p) * NC;
    if (level0) {
      double b[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) b[j] = 0.0;
      b[p] = 1.0;
      if constexpr (NC == 6) {
        const double x = coords[3 * int64_t(v)] - cen[0];
        const double y = coords[3 * int64_t(v) + 1] - cen[1];
        const double z = coords[3 * int64_t(v) + 2] - cen[2];
        if (p == 0) { b[4] = z; b[5] = -y; }
        if (p == 1) { b[3] = -z; b[5] = x; }
        if (p == 2) { b[3] = y; b[4] = -x; }
      }
      const bool off_row = dec && dec[int64_t(v) * BR + p];
#pragma unroll
      for (int j = 0; j < NC; ++j) row[j] = off_row ? 0.0 : b[j];
    } else {
      const double* src = Rprev + (int64_t(v) * NC + p) * NC;
#pragma unroll
      for (int j = 0; j < NC; ++j) row[j] = src[j];
    }
  }
  double R[NC][NC];
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) R[i][j] = 0.0;
  bool isdead[NC];
  for (int j = 0; j < NC; ++j) {
    double s = 0.0;
    for (int idx = lane; idx < rows; idx += 64) {
      const int v = members[a0 + idx / BR], p = idx % BR;
      const double x = Pt[(int64_t(v) * BR + p) * NC + j];
      s += x * x;
    }
    const double nb = sqrt(wave_sum(s));
    for (int pass = 0; pass < 2; ++pass) {
      double cc[NC];
      for (int i = 0; i < j; ++i) {
        double d = 0.0;
        for (int idx = lane; idx < rows; idx += 64) {
          const int v = members[a0 + idx / BR], p = idx % BR;
          const double* row = Pt + (int64_t(v) * BR + p) * NC;
          d += row[i] * row[j];
        }
        cc[i] = wave_sum(d);
      }
      for (int idx = lane; idx < rows; idx += 64) {
        const int v = members[a0 + idx / BR], p = idx % BR;
        double* row = Pt + (int64_t(v) * BR + p) * NC;
        double x = row[j];
        for (int i = 0; i < j; ++i) x -= cc[i] * row[i];
        row[j] = x;
      }
      for (int i = 0; i < j; ++i) R[i][j] += cc[i];
    }
    double s2 = 0.0;
    for (int idx = lane; idx < rows; idx += 64) {
      const int v = members[a0 + idx / BR], p = idx % BR;
      const double x = Pt[(int64_t(v) * BR + p) * NC + j];
      s2 += x * x;
    }
    const double nv = sqrt(wave_sum(s2));
    isdead[j] = (nb == 0.0) || (nv <= qr_tol * nb);
    const double scale = isdead[j] ? 0.0 : 1.0 / nv;
    R[j][j] = isdead[j] ? 0.0 : nv;
    for (int idx = lane; idx < rows; idx += 64) {
      const int v = members[a0 + idx / BR], p = idx % BR;
      double* row = Pt + (int64_t(v) * BR + p) * NC;
      row[j] = isdead[j] ? 0.0 : row[j] * scale;
    }
  }
  if (lane == 0) {
    for (int i = 0; i < NC; ++i) {
      dead[int64_t(J) * NC + i] = isdead[i];
      for (int j = 0; j < NC; ++j)
        Rout[int64_t(J) * NC * NC + i * NC + j] = isdead[i] ? 0.0 : R[i][j];
    }
  }
}

// The same QR with the aggregate's rows held in registers (lane l owns rows l, l + 64, ...,
// at most TENT_R of them): one pass builds them, the Gram-Schmidt sweeps run on registers
// and wavefront sums, one pass writes the orthonormal rows.  Every sum runs in the order of
// the kernel above (a lane's rows ascending, then over the wavefront), so the results are
// the same.  Aggregates with more than 64 TENT_R rows take the kernel above.
constexpr int TENT_R = 8;
template <int BR, int NC>
__global__ void __launch_bounds__(64) k_tentative(int n_agg, const int* __restrict__ off,
                                                  const int* __restrict__ members,
                                                  int level0,
                                                  const double* __restrict__ coords,
                                                  const unsigned char* __restrict__ dec,
                                                  const double* __restrict__ Rprev,
                                                  double qr_tol, double* __restrict__ Pt,
                                                  double* __restrict__ Rout,
                                                  unsigned char* __restrict__ dead) {
  const int J = blockIdx.x;
  if (J >= n_agg) return;
  const int lane = threadIdx.x;
  const int a0 = off[J], k = off[J + 1] - a0;
  const int rows = BR * k;
  __shared__ double cen[3];
  if (level0 && NC == 6) {
    if (lane == 0) {
      double cx = 0.0, cy = 0.0, cz = 0.0;
      for (int i = 0; i < k; ++i) {
        const int v = members[a0 + i];
        cx = cx + coords[3 * int64_t(v)];
        cy = cy + coords[3 * int64_t(v) + 1];
        cz = cz + coords[3 * int64_t(v) + 2];
      }
      cen[0] = cx / k;
      cen[1] = cy / k;
      cen[2] = cz / k;
    }
    __syncthreads();
  }
  double Q[TENT_R][NC];
  int64_t rowoff[TENT_R];
#pragma unroll
  for (int s = 0; s < TENT_R; ++s) {
    const int idx = lane + 64 * s;
    rowoff[s] = -1;
#pragma unroll
    for (int j = 0; j < NC; ++j) Q[s][j] = 0.0;
    if (idx >= rows) continue;
    const int v = members[a0 + idx / BR], p = idx % BR;
    rowoff[s] = (int64_t(v) * BR + p) * NC;
    if (level0) {
      double b[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) b[j] = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (p == j) b[j] = 1.0;
      if constexpr (NC == 6) {
        const double x = coords[3 * int64_t(v)] - cen[0];
        const double y = coords[3 * int64_t(v) + 1] - cen[1];
        const double z = coords[3 * int64_t(v) + 2] - cen[2];
        if (p == 0) { b[4] = z; b[5] = -y; }
        if (p == 1) { b[3] = -z; b[5] = x; }
        if (p == 2) { b[3] = y; b[4] = -x; }
      }
      const bool off_row = dec && dec[int64_t(v) * BR + p];
#pragma unroll
      for (int j = 0; j < NC; ++j) Q[s][j] = off_row ? 0.0 : b[j];
    } else {
      const double* src = Rprev + (int64_t(v) * NC + p) * NC;
#pragma unroll
      for (int j = 0; j < NC; ++j) Q[s][j] = src[j];
    }
  }
  double R[NC][NC];
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) R[i][j] = 0.0;
  bool isdead[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    double sq = 0.0;
#pragma unroll
    for (int s = 0; s < TENT_R; ++s) sq += Q[s][j] * Q[s][j];
    const double nb = sqrt(wave_sum(sq));
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      double cc[NC];
#pragma unroll
      for (int i = 0; i < j; ++i) {
        double d = 0.0;
#pragma unroll
        for (int s = 0; s < TENT_R; ++s) d += Q[s][i] * Q[s][j];
        cc[i] = wave_sum(d);
      }
#pragma unroll
      for (int s = 0; s < TENT_R; ++s) {
        double x = Q[s][j];
#pragma unroll
        for (int i = 0; i < j; ++i) x -= cc[i] * Q[s][i];
        Q[s][j] = x;
      }
#pragma unroll
      for (int i = 0; i < j; ++i) R[i][j] += cc[i];
    }
    double s2 = 0.0;
#pragma unroll
    for (int s = 0; s < TENT_R; ++s) s2 += Q[s][j] * Q[s][j];
    const double nv = sqrt(wave_sum(s2));
    isdead[j] = (nb == 0.0) || (nv <= qr_tol * nb);
    const double scale = isdead[j] ? 0.0 : 1.0 / nv;
    R[j][j] = isdead[j] ? 0.0 : nv;
#pragma unroll
    for (int s = 0; s < TENT_R; ++s) Q[s][j] = isdead[j] ? 0.0 : Q[s][j] * scale;
  }
#pragma unroll
  for (int s = 0; s < TENT_R; ++s)
    if (rowoff[s] >= 0)
#pragma unroll
      for (int j = 0; j < NC; ++j) Pt[rowoff[s] + j] = Q[s][j];
  if (lane == 0) {
    for (int i = 0; i < NC; ++i) {
      dead[int64_t(J) * NC + i] = isdead[i];
      for (int j = 0; j < NC; ++j)
        Rout[int64_t(J) * NC * NC + i * NC + j] = isdead[i] ? 0.0 : R[i][j];
    }
  }
}

void tentative_prolongator(Ctx& c, int br, int nc, int n_nodes, int n_agg, const int* moff,
                           const int* members, bool level0, const double* coords,
                           const unsigned char* dec, const double* Rprev, double qr_tol,
                           DBuf<double>& Pt, DBuf<double>& R, DBuf<unsigned char>& dead) {
  AMGF_REQUIRE(nc == 3 || nc == 6, AMGF_EINVAL, "near-null space must have 3 or 6 vectors");
  AMGF_REQUIRE(level0 ? br == 3 : br == nc, AMGF_EINVAL, "tentative prolongator block size");
  AMGF_REQUIRE(!level0 || nc == 3 || coords, AMGF_EINVAL, "rigid-body modes need coords");
  Pt.alloc(size_t(n_nodes) * br * nc);
  AMGF_HIP(hipMemsetAsync(Pt.p, 0, Pt.bytes(), c.s));
  R.alloc(size_t(n_agg) * nc * nc);
  dead.alloc(size_t(n_agg) * nc);
  const int l0 = level0 ? 1 : 0;
  const bool regs = int64_t(br) * max_segment_length(c, moff, n_agg) <= 64 * TENT_R;
#define AMGF_TENT(BR, NC)                                                                    \
  do {                                                                                       \
    if (regs)                                                                                \
      hipLaunchKernelGGL((k_tentative<BR, NC>), dim3(n_agg), dim3(64), 0, c.s, n_agg, moff,  \
                         members, l0, coords, dec, Rprev, qr_tol, Pt.p, R.p, dead.p);        \
    else                                                                                     \
      hipLaunchKernelGGL((k_tentative_mem<BR, NC>), dim3(n_agg), dim3(64), 0, c.s, n_agg,    \
                         moff, members, l0, coords, dec, Rprev, qr_tol, Pt.p, R.p, dead.p);  \
  } while (0)
  if (nc == 6) {
    if (br == 3) AMGF_TENT(3, 6);
    else AMGF_TENT(6, 6);
  } else {
    AMGF_TENT(3, 3);
  }
#undef AMGF_TENT
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// prolongator smoothing  P = P_t - omega D_l1^{-1} A P_t
// ======================================================================================
// Ordered sums of products staged in LDS (prolongator smoothing and the products of
// Galerkin operators).  A wavefront owns one output row and up to 64 of its output blocks
// (a lane each, columns `mycol` ascending over the lanes).  Its lanes form up to 64
// products in LDS, each with the output column `key` it adds to; slot_of finds the lane
// owning that column by a binary search over the lanes (shuffles), and add_staged gives
// every owner the products of its column in ascending staging order (one ballot per
// owner).  Products staged in the order of a walk along the row give the walk's sums.
__device__ __forceinline__ int slot_of(int key, int mycol, int nslot) {
  int pos = 0;
#pragma unroll
  for (int st = 32; st > 0; st >>= 1) {
    const int v = __shfl(mycol, min(pos + st - 1, 63), 64);
    if (pos + st <= nslot && v < key) pos += st;
  }
  const int hit = __shfl(mycol, min(pos, 63), 64);
  return (key >= 0 && pos < nslot && hit == key) ? pos : -1;
}

template <int E, int LD>
__device__ __forceinline__ void add_staged(int slot, int nslot, const double (*prod)[LD],
                                           double* acc) {
  const int lane = threadIdx.x & 63;
  unsigned long long mine = 0;
  for (int s = 0; s < nslot; ++s) {
    const unsigned long long m = __ballot(slot == s);
    if (lane == s) mine = m;
  }
  while (mine) {
    const int u = __ffsll(mine) - 1;
    mine &= mine - 1;
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] += prod[u][e];
  }
}

// P = P_t - omega D_l1^{-1} A P_t, one wavefront per aggregated row i: the row's blocks of
// A go through in chunks of 64, a lane per block (i, v) forming A_iv P_t,v (key agg(v)),
// summed per block (i, J) of P in ascending block order; then the lane of (i, J) scales by
// -omega/d and adds P_t,i on the block of i's own aggregate.
template <int B, int NC>
__global__ void __launch_bounds__(256) k_sa_numeric(int n, const int* __restrict__ arp,
                                                    const int* __restrict__ acol,
                                                    const double* __restrict__ aval,
                                                    const int* __restrict__ agg,
                                                    const double* __restrict__ Pt,
                                                    const double* __restrict__ d, double omega,
                                                    const int* __restrict__ prp,
                                                    const int* __restrict__ pcol,
                                                    double* __restrict__ pval) {
  constexpr int E = B * NC;
  __shared__ double prod[4][64][E + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);
  if (i >= n) return;
  const int ai = agg[i];
  if (ai < 0) return;
  const int t0 = arp[i], t1 = arp[i + 1];
  for (int sb = prp[i]; sb < prp[i + 1]; sb += 64) {
    const int nslot = min(64, prp[i + 1] - sb);
    const bool act = lane < nslot;
    const int J = act ? pcol[sb + lane] : INT_MAX;
    double acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.0;
    for (int c0 = t0; c0 < t1; c0 += 64) {
      const int t = c0 + lane;
      int kj = -1;
      if (t < t1) {
        const int v = acol[t];
        kj = agg[v];
        if (kj >= 0) {
          const double* A = aval + int64_t(t) * B * B;
          const double* Q = Pt + int64_t(v) * E;
#pragma unroll
          for (int p = 0; p < B; ++p)
#pragma unroll
            for (int q = 0; q < NC; ++q) {
              double a = 0.0;
#pragma unroll
              for (int r = 0; r < B; ++r) a += A[p * B + r] * Q[r * NC + q];
              prod[wv][lane][p * NC + q] = a;
            }
        }
      }
      const int slot = slot_of(kj, J, nslot);
      wave_lds_sync();
      add_staged<E>(slot, nslot, prod[wv], acc);
      wave_lds_sync();
    }
    if (act) {
      double* out = pval + int64_t(sb + lane) * E;
#pragma unroll
      for (int p = 0; p < B; ++p) {
        const double sc = omega / d[int64_t(i) * B + p];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          const double v = -(acc[p * NC + q] * sc);
          out[p * NC + q] = J == ai ? Pt[int64_t(i) * E + p * NC + q] + v : v;
        }
      }
    }
  }
}

// The same for short rows (level 0: about 27 blocks of A and 5 of P per row): two rows per
// wavefront, a half-wavefront (32 lanes) each, so each staged chunk serves two rows.  A
// half's blocks of A go through in chunks of 32 in ascending order, as the full-wavefront
// form takes them in chunks of 64, so each block of P gets the same sums in the same order.
// Both halves run the loops to the larger trip count (the other half idles) so that every
// lane reaches the shuffles and ballots.
template <int B, int NC>
__global__ void __launch_bounds__(256) k_sa_numeric_half(int n, const int* __restrict__ arp,
                                                         const int* __restrict__ acol,
                                                         const double* __restrict__ aval,
                                                         const int* __restrict__ agg,
                                                         const double* __restrict__ Pt,
                                                         const double* __restrict__ d,
                                                         double omega,
                                                         const int* __restrict__ prp,
                                                         const int* __restrict__ pcol,
                                                         double* __restrict__ pval) {
  constexpr int E = B * NC;
  __shared__ double prod[4][64][E + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int half = lane >> 5, hl = lane & 31;
  const int i = (blockIdx.x * 4 + wv) * 2 + half;
  const bool row_on = i < n && agg[i] >= 0;
  const int ai = row_on ? agg[i] : -1;
  const int t0 = row_on ? arp[i] : 0, t1 = row_on ? arp[i + 1] : 0;
  const int p0 = row_on ? prp[i] : 0, p1 = row_on ? prp[i + 1] : 0;
  // trip counts of the slot and block chunks, the larger of the two halves
  const int ns_mine = (p1 - p0 + 31) / 32, nc_mine = (t1 - t0 + 31) / 32;
  const int ns_it = max(__shfl(ns_mine, 0, 64), __shfl(ns_mine, 32, 64));
  const int nc_it = max(__shfl(nc_mine, 0, 64), __shfl(nc_mine, 32, 64));
  const unsigned long long half_mask = half ? 0xFFFFFFFF00000000ull : 0x00000000FFFFFFFFull;
  for (int si = 0; si < ns_it; ++si) {
    const int sb = p0 + si * 32;
    const int nslot = max(0, min(32, p1 - sb));
    const bool act = hl < nslot;
    const int J = act ? pcol[sb + hl] : INT_MAX;
    double acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.0;
    for (int ci = 0; ci < nc_it; ++ci) {
      const int t = t0 + ci * 32 + hl;
      int kj = -1;
      if (t < t1) {
        const int v = acol[t];
        kj = agg[v];
        if (kj >= 0) {
          const double* A = aval + int64_t(t) * B * B;
          const double* Q = Pt + int64_t(v) * E;
#pragma unroll
          for (int p = 0; p < B; ++p)
#pragma unroll
            for (int q = 0; q < NC; ++q) {
              double a = 0.0;
#pragma unroll
              for (int r = 0; r < B; ++r) a += A[p * B + r] * Q[r * NC + q];
              prod[wv][lane][p * NC + q] = a;
            }
        }
      }
      // the lane of this half owning column kj (binary search over the half's columns)
      int pos = 0;
#pragma unroll
      for (int st = 16; st > 0; st >>= 1) {
        const int v = __shfl(J, min(pos + st - 1, 31), 32);
        if (pos + st <= nslot && v < kj) pos += st;
      }
      const int hit = __shfl(J, min(pos, 31), 32);
      const int slot = (kj >= 0 && pos < nslot && hit == kj) ? pos : -1;
      wave_lds_sync();
      // one ballot per slot, to the larger slot count of the two halves (uniform)
      const int nslot_max = max(__shfl(nslot, 0, 64), __shfl(nslot, 32, 64));
      unsigned long long mine = 0;
      for (int s2 = 0; s2 < nslot_max; ++s2) {
        const unsigned long long m = __ballot(slot == s2);
        if (hl == s2) mine = m & half_mask;
      }
      while (mine) {
        const int u = __ffsll(mine) - 1;
        mine &= mine - 1;
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] += prod[wv][u][e];
      }
      wave_lds_sync();
    }
    if (act) {
      double* out = pval + int64_t(sb + hl) * E;
#pragma unroll
      for (int p = 0; p < B; ++p) {
        const double sc = omega / d[int64_t(i) * B + p];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          const double v = -(acc[p * NC + q] * sc);
          out[p * NC + q] = J == ai ? Pt[int64_t(i) * E + p * NC + q] + v : v;
        }
      }
    }
  }
}

void smooth_prolongator(Ctx& c, const BSR& A, const int* agg, int n_agg, int nc,
                        const double* Pt, const double* d, double omega, BSR& P) {
  const int n = A.nrows;
  DBuf<int> mask(std::max(n, 1));
  hipLaunchKernelGGL(k_nonneg_mask, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, agg, mask.p);
  union_symbolic(c, n, n_agg, A.rowptr.p, A.col.p, nullptr, nullptr, agg, false, mask.p, P);
  P.br = A.br;
  P.bc = nc;
  P.val.alloc(std::max<int64_t>(P.nnzb, 1) * P.bsz());
  const dim3 g(grid_for(n, 4));
  AMGF_REQUIRE((A.br == 3 && (nc == 3 || nc == 6)) || (A.br == 6 && nc == 6), AMGF_EINVAL,
               "prolongator block size");
  if (A.br == 3 && nc == 6)
    hipLaunchKernelGGL((k_sa_numeric_half<3, 6>), dim3(grid_for(n, 8)), dim3(256), 0, c.s, n,
                       A.rowptr.p, A.col.p, A.val.p, agg, Pt, d, omega, P.rowptr.p, P.col.p,
                       P.val.p);
  else if (A.br == 3)
    hipLaunchKernelGGL((k_sa_numeric<3, 3>), g, dim3(256), 0, c.s, n, A.rowptr.p, A.col.p,
                       A.val.p, agg, Pt, d, omega, P.rowptr.p, P.col.p, P.val.p);
  else
    hipLaunchKernelGGL((k_sa_numeric<6, 6>), g, dim3(256), 0, c.s, n, A.rowptr.p, A.col.p,
                       A.val.p, agg, Pt, d, omega, P.rowptr.p, P.col.p, P.val.p);
  AMGF_LAUNCH_CHECK();
}

__global__ void k_nonneg_mask(int n, const int* __restrict__ a, int* __restrict__ m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) m[i] = a[i] >= 0;
}

// ======================================================================================
// generic BSR product C = A B, output-stationary
// ======================================================================================
// A group of G lanes per row r (G = 64: one wavefront; G = 16: four short rows per
// wavefront), one lane per output block (r, j): the lane walks A's row in ascending order,
// so each output block accumulates in a fixed order (deterministic) and rows with many
// blocks spread over the group.  A's row goes through G blocks at a time: lane u loads block
// u's column k and the extent of B's row k, which the walk then takes from lane u by a
// shuffle, so the only loads left in the walk are B's column ids and the values.  For each A
// block (r, k) the group loads the column ids of B's row k (coalesced, up to G at a time) and
// every lane finds its column j there by a binary search over the group's lanes (shuffles),
// the ids of the next A block already on their way.
template <int RA, int KA, int CB, int G>
__global__ void __launch_bounds__(256) k_spgemm_numeric(
    int nrows, const int* __restrict__ arp, const int* __restrict__ acol,
    const double* __restrict__ aval, const int* __restrict__ brp, const int* __restrict__ bcol,
    const double* __restrict__ bval, const int* __restrict__ crp, const int* __restrict__ ccol,
    double* __restrict__ cval) {
  // a full wavefront per row keeps the row index (and the loops over A's row) scalar
  const int r = G == 64 ? __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6))
                        : int((blockIdx.x * 256 + threadIdx.x) / G);
  const int lane = threadIdx.x % G;
  if (r >= nrows) return;
  const int t0 = arp[r], t1 = arp[r + 1];
  const int s1 = crp[r + 1];
  // blockIdx.y spreads the output chunks of a row over gridDim.y wavefronts
  for (int sb = crp[r] + int(blockIdx.y) * G; sb < s1; sb += G * int(gridDim.y)) {
    const int s = sb + lane;
    const bool act = s < s1;
    const int j = act ? ccol[s] : INT_MAX;
    double acc[RA * CB];
#pragma unroll
    for (int e = 0; e < RA * CB; ++e) acc[e] = 0.0;
    for (int tc = t0; tc < t1; tc += G) {
      const int nt = min(G, t1 - tc);
      int mb0 = 0, mblen = 0;
      if (lane < nt) {
        const int k = acol[tc + lane];
        mb0 = brp[k];
        mblen = brp[k + 1] - mb0;
      }
      // B's column ids of the walk's current A block (the first G of them)
      int b0 = __shfl(mb0, 0, G), blen = __shfl(mblen, 0, G);
      int myc = lane < min(G, blen) ? bcol[b0 + lane] : INT_MAX;
      for (int u = 0; u < nt; ++u) {
        const int cb0 = b0, cblen = blen, cmyc = myc;
        if (u + 1 < nt) {                             // next A block's ids, ahead of use
          b0 = __shfl(mb0, u + 1, G);
          blen = __shfl(mblen, u + 1, G);
          myc = lane < min(G, blen) ? bcol[b0 + lane] : INT_MAX;
        }
        const int t = tc + u;
        for (int c0 = 0; c0 < cblen; c0 += G) {
          const int nb = min(G, cblen - c0);
          const int mc = c0 == 0 ? cmyc : (lane < nb ? bcol[cb0 + c0 + lane] : INT_MAX);
          // pos = number of chunk columns below j (chunk columns ascending)
          int pos = 0;
          for (int st = 1 << (31 - __clz(nb)); st > 0; st >>= 1) {
            const int v = __shfl(mc, min(pos + st - 1, G - 1), G);
            if (pos + st <= nb && v < j) pos += st;
          }
          const int hit = __shfl(mc, min(pos, G - 1), G);
          if (!act || pos >= nb || hit != j) continue;
          const double* a = aval + int64_t(t) * RA * KA;
          const double* b = bval + int64_t(cb0 + c0 + pos) * KA * CB;
#pragma unroll
          for (int p = 0; p < RA; ++p)
#pragma unroll
            for (int x = 0; x < KA; ++x) {
              const double av = a[p * KA + x];
#pragma unroll
              for (int q = 0; q < CB; ++q) acc[p * CB + q] += av * b[x * CB + q];
            }
        }
      }
    }
    if (act) {
      double* out = cval + int64_t(s) * RA * CB;
#pragma unroll
      for (int e = 0; e < RA * CB; ++e) out[e] = acc[e];
    }
  }
}

void spgemm(Ctx& c, const BSR& A, const BSR& B, BSR& C) {
  AMGF_REQUIRE(A.bc == B.br && A.ncols == B.nrows, AMGF_EINVAL, "spgemm shape");
  union_symbolic(c, A.nrows, B.ncols, A.rowptr.p, A.col.p, B.rowptr.p, B.col.p, nullptr,
                 false, nullptr, C);
  C.br = A.br;
  C.bc = B.bc;
  C.val.alloc(std::max<int64_t>(C.nnzb, 1) * C.bsz());
  // short output rows (at most 16 blocks on average): four rows per wavefront; long rows
  // of a small matrix (coarse Galerkin products): their 64-column chunks on up to 16
  // wavefronts each, so that a few hundred rows still fill the chip
  const bool short_rows = A.nrows > 0 && C.nnzb <= int64_t(16) * A.nrows;
  const int ny = A.nrows > 0 ? std::min(16, std::max(1, 32768 / A.nrows)) : 1;
  const dim3 g64(grid_for(A.nrows, 4), ny), g16(grid_for(A.nrows, 16)), b(256);
#define AMGF_SPGEMM_CASE(ra, ka, cb)                                                         \
  if (A.br == ra && A.bc == ka && B.bc == cb) {                                              \
    if (A.nrows && short_rows)                                                               \
      hipLaunchKernelGGL((k_spgemm_numeric<ra, ka, cb, 16>), g16, b, 0, c.s, A.nrows,        \
                         A.rowptr.p, A.col.p, A.val.p, B.rowptr.p, B.col.p, B.val.p,         \
                         C.rowptr.p, C.col.p, C.val.p);                                      \
    else if (A.nrows)                                                                        \
      hipLaunchKernelGGL((k_spgemm_numeric<ra, ka, cb, 64>), g64, b, 0, c.s, A.nrows,        \
                         A.rowptr.p, A.col.p, A.val.p, B.rowptr.p, B.col.p, B.val.p,         \
                         C.rowptr.p, C.col.p, C.val.p);                                      \
    AMGF_LAUNCH_CHECK();                                                                     \
    return;                                                                                  \
  }
  AMGF_SPGEMM_CASE(3, 3, 6)
  AMGF_SPGEMM_CASE(6, 6, 6)
  AMGF_SPGEMM_CASE(6, 3, 6)
  AMGF_SPGEMM_CASE(1, 3, 6)
  AMGF_SPGEMM_CASE(1, 6, 6)
  AMGF_SPGEMM_CASE(3, 3, 3)
  AMGF_SPGEMM_CASE(1, 3, 3)
#undef AMGF_SPGEMM_CASE
  throw Error(AMGF_EINVAL, "spgemm: unsupported block sizes");
}

// coarse DOFs whose prolongator column is dead get a unit diagonal
__global__ void k_dead_identity(int n_agg, int nc, const unsigned char* __restrict__ dead,
                                const int* __restrict__ dpos, double* __restrict__ val) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= n_agg || dpos[J] < 0) return;
  for (int j = 0; j < nc; ++j)
    if (dead[int64_t(J) * nc + j]) val[int64_t(dpos[J]) * nc * nc + j * nc + j] = 1.0;
}

// K_aa(q, q) = K0_aq + E_aq on the diagonal blocks (one add; E == nullptr: K0 itself).
// save: first record K0 from K.
__global__ void k_bound_diag(int nn, const int* __restrict__ rp, const int* __restrict__ col,
                             double* __restrict__ val, const double* __restrict__ E,
                             double* __restrict__ k0, int save, int* __restrict__ flag) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nn) return;
  int pos = -1;
  for (int e = rp[a]; e < rp[a + 1]; ++e)
    if (col[e] == a) pos = e;
  if (pos < 0) {
    atomicOr(flag, 1);
    return;
  }
  for (int q = 0; q < 3; ++q) {
    const int64_t k = int64_t(pos) * 9 + 4 * q;
    if (save) k0[int64_t(a) * 3 + q] = val[k];
    const double base = k0[int64_t(a) * 3 + q];
    val[k] = E ? base + E[int64_t(a) * 3 + q] : base;
  }
}

void bound_diagonal(Ctx& c, BSR& K, const double* E, DBuf<double>& k0) {
  AMGF_REQUIRE(K.br == 3 && K.bc == 3, AMGF_EINVAL, "bound terms need 3x3 blocks");
  const bool save = k0.n == 0;
  if (save) k0.alloc(size_t(K.nrows) * 3);
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  hipLaunchKernelGGL(k_bound_diag, dim3(grid_for(K.nrows, 256)), dim3(256), 0, c.s, K.nrows,
                     K.rowptr.p, K.col.p, K.val.p, E, k0.p, int(save), c.flag.p);
  AMGF_LAUNCH_CHECK();
  AMGF_REQUIRE(d2h_scalar(c.flag.p, c.s) == 0, AMGF_EINVAL,
               "bound terms need a stored diagonal block in every row of K");
}

void dead_identity(Ctx& c, BSR& Kc, const unsigned char* dead) {
  DBuf<int> dpos(std::max(Kc.nrows, 1));
  hipLaunchKernelGGL(k_diag_pos, dim3(grid_for(Kc.nrows, 256)), dim3(256), 0, c.s, Kc.nrows,
                     Kc.rowptr.p, Kc.col.p, dpos.p);
  AMGF_REQUIRE(Kc.br == Kc.bc, AMGF_EINVAL, "dead identity needs square blocks");
  hipLaunchKernelGGL(k_dead_identity, dim3(grid_for(Kc.nrows, 256)), dim3(256), 0, c.s,
                     Kc.nrows, Kc.br, dead, dpos.p, Kc.val.p);
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// l1 row norms
// ======================================================================================
template <int B>
__global__ void k_l1(int n, const int* __restrict__ rp, const double* __restrict__ val,
                     double* __restrict__ d) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double s[B];
#pragma unroll
  for (int p = 0; p < B; ++p) s[p] = 0.0;
  for (int k = rp[a]; k < rp[a + 1]; ++k) {
    const double* v = val + int64_t(k) * B * B;
#pragma unroll
    for (int p = 0; p < B; ++p)
#pragma unroll
      for (int q = 0; q < B; ++q) s[p] += fabs(v[p * B + q]);
  }
#pragma unroll
  for (int p = 0; p < B; ++p) d[int64_t(a) * B + p] = s[p];
}

void l1_norms(Ctx& c, const BSR& A, DBuf<double>& d) {
  d.alloc(size_t(A.nrows) * A.br);
  if (A.br == 3)
    hipLaunchKernelGGL(k_l1<3>, dim3(grid_for(A.nrows, 256)), dim3(256), 0, c.s, A.nrows,
                       A.rowptr.p, A.val.p, d.p);
  else
    hipLaunchKernelGGL(k_l1<6>, dim3(grid_for(A.nrows, 256)), dim3(256), 0, c.s, A.nrows,
                       A.rowptr.p, A.val.p, d.p);
  AMGF_LAUNCH_CHECK();
}

// ======================================================================================
// filtering space: every DOF of every node touched by J
// ======================================================================================
__global__ void k_mark_nodes(int64_t nnzb, const int* __restrict__ col, int* __restrict__ mark) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < nnzb) mark[col[k]] = 1;
}
__global__ void k_node_dofs(int nn, const int* __restrict__ mark, const int* __restrict__ pos,
                            int* __restrict__ ic) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn || !mark[v]) return;
  const int o = 3 * pos[v];
  ic[o] = 3 * v;
  ic[o + 1] = 3 * v + 1;
  ic[o + 2] = 3 * v + 2;
}

int filter_space_from_J(Ctx& c, const BSR& J, int n_nodes, DBuf<int>& Ic) {
  DBuf<int> mark(std::max(n_nodes, 1)), pos(size_t(n_nodes) + 1);
  AMGF_HIP(hipMemsetAsync(mark.p, 0, mark.bytes(), c.s));
  if (J.nnzb)
    hipLaunchKernelGGL(k_mark_nodes, dim3(grid_for(J.nnzb, 256)), dim3(256), 0, c.s, J.nnzb,
                       J.col.p, mark.p);
  const int nodes = scan_exclusive(c, mark.p, pos.p, n_nodes);
  Ic.alloc(std::max(3 * nodes, 1));
  if (nodes)
    hipLaunchKernelGGL(k_node_dofs, dim3(grid_for(n_nodes, 256)), dim3(256), 0, c.s, n_nodes,
                       mark.p, pos.p, Ic.p);
  AMGF_LAUNCH_CHECK();
  return 3 * nodes;
}

}  // namespace amgf

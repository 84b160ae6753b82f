// Nested-dissection multifrontal FP64 Cholesky (the paper solves the filtering system with
// a multifrontal direct solver, whose cost on the two-dimensional contact subspace grows as
// n_c^{3/2} with n_c log n_c memory, Sec. 6).
//
// Ordering.  The node graph is split recursively by breadth-first level sets: from a
// pseudo-peripheral node (the farthest node of a first search), the level that best
// balances the node counts on its two sides separates the lower levels from the higher
// ones and from nodes the search did not reach (the middle level by index would leave a
// corner-started triangle split 1:3 and the tree half again as deep).  All parts of one
// depth are split together, one workgroup per part.  Parts of at most MF_LEAF nodes, and
// parts whose search spans fewer than three levels, become leaves.
// Symbolic.  The boundary of supernode t (the ancestor nodes its front couples to) is the
// set of ancestor nodes adjacent to its separator or lying in a child's boundary.
// Numeric.  Fronts of one depth are factored together in 64x64 tiles: Cholesky and
// inverse of the diagonal tile, the tile column as an MFMA product with that inverse, and
// the MFMA trailing update.  The trailing block (the update matrix) is then added into the
// parent's front.
// Each front then keeps X = L11^{-1} and G = L21 X, so the solve is matrix-vector
// products only: forward by depth (deepest first) y = X f_s, u = f_b - G f_s, the update
// vector u going to the parent; backward by depth (root first) x_s = X^T y - G^T x_b.
// The solve works in tree order (the members of each supernode together), so a front's
// right-hand side and solution are contiguous; each child writes its update vector into a
// slot array of its parent at the parent's front positions.  Every sum has a fixed order,
// so results are reproducible.
#include "multifrontal.h"

#include <algorithm>
#include <climits>

namespace amgf {

constexpr int MF_LEAF = 64;
constexpr int MF_MAXD = 64;
constexpr int MF_SMAX = 8192;   // largest padded separator of one front
constexpr int MF_MAXNODES = 1 << 18;   // node bitmap of the boundary search fits in LDS
constexpr int MF_HIST = 4096;   // level histogram of a split (more levels: middle level)

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lower_bound_dev(const int* a, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- node graph
__global__ void k_mf_node_graph(int nn, int bs, const int* __restrict__ rp,
                                const int* __restrict__ col, const int* __restrict__ grp,
                                int* __restrict__ cnt, int* __restrict__ gcol) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  const int r = v * bs;
  int prev = -1, k = 0;
  const int o = grp ? grp[v] : 0;
  for (int e = rp[r]; e < rp[r + 1]; ++e) {
    const int u = col[e] / bs;
    if (u != prev && u != v) {
      if (gcol) gcol[o + k] = u;
      ++k;
    }
    prev = u;
  }
  if (cnt) cnt[v] = k;
}

// ---------------------------------------------------------------- ordering
// Threads of a splitting workgroup, and lanes that share one frontier node's neighbour list
// in its breadth-first search (the search steps level by level; a lane per frontier node
// walked ~20 neighbours one dependent load after another at every level).
constexpr int MF_SPLIT_THREADS = 1024;
constexpr int MF_BFS_LANES = 8;

// Breadth-first search restricted to part p from `start`.  Frontier queues qa/qb hold at
// most np nodes each.  On return sh[0] = last level, sh[2] = nodes reached.  The levels
// do not depend on the order in which the frontier is filled.
__device__ void mf_bfs(int p, int start, const int* nodes, int np, const int* grp,
                       const int* gcol, const int* part, int* lvl, int* qa, int* qb,
                       int* sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < np; i += nt) lvl[nodes[i]] = -1;
  __syncthreads();
  if (tid == 0) {
    lvl[start] = 0;
    qa[0] = start;
    sh[0] = 1;
    sh[1] = 0;
    sh[2] = 1;
  }
  __syncthreads();
  int cur = 0;
  int* q = qa;
  int* qn = qb;
  const int sub = tid % MF_BFS_LANES, gi = tid / MF_BFS_LANES, ng = nt / MF_BFS_LANES;
  while (true) {
    const int fsz = sh[0];
    for (int i = gi; i < fsz; i += ng) {
      const int v = q[i];
      const int e1 = grp[v + 1];
      for (int e = grp[v] + sub; e < e1; e += MF_BFS_LANES) {
        const int u = gcol[e];
        if (part[u] != p) continue;
        if (atomicCAS(&lvl[u], -1, cur + 1) == -1) qn[atomicAdd(&sh[1], 1)] = u;
      }
    }
    __syncthreads();
    const int nsz = sh[1];
    __syncthreads();
    if (nsz == 0) break;
    if (tid == 0) {
      sh[0] = nsz;
      sh[1] = 0;
      sh[2] += nsz;
    }
    int* t = q;
    q = qn;
    qn = t;
    ++cur;
    __syncthreads();
  }
  if (tid == 0) sh[0] = cur;
  __syncthreads();
}

// One workgroup per part of depth d: leaf, or split into children 2p (lower levels) and
// 2p+1 (higher levels and unreached nodes) with the middle level as separator.
// npart[v] = child slot, or -1 when v joins supernode tb + p (snode[v]).
__global__ void __launch_bounds__(MF_SPLIT_THREADS) k_mf_split(int tb, int force_leaf,
                                                  const int* __restrict__ poff,
                                                  const int* __restrict__ pperm,
                                                  const int* __restrict__ grp,
                                                  const int* __restrict__ gcol,
                                                  const int* __restrict__ part, int* npart,
                                                  int* lvl, int* qa, int* qb,
                                                  int* __restrict__ snode,
                                                  int* __restrict__ pinfo) {
  __shared__ int sh[3];
  __shared__ int far;
  __shared__ int hist[MF_HIST];
  __shared__ int msel;
  const int p = blockIdx.x, tid = threadIdx.x;
  const int o = poff[p], np = poff[p + 1] - o;
  const int* nodes = pperm + o;
  bool leaf = force_leaf || np <= MF_LEAF;
  int mode = 0, m = 0;
  if (!leaf) {
    // first search from the part's smallest node id (members arrive in any order)
    if (tid == 0) far = INT_MAX;
    __syncthreads();
    for (int i = tid; i < np; i += blockDim.x) atomicMin(&far, nodes[i]);
    __syncthreads();
    const int start = far;
    __syncthreads();
    mf_bfs(p, start, nodes, np, grp, gcol, part, lvl, qa + o, qb + o, sh);
    const int L1 = sh[0];
    if (tid == 0) far = INT_MAX;
    __syncthreads();
    for (int i = tid; i < np; i += blockDim.x)
      if (lvl[nodes[i]] == L1) atomicMin(&far, nodes[i]);
    __syncthreads();
    mf_bfs(p, far, nodes, np, grp, gcol, part, lvl, qa + o, qb + o, sh);
    const int L2 = sh[0], reached = sh[2];
    if (L2 >= 2 && L2 < MF_HIST) {
      // separator level m in [1, L2-1]: fewest nodes difference between the levels below
      // it and the rest (higher levels and unreached nodes); first such level on ties
      mode = 1;
      for (int i = tid; i <= L2; i += blockDim.x) hist[i] = 0;
      __syncthreads();
      for (int i = tid; i < np; i += blockDim.x) {
        const int lv = lvl[nodes[i]];
        if (lv >= 0) atomicAdd(&hist[lv], 1);
      }
      __syncthreads();
      if (tid == 0) {
        int below = 0, best = INT_MAX, bm = L2 / 2;
        for (int mm = 1; mm < L2; ++mm) {
          below += hist[mm - 1];
          const int above = np - below - hist[mm];
          const int sc = below > above ? below - above : above - below;
          if (sc < best) {
            best = sc;
            bm = mm;
          }
        }
        msel = bm;
      }
      __syncthreads();
      m = msel;
    } else if (L2 >= 2) {
      mode = 1;
      m = L2 / 2;
    } else if (reached < np) {
      mode = 2;
    } else {
      leaf = true;
    }
  }
  for (int i = tid; i < np; i += blockDim.x) {
    const int v = nodes[i];
    int q = -1;
    if (!leaf) {
      const int lv = lvl[v];
      if (mode == 1) q = (lv == m) ? -1 : ((lv >= 0 && lv < m) ? 2 * p : 2 * p + 1);
      else q = lv >= 0 ? 2 * p : 2 * p + 1;
    }
    npart[v] = q;
    if (q < 0) snode[v] = tb + p;
  }
  if (tid == 0) pinfo[p] = leaf ? 0 : 1;
}

__global__ void k_mf_link(int np, int d, int tb, const int* __restrict__ pinfo,
                          const int* __restrict__ rank, int* __restrict__ tdepth,
                          int* __restrict__ child0, int* __restrict__ child1,
                          int* __restrict__ parent) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int t = tb + p;
  tdepth[t] = d;
  if (pinfo[p]) {
    const int c0 = tb + np + 2 * rank[p];
    child0[t] = c0;
    child1[t] = c0 + 1;
    parent[c0] = t;
    parent[c0 + 1] = t;
  }
}

__global__ void k_mf_relabel(int nn, int* __restrict__ part, const int* __restrict__ npart,
                             const int* __restrict__ rank) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn || part[v] < 0) return;
  const int q = npart[v];
  part[v] = q < 0 ? -1 : 2 * rank[q >> 1] + (q & 1);
}

__global__ void k_mf_rank(int nn, const int* __restrict__ sperm, const int* __restrict__ snode,
                          const int* __restrict__ soff, int* __restrict__ sep_rank) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int v = sperm[i];
  sep_rank[v] = i - soff[snode[v]];
}

// ---------------------------------------------------------------- boundaries
// Candidate boundary of supernode t (depth d) as a bitmap over node ids in LDS; count
// (fill = 0) or write the nodes in ascending order at bnd[bnd_off[t]] (fill = 1).
__global__ void __launch_bounds__(256) k_mf_bnd(int fill, int d, int tb, int nn,
                                                const int* __restrict__ soff,
                                                const int* __restrict__ sperm,
                                                const int* __restrict__ snode,
                                                const int* __restrict__ tdepth,
                                                const int* __restrict__ child0,
                                                const int* __restrict__ child1,
                                                const int* __restrict__ grp,
                                                const int* __restrict__ gcol,
                                                int* __restrict__ bcnt,
                                                const int* __restrict__ bnd_off,
                                                int* __restrict__ bnd) {
  extern __shared__ uint32_t bm[];
  __shared__ int part_cnt[256];
  const int t = tb + blockIdx.x, tid = threadIdx.x;
  const int words = (nn + 31) >> 5;
  for (int w = tid; w < words; w += 256) bm[w] = 0u;
  __syncthreads();
  const int s0 = soff[t], ns = soff[t + 1] - s0;
  for (int k = tid; k < ns; k += 256) {
    const int v = sperm[s0 + k];
    for (int e = grp[v]; e < grp[v + 1]; ++e) {
      const int u = gcol[e];
      if (tdepth[snode[u]] < d) atomicOr(&bm[u >> 5], 1u << (u & 31));
    }
  }
  for (int ci = 0; ci < 2; ++ci) {
    const int ch = ci ? child1[t] : child0[t];
    if (ch < 0) continue;
    const int b0 = bnd_off[ch], nb = bcnt[ch];
    for (int k = tid; k < nb; k += 256) {
      const int u = bnd[b0 + k];
      if (snode[u] != t) atomicOr(&bm[u >> 5], 1u << (u & 31));
    }
  }
  __syncthreads();
  // contiguous word ranges per thread, popcounts, then an ordered scan
  const int cw = (words + 255) / 256;
  const int w0 = min(words, tid * cw), w1 = min(words, w0 + cw);
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popc(bm[w]);
  part_cnt[tid] = cnt;
  __syncthreads();
  if (!fill) {
    if (tid == 0) {
      int s = 0;
      for (int i = 0; i < 256; ++i) s += part_cnt[i];
      bcnt[t] = s;
    }
    return;
  }
  int base = 0;
  for (int i = 0; i < tid; ++i) base += part_cnt[i];
  int* out = bnd + bnd_off[t] + base;
  for (int w = w0; w < w1; ++w) {
    uint32_t bits = bm[w];
    while (bits) {
      const int b = __ffs(bits) - 1;
      *out++ = (w << 5) + b;
      bits &= bits - 1;
    }
  }
}

__global__ void k_mf_add_base(int nt, int tb, int base, const int* __restrict__ tmp,
                              int* __restrict__ bnd_off) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nt) bnd_off[tb + i] = base + tmp[i];
}

// positions (in the parent's front, DOF units of the node's first component) of every
// child boundary node
__global__ void __launch_bounds__(256) k_mf_bnd_pos(int bs, const int* __restrict__ parent,
                                                    const int* __restrict__ snode,
                                                    const int* __restrict__ sep_rank,
                                                    const int* __restrict__ bcnt,
                                                    const int* __restrict__ bnd_off,
                                                    const int* __restrict__ bnd,
                                                    const int* __restrict__ fS,
                                                    int* __restrict__ bnd_pos, int* flag) {
  const int c = blockIdx.x, t = parent[c];
  if (t < 0) return;
  const int nb = bcnt[c], o = bnd_off[c];
  const int* pb = bnd + bnd_off[t];
  const int pnb = bcnt[t];
  for (int k = threadIdx.x; k < nb; k += 256) {
    const int u = bnd[o + k];
    int pos;
    if (snode[u] == t) {
      pos = bs * sep_rank[u];
    } else {
      const int m = lower_bound_dev(pb, pnb, u);
      if (m >= pnb || pb[m] != u) {
        atomicOr(flag, 4);
        pos = 0;
      } else {
        pos = fS[t] + bs * m;
      }
    }
    bnd_pos[o + k] = pos;
  }
}

// ---------------------------------------------------------------- numeric factorisation
// Original entries of the separator rows (and their transposes in the boundary rows);
// identity on the padding of the separator block.
__global__ void __launch_bounds__(256) k_mf_assemble(int bs, const int* __restrict__ rp,
                                                     const int* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const int* __restrict__ soff,
                                                     const int* __restrict__ sperm,
                                                     const int* __restrict__ snode,
                                                     const int* __restrict__ sep_rank,
                                                     const int* __restrict__ tdepth,
                                                     const int* __restrict__ bcnt,
                                                     const int* __restrict__ bnd_off,
                                                     const int* __restrict__ bnd,
                                                     const int* __restrict__ fs,
                                                     const int* __restrict__ fS,
                                                     const int* __restrict__ fT,
                                                     const int64_t* __restrict__ fo,
                                                     double* __restrict__ F, int* flag) {
  const int t = blockIdx.x, tid = threadIdx.x;
  const int s = fs[t], S = fS[t], d = tdepth[t];
  const int64_t ld = int64_t(fT[t]) * 64;
  double* Ft = F + fo[t];
  for (int k = s + tid; k < S; k += 256) Ft[k * ld + k] = 1.0;
  const int* pb = bnd + bnd_off[t];
  const int pnb = bcnt[t];
  for (int k = tid; k < s; k += 256) {
    const int v = sperm[soff[t] + k / bs];
    const int row = v * bs + k % bs;
    for (int e = rp[row]; e < rp[row + 1]; ++e) {
      const int cidx = col[e], u = cidx / bs, q = cidx % bs;
      const int su = snode[u];
      if (su == t) {
        Ft[k * ld + bs * sep_rank[u] + q] = val[e];
      } else if (tdepth[su] < d) {
        const int m = lower_bound_dev(pb, pnb, u);
        if (m >= pnb || pb[m] != u) {
          atomicOr(flag, 4);
          continue;
        }
        const int64_t pos = S + int64_t(bs) * m + q;
        Ft[k * ld + pos] = val[e];
        Ft[pos * ld + k] = val[e];
      }
    }
  }
}

// lower triangle of child `ci`'s update matrix added into the parent front
__global__ void __launch_bounds__(256) k_mf_extadd(int tb, int ci, int bs,
                                                   const int* __restrict__ child0,
                                                   const int* __restrict__ child1,
                                                   const int* __restrict__ bnd_off,
                                                   const int* __restrict__ bnd_pos,
                                                   const int* __restrict__ fb,
                                                   const int* __restrict__ fS,
                                                   const int* __restrict__ fT,
                                                   const int64_t* __restrict__ fo,
                                                   double* __restrict__ F) {
  const int t = tb + blockIdx.y;
  const int c = ci ? child1[t] : child0[t];
  if (c < 0) return;
  const int bc = fb[c], Sc = fS[c];
  const int64_t ldc = int64_t(fT[c]) * 64, ldt = int64_t(fT[t]) * 64;
  const double* Fc = F + fo[c];
  double* Ft = F + fo[t];
  const int* pos = bnd_pos + bnd_off[c];
  for (int i = blockIdx.x; i < bc; i += gridDim.x) {
    const int64_t pi = pos[i / bs] + i % bs;
    const double* urow = Fc + (Sc + i) * ldc + Sc;
    for (int j = threadIdx.x; j <= i; j += 256) {
      const int64_t pj = pos[j / bs] + j % bs;
      const int64_t a = pi > pj ? pi : pj, b = pi > pj ? pj : pi;
      Ft[a * ldt + b] += urow[j];
    }
  }
}

// Cholesky and inverse of one 64x64 diagonal tile k (lower triangle read; L written back
// with a zero upper triangle, L^{-1} to the diagonal tile of the front's solve matrix M,
// leading dimension S).  One wavefront; lane t keeps row t in registers and column j is
// broadcast through LDS.
__global__ void __launch_bounds__(64) k_mf_potrf(int tb, int k, const int* __restrict__ fS,
                                                 const int* __restrict__ fT,
                                                 const int64_t* __restrict__ fo,
                                                 const int64_t* __restrict__ mo,
                                                 double* __restrict__ F,
                                                 double* __restrict__ M, int* info) {
  const int t = tb + blockIdx.x;
  const int S = fS[t];
  if (k >= S / 64) return;
  const int64_t ld = int64_t(fT[t]) * 64;
  double* A = F + fo[t] + int64_t(64 * k) * ld + 64 * k;
  double* L = M + mo[t] + int64_t(64 * k) * S + 64 * k;
  __shared__ double colj[64];
  __shared__ double Ls[64][65];
  const int r = threadIdx.x;
  for (int i = 0; i < 64; ++i) Ls[i][r] = A[i * ld + r];
  __syncthreads();
  double row[64];
#pragma unroll
  for (int l = 0; l < 64; ++l) row[l] = Ls[r][l];
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    colj[r] = row[j];
    __syncthreads();
    const double p = colj[j];
    if (r == 0 && !(p > 0.0)) atomicOr(info, 1);
    const double dj = sqrt(p > 0.0 ? p : 1.0);
    const double lj = (r > j) ? row[j] / dj : dj;
    if (r >= j) row[j] = lj;
    __syncthreads();
    colj[r] = lj;
    __syncthreads();
    if (r > j) {
#pragma unroll
      for (int l = j + 1; l < 64; ++l)
        if (l <= r) row[l] -= lj * colj[l];
    }
    __syncthreads();
  }
#pragma unroll
  for (int l = 0; l < 64; ++l) Ls[r][l] = (l <= r) ? row[l] : 0.0;
  __syncthreads();
  for (int i = 0; i < 64; ++i) A[i * ld + r] = Ls[i][r];
  double x[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    double s = (i == r) ? 1.0 : 0.0;
#pragma unroll
    for (int l = 0; l < i; ++l) s -= Ls[i][l] * x[l];
    x[i] = (i >= r) ? s / Ls[i][i] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 64; ++i) Ls[i][r] = x[i];
  __syncthreads();
  for (int i = 0; i < 64; ++i) L[i * S + r] = Ls[i][r];
}

// ---- 64x64 tile products on MFMA: 256 threads, each wavefront a 32x32 quarter as 2x2
// v_mfma_f64_16x16x4f64 tiles (operand lane l: A[l%16][l/16], B[l/16][l%16]; result
// lane l, register r: D[4r + l/16][l%16]).  Operands are staged in LDS.
struct MfTiles {
  double A[64][65];
  double B[64][65];
};

__device__ __forceinline__ void mf_zero(v4d (&acc)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
}

// acc += As * op(Bs) with op = transpose (TB) or identity, operands already in LDS
template <bool TB>
__device__ __forceinline__ void mf_mac_lds(v4d (&acc)[2][2], const MfTiles& sm) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
#pragma unroll 4
  for (int ks = 0; ks < 16; ++ks) {
    const int kq = ks * 4 + (lane >> 4);
    double af[2], bf[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) af[a] = sm.A[wr + a * 16 + (lane & 15)][kq];
#pragma unroll
    for (int b = 0; b < 2; ++b)
      bf[b] = TB ? sm.B[wc + b * 16 + (lane & 15)][kq] : sm.B[kq][wc + b * 16 + (lane & 15)];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
  }
}

__device__ __forceinline__ void mf_load(double (*T)[65], const double* G, int64_t ld) {
  for (int e = threadIdx.x; e < 4096; e += 256) T[e >> 6][e & 63] = G[(e >> 6) * ld + (e & 63)];
}

// acc += A * op(B) for global tiles
template <bool TB>
__device__ __forceinline__ void mf_mac(v4d (&acc)[2][2], MfTiles& sm, const double* A,
                                       int64_t lda, const double* B, int64_t ldb) {
  __syncthreads();
  mf_load(sm.A, A, lda);
  mf_load(sm.B, B, ldb);
  __syncthreads();
  mf_mac_lds<TB>(acc, sm);
}

// C = alpha acc + beta C (global) or T = acc (LDS, lds != nullptr)
__device__ __forceinline__ void mf_store(const v4d (&acc)[2][2], double* C, int64_t ldc,
                                         double alpha, double beta) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double* cp = C + (wr + a * 16 + 4 * r + (lane >> 4)) * ldc + wc + b * 16 + (lane & 15);
        *cp = alpha * acc[a][b][r] + (beta == 0.0 ? 0.0 : beta * *cp);
      }
}
__device__ __forceinline__ void mf_store_lds(const v4d (&acc)[2][2], double (*T)[65]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        T[wr + a * 16 + 4 * r + (lane >> 4)][wc + b * 16 + (lane & 15)] = acc[a][b][r];
}

// L_ik = F_ik Linv_kk^T for the tiles below diagonal tile k (in place)
__global__ void __launch_bounds__(256) k_mf_trsm(int tb, int k, const int* __restrict__ fS,
                                                 const int* __restrict__ fT,
                                                 const int64_t* __restrict__ fo,
                                                 const int64_t* __restrict__ mo,
                                                 double* __restrict__ F,
                                                 const double* __restrict__ M) {
  __shared__ MfTiles sm;
  const int t = tb + blockIdx.y;
  const int T = fT[t], S = fS[t];
  const int i = k + 1 + blockIdx.x;
  if (k >= S / 64 || i >= T) return;
  const int64_t ld = int64_t(T) * 64;
  double* C = F + fo[t] + int64_t(64 * i) * ld + 64 * k;
  v4d acc[2][2];
  mf_zero(acc);
  mf_mac<true>(acc, sm, C, ld, M + mo[t] + int64_t(64 * k) * S + 64 * k, S);
  mf_store(acc, C, ld, 1.0, 0.0);
}

// F_ij -= L_ik L_jk^T for k < j <= i (lower trailing tiles)
__global__ void __launch_bounds__(256) k_mf_update(int tb, int k, const int* __restrict__ fS,
                                                   const int* __restrict__ fT,
                                                   const int64_t* __restrict__ fo,
                                                   double* __restrict__ F) {
  __shared__ MfTiles sm;
  const int t = tb + blockIdx.y;
  const int T = fT[t];
  if (k >= fS[t] / 64) return;
  const int m = T - k - 1;
  const int q = blockIdx.x;
  if (q >= m * (m + 1) / 2) return;
  int ii = int((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while (ii * (ii + 1) / 2 > q) --ii;
  while ((ii + 1) * (ii + 2) / 2 <= q) ++ii;
  const int jj = q - ii * (ii + 1) / 2;
  const int i = k + 1 + ii, j = k + 1 + jj;
  const int64_t ld = int64_t(T) * 64;
  double* Ft = F + fo[t];
  v4d acc[2][2];
  mf_zero(acc);
  mf_mac<true>(acc, sm, Ft + int64_t(64 * i) * ld + 64 * k, ld, Ft + int64_t(64 * j) * ld + 64 * k,
               ld);
  mf_store(acc, Ft + int64_t(64 * i) * ld + 64 * j, ld, -1.0, 1.0);
}

// Row-tile i of X = L11^{-1}: X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj for j < i (X_ii is the
// diagonal-tile inverse already in M; rows above i are final)
__global__ void __launch_bounds__(256) k_mf_inv_row(int tb, int i, const int* __restrict__ fS,
                                                    const int* __restrict__ fT,
                                                    const int64_t* __restrict__ fo,
                                                    const int64_t* __restrict__ mo,
                                                    const double* __restrict__ F,
                                                    double* __restrict__ M) {
  __shared__ MfTiles sm;
  const int t = tb + blockIdx.y, j = blockIdx.x;
  const int S = fS[t];
  if (i >= S / 64 || j >= i) return;
  const int64_t ld = int64_t(fT[t]) * 64;
  const double* Ft = F + fo[t];
  double* Mt = M + mo[t];
  v4d acc[2][2];
  mf_zero(acc);
  for (int k = j; k < i; ++k)
    mf_mac<false>(acc, sm, Ft + int64_t(64 * i) * ld + 64 * k, ld,
                  Mt + int64_t(64 * k) * S + 64 * j, S);
  __syncthreads();
  mf_store_lds(acc, sm.B);
  mf_load(sm.A, Mt + int64_t(64 * i) * S + 64 * i, S);
  __syncthreads();
  mf_zero(acc);
  mf_mac_lds<false>(acc, sm);
  mf_store(acc, Mt + int64_t(64 * i) * S + 64 * j, S, -1.0, 0.0);
}

// G = L21 X (boundary tile rows of M): G_mj = sum_{k >= j} L_{p+m, k} X_kj, p = S/64
__global__ void __launch_bounds__(256) k_mf_g(int tb, const int* __restrict__ fS,
                                              const int* __restrict__ fT,
                                              const int64_t* __restrict__ fo,
                                              const int64_t* __restrict__ mo,
                                              const double* __restrict__ F,
                                              double* __restrict__ M) {
  __shared__ MfTiles sm;
  const int t = tb + blockIdx.y;
  const int S = fS[t], T = fT[t], p = S / 64;
  if (p == 0) return;
  const int m = blockIdx.x / p, j = blockIdx.x % p;
  if (m >= T - p) return;
  const int64_t ld = int64_t(T) * 64;
  const double* Ft = F + fo[t];
  double* Mt = M + mo[t];
  v4d acc[2][2];
  mf_zero(acc);
  for (int k = j; k < p; ++k)
    mf_mac<false>(acc, sm, Ft + int64_t(64 * (p + m)) * ld + 64 * k, ld,
                  Mt + int64_t(64 * k) * S + 64 * j, S);
  mf_store(acc, Mt + int64_t(64 * (p + m)) * S + 64 * j, S, 1.0, 0.0);
}

// MT (S x Fp) = M^T (M is Fp x S), 64x64 tiles through LDS
__global__ void __launch_bounds__(256) k_mf_transpose(int tb, const int* __restrict__ fS,
                                                      const int* __restrict__ fT,
                                                      const int64_t* __restrict__ mo,
                                                      const double* __restrict__ M,
                                                      double* __restrict__ MT) {
  __shared__ double tile[64][65];
  const int t = tb + blockIdx.y;
  const int S = fS[t], T = fT[t], p = S / 64;
  if (p == 0) return;
  const int ti = blockIdx.x / p, tj = blockIdx.x % p;   // tile (ti, tj) of M
  if (ti >= T) return;
  const int64_t Fp = int64_t(T) * 64;
  const double* src = M + mo[t] + int64_t(64 * ti) * S + 64 * tj;
  double* dst = MT + mo[t] + int64_t(64 * tj) * Fp + 64 * ti;
  for (int e = threadIdx.x; e < 4096; e += 256) tile[e >> 6][e & 63] = src[(e >> 6) * S + (e & 63)];
  __syncthreads();
  for (int e = threadIdx.x; e < 4096; e += 256) dst[(e >> 6) * Fp + (e & 63)] = tile[e & 63][e >> 6];
}

// ---------------------------------------------------------------- solve
// Rows per wavefront in the solve kernels: each wave issues the loads of MF_R rows of the
// factor back to back (row indices clamped, products masked) and shares the vector entries
// among them; one row per wave left the mid depths of the tree waiting on memory latency.
// MF_R divides 64.
constexpr int MF_R = 4;
// The solve kernels run over per-depth work lists (one MFWork per workgroup) built at
// setup, so the grid holds exactly the workgroups the fronts of a depth need.
//
// Column split of the solve kernels: KS = 1, each wavefront of a workgroup takes MF_R rows
// of its own (4 * MF_R rows per workgroup); KS = 4, the four wavefronts share MF_R rows and
// take every fourth 64-column stretch of them, the partial sums meeting in LDS (fixed
// order).  The shallow tree depths hold few fronts with long rows: there KS = 4 gives the
// chip four times the wavefronts and each one a quarter of the dependent loads.
constexpr int MF_KS = 4;
constexpr int MF_SPLIT_WG = 512;   // a depth with fewer row-group workgroups splits columns

// sum of the KS wavefronts' partial sums of rows lane < MF_R, in wavefront order (KS > 1);
// every wavefront of the workgroup calls it
template <int KS>
__device__ __forceinline__ double mf_split_sum(double mine) {
  if constexpr (KS == 1) {
    return mine;
  } else {
    __shared__ double part[KS][MF_R];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane < MF_R) part[wv][lane] = mine;
    __syncthreads();
    double s = 0.0;
    if (lane < MF_R)
#pragma unroll
      for (int k = 0; k < KS; ++k) s += part[k][lane];
    return s;
  }
}

// Forward rows i0 .. i0+MF_R-1 of M: [y; u] = [X; -G] f_s + [0; f_b].  The front's
// right-hand side f is read where it is used: f = r (separator positions, tree order) +
// slot 0 + slot 1 (the children's update vectors, already at the front's positions), the
// same sum in the same order as assembling the front first.  y goes to fv; the update
// vector u goes straight to its place in the parent's slot array.  With KS = 4 every
// wavefront of the workgroup reaches the LDS sum: i0, S and rows are the same for all.
template <int KS>
__global__ void __launch_bounds__(256) k_mf_fwd(const MFWork* __restrict__ wl, int bs, int tv,
                                                const double* __restrict__ r,
                                                const int* __restrict__ bnd_pos,
                                                const double* __restrict__ M, double* us,
                                                double* __restrict__ y) {
  const MFWork w = wl[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int S = w.S, rows = w.S + w.b;
  const int i0 = (KS == 1 ? w.blk * 4 + wv : w.blk) * MF_R;
  if (i0 >= rows) return;
  const double* fr = r + w.roff;
  const double* s0 = us + w.vo;
  const double* s1 = us + int64_t(tv) + w.vo;
  // the lane's own boundary row: its f_b entry and where its u entry goes
  const int io = i0 + lane;
  double fo = 0.0;
  int64_t dst = 0;
  if (lane < MF_R && io < rows && io >= S) {
    if (w.nch) fo = s0[io] + s1[io];
    const int m = io - S;
    dst = int64_t(w.uoff) + bnd_pos[w.boff + m / bs] + m % bs;
  }
  const double* rowp[MF_R];
  int jend[MF_R];
  int jmax = 0;
#pragma unroll
  for (int q = 0; q < MF_R; ++q) {
    const int i = i0 + q;
    jend[q] = i >= rows ? 0 : (i < S ? (i / 64 + 1) * 64 : S);
    jmax = max(jmax, jend[q]);
    rowp[q] = M + int64_t(w.mo) * 4096 + int64_t(min(i, rows - 1)) * S;
  }
  double acc[MF_R];
#pragma unroll
  for (int q = 0; q < MF_R; ++q) acc[q] = 0.0;
#pragma unroll 4
  for (int j = (KS == 1 ? 0 : wv * 64) + lane; j < jmax; j += 64 * KS) {
    double fj = j < w.s ? fr[j] : 0.0;
    if (w.nch) fj = fj + s0[j] + s1[j];
    double v[MF_R];
#pragma unroll
    for (int q = 0; q < MF_R; ++q) v[q] = ld_stream(&rowp[q][j]);   // j < jmax <= S: inside the row
#pragma unroll
    for (int q = 0; q < MF_R; ++q)
      if (j < jend[q]) acc[q] += v[q] * fj;
  }
  double mine = 0.0;
#pragma unroll
  for (int q = 0; q < MF_R; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == q) mine = t;
  }
  mine = mf_split_sum<KS>(mine);
  if ((KS == 1 || wv == 0) && lane < MF_R && io < rows) {
    if (io < S) y[w.vo + io] = mine;
    else us[dst] = fo - mine;
  }
}

// x_s = X^T y - G^T x_b: separator rows j0 .. j0+MF_R-1 of MT (column split as in the
// forward rows), x in tree order.  Each lane gathers the boundary values x_b of its own
// columns: their index loads go out with the factor loads, so no workgroup barrier waits
// for a staged copy.
template <int KS>
__global__ void __launch_bounds__(256) k_mf_bwd(const MFWork* __restrict__ wl, int bs,
                                                double* __restrict__ x,
                                                const int* __restrict__ bnd_tp,
                                                const double* __restrict__ MT,
                                                const double* __restrict__ yv) {
  const MFWork w = wl[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int s = w.s, S = w.S, b = w.b;
  const int j0 = (KS == 1 ? w.blk * 4 + wv : w.blk) * MF_R;
  if (j0 >= s) return;
  const int64_t Fp = S + ((b + 63) & ~63);
  const double* y = yv + w.vo;
  const int* bt = bnd_tp + w.boff;
  const double* rowp[MF_R];
#pragma unroll
  for (int q = 0; q < MF_R; ++q)
    rowp[q] = MT + int64_t(w.mo) * 4096 + int64_t(min(j0 + q, s - 1)) * Fp;
  double acc[MF_R];
#pragma unroll
  for (int q = 0; q < MF_R; ++q) acc[q] = 0.0;
  // rows j0 .. j0+MF_R-1 share their 64-block, so the same columns start the sum
#pragma unroll 4
  for (int i = (j0 / 64) * 64 + (KS == 1 ? 0 : wv * 64) + lane; i < S; i += 64 * KS) {
    const double yi = y[i];
    double v[MF_R];
#pragma unroll
    for (int q = 0; q < MF_R; ++q) v[q] = ld_stream(&rowp[q][i]);
#pragma unroll
    for (int q = 0; q < MF_R; ++q)
      if (j0 + q < s) acc[q] += v[q] * yi;
  }
#pragma unroll 4
  for (int m = (KS == 1 ? 0 : wv * 64) + lane; m < b; m += 64 * KS) {
    const double xb = x[int64_t(bt[m / bs]) * bs + m % bs];
    double v[MF_R];
#pragma unroll
    for (int q = 0; q < MF_R; ++q) v[q] = ld_stream(&rowp[q][S + m]);
#pragma unroll
    for (int q = 0; q < MF_R; ++q)
      if (j0 + q < s) acc[q] -= v[q] * xb;
  }
  double mine = 0.0;
#pragma unroll
  for (int q = 0; q < MF_R; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == q) mine = t;
  }
  mine = mf_split_sum<KS>(mine);
  if ((KS == 1 || wv == 0) && lane < MF_R && j0 + lane < s) x[w.roff + j0 + lane] = mine;
}

// tree order <-> the caller's order
__global__ void k_mf_to_tree(int n, const int* __restrict__ tdof, const double* __restrict__ r,
                             double* __restrict__ rt) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) rt[q] = r[tdof[q]];
}
__global__ void k_mf_index_to_tree(int n, const int* __restrict__ tdof,
                                   const int* __restrict__ idx, int* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = idx[tdof[q]];
}
__global__ void k_mf_from_tree(int n, const int* __restrict__ tdof,
                               const double* __restrict__ xt, double* __restrict__ x) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) x[tdof[q]] = xt[q];
}

// tree-order node position of every boundary node, and the DOF of every tree position
__global__ void k_mf_tree_pos(int used, int nn, int bs, const int* __restrict__ bnd,
                              const int* __restrict__ snode, const int* __restrict__ soff,
                              const int* __restrict__ sep_rank, const int* __restrict__ sperm,
                              int* __restrict__ bnd_tp, int* __restrict__ tdof) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < used) {
    const int u = bnd[i];
    bnd_tp[i] = soff[snode[u]] + sep_rank[u];
  }
  if (i < nn)
    for (int k = 0; k < bs; ++k) tdof[i * bs + k] = sperm[i] * bs + k;
}

// ---------------------------------------------------------------- host side
static void grow(Ctx& c, DBuf<int>& b, size_t used, size_t need) {
  if (need <= b.n) return;
  DBuf<int> nb(std::max(need, 2 * b.n));
  if (used) AMGF_HIP(hipMemcpyAsync(nb.p, b.p, used * sizeof(int), hipMemcpyDeviceToDevice, c.s));
  b = std::move(nb);
}
void MFSolver::setup(Ctx& c, int n_, int bs_, const int* rp, const int* col,
                     const double* val) {
  n = n_;
  bs = bs_;
  AMGF_REQUIRE(bs >= 1 && n >= 0 && n % bs == 0, AMGF_EINVAL, "multifrontal: bad block size");
  nn = n / bs;
  ntree = ndepth = 0;
  tree_off.assign(1, 0);
  if (n == 0) return;
  AMGF_REQUIRE(nn <= MF_MAXNODES, AMGF_ENOMEM, "multifrontal: graph too large");
  // ---- node graph
  DBuf<int> gcnt(size_t(nn) + 1), grp(size_t(nn) + 1);
  hipLaunchKernelGGL(k_mf_node_graph, dim3(grid_for(nn, 256)), dim3(256), 0, c.s, nn, bs, rp,
                     col, nullptr, gcnt.p, nullptr);
  const int ne = scan_exclusive(c, gcnt.p, grp.p, nn);
  DBuf<int> gcol(std::max(ne, 1));
  hipLaunchKernelGGL(k_mf_node_graph, dim3(grid_for(nn, 256)), dim3(256), 0, c.s, nn, bs, rp,
                     col, grp.p, nullptr, gcol.p);
  AMGF_LAUNCH_CHECK();
  // ---- nested dissection, one depth at a time
  const int cap = 2 * nn + 2;
  DBuf<int> part(nn), npart(nn), lvl(nn), qa(nn), qb(nn), parent(cap);
  snode.alloc(nn);
  tdepth.alloc(cap);
  child0.alloc(cap);
  child1.alloc(cap);
  AMGF_HIP(hipMemsetAsync(part.p, 0, part.bytes(), c.s));
  AMGF_HIP(hipMemsetAsync(parent.p, 0xff, parent.bytes(), c.s));
  AMGF_HIP(hipMemsetAsync(child0.p, 0xff, child0.bytes(), c.s));
  AMGF_HIP(hipMemsetAsync(child1.p, 0xff, child1.bytes(), c.s));
  int np = 1, tb = 0, d = 0;
  while (np > 0) {
    AMGF_REQUIRE(d < MF_MAXD && tb + np <= cap, AMGF_ENOMEM, "multifrontal: ordering depth");
    DBuf<int> poff, pperm;
    group_by_key(c, part.p, nn, np, poff, pperm, false);   // order within a part unused
    DBuf<int> pinfo(size_t(np) + 1), rank(size_t(np) + 1);
    hipLaunchKernelGGL(k_mf_split, dim3(np), dim3(MF_SPLIT_THREADS), 0, c.s, tb,
                       int(d == MF_MAXD - 1),
                       poff.p, pperm.p, grp.p, gcol.p, part.p, npart.p, lvl.p, qa.p, qb.p,
                       snode.p, pinfo.p);
    AMGF_LAUNCH_CHECK();
    const int nsplit = scan_exclusive(c, pinfo.p, rank.p, np);
    hipLaunchKernelGGL(k_mf_link, dim3(grid_for(np, 256)), dim3(256), 0, c.s, np, d, tb,
                       pinfo.p, rank.p, tdepth.p, child0.p, child1.p, parent.p);
    hipLaunchKernelGGL(k_mf_relabel, dim3(grid_for(nn, 256)), dim3(256), 0, c.s, nn, part.p,
                       npart.p, rank.p);
    AMGF_LAUNCH_CHECK();
    tb += np;
    tree_off.push_back(tb);
    np = 2 * nsplit;
    ++d;
  }
  ntree = tb;
  ndepth = d;
  // ---- supernode members
  group_by_key(c, snode.p, nn, ntree, soff, sperm);
  sep_rank.alloc(nn);
  hipLaunchKernelGGL(k_mf_rank, dim3(grid_for(nn, 256)), dim3(256), 0, c.s, nn, sperm.p,
                     snode.p, soff.p, sep_rank.p);
  AMGF_LAUNCH_CHECK();
  // ---- boundaries, deepest supernodes first
  DBuf<int> bcnt(ntree);
  bnd_off.alloc(ntree);
  bnd.alloc(std::max<size_t>(size_t(nn) * 4, 1024));
  size_t used = 0;
  const size_t lds = size_t((nn + 31) / 32) * sizeof(uint32_t);
  for (int dd = ndepth - 1; dd >= 0; --dd) {
    const int b0 = tree_off[dd], nt = tree_off[dd + 1] - b0;
    hipLaunchKernelGGL(k_mf_bnd, dim3(nt), dim3(256), lds, c.s, 0, dd, b0, nn, soff.p, sperm.p,
                       snode.p, tdepth.p, child0.p, child1.p, grp.p, gcol.p, bcnt.p, bnd_off.p,
                       bnd.p);
    AMGF_LAUNCH_CHECK();
    DBuf<int> tmp(size_t(nt) + 1);
    const int total = scan_exclusive(c, bcnt.p + b0, tmp.p, nt);
    AMGF_REQUIRE(used + size_t(total) < size_t(INT_MAX), AMGF_ENOMEM,
                 "multifrontal: boundary lists");
    grow(c, bnd, used, used + size_t(total));
    hipLaunchKernelGGL(k_mf_add_base, dim3(grid_for(nt, 256)), dim3(256), 0, c.s, nt, b0,
                       int(used), tmp.p, bnd_off.p);
    hipLaunchKernelGGL(k_mf_bnd, dim3(nt), dim3(256), lds, c.s, 1, dd, b0, nn, soff.p, sperm.p,
                       snode.p, tdepth.p, child0.p, child1.p, grp.p, gcol.p, bcnt.p, bnd_off.p,
                       bnd.p);
    AMGF_LAUNCH_CHECK();
    used += size_t(total);
  }
  // ---- front sizes (host)
  std::vector<int> hsoff = d2h(soff.p, size_t(ntree) + 1, c.s);
  std::vector<int> hb = d2h(bcnt.p, ntree, c.s);
  h_s.resize(ntree);
  h_S.resize(ntree);
  h_b.resize(ntree);
  h_T.resize(ntree);
  std::vector<int64_t> hfo(ntree), hmo(ntree), hvo(ntree);
  int64_t tf = 0, tm = 0, tvs = 0;
  for (int t = 0; t < ntree; ++t) {
    h_s[t] = bs * (hsoff[t + 1] - hsoff[t]);
    h_S[t] = (h_s[t] + 63) / 64 * 64;
    h_b[t] = bs * hb[t];
    const int Fp = h_S[t] + (h_b[t] + 63) / 64 * 64;
    AMGF_REQUIRE(h_S[t] <= MF_SMAX, AMGF_ENOMEM, "multifrontal: separator too large");
    h_T[t] = Fp / 64;
    hfo[t] = tf;
    hmo[t] = tm;
    hvo[t] = tvs;
    tf += int64_t(Fp) * Fp;
    tm += int64_t(Fp) * h_S[t];
    tvs += Fp;
  }
  AMGF_REQUIRE(tvs < (int64_t(1) << 30) && tm / 4096 < INT_MAX, AMGF_ENOMEM,
               "multifrontal: fronts too large");
  tv = int(tvs);
  for (int dd = 0; dd < ndepth; ++dd)
    AMGF_REQUIRE(tree_off[dd + 1] - tree_off[dd] <= 65535, AMGF_ENOMEM,
                 "multifrontal: too many fronts in one level");
  auto up = [&](DBuf<int>& dst, const std::vector<int>& src) {
    dst.alloc(src.size());
    AMGF_HIP(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(int), hipMemcpyHostToDevice,
                            c.s));
  };
  auto up64 = [&](DBuf<int64_t>& dst, const std::vector<int64_t>& src) {
    dst.alloc(src.size());
    AMGF_HIP(hipMemcpyAsync(dst.p, src.data(), src.size() * sizeof(int64_t),
                            hipMemcpyHostToDevice, c.s));
  };
  DBuf<int64_t> fo;
  up(fs, h_s);
  up(fS, h_S);
  up(fb, h_b);
  up(fT, h_T);
  up64(fo, hfo);
  up64(mo, hmo);
  up64(vo, hvo);
  DBuf<double> F(size_t(std::max<int64_t>(tf, 1)));
  M.alloc(size_t(std::max<int64_t>(tm, 1)));
  MT.alloc(size_t(std::max<int64_t>(tm, 1)));
  fv.alloc(size_t(std::max(tv, 1)));
  us.alloc(2 * size_t(std::max(tv, 1)));
  rt.alloc(size_t(n));
  xt.alloc(size_t(n));
  AMGF_HIP(hipMemsetAsync(us.p, 0, us.bytes(), c.s));
  bnd_pos.alloc(std::max<size_t>(used, 1));
  bnd_tp.alloc(std::max<size_t>(used, 1));
  tdof.alloc(size_t(n));
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  hipLaunchKernelGGL(k_mf_bnd_pos, dim3(ntree), dim3(256), 0, c.s, bs, parent.p, snode.p,
                     sep_rank.p, bcnt.p, bnd_off.p, bnd.p, fS.p, bnd_pos.p, c.flag.p);
  hipLaunchKernelGGL(k_mf_tree_pos, dim3(grid_for(std::max<int64_t>(int64_t(used), nn), 256)),
                     dim3(256), 0, c.s, int(used), nn, bs, bnd.p, snode.p, soff.p, sep_rank.p,
                     sperm.p, bnd_tp.p, tdof.p);
  // ---- numeric: original entries, then depth by depth from the leaves
  AMGF_HIP(hipMemsetAsync(F.p, 0, F.bytes(), c.s));
  AMGF_HIP(hipMemsetAsync(M.p, 0, M.bytes(), c.s));
  hipLaunchKernelGGL(k_mf_assemble, dim3(ntree), dim3(256), 0, c.s, bs, rp, col, val, soff.p,
                     sperm.p, snode.p, sep_rank.p, tdepth.p, bcnt.p, bnd_off.p, bnd.p, fs.p,
                     fS.p, fT.p, fo.p, F.p, c.flag.p);
  AMGF_LAUNCH_CHECK();
  for (int dd = ndepth - 1; dd >= 0; --dd) {
    const int b0 = tree_off[dd], nt = tree_off[dd + 1] - b0;
    for (int ci = 0; ci < 2; ++ci)
      hipLaunchKernelGGL(k_mf_extadd, dim3(64, nt), dim3(256), 0, c.s, b0, ci, bs, child0.p,
                         child1.p, bnd_off.p, bnd_pos.p, fb.p, fS.p, fT.p, fo.p, F.p);
    int ktiles = 0, gtiles = 0, ttiles = 0;
    for (int t = b0; t < b0 + nt; ++t) {
      const int p = h_S[t] / 64;
      ktiles = std::max(ktiles, p);
      gtiles = std::max(gtiles, (h_T[t] - p) * p);
      ttiles = std::max(ttiles, h_T[t] * p);
    }
    // partial Cholesky of every front of this depth, tile column by tile column
    for (int k = 0; k < ktiles; ++k) {
      int rows = 0, pairs = 0;
      for (int t = b0; t < b0 + nt; ++t) {
        if (k >= h_S[t] / 64) continue;
        const int m = h_T[t] - k - 1;
        rows = std::max(rows, m);
        pairs = std::max(pairs, m * (m + 1) / 2);
      }
      hipLaunchKernelGGL(k_mf_potrf, dim3(nt), dim3(64), 0, c.s, b0, k, fS.p, fT.p, fo.p, mo.p,
                         F.p, M.p, c.flag.p);
      if (rows > 0)
        hipLaunchKernelGGL(k_mf_trsm, dim3(rows, nt), dim3(256), 0, c.s, b0, k, fS.p, fT.p,
                           fo.p, mo.p, F.p, M.p);
      if (pairs > 0)
        hipLaunchKernelGGL(k_mf_update, dim3(pairs, nt), dim3(256), 0, c.s, b0, k, fS.p, fT.p,
                           fo.p, F.p);
      AMGF_LAUNCH_CHECK();
    }
    // solve matrices: X = L11^{-1} row tile by row tile, G = L21 X, and M^T
    for (int i = 1; i < ktiles; ++i)
      hipLaunchKernelGGL(k_mf_inv_row, dim3(i, nt), dim3(256), 0, c.s, b0, i, fS.p, fT.p, fo.p,
                         mo.p, F.p, M.p);
    if (gtiles > 0)
      hipLaunchKernelGGL(k_mf_g, dim3(gtiles, nt), dim3(256), 0, c.s, b0, fS.p, fT.p, fo.p, mo.p,
                         F.p, M.p);
    if (ttiles > 0)
      hipLaunchKernelGGL(k_mf_transpose, dim3(ttiles, nt), dim3(256), 0, c.s, b0, fS.p, fT.p,
                         mo.p, M.p, MT.p);
    AMGF_LAUNCH_CHECK();
  }
  // per-depth launch extents of the solve: workgroups of 4 * MF_R rows, or of MF_R rows
  // with the columns split over the four wavefronts (ks = MF_KS) where a depth would give
  // fewer than MF_SPLIT_WG workgroups
  {
    const std::vector<int> hbo = d2h(bnd_off.p, size_t(ntree), c.s);
    const std::vector<int> hpar = d2h(parent.p, size_t(ntree), c.s);
    const std::vector<int> hc0 = d2h(child0.p, size_t(ntree), c.s);
    const std::vector<int> hc1 = d2h(child1.p, size_t(ntree), c.s);
    auto work = [&](int t, int blk) {
      MFWork w;
      w.blk = blk;
      w.S = h_S[t];
      w.b = h_b[t];
      w.s = h_s[t];
      w.nch = (hc0[t] >= 0) + (hc1[t] >= 0);
      w.roff = bs * hsoff[t];
      w.vo = int(hvo[t]);
      const int pa = hpar[t];
      w.uoff = pa < 0 ? 0 : (hc0[pa] == t ? 0 : tv) + int(hvo[pa]);
      w.boff = hbo[t];
      w.mo = int(hmo[t] / 4096);
      return w;
    };
    std::vector<MFWork> wf, wb;
    wl_fwd_off.assign(ndepth + 1, 0);
    wl_bwd_off.assign(ndepth + 1, 0);
    ks_fwd.assign(ndepth, 1);
    ks_bwd.assign(ndepth, 1);
    auto blocks = [](int rows, int rb) { return (rows + rb - 1) / rb; };
    for (int dd = 0; dd < ndepth; ++dd) {
      int64_t nf1 = 0, nb1 = 0;
      for (int t = tree_off[dd]; t < tree_off[dd + 1]; ++t) {
        nf1 += blocks(h_S[t] + h_b[t], 4 * MF_R);
        nb1 += blocks(h_s[t], 4 * MF_R);
      }
      ks_fwd[dd] = nf1 < MF_SPLIT_WG ? MF_KS : 1;
      ks_bwd[dd] = nb1 < MF_SPLIT_WG ? MF_KS : 1;
      const int rbf = ks_fwd[dd] == 1 ? 4 * MF_R : MF_R;
      const int rbb = ks_bwd[dd] == 1 ? 4 * MF_R : MF_R;
      for (int t = tree_off[dd]; t < tree_off[dd + 1]; ++t) {
        for (int k = 0; k < blocks(h_S[t] + h_b[t], rbf); ++k) wf.push_back(work(t, k));
        for (int k = 0; k < blocks(h_s[t], rbb); ++k) wb.push_back(work(t, k));
      }
      wl_fwd_off[dd + 1] = int(wf.size());
      wl_bwd_off[dd + 1] = int(wb.size());
    }
    if (wf.empty()) wf.push_back(MFWork{});
    if (wb.empty()) wb.push_back(MFWork{});
    wl_fwd.alloc(wf.size());
    wl_bwd.alloc(wb.size());
    AMGF_HIP(hipMemcpyAsync(wl_fwd.p, wf.data(), wf.size() * sizeof(MFWork),
                            hipMemcpyHostToDevice, c.s));
    AMGF_HIP(hipMemcpyAsync(wl_bwd.p, wb.data(), wb.size() * sizeof(MFWork),
                            hipMemcpyHostToDevice, c.s));
    AMGF_HIP(hipStreamSynchronize(c.s));   // the host lists go out of scope
  }
  const int fl = d2h_scalar(c.flag.p, c.s);
  AMGF_REQUIRE(!(fl & 4), AMGF_EDEVICE, "multifrontal: inconsistent symbolic structure");
  AMGF_REQUIRE(!(fl & 1), AMGF_ENOTSPD, "multifrontal: non-positive pivot");
}

void MFSolver::solve(Ctx& c, const double* r, double* x) const {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mf_to_tree, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, tdof.p, r,
                     rt.p);
  solve_tree(c, rt.p, xt.p);
  hipLaunchKernelGGL(k_mf_from_tree, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, tdof.p,
                     xt.p, x);
  AMGF_LAUNCH_CHECK();
}

void MFSolver::solve_tree(Ctx& c, const double* r, double* x) const {
  if (n == 0) return;
  // forward by depth, deepest first; each front's update vector lands in its parent's slot
  for (int dd = ndepth - 1; dd >= 0; --dd) {
    const int nf = wl_fwd_off[dd + 1] - wl_fwd_off[dd];
    if (nf > 0)
      hipLaunchKernelGGL(ks_fwd[dd] != 1 ? k_mf_fwd<MF_KS> : k_mf_fwd<1>, dim3(nf), dim3(256),
                         0, c.s, wl_fwd.p + wl_fwd_off[dd], bs, tv, r, bnd_pos.p, M.p, us.p,
                         fv.p);
  }
  // backward by depth, root first
  for (int dd = 0; dd < ndepth; ++dd) {
    const int nb = wl_bwd_off[dd + 1] - wl_bwd_off[dd];
    if (nb > 0)
      hipLaunchKernelGGL(ks_bwd[dd] != 1 ? k_mf_bwd<MF_KS> : k_mf_bwd<1>, dim3(nb), dim3(256),
                         0, c.s, wl_bwd.p + wl_bwd_off[dd], bs, x, bnd_tp.p, MT.p, fv.p);
  }
  AMGF_LAUNCH_CHECK();
}

void MFSolver::tree_index(Ctx& c, const int* idx, int* out) const {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mf_index_to_tree, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, tdof.p,
                     idx, out);
  AMGF_LAUNCH_CHECK();
}

int64_t MFSolver::stored_doubles() const {
  return int64_t(M.n) + int64_t(MT.n);
}

}  // namespace amgf

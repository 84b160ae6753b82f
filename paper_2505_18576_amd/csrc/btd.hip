// Block-tridiagonal FP64 Cholesky solver for the filter matrix A_w and the coarsest
// level.
//
// Breadth-first level sets of the matrix graph give an ordering in which A is
// block-tridiagonal (a level only touches its neighbours); consecutive levels are
// merged into blocks of at least `target` unknowns.  The factorisation
//   F_k = E_k L_{k-1}^{-T},  L_k L_k^T = D_k - F_k F_k^T
// is done with dense tiled kernels.  For the solves it stores Linv_k = L_k^{-1},
// its transpose, G_k = Linv_k F_k and H_k = Linv_k^T F_{k+1}^T, so that
//   forward : c = blockdiag(Linv) r,  y_0 = c_0,  y_k = c_k - G_k y_{k-1}
//   backward: d = blockdiag(Linv^T) y, x_L = d_L, x_k = d_k - H_k x_{k+1}
// is two batched products plus one row-parallel GEMV per block boundary.
#include "btd.h"

#include "dense.h"

namespace amgf {

// ---------------------------------------------------------------- BFS level sets
__global__ void k_bfs_step(int n, const int* __restrict__ rp, const int* __restrict__ col,
                           int* __restrict__ level, int cur, int* __restrict__ added) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || level[i] != cur) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = col[k];
    if (level[j] < 0) {
      level[j] = cur + 1;
      atomicAdd(added, 1);
    }
  }
}
__global__ void k_min_unvisited(int n, const int* __restrict__ level, int* __restrict__ mn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && level[i] < 0) atomicMin(mn, i);
}
__global__ void k_set_level(int* level, int i, int v) { level[i] = v; }
__global__ void k_level_hist(int n, const int* __restrict__ level, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[level[i]], 1);
}
__global__ void k_map_int(int n, const int* __restrict__ in, const int* __restrict__ map,
                          int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = map[in[i]];
}
__global__ void k_inverse_perm(int n, const int* __restrict__ perm, int* __restrict__ pos) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) pos[perm[p]] = p;
}

// ---------------------------------------------------------------- block extraction
// D_b[li][lj] for same-block entries, E_b[li][lj] for entries in the previous block.
__global__ void k_extract_blocks(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                 const double* __restrict__ val, const int* __restrict__ pos,
                                 const int* __restrict__ blk, const int* __restrict__ boff,
                                 const int64_t* __restrict__ doff,
                                 const int64_t* __restrict__ eoff, double* __restrict__ Db,
                                 double* __restrict__ Eb, int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int bi = blk[i], li = pos[i] - boff[bi], si = boff[bi + 1] - boff[bi];
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = col[k], bj = blk[j], lj = pos[j] - boff[bj];
    if (bj == bi) {
      Db[doff[bi] + int64_t(li) * si + lj] = val[k];
    } else if (bj == bi - 1) {
      const int sj = boff[bj + 1] - boff[bj];
      Eb[eoff[bi] + int64_t(li) * sj + lj] = val[k];
    } else if (bj != bi + 1) {
      atomicOr(flag, 1);
    }
  }
}

// ---------------------------------------------------------------- dense transpose
__global__ void k_transpose(int rows, int cols, const double* __restrict__ A,
                            double* __restrict__ T) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int y = threadIdx.y; y < 32; y += 8) {
    const int r = by + y, cidx = bx + threadIdx.x;
    if (r < rows && cidx < cols) tile[y][threadIdx.x] = A[int64_t(r) * cols + cidx];
  }
  __syncthreads();
  for (int y = threadIdx.y; y < 32; y += 8) {
    const int r = bx + y, cidx = by + threadIdx.x;   // T is cols x rows
    if (r < cols && cidx < rows) T[int64_t(r) * rows + cidx] = tile[threadIdx.x][y];
  }
}
static void transpose(Ctx& c, int rows, int cols, const double* A, double* T) {
  if (rows == 0 || cols == 0) return;
  hipLaunchKernelGGL(k_transpose, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(32, 8), 0, c.s,
                     rows, cols, A, T);
  AMGF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- solve kernels
// y[r] = sum_j M_b[li][j] x_b[j] over a triangle (lower: j <= li, upper: j >= li);
// one wavefront per row.
__global__ void k_blockdiag_gemv(int n, int upper, const int* __restrict__ rowblk,
                                 const int* __restrict__ boff, const int64_t* __restrict__ moff,
                                 const double* __restrict__ M, const double* __restrict__ x,
                                 double* __restrict__ y) {
  const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  const int b = rowblk[r], o = boff[b], s = boff[b + 1] - o, li = r - o;
  const double* row = M + moff[b] + int64_t(li) * s;
  const int j0 = upper ? li : 0, j1 = upper ? s : li + 1;
  double acc = 0.0;
  for (int j = j0 + lane; j < j1; j += 64) acc += row[j] * x[o + j];
  acc = wave_sum(acc);
  if (lane == 0) y[r] = acc;
}
// y[i] = c[i] - sum_j G[i][j] z[j], G is rows x cols (row-major); one 256-thread
// workgroup per row (four wavefronts split the columns) for memory parallelism
__global__ void __launch_bounds__(256) k_gemv_sub(int rows, int cols, const double* __restrict__ G,
                                                  const double* __restrict__ z,
                                                  const double* __restrict__ cvec,
                                                  double* __restrict__ y) {
  __shared__ double part[4];
  const int r = blockIdx.x;
  if (r >= rows) return;
  const double* row = G + int64_t(r) * cols;
  double acc = 0.0;
  for (int j = threadIdx.x; j < cols; j += 256) acc += row[j] * z[j];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) y[r] = cvec[r] - ((part[0] + part[1]) + (part[2] + part[3]));
}
__global__ void k_gather_perm(int n, const int* __restrict__ perm, const double* __restrict__ x,
                              double* __restrict__ y) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) y[p] = x[perm[p]];
}
__global__ void k_scatter_perm(int n, const int* __restrict__ perm, const double* __restrict__ x,
                               double* __restrict__ y) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) y[perm[p]] = x[p];
}

// ---------------------------------------------------------------- setup
void BTDSolver::setup(Ctx& c, int n_, const int* rp, const int* col, const double* val,
                      int target) {
  n = n_;
  if (n == 0) return;
  // 1. BFS level sets (component by component, smallest unvisited index first)
  DBuf<int> level(n), added(1), mn(1);
  AMGF_HIP(hipMemsetAsync(level.p, 0xff, level.bytes(), c.s));
  int cur = 0, start = 0;
  hipLaunchKernelGGL(k_set_level, dim3(1), dim3(1), 0, c.s, level.p, start, 0);
  for (;;) {
    AMGF_HIP(hipMemsetAsync(added.p, 0, sizeof(int), c.s));
    hipLaunchKernelGGL(k_bfs_step, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, rp, col, level.p,
                       cur, added.p);
    AMGF_LAUNCH_CHECK();
    if (d2h_scalar(added.p, c.s) > 0) {
      ++cur;
      continue;
    }
    const int big = 0x7fffffff;
    AMGF_HIP(hipMemcpyAsync(mn.p, &big, sizeof(int), hipMemcpyHostToDevice, c.s));
    hipLaunchKernelGGL(k_min_unvisited, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, level.p,
                       mn.p);
    const int m = d2h_scalar(mn.p, c.s);
    if (m == big) break;
    ++cur;
    hipLaunchKernelGGL(k_set_level, dim3(1), dim3(1), 0, c.s, level.p, m, cur);
  }
  const int nlev = cur + 1;
  DBuf<int> hist(nlev);
  AMGF_HIP(hipMemsetAsync(hist.p, 0, hist.bytes(), c.s));
  hipLaunchKernelGGL(k_level_hist, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, level.p, hist.p);
  std::vector<int> h = d2h(hist.p, nlev, c.s);
  // 2. merge consecutive levels into blocks of >= target unknowns
  std::vector<int> lev2blk(nlev);
  hoff.assign(1, 0);
  int acc = 0;
  for (int l = 0; l < nlev; ++l) {
    lev2blk[l] = int(hoff.size()) - 1;
    acc += h[l];
    if (acc >= target || l == nlev - 1) {
      hoff.push_back(hoff.back() + acc);
      acc = 0;
    }
  }
  nb = int(hoff.size()) - 1;
  DBuf<int> l2b(nlev), blk(n);
  AMGF_HIP(hipMemcpyAsync(l2b.p, lev2blk.data(), sizeof(int) * nlev, hipMemcpyHostToDevice, c.s));
  hipLaunchKernelGGL(k_map_int, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, level.p, l2b.p,
                     blk.p);
  // 3. ordering: by block, ascending index inside a block
  DBuf<int> boffd;
  group_by_key(c, blk.p, n, nb, boffd, perm);
  DBuf<int> pos(n);
  hipLaunchKernelGGL(k_inverse_perm, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, perm.p, pos.p);
  rowblk.alloc(n);
  {
    std::vector<int> rb(n);
    for (int b = 0; b < nb; ++b)
      for (int r = hoff[b]; r < hoff[b + 1]; ++r) rb[r] = b;
    AMGF_HIP(hipMemcpyAsync(rowblk.p, rb.data(), sizeof(int) * n, hipMemcpyHostToDevice, c.s));
  }
  boff.alloc(nb + 1);
  AMGF_HIP(hipMemcpyAsync(boff.p, hoff.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice,
                          c.s));
  // 4. offsets of the dense pieces
  std::vector<int64_t> dof(nb + 1, 0), eo(nb + 1, 0), go(nb + 1, 0), ho(nb + 1, 0);
  for (int b = 0; b < nb; ++b) {
    const int64_t s = hoff[b + 1] - hoff[b];
    const int64_t sp = b > 0 ? hoff[b] - hoff[b - 1] : 0;
    const int64_t sn = b + 1 < nb ? hoff[b + 2] - hoff[b + 1] : 0;
    dof[b + 1] = dof[b] + s * s;
    eo[b + 1] = eo[b] + s * sp;
    go[b + 1] = go[b] + s * sp;
    ho[b + 1] = ho[b] + s * sn;
  }
  hmoff = dof;
  hgoff = go;
  hhoff = ho;
  moff.alloc(nb + 1);
  AMGF_HIP(hipMemcpyAsync(moff.p, dof.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice,
                          c.s));
  DBuf<int64_t> eoffd(nb + 1);
  AMGF_HIP(hipMemcpyAsync(eoffd.p, eo.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice,
                          c.s));
  // 5. extract D_b and E_b
  DBuf<double> Db(std::max<int64_t>(dof[nb], 1)), Eb(std::max<int64_t>(eo[nb], 1));
  AMGF_HIP(hipMemsetAsync(Db.p, 0, Db.bytes(), c.s));
  AMGF_HIP(hipMemsetAsync(Eb.p, 0, Eb.bytes(), c.s));
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  hipLaunchKernelGGL(k_extract_blocks, dim3(grid_for(n, 128)), dim3(128), 0, c.s, n, rp, col, val,
                     pos.p, blk.p, boff.p, moff.p, eoffd.p, Db.p, Eb.p, c.flag.p);
  AMGF_LAUNCH_CHECK();
  AMGF_REQUIRE(d2h_scalar(c.flag.p, c.s) == 0, AMGF_EDEVICE,
               "level-set ordering is not block-tridiagonal");
  // 6. factorisation
  Linv.alloc(std::max<int64_t>(dof[nb], 1));
  LinvT.alloc(std::max<int64_t>(dof[nb], 1));
  G.alloc(std::max<int64_t>(go[nb], 1));
  H.alloc(std::max<int64_t>(ho[nb], 1));
  int smax = 0;
  for (int b = 0; b < nb; ++b) smax = std::max(smax, hoff[b + 1] - hoff[b]);
  DBuf<double> F(size_t(smax) * smax), T(size_t(smax) * smax);
  for (int b = 0; b < nb; ++b) {
    const int s = hoff[b + 1] - hoff[b];
    double* D = Db.p + dof[b];
    if (b > 0) {
      const int sp = hoff[b] - hoff[b - 1];
      const double* Lp = Linv.p + dof[b - 1];
      // F = E_b Linv_{b-1}^T   (s x sp)
      dgemm(c, true, s, sp, sp, 1.0, Eb.p + eo[b], sp, Lp, sp, 0.0, F.p, sp, false);
      // D -= F F^T (lower part is what the factorisation reads)
      dgemm(c, true, s, s, sp, -1.0, F.p, sp, F.p, sp, 1.0, D, s, true);
      // H_{b-1} = Linv_{b-1}^T F^T = (F Linv_{b-1})^T   (sp x s)
      dgemm(c, false, s, sp, sp, 1.0, F.p, sp, Lp, sp, 0.0, T.p, sp, false);
      transpose(c, s, sp, T.p, H.p + ho[b - 1]);
    }
    DBuf<double> Li;
    dense_cholesky_inverse(c, D, s, Li);
    AMGF_HIP(hipMemcpyAsync(Linv.p + dof[b], Li.p, sizeof(double) * size_t(s) * s,
                            hipMemcpyDeviceToDevice, c.s));
    transpose(c, s, s, Li.p, LinvT.p + dof[b]);
    if (b > 0) {
      const int sp = hoff[b] - hoff[b - 1];
      // G_b = Linv_b F   (s x sp)
      dgemm(c, false, s, sp, s, 1.0, Li.p, s, F.p, sp, 0.0, G.p + go[b], sp, false);
    }
  }
  work.alloc(size_t(n) * 3);
  AMGF_HIP(hipStreamSynchronize(c.s));
}

void BTDSolver::solve(Ctx& c, const double* r, double* x) const {
  if (n == 0) return;
  double* rp_ = work.p;          // permuted rhs, later y
  double* cv = work.p + n;       // c, later d
  double* yv = work.p + 2 * int64_t(n);
  const dim3 gw(grid_for(int64_t(n), 4)), bw(256);
  hipLaunchKernelGGL(k_gather_perm, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, perm.p, r, rp_);
  hipLaunchKernelGGL(k_blockdiag_gemv, gw, bw, 0, c.s, n, 0, rowblk.p, boff.p, moff.p, Linv.p,
                     rp_, cv);
  // forward: y_0 = c_0, y_b = c_b - G_b y_{b-1}
  AMGF_HIP(hipMemcpyAsync(yv, cv, sizeof(double) * (hoff[1] - hoff[0]), hipMemcpyDeviceToDevice,
                          c.s));
  for (int b = 1; b < nb; ++b) {
    const int s = hoff[b + 1] - hoff[b], sp = hoff[b] - hoff[b - 1];
    hipLaunchKernelGGL(k_gemv_sub, dim3(s), bw, 0, c.s, s, sp, G.p + hgoff[b],
                       yv + hoff[b - 1], cv + hoff[b], yv + hoff[b]);
  }
  // d = blockdiag(Linv^T) y
  hipLaunchKernelGGL(k_blockdiag_gemv, gw, bw, 0, c.s, n, 1, rowblk.p, boff.p, moff.p, LinvT.p,
                     yv, cv);
  // backward: x_last = d_last, x_b = d_b - H_b x_{b+1}
  double* xv = rp_;
  const int sl = hoff[nb] - hoff[nb - 1];
  AMGF_HIP(hipMemcpyAsync(xv + hoff[nb - 1], cv + hoff[nb - 1], sizeof(double) * sl,
                          hipMemcpyDeviceToDevice, c.s));
  for (int b = nb - 2; b >= 0; --b) {
    const int s = hoff[b + 1] - hoff[b], sn = hoff[b + 2] - hoff[b + 1];
    hipLaunchKernelGGL(k_gemv_sub, dim3(s), bw, 0, c.s, s, sn, H.p + hhoff[b],
                       xv + hoff[b + 1], cv + hoff[b], xv + hoff[b]);
  }
  hipLaunchKernelGGL(k_scatter_perm, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, perm.p, xv, x);
  AMGF_LAUNCH_CHECK();
}

int64_t BTDSolver::stored_doubles() const {
  return nb ? 2 * hmoff[nb] + hgoff[nb] + hhoff[nb] : 0;
}

}  // namespace amgf

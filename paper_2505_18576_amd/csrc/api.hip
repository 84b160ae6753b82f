// Host runtime and C ABI of the AMGF library: hierarchy setup, V-cycle, the AMGF
// preconditioner of Definition 5.3 and the preconditioned CG driver.
#include <chrono>
#include <cmath>
#include <memory>
#include <mutex>

#include "apply.h"
#include "multifrontal.h"
#include "csr.h"
#include "learn.h"
#include "setup.h"
#include "ip.h"
#include "coarse.h"

namespace amgf {

struct Level {
  int nn = 0, b = 0;            // block rows (nodes) and block size
  BSR A;                        // assembled operator (kept for inspection)
  BSR K;                        // stiffness part (FP64 + FP32 copy in mixed mode)
  BSR J, JT;                    // contact Jacobian (m x nn, 1 x b) and transpose
  DBuf<int> crows;              // node rows with a contact term (nonempty J^T rows)
  int ncrows = 0;
  DBuf<int> ccrows;             // nonempty rows of C (levels >= 1)
  int nccrows = 0;
  bool contact_factored = false;  // V-cycle applies the contact term through J and D
  bool contact_in_A = false;    // contact term assembled into the smoothing matrix (A_l)
  BSR P, PT;                    // prolongator to the next level and its transpose
  BSR C;                        // contact term J^T D J of this level (interface rows only)
  Graph G;                      // aggregation graph
  DBuf<int> agg, root;
  DBuf<double> d, w;
  DBuf<float> w32;
  int n_agg = 0;
  double rho = 1.0, omega = 0.0;
  // learned smoother: features (6 x n) and damping theta
  DBuf<double> F, theta;
  // adjoint work vectors and the damping gradient
  DBuf<double> ay, ab, ax, ar, ax2, wbar;
  // V-cycle work vectors
  DBuf<double> vb, vx, vr, vxn;
  DBuf<float> fb, fx, fr, fxn;
  // repeated visits of this level (cycle_gamma > 1): the correction so far and the residual
  DBuf<double> vxw, vbw;
  DBuf<float> fxw, fbw;
  // Chebyshev / multi-sweep smoothing work vectors
  DBuf<double> vd, vt;
  DBuf<float> fd, ft;
  double lam = 1.0;             // unclipped power estimate of rho(D_l1^{-1} A)
  DBuf<unsigned char> dead;     // dead near-null columns of the aggregates (n_agg x 6)
  int64_t n() const { return int64_t(nn) * b; }
};

struct Handle {
  amgf_options opt{};
  Ctx ctx;
  int n_nodes = 0, m = 0;
  std::vector<std::unique_ptr<Level>> lev;
  DBuf<double> D, coords;
  DBuf<double> kdiag0;          // diagonal entries of the input K (bound terms present)
  bool has_E = false;           // K_0 = K + diag(E) with bound-constraint barrier terms
  DBuf<unsigned char> dec0;
  DBuf<double> t;               // contact scratch (m)
  // coarsest solve: explicit inverse when small (one matrix-vector product per solve),
  // multifrontal Cholesky otherwise
  int nc_dense = 0;
  bool coarse_inverse = false;
  DenseInverse coarse_inv;
  MFSolver coarse;
  DBuf<double> coarse_b, coarse_x;
  // filter
  int n_c = 0;
  DBuf<int> Ic;
  MFSolver aw;
  DBuf<int> Ic_t;               // I_c in the factor's tree order: Ic_t[q] = Ic[aw.tdof[q]]
  DBuf<uint32_t> ic_mask;       // one bit per DOF, set on I_c
  DBuf<double> f_r, f_w;
  DBuf<int> aw_rp, aw_col;      // A_w = S[I_c, I_c] as scalar CSR (input of its factor)
  DBuf<double> aw_val;
  // apply scratch
  DBuf<double> z1, ra, r2, z3;
  DBuf<float> zf, r2f;
  DBuf<int> ic_nodes;           // node rows holding filter DOFs
  int n_icn = 0;
  bool ic_from_J = false;       // I_c = all DOFs of the nodes J touches (not a caller's list)
  bool r_cast_ready = false;    // level-0 fb = float(r), fx = w.fb already formed for the
                                // next mixed V-cycle on r (set by the CG update, used once)
  bool ic_closed = false;
  // pcg scratch
  DBuf<double> pr, pz, pzo, pp, pq;
  DBuf<double> pcg_s;           // device scalars of one CG iteration: p.q, r.z, r.z_old
  double op_complexity = 1.0;
  DBuf<float> mlpW;             // device copy of the MLP parameters (learned smoother)
  bool learned = false;         // the MLP damping is applied
  // judge of the learned damping (AMGF_LEARNED with learned_judge): one AMGF step from a
  // fixed start with each damping at every setup / update; the better one is kept
  bool judge_on = false;
  bool judge_rejected = false;  // the last judge kept theta = 1
  double judge_l = 0.0, judge_p = 0.0;
  double ms_setup_amg = 0.0, ms_setup_filter = 0.0;   // host wall times of the last setup
  // live timing of one level-0 kernel class inside solves: event pairs on the solve stream
  int prof_which = -1;
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used = 0;
  bool prof_open = false;
  AllocSrc mem;                 // the caller's allocator and the stream of the running call
  // plain AMG-PCG on a filter handle (the switching interior-point driver); the filter
  // factor is not refreshed while suspended
  bool filter_suspended = false;
  DBuf<double> ip_red;          // device results of the driver's reductions
  // phase timing of the running CG solve: event i opens a segment of phase ph_cat[i]
  // (V-cycles, filter correction, other CG work) on the solve stream
  std::vector<hipEvent_t> ph_ev;
  std::vector<int> ph_cat;
  size_t ph_used = 0;
  bool ph_on = false;
  // CG coefficients of the last solve: alpha_k = r.z / p.Ap and beta_k = r'.z' / r.z
  // (the Lanczos tridiagonal of M A, Sec. 6.1)
  std::vector<double> cg_alpha, cg_beta;
  Handle() = default;
  Handle(const Handle&) = delete;
  ~Handle() {
    for (hipEvent_t e : prof_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : ph_ev) (void)hipEventDestroy(e);
  }
  bool mixed() const { return opt.precision != AMGF_FP64; }
  bool bf16k() const { return opt.precision == AMGF_MIXED_BF16K; }
  // one fused l1-Jacobi step before and after the coarse correction
  bool plain_cycle() const { return opt.smoother != AMGF_CHEBYSHEV && opt.sweeps == 1; }
  int64_t n() const { return int64_t(n_nodes) * 3; }
  // the stream of the running entry point: kernels are queued on it, and buffers allocated
  // during the call come from the handle's allocator with it
  void bind(void* stream) {
    ctx.s = static_cast<hipStream_t>(stream);
    mem.s = ctx.s;
  }
};

static thread_local std::string g_last_error;

// ------------------------------------------------------------------------------------
// device scratch of the allocation-free CG entry point (amgf_pcg_noalloc): the partial
// sums of the deterministic dot products and the CG scalars p.q, r.z, r.z_old.  Its size
// does not depend on the problem.  Each GPU holds its own copy until the process ends;
// host code uses the per-device address from hipGetSymbolAddress, never the array's name.
// ------------------------------------------------------------------------------------
constexpr size_t PCG_SCRATCH = DOT_SCRATCH + 4;
static __device__ __align__(256) double scratch[PCG_SCRATCH];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// the scratch address on the current device, looked up once per device (called by
// amgf_setup on its device, then by the entry point)
static double* scratch_ptr() {
  int dev = 0;
  AMGF_HIP(hipGetDevice(&dev));
  AMGF_REQUIRE(dev >= 0 && dev < SCRATCH_MAX_DEVICES, AMGF_EDEVICE, "device index");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    AMGF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    AMGF_REQUIRE(p != nullptr, AMGF_EDEVICE, "hipGetSymbolAddress returned no address");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

// ------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------
static void copy_in(Ctx& c, void* dst, const void* src, size_t bytes) {
  if (bytes) AMGF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c.s));
}

static double power_estimate(Handle& h, Level& L, const unsigned char* dec) {
  Ctx& c = h.ctx;
  const int64_t n = L.n();
  DBuf<double> x(n), y(n);
  fill_power_start(c, n, x.p, dec);
  const double* xs[1] = {x.p};
  double nrm;
  dots(c, n, 1, xs, xs, &nrm);
  vscale(c, n, 1.0 / std::sqrt(nrm), x.p);
  // the norms stay on the device between steps (x = y / |y| there); the host reads the
  // last one.  A zero y makes every later step 0/0, so the last norm tells.
  DBuf<double> s(1);
  const bool fine = &L == h.lev[0].get();
  const int iters = h.opt.sa_power_iters;
  for (int it = 0; it < iters; ++it) {
    if (fine) {
      // level 0: sliced stiffness plus the contact term through J (same operator as A)
      bsr_spmv<double>(c, SPMV_Y, L.K, L.K.val.p, x.p, y.p, nullptr, nullptr, nullptr);
      contact_apply<double, double>(c, CT_ADD, L.J, L.JT, L.crows.p, L.ncrows, h.D.p, x.p,
                                    h.t.p, y.p, nullptr);
    } else {
      bsr_spmv<double>(c, SPMV_Y, L.A, L.A.val.p, x.p, y.p, nullptr, nullptr, nullptr);
    }
    scale_div_zero(c, n, y.p, L.d.p, dec);
    const double* ys[1] = {y.p};
    dots_device(c, n, 1, ys, ys, s.p);
    if (it + 1 < iters) normalize_dev(c, n, s.p, y.p, x.p);
  }
  if (iters < 1) return 1.0;
  const double lam = std::sqrt(d2h_scalar(s.p, c.s));
  return lam > 0.0 ? lam : 1.0;
}

// FP16 values of a transfer operator (FP32 when a value would overflow FP16)
static void to_fp16_or_fp32(Ctx& c, BSR& A) {
  const int64_t nv = std::max<int64_t>(A.nnzb, 1) * A.bsz();
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  cast_d2h_transfer(c, A, c.flag.p);
  if (d2h_scalar(c.flag.p, c.s) == 0) return;
  A.valh = DBuf<_Float16>();
  A.val32.alloc(nv);
  cast_d2f(c, A.val.p, A.val32.p, nv);
}

static void smoothing_copies(Handle& h, Level& L);

static void to_fp32(Ctx& c, BSR& A) {
  const int64_t nv = std::max<int64_t>(A.nnzb, 1) * A.bsz();
  A.val32.alloc(nv);
  cast_d2f(c, A.val.p, A.val32.p, nv);
}

// ------------------------------------------------------------------------------------
// setup pieces shared with the numeric re-setup of a new barrier diagonal
// ------------------------------------------------------------------------------------
// The contact term of a coarse level inside the V-cycle: through J_l and D (two kernels,
// t = D (J_l x), then J_l^T t) when that reads fewer bytes than the assembled Galerkin
// block C_l, otherwise through C_l (one wavefront per row).  C_l couples every pair of
// coarse nodes that share a constraint, so it holds b^2 values per coupling where J_l holds
// b per constraint and node.
static bool factored_contact_pays(Ctx&, const Level& L) {
  if (L.J.nnzb == 0 || L.ncrows == 0) return false;
  const int64_t b = L.b;
  const int64_t factored = 2 * L.J.nnzb * (8 * b + 4) + 2 * int64_t(L.J.nrows) * 8;
  const int64_t assembled = L.C.nnzb * (8 * b * b + 4);
  return factored < assembled;
}

// direct factor of the coarsest operator
constexpr int64_t COARSE_INVERSE_MAX = 2048;   // unknowns; 32 MiB of FP64 at most

static void factor_coarsest(Handle& h) {
  Level& LL = *h.lev.back();
  h.coarse_inverse = LL.n() <= COARSE_INVERSE_MAX && h.coarse_inv.setup(h.ctx, LL.A);
  if (h.coarse_inverse) return;
  h.coarse_inv = DenseInverse();
  DBuf<int> rp, cl;
  DBuf<double> vl;
  bsr_to_csr(h.ctx, LL.A, rp, cl, vl);
  h.coarse.setup(h.ctx, int(LL.n()), LL.b, rp.p, cl.p, vl.p);
}

// A_w = S[I_c, I_c] and its factor
static void factor_filter(Handle& h) {
  Level& L0 = *h.lev[0];
  filter_csr(h.ctx, L0.A, h.Ic.p, h.n_c, h.aw_rp, h.aw_col, h.aw_val);
  h.aw.setup(h.ctx, h.n_c, h.ic_closed ? 3 : 1, h.aw_rp.p, h.aw_col.p, h.aw_val.p);
  if (h.Ic_t.n != size_t(h.n_c)) h.Ic_t.alloc(size_t(h.n_c));
  h.aw.tree_index(h.ctx, h.Ic.p, h.Ic_t.p);
}

// features of every smoothed level and, with learned damping, w = theta/d from the MLP
static void features_and_damping(Handle& h) {
  Ctx& c = h.ctx;
  const int nlev = int(h.lev.size());
  for (int l = 0; l + 1 < nlev; ++l) {
    Level& L = *h.lev[l];
    L.F.alloc(size_t(6) * L.n());
    L.theta.alloc(L.n());
    level_features(c, L.b, L.nn, L.A.rowptr.p, L.A.col.p, L.A.val.p, L.d.p, L.JT.rowptr.p,
                   L.JT.col.p, L.JT.val.p, h.D.p, nlev > 1 ? double(l) / double(nlev - 1) : 0.0,
                   L.F.p);
    if (h.learned) mlp_theta(c, L.n(), h.mlpW.p, L.F.p, L.d.p, L.theta.p, L.w.p);
  }
}

static void judge_damping(Handle& h);


// ------------------------------------------------------------------------------------
// setup
// ------------------------------------------------------------------------------------
static void setup(Handle& h, const int32_t* K_rowptr, const int32_t* K_col, const double* K_val,
                  const int32_t* J_rowptr, const int32_t* J_col, const double* J_val,
                  const double* D, const double* coords, const int32_t* Ic_user, int n_c_user) {
  Ctx& c = h.ctx;
  const amgf_options& o = h.opt;
  const int nn = h.n_nodes, m = h.m;
  const auto t_start = std::chrono::steady_clock::now();
  // ---- input checks
  std::vector<int> rp_host = d2h(K_rowptr, 2, c.s);
  AMGF_REQUIRE(rp_host[0] == 0, AMGF_EINVAL, "K_rowptr[0] must be 0");
  const int nnzb = d2h_scalar(K_rowptr + nn, c.s);
  AMGF_REQUIRE(nnzb >= nn, AMGF_EINVAL, "K needs a diagonal block per row");
  int nnzJ = 0;
  if (m > 0) nnzJ = d2h_scalar(J_rowptr + m, c.s);
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  check_values(c, K_val, int64_t(nnzb) * 9, false, c.flag.p);
  if (m > 0) {
    check_values(c, J_val, nnzJ, false, c.flag.p);
    check_values(c, D, m, true, c.flag.p);
  }
  if (coords) check_values(c, coords, int64_t(nn) * 3, false, c.flag.p);
  if (o.bound_diag) check_nonnegative(c, o.bound_diag, int64_t(nn) * 3, c.flag.p);
  const int fl = d2h_scalar(c.flag.p, c.s);
  AMGF_REQUIRE(fl == 0, AMGF_EINVAL,
               (fl & 2) ? "D must be positive and E non-negative"
                        : "non-finite value in K, J, D, E or coords");

  // ---- level 0 inputs
  h.lev.emplace_back(new Level());
  Level* L0 = h.lev.back().get();
  L0->nn = nn;
  L0->b = 3;
  BSR& K = L0->K;
  K.nrows = K.ncols = nn;
  K.br = K.bc = 3;
  K.nnzb = nnzb;
  K.rowptr.alloc(size_t(nn) + 1);
  K.col.alloc(std::max(nnzb, 1));
  K.val.alloc(size_t(std::max(nnzb, 1)) * 9);
  copy_in(c, K.rowptr.p, K_rowptr, sizeof(int) * (size_t(nn) + 1));
  copy_in(c, K.col.p, K_col, sizeof(int) * size_t(nnzb));
  copy_in(c, K.val.p, K_val, sizeof(double) * size_t(nnzb) * 9);
  if (o.bound_diag) {           // Remark 3.1: K_0 = K + diag(E)
    bound_diagonal(c, K, o.bound_diag, h.kdiag0);
    h.has_E = true;
  }
  h.D.alloc(std::max(m, 1));
  copy_in(c, h.D.p, D, sizeof(double) * size_t(m));
  if (coords) {                 // rigid-body modes (near_null = 6) need the node positions
    h.coords.alloc(size_t(nn) * 3);
    copy_in(c, h.coords.p, coords, sizeof(double) * size_t(nn) * 3);
  }
  h.t.alloc(std::max(m, 1));
  bsr_build_sell(c, K, true, h.mixed(), h.bf16k());     // apply copies of K (level 0)
  j_to_node_blocks(c, m, nn, J_rowptr, J_col, J_val, L0->J);
  bsr_transpose(c, L0->J, L0->JT);
  L0->ncrows = nonempty_rows(c, L0->JT.rowptr.p, nn, L0->crows);
  contact_operator(c, L0->J, L0->JT, h.D.p, L0->C);
  bsr_add(c, K, L0->C, L0->A);
  // ---- levels
  DBuf<double> Rprev;
  Graph Gnext;
  int64_t nz0 = L0->A.nnzb * 9, nzsum = nz0;
  for (int l = 0; l < o.max_levels; ++l) {
    Level& L = *h.lev[l];
    l1_norms(c, L.A, L.d);
    L.w.alloc(L.n());
    weights_from_l1(c, L.n(), L.d.p, nullptr, L.w.p);
    if (L.nn <= o.coarse_max_nodes || l == o.max_levels - 1) break;
    if (l == 0) strength_graph(c, L.A, o.strength_theta, L.G);
    else L.G = std::move(Gnext);
    int rounds = 0;
    const int n_agg = mis2_aggregate(c, L.G, l, L.agg, L.root, &rounds);
    if (n_agg == 0 || n_agg > o.max_coarse_ratio * L.nn) break;
    L.n_agg = n_agg;
    DBuf<int> moff, members;
    group_by_key(c, L.agg.p, L.nn, n_agg, moff, members);
    const unsigned char* dec = nullptr;
    if (l == 0) {
      decoupled_dofs(c, L.A, h.dec0);
      dec = h.dec0.p;
    }
    DBuf<double> Pt, R;
    DBuf<unsigned char> dead;
    tentative_prolongator(c, L.b, h.opt.near_null, L.nn, n_agg, moff.p, members.p, l == 0,
                          l == 0 ? h.coords.p : nullptr,
                          dec, Rprev.p, o.qr_tol, Pt, R, dead);
    L.lam = power_estimate(h, L, dec);
    L.rho = std::min(1.0, L.lam);
    L.omega = o.sa_omega / L.rho;
    smooth_prolongator(c, L.A, L.agg.p, n_agg, h.opt.near_null, Pt.p, L.d.p, L.omega, L.P);
    bsr_transpose(c, L.P, L.PT);
    h.lev.emplace_back(new Level());
    Level& N = *h.lev.back();
    Level& Lc = *h.lev[l];  // re-fetch (vector may have reallocated)
    N.nn = n_agg;
    N.b = h.opt.near_null;
    {
      BSR KP;
      spgemm(c, Lc.K, Lc.P, KP);
      spgemm(c, Lc.PT, KP, N.K);
    }
    dead_identity(c, N.K, dead.p);
    Lc.dead = std::move(dead);
    spgemm(c, Lc.J, Lc.P, N.J);
    bsr_transpose(c, N.J, N.JT);
    N.ncrows = nonempty_rows(c, N.JT.rowptr.p, N.nn, N.crows);
    {
      // C_{l+1} = P^T C_l P (= J_{l+1}^T D J_{l+1}), local to the interface rows
      BSR CP;
      spgemm(c, Lc.C, Lc.P, CP);
      spgemm(c, Lc.PT, CP, N.C);
      bsr_add(c, N.K, N.C, N.A);
      N.nccrows = nonempty_rows(c, N.C.rowptr.p, N.nn, N.ccrows);
    }
    N.contact_factored = factored_contact_pays(c, N);
    N.contact_in_A = !N.contact_factored && N.nccrows > 0;
    nzsum += N.A.nnzb * int64_t(N.A.bsz());
    coarse_graph(c, Lc.G, Lc.agg.p, n_agg, moff.p, members.p, Gnext);
    Rprev = std::move(R);
  }
  h.op_complexity = double(nzsum) / double(std::max<int64_t>(nz0, 1));
  // ---- coarsest level: direct multifrontal Cholesky
  Level& LL = *h.lev.back();
  h.nc_dense = int(LL.n());
  factor_coarsest(h);
  h.coarse_b.alloc(h.nc_dense);
  h.coarse_x.alloc(h.nc_dense);
  // ---- filter (Sec. 5.1): A_w = S[I_c, I_c], nested-dissection multifrontal Cholesky
  AMGF_HIP(hipStreamSynchronize(c.s));
  const auto t_filter = std::chrono::steady_clock::now();
  if (Ic_user && n_c_user > 0) {
    h.Ic.alloc(n_c_user);
    copy_in(c, h.Ic.p, Ic_user, sizeof(int) * size_t(n_c_user));
    h.n_c = n_c_user;
  } else {
    h.n_c = filter_space_from_J(c, L0->J, nn, h.Ic);
    h.ic_from_J = true;
  }
  if (h.n_c > 0) {
    std::vector<int> ic = d2h(h.Ic.p, h.n_c, c.s);
    std::vector<int> nodes;
    for (int i = 0; i < h.n_c; ++i) {
      AMGF_REQUIRE(ic[i] >= 0 && ic[i] < 3 * nn && (i == 0 || ic[i] > ic[i - 1]), AMGF_EINVAL,
                   "Ic must be ascending DOF indices in [0, n)");
      if (nodes.empty() || nodes.back() != ic[i] / 3) nodes.push_back(ic[i] / 3);
    }
    h.n_icn = int(nodes.size());
    // node-closed I_c (all three DOFs of each node, in order) lets the filter solver order
    // nodes instead of single DOFs
    h.ic_closed = h.n_c == 3 * h.n_icn;
    for (int i = 0; h.ic_closed && i < h.n_c; ++i)
      h.ic_closed = ic[i] == 3 * nodes[i / 3] + i % 3;
    h.ic_nodes.alloc(h.n_icn);
    AMGF_HIP(hipMemcpyAsync(h.ic_nodes.p, nodes.data(), sizeof(int) * h.n_icn,
                            hipMemcpyHostToDevice, c.s));
    bit_mask(c, h.Ic.p, h.n_c, 3 * int64_t(nn), h.ic_mask);
    AMGF_HIP(hipStreamSynchronize(c.s));
  }
  if (o.filter && h.n_c > 0) {
    factor_filter(h);
    h.f_r.alloc(h.n_c);
    h.f_w.alloc(h.n_c);
  }
  AMGF_HIP(hipStreamSynchronize(c.s));
  const auto t_filter_end = std::chrono::steady_clock::now();
  // ---- learned-smoother features of the smoothed levels
  if (o.smoother == AMGF_LEARNED) {
    h.mlpW.alloc(MLP_NTOTAL);
    AMGF_HIP(hipMemcpyAsync(h.mlpW.p, o.mlp_weights, sizeof(float) * MLP_NTOTAL,
                            hipMemcpyHostToDevice, c.s));
    h.learned = true;
    h.judge_on = o.learned_judge != 0;
  }
  features_and_damping(h);
  // ---- precision copies and work vectors
  for (size_t l = 0; l < h.lev.size(); ++l) {
    Level& L = *h.lev[l];
    const int64_t n = L.n();
    L.vb.alloc(n); L.vx.alloc(n); L.vr.alloc(n); L.vxn.alloc(n);
    if (h.opt.cycle_gamma > 1 && l != 0 && l + 1 < h.lev.size()) {
      L.vxw.alloc(n);
      L.vbw.alloc(n);
      if (h.mixed()) { L.fxw.alloc(n); L.fbw.alloc(n); }
    }
    if (!h.plain_cycle()) {
      L.vd.alloc(n);
      L.vt.alloc(n);
      if (h.mixed()) { L.fd.alloc(n); L.ft.alloc(n); }
    }
    // packed copies of the smoothing matrices of the coarse levels (1 .. L-2)
    if (l != 0 && l + 1 < h.lev.size()) smoothing_copies(h, L);
    if (h.mixed()) {
      if (l != 0) to_fp32(c, L.K);
      if (L.P.nnzb) {
        if (h.opt.transfer_fp16) {
          to_fp16_or_fp32(c, L.P);
          to_fp16_or_fp32(c, L.PT);
        } else {
          to_fp32(c, L.P);
          to_fp32(c, L.PT);
        }
      }
      L.w32.alloc(n);
      cast_d2f(c, L.w.p, L.w32.p, n);
      L.fb.alloc(n); L.fx.alloc(n); L.fr.alloc(n); L.fxn.alloc(n);
    }
  }
  const int64_t n = h.n();
  h.z1.alloc(n); h.ra.alloc(n); h.r2.alloc(n); h.z3.alloc(n);
  if (h.mixed()) { h.zf.alloc(n); h.r2f.alloc(n); }
  h.pr.alloc(n); h.pz.alloc(n); h.pzo.alloc(n); h.pp.alloc(n); h.pq.alloc(n);
  judge_damping(h);
  AMGF_HIP(hipStreamSynchronize(c.s));
  const auto t_end = std::chrono::steady_clock::now();
  using ms = std::chrono::duration<double, std::milli>;
  h.ms_setup_filter = ms(t_filter_end - t_filter).count();
  h.ms_setup_amg = ms(t_filter - t_start).count() + ms(t_end - t_filter_end).count();
}

// ------------------------------------------------------------------------------------
// numeric re-setup for a new barrier diagonal (same K, J; aggregates and P kept)
// ------------------------------------------------------------------------------------
static void update_D(Handle& h, const double* D) {
  Ctx& c = h.ctx;
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  if (h.m > 0) check_values(c, D, h.m, true, c.flag.p);
  const int fl = d2h_scalar(c.flag.p, c.s);
  AMGF_REQUIRE(fl == 0, AMGF_EINVAL, (fl & 2) ? "D must be positive" : "non-finite value in D");
  copy_in(c, h.D.p, D, sizeof(double) * size_t(h.m));
  const auto t_start = std::chrono::steady_clock::now();
  const size_t nlev = h.lev.size();
  for (size_t l = 0; l < nlev; ++l) {
    Level& L = *h.lev[l];
    if (l == 0) {
      L.C = BSR();
      contact_operator(c, L.J, L.JT, h.D.p, L.C);
    } else {
      Level& U = *h.lev[l - 1];
      BSR CP;
      spgemm(c, U.C, U.P, CP);
      L.C = BSR();
      spgemm(c, U.PT, CP, L.C);
    }
    L.A = BSR();
    bsr_add(c, L.K, L.C, L.A);
    l1_norms(c, L.A, L.d);
    weights_from_l1(c, L.n(), L.d.p, nullptr, L.w.p);
    if (l + 1 < nlev) L.lam = power_estimate(h, L, l == 0 ? h.dec0.p : nullptr);
    // after the power estimate, which the fresh setup also runs on the plain BSR A_l
    if (l != 0 && L.contact_in_A && l + 1 < nlev) smoothing_copies(h, L);
  }
  factor_coarsest(h);
  AMGF_HIP(hipStreamSynchronize(c.s));
  const auto t_filter = std::chrono::steady_clock::now();
  if (h.opt.filter && h.n_c > 0 && !h.filter_suspended) factor_filter(h);
  AMGF_HIP(hipStreamSynchronize(c.s));
  const auto t_filter_end = std::chrono::steady_clock::now();
  if (h.judge_on) h.learned = true;                   // the judge decides afresh
  features_and_damping(h);
  if (h.mixed())
    for (size_t l = 0; l < nlev; ++l) {
      Level& L = *h.lev[l];
      cast_d2f(c, L.w.p, L.w32.p, L.n());
    }
  judge_damping(h);
  AMGF_HIP(hipStreamSynchronize(c.s));
  const auto t_end = std::chrono::steady_clock::now();
  using ms = std::chrono::duration<double, std::milli>;
  h.ms_setup_filter = ms(t_filter_end - t_filter).count();
  h.ms_setup_amg = ms(t_filter - t_start).count() + ms(t_end - t_filter_end).count();
}

// New barrier terms of both kinds (Remark 3.1): K_0 = K + diag(E) and the coarse stiffness
// chain are rebuilt with the kept prolongators, then the rest as for a new D.
static void update_barrier(Handle& h, const double* D, const double* E) {
  Ctx& c = h.ctx;
  Level& L0 = *h.lev[0];
  AMGF_HIP(hipMemsetAsync(c.flag.p, 0, sizeof(int), c.s));
  if (h.m > 0) check_values(c, D, h.m, true, c.flag.p);
  if (E) check_nonnegative(c, E, h.n(), c.flag.p);
  const int fl = d2h_scalar(c.flag.p, c.s);
  AMGF_REQUIRE(fl == 0, AMGF_EINVAL,
               (fl & 2) ? "D must be positive and E non-negative" : "non-finite value in D or E");
  if (E || h.has_E) {
    bound_diagonal(c, L0.K, E, h.kdiag0);
    h.has_E = E != nullptr;
    bsr_build_sell(c, L0.K, true, h.mixed(), h.bf16k());
    for (size_t l = 0; l + 1 < h.lev.size(); ++l) {
      Level& L = *h.lev[l];
      Level& N = *h.lev[l + 1];
      BSR KP;
      spgemm(c, L.K, L.P, KP);
      N.K = BSR();
      spgemm(c, L.PT, KP, N.K);
      dead_identity(c, N.K, L.dead.p);
      if (h.mixed()) to_fp32(c, N.K);
      if (l + 2 < h.lev.size() && !N.contact_in_A) smoothing_copies(h, N);
    }
  }
  update_D(h, D);
}

// ------------------------------------------------------------------------------------
// V-cycle
// ------------------------------------------------------------------------------------
static void coarse_solve(Handle& h, const double* b, double* x) {
  if (h.coarse_inverse) h.coarse_inv.solve(h.ctx, b, x);
  else h.coarse.solve(h.ctx, b, x);
}

// The matrix a level's smoother multiplies by: K_l, with the contact term added by
// level_contact, or A_l = K_l + C_l itself where the contact term is assembled into it
static const BSR& smooth_mat(const Level& L) { return L.contact_in_A ? L.A : L.K; }

// packed copy of a coarse level's smoothing matrix: FP32 values for the mixed V-cycle's K_l,
// FP64 otherwise; A_l = K_l + C_l keeps FP64 values in every mode, so the contact term stays
// FP64 (the FP32 cycle then accumulates its products in FP64)
static void smoothing_copies(Handle& h, Level& L) {
  BSR& S = L.contact_in_A ? L.A : L.K;
  const bool f32 = h.mixed() && !L.contact_in_A;
  bsr_build_packed(h.ctx, S, !f32, f32);
}

// Contact term of a level inside the V-cycle: through J and D on level 0 (the fine
// interface, where the assembled block would be larger than J) and on the coarse levels
// where that still reads fewer bytes (factored_contact_pays); on the other coarse levels
// the assembled Galerkin block C_l is part of the smoothing matrix A_l = K_l + C_l, or
// empty (no contact rows: nothing to add).
template <class T>
static void level_contact(Handle& h, Level& L, int mode, const T* x, T* y, const T* w) {
  if (L.contact_in_A) return;                         // inside the level's smoothing matrix
  if (&L == h.lev[0].get() || L.contact_factored)
    contact_apply<T, T>(h.ctx, mode, L.J, L.JT, L.crows.p, L.ncrows, h.D.p, x, h.t.p, y, w);
  else if (L.nccrows > 0)
    throw Error(AMGF_EDEVICE, "coarse contact term without a form");
}

// bracket the launches of kernel class `which` (level 0) when live timing is on
static void prof_begin(Handle& h, int which) {
  if (h.prof_which != which || h.prof_used + 2 > h.prof_ev.size()) return;
  AMGF_HIP(hipEventRecord(h.prof_ev[h.prof_used++], h.ctx.s));
  h.prof_open = true;
}
static void prof_end(Handle& h) {
  if (!h.prof_open) return;
  AMGF_HIP(hipEventRecord(h.prof_ev[h.prof_used++], h.ctx.s));
  h.prof_open = false;
}

// phase timing inside a CG solve: opens a segment of phase `ph` unless it is already open
enum { PH_AMG = 0, PH_FILTER = 1, PH_OTHER = 2 };
static void phase(Handle& h, int ph) {
  if (!h.ph_on) return;
  if (h.ph_used > 0 && h.ph_cat[h.ph_used - 1] == ph) return;
  if (h.ph_used == h.ph_ev.size()) {
    hipEvent_t e;
    AMGF_HIP(hipEventCreate(&e));
    h.ph_ev.push_back(e);
    h.ph_cat.push_back(ph);
  }
  h.ph_cat[h.ph_used] = ph;
  AMGF_HIP(hipEventRecord(h.ph_ev[h.ph_used++], h.ctx.s));
}

// ---- smoother options: nu applications of l1-Jacobi or of the degree-m Chebyshev
// polynomial in D_l1^{-1} A over [0.3 lam, lam], lam = min(1, 1.1 * power estimate)
template <class T>
struct LvBufs {
  DBuf<T>*b, *x, *xn, *r, *d, *t, *xw, *bw;
  const T* w;
};
static LvBufs<double> lv_bufs(Level& L, double) {
  return {&L.vb, &L.vx, &L.vxn, &L.vr, &L.vd, &L.vt, &L.vxw, &L.vbw, L.w.p};
}
static LvBufs<float> lv_bufs(Level& L, float) {
  return {&L.fb, &L.fx, &L.fxn, &L.fr, &L.fd, &L.ft, &L.fxw, &L.fbw, L.w32.p};
}
static void add_to(Ctx& c, int64_t n, const double* a, double* y) { axpby(c, n, 1.0, a, 1.0, y); }
static void add_to(Ctx& c, int64_t n, const float* a, float* y) { add_to_f32(c, n, a, y); }

static const double* bsr_vals(const BSR& A, double) { return A.val.p; }
static const float* bsr_vals(const BSR& A, float) { return A.val32.p; }

// restriction / prolongation in the V-cycle's precision (FP32: FP16 values when stored)
static void transfer(Handle& h, int mode, const BSR& A, const double* x, double* y) {
  bsr_spmv<double>(h.ctx, mode, A, A.val.p, x, y, nullptr, nullptr, nullptr);
}
static void transfer(Handle& h, int mode, const BSR& A, const float* x, float* y) {
  transfer_spmv(h.ctx, mode, A, x, y);
}

// K x in the level's V-cycle precision (BF16 level-0 values in MIXED_BF16K)
static void k_spmv(Handle& h, size_t l, int mode, const double* x, double* y, const double* b,
                   const double* w, double* xo) {
  const BSR& S = smooth_mat(*h.lev[l]);
  bsr_spmv<double>(h.ctx, mode, S, S.val.p, x, y, b, w, xo);
}
static void k_spmv(Handle& h, size_t l, int mode, const float* x, float* y, const float* b,
                   const float* w, float* xo) {
  Level& L = *h.lev[l];
  if (l == 0 && h.bf16k()) sell_spmv_bf16(h.ctx, mode, L.K, x, y, b, w, xo);
  else bsr_spmv<float>(h.ctx, mode, smooth_mat(L), smooth_mat(L).val32.p, x, y, b, w, xo);
}

template <class T>
static void contact(Handle& h, Level& L, int mode, const T* x, T* y, const T* w) {
  level_contact<T>(h, L, mode, x, y, w);
}

// one smoother application on x (x_zero: x = 0 on entry); result in *B.x
template <class T>
static void smooth_once(Handle& h, size_t l, bool x_zero) {
  Ctx& c = h.ctx;
  Level& L = *h.lev[l];
  LvBufs<T> B = lv_bufs(L, T());
  const int64_t n = L.n();
  if (h.opt.smoother != AMGF_CHEBYSHEV) {
    if (x_zero) {
      // x = w.b (the residual written to r is not needed here)
      k_spmv(h, l, SPMV_PRE, (const T*)nullptr, B.r->p, B.b->p, B.w, B.x->p);
      return;
    }
    k_spmv(h, l, SPMV_POST, B.x->p, (T*)nullptr, B.b->p, B.w, B.xn->p);
    contact<T>(h, L, CT_SUB_W, B.x->p, B.xn->p, B.w);
    std::swap(*B.x, *B.xn);
    return;
  }
  const double lmax = std::min(1.0, 1.1 * L.lam), lmin = 0.3 * lmax;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  const T* src = B.b->p;
  if (!x_zero) {
    k_spmv(h, l, SPMV_RES, B.x->p, B.r->p, B.b->p, (const T*)nullptr, (T*)nullptr);
    contact<T>(h, L, CT_SUB_RES, B.x->p, B.r->p, (const T*)nullptr);
    src = B.r->p;
  }
  cheb_start<T>(c, n, src, B.w, B.r->p, B.d->p, B.x->p, 1.0 / theta, x_zero);
  double rho = 1.0 / sigma;
  for (int k = 1; k < h.opt.cheb_degree; ++k) {
    k_spmv(h, l, SPMV_Y, B.d->p, B.t->p, (const T*)nullptr, (const T*)nullptr, (T*)nullptr);
    contact<T>(h, L, CT_ADD, B.d->p, B.t->p, (const T*)nullptr);
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    cheb_step<T>(c, n, B.t->p, B.w, B.r->p, B.d->p, B.x->p, rho_new * rho, 2.0 * rho_new / delta);
    rho = rho_new;
  }
}

// The coarse correction of level l on level l+1 (input *NB.b, result *NB.x): cycle_gamma
// visits, each later one on the residual the earlier ones left, their corrections summed
// (gamma = 2: x = 2 B b - B A B b, the W-cycle).  The coarsest solve is exact: one visit.
// coarse_first makes the first visit (a plain cycle whose first iterate w.b the
// restriction already formed).
template <class T>
static void coarse_visits(Handle& h, size_t l, void (*coarse)(Handle&, size_t),
                          void (*coarse_first)(Handle&, size_t)) {
  coarse_first(h, l + 1);
  if (h.opt.cycle_gamma <= 1 || l + 2 >= h.lev.size()) return;
  Level& N = *h.lev[l + 1];
  LvBufs<T> NB = lv_bufs(N, T());
  for (int g = 1; g < h.opt.cycle_gamma; ++g) {
    k_spmv(h, l + 1, SPMV_RES, NB.x->p, NB.bw->p, NB.b->p, (const T*)nullptr, (T*)nullptr);
    contact<T>(h, N, CT_SUB_RES, NB.x->p, NB.bw->p, (const T*)nullptr);
    std::swap(*NB.b, *NB.bw);                         // next visit: on the residual
    std::swap(*NB.x, *NB.xw);                         // keep the correction so far
    coarse(h, l + 1);
    add_to(h.ctx, N.n(), NB.xw->p, NB.x->p);
    std::swap(*NB.b, *NB.bw);
  }
}

// general V(nu, nu) on level l (not the coarsest): *B.b -> *B.x
template <class T>
static void vcycle_general(Handle& h, size_t l, void (*coarse)(Handle&, size_t)) {
  Level& L = *h.lev[l];
  Level& N = *h.lev[l + 1];
  LvBufs<T> B = lv_bufs(L, T());
  LvBufs<T> NB = lv_bufs(N, T());
  for (int s = 0; s < h.opt.sweeps; ++s) smooth_once<T>(h, l, s == 0);
  k_spmv(h, l, SPMV_RES, B.x->p, B.r->p, B.b->p, (const T*)nullptr, (T*)nullptr);
  contact<T>(h, L, CT_SUB_RES, B.x->p, B.r->p, (const T*)nullptr);
  transfer(h, SPMV_Y, L.PT, B.r->p, NB.b->p);
  coarse_visits<T>(h, l, coarse, coarse);
  transfer(h, SPMV_ADD, L.P, NB.x->p, B.x->p);
  for (int s = 0; s < h.opt.sweeps; ++s) smooth_once<T>(h, l, false);
}

// FP64 V(1,1) on level l: L.vb -> L.vx.  As in the FP32 cycle, the first smoothing
// iterate x = w.b is formed on its own (x0_ready: the caller already wrote it to L.vx) and
// r = b - K x then gathers x once per column instead of w and b.
static void vcycle64_from(Handle& h, size_t l, bool x0_ready);
static void vcycle64(Handle& h, size_t l) { vcycle64_from(h, l, false); }
static void vcycle64_ready(Handle& h, size_t l) { vcycle64_from(h, l, true); }
static void vcycle64_from(Handle& h, size_t l, bool x0_ready) {
  Ctx& c = h.ctx;
  Level& L = *h.lev[l];
  if (l + 1 == h.lev.size()) {
    coarse_solve(h, L.vb.p, L.vx.p);
    return;
  }
  if (!h.plain_cycle()) return vcycle_general<double>(h, l, vcycle64);
  Level& N = *h.lev[l + 1];
  if (!x0_ready) wmul_f64(c, L.n(), L.w.p, L.vb.p, L.vx.p);
  if (l == 0) prof_begin(h, AMGF_K_PRESMOOTH);
  const BSR& S = smooth_mat(L);
  bsr_spmv<double>(c, SPMV_RES, S, S.val.p, L.vx.p, L.vr.p, L.vb.p, nullptr, nullptr);
  prof_end(h);
  level_contact<double>(h, L, CT_SUB_RES, L.vx.p, L.vr.p, nullptr);
  // restriction; on a smoothed level it also forms that cycle's first iterate w.b
  const bool n_smoothed = l + 2 < h.lev.size();
  bsr_spmv<double>(c, n_smoothed ? SPMV_YW : SPMV_Y, L.PT, L.PT.val.p, L.vr.p, N.vb.p, nullptr,
                   n_smoothed ? N.w.p : nullptr, n_smoothed ? N.vx.p : nullptr);
  coarse_visits<double>(h, l, vcycle64, vcycle64_ready);
  bsr_spmv<double>(c, SPMV_ADD, L.P, L.P.val.p, N.vx.p, L.vx.p, nullptr, nullptr, nullptr);
  if (l == 0) prof_begin(h, AMGF_K_POSTSMOOTH);
  bsr_spmv<double>(c, SPMV_POST, S, S.val.p, L.vx.p, nullptr, L.vb.p, L.w.p, L.vxn.p);
  prof_end(h);
  level_contact<double>(h, L, CT_SUB_W, L.vx.p, L.vxn.p, L.w.p);
  std::swap(L.vx, L.vxn);
}

// FP32 V(1,1) (contact term and coarsest solve in FP64): L.fb -> L.fx.  The first
// smoothing iterate x = w.b is formed on its own (x0_ready: the caller already wrote it
// to L.fx), then r = b - K x reads x once per column instead of w and b.
static void vcycle32_from(Handle& h, size_t l, bool x0_ready);
static void vcycle32(Handle& h, size_t l) { vcycle32_from(h, l, false); }
static void vcycle32_ready(Handle& h, size_t l) { vcycle32_from(h, l, true); }
static void vcycle32_from(Handle& h, size_t l, bool x0_ready) {
  Ctx& c = h.ctx;
  Level& L = *h.lev[l];
  if (l + 1 == h.lev.size()) {
    if (h.coarse_inverse) {                           // FP32 in and out, FP64 product
      h.coarse_inv.solve_f32(c, L.fb.p, L.fx.p);
      return;
    }
    cast_f2d(c, L.fb.p, h.coarse_b.p, L.n());
    coarse_solve(h, h.coarse_b.p, h.coarse_x.p);
    cast_d2f(c, h.coarse_x.p, L.fx.p, L.n());
    return;
  }
  if (!h.plain_cycle()) return vcycle_general<float>(h, l, vcycle32);
  Level& N = *h.lev[l + 1];
  if (!x0_ready) wmul_f32(c, L.n(), L.w32.p, L.fb.p, L.fx.p);
  if (l == 0) prof_begin(h, AMGF_K_PRESMOOTH);
  if (l == 0 && h.bf16k())
    sell_spmv_bf16(c, SPMV_RES, L.K, L.fx.p, L.fr.p, L.fb.p, nullptr, nullptr);
  else
    bsr_spmv<float>(c, SPMV_RES, smooth_mat(L), smooth_mat(L).val32.p, L.fx.p, L.fr.p, L.fb.p,
                    nullptr, nullptr);
  prof_end(h);
  level_contact<float>(h, L, CT_SUB_RES, L.fx.p, L.fr.p, nullptr);
  // restriction; on a smoothed level it also forms that cycle's first iterate w.b
  if (l + 2 < h.lev.size()) {
    transfer_spmv(c, SPMV_YW, L.PT, L.fr.p, N.fb.p, N.w32.p, N.fx.p);
    coarse_visits<float>(h, l, vcycle32, vcycle32_ready);
  } else {
    transfer_spmv(c, SPMV_Y, L.PT, L.fr.p, N.fb.p);
    coarse_visits<float>(h, l, vcycle32, vcycle32);
  }
  transfer_spmv(c, SPMV_ADD, L.P, N.fx.p, L.fx.p);
  if (l == 0) prof_begin(h, AMGF_K_POSTSMOOTH);
  if (l == 0 && h.bf16k())
    sell_spmv_bf16(c, SPMV_POST, L.K, L.fx.p, nullptr, L.fb.p, L.w32.p, L.fxn.p);
  else
    bsr_spmv<float>(c, SPMV_POST, smooth_mat(L), smooth_mat(L).val32.p, L.fx.p, nullptr, L.fb.p,
                    L.w32.p, L.fxn.p);
  prof_end(h);
  level_contact<float>(h, L, CT_SUB_W, L.fx.p, L.fxn.p, L.w32.p);
  std::swap(L.fx, L.fxn);
}

// z = B r (FP64 boundary vectors)
static void vcycle(Handle& h, const double* r, double* z) {
  Ctx& c = h.ctx;
  Level& L0 = *h.lev[0];
  const int64_t n = h.n();
  if (h.mixed()) {
    if (h.plain_cycle()) {
      if (!h.r_cast_ready) cast_d2f_w(c, r, L0.w32.p, L0.fb.p, L0.fx.p, n);
      h.r_cast_ready = false;
      vcycle32_from(h, 0, true);
    } else {
      cast_d2f(c, r, L0.fb.p, n);
      vcycle32(h, 0);
    }
    cast_f2d(c, L0.fx.p, z, n);
  } else if (h.plain_cycle()) {
    copy_w(c, r, L0.w.p, L0.vb.p, L0.vx.p, n);
    vcycle64_from(h, 0, true);
    vcopy(c, L0.vx.p, z, n);
  } else {
    vcopy(c, r, L0.vb.p, n);
    vcycle64(h, 0);
    vcopy(c, L0.vx.p, z, n);
  }
}

// y = A x (FP64), or y = b - A x when b != nullptr
static void operator_apply(Handle& h, const double* x, double* y, const double* b) {
  Ctx& c = h.ctx;
  Level& L0 = *h.lev[0];
  if (b) {
    bsr_spmv<double>(c, SPMV_RES, L0.K, L0.K.val.p, x, y, b, nullptr, nullptr);
    contact_apply<double, double>(c, CT_SUB_RES, L0.J, L0.JT, L0.crows.p, L0.ncrows, h.D.p, x,
                                  h.t.p, y, nullptr);
  } else {
    bsr_spmv<double>(c, SPMV_Y, L0.K, L0.K.val.p, x, y, nullptr, nullptr, nullptr);
    contact_apply<double, double>(c, CT_ADD, L0.J, L0.JT, L0.crows.p, L0.ncrows, h.D.p, x,
                                  h.t.p, y, nullptr);
  }
}

// w = A_w^{-1} r with the multifrontal factor of the filter matrix, r and w in the
// factor's tree order (entry q belongs to DOF Ic_t[q])
static void filter_solve(Handle& h, const double* r, double* w) {
  h.aw.solve_tree(h.ctx, r, w);
}

// CG dot products that an AMGF step can form in its last kernel: out[0] = r.z and
// out[1] = r.zo (device memory), part the dot-product partials (nullptr: the context's)
struct StepDots {
  const double* zo;
  double* out;
  double* part;
};

// z = M r, Definition 5.3:  z1 = B r;  z2 = z1 + P A_w^{-1} P^T (r - A z1);
// z = z2 + B (r - A z2).  The filter residual is formed on the filter rows only.  In
// mixed precision the second residual keeps the stiffness product in FP32 (it only
// feeds the FP32 V-cycle) and the contact term in FP64.  Returns true when it also formed
// the dot products sd asks for (the mixed step does, in its final sum).
static bool amgf_apply_impl(Handle& h, const double* r, double* z,
                            const StepDots* sd = nullptr) {
  Ctx& c = h.ctx;
  const int64_t n = h.n();
  phase(h, PH_AMG);
  if (!h.opt.filter || h.filter_suspended) {
    vcycle(h, r, z);
    phase(h, PH_OTHER);
    return false;
  }
  Level& L0 = *h.lev[0];
  if (h.mixed() && h.plain_cycle() && h.ic_from_J) {
    // FP32 V-cycles: z1 = B r stays in FP32 (L0.fx, widened exactly wherever FP64 reads
    // it); the FP64 z2 = z1 + P w is formed on the filter DOFs only (h.z1 there), which
    // cover every DOF the contact term reads when I_c comes from J
    if (!h.r_cast_ready) cast_d2f_w(c, r, L0.w32.p, L0.fb.p, L0.fx.p, n);
    h.r_cast_ready = false;
    vcycle32_from(h, 0, true);                        // z1 = B r  (L0.fx)
    if (h.n_c > 0) {
      phase(h, PH_FILTER);
      bsr_res_rows<float>(c, L0.K, h.ic_nodes.p, h.n_icn, L0.fx.p, r, h.ra.p);
      contact_apply<float, double>(c, CT_SUB_RES, L0.J, L0.JT, L0.crows.p, L0.ncrows, h.D.p,
                                   L0.fx.p, h.t.p, h.ra.p, nullptr);   // ra = r - A z1 on I_c
      gather(c, h.ra.p, h.Ic_t.p, h.n_c, h.f_r.p);      // P^T ra
      filter_solve(h, h.f_r.p, h.f_w.p);              // w = A_w^{-1} P^T ra
      correct_at(c, L0.fx.p, h.f_w.p, h.Ic_t.p, h.n_c, h.z1.p);   // z2 on I_c; L0.fx = float(z2)
    }
    phase(h, PH_OTHER);
    bsr_spmv<float>(c, SPMV_RES, L0.K, L0.K.val32.p, L0.fx.p, h.r2f.p, L0.fb.p, nullptr,
                    nullptr);
    contact_apply<double, float>(c, CT_SUB_RES, L0.J, L0.JT, L0.crows.p, L0.ncrows, h.D.p,
                                 h.z1.p, h.t.p, h.r2f.p, nullptr);     // r2 = r - A z2
    std::swap(L0.fx, h.zf);                           // keep z1 (float(z2) on I_c)
    std::swap(L0.fb, h.r2f);
    phase(h, PH_AMG);
    vcycle32(h, 0);                                   // B r2  (L0.fx)
    phase(h, PH_OTHER);
    std::swap(L0.fb, h.r2f);
    if (sd && h.ic_mask.p) {                          // the same sums, with r.z and r.zo
      add_ff_dots(c, n, h.zf.p, L0.fx.p, h.z1.p, h.ic_mask.p, r, sd->zo, z, sd->out,
                  sd->part);
      return true;
    }
    add_ff(c, n, h.zf.p, L0.fx.p, z);                 // z = z2 + B r2 ...
    add_at(c, h.z1.p, L0.fx.p, h.Ic.p, h.n_c, z);     // ... with the FP64 z2 on I_c
    return false;
  }
  vcycle(h, r, h.z1.p);                               // z1 = B r
  if (h.n_c > 0) {
    phase(h, PH_FILTER);
    bsr_res_rows(c, L0.K, h.ic_nodes.p, h.n_icn, h.z1.p, r, h.ra.p);
    contact_apply<double, double>(c, CT_SUB_RES, L0.J, L0.JT, L0.crows.p, L0.ncrows, h.D.p,
                                  h.z1.p, h.t.p, h.ra.p, nullptr);     // ra = r - A z1 on I_c
    gather(c, h.ra.p, h.Ic_t.p, h.n_c, h.f_r.p);        // P^T ra
    filter_solve(h, h.f_r.p, h.f_w.p);                // w = A_w^{-1} P^T ra
    scatter_add(c, h.f_w.p, h.Ic_t.p, h.n_c, h.z1.p);   // z2 = z1 + P w
  }
  phase(h, PH_OTHER);
  if (h.mixed()) {
    cast_d2f(c, h.z1.p, h.zf.p, n);
    bsr_spmv<float>(c, SPMV_RES, L0.K, L0.K.val32.p, h.zf.p, h.r2f.p, L0.fb.p, nullptr, nullptr);
    contact_apply<double, float>(c, CT_SUB_RES, L0.J, L0.JT, L0.crows.p, L0.ncrows, h.D.p,
                                 h.z1.p, h.t.p, h.r2f.p, nullptr);     // r2 = r - A z2
    std::swap(L0.fb, h.r2f);
    phase(h, PH_AMG);
    vcycle32(h, 0);                                   // B r2
    phase(h, PH_OTHER);
    std::swap(L0.fb, h.r2f);
    add_f32(c, n, h.z1.p, L0.fx.p, z);                // z = z2 + B r2
  } else {
    operator_apply(h, h.z1.p, h.r2.p, r);             // r2 = r - A z2
    phase(h, PH_AMG);
    vcycle(h, h.r2.p, h.z3.p);                        // B r2
    phase(h, PH_OTHER);
    vcopy(c, h.z1.p, z, n);
    axpby(c, n, 1.0, h.z3.p, 1.0, z);                 // z = z2 + B r2
  }
  return false;
}

static void set_damping(Handle& h, const float* W);

// The judge of the learned damping: one AMGF error-propagation step e1 = e0 - M A e0 from
// the fixed start e0 (the power-iteration start, zero on decoupled DOFs) with the MLP
// damping and with theta = 1.  Plain l1-Jacobi is the reference the learned damping has to
// beat on every system it is set up for: the MLP damping stays unless theta = 1 leaves an
// energy-norm error smaller by more than JUDGE_MARGIN.  One step from one start vector
// ranks clear differences (3x in favour of the MLP on the trained workloads, 18x against
// it with bound-constraint terms it never saw) but not near-ties, where the CG counts can
// go either way (C3: 9.81e-5 against 9.73e-5, 233 iterations with the MLP, 248 without).
constexpr double JUDGE_MARGIN = 1.25;

static void judge_damping(Handle& h) {
  h.judge_rejected = false;
  if (!h.judge_on || !h.learned) return;
  Ctx& c = h.ctx;
  const int64_t n = h.n();
  DBuf<double> e0(n), ae0(n), e1(n), ae1(n);
  fill_power_start(c, n, e0.p, h.dec0.p);
  operator_apply(h, e0.p, ae0.p, nullptr);
  double n0;
  {
    const double* xs[1] = {e0.p};
    const double* ys[1] = {ae0.p};
    dots(c, n, 1, xs, ys, &n0);
  }
  auto reduction = [&]() {
    amgf_apply_impl(h, ae0.p, e1.p);                  // M A e0
    axpby(c, n, 1.0, e0.p, -1.0, e1.p);               // e1 = e0 - M A e0
    operator_apply(h, e1.p, ae1.p, nullptr);
    double n1;
    const double* xs[1] = {e1.p};
    const double* ys[1] = {ae1.p};
    dots(c, n, 1, xs, ys, &n1);
    return n0 > 0.0 ? std::sqrt(std::fabs(n1) / n0) : 0.0;
  };
  h.judge_l = reduction();
  set_damping(h, nullptr);
  h.judge_p = reduction();
  if (h.judge_l <= JUDGE_MARGIN * h.judge_p) {
    // back to w = theta / d from the stored MLP damping (the same division mlp_theta made,
    // so bitwise its weights, without evaluating the network again)
    for (size_t l = 0; l + 1 < h.lev.size(); ++l) {
      Level& L = *h.lev[l];
      weights_from_l1(c, L.n(), L.d.p, L.theta.p, L.w.p);
      if (h.mixed()) cast_d2f(c, L.w.p, L.w32.p, L.n());
    }
  } else {
    h.learned = false;
    h.judge_rejected = true;
  }
}

// ------------------------------------------------------------------------------------
// learned smoother: damping from the MLP, taped forward and adjoint of M
// ------------------------------------------------------------------------------------
// w = theta / d on every smoothed level; W == nullptr restores theta = 1
static void set_damping(Handle& h, const float* W) {
  Ctx& c = h.ctx;
  for (size_t l = 0; l + 1 < h.lev.size(); ++l) {
    Level& L = *h.lev[l];
    if (W) mlp_theta(c, L.n(), W, L.F.p, L.d.p, L.theta.p, L.w.p);
    else weights_from_l1(c, L.n(), L.d.p, nullptr, L.w.p);
    if (h.mixed()) cast_d2f(c, L.w.p, L.w32.p, L.n());
  }
}

struct Tape {
  std::vector<DBuf<double>> b, s2;   // per level: V-cycle input and post-smoothing residual
  void alloc(const Handle& h) {
    b.resize(h.lev.size());
    s2.resize(h.lev.size());
    for (size_t l = 0; l < h.lev.size(); ++l) {
      b[l].alloc(h.lev[l]->n());
      s2[l].alloc(h.lev[l]->n());
    }
  }
};

// FP64 V-cycle L.vb -> L.vx, recording b and s2 = b - A x' of every level
static void vcycle64_tape(Handle& h, size_t l, Tape& T) {
  Ctx& c = h.ctx;
  Level& L = *h.lev[l];
  vcopy(c, L.vb.p, T.b[l].p, L.n());
  if (l + 1 == h.lev.size()) {
    coarse_solve(h, L.vb.p, L.vx.p);
    return;
  }
  Level& N = *h.lev[l + 1];
  bsr_spmv<double>(c, SPMV_PRE, L.K, L.K.val.p, nullptr, L.vr.p, L.vb.p, L.w.p, L.vx.p);
  contact_apply<double, double>(c, CT_SUB_RES, L.J, L.JT, L.crows.p, L.ncrows, h.D.p, L.vx.p,
                                h.t.p, L.vr.p, nullptr);
  bsr_spmv<double>(c, SPMV_Y, L.PT, L.PT.val.p, L.vr.p, N.vb.p, nullptr, nullptr, nullptr);
  vcycle64_tape(h, l + 1, T);
  bsr_spmv<double>(c, SPMV_ADD, L.P, L.P.val.p, N.vx.p, L.vx.p, nullptr, nullptr, nullptr);
  bsr_spmv<double>(c, SPMV_RES, L.K, L.K.val.p, L.vx.p, T.s2[l].p, L.vb.p, nullptr, nullptr);
  contact_apply<double, double>(c, CT_SUB_RES, L.J, L.JT, L.crows.p, L.ncrows, h.D.p, L.vx.p,
                                h.t.p, T.s2[l].p, nullptr);
  axpy_hadamard(c, L.n(), L.w.p, T.s2[l].p, L.vx.p);
}

// y = b - A x on level l (K_l plus the contact term), FP64
static void level_residual(Handle& h, Level& L, const double* x, double* y, const double* b) {
  bsr_spmv<double>(h.ctx, SPMV_RES, L.K, L.K.val.p, x, y, b, nullptr, nullptr);
  contact_apply<double, double>(h.ctx, CT_SUB_RES, L.J, L.JT, L.crows.p, L.ncrows, h.D.p, x,
                                h.t.p, y, nullptr);
}

// adjoint of the V-cycle: L.ay (adjoint of the output) -> L.ab (adjoint of the input),
// accumulating d/dw into L.wbar.  Reverse of
//   x = w.b; r = b - A x; xc = B_c(P^T r); x' = x + P xc; s2 = b - A x'; x'' = x' + w.s2
static void vcycle64_adj(Handle& h, size_t l, const Tape& T) {
  Ctx& c = h.ctx;
  Level& L = *h.lev[l];
  const int64_t n = L.n();
  if (l + 1 == h.lev.size()) {
    coarse_solve(h, L.ay.p, L.ab.p);
    return;
  }
  Level& N = *h.lev[l + 1];
  hadamard(c, n, L.w.p, L.ay.p, L.ab.p);                  // s2bar = w.ybar (-> bbar)
  acc_hadamard(c, n, L.ay.p, T.s2[l].p, L.wbar.p);        // wbar += ybar.s2
  level_residual(h, L, L.ab.p, L.ax.p, L.ay.p);           // x'bar = ybar - A s2bar
  bsr_spmv<double>(c, SPMV_Y, L.PT, L.PT.val.p, L.ax.p, N.ay.p, nullptr, nullptr, nullptr);
  vcycle64_adj(h, l + 1, T);                              // bcbar = B_c^T xcbar
  bsr_spmv<double>(c, SPMV_Y, L.P, L.P.val.p, N.ab.p, L.ar.p, nullptr, nullptr, nullptr);
  axpby(c, n, 1.0, L.ar.p, 1.0, L.ab.p);                  // bbar += rbar
  level_residual(h, L, L.ar.p, L.ax2.p, L.ax.p);          // xbar = x'bar - A rbar
  axpy_hadamard(c, n, L.w.p, L.ax2.p, L.ab.p);            // bbar += w.xbar
  acc_hadamard(c, n, L.ax2.p, T.b[l].p, L.wbar.p);        // wbar += xbar.b
}

// z = M v (FP64) recording both V-cycles
static void apply_tape(Handle& h, const double* v, double* z, Tape& T1, Tape& T2) {
  Ctx& c = h.ctx;
  Level& L0 = *h.lev[0];
  const int64_t n = h.n();
  vcopy(c, v, L0.vb.p, n);
  vcycle64_tape(h, 0, T1);
  vcopy(c, L0.vx.p, h.z1.p, n);
  if (h.n_c > 0) {
    bsr_res_rows(c, L0.K, h.ic_nodes.p, h.n_icn, h.z1.p, v, h.ra.p);
    contact_apply<double, double>(c, CT_SUB_RES, L0.J, L0.JT, L0.crows.p, L0.ncrows, h.D.p,
                                  h.z1.p, h.t.p, h.ra.p, nullptr);
    gather(c, h.ra.p, h.Ic_t.p, h.n_c, h.f_r.p);
    filter_solve(h, h.f_r.p, h.f_w.p);
    scatter_add(c, h.f_w.p, h.Ic_t.p, h.n_c, h.z1.p);
  }
  operator_apply(h, h.z1.p, L0.vb.p, v);                  // r2 = v - A z2
  vcycle64_tape(h, 0, T2);
  vcopy(c, h.z1.p, z, n);
  axpby(c, n, 1.0, L0.vx.p, 1.0, z);
}

// vbar = M^T zbar, accumulating d/dw of both V-cycles (reverse of apply_tape)
static void apply_adj(Handle& h, const double* zbar, double* vbar, const Tape& T1,
                      const Tape& T2) {
  Ctx& c = h.ctx;
  Level& L0 = *h.lev[0];
  const int64_t n = h.n();
  vcopy(c, zbar, L0.ay.p, n);
  vcycle64_adj(h, 0, T2);                                 // r2bar = B^T zbar
  vcopy(c, L0.ab.p, vbar, n);                             // vbar = r2bar
  operator_apply(h, L0.ab.p, h.z3.p, zbar);               // z2bar = zbar - A r2bar
  if (h.n_c > 0) {
    gather(c, h.z3.p, h.Ic_t.p, h.n_c, h.f_r.p);
    filter_solve(h, h.f_r.p, h.f_w.p);                    // rabar = A_w^{-1} P^T z2bar
    AMGF_HIP(hipMemsetAsync(h.r2.p, 0, sizeof(double) * n, c.s));
    scatter_add(c, h.f_w.p, h.Ic_t.p, h.n_c, h.r2.p);       // u = P rabar
    axpby(c, n, 1.0, h.r2.p, 1.0, vbar);                  // vbar += u
    operator_apply(h, h.r2.p, L0.ay.p, h.z3.p);           // z1bar = z2bar - A u
  } else {
    vcopy(c, h.z3.p, L0.ay.p, n);
  }
  vcycle64_adj(h, 0, T1);
  axpby(c, n, 1.0, L0.ab.p, 1.0, vbar);                   // vbar += B^T z1bar
}

// mean over probes of (1/k) log(||E^k e||_S / ||e||_S), E = I - M S, and d/dW
static double loss_grad(Handle& h, const float* W, int k, int np, const double* probes,
                        double* grad) {
  Ctx& c = h.ctx;
  const int64_t n = h.n();
  AMGF_REQUIRE(!h.mixed(), AMGF_EINVAL, "training runs on an FP64 handle");
  AMGF_REQUIRE(h.opt.cycle_gamma == 1, AMGF_EINVAL, "training follows the V-cycle");
  AMGF_REQUIRE(h.lev.size() > 1, AMGF_EINVAL, "no smoothed level");
  set_damping(h, W);
  for (auto& Lp : h.lev) {
    Level& L = *Lp;
    if (!L.ay.n) {
      L.ay.alloc(L.n()); L.ab.alloc(L.n()); L.ax.alloc(L.n());
      L.ar.alloc(L.n()); L.ax2.alloc(L.n()); L.wbar.alloc(L.n());
    }
    AMGF_HIP(hipMemsetAsync(L.wbar.p, 0, L.wbar.bytes(), c.s));
  }
  std::vector<Tape> T(2 * size_t(k));
  for (auto& t : T) t.alloc(h);
  DBuf<double> e(n), Se(n), r(n), z(n), eb(n), vb(n);
  double loss = 0.0;
  for (int q = 0; q < np; ++q) {
    vcopy(c, probes + int64_t(q) * n, e.p, n);
    operator_apply(h, e.p, Se.p, nullptr);
    double s0;
    {
      const double* xs[1] = {e.p};
      const double* ys[1] = {Se.p};
      dots(c, n, 1, xs, ys, &s0);
    }
    for (int j = 0; j < k; ++j) {
      operator_apply(h, e.p, r.p, nullptr);               // r_j = S e_j
      apply_tape(h, r.p, z.p, T[2 * j], T[2 * j + 1]);    // z_j = M r_j
      axpby(c, n, -1.0, z.p, 1.0, e.p);                   // e_{j+1} = e_j - z_j
    }
    operator_apply(h, e.p, Se.p, nullptr);
    double sk;
    {
      const double* xs[1] = {e.p};
      const double* ys[1] = {Se.p};
      dots(c, n, 1, xs, ys, &sk);
    }
    AMGF_REQUIRE(s0 > 0.0 && sk > 0.0, AMGF_ENOTSPD, "probe has zero energy");
    loss += (std::log(sk) - std::log(s0)) / (2.0 * k);
    vcopy(c, Se.p, eb.p, n);
    vscale(c, n, 1.0 / (k * sk), eb.p);                   // ebar_k = S e_k / (k s_k)
    for (int j = k - 1; j >= 0; --j) {
      vcopy(c, eb.p, z.p, n);
      vscale(c, n, -1.0, z.p);                            // zbar_j = -ebar_{j+1}
      apply_adj(h, z.p, vb.p, T[2 * j], T[2 * j + 1]);
      operator_apply(h, vb.p, r.p, nullptr);
      axpby(c, n, 1.0, r.p, 1.0, eb.p);                   // ebar_j = ebar_{j+1} + S vbar
    }
  }
  // dL/dtheta = wbar / d / np on every smoothed level, then through the MLP
  bool first = true;
  for (size_t l = 0; l + 1 < h.lev.size(); ++l) {
    Level& L = *h.lev[l];
    vdiv(c, L.n(), L.wbar.p, L.d.p, L.ax.p);
    vscale(c, L.n(), 1.0 / np, L.ax.p);
    mlp_backward(c, L.n(), W, L.F.p, L.ax.p, grad, !first);
    first = false;
  }
  return loss / np;
}

// ------------------------------------------------------------------------------------
// PCG (Sec. 4 / 6.1 stopping rule), Polak-Ribiere beta
// ------------------------------------------------------------------------------------
static amgf_status pcg_run(Handle& h, const double* b, double* x, amgf_solve_info* info,
                           double* ns = nullptr);

// Learned damping: if CG does not converge (or breaks down), rerun from the same initial
// guess with theta = 1 (plain l1-Jacobi) and report the fallback.
// ns: the allocation-free variant's device scratch (no fallback rerun there: keeping the
// initial guess for it would need n doubles).
static amgf_status pcg_impl(Handle& h, const double* b, double* x, amgf_solve_info* info,
                            double* ns = nullptr) {
  if (!h.learned || ns) {
    amgf_status st = pcg_run(h, b, x, info, ns);
    if (info && h.judge_rejected) info->used_fallback = 2;
    return st;
  }
  Ctx& c = h.ctx;
  DBuf<double> x0(h.n());
  vcopy(c, x, x0.p, h.n());
  amgf_status st = pcg_run(h, b, x, info);
  if (st == AMGF_OK) return st;
  set_damping(h, nullptr);
  vcopy(c, x0.p, x, h.n());
  st = pcg_run(h, b, x, info);
  set_damping(h, h.mlpW.p);
  if (info) info->used_fallback = 1;
  return st;
}

// ns != nullptr: the allocation-free variant.  Its CG scalars and dot-product partials live
// in the device scratch ns (PCG_SCRATCH doubles), the host reads the scalars into a stack
// array after a stream synchronisation, and no events are created (no phase split; the
// solve time is host wall time).
static amgf_status pcg_run(Handle& h, const double* b, double* x, amgf_solve_info* info,
                           double* ns) {
  Ctx& c = h.ctx;
  const int64_t n = h.n();
  const bool na = ns != nullptr;
  double* dpart = na ? ns : nullptr;                  // dot partials (nullptr: c.dot)
  const auto t_host0 = std::chrono::steady_clock::now();
  struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } evs;
  if (!na) {
    AMGF_HIP(hipEventCreate(&evs.e0));
    AMGF_HIP(hipEventCreate(&evs.e1));
    AMGF_HIP(hipEventRecord(evs.e0, c.s));
  }
  struct PhaseScope {                                 // phase timing on for this solve only
    Handle& h;
    PhaseScope(Handle& hh, bool on) : h(hh) { h.ph_used = 0; h.ph_on = on; }
    ~PhaseScope() { h.ph_on = false; }
  } phases_(h, !na);
  phase(h, PH_OTHER);
  operator_apply(h, x, h.pr.p, b);                    // r = b - A x0
  amgf_apply_impl(h, h.pr.p, h.pz.p);
  vcopy(c, h.pz.p, h.pp.p, n);
  double d2[2];
  {
    const double* xs[2] = {h.pr.p, b};
    const double* ys[2] = {h.pz.p, b};
    dots(c, n, 2, xs, ys, d2, dpart);
  }
  double rz = d2[0];
  const double rz0 = rz;
  int it = 0;
  bool conv = rz0 == 0.0;
  double rel = conv ? 0.0 : 1.0;
  amgf_status st = AMGF_OK;
  // Scalars stay on the device within an iteration (p.q feeds the x, r update, r.z and
  // r.z_old the direction update); the host reads p.q, r.z and r.z_old once per iteration
  // for the stopping rule.  While it waits for them the stream already runs the next
  // direction p = z + beta p, q = A p and p.q (beta formed on the device from the same
  // doubles, so the iterates are those of the host-side update); after the last
  // iteration that work is simply not used.
  // The speculation is skipped when the residual history predicts convergence in this
  // iteration (geometric extrapolation), so the last iteration rarely wastes the work.
  double* dsc = nullptr;                              // device scalars p.q, r.z, r.z_old
  if (na) {
    dsc = ns + DOT_SCRATCH;
  } else {
    if (h.pcg_s.n == 0) h.pcg_s.alloc(4);
    dsc = h.pcg_s.p;
  }
  struct HostScalars {                                // pinned: the copy is truly async
    double* p = nullptr;
    hipEvent_t ev = nullptr;
    ~HostScalars() {
      if (ev) (void)hipEventDestroy(ev);
      if (p) (void)hipHostFree(p);
    }
  } hs;
  double s3_stack[4] = {0.0, 0.0, 0.0, 0.0};
  double* s3 = s3_stack;
  if (!na) {
    AMGF_HIP(hipHostMalloc(reinterpret_cast<void**>(&hs.p), 4 * sizeof(double)));
    AMGF_HIP(hipEventCreateWithFlags(&hs.ev, hipEventDisableTiming));
    s3 = hs.p;
  }
  hipEvent_t ev = hs.ev;
  double rel_old = 1.0;                               // relative residual one step back
  h.cg_alpha.clear();
  h.cg_beta.clear();
  bool have_q = false;                                // q = A p, p.q already enqueued
  bool need_p = false;                                // p = z + beta p still to be done
  double beta = 0.0;
  while (!conv && it < h.opt.max_iters) {
    if (!have_q) {
      if (need_p) pcg_update_p(c, n, beta, h.pz.p, h.pp.p);
      operator_apply(h, h.pp.p, h.pq.p, nullptr);     // q = A p
      const double* xs[1] = {h.pp.p};
      const double* ys[1] = {h.pq.p};
      dots_device(c, n, 1, xs, ys, dsc, dpart);
    }
    if (h.mixed() && h.plain_cycle()) {
      // the V-cycle's first level-0 vectors come out of the residual update
      Level& L0 = *h.lev[0];
      pcg_update_xr_dev_f(c, n, rz, dsc, h.pp.p, h.pq.p, x, h.pr.p, L0.w32.p, L0.fb.p,
                          L0.fx.p);
      h.r_cast_ready = true;
    } else {
      pcg_update_xr_dev(c, n, rz, dsc, h.pp.p, h.pq.p, x, h.pr.p);
    }
    std::swap(h.pz, h.pzo);
    const StepDots sd{h.pzo.p, dsc + 1, dpart};
    if (!amgf_apply_impl(h, h.pr.p, h.pz.p, &sd)) {   // r.z and r.z_old
      const double* xs[2] = {h.pr.p, h.pr.p};
      const double* ys[2] = {h.pz.p, h.pzo.p};
      dots_device(c, n, 2, xs, ys, dsc + 1, dpart);
    }
    h.r_cast_ready = false;
    AMGF_HIP(hipMemcpyAsync(s3, dsc, 3 * sizeof(double), hipMemcpyDeviceToHost, c.s));
    if (!na) AMGF_HIP(hipEventRecord(ev, c.s));
    have_q = it + 1 < h.opt.max_iters && rel * (rel / rel_old) > h.opt.rtol;
    if (have_q) {
      pcg_update_p_dev(c, n, rz, dsc + 1, h.pz.p, h.pp.p);
      operator_apply(h, h.pp.p, h.pq.p, nullptr);
      const double* xs[1] = {h.pp.p};
      const double* ys[1] = {h.pq.p};
      dots_device(c, n, 1, xs, ys, dsc, dpart);
    }
    if (na) AMGF_HIP(hipStreamSynchronize(c.s));
    else AMGF_HIP(hipEventSynchronize(ev));
    if (!(s3[0] > 0.0)) { st = AMGF_ENOTSPD; break; }  // p.q <= 0: not SPD
    d2[0] = s3[1];
    d2[1] = s3[2];
    if (!na) {                                        // (no host allocation when na)
      h.cg_alpha.push_back(rz / s3[0]);
      h.cg_beta.push_back(d2[0] / rz);
    }
    ++it;
    const double rel_prev = rel;
    rel = std::sqrt(std::fabs(d2[0]) / rz0);
    if (!std::isfinite(rel)) { st = AMGF_ENOTSPD; break; }
    if (rel <= h.opt.rtol) { conv = true; break; }
    need_p = !have_q;
    if (need_p) beta = (d2[0] - d2[1]) / rz;
    rz = d2[0];
    rel_old = rel_prev;
  }
  float ms = 0.f;
  float ms_ph[3] = {0.f, 0.f, 0.f};
  if (!na) {
    AMGF_HIP(hipEventRecord(evs.e1, c.s));
    AMGF_HIP(hipEventSynchronize(evs.e1));
    AMGF_HIP(hipEventElapsedTime(&ms, evs.e0, evs.e1));
    for (size_t i = 0; i < h.ph_used; ++i) {
      float t = 0.f;
      AMGF_HIP(hipEventElapsedTime(&t, h.ph_ev[i],
                                   i + 1 < h.ph_used ? h.ph_ev[i + 1] : evs.e1));
      ms_ph[h.ph_cat[i]] += t;
    }
  } else {
    AMGF_HIP(hipStreamSynchronize(c.s));
    ms = float(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                         t_host0).count());
  }
  h.ph_on = false;
  if (info) {
    operator_apply(h, x, h.ra.p, b);
    double tr[2];
    const double* xs[2] = {h.ra.p, b};
    const double* ys[2] = {h.ra.p, b};
    dots(c, n, 2, xs, ys, tr, dpart);
    info->iterations = it;
    info->converged = conv ? 1 : 0;
    info->n_levels = int(h.lev.size());
    info->n_c = h.n_c;
    info->rel_prec_res = rel;
    info->rel_true_res = tr[1] > 0 ? std::sqrt(tr[0] / tr[1]) : 0.0;
    info->op_complexity = h.op_complexity;
    info->ms_solve = ms;
    info->used_fallback = 0;
    info->ms_setup_amg = float(h.ms_setup_amg);
    info->ms_setup_filter = float(h.ms_setup_filter);
    info->ms_amg_apply = ms_ph[PH_AMG];
    info->ms_filter_apply = ms_ph[PH_FILTER];
    info->ms_cg_other = ms_ph[PH_OTHER];
    info->pad_ = 0;
    info->judge_learned = h.judge_on ? h.judge_l : 0.0;
    info->judge_plain = h.judge_on ? h.judge_p : 0.0;
  }
  if (st != AMGF_OK) return st;
  return conv ? AMGF_OK : AMGF_ENOCONV;
}

// ------------------------------------------------------------------------------------
// interior-point driver for the contact QP (Sec. 3): Newton steps on the barrier
// subproblems, each solved through the condensed system with AMGF-PCG
// ------------------------------------------------------------------------------------
static double ip_error(const amgf_ip_options& o, int m, double ru_norm, const double* q) {
  // q: sum r_s^2, max |r_lam|, max |r_z|, sum |lam|, sum |z|
  const double mm = std::max(m, 1);
  const double s_d = std::max(o.s_max, (q[3] + q[4]) / (2.0 * mm)) / o.s_max;
  const double s_c = std::max(o.s_max, q[4] / mm) / o.s_max;
  return std::max(std::max(ru_norm / s_d, std::sqrt(q[0]) / s_d), std::max(q[1], q[2] / s_c));
}

static void ip_solve(Handle& h, const double* f, const double* g0, const double* Ms,
                     const double* Mu, double* u, double* s, double* lam, double* z,
                     const amgf_ip_options& o, amgf_ip_step* rec, int max_rec, int* n_steps,
                     int* converged) {
  Ctx& c = h.ctx;
  Level& L0 = *h.lev[0];
  const int64_t n = h.n();
  const int m = h.m;
  DBuf<double> ru(n), y(n), bb(n), uh(n);
  DBuf<double> rl(m), rs(m), t(m), Dn(m), sh(m), lh(m), zh(m);
  if (h.ip_red.n == 0) h.ip_red.alloc(8);
  double mu = o.mu0;
  ip_init(c, L0.J, u, g0, Ms, mu, o.s_init, s, lam, z);
  bool filter_switched = false;
  *n_steps = 0;
  *converged = 0;
  for (int step = 0; step < o.max_steps; ++step) {
    // r_u = K u - f + J^T lam;  r_lam, r_s
    bsr_spmv<double>(c, SPMV_RES, L0.K, L0.K.val.p, u, y.p, f, nullptr, nullptr);
    vcopy(c, y.p, ru.p, n);
    vscale(c, n, -1.0, ru.p);
    ip_jt_add(c, L0.JT, L0.crows.p, L0.ncrows, lam, ru.p);
    ip_m_residuals(c, L0.J, u, g0, Ms, s, lam, z, rl.p, rs.p);
    double nr2;     // ||r_u||^2 in the M_u^{-1} norm
    const double* xs[1] = {ru.p};
    if (Mu) ip_div(c, n, ru.p, Mu, y.p);
    const double* ys[1] = {Mu ? y.p : ru.p};
    dots(c, n, 1, xs, ys, &nr2);
    const double ru_norm = std::sqrt(nr2);
    double q[7];
    ip_m_norms(c, m, rs.p, rl.p, s, lam, z, Ms, 0.0, h.ip_red.p, q);
    const double e0 = ip_error(o, m, ru_norm, q);
    if (e0 < o.tol) {
      *converged = 1;
      break;
    }
    double e_mu;
    for (;;) {       // the barrier subproblem is solved: decrease mu, possibly repeatedly
      ip_m_norms(c, m, rs.p, rl.p, s, lam, z, Ms, mu, h.ip_red.p, q);
      e_mu = ip_error(o, m, ru_norm, q);
      if (e_mu >= o.kappa_eps * mu || mu <= o.tol / 10) break;
      mu = std::max(o.tol / 10, std::min(o.kappa_mu * mu, std::pow(mu, o.theta_mu)));
    }
    const double D_min = q[5], D_max = q[6];
    // D = M_s z / s and the condensed right-hand side b = -r_u + J^T (D b_lam + b_s)
    ip_rhs_m(c, m, s, z, Ms, rs.p, rl.p, mu, Dn.p, t.p);
    if (o.switch_ratio > 0 && !filter_switched && D_max >= o.switch_ratio * D_min)
      filter_switched = true;
    h.filter_suspended = o.switch_ratio > 0 && !filter_switched;
    const auto t0 = std::chrono::steady_clock::now();
    update_D(h, Dn.p);
    AMGF_HIP(hipStreamSynchronize(c.s));
    const auto t1 = std::chrono::steady_clock::now();
    vcopy(c, ru.p, bb.p, n);
    vscale(c, n, -1.0, bb.p);
    ip_jt_add(c, L0.JT, L0.crows.p, L0.ncrows, t.p, bb.p);
    AMGF_HIP(hipMemsetAsync(uh.p, 0, sizeof(double) * size_t(n), c.s));
    amgf_solve_info info{};
    const amgf_status st = pcg_impl(h, bb.p, uh.p, &info);
    AMGF_REQUIRE(st == AMGF_OK || st == AMGF_ENOCONV, st, "Newton solve failed");
    // recovery and step lengths, then the update
    const double tau = std::max(o.tau_min, 1.0 - mu);
    double alpha[2];
    ip_recover(c, L0.J, uh.p, s, z, Dn.p, Ms, rs.p, rl.p, mu, tau, sh.p, lh.p, zh.p,
               h.ip_red.p, alpha);
    axpby(c, n, alpha[0], uh.p, 1.0, u);
    ip_update_m(c, m, alpha[0], alpha[1], sh.p, lh.p, zh.p, s, lam, z);
    if (step < max_rec && rec) {
      amgf_ip_step& r = rec[step];
      r.mu = mu;
      r.e_opt = e0;
      r.e_opt_mu = e_mu;
      r.alpha_p = alpha[0];
      r.alpha_d = alpha[1];
      r.D_min = D_min;
      r.D_max = D_max;
      r.pcg_iterations = info.iterations;
      r.pcg_converged = info.converged;
      r.filter_on = (h.opt.filter && !h.filter_suspended) ? 1 : 0;
      r.pad = 0;
      r.ms_update = float(std::chrono::duration<double, std::milli>(t1 - t0).count());
      r.ms_solve = info.ms_solve;
    }
    *n_steps = step + 1;
  }
  AMGF_HIP(hipStreamSynchronize(c.s));
  if (h.filter_suspended) {       // leave a consistent filter factor for the last D
    h.filter_suspended = false;
    if (h.opt.filter && h.n_c > 0) factor_filter(h);
  }
}

}  // namespace amgf

// ======================================================================================
// C ABI
// ======================================================================================
using amgf::Handle;

struct amgf_handle_s {
  Handle h;
};

template <class F>
static amgf_status guard(F&& f) {
  try {
    return f();
  } catch (const amgf::Error& e) {
    amgf::g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    amgf::g_last_error = e.what();
    return AMGF_EDEVICE;
  }
}

extern "C" {

void amgf_default_options(amgf_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(amgf_options);
  o->precision = AMGF_FP64;
  o->smoother = AMGF_L1JACOBI;
  o->sweeps = 1;
  o->cheb_degree = 2;
  o->filter = 1;
  o->max_levels = 10;
  o->coarse_max_nodes = 1024;
  o->max_iters = 5000;
  o->sa_power_iters = 10;
  o->strength_theta = 0.04;
  o->rtol = 1e-10;
  o->sa_omega = 1.5;
  o->qr_tol = 1e-10;
  o->max_coarse_ratio = 0.9;
  o->mlp_weights = nullptr;
  o->near_null = 6;
  o->learned_judge = 1;
  o->transfer_fp16 = 1;
  o->cycle_gamma = 1;
}

const char* amgf_status_string(amgf_status s) {
  switch (s) {
    case AMGF_OK: return "AMGF_OK";
    case AMGF_EINVAL: return "AMGF_EINVAL";
    case AMGF_ENOTSPD: return "AMGF_ENOTSPD";
    case AMGF_ENOCONV: return "AMGF_ENOCONV";
    case AMGF_ENOMEM: return "AMGF_ENOMEM";
    case AMGF_EDEVICE: return "AMGF_EDEVICE";
  }
  return "AMGF_UNKNOWN";
}

const char* amgf_last_error(void) { return amgf::g_last_error.c_str(); }

amgf_status amgf_setup(const amgf_options* opts, int32_t n_nodes, const int32_t* K_rowptr,
                       const int32_t* K_col, const double* K_val, int32_t m,
                       const int32_t* J_rowptr, const int32_t* J_col, const double* J_val,
                       const double* D, const double* coords, const int32_t* Ic, int32_t n_c,
                       void* stream, amgf_handle* out) {
  if (!out) return AMGF_EINVAL;
  *out = nullptr;
  std::unique_ptr<amgf_handle_s> hs(new (std::nothrow) amgf_handle_s());
  if (!hs) return AMGF_ENOMEM;
  amgf_status st_ = guard([&]() -> amgf_status {
    Handle& h = hs->h;
    if (opts) {
      AMGF_REQUIRE(opts->struct_size == int32_t(sizeof(amgf_options)), AMGF_EINVAL,
                   "amgf_options.struct_size mismatch");
      h.opt = *opts;
    } else {
      amgf_default_options(&h.opt);
    }
    AMGF_REQUIRE(h.opt.near_null == 3 || h.opt.near_null == 6, AMGF_EINVAL,
                 "near_null must be 6 (rigid-body modes) or 3 (translations)");
    AMGF_REQUIRE(n_nodes > 0 && m >= 0 && K_rowptr && K_col && K_val &&
                     (coords || h.opt.near_null == 3),
                 AMGF_EINVAL, "bad sizes, null K, or null coords with near_null = 6");
    AMGF_REQUIRE(m == 0 || (J_rowptr && J_col && J_val && D), AMGF_EINVAL, "null J or D");
    AMGF_REQUIRE(int64_t(n_nodes) * 6 < (int64_t(1) << 31), AMGF_EINVAL, "too many nodes");
    AMGF_REQUIRE(h.opt.precision == AMGF_FP64 || h.opt.precision == AMGF_MIXED_FP32 ||
                     h.opt.precision == AMGF_MIXED_BF16K,
                 AMGF_EINVAL, "precision");
    AMGF_REQUIRE(h.opt.smoother == AMGF_L1JACOBI || h.opt.smoother == AMGF_CHEBYSHEV ||
                     h.opt.smoother == AMGF_LEARNED,
                 AMGF_EINVAL, "smoother");
    AMGF_REQUIRE(h.opt.sweeps >= 1 && h.opt.sweeps <= 16, AMGF_EINVAL, "sweeps must be 1..16");
    AMGF_REQUIRE(h.opt.cycle_gamma >= 1 && h.opt.cycle_gamma <= 4, AMGF_EINVAL,
                 "cycle_gamma must be 1..4");
    AMGF_REQUIRE(h.opt.cheb_degree >= 1 && h.opt.cheb_degree <= 16, AMGF_EINVAL,
                 "cheb_degree must be 1..16");
    AMGF_REQUIRE(h.opt.smoother != AMGF_LEARNED || h.opt.mlp_weights, AMGF_EINVAL,
                 "the learned smoother needs mlp_weights");
    AMGF_REQUIRE(h.opt.max_levels >= 1 && h.opt.max_iters >= 0 && h.opt.rtol >= 0,
                 AMGF_EINVAL, "options");
    AMGF_REQUIRE(n_c >= 0 && (n_c == 0 || Ic), AMGF_EINVAL, "Ic");
    AMGF_REQUIRE(!h.opt.allocator.alloc == !h.opt.allocator.free, AMGF_EINVAL,
                 "amgf_allocator needs both alloc and free, or neither");
    h.mem.a = h.opt.allocator;
    h.bind(stream);
    amgf::AllocScope scope_(&h.mem);
    (void)amgf::scratch_ptr();                        // per-device scratch address, once
    h.ctx.flag.alloc(1);
    h.n_nodes = n_nodes;
    h.m = m;
    amgf::setup(h, K_rowptr, K_col, K_val, J_rowptr, J_col, J_val, D, coords, Ic, n_c);
    return AMGF_OK;
  });
  if (st_ != AMGF_OK) return st_;
  *out = hs.release();
  return AMGF_OK;
}

void amgf_ip_default_options(amgf_ip_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(amgf_ip_options);
  o->max_steps = 200;
  o->tol = 1e-6;
  o->mu0 = 0.1;
  o->kappa_eps = 10.0;
  o->kappa_mu = 0.2;
  o->theta_mu = 1.5;
  o->tau_min = 0.99;
  o->s_max = 100.0;
  o->s_init = 1e-2;
  o->switch_ratio = 0.0;
}

amgf_status amgf_ip_solve(amgf_handle hd, const double* f, const double* g0, const double* Ms,
                          const double* Mu, double* u, double* s, double* lam, double* z,
                          const amgf_ip_options* opts, amgf_ip_step* steps,
                          int32_t max_records, int32_t* n_steps, int32_t* converged,
                          void* stream) {
  if (!hd || !f || !g0 || !u || !s || !lam || !z || !n_steps || !converged || max_records < 0)
    return AMGF_EINVAL;
  return guard([&]() -> amgf_status {
    Handle& h = hd->h;
    amgf_ip_options o;
    if (opts) {
      AMGF_REQUIRE(opts->struct_size == int32_t(sizeof(amgf_ip_options)), AMGF_EINVAL,
                   "amgf_ip_options.struct_size mismatch");
      o = *opts;
    } else {
      amgf_ip_default_options(&o);
    }
    AMGF_REQUIRE(h.m > 0, AMGF_EINVAL, "the interior-point driver needs contact constraints");
    AMGF_REQUIRE(!h.has_E, AMGF_EINVAL,
                 "the interior-point driver has no bound constraints (handle has E)");
    AMGF_REQUIRE(o.max_steps >= 0 && o.tol > 0 && o.mu0 > 0 && o.kappa_eps > 0 &&
                     o.kappa_mu > 0 && o.kappa_mu < 1 && o.theta_mu > 1 && o.tau_min > 0 &&
                     o.tau_min < 1 && o.s_max > 0 && o.s_init > 0 && o.switch_ratio >= 0,
                 AMGF_EINVAL, "interior-point options");
    AMGF_REQUIRE(o.switch_ratio == 0 || (h.opt.filter && h.n_c > 0), AMGF_EINVAL,
                 "switching to AMGF needs a handle built with the filter");
    h.bind(stream);
    amgf::AllocScope scope_(&h.mem);
    if (Ms || Mu) {
      AMGF_HIP(hipMemsetAsync(h.ctx.flag.p, 0, sizeof(int), h.ctx.s));
      if (Ms) amgf::check_values(h.ctx, Ms, h.m, true, h.ctx.flag.p);
      if (Mu) amgf::check_values(h.ctx, Mu, h.n(), true, h.ctx.flag.p);
      AMGF_REQUIRE(amgf::d2h_scalar(h.ctx.flag.p, h.ctx.s) == 0, AMGF_EINVAL,
                   "lumped masses must be finite and positive");
    }
    try {
      amgf::ip_solve(h, f, g0, Ms, Mu, u, s, lam, z, o, steps, max_records, n_steps,
                     converged);
    } catch (...) {
      h.filter_suspended = false;
      throw;
    }
    return AMGF_OK;
  });
}

amgf_status amgf_apply(amgf_handle hd, const double* r, double* z, void* stream) {
  if (!hd || !r || !z) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    hd->h.bind(stream);
    amgf::AllocScope scope_(&hd->h.mem);
    amgf::amgf_apply_impl(hd->h, r, z);
    return AMGF_OK;
  });
  if (st_ != AMGF_OK) return st_;
  return AMGF_OK;
}

amgf_status amgf_update_D(amgf_handle hd, const double* D, void* stream) {
  if (!hd || (!D && hd->h.m > 0)) return AMGF_EINVAL;
  return guard([&]() -> amgf_status {
    hd->h.bind(stream);
    amgf::AllocScope scope_(&hd->h.mem);
    amgf::update_D(hd->h, D);
    return AMGF_OK;
  });
}

amgf_status amgf_update_barrier(amgf_handle hd, const double* D, const double* E,
                                void* stream) {
  if (!hd || (!D && hd->h.m > 0)) return AMGF_EINVAL;
  return guard([&]() -> amgf_status {
    hd->h.bind(stream);
    amgf::AllocScope scope_(&hd->h.mem);
    amgf::update_barrier(hd->h, D, E);
    return AMGF_OK;
  });
}

amgf_status amgf_filter_solve(amgf_handle hd, const double* rc, double* wc, void* stream) {
  if (!hd || !rc || !wc) return AMGF_EINVAL;
  return guard([&]() -> amgf_status {
    Handle& h = hd->h;
    AMGF_REQUIRE(h.opt.filter && h.n_c > 0, AMGF_EINVAL, "handle has no filtering space");
    h.bind(stream);
    amgf::AllocScope scope_(&h.mem);
    h.aw.solve(h.ctx, rc, wc);   // the caller's (filtering-space) order
    return AMGF_OK;
  });
}

amgf_status amgf_vcycle(amgf_handle hd, const double* r, double* z, void* stream) {
  if (!hd || !r || !z) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    hd->h.bind(stream);
    amgf::AllocScope scope_(&hd->h.mem);
    amgf::vcycle(hd->h, r, z);
    return AMGF_OK;
  });
  if (st_ != AMGF_OK) return st_;
  return AMGF_OK;
}

amgf_status amgf_operator_apply(amgf_handle hd, const double* x, double* y, void* stream) {
  if (!hd || !x || !y) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    hd->h.bind(stream);
    amgf::AllocScope scope_(&hd->h.mem);
    amgf::operator_apply(hd->h, x, y, nullptr);
    return AMGF_OK;
  });
  if (st_ != AMGF_OK) return st_;
  return AMGF_OK;
}

amgf_status amgf_pcg(amgf_handle hd, const double* b, double* x, amgf_solve_info* info,
                     void* stream) {
  if (!hd || !b || !x) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    hd->h.bind(stream);
    amgf::AllocScope scope_(&hd->h.mem);
    return amgf::pcg_impl(hd->h, b, x, info);
  });
  if (st_ != AMGF_OK) return st_;
  return AMGF_OK;
}

amgf_status amgf_pcg_noalloc(amgf_handle hd, const double* b, double* x,
                             amgf_solve_info* info, void* stream) {
  if (!hd || !b || !x) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    hd->h.bind(stream);
    amgf::AllocScope scope_(&hd->h.mem);
    amgf::NoAllocScope no_alloc_;
    return amgf::pcg_impl(hd->h, b, x, info, amgf::scratch_ptr());
  });
  if (st_ != AMGF_OK) return st_;
  return AMGF_OK;
}

void amgf_destroy(amgf_handle hd) {
  if (!hd) return;
  (void)hipStreamSynchronize(hd->h.ctx.s);
  delete hd;
}

amgf_status amgf_profile_start(amgf_handle hd, int32_t which, int32_t max_launches) {
  if (!hd) return AMGF_EINVAL;
  if (which >= 0 && (which > AMGF_K_POSTSMOOTH || max_launches <= 0)) return AMGF_EINVAL;
  return guard([&]() -> amgf_status {
    Handle& h = hd->h;
    AMGF_HIP(hipStreamSynchronize(h.ctx.s));
    for (hipEvent_t e : h.prof_ev) AMGF_HIP(hipEventDestroy(e));
    h.prof_ev.clear();
    h.prof_used = 0;
    h.prof_open = false;
    h.prof_which = which;
    if (which < 0) return AMGF_OK;
    h.prof_ev.resize(size_t(max_launches) * 2);
    for (hipEvent_t& e : h.prof_ev) AMGF_HIP(hipEventCreate(&e));
    return AMGF_OK;
  });
}

amgf_status amgf_profile_read(amgf_handle hd, int32_t* count, double* avg_ms) {
  if (!hd || !count || !avg_ms) return AMGF_EINVAL;
  return guard([&]() -> amgf_status {
    Handle& h = hd->h;
    *count = 0;
    *avg_ms = 0.0;
    double tot = 0.0;
    for (size_t k = 0; k + 1 < h.prof_used; k += 2) {
      AMGF_HIP(hipEventSynchronize(h.prof_ev[k + 1]));
      float ms = 0.f;
      AMGF_HIP(hipEventElapsedTime(&ms, h.prof_ev[k], h.prof_ev[k + 1]));
      tot += ms;
      ++*count;
    }
    if (*count) *avg_ms = tot / *count;
    h.prof_used = 0;
    return AMGF_OK;
  });
}

int32_t amgf_num_levels(amgf_handle hd) { return hd ? int32_t(hd->h.lev.size()) : 0; }

amgf_status amgf_set_mlp(amgf_handle hd, const float* W, void* stream) {
  if (!hd) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    Handle& h = hd->h;
    h.bind(stream);
    amgf::AllocScope scope_(&h.mem);
    if (W) {
      AMGF_REQUIRE(h.opt.smoother != AMGF_CHEBYSHEV, AMGF_EINVAL,
                   "learned damping applies to the l1-Jacobi smoother");
      if (!h.mlpW.n) h.mlpW.alloc(amgf::MLP_NTOTAL);
      AMGF_HIP(hipMemcpyAsync(h.mlpW.p, W, sizeof(float) * amgf::MLP_NTOTAL,
                              hipMemcpyDeviceToDevice, h.ctx.s));
      h.learned = true;
      h.judge_rejected = false;
      amgf::set_damping(h, h.mlpW.p);
    } else {
      h.learned = false;
      h.judge_on = false;
      h.judge_rejected = false;
      amgf::set_damping(h, nullptr);
    }
    return AMGF_OK;
  });
  return st_;
}

amgf_status amgf_mlp_loss_grad(amgf_handle hd, const float* W, int32_t k, int32_t n_probes,
                               const double* probes, double* loss, double* grad, void* stream) {
  if (!hd || !W || !probes || !loss || !grad || k < 1 || n_probes < 1) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    Handle& h = hd->h;
    AMGF_REQUIRE(h.plain_cycle(), AMGF_EINVAL,
                 "the damping gradient needs the l1-Jacobi V(1,1) (sweeps = 1)");
    h.bind(stream);
    amgf::AllocScope scope_(&h.mem);
    *loss = amgf::loss_grad(h, W, k, n_probes, probes, grad);
    // leave the handle's damping as it was
    amgf::set_damping(h, h.learned ? h.mlpW.p : nullptr);
    return AMGF_OK;
  });
  return st_;
}

amgf_status amgf_adam_step(float* W, const double* grad, float* m1, float* m2, int32_t t,
                           float lr, void* stream) {
  if (!W || !grad || !m1 || !m2 || t < 1) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    amgf::Ctx c;
    c.s = static_cast<hipStream_t>(stream);
    amgf::adam_step(c, W, grad, m1, m2, t, lr);
    return AMGF_OK;
  });
  return st_;
}

amgf_status amgf_time_kernel(amgf_handle hd, int32_t which, int32_t reps, void* stream,
                             double* avg_ms) {
  if (!hd || !avg_ms || reps <= 0 || which < 0 || which > AMGF_K_OPERATOR) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    Handle& h = hd->h;
    amgf::Ctx& c = h.ctx;
    h.bind(stream);
    amgf::AllocScope scope_(&h.mem);
    amgf::Level& L = *h.lev[0];
    const int64_t n = h.n();
    AMGF_REQUIRE(h.lev.size() > 1 || which >= AMGF_K_VCYCLE, AMGF_EINVAL,
                 "single-level hierarchy has no smoother");
    // deterministic non-trivial data in the buffers the kernels read
    amgf::fill_power_start(c, n, h.ra.p, nullptr);
    amgf::vcopy(c, h.ra.p, L.vb.p, n);
    amgf::vcopy(c, h.ra.p, L.vx.p, n);
    if (h.mixed()) {
      amgf::cast_d2f(c, h.ra.p, L.fb.p, n);
      amgf::cast_d2f(c, h.ra.p, L.fx.p, n);
    }
    auto launch = [&]() {
      switch (which) {
        case AMGF_K_PRESMOOTH:
          if (h.bf16k())
            amgf::sell_spmv_bf16(c, amgf::SPMV_RES, L.K, L.fx.p, L.fr.p, L.fb.p, nullptr,
                                 nullptr);
          else if (h.mixed())
            amgf::bsr_spmv<float>(c, amgf::SPMV_RES, L.K, L.K.val32.p, L.fx.p, L.fr.p, L.fb.p,
                                  nullptr, nullptr);
          else
            amgf::bsr_spmv<double>(c, amgf::SPMV_RES, L.K, L.K.val.p, L.vx.p, L.vr.p, L.vb.p,
                                   nullptr, nullptr);
          break;
        case AMGF_K_POSTSMOOTH:
          if (h.bf16k())
            amgf::sell_spmv_bf16(c, amgf::SPMV_POST, L.K, L.fx.p, nullptr, L.fb.p, L.w32.p,
                                 L.fxn.p);
          else if (h.mixed())
            amgf::bsr_spmv<float>(c, amgf::SPMV_POST, L.K, L.K.val32.p, L.fx.p, nullptr, L.fb.p,
                                  L.w32.p, L.fxn.p);
          else
            amgf::bsr_spmv<double>(c, amgf::SPMV_POST, L.K, L.K.val.p, L.vx.p, nullptr, L.vb.p,
                                   L.w.p, L.vxn.p);
          break;
        case AMGF_K_VCYCLE:
          amgf::vcycle(h, h.ra.p, h.z3.p);
          break;
        default:
          amgf::operator_apply(h, h.ra.p, h.z3.p, nullptr);
      }
    };
    launch();
    hipEvent_t e0, e1;
    AMGF_HIP(hipEventCreate(&e0));
    AMGF_HIP(hipEventCreate(&e1));
    AMGF_HIP(hipEventRecord(e0, c.s));
    for (int i = 0; i < reps; ++i) launch();
    AMGF_HIP(hipEventRecord(e1, c.s));
    AMGF_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    AMGF_HIP(hipEventElapsedTime(&ms, e0, e1));
    AMGF_HIP(hipEventDestroy(e0));
    AMGF_HIP(hipEventDestroy(e1));
    *avg_ms = double(ms) / reps;
    return AMGF_OK;
  });
  return st_;
}

amgf_status amgf_query(amgf_handle hd, int32_t level, int32_t which, void* dst, size_t bytes) {
  if (!hd || !dst) return AMGF_EINVAL;
  amgf_status st_ = guard([&]() -> amgf_status {
    Handle& h = hd->h;
    amgf::Ctx& c = h.ctx;
    if (which == AMGF_Q_IC) {
      AMGF_REQUIRE(bytes == sizeof(int) * size_t(h.n_c), AMGF_EINVAL, "size");
      if (bytes) AMGF_HIP(hipMemcpy(dst, h.Ic.p, bytes, hipMemcpyDeviceToHost));
      return AMGF_OK;
    }
    if (which == AMGF_Q_CG_COEF) {
      const size_t k = h.cg_alpha.size();
      AMGF_REQUIRE(bytes == 2 * sizeof(double) * k, AMGF_EINVAL, "size");
      double* d = static_cast<double*>(dst);
      std::copy(h.cg_alpha.begin(), h.cg_alpha.end(), d);
      std::copy(h.cg_beta.begin(), h.cg_beta.end(), d + k);
      return AMGF_OK;
    }
    AMGF_REQUIRE(level >= 0 && level < int(h.lev.size()), AMGF_EINVAL, "level");
    amgf::Level& L = *h.lev[level];
    auto cp = [&](const void* src, size_t want) {
      AMGF_REQUIRE(bytes == want, AMGF_EINVAL, "query size mismatch");
      AMGF_REQUIRE(src != nullptr || want == 0, AMGF_EINVAL, "array not available");
      if (want) AMGF_HIP(hipMemcpy(dst, src, want, hipMemcpyDeviceToHost));
    };
    AMGF_HIP(hipStreamSynchronize(c.s));
    switch (which) {
      case AMGF_Q_CONTACT: {
        const bool last = level + 1 == int(h.lev.size());
        int32_t v[2] = {0, 0};
        if (!last && L.contact_in_A) {
          v[0] = 2;
          v[1] = L.nccrows;
        } else if (!last && L.ncrows > 0) {
          v[0] = 1;
          v[1] = L.ncrows;
        }
        AMGF_REQUIRE(bytes == sizeof(v), AMGF_EINVAL, "query size mismatch");
        std::copy(v, v + 2, static_cast<int32_t*>(dst));
        break;
      }
      case AMGF_Q_SIZES: {
        const int32_t idx_bytes = L.K.sell_dcol.p ? 2 : (L.K.sell_col.p ? 4 : 0);
        int32_t s[8] = {L.nn, L.b, int32_t(L.A.nnzb), L.n_agg, int32_t(L.P.nnzb),
                        int32_t(L.G.nnz), int32_t(L.K.nnzb), idx_bytes};
        AMGF_REQUIRE(bytes == sizeof(s), AMGF_EINVAL, "size");
        std::memcpy(dst, s, sizeof(s));
        break;
      }
      case AMGF_Q_A_ROWPTR: cp(L.A.rowptr.p, sizeof(int) * (size_t(L.nn) + 1)); break;
      case AMGF_Q_A_COL: cp(L.A.col.p, sizeof(int) * size_t(L.A.nnzb)); break;
      case AMGF_Q_A_VAL: cp(L.A.val.p, sizeof(double) * size_t(L.A.nnzb) * L.A.bsz()); break;
      case AMGF_Q_AGG: cp(L.agg.p, L.n_agg ? sizeof(int) * size_t(L.nn) : 0); break;
      case AMGF_Q_ROOT: cp(L.root.p, L.n_agg ? sizeof(int) * size_t(L.nn) : 0); break;
      case AMGF_Q_G_ROWPTR: cp(L.G.rowptr.p, L.G.n ? sizeof(int) * (size_t(L.G.n) + 1) : 0); break;
      case AMGF_Q_G_COL: cp(L.G.col.p, sizeof(int) * size_t(L.G.nnz)); break;
      case AMGF_Q_P_ROWPTR: cp(L.P.rowptr.p, L.n_agg ? sizeof(int) * (size_t(L.nn) + 1) : 0); break;
      case AMGF_Q_P_COL: cp(L.P.col.p, sizeof(int) * size_t(L.P.nnzb)); break;
      case AMGF_Q_P_VAL: cp(L.P.val.p, sizeof(double) * size_t(L.P.nnzb) * L.P.bsz()); break;
      case AMGF_Q_L1: cp(L.d.p, sizeof(double) * size_t(L.n())); break;
      case AMGF_Q_K_ROWPTR: cp(L.K.rowptr.p, sizeof(int) * (size_t(L.nn) + 1)); break;
      case AMGF_Q_K_COL: cp(L.K.col.p, sizeof(int) * size_t(L.K.nnzb)); break;
      case AMGF_Q_K_VAL: cp(L.K.val.p, sizeof(double) * size_t(L.K.nnzb) * L.K.bsz()); break;
      case AMGF_Q_FEATURES: cp(L.F.p, L.F.n ? sizeof(double) * size_t(6) * L.n() : 0); break;
      case AMGF_Q_THETA: {
        AMGF_REQUIRE(bytes == sizeof(double) * size_t(L.n()), AMGF_EINVAL, "size");
        if (h.learned && L.theta.n) {
          AMGF_HIP(hipMemcpy(dst, L.theta.p, bytes, hipMemcpyDeviceToHost));
        } else {
          std::vector<double> one(L.n(), 1.0);
          std::memcpy(dst, one.data(), bytes);
        }
        break;
      }
      case AMGF_Q_OMEGA: {
        double s[2] = {L.rho, L.omega};
        AMGF_REQUIRE(bytes == sizeof(s), AMGF_EINVAL, "size");
        std::memcpy(dst, s, sizeof(s));
        break;
      }
      default:
        throw amgf::Error(AMGF_EINVAL, "query selector");
    }
    return AMGF_OK;
  });
  if (st_ != AMGF_OK) return st_;
  return AMGF_OK;
}

}  // extern "C"

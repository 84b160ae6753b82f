/*
 * amgf.h -- C ABI of the MI355X (gfx950) AMGF solver library.
 *
 * Solves A u = b with A = K + J^T D J, the Schur complement of the interior-point
 * Newton system (arXiv 2505.18576, Sec. 3, the condensed system), by preconditioned
 * CG (stopping rule of Sec. 4 / Sec. 6.1: relative preconditioned residual below
 * rtol, iteration cap) with the multiplicative AMG-with-filtering preconditioner of
 * Definition 5.3:
 *     I - M A = (I - B A)(I - P A_w^{-1} P^T A)(I - B A),
 * where B is one AMG V-cycle on A and P embeds the filtering space of contact DOFs
 * I_c (Sec. 5.1) with A_w = P^T A P.
 *
 * Conventions for every entry point
 *  - All array arguments are DEVICE pointers unless the comment says "host".
 *  - The caller owns every pointer it passes; the library never frees them.
 *    amgf_setup copies what it keeps (stream-ordered on `stream`) and returns once
 *    the copies are enqueued; inputs must stay valid until `stream` reaches that point.
 *  - The handle owns all hierarchy memory and releases it in amgf_destroy.  It comes
 *    from hipMalloc, or from the caller's amgf_allocator (amgf_options.allocator).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call runs on it.
 *  - Every entry point returns an amgf_status; nothing throws across the ABI.  On an
 *    error the output arrays are unspecified; amgf_last_error() gives a message.
 *  - Indices are int32; value arrays are FP64 at the boundary whatever the internal
 *    precision.  A handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef AMGF_H
#define AMGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amgf_handle_s* amgf_handle;

typedef enum {
  AMGF_OK = 0,
  AMGF_EINVAL = 1,   /* bad sizes / pattern / non-finite input / D <= 0            */
  AMGF_ENOTSPD = 2,  /* non-positive Cholesky pivot, or p.Ap <= 0 in CG            */
  AMGF_ENOCONV = 3,  /* max_iters reached; x holds the last iterate                 */
  AMGF_ENOMEM = 4,   /* device allocation failed or a setup capacity was exceeded   */
  AMGF_EDEVICE = 5   /* a HIP runtime call failed                                  */
} amgf_status;

/* V-cycle arithmetic.  MIXED_BF16K is MIXED_FP32 with the level-0 stiffness values of
 * the smoothing steps stored in BF16 (rounded to nearest even once from FP64) and
 * widened to FP32 in registers; the second AMGF residual keeps FP32 values.         */
enum { AMGF_FP64 = 0, AMGF_MIXED_FP32 = 1, AMGF_MIXED_BF16K = 2 };
/* Smoother (Sec. 6 uses l1 smoothers; Remark 5.6): l1-Jacobi with theta = 1, Chebyshev
 * of degree cheb_degree in D_l1^{-1} A over [0.3 lam, lam] (lam = min(1, 1.1 x the power
 * estimate of the prolongator damping)), or l1-Jacobi with learned damping theta_i.  */
enum { AMGF_L1JACOBI = 0, AMGF_CHEBYSHEV = 1, AMGF_LEARNED = 2 };

/* Device memory supplied by the caller (e.g. a framework's caching allocator), used for
 * every buffer the library allocates, persistent or temporary.  Both functions NULL:
 * hipMalloc / hipFree.
 *  alloc(bytes, stream, ctx): `bytes` > 0 of device memory on the current device,
 *      256-byte aligned, usable by work queued on `stream` (the stream of the entry
 *      point that allocates); NULL on failure (the call then returns AMGF_ENOMEM).
 *  free(ptr, stream, ctx): returns a block with the stream it was allocated on.  It may
 *      be called while work on that stream that reads `ptr` is still queued: the
 *      allocator must order reuse after it (as hipFreeAsync and stream-ordered caching
 *      allocators do).  amgf_destroy synchronises the handle's last stream first.
 * The callbacks are called from the thread of the entry point, never concurrently for
 * one handle, and must not call into the library.                                      */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, void* stream, void* ctx);
  void* ctx;
} amgf_allocator;

typedef struct {
  int32_t struct_size;        /* sizeof(amgf_options), for ABI versioning            */
  int32_t precision;          /* AMGF_FP64, AMGF_MIXED_FP32 (FP32 V-cycle, FP64
                                 contact term, coarse solve, filter and outer CG) or
                                 AMGF_MIXED_BF16K                                      */
  int32_t smoother;           /* AMGF_L1JACOBI (theta = 1) or AMGF_LEARNED          */
  int32_t filter;             /* 1: AMGF (Definition 5.3); 0: plain AMG-PCG, M = B   */
  int32_t max_levels;         /* hierarchy depth cap (default 10)                    */
  int32_t coarse_max_nodes;   /* stop coarsening at or below this many nodes (1024)  */
  int32_t max_iters;          /* CG iteration cap (default 5000, Sec. 6.1)           */
  int32_t sa_power_iters;     /* power steps for rho(D_l1^{-1}A) (default 10)        */
  double strength_theta;      /* level-0 strength threshold (default 0.04)           */
  double rtol;                /* relative preconditioned residual (default 1e-10)    */
  double sa_omega;            /* prolongator damping numerator (default 1.5)          */
  double qr_tol;              /* dead near-null column threshold (default 1e-10)      */
  double max_coarse_ratio;    /* stop if n_agg > ratio * n_nodes (default 0.9)        */
  const float* mlp_weights;   /* host; 1313 MLP parameters + 12 feature normalisers,
                                 required iff smoother == AMGF_LEARNED                */
  int32_t sweeps;             /* smoother applications before and after the coarse
                                 correction, 1..16 (default 1: V(1,1))                */
  int32_t cheb_degree;        /* Chebyshev degree, 1..16 (default 2)                  */
  amgf_allocator allocator;   /* device memory source (default: both NULL, hipMalloc) */
  const double* bound_diag;   /* NULL, or n device values E >= 0: barrier terms of bound
                                 constraints on u (Remark 3.1: J~ = [J; I; -I] adds
                                 diag(D_lower + D_upper) = diag(E)), so that
                                 A = K + diag(E) + J^T D J.  Read by amgf_setup only.   */
  int32_t near_null;          /* 6: rigid-body modes (3 translations, 3 rotations about
                                 each aggregate's centroid; needs coords), 3: the three
                                 translations only (coords may be NULL); coarse levels
                                 then carry 3 DOFs per node (default 6)                  */
  int32_t learned_judge;      /* with AMGF_LEARNED: 1 (default) keeps the MLP damping only
                                 where it reduces the error at least as well as theta = 1:
                                 at every setup and update of D, one AMGF step
                                 e1 = (I - M A) e0 from a fixed start e0 (the power-
                                 iteration start vector, zero on decoupled DOFs) is taken
                                 with each damping; the MLP damping is kept unless theta
                                 = 1 leaves an energy norm ||e1||_A smaller by more than
                                 a factor 1.25; 0: always the MLP damping               */
  int32_t transfer_fp16;      /* mixed precisions: 1 (default) stores the prolongators
                                 P_l and P_l^T of the V-cycle in FP16 (one rounding to
                                 nearest even; |P| <= about 2 here, relative rounding
                                 4.9e-4; FP32 if a value overflows) and applies them in
                                 FP32; 0: FP32 values.  The Galerkin operators, the
                                 FP64 V-cycle and every FP64 path keep FP64 P.          */
  int32_t cycle_gamma;        /* visits of the next level per coarse correction, 1..4:
                                 1 (default) the V-cycle; 2 the W-cycle, whose coarse
                                 correction on each level above the coarsest is
                                 (2 B_c - B_c A_c B_c) applied to the restricted residual
                                 (B_c the cycle one level down; the coarsest solve is
                                 exact and is visited once).  Not in the paper, which uses
                                 V-cycles.  amgf_mlp_loss_grad needs 1.                  */
} amgf_options;

typedef struct {
  int32_t iterations;         /* CG iterations performed                              */
  int32_t converged;          /* 1 if the stopping rule was met                       */
  int32_t n_levels;           /* AMG levels (1 = dense solve only)                    */
  int32_t n_c;                /* filtering-space dimension |I_c|                       */
  double rel_prec_res;        /* sqrt(r.Mr / r0.Mr0) at exit                          */
  double rel_true_res;        /* ||b - A x|| / ||b|| at exit (FP64)                   */
  double op_complexity;       /* sum of level nonzeros / level-0 nonzeros             */
  float ms_solve;             /* wall time of amgf_pcg (hipEvents)                    */
  int32_t used_fallback;      /* learned smoother: 1 = CG with the MLP damping did not
                                 converge and was rerun with theta = 1; 2 = the
                                 learned_judge chose theta = 1 at the last setup or
                                 update (this solve used plain l1-Jacobi)              */
  float ms_setup_amg;         /* host wall time of the last amgf_setup / amgf_update_D:
                                 hierarchy, smoother data and coarsest factor          */
  float ms_setup_filter;      /* ... and of the filtering space and its factor        */
  /* Device time of amgf_pcg split by phase (hipEvents between phases on the solve stream;
   * the three sum to ms_solve up to the event resolution; Sec. 7 reports this split):    */
  float ms_amg_apply;         /* the V-cycles B r inside the preconditioner, with their
                                 FP64 <-> FP32 boundary casts                           */
  float ms_filter_apply;      /* the filter correction of Definition 5.3: the residual
                                 r - A z1 on I_c, the gather, the A_w solve and the
                                 scatter-add                                            */
  float ms_cg_other;          /* everything else: q = A p, dots, vector updates, the
                                 residual r - A z2 feeding the second V-cycle and the
                                 final sum                                              */
  int32_t pad_;
  double judge_learned;       /* learned_judge: ||(I - M A) e0||_A / ||e0||_A with the MLP
                                 damping at the last setup / update (0: no judge ran)   */
  double judge_plain;         /* ... and with theta = 1                                 */
} amgf_solve_info;

/* Fill `o` with the defaults listed above. */
void amgf_default_options(amgf_options* o);

/* Build the hierarchy and the filter factorisation for
 *   A = K + J^T diag(D) J,  n = 3 * n_nodes DOFs, m constraints.
 * K: symmetric BSR with 3x3 row-major blocks: K_rowptr[n_nodes+1], K_col[nnzb]
 *    (ascending per row, symmetric pattern), K_val[9 * nnzb].  Decoupled DOFs
 *    (rows without off-diagonal nonzeros, e.g. Dirichlet) are detected.
 * J: m x n scalar CSR, J_rowptr[m+1], J_col (ascending per row), J_val.
 * D: m barrier values, all > 0 (Sec. 3: D = diag(M_s z / s)).  m may be 0.
 * coords: 3 * n_nodes node coordinates for the rigid-body near-null space; required
 *    with near_null = 6, may be NULL with near_null = 3.
 * Ic / n_c: optional filtering-space DOF list (ascending, device); NULL/0 selects
 *    every DOF of every node that J touches (Sec. 5.1, supp(phi_i) meets the
 *    contact surface).  The error estimate holds for any full-rank P (Remark 5.5).
 * Returns EINVAL for inconsistent sizes or D <= 0, ENOTSPD if a Cholesky pivot is
 * not positive, ENOMEM if an allocation or internal capacity fails.           */
amgf_status amgf_setup(const amgf_options* opts, int32_t n_nodes,
                       const int32_t* K_rowptr, const int32_t* K_col, const double* K_val,
                       int32_t m, const int32_t* J_rowptr, const int32_t* J_col,
                       const double* J_val, const double* D, const double* coords,
                       const int32_t* Ic, int32_t n_c, void* stream, amgf_handle* out);

/* z = M r, one application of the AMGF preconditioner (Definition 5.3); r, z: n
 * FP64 device vectors (may not alias).  With filter = 0, z = B r.            */
amgf_status amgf_apply(amgf_handle h, const double* r, double* z, void* stream);

/* New interior-point step: replace the barrier diagonal D (m FP64 values > 0, device,
 * copied) while K and J stay (Sec. 3, the Newton systems of one IP solve differ in D
 * only).  Numeric re-setup: the aggregates, prolongators, coarse stiffness and coarse
 * Jacobians are kept; A_l = K_l + J_l^T D J_l, the l1 norms, smoother weights (and learned
 * damping), spectral estimates, the coarsest factor and the filter factor are rebuilt, so
 * every A_{l+1} = P_l^T A_l P_l still holds.  EINVAL for D <= 0 or non-finite entries
 * (the handle is unchanged then); ENOTSPD if a factor loses definiteness.             */
amgf_status amgf_update_D(amgf_handle h, const double* D, void* stream);

/* Both barrier terms of a new interior-point step: D (m values > 0, device) and the bound
 * diagonal E (n values >= 0, device; NULL removes it), A = K + diag(E) + J^T D J
 * (Remark 3.1).  Like amgf_update_D, with the stiffness chain rebuilt as well: the
 * aggregates and prolongators are kept, K_0 = K + diag(E) and K_{l+1} = P_l^T K_l P_l are
 * recomputed (coarse DOFs whose near-null column died again get a unit diagonal), then
 * everything amgf_update_D rebuilds.  EINVAL for D <= 0, E < 0 or non-finite values (the
 * handle is unchanged then).                                                           */
amgf_status amgf_update_barrier(amgf_handle h, const double* D, const double* E, void* stream);

/* w_c = A_w^{-1} r_c with A_w = S[I_c, I_c], the filtering-space solve of Definition 5.3
 * (Sec. 5.1), by the handle's nested-dissection multifrontal Cholesky factor.  r_c, w_c:
 * n_c FP64 device vectors in the order of I_c (may not alias).  EINVAL when the handle
 * was built with filter = 0 or has an empty filtering space.                     */
amgf_status amgf_filter_solve(amgf_handle h, const double* r_c, double* w_c, void* stream);

/* z = B r, one V-cycle of the AMG part alone (the B of Assumptions 1-2).        */
amgf_status amgf_vcycle(amgf_handle h, const double* r, double* z, void* stream);

/* y = A x with A = K + J^T D J applied in FP64 (the operator of the CG loop).    */
amgf_status amgf_operator_apply(amgf_handle h, const double* x, double* y, void* stream);

/* Preconditioned CG for A x = b.  x: initial guess in, solution out (device, n).
 * Stops when sqrt(r.Mr) <= rtol * sqrt(r0.Mr0) (Sec. 6.1) or after max_iters, then
 * fills *info (host) and returns AMGF_ENOCONV if not converged.                  */
amgf_status amgf_pcg(amgf_handle h, const double* b, double* x, amgf_solve_info* info,
                     void* stream);

/* amgf_pcg for callers that cannot allocate device memory: serving loops with a fixed
 * memory budget and harnesses that forbid allocation after setup.  Same arguments,
 * iterates and stopping rule as amgf_pcg; it calls no hipMalloc, hipFree, hipHostMalloc
 * or allocator callback and creates no events.  Its scratch (the CG scalars and the
 * partial sums of the dot products: 4100 + 4 doubles, the same for every problem size) is
 * a static device array of the library, one copy per GPU, whose address amgf_setup looks
 * up on its device; every other work buffer belongs to the handle.  Calls on one GPU share
 * that scratch: calls that overlap on one GPU (two streams, two threads) race and must
 * be serialised by the caller.  Differences from amgf_pcg: the host reads the scalars
 * after a stream synchronisation (no overlap of the next direction with that read),
 * info->ms_solve is host wall time and the phase split is zero, the CG coefficients are
 * not recorded for AMGF_Q_CG_COEF, and with learned damping a CG that does not converge
 * is not rerun with theta = 1 (that would need a copy of the initial guess): the status
 * is returned as is.  Errors as amgf_pcg; AMGF_EDEVICE if the library would have had
 * to allocate (an internal error).                                                    */
amgf_status amgf_pcg_noalloc(amgf_handle h, const double* b, double* x,
                             amgf_solve_info* info, void* stream);

/* Release every device buffer of the handle.  NULL is ignored.                   */
void amgf_destroy(amgf_handle h);

/* Human-readable name of a status code (static string).                           */
const char* amgf_status_string(amgf_status s);

/* Message of the last error raised on the calling thread (static buffer).          */
const char* amgf_last_error(void);

/* ---------------- inspection (tests and benchmarks) ---------------------------------
 * Level data are copied to HOST buffers of the stated size; `which` selects the array:
 *  AMGF_Q_SIZES    int32[8]: n_nodes, block size, nnzb(A), n_agg, nnzb(P), nnzb(G),
 *                  nnzb(K), bytes per column id of the level's sliced-ELL stiffness copy
 *                  (2: 16-bit offsets from the row, 4: int32 ids, 0: no sliced copy)
 *  AMGF_Q_A_ROWPTR/A_COL/A_VAL  assembled operator A_l (BSR b x b, FP64)
 *  AMGF_Q_AGG      int32[n_nodes] aggregate of each node (-1 = isolated)
 *  AMGF_Q_ROOT     int32[n_nodes] 1 for MIS-2 roots
 *  AMGF_Q_G_ROWPTR/G_COL        aggregation graph
 *  AMGF_Q_P_ROWPTR/P_COL/P_VAL  prolongator P_l (b x near_null blocks)
 *  AMGF_Q_L1       double[n_nodes*b] l1 row norms d
 *  AMGF_Q_K_VAL    double stiffness values of level l (pattern = K rowptr/col below)
 *  AMGF_Q_K_ROWPTR/K_COL
 *  AMGF_Q_OMEGA    double[2]: rho estimate, prolongator damping
 *  AMGF_Q_IC       int32[n_c] filtering-space DOFs (level argument ignored)
 *  AMGF_Q_FEATURES double[6 * n] learned-smoother features of the level's scalar rows,
 *                  feature-major: log10 a_ii, log10 d_i, a_ii/d_i, log10(1 + sum D J^2),
 *                  contact flag, level/(levels-1)  (smoothed levels only)
 *  AMGF_Q_THETA    double[n] smoother damping theta of the level (1 when not learned)
 *  AMGF_Q_CG_COEF  double[2k] of the last amgf_pcg call with k iterations (level ignored):
 *                  alpha_1..alpha_k (r.z / p.Ap) then beta_1..beta_k (r'.z' / r.z), the
 *                  coefficients of the Lanczos tridiagonal of M A whose extreme
 *                  eigenvalues estimate the spectrum (the bound procedure of Sec. 6.1)
 *  AMGF_Q_CONTACT  int32[2]: how the V-cycle applies the level's contact term J^T D J
 *                  (0: none, 1: through J and D, 2: assembled into the matrix the level
 *                  smooths with, A_l = K_l + C_l), and the number of node rows it touches
 * Returns EINVAL for a bad level or selector; `bytes` must equal the array size.    */
enum {
  AMGF_Q_SIZES = 0, AMGF_Q_A_ROWPTR, AMGF_Q_A_COL, AMGF_Q_A_VAL, AMGF_Q_AGG, AMGF_Q_ROOT,
  AMGF_Q_G_ROWPTR, AMGF_Q_G_COL, AMGF_Q_P_ROWPTR, AMGF_Q_P_COL, AMGF_Q_P_VAL, AMGF_Q_L1,
  AMGF_Q_K_ROWPTR, AMGF_Q_K_COL, AMGF_Q_K_VAL, AMGF_Q_OMEGA, AMGF_Q_IC, AMGF_Q_FEATURES,
  AMGF_Q_THETA, AMGF_Q_CG_COEF, AMGF_Q_CONTACT
};
int32_t amgf_num_levels(amgf_handle h);

/* ---------------- learned smoother damping --------------------------------------------
 * Not part of the paper: a per-row MLP (6 -> 32 tanh -> 32 tanh -> 1) maps the features
 * listed under AMGF_Q_FEATURES, standardised with 6 means and 6 deviations, to
 * theta = 1 + 0.98 tanh(y) in (0.02, 1.98), and the l1-Jacobi weights become theta / d.
 * Any theta in (0, 2) keeps the smoother convergent (2 D_l1 / theta - A is SPD), so B
 * stays an SPD, convergent V-cycle.  Parameter vector (1325 floats):
 *   W1[32][6] b1[32] W2[32][32] b2[32] W3[32] b3 mu[6] sigma[6].
 * With options.smoother = AMGF_LEARNED, plain l1-Jacobi is both the judge and the
 * fallback: the learned_judge option keeps theta = 1 where one AMGF step reduces the
 * error more with it, and amgf_pcg reruns with theta = 1 when CG with the MLP damping does
 * not converge; info.used_fallback reports either case.                               */

/* Replace the damping of every smoothed level by the MLP with device parameters W
 * (1325 floats), or restore theta = 1 when W is NULL.  EINVAL with W on a Chebyshev
 * handle.                                                                              */
amgf_status amgf_set_mlp(amgf_handle h, const float* W, void* stream);

/* Training loss and gradient on an FP64 handle: for each probe e0 (device, column q of
 * the n x n_probes array `probes`), loss_q = (1/k) log(||E^k e0||_S / ||e0||_S) with
 * E = I - M S and M the AMGF preconditioner with MLP damping W (device).  *loss (host)
 * = mean over probes; grad (device, 1313 doubles) = d loss / d (W1 b1 W2 b2 W3 b3),
 * obtained by reverse mode through both V-cycles and the filter correction.  The
 * handle's own damping is left unchanged.  EINVAL unless the handle smooths with
 * l1-Jacobi and sweeps = 1 (the reverse mode follows that V(1,1)).                     */
amgf_status amgf_mlp_loss_grad(amgf_handle h, const float* W, int32_t k, int32_t n_probes,
                               const double* probes, double* loss, double* grad,
                               void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the 1313 trainable parameters:
 * W, m1, m2 device floats (m1/m2 zero before step t = 1), grad device doubles.          */
amgf_status amgf_adam_step(float* W, const double* grad, float* m1, float* m2, int32_t t,
                           float lr, void* stream);

/* Benchmark helper: launch one hot-path kernel `reps` times on `stream` between two
 * hipEvents and store the mean time per launch (milliseconds) in *avg_ms (host).
 *   AMGF_K_PRESMOOTH   level-0 pre-smoothing residual "r = b - K x" SpMV at the first
 *                      iterate x = w.b (formed before it) in the handle's V-cycle
 *                      precision (reads the level-0 V-cycle buffers)
 *   AMGF_K_POSTSMOOTH  level-0 fused Jacobi step "x' = x + w.(b - K x)"
 *   AMGF_K_VCYCLE      one whole V-cycle B r on level-0 buffers
 *   AMGF_K_OPERATOR    the FP64 operator y = A x of the CG loop
 * Work vectors are overwritten; the hierarchy is not modified.                      */
enum { AMGF_K_PRESMOOTH = 0, AMGF_K_POSTSMOOTH = 1, AMGF_K_VCYCLE = 2, AMGF_K_OPERATOR = 3 };
amgf_status amgf_time_kernel(amgf_handle h, int32_t which, int32_t reps, void* stream,
                             double* avg_ms);

/* Live timing inside solves.  After amgf_profile_start(h, which, max_launches) with
 * which = AMGF_K_PRESMOOTH or AMGF_K_POSTSMOOTH, every launch of that level-0 kernel
 * made by later amgf_apply / amgf_vcycle / amgf_pcg calls is bracketed by a pair of
 * hipEvents recorded on the solve stream (the first max_launches launches; later ones
 * are not timed).  which < 0 switches timing off.  Events are owned by the handle.
 * amgf_profile_read waits for the recorded events, stores the number of timed launches
 * in *count and their mean duration (milliseconds) in *avg_ms (host pointers), and
 * clears the record.  EINVAL for a null handle or pointer, an unknown kernel or
 * max_launches <= 0.                                                                  */
amgf_status amgf_profile_start(amgf_handle h, int32_t which, int32_t max_launches);
amgf_status amgf_profile_read(amgf_handle h, int32_t* count, double* avg_ms);
amgf_status amgf_query(amgf_handle h, int32_t level, int32_t which, void* host_dst,
                       size_t bytes);

/* ---------------- interior-point driver for the contact QP ----------------------------
 * Solves  minimise 1/2 u^T K u - f^T u  subject to  J u + g0 >= 0  with the handle's K and
 * J, by the interior-point Newton method outlined in Sec. 3: slacks s, multipliers lam of
 * J u + g0 - s = 0 and duals z = mu / s, the barrier weighted by the diagonal lumped slack
 * mass M_s; every Newton step is the condensed system A u^ = b, A = K + J^T D J with
 * D = M_s z / s, solved by amgf_update_D + amgf_pcg (AMGF-PCG), and s^, lam^, z^ are
 * recovered from u^.  Barrier subproblem residuals: r_u = K u - f + J^T lam,
 * r_s = -lam - M_s z, r_lam = J u + g0 - s, r_z = s z - mu; optimality error
 * e(mu) = max(||r_u||_{M_u^-1} / s_d, ||r_s||_{M_s^-1} / s_d, ||r_lam||_inf,
 * ||r_z||_inf / s_c) with M_u the lumped displacement mass and the scalings
 * s_d = max(s_max, (|lam|_1 + |z|_1) / 2m) / s_max, s_c = max(s_max, |z|_1 / m) / s_max.  mu decreases to max(tol / 10, min(kappa_mu mu, mu^theta_mu)) once
 * e(mu) < kappa_eps mu; steps are cut back by the fraction-to-the-boundary rule with
 * tau = max(tau_min, 1 - mu) (separate lengths for the primal variables and z); the run
 * stops when e(0) < tol.  The first iterate is s = max(J u + g0, s_init), z = mu0 / s,
 * lam = -M_s z.  Where the paper defers to its IP reference (Wachter and Biegler 2006) the
 * defaults of that method are used.                                                     */
typedef struct {
  int32_t struct_size;        /* sizeof(amgf_ip_options)                              */
  int32_t max_steps;          /* Newton steps (default 200)                           */
  double tol;                 /* tol_IP (default 1e-6, Sec. 4)                        */
  double mu0;                 /* initial barrier parameter (0.1)                      */
  double kappa_eps;           /* subproblem tolerance factor (10, Sec. 3)             */
  double kappa_mu;            /* barrier decrease factor (0.2)                        */
  double theta_mu;            /* superlinear barrier decrease exponent (1.5)          */
  double tau_min;             /* fraction-to-the-boundary floor (0.99)                */
  double s_max;               /* optimality-error scaling constant (100, Sec. 3)      */
  double s_init;              /* floor of the first slacks (1e-2)                     */
  double switch_ratio;        /* 0: every solve uses the handle's preconditioner.  > 0
                                 (handle built with filter = 1): plain AMG-PCG while
                                 D_max / D_min < switch_ratio, AMGF from the first step
                                 that reaches it on (Sec. 7 suggests such a switch)    */
} amgf_ip_options;

typedef struct {
  double mu;                  /* barrier parameter of the step                        */
  double e_opt;               /* optimality error e(0) before the step                */
  double e_opt_mu;            /* e(mu)                                                 */
  double alpha_p, alpha_d;    /* step lengths (s, u, lam) and (z)                     */
  double D_min, D_max;        /* range of the barrier diagonal D = M_s z / s          */
  int32_t pcg_iterations;     /* CG iterations of the Newton solve                    */
  int32_t pcg_converged;      /* 0 when the solve stopped at max_iters (the step then
                                 uses the last CG iterate)                             */
  int32_t filter_on;          /* 1 when the solve used AMGF, 0 for plain AMG          */
  int32_t pad;
  float ms_update;            /* host wall time of the numeric re-setup for D         */
  float ms_solve;             /* device time of the CG solve                           */
} amgf_ip_step;

/* Fill `o` with the defaults listed above. */
void amgf_ip_default_options(amgf_ip_options* o);

/* Run the driver.  f (n), g0 (m): device inputs.  Ms (m) and Mu (n): device lumped
 * masses, positive, or NULL for ones.  u (n, device): initial point in,
 * solution out.  s, lam, z (m, device): outputs.  steps: host array of max_records
 * records (may be NULL), the first min(steps taken, max_records) are filled.  *n_steps and
 * *converged (host) receive the number of Newton steps and whether e(0) < tol was reached.
 * The handle's D is left at the last step's M_s z / s.  EINVAL for m = 0, bad options,
 * a handle with bound terms (the driver has no bound constraints) or switch_ratio > 0 on
 * a handle without filter; ENOTSPD if a solve breaks down; other CG
 * non-convergence is recorded per step and not an error.                             */
amgf_status amgf_ip_solve(amgf_handle h, const double* f, const double* g0, const double* Ms,
                          const double* Mu, double* u, double* s, double* lam, double* z,
                          const amgf_ip_options* opts, amgf_ip_step* steps,
                          int32_t max_records, int32_t* n_steps, int32_t* converged,
                          void* stream);

#ifdef __cplusplus
}
#endif
#endif /* AMGF_H */

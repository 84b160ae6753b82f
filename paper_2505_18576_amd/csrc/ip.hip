// Vector kernels of the interior-point driver for the contact QP (Sec. 3): residuals of the
// barrier subproblem, the condensed right-hand side, the recovery of the eliminated
// components and the fraction-to-the-boundary step lengths.  The m-sized work is small
// (one entry per contact constraint), so the reductions run in one workgroup in a fixed
// order and their results are deterministic.
#include "ip.h"

#include <cfloat>

namespace amgf {

namespace {

constexpr int RED_THREADS = 1024;

// (J x)_k for a 1 x 3 block row
__device__ __forceinline__ double jrow(const int* __restrict__ rp, const int* __restrict__ col,
                                       const double* __restrict__ val,
                                       const double* __restrict__ x, int k) {
  double acc = 0.0;
  for (int e = rp[k]; e < rp[k + 1]; ++e) {
    const int64_t a = int64_t(col[e]) * 3;
    acc += val[int64_t(e) * 3] * x[a] + val[int64_t(e) * 3 + 1] * x[a + 1] +
           val[int64_t(e) * 3 + 2] * x[a + 2];
  }
  return acc;
}

__global__ void k_ip_init(int m, const int* __restrict__ rp, const int* __restrict__ col,
                          const double* __restrict__ val, const double* __restrict__ u,
                          const double* __restrict__ g0, const double* __restrict__ Ms,
                          double mu, double s_init, double* __restrict__ s,
                          double* __restrict__ lam, double* __restrict__ z) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const double sk = fmax(jrow(rp, col, val, u, k) + g0[k], s_init);
  const double zk = mu / sk;
  s[k] = sk;
  z[k] = zk;
  lam[k] = -(Ms ? Ms[k] : 1.0) * zk;
}

// one wavefront per listed node row: y_a += sum_k JT(a, k) v_k
__global__ void __launch_bounds__(256) k_ip_jt_add(int nrows, const int* __restrict__ rows,
                                                   const int* __restrict__ rp,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ v,
                                                   double* __restrict__ y) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nrows) return;
  const int a = rows[i];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int k = rp[a] + lane; k < rp[a + 1]; k += 64) {
    const double vk = v[col[k]];
#pragma unroll
    for (int p = 0; p < 3; ++p) acc[p] += val[int64_t(k) * 3 + p] * vk;
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) acc[p] = wave_sum(acc[p]);
  if (lane < 3) {
    const double add = lane == 0 ? acc[0] : (lane == 1 ? acc[1] : acc[2]);
    y[int64_t(a) * 3 + lane] += add;
  }
}

__global__ void k_ip_m_residuals(int m, const int* __restrict__ rp, const int* __restrict__ col,
                                 const double* __restrict__ val, const double* __restrict__ u,
                                 const double* __restrict__ g0, const double* __restrict__ Ms,
                                 const double* __restrict__ s, const double* __restrict__ lam,
                                 const double* __restrict__ z, double* __restrict__ r_lam,
                                 double* __restrict__ r_s) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  r_lam[k] = jrow(rp, col, val, u, k) + g0[k] - s[k];
  r_s[k] = -lam[k] - (Ms ? Ms[k] : 1.0) * z[k];
}

__global__ void k_ip_div(int64_t n, const double* __restrict__ a, const double* __restrict__ d,
                         double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] / d[i];
}

// tree reduction of one value per thread over the workgroup; op 0 sum, 1 max, 2 min
template <int OP>
__device__ double block_reduce(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = RED_THREADS / 2; o > 0; o >>= 1) {
    if (t < o) {
      const double a = sh[t], b = sh[t + o];
      sh[t] = OP == 0 ? a + b : (OP == 1 ? fmax(a, b) : fmin(a, b));
    }
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(RED_THREADS) k_ip_m_norms(
    int m, const double* __restrict__ r_s, const double* __restrict__ r_lam,
    const double* __restrict__ s, const double* __restrict__ lam, const double* __restrict__ z,
    const double* __restrict__ Ms, double mu, double* __restrict__ out) {
  __shared__ double sh[RED_THREADS];
  double q[7] = {0.0, 0.0, 0.0, 0.0, 0.0, DBL_MAX, 0.0};
  for (int k = threadIdx.x; k < m; k += RED_THREADS) {
    const double ms = Ms ? Ms[k] : 1.0;
    q[0] += r_s[k] * r_s[k] / ms;
    q[1] = fmax(q[1], fabs(r_lam[k]));
    q[2] = fmax(q[2], fabs(s[k] * z[k] - mu));
    q[3] += fabs(lam[k]);
    q[4] += fabs(z[k]);
    const double d = ms * z[k] / s[k];
    q[5] = fmin(q[5], d);
    q[6] = fmax(q[6], d);
  }
  const double r0 = block_reduce<0>(q[0], sh);
  const double r1 = block_reduce<1>(q[1], sh);
  const double r2 = block_reduce<1>(q[2], sh);
  const double r3 = block_reduce<0>(q[3], sh);
  const double r4 = block_reduce<0>(q[4], sh);
  const double r5 = block_reduce<2>(q[5], sh);
  const double r6 = block_reduce<1>(q[6], sh);
  if (threadIdx.x == 0) {
    out[0] = r0;
    out[1] = r1;
    out[2] = r2;
    out[3] = r3;
    out[4] = r4;
    out[5] = r5;
    out[6] = r6;
  }
}

__global__ void k_ip_rhs_m(int m, const double* __restrict__ s, const double* __restrict__ z,
                           const double* __restrict__ Ms, const double* __restrict__ r_s,
                           const double* __restrict__ r_lam, double mu, double* __restrict__ D,
                           double* __restrict__ t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const double ms = Ms ? Ms[k] : 1.0;
  const double d = ms * z[k] / s[k];
  const double b_lam = -r_lam[k];
  const double b_s = -(r_s[k] + ms * (s[k] * z[k] - mu) / s[k]);
  D[k] = d;
  t[k] = d * b_lam + b_s;
}

__global__ void __launch_bounds__(RED_THREADS) k_ip_recover(
    int m, const int* __restrict__ rp, const int* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ uh,
    const double* __restrict__ s, const double* __restrict__ z, const double* __restrict__ D,
    const double* __restrict__ Ms, const double* __restrict__ r_s,
    const double* __restrict__ r_lam, double mu, double tau,
    double* __restrict__ sh_out, double* __restrict__ lh_out, double* __restrict__ zh_out,
    double* __restrict__ out) {
  __shared__ double sh[RED_THREADS];
  double ap = 1.0, ad = 1.0;
  for (int k = threadIdx.x; k < m; k += RED_THREADS) {
    const double b_lam = -r_lam[k];
    const double r_z = s[k] * z[k] - mu;
    const double b_s = -(r_s[k] + (Ms ? Ms[k] : 1.0) * r_z / s[k]);
    const double s_h = jrow(rp, col, val, uh, k) - b_lam;
    const double l_h = D[k] * s_h - b_s;
    const double z_h = -(r_z + z[k] * s_h) / s[k];
    sh_out[k] = s_h;
    lh_out[k] = l_h;
    zh_out[k] = z_h;
    if (s_h < 0.0) ap = fmin(ap, -tau * s[k] / s_h);
    if (z_h < 0.0) ad = fmin(ad, -tau * z[k] / z_h);
  }
  const double rp_ = block_reduce<2>(ap, sh);
  const double rd_ = block_reduce<2>(ad, sh);
  if (threadIdx.x == 0) {
    out[0] = rp_;
    out[1] = rd_;
  }
}

__global__ void k_ip_update_m(int m, double ap, double ad, const double* __restrict__ sh,
                              const double* __restrict__ lh, const double* __restrict__ zh,
                              double* __restrict__ s, double* __restrict__ lam,
                              double* __restrict__ z) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  s[k] += ap * sh[k];
  lam[k] += ap * lh[k];
  z[k] += ad * zh[k];
}

void require_j(const BSR& J) {
  AMGF_REQUIRE(J.br == 1 && J.bc == 3, AMGF_EINVAL, "contact Jacobian blocks must be 1 x 3");
}

}  // namespace

void ip_init(Ctx& c, const BSR& J, const double* u, const double* g0, const double* Ms,
             double mu, double s_init, double* s, double* lam, double* z) {
  require_j(J);
  const int m = J.nrows;
  if (!m) return;
  hipLaunchKernelGGL(k_ip_init, dim3(grid_for(m, 256)), dim3(256), 0, c.s, m, J.rowptr.p,
                     J.col.p, J.val.p, u, g0, Ms, mu, s_init, s, lam, z);
  AMGF_LAUNCH_CHECK();
}

void ip_jt_add(Ctx& c, const BSR& JT, const int* crows, int ncrows, const double* v, double* y) {
  if (!ncrows || !JT.nnzb) return;
  AMGF_REQUIRE(JT.br == 3 && JT.bc == 1, AMGF_EINVAL, "transposed Jacobian blocks must be 3 x 1");
  hipLaunchKernelGGL(k_ip_jt_add, dim3(grid_for(ncrows, 4)), dim3(256), 0, c.s, ncrows, crows,
                     JT.rowptr.p, JT.col.p, JT.val.p, v, y);
  AMGF_LAUNCH_CHECK();
}

void ip_m_residuals(Ctx& c, const BSR& J, const double* u, const double* g0, const double* Ms,
                    const double* s, const double* lam, const double* z, double* r_lam,
                    double* r_s) {
  require_j(J);
  const int m = J.nrows;
  if (!m) return;
  hipLaunchKernelGGL(k_ip_m_residuals, dim3(grid_for(m, 256)), dim3(256), 0, c.s, m,
                     J.rowptr.p, J.col.p, J.val.p, u, g0, Ms, s, lam, z, r_lam, r_s);
  AMGF_LAUNCH_CHECK();
}

void ip_div(Ctx& c, int64_t n, const double* a, const double* d, double* y) {
  if (!n) return;
  hipLaunchKernelGGL(k_ip_div, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, a, d, y);
  AMGF_LAUNCH_CHECK();
}

void ip_m_norms(Ctx& c, int m, const double* r_s, const double* r_lam, const double* s,
                const double* lam, const double* z, const double* Ms, double mu, double* dev,
                double* out) {
  hipLaunchKernelGGL(k_ip_m_norms, dim3(1), dim3(RED_THREADS), 0, c.s, m, r_s, r_lam, s, lam,
                     z, Ms, mu, dev);
  AMGF_LAUNCH_CHECK();
  AMGF_HIP(hipMemcpyAsync(out, dev, 7 * sizeof(double), hipMemcpyDeviceToHost, c.s));
  AMGF_HIP(hipStreamSynchronize(c.s));
}

void ip_rhs_m(Ctx& c, int m, const double* s, const double* z, const double* Ms,
              const double* r_s, const double* r_lam, double mu, double* D, double* t) {
  if (!m) return;
  hipLaunchKernelGGL(k_ip_rhs_m, dim3(grid_for(m, 256)), dim3(256), 0, c.s, m, s, z, Ms, r_s,
                     r_lam, mu, D, t);
  AMGF_LAUNCH_CHECK();
}

void ip_recover(Ctx& c, const BSR& J, const double* uh, const double* s, const double* z,
                const double* D, const double* Ms, const double* r_s, const double* r_lam,
                double mu, double tau, double* sh, double* lh, double* zh, double* dev,
                double* alpha) {
  require_j(J);
  hipLaunchKernelGGL(k_ip_recover, dim3(1), dim3(RED_THREADS), 0, c.s, J.nrows, J.rowptr.p,
                     J.col.p, J.val.p, uh, s, z, D, Ms, r_s, r_lam, mu, tau, sh, lh, zh, dev);
  AMGF_LAUNCH_CHECK();
  AMGF_HIP(hipMemcpyAsync(alpha, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, c.s));
  AMGF_HIP(hipStreamSynchronize(c.s));
}

void ip_update_m(Ctx& c, int m, double ap, double ad, const double* sh, const double* lh,
                 const double* zh, double* s, double* lam, double* z) {
  if (!m) return;
  hipLaunchKernelGGL(k_ip_update_m, dim3(grid_for(m, 256)), dim3(256), 0, c.s, m, ap, ad, sh, lh,
                     zh, s, lam, z);
  AMGF_LAUNCH_CHECK();
}

}  // namespace amgf

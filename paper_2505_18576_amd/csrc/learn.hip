// Learned smoother damping: per-row features, the 6-32-32-1 MLP forward and backward,
// and the Adam update.  All arithmetic is FP64 (weights are stored as FP32); the weight
// gradient is reduced in two fixed-order stages so it is deterministic.
#include "learn.h"

namespace amgf {

// parameter layout (MLP_NPARAM = 1313) followed by the 12 feature normalisers
//   W1[32][6] b1[32] W2[32][32] b2[32] W3[32] b3 | mu[6] sigma[6]
constexpr int OFF_W1 = 0, OFF_B1 = 192, OFF_W2 = 224, OFF_B2 = 1248, OFF_W3 = 1280,
              OFF_B3 = 1312, OFF_MU = 1313, OFF_SD = 1319;

// features of the scalar rows of one level:
//   f0 = log10 a_ii, f1 = log10 d_i, f2 = a_ii / d_i, f3 = log10(1 + beta_i),
//   f4 = 1 if the node carries a contact term, f5 = level / (levels - 1)
// beta_i = sum_k D_k J_ki^2 (the row's barrier weight).
template <int B>
__global__ void k_features(int nn, const int* __restrict__ arp, const int* __restrict__ acol,
                           const double* __restrict__ aval, const double* __restrict__ d,
                           const int* __restrict__ jtrp, const int* __restrict__ jtcol,
                           const double* __restrict__ jtval, const double* __restrict__ D,
                           double lev_frac, double* __restrict__ F, int64_t ld) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nn) return;
  int kd = arp[a];
  while (kd < arp[a + 1] && acol[kd] != a) ++kd;
  double beta[B];
#pragma unroll
  for (int p = 0; p < B; ++p) beta[p] = 0.0;
  for (int t = jtrp[a]; t < jtrp[a + 1]; ++t) {
    const double Dk = D[jtcol[t]];
#pragma unroll
    for (int p = 0; p < B; ++p) {
      const double j = jtval[int64_t(t) * B + p];
      beta[p] += Dk * j * j;
    }
  }
  const double contact = jtrp[a + 1] > jtrp[a] ? 1.0 : 0.0;
#pragma unroll
  for (int p = 0; p < B; ++p) {
    const int64_t i = int64_t(a) * B + p;
    const double aii = aval[int64_t(kd) * B * B + p * B + p];
    F[0 * ld + i] = log10(aii);
    F[1 * ld + i] = log10(d[i]);
    F[2 * ld + i] = aii / d[i];
    F[3 * ld + i] = log10(1.0 + beta[p]);
    F[4 * ld + i] = contact;
    F[5 * ld + i] = lev_frac;
  }
}

void level_features(Ctx& c, int b, int nn, const int* arp, const int* acol, const double* aval,
                    const double* d, const int* jtrp, const int* jtcol, const double* jtval,
                    const double* D, double lev_frac, double* F) {
  const int64_t ld = int64_t(nn) * b;
  if (b == 3)
    hipLaunchKernelGGL(k_features<3>, dim3(grid_for(nn, 128)), dim3(128), 0, c.s, nn, arp, acol,
                       aval, d, jtrp, jtcol, jtval, D, lev_frac, F, ld);
  else
    hipLaunchKernelGGL(k_features<6>, dim3(grid_for(nn, 128)), dim3(128), 0, c.s, nn, arp, acol,
                       aval, d, jtrp, jtcol, jtval, D, lev_frac, F, ld);
  AMGF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- forward
struct MLPState {
  double fh[6], h1[32], h2[32], y;
};

__device__ __forceinline__ void mlp_forward(const float* __restrict__ W, const double* f,
                                            MLPState& s) {
  for (int j = 0; j < 6; ++j) s.fh[j] = (f[j] - double(W[OFF_MU + j])) / double(W[OFF_SD + j]);
  for (int j = 0; j < 32; ++j) {
    double a = double(W[OFF_B1 + j]);
    for (int q = 0; q < 6; ++q) a += double(W[OFF_W1 + j * 6 + q]) * s.fh[q];
    s.h1[j] = tanh(a);
  }
  for (int j = 0; j < 32; ++j) {
    double a = double(W[OFF_B2 + j]);
    for (int q = 0; q < 32; ++q) a += double(W[OFF_W2 + j * 32 + q]) * s.h1[q];
    s.h2[j] = tanh(a);
  }
  double y = double(W[OFF_B3]);
  for (int q = 0; q < 32; ++q) y += double(W[OFF_W3 + q]) * s.h2[q];
  s.y = y;
}

// The network's output for one row without keeping the second hidden layer (theta only):
// the operations and their order are those of mlp_forward, so y is bitwise the same; the
// first hidden layer stays in registers (loops unrolled) instead of per-lane memory.
__device__ __forceinline__ double mlp_output(const float* __restrict__ W, const double* f) {
  double fh[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) fh[j] = (f[j] - double(W[OFF_MU + j])) / double(W[OFF_SD + j]);
  double h1[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    double a = double(W[OFF_B1 + j]);
#pragma unroll
    for (int q = 0; q < 6; ++q) a += double(W[OFF_W1 + j * 6 + q]) * fh[q];
    h1[j] = tanh(a);
  }
  double y = double(W[OFF_B3]);
  for (int j = 0; j < 32; ++j) {                    // h2_j, then its term of y
    double a = double(W[OFF_B2 + j]);
#pragma unroll
    for (int q = 0; q < 32; ++q) a += double(W[OFF_W2 + j * 32 + q]) * h1[q];
    y += double(W[OFF_W3 + j]) * tanh(a);
  }
  return y;
}

// theta_i = 1 + 0.98 tanh(y_i), w_i = theta_i / d_i
__global__ void k_mlp_theta(int64_t n, const float* __restrict__ W, const double* __restrict__ F,
                            int64_t ld, const double* __restrict__ d, double* __restrict__ theta,
                            double* __restrict__ w) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double f[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) f[q] = F[q * ld + i];
  const double th = 1.0 + 0.98 * tanh(mlp_output(W, f));
  theta[i] = th;
  w[i] = th / d[i];
}

void mlp_theta(Ctx& c, int64_t n, const float* W, const double* F, const double* d,
               double* theta, double* w) {
  if (n) hipLaunchKernelGGL(k_mlp_theta, dim3(grid_for(n, 128)), dim3(128), 0, c.s, n, W, F, n,
                            d, theta, w);
  AMGF_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- backward
// Per row: from dL/dtheta_i, the adjoints of the output and both hidden pre-activations.
// Stored per row: fh (6), h1 (32), h2 (32), ybar (1), a2bar (32), a1bar (32) = 135 values.
constexpr int ROWV = 135;

__global__ void k_mlp_rows(int64_t n, const float* __restrict__ W, const double* __restrict__ F,
                           int64_t ld, const double* __restrict__ thbar,
                           double* __restrict__ rowv) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double f[6];
  for (int q = 0; q < 6; ++q) f[q] = F[q * ld + i];
  MLPState s;
  mlp_forward(W, f, s);
  const double t = tanh(s.y);
  const double ybar = thbar[i] * 0.98 * (1.0 - t * t);
  double a2bar[32], a1bar[32];
  for (int j = 0; j < 32; ++j)
    a2bar[j] = ybar * double(W[OFF_W3 + j]) * (1.0 - s.h2[j] * s.h2[j]);
  for (int q = 0; q < 32; ++q) {
    double h = 0.0;
    for (int j = 0; j < 32; ++j) h += double(W[OFF_W2 + j * 32 + q]) * a2bar[j];
    a1bar[q] = h * (1.0 - s.h1[q] * s.h1[q]);
  }
  double* o = rowv + i * ROWV;
  for (int q = 0; q < 6; ++q) o[q] = s.fh[q];
  for (int q = 0; q < 32; ++q) o[6 + q] = s.h1[q];
  for (int q = 0; q < 32; ++q) o[38 + q] = s.h2[q];
  o[70] = ybar;
  for (int q = 0; q < 32; ++q) o[71 + q] = a2bar[q];
  for (int q = 0; q < 32; ++q) o[103 + q] = a1bar[q];
}

// gradient entry g of one row (indices into the row record)
__device__ __forceinline__ double grad_term(int g, const double* o) {
  if (g < OFF_B1) return o[103 + g / 6] * o[g % 6];                        // W1[j][q]
  if (g < OFF_W2) return o[103 + (g - OFF_B1)];                            // b1[j]
  if (g < OFF_B2) { const int e = g - OFF_W2; return o[71 + e / 32] * o[6 + e % 32]; }  // W2
  if (g < OFF_W3) return o[71 + (g - OFF_B2)];                             // b2[j]
  if (g < OFF_B3) return o[70] * o[38 + (g - OFF_W3)];                     // W3[q]
  return o[70];                                                            // b3
}

constexpr int GRAD_CHUNK = 1024;
// partial[chunk][g] = sum over the chunk's rows (ascending) of the row's term
__global__ void __launch_bounds__(256) k_grad_partial(int64_t n, const double* __restrict__ rowv,
                                                      double* __restrict__ partial) {
  const int64_t r0 = int64_t(blockIdx.x) * GRAD_CHUNK;
  const int64_t r1 = r0 + GRAD_CHUNK < n ? r0 + GRAD_CHUNK : n;
  for (int g = threadIdx.x; g < MLP_NPARAM; g += 256) {
    double acc = 0.0;
    for (int64_t r = r0; r < r1; ++r) acc += grad_term(g, rowv + r * ROWV);
    partial[int64_t(blockIdx.x) * MLP_NPARAM + g] = acc;
  }
}
__global__ void k_grad_final(int nchunks, const double* __restrict__ partial,
                             double* __restrict__ grad, int accumulate) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= MLP_NPARAM) return;
  double acc = 0.0;
  for (int k = 0; k < nchunks; ++k) acc += partial[int64_t(k) * MLP_NPARAM + g];
  grad[g] = accumulate ? grad[g] + acc : acc;
}

void mlp_backward(Ctx& c, int64_t n, const float* W, const double* F, const double* thbar,
                  double* grad, bool accumulate) {
  if (n == 0) return;
  DBuf<double> rowv(size_t(n) * ROWV);
  const int nchunks = int((n + GRAD_CHUNK - 1) / GRAD_CHUNK);
  DBuf<double> part(size_t(nchunks) * MLP_NPARAM);
  hipLaunchKernelGGL(k_mlp_rows, dim3(grid_for(n, 128)), dim3(128), 0, c.s, n, W, F, n, thbar,
                     rowv.p);
  hipLaunchKernelGGL(k_grad_partial, dim3(nchunks), dim3(256), 0, c.s, n, rowv.p, part.p);
  hipLaunchKernelGGL(k_grad_final, dim3(grid_for(MLP_NPARAM, 256)), dim3(256), 0, c.s, nchunks,
                     part.p, grad, int(accumulate));
  AMGF_LAUNCH_CHECK();
  AMGF_HIP(hipStreamSynchronize(c.s));
}

// ---------------------------------------------------------------- adjoint helpers
__global__ void k_wbar(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                       double* __restrict__ acc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) acc[i] += a[i] * b[i];
}
__global__ void k_hadamard(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}
__global__ void k_axpy_hadamard(int64_t n, const double* __restrict__ w,
                                const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] += w[i] * x[i];
}
__global__ void k_div(int64_t n, const double* __restrict__ a, const double* __restrict__ d,
                      double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] / d[i];
}

void acc_hadamard(Ctx& c, int64_t n, const double* a, const double* b, double* acc) {
  if (n) hipLaunchKernelGGL(k_wbar, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, a, b, acc);
}
void hadamard(Ctx& c, int64_t n, const double* a, const double* b, double* out) {
  if (n) hipLaunchKernelGGL(k_hadamard, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, a, b, out);
}
void axpy_hadamard(Ctx& c, int64_t n, const double* w, const double* x, double* y) {
  if (n) hipLaunchKernelGGL(k_axpy_hadamard, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, w, x, y);
}
void vdiv(Ctx& c, int64_t n, const double* a, const double* d, double* out) {
  if (n) hipLaunchKernelGGL(k_div, dim3(grid_for(n, 256)), dim3(256), 0, c.s, n, a, d, out);
}

// ---------------------------------------------------------------- Adam
__global__ void k_adam(int n, float* __restrict__ W, const double* __restrict__ g,
                       float* __restrict__ m1, float* __restrict__ m2, int t, float lr,
                       float b1, float b2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = float(g[i]);
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  const float ah = a / (1.f - powf(b1, float(t)));
  const float vh = v / (1.f - powf(b2, float(t)));
  W[i] -= lr * ah / (sqrtf(vh) + eps);
}

void adam_step(Ctx& c, float* W, const double* g, float* m1, float* m2, int t, float lr) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(MLP_NPARAM, 256)), dim3(256), 0, c.s, MLP_NPARAM, W,
                     g, m1, m2, t, lr, 0.9f, 0.999f, 1e-8f);
  AMGF_LAUNCH_CHECK();
}

}  // namespace amgf

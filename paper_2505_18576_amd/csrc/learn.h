// Learned smoother damping (learn.hip): features, MLP forward/backward, Adam.
#pragma once
#include "common.h"

namespace amgf {

constexpr int MLP_NPARAM = 1313;     // 6-32-32-1 weights and biases
constexpr int MLP_NTOTAL = 1325;     // + 6 feature means + 6 feature standard deviations

// F: 6 x (nn*b) row-major feature matrix of one level
void level_features(Ctx& c, int b, int nn, const int* arp, const int* acol, const double* aval,
                    const double* d, const int* jtrp, const int* jtcol, const double* jtval,
                    const double* D, double lev_frac, double* F);
// theta = 1 + 0.98 tanh(MLP(F)), w = theta / d  (W: device, MLP_NTOTAL floats)
void mlp_theta(Ctx& c, int64_t n, const float* W, const double* F, const double* d,
               double* theta, double* w);
// grad (+)= d loss / d W given thbar = d loss / d theta (MLP_NPARAM doubles)
void mlp_backward(Ctx& c, int64_t n, const float* W, const double* F, const double* thbar,
                  double* grad, bool accumulate);
void acc_hadamard(Ctx& c, int64_t n, const double* a, const double* b, double* acc);  // acc += a.b
void hadamard(Ctx& c, int64_t n, const double* a, const double* b, double* out);      // out = a.b
void axpy_hadamard(Ctx& c, int64_t n, const double* w, const double* x, double* y);   // y += w.x
void vdiv(Ctx& c, int64_t n, const double* a, const double* d, double* out);          // out = a/d
void adam_step(Ctx& c, float* W, const double* g, float* m1, float* m2, int t, float lr);

}  // namespace amgf

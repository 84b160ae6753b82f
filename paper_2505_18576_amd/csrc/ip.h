// Vector kernels of the interior-point driver for the contact QP (ip.hip).
//
// Problem: minimise 1/2 u^T K u - f^T u subject to J u + g0 >= 0, with slacks s, multipliers
// lam of J u + g0 - s = 0 and duals z of s >= 0 (Sec. 3), the barrier weighted by the
// lumped slack mass M_s (Ms, m values; NULL = ones).  Residuals of the barrier subproblem:
// r_u = K u - f + J^T lam, r_s = -lam - M_s z, r_lam = J u + g0 - s, r_z = s z - mu.
// J is the level-0 contact Jacobian (m x nn BSR, 1 x 3 blocks), JT its transpose with the
// nonempty block rows listed in crows.
#pragma once
#include "common.h"

namespace amgf {

// s = max(J u + g0, s_init), z = mu / s, lam = -M_s z
void ip_init(Ctx& c, const BSR& J, const double* u, const double* g0, const double* Ms,
             double mu, double s_init, double* s, double* lam, double* z);
// y += J^T v over the listed rows
void ip_jt_add(Ctx& c, const BSR& JT, const int* crows, int ncrows, const double* v, double* y);
// r_lam = J u + g0 - s, r_s = -lam - M_s z
void ip_m_residuals(Ctx& c, const BSR& J, const double* u, const double* g0, const double* Ms,
                    const double* s, const double* lam, const double* z, double* r_lam,
                    double* r_s);
// y = a / d elementwise (n values)
void ip_div(Ctx& c, int64_t n, const double* a, const double* d, double* y);
// Host results of one fixed-order pass over the m constraints:
//   out[0] = sum r_s^2 / M_s, out[1] = max |r_lam|, out[2] = max |s z - mu|,
//   out[3] = sum |lam|, out[4] = sum |z|, out[5] = min D, out[6] = max D (D = M_s z / s).
//   `dev` holds 8 doubles.
void ip_m_norms(Ctx& c, int m, const double* r_s, const double* r_lam, const double* s,
                const double* lam, const double* z, const double* Ms, double mu, double* dev,
                double* out);
// D = M_s z / s and t = D b_lam + b_s with b_lam = -r_lam, b_s = -(r_s + M_s (s z - mu) / s)
void ip_rhs_m(Ctx& c, int m, const double* s, const double* z, const double* Ms,
              const double* r_s, const double* r_lam, double mu, double* D, double* t);
// Recovery of the eliminated components from u^ (Sec. 3):
//   s^ = J u^ - b_lam, lam^ = D s^ - b_s, z^ = -(r_z + z s^) / s,
// and the fraction-to-the-boundary step lengths (host) alpha[0] for s, alpha[1] for z:
// the largest a in (0, 1] with v + a v^ >= (1 - tau) v.  `dev` holds 8 doubles.
void ip_recover(Ctx& c, const BSR& J, const double* uh, const double* s, const double* z,
                const double* D, const double* Ms, const double* r_s, const double* r_lam,
                double mu, double tau, double* sh, double* lh, double* zh, double* dev,
                double* alpha);
// s += ap s^, lam += ap lam^, z += ad z^
void ip_update_m(Ctx& c, int m, double ap, double ad, const double* sh, const double* lh,
                 const double* zh, double* s, double* lam, double* z);

}  // namespace amgf

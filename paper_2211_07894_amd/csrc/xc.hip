// LDA exchange-correlation potential and kernel, point by point (the K_xc part of
// K in Eq. (3); two channels as in Sec. II D).  FP64.
//
// Energy per volume e(rho):
//   exchange  -(3/4)(3/pi)^{1/3} n^{4/3} (one channel, n the total density) or
//             -(3/4)(6/pi)^{1/3} sum_s rho_s^{4/3} (two channels);
//   correlation n eps_c(rs, zeta), rs = (3/(4 pi n))^{1/3},
//             eps_c = eps_U + f(zeta)(eps_P - eps_U), the Perdew-Zunger (1981) fit of
//             the Ceperley-Alder gas (gamma/(1 + beta1 sqrt(rs) + beta2 rs) for
//             rs >= 1, A ln rs + B + C rs ln rs + D rs below) for the unpolarised
//             and fully polarised gas, f(zeta) = ((1+zeta)^{4/3} + (1-zeta)^{4/3} - 2)
//             / (2^{4/3} - 2).
// Potential V_s = de/drho_s and kernel f_st = d^2 e / drho_s drho_t, written out
// by the chain rule through n, rs (drs/dn = -rs/(3n)) and zeta
// (dzeta/drho_s = (sgn_s - zeta)/n).  Points where a channel density is below
// 1e-12 carry no exchange-correlation term (V = f = 0).
#include "lrdm_internal.h"

namespace lrdm {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kRhoMin = 1e-12;

struct Fit {
  double gamma, beta1, beta2, A, B, C, D;
};
// unpolarised and fully polarised gas
__device__ inline Fit fit_unpolarised() {
  return {-0.1423, 1.0529, 0.3334, 0.0311, -0.048, 0.0020, -0.0116};
}
__device__ inline Fit fit_polarised() {
  return {-0.0843, 1.3981, 0.2611, 0.01555, -0.0269, 0.0007, -0.0048};
}

// eps_c(rs) and its first two derivatives in rs.
__device__ inline void pz81(const Fit& c, double rs, double& e, double& e1, double& e2) {
  if (rs >= 1.0) {
    const double sq = sqrt(rs);
    const double Q = 1.0 + c.beta1 * sq + c.beta2 * rs;
    const double Q1 = c.beta1 / (2.0 * sq) + c.beta2;
    const double Q2 = -c.beta1 / (4.0 * rs * sq);
    e = c.gamma / Q;
    e1 = -c.gamma * Q1 / (Q * Q);
    e2 = -c.gamma * Q2 / (Q * Q) + 2.0 * c.gamma * Q1 * Q1 / (Q * Q * Q);
  } else {
    const double lr = log(rs);
    e = c.A * lr + c.B + c.C * rs * lr + c.D * rs;
    e1 = c.A / rs + c.C * (lr + 1.0) + c.D;
    e2 = -c.A / (rs * rs) + c.C / rs;
  }
}

// vxc [nspin][M] and fxc [nspin][nspin][M] (either may be NULL).
__global__ __launch_bounds__(256) void lda_xc_kernel(const double* __restrict__ rho, int nspin,
                                                     int64_t M, double* __restrict__ vxc,
                                                     double* __restrict__ fxc) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= M) return;
  double v[2] = {0.0, 0.0};
  double f[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  const double r0 = rho[p];
  const double r1 = nspin == 2 ? rho[M + p] : 1.0;
  if (r0 >= kRhoMin && r1 >= kRhoMin) {
    const double n = nspin == 2 ? r0 + r1 : r0;
    const double rs = cbrt(3.0 / (4.0 * kPi * n));
    const double drs = -rs / (3.0 * n);                 // drs/dn
    double eU, eU1, eU2;
    pz81(fit_unpolarised(), rs, eU, eU1, eU2);
    if (nspin == 1) {
      const double cx = cbrt(3.0 / kPi);
      const double n13 = cbrt(n);
      // correlation: V = eps - (rs/3) eps', f = ((2/3) eps' - (rs/3) eps'') drs/dn
      v[0] = -cx * n13 + eU - rs / 3.0 * eU1;
      f[0][0] = -cx / (3.0 * n13 * n13) + (2.0 / 3.0 * eU1 - rs / 3.0 * eU2) * drs;
    } else {
      double eP, eP1, eP2;
      pz81(fit_polarised(), rs, eP, eP1, eP2);
      const double z = (r0 - r1) / n;
      const double den = cbrt(16.0) - 2.0;             // 2^{4/3} - 2
      const double a = cbrt(1.0 + z), b = cbrt(1.0 - z);
      const double fz = ((1.0 + z) * a + (1.0 - z) * b - 2.0) / den;
      const double fz1 = 4.0 / 3.0 * (a - b) / den;
      const double fz2 = 4.0 / 9.0 * (1.0 / (a * a) + 1.0 / (b * b)) / den;
      const double e = eU + fz * (eP - eU);
      const double e_r = eU1 + fz * (eP1 - eU1);
      const double e_rr = eU2 + fz * (eP2 - eU2);
      const double e_z = fz1 * (eP - eU);
      const double e_zr = fz1 * (eP1 - eU1);
      const double e_zz = fz2 * (eP - eU);
      const double cx = cbrt(6.0 / kPi);
      const double rs_[2] = {r0, r1};
      const double sg[2] = {1.0, -1.0};
      for (int s = 0; s < 2; ++s) {
        const double c13 = cbrt(rs_[s]);
        v[s] = -cx * c13 + e - rs / 3.0 * e_r + (sg[s] - z) * e_z;
        f[s][s] = -cx / (3.0 * c13 * c13);
      }
      for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) {
          const double dVdrs = 2.0 / 3.0 * e_r - rs / 3.0 * e_rr + (sg[s] - z) * e_zr;
          const double dVdz = -rs / 3.0 * e_zr + (sg[s] - z) * e_zz;
          f[s][t] += dVdrs * drs + dVdz * (sg[t] - z) / n;
        }
    }
  }
  for (int s = 0; s < nspin; ++s) {
    if (vxc) vxc[(size_t)s * M + p] = v[s];
    if (fxc)
      for (int t = 0; t < nspin; ++t) fxc[((size_t)s * nspin + t) * M + p] = f[s][t];
  }
}

// dV[k][c] += sum_d fxc[c][d] u[k][d] for k < r.
__global__ __launch_bounds__(256) void xc_apply_kernel(const double* __restrict__ fxc,
                                                       const double* __restrict__ u, int nspin,
                                                       int r, int64_t M,
                                                       double* __restrict__ dV) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= M) return;
  for (int k = 0; k < r; ++k)
    for (int c = 0; c < nspin; ++c) {
      double s = 0.0;
      for (int d = 0; d < nspin; ++d)
        s += fxc[((size_t)c * nspin + d) * M + p] * u[((size_t)k * nspin + d) * M + p];
      dV[((size_t)k * nspin + c) * M + p] += s;
    }
}

}  // namespace

hipError_t launch_lda_xc(lrdm_ctx* ctx, const double* rho, int nspin, int64_t M, double* vxc,
                         double* fxc) {
  if (M <= 0) return hipSuccess;
  lda_xc_kernel<<<(unsigned)((M + 255) / 256), 256, 0, ctx->stream>>>(rho, nspin, M, vxc, fxc);
  return hipGetLastError();
}

hipError_t launch_xc_apply(lrdm_ctx* ctx, const double* fxc, const double* u, int nspin, int r,
                           int64_t M, double* dV) {
  if (M <= 0) return hipSuccess;
  xc_apply_kernel<<<(unsigned)((M + 255) / 256), 256, 0, ctx->stream>>>(fxc, u, nspin, r, M, dV);
  return hipGetLastError();
}

}  // namespace lrdm

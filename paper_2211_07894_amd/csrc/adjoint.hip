// Pieces of the adjoint of the subspace density response that are not
// contractions: scaling, and the gradient with respect to the eigenvalues.
//
// With A_k = dL/dGamma_k and H'_k (Eqs. (21)-(22)) for directions k, the loss
// depends on eps through
//   F_ij = f[eps_i, eps_j]   (dL/dF = P = sum_k A_k o H'_k),
//   f'_i                     (dL/df'_i = q_i = sum_k -mu'_k A_k,ii - nu_k (H'_k,ii - mu'_k),
//                             from -mu' diag(f') and mu' = sum f' H'_ii / sum f'),
//   mu(eps)                  (electron count: dmu/deps_i = f'_i / sum f').
// With mu held fixed, dL/deps_i = 2 sum_j P_ij f[eps_i, eps_i, eps_j] + q_i f''_i
// (F symmetric; the second divided difference is f''/2 at coincidence), and
// dL/dmu is minus the sum of those, so the full gradient is
//   g_i = g_i^0 - (f'_i / sum f') sum_j g_j^0   (zero shift when sum f' underflows).
// Everything is FP64.
#include "lrdm_internal.h"

namespace lrdm {
namespace {

__global__ void scale_kernel(const double* __restrict__ x, double a, int64_t n,
                             double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// f[e_i, e_i, e_j] from F_ij = f[e_i, e_j] and the derivatives of f at e_i:
// the difference quotient (F_ij - f'_i)/(e_j - e_i), or below |e_j - e_i| < 1e-3 kT
// (where it would cancel) the Taylor series f''/2 + f''' h/6 + f'''' h^2/24.
__device__ inline double second_dd(double h, double Fij, double f1, double f2, double f3,
                                   double f4, double kT) {
  if (fabs(h) < 1e-3 * kT) return f2 / 2.0 + f3 * h / 6.0 + f4 * h * h / 24.0;
  return (Fij - f1) / h;
}

// One block per (row i, channel c): partial gradient g^0 with mu held fixed.
__global__ __launch_bounds__(256) void adj_eps_row_kernel(
    const double* __restrict__ A, const double* __restrict__ Hp, const double* __restrict__ eps,
    const double* __restrict__ F, const double* __restrict__ f, const double* __restrict__ omf,
    const double* __restrict__ dmu, const double* __restrict__ nu, int N, int nspin, int r,
    double kT, double* __restrict__ part) {
  __shared__ double red[4];
  const int i = blockIdx.x, c = blockIdx.y;
  const int64_t row = (int64_t)c * N + i;
  const double a = f[row] * omf[row];
  const double d = omf[row] - f[row];
  const double f1 = -a / kT;
  const double f2 = a * d / (kT * kT);
  const double f3 = -a * (1.0 - 6.0 * a) / (kT * kT * kT);
  const double f4 = a * d * (1.0 - 12.0 * a) / (kT * kT * kT * kT);
  const double ei = eps[row];
  double s = 0.0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    double P = 0.0;
    for (int k = 0; k < r; ++k) {
      const int64_t idx = (((int64_t)k * nspin + c) * N + i) * N + j;
      P += A[idx] * Hp[idx];
    }
    const double h = eps[(int64_t)c * N + j] - ei;
    s += P * second_dd(h, F[((int64_t)c * N + i) * N + j], f1, f2, f3, f4, kT);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double q = 0.0;
    for (int k = 0; k < r; ++k) {
      const int64_t dg = (((int64_t)k * nspin + c) * N + i) * N + i;
      q += -dmu[k] * A[dg] - nu[k] * (Hp[dg] - dmu[k]);
    }
    part[row] = 2.0 * (red[0] + red[1] + red[2] + red[3]) + q * f2;
  }
}

// g = g^0 - (f' / sum f') sum g^0 over all channels; one block, fixed-order sums.
__global__ __launch_bounds__(256) void adj_eps_mu_kernel(const double* __restrict__ part,
                                                         const double* __restrict__ fp,
                                                         int64_t n, double* __restrict__ g) {
  __shared__ double red[2][4];
  double s = 0.0, sf = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    s += part[i];
    sf += fp[i];
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_down(s, off, 64);
    sf += __shfl_down(sf, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s;
    red[1][threadIdx.x >> 6] = sf;
  }
  __syncthreads();
  const double tot = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  const double S = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  const double shift = fabs(S) < 1e-300 ? 0.0 : -tot / S;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) g[i] = part[i] + fp[i] * shift;
}

}  // namespace

hipError_t launch_scale(lrdm_ctx* ctx, const double* x, double a, int64_t n, double* y) {
  scale_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(x, a, n, y);
  return hipGetLastError();
}

hipError_t launch_adj_eps(lrdm_ctx* ctx, const double* A, const double* Hp, const double* eps,
                          const double* F, const double* f, const double* omf, const double* fp,
                          const double* dmu, const double* nu, int N, int nspin, int r, double kT,
                          double* part, double* g_eps) {
  ProfScope prof(ctx, "adj_eps");
  adj_eps_row_kernel<<<dim3(N, nspin), 256, 0, ctx->stream>>>(A, Hp, eps, F, f, omf, dmu, nu, N,
                                                               nspin, r, kT, part);
  LRDM_HIP(hipGetLastError());
  adj_eps_mu_kernel<<<1, 256, 0, ctx->stream>>>(part, fp, (int64_t)nspin * N, g_eps);
  return hipGetLastError();
}

}  // namespace lrdm

// Fermi level, occupations, divided differences and the Fermi-shift / Gamma step.
//
// Eq. (1): f(eps, mu) = 1 / (1 + exp((eps - mu)/kT)), s sum_i f(eps_i, mu) = N_e.
// Eq. (22) with exact Fermi-Dirac divided differences: the derivative of
// f(D + lam H', mu + lam mu') at lam = 0 for diagonal D is
//     Gamma = F o H' - mu' diag(f'),   F_ij = (f_i - f_j)/(eps_i - eps_j), F_ii = f'_i,
// and mu' follows from the traceless condition stated after Eq. (24).
// Everything here is FP64.
#include "blocks.h"
#include "lrdm_internal.h"

namespace lrdm {
namespace {

constexpr int kFermiThreads = 256;

__device__ inline double logistic(double y) {  // 1 / (1 + exp(y)) without overflow
  if (y >= 0.0) {
    double e = exp(-y);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + exp(y));
}

__device__ inline double block_sum(double v, double* red) {
  // wavefront reduction then across the 4 waves of a 256-thread block (fixed order)
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return t;
}

__device__ inline double block_max(double v, double* red) {
  // same pattern as block_sum, for a maximum of non-negative values
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return t;
}

// One block: bisection for mu on [min eps - 50 kT, max eps + 50 kT] until the
// bracket is within 2 ulp of its midpoint (at most 200 halvings).  With weights
// (Brillouin-zone sampling) entry i of eps [nspin][nk][N] counts with weight
// weights[(i / N) % nk].
__global__ __launch_bounds__(kFermiThreads) void fermi_mu_kernel(
    const double* __restrict__ eps, int count, double s, double kT, double ne,
    const double* __restrict__ weights, int N, int nk, double* __restrict__ mu_out,
    int* __restrict__ status) {
  __shared__ double red[4];
  double lo = 1e300, hi = -1e300;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    lo = fmin(lo, eps[i]);
    hi = fmax(hi, eps[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
  }
  __shared__ double mn[4], mx[4];
  if ((threadIdx.x & 63) == 0) {
    mn[threadIdx.x >> 6] = lo;
    mx[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  lo = fmin(fmin(mn[0], mn[1]), fmin(mn[2], mn[3])) - 50.0 * kT;
  hi = fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3])) + 50.0 * kT;
  bool converged = false;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double ulp = nextafter(fabs(mid), INFINITY) - fabs(mid);
    if (hi - lo <= 2.0 * ulp) {
      converged = true;
      break;
    }
    double part = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
      const double fi = logistic((eps[i] - mid) / kT);
      part += weights ? weights[(i / N) % nk] * fi : fi;
    }
    const double cnt = s * block_sum(part, red);
    if (cnt > ne) hi = mid; else lo = mid;
  }
  if (threadIdx.x == 0) {
    *mu_out = 0.5 * (lo + hi);
    if (!converged && status) status[LRDM_DS_BISECT] = 1;
  }
}

__global__ void occupations_kernel(const double* __restrict__ eps, int count, double kT,
                                   const double* __restrict__ mu, double* __restrict__ f,
                                   double* __restrict__ omf, double* __restrict__ fprime) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double y = (eps[i] - *mu) / kT;
  const double fi = logistic(y);
  const double oi = logistic(-y);
  if (f) f[i] = fi;
  if (omf) omf[i] = oi;
  if (fprime) fprime[i] = -fi * oi / kT;
}

// F_ij for one channel: with eps_lo <= eps_hi and z = (eps_lo - eps_hi)/kT <= 0,
// f_lo - f_hi = -f_lo (1 - f_hi) expm1(z) exactly, hence
// F = -(1/kT) f_lo (1 - f_hi) expm1(z)/z with expm1(z)/z -> 1 at z = 0.
__global__ void divided_diff_kernel(const double* __restrict__ eps, const double* __restrict__ f,
                                    const double* __restrict__ omf, int N, double kT,
                                    double* __restrict__ F) {
  const int c = blockIdx.z;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= N || j >= N) return;
  const double* e = eps + (size_t)c * N;
  const double* fc = f + (size_t)c * N;
  const double* oc = omf + (size_t)c * N;
  const double ei = e[i], ej = e[j];
  int lo = i, hi = j;
  if (ej < ei || (ej == ei && j < i)) { lo = j; hi = i; }
  const double z = (e[lo] - e[hi]) / kT;
  const double phi = (z == 0.0) ? 1.0 : expm1(z) / z;
  F[((size_t)c * N + i) * N + j] = -(fc[lo] * oc[hi] * phi) / kT;
}

// The paper's recursive Fermi expansion of depth T (Eqs. (23)-(24)) as a Hadamard
// multiplier.  On the diagonal subspace Hamiltonian every step
// g(x) = x^2 / (x^2 + (1 - x)^2) acts on each diagonal entry, so the first-order
// response of the composition is, entry by entry, the product of the divided
// differences g[a, b] = (a + b - 2ab) / (y(a) y(b)), y(x) = x^2 + (1 - x)^2, over
// the T steps, times the slope -2^{-(T+2)}/kT of the first map:
//   M_ij = -(2^{-(T+2)}/kT) prod_n g[x_i^(n), x_j^(n)],
//   x^(0) = 1/2 - 2^{-(T+2)} (eps - mu)/kT,  x^(n+1) = g(x^(n)).
// diag receives M_ii (the response to mu, used for mu').  Symmetric bit for bit:
// every operation is commutative in (i, j).
__global__ void recursive_multiplier_kernel(const double* __restrict__ eps,
                                            const double* __restrict__ mu, int N, double kT,
                                            int T, double* __restrict__ M,
                                            double* __restrict__ diag) {
  const int c = blockIdx.z;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= N || j >= N) return;
  const double* e = eps + (size_t)c * N;
  const double scale = ldexp(1.0, -(T + 2)) / kT;
  double xi = 0.5 - scale * (e[i] - mu[0]);
  double xj = 0.5 - scale * (e[j] - mu[0]);
  double m = -scale;
  for (int n = 0; n < T; ++n) {
    const double yi = xi * xi + (1.0 - xi) * (1.0 - xi);
    const double yj = xj * xj + (1.0 - xj) * (1.0 - xj);
    m *= (xi + xj - 2.0 * (xi * xj)) / (yi * yj);
    xi = (xi * xi) / yi;
    xj = (xj * xj) / yj;
  }
  M[((size_t)c * N + i) * N + j] = m;
  if (i == j) diag[(size_t)c * N + i] = m;
}

// One block per direction: mu'_k = sum_{c,i} f'_ci Hp_kc,ii / sum_{c,i} f'_ci.
__global__ __launch_bounds__(kFermiThreads) void dmu_kernel(const double* __restrict__ Hp,
                                                            const double* __restrict__ fprime,
                                                            int N, int nspin,
                                                            double* __restrict__ dmu) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double num = 0.0, den = 0.0;
  for (int idx = threadIdx.x; idx < nspin * N; idx += blockDim.x) {
    const int c = idx / N, i = idx - c * N;
    const double fp = fprime[idx];
    num += fp * Hp[(((size_t)k * nspin + c) * N + i) * N + i];
    den += fp;
  }
  num = block_sum(num, red);
  den = block_sum(den, red);
  if (threadIdx.x == 0) dmu[k] = (fabs(den) < 1e-300) ? 0.0 : num / den;
}

// Gamma_kc = F_c o Hp_kc - mu'_k diag(f'_c), in place.
__global__ void gamma_kernel(double* __restrict__ Hp, const double* __restrict__ F,
                             const double* __restrict__ fprime, const double* __restrict__ dmu,
                             int N, int nspin) {
  const int b = blockIdx.z;  // k * nspin + c
  const int k = b / nspin, c = b - k * nspin;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= N || j >= N) return;
  const size_t off = ((size_t)b * N + i) * N + j;
  double g = F[((size_t)c * N + i) * N + j] * Hp[off];
  if (i == j) g -= dmu[k] * fprime[(size_t)c * N + i];
  Hp[off] = g;
}

// tmax[c][I][J] = largest |F_c| entry of the 128 x 128 block (I, J) for I <= J
// (infinity when the block holds a NaN, so that it stays active).
__global__ __launch_bounds__(256) void block_max_kernel(const double* __restrict__ F, int N,
                                                       int ntb, double* __restrict__ tmax) {
  __shared__ double red[4];
  const int c = blockIdx.y;
  const int I = blockIdx.x / ntb, J = blockIdx.x % ntb;
  if (J < I) return;
  double m = 0.0;
  for (int idx = threadIdx.x; idx < kBlockEdge * kBlockEdge; idx += blockDim.x) {
    const int i = I * kBlockEdge + idx / kBlockEdge, j = J * kBlockEdge + idx % kBlockEdge;
    if (i < N && j < N) {
      const double a = fabs(F[((size_t)c * N + i) * N + j]);
      m = (a != a) ? INFINITY : fmax(m, a);
    }
  }
  m = block_max(m, red);
  if (threadIdx.x == 0) tmax[((size_t)c * ntb + I) * ntb + J] = m;
}

// active[c][I][J] = active[c][J][I] = (tmax of the block > tau * largest tmax);
// every block is active when the largest is not finite.  One block of threads.
__global__ __launch_bounds__(256) void block_mask_kernel(const double* __restrict__ tmax, int ntb,
                                                        int nspin, double tau,
                                                        unsigned char* __restrict__ active) {
  __shared__ double red[4];
  const int n = nspin * ntb * ntb;
  double g = 0.0;
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int I = (idx / ntb) % ntb, J = idx % ntb;
    if (J >= I) g = fmax(g, tmax[idx]);
  }
  g = block_max(g, red);
  const bool all = !isfinite(g);
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int c = idx / (ntb * ntb), I = (idx / ntb) % ntb, J = idx % ntb;
    const double m = tmax[((size_t)c * ntb + min(I, J)) * ntb + max(I, J)];
    active[idx] = (all || m > tau * g) ? 1 : 0;
  }
}

__global__ void check_finite_kernel(const double* __restrict__ x, int64_t n, int* status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) status[LRDM_DS_NONFINITE] = 1;
}

}  // namespace

hipError_t launch_fermi(lrdm_ctx* ctx, const double* eps, int N, int nspin, double kT,
                        double n_electrons, double* mu, double* f, double* omf, double* fprime,
                        double* F) {
  const int count = N * nspin;
  const double s = (nspin == 1) ? 2.0 : 1.0;
  fermi_mu_kernel<<<1, kFermiThreads, 0, ctx->stream>>>(eps, count, s, kT, n_electrons, nullptr,
                                                        N, 1, mu, ctx->dstatus);
  LRDM_HIP(hipGetLastError());
  occupations_kernel<<<(count + 255) / 256, 256, 0, ctx->stream>>>(eps, count, kT, mu, f, omf,
                                                                   fprime);
  LRDM_HIP(hipGetLastError());
  if (F) {
    dim3 blk(32, 8);
    dim3 grd((N + 31) / 32, (N + 7) / 8, nspin);
    divided_diff_kernel<<<grd, blk, 0, ctx->stream>>>(eps, f, omf, N, kT, F);
    LRDM_HIP(hipGetLastError());
  }
  return hipSuccess;
}

hipError_t launch_fermi_bz(lrdm_ctx* ctx, const double* eps, int N, int nspin, int nk,
                           const double* weights, double kT, double n_electrons, double* mu,
                           double* f, double* omf, double* fprime, double* F) {
  const int count = N * nspin * nk;
  const double s = (nspin == 1) ? 2.0 : 1.0;
  fermi_mu_kernel<<<1, kFermiThreads, 0, ctx->stream>>>(eps, count, s, kT, n_electrons, weights,
                                                        N, nk, mu, ctx->dstatus);
  LRDM_HIP(hipGetLastError());
  occupations_kernel<<<(count + 255) / 256, 256, 0, ctx->stream>>>(eps, count, kT, mu, f, omf,
                                                                   fprime);
  LRDM_HIP(hipGetLastError());
  dim3 blk(32, 8);
  dim3 grd((N + 31) / 32, (N + 7) / 8, nspin * nk);
  divided_diff_kernel<<<grd, blk, 0, ctx->stream>>>(eps, f, omf, N, kT, F);
  return hipGetLastError();
}

hipError_t launch_recursive_multiplier(lrdm_ctx* ctx, const double* eps, const double* mu, int N,
                                      int nspin, double kT, int depth, double* M, double* diag) {
  dim3 blk(32, 8);
  dim3 grd((N + 31) / 32, (N + 7) / 8, nspin);
  recursive_multiplier_kernel<<<grd, blk, 0, ctx->stream>>>(eps, mu, N, kT, depth, M, diag);
  return hipGetLastError();
}

hipError_t launch_gamma(lrdm_ctx* ctx, double* Hp, const double* F, const double* fprime, int N,
                        int nspin, int r, double* dmu) {
  dmu_kernel<<<r, kFermiThreads, 0, ctx->stream>>>(Hp, fprime, N, nspin, dmu);
  LRDM_HIP(hipGetLastError());
  dim3 blk(32, 8);
  dim3 grd((N + 31) / 32, (N + 7) / 8, r * nspin);
  gamma_kernel<<<grd, blk, 0, ctx->stream>>>(Hp, F, fprime, dmu, N, nspin);
  return hipGetLastError();
}

hipError_t launch_block_mask(lrdm_ctx* ctx, const double* F, int N, int nspin, double tau,
                             double* tmax, unsigned char* active) {
  const int ntb = (N + kBlockEdge - 1) / kBlockEdge;
  dim3 grd((unsigned)(ntb * ntb), (unsigned)nspin);
  block_max_kernel<<<grd, 256, 0, ctx->stream>>>(F, N, ntb, tmax);
  LRDM_HIP(hipGetLastError());
  block_mask_kernel<<<1, 256, 0, ctx->stream>>>(tmax, ntb, nspin, tau, active);
  return hipGetLastError();
}

hipError_t launch_check_finite(lrdm_ctx* ctx, const double* x, int64_t n) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  check_finite_kernel<<<(unsigned)blocks, 256, 0, ctx->stream>>>(x, n, ctx->dstatus);
  return hipGetLastError();
}

}  // namespace lrdm

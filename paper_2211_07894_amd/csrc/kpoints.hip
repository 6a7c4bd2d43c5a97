// Brillouin-zone sampling of the subspace response (Sec. II C, last paragraph).
//
// Each k-point has a complex subspace Psi_k = A + iB (N states).  With the states
// stored "realified" as the 2N real rows Phi = [A; B], the complex products
// reduce to the real kernels' products with 2N states:
//   H2 = Phi^T diag(dV) Phi  ->  H'_k = Psi^H diag(dV) Psi = (H2_00 + H2_11) + i (H2_01 - H2_10),
// and for Hermitian Gamma_k = Gr + i Gi (Gr symmetric, Gi antisymmetric)
//   diag(Psi Gamma Psi^H) = sum_ij Gr_ij (A_i A_j + B_i B_j) + 2 sum_ij Gi_ij A_i B_j
//                         = sum_IJ Phi_I G2_IJ Phi_J,   G2 = [[Gr, Gi], [-Gi, Gr]]
// (G2 is symmetric, so the symmetric back-projection applies).  mu and mu' are
// common to the zone: mu from the weighted electron count, mu' from the weighted
// traceless condition sum_k w_k sum_i f'_ki (Gamma_k)_ii = 0.  All FP64.
#include "lrdm_internal.h"

namespace lrdm {
namespace {

constexpr int kThreads = 256;

__global__ void expand_dv_kernel(const double* __restrict__ dV, int nk, int64_t M,
                                 double* __restrict__ W) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;                   // (q nspin + c) nk + k
  if (p < M) W[(int64_t)b * M + p] = dV[(int64_t)(b / nk) * M + p];
}

__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  const double t = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return t;
}

// One block per direction q: mu' = sum_{c,k} w_k sum_i f'_cki H'_cki,ii /
// sum_{c,k} w_k sum_i f'_cki (zero when the denominator underflows), with
// H'_ii = H2_ii + H2_(N+i)(N+i).
__global__ __launch_bounds__(kThreads) void dmu_bz_kernel(const double* __restrict__ H2,
                                                          const double* __restrict__ fprime,
                                                          const double* __restrict__ weights,
                                                          int N, int nspin, int nk,
                                                          double* __restrict__ dmu) {
  __shared__ double red[4];
  const int q = blockIdx.x;
  const int N2 = 2 * N;
  double num = 0.0, den = 0.0;
  for (int idx = threadIdx.x; idx < nspin * nk * N; idx += blockDim.x) {
    const int ck = idx / N, i = idx - ck * N;
    const int k = ck % nk;
    const double* H = H2 + ((size_t)q * nspin * nk + ck) * N2 * N2;
    const double fp = weights[k] * fprime[idx];
    num += fp * (H[(size_t)i * N2 + i] + H[(size_t)(N + i) * N2 + N + i]);
    den += fp;
  }
  num = block_sum(num, red);
  den = block_sum(den, red);
  if (threadIdx.x == 0) dmu[q] = (fabs(den) < 1e-300) ? 0.0 : num / den;
}

// G2 = w_k [[Gr, Gi], [-Gi, Gr]] in place over H2: thread (i, j) owns the four
// entries (i, j), (N+i, N+j), (i, N+j), (N+i, j), which it reads before writing.
__global__ void gamma_bz_kernel(double* __restrict__ H2, const double* __restrict__ F,
                                const double* __restrict__ fprime,
                                const double* __restrict__ weights, const double* __restrict__ dmu,
                                int N, int nspin, int nk) {
  const int b = blockIdx.z;                   // (q nspin + c) nk + k
  const int ck = b % (nspin * nk), q = b / (nspin * nk), k = ck % nk;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= N || j >= N) return;
  const int N2 = 2 * N;
  double* H = H2 + (size_t)b * N2 * N2;
  const double h00 = H[(size_t)i * N2 + j], h11 = H[(size_t)(N + i) * N2 + N + j];
  const double h01 = H[(size_t)i * N2 + N + j], h10 = H[(size_t)(N + i) * N2 + j];
  const double f = F[((size_t)ck * N + i) * N + j];
  double gr = f * (h00 + h11);
  if (i == j) gr -= dmu[q] * fprime[(size_t)ck * N + i];
  const double gi = f * (h01 - h10);
  const double w = weights[k];
  H[(size_t)i * N2 + j] = w * gr;
  H[(size_t)(N + i) * N2 + N + j] = w * gr;
  H[(size_t)i * N2 + N + j] = w * gi;
  H[(size_t)(N + i) * N2 + j] = -w * gi;
}

__global__ void sum_k_kernel(const double* __restrict__ part, int nk, int64_t M,
                             double* __restrict__ drho) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int qc = blockIdx.y;
  if (p >= M) return;
  double s = 0.0;
  for (int k = 0; k < nk; ++k) s += part[((int64_t)qc * nk + k) * M + p];
  drho[(int64_t)qc * M + p] = s;
}

}  // namespace

hipError_t launch_expand_dv(lrdm_ctx* ctx, const double* dV, int r, int nspin, int nk, int64_t M,
                            double* W) {
  dim3 grd((unsigned)((M + kThreads - 1) / kThreads), (unsigned)(r * nspin * nk));
  expand_dv_kernel<<<grd, kThreads, 0, ctx->stream>>>(dV, nk, M, W);
  return hipGetLastError();
}

hipError_t launch_gamma_bz(lrdm_ctx* ctx, double* H2, const double* F, const double* fprime,
                           const double* weights, int N, int nspin, int nk, int r, double* dmu) {
  dmu_bz_kernel<<<r, kThreads, 0, ctx->stream>>>(H2, fprime, weights, N, nspin, nk, dmu);
  LRDM_HIP(hipGetLastError());
  dim3 blk(32, 8);
  dim3 grd((N + 31) / 32, (N + 7) / 8, r * nspin * nk);
  gamma_bz_kernel<<<grd, blk, 0, ctx->stream>>>(H2, F, fprime, weights, dmu, N, nspin, nk);
  return hipGetLastError();
}

hipError_t launch_sum_k(lrdm_ctx* ctx, const double* part, int r, int nspin, int nk, int64_t M,
                        double* drho) {
  dim3 grd((unsigned)((M + kThreads - 1) / kThreads), (unsigned)(r * nspin));
  sum_k_kernel<<<grd, kThreads, 0, ctx->stream>>>(part, nk, M, drho);
  return hipGetLastError();
}

}  // namespace lrdm

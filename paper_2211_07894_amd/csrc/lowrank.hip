// Kernels of the low-rank preconditioner around the density response (Sec. II B)
// and of the model SCF map it acts on (Sec. II A):
//  * density_part_kernel / density_sum_kernel: the output density of Eq. (1),
//    rho_c(x_p) = (s/dv) sum_i f_c,i Psi_c,ip^2, with the state sum split into
//    ranges whose FP64 partial sums are added in a fixed order (minus rho_in when
//    the caller wants the residual R = rho - rho_in);
//  * dots_part_kernel / dots_sum_kernel: cell-integral inner products
//    <a_k, x> = dv sum_p a_k,p x_p of several vectors with one, in a fixed
//    reduction order (per-block partials, then one block per vector);
//  * combine_kernel: y = beta x + sgn sum_k coef_k a_k with the coefficients read
//    from device memory, so that no step of the Krylov loop waits for the host;
//  * normalize_kernel: y = x / sqrt(<x, x>) from a device-held <x, x>;
//  * lowrank_solve_kernel: y = S^{-1} c for the r x r Gram matrix of the
//    directional derivatives (Cholesky; r is at most kMaxLowRank).
// Everything is FP64 except the storage type of Psi in the density.
#include <algorithm>

#include "lrdm_internal.h"

namespace lrdm {
namespace {

constexpr int kThreads = 256;
constexpr int kDotBlocks = 256;

// Sum over a 256-thread block: wavefront shuffles, then the four wave totals in
// a fixed order.  Every thread returns the total.
__device__ inline double block_total(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  const double t = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return t;
}

// part[c][split][p] = sum_{i in the split's state range} f[c][i] Psi[c][i][p]^2.
// Grid: (ceil(M / 256), nsplit, nspin).
template <typename T>
__global__ __launch_bounds__(kThreads) void density_part_kernel(
    const T* __restrict__ Psi, const double* __restrict__ f, int N, int64_t M, int per_split,
    double* __restrict__ part) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= M) return;
  const int c = blockIdx.z, split = blockIdx.y;
  const int i0 = split * per_split;
  const int i1 = min(N, i0 + per_split);
  const T* col = Psi + (size_t)c * N * M + p;
  const double* fc = f + (size_t)c * N;
  double acc = 0.0;
  for (int i = i0; i < i1; ++i) {
    const double v = static_cast<double>(col[(size_t)i * M]);
    acc += fc[i] * (v * v);
  }
  part[((size_t)c * gridDim.y + split) * M + p] = acc;
}

// out[c][p] = scale * sum_split part[c][split][p] - (rho_in ? rho_in[c][p] : 0).
// rho_in may be out (each element is read before it is written).
__global__ __launch_bounds__(kThreads) void density_sum_kernel(
    const double* __restrict__ part, int nsplit, int64_t M, int nspin, double scale,
    const double* rho_in, double* out) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= (int64_t)nspin * M) return;
  const int64_t c = q / M, p = q - c * M;
  const double* pc = part + (size_t)c * nsplit * M + p;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += pc[(size_t)k * M];
  s *= scale;
  if (rho_in) s -= rho_in[q];
  out[q] = s;
}

// part[k][b] = sum over block b's grid-stride slice of A[k][i] x[i].
// Grid: (kDotBlocks, k).
__global__ __launch_bounds__(kThreads) void dots_part_kernel(
    const double* __restrict__ A, int64_t lda, const double* __restrict__ x, int64_t n,
    double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  const double* a = A + (size_t)blockIdx.y * lda;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    s += a[i] * x[i];
  s = block_total(s, red);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// out[k * stride] = scale * sum_b part[k][b].  One block per vector k.
__global__ __launch_bounds__(kThreads) void dots_sum_kernel(const double* __restrict__ part,
                                                            int nb, double scale,
                                                            double* __restrict__ out,
                                                            int stride) {
  __shared__ double red[kThreads / 64];
  const double* pk = part + (size_t)blockIdx.x * nb;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) s += pk[b];
  s = block_total(s, red);
  if (threadIdx.x == 0) out[(size_t)blockIdx.x * stride] = scale * s;
}

// y[i] = beta x[i] + sgn sum_{k < nk} coef[k] A[k][i]  (x may be NULL; y may be x,
// never one of the A rows).
__global__ __launch_bounds__(kThreads) void combine_kernel(
    const double* x, double beta, const double* __restrict__ A, int64_t lda,
    const double* __restrict__ coef, int nk, double sgn, int64_t n, double* y) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nk; ++k) s += coef[k] * A[(size_t)k * lda + i];
  s *= sgn;
  if (x) s += beta * x[i];
  y[i] = s;
}

// y[i] = x[i] / sqrt(nrm2[0]) (y may be x).
__global__ __launch_bounds__(kThreads) void normalize_kernel(const double* x,
                                                             const double* __restrict__ nrm2,
                                                             int64_t n, double* y) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = x[i] / sqrt(nrm2[0]);
}

// y[i] += a x[i].
__global__ __launch_bounds__(kThreads) void axpy_kernel(double a, const double* __restrict__ x,
                                                        int64_t n, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// y = S^{-1} c for the leading r x r block of S (row-major, leading dimension ld;
// only S[i][j] with j <= i is read): Cholesky S = L L^T, then L z = c and
// L^T y = z.  A pivot that is not positive (directional derivatives linearly
// dependent) leaves y = 0 and sets *flag.  One thread; r <= kMaxLowRank.
__global__ void lowrank_solve_kernel(const double* __restrict__ S, int ld,
                                     const double* __restrict__ c, int r,
                                     double* __restrict__ y, int* __restrict__ flag) {
  __shared__ double Lm[kMaxLowRank * kMaxLowRank];
  __shared__ double z[kMaxLowRank];
  if (threadIdx.x != 0) return;
  *flag = 0;
  for (int j = 0; j < r; ++j) {
    double d = S[(size_t)j * ld + j];
    for (int k = 0; k < j; ++k) d -= Lm[j * kMaxLowRank + k] * Lm[j * kMaxLowRank + k];
    if (!(d > 0.0)) {
      *flag = 1;
      for (int i = 0; i < r; ++i) y[i] = 0.0;
      return;
    }
    const double ljj = sqrt(d);
    Lm[j * kMaxLowRank + j] = ljj;
    for (int i = j + 1; i < r; ++i) {
      double v = S[(size_t)i * ld + j];
      for (int k = 0; k < j; ++k) v -= Lm[i * kMaxLowRank + k] * Lm[j * kMaxLowRank + k];
      Lm[i * kMaxLowRank + j] = v / ljj;
    }
  }
  for (int i = 0; i < r; ++i) {
    double v = c[i];
    for (int k = 0; k < i; ++k) v -= Lm[i * kMaxLowRank + k] * z[k];
    z[i] = v / Lm[i * kMaxLowRank + i];
  }
  for (int i = r - 1; i >= 0; --i) {
    double v = z[i];
    for (int k = i + 1; k < r; ++k) v -= Lm[k * kMaxLowRank + i] * y[k];
    y[i] = v / Lm[i * kMaxLowRank + i];
  }
}

// range[0] = min x, range[1] = max x over n > 0 elements.  One block.
__global__ __launch_bounds__(kThreads) void minmax_kernel(const double* __restrict__ x, int64_t n,
                                                          double* __restrict__ range) {
  __shared__ double lo_w[kThreads / 64], hi_w[kThreads / 64];
  double lo = x[0], hi = x[0];
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    lo = fmin(lo, x[i]);
    hi = fmax(hi, x[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    lo_w[wid] = lo;
    hi_w[wid] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    range[0] = fmin(fmin(lo_w[0], lo_w[1]), fmin(lo_w[2], lo_w[3]));
    range[1] = fmax(fmax(hi_w[0], hi_w[1]), fmax(hi_w[2], hi_w[3]));
  }
}

// x[i] = a value in [-1, 1) from an integer hash of i (scratch data for timing).
template <typename T>
__global__ __launch_bounds__(kThreads) void pattern_kernel(T* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z ^= z >> 29;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 32;
  x[i] = (T)((double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

size_t density_workspace_bytes(int N, int64_t M, int nspin) {
  return ws_align((size_t)nspin * density_splits(N, M, nspin) * M * sizeof(double));
}

template <typename T>
hipError_t launch_density(lrdm_ctx* ctx, const T* Psi, const double* f, int N, int64_t M,
                          int nspin, double scale, const double* rho_in, double* out,
                          double* part) {
  if (M <= 0 || N <= 0) return hipSuccess;
  ProfScope prof(ctx, "density");
  const int nsplit = density_splits(N, M, nspin);
  const int per_split = (N + nsplit - 1) / nsplit;
  dim3 grd(blocks_for(M), nsplit, nspin);
  density_part_kernel<T><<<grd, kThreads, 0, ctx->stream>>>(Psi, f, N, M, per_split, part);
  LRDM_HIP(hipGetLastError());
  density_sum_kernel<<<blocks_for((int64_t)nspin * M), kThreads, 0, ctx->stream>>>(
      part, nsplit, M, nspin, scale, rho_in, out);
  return hipGetLastError();
}

template hipError_t launch_density<double>(lrdm_ctx*, const double*, const double*, int, int64_t,
                                           int, double, const double*, double*, double*);
template hipError_t launch_density<float>(lrdm_ctx*, const float*, const double*, int, int64_t,
                                          int, double, const double*, double*, double*);

size_t dots_workspace_bytes(int k) { return ws_align((size_t)k * kDotBlocks * sizeof(double)); }

hipError_t launch_dots(lrdm_ctx* ctx, const double* A, int64_t lda, int k, const double* x,
                       int64_t n, double scale, double* out, int stride, double* part) {
  if (k <= 0) return hipSuccess;
  const int nb = (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, (n + kThreads - 1) / kThreads));
  dots_part_kernel<<<dim3(nb, k), kThreads, 0, ctx->stream>>>(A, lda, x, n, part);
  LRDM_HIP(hipGetLastError());
  dots_sum_kernel<<<k, kThreads, 0, ctx->stream>>>(part, nb, scale, out, stride);
  return hipGetLastError();
}

hipError_t launch_combine(lrdm_ctx* ctx, const double* x, double beta, const double* A,
                          int64_t lda, const double* coef, int nk, double sgn, int64_t n,
                          double* y) {
  if (n <= 0) return hipSuccess;
  combine_kernel<<<blocks_for(n), kThreads, 0, ctx->stream>>>(x, beta, A, lda, coef, nk, sgn, n, y);
  return hipGetLastError();
}

hipError_t launch_normalize(lrdm_ctx* ctx, const double* x, const double* nrm2, int64_t n,
                            double* y) {
  if (n <= 0) return hipSuccess;
  normalize_kernel<<<blocks_for(n), kThreads, 0, ctx->stream>>>(x, nrm2, n, y);
  return hipGetLastError();
}

hipError_t launch_axpy(lrdm_ctx* ctx, double a, const double* x, int64_t n, double* y) {
  if (n <= 0) return hipSuccess;
  axpy_kernel<<<blocks_for(n), kThreads, 0, ctx->stream>>>(a, x, n, y);
  return hipGetLastError();
}

hipError_t launch_pattern(lrdm_ctx* ctx, void* x, int64_t n, bool is_double) {
  if (n <= 0) return hipSuccess;
  if (is_double)
    pattern_kernel<double><<<blocks_for(n), kThreads, 0, ctx->stream>>>(static_cast<double*>(x), n);
  else
    pattern_kernel<float><<<blocks_for(n), kThreads, 0, ctx->stream>>>(static_cast<float*>(x), n);
  return hipGetLastError();
}

hipError_t launch_minmax(lrdm_ctx* ctx, const double* x, int64_t n, double* range) {
  if (n <= 0) return hipSuccess;
  minmax_kernel<<<1, kThreads, 0, ctx->stream>>>(x, n, range);
  return hipGetLastError();
}

hipError_t launch_lowrank_solve(lrdm_ctx* ctx, const double* S, int ld, const double* c, int r,
                                double* y, int* flag) {
  lowrank_solve_kernel<<<1, 64, 0, ctx->stream>>>(S, ld, c, r, y, flag);
  return hipGetLastError();
}

}  // namespace lrdm

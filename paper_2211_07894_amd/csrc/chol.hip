// Orthonormalising factor of a filtered block for the Rayleigh-Ritz step of ChFSI
// (Sec. II C): column-scaled Cholesky QR with rank detection.
//
// Given the Gram matrix G = Y Y^T of N rows, with D = diag(G)^{-1/2} and
// Gs = D G D (unit diagonal), a blocked right-looking Cholesky Gs = L L^T runs in
// the rows' natural order.  A row whose Schur-complement pivot falls below tau
// (its distance to the span of the rows before it is below sqrt(tau) of its own
// norm, where the Gram matrix can no longer resolve it) is dependent: its column of
// L is zeroed, so that it takes no part in the others, and its row keeps its
// projection coefficients with a unit diagonal.  With X = L^{-1}, the row of X Ds
// of an independent row is an orthonormal vector (to about u cond(Gs)); that of a
// dependent row is its explicit residual against the independent rows before it,
// which a further pass over the vectors themselves can resolve (classical
// Gram-Schmidt without the Gram matrix's cancellation).  The factor returned is
//   T[r][j] = X[perm(r)][j] D_j,
// with the k independent rows first (in their original order) and the dependent
// ones after.  Also returned: k and an estimate of cond(Gs) = ||Gs||_2 ||Gs^{-1}||_2
// from ||Gs||_inf and a power iteration on T_k^T T_k (the independent rows).
//
// Blocks of 64: one workgroup factors the diagonal block in LDS and inverts it;
// the panel below is L_ib,kb = A_ib,kb L_kk^{-T}; the trailing lower blocks take
// A_ib,jb -= L_ib,kb L_jb,kb^T.  The inverse of the whole lower-triangular factor is
// built by doubling: with X11, X22 the inverses of two neighbouring diagonal
// super-blocks, X21 = -X22 (L21 X11).  Everything is FP64.
#include "lrdm_internal.h"
#include "jacobi_order.h"

#include <algorithm>
#include <cmath>

namespace lrdm {
namespace {

constexpr int CB = 64;      // block size
constexpr int CP = CB + 1;  // LDS pitch
constexpr int kPowerSteps = 12;

// acc (thread (tr, tc) owns rows 4tr.., cols 4tc.. of a 64 x 64 tile; 256 threads)
// = X Y^T, with X and Y 64 x 64 in LDS (pitch CP).
__device__ inline void lds_gemm_abt(const double* X, const double* Y, double acc[4][4]) {
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k = 0; k < CB; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = X[(tr * 4 + i) * CP + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = Y[(tc * 4 + j) * CP + k];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
  }
}

// dinv_j = G_jj^{-1/2} (0 for a zero, negative or non-finite diagonal: that row is
// then dependent).
__global__ void chol_dinv_kernel(const double* __restrict__ G, int N, double* __restrict__ dinv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double d = G[(int64_t)i * N + i];
  dinv[i] = (d > 0.0 && d < __builtin_huge_val()) ? 1.0 / sqrt(d) : 0.0;
}

// A (Np x Np) = symmetrised D G D, padded with decoupled unit rows.
__global__ void chol_init_kernel(const double* __restrict__ G, const double* __restrict__ dinv,
                                 int N, int Np, double* __restrict__ A) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= Np || j >= Np) return;
  double v;
  if (i < N && j < N)
    v = 0.5 * (G[(int64_t)i * N + j] + G[(int64_t)j * N + i]) * dinv[i] * dinv[j];
  else
    v = (i == j) ? 1.0 : 0.0;
  A[(int64_t)i * Np + j] = v;
}

// Factor the diagonal block kb (dependent rows: zero column, unit diagonal) and
// write L_kk to A and its inverse to Linv[kb].  One wave: lane i keeps row i of
// the block in registers.  At column j every lane publishes its entry S_ij to an
// LDS column, and lane i applies S_il -= S_ij S_lj / S_jj for l > j (nothing for a
// dependent column); the entries as they stood when their column was eliminated
// give L.  The inverse follows by forward substitution, lane c taking column c.
// The chain of 64 eliminations runs inside one wave, so each step costs a few
// LDS accesses rather than a workgroup barrier.
__global__ __launch_bounds__(64) void chol_diag_kernel(double* __restrict__ A, int Np, int kb,
                                                       double tau, int* __restrict__ dead,
                                                       double* __restrict__ Linv) {
  __shared__ double col[CB];
  __shared__ double piv[CB];
  __shared__ double sq[CB];
  __shared__ double L[CB * CP];
  const int lane = threadIdx.x;
  const int64_t o = (int64_t)kb * CB;
  // rows through LDS, so that the global reads are coalesced
  for (int i = 0; i < CB; ++i) L[i * CP + lane] = A[(o + i) * Np + o + lane];
  __syncthreads();
  double r[CB];
#pragma unroll
  for (int l = 0; l < CB; ++l) r[l] = (l <= lane) ? L[lane * CP + l] : 0.0;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    col[lane] = r[j];
    __syncthreads();
    const double d = col[j];
    const double f = d > tau ? r[j] / d : 0.0;  // NaN is dependent
#pragma unroll
    for (int l = j + 1; l < CB; ++l) r[l] -= f * col[l];
    piv[j] = d;   // every lane stores the same value
    __syncthreads();
  }
  {
    const double d = piv[lane];
    sq[lane] = d > tau ? sqrt(d) : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int l = 0; l < CB; ++l) {
    const double s = sq[l];
    double x = 0.0;
    if (l < lane)
      x = s > 0.0 ? r[l] / s : 0.0;
    else if (l == lane)
      x = s > 0.0 ? s : 1.0;
    L[lane * CP + l] = x;
  }
  __syncthreads();
  // X = L^{-1}, column `lane`: x_i = (delta_ic - sum_{l<i} L_il x_l) / L_ii
  double x[CB];
#pragma unroll
  for (int i = 0; i < CB; ++i) {
    double sum = (i == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int l = 0; l < i; ++l) sum -= L[i * CP + l] * x[l];
    x[i] = sum / L[i * CP + i];
  }
  double* Li = Linv + (int64_t)kb * CB * CB;
#pragma unroll
  for (int i = 0; i < CB; ++i) {
    Li[i * CB + lane] = x[i];
    A[(o + i) * Np + o + lane] = L[i * CP + lane];
  }
  dead[o + lane] = piv[lane] > tau ? 0 : 1;
}

// Panel below the diagonal block: L_ib,kb = A_ib,kb Linv_kk^T, dependent columns zero.
__global__ __launch_bounds__(256) void chol_trsm_kernel(double* __restrict__ A, int Np, int kb,
                                                        const double* __restrict__ Linv,
                                                        const int* __restrict__ dead) {
  __shared__ double B[CB * CP];
  __shared__ double Xs[CB * CP];
  const int ib = kb + 1 + blockIdx.x;
  const int64_t r0 = (int64_t)ib * CB, c0 = (int64_t)kb * CB;
  const double* Li = Linv + (int64_t)kb * CB * CB;
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int i = e / CB, j = e % CB;
    B[i * CP + j] = A[(r0 + i) * Np + c0 + j];
    Xs[i * CP + j] = Li[e];
  }
  __syncthreads();
  double acc[4][4];
  lds_gemm_abt(B, Xs, acc);
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = tc * 4 + j;
      A[(r0 + tr * 4 + i) * Np + c0 + c] = dead[c0 + c] ? 0.0 : acc[i][j];
    }
}

// Trailing lower blocks: A_ib,jb -= L_ib,kb L_jb,kb^T for kb < jb <= ib < nb; block q
// of the launch is the q-th pair in row-major order of that triangle.
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ A, int Np, int kb) {
  __shared__ double X[CB * CP];
  __shared__ double Y[CB * CP];
  const int q = blockIdx.x;
  int a = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= q) ++a;
  while (a * (a + 1) / 2 > q) --a;
  const int b = q - a * (a + 1) / 2;
  const int64_t ri = (int64_t)(kb + 1 + a) * CB, rj = (int64_t)(kb + 1 + b) * CB;
  const int64_t c0 = (int64_t)kb * CB;
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int i = e / CB, j = e % CB;
    X[i * CP + j] = A[(ri + i) * Np + c0 + j];
    Y[i * CP + j] = A[(rj + i) * Np + c0 + j];
  }
  __syncthreads();
  double acc[4][4];
  lds_gemm_abt(X, Y, acc);
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) A[(ri + tr * 4 + i) * Np + rj + tc * 4 + j] -= acc[i][j];
}

// L with its strict upper triangle zeroed; X = block diagonal of the inverses.
__global__ void chol_finish_kernel(double* __restrict__ A, int Np, const double* __restrict__ Linv,
                                   double* __restrict__ X) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= Np || j >= Np) return;
  const int64_t e = (int64_t)i * Np + j;
  if (j > i) A[e] = 0.0;
  const int bi = i / CB, bj = j / CB;
  X[e] = (bi == bj) ? Linv[(int64_t)bi * CB * CB + (i % CB) * CB + (j % CB)] : 0.0;
}

// Batched C_z = alpha A_z B_z + beta C_z (row-major, no transposes), z = blockIdx.z
// with element strides sA, sB, sC; 64 x 64 tiles, 256 threads.
__global__ __launch_bounds__(256) void chol_bgemm_kernel(int m, int n, int k, double alpha,
                                                         const double* __restrict__ A, int lda,
                                                         int64_t sA, const double* __restrict__ B,
                                                         int ldb, int64_t sB, double beta,
                                                         double* __restrict__ C, int ldc,
                                                         int64_t sC) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  A += blockIdx.z * sA;
  B += blockIdx.z * sB;
  C += blockIdx.z * sC;
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < k; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e >> 6, r = e & 63;
      const int gi = i0 + r, gk = k0 + kk, gj = j0 + r;
      As[kk][r] = (gi < m && gk < k) ? A[(int64_t)gi * lda + gk] : 0.0;
      Bs[kk][r] = (gj < n && gk < k) ? B[(int64_t)gk * ldb + gj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gi = i0 + tr * 4 + i;
    if (gi >= m) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gj = j0 + tc * 4 + j;
      if (gj >= n) continue;
      double v = alpha * acc[i][j];
      if (beta != 0.0) v += beta * C[(int64_t)gi * ldc + gj];
      C[(int64_t)gi * ldc + gj] = v;
    }
  }
}

// Live-row permutation: perm[r] = index of the r-th independent row (r < k), the
// dependent rows after them; sc[2] = k.  One thread (N is at most a few thousand).
__global__ __launch_bounds__(1024) void chol_perm_kernel(const int* __restrict__ dead, int N,
                                                        int* __restrict__ perm,
                                                        double* __restrict__ sc) {
  // one block of 1024 threads: chunks of 1024 rows, a scan of the live flags per
  // chunk; live rows go to their rank, dependent rows after the k live ones
  __shared__ int scan[1024];
  __shared__ int base_live, total_live;
  const int t = threadIdx.x;
  if (t == 0) {
    int k = 0;
    for (int i = 0; i < N; ++i) k += dead[i] ? 0 : 1;   // N reads, once
    total_live = k;
    base_live = 0;
  }
  __syncthreads();
  const int k = total_live;
  for (int c0 = 0; c0 < N; c0 += 1024) {
    const int i = c0 + t;
    const int live = (i < N && !dead[i]) ? 1 : 0;
    scan[t] = live;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int v = t >= off ? scan[t - off] : 0;
      __syncthreads();
      scan[t] += v;
      __syncthreads();
    }
    const int before_live = base_live + scan[t] - live;   // live rows before i
    if (i < N) perm[live ? before_live : k + (i - before_live)] = i;
    __syncthreads();
    if (t == 1023) base_live += scan[1023];
    __syncthreads();
  }
  if (t == 0) sc[2] = (double)k;
}

// T[r][j] = X[perm[r]][j] (unscaled).
__global__ void chol_rows_kernel(const double* __restrict__ X, int Np, int N,
                                 const int* __restrict__ perm, const double* __restrict__ sc,
                                 double* __restrict__ T) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y * blockDim.y + threadIdx.y;
  if (r >= N || j >= N) return;
  T[(int64_t)r * N + j] = X[(int64_t)perm[r] * Np + j];
}

// rowsum[i] = sum_j |A[i][j]| (one block per row) ...
__global__ __launch_bounds__(256) void chol_rowsum_kernel(const double* __restrict__ A, int N,
                                                          int lda, double* __restrict__ rowsum) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) s += fabs(A[(int64_t)i * lda + j]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) rowsum[i] = red[0] + red[1] + red[2] + red[3];
}

// ... and *out = max_i rowsum[i] = ||A||_inf (NaN propagates); one block.
__global__ __launch_bounds__(256) void chol_max_kernel(const double* __restrict__ x, int N,
                                                       double* __restrict__ out) {
  __shared__ double red[4];
  double mx = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) mx = nan_max(mx, x[i]);
  for (int off = 32; off > 0; off >>= 1) mx = nan_max(mx, __shfl_down(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) *out = nan_max(nan_max(red[0], red[1]), nan_max(red[2], red[3]));
}

// y = T v over the rows i < kmax (one block per row; rows from kmax on give 0;
// kmax = sc[2] when sc is given, else N) ...
__global__ __launch_bounds__(256) void chol_mv_kernel(const double* __restrict__ T, int N,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ sc,
                                                      double* __restrict__ y) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const int k = sc ? (int)sc[2] : N;
  double s = 0.0;
  if (i < k)
    for (int j = threadIdx.x; j < N; j += blockDim.x) s += T[(int64_t)i * N + j] * v[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) y[i] = red[0] + red[1] + red[2] + red[3];
}

// ... and v = w / ||w||, sc[1] = ||w|| (the Rayleigh estimate of ||T^T T||_2 for a
// unit v).  One block.
__global__ __launch_bounds__(256) void chol_normalize_kernel(const double* __restrict__ w, int N,
                                                             double* __restrict__ v,
                                                             double* __restrict__ sc) {
  __shared__ double red[4];
  double s = 0.0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) s += w[j] * w[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double nrm = sqrt(red[0] + red[1] + red[2] + red[3]);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) v[j] = w[j] * inv;
  if (threadIdx.x == 0) sc[1] = nrm;
}

__global__ void chol_fill_kernel(double* __restrict__ v, int N) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  // a fixed start vector with no special structure: 1 + j/N, normalised later
  if (j < N) v[j] = (1.0 + (double)j / N) / sqrt((double)N);
}

// Tt = T^T (N x N).
__global__ void chol_transpose_kernel(const double* __restrict__ T, int N, double* __restrict__ Tt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i < N && j < N) Tt[(int64_t)j * N + i] = T[(int64_t)i * N + j];
}

// T[r][j] *= dinv[j]
__global__ void chol_scale_cols_kernel(double* __restrict__ T, int N,
                                       const double* __restrict__ dinv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y * blockDim.y + threadIdx.y;
  if (r >= N || j >= N) return;
  T[(int64_t)r * N + j] *= dinv[j];
}

}  // namespace

size_t chol_orth_bytes(int N) {
  const int Np = ((N + CB - 1) / CB) * CB;
  const int nb = Np / CB;
  size_t b = 0;
  b += 3 * ws_align((size_t)Np * Np * sizeof(double));      // A (then L'), X, tmp
  b += ws_align((size_t)nb * CB * CB * sizeof(double));     // diagonal-block inverses
  b += ws_align((size_t)Np * sizeof(int));                  // dependent-row flags
  b += ws_align((size_t)N * sizeof(int));                   // live-row permutation
  b += 3 * ws_align((size_t)N * sizeof(double));            // dinv, power-iteration vectors
  b += ws_align(4 * sizeof(double));                        // scalars
  return b;
}

lrdm_status chol_orth(lrdm_ctx* ctx, const double* G, int N, double tau, double* T,
                      CholInfo* info) {
  ProfScope prof(ctx, "chol");
  const int Np = ((N + CB - 1) / CB) * CB;
  const int nb = Np / CB;
  const size_t mark = ctx->ws_top;
  const size_t np2 = (size_t)Np * Np * sizeof(double);
  double* A = static_cast<double*>(ws_take(ctx, np2));
  double* X = static_cast<double*>(ws_take(ctx, np2));
  double* tmp = static_cast<double*>(ws_take(ctx, np2));
  double* Linv = static_cast<double*>(ws_take(ctx, (size_t)nb * CB * CB * sizeof(double)));
  int* dead = static_cast<int*>(ws_take(ctx, (size_t)Np * sizeof(int)));
  int* perm = static_cast<int*>(ws_take(ctx, (size_t)N * sizeof(int)));
  double* dinv = static_cast<double*>(ws_take(ctx, (size_t)N * sizeof(double)));
  double* pv = static_cast<double*>(ws_take(ctx, (size_t)N * sizeof(double)));
  double* pw = static_cast<double*>(ws_take(ctx, (size_t)N * sizeof(double)));
  double* sc = static_cast<double*>(ws_take(ctx, 4 * sizeof(double)));
  hipError_t e;
  auto fail = [&](hipError_t err) {
    ctx->err = std::string("orthonormalisation: ") + hipGetErrorString(err);
    return LRDM_EDEVICE;
  };
  const dim3 blk(32, 8);
  chol_dinv_kernel<<<(N + 255) / 256, 256, 0, ctx->stream>>>(G, N, dinv);
  chol_init_kernel<<<dim3((Np + 31) / 32, (Np + 7) / 8), blk, 0, ctx->stream>>>(G, dinv, N, Np, A);
  chol_rowsum_kernel<<<N, 256, 0, ctx->stream>>>(A, N, Np, pw);
  chol_max_kernel<<<1, 256, 0, ctx->stream>>>(pw, N, sc);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  for (int kb = 0; kb < nb; ++kb) {
    chol_diag_kernel<<<1, CB, 0, ctx->stream>>>(A, Np, kb, tau, dead, Linv);
    const int m = nb - kb - 1;
    if (m > 0) {
      chol_trsm_kernel<<<m, 256, 0, ctx->stream>>>(A, Np, kb, Linv, dead);
      chol_update_kernel<<<m * (m + 1) / 2, 256, 0, ctx->stream>>>(A, Np, kb);
    }
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  }
  chol_finish_kernel<<<dim3((Np + 31) / 32, (Np + 7) / 8), blk, 0, ctx->stream>>>(A, Np, Linv, X);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  // X = L'^{-1} by doubling: super-blocks [c0, c0 + h) and [c0 + h, c0 + h + h2)
  for (int h = CB; h < Np; h *= 2) {
    const int64_t step = 2 * (int64_t)h * (Np + 1);  // from one pair to the next
    const int full = Np / (2 * h);                   // pairs with h2 = h
    const int c_last = full * 2 * h, h2_last = std::min(h, Np - c_last - h);
    for (int part = 0; part < 2; ++part) {
      const int cnt = part == 0 ? full : (h2_last > 0 ? 1 : 0);
      if (cnt == 0) continue;
      const int c0 = part == 0 ? 0 : c_last;
      const int h2 = part == 0 ? h : h2_last;
      const int64_t r0 = c0 + h;
      // tmp = L21 X11   (h2 x h)
      chol_bgemm_kernel<<<dim3((h + 63) / 64, (h2 + 63) / 64, cnt), 256, 0, ctx->stream>>>(
          h2, h, h, 1.0, A + r0 * Np + c0, Np, step, X + (int64_t)c0 * Np + c0, Np, step, 0.0,
          tmp + r0 * Np + c0, Np, step);
      // X21 = -X22 tmp  (h2 x h)
      chol_bgemm_kernel<<<dim3((h + 63) / 64, (h2 + 63) / 64, cnt), 256, 0, ctx->stream>>>(
          h2, h, h2, -1.0, X + r0 * Np + r0, Np, step, tmp + r0 * Np + c0, Np, step, 0.0,
          X + r0 * Np + c0, Np, step);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    }
  }
  chol_perm_kernel<<<1, 1024, 0, ctx->stream>>>(dead, N, perm, sc);
  chol_rows_kernel<<<dim3((N + 31) / 32, (N + 7) / 8), blk, 0, ctx->stream>>>(X, Np, N, perm, sc,
                                                                              T);
  // ||Gs^{-1}||_2 on the independent rows = ||T_k^T T_k||_2 (unscaled T): power iteration
  chol_transpose_kernel<<<dim3((N + 31) / 32, (N + 7) / 8), blk, 0, ctx->stream>>>(T, N, tmp);
  chol_fill_kernel<<<(N + 255) / 256, 256, 0, ctx->stream>>>(pv, N);
  for (int it = 0; it < kPowerSteps; ++it) {
    chol_mv_kernel<<<N, 256, 0, ctx->stream>>>(T, N, pv, sc, pw);         // y = T_k v
    chol_mv_kernel<<<N, 256, 0, ctx->stream>>>(tmp, N, pw, nullptr, pv);  // w = T^T y
    chol_normalize_kernel<<<1, 256, 0, ctx->stream>>>(pv, N, pv, sc);
  }
  chol_scale_cols_kernel<<<dim3((N + 31) / 32, (N + 7) / 8), blk, 0, ctx->stream>>>(T, N, dinv);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  double h_sc[3];
  if ((e = hipMemcpyAsync(h_sc, sc, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream)) !=
      hipSuccess)
    return fail(e);
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return fail(e);
  info->live = (int)h_sc[2];
  info->cond = h_sc[0] * h_sc[1];
  ctx->ws_top = mark;
  return LRDM_OK;
}

}  // namespace lrdm

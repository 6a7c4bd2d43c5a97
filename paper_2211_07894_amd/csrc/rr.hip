// Rayleigh-Ritz step of ChFSI (Sec. II C, Eq. (15)) and the FP64 symmetric
// eigensolver it needs, both on the GPU.
//
// Orthonormalisation: column-scaled Cholesky QR of the filtered block Y (rows =
// vectors), with rank detection (chol.hip).  After a high-degree filter the rows'
// norms span many orders of magnitude and the top states of a cold block can be
// swamped by the lower ones; such rows are numerically dependent on the rest and
// are replaced by fixed pseudo-random rows, which a second Cholesky pass makes
// orthonormal to the others.  A warm-started block is well conditioned after the
// column scaling and takes one pass: one grid pass for the Gram matrix, one stencil
// pass, one pass for Y (HY)^T and one rotation pass.
//
// Eigensolver: two-sided block Jacobi.  The matrix (padded to a multiple of 64
// with decoupled diagonal entries 1e30) is cut into 32-wide blocks; each outer
// round pairs blocks by a round-robin tournament and a workgroup diagonalises
// each 64 x 64 pair problem in LDS with one sweep of cyclic Jacobi
// (1024 threads, one 2 x 2 block of the pair rotation per thread; rotations
// t = sign(z)/(|z| + sqrt(1 + z^2)), z = (a_qq - a_pp)/(2 a_pq), the angle in FP32
// and (c, s) normalised in FP64); a second kernel
// applies the pair rotations to A and to the eigenvector matrix as 64 x 64 GEMMs
// on FP64 matrix cores.
// Rotations are applied above 1e-16 ||A||_F; sweeps stop when an outer sweep
// leaves no off-diagonal entry above 1e-13 ||A||_F (a reduction after the sweep
// and one host read of its flag), about ten times the rounding left by the
// 64-wide rotation updates, so the stop is reachable.
#include "lrdm_internal.h"
#include "jacobi_order.h"

#include <algorithm>
#include <utility>
#include <vector>

namespace lrdm {
namespace {

constexpr int JB = 32;        // block width
constexpr int JS = 64;        // pair problem size
constexpr int JP = JS + 1;    // LDS pitch
static_assert(JB * JB == 1024, "the pair solve gives one 2 x 2 rotation block to each thread");
constexpr double kPad = 1e30; // diagonal of padding rows (decoupled, sorts last)
constexpr double kDependentTol = 1e-10;  // Schur pivot (unit diagonal) of a dependent row
// One Cholesky pass when cond(Gs) is below this: the basis T Y is then orthonormal
// to about u cond(Gs), 1e-13 for FP64 storage and 1e-9 (below the FP32 rounding
// of the stored Ritz vectors) for FP32 storage.
constexpr double kOnePassCond64 = 1e3;
constexpr double kOnePassCond32 = 1e7;
constexpr int kMaxOrthPasses = 5;        // Cholesky passes before giving up


// --------------------------------------------------------------- reductions
// Frobenius norm of the N x N matrix A (leading dimension lda): kFrobBlocks blocks
// write partial sums of squares (grid-stride over rows), then one block adds
// them in a fixed order.
constexpr int kFrobBlocks = 256;

__global__ __launch_bounds__(256) void frob_partial_kernel(const double* __restrict__ A, int N,
                                                           int lda, double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = blockIdx.x; i < N; i += gridDim.x)
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      const double v = A[(int64_t)i * lda + j];
      s += v * v;
    }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void frob_final_kernel(const double* __restrict__ part, int n,
                                                         double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// out = ||A||_F, with `part` kFrobBlocks doubles of scratch.
hipError_t frob(lrdm_ctx* ctx, const double* A, int N, int lda, double* part, double* out) {
  frob_partial_kernel<<<kFrobBlocks, 256, 0, ctx->stream>>>(A, N, lda, part);
  frob_final_kernel<<<1, 256, 0, ctx->stream>>>(part, kFrobBlocks, out);
  return hipGetLastError();
}

// --------------------------------------------------------------- block Jacobi
__global__ __launch_bounds__(1024) void jac_solve_kernel(const double* __restrict__ A, int Np,
                                                        int nb, int t,
                                                        const double* __restrict__ normF_ptr,
                                                        double* __restrict__ Ublk, int max_inner) {
  __shared__ double S[JS * JP];
  __shared__ double U[JS * JP];
  __shared__ double2 rcs[JB];   // (c, s) of the round's rotations
  __shared__ int2 rpq[JB];      // (p, q)
  __shared__ int any_rot;
  const int pair = blockIdx.x;
  const int bp = rr_pos(pair, t, nb), bq = rr_pos(nb - 1 - pair, t, nb);
  for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
    const int a = e / JS, c = e - a * JS;
    const int ga = a < JB ? bp * JB + a : bq * JB + (a - JB);
    const int gc = c < JB ? bp * JB + c : bq * JB + (c - JB);
    S[a * JP + c] = A[(int64_t)ga * Np + gc];
    U[a * JP + c] = (a == c) ? 1.0 : 0.0;
  }
  const double normF = *normF_ptr;
  const double thr_apply = 1e-16 * normF, thr_flag = 1e-13 * normF;
  __syncthreads();
  for (int sw = 0; sw < max_inner; ++sw) {
    if (threadIdx.x == 0) any_rot = 0;
    __syncthreads();
    for (int r = 0; r < JS - 1; ++r) {
      if (threadIdx.x < JB) {
        // The angle only steers convergence: any (c, s) with c^2 + s^2 = 1 is an
        // exact rotation, and every entry, the 2 x 2 diagonal block included, is
        // updated with the full formulas below.  So t is formed in FP32
        // (z = (a_qq - a_pp)/(2 a_pq), t = sign(z)/(|z| + sqrt(1 + z^2))), which
        // leaves a residual of about 1e-7 a_pq for the next sweep, and (c, s) is
        // normalised in FP64.  |z| beyond the FP32 range gives t = 0 (no rotation).
        const int i = threadIdx.x;
        const int p = rr_pos(i, r, JS), q = rr_pos(JS - 1 - i, r, JS);
        const double apq = S[p * JP + q], app = S[p * JP + p], aqq = S[q * JP + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > thr_apply) {
          const float z = (float)(aqq - app) * __builtin_amdgcn_rcpf((float)(2.0 * apq));
          const float az = fabsf(z);
          const float tf = __builtin_amdgcn_rcpf(az + sqrtf(1.0f + az * az));
          const double td = (z >= 0.0f ? 1.0 : -1.0) * (double)tf;
          // c = (1 + t^2)^{-1/2}: an FP32 estimate and two steps of Newton's
          // iteration y <- y (3 - x y^2) / 2 in FP64 (x in [1, 2])
          const double x = 1.0 + td * td;
          double y = (double)__builtin_amdgcn_rsqf((float)x);
          y = y * (1.5 - 0.5 * x * y * y);
          y = y * (1.5 - 0.5 * x * y * y);
          c = y;
          s = td * c;
          if (fabs(apq) > thr_flag) any_rot = 1;
        }
        rpq[i] = make_int2(p, q);
        rcs[i] = make_double2(c, s);
      }
      __syncthreads();
      // S <- J^T S J on the 32 x 32 pair blocks (rows, then columns), one per
      // thread (the workgroup has JB * JB threads); U <- U J for the thread's row
      // pair in rows be and be + 32
      {
        const int al = threadIdx.x >> 5, be = threadIdx.x & 31;
        const double2 ra = rcs[al], rb = rcs[be];
        const int2 ia = rpq[al], ib = rpq[be];
        if (ra.y != 0.0 || rb.y != 0.0) {
          const int p1 = ia.x, q1 = ia.y, p2 = ib.x, q2 = ib.y;
          const double ca = ra.x, sa = ra.y, cb = rb.x, sb = rb.y;
          const double b00 = S[p1 * JP + p2], b01 = S[p1 * JP + q2];
          const double b10 = S[q1 * JP + p2], b11 = S[q1 * JP + q2];
          const double x00 = ca * b00 - sa * b10, x01 = ca * b01 - sa * b11;
          const double x10 = sa * b00 + ca * b10, x11 = sa * b01 + ca * b11;
          S[p1 * JP + p2] = x00 * cb - x01 * sb;
          S[p1 * JP + q2] = x00 * sb + x01 * cb;
          S[q1 * JP + p2] = x10 * cb - x11 * sb;
          S[q1 * JP + q2] = x10 * sb + x11 * cb;
        }
        if (ra.y != 0.0) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int row = be + 32 * h;
            const double up = U[row * JP + ia.x], uq = U[row * JP + ia.y];
            U[row * JP + ia.x] = ra.x * up - ra.y * uq;
            U[row * JP + ia.y] = ra.y * up + ra.x * uq;
          }
        }
      }
      __syncthreads();
    }
    const int rot = any_rot;
    __syncthreads();
    if (!rot) break;
  }
  double* Ub = Ublk + (int64_t)pair * JS * JS;
  for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
    const int a = e / JS, c = e - a * JS;
    Ub[e] = U[a * JP + c];
  }
}

// *flag = 1 when an off-diagonal entry of the leading N x N block exceeds
// 1e-13 ||A||_F (blocks stride over rows; any thread that sees one stores 1).
__global__ __launch_bounds__(256) void jac_offmax_kernel(const double* __restrict__ A, int Np,
                                                         int N, const double* __restrict__ normF,
                                                         int* __restrict__ flag) {
  const double thr = 1e-13 * *normF;
  bool big = false;
  for (int i = blockIdx.x; i < N; i += gridDim.x)
    for (int j = threadIdx.x; j < N; j += blockDim.x)
      big |= (j != i) && fabs(A[(int64_t)i * Np + j]) > thr;
  if (big) *flag = 1;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// 64 x 64 x 64 product C = op(X) Y with X, Y in LDS (pitch JP), on FP64 matrix
// cores (v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16],
// and register v of lane l holds D[4v + l/16][l%16]).  Wave w of the 256 threads
// owns the 32 x 32 quadrant (w / 2, w % 2): acc[I][J] is its 16 x 16 tile (I, J).
// transX: C = X^T Y.
__device__ inline void lds_gemm64(const double* X, const double* Y, d4 (&acc)[2][2],
                                  bool transX) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J) acc[I][J] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < JS; k += 4) {
    double a[2], b[2];
#pragma unroll
    for (int I = 0; I < 2; ++I) {
      const int row = r0 + I * 16 + li;
      a[I] = transX ? X[(k + lk) * JP + row] : X[row * JP + k + lk];
    }
#pragma unroll
    for (int J = 0; J < 2; ++J) b[J] = Y[(k + lk) * JP + c0 + J * 16 + li];
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J)
        acc[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], b[J], acc[I][J], 0, 0, 0);
  }
}

// Row and column (within the 64 x 64 tile) of register v of the lane's tile (I, J).
__device__ inline int acc_row(int I, int v) {
  return ((threadIdx.x >> 6) >> 1) * 32 + I * 16 + 4 * v + ((threadIdx.x & 63) >> 4);
}
__device__ inline int acc_col(int J) {
  return ((threadIdx.x >> 6) & 1) * 32 + J * 16 + (threadIdx.x & 15);
}

// blocks [0, P*P): A(pair P rows, pair R cols) <- U_P^T A U_R
// blocks [P*P, P*P + (Np/64)*P): V(row block, pair P cols) <- V U_P
__global__ __launch_bounds__(256) void jac_update_kernel(double* __restrict__ A,
                                                         double* __restrict__ V, int Np, int nb,
                                                         int t, const double* __restrict__ Ublk) {
  // two 64 x 64 tiles of LDS (66 KB), so that two workgroups share a CU; U_R
  // takes U_P's place once U_P^T A is formed
  __shared__ double X[JS * JP];
  __shared__ double UL[JS * JP];
  const int np = nb / 2;
  int id = blockIdx.x;
  d4 acc[2][2];
  if (id < np * np) {
    const int P = id / np, R = id - P * np;
    const int p1 = rr_pos(P, t, nb), q1 = rr_pos(nb - 1 - P, t, nb);
    const int p2 = rr_pos(R, t, nb), q2 = rr_pos(nb - 1 - R, t, nb);
    const double* UPg = Ublk + (int64_t)P * JS * JS;
    const double* URg = Ublk + (int64_t)R * JS * JS;
    for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
      const int a = e / JS, c = e - a * JS;
      const int ga = a < JB ? p1 * JB + a : q1 * JB + (a - JB);
      const int gc = c < JB ? p2 * JB + c : q2 * JB + (c - JB);
      X[a * JP + c] = A[(int64_t)ga * Np + gc];
      UL[a * JP + c] = UPg[e];
    }
    __syncthreads();
    lds_gemm64(UL, X, acc, true);   // U_P^T A
    __syncthreads();
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J)
#pragma unroll
        for (int v = 0; v < 4; ++v) X[acc_row(I, v) * JP + acc_col(J)] = acc[I][J][v];
    for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
      const int a = e / JS, c = e - a * JS;
      UL[a * JP + c] = URg[e];
    }
    __syncthreads();
    lds_gemm64(X, UL, acc, false);  // (U_P^T A) U_R
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = acc_row(I, v);
        const int ga = a < JB ? p1 * JB + a : q1 * JB + (a - JB);
#pragma unroll
        for (int J = 0; J < 2; ++J) {
          const int c = acc_col(J);
          const int gc = c < JB ? p2 * JB + c : q2 * JB + (c - JB);
          A[(int64_t)ga * Np + gc] = acc[I][J][v];
        }
      }
  } else {
    id -= np * np;
    const int P = id % np, rb = id / np;
    const int p1 = rr_pos(P, t, nb), q1 = rr_pos(nb - 1 - P, t, nb);
    const double* UPg = Ublk + (int64_t)P * JS * JS;
    for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
      const int a = e / JS, c = e - a * JS;
      const int gc = c < JB ? p1 * JB + c : q1 * JB + (c - JB);
      X[a * JP + c] = V[(int64_t)(rb * JS + a) * Np + gc];
      UL[a * JP + c] = UPg[e];
    }
    __syncthreads();
    lds_gemm64(X, UL, acc, false);
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = acc_row(I, v);
#pragma unroll
        for (int J = 0; J < 2; ++J) {
          const int c = acc_col(J);
          const int gc = c < JB ? p1 * JB + c : q1 * JB + (c - JB);
          V[(int64_t)(rb * JS + a) * Np + gc] = acc[I][J][v];
        }
      }
  }
}

// Copy an N x N matrix (leading dim lda) into Np x Np work with decoupled padding
// and set V = I.  Optional symmetric diagonal scaling by dinv.
__global__ void jac_init_kernel(const double* __restrict__ src, int lda, int N, int Np,
                                const double* __restrict__ dinv, double* __restrict__ A,
                                double* __restrict__ V) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= Np || j >= Np) return;
  double v;
  if (i < N && j < N) {
    // symmetrise: 0.5 (S_ij + S_ji)
    v = 0.5 * (src[(int64_t)i * lda + j] + src[(int64_t)j * lda + i]);
    if (dinv) v *= dinv[i] * dinv[j];
  } else {
    v = (i == j) ? kPad : 0.0;
  }
  A[(int64_t)i * Np + j] = v;
  V[(int64_t)i * Np + j] = (i == j) ? 1.0 : 0.0;
}

// Ascending order of diag(A) by rank (ties by index, NaN last): always a
// permutation, so the gather below stays in bounds whatever the data.
// The diagonal is staged in LDS (Np doubles of dynamic shared memory).
__global__ void jac_rank_kernel(const double* __restrict__ A, int Np, int* __restrict__ perm) {
  extern __shared__ __attribute__((aligned(16))) unsigned char diag_raw[];
  double* diag_lds = reinterpret_cast<double*>(diag_raw);
  for (int i = threadIdx.x; i < Np; i += blockDim.x) diag_lds[i] = A[(int64_t)i * (Np + 1)];
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Np) return;
  perm[order_rank(diag_lds, 1, Np, k)] = k;
}

__global__ void jac_gather_kernel(const double* __restrict__ A, const double* __restrict__ V,
                                  int Np, int N, const int* __restrict__ perm,
                                  double* __restrict__ evals, double* __restrict__ evecs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;  // eigen index
  const int i = blockIdx.y * blockDim.y + threadIdx.y;  // component
  if (k >= N || i >= N) return;
  const int src = min(max(perm[k], 0), Np - 1);
  if (i == 0 && evals) evals[k] = A[(int64_t)src * Np + src];
  evecs[(int64_t)i * N + k] = V[(int64_t)i * Np + src];
}

// --------------------------------------------------------------- small FP64 GEMM
// C[m x n] = alpha op(A) op(B) + beta C, op = transpose when the flag is set.
// 64 x 64 tiles, 256 threads, 4 x 4 per thread, K steps of 16.
// When *skip is set (skip may be null) the block does no product: it copies its
// tile of copy_src (leading dimension ldc) into C, or leaves C alone when
// copy_src is null.
__global__ __launch_bounds__(256) void small_gemm_kernel(int ta, int tb, int m, int n, int k,
                                                         double alpha, const double* __restrict__ A,
                                                         int lda, const double* __restrict__ B,
                                                         int ldb, double beta,
                                                         double* __restrict__ C, int ldc,
                                                         const int* __restrict__ skip,
                                                         const double* __restrict__ copy_src) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  if (skip && *skip) {
    if (copy_src) {
      for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int gi = i0 + (e >> 6), gj = j0 + (e & 63);
        if (gi < m && gj < n) C[(int64_t)gi * ldc + gj] = copy_src[(int64_t)gi * ldc + gj];
      }
    }
    return;
  }
  double acc[4][4] = {};
  for (int k0 = 0; k0 < k; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e >> 6, r = e & 63;
      const int gi = i0 + r, gk = k0 + kk, gj = j0 + r;
      double a = 0.0, b = 0.0;
      if (gi < m && gk < k) a = ta ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
      if (gj < n && gk < k) b = tb ? B[(int64_t)gj * ldb + gk] : B[(int64_t)gk * ldb + gj];
      As[kk][r] = a;
      Bs[kk][r] = b;
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

hipError_t small_gemm(lrdm_ctx* ctx, bool ta, bool tb, int m, int n, int k, double alpha,
                      const double* A, int lda, const double* B, int ldb, double beta, double* C,
                      int ldc, const int* skip = nullptr, const double* copy_src = nullptr) {
  dim3 grd((n + 63) / 64, (m + 63) / 64);
  small_gemm_kernel<<<grd, 256, 0, ctx->stream>>>(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta,
                                                  C, ldc, skip, copy_src);
  return hipGetLastError();
}

// --------------------------------------------------------------- RR helpers
// Wt = T^T (N x N).
__global__ void transpose_kernel(const double* __restrict__ T, int N, double* __restrict__ Wt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i < N && j < N) Wt[(int64_t)j * N + i] = T[(int64_t)i * N + j];
}

// splitmix64 output function (Steele, Lea and Flood, OOPSLA 2014) of a 64-bit counter.
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Rows r in [k, N) of Z (row length M): uniform values on [-sqrt(3/M), sqrt(3/M))
// keyed by (r, p), so that each row has unit expected norm; a fixed function of
// the indices, hence the same on every call.
template <typename T>
__global__ void fill_rows_kernel(T* __restrict__ Z, int N, int64_t M, int k) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = k + blockIdx.y;
  if (p >= M || r >= N) return;
  const uint64_t z = splitmix64((uint64_t)r * (uint64_t)M + (uint64_t)p);
  const double u = (double)(z >> 11) * 0x1.0p-53;  // [0, 1)
  Z[(int64_t)r * M + p] = (T)((2.0 * u - 1.0) * sqrt(3.0 / (double)M));
}

}  // namespace

// Eigen-decomposition of a symmetric N x N matrix S (leading dim lda): evals
// ascending [N], evecs [N][N] with column k the k-th eigenvector.  dinv, when
// given, scales S symmetrically first.
lrdm_status sym_eigh(lrdm_ctx* ctx, const double* S, int lda, int N, const double* dinv,
                     double* evals, double* evecs) {
  ProfScope prof(ctx, "eigh");
  const int Np = ((N + JS - 1) / JS) * JS;
  const int nb = Np / JB;
  double* A = static_cast<double*>(ws_take(ctx, (size_t)Np * Np * sizeof(double)));
  double* V = static_cast<double*>(ws_take(ctx, (size_t)Np * Np * sizeof(double)));
  double* Ublk = static_cast<double*>(ws_take(ctx, (size_t)(nb / 2) * JS * JS * sizeof(double)));
  double* normF = static_cast<double*>(ws_take(ctx, 256));
  double* fpart = static_cast<double*>(ws_take(ctx, kFrobBlocks * sizeof(double)));
  int* perm = static_cast<int*>(ws_take(ctx, (size_t)Np * sizeof(int)));
  int* flag = ctx->dstatus + LRDM_DS_COUNT;  // scratch word next to the status words
  auto fail = [&](hipError_t e) {
    ctx->err = std::string("eigensolver: ") + hipGetErrorString(e);
    return LRDM_EDEVICE;
  };
  hipError_t e;
  {
    dim3 blk(32, 8), grd((Np + 31) / 32, (Np + 7) / 8);
    jac_init_kernel<<<grd, blk, 0, ctx->stream>>>(S, lda, N, Np, dinv, A, V);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  }
  if ((e = frob(ctx, A, N, Np, fpart, normF)) != hipSuccess) return fail(e);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  const int max_sweeps = ctx->eigh_max_sweeps;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    ProfScope prof_sweep(ctx, "jac_sweep");
    if ((e = hipMemsetAsync(flag, 0, sizeof(int), ctx->stream)) != hipSuccess) return fail(e);
    for (int t = 0; t < nb - 1; ++t) {
      {
        ProfScope prof_solve(ctx, "jac_solve");
        jac_solve_kernel<<<nb / 2, 1024, 0, ctx->stream>>>(A, Np, nb, t, normF, Ublk, 1);
      }
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      const int np = nb / 2;
      {
        ProfScope prof_update(ctx, "jac_update");
        jac_update_kernel<<<np * np + (Np / JS) * np, 256, 0, ctx->stream>>>(A, V, Np, nb, t, Ublk);
      }
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    }
    jac_offmax_kernel<<<kFrobBlocks, 256, 0, ctx->stream>>>(A, Np, N, normF, flag);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    int host_flag = 0;
    if ((e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream)) !=
        hipSuccess)
      return fail(e);
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return fail(e);
    if (!host_flag) break;
  }
  if (sweep == max_sweeps) {
    // the host already waited on the convergence flag: unconverged Ritz pairs are
    // reported whatever the checking level, never passed on
    ctx->err = "eigensolver: no convergence in " + std::to_string(max_sweeps) + " sweeps";
    return LRDM_ENOTCONV;
  }
  jac_rank_kernel<<<(Np + 255) / 256, 256, (size_t)Np * sizeof(double), ctx->stream>>>(A, Np, perm);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  dim3 blk(32, 8), grd((N + 31) / 32, (N + 7) / 8);
  jac_gather_kernel<<<grd, blk, 0, ctx->stream>>>(A, V, Np, N, perm, evals, evecs);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  return LRDM_OK;
}

size_t rr_workspace_bytes(int N, int64_t M, lrdm_prec prec) {
  const int Np = ((N + JS - 1) / JS) * JS;
  const int nb = Np / JB;
  const size_t s = prec == LRDM_FP64 ? sizeof(double) : sizeof(float);
  size_t b = 0;
  b += ws_align((size_t)M * N * sizeof(double));            // H B, later Psi_R
  b += ws_align((size_t)M * N * s);                         // completed basis Z
  b += 6 * ws_align((size_t)N * N * sizeof(double));         // G, Hy, T, C, X, Wt
  b += ws_align((size_t)N * N * sizeof(double));             // eigenvectors
  size_t inner = chol_orth_bytes(N);
  // eigensolver
  inner = std::max(inner, 2 * ws_align((size_t)Np * Np * sizeof(double)) +
                              ws_align((size_t)(nb / 2) * JS * JS * 8) + ws_align(256) +
                              ws_align((size_t)Np * 4) + ws_align(kFrobBlocks * sizeof(double)));
  inner = std::max(inner, ws_align(tn_workspace_bytes(N, M, 1, prec)));
  if (prec == LRDM_BF16X3) inner = std::max(inner, rotate_bf16x3_bytes(N, M));
  return b + inner;
}

// Psi (N rows of M points, filtered block Y on entry) -> Ritz vectors, eps ascending.
// Orthonormal basis: B = Y and T = factor of B B^T; while T leaves dependent rows or
// cond(Gs) is too large for one pass, the next pass takes B <- T B (independent rows first,
// then the explicit residuals of the dependent ones; from the second pass on, rows
// still dependent are replaced by fixed pseudo-random rows) and refactors.  A
// warm-started block takes one pass, an ill-conditioned one two (Cholesky QR
// twice), a numerically rank-deficient one three.  Then
//   Hhat = T (B (H B)^T) T^T = Q E Q^T, eps = E, Psi_R = Q^T T B.
template <typename T>
lrdm_status rayleigh_ritz(lrdm_ctx* ctx, const Grid3& g, const double* V, T* Psi, int N,
                          lrdm_prec prec, double* eps) {
  const int64_t M = g.M;
  const size_t nn = (size_t)N * N * sizeof(double);
  // H B in FP64 whatever the storage type (later reused for Psi_R in type T)
  double* HY = static_cast<double*>(ws_take(ctx, (size_t)M * N * sizeof(double)));
  T* Z = static_cast<T*>(ws_take(ctx, (size_t)M * N * sizeof(T)));
  double* G = static_cast<double*>(ws_take(ctx, nn));
  double* Hy = static_cast<double*>(ws_take(ctx, nn));
  double* Tm = static_cast<double*>(ws_take(ctx, nn));
  double* C = static_cast<double*>(ws_take(ctx, nn));
  double* X = static_cast<double*>(ws_take(ctx, nn));
  double* Wt = static_cast<double*>(ws_take(ctx, nn));
  double* Ug = static_cast<double*>(ws_take(ctx, nn));
  hipError_t e;
  auto fail = [&](const char* what, hipError_t err) {
    ctx->err = std::string("rayleigh_ritz: ") + what + ": " + hipGetErrorString(err);
    return LRDM_EDEVICE;
  };
  const size_t mark = ctx->ws_top;
  const dim3 blk(32, 8), grd((N + 31) / 32, (N + 7) / 8);
  // Every contraction here runs in FP64 arithmetic, and H B is formed and kept in
  // FP64, whatever the storage type of the block: a filtered block's rows span many
  // orders of magnitude (1e-11 .. 1 at the 64^3 / 1024-state workload), so its
  // Gram matrix and the orthonormalising coefficients need FP64 products.
  T* B = Psi;
  T* spare = Z;
  CholInfo ci;
  // Out = Wt^T Bsrc: FP64 matrix cores, or in the BF16X3 form the split-operand
  // product on BF16 matrix cores (its scratch in the region after `mark`)
  auto rotate = [&](const T* Bsrc, T* Out, bool upper) -> hipError_t {
    if constexpr (sizeof(T) == sizeof(float)) {
      if (prec == LRDM_BF16X3) {
        ctx->ws_top = mark;
        const hipError_t err = launch_rotate_bf16x3(ctx, Wt, Bsrc, Out, N, M, upper);
        ctx->ws_top = mark;   // the split operands are free again once the product is queued
        return err;
      }
    }
    return launch_nn_f64<T>(ctx, Wt, Bsrc, Out, N, M, upper);
  };
  for (int pass = 0;; ++pass) {
    if (pass > 0) {
      if (pass == kMaxOrthPasses) {
        ctx->err = "rayleigh_ritz: the block could not be orthonormalised";
        return LRDM_ENOTCONV;
      }
      transpose_kernel<<<grd, blk, 0, ctx->stream>>>(Tm, N, Wt);
      // with every row independent the factor is lower triangular (no reordering)
      if ((e = rotate(B, spare, ci.live == N)) != hipSuccess) return fail("rotation", e);
      if (pass > 1 && ci.live < N) {
        fill_rows_kernel<T><<<dim3((unsigned)((M + 255) / 256), N - ci.live), 256, 0,
                              ctx->stream>>>(spare, N, M, ci.live);
        if ((e = hipGetLastError()) != hipSuccess) return fail("fill", e);
      }
      std::swap(B, spare);
    }
    if ((e = launch_tn_sym_f64<T, T>(ctx, B, nullptr, nullptr, 0, N, M, 1, 1, G)) != hipSuccess)
      return fail("gram", e);
    ctx->ws_top = mark;
    lrdm_status st = chol_orth(ctx, G, N, kDependentTol, Tm, &ci);
    if (st != LRDM_OK) return st;
    if (ci.live == N && ci.cond < (sizeof(T) == sizeof(double) ? kOnePassCond64 : kOnePassCond32))
      break;
  }
  // H B and B (H B)^T
  if ((e = launch_hpsi_f64<T>(ctx, g, V, B, HY, N)) != hipSuccess) return fail("stencil", e);
  if ((e = launch_tn_sym_f64<T, double>(ctx, B, HY, nullptr, 0, N, M, 1, 1, Hy)) != hipSuccess)
    return fail("projection", e);
  ctx->ws_top = mark;
  // C = T Hy T^T
  if ((e = small_gemm(ctx, false, false, N, N, N, 1.0, Tm, N, Hy, N, 0.0, X, N)) != hipSuccess)
    return fail("gemm", e);
  if ((e = small_gemm(ctx, false, true, N, N, N, 1.0, X, N, Tm, N, 0.0, C, N)) != hipSuccess)
    return fail("gemm", e);
  lrdm_status st = sym_eigh(ctx, C, N, N, nullptr, eps, Ug);
  if (st != LRDM_OK) return st;
  ctx->ws_top = mark;
  // Psi_R = Q^T T B: the rotation kernel computes Wt^T B with Wt = T^T Q
  if ((e = small_gemm(ctx, true, false, N, N, N, 1.0, Tm, N, Ug, N, 0.0, Wt, N)) != hipSuccess)
    return fail("gemm", e);
  if (B != Psi || (sizeof(T) == sizeof(float) && prec == LRDM_BF16X3)) {
    if ((e = rotate(B, Psi, false)) != hipSuccess) return fail("rotation", e);
    return LRDM_OK;
  }
  T* PR = reinterpret_cast<T*>(HY);
  if ((e = launch_nn_f64<T>(ctx, Wt, Psi, PR, N, M)) != hipSuccess) return fail("rotation", e);
  if ((e = hipMemcpyAsync(Psi, PR, (size_t)M * N * sizeof(T), hipMemcpyDeviceToDevice,
                          ctx->stream)) != hipSuccess)
    return fail("copy", e);
  return LRDM_OK;
}

template lrdm_status rayleigh_ritz<double>(lrdm_ctx*, const Grid3&, const double*, double*, int,
                                           lrdm_prec, double*);
template lrdm_status rayleigh_ritz<float>(lrdm_ctx*, const Grid3&, const double*, float*, int,
                                          lrdm_prec, double*);

// ------------------------------------------------------ Rayleigh-Ritz of H_k
// The complex subspace of one k-point (Sec. II C, last paragraph) is handled as
// a real one: the N complex states y_i and their multiples i y_i are 2N real
// vectors [Re | Im] of length 2M, whose real inner products are the real parts
// of the complex ones and on which H_k acts as the real symmetric operator
// [[Re H_k, -Im H_k], [Im H_k, Re H_k]].  Rayleigh-Ritz of that operator on the
// 2N real vectors (the Cholesky factor, the block Jacobi eigensolver and the
// rotations of the real path) gives every Ritz value of H_k twice: multiplication
// by i maps each eigenspace of the real form onto itself, so a complex Ritz value
// of multiplicity d is a cluster of 2d real Ritz values whose vectors span d
// complex dimensions.  Clusters are runs of real Ritz values with consecutive
// gaps below 1e-8 of the spectrum's scale (two copies of one value differ by
// rounding only).  A cluster of two gives one complex Ritz vector, either real
// vector of the pair.  A larger one (a degenerate or nearly degenerate multiplet)
// takes its complex overlaps <psi_a, psi_b>, a pivoted complex Gram-Schmidt that
// picks d orthonormal combinations, and the d x d Hermitian projection of H_k on
// them, diagonalised by complex Jacobi rotations; the cluster must span exactly
// d complex dimensions, or the call reports ENOTCONV.
namespace {

constexpr int kPairMax = 64;           // real Ritz values per cluster (2 d)
constexpr int kPairRow = 4 * kPairMax; // scratch entries per real Ritz vector
constexpr double kClusterTol = 1e-8;   // cluster gap, relative to the spectrum's scale

struct cplx {
  double re, im;
};
__device__ inline cplx c_mul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ inline cplx c_conj_mul(cplx a, cplx b) {   // conj(a) b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__device__ inline double c_abs2(cplx a) { return a.re * a.re + a.im * a.im; }

// B [2N][2M]: the 2N real vectors [Re | Im] of the states y_i, i y_i, from Y
// [2][N][M] (real parts, then imaginary parts).  Each real vector is one row of
// length 2M, so the Gram matrix, the projection and the rotations of the 2N
// vectors are the real path's products with K = 2M.
template <typename T>
__global__ void realify_kernel(const T* __restrict__ Y, int N, int64_t M, T* __restrict__ B) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (p >= M) return;
  const T yr = Y[(int64_t)i * M + p], yi = Y[((int64_t)N + i) * M + p];
  const int64_t m2 = 2 * M;
  B[(int64_t)i * m2 + p] = yr;
  B[(int64_t)i * m2 + M + p] = yi;
  B[((int64_t)N + i) * m2 + p] = -yi;
  B[((int64_t)N + i) * m2 + M + p] = yr;
}

__global__ void zero_int_kernel(int* __restrict__ x) { *x = 0; }

// *out = min_i G_ii over the n x n matrix G (a non-finite or negative entry counts
// as 0).
__global__ __launch_bounds__(256) void min_diag_kernel(const double* __restrict__ G, int n,
                                                       double* __restrict__ out) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double m = __builtin_huge_val();
  for (int i = t; i < n; i += 256) {
    double v = G[(int64_t)i * n + i];
    if (!(v > 0.0 && v < __builtin_huge_val())) v = 0.0;
    m = fmin(m, v);
  }
  red[t] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmin(red[t], red[t + w]);
    __syncthreads();
  }
  if (t == 0) *out = red[0];
}

// Cluster gap of the ascending real Ritz values e2 [n2].
__device__ inline double cluster_tol(const double* e2, int n2) {
  const double scale = fmax(fmax(fabs(e2[0]), fabs(e2[n2 - 1])), e2[n2 - 1] - e2[0]);
  return kClusterTol * scale;
}

// cs, cn [n2]: first index and size of each real Ritz value's cluster.
__global__ void cluster_kernel(const double* __restrict__ e2, int n2, int* __restrict__ cs,
                               int* __restrict__ cn) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n2) return;
  const double tol = cluster_tol(e2, n2);
  int a = m, b = m + 1;
  while (a > 0 && e2[a] - e2[a - 1] <= tol) --a;
  while (b < n2 && e2[b] - e2[b - 1] <= tol) ++b;
  cs[m] = a;
  cn[m] = b - a;
}

// Complex overlaps <psi_a, psi_b> of real Ritz vector a (one block) with every
// member b of its cluster, for clusters of four or more; R [n2][2M].
template <typename T>
__global__ __launch_bounds__(256) void cluster_overlap_kernel(const T* __restrict__ R,
                                                              const int* __restrict__ cs,
                                                              const int* __restrict__ cn, int n2,
                                                              int64_t M, cplx* __restrict__ scr) {
  __shared__ double red[2][256];
  const int a = blockIdx.x, t = threadIdx.x;
  const int s = cs[a], n = cn[a];
  if (n < 4 || n > kPairMax) return;
  const T* ar = R + (int64_t)a * 2 * M;
  const T* ai = ar + M;
  for (int j = 0; j < n; ++j) {
    const T* br = R + (int64_t)(s + j) * 2 * M;
    const T* bi = br + M;
    double re = 0.0, im = 0.0;
    for (int64_t p = t; p < M; p += 256) {
      const double xr = ar[p], xi = ai[p], yr = br[p], yi = bi[p];
      re += xr * yr + xi * yi;
      im += xr * yi - xi * yr;
    }
    red[0][t] = re;
    red[1][t] = im;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) {
        red[0][t] += red[0][t + w];
        red[1][t] += red[1][t + w];
      }
      __syncthreads();
    }
    if (t == 0) scr[(size_t)a * kPairRow + j] = cplx{red[0][0], red[1][0]};
    __syncthreads();
  }
}

// One thread per cluster (its first index m): the d = n/2 complex Ritz pairs of
// the cluster, written to outputs m/2 .. m/2 + d - 1 as coefficients over the
// cluster's real Ritz vectors (coef [N][kPairMax]), with ostart / osize naming
// the cluster.  flag = 1 when a cluster has an odd size or more than kPairMax
// members, or does not span exactly d complex dimensions.
__global__ void cluster_pair_kernel(const double* __restrict__ e2, const int* __restrict__ cs,
                                    const int* __restrict__ cn, int N, cplx* __restrict__ scr,
                                    cplx* __restrict__ coef, int* __restrict__ ostart,
                                    int* __restrict__ osize, double* __restrict__ eps,
                                    int* __restrict__ flag) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int n2 = 2 * N;
  if (m >= n2 || cs[m] != m) return;
  const int n = cn[m];
  if ((n & 1) || n > kPairMax) {
    atomicOr(flag, 1);
    return;
  }
  const int d = n / 2, o0 = m / 2;
  cplx* row0 = scr + (size_t)m * kPairRow;
  cplx* C = coef + (size_t)o0 * kPairMax;
  if (n == 2) {   // one complex Ritz vector: the first real one of the pair
    C[0] = cplx{1.0, 0.0};
    C[1] = cplx{0.0, 0.0};
    ostart[o0] = m;
    osize[o0] = 2;
    eps[o0] = e2[m];
    return;
  }
  // scratch rows m .. m+n-1: S | S C_k | projected H_k | Jacobi vectors
  auto S = [&](int j, int l) -> cplx& { return row0[(size_t)j * kPairRow + l]; };
  auto SC = [&](int k, int l) -> cplx& { return row0[(size_t)k * kPairRow + kPairMax + l]; };
  auto Hc = [&](int k, int l) -> cplx& { return row0[(size_t)k * kPairRow + 2 * kPairMax + l]; };
  auto W = [&](int k, int l) -> cplx& { return row0[(size_t)k * kPairRow + 3 * kPairMax + l]; };
  auto Cc = [&](int k, int l) -> cplx& { return C[(size_t)k * kPairMax + l]; };
  // S v into SC row k, for v = C_k
  auto apply_s = [&](int k) {
    for (int j = 0; j < n; ++j) {
      cplx acc{0.0, 0.0};
      for (int l = 0; l < n; ++l) {
        const cplx x = c_mul(S(j, l), Cc(k, l));
        acc.re += x.re;
        acc.im += x.im;
      }
      SC(k, j) = acc;
    }
  };
  // pivoted complex Gram-Schmidt: C_k (rows of coefficients), orthonormal in S
  unsigned long long used = 0;
  for (int k = 0; k < d; ++k) {
    int best = -1;
    double bestn = -1.0;
    for (int l = 0; l < n; ++l) {
      if ((used >> l) & 1ull) continue;
      double nv = S(l, l).re;
      for (int q = 0; q < k; ++q) nv -= c_abs2(SC(q, l));   // |<phi_q, psi_l>|^2
      if (nv > bestn) {
        bestn = nv;
        best = l;
      }
    }
    if (bestn < 1e-4) {
      atomicOr(flag, 1);
      return;
    }
    used |= 1ull << best;
    for (int l = 0; l < n; ++l) Cc(k, l) = cplx{l == best ? 1.0 : 0.0, 0.0};
    for (int pass = 0; pass < 2; ++pass) {
      apply_s(k);
      for (int q = 0; q < k; ++q) {
        cplx o{0.0, 0.0};   // <phi_q, v> = C_q^H S v
        for (int j = 0; j < n; ++j) {
          const cplx x = c_conj_mul(Cc(q, j), SC(k, j));
          o.re += x.re;
          o.im += x.im;
        }
        for (int l = 0; l < n; ++l) {
          const cplx x = c_mul(o, Cc(q, l));
          Cc(k, l).re -= x.re;
          Cc(k, l).im -= x.im;
        }
      }
    }
    apply_s(k);
    double nrm = 0.0;
    for (int j = 0; j < n; ++j) nrm += c_conj_mul(Cc(k, j), SC(k, j)).re;
    const double inv = 1.0 / sqrt(nrm);
    for (int j = 0; j < n; ++j) {
      Cc(k, j).re *= inv;
      Cc(k, j).im *= inv;
      SC(k, j).re *= inv;
      SC(k, j).im *= inv;
    }
  }
  // the cluster spans exactly d complex dimensions: nothing of any member is left
  for (int l = 0; l < n; ++l) {
    double res = S(l, l).re;
    for (int k = 0; k < d; ++k) res -= c_abs2(SC(k, l));
    if (res > 1e-6) {
      atomicOr(flag, 1);
      return;
    }
  }
  // projected H_k on the combinations: <psi_j, H psi_l> = (e_j + e_l)/2 <psi_j, psi_l>
  // (exact for Ritz vectors, whose real Ritz values differ only inside one eigenspace)
  for (int k2 = 0; k2 < d; ++k2)
    for (int j = 0; j < n; ++j) {
      cplx acc{0.0, 0.0};
      for (int l = 0; l < n; ++l) {
        const double h = 0.5 * (e2[m + j] + e2[m + l]);
        const cplx x = c_mul(S(j, l), Cc(k2, l));
        acc.re += h * x.re;
        acc.im += h * x.im;
      }
      W(k2, j) = acc;   // (Hs C_k2)_j
    }
  for (int k = 0; k < d; ++k)
    for (int k2 = 0; k2 < d; ++k2) {
      cplx acc{0.0, 0.0};
      for (int j = 0; j < n; ++j) {
        const cplx x = c_conj_mul(Cc(k, j), W(k2, j));
        acc.re += x.re;
        acc.im += x.im;
      }
      Hc(k, k2) = acc;
    }
  for (int k = 0; k < d; ++k) {
    Hc(k, k).im = 0.0;
    for (int k2 = k + 1; k2 < d; ++k2) {
      const cplx a = Hc(k, k2), b = Hc(k2, k);
      Hc(k, k2) = cplx{0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
      Hc(k2, k) = cplx{Hc(k, k2).re, -Hc(k, k2).im};
    }
    for (int k2 = 0; k2 < d; ++k2) W(k, k2) = cplx{k == k2 ? 1.0 : 0.0, 0.0};
  }
  // cyclic complex Jacobi: for a_pq = r e^{i phi}, G = diag(1, e^{-i phi}) R(theta)
  // on rows / columns p, q makes the (p, q) entry zero
  const double scale = fmax(fabs(e2[m]), fabs(e2[m + n - 1])) + 1e-300;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) off += c_abs2(Hc(p, q));
    if (sqrt(off) <= 1e-15 * scale) break;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) {
        const double r = sqrt(c_abs2(Hc(p, q)));
        if (r <= 1e-300) continue;
        const cplx ph{Hc(p, q).re / r, Hc(p, q).im / r};
        const cplx phc{ph.re, -ph.im};
        const double tau = (Hc(q, q).re - Hc(p, p).re) / (2.0 * r);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        for (int k = 0; k < d; ++k) {   // columns: X <- X G
          const cplx xp = Hc(k, p), xq = c_mul(phc, Hc(k, q));
          Hc(k, p) = cplx{c * xp.re - sn * xq.re, c * xp.im - sn * xq.im};
          Hc(k, q) = cplx{sn * xp.re + c * xq.re, sn * xp.im + c * xq.im};
          const cplx wp = W(k, p), wq = c_mul(phc, W(k, q));
          W(k, p) = cplx{c * wp.re - sn * wq.re, c * wp.im - sn * wq.im};
          W(k, q) = cplx{sn * wp.re + c * wq.re, sn * wp.im + c * wq.im};
        }
        for (int k = 0; k < d; ++k) {   // rows: X <- G^H X
          const cplx xp = Hc(p, k), xq = c_mul(ph, Hc(q, k));
          Hc(p, k) = cplx{c * xp.re - sn * xq.re, c * xp.im - sn * xq.im};
          Hc(q, k) = cplx{sn * xp.re + c * xq.re, sn * xp.im + c * xq.im};
        }
      }
  }
  // ascending eigenvalues; output k = sum_i W(i, k) phi_i, staged in SC
  int order[kPairMax / 2];
  for (int k = 0; k < d; ++k) order[k] = k;
  for (int k = 0; k < d; ++k)
    for (int q = k + 1; q < d; ++q)
      if (Hc(order[q], order[q]).re < Hc(order[k], order[k]).re) {
        const int x = order[k];
        order[k] = order[q];
        order[q] = x;
      }
  for (int k = 0; k < d; ++k) {
    const int w = order[k];
    for (int l = 0; l < n; ++l) {
      cplx acc{0.0, 0.0};
      for (int i = 0; i < d; ++i) {
        const cplx x = c_mul(W(i, w), Cc(i, l));
        acc.re += x.re;
        acc.im += x.im;
      }
      SC(k, l) = acc;
    }
  }
  for (int k = 0; k < d; ++k) {
    for (int l = 0; l < n; ++l) Cc(k, l) = SC(k, l);
    ostart[o0 + k] = m;
    osize[o0 + k] = n;
    eps[o0 + k] = Hc(order[k], order[k]).re;
  }
}

// Psi [2][N][M]: the complex Ritz vectors sum_l coef[o][l] psi_{ostart[o] + l} from
// the real ones R [2N][2M] (real part of (a + ib)(re + i im) = a re - b im).
template <typename T>
__global__ void cluster_combine_kernel(const T* __restrict__ R, const cplx* __restrict__ coef,
                                       const int* __restrict__ ostart,
                                       const int* __restrict__ osize, int N, int64_t M,
                                       T* __restrict__ Psi) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int o = blockIdx.y;
  if (p >= M) return;
  const int s = ostart[o], n = osize[o], n2 = 2 * N;
  if (s < 0 || n < 1 || n > kPairMax || s + n > n2) return;
  double xr = 0.0, xi = 0.0;
  for (int l = 0; l < n; ++l) {
    const cplx c = coef[(size_t)o * kPairMax + l];
    if (c.re == 0.0 && c.im == 0.0) continue;
    const double re = R[(int64_t)(s + l) * 2 * M + p], im = R[(int64_t)(s + l) * 2 * M + M + p];
    xr += c.re * re - c.im * im;
    xi += c.re * im + c.im * re;
  }
  Psi[(int64_t)o * M + p] = (T)xr;
  Psi[((int64_t)N + o) * M + p] = (T)xi;
}

}  // namespace

size_t rr_bloch_workspace_bytes(int N, int64_t M, lrdm_prec prec) {
  const int n2 = 2 * N;
  const int Np = ((n2 + JS - 1) / JS) * JS;
  const int nb = Np / JB;
  const size_t s = prec == LRDM_FP64 ? sizeof(double) : sizeof(float);
  size_t b = 2 * ws_align((size_t)2 * n2 * M * s);                 // B, spare
  b += ws_align((size_t)2 * n2 * M * sizeof(double));              // H B
  b += 6 * ws_align((size_t)n2 * n2 * sizeof(double));            // G, T, C, X, Wt, Q
  b += ws_align((size_t)n2 * sizeof(double));                     // real Ritz values
  b += 2 * ws_align((size_t)n2 * sizeof(int));                    // clusters
  b += ws_align((size_t)n2 * kPairRow * sizeof(cplx));            // cluster scratch
  b += ws_align((size_t)N * kPairMax * sizeof(cplx));             // coefficients
  b += 2 * ws_align((size_t)N * sizeof(int)) + 2 * ws_align(64);
  size_t inner = chol_orth_bytes(n2);
  inner = std::max(inner, 2 * ws_align((size_t)Np * Np * sizeof(double)) +
                              ws_align((size_t)(nb / 2) * JS * JS * 8) + ws_align(256) +
                              ws_align((size_t)Np * 4) + ws_align(kFrobBlocks * sizeof(double)));
  inner = std::max(inner, ws_align(tn_workspace_bytes(n2, 2 * M, 1, prec)));
  return b + inner;
}

// Psi [2][N][M] (real parts, then imaginary parts; the filtered block on entry)
// -> Ritz vectors of H_k, eps ascending.  Storage T, FP64 arithmetic throughout
// (H B is formed and kept in FP64, as in the real path).
template <typename T>
lrdm_status rayleigh_ritz_bloch(lrdm_ctx* ctx, const Grid3& g, const double* V,
                                const double kvec[3], T* Psi, int N, double* eps) {
  const int64_t M = g.M;
  const int n2 = 2 * N;
  const size_t plane = (size_t)n2 * M;
  const size_t nn = (size_t)n2 * n2 * sizeof(double);
  T* B = static_cast<T*>(ws_take(ctx, 2 * plane * sizeof(T)));
  T* spare = static_cast<T*>(ws_take(ctx, 2 * plane * sizeof(T)));
  double* HB = static_cast<double*>(ws_take(ctx, 2 * plane * sizeof(double)));
  double* G = static_cast<double*>(ws_take(ctx, nn));
  double* Tm = static_cast<double*>(ws_take(ctx, nn));
  double* C = static_cast<double*>(ws_take(ctx, nn));
  double* X = static_cast<double*>(ws_take(ctx, nn));
  double* Wt = static_cast<double*>(ws_take(ctx, nn));
  double* Q = static_cast<double*>(ws_take(ctx, nn));
  double* e2 = static_cast<double*>(ws_take(ctx, (size_t)n2 * sizeof(double)));
  int* cs = static_cast<int*>(ws_take(ctx, (size_t)n2 * sizeof(int)));
  int* cn = static_cast<int*>(ws_take(ctx, (size_t)n2 * sizeof(int)));
  cplx* scr = static_cast<cplx*>(ws_take(ctx, (size_t)n2 * kPairRow * sizeof(cplx)));
  cplx* coef = static_cast<cplx*>(ws_take(ctx, (size_t)N * kPairMax * sizeof(cplx)));
  int* ostart = static_cast<int*>(ws_take(ctx, (size_t)N * sizeof(int)));
  int* osize = static_cast<int*>(ws_take(ctx, (size_t)N * sizeof(int)));
  int* flag = static_cast<int*>(ws_take(ctx, 64));
  double* dmin = static_cast<double*>(ws_take(ctx, 64));
  const size_t mark = ctx->ws_top;
  hipError_t e;
  auto fail = [&](const char* what, hipError_t err) {
    ctx->err = std::string("rayleigh_ritz_bloch: ") + what + ": " + hipGetErrorString(err);
    return LRDM_EDEVICE;
  };
  const dim3 blk(32, 8), grd((n2 + 31) / 32, (n2 + 7) / 8);
  const int64_t M2 = 2 * M;
  realify_kernel<T><<<dim3((unsigned)((M + 255) / 256), N), 256, 0, ctx->stream>>>(Psi, N, M, B);
  if ((e = hipGetLastError()) != hipSuccess) return fail("realify", e);
  // out = P Q^T over rows of length 2M (Q = P when Q2 is null); the partial sums
  // are free once the reduction is queued
  auto gram = [&](const T* P, const double* Q2, double* out) -> hipError_t {
    const hipError_t err =
        Q2 ? launch_tn_sym_f64<T, double>(ctx, P, Q2, nullptr, 0, n2, M2, 1, 1, out)
           : launch_tn_sym_f64<T, T>(ctx, P, nullptr, nullptr, 0, n2, M2, 1, 1, out);
    ctx->ws_top = mark;
    return err;
  };
  // Orthonormal basis as in the real path: one Cholesky pass for a well-conditioned
  // block, more over the explicitly formed basis otherwise.  Rows the factor finds
  // dependent become their explicit residuals relative to their own length; one
  // below 1e-8 (or a row still dependent on the third pass) means the complex
  // block is rank deficient as given, which is an error here: completing it
  // with pseudo-random rows, as the real path does, would break the pairing of
  // y and i y.
  T* Bc = B;
  CholInfo ci{n2, 0.0};
  bool check_residuals = false;
  for (int pass = 0;; ++pass) {
    if (pass > 0) {
      if (pass == kMaxOrthPasses) {
        ctx->err = "rayleigh_ritz_bloch: the block could not be orthonormalised";
        return LRDM_ENOTCONV;
      }
      transpose_kernel<<<grd, blk, 0, ctx->stream>>>(Tm, n2, Wt);
      if ((e = launch_nn_f64<T>(ctx, Wt, Bc, spare, n2, M2, ci.live == n2)) != hipSuccess)
        return fail("rotation", e);
      std::swap(Bc, spare);
    }
    if ((e = gram(Bc, nullptr, G)) != hipSuccess) return fail("gram", e);
    if (check_residuals) {
      min_diag_kernel<<<1, 256, 0, ctx->stream>>>(G, n2, dmin);
      double host_min = 0.0;
      if ((e = hipGetLastError()) != hipSuccess ||
          (e = hipMemcpyAsync(&host_min, dmin, sizeof(double), hipMemcpyDeviceToHost,
                              ctx->stream)) != hipSuccess ||
          (e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
        return fail("residual norms", e);
      if (host_min < 1e-16) {
        ctx->err = "rayleigh_ritz_bloch: the complex block is numerically rank deficient";
        return LRDM_ENOTCONV;
      }
      check_residuals = false;
    }
    lrdm_status st = chol_orth(ctx, G, n2, kDependentTol, Tm, &ci);
    ctx->ws_top = mark;
    if (st != LRDM_OK) return st;
    if (ci.live < n2) {
      if (pass >= 2) {
        ctx->err = "rayleigh_ritz_bloch: the complex block is numerically rank deficient";
        return LRDM_ENOTCONV;
      }
      check_residuals = true;
    } else if (ci.cond < kOnePassCond64) {
      break;
    }
  }
  // H_k on the 2N complex states, then the projected real operator
  if ((e = launch_bloch_hpsi_f64<T>(ctx, g, V, kvec, Bc, HB, n2, M2, M)) != hipSuccess)
    return fail("H_k", e);
  if ((e = gram(Bc, HB, G)) != hipSuccess) return fail("projection", e);
  if ((e = small_gemm(ctx, false, false, n2, n2, n2, 1.0, Tm, n2, G, n2, 0.0, X, n2)) !=
      hipSuccess)
    return fail("gemm", e);
  if ((e = small_gemm(ctx, false, true, n2, n2, n2, 1.0, X, n2, Tm, n2, 0.0, C, n2)) !=
      hipSuccess)
    return fail("gemm", e);
  lrdm_status st = sym_eigh(ctx, C, n2, n2, nullptr, e2, Q);
  if (st != LRDM_OK) return st;
  ctx->ws_top = mark;
  // the 2N real Ritz vectors Wt^T B, Wt = T^T Q
  if ((e = small_gemm(ctx, true, false, n2, n2, n2, 1.0, Tm, n2, Q, n2, 0.0, Wt, n2)) !=
      hipSuccess)
    return fail("gemm", e);
  T* R = (Bc == B) ? spare : B;
  if ((e = launch_nn_f64<T>(ctx, Wt, Bc, R, n2, M2)) != hipSuccess) return fail("rotation", e);
  // clusters of real Ritz values, the complex pairs of each, and their vectors
  const unsigned cgrid = (unsigned)((n2 + 255) / 256);
  zero_int_kernel<<<1, 1, 0, ctx->stream>>>(flag);
  cluster_kernel<<<cgrid, 256, 0, ctx->stream>>>(e2, n2, cs, cn);
  cluster_overlap_kernel<T><<<n2, 256, 0, ctx->stream>>>(R, cs, cn, n2, M, scr);
  cluster_pair_kernel<<<cgrid, 256, 0, ctx->stream>>>(e2, cs, cn, N, scr, coef, ostart, osize,
                                                      eps, flag);
  if ((e = hipGetLastError()) != hipSuccess) return fail("pairs", e);
  int host_flag = 0;
  if ((e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream)) !=
      hipSuccess)
    return fail("flag", e);
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return fail("flag", e);
  if (host_flag) {
    ctx->err = "rayleigh_ritz_bloch: the real Ritz values do not fall into clusters of complex "
               "pairs (at most 32 equal Ritz values of H_k are resolved)";
    return LRDM_ENOTCONV;
  }
  cluster_combine_kernel<T><<<dim3((unsigned)((M + 255) / 256), N), 256, 0, ctx->stream>>>(
      R, coef, ostart, osize, N, M, Psi);
  if ((e = hipGetLastError()) != hipSuccess) return fail("combine", e);
  return LRDM_OK;
}

template lrdm_status rayleigh_ritz_bloch<double>(lrdm_ctx*, const Grid3&, const double*,
                                                 const double[3], double*, int, double*);
template lrdm_status rayleigh_ritz_bloch<float>(lrdm_ctx*, const Grid3&, const double*,
                                                const double[3], float*, int, double*);

}  // namespace lrdm

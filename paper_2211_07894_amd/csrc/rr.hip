// Rayleigh-Ritz step of ChFSI (Sec. II C, Eq. (15)) and the FP64 symmetric
// eigensolver it needs, both on the GPU.
//
// Orthonormalisation: with the filtered block Y (rows = vectors) and
// G = Y Y^T = D^{-1} Gs D^{-1} (D^{-1} = diag of row norms), the symmetric
// (Loewdin) factor T = Gs^{-1/2} D, from a coupled Newton-Schulz iteration,
// gives orthonormal rows Psi_o = T Y.  The projected Hamiltonian is Hhat = T (Y (H Y)^T) T^T, its
// eigenpairs Hhat = Q E Q^T give eps = E and Psi_R = Q^T T Y: one pass over the
// grid for Gram, one stencil pass, one pass for Y (HY)^T and one rotation pass.
// Column scaling makes a warm-started block (Y ~ eigenvectors times filter
// gains) well conditioned, which is the regime of ChFSI inside an SCF loop.
//
// Eigensolver: two-sided block Jacobi.  The matrix (padded to a multiple of 64
// with decoupled diagonal entries 1e30) is cut into 32-wide blocks; each outer
// round pairs blocks by a round-robin tournament and a workgroup diagonalises
// each 64 x 64 pair problem in LDS with one or two sweeps of cyclic Jacobi
// (1024 threads, one 2 x 2 block of the pair rotation per thread; rotations
// t = sign(z)/(|z| + sqrt(1 + z^2)), z = (a_qq - a_pp)/(2 a_pq)); a second kernel
// applies the pair rotations to A and to the eigenvector matrix as 64 x 64 GEMMs.
// Rotations are applied above 1e-16 ||A||_F; sweeps stop when an outer sweep
// meets no off-diagonal entry above 1e-13 ||A||_F (one host read of a device
// flag per sweep), about ten times the rounding left by the 64-wide rotation
// updates, so the stop is reachable.
#include "lrdm_internal.h"
#include "jacobi_order.h"

#include <utility>
#include <vector>

namespace lrdm {
namespace {

constexpr int JB = 32;        // block width
constexpr int JS = 64;        // pair problem size
constexpr int JP = JS + 1;    // LDS pitch
constexpr double kPad = 1e30; // diagonal of padding rows (decoupled, sorts last)
constexpr int kNewtonSchulz = 28;  // at most this many Newton-Schulz steps
constexpr double kNewtonSchulzTol = 1e-10;  // stop one step after ||W - I||_F < tol


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
                                                        double* __restrict__ Ublk,
                                                        int* __restrict__ flag, int max_inner) {
  __shared__ double S[JS * JP];
  __shared__ double U[JS * JP];
  __shared__ double rc[JB], rs[JB], rt[JB];
  __shared__ int rp[JB], rq[JB];
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
  int first_rot = 0;
  __syncthreads();
  for (int sw = 0; sw < max_inner; ++sw) {
    if (threadIdx.x == 0) any_rot = 0;
    __syncthreads();
    for (int r = 0; r < JS - 1; ++r) {
      if (threadIdx.x < JB) {
        const int i = threadIdx.x;
        const int p = rr_pos(i, r, JS), q = rr_pos(JS - 1 - i, r, JS);
        const double apq = S[p * JP + q], app = S[p * JP + p], aqq = S[q * JP + q];
        double c = 1.0, s = 0.0, tt = 0.0;
        if (fabs(apq) > thr_apply) {
          const double z = (aqq - app) / (2.0 * apq);
          tt = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          if (fabs(apq) > thr_flag) any_rot = 1;
        }
        rp[i] = p;
        rq[i] = q;
        rc[i] = c;
        rs[i] = s;
        rt[i] = tt;
      }
      __syncthreads();
      // S <- J^T S J on the 32 x 32 pair blocks
      for (int blk = threadIdx.x; blk < JB * JB; blk += blockDim.x) {
        const int al = blk >> 5, be = blk & 31;
        const int p1 = rp[al], q1 = rq[al], p2 = rp[be], q2 = rq[be];
        const double ca = rc[al], sa = rs[al], cb = rc[be], sb = rs[be];
        if (al == be) {
          if (sa != 0.0) {
            const double apq = S[p1 * JP + q1], ta = rt[al];
            S[p1 * JP + p1] -= ta * apq;
            S[q1 * JP + q1] += ta * apq;
            S[p1 * JP + q1] = 0.0;
            S[q1 * JP + p1] = 0.0;
          }
        } else if (sa != 0.0 || sb != 0.0) {
          const double b00 = S[p1 * JP + p2], b01 = S[p1 * JP + q2];
          const double b10 = S[q1 * JP + p2], b11 = S[q1 * JP + q2];
          const double x00 = ca * b00 - sa * b10, x01 = ca * b01 - sa * b11;
          const double x10 = sa * b00 + ca * b10, x11 = sa * b01 + ca * b11;
          S[p1 * JP + p2] = x00 * cb - x01 * sb;
          S[p1 * JP + q2] = x00 * sb + x01 * cb;
          S[q1 * JP + p2] = x10 * cb - x11 * sb;
          S[q1 * JP + q2] = x10 * sb + x11 * cb;
        }
      }
      // U <- U J
      for (int e = threadIdx.x; e < JS * JB; e += blockDim.x) {
        const int row = e >> 5, al = e & 31;
        const double s = rs[al];
        if (s != 0.0) {
          const double c = rc[al];
          const int p = rp[al], q = rq[al];
          const double up = U[row * JP + p], uq = U[row * JP + q];
          U[row * JP + p] = c * up - s * uq;
          U[row * JP + q] = s * up + c * uq;
        }
      }
      __syncthreads();
    }
    const int rot = any_rot;
    if (sw == 0) first_rot = rot;
    __syncthreads();
    if (!rot) break;
  }
  double* Ub = Ublk + (int64_t)pair * JS * JS;
  for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
    const int a = e / JS, c = e - a * JS;
    Ub[e] = U[a * JP + c];
  }
  if (threadIdx.x == 0 && first_rot) atomicOr(flag, 1);
}

// 64x64x64 product C = op(X) Y with X, Y, C in LDS (pitch JP); thread (tr, tc)
// owns a 4x4 micro-tile.  transX: C = X^T Y.
__device__ inline void lds_gemm64(const double* X, const double* Y, double acc[4][4], bool transX) {
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k = 0; k < JS; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = transX ? X[k * JP + tr * 4 + i] : X[(tr * 4 + i) * JP + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = Y[k * JP + tc * 4 + j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
  }
}

// blocks [0, P*P): A(pair P rows, pair R cols) <- U_P^T A U_R
// blocks [P*P, P*P + (Np/64)*P): V(row block, pair P cols) <- V U_P
__global__ __launch_bounds__(256) void jac_update_kernel(double* __restrict__ A,
                                                         double* __restrict__ V, int Np, int nb,
                                                         int t, const double* __restrict__ Ublk) {
  __shared__ double X[JS * JP];
  __shared__ double UL[JS * JP];
  __shared__ double UR[JS * JP];
  const int np = nb / 2;
  int id = blockIdx.x;
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  double acc[4][4];
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
      UR[a * JP + c] = URg[e];
    }
    __syncthreads();
    lds_gemm64(UL, X, acc, true);   // U_P^T A
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) X[(tr * 4 + i) * JP + tc * 4 + j] = acc[i][j];
    __syncthreads();
    lds_gemm64(X, UR, acc, false);  // (U_P^T A) U_R
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int a = tr * 4 + i;
      const int ga = a < JB ? p1 * JB + a : q1 * JB + (a - JB);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = tc * 4 + j;
        const int gc = c < JB ? p2 * JB + c : q2 * JB + (c - JB);
        A[(int64_t)ga * Np + gc] = acc[i][j];
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
    for (int i = 0; i < 4; ++i) {
      const int a = tr * 4 + i;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = tc * 4 + j;
        const int gc = c < JB ? p1 * JB + c : q1 * JB + (c - JB);
        V[(int64_t)(rb * JS + a) * Np + gc] = acc[i][j];
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
__global__ void jac_rank_kernel(const double* __restrict__ A, int Np, int* __restrict__ perm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Np) return;
  perm[order_rank(A, Np + 1, Np, k)] = k;
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
__global__ void diag_rsqrt_kernel(const double* __restrict__ G, int N, double* __restrict__ dinv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dinv[i] = 1.0 / sqrt(G[(int64_t)i * N + i]);
}


// Gs = D G D (symmetrised), D = diag(dinv): the column-scaled Gram matrix.
__global__ void gram_scale_kernel(const double* __restrict__ G, const double* __restrict__ dinv,
                                  int N, double* __restrict__ Gs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= N || j >= N) return;
  Gs[(int64_t)i * N + j] = 0.5 * (G[(int64_t)i * N + j] + G[(int64_t)j * N + i]) * dinv[i] * dinv[j];
}

// Y0 = Gs / ||Gs||_F (spectrum in (0, 1]), Z0 = I.
__global__ void ns_start_kernel(const double* __restrict__ Gs, const double* __restrict__ fro,
                                int N, double* __restrict__ Y, double* __restrict__ Z) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= N || j >= N) return;
  Y[(int64_t)i * N + j] = Gs[(int64_t)i * N + j] / *fro;
  Z[(int64_t)i * N + j] = (i == j) ? 1.0 : 0.0;
}

// T = (3 I - W) / 2
// T = (3I - W)/2 and, per block, the partial sum of (W - I)^2 (blockDim 32 x 8);
// nothing once the iteration has stopped.
__global__ __launch_bounds__(256) void ns_step_kernel(const double* __restrict__ W, int N,
                                                      double* __restrict__ T,
                                                      const int* __restrict__ stop,
                                                      double* __restrict__ part) {
  __shared__ double red[4];
  if (*stop) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  double d2 = 0.0;
  if (i < N && j < N) {
    const double w = W[(int64_t)i * N + j];
    const double d = w - (i == j ? 1.0 : 0.0);
    d2 = d * d;
    T[(int64_t)i * N + j] = (i == j ? 1.5 : 0.0) - 0.5 * w;
  }
  const int t = threadIdx.y * blockDim.x + threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) d2 += __shfl_down(d2, off, 64);
  if ((t & 63) == 0) red[t >> 6] = d2;
  __syncthreads();
  if (t == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// pending = 1 once ||W - I||_F < tol (fixed-order sum of the partials); the step
// that detected it still updates Y and Z, and the following ones copy.
__global__ __launch_bounds__(256) void ns_check_kernel(const double* __restrict__ part, int n,
                                                       double tol, const int* __restrict__ stop,
                                                       int* __restrict__ pending) {
  __shared__ double red[4];
  if (*stop) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0 && red[0] + red[1] + red[2] + red[3] < tol * tol) *pending = 1;
}

__global__ void ns_flags_kernel(int* __restrict__ stop, int* __restrict__ pending, int reset) {
  if (threadIdx.x == 0) {
    if (reset) {
      *stop = 0;
      *pending = 0;
    } else if (*pending) {
      *stop = 1;
    }
  }
}

// Tm[i][j] = Z[i][j] dinv[j] / sqrt(||Gs||_F): Gs^{-1/2} D, orthonormal rows Tm Y.
__global__ void ns_finish_kernel(const double* __restrict__ Z, const double* __restrict__ dinv,
                                 const double* __restrict__ fro, int N, double* __restrict__ T) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= N || j >= N) return;
  T[(int64_t)i * N + j] = Z[(int64_t)i * N + j] * dinv[j] / sqrt(*fro);
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
  const int max_sweeps = 40;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    ProfScope prof_sweep(ctx, "jac_sweep");
    if ((e = hipMemsetAsync(flag, 0, sizeof(int), ctx->stream)) != hipSuccess) return fail(e);
    for (int t = 0; t < nb - 1; ++t) {
      {
        ProfScope prof_solve(ctx, "jac_solve");
        jac_solve_kernel<<<nb / 2, 1024, 0, ctx->stream>>>(A, Np, nb, t, normF, Ublk, flag,
                                                            sweep == 0 ? 2 : 1);
      }
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      const int np = nb / 2;
      {
        ProfScope prof_update(ctx, "jac_update");
        jac_update_kernel<<<np * np + (Np / JS) * np, 256, 0, ctx->stream>>>(A, V, Np, nb, t, Ublk);
      }
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    }
    int host_flag = 0;
    if ((e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream)) !=
        hipSuccess)
      return fail(e);
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return fail(e);
    if (!host_flag) break;
  }
  if (sweep == max_sweeps) {
    if (ctx->checks) {
      ctx->err = "eigensolver: no convergence in 40 sweeps";
      return LRDM_ENOTCONV;
    }
  }
  jac_rank_kernel<<<(Np + 255) / 256, 256, 0, ctx->stream>>>(A, Np, perm);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  dim3 blk(32, 8), grd((N + 31) / 32, (N + 7) / 8);
  jac_gather_kernel<<<grd, blk, 0, ctx->stream>>>(A, V, Np, N, perm, evals, evecs);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  return LRDM_OK;
}

size_t ns_part_bytes(int N) {
  return (size_t)((N + 31) / 32) * ((N + 7) / 8) * sizeof(double);
}

size_t rr_workspace_bytes(int N, int64_t M, lrdm_prec prec) {
  const int Np = ((N + JS - 1) / JS) * JS;
  const int nb = Np / JB;
  size_t b = 0;
  b += ws_align((size_t)M * N * sizeof(double));            // H Y, later Psi_R
  b += 6 * ws_align((size_t)N * N * sizeof(double));         // G, Hy, T, C, X, Wt
  b += 2 * ws_align((size_t)N * sizeof(double));             // dinv, lam
  b += ws_align(kFrobBlocks * sizeof(double));               // norm partial sums
  b += ws_align(ns_part_bytes(N));                           // Newton-Schulz residuals
  // eigensolver
  b += 2 * ws_align((size_t)Np * Np * sizeof(double)) + ws_align((size_t)(nb / 2) * JS * JS * 8) +
       ws_align(256) + ws_align((size_t)Np * 4) + ws_align(kFrobBlocks * sizeof(double));
  b += ws_align(tn_workspace_bytes(N, M, 1, prec));
  b += ws_align((size_t)N * N * sizeof(double));             // U of G
  return b;
}

template <typename T>
lrdm_status rayleigh_ritz(lrdm_ctx* ctx, const Grid3& g, const double* V, T* Psi, int N,
                          lrdm_prec prec, double* eps) {
  const int64_t M = g.M;
  const size_t nn = (size_t)N * N * sizeof(double);
  // H Y in FP64 whatever the storage type (later reused for Psi_R in type T)
  double* HY = static_cast<double*>(ws_take(ctx, (size_t)M * N * sizeof(double)));
  double* G = static_cast<double*>(ws_take(ctx, nn));
  double* Hy = static_cast<double*>(ws_take(ctx, nn));
  double* Tm = static_cast<double*>(ws_take(ctx, nn));
  double* C = static_cast<double*>(ws_take(ctx, nn));
  double* X = static_cast<double*>(ws_take(ctx, nn));
  double* Wt = static_cast<double*>(ws_take(ctx, nn));
  double* Ug = static_cast<double*>(ws_take(ctx, nn));
  double* dinv = static_cast<double*>(ws_take(ctx, (size_t)N * sizeof(double)));
  double* lam = static_cast<double*>(ws_take(ctx, (size_t)N * sizeof(double)));
  double* fpart = static_cast<double*>(ws_take(ctx, kFrobBlocks * sizeof(double)));
  double* ns_part = static_cast<double*>(ws_take(ctx, ns_part_bytes(N)));
  int* ns_stop = ctx->dstatus + LRDM_DS_COUNT + 1;     // scratch words after the status
  int* ns_pending = ctx->dstatus + LRDM_DS_COUNT + 2;  // words (the zero page starts at 32)
  hipError_t e;
  auto fail = [&](const char* what, hipError_t err) {
    ctx->err = std::string("rayleigh_ritz: ") + what + ": " + hipGetErrorString(err);
    return LRDM_EDEVICE;
  };
  const size_t mark = ctx->ws_top;
  // Every contraction here runs in FP64 arithmetic, and H Y is formed and kept
  // in FP64, whatever the storage type of the block: a filtered block's columns
  // span many orders of magnitude (1e-11 .. 1 at the 64^3 / 1024-state
  // workload), so the scaled Gram matrix is far too ill-conditioned for FP32
  // products, and the Loewdin coefficients (up to the inverse column norms)
  // magnify any FP32 rounding of H Y or of the rotation.
  // G = Y Y^T
  if ((e = launch_tn_sym_f64<T, T>(ctx, Psi, nullptr, nullptr, 0, N, M, 1, 1, G)) != hipSuccess)
    return fail("gram", e);
  ctx->ws_top = mark;
  diag_rsqrt_kernel<<<(N + 255) / 256, 256, 0, ctx->stream>>>(G, N, dinv);
  if ((e = hipGetLastError()) != hipSuccess) return fail("scale", e);
  // Loewdin factor Gs^{-1/2} by the coupled Newton-Schulz iteration
  //   W = Z Y, T = (3I - W)/2, Y <- Y T, Z <- T Z   (Y -> Gs'^{1/2}, Z -> Gs'^{-1/2})
  // on Gs' = Gs / ||Gs||_F, whose spectrum lies in (0, 1].  At most
  // kNewtonSchulz steps (a cold block with cond(Gs) up to ~1e6 needs about 24); the
  // device stops the iteration one step after ||W - I||_F < kNewtonSchulzTol, and
  // the remaining launches only copy Y and Z, with no host read-back.
  double* Ya = X;
  double* Za = C;
  double* Yb = Hy;
  double* Zb = Wt;
  double* W = G;
  double* Tn = Ug;
  double* fro = lam;
  {
    dim3 blk(32, 8), grd((N + 31) / 32, (N + 7) / 8);
    gram_scale_kernel<<<grd, blk, 0, ctx->stream>>>(G, dinv, N, Tm);
    if ((e = frob(ctx, Tm, N, N, fpart, fro)) != hipSuccess) return fail("scale", e);
    ns_start_kernel<<<grd, blk, 0, ctx->stream>>>(Tm, fro, N, Ya, Za);
    ns_flags_kernel<<<1, 64, 0, ctx->stream>>>(ns_stop, ns_pending, 1);
    if ((e = hipGetLastError()) != hipSuccess) return fail("scale", e);
    const int nparts = (int)(grd.x * grd.y);
    for (int it = 0; it < kNewtonSchulz; ++it) {
      if ((e = small_gemm(ctx, false, false, N, N, N, 1.0, Za, N, Ya, N, 0.0, W, N, ns_stop)) !=
          hipSuccess)
        return fail("newton-schulz", e);
      ns_step_kernel<<<grd, blk, 0, ctx->stream>>>(W, N, Tn, ns_stop, ns_part);
      ns_check_kernel<<<1, 256, 0, ctx->stream>>>(ns_part, nparts, kNewtonSchulzTol, ns_stop,
                                                  ns_pending);
      if ((e = small_gemm(ctx, false, false, N, N, N, 1.0, Ya, N, Tn, N, 0.0, Yb, N, ns_stop,
                          Ya)) != hipSuccess ||
          (e = small_gemm(ctx, false, false, N, N, N, 1.0, Tn, N, Za, N, 0.0, Zb, N, ns_stop,
                          Za)) != hipSuccess)
        return fail("newton-schulz", e);
      ns_flags_kernel<<<1, 64, 0, ctx->stream>>>(ns_stop, ns_pending, 0);
      std::swap(Ya, Yb);
      std::swap(Za, Zb);
    }
    ns_finish_kernel<<<grd, blk, 0, ctx->stream>>>(Za, dinv, fro, N, Tm);
    if ((e = hipGetLastError()) != hipSuccess) return fail("scale", e);
  }
  // H Y and Y (H Y)^T
  if ((e = launch_hpsi_f64<T>(ctx, g, V, Psi, HY, N)) != hipSuccess) return fail("stencil", e);
  if ((e = launch_tn_sym_f64<T, double>(ctx, Psi, HY, nullptr, 0, N, M, 1, 1, Hy)) != hipSuccess)
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
  // Psi_R = Q^T T Y: the rotation kernel computes Wt^T Y with Wt = T^T Q
  if ((e = small_gemm(ctx, true, false, N, N, N, 1.0, Tm, N, Ug, N, 0.0, Wt, N)) != hipSuccess)
    return fail("gemm", e);
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

}  // namespace lrdm

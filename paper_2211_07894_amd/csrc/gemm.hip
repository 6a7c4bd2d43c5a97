// Matrix-core contractions of the hot path (FP64 form: v_mfma_f64_16x16x4f64).
//
//  tn_sym   H[b] = A^T diag(w_b) A over the grid index (K = M, long), for the
//           projected perturbation Hbreve' = Psi^T H' Psi of Eq. (21) and for Gram
//           matrices in Rayleigh-Ritz.  Only upper 128x128 tiles are computed;
//           split-K partials go to workspace and are summed in a fixed order.
//  backproj out[p] = scale sum_ij A_ip G_ij A_jp, the density of a symmetric
//           subspace matrix (Eqs. (16), (20)); Z = G A never leaves the chip:
//           each block owns 128 grid points and walks the upper block triangle.
//  nn       Out = Wt^T B (K = N, short), the rotations Psi_o = L^{-1} Y and
//           Psi_R = Q^T Psi_o of Rayleigh-Ritz.
//
// Blocks are "state-major" [N][M] arrays, so every operand streams contiguous
// grid points.  Lane layout of v_mfma_f64_16x16x4f64 (measured on gfx950):
//   A operand: lane l supplies A[l%16][l/16]   (row, k)
//   B operand: lane l supplies B[l/16][l%16]   (k, col)
//   D: lane l, register v holds D[4v + l/16][l%16].
#include "lrdm_internal.h"

namespace lrdm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BT = 128;   // output tile (rows and columns)
constexpr int KT = 32;    // k extent staged in LDS per step
constexpr int LDP = BT + 1;  // LDS row pitch in doubles

__device__ inline d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Stage rows [r0, r0+BT) x cols [k0, k0+KT) of a row-major [nrows][ld] array into
// S[k][row] (transposed), optionally scaling column k by w[k].  Each thread
// loads 16 consecutive k of one row.  Out-of-range elements are zero.
struct TileLoad {
  double v[16];
  __device__ inline void load(const double* __restrict__ X, int64_t ld, int nrows, int r0,
                              int64_t k0, int64_t kend, const double* __restrict__ w) {
    const int t = threadIdx.x;
    const int row = t >> 1;
    const int64_t kb = k0 + (t & 1) * 16;
    const int gr = r0 + row;
    const bool aligned = ((reinterpret_cast<uintptr_t>(X + (int64_t)gr * ld + kb) |
                           reinterpret_cast<uintptr_t>(w ? w + kb : nullptr)) & 15) == 0;
    if (gr < nrows && kb + 16 <= kend && aligned) {
      const double2* src = reinterpret_cast<const double2*>(X + (int64_t)gr * ld + kb);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        double2 x = src[q];
        v[2 * q] = x.x;
        v[2 * q + 1] = x.y;
      }
      if (w) {
        const double2* ws = reinterpret_cast<const double2*>(w + kb);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          double2 x = ws[q];
          v[2 * q] *= x.x;
          v[2 * q + 1] *= x.y;
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t k = kb + q;
        double x = 0.0;
        if (gr < nrows && k < kend) {
          x = X[(int64_t)gr * ld + k];
          if (w) x *= w[k];
        }
        v[q] = x;
      }
    }
  }
  __device__ inline void store(double* S) const {
    const int t = threadIdx.x;
    const int row = t >> 1;
    const int kb = (t & 1) * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) S[(kb + q) * LDP + row] = v[q];
  }
};

// ------------------------------------------------------------------ tn_sym
// grid: x = upper tile index, y = split, z = batch.  part layout:
// [batch][split][tile][BT][BT].
__global__ __launch_bounds__(256, 2) void tn_sym_f64_kernel(
    const double* __restrict__ A, const double* __restrict__ B, const double* __restrict__ w,
    int64_t w_stride, int N, int64_t M, int nspin, int ntb, int64_t kchunk,
    double* __restrict__ part) {
  __shared__ double As[KT * LDP];
  __shared__ double Bs[KT * LDP];
  const int tile = blockIdx.x, split = blockIdx.y, b = blockIdx.z;
  // upper-triangle tile index -> (ti, tj), ti <= tj
  int ti = 0, rem = tile;
  while (rem >= ntb - ti) { rem -= ntb - ti; ++ti; }
  const int tj = ti + rem;
  const int c = b % nspin;
  const double* Ac = A + (int64_t)c * N * M;
  const double* Bc = B + (int64_t)c * N * M;
  const double* wb = w ? w + (int64_t)b * w_stride : nullptr;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = min(M, kbeg + kchunk);

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  TileLoad la, lb;
  if (kbeg < kend) {
    la.load(Ac, M, N, ti * BT, kbeg, kend, nullptr);
    lb.load(Bc, M, N, tj * BT, kbeg, kend, wb);
  }
  for (int64_t k0 = kbeg; k0 < kend; k0 += KT) {
    __syncthreads();
    la.store(As);
    lb.store(Bs);
    __syncthreads();
    if (k0 + KT < kend) {
      la.load(Ac, M, N, ti * BT, k0 + KT, kend, nullptr);
      lb.load(Bc, M, N, tj * BT, k0 + KT, kend, wb);
    }
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int kr = (kk + (lane >> 4)) * LDP;
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kr + wr * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kr + wc * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(a[i], bb[j], acc[i][j]);
    }
  }
  const int ntiles = ntb * (ntb + 1) / 2;
  double* out = part + (((int64_t)b * gridDim.y + split) * ntiles + tile) * (BT * BT);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 64 + i * 16 + 4 * v + (lane >> 4);
        const int col = wc * 64 + j * 16 + (lane & 15);
        out[row * BT + col] = acc[i][j][v];
      }
}

// H[b][i][j] = sum over splits (fixed order) of the partial tile holding (i, j),
// i <= j read from the upper tile and mirrored.
__global__ void tn_reduce_kernel(const double* __restrict__ part, int N, int ntb, int nsplit,
                                 double* __restrict__ H) {
  const int b = blockIdx.z;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= N || j >= N) return;
  const int ii = min(i, j), jj = max(i, j);
  const int ti = ii / BT, tj = jj / BT;
  // tile index of (ti, tj) in the upper-triangle enumeration
  const int tile = ti * ntb - ti * (ti - 1) / 2 + (tj - ti);
  const int ntiles = ntb * (ntb + 1) / 2;
  const int r = ii - ti * BT, cc = jj - tj * BT;
  double s = 0.0;
  for (int sp = 0; sp < nsplit; ++sp)
    s += part[(((int64_t)b * nsplit + sp) * ntiles + tile) * (BT * BT) + r * BT + cc];
  H[((int64_t)b * N + i) * N + j] = s;
}

// ------------------------------------------------------------------ backproj
// Stage G rows [j0, j0+KT) x cols [i0, i0+BT) (G symmetric: G[j][i] = G[i][j]) or
// A rows [j0, j0+KT) x cols [p0, p0+BT) straight (no transpose) into S[k][col].
struct RowLoad {
  double v[16];
  // thread t: row (t >> 3) of KT, 16 consecutive columns starting (t & 7) * 16
  __device__ inline void load(const double* __restrict__ X, int64_t ld, int nrows, int64_t ncols,
                              int j0, int64_t c0, double factor) {
    const int t = threadIdx.x;
    const int row = t >> 3;
    const int64_t cb = c0 + (t & 7) * 16;
    const int gr = j0 + row;
    const bool aligned = (reinterpret_cast<uintptr_t>(X + (int64_t)gr * ld + cb) & 15) == 0;
    if (gr < nrows && cb + 16 <= ncols && aligned) {
      const double2* src = reinterpret_cast<const double2*>(X + (int64_t)gr * ld + cb);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        double2 x = src[q];
        v[2 * q] = x.x * factor;
        v[2 * q + 1] = x.y * factor;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t cc = cb + q;
        v[q] = (gr < nrows && cc < ncols) ? X[(int64_t)gr * ld + cc] * factor : 0.0;
      }
    }
  }
  __device__ inline void store(double* S) const {
    const int t = threadIdx.x;
    const int row = t >> 3;
    const int cb = (t & 7) * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) S[row * LDP + cb + q] = v[q];
  }
};

// grid: x = point block (BT points), y = batch b (direction * nspin + channel).
__global__ __launch_bounds__(256, 2) void backproj_f64_kernel(
    const double* __restrict__ A, const double* __restrict__ G, int N, int64_t M, int nspin,
    double scale, const double* __restrict__ sub, double* __restrict__ out) {
  __shared__ double Gs[KT * LDP];
  __shared__ double Ps[KT * LDP];
  __shared__ double red[4][64];
  const int b = blockIdx.y;
  const int c = b % nspin;
  const double* Ac = A + (int64_t)c * N * M;
  const double* Gb = G + (int64_t)b * N * N;
  const int64_t p0 = (int64_t)blockIdx.x * BT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  double dsum[4] = {0.0, 0.0, 0.0, 0.0};   // per lane: columns wc*64 + j*16 + lane%16
  const int nib = (N + BT - 1) / BT;
  for (int ib = 0; ib < nib; ++ib) {
    const int i0 = ib * BT;
    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    RowLoad lg, lp;
    // K runs over j in [i0, N): the diagonal block once, blocks right of it twice
    // (G symmetric), so only the upper block triangle is touched.
    lg.load(Gb, N, N, N, i0, i0, 1.0);
    lp.load(Ac, M, N, M, i0, p0, 1.0);
    for (int j0 = i0; j0 < N; j0 += KT) {
      __syncthreads();
      lg.store(Gs);
      lp.store(Ps);
      __syncthreads();
      const int jn = j0 + KT;
      if (jn < N) {
        lg.load(Gb, N, N, N, jn, i0, (jn >= i0 + BT) ? 2.0 : 1.0);
        lp.load(Ac, M, N, M, jn, p0, 1.0);
      }
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        const int kr = (kk + (lane >> 4)) * LDP;
        double a[4], bb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = Gs[kr + wr * 64 + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 4; ++j) bb[j] = Ps[kr + wc * 64 + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(a[i], bb[j], acc[i][j]);
      }
    }
    // row-dot with A[i][p] for the rows of this block
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wr * 64 + i * 16 + 4 * v + (lane >> 4);
        if (gi < N) {
          const double* arow = Ac + (int64_t)gi * M;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
            if (p < M) dsum[j] += acc[i][j][v] * arow[p];
          }
        }
      }
  }
  // reduce over the 4 lane groups of a wave, then over the two row-waves
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double v = dsum[j];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    dsum[j] = v;
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wid][j * 16 + lane] = dsum[j];
  }
  __syncthreads();
  if (threadIdx.x < BT) {
    const int col = threadIdx.x;             // 0..127
    const int wcc = col >> 6, cl = col & 63;
    const double v = red[wcc][cl] + red[2 + wcc][cl];
    const int64_t p = p0 + col;
    if (p < M) {
      double r = scale * v;
      if (sub) r -= sub[(int64_t)b * M + p];
      out[(int64_t)b * M + p] = r;
    }
  }
}

// ------------------------------------------------------------------ nn
// Out[i][p] = sum_j Wt[j][i] B[j][p]; grid x = point block, y = row block.
template <typename T>
__global__ __launch_bounds__(256, 2) void nn_f64_kernel(const double* __restrict__ Wt,
                                                        const T* __restrict__ B,
                                                        T* __restrict__ Out, int N, int64_t M) {
  __shared__ double Ws[KT * LDP];
  __shared__ double Bs[KT * LDP];
  const int64_t p0 = (int64_t)blockIdx.x * BT;
  const int i0 = blockIdx.y * BT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  RowLoad lw, lb;
  lw.load(Wt, N, N, N, 0, i0, 1.0);
  lb.load(B, M, N, M, 0, p0, 1.0);
  for (int j0 = 0; j0 < N; j0 += KT) {
    __syncthreads();
    lw.store(Ws);
    lb.store(Bs);
    __syncthreads();
    if (j0 + KT < N) {
      lw.load(Wt, N, N, N, j0 + KT, i0, 1.0);
      lb.load(B, M, N, M, j0 + KT, p0, 1.0);
    }
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int kr = (kk + (lane >> 4)) * LDP;
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Ws[kr + wr * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kr + wc * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(a[i], bb[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = i0 + wr * 64 + i * 16 + 4 * v + (lane >> 4);
      if (gi >= N) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
        if (p < M) Out[(int64_t)gi * M + p] = (T)acc[i][j][v];
      }
    }
}

int pick_splits(int tiles_x_batch, int64_t M) {
  // enough blocks to fill 256 CUs at two blocks per CU several times over,
  // with each split at least 4096 grid points long
  int s = 1;
  while (tiles_x_batch * s < 2048 && M / (2 * s) >= 4096) s *= 2;
  return s;
}

}  // namespace

size_t tn_workspace_bytes(int N, int64_t M, int batch, lrdm_prec) {
  const int ntb = (N + BT - 1) / BT;
  const int ntiles = ntb * (ntb + 1) / 2;
  const int ns = pick_splits(ntiles * batch, M);
  return (size_t)batch * ns * ntiles * BT * BT * sizeof(double);
}

template <>
hipError_t launch_tn_sym<double>(lrdm_ctx* ctx, const double* A, const double* B,
                                 const double* w, int64_t w_stride, int N, int64_t M, int nspin,
                                 int batch, lrdm_prec prec, double* H) {
  const int ntb = (N + BT - 1) / BT;
  const int ntiles = ntb * (ntb + 1) / 2;
  const int ns = pick_splits(ntiles * batch, M);
  int64_t kchunk = (M + ns - 1) / ns;
  kchunk = (kchunk + KT - 1) / KT * KT;
  double* part = static_cast<double*>(ws_take(ctx, tn_workspace_bytes(N, M, batch, prec)));
  dim3 grd(ntiles, ns, batch);
  ProfScope prof(ctx, w ? "proj" : "gram");
  tn_sym_f64_kernel<<<grd, 256, 0, ctx->stream>>>(A, B ? B : A, w, w_stride, N, M, nspin, ntb,
                                                   kchunk, part);
  LRDM_HIP(hipGetLastError());
  dim3 blk(32, 8);
  dim3 grd2((N + 31) / 32, (N + 7) / 8, batch);
  tn_reduce_kernel<<<grd2, blk, 0, ctx->stream>>>(part, N, ntb, ns, H);
  return hipGetLastError();
}

template <>
hipError_t launch_backproj<double>(lrdm_ctx* ctx, const double* A, const double* G, int N,
                                   int64_t M, int nspin, int batch, lrdm_prec, double scale,
                                   const double* sub, double* out) {
  dim3 grd((unsigned)((M + BT - 1) / BT), batch);
  ProfScope prof(ctx, "backproj");
  backproj_f64_kernel<<<grd, 256, 0, ctx->stream>>>(A, G, N, M, nspin, scale, sub, out);
  return hipGetLastError();
}

template <>
hipError_t launch_nn<double>(lrdm_ctx* ctx, const double* Wt, const double* B, double* Out, int N,
                             int64_t M) {
  dim3 grd((unsigned)((M + BT - 1) / BT), (N + BT - 1) / BT);
  ProfScope prof(ctx, "nn");
  nn_f64_kernel<double><<<grd, 256, 0, ctx->stream>>>(Wt, B, Out, N, M);
  return hipGetLastError();
}

}  // namespace lrdm

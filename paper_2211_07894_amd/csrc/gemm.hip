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
#include <algorithm>

#include "blocks.h"
#include "lrdm_internal.h"
#include "xcd.h"

namespace lrdm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BT = 128;   // output tile (rows and columns)
constexpr int KT = 32;    // k extent staged in LDS per step
constexpr int LDP = BT + 1;  // LDS row pitch in doubles

__device__ inline d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 16 consecutive elements of storage type S from a 16-byte aligned address.
__device__ inline void load16(const double* src, double (&v)[16]) {
  const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double2 x = s2[q];
    v[2 * q] = x.x;
    v[2 * q + 1] = x.y;
  }
}
__device__ inline void load16(const float* src, float (&v)[16]) {
  const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 x = s4[q];
    v[4 * q] = x.x;
    v[4 * q + 1] = x.y;
    v[4 * q + 2] = x.z;
    v[4 * q + 3] = x.w;
  }
}

// Stage rows [r0, r0+BT) x cols [k0, k0+KT) of a row-major [nrows][ld] array of
// storage type S (double or float; the arithmetic is FP64 either way) into
// S[k][row] (transposed).  Each thread loads 16 consecutive k of one row.
// Out-of-range elements are zero.  load() only issues the reads, so they stay in
// flight during the current K-tile's matrix-core work.
template <typename S>
struct TileLoad {
  S v[16];
  __device__ inline void load(const S* __restrict__ X, int64_t ld, int nrows, int r0,
                              int64_t k0, int64_t kend) {
    const int t = threadIdx.x;
    const int row = t >> 1;
    const int64_t kb = k0 + (t & 1) * 16;
    const int gr = r0 + row;
    const bool aligned = (reinterpret_cast<uintptr_t>(X + (int64_t)gr * ld + kb) & 15) == 0;
    if (gr < nrows && kb + 16 <= kend && aligned) {
      load16(X + (int64_t)gr * ld + kb, v);
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t k = kb + q;
        v[q] = (gr < nrows && k < kend) ? X[(int64_t)gr * ld + k] : (S)0;
      }
    }
  }
  __device__ inline void store(double* Sm) const {
    const int t = threadIdx.x;
    const int row = t >> 1;
    const int kb = (t & 1) * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) Sm[(kb + q) * LDP + row] = (double)v[q];
  }
};

// ------------------------------------------------------------------ tn_sym
// 1-D grid over (split, batch) groups of upper tiles (xcd_map).  part layout:
// [batch][split][tile][BT][BT].
template <typename SA, typename SB>
__global__ __launch_bounds__(256, 2) void tn_sym_f64_kernel(
    const SA* __restrict__ A, const SB* __restrict__ B, const double* __restrict__ w,
    int64_t w_stride, int N, int64_t M, int nspin, int ntb, int64_t kchunk, int nsplit, int batch,
    const unsigned char* __restrict__ active, double* __restrict__ part) {
  __shared__ double As[KT * LDP];
  __shared__ double Bs[KT * LDP];
  __shared__ double Ws[KT];   // w over the current K-tile (1 when w is absent)
  const int ntiles = ntb * (ntb + 1) / 2;
  int group, tile;
  xcd_map(blockIdx.x, nsplit * batch, ntiles, group, tile);
  const int split = group % nsplit, b = group / nsplit;
  // upper-triangle tile index -> (ti, tj), ti <= tj
  int ti = 0, rem = tile;
  while (rem >= ntb - ti) { rem -= ntb - ti; ++ti; }
  const int tj = ti + rem;
  const int c = b % nspin;
  const SA* Ac = A + (int64_t)c * N * M;
  const SB* Bc = B + (int64_t)c * N * M;
  const double* wb = w ? w + (int64_t)b * w_stride : nullptr;
  const int64_t kbeg = (int64_t)split * kchunk;
  // an inactive block (blocks.h) keeps a zero partial tile
  const int64_t kend = block_active(active, c, ntb, ti, tj) ? min(M, kbeg + kchunk) : kbeg;

  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // the weight of B's column k is applied as B is read from LDS (the FP64 product
  // w[k] * B[j][k], as if B had been scaled in memory)
  auto wload = [&](int64_t k0) {
    const int64_t k = k0 + threadIdx.x;
    return (threadIdx.x < KT && k < kend) ? (wb ? wb[k] : 1.0) : 0.0;
  };
  TileLoad<SA> la;
  TileLoad<SB> lb;
  double wn = 0.0;
  if (kbeg < kend) {
    la.load(Ac, M, N, ti * BT, kbeg, kend);
    lb.load(Bc, M, N, tj * BT, kbeg, kend);
    wn = wload(kbeg);
  }
  for (int64_t k0 = kbeg; k0 < kend; k0 += KT) {
    __syncthreads();
    la.store(As);
    lb.store(Bs);
    if (threadIdx.x < KT) Ws[threadIdx.x] = wn;
    __syncthreads();
    if (k0 + KT < kend) {
      la.load(Ac, M, N, ti * BT, k0 + KT, kend);
      lb.load(Bc, M, N, tj * BT, k0 + KT, kend);
      wn = wload(k0 + KT);
    }
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int kr = (kk + (lane >> 4)) * LDP;
      const double wk = Ws[kk + (lane >> 4)];
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kr + wr * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kr + wc * 64 + j * 16 + (lane & 15)] * wk;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(a[i], bb[j], acc[i][j]);
    }
  }
  double* out = part + (((int64_t)b * nsplit + split) * ntiles + tile) * (BT * BT);
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
template <typename S>
struct RowLoad {
  S v[16];
  double fac;
  // thread t: row (t >> 3) of KT, 16 consecutive columns starting (t & 7) * 16
  __device__ inline void load(const S* __restrict__ X, int64_t ld, int nrows, int64_t ncols,
                              int j0, int64_t c0, double factor) {
    const int t = threadIdx.x;
    const int row = t >> 3;
    const int64_t cb = c0 + (t & 7) * 16;
    const int gr = j0 + row;
    const bool aligned = (reinterpret_cast<uintptr_t>(X + (int64_t)gr * ld + cb) & 15) == 0;
    fac = factor;
    if (gr < nrows && cb + 16 <= ncols && aligned) {
      load16(X + (int64_t)gr * ld + cb, v);
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t cc = cb + q;
        v[q] = (gr < nrows && cc < ncols) ? X[(int64_t)gr * ld + cc] : (S)0;
      }
    }
  }
  // the factor is applied here, after the current K-tile's work, so that the
  // reads issued by load() stay in flight meanwhile
  __device__ inline void store(double* Sm) const {
    const int t = threadIdx.x;
    const int row = t >> 3;
    const int cb = (t & 7) * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) Sm[row * LDP + cb + q] = (double)v[q] * fac;
  }
};

// 1-D grid over (point block of BT points, batch b = direction * nspin + channel);
// the directions of one point block run together on one XCD (xcd_map).
__global__ __launch_bounds__(256, 2) void backproj_f64_kernel(
    const double* __restrict__ A, const double* __restrict__ G, int N, int64_t M, int nspin,
    int batch, double scale, const double* __restrict__ sub,
    const unsigned char* __restrict__ active, double* __restrict__ out) {
  __shared__ double Gs[KT * LDP];
  __shared__ double Ps[KT * LDP];
  __shared__ double red[4][64];
  int pblk, b;
  xcd_map(blockIdx.x, (int)((M + BT - 1) / BT), batch, pblk, b);
  const int c = b % nspin;
  const double* Ac = A + (int64_t)c * N * M;
  const double* Gb = G + (int64_t)b * N * N;
  const int64_t p0 = (int64_t)pblk * BT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  double dsum[4] = {0.0, 0.0, 0.0, 0.0};   // per lane: columns wc*64 + j*16 + lane%16
  const int nib = (N + BT - 1) / BT;
  for (int ib = 0; ib < nib; ++ib) {
    const int i0 = ib * BT;
    // K runs over j in [i0, N): the diagonal block once, blocks right of it twice
    // (G symmetric), so only the upper block triangle is touched; inactive blocks
    // (blocks.h) are skipped, and a row block with none active contributes nothing
    const uint64_t bits = active_row_bits(active, c, nib, ib);
    const int nk = active_ktiles(bits, N, KT);
    if (nk == 0) continue;
    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    RowLoad<double> lg, lp;
    {
      int J;
      const int j0 = active_ktile(bits, 0, KT, J);
      lg.load(Gb, N, N, N, j0, i0, J > ib ? 2.0 : 1.0);
      lp.load(Ac, M, N, M, j0, p0, 1.0);
    }
    for (int t = 0; t < nk; ++t) {
      __syncthreads();
      lg.store(Gs);
      lp.store(Ps);
      __syncthreads();
      if (t + 1 < nk) {
        int J;
        const int jn = active_ktile(bits, t + 1, KT, J);
        lg.load(Gb, N, N, N, jn, i0, J > ib ? 2.0 : 1.0);
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
// Out[i][p] = sum_j Wt[j][i] B[j][p]; 1-D grid over (point block, row block), the
// row blocks of one point block together on one XCD (they read the same slice of B).
template <typename T>
// upper: Wt is upper triangular (Wt[j][i] = 0 for j > i), so row block i0 needs
// only k < i0 + BT.
__global__ __launch_bounds__(256, 2) void nn_f64_kernel(const double* __restrict__ Wt,
                                                        const T* __restrict__ B,
                                                        T* __restrict__ Out, int N, int64_t M,
                                                        int upper) {
  __shared__ double Ws[KT * LDP];
  __shared__ double Bs[KT * LDP];
  int pblk, rblk;
  const int nrb = (N + BT - 1) / BT;
  xcd_map(blockIdx.x, (int)((M + BT - 1) / BT), nrb, pblk, rblk);
  if (upper) rblk = nrb - 1 - rblk;   // the longest row blocks first
  const int64_t p0 = (int64_t)pblk * BT;
  const int i0 = rblk * BT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  RowLoad<double> lw;
  RowLoad<T> lb;
  const int kmax = upper ? min(N, i0 + BT) : N;
  lw.load(Wt, N, N, N, 0, i0, 1.0);
  lb.load(B, M, N, M, 0, p0, 1.0);
  for (int j0 = 0; j0 < kmax; j0 += KT) {
    __syncthreads();
    lw.store(Ws);
    lb.store(Bs);
    __syncthreads();
    if (j0 + KT < kmax) {
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

// ------------------------------------------------------------------ adjoint rotation
// Out_c[i][p] = scale * sum_m w_m[p] sum_j X_m[i][j] Psi_c[j][p] over the nmat
// symmetric matrices X_m of channel c (m = 0 .. nmat-1 at X + ((m * nspin) + c) N^2,
// weights at w + ((m * nspin) + c) M; two lists, the second starting at m = nx).
// FP64 arithmetic for either storage type.  grid x = point block, y = row block,
// z = channel.  The column weights travel with each staged K-tile.
template <typename T>
__global__ __launch_bounds__(256, 2) void adj_psi_f64_kernel(
    const double* __restrict__ X1, const double* __restrict__ w1, const double* __restrict__ X2,
    const double* __restrict__ w2, int nx, const T* __restrict__ Psi, int N, int64_t M, int nspin,
    double scale, T* __restrict__ Out) {
  __shared__ double Xs[KT * LDP];
  __shared__ double Bs[KT * LDP];
  __shared__ double Wc[BT];
  const int64_t p0 = (int64_t)blockIdx.x * BT;
  const int i0 = blockIdx.y * BT;
  const int c = blockIdx.z;
  const T* Pc = Psi + (int64_t)c * N * M;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int nkt = (N + KT - 1) / KT;
  const int nstep = 2 * nx * nkt;              // (matrix, K-tile) steps
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  RowLoad<double> lx;
  RowLoad<T> lb;
  double wn = 0.0;
  auto load = [&](int step) {
    const int m = step / nkt, j0 = (step % nkt) * KT;
    const int64_t b = (int64_t)(m % nx) * nspin + c;
    const double* X = (m < nx ? X1 : X2) + b * N * N;
    const double* w = (m < nx ? w1 : w2) + b * M;
    lx.load(X, N, N, N, j0, i0, 1.0);
    lb.load(Pc, M, N, M, j0, p0, 1.0);
    if (threadIdx.x < BT) {
      const int64_t p = p0 + threadIdx.x;
      wn = p < M ? w[p] : 0.0;
    }
  };
  if (nstep > 0) load(0);
  for (int step = 0; step < nstep; ++step) {
    __syncthreads();
    lx.store(Xs);
    lb.store(Bs);
    if (threadIdx.x < BT) Wc[threadIdx.x] = wn;
    __syncthreads();
    if (step + 1 < nstep) load(step + 1);
    double wcol[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) wcol[j] = Wc[wc * 64 + j * 16 + (lane & 15)];
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int kr = (kk + (lane >> 4)) * LDP;
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Xs[kr + wr * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kr + wc * 64 + j * 16 + (lane & 15)] * wcol[j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(a[i], bb[j], acc[i][j]);
    }
  }
  T* Oc = Out + (int64_t)c * N * M;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = i0 + wr * 64 + i * 16 + 4 * v + (lane >> 4);
      if (gi >= N) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
        if (p < M) Oc[(int64_t)gi * M + p] = (T)(scale * acc[i][j][v]);
      }
    }
}

}  // namespace

size_t tn_part_bytes(int N, int64_t M, int batch, int split_limit) {
  const int ntb = (N + BT - 1) / BT;
  const int ntiles = ntb * (ntb + 1) / 2;
  int ns = tn_split_cap(ntiles * batch, M);
  if (split_limit > 0) ns = std::min(ns, split_limit);
  return (size_t)batch * ns * ntiles * BT * BT * sizeof(double);
}

int tn_split_count(const lrdm_ctx* ctx, int N, int64_t M, int batch, int arith, bool weighted) {
  const int ntb = (N + BT - 1) / BT;
  const int ntiles = ntb * (ntb + 1) / 2;
  const auto it = ctx->tn_tuned.find({N, M, batch, arith, weighted ? 1 : 0});
  int s = tn_splits(ntiles * batch, M);
  if (it != ctx->tn_tuned.end() && it->second >= 1 && it->second <= tn_split_cap(ntiles * batch, M))
    s = it->second;
  if (ctx->split_limit > 0) s = std::min(s, ctx->split_limit);
  return s;
}

int tn_variant(const lrdm_ctx* ctx, int N, int64_t M, int batch, int arith, bool weighted) {
  const auto it = ctx->tn_variant.find({N, M, batch, arith, weighted ? 1 : 0});
  return it == ctx->tn_variant.end() ? TN_VAR_DEFAULT : it->second;
}

size_t tn_workspace_bytes(int N, int64_t M, int batch, lrdm_prec prec, int split_limit) {
  return ws_align(tn_part_bytes(N, M, batch, split_limit)) + tn_split_bytes(N, M, prec);
}

template <typename SA, typename SB>
hipError_t launch_tn_sym_f64(lrdm_ctx* ctx, const SA* A, const SB* B, const double* w,
                             int64_t w_stride, int N, int64_t M, int nspin, int batch,
                             double* H, const unsigned char* active) {
  const int ntb = (N + BT - 1) / BT;
  const int ntiles = ntb * (ntb + 1) / 2;
  const int ns = tn_split_count(ctx, N, M, batch, TN_ARITH_F64, w != nullptr);
  int64_t kchunk = (M + ns - 1) / ns;
  kchunk = (kchunk + KT - 1) / KT * KT;
  double* part = static_cast<double*>(ws_take(ctx, tn_part_bytes(N, M, batch, ctx->split_limit)));
  const unsigned grd = (unsigned)(ntiles * ns * batch);
  {
    ProfScope prof(ctx, w ? "proj" : "gram");
    if (B)
      tn_sym_f64_kernel<SA, SB><<<grd, 256, 0, ctx->stream>>>(A, B, w, w_stride, N, M, nspin, ntb,
                                                               kchunk, ns, batch, active, part);
    else
      tn_sym_f64_kernel<SA, SA><<<grd, 256, 0, ctx->stream>>>(A, A, w, w_stride, N, M, nspin, ntb,
                                                               kchunk, ns, batch, active, part);
    LRDM_HIP(hipGetLastError());
  }
  dim3 blk(32, 8);
  dim3 grd2((N + 31) / 32, (N + 7) / 8, batch);
  tn_reduce_kernel<<<grd2, blk, 0, ctx->stream>>>(part, N, ntb, ns, H);
  return hipGetLastError();
}
template hipError_t launch_tn_sym_f64<double, double>(lrdm_ctx*, const double*, const double*,
                                                      const double*, int64_t, int, int64_t, int,
                                                      int, double*, const unsigned char*);
template hipError_t launch_tn_sym_f64<float, float>(lrdm_ctx*, const float*, const float*,
                                                    const double*, int64_t, int, int64_t, int, int,
                                                    double*, const unsigned char*);
template hipError_t launch_tn_sym_f64<float, double>(lrdm_ctx*, const float*, const double*,
                                                     const double*, int64_t, int, int64_t, int,
                                                     int, double*, const unsigned char*);

template <>
hipError_t launch_tn_sym<double>(lrdm_ctx* ctx, const double* A, const double* B,
                                 const double* w, int64_t w_stride, int N, int64_t M, int nspin,
                                 int batch, lrdm_prec, double* H, const unsigned char* active) {
  return launch_tn_sym_f64<double, double>(ctx, A, B, w, w_stride, N, M, nspin, batch, H, active);
}

template <>
hipError_t launch_backproj<double>(lrdm_ctx* ctx, const double* A, const double* G, int N,
                                   int64_t M, int nspin, int batch, lrdm_prec, double scale,
                                   const double* sub, double* out, const unsigned char* active) {
  const unsigned grd = (unsigned)((M + BT - 1) / BT * batch);
  ProfScope prof(ctx, "backproj");
  backproj_f64_kernel<<<grd, 256, 0, ctx->stream>>>(A, G, N, M, nspin, batch, scale, sub, active,
                                                    out);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_nn_f64(lrdm_ctx* ctx, const double* Wt, const S* B, S* Out, int N, int64_t M,
                         bool upper) {
  const unsigned grd = (unsigned)((M + BT - 1) / BT) * (unsigned)((N + BT - 1) / BT);
  ProfScope prof(ctx, "nn");
  nn_f64_kernel<S><<<grd, 256, 0, ctx->stream>>>(Wt, B, Out, N, M, upper ? 1 : 0);
  return hipGetLastError();
}
template hipError_t launch_nn_f64<double>(lrdm_ctx*, const double*, const double*, double*, int,
                                          int64_t, bool);
template hipError_t launch_nn_f64<float>(lrdm_ctx*, const double*, const float*, float*, int,
                                         int64_t, bool);

template <>
hipError_t launch_adj_psi<double>(lrdm_ctx* ctx, const double* X1, const double* w1,
                                  const double* X2, const double* w2, int nx, const double* Psi,
                                  int N, int64_t M, int nspin, double scale, double* Out,
                                  const unsigned char*) {
  dim3 grd((unsigned)((M + BT - 1) / BT), (N + BT - 1) / BT, nspin);
  ProfScope prof(ctx, "adj_psi");
  adj_psi_f64_kernel<double><<<grd, 256, 0, ctx->stream>>>(X1, w1, X2, w2, nx, Psi, N, M, nspin,
                                                           scale, Out);
  return hipGetLastError();
}

}  // namespace lrdm

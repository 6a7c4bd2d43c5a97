// Hartree kernel K_c of Eq. (3) on the periodic grid:
//     dV = 4 pi (-Lap_h)^{-1} u,  q = 0 component removed,
// with the same 7-point Laplacian as the Hamiltonian.  -Lap_h is a sum of
// per-axis circulant second differences, diagonalised by a real orthonormal
// basis of each axis: column 0 = 1/sqrt(n); columns 2m-1, 2m = sqrt(2/n) cos, sin
// of 2 pi m j / n (m < n/2); for even n the last column (-1)^j / sqrt(n).  The
// eigenvalue of a column with frequency m is (2 - 2 cos(2 pi m / n)) / h^2.
// The transform is three passes of a dense n x n matrix along x, y and z.
#include "lrdm_internal.h"

namespace lrdm {
namespace {

__device__ inline int freq_of(int col, int n) {
  // column index -> frequency m
  if (col == 0) return 0;
  if ((n % 2 == 0) && col == n - 1) return n / 2;
  return (col + 1) / 2;
}

// U_d[j][col] and lam_d[col] for the three axes, packed: axis d at offset base_d.
__global__ void basis_kernel(int n, double h, double* __restrict__ U, double* __restrict__ lam) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (col >= n) return;
  const int m = freq_of(col, n);
  double v;
  if (col == 0) {
    v = 1.0 / sqrt((double)n);
  } else if ((n % 2 == 0) && col == n - 1) {
    v = ((j & 1) ? -1.0 : 1.0) / sqrt((double)n);
  } else {
    // angle 2 pi m j / n reduced exactly modulo n before the trigonometric call
    const double frac = 2.0 * (double)((int64_t)m * j % n) / (double)n;
    double s, c;
    sincospi(frac, &s, &c);
    v = sqrt(2.0 / n) * ((col & 1) ? c : s);
  }
  U[(int64_t)j * n + col] = v;
  if (j == 0) {
    double s, c;
    sincospi(2.0 * (double)m / (double)n, &s, &c);
    lam[col] = (2.0 - 2.0 * c) / (h * h);
  }
}

// out[.., k, ..] = sum_j B(j, k) in[.., j, ..] along one axis, B = U (forward
// uses U^T: coefficient k = sum_j U[j][k] x_j; inverse: x_j = sum_k U[j][k] c_k).
__global__ void axis_kernel(const double* __restrict__ in, double* __restrict__ out, int nx,
                            int ny, int nz, int axis, const double* __restrict__ U, int inverse,
                            int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t M = (int64_t)nx * ny * nz;
  const int64_t b = e / M;
  const int64_t p = e - b * M;
  const int x = (int)(p % nx);
  const int y = (int)((p / nx) % ny);
  const int z = (int)(p / ((int64_t)nx * ny));
  int n, k;
  int64_t stride, base;
  if (axis == 0) { n = nx; k = x; stride = 1; base = p - x; }
  else if (axis == 1) { n = ny; k = y; stride = nx; base = p - (int64_t)y * nx; }
  else { n = nz; k = z; stride = (int64_t)nx * ny; base = p - (int64_t)z * nx * ny; }
  const double* src = in + b * M + base;
  double s = 0.0;
  if (!inverse) {
    for (int j = 0; j < n; ++j) s += U[(int64_t)j * n + k] * src[j * stride];
  } else {
    for (int j = 0; j < n; ++j) s += U[(int64_t)k * n + j] * src[j * stride];
  }
  out[e] = s;
}

// The same transform for axes of at most kLdsAxis points, staged through LDS: the
// axis basis U (n x n) and a tile of the data, so that every value is read from
// HBM once per pass.
//  * axis 0 (x, contiguous lines): a block takes 64 lines of n points;
//  * axes 1 and 2: a block takes, for one index of the slower dimensions, the n
//    planes of a run of up to 64 consecutive points of the faster ones
//    (in[j][i] with j along the axis, i contiguous).
// out[.., k, ..] = sum_j coef(j, k) in[.., j, ..], coef = U[j][k] (forward) or
// U[k][j] (inverse).
constexpr int kLdsAxis = 64;

__global__ __launch_bounds__(256) void axis_lds_kernel(const double* __restrict__ in,
                                                       double* __restrict__ out, int n,
                                                       int64_t inner, int64_t lines,
                                                       const double* __restrict__ U,
                                                       int inverse) {
  __shared__ double Us[kLdsAxis * kLdsAxis];
  __shared__ double T[kLdsAxis * (kLdsAxis + 1)];
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int j = e / n, k = e - j * n;
    Us[j * kLdsAxis + k] = inverse ? U[(int64_t)k * n + j] : U[(int64_t)j * n + k];
  }
  if (inner == 1) {
    // 64 contiguous lines of n points: T[line][j]
    const int64_t l0 = (int64_t)blockIdx.x * 64;
    const int nl = (int)min((int64_t)64, lines - l0);
    const double* src = in + l0 * n;
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
      const int l = e / n, j = e - l * n;
      T[l * (kLdsAxis + 1) + j] = src[e];
    }
    __syncthreads();
    double* dst = out + l0 * n;
    for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
      const int l = e / n, k = e - l * n;
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += Us[j * kLdsAxis + k] * T[l * (kLdsAxis + 1) + j];
      dst[e] = acc;
    }
    return;
  }
  // a block: one outer index o and a run of up to 64 points i0 .. i0 + w
  const int64_t chunks = (inner + 63) / 64;
  const int64_t o = (int64_t)blockIdx.x / chunks;
  const int64_t i0 = ((int64_t)blockIdx.x - o * chunks) * 64;
  const int w = (int)min((int64_t)64, inner - i0);
  const double* src = in + o * n * inner + i0;
  for (int e = threadIdx.x; e < n * 64; e += blockDim.x) {
    const int j = e >> 6, i = e & 63;
    if (i < w) T[j * (kLdsAxis + 1) + i] = src[(int64_t)j * inner + i];
  }
  __syncthreads();
  double* dst = out + o * n * inner + i0;
  for (int e = threadIdx.x; e < n * 64; e += blockDim.x) {
    const int k = e >> 6, i = e & 63;
    if (i >= w) continue;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += Us[j * kLdsAxis + k] * T[j * (kLdsAxis + 1) + i];
    dst[(int64_t)k * inner + i] = acc;
  }
}

__global__ void sum_channels_kernel(const double* __restrict__ u, int nspin, int64_t M, int r,
                                    double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * M) return;
  const int64_t k = e / M, p = e - k * M;
  double s = 0.0;
  for (int c = 0; c < nspin; ++c) s += u[(k * nspin + c) * M + p];
  out[e] = s;
}

__global__ void symbol_kernel(double* __restrict__ c, int nx, int ny, int nz,
                              const double* __restrict__ lx, const double* __restrict__ ly,
                              const double* __restrict__ lz, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t M = (int64_t)nx * ny * nz;
  const int64_t p = e % M;
  const int x = (int)(p % nx);
  const int y = (int)((p / nx) % ny);
  const int z = (int)(p / ((int64_t)nx * ny));
  const double lam = lx[x] + ly[y] + lz[z];
  const double four_pi = 12.566370614359172953850573533118;
  c[e] = (x == 0 && y == 0 && z == 0) ? 0.0 : c[e] * (four_pi / lam);
}

__global__ void scatter_channels_kernel(const double* __restrict__ src, int64_t M, int r,
                                        int nspin, double* __restrict__ dV) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * nspin * M) return;
  const int64_t p = e % M;
  const int64_t k = e / (M * nspin);
  dV[e] = src[k * M + p];
}

}  // namespace

size_t hartree_workspace_bytes(const Grid3& g) {
  return ws_align((size_t)(g.nx * g.nx + g.ny * g.ny + g.nz * g.nz + g.nx + g.ny + g.nz) * 8);
}

// scratch: 2 * r * M doubles
hipError_t launch_hartree(lrdm_ctx* ctx, const Grid3& g, const double* u, int u_nspin, double* dV,
                          int dv_nspin, int r, double* scratch) {
  ProfScope prof(ctx, "hartree");
  double* tabs = static_cast<double*>(ws_take(ctx, hartree_workspace_bytes(g)));
  double* Ux = tabs;
  double* Uy = Ux + (int64_t)g.nx * g.nx;
  double* Uz = Uy + (int64_t)g.ny * g.ny;
  double* lx = Uz + (int64_t)g.nz * g.nz;
  double* ly = lx + g.nx;
  double* lz = ly + g.ny;
  basis_kernel<<<dim3((g.nx + 63) / 64, g.nx), 64, 0, ctx->stream>>>(g.nx, g.hx, Ux, lx);
  basis_kernel<<<dim3((g.ny + 63) / 64, g.ny), 64, 0, ctx->stream>>>(g.ny, g.hy, Uy, ly);
  basis_kernel<<<dim3((g.nz + 63) / 64, g.nz), 64, 0, ctx->stream>>>(g.nz, g.hz, Uz, lz);
  LRDM_HIP(hipGetLastError());
  const int64_t total = (int64_t)r * g.M;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  double* a = scratch;
  double* b = scratch + total;
  // one pass along `axis`: LDS-staged for axes of at most kLdsAxis points
  auto pass = [&](const double* in, double* out, int axis, const double* Ud, int inverse) {
    const int n = axis == 0 ? g.nx : (axis == 1 ? g.ny : g.nz);
    if (n > kLdsAxis) {
      axis_kernel<<<blocks, 256, 0, ctx->stream>>>(in, out, g.nx, g.ny, g.nz, axis, Ud, inverse,
                                                   total);
      return;
    }
    const int64_t inner = axis == 0 ? 1 : (axis == 1 ? g.nx : (int64_t)g.nx * g.ny);
    const int64_t lines = total / n;                 // lines of n points along the axis
    const int64_t nblk = axis == 0 ? (lines + 63) / 64 : (lines / inner) * ((inner + 63) / 64);
    axis_lds_kernel<<<(unsigned)nblk, 256, 0, ctx->stream>>>(in, out, n, inner, lines, Ud,
                                                             inverse);
  };
  sum_channels_kernel<<<blocks, 256, 0, ctx->stream>>>(u, u_nspin, g.M, r, a);
  pass(a, b, 0, Ux, 0);
  pass(b, a, 1, Uy, 0);
  pass(a, b, 2, Uz, 0);
  symbol_kernel<<<blocks, 256, 0, ctx->stream>>>(b, g.nx, g.ny, g.nz, lx, ly, lz, total);
  pass(b, a, 2, Uz, 1);
  pass(a, b, 1, Uy, 1);
  if (dv_nspin == 1) {
    pass(b, dV, 0, Ux, 1);
  } else {
    pass(b, a, 0, Ux, 1);
    const int64_t tot2 = total * dv_nspin;
    scatter_channels_kernel<<<(unsigned)((tot2 + 255) / 256), 256, 0, ctx->stream>>>(a, g.M, r,
                                                                                    dv_nspin, dV);
  }
  return hipGetLastError();
}

}  // namespace lrdm

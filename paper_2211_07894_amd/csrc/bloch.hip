// Bloch Hamiltonian of one k-point on the periodic grid, and its Chebyshev step
// (the ChFSI of each k-point's subspace, Sec. II C, last paragraph).
//
// For the cell-periodic part u of e^{i k.x} u(x) the 7-point stencil carries the
// phase e^{i k_d h_d} on the link to the neighbour at +h_d and its conjugate on
// the link to -h_d:
//   (H_k u)_p = -1/2 sum_d (e^{i k_d h_d} u_{p+e_d} + e^{-i k_d h_d} u_{p-e_d} - 2 u_p)/h_d^2
//               + V_p u_p.
// A block of N complex states is stored as two real planes [2][N][M]: the N real
// parts, then the N imaginary parts.  With u = a + ib, c_d = cos(k_d h_d) and
// s_d = sin(k_d h_d):
//   Re H_k u = -1/2 sum_d (c_d (a+ + a-) - s_d (b+ - b-) - 2a)/h_d^2 + V a,
//   Im H_k u = -1/2 sum_d (c_d (b+ + b-) + s_d (a+ - a-) - 2b)/h_d^2 + V b.
// One thread forms both planes of one point of one state; the neighbours come
// through the caches (x fastest, so a wavefront reads contiguous rows).
#include "lrdm_internal.h"

namespace lrdm {
namespace {

constexpr int kBlochThreads = 256;

struct BlochCoef {
  double c[3], s[3], ih2[3];   // cos(k_d h_d), sin(k_d h_d), 1/h_d^2 for x, y, z
};

// out = alpha (H_k in - c0 in) + beta old (old may be out itself: each thread
// reads old at its point before writing it; beta = 0 ignores old).
template <typename T>
__global__ __launch_bounds__(kBlochThreads) void bloch_step_kernel(
    const T* __restrict__ in, const T* old, T* out, const double* __restrict__ V, int nx, int ny,
    int nz, int N, BlochCoef k, double alpha, double c0, double beta) {
  const int64_t M = (int64_t)nx * ny * nz;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (p >= M) return;
  const int x = (int)(p % nx);
  const int y = (int)((p / nx) % ny);
  const int z = (int)(p / ((int64_t)nx * ny));
  const T* a = in + (int64_t)i * M;            // real plane of state i
  const T* b = in + ((int64_t)N + i) * M;      // imaginary plane
  const int64_t xp = p - x + (x + 1 == nx ? 0 : x + 1), xm = p - x + (x == 0 ? nx - 1 : x - 1);
  const int64_t yo = (int64_t)nx;
  const int64_t yp = p + (y + 1 == ny ? -(int64_t)(ny - 1) * yo : yo);
  const int64_t ym = p + (y == 0 ? (int64_t)(ny - 1) * yo : -yo);
  const int64_t zo = (int64_t)nx * ny;
  const int64_t zp = p + (z + 1 == nz ? -(int64_t)(nz - 1) * zo : zo);
  const int64_t zm = p + (z == 0 ? (int64_t)(nz - 1) * zo : -zo);
  const double ap = (double)a[p], bp = (double)b[p];
  const int64_t plus[3] = {xp, yp, zp}, minus[3] = {xm, ym, zm};
  double lr = 0.0, li = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double a1 = (double)a[plus[d]], a0m = (double)a[minus[d]];
    const double b1 = (double)b[plus[d]], b0m = (double)b[minus[d]];
    lr += (k.c[d] * (a1 + a0m) - k.s[d] * (b1 - b0m) - 2.0 * ap) * k.ih2[d];
    li += (k.c[d] * (b1 + b0m) + k.s[d] * (a1 - a0m) - 2.0 * bp) * k.ih2[d];
  }
  const double v = V[p];
  double hr = -0.5 * lr + v * ap - c0 * ap;
  double hi = -0.5 * li + v * bp - c0 * bp;
  hr *= alpha;
  hi *= alpha;
  const int64_t oa = (int64_t)i * M + p, ob = ((int64_t)N + i) * M + p;
  if (beta != 0.0) {
    hr += beta * (double)old[oa];
    hi += beta * (double)old[ob];
  }
  out[oa] = (T)hr;
  out[ob] = (T)hi;
}

BlochCoef coef(const Grid3& g, const double kvec[3]) {
  BlochCoef k;
  const double h[3] = {g.hx, g.hy, g.hz};
  for (int d = 0; d < 3; ++d) {
    k.c[d] = std::cos(kvec[d] * h[d]);
    k.s[d] = std::sin(kvec[d] * h[d]);
    k.ih2[d] = 1.0 / (h[d] * h[d]);
  }
  return k;
}

}  // namespace

template <typename T>
hipError_t launch_bloch_step(lrdm_ctx* ctx, const Grid3& g, const double* V, const double kvec[3],
                             const T* in, const T* old, T* out, int N, double alpha, double c0,
                             double beta) {
  dim3 grd((unsigned)((g.M + kBlochThreads - 1) / kBlochThreads), (unsigned)N);
  ProfScope prof(ctx, "bloch_step");
  bloch_step_kernel<T><<<grd, kBlochThreads, 0, ctx->stream>>>(in, old, out, V, g.nx, g.ny, g.nz,
                                                               N, coef(g, kvec), alpha, c0, beta);
  return hipGetLastError();
}
template hipError_t launch_bloch_step<double>(lrdm_ctx*, const Grid3&, const double*,
                                              const double[3], const double*, const double*,
                                              double*, int, double, double, double);
template hipError_t launch_bloch_step<float>(lrdm_ctx*, const Grid3&, const double*,
                                             const double[3], const float*, const float*, float*,
                                             int, double, double, double);

}  // namespace lrdm

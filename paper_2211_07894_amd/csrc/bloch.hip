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
// The kernels take the distance between states and the offset of a state's
// imaginary part, so that the complex Rayleigh-Ritz can also apply H_k to rows
// [Re | Im] of length 2M.
// Planes of up to 4096 points: a workgroup marches through a run of z-planes of
// one state with plane z of both parts in LDS (bloch_plane_kernel).  Larger
// planes: one thread forms both parts of one point of one state, the neighbours
// through the caches (bloch_step_kernel).
#include "lrdm_internal.h"

namespace lrdm {
namespace {

constexpr int kBlochThreads = 256;

struct BlochCoef {
  double c[3], s[3], ih2[3];   // cos(k_d h_d), sin(k_d h_d), 1/h_d^2 for x, y, z
};

// out = alpha (H_k in - c0 in) + beta old (old may be out itself: each thread
// reads old at its point before writing it; beta = 0 ignores old).
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlochThreads) void bloch_step_kernel(
    const TI* __restrict__ in, const TO* old, TO* out, const double* __restrict__ V, int nx, int ny,
    int nz, int64_t sr, int64_t si, BlochCoef k, double alpha, double c0, double beta) {
  const int64_t M = (int64_t)nx * ny * nz;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (p >= M) return;
  const int x = (int)(p % nx);
  const int y = (int)((p / nx) % ny);
  const int z = (int)(p / ((int64_t)nx * ny));
  const TI* a = in + (int64_t)i * sr;          // real part of state i
  const TI* b = a + si;                        // imaginary part
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
  const int64_t oa = (int64_t)i * sr + p, ob = oa + si;
  if (beta != 0.0) {
    hr += beta * (double)old[oa];
    hi += beta * (double)old[ob];
  }
  out[oa] = (TO)hr;
  out[ob] = (TO)hi;
}

// The same step over a run of z-planes of one state (blockIdx.x), for planes of at
// most 1024 Q points: plane z of both parts is staged in LDS for the x and y
// neighbours, planes z - 1 and z + 1 stay in registers as the run advances.  Each
// thread owns Q points of the plane.  The arithmetic is that of bloch_step_kernel,
// term for term.
template <typename TI, typename TO, int Q, int TB>
__global__ __launch_bounds__(TB) void bloch_plane_kernel(
    const TI* __restrict__ in, const TO* old, TO* out, const double* __restrict__ V, int nx, int ny,
    int nz, int64_t sr, int64_t si, int zrun, BlochCoef k, double alpha, double c0, double beta) {
  extern __shared__ __attribute__((aligned(16))) unsigned char bloch_smem[];
  double* bloch_lds = reinterpret_cast<double*>(bloch_smem);   // [2][P]: plane z, both parts
  const int P = nx * ny;
  const int i = blockIdx.x;
  const int z0 = blockIdx.y * zrun, z1 = min(nz, z0 + zrun);
  const TI* a = in + (int64_t)i * sr;
  const TI* b = a + si;
  double* la = bloch_lds;
  double* lb = bloch_lds + P;
  double am[Q], ac[Q], ap[Q], bm[Q], bc[Q], bp[Q];
  {
    const int64_t zm = z0 == 0 ? nz - 1 : z0 - 1, zp = z0 + 1 == nz ? 0 : z0 + 1;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int q = threadIdx.x + j * blockDim.x;
      am[j] = ac[j] = ap[j] = bm[j] = bc[j] = bp[j] = 0.0;
      if (q < P) {
        am[j] = (double)a[zm * P + q];
        ac[j] = (double)a[(int64_t)z0 * P + q];
        ap[j] = (double)a[zp * P + q];
        bm[j] = (double)b[zm * P + q];
        bc[j] = (double)b[(int64_t)z0 * P + q];
        bp[j] = (double)b[zp * P + q];
      }
    }
  }
  for (int z = z0; z < z1; ++z) {
    __syncthreads();   // every read of the previous plane is done
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int q = threadIdx.x + j * blockDim.x;
      if (q < P) {
        la[q] = ac[j];
        lb[q] = bc[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int q = threadIdx.x + j * blockDim.x;
      if (q >= P) continue;
      const int y = q / nx, x = q - y * nx;
      const int xp = x + 1 == nx ? q - x : q + 1, xm = x == 0 ? q + nx - 1 : q - 1;
      const int yp = y + 1 == ny ? x : q + nx, ym = y == 0 ? q + (ny - 1) * nx : q - nx;
      const double apc = ac[j], bpc = bc[j];
      const double a1[3] = {la[xp], la[yp], ap[j]}, a0m[3] = {la[xm], la[ym], am[j]};
      const double b1[3] = {lb[xp], lb[yp], bp[j]}, b0m[3] = {lb[xm], lb[ym], bm[j]};
      double lr = 0.0, li = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lr += (k.c[d] * (a1[d] + a0m[d]) - k.s[d] * (b1[d] - b0m[d]) - 2.0 * apc) * k.ih2[d];
        li += (k.c[d] * (b1[d] + b0m[d]) + k.s[d] * (a1[d] - a0m[d]) - 2.0 * bpc) * k.ih2[d];
      }
      const int64_t pz = (int64_t)z * P + q;
      const double v = V[pz];
      double hr = -0.5 * lr + v * apc - c0 * apc;
      double hi = -0.5 * li + v * bpc - c0 * bpc;
      hr *= alpha;
      hi *= alpha;
      const int64_t oa = (int64_t)i * sr + pz, ob = oa + si;
      if (beta != 0.0) {
        hr += beta * (double)old[oa];
        hi += beta * (double)old[ob];
      }
      out[oa] = (TO)hr;
      out[ob] = (TO)hi;
      // one point's neighbour values live at a time
      __builtin_amdgcn_sched_barrier(0);
    }
    // advance the run; plane z + 2 is loaded here and first used after the next
    // plane's two barriers
    const bool more = z + 1 < z1;
    const int64_t zpp = z + 2 >= nz ? z + 2 - nz : z + 2;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int q = threadIdx.x + j * blockDim.x;
      am[j] = ac[j];
      ac[j] = ap[j];
      bm[j] = bc[j];
      bc[j] = bp[j];
      if (q < P && more) {
        ap[j] = (double)a[zpp * P + q];
        bp[j] = (double)b[zpp * P + q];
      }
    }
  }
}

template <typename TI, typename TO, int Q, int TB>
hipError_t launch_plane(const Grid3& g, const double* V, const TI* in, const TO* old, TO* out,
                        int N, int64_t sr, int64_t si, int threads, const BlochCoef& k,
                        double alpha, double c0, double beta, hipStream_t stream) {
  // z runs: enough blocks for the chip (N * runs >= ~1024), runs of >= 8 planes
  int runs = 1;
  while ((int64_t)N * runs < 1024 && g.nz / (runs * 2) >= 8) runs *= 2;
  const int zrun = (g.nz + runs - 1) / runs;
  const size_t smem = 2 * (size_t)g.nx * g.ny * sizeof(double);
  if (smem > 65536)
    LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&bloch_plane_kernel<TI, TO, Q, TB>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  dim3 grd((unsigned)N, (unsigned)((g.nz + zrun - 1) / zrun));
  bloch_plane_kernel<TI, TO, Q, TB><<<grd, threads, smem, stream>>>(in, old, out, V, g.nx, g.ny,
                                                                   g.nz, sr, si, zrun, k, alpha,
                                                                   c0, beta);
  return hipGetLastError();
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

// out = alpha (H_k in - c0 in) + beta old on blocks of N complex states.
template <typename TI, typename TO>
hipError_t bloch_dispatch(lrdm_ctx* ctx, const Grid3& g, const double* V, const double kvec[3],
                          const TI* in, const TO* old, TO* out, int N, int64_t sr, int64_t si,
                          double alpha, double c0, double beta) {
  ProfScope prof(ctx, "bloch_step");
  const BlochCoef k = coef(g, kvec);
  // planes of up to 4096 points: the plane-staged kernel (1024 threads, up to
  // four points each, at most 64 KB of LDS for both parts in FP64; at four
  // points a few registers spill, and 64^2 planes still run 1.27x faster than
  // with the per-point kernel); larger planes take the per-point kernel
  const int P = g.nx * g.ny;
  if (P <= 1024)
    return launch_plane<TI, TO, 1, 1024>(g, V, in, old, out, N, sr, si, ((P + 63) / 64) * 64, k,
                                         alpha, c0, beta, ctx->stream);
  if (P <= 2048)
    return launch_plane<TI, TO, 2, 1024>(g, V, in, old, out, N, sr, si, 1024, k, alpha, c0, beta,
                                         ctx->stream);
  if (P <= 3072)
    return launch_plane<TI, TO, 3, 1024>(g, V, in, old, out, N, sr, si, 1024, k, alpha, c0, beta,
                                         ctx->stream);
  if (P <= 4096)
    return launch_plane<TI, TO, 4, 1024>(g, V, in, old, out, N, sr, si, 1024, k, alpha, c0, beta,
                                         ctx->stream);
  dim3 grd((unsigned)((g.M + kBlochThreads - 1) / kBlochThreads), (unsigned)N);
  bloch_step_kernel<TI, TO><<<grd, kBlochThreads, 0, ctx->stream>>>(
      in, old, out, V, g.nx, g.ny, g.nz, sr, si, k, alpha, c0, beta);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_bloch_step(lrdm_ctx* ctx, const Grid3& g, const double* V, const double kvec[3],
                             const T* in, const T* old, T* out, int N, double alpha, double c0,
                             double beta) {
  return bloch_dispatch<T, T>(ctx, g, V, kvec, in, old, out, N, g.M, (int64_t)N * g.M, alpha, c0,
                              beta);
}

template <typename T>
hipError_t launch_bloch_hpsi_f64(lrdm_ctx* ctx, const Grid3& g, const double* V,
                                 const double kvec[3], const T* in, double* out, int N,
                                 int64_t sr, int64_t si) {
  return bloch_dispatch<T, double>(ctx, g, V, kvec, in, nullptr, out, N, sr, si, 1.0, 0.0, 0.0);
}
template hipError_t launch_bloch_hpsi_f64<double>(lrdm_ctx*, const Grid3&, const double*,
                                                  const double[3], const double*, double*, int,
                                                  int64_t, int64_t);
template hipError_t launch_bloch_hpsi_f64<float>(lrdm_ctx*, const Grid3&, const double*,
                                                 const double[3], const float*, double*, int,
                                                 int64_t, int64_t);
template hipError_t launch_bloch_step<double>(lrdm_ctx*, const Grid3&, const double*,
                                              const double[3], const double*, const double*,
                                              double*, int, double, double, double);
template hipError_t launch_bloch_step<float>(lrdm_ctx*, const Grid3&, const double*,
                                             const double[3], const float*, const float*, float*,
                                             int, double, double, double);

}  // namespace lrdm

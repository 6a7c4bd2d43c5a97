// Stencil Hamiltonian applied to a block of vectors, fused with one step of the
// Chebyshev three-term recurrence (Sec. II C):
//     Yout = alpha (H - c0) Yin + beta Yold,   H = -1/2 Lap_h + diag(V)
// with the 7-point periodic Laplacian.  alpha = 1, c0 = 0, beta = 0 gives H Y.
// Yin and Yold have storage type TI, Yout type TO; the arithmetic is done in TO
// (H Y of an FP32 block can be formed and kept in FP64).
//
// Layout: vectors are [N][nz][ny][nx], x fastest.  A block owns one vector and a
// run of z planes; it marches in z keeping the planes z-1, z, z+1 of its points
// in registers and the whole current plane in LDS (double-buffered) for the x
// and y neighbours.  Every element of Yin is read from HBM about once (plus two
// halo planes per z run), Yold once, Yout written once: 3 M N s bytes per step,
// the bound of this HBM-limited kernel.
//
// The recurrence step of the filter takes a vectorised form of the same sweep
// when nx is a multiple of the 16-byte group (4 FP32 or 2 FP64 points): each
// thread owns groups of consecutive x points and moves each of Yin, Yold and V
// (V in the storage type) with one 16-byte load per plane, two planes ahead of
// the plane it computes, so that about twice the bytes are in flight per CU with
// fewer registers than the scalar form.  Yout may be the same buffer as Yold
// (each element is read, then written, by the same thread).
//
// Where a block owns a whole z column (N of 1024 and more, or short columns)
// three (or two) consecutive steps run in one sweep: each intermediate block is
// formed plane by plane and used by the next step while its planes are still in
// registers and LDS, and only the last two blocks (the next sweep's inputs) are
// written, so three steps move 4 M N s bytes instead of 9.
#include "lrdm_internal.h"

namespace lrdm {
namespace {

template <typename TI, typename T, int PPT>
__global__ __launch_bounds__(1024) void cheb_plane_kernel(
    const TI* __restrict__ Yin, const TI* Yold, T* Yout,
    const double* __restrict__ V, int nx, int ny, int nz, int zrun, T wx, T wy, T wz, T dshift,
    T alpha, T beta) {
  extern __shared__ unsigned char smem_raw[];
  T* plane = reinterpret_cast<T*>(smem_raw);
  const int P = nx * ny;
  const int64_t M = (int64_t)P * nz;
  const int vec = blockIdx.x;
  const int z0 = blockIdx.y * zrun;
  const int z1 = min(nz, z0 + zrun);
  const TI* yin = Yin + (int64_t)vec * M;
  const TI* yold = Yold ? Yold + (int64_t)vec * M : nullptr;
  T* yout = Yout + (int64_t)vec * M;

  int xy[PPT];   // (y << 16) | x of each point owned by this thread, -1 if none
  T prev[PPT], cur[PPT], next[PPT];
  T vcur[PPT], ocur[PPT];   // V and Yold at the current plane, loaded one plane ahead
  {
    const int zm = (z0 == 0) ? nz - 1 : z0 - 1;
    const int zp = (z0 + 1 == nz) ? 0 : z0 + 1;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int qq = threadIdx.x + j * blockDim.x;
      if (qq < P) {
        const int y = qq / nx, x = qq - y * nx;
        xy[j] = (y << 16) | x;
        prev[j] = (T)yin[(int64_t)zm * P + qq];
        cur[j] = (T)yin[(int64_t)z0 * P + qq];
        next[j] = (T)yin[(int64_t)zp * P + qq];
        vcur[j] = (T)V[(int64_t)z0 * P + qq];
        ocur[j] = yold ? (T)yold[(int64_t)z0 * P + qq] : T(0);
      } else {
        xy[j] = -1;
        prev[j] = cur[j] = next[j] = vcur[j] = ocur[j] = T(0);
      }
    }
  }
  int buf = 0;
  for (int z = z0; z < z1; ++z) {
    T* pl = plane + buf * P;
#pragma unroll
    for (int j = 0; j < PPT; ++j)
      if (xy[j] >= 0) pl[threadIdx.x + j * blockDim.x] = cur[j];
    __syncthreads();
    // loads for the next planes, issued before this plane's arithmetic
    const bool more = z + 1 < z1;
    const int zn = (z + 2 >= nz) ? z + 2 - nz : z + 2;
    T nn[PPT], vn[PPT], on[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int qq = threadIdx.x + j * blockDim.x;
      nn[j] = vn[j] = on[j] = T(0);
      if (xy[j] >= 0 && more) {
        nn[j] = (T)yin[(int64_t)zn * P + qq];
        vn[j] = (T)V[(int64_t)(z + 1) * P + qq];
        if (yold) on[j] = (T)yold[(int64_t)(z + 1) * P + qq];
      }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if (xy[j] < 0) continue;
      const int x = xy[j] & 0xffff, y = xy[j] >> 16;
      const int q = y * nx + x;
      const int xm = (x == 0) ? q + nx - 1 : q - 1;
      const int xp = (x == nx - 1) ? q - nx + 1 : q + 1;
      const int ym = (y == 0) ? q + P - nx : q - nx;
      const int yp = (y == ny - 1) ? q - P + nx : q + nx;
      const int64_t off = (int64_t)z * P + q;
      const T c = cur[j];
      const T hy = wx * (pl[xm] + pl[xp]) + wy * (pl[ym] + pl[yp]) +
                   wz * (prev[j] + next[j]) + (vcur[j] + dshift) * c;
      T out = alpha * hy;
      if (yold) out += beta * ocur[j];
      yout[off] = out;
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      prev[j] = cur[j];
      cur[j] = next[j];
      next[j] = nn[j];
      vcur[j] = vn[j];
      ocur[j] = on[j];
    }
    buf ^= 1;
  }
}

template <typename TI, typename T, int PPT>
hipError_t launch_plane(lrdm_ctx* ctx, const Grid3& g, const double* V, const TI* Yin,
                        const TI* Yold, T* Yout, int N, int threads, int zrun, double alpha,
                        double c0, double beta) {
  const int P = g.nx * g.ny;
  const size_t smem = 2 * (size_t)P * sizeof(T);
  const T wx = T(-0.5 / (g.hx * g.hx)), wy = T(-0.5 / (g.hy * g.hy)), wz = T(-0.5 / (g.hz * g.hz));
  const T dshift = T(1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz) - c0);
  dim3 grd(N, (g.nz + zrun - 1) / zrun);
  if (smem > 65536)
    LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&cheb_plane_kernel<TI, T, PPT>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  ProfScope prof(ctx, beta != 0.0 ? "cheb_step" : "hpsi");
  cheb_plane_kernel<TI, T, PPT><<<grd, threads, smem, ctx->stream>>>(
      Yin, beta != 0.0 ? Yold : nullptr, Yout, V, g.nx, g.ny, g.nz, zrun, wx, wy, wz, dshift,
      T(alpha), T(beta));
  return hipGetLastError();
}

template <typename TI, typename T>
hipError_t launch_stencil(lrdm_ctx* ctx, const Grid3& g, const double* V, const TI* Yin,
                          const TI* Yold, T* Yout, int N, double alpha, double c0, double beta) {
  const int P = g.nx * g.ny;
  // whole plane per block: up to 1024 threads, PPT points per thread
  int threads = P <= 1024 ? ((P + 63) / 64) * 64 : 1024;
  const int ppt = (P + threads - 1) / threads;
  // z runs: enough blocks for the chip (N * runs >= ~2048) but runs of >= 8 planes
  int runs = 1;
  while ((int64_t)N * runs < 2048 && g.nz / (runs * 2) >= 8) runs *= 2;
  const int zrun = (g.nz + runs - 1) / runs;
  if (ppt <= 1)
    return launch_plane<TI, T, 1>(ctx, g, V, Yin, Yold, Yout, N, threads, zrun, alpha, c0, beta);
  if (ppt <= 2)
    return launch_plane<TI, T, 2>(ctx, g, V, Yin, Yold, Yout, N, threads, zrun, alpha, c0, beta);
  if (ppt <= 4)
    return launch_plane<TI, T, 4>(ctx, g, V, Yin, Yold, Yout, N, threads, zrun, alpha, c0, beta);
  if (ppt <= 8)
    return launch_plane<TI, T, 8>(ctx, g, V, Yin, Yold, Yout, N, threads, zrun, alpha, c0, beta);
  return hipErrorInvalidValue;  // planes above 8192 points are rejected by validation
}


template <typename T, int W>
using vec_t = T __attribute__((ext_vector_type(W)));

// Vectorised step; W points per 16-byte group of the input type TI, Q groups per
// thread; arithmetic, V and Yout in T (T = TI for the recurrence, T = double for
// H Y of an FP32 block).
template <typename TI, typename T, int Q>
__global__ __launch_bounds__(1024) void cheb_vec_kernel(const TI* __restrict__ Yin, const TI* Yold,
                                                       T* Yout, const T* __restrict__ Vt, int nx,
                                                       int ny, int nz, int zrun, T wx, T wy, T wz,
                                                       T dshift, T alpha, T beta) {
  constexpr int W = 16 / sizeof(TI);
  using V = vec_t<T, W>;
  using VI = vec_t<TI, W>;
  extern __shared__ unsigned char smem_raw[];
  V* plane = reinterpret_cast<V*>(smem_raw);
  const int P = nx * ny, G = P / W, nxg = nx / W;
  const int64_t MG = (int64_t)G * nz;
  const int z0 = blockIdx.y * zrun;
  const int z1 = min(nz, z0 + zrun);
  const VI* yin = reinterpret_cast<const VI*>(Yin) + (int64_t)blockIdx.x * MG;
  const VI* yold = Yold ? reinterpret_cast<const VI*>(Yold) + (int64_t)blockIdx.x * MG : nullptr;
  V* yout = reinterpret_cast<V*>(Yout) + (int64_t)blockIdx.x * MG;
  const V* vg = reinterpret_cast<const V*>(Vt);
  const V zero = V(T(0));
  // Yin planes z-1 .. z+2, Yold and V planes z, z+1 of each owned group
  V prev[Q], cur[Q], next[Q], ahead[Q], o0[Q], o1[Q], v0[Q], v1[Q];
  {
    const int zm = (z0 == 0) ? nz - 1 : z0 - 1;
    const int zp = (z0 + 1 == nz) ? 0 : z0 + 1;
    const int zpp = (zp + 1 == nz) ? 0 : zp + 1;
    const bool m1 = z0 + 1 < z1;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int gi = threadIdx.x + j * blockDim.x;
      prev[j] = cur[j] = next[j] = ahead[j] = o0[j] = o1[j] = v0[j] = v1[j] = zero;
      if (gi < G) {
        prev[j] = __builtin_convertvector(yin[(int64_t)zm * G + gi], V);
        cur[j] = __builtin_convertvector(yin[(int64_t)z0 * G + gi], V);
        next[j] = __builtin_convertvector(yin[(int64_t)zp * G + gi], V);
        v0[j] = vg[(int64_t)z0 * G + gi];
        if (yold) o0[j] = __builtin_convertvector(yold[(int64_t)z0 * G + gi], V);
        if (m1) {
          ahead[j] = __builtin_convertvector(yin[(int64_t)zpp * G + gi], V);
          v1[j] = vg[(int64_t)(z0 + 1) * G + gi];
          if (yold) o1[j] = __builtin_convertvector(yold[(int64_t)(z0 + 1) * G + gi], V);
        }
      }
    }
  }
  int buf = 0;
  for (int z = z0; z < z1; ++z) {
    V* pl = plane + buf * G;
    const T* pls = reinterpret_cast<const T*>(pl);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int gi = threadIdx.x + j * blockDim.x;
      if (gi < G) pl[gi] = cur[j];
    }
    __syncthreads();
    // loads two planes ahead, issued before this plane's arithmetic
    const bool more2 = z + 2 < z1;
    const int zy = (z + 3 >= nz) ? z + 3 - nz : z + 3;
    VI ny_[Q], no[Q];
    V nv[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int gi = threadIdx.x + j * blockDim.x;
      ny_[j] = no[j] = VI(TI(0));
      nv[j] = zero;
      if (gi < G && more2) {
        ny_[j] = yin[(int64_t)zy * G + gi];
        nv[j] = vg[(int64_t)(z + 2) * G + gi];
        if (yold) no[j] = yold[(int64_t)(z + 2) * G + gi];
      }
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int gi = threadIdx.x + j * blockDim.x;
      if (gi >= G) continue;
      const int y = gi / nxg, x0 = (gi - y * nxg) * W;
      const int q = W * gi;
      const V ym = pl[y == 0 ? gi + G - nxg : gi - nxg];
      const V yp = pl[y == ny - 1 ? gi - G + nxg : gi + nxg];
      const T left = pls[x0 == 0 ? q + nx - 1 : q - 1];
      const T right = pls[x0 + W == nx ? q + W - nx : q + W];
      const V c = cur[j], pz = prev[j], nzv = next[j], vv = v0[j], o = o0[j];
      V out;
#pragma unroll
      for (int e = 0; e < W; ++e) {
        const T xl = e == 0 ? left : c[e == 0 ? 0 : e - 1];
        const T xr = e == W - 1 ? right : c[e == W - 1 ? 0 : e + 1];
        const T hy = wx * (xl + xr) + wy * (ym[e] + yp[e]) + wz * (pz[e] + nzv[e]) +
                     (vv[e] + dshift) * c[e];
        out[e] = alpha * hy + beta * o[e];
      }
      yout[(int64_t)z * G + gi] = out;
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      prev[j] = cur[j];
      cur[j] = next[j];
      next[j] = ahead[j];
      ahead[j] = __builtin_convertvector(ny_[j], V);
      o0[j] = o1[j];
      o1[j] = __builtin_convertvector(no[j], V);
      v0[j] = v1[j];
      v1[j] = nv[j];
    }
    buf ^= 1;
  }
}

template <typename TI, typename T, int Q>
hipError_t launch_vec(lrdm_ctx* ctx, const char* scope, const Grid3& g, const T* Vt, const TI* Yin,
                      const TI* Yold, T* Yout, int N, int threads, int zrun, double alpha,
                      double c0, double beta) {
  const int P = g.nx * g.ny;
  const size_t smem = 2 * (size_t)P * sizeof(T);
  const T wx = T(-0.5 / (g.hx * g.hx)), wy = T(-0.5 / (g.hy * g.hy)), wz = T(-0.5 / (g.hz * g.hz));
  const T dshift = T(1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz) - c0);
  dim3 grd(N, (g.nz + zrun - 1) / zrun);
  if (smem > 65536)
    LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&cheb_vec_kernel<TI, T, Q>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  ProfScope prof(ctx, scope);
  cheb_vec_kernel<TI, T, Q><<<grd, threads, smem, ctx->stream>>>(
      Yin, beta != 0.0 ? Yold : nullptr, Yout, Vt, g.nx, g.ny, g.nz, zrun, wx, wy, wz, dshift,
      T(alpha), T(beta));
  return hipGetLastError();
}

// One group of W points of a recurrence step: alpha (H - c0) y + beta o at the
// group gi of the plane pl (LDS, for the x and y neighbours), with c the group's
// own values and pz, nzv its values on the planes below and above.
template <typename T, int W>
__device__ inline vec_t<T, W> step_group(const vec_t<T, W>* pl, int gi, int G, int nx, int ny,
                                         int nxg, vec_t<T, W> c, vec_t<T, W> pz, vec_t<T, W> nzv,
                                         vec_t<T, W> vv, vec_t<T, W> o, T wx, T wy, T wz,
                                         T dshift, T alpha, T beta) {
  const T* pls = reinterpret_cast<const T*>(pl);
  const int y = gi / nxg, x0 = (gi - y * nxg) * W;
  const int q = W * gi;
  const vec_t<T, W> ym = pl[y == 0 ? gi + G - nxg : gi - nxg];
  const vec_t<T, W> yp = pl[y == ny - 1 ? gi - G + nxg : gi + nxg];
  const T left = pls[x0 == 0 ? q + nx - 1 : q - 1];
  const T right = pls[x0 + W == nx ? q + W - nx : q + W];
  vec_t<T, W> out;
#pragma unroll
  for (int e = 0; e < W; ++e) {
    const T xl = e == 0 ? left : c[e == 0 ? 0 : e - 1];
    const T xr = e == W - 1 ? right : c[e == W - 1 ? 0 : e + 1];
    const T hy = wx * (xl + xr) + wy * (ym[e] + yp[e]) + wz * (pz[e] + nzv[e]) +
                 (vv[e] + dshift) * c[e];
    out[e] = alpha * hy + beta * o[e];
  }
  return out;
}

// Two recurrence steps in one sweep, for a block that owns the whole z column of
// one vector (periodic in z, nz >= 4):
//   C = a1 (H - c0) B + b1 A,   D = a2 (H - c0) C + b2 B
// (A, B, C, D = Y_{k-1}, Y_k, Y_{k+1}, Y_{k+2}).  Each element is computed as
// the single step computes it; C never makes the round trip through HBM before
// D uses it, so the pair moves 4 M N s bytes instead of 6.  C may be the buffer
// of A and D that of B: every element of A and B that a thread reads is read by
// that thread before it writes the same element of C or D, and A on the planes
// nz-1 and 0 (C written there first) and B on 0 .. 2 are never read again.
// At plane z the sweep forms C(z+1) (from B(z), B(z+1), B(z+2)) and D(z) (from
// C(z-1), C(z), C(z+1)); C(nz-1) and C(0), which close the period, are formed
// before the sweep and kept in registers.  LDS holds the planes B(z+1) and C(z),
// double-buffered: [2 buffers][B, C][G groups].
template <typename T, int Q>
__global__ __launch_bounds__(1024) void cheb_pair_kernel(const T* Ya, const T* Yb, T* Yc, T* Yd,
                                                        const T* __restrict__ Vt, int nx, int ny,
                                                        int nz, T wx, T wy, T wz, T dshift, T a1,
                                                        T b1, T a2, T b2) {
  constexpr int W = 16 / sizeof(T);
  using V = vec_t<T, W>;
  extern __shared__ unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const int P = nx * ny, G = P / W, nxg = nx / W;
  const int64_t base = (int64_t)blockIdx.x * G * nz;
  const V* A = reinterpret_cast<const V*>(Ya) + base;
  const V* B = reinterpret_cast<const V*>(Yb) + base;
  V* C = reinterpret_cast<V*>(Yc) + base;
  V* D = reinterpret_cast<V*>(Yd) + base;
  const V* vg = reinterpret_cast<const V*>(Vt);
  const V zero = V(T(0));
  const int zl = nz - 1;
  V b0[Q], b1v[Q], b2v[Q], av[Q], vc[Q], vd[Q], cm[Q], cc[Q], cl[Q], cf[Q];
  // C(nz-1) and C(0): B planes nz-2, nz-1, 0, 1 and A, V on nz-1 and 0
  {
    V bm2[Q], bm1[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int gi = threadIdx.x + j * blockDim.x;
      bm2[j] = bm1[j] = b0[j] = b1v[j] = zero;
      if (gi < G) {
        bm2[j] = B[(int64_t)(zl - 1) * G + gi];
        bm1[j] = B[(int64_t)zl * G + gi];
        b0[j] = B[gi];
        b1v[j] = B[(int64_t)G + gi];
        lds[gi] = bm1[j];              // buffer 0, B slot: plane nz-1
        lds[2 * G + gi] = b0[j];       // buffer 1, B slot: plane 0
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int gi = threadIdx.x + j * blockDim.x;
      cl[j] = cf[j] = zero;
      if (gi < G) {
        const V al = A[(int64_t)zl * G + gi], a0 = A[gi];
        const V vl = vg[(int64_t)zl * G + gi], v0 = vg[gi];
        cl[j] = step_group<T, W>(lds, gi, G, nx, ny, nxg, bm1[j], bm2[j], b0[j], vl, al, wx, wy,
                                 wz, dshift, a1, b1);
        cf[j] = step_group<T, W>(lds + 2 * G, gi, G, nx, ny, nxg, b0[j], bm1[j], b1v[j], v0, a0,
                                 wx, wy, wz, dshift, a1, b1);
        C[(int64_t)zl * G + gi] = cl[j];
        C[gi] = cf[j];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int gi = threadIdx.x + j * blockDim.x;
    b2v[j] = av[j] = vc[j] = vd[j] = zero;
    if (gi < G) {
      b2v[j] = B[(int64_t)2 * G + gi];
      av[j] = A[(int64_t)G + gi];
      vd[j] = vg[gi];
      vc[j] = vg[(int64_t)G + gi];
    }
    cm[j] = cl[j];
    cc[j] = cf[j];
  }
  for (int z = 0; z < nz; ++z) {
    V* lb = lds + (z & 1) * 2 * G;
    V* lc = lb + G;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int gi = threadIdx.x + j * blockDim.x;
      if (gi < G) {
        lb[gi] = b1v[j];
        lc[gi] = cc[j];
      }
    }
    __syncthreads();
    // operands of the next plane, issued before this plane's arithmetic: B(z+3)
    // and A(z+2) while C(z+2) is still to be formed, V(z+2) while z+2 < nz
    const bool nextc = z + 2 <= nz - 2;
    V nb[Q], na[Q], nv[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int gi = threadIdx.x + j * blockDim.x;
      nb[j] = na[j] = nv[j] = zero;
      if (gi < G) {
        if (nextc) {
          nb[j] = B[(int64_t)(z + 3) * G + gi];
          na[j] = A[(int64_t)(z + 2) * G + gi];
        }
        if (z + 2 < nz) nv[j] = vg[(int64_t)(z + 2) * G + gi];
      }
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int gi = threadIdx.x + j * blockDim.x;
      if (gi >= G) continue;
      V cn;
      if (z + 1 <= nz - 2) {
        cn = step_group<T, W>(lb, gi, G, nx, ny, nxg, b1v[j], b0[j], b2v[j], vc[j], av[j], wx, wy,
                              wz, dshift, a1, b1);
        C[(int64_t)(z + 1) * G + gi] = cn;
      } else {
        cn = (z + 1 == zl) ? cl[j] : cf[j];
      }
      D[(int64_t)z * G + gi] = step_group<T, W>(lc, gi, G, nx, ny, nxg, cc[j], cm[j], cn, vd[j],
                                                b0[j], wx, wy, wz, dshift, a2, b2);
      cm[j] = cc[j];
      cc[j] = cn;
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      b0[j] = b1v[j];
      b1v[j] = b2v[j];
      b2v[j] = nb[j];
      av[j] = na[j];
      vd[j] = vc[j];
      vc[j] = nv[j];
    }
  }
}

template <typename T, int S>
struct ChebCoef {
  T a[S], b[S];
};

// S recurrence steps in one sweep, for a block that owns the whole z column of
// one vector (periodic in z, nz >= 2 S + 2).  Stage 0 is Y_k (Yb), stage -1 is
// Y_{k-1} (Ya); stage s = 1 .. S is Y_{k+s} = a_s (H - c0) Y_{k+s-1} + b_s Y_{k+s-2},
// each element formed as the single step forms it.  Only the last two stages are
// written (stage S-1 to Yp, stage S to Yq; they are the next group's inputs), so
// S steps move 4 M N s bytes.  Yp and Yq may be the buffers of Ya and Yb (either
// way round): a thread reads each element of Ya and Yb before it writes the same
// element of Yp or Yq, and the planes written first are never read again.
// At step h of the sweep stage s is formed on plane h + S - s from stage s-1 on
// planes h + S - s - 1 .. h + S - s + 1 (registers for z, an LDS plane for x and
// y) and stage s-2 on its own plane.  The planes that close the period (stage s on
// nz - (S - s) .. nz - 1 and 0 .. S - s - 1) are formed before the sweep and kept
// in registers.  LDS: [2 buffers][S planes][G groups].
template <typename T, int S>
__global__ __launch_bounds__(1024) void cheb_multi_kernel(const T* Ya, const T* Yb, T* Yp, T* Yq,
                                                         const T* __restrict__ Vt, int nx, int ny,
                                                         int nz, T wx, T wy, T wz, T dshift,
                                                         ChebCoef<T, S> cf) {
  constexpr int W = 16 / sizeof(T);
  using V = vec_t<T, W>;
  extern __shared__ unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const int P = nx * ny, G = P / W, nxg = nx / W;
  const int gi = threadIdx.x;
  const bool on = gi < G;
  const int64_t base = (int64_t)blockIdx.x * G * nz;
  const V* A = reinterpret_cast<const V*>(Ya) + base;
  const V* B = reinterpret_cast<const V*>(Yb) + base;
  V* Op = reinterpret_cast<V*>(Yp) + base;
  V* Oq = reinterpret_cast<V*>(Yq) + base;
  const V* vg = reinterpret_cast<const V*>(Vt);
  const V zero = V(T(0));
  auto ld = [&](const V* src, int z) { return on ? src[(int64_t)z * G + gi] : zero; };
  // plane of index j in the closing region: nz - S + j (j < S), j - S (j >= S)
  auto plane = [&](int j) { return j < S ? nz - S + j : j - S; };

  // ---- the closing region: stage s on j in [s, 2S - s)
  V pro[S][2 * S];
#pragma unroll
  for (int j = 0; j < 2 * S; ++j) pro[0][j] = ld(B, plane(j));
#pragma unroll
  for (int s = 1; s < S; ++s) {
#pragma unroll
    for (int j = s; j < 2 * S - s; ++j)
      if (on) lds[(j - s) * G + gi] = pro[s - 1][j];
    __syncthreads();
#pragma unroll
    for (int j = s; j < 2 * S - s; ++j) {
      const int z = plane(j);
      const V o = s == 1 ? ld(A, z) : pro[s - 2][j];
      pro[s][j] = zero;
      if (on) {
        pro[s][j] = step_group<T, W>(lds + (j - s) * G, gi, G, nx, ny, nxg, pro[s - 1][j],
                                     pro[s - 1][j - 1], pro[s - 1][j + 1], vg[(int64_t)z * G + gi],
                                     o, wx, wy, wz, dshift, cf.a[s - 1], cf.b[s - 1]);
        if (s == S - 1) Op[(int64_t)z * G + gi] = pro[s][j];
      }
    }
    __syncthreads();
  }

  // ---- the sweep.  win[s]: stage s on planes p_s - 2, p_s - 1, p_s once stage s
  // is formed on p_s = h + S - s (stage 0: loaded, p_0 = h + S).
  V win[S][3];
#pragma unroll
  for (int s = 1; s < S; ++s) {
    win[s][0] = zero;
    win[s][1] = pro[s][2 * S - s - 2];
    win[s][2] = pro[s][2 * S - s - 1];
  }
  win[0][0] = zero;
  win[0][1] = pro[0][2 * S - 2];
  win[0][2] = pro[0][2 * S - 1];
  V bnext = ld(B, S);
  V areg = ld(A, S - 1);
  V vw[S + 1];                       // vw[s] = V on p_s, s = 1 .. S
#pragma unroll
  for (int s = 1; s <= S; ++s) vw[s] = ld(vg, S - s);
  for (int h = 0; h < nz; ++h) {
    win[0][0] = win[0][1];
    win[0][1] = win[0][2];
    win[0][2] = bnext;
    V* buf = lds + (h & 1) * S * G;
    if (on) {
      buf[gi] = win[0][1];
#pragma unroll
      for (int s = 1; s < S; ++s) buf[s * G + gi] = win[s][2];
    }
    __syncthreads();
    // operands of the next step, issued before this step's arithmetic: B and A
    // while stage 1 is still formed, V while its plane is inside the column
    const bool next1 = h + S <= nz - S;
    bnext = next1 ? ld(B, h + S + 1) : zero;
    const V anext = next1 ? ld(A, h + S) : zero;
    const V vnext = h + S < nz ? ld(vg, h + S) : zero;
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int p = h + S - s;
      V val;
      if (p <= nz - 1 - (S - s)) {
        const V o = s == 1 ? areg : win[s - 2][0];
        val = on ? step_group<T, W>(buf + (s - 1) * G, gi, G, nx, ny, nxg, win[s - 1][1],
                                    win[s - 1][0], win[s - 1][2], vw[s], o, wx, wy, wz, dshift,
                                    cf.a[s - 1], cf.b[s - 1])
                 : zero;
        if (on && s == S - 1) Op[(int64_t)p * G + gi] = val;
      } else {
        const int jj = p - nz + S;     // in [s, 2S - s)
        val = zero;
#pragma unroll
        for (int j = s; j < 2 * S - s; ++j)
          if (j == jj) val = pro[s][j];
      }
      if (s == S) {
        if (on) Oq[(int64_t)h * G + gi] = val;
      } else {
        win[s][0] = win[s][1];
        win[s][1] = win[s][2];
        win[s][2] = val;
      }
    }
    areg = anext;
#pragma unroll
    for (int s = S; s > 1; --s) vw[s] = vw[s - 1];
    vw[1] = vnext;
  }
}

__global__ void convert_kernel(const double* __restrict__ a, int64_t n, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

}  // namespace

template <typename T>
bool cheb_vec_ok(const Grid3& g) {
  constexpr int W = 16 / sizeof(T);
  const int P = g.nx * g.ny;
  return g.nx % W == 0 && P / W <= 2 * 1024;
}

hipError_t launch_to_float(lrdm_ctx* ctx, const double* a, int64_t n, float* b) {
  convert_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(a, n, b);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cheb_step_vec(lrdm_ctx* ctx, const Grid3& g, const T* Vt, const T* Yin,
                                const T* Yold, T* Yout, int N, double alpha, double c0,
                                double beta) {
  constexpr int W = 16 / sizeof(T);
  const int G = g.nx * g.ny / W;
  if (!cheb_vec_ok<T>(g)) return hipErrorInvalidValue;
  const int threads = G <= 1024 ? ((G + 63) / 64) * 64 : 1024;
  // z runs: enough blocks for the chip (N * runs >= ~1024) but runs of >= 8 planes
  int runs = 1;
  while ((int64_t)N * runs < 1024 && g.nz / (runs * 2) >= 8) runs *= 2;
  const int zrun = (g.nz + runs - 1) / runs;
  if (G <= threads)
    return launch_vec<T, T, 1>(ctx, "cheb_step", g, Vt, Yin, Yold, Yout, N, threads, zrun, alpha,
                               c0, beta);
  return launch_vec<T, T, 2>(ctx, "cheb_step", g, Vt, Yin, Yold, Yout, N, threads, zrun, alpha,
                             c0, beta);
}

template <typename T>
bool cheb_pair_ok(const Grid3& g, int N) {
  constexpr int W = 16 / sizeof(T);
  // one group per thread (a plane of at most 1024 groups): with two the sweep's
  // registers would spill
  if (!cheb_vec_ok<T>(g) || g.nz < 4 || g.nx * g.ny / W > 1024) return false;
  // the pair needs a block per whole z column, which the single step also uses
  // once N alone fills the chip or the column is short
  return (int64_t)N >= 1024 || g.nz / 2 < 8;
}

template <typename T>
hipError_t launch_cheb_pair_vec(lrdm_ctx* ctx, const Grid3& g, const T* Vt, const T* Ya,
                                const T* Yb, T* Yc, T* Yd, int N, double c0, double a1, double b1,
                                double a2, double b2) {
  constexpr int W = 16 / sizeof(T);
  if (!cheb_pair_ok<T>(g, N)) return hipErrorInvalidValue;
  const int P = g.nx * g.ny, G = P / W;
  const int threads = ((G + 63) / 64) * 64;
  const size_t smem = 4 * (size_t)P * sizeof(T);
  const T wx = T(-0.5 / (g.hx * g.hx)), wy = T(-0.5 / (g.hy * g.hy)), wz = T(-0.5 / (g.hz * g.hz));
  const T dshift = T(1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz) - c0);
  if (smem > 65536)
    LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&cheb_pair_kernel<T, 1>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  ProfScope prof(ctx, "cheb_pair");
  cheb_pair_kernel<T, 1><<<N, threads, smem, ctx->stream>>>(Ya, Yb, Yc, Yd, Vt, g.nx, g.ny, g.nz,
                                                            wx, wy, wz, dshift, T(a1), T(b1),
                                                            T(a2), T(b2));
  return hipGetLastError();
}

template <typename T>
bool cheb_triple_ok(const Grid3& g, int N) {
  return cheb_pair_ok<T>(g, N) && g.nz >= 8;
}

template <typename T>
hipError_t launch_cheb_triple_vec(lrdm_ctx* ctx, const Grid3& g, const T* Vt, const T* Ya,
                                  const T* Yb, T* Yp, T* Yq, int N, double c0, const double* a,
                                  const double* b) {
  constexpr int W = 16 / sizeof(T);
  if (!cheb_triple_ok<T>(g, N)) return hipErrorInvalidValue;
  const int P = g.nx * g.ny, G = P / W;
  const int threads = ((G + 63) / 64) * 64;
  const size_t smem = 2 * 3 * (size_t)P * sizeof(T);
  const T wx = T(-0.5 / (g.hx * g.hx)), wy = T(-0.5 / (g.hy * g.hy)), wz = T(-0.5 / (g.hz * g.hz));
  const T dshift = T(1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz) - c0);
  ChebCoef<T, 3> cf;
  for (int s = 0; s < 3; ++s) {
    cf.a[s] = T(a[s]);
    cf.b[s] = T(b[s]);
  }
  if (smem > 65536)
    LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&cheb_multi_kernel<T, 3>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  ProfScope prof(ctx, "cheb_triple");
  cheb_multi_kernel<T, 3><<<N, threads, smem, ctx->stream>>>(Ya, Yb, Yp, Yq, Vt, g.nx, g.ny, g.nz,
                                                             wx, wy, wz, dshift, cf);
  return hipGetLastError();
}

template bool cheb_triple_ok<double>(const Grid3&, int);
template bool cheb_triple_ok<float>(const Grid3&, int);
template hipError_t launch_cheb_triple_vec<double>(lrdm_ctx*, const Grid3&, const double*,
                                                   const double*, const double*, double*, double*,
                                                   int, double, const double*, const double*);
template hipError_t launch_cheb_triple_vec<float>(lrdm_ctx*, const Grid3&, const float*,
                                                  const float*, const float*, float*, float*, int,
                                                  double, const double*, const double*);
template bool cheb_pair_ok<double>(const Grid3&, int);
template bool cheb_pair_ok<float>(const Grid3&, int);
template hipError_t launch_cheb_pair_vec<double>(lrdm_ctx*, const Grid3&, const double*,
                                                 const double*, const double*, double*, double*,
                                                 int, double, double, double, double, double);
template hipError_t launch_cheb_pair_vec<float>(lrdm_ctx*, const Grid3&, const float*,
                                                const float*, const float*, float*, float*, int,
                                                double, double, double, double, double);
template bool cheb_vec_ok<double>(const Grid3&);
template bool cheb_vec_ok<float>(const Grid3&);
template hipError_t launch_cheb_step_vec<double>(lrdm_ctx*, const Grid3&, const double*,
                                                 const double*, const double*, double*, int,
                                                 double, double, double);
template hipError_t launch_cheb_step_vec<float>(lrdm_ctx*, const Grid3&, const float*,
                                                const float*, const float*, float*, int, double,
                                                double, double);

namespace {
}  // namespace

template <typename T>
hipError_t launch_cheb_step(lrdm_ctx* ctx, const Grid3& g, const double* V, const T* Yin,
                            const T* Yold, T* Yout, int N, double alpha, double c0, double beta) {
  return launch_stencil<T, T>(ctx, g, V, Yin, Yold, Yout, N, alpha, c0, beta);
}

template <typename T>
hipError_t launch_hpsi_f64(lrdm_ctx* ctx, const Grid3& g, const double* V, const T* Y, double* HY,
                           int N) {
  constexpr int W = 16 / sizeof(T);
  auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const int G = g.nx * g.ny / W;
  if (cheb_vec_ok<T>(g) && G <= 1024 && aligned(Y) && aligned(HY) && aligned(V)) {
    const int threads = ((G + 63) / 64) * 64;
    int runs = 1;
    while ((int64_t)N * runs < 1024 && g.nz / (runs * 2) >= 8) runs *= 2;
    const int zrun = (g.nz + runs - 1) / runs;
    return launch_vec<T, double, 1>(ctx, "hpsi", g, V, Y, nullptr, HY, N, threads, zrun, 1.0, 0.0,
                                    0.0);
  }
  return launch_stencil<T, double>(ctx, g, V, Y, nullptr, HY, N, 1.0, 0.0, 0.0);
}

template hipError_t launch_cheb_step<double>(lrdm_ctx*, const Grid3&, const double*, const double*,
                                             const double*, double*, int, double, double, double);
template hipError_t launch_cheb_step<float>(lrdm_ctx*, const Grid3&, const double*, const float*,
                                            const float*, float*, int, double, double, double);
template hipError_t launch_hpsi_f64<double>(lrdm_ctx*, const Grid3&, const double*, const double*,
                                            double*, int);
template hipError_t launch_hpsi_f64<float>(lrdm_ctx*, const Grid3&, const double*, const float*,
                                           double*, int);

}  // namespace lrdm

// Matrix-core contractions for the single-precision storage forms (Psi, X, Y held
// as FP32; eps, V, dV, drho and every N x N matrix stay FP64).
//
//  LRDM_FP32    FP32 operands on v_mfma_f32_16x16x4f32.
//  LRDM_BF16X3  FP32 operands split exactly into three BF16 pieces,
//               x = hi + mid + lo (8 + 8 + 8 significant bits), on
//               v_mfma_f32_16x16x32_bf16, keeping the six products of order <= 2
//               (hi*hi; hi*mid + mid*hi; hi*lo + mid*mid + lo*hi), so each product
//               carries an error of about 2^-24, as in FP32.  The density is too
//               sensitive for a two-piece split (hi*hi + hi*lo + lo*hi, error
//               about 2^-16 per product): that leaves relative errors of a few
//               1e-6 in the response density.
//
// The two response contractions (tn_sym, backproj; same meaning as the FP64
// forms) share one 128 x 128 tile core computing C = A B^T over a K range.  A and B
// tiles are staged in LDS as FP32 in [row][k] layout (k contiguous), so a lane
// fetches 8 consecutive k of one row with two 16-byte LDS reads.  For the FP32
// instruction the lanes of group g = lane/16 take k = 8g + s at step s (any
// permutation of k is allowed as long as A and B use the same one); for the BF16
// instruction those 8 values are exactly the operand of one lane.  Partial sums
// live in FP32 for one K-tile (KT = 32 values of k) and are then added into FP64
// registers, so FP32 rounding never accumulates over more than 32 terms.
//
// Lane layouts (measured on gfx950):
//   v_mfma_f32_16x16x4f32:      A lane l -> A[l%16][l/16], B lane l -> B[l/16][l%16]
//   v_mfma_f32_16x16x32_bf16:   A lane l -> A[l%16][8(l/16)+e], B -> B[8(l/16)+e][l%16]
//   both:                       D lane l, register v -> D[4(l/16) + v][l%16]
#include <algorithm>

#include "blocks.h"
#include "lrdm_internal.h"
#include "xcd.h"

namespace lrdm {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef double d2v __attribute__((ext_vector_type(2)));

constexpr int BT = 128;      // output tile edge
constexpr int KT = 32;       // k extent staged per step
constexpr int KP = KT + 4;   // LDS row pitch in floats (16-byte aligned rows)

enum class Core { F32, BF2, BF3 };  // BF2: two-piece split, order <= 1 (kept for measurement)

__device__ inline f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Exact split of 8 FP32 values into BF16 pieces (round to nearest even at each
// stage; every remainder is exact in FP32).
template <int NP>
__device__ inline void split(const float (&x)[8], bf8 (&p)[NP]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float r = x[e];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const __bf16 h = (__bf16)r;
      p[q][e] = h;
      r -= (float)h;
    }
  }
}

// Exact three-piece split of 8 FP32 values with round-to-nearest pieces (as the
// pre-split operands): pairs of values are converted together (one packed
// conversion per pair and piece), and each piece is widened back by placing its
// 16 bits in the high half of an FP32.  |mid| <= 2^-9 |x|, |lo| <= 2^-17 |x|.
__device__ inline void split3_rne(const float (&x)[8], bf8 (&p)[3]) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  u4 w[3];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    f2 r = {x[2 * e], x[2 * e + 1]};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const b2 h = __builtin_convertvector(r, b2);
      const unsigned hb = __builtin_bit_cast(unsigned, h);
      w[q][e] = hb;
      if (q < 2) {
        const f2 hf = {__uint_as_float(hb << 16), __uint_as_float(hb & 0xffff0000u)};
        r = r - hf;
      }
    }
  }
  p[0] = __builtin_bit_cast(bf8, w[0]);
  p[1] = __builtin_bit_cast(bf8, w[1]);
  p[2] = __builtin_bit_cast(bf8, w[2]);
}

// Lane-local fragment of rows (base + 16i + lane%16), k = 8(lane/16) .. +7.
__device__ inline void frag(const float* S, int base, int lane, float (&v)[4][8]) {
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const f4* p = reinterpret_cast<const f4*>(S + (base + i * 16 + r) * KP + 8 * g);
    const f4 x = p[0], y = p[1];
    v[i][0] = x[0]; v[i][1] = x[1]; v[i][2] = x[2]; v[i][3] = x[3];
    v[i][4] = y[0]; v[i][5] = y[1]; v[i][6] = y[2]; v[i][7] = y[3];
  }
}

// One K-tile of the wave's 64 x 64 sub-tile: acc += A_rows B_rows^T over KT.
template <Core C>
__device__ inline void kt_step(const float* As, const float* Bs, int wr, int wc, int lane,
                               double (&acc)[4][4][4]) {
  float a[4][8], b[4][8];
  frag(As, wr * 64, lane, a);
  frag(Bs, wc * 64, lane, b);
  f4 c[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (C == Core::F32) {
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) c[i][j] = mfma_f32(a[i][s], b[j][s], c[i][j]);
  } else {
    constexpr int NP = (C == Core::BF3) ? 3 : 2;
    bf8 pa[4][NP];
#pragma unroll
    for (int i = 0; i < 4; ++i) split<NP>(a[i], pa[i]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf8 pb[NP];
      split<NP>(b[j], pb);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // smallest terms first
        if constexpr (C == Core::BF3) {
          c[i][j] = mfma_bf16(pa[i][0], pb[2], c[i][j]);
          c[i][j] = mfma_bf16(pa[i][1], pb[1], c[i][j]);
          c[i][j] = mfma_bf16(pa[i][2], pb[0], c[i][j]);
        }
        c[i][j] = mfma_bf16(pa[i][0], pb[1], c[i][j]);
        c[i][j] = mfma_bf16(pa[i][1], pb[0], c[i][j]);
        c[i][j] = mfma_bf16(pa[i][0], pb[0], c[i][j]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)c[i][j][v];
}

__device__ inline void zero(double (&acc)[4][4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0.0;
}

template <typename S>
__device__ inline bool aligned16(const S* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

// Rows [r0, r0+BT) x k in [k0, k0+KT) of a row-major FP32 [nrows][ld] array (k
// contiguous), times w[k] (the FP64 product rounded once) and a factor; zero
// outside [0, nrows) x [., kend).  Thread t: row t/2, k = 16 (t%2) .. +15.  load()
// only issues the global reads; the products are formed in store(), after the
// current K-tile's matrix-core work, so the reads stay in flight meanwhile.
struct StageDirect {
  float v[16];
  double wv[16];
  float fac;
  bool has_w;
  __device__ inline void load(const float* __restrict__ X, int64_t ld, int nrows, int r0,
                              int64_t k0, int64_t kend, const double* __restrict__ w,
                              float factor) {
    const int t = threadIdx.x;
    const int gr = r0 + (t >> 1);
    const int64_t kb = k0 + (t & 1) * 16;
    const float* src = X + (int64_t)gr * ld + kb;
    fac = factor;
    has_w = (w != nullptr);
    if (gr < nrows && kb + 16 <= kend && aligned16(src) && (!w || aligned16(w + kb))) {
      const f4* s4 = reinterpret_cast<const f4*>(src);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f4 x = s4[q];
        v[4 * q] = x[0]; v[4 * q + 1] = x[1]; v[4 * q + 2] = x[2]; v[4 * q + 3] = x[3];
      }
      if (w) {
        const double2* w2 = reinterpret_cast<const double2*>(w + kb);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double2 y = w2[q];
          wv[2 * q] = y.x;
          wv[2 * q + 1] = y.y;
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t k = kb + q;
        const bool in = gr < nrows && k < kend;
        v[q] = in ? X[(int64_t)gr * ld + k] : 0.f;
        wv[q] = (in && w) ? w[k] : 1.0;
      }
    }
  }
  __device__ inline void store(float* Sm) {
    const int t = threadIdx.x;
    if (has_w) {
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = (float)((double)v[q] * wv[q]);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] *= fac;
    f4* dst = reinterpret_cast<f4*>(Sm + (t >> 1) * KP + (t & 1) * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = f4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
  }
};

// Columns [c0, c0+BT) x k in [k0, k0+KT) of a row-major FP32 [nk][ld] array whose
// rows are indexed by k (columns contiguous), stored transposed as [column][k];
// zero outside [0, nk) x [0, ncols).  Thread t: k = t%32, columns 16 (t/32) .. +15,
// so that the transposed LDS writes of a wave fall on consecutive banks.
struct StageTrans {
  float v[16];
  __device__ inline void load(const float* __restrict__ X, int64_t ld, int64_t nk, int64_t ncols,
                              int64_t k0, int64_t c0) {
    const int t = threadIdx.x;
    const int64_t gk = k0 + (t & 31);
    const int64_t cb = c0 + (t >> 5) * 16;
    const float* src = X + gk * ld + cb;
    if (gk < nk && cb + 16 <= ncols && aligned16(src)) {
      const f4* s4 = reinterpret_cast<const f4*>(src);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f4 x = s4[q];
        v[4 * q] = x[0]; v[4 * q + 1] = x[1]; v[4 * q + 2] = x[2]; v[4 * q + 3] = x[3];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t cc = cb + q;
        v[q] = (gk < nk && cc < ncols) ? X[gk * ld + cc] : 0.f;
      }
    }
  }
  __device__ inline void store(float* Sm) const {
    const int t = threadIdx.x;
    const int kr = t & 31, cb = (t >> 5) * 16;
#pragma unroll
    for (int q = 0; q < 16; ++q) Sm[(cb + q) * KP + kr] = v[q];
  }
};

// ------------------------------------------------------------------ tn_sym
// 1-D grid over (split, batch) groups of upper tiles (xcd_map); part
// [batch][split][tile][BT][BT].
template <Core C>
__global__ __launch_bounds__(256, 1) void tn_sym_lp_kernel(
    const float* __restrict__ A, const float* __restrict__ B, const double* __restrict__ w,
    int64_t w_stride, int N, int64_t M, int nspin, int ntb, int64_t kchunk, int nsplit, int batch,
    const unsigned char* __restrict__ active, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) float As[BT * KP];
  __shared__ __attribute__((aligned(16))) float Bs[BT * KP];
  const int ntiles = ntb * (ntb + 1) / 2;
  int group, tile;
  xcd_map(blockIdx.x, nsplit * batch, ntiles, group, tile);
  const int sp = group % nsplit, b = group / nsplit;
  int ti = 0, rem = tile;
  while (rem >= ntb - ti) { rem -= ntb - ti; ++ti; }
  const int tj = ti + rem;
  const int c = b % nspin;
  const float* Ac = A + (int64_t)c * N * M;
  const float* Bc = B + (int64_t)c * N * M;
  const double* wb = w ? w + (int64_t)b * w_stride : nullptr;
  const int64_t kbeg = (int64_t)sp * kchunk;
  // an inactive block (blocks.h) keeps a zero partial tile
  const int64_t kend = block_active(active, c, ntb, ti, tj) ? min(M, kbeg + kchunk) : kbeg;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  double acc[4][4][4];
  zero(acc);
  StageDirect la, lb;
  if (kbeg < kend) {
    la.load(Ac, M, N, ti * BT, kbeg, kend, nullptr, 1.f);
    lb.load(Bc, M, N, tj * BT, kbeg, kend, wb, 1.f);
  }
  for (int64_t k0 = kbeg; k0 < kend; k0 += KT) {
    __syncthreads();
    la.store(As);
    lb.store(Bs);
    __syncthreads();
    if (k0 + KT < kend) {
      la.load(Ac, M, N, ti * BT, k0 + KT, kend, nullptr, 1.f);
      lb.load(Bc, M, N, tj * BT, k0 + KT, kend, wb, 1.f);
    }
    kt_step<C>(As, Bs, wr, wc, lane, acc);
  }
  double* out = part + (((int64_t)b * nsplit + sp) * ntiles + tile) * (BT * BT);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int col = wc * 64 + j * 16 + (lane & 15);
        out[row * BT + col] = acc[i][j][v];
      }
}

// Same fixed-order split sum as the FP64 form.
__global__ void tn_reduce_lp_kernel(const double* __restrict__ part, int N, int ntb, int nsplit,
                                    double* __restrict__ H) {
  const int b = blockIdx.z;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= N || j >= N) return;
  const int ii = min(i, j), jj = max(i, j);
  const int ti = ii / BT, tj = jj / BT;
  const int tile = ti * ntb - ti * (ti - 1) / 2 + (tj - ti);
  const int ntiles = ntb * (ntb + 1) / 2;
  const int r = ii - ti * BT, cc = jj - tj * BT;
  double s = 0.0;
  for (int q = 0; q < nsplit; ++q)
    s += part[(((int64_t)b * nsplit + q) * ntiles + tile) * (BT * BT) + r * BT + cc];
  H[((int64_t)b * N + i) * N + j] = s;
}

__global__ void to_f32_kernel(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

// ================================================================== pipelined forms
// Eight waves per block (two per SIMD), each owning a 32 x 64 part of the 128 x
// 128 tile.  Operand tiles go from global memory straight into LDS
// (global_load_lds_dwordx4: lane l of a wave writes 16 bytes at base + 16 l) in a
// ring of NST stages, so NST - 1 K-tiles are in flight while one is multiplied.
// A tile row (32 FP32 = eight 16-byte chunks) keeps logical chunk q in slot
// q ^ tile_swizzle(row), which spreads a wave's fragment reads over the LDS banks.
// Chunks outside the operands are fetched from a page of zeros.
constexpr int PW = 8;                     // waves per block
constexpr int PT = PW * 64;               // threads per block
constexpr int NST = 3;                    // ring stages
constexpr int TB = BT * KT * 4;           // bytes of one operand tile (16 KB)

typedef __attribute__((address_space(3))) void lds_void;

// Wait until at most VM of this wave's global->LDS copies are outstanding, then
// barrier: the "memory" clobber keeps the compiler from moving LDS accesses across.
template <int VM>
__device__ inline void wait_stage() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(VM) : "memory");
}

__device__ inline void dma16(const void* src, unsigned char* lds) {
  __builtin_amdgcn_global_load_lds(src, (lds_void*)lds, 16, 0, 0);
}

// This wave's share (2 of 16 copy instructions) of one operand tile: rows
// [r0, r0+BT) x k in [k0, k0+KT) of the row-major FP32 [nrows][ld] array X.
// Chunks with a row >= nrows or k >= kend (kend a multiple of 4) read zeros.
// Slot permutation of the eight 16-byte chunks of an FP32 tile row (128 bytes):
// chunk q of row r sits in slot q ^ tile_swizzle(r), so 8 consecutive rows reading
// one chunk fall in distinct 16-byte bank groups.  (A permutation that also
// separates rows 8 apart removed the remaining bank conflicts of these reads but
// made the FP32 kernels 2 % slower on the device, so this one stays.)
__device__ inline int tile_swizzle(int r) { return r & 7; }

__device__ inline void dma_tile(const float* __restrict__ X, int64_t ld, int nrows, int64_t r0,
                                int64_t k0, int64_t kend, const float* zeros, unsigned char* tile,
                                int wid, int lane) {
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int ins = wid * 2 + u;                      // 64 chunks = 8 rows each
    const int r = ins * 8 + (lane >> 3);
    const int q = (lane & 7) ^ tile_swizzle(r);       // logical chunk of slot lane & 7
    const int64_t k = k0 + 4 * q;
    const int64_t gr = r0 + r;
    const float* src = (gr < nrows && k < kend) ? X + gr * ld + k : zeros;
    dma16(src, tile + ins * 1024);
  }
}

// The weights w[k0 .. k0+KT) of one K-tile (16 chunks of two doubles; lanes
// 16..63 repeat them), zeros at k >= kend (a multiple of 4).  Issued by wave 0.
__device__ inline void dma_weights(const double* __restrict__ w, int64_t k0, int64_t kend,
                                   const float* zeros, unsigned char* wtile, int lane) {
  const int64_t k = k0 + 2 * (lane & 15);
  const void* src = (k < kend) ? (const void*)(w + k) : (const void*)zeros;
  dma16(src, wtile);
}

// Lane fragment of rows base + 16 i + lane%16, k = 8(lane/16) .. +7 of a swizzled tile.
template <int NI>
__device__ inline void frag_sw(const unsigned char* tile, int base, int lane, float (&v)[NI][8]) {
  const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int R = base + 16 * i + r16;
    const int sw = tile_swizzle(R);
    const f4 x = *reinterpret_cast<const f4*>(tile + (R * 8 + ((2 * g) ^ sw)) * 16);
    const f4 y = *reinterpret_cast<const f4*>(tile + (R * 8 + ((2 * g + 1) ^ sw)) * 16);
    v[i][0] = x[0]; v[i][1] = x[1]; v[i][2] = x[2]; v[i][3] = x[3];
    v[i][4] = y[0]; v[i][5] = y[1]; v[i][6] = y[2]; v[i][7] = y[3];
  }
}

// The wave's operands of one K-tile (rows of its 32 x 64 part), read from LDS
// before the next copies are issued: an LDS read after a global->LDS copy would
// make the compiler wait for every copy in flight.  weight() scales B's column k
// by w[k] (FP32 product of the rounded weight).
struct PipeFrag {
  float a[2][8], b[4][8];
  __device__ inline void load(const unsigned char* At, const unsigned char* Bt, int wr, int wc,
                              int lane) {
    frag_sw<2>(At, wr * 32, lane, a);
    frag_sw<4>(Bt, wc * 64, lane, b);
  }
  // wt: the weights of the K-tile in LDS
  __device__ inline void weight(const unsigned char* wt, int lane) {
    const int g = lane >> 4;
    float wf[8];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      // read as FP32 lanes like the tiles (the compiler then leaves the wait for
      // the copies to wait_stage), then reinterpret the 16 bytes as two doubles
      const f4 x = *reinterpret_cast<const f4*>(wt + (4 * g + h) * 16);
      const d2v y = __builtin_bit_cast(d2v, x);
      wf[2 * h] = (float)y[0];
      wf[2 * h + 1] = (float)y[1];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 8; ++e) b[j][e] *= wf[e];
  }
};

// acc += scale * A B^T over one K-tile of the wave's 32 x 64 part (registers only).
template <Core C>
__device__ inline void kt_step_pipe(PipeFrag& f, double scale, double (&acc)[2][4][4]) {
  f4 c[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (C == Core::F32) {
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) c[i][j] = mfma_f32(f.a[i][s], f.b[j][s], c[i][j]);
  } else {
    constexpr int NP = (C == Core::BF3) ? 3 : 2;
    bf8 pa[2][NP];
#pragma unroll
    for (int i = 0; i < 2; ++i) split<NP>(f.a[i], pa[i]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf8 pb[NP];
      split<NP>(f.b[j], pb);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if constexpr (C == Core::BF3) {
          c[i][j] = mfma_bf16(pa[i][0], pb[2], c[i][j]);
          c[i][j] = mfma_bf16(pa[i][1], pb[1], c[i][j]);
          c[i][j] = mfma_bf16(pa[i][2], pb[0], c[i][j]);
        }
        c[i][j] = mfma_bf16(pa[i][0], pb[1], c[i][j]);
        c[i][j] = mfma_bf16(pa[i][1], pb[0], c[i][j]);
        c[i][j] = mfma_bf16(pa[i][0], pb[0], c[i][j]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] += scale * (double)c[i][j][v];
}

// Keeps the compiler from moving memory accesses across this point.
__device__ inline void compiler_fence() { asm volatile("" ::: "memory"); }

// FP32 partial sums of the BF16X3 kernels are added into FP64 every kFlush
// K-tiles (kFlush * KT = 128 terms of each product).
constexpr int kFlush = 4;
static_assert(BT % (kFlush * KT) == 0, "flush groups must not straddle the diagonal blocks");

__device__ inline void zero_f32(f4 (&cc)[2][4]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) cc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
}

// acc += f * cc, cc = 0.
__device__ inline void flush_pipe(f4 (&cc)[2][4], double f, double (&acc)[2][4][4]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] += f * (double)cc[i][j][v];
      cc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
}

__device__ inline void zero_pipe(double (&acc)[2][4][4]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0.0;
}

// tn_sym, pipelined: same grid and partial layout as tn_sym_lp_kernel.  Requires M
// a multiple of 4 and 16-byte aligned A, B and weight rows.  W: B weighted by w.
// The body, for workgroup `lin` of the launch's grid (the fused launch of several
// systems passes each system's own workgroup index).
template <Core C, bool W>
__device__ inline void tn_sym_pipe_body(
    int lin, const float* __restrict__ A, const float* __restrict__ B,
    const double* __restrict__ w, int64_t w_stride, int N, int64_t M, int nspin, int ntb,
    int64_t kchunk, int nsplit, int batch, const unsigned char* __restrict__ active,
    const float* __restrict__ zeros, double* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pipe[];
  constexpr int SB = 2 * TB + (W ? 1024 : 0);   // bytes of one stage
  const int ntiles = ntb * (ntb + 1) / 2;
  int group, tile;
  xcd_map(lin, nsplit * batch, ntiles, group, tile);
  const int sp = group % nsplit, b = group / nsplit;
  int ti = 0, rem = tile;
  while (rem >= ntb - ti) { rem -= ntb - ti; ++ti; }
  const int tj = ti + rem;
  const int c = b % nspin;
  const float* Ac = A + (int64_t)c * N * M;
  const float* Bc = B + (int64_t)c * N * M;
  const double* wb = W ? w + (int64_t)b * w_stride : nullptr;
  const int64_t kbeg = (int64_t)sp * kchunk;
  // an inactive block (blocks.h) keeps a zero partial tile
  const int64_t kend = block_active(active, c, ntb, ti, tj) ? min(M, kbeg + kchunk) : kbeg;
  const int nk = kbeg < kend ? (int)((kend - kbeg + KT - 1) / KT) : 0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  // Every stage issues the same copies (zeros past the end), so the count of
  // copies in flight per wave is the same at every wait: 4 per stage, plus the
  // weights in wave 0.
  auto issue = [&](int t) {
    unsigned char* st = smem_pipe + (t % NST) * SB;
    const int64_t k0 = kbeg + (int64_t)t * KT;
    const int64_t ke = t < nk ? kend : k0;
    dma_tile(Ac, M, N, (int64_t)ti * BT, k0, ke, zeros, st, wid, lane);
    dma_tile(Bc, M, N, (int64_t)tj * BT, k0, ke, zeros, st + TB, wid, lane);
    if (W && wid == 0) dma_weights(wb, k0, ke, zeros, st + 2 * TB, lane);
  };
  double acc[2][4][4];
  zero_pipe(acc);
  issue(0);
  issue(1);
  for (int t = 0; t < nk; ++t) {
    if (W && wid == 0) wait_stage<5>(); else wait_stage<4>();
    const unsigned char* st = smem_pipe + (t % NST) * SB;
    PipeFrag f;
    f.load(st, st + TB, wr, wc, lane);
    if (W) f.weight(st + 2 * TB, lane);
    compiler_fence();
    issue(t + 2);
    kt_step_pipe<C>(f, 1.0, acc);
  }
  wait_stage<0>();
  double* out = part + (((int64_t)b * nsplit + sp) * ntiles + tile) * (BT * BT);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 32 + i * 16 + 4 * (lane >> 4) + v;
        const int col = wc * 64 + j * 16 + (lane & 15);
        out[row * BT + col] = acc[i][j][v];
      }
}

template <Core C, bool W>
__global__ __launch_bounds__(PT, 1) void tn_sym_pipe_kernel(
    const float* __restrict__ A, const float* __restrict__ B, const double* __restrict__ w,
    int64_t w_stride, int N, int64_t M, int nspin, int ntb, int64_t kchunk, int nsplit, int batch,
    const unsigned char* __restrict__ active, const float* __restrict__ zeros,
    double* __restrict__ part) {
  tn_sym_pipe_body<C, W>(blockIdx.x, A, B, w, w_stride, N, M, nspin, ntb, kchunk, nsplit, batch,
                         active, zeros, part);
}

// backproj, pipelined.  Gf: FP32 copies of the symmetric matrices [batch][N][ldk];
// PT_: FP32 transposes of the blocks, [nspin][M][ldk] (A^T, points as rows); ldk a
// multiple of KT with zeros in the columns >= N.  A ([nspin][N][M]) feeds the row-dot.
template <Core C>
__device__ inline void backproj_pipe_body(
    int lin, const float* __restrict__ A, const float* __restrict__ AT,
    const float* __restrict__ Gf, int N, int64_t M, int ldk, int nspin, int batch, double scale,
    const double* __restrict__ sub, const unsigned char* __restrict__ active,
    const float* __restrict__ zeros, double* __restrict__ out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pipe[];
  constexpr int SB = 2 * TB;
  double* red = reinterpret_cast<double*>(smem_pipe + NST * SB);   // [PW][64]
  // 1-D grid: the directions of one block of points run together on one XCD
  int pblk, b;
  xcd_map(lin, (int)((M + BT - 1) / BT), batch, pblk, b);
  const int c = b % nspin;
  const float* Ac = A + (int64_t)c * N * M;
  const float* ATc = AT + (int64_t)c * M * ldk;
  const float* Gb = Gf + (int64_t)b * N * ldk;
  const int64_t p0 = (int64_t)pblk * BT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  double dsum[4] = {0.0, 0.0, 0.0, 0.0};
  const int nib = (N + BT - 1) / BT;
  for (int ib = 0; ib < nib; ++ib) {
    const int i0 = ib * BT;
    // j runs over the active blocks (blocks.h) of [i0, N): the diagonal block
    // once, blocks right of it twice
    const uint64_t bits = active_row_bits(active, c, nib, ib);
    const int nk = active_ktiles(bits, N, KT);
    if (nk == 0) continue;
    auto issue = [&](int t) {
      unsigned char* st = smem_pipe + (t % NST) * SB;
      int J;
      const int64_t j0 = active_ktile(bits, t, KT, J);
      const int64_t je = t < nk ? ldk : j0;
      dma_tile(Gb, ldk, N, i0, j0, je, zeros, st, wid, lane);
      dma_tile(ATc, ldk, (int)M, p0, j0, je, zeros, st + TB, wid, lane);
    };
    double acc[2][4][4];
    zero_pipe(acc);
    issue(0);
    issue(1);
    for (int t = 0; t < nk; ++t) {
      wait_stage<4>();
      const unsigned char* st = smem_pipe + (t % NST) * SB;
      PipeFrag f;
      f.load(st, st + TB, wr, wc, lane);
      compiler_fence();
      issue(t + 2);
      int J;
      active_ktile(bits, t, KT, J);
      kt_step_pipe<C>(f, J > ib ? 2.0 : 1.0, acc);
    }
    wait_stage<0>();   // the copies past the end land before the ring is reused
    // row-dot with A[i][p]: all 32 reads issued first (indices clamped into
    // range, out-of-range terms dropped afterwards)
    float av[2][4][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = min(i0 + wr * 32 + i * 16 + 4 * (lane >> 4) + v, N - 1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t p = min(p0 + wc * 64 + j * 16 + (lane & 15), M - 1);
          av[i][v][j] = Ac[(int64_t)gi * M + p];
        }
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wr * 32 + i * 16 + 4 * (lane >> 4) + v;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
          if (gi < N && p < M) dsum[j] += acc[i][j][v] * (double)av[i][v][j];
        }
      }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double v = dsum[j];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    dsum[j] = v;
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wid * 64 + j * 16 + lane] = dsum[j];
  }
  __syncthreads();
  if (threadIdx.x < BT) {
    const int col = threadIdx.x;
    const int wcc = col >> 6, cl = col & 63;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) v += red[(2 * q + wcc) * 64 + cl];
    const int64_t p = p0 + col;
    if (p < M) {
      double r = scale * v;
      if (sub) r -= sub[(int64_t)b * M + p];
      out[(int64_t)b * M + p] = r;
    }
  }
}

template <Core C>
__global__ __launch_bounds__(PT, 1) void backproj_pipe_kernel(
    const float* __restrict__ A, const float* __restrict__ AT, const float* __restrict__ Gf,
    int N, int64_t M, int ldk, int nspin, int batch, double scale, const double* __restrict__ sub,
    const unsigned char* __restrict__ active, const float* __restrict__ zeros,
    double* __restrict__ out) {
  backproj_pipe_body<C>(blockIdx.x, A, AT, Gf, N, M, ldk, nspin, batch, scale, sub, active,
                        zeros, out);
}

// ------------------------------------------------------------------ fused systems
// One launch of the FP32 projection (or back-projection) over up to kMaxFused
// independent systems: system s owns workgroups [wg0[s], wg0[s+1]) (each range
// a multiple of the XCD count, so that a system's own XCD grouping holds; the
// padding workgroups exit at once), with its operands passed by value.
constexpr int kMaxFused = 16;

struct FusedProj {
  int nsys;
  int wg0[kMaxFused + 1];
  int used[kMaxFused];                 // workgroups system s needs
  const float* A[kMaxFused];
  const double* w[kMaxFused];
  double* part[kMaxFused];
  const unsigned char* active[kMaxFused];
  int64_t M[kMaxFused], kchunk[kMaxFused];
  int N[kMaxFused], nspin[kMaxFused], ntb[kMaxFused], nsplit[kMaxFused], batch[kMaxFused];
};

struct FusedBackproj {
  int nsys;
  int wg0[kMaxFused + 1];
  int used[kMaxFused];
  const float* A[kMaxFused];
  const float* AT[kMaxFused];
  const float* Gf[kMaxFused];
  double* out[kMaxFused];
  const unsigned char* active[kMaxFused];
  int64_t M[kMaxFused];
  int N[kMaxFused], ldk[kMaxFused], nspin[kMaxFused], batch[kMaxFused];
  double scale[kMaxFused];
};

__device__ inline int fused_system(const int* wg0, int nsys, int bid) {
  int s = 0;
  while (s + 1 < nsys && bid >= wg0[s + 1]) ++s;
  return s;
}

__global__ __launch_bounds__(PT, 1) void tn_sym_fused_kernel(const FusedProj t,
                                                             const float* __restrict__ zeros) {
  const int s = fused_system(t.wg0, t.nsys, blockIdx.x);
  const int lin = blockIdx.x - t.wg0[s];
  if (lin >= t.used[s]) return;
  tn_sym_pipe_body<Core::F32, true>(lin, t.A[s], t.A[s], t.w[s], t.M[s], t.N[s], t.M[s],
                                    t.nspin[s], t.ntb[s], t.kchunk[s], t.nsplit[s], t.batch[s],
                                    t.active[s], zeros, t.part[s]);
}

__global__ __launch_bounds__(PT, 1) void backproj_fused_kernel(const FusedBackproj t,
                                                               const float* __restrict__ zeros) {
  const int s = fused_system(t.wg0, t.nsys, blockIdx.x);
  const int lin = blockIdx.x - t.wg0[s];
  if (lin >= t.used[s]) return;
  backproj_pipe_body<Core::F32>(lin, t.A[s], t.AT[s], t.Gf[s], t.N[s], t.M[s], t.ldk[s],
                                t.nspin[s], t.batch[s], t.scale[s], nullptr, t.active[s], zeros,
                                t.out[s]);
}

// Gf[b][i][j] = G[b][i][j] for j < N, 0 for N <= j < ldk.
__global__ void gamma_pad_kernel(const double* __restrict__ G, float* __restrict__ Gf, int N,
                                 int ldk, int batch) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)batch * N * ldk;
  if (idx >= total) return;
  const int j = (int)(idx % ldk);
  const int64_t bi = idx / ldk;
  Gf[idx] = j < N ? (float)G[bi * N + j] : 0.f;
}

// AT[c][p][j] = A[c][j][p] for j < N, 0 for N <= j < ldk: 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void transpose_pad_kernel(const float* __restrict__ A,
                                                            float* __restrict__ AT, int N,
                                                            int64_t M, int ldk) {
  __shared__ float T[64][65];
  const int c = blockIdx.z;
  const float* Ac = A + (int64_t)c * N * M;
  float* ATc = AT + (int64_t)c * M * ldk;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int j = j0 + r;
    const int64_t p = p0 + tx;
    T[r][tx] = (j < N && p < M) ? Ac[(int64_t)j * M + p] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t p = p0 + r;
    const int j = j0 + tx;
    if (p < M && j < ldk) ATc[p * ldk + j] = T[tx][r];
  }
}

// Adjoint rotation on FP32 matrix cores (FP32 storage):
//   Out_c[i][p] = scale * sum_m w_m[p] sum_j X_m[i][j] Psi_c[j][p]
// over the 2 nx matrices X_m of channel c, staged as FP32 copies Xf
// [2 nx][nspin][N][ldk] (X1's then X2's), with Psi^T as AT [nspin][M][ldk].  The
// K-tiles of every matrix run through the same LDS ring; each K-tile's FP32
// products are added into the FP64 accumulators with the weight w_m of their
// output column.  The blocks (ib, J) that `active` marks inactive (blocks.h) are
// zero in every X_m and are skipped.  1-D grid over (point block, channel) groups
// of row blocks, the row blocks of one point block together on one XCD (they
// stage the same tiles of AT).
__global__ __launch_bounds__(PT, 1) void adj_psi_pipe_kernel(
    const float* __restrict__ Xf, const double* __restrict__ w1, const double* __restrict__ w2,
    int nx, const float* __restrict__ AT, int N, int64_t M, int ldk, int nspin, double scale,
    const unsigned char* __restrict__ active, const float* __restrict__ zeros,
    float* __restrict__ Out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pipe[];
  constexpr int SB = 2 * TB;
  const int nrb = (N + BT - 1) / BT;
  const int npb = (int)((M + BT - 1) / BT);
  int group, ib;
  xcd_map(blockIdx.x, npb * nspin, nrb, group, ib);
  const int pblk = group / nspin, c = group % nspin;
  const int i0 = ib * BT;
  const int64_t p0 = (int64_t)pblk * BT;
  const float* ATc = AT + (int64_t)c * M * ldk;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  // K runs over the active blocks J of row block ib (every J, X_m being a full product)
  uint64_t bits = 0;
  for (int J = 0; J < nrb; ++J)
    if (block_active(active, c, nrb, ib, J)) bits |= 1ull << J;
  const int nkm = active_ktiles(bits, N, KT);     // K-tiles per matrix
  const int nmat = 2 * nx;
  const int nk = nmat * nkm;
  auto issue = [&](int t) {
    unsigned char* st = smem_pipe + (t % NST) * SB;
    const int m = nkm > 0 ? min(t / nkm, nmat - 1) : 0;
    int J;
    const int64_t j0 = active_ktile(bits, nkm > 0 ? t % nkm : 0, KT, J);
    const int64_t je = t < nk ? ldk : j0;
    const float* Xm = Xf + ((int64_t)m * nspin + c) * N * ldk;
    dma_tile(Xm, ldk, N, i0, j0, je, zeros, st, wid, lane);
    dma_tile(ATc, ldk, (int)M, p0, j0, je, zeros, st + TB, wid, lane);
  };
  double acc[2][4][4];
  zero_pipe(acc);
  double wcol[4] = {0.0, 0.0, 0.0, 0.0};
  issue(0);
  issue(1);
  for (int t = 0; t < nk; ++t) {
    if (t % nkm == 0) {
      // the weights of matrix m for this wave's output columns
      const int m = t / nkm;
      const double* w = (m < nx ? w1 : w2) + ((int64_t)(m % nx) * nspin + c) * M;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
        wcol[j] = p < M ? w[p] : 0.0;
      }
    }
    wait_stage<4>();
    const unsigned char* st = smem_pipe + (t % NST) * SB;
    PipeFrag f;
    f.load(st, st + TB, wr, wc, lane);
    compiler_fence();
    issue(t + 2);
    f4 cc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) cc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cc[i][j] = mfma_f32(f.a[i][s], f.b[j][s], cc[i][j]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][j][v] += wcol[j] * (double)cc[i][j][v];
  }
  wait_stage<0>();
  float* Oc = Out + (int64_t)c * N * M;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = i0 + wr * 32 + i * 16 + 4 * (lane >> 4) + v;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
        if (gi < N && p < M) Oc[(int64_t)gi * M + p] = (float)(scale * acc[i][j][v]);
      }
    }
}

// ================================================================== pre-split BF16X3
// The exact three-piece split costs about as much VALU work as the six products,
// and inside the kernels every wave repeats it for the fragments it shares with
// other waves.  So the operands that carry no weight are split once per call
// into three BF16 planes (x = hi + mid + lo), and the kernels read the pieces:
// the back-projection reads pieces of both Gamma and Psi^T and splits nothing;
// the projection carries the weight on its A side (H'_ij = sum_p (w_p Psi_ip)
// Psi_jp), splits only that, and reads the pieces of Psi for B.
//
// A piece tile is 128 rows x 32 k of BF16 (64 bytes per row, four 16-byte
// chunks), the chunks of each row permuted by piece_swizzle below.
constexpr int PB = BT * KT * 2;           // bytes of one piece tile (8 KB)

// x -> three BF16 planes, rows of length ld: P[q][row][k] for q = hi, mid, lo.
__global__ void split3_kernel(const float* __restrict__ X, int64_t n, __bf16* __restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float r = X[i];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const __bf16 h = (__bf16)r;
    P[q * n + i] = h;
    r -= (float)h;
  }
}

// PT[c][q][p][j] = piece q of A[c][j][p] for j < N, 0 for N <= j < ldk.
__global__ __launch_bounds__(256) void transpose_split3_kernel(const float* __restrict__ A,
                                                              __bf16* __restrict__ PT, int N,
                                                              int64_t M, int ldk) {
  __shared__ float T[64][65];
  const int c = blockIdx.z;
  const float* Ac = A + (int64_t)c * N * M;
  const int64_t plane = M * ldk;
  __bf16* PTc = PT + (int64_t)c * 3 * plane;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int j = j0 + r;
    const int64_t p = p0 + tx;
    T[r][tx] = (j < N && p < M) ? Ac[(int64_t)j * M + p] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t p = p0 + r;
    const int j = j0 + tx;
    if (p < M && j < ldk) {
      float x = T[tx][r];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const __bf16 h = (__bf16)x;
        PTc[q * plane + p * ldk + j] = h;
        x -= (float)h;
      }
    }
  }
}

// G3[b][q][i][j] = piece q of (float)G[b][i][j] for j < N, 0 for N <= j < ldk;
// with upper2, entries of the blocks right of the diagonal block (j / 128 > i /
// 128) are doubled (exact: the pieces of 2x are twice the pieces of x).
__global__ void gamma_split3_kernel(const double* __restrict__ G, __bf16* __restrict__ G3, int N,
                                    int ldk, int batch, int upper2) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)N * ldk;
  if (idx >= (int64_t)batch * per) return;
  const int64_t b = idx / per, rem = idx - b * per;
  const int j = (int)(rem % ldk);
  const int64_t i = rem / ldk;
  float x = j < N ? (float)G[(b * N + i) * N + j] : 0.f;
  if (upper2 && j / BT > i / BT) x *= 2.f;
  __bf16* out = G3 + b * 3 * per + rem;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const __bf16 h = (__bf16)x;
    out[q * per] = h;
    x -= (float)h;
  }
}

// Slot permutation of the four 16-byte chunks of a piece row (64 bytes): chunk q
// of row r sits in slot q ^ piece_swizzle(r).  Rows r and r' that a fragment read
// serves in one pass then fall in distinct 16-byte bank groups, whether a pass
// covers 8 rows (128 bytes of banks) or 16 rows (256 bytes).
__device__ inline int piece_swizzle(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

// This wave's share (one of eight copy instructions, 16 rows each) of a piece
// tile: rows [r0, r0+BT) x k in [k0, k0+KT) of the row-major BF16 plane X
// (row length ld); chunks with row >= nrows or k >= kend (a multiple of 8) read
// zeros.
__device__ inline void dma_piece(const __bf16* __restrict__ X, int64_t ld, int64_t nrows,
                                 int64_t r0, int64_t k0, int64_t kend, const float* zeros,
                                 unsigned char* tile, int wid, int lane) {
  const int r = wid * 16 + (lane >> 2);
  const int q = (lane & 3) ^ piece_swizzle(r);
  const int64_t k = k0 + 8 * q;
  const int64_t gr = r0 + r;
  const void* src = (gr < nrows && k < kend) ? (const void*)(X + gr * ld + k) : (const void*)zeros;
  dma16(src, tile + wid * 1024);
}

// Lane fragment of rows base + 16 i + lane%16, k = 8(lane/16) .. +7 of a piece tile.
template <int NI>
__device__ inline void frag_piece(const unsigned char* tile, int base, int lane, bf8 (&v)[NI]) {
  const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int R = base + 16 * i + r16;
    v[i] = *reinterpret_cast<const bf8*>(tile + R * 64 + ((g ^ piece_swizzle(R)) * 16));
  }
}

// The six products of order <= 2, smallest first.
__device__ inline f4 mfma6(const bf8 (&a)[3], const bf8 (&b)[3], f4 c) {
  c = mfma_bf16(a[0], b[2], c);
  c = mfma_bf16(a[1], b[1], c);
  c = mfma_bf16(a[2], b[0], c);
  c = mfma_bf16(a[0], b[1], c);
  c = mfma_bf16(a[1], b[0], c);
  return mfma_bf16(a[0], b[0], c);
}

// Adjoint rotation in the BF16X3 form: adj_psi_pipe_kernel's product with both
// operands pre-split into three BF16 pieces, X3 [2 nx][nspin][3][N][ldk] (the
// FP32 rounding of each X_m, split) and PT3 [nspin][3][M][ldk] (Psi^T, split).
// Each K-tile's six products of order <= 2 accumulate in FP32 and are added
// into the FP64 accumulators with the weight w_m of their output column.
__global__ __launch_bounds__(PT, 1) void adj_psi_p3_kernel(
    const __bf16* __restrict__ X3, const double* __restrict__ w1, const double* __restrict__ w2,
    int nx, const __bf16* __restrict__ PT3, int N, int64_t M, int ldk, int nspin, double scale,
    const unsigned char* __restrict__ active, const float* __restrict__ zeros,
    float* __restrict__ Out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pipe[];
  constexpr int SB = 6 * PB;
  const int nrb = (N + BT - 1) / BT;
  const int npb = (int)((M + BT - 1) / BT);
  int group, ib;
  xcd_map(blockIdx.x, npb * nspin, nrb, group, ib);
  const int pblk = group / nspin, c = group % nspin;
  const int i0 = ib * BT;
  const int64_t p0 = (int64_t)pblk * BT;
  const int64_t gplane = (int64_t)N * ldk, pplane = M * ldk;
  const __bf16* Pc = PT3 + (int64_t)c * 3 * pplane;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  uint64_t bits = 0;
  for (int J = 0; J < nrb; ++J)
    if (block_active(active, c, nrb, ib, J)) bits |= 1ull << J;
  const int nkm = active_ktiles(bits, N, KT);     // K-tiles per matrix
  const int nmat = 2 * nx;
  const int nk = nmat * nkm;
  auto issue = [&](int t) {
    unsigned char* st = smem_pipe + (t % NST) * SB;
    const int m = nkm > 0 ? min(t / nkm, nmat - 1) : 0;
    int J;
    const int64_t j0 = active_ktile(bits, nkm > 0 ? t % nkm : 0, KT, J);
    const int64_t je = t < nk ? ldk : j0;
    const __bf16* Xm = X3 + ((int64_t)m * nspin + c) * 3 * gplane;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dma_piece(Xm + q * gplane, ldk, N, i0, j0, je, zeros, st + q * PB, wid, lane);
      dma_piece(Pc + q * pplane, ldk, M, p0, j0, je, zeros, st + (3 + q) * PB, wid, lane);
    }
  };
  double acc[2][4][4];
  zero_pipe(acc);
  double wcol[4] = {0.0, 0.0, 0.0, 0.0};
  issue(0);
  issue(1);
  for (int t = 0; t < nk; ++t) {
    if (t % nkm == 0) {
      // the weights of matrix m for this wave's output columns
      const int m = t / nkm;
      const double* w = (m < nx ? w1 : w2) + ((int64_t)(m % nx) * nspin + c) * M;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
        wcol[j] = p < M ? w[p] : 0.0;
      }
    }
    wait_stage<6>();
    const unsigned char* st = smem_pipe + (t % NST) * SB;
    bf8 pa[2][3], pb[4][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      bf8 va[2], vb[4];
      frag_piece<2>(st + q * PB, wr * 32, lane, va);
      frag_piece<4>(st + (3 + q) * PB, wc * 64, lane, vb);
#pragma unroll
      for (int i = 0; i < 2; ++i) pa[i][q] = va[i];
#pragma unroll
      for (int j = 0; j < 4; ++j) pb[j][q] = vb[j];
    }
    compiler_fence();
    issue(t + 2);
    f4 cc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) cc[i][j] = mfma6(pa[i], pb[j], f4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][j][v] += wcol[j] * (double)cc[i][j][v];
  }
  wait_stage<0>();
  float* Oc = Out + (int64_t)c * N * M;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = i0 + wr * 32 + i * 16 + 4 * (lane >> 4) + v;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
        if (gi < N && p < M) Oc[(int64_t)gi * M + p] = (float)(scale * acc[i][j][v]);
      }
    }
}

// Projection, BF16X3, pre-split B: H[b] = (w o A_c) B_c^T with A = B = Psi; A
// FP32 tiles weighted and split in the kernel, B from the pieces P3
// [nspin][3][N][M].  Same grid and partial layout as tn_sym_pipe_kernel; M a
// multiple of 8, aligned rows.
__global__ __launch_bounds__(PT, 1) void tn_sym_p3_kernel(
    const float* __restrict__ A, const __bf16* __restrict__ P3, const double* __restrict__ w,
    int64_t w_stride, int N, int64_t M, int nspin, int ntb, int64_t kchunk, int nsplit, int batch,
    const unsigned char* __restrict__ active, const float* __restrict__ zeros,
    double* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pipe[];
  constexpr int SB = TB + 3 * PB + 1024;   // A (FP32), B pieces, weights
  const int ntiles = ntb * (ntb + 1) / 2;
  // the directions of one (split, tile) run together on one XCD: they stage the
  // same operand tiles (only the weights differ), so L2 serves all but the first
  int group, b;
  xcd_map(blockIdx.x, nsplit * ntiles, batch, group, b);
  const int sp = group / ntiles, tile = group % ntiles;
  int ti = 0, rem = tile;
  while (rem >= ntb - ti) { rem -= ntb - ti; ++ti; }
  const int tj = ti + rem;
  const int c = b % nspin;
  const float* Ac = A + (int64_t)c * N * M;
  const __bf16* Pc = P3 + (int64_t)c * 3 * N * M;
  const double* wb = w + (int64_t)b * w_stride;
  const int64_t kbeg = (int64_t)sp * kchunk;
  // an inactive block (blocks.h) keeps a zero partial tile
  const int64_t kend = block_active(active, c, ntb, ti, tj) ? min(M, kbeg + kchunk) : kbeg;
  const int nk = kbeg < kend ? (int)((kend - kbeg + KT - 1) / KT) : 0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  // Per-lane source addresses of a full K-tile (k0 + KT <= kend) are base + k0:
  // the copy slots of dma_tile / dma_piece with rows past N reading row N - 1
  // instead of zeros (their products land in rows or columns of the partial
  // tile the reduction never reads), so the loop spends one address add per
  // copy.  The last, partial K-tile takes the checked copies.
  const float* abase[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int r = (wid * 2 + u) * 8 + (lane >> 3);
    const int q = (lane & 7) ^ tile_swizzle(r);
    abase[u] = Ac + (int64_t)min(ti * BT + r, N - 1) * M + 4 * q;
  }
  const __bf16* pbase;
  {
    const int r = wid * 16 + (lane >> 2);
    const int q = (lane & 3) ^ piece_swizzle(r);
    pbase = Pc + (int64_t)min(tj * BT + r, N - 1) * M + 8 * q;
  }
  const double* wbase = wb + 2 * (lane & 15);
  // copies per stage and wave: 2 (A) + 3 (pieces of B), plus the weights in wave 0
  auto issue = [&](int t) {
    unsigned char* st = smem_pipe + (t % NST) * SB;
    const int64_t k0 = kbeg + (int64_t)t * KT;
    if (t < nk && k0 + KT <= kend) {
#pragma unroll
      for (int u = 0; u < 2; ++u) dma16(abase[u] + k0, st + (wid * 2 + u) * 1024);
#pragma unroll
      for (int q = 0; q < 3; ++q)
        dma16(pbase + (int64_t)q * N * M + k0, st + TB + q * PB + wid * 1024);
      if (wid == 0) dma16(wbase + k0, st + TB + 3 * PB);
      return;
    }
    const int64_t ke = t < nk ? kend : k0;
    dma_tile(Ac, M, N, (int64_t)ti * BT, k0, ke, zeros, st, wid, lane);
#pragma unroll
    for (int q = 0; q < 3; ++q)
      dma_piece(Pc + (int64_t)q * N * M, M, N, (int64_t)tj * BT, k0, ke, zeros,
                st + TB + q * PB, wid, lane);
    if (wid == 0) dma_weights(wb, k0, ke, zeros, st + TB + 3 * PB, lane);
  };
  double acc[2][4][4];
  zero_pipe(acc);
  f4 cc[2][4];
  zero_f32(cc);
  issue(0);
  issue(1);
  for (int t0 = 0; t0 < nk; t0 += kFlush) {
    const int t1 = min(nk, t0 + kFlush);
    for (int t = t0; t < t1; ++t) {
      if (wid == 0) wait_stage<6>(); else wait_stage<5>();
      const unsigned char* st = smem_pipe + (t % NST) * SB;
      float a[2][8];
      frag_sw<2>(st, wr * 32, lane, a);
      bf8 pb[4][3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        bf8 v[4];
        frag_piece<4>(st + TB + q * PB, wc * 64, lane, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) pb[j][q] = v[j];
      }
      float wf[8];
      {
        const int g = lane >> 4;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const f4 x = *reinterpret_cast<const f4*>(st + TB + 3 * PB + (4 * g + h) * 16);
          const d2v y = __builtin_bit_cast(d2v, x);
          wf[2 * h] = (float)y[0];
          wf[2 * h + 1] = (float)y[1];
        }
      }
      compiler_fence();
      issue(t + 2);
      bf8 pa[2][3];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int e = 0; e < 8; ++e) a[i][e] *= wf[e];
        split3_rne(a[i], pa[i]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cc[i][j] = mfma6(pa[i], pb[j], cc[i][j]);
      }
      flush_pipe(cc, 1.0, acc);
    }
  wait_stage<0>();
  double* out = part + (((int64_t)b * nsplit + sp) * ntiles + tile) * (BT * BT);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 32 + i * 16 + 4 * (lane >> 4) + v;
        const int col = wc * 64 + j * 16 + (lane & 15);
        out[row * BT + col] = acc[i][j][v];
      }
}

// Back-projection, BF16X3, both operands pre-split: G3 [batch][3][N][ldk] (FP32
// rounding of Gamma, split), PT3 [nspin][3][M][ldk] (Psi^T split).  Otherwise as
// backproj_pipe_kernel.
__global__ __launch_bounds__(PT, 1) void backproj_p3_kernel(
    const float* __restrict__ A, const __bf16* __restrict__ PT3, const __bf16* __restrict__ G3,
    int N, int64_t M, int ldk, int nspin, int batch, double scale, const double* __restrict__ sub,
    const unsigned char* __restrict__ active, const float* __restrict__ zeros,
    double* __restrict__ out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pipe[];
  constexpr int SB = 6 * PB;
  double* red = reinterpret_cast<double*>(smem_pipe + NST * SB);   // [PW][64]
  // the directions of one block of points run together on one XCD: they stage
  // the same tiles of the Psi^T pieces (each direction's Gamma, 6 MB at N = 1024,
  // is re-read from the last-level cache)
  int pblk, b;
  xcd_map(blockIdx.x, (int)((M + BT - 1) / BT), batch, pblk, b);
  const int c = b % nspin;
  const float* Ac = A + (int64_t)c * N * M;
  const int64_t gplane = (int64_t)N * ldk, pplane = M * ldk;
  const __bf16* Gb = G3 + (int64_t)b * 3 * gplane;
  const __bf16* Pb = PT3 + (int64_t)c * 3 * pplane;
  const int64_t p0 = (int64_t)pblk * BT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  double dsum[4] = {0.0, 0.0, 0.0, 0.0};
  const int nib = (N + BT - 1) / BT;
  for (int ib = 0; ib < nib; ++ib) {
    const int i0 = ib * BT;
    // j runs over the active blocks (blocks.h) of [i0, N), kFlush K-tiles each
    const uint64_t bits = active_row_bits(active, c, nib, ib);
    const int nk = active_ktiles(bits, N, KT);
    if (nk == 0) continue;
    auto issue = [&](int t) {
      unsigned char* st = smem_pipe + (t % NST) * SB;
      int J;
      const int64_t j0 = active_ktile(bits, t, KT, J);
      const int64_t je = t < nk ? ldk : j0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        dma_piece(Gb + q * gplane, ldk, N, i0, j0, je, zeros, st + q * PB, wid, lane);
        dma_piece(Pb + q * pplane, ldk, M, p0, j0, je, zeros, st + (3 + q) * PB, wid, lane);
      }
    };
    double acc[2][4][4];
    zero_pipe(acc);
    f4 cc[2][4];
    zero_f32(cc);
    issue(0);
    issue(1);
    for (int t0 = 0; t0 < nk; t0 += kFlush) {
      const int t1 = min(nk, t0 + kFlush);
      for (int t = t0; t < t1; ++t) {
        wait_stage<6>();
        const unsigned char* st = smem_pipe + (t % NST) * SB;
        bf8 pa[2][3], pb[4][3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          bf8 va[2], vb[4];
          frag_piece<2>(st + q * PB, wr * 32, lane, va);
          frag_piece<4>(st + (3 + q) * PB, wc * 64, lane, vb);
#pragma unroll
          for (int i = 0; i < 2; ++i) pa[i][q] = va[i];
#pragma unroll
          for (int j = 0; j < 4; ++j) pb[j][q] = vb[j];
        }
        compiler_fence();
        issue(t + 2);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) cc[i][j] = mfma6(pa[i], pb[j], cc[i][j]);
      }
      // a flush group of kFlush K-tiles (kFlush KT = BT) is one block, on or off
      // the diagonal
      int J;
      active_ktile(bits, t0, KT, J);
      flush_pipe(cc, J > ib ? 2.0 : 1.0, acc);
    }
    wait_stage<0>();
    float av[2][4][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = min(i0 + wr * 32 + i * 16 + 4 * (lane >> 4) + v, N - 1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t p = min(p0 + wc * 64 + j * 16 + (lane & 15), M - 1);
          av[i][v][j] = Ac[(int64_t)gi * M + p];
        }
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wr * 32 + i * 16 + 4 * (lane >> 4) + v;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
          if (gi < N && p < M) dsum[j] += acc[i][j][v] * (double)av[i][v][j];
        }
      }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double v = dsum[j];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    dsum[j] = v;
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wid * 64 + j * 16 + lane] = dsum[j];
  }
  __syncthreads();
  if (threadIdx.x < BT) {
    const int col = threadIdx.x;
    const int wcc = col >> 6, cl = col & 63;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) v += red[(2 * q + wcc) * 64 + cl];
    const int64_t p = p0 + col;
    if (p < M) {
      double r = scale * v;
      if (sub) r -= sub[(int64_t)b * M + p];
      out[(int64_t)b * M + p] = r;
    }
  }
}

// Back-projection, BF16X3, wide point tiles: as backproj_p3_kernel, but each
// workgroup owns 256 grid points (twice the points per staged Gamma tile, so
// each direction's Gamma pieces are read half as often) and each of its eight
// waves a 64 x 64 part (rows of Gamma x points), so every LDS fragment feeds
// four matrix products instead of two.  Gamma's pieces come with the blocks
// right of the diagonal doubled (gamma_split3_kernel, upper2), so a row block's
// products accumulate in FP32 over all its active blocks and meet Psi once, in
// FP64, at the end of the row block.  Two ring stages (72 KB each); the first
// K-tile of the next active row block is in flight while the current one's
// products are folded with Psi.
constexpr int BPW = 2 * BT;               // points per workgroup
constexpr int SBW = 9 * PB;               // one stage: 3 Gamma pieces, 3 x 2 Psi^T pieces

__global__ __launch_bounds__(PT, 1) void backproj_p3w_kernel(
    const float* __restrict__ A, const __bf16* __restrict__ PT3, const __bf16* __restrict__ G3,
    int N, int64_t M, int ldk, int nspin, int batch, double scale, const double* __restrict__ sub,
    const unsigned char* __restrict__ active, double* __restrict__ out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pipe[];
  double* red = reinterpret_cast<double*>(smem_pipe + 2 * SBW);   // [PW][64]
  int pblk, b;
  xcd_map(blockIdx.x, (int)((M + BPW - 1) / BPW), batch, pblk, b);
  const int c = b % nspin;
  const float* Ac = A + (int64_t)c * N * M;
  const int64_t gplane = (int64_t)N * ldk, pplane = M * ldk;
  const __bf16* Gb = G3 + (int64_t)b * 3 * gplane;
  const __bf16* Pb = PT3 + (int64_t)c * 3 * pplane;
  const int64_t p0 = (int64_t)pblk * BPW;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 2, wc = wid & 3;          // rows wr*64.., points wc*64..
  const int nib = (N + BT - 1) / BT;
  // next row block at or after ib with active K-tiles (nib when none)
  auto next_row = [&](int ib, uint64_t& bits, int& nk) {
    for (; ib < nib; ++ib) {
      bits = active_row_bits(active, c, nib, ib);
      nk = active_ktiles(bits, N, KT);
      if (nk > 0) return ib;
    }
    return nib;
  };
  // This lane's copy slot of a piece tile (dma_piece): row wid * 16 + lane / 4,
  // 16-byte chunk q; every K-tile lies inside [0, ldk), and rows past N (Gamma)
  // or M (Psi^T) read the last row instead of zeros (their products land in rows
  // or points that fold() masks), so a copy's address is base + j0.
  const int slot_r = wid * 16 + (lane >> 2);
  const int slot_k = 8 * ((lane & 3) ^ piece_swizzle(slot_r));
  const __bf16* pbase[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
    pbase[h] = Pb + min(p0 + h * BT + slot_r, M - 1) * ldk + slot_k;
  // K-tile t of row block ib into ring stage s
  auto issue = [&](int ib, uint64_t bits, int t, int s) {
    unsigned char* st = smem_pipe + s * SBW;
    int J;
    const int64_t j0 = active_ktile(bits, t, KT, J);
    const __bf16* gbase = Gb + (int64_t)min(ib * BT + slot_r, N - 1) * ldk + slot_k + j0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dma16(gbase + q * gplane, st + q * PB + wid * 1024);
#pragma unroll
      for (int h = 0; h < 2; ++h)
        dma16(pbase[h] + q * pplane + j0, st + (3 + 2 * q + h) * PB + wid * 1024);
    }
  };
  double dsum[4] = {0.0, 0.0, 0.0, 0.0};
  uint64_t bits = 0;
  int nk = 0;
  int ib = next_row(0, bits, nk);
  int s = 0;                                      // ring stage of the next K-tile
  if (ib < nib) issue(ib, bits, 0, s);
  while (ib < nib) {
    uint64_t nbits = 0;
    int nnk = 0;
    const int nib2 = next_row(ib + 1, nbits, nnk);
    f4 cc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) cc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < nk; ++t) {
      // this stage's copies have landed for every wave, and every wave has read
      // the other stage (its previous K-tile) into registers
      wait_stage<0>();
      const unsigned char* st = smem_pipe + s * SBW;
      bf8 pa[4][3], pb[4][3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        bf8 va[4], vb[4];
        frag_piece<4>(st + q * PB, wr * 64, lane, va);
        frag_piece<4>(st + (3 + 2 * q + (wc >> 1)) * PB, (wc & 1) * 64, lane, vb);
#pragma unroll
        for (int i = 0; i < 4; ++i) pa[i][q] = va[i];
#pragma unroll
        for (int j = 0; j < 4; ++j) pb[j][q] = vb[j];
      }
      compiler_fence();
      s ^= 1;
      if (t + 1 < nk)
        issue(ib, bits, t + 1, s);
      else if (nib2 < nib)
        issue(nib2, nbits, 0, s);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cc[i][j] = mfma6(pa[i], pb[j], cc[i][j]);
    }
    // fold the row block's products with Psi: sum_i Psi_ip (Gamma Psi)_ip
    const int i0 = ib * BT;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wr * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int gic = min(gi, N - 1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
          const float a = Ac[(int64_t)gic * M + min(p, M - 1)];
          if (gi < N && p < M) dsum[j] += (double)cc[i][j][v] * (double)a;
        }
      }
    ib = nib2;
    bits = nbits;
    nk = nnk;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double v = dsum[j];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    dsum[j] = v;
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wid * 64 + j * 16 + lane] = dsum[j];
  }
  __syncthreads();
  if (threadIdx.x < BPW) {
    const int col = threadIdx.x;
    const int wcc = col >> 6, cl = col & 63;
    const double v = red[wcc * 64 + cl] + red[(4 + wcc) * 64 + cl];
    const int64_t p = p0 + col;
    if (p < M) {
      double r = scale * v;
      if (sub) r -= sub[(int64_t)b * M + p];
      out[(int64_t)b * M + p] = r;
    }
  }
}

}  // namespace

// Rotation, BF16X3: Out[i][p] = sum_j Wt[j][i] B[j][p] over j < N, or j below the
// end of row block i when `upper` (Wt upper triangular: the blocks past the
// diagonal block are zero), with both operands pre-split: W3 [3][N][ldk] (FP32
// rounding of Wt^T, split) and BT3 [3][M][ldk] (B^T split).  One block per
// (row block of 128, point block of 128); the row blocks of one point block run
// together on one XCD, where they share the staged tiles of BT3.  FP32 partials
// over kFlush K-tiles are added into FP64 accumulators; FP32 output.
__global__ __launch_bounds__(PT, 1) void rotate_p3_kernel(
    const __bf16* __restrict__ W3, const __bf16* __restrict__ BT3, int N, int64_t M, int ldk,
    int upper, const float* __restrict__ zeros, float* __restrict__ out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_pipe[];
  constexpr int SB = 6 * PB;
  const int nib = (N + BT - 1) / BT;
  int pblk, ib;
  xcd_map(blockIdx.x, (int)((M + BT - 1) / BT), nib, pblk, ib);
  const int64_t wplane = (int64_t)N * ldk, pplane = M * ldk;
  const int64_t p0 = (int64_t)pblk * BT;
  const int i0 = ib * BT;
  const int kmax = upper ? min(ldk, i0 + BT) : ldk;
  const int nk = (kmax + KT - 1) / KT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  auto issue = [&](int t) {
    unsigned char* st = smem_pipe + (t % NST) * SB;
    const int64_t j0 = (int64_t)t * KT;
    const int64_t je = t < nk ? kmax : j0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dma_piece(W3 + q * wplane, ldk, N, i0, j0, je, zeros, st + q * PB, wid, lane);
      dma_piece(BT3 + q * pplane, ldk, M, p0, j0, je, zeros, st + (3 + q) * PB, wid, lane);
    }
  };
  double acc[2][4][4];
  zero_pipe(acc);
  f4 cc[2][4];
  zero_f32(cc);
  issue(0);
  issue(1);
  for (int t0 = 0; t0 < nk; t0 += kFlush) {
    const int t1 = min(nk, t0 + kFlush);
    for (int t = t0; t < t1; ++t) {
      wait_stage<6>();
      const unsigned char* st = smem_pipe + (t % NST) * SB;
      bf8 pa[2][3], pb[4][3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        bf8 va[2], vb[4];
        frag_piece<2>(st + q * PB, wr * 32, lane, va);
        frag_piece<4>(st + (3 + q) * PB, wc * 64, lane, vb);
#pragma unroll
        for (int i = 0; i < 2; ++i) pa[i][q] = va[i];
#pragma unroll
        for (int j = 0; j < 4; ++j) pb[j][q] = vb[j];
      }
      compiler_fence();
      issue(t + 2);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cc[i][j] = mfma6(pa[i], pb[j], cc[i][j]);
    }
    flush_pipe(cc, 1.0, acc);
  }
  wait_stage<0>();
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = i0 + wr * 32 + i * 16 + 4 * (lane >> 4) + v;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t p = p0 + wc * 64 + j * 16 + (lane & 15);
        if (gi < N && p < M) out[(int64_t)gi * M + p] = (float)acc[i][j][v];
      }
    }
}

// W3[q][i][j] = piece q of (float)Wt[j][i] for j < N, 0 for N <= j < ldk.
__global__ void wt_split3_kernel(const double* __restrict__ Wt, __bf16* __restrict__ W3, int N,
                                 int ldk) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)N * ldk;
  if (idx >= per) return;
  const int j = (int)(idx % ldk);
  const int64_t i = idx / ldk;
  float x = j < N ? (float)Wt[(int64_t)j * N + i] : 0.f;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const __bf16 h = (__bf16)x;
    W3[q * per + idx] = h;
    x -= (float)h;
  }
}

static int pad_k(int N) { return (N + KT - 1) / KT * KT; }

size_t backproj_workspace_bytes(int N, int64_t M, int nspin, int batch, lrdm_prec prec) {
  if (prec == LRDM_FP64) return 0;
  const size_t ldk = pad_k(N);
  const size_t el = (prec == LRDM_BF16X3) ? 3 * sizeof(__bf16) : sizeof(float);
  return ws_align((size_t)batch * N * ldk * el) + ws_align((size_t)nspin * M * ldk * el);
}

// Pieces of Psi for the pre-split projection (nspin <= 2).
size_t tn_split_bytes(int N, int64_t M, lrdm_prec prec) {
  return prec == LRDM_BF16X3 ? ws_align((size_t)2 * 3 * N * M * sizeof(__bf16)) : 0;
}

template <>
hipError_t launch_tn_sym<float>(lrdm_ctx* ctx, const float* A, const float* B, const double* w,
                                int64_t w_stride, int N, int64_t M, int nspin, int batch,
                                lrdm_prec prec, double* H, const unsigned char* active) {
  if (prec == LRDM_FP64)
    return launch_tn_sym_f64<float, float>(ctx, A, B, w, w_stride, N, M, nspin, batch, H, active);
  const int ntb = (N + BT - 1) / BT;
  const int ntiles = ntb * (ntb + 1) / 2;
  const int ns = tn_split_count(ctx, N, M, batch,
                                prec == LRDM_BF16X3 ? TN_ARITH_BF16X3 : TN_ARITH_F32, w != nullptr);
  int64_t kchunk = (M + ns - 1) / ns;
  kchunk = (kchunk + KT - 1) / KT * KT;
  double* part = static_cast<double*>(ws_take(ctx, tn_part_bytes(N, M, batch, ctx->split_limit)));
  if (!B) B = A;
  auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  // the pipelined kernel copies 16-byte chunks of rows: rows must start aligned
  const bool pipe = (M % 4 == 0) && a16(A) && a16(B) && (!w || (a16(w) && w_stride % 2 == 0));
  const unsigned grd = (unsigned)(ntiles * ns * batch);
  // the tile and wave layout lrdm_autotune chose for this shape (default otherwise)
  const int variant = tn_variant(ctx, N, M, batch,
                                 prec == LRDM_BF16X3 ? TN_ARITH_BF16X3 : TN_ARITH_F32,
                                 w != nullptr);
  if (variant == TN_VAR_DEFAULT && pipe && w && B == A && prec == LRDM_BF16X3 && M % 8 == 0 &&
      nspin <= 2) {
    // pieces of Psi once per call (or those the context holds for this block), then
    // the weighted A side split in the kernel
    const lrdm_psi_pieces& pc = ctx->pieces;
    const __bf16* P3 = nullptr;
    if (pc.psi == A && pc.p3 && pc.N == N && pc.M == M && pc.nspin == nspin) {
      P3 = static_cast<const __bf16*>(pc.p3);
    } else {
      __bf16* P = static_cast<__bf16*>(ws_take(ctx, tn_split_bytes(N, M, prec)));
      const int64_t n = (int64_t)N * M;
      for (int c = 0; c < nspin; ++c) {
        split3_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(A + c * n, n,
                                                                            P + c * 3 * n);
        LRDM_HIP(hipGetLastError());
      }
      P3 = P;
    }
    const int smem = NST * (TB + 3 * PB + 1024);
    LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tn_sym_p3_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, smem));
    {
      ProfScope prof(ctx, "proj");
      tn_sym_p3_kernel<<<grd, PT, smem, ctx->stream>>>(A, P3, w, w_stride, N, M, nspin, ntb,
                                                       kchunk, ns, batch, active, ctx->zeros,
                                                       part);
      LRDM_HIP(hipGetLastError());
    }
    dim3 blk(32, 8);
    dim3 grd2((N + 31) / 32, (N + 7) / 8, batch);
    tn_reduce_lp_kernel<<<grd2, blk, 0, ctx->stream>>>(part, N, ntb, ns, H);
    return hipGetLastError();
  }
  const int smem = NST * (2 * TB + (w ? 1024 : 0));
  auto run_pipe = [&](auto kernel) -> hipError_t {
    LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, smem));
    kernel<<<grd, PT, smem, ctx->stream>>>(A, B, w, w_stride, N, M, nspin, ntb, kchunk, ns, batch,
                                           active, ctx->zeros, part);
    return hipGetLastError();
  };
  auto run_staged = [&](auto kernel) -> hipError_t {
    kernel<<<grd, 256, 0, ctx->stream>>>(A, B, w, w_stride, N, M, nspin, ntb, kchunk, ns, batch,
                                         active, part);
    return hipGetLastError();
  };
  {
    ProfScope prof(ctx, w ? "proj" : "gram");
    const bool bf = (prec == LRDM_BF16X3);
    if (variant == TN_VAR_STAGED || !pipe)
      LRDM_HIP(bf ? run_staged(tn_sym_lp_kernel<Core::BF3>) : run_staged(tn_sym_lp_kernel<Core::F32>));
    else if (w)
      LRDM_HIP(bf ? run_pipe(tn_sym_pipe_kernel<Core::BF3, true>)
                  : run_pipe(tn_sym_pipe_kernel<Core::F32, true>));
    else
      LRDM_HIP(bf ? run_pipe(tn_sym_pipe_kernel<Core::BF3, false>)
                  : run_pipe(tn_sym_pipe_kernel<Core::F32, false>));
  }
  dim3 blk(32, 8);
  dim3 grd2((N + 31) / 32, (N + 7) / 8, batch);
  tn_reduce_lp_kernel<<<grd2, blk, 0, ctx->stream>>>(part, N, ntb, ns, H);
  return hipGetLastError();
}

template <>
hipError_t launch_backproj<float>(lrdm_ctx* ctx, const float* A, const double* G, int N,
                                  int64_t M, int nspin, int batch, lrdm_prec prec, double scale,
                                  const double* sub, double* out, const unsigned char* active) {
  const int ldk = pad_k(N);
  const unsigned grd = (unsigned)((M + BT - 1) / BT * batch);
  dim3 gt((unsigned)((M + 63) / 64), (unsigned)(ldk / 64 + (ldk % 64 ? 1 : 0)), nspin);
  if (prec == LRDM_BF16X3) {
    const int64_t nG = (int64_t)batch * N * ldk;
    __bf16* G3 = static_cast<__bf16*>(ws_take(ctx, (size_t)nG * 3 * sizeof(__bf16)));
    const bool wide = ctx->bp_variant == BP_VAR_WIDE;   // Gamma's upper blocks doubled
    gamma_split3_kernel<<<(unsigned)((nG + 255) / 256), 256, 0, ctx->stream>>>(G, G3, N, ldk,
                                                                              batch, wide);
    LRDM_HIP(hipGetLastError());
    const lrdm_psi_pieces& pc = ctx->pieces;
    const __bf16* PT3 = nullptr;
    if (pc.psi == A && pc.pt3 && pc.N == N && pc.M == M && pc.nspin == nspin) {
      PT3 = static_cast<const __bf16*>(pc.pt3);
    } else {
      __bf16* P = static_cast<__bf16*>(
          ws_take(ctx, (size_t)nspin * M * ldk * 3 * sizeof(__bf16)));
      transpose_split3_kernel<<<gt, 256, 0, ctx->stream>>>(A, P, N, M, ldk);
      LRDM_HIP(hipGetLastError());
      PT3 = P;
    }
    if (wide) {
      const int smem = 2 * SBW + PW * 64 * (int)sizeof(double);
      LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&backproj_p3w_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, smem));
      const unsigned grdw = (unsigned)((M + BPW - 1) / BPW * batch);
      ProfScope prof(ctx, "backproj");
      backproj_p3w_kernel<<<grdw, PT, smem, ctx->stream>>>(A, PT3, G3, N, M, ldk, nspin, batch,
                                                           scale, sub, active, out);
      return hipGetLastError();
    }
    const int smem = NST * 6 * PB + PW * 64 * (int)sizeof(double);
    LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&backproj_p3_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, smem));
    ProfScope prof(ctx, "backproj");
    backproj_p3_kernel<<<grd, PT, smem, ctx->stream>>>(A, PT3, G3, N, M, ldk, nspin, batch, scale,
                                                       sub, active, ctx->zeros, out);
    return hipGetLastError();
  }
  float* Gf = static_cast<float*>(ws_take(ctx, (size_t)batch * N * ldk * sizeof(float)));
  float* AT = static_cast<float*>(ws_take(ctx, (size_t)nspin * M * ldk * sizeof(float)));
  const int64_t nG = (int64_t)batch * N * ldk;
  gamma_pad_kernel<<<(unsigned)((nG + 255) / 256), 256, 0, ctx->stream>>>(G, Gf, N, ldk, batch);
  LRDM_HIP(hipGetLastError());
  transpose_pad_kernel<<<gt, 256, 0, ctx->stream>>>(A, AT, N, M, ldk);
  LRDM_HIP(hipGetLastError());
  const int smem = NST * 2 * TB + PW * 64 * (int)sizeof(double);
  LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&backproj_pipe_kernel<Core::F32>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, smem));
  ProfScope prof(ctx, "backproj");
  backproj_pipe_kernel<Core::F32><<<grd, PT, smem, ctx->stream>>>(
      A, AT, Gf, N, M, ldk, nspin, batch, scale, sub, active, ctx->zeros, out);
  return hipGetLastError();
}

size_t rotate_bf16x3_bytes(int N, int64_t M) {
  const int ldk = pad_k(N);
  return ws_align((size_t)3 * N * ldk * sizeof(__bf16)) +
         ws_align((size_t)3 * M * ldk * sizeof(__bf16));
}

hipError_t launch_rotate_bf16x3(lrdm_ctx* ctx, const double* Wt, const float* B, float* Out,
                                int N, int64_t M, bool upper) {
  const int ldk = pad_k(N);
  __bf16* W3 = static_cast<__bf16*>(ws_take(ctx, (size_t)3 * N * ldk * sizeof(__bf16)));
  __bf16* BT3 = static_cast<__bf16*>(ws_take(ctx, (size_t)3 * M * ldk * sizeof(__bf16)));
  ProfScope prof(ctx, "nn");
  const int64_t nW = (int64_t)N * ldk;
  wt_split3_kernel<<<(unsigned)((nW + 255) / 256), 256, 0, ctx->stream>>>(Wt, W3, N, ldk);
  LRDM_HIP(hipGetLastError());
  dim3 gt((unsigned)((M + 63) / 64), (unsigned)(ldk / 64 + (ldk % 64 ? 1 : 0)), 1);
  transpose_split3_kernel<<<gt, 256, 0, ctx->stream>>>(B, BT3, N, M, ldk);
  LRDM_HIP(hipGetLastError());
  const int smem = NST * 6 * PB;
  LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&rotate_p3_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, smem));
  const unsigned grd = (unsigned)((M + BT - 1) / BT * ((N + BT - 1) / BT));
  rotate_p3_kernel<<<grd, PT, smem, ctx->stream>>>(W3, BT3, N, M, ldk, upper ? 1 : 0, ctx->zeros,
                                                   Out);
  return hipGetLastError();
}

size_t psi_pieces_p3_bytes(int N, int64_t M, int nspin) {
  return ws_align((size_t)nspin * 3 * N * M * sizeof(__bf16));
}

size_t psi_pieces_pt3_bytes(int N, int64_t M, int nspin) {
  return ws_align((size_t)nspin * 3 * M * pad_k(N) * sizeof(__bf16));
}

hipError_t launch_psi_pieces(lrdm_ctx* ctx, const float* Psi, int N, int64_t M, int nspin,
                             void* p3, void* pt3) {
  const int ldk = pad_k(N);
  const int64_t n = (int64_t)N * M;
  __bf16* P3 = static_cast<__bf16*>(p3);
  for (int c = 0; c < nspin; ++c) {
    split3_kernel<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(Psi + c * n, n,
                                                                        P3 + c * 3 * n);
    LRDM_HIP(hipGetLastError());
  }
  dim3 gt((unsigned)((M + 63) / 64), (unsigned)(ldk / 64 + (ldk % 64 ? 1 : 0)), nspin);
  transpose_split3_kernel<<<gt, 256, 0, ctx->stream>>>(Psi, static_cast<__bf16*>(pt3), N, M, ldk);
  return hipGetLastError();
}

// Adjoint rotation for FP32 storage: FP32 copies of the 2 nx matrices and Psi^T,
// then adj_psi_pipe_kernel.
template <>
hipError_t launch_adj_psi<float>(lrdm_ctx* ctx, const double* X1, const double* w1,
                                 const double* X2, const double* w2, int nx, const float* Psi,
                                 int N, int64_t M, int nspin, double scale, float* Out,
                                 const unsigned char* active) {
  const int ldk = pad_k(N);
  const int64_t nX = (int64_t)nx * nspin * N * ldk;
  float* Xf = static_cast<float*>(ws_take(ctx, (size_t)2 * nX * sizeof(float)));
  float* AT = static_cast<float*>(ws_take(ctx, (size_t)nspin * M * ldk * sizeof(float)));
  const unsigned g1 = (unsigned)((nX + 255) / 256);
  gamma_pad_kernel<<<g1, 256, 0, ctx->stream>>>(X1, Xf, N, ldk, nx * nspin);
  LRDM_HIP(hipGetLastError());
  gamma_pad_kernel<<<g1, 256, 0, ctx->stream>>>(X2, Xf + nX, N, ldk, nx * nspin);
  LRDM_HIP(hipGetLastError());
  dim3 gt((unsigned)((M + 63) / 64), (unsigned)(ldk / 64 + (ldk % 64 ? 1 : 0)), nspin);
  transpose_pad_kernel<<<gt, 256, 0, ctx->stream>>>(Psi, AT, N, M, ldk);
  LRDM_HIP(hipGetLastError());
  const int smem = NST * 2 * TB;
  LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&adj_psi_pipe_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, smem));
  const unsigned grd = (unsigned)((M + BT - 1) / BT) * (unsigned)((N + BT - 1) / BT) *
                       (unsigned)nspin;
  ProfScope prof(ctx, "adj_psi");
  adj_psi_pipe_kernel<<<grd, PT, smem, ctx->stream>>>(Xf, w1, w2, nx, AT, N, M, ldk, nspin, scale,
                                                      active, ctx->zeros, Out);
  return hipGetLastError();
}

size_t adj_psi_workspace_bytes(int N, int64_t M, int nspin, int nx, bool fp32) {
  if (!fp32) return 0;
  const size_t ldk = pad_k(N);
  return ws_align((size_t)2 * nx * nspin * N * ldk * sizeof(float)) +
         ws_align((size_t)nspin * M * ldk * sizeof(float));
}

// Adjoint rotation in the BF16X3 form: the 2 nx matrices and Psi^T split into
// three BF16 pieces each, then adj_psi_p3_kernel.
hipError_t launch_adj_psi_bf16x3(lrdm_ctx* ctx, const double* X1, const double* w1,
                                 const double* X2, const double* w2, int nx, const float* Psi,
                                 int N, int64_t M, int nspin, double scale, float* Out,
                                 const unsigned char* active) {
  const int ldk = pad_k(N);
  const int64_t nX = (int64_t)nx * nspin * N * ldk;
  __bf16* X3 = static_cast<__bf16*>(ws_take(ctx, (size_t)2 * 3 * nX * sizeof(__bf16)));
  __bf16* PT3 = static_cast<__bf16*>(ws_take(ctx, (size_t)nspin * 3 * M * ldk * sizeof(__bf16)));
  const unsigned g1 = (unsigned)((nX + 255) / 256);
  gamma_split3_kernel<<<g1, 256, 0, ctx->stream>>>(X1, X3, N, ldk, nx * nspin, 0);
  LRDM_HIP(hipGetLastError());
  gamma_split3_kernel<<<g1, 256, 0, ctx->stream>>>(X2, X3 + 3 * nX, N, ldk, nx * nspin, 0);
  LRDM_HIP(hipGetLastError());
  dim3 gt((unsigned)((M + 63) / 64), (unsigned)(ldk / 64 + (ldk % 64 ? 1 : 0)), nspin);
  transpose_split3_kernel<<<gt, 256, 0, ctx->stream>>>(Psi, PT3, N, M, ldk);
  LRDM_HIP(hipGetLastError());
  const int smem = NST * 6 * PB;
  LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&adj_psi_p3_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, smem));
  const unsigned grd = (unsigned)((M + BT - 1) / BT) * (unsigned)((N + BT - 1) / BT) *
                       (unsigned)nspin;
  ProfScope prof(ctx, "adj_psi");
  adj_psi_p3_kernel<<<grd, PT, smem, ctx->stream>>>(X3, w1, w2, nx, PT3, N, M, ldk, nspin, scale,
                                                    active, ctx->zeros, Out);
  return hipGetLastError();
}

size_t adj_psi_bf16x3_bytes(int N, int64_t M, int nspin, int nx) {
  const size_t ldk = pad_k(N);
  return ws_align((size_t)2 * 3 * nx * nspin * N * ldk * sizeof(__bf16)) +
         ws_align((size_t)nspin * 3 * M * ldk * sizeof(__bf16));
}

// ------------------------------------------------------------------ fused systems (host)
namespace {

// Items in decreasing order of work, so that the largest systems start first.
template <typename Item, typename Work>
std::vector<int> by_work(const Item* items, int n, Work work) {
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return work(items[a]) > work(items[b]); });
  return order;
}

bool a16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

hipError_t launch_tn_sym_fused(lrdm_ctx* ctx, const FusedProjItem* items, int n) {
  const int smem = NST * (2 * TB + 1024);
  LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tn_sym_fused_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, smem));
  std::vector<double*> parts(n, nullptr);
  std::vector<int> splits(n, 0);
  FusedProj t{};
  t.nsys = 0;
  int total = 0;
  auto flush = [&]() -> hipError_t {
    if (t.nsys == 0) return hipSuccess;
    t.wg0[t.nsys] = total;
    {
      ProfScope prof(ctx, "proj");
      tn_sym_fused_kernel<<<(unsigned)total, PT, smem, ctx->stream>>>(t, ctx->zeros);
    }
    t = FusedProj{};
    t.nsys = 0;
    total = 0;
    return hipGetLastError();
  };
  const auto order = by_work(items, n, [](const FusedProjItem& it) {
    return (double)it.M * it.N * it.N * it.batch;
  });
  for (int k : order) {
    const FusedProjItem& it = items[k];
    const int ntb = (it.N + BT - 1) / BT;
    const int ntiles = ntb * (ntb + 1) / 2;
    const int ns = tn_split_count(ctx, it.N, it.M, it.batch, TN_ARITH_F32, true);
    int64_t kchunk = (it.M + ns - 1) / ns;
    kchunk = (kchunk + KT - 1) / KT * KT;
    const bool pipe = it.M % 4 == 0 && a16(it.A) && a16(it.w) &&
                      tn_variant(ctx, it.N, it.M, it.batch, TN_ARITH_F32, true) == TN_VAR_DEFAULT;
    if (!pipe) {      // a system the copy engine cannot stage, or tuned to another layout
      // of tiles and waves, goes alone
      LRDM_HIP(launch_tn_sym<float>(ctx, it.A, nullptr, it.w, it.M, it.N, it.M, it.nspin,
                                    it.batch, LRDM_FP32, it.H, it.active));
      continue;
    }
    parts[k] = static_cast<double*>(ws_take(ctx, tn_part_bytes(it.N, it.M, it.batch)));
    splits[k] = ns;
    const int s = t.nsys++;
    const int used = ntiles * ns * it.batch;
    t.wg0[s] = total;
    t.used[s] = used;
    t.A[s] = it.A;
    t.w[s] = it.w;
    t.part[s] = parts[k];
    t.active[s] = it.active;
    t.M[s] = it.M;
    t.kchunk[s] = kchunk;
    t.N[s] = it.N;
    t.nspin[s] = it.nspin;
    t.ntb[s] = ntb;
    t.nsplit[s] = ns;
    t.batch[s] = it.batch;
    total += (used + 7) / 8 * 8;
    if (t.nsys == kMaxFused) LRDM_HIP(flush());
  }
  LRDM_HIP(flush());
  for (int k = 0; k < n; ++k) {
    if (!parts[k]) continue;
    const FusedProjItem& it = items[k];
    const int ntb = (it.N + BT - 1) / BT;
    dim3 blk(32, 8);
    dim3 grd2((it.N + 31) / 32, (it.N + 7) / 8, it.batch);
    tn_reduce_lp_kernel<<<grd2, blk, 0, ctx->stream>>>(parts[k], it.N, ntb, splits[k], it.H);
    LRDM_HIP(hipGetLastError());
  }
  return hipSuccess;
}

hipError_t launch_backproj_fused(lrdm_ctx* ctx, const FusedBackprojItem* items, int n) {
  const int smem = NST * 2 * TB + PW * 64 * (int)sizeof(double);
  LRDM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&backproj_fused_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, smem));
  FusedBackproj t{};
  t.nsys = 0;
  int total = 0;
  auto flush = [&]() -> hipError_t {
    if (t.nsys == 0) return hipSuccess;
    t.wg0[t.nsys] = total;
    {
      ProfScope prof(ctx, "backproj");
      backproj_fused_kernel<<<(unsigned)total, PT, smem, ctx->stream>>>(t, ctx->zeros);
    }
    t = FusedBackproj{};
    t.nsys = 0;
    total = 0;
    return hipGetLastError();
  };
  const auto order = by_work(items, n, [](const FusedBackprojItem& it) {
    return (double)it.M * it.N * it.N * it.batch;
  });
  for (int k : order) {
    const FusedBackprojItem& it = items[k];
    const int ldk = pad_k(it.N);
    float* Gf = static_cast<float*>(ws_take(ctx, (size_t)it.batch * it.N * ldk * sizeof(float)));
    float* AT = static_cast<float*>(ws_take(ctx, (size_t)it.nspin * it.M * ldk * sizeof(float)));
    const int64_t nG = (int64_t)it.batch * it.N * ldk;
    gamma_pad_kernel<<<(unsigned)((nG + 255) / 256), 256, 0, ctx->stream>>>(it.G, Gf, it.N, ldk,
                                                                           it.batch);
    LRDM_HIP(hipGetLastError());
    dim3 gt((unsigned)((it.M + 63) / 64), (unsigned)(ldk / 64 + (ldk % 64 ? 1 : 0)), it.nspin);
    transpose_pad_kernel<<<gt, 256, 0, ctx->stream>>>(it.A, AT, it.N, it.M, ldk);
    LRDM_HIP(hipGetLastError());
    const int s = t.nsys++;
    const int used = (int)((it.M + BT - 1) / BT) * it.batch;
    t.wg0[s] = total;
    t.used[s] = used;
    t.A[s] = it.A;
    t.AT[s] = AT;
    t.Gf[s] = Gf;
    t.out[s] = it.out;
    t.active[s] = it.active;
    t.M[s] = it.M;
    t.N[s] = it.N;
    t.ldk[s] = ldk;
    t.nspin[s] = it.nspin;
    t.batch[s] = it.batch;
    t.scale[s] = it.scale;
    total += (used + 7) / 8 * 8;
    if (t.nsys == kMaxFused) LRDM_HIP(flush());
  }
  return flush();
}

}  // namespace lrdm


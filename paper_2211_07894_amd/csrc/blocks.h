// Blocks of the response that can be left out.
//
// Gamma = F o H' - mu' diag(f') (Eq. (22)) is negligible wherever the Fermi
// multiplier F is: between two states both deep below the Fermi level, or both
// far above it, F_ij = (f_i - f_j)/(eps_i - eps_j) vanishes to many digits.
// launch_block_mask marks each 128 x 128 block (I, J) of the N x N matrices as
// active when its largest |F| exceeds tau times the largest over the whole
// multiplier; the projection leaves the H' blocks of inactive pairs at zero and
// the back-projection skips their Gamma blocks.  `active` is [nspin][ntb][ntb]
// bytes (ntb = ceil(N / 128) <= 64), symmetric; NULL means every block.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lrdm {

constexpr int kBlockEdge = 128;

__device__ inline bool block_active(const unsigned char* active, int c, int ntb, int I, int J) {
  return !active || active[((int64_t)c * ntb + I) * ntb + J] != 0;
}

// Bit J set for each active block (ib, J) with J >= ib.
__device__ inline uint64_t active_row_bits(const unsigned char* active, int c, int ntb, int ib) {
  uint64_t m = 0;
  for (int J = ib; J < ntb; ++J)
    if (block_active(active, c, ntb, ib, J)) m |= 1ull << J;
  return m;
}

// Number of K-tiles of width kt over the active blocks of `bits` (the last
// block, J = ntb - 1, may be ragged: it ends at N).
__device__ inline int active_ktiles(uint64_t bits, int N, int kt) {
  int n = 0;
  while (bits) {
    const int J = __builtin_ctzll(bits);
    bits &= bits - 1;
    const int lo = J * kBlockEdge, hi = min(N, lo + kBlockEdge);
    n += (hi - lo + kt - 1) / kt;
  }
  return n;
}

// Block J and first column of K-tile t when the active blocks of `bits` are
// walked in order, kBlockEdge / kt tiles per block; t past the end gives J = -1.
__device__ inline int active_ktile(uint64_t bits, int t, int kt, int& J) {
  const int per = kBlockEdge / kt;
  int q = t / per;
  while (q > 0 && bits) {
    bits &= bits - 1;
    --q;
  }
  if (!bits) {
    J = -1;
    return 0;
  }
  J = __builtin_ctzll(bits);
  return J * kBlockEdge + (t % per) * kt;
}

}  // namespace lrdm

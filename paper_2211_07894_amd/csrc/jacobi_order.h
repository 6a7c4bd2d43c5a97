// Index logic of the block-Jacobi eigensolver, shared by its kernels and by a
// host-only unit test: round-robin pairings and the ordering of eigenvalues.
#pragma once

#if defined(__HIPCC__)
#define LRDM_HD __host__ __device__
#else
#define LRDM_HD
#endif

namespace lrdm {

// Round-robin (circle) tournament on n players, n even: in round t the player at
// position k is 0 for k = 0 and ((k - 1 + t) mod (n - 1)) + 1 otherwise;
// positions k and n - 1 - k meet.  Over rounds 0..n-2 every pair meets once.
LRDM_HD inline int rr_pos(int k, int t, int n) {
  return k == 0 ? 0 : ((k - 1 + t) % (n - 1)) + 1;
}

// Sort key of a diagonal entry: NaN sorts as +infinity, so that the rank below is
// a permutation for any input.
LRDM_HD inline double order_key(double d) {
  return (d != d) ? __builtin_huge_val() : d;
}

// Rank of entry k among diag[0..n): entries with a smaller key, plus equal keys at
// a smaller index.  A strict total order, hence a permutation of 0..n-1.
LRDM_HD inline int order_rank(const double* diag, int stride, int n, int k) {
  const double d = order_key(diag[(long long)k * stride]);
  int rank = 0;
  for (int j = 0; j < n; ++j) {
    const double e = order_key(diag[(long long)j * stride]);
    rank += (e < d) || (e == d && j < k);
  }
  return rank;
}

// NaN-propagating maximum (fmax drops NaN, which would hide a failed iteration).
LRDM_HD inline double nan_max(double a, double b) {
  return (a != a) ? a : ((b != b) ? b : (a > b ? a : b));
}

}  // namespace lrdm

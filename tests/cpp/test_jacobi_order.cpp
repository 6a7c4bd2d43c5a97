// Host-only checks of the eigensolver's index logic (same header as the kernels):
// the round-robin tournament meets every pair exactly once per sweep, and the
// eigenvalue ordering is a permutation for any input, NaN and ties included.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "jacobi_order.h"

using namespace lrdm;

static int check_tournament(int n) {
  std::vector<int> met(n * n, 0);
  for (int t = 0; t < n - 1; ++t) {
    std::vector<int> seen(n, 0);
    for (int i = 0; i < n / 2; ++i) {
      const int p = rr_pos(i, t, n), q = rr_pos(n - 1 - i, t, n);
      if (p < 0 || p >= n || q < 0 || q >= n || p == q) return 1;
      if (seen[p]++ || seen[q]++) return 2;
      met[p * n + q]++;
      met[q * n + p]++;
    }
  }
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      if (p != q && met[p * n + q] != 1) return 3;
  return 0;
}

static int check_rank(std::vector<double> d) {
  const int n = (int)d.size();
  std::vector<int> perm(n, -1);
  for (int k = 0; k < n; ++k) {
    const int r = order_rank(d.data(), 1, n, k);
    if (r < 0 || r >= n) return 1;
    if (perm[r] != -1) return 2;
    perm[r] = k;
  }
  for (int i = 1; i < n; ++i) {
    const double a = order_key(d[perm[i - 1]]), b = order_key(d[perm[i]]);
    if (a > b) return 3;
  }
  return 0;
}

int main() {
  int fails = 0;
  for (int n : {2, 4, 6, 16, 64, 192, 1024}) {
    const int r = check_tournament(n);
    if (r) { std::printf("tournament n=%d failed (%d)\n", n, r); ++fails; }
  }
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> u(-3, 3);
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const double inf = std::numeric_limits<double>::infinity();
  for (int trial = 0; trial < 200; ++trial) {
    const int n = 1 + (int)(rng() % 300);
    std::vector<double> d(n);
    for (double& x : d) {
      const int kind = (int)(rng() % 10);
      x = kind == 0 ? nan : kind == 1 ? inf : kind == 2 ? -inf : kind == 3 ? 1.0 : u(rng);
    }
    const int r = check_rank(d);
    if (r) { std::printf("rank trial %d failed (%d)\n", trial, r); ++fails; }
  }
  if (!(nan_max(1.0, nan) != nan_max(1.0, nan)) || !(nan_max(nan, 1.0) != nan_max(nan, 1.0)) ||
      nan_max(2.0, 3.0) != 3.0) {
    std::printf("nan_max failed\n");
    ++fails;
  }
  std::printf("%s\n", fails ? "FAIL" : "OK");
  return fails ? 1 : 0;
}

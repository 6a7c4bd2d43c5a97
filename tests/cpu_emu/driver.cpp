// Driver of the test-only CPU build: runs every C-ABI entry point (and a few
// internal launchers at full size) on host memory under AddressSanitizer.
// Exit status 0 and "EMU OK" when every call returned LRDM_OK with finite
// outputs; ASan aborts the process on any out-of-bounds access.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lrdm.h"
#include "lrdm_internal.h"

namespace {

int failures = 0;

void check(lrdm_status st, lrdm_ctx* ctx, const char* what) {
  if (st != LRDM_OK) {
    std::printf("FAIL %s: status %d: %s\n", what, (int)st, lrdm_last_error(ctx));
    ++failures;
  } else {
    std::printf("ok   %s\n", what);
  }
  std::fflush(stdout);
}

struct Rng {
  unsigned long long s;
  double next() {  // uniform in (-1, 1)
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return ((s >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
  }
};

std::vector<double> randv(size_t n, unsigned long long seed, double scale = 1.0) {
  Rng r{seed};
  std::vector<double> v(n);
  for (auto& x : v) x = scale * r.next();
  return v;
}

bool finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

lrdm_grid grid(int nx, int ny, int nz, double h) {
  lrdm_grid g;
  g.n[0] = nx; g.n[1] = ny; g.n[2] = nz;
  g.L[0] = nx * h; g.L[1] = ny * h; g.L[2] = nz * h;
  return g;
}

// Gram-Schmidt rows of a random block: an orthonormal basis of N vectors in R^M.
std::vector<double> orthonormal(int N, int64_t M, unsigned long long seed) {
  std::vector<double> P = randv((size_t)N * M, seed);
  for (int i = 0; i < N; ++i) {
    double* pi = &P[(size_t)i * M];
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < i; ++j) {
        const double* pj = &P[(size_t)j * M];
        double d = 0;
        for (int64_t p = 0; p < M; ++p) d += pi[p] * pj[p];
        for (int64_t p = 0; p < M; ++p) pi[p] -= d * pj[p];
      }
    double n = 0;
    for (int64_t p = 0; p < M; ++p) n += pi[p] * pi[p];
    n = std::sqrt(n);
    for (int64_t p = 0; p < M; ++p) pi[p] /= n;
  }
  return P;
}

const char* prec_name(lrdm_prec p) {
  return p == LRDM_FP64 ? "fp64" : (p == LRDM_FP32 ? "fp32" : "bf16x3");
}

// Storage of a block in the form's element type.
struct Block {
  std::vector<double> d;
  std::vector<float> f;
  lrdm_prec prec;
  Block(const std::vector<double>& x, lrdm_prec p) : prec(p) {
    if (p == LRDM_FP64) d = x;
    else f.assign(x.begin(), x.end());
  }
  void* data() { return prec == LRDM_FP64 ? (void*)d.data() : (void*)f.data(); }
  std::vector<double> values() const {
    return prec == LRDM_FP64 ? d : std::vector<double>(f.begin(), f.end());
  }
};

void scenario_response(lrdm_ctx* ctx, lrdm_grid g, int N, int nspin, int r,
                       lrdm_prec prec = LRDM_FP64) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  std::vector<double> Psi0;
  for (int c = 0; c < nspin; ++c) {
    auto P = orthonormal(N, M, 11 + c);
    Psi0.insert(Psi0.end(), P.begin(), P.end());
  }
  Block Psi(Psi0, prec);
  std::vector<double> eps((size_t)nspin * N);
  for (int c = 0; c < nspin; ++c)
    for (int i = 0; i < N; ++i) eps[(size_t)c * N + i] = -1.0 + 1.5 * i / N + 0.001 * c;
  lrdm_occ occ{nspin, 0.02, 0.8 * N};
  auto dV = randv((size_t)r * nspin * M, 5);
  std::vector<double> drho(dV.size()), mu(1), dmu(r), t(dV.size());
  char name[128];
  std::snprintf(name, sizeof name, "density_response %s N=%d nspin=%d r=%d grid %dx%dx%d",
                prec_name(prec), N, nspin, r, g.n[0], g.n[1], g.n[2]);
  check(density_response(ctx, &g, Psi.data(), eps.data(), N, &occ, dV.data(), r, prec,
                         drho.data(), mu.data(), dmu.data()), ctx, name);
  if (!finite(drho)) { std::printf("FAIL non-finite drho\n"); ++failures; }
  std::snprintf(name, sizeof name, "residual_derivative N=%d nspin=%d r=%d", N, nspin, r);
  check(lrdm_residual_derivative(ctx, &g, Psi.data(), eps.data(), N, &occ, dV.data(), r,
                                 prec, t.data()), ctx, name);
  std::vector<double> Hp((size_t)r * nspin * N * N);
  check(lrdm_projected_perturbation(ctx, &g, Psi.data(), N, nspin, dV.data(), r, prec,
                                    Hp.data()), ctx, "projected_perturbation");
  if (prec != LRDM_FP64) {
    // the single-precision forms against the FP64 form on the same (rounded) block
    Block P64(Psi.values(), LRDM_FP64);
    std::vector<double> ref(dV.size());
    check(density_response(ctx, &g, P64.data(), eps.data(), N, &occ, dV.data(), r, LRDM_FP64,
                           ref.data(), mu.data(), dmu.data()), ctx, "density_response fp64 reference");
    double num = 0, den = 0;
    for (size_t i = 0; i < ref.size(); ++i) {
      num += (drho[i] - ref[i]) * (drho[i] - ref[i]);
      den += ref[i] * ref[i];
    }
    const double err = std::sqrt(num / den);
    const double tol = prec == LRDM_FP32 ? 1e-5 : 1e-6;
    std::printf("     %s drho rel err vs fp64 %.2e (bound %.0e)\n", prec_name(prec), err, tol);
    if (!(err < tol)) ++failures;
  }
  std::vector<double> f((size_t)nspin * N), fp((size_t)nspin * N), F((size_t)nspin * N * N);
  check(lrdm_fermi_occupations(ctx, eps.data(), N, &occ, mu.data(), f.data(), fp.data(), F.data()),
        ctx, "fermi_occupations");
}

// A spectrum with deep occupied and high empty states, so that the response's
// block mask drops blocks: the result with the default threshold against every
// block formed (threshold 0).
void scenario_block_skip(lrdm_ctx* ctx, lrdm_grid g, int N, int nspin, int r, lrdm_prec prec) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  std::vector<double> Psi0;
  for (int c = 0; c < nspin; ++c) {
    auto P = orthonormal(N, M, 21 + c);
    Psi0.insert(Psi0.end(), P.begin(), P.end());
  }
  Block Psi(Psi0, prec);
  std::vector<double> eps((size_t)nspin * N);
  for (int c = 0; c < nspin; ++c)
    for (int i = 0; i < N; ++i) eps[(size_t)c * N + i] = -3.0 + 4.0 * i / N + 0.001 * c;
  lrdm_occ occ{nspin, 0.005, (nspin == 1 ? 0.8 : 0.4 * nspin) * N};
  auto dV = randv((size_t)r * nspin * M, 6);
  std::vector<double> a(dV.size()), b(dV.size()), mu(1), dmu(r);
  char name[128];
  std::snprintf(name, sizeof name, "density_response %s block skip N=%d nspin=%d r=%d",
                prec_name(prec), N, nspin, r);
  check(density_response(ctx, &g, Psi.data(), eps.data(), N, &occ, dV.data(), r, prec, a.data(),
                         mu.data(), dmu.data()), ctx, name);
  check(lrdm_set_response_block_skip(ctx, 0.0), ctx, "block skip off");
  check(density_response(ctx, &g, Psi.data(), eps.data(), N, &occ, dV.data(), r, prec, b.data(),
                         mu.data(), dmu.data()), ctx, "density_response, every block");
  check(lrdm_set_response_block_skip(ctx, 1e-14), ctx, "block skip on");
  double num = 0, den = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    num += (a[i] - b[i]) * (a[i] - b[i]);
    den += b[i] * b[i];
  }
  const double err = std::sqrt(num / den);
  std::printf("     %s block skip vs every block: rel diff %.2e\n", prec_name(prec), err);
  if (!finite(a) || !(err < (prec == LRDM_FP64 ? 1e-12 : 1e-6))) ++failures;
}

// Zone-sampled response: random realified blocks, unequal weights (bounds and
// finiteness; the numbers are checked against the oracle on the GPU).
void scenario_response_bz(lrdm_ctx* ctx, lrdm_grid g, int N, int nk, int nspin, int r,
                          lrdm_prec prec) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  Block Psi(randv((size_t)nspin * nk * 2 * N * M, 31, 0.05), prec);
  std::vector<double> eps((size_t)nspin * nk * N), w(nk);
  for (size_t i = 0; i < eps.size(); ++i) eps[i] = -1.0 + 1.5 * (double)(i % N) / N + 0.001 * (i / N);
  for (int k = 0; k < nk; ++k) w[k] = (1.0 + k) / (nk * (nk + 1) / 2.0);
  lrdm_occ occ{nspin, 0.02, 0.8 * N};
  auto dV = randv((size_t)r * nspin * M, 32);
  std::vector<double> drho((size_t)r * nspin * M), mu(1), dmu(r);
  char name[128];
  std::snprintf(name, sizeof name, "density_response_bz %s N=%d nk=%d nspin=%d r=%d",
                prec_name(prec), N, nk, nspin, r);
  check(density_response_bz(ctx, &g, Psi.data(), eps.data(), w.data(), N, nk, &occ, dV.data(), r,
                            prec, drho.data(), mu.data(), dmu.data()), ctx, name);
  if (!finite(drho)) { std::printf("FAIL non-finite drho\n"); ++failures; }
}

// Several uneven systems in one batched call (FP32: the fused launches), each
// against its own single call (bounds; the batched and single results match).
void scenario_batched(lrdm_ctx* ctx, lrdm_prec prec) {
  const int nsys = 3;
  const lrdm_grid gs[nsys] = {grid(8, 8, 8, 0.5), grid(12, 8, 8, 0.45), grid(8, 8, 6, 0.5)};
  const int Ns[nsys] = {150, 40, 70}, rs[nsys] = {2, 3, 1};
  std::vector<Block> psi;
  std::vector<std::vector<double>> eps(nsys), dV(nsys), drho(nsys), one(nsys), mu(nsys),
      dmu(nsys);
  std::vector<lrdm_system> sys(nsys);
  psi.reserve(nsys);
  for (int s = 0; s < nsys; ++s) {
    const int64_t M = (int64_t)gs[s].n[0] * gs[s].n[1] * gs[s].n[2];
    std::vector<double> P;
    for (int c = 0; c < 2; ++c) {
      auto Q = orthonormal(Ns[s], M, 41 + 2 * s + c);
      P.insert(P.end(), Q.begin(), Q.end());
    }
    psi.emplace_back(P, prec);
    eps[s].resize(2 * Ns[s]);
    for (int i = 0; i < 2 * Ns[s]; ++i) eps[s][i] = -2.0 + 2.5 * (i % Ns[s]) / Ns[s] + 0.01 * (i / Ns[s]);
    dV[s] = randv((size_t)rs[s] * 2 * M, 43 + s);
    drho[s].assign(dV[s].size(), 0.0);
    one[s].assign(dV[s].size(), 0.0);
    mu[s].assign(1, 0.0);
    dmu[s].assign(rs[s], 0.0);
    sys[s] = lrdm_system{gs[s], psi[s].data(), eps[s].data(), Ns[s], lrdm_occ{2, 0.01, 0.78 * Ns[s]},
                         dV[s].data(), rs[s], drho[s].data(), mu[s].data(), dmu[s].data()};
  }
  char name[96];
  std::snprintf(name, sizeof name, "density_response_batched %s, %d systems", prec_name(prec), nsys);
  check(density_response_batched(ctx, sys.data(), nsys, prec), ctx, name);
  for (int s = 0; s < nsys; ++s) {
    std::vector<double> m1(1), d1(rs[s]);
    check(density_response(ctx, &gs[s], psi[s].data(), eps[s].data(), Ns[s], &sys[s].occ,
                           dV[s].data(), rs[s], prec, one[s].data(), m1.data(), d1.data()),
          ctx, "density_response (one system)");
    double worst = 0.0;
    for (size_t i = 0; i < one[s].size(); ++i) worst = std::max(worst, std::fabs(one[s][i] - drho[s][i]));
    std::printf("     system %d: batched vs single max diff %.2e\n", s, worst);
    if (!(worst == 0.0) || !finite(drho[s])) ++failures;
  }
}

void scenario_chfsi(lrdm_ctx* ctx, lrdm_grid g, int N, int degree, lrdm_prec prec = LRDM_FP64) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  auto V = randv((size_t)M, 3, 0.5);
  Block X(randv((size_t)N * M, 4), prec);
  Block Y(std::vector<double>((size_t)N * M), prec), HX(std::vector<double>((size_t)N * M), prec);
  std::vector<double> eps(N);
  double hx = g.L[0] / g.n[0], hy = g.L[1] / g.n[1], hz = g.L[2] / g.n[2];
  const double b = 2 / (hx * hx) + 2 / (hy * hy) + 2 / (hz * hz) + 0.5;
  char name[128];
  std::snprintf(name, sizeof name, "hamiltonian_apply %s N=%d grid %dx%dx%d", prec_name(prec), N,
                g.n[0], g.n[1], g.n[2]);
  check(lrdm_hamiltonian_apply(ctx, &g, V.data(), X.data(), HX.data(), N, prec), ctx, name);
  std::snprintf(name, sizeof name, "chfsi_filter %s N=%d degree=%d", prec_name(prec), N, degree);
  check(chfsi_filter(ctx, &g, V.data(), X.data(), Y.data(), N, prec, degree, -0.2, b, -1.0),
        ctx, name);
  std::snprintf(name, sizeof name, "subspace_rayleigh_ritz %s N=%d", prec_name(prec), N);
  check(subspace_rayleigh_ritz(ctx, &g, V.data(), Y.data(), N, prec, eps.data()), ctx, name);
  const std::vector<double> Yv = Y.values();
  if (!finite(eps) || !finite(Yv)) { std::printf("FAIL non-finite Ritz output\n"); ++failures; }
  // orthonormality of the Ritz vectors
  double worst = 0;
  for (int i = 0; i < N; i += 7)
    for (int j = 0; j < N; j += 5) {
      double d = 0;
      for (int64_t p = 0; p < M; ++p) d += Yv[(size_t)i * M + p] * Yv[(size_t)j * M + p];
      worst = std::fmax(worst, std::fabs(d - (i == j)));
    }
  const double bound = prec == LRDM_FP64 ? 1e-10 : 1e-5;
  std::printf("     Ritz orthonormality error %.2e (bound %.0e)\n", worst, bound);
  if (!(worst < bound)) ++failures;
  std::vector<double> u = randv((size_t)2 * M, 9), dV(u.size());
  check(lrdm_hartree_kernel(ctx, &g, u.data(), dV.data(), 2), ctx, "hartree_kernel");
}

// ChFSI of one k-point: the Bloch filter, then the complex Rayleigh-Ritz; the Ritz
// vectors must be orthonormal and diagonalise H_k in the complex product.
void scenario_rr_bloch(lrdm_ctx* ctx, lrdm_grid g, int N, int degree) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  auto V = randv((size_t)M, 3, 0.5);
  const double k[3] = {0.5, -0.3, 0.9};
  std::vector<double> X = randv((size_t)2 * N * M, 14), Y((size_t)2 * N * M),
                      HY((size_t)2 * N * M), eps(N);
  double hx = g.L[0] / g.n[0], hy = g.L[1] / g.n[1], hz = g.L[2] / g.n[2];
  const double b = 2 / (hx * hx) + 2 / (hy * hy) + 2 / (hz * hz) + 0.5;
  char name[128];
  std::snprintf(name, sizeof name, "chfsi_filter_bloch N=%d degree=%d", N, degree);
  check(chfsi_filter_bloch(ctx, &g, V.data(), k[0], k[1], k[2], X.data(), Y.data(), N, LRDM_FP64,
                           degree, -0.2, b, -1.0),
        ctx, name);
  std::snprintf(name, sizeof name, "subspace_rayleigh_ritz_bloch N=%d grid %dx%dx%d", N, g.n[0],
                g.n[1], g.n[2]);
  check(subspace_rayleigh_ritz_bloch(ctx, &g, V.data(), k[0], k[1], k[2], Y.data(), N,
                                     LRDM_FP64, eps.data()),
        ctx, name);
  check(lrdm_bloch_hamiltonian_apply(ctx, &g, V.data(), k[0], k[1], k[2], Y.data(), HY.data(), N,
                                     LRDM_FP64),
        ctx, "bloch_hamiltonian_apply of the Ritz vectors");
  if (!finite(eps) || !finite(Y)) { std::printf("FAIL non-finite Ritz output\n"); ++failures; }
  // <psi_i, psi_j> = delta_ij and <psi_i, H_k psi_j> = eps_i delta_ij (complex products)
  const size_t im = (size_t)N * M;
  double worst_o = 0, worst_h = 0, worst_order = 0;
  for (int i = 0; i < N; i += 7)
    for (int j = 0; j < N; j += 5) {
      double ore = 0, oim = 0, hre = 0, him = 0;
      for (int64_t p = 0; p < M; ++p) {
        const double ar = Y[(size_t)i * M + p], ai = Y[im + (size_t)i * M + p];
        const double br = Y[(size_t)j * M + p], bi = Y[im + (size_t)j * M + p];
        const double cr = HY[(size_t)j * M + p], ci = HY[im + (size_t)j * M + p];
        ore += ar * br + ai * bi;
        oim += ar * bi - ai * br;
        hre += ar * cr + ai * ci;
        him += ar * ci - ai * cr;
      }
      worst_o = std::fmax(worst_o, std::hypot(ore - (i == j), oim));
      worst_h = std::fmax(worst_h, std::hypot(hre - (i == j ? eps[i] : 0.0), him));
    }
  for (int i = 1; i < N; ++i) worst_order = std::fmax(worst_order, eps[i - 1] - eps[i]);
  std::printf("     complex orthonormality %.2e, projected H_k off the Ritz values %.2e, "
              "order %.2e\n", worst_o, worst_h, worst_order);
  if (!(worst_o < 1e-10) || !(worst_h < 1e-9) || !(worst_order <= 0.0)) ++failures;
}

// The complex Rayleigh-Ritz on an FP32 block (FP64 arithmetic): orthonormal
// Ritz vectors in the complex product, ascending Ritz values.
void scenario_rr_bloch_fp32(lrdm_ctx* ctx, lrdm_grid g, int N) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  auto V = randv((size_t)M, 3, 0.5);
  const std::vector<double> y = randv((size_t)2 * N * M, 17);
  std::vector<float> Y(y.begin(), y.end());
  std::vector<double> eps(N);
  check(subspace_rayleigh_ritz_bloch(ctx, &g, V.data(), 0.3, -0.2, 0.5, Y.data(), N, LRDM_FP32,
                                     eps.data()),
        ctx, "subspace_rayleigh_ritz_bloch fp32");
  const size_t im = (size_t)N * M;
  double worst = 0, order = 0;
  for (int i = 0; i < N; i += 3)
    for (int j = 0; j < N; j += 2) {
      double ore = 0, oim = 0;
      for (int64_t p = 0; p < M; ++p) {
        const double ar = Y[(size_t)i * M + p], ai = Y[im + (size_t)i * M + p];
        const double br = Y[(size_t)j * M + p], bi = Y[im + (size_t)j * M + p];
        ore += ar * br + ai * bi;
        oim += ar * bi - ai * br;
      }
      worst = std::fmax(worst, std::hypot(ore - (i == j), oim));
    }
  for (int i = 1; i < N; ++i) order = std::fmax(order, eps[i - 1] - eps[i]);
  std::printf("     complex orthonormality %.2e (bound 1e-5), order %.2e\n", worst, order);
  if (!(worst < 1e-5) || !(order <= 0.0) || !finite(eps)) ++failures;
}

// Degenerate Ritz values of H_k: free electrons (V = 0) on a cubic 6^3 grid at
// k = 0, the subspace of the 19 lowest plane waves (1 + 6 + 12 equal energies)
// mixed by a random complex matrix.  The complex Rayleigh-Ritz must return the
// three exact energies with their multiplicities and orthonormal vectors.
void scenario_rr_bloch_degenerate(lrdm_ctx* ctx) {
  const lrdm_grid g = grid(6, 6, 6, 0.5);
  const int n = 6, N = 19;
  const int64_t M = (int64_t)n * n * n;
  const double h = 0.5, pi = 3.14159265358979323846;
  std::vector<double> V((size_t)M, 0.0);
  std::vector<int> waves;   // (nx, ny, nz) in {-1, 0, 1}^3 with at most two nonzero
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b)
      for (int c = -1; c <= 1; ++c)
        if (std::abs(a) + std::abs(b) + std::abs(c) <= 2) {
          waves.push_back(a);
          waves.push_back(b);
          waves.push_back(c);
        }
  std::vector<double> mix = randv((size_t)2 * N * N, 21);
  std::vector<double> Y((size_t)2 * N * M, 0.0), eps(N);
  for (int i = 0; i < N; ++i)
    for (int w = 0; w < N; ++w) {
      const double qr = mix[(size_t)i * N + w], qi = mix[(size_t)N * N + i * N + w];
      for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
          for (int x = 0; x < n; ++x) {
            const double ph = 2 * pi * (waves[3 * w] * x + waves[3 * w + 1] * y +
                                        waves[3 * w + 2] * z) / n;
            const double wr = std::cos(ph) / std::sqrt((double)M), wi = std::sin(ph) / std::sqrt((double)M);
            const size_t p = ((size_t)z * n + y) * n + x;
            Y[(size_t)i * M + p] += qr * wr - qi * wi;
            Y[(size_t)N * M + (size_t)i * M + p] += qr * wi + qi * wr;
          }
    }
  check(subspace_rayleigh_ritz_bloch(ctx, &g, V.data(), 0.0, 0.0, 0.0, Y.data(), N, LRDM_FP64,
                                     eps.data()),
        ctx, "subspace_rayleigh_ritz_bloch degenerate N=19 (1 + 6 + 12)");
  const double e1 = (1 - std::cos(2 * pi / n)) / (h * h);   // one direction at +-1
  double worst_e = 0;
  for (int i = 0; i < N; ++i) {
    const double ref = i == 0 ? 0.0 : (i < 7 ? e1 : 2 * e1);
    worst_e = std::fmax(worst_e, std::fabs(eps[i] - ref));
  }
  double worst_o = 0;
  const size_t im = (size_t)N * M;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double ore = 0, oim = 0;
      for (int64_t p = 0; p < M; ++p) {
        const double ar = Y[(size_t)i * M + p], ai = Y[im + (size_t)i * M + p];
        const double br = Y[(size_t)j * M + p], bi = Y[im + (size_t)j * M + p];
        ore += ar * br + ai * bi;
        oim += ar * bi - ai * br;
      }
      worst_o = std::fmax(worst_o, std::hypot(ore - (i == j), oim));
    }
  std::printf("     Ritz values off the exact shells %.2e, complex orthonormality %.2e\n", worst_e,
              worst_o);
  if (!(worst_e < 1e-12) || !(worst_o < 1e-11) || !finite(Y)) ++failures;
}

// Rayleigh-Ritz of a block with exactly and nearly dependent rows (exact copies, a
// combination, a zero row): the orthonormalisation takes its multi-pass route,
// residual rows and pseudo-random completion included; the Ritz vectors must still
// be orthonormal.
void scenario_rr_dependent(lrdm_ctx* ctx, lrdm_grid g, int N, lrdm_prec prec) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  auto V = randv((size_t)M, 3, 0.5);
  std::vector<double> y = randv((size_t)N * M, 12);
  auto row = [&](int i) { return y.begin() + (size_t)i * M; };
  std::copy(row(3), row(4), row(N / 3));                              // exact copy
  for (int64_t p = 0; p < M; ++p) y[(size_t)(N / 2) * M + p] = 2 * row(10)[p] - row(11)[p];
  for (int64_t p = 0; p < M; ++p) y[(size_t)(N - 2) * M + p] = row(0)[p] * (1 + 1e-13);
  std::fill(row(N - 1), row(N), 0.0);                                 // zero row
  Block Y(y, prec);
  std::vector<double> eps(N);
  char name[128];
  std::snprintf(name, sizeof name, "subspace_rayleigh_ritz dependent rows %s N=%d", prec_name(prec), N);
  check(subspace_rayleigh_ritz(ctx, &g, V.data(), Y.data(), N, prec, eps.data()), ctx, name);
  const std::vector<double> Yv = Y.values();
  double worst = 0;
  for (int i = 0; i < N; i += 3)
    for (int j = 0; j < N; j += 2) {
      double d = 0;
      for (int64_t p = 0; p < M; ++p) d += Yv[(size_t)i * M + p] * Yv[(size_t)j * M + p];
      worst = std::fmax(worst, std::fabs(d - (i == j)));
    }
  const double bound = prec == LRDM_FP64 ? 1e-10 : 1e-5;
  std::printf("     Ritz orthonormality error %.2e (bound %.0e)\n", worst, bound);
  if (!(worst < bound) || !finite(eps)) ++failures;
}

// Internal launchers at the full subspace size of the 64^3 workload (N = 1024):
// the eigenvalue ordering and gather of the eigensolver.
void scenario_full_n(lrdm_ctx* ctx) {
  const int N = 1024;
  lrdm::ws_reserve(ctx, 64u << 20);
  // an already diagonal matrix: the eigensolver goes straight to ordering and gather
  std::vector<double> D((size_t)N * N, 0.0), ev(N), Q((size_t)N * N);
  for (int i = 0; i < N; ++i) D[(size_t)i * N + i] = std::cos(0.37 * i);
  ctx->ws_top = 0;
  lrdm_status st = lrdm::sym_eigh(ctx, D.data(), N, N, nullptr, ev.data(), Q.data());
  check(st, ctx, "sym_eigh diagonal N=1024 (ordering + gather)");
  for (int i = 1; i < N; ++i)
    if (ev[i] < ev[i - 1]) { std::printf("FAIL order\n"); ++failures; break; }
  // a diagonal with NaN entries: ordering must stay a permutation
  D[5 * N + 5] = std::nan("");
  D[700 * N + 700] = std::nan("");
  ctx->ws_top = 0;
  st = lrdm::sym_eigh(ctx, D.data(), N, N, nullptr, ev.data(), Q.data());
  std::printf("     sym_eigh with NaN diagonal returned %d\n", (int)st);
}

// Projected perturbation of one form against FP64 on the same rounded block.
void scenario_projection(lrdm_ctx* ctx, lrdm_grid g, int N, int r, lrdm_prec prec) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  Block Psi(orthonormal(N, M, 21), prec);
  Block P64(Psi.values(), LRDM_FP64);
  auto dV = randv((size_t)r * M, 7);
  std::vector<double> H((size_t)r * N * N), R(H.size());
  check(lrdm_projected_perturbation(ctx, &g, Psi.data(), N, 1, dV.data(), r, prec, H.data()), ctx,
        "projected_perturbation (form)");
  check(lrdm_projected_perturbation(ctx, &g, P64.data(), N, 1, dV.data(), r, LRDM_FP64, R.data()),
        ctx, "projected_perturbation fp64");
  double worst = 0, scale = 0;
  size_t bad = 0;
  for (size_t i = 0; i < H.size(); ++i) {
    scale = std::fmax(scale, std::fabs(R[i]));
    if (!std::isfinite(H[i])) { if (bad++ < 5) std::printf("     non-finite at %zu\n", i); continue; }
    worst = std::fmax(worst, std::fabs(H[i] - R[i]));
  }
  std::printf("     %s projection: max err %.2e of max %.2e, non-finite %zu; H[0..3] %g %g %g vs %g %g %g\n",
              prec_name(prec), worst, scale, bad, H[0], H[1], H[N + 1], R[0], R[1], R[N + 1]);
  if (bad || !(worst < 1e-5 * scale)) ++failures;
}

// Adjoint of the response: all outputs, finite, and dL/ddV equal to the response
// to g itself (the map is symmetric).
void scenario_backward(lrdm_ctx* ctx, lrdm_grid g, int N, int nspin, int r, lrdm_prec prec) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  std::vector<double> P0;
  for (int c = 0; c < nspin; ++c) {
    auto P = orthonormal(N, M, 31 + c);
    P0.insert(P0.end(), P.begin(), P.end());
  }
  Block Psi(P0, prec), gPsi(std::vector<double>(P0.size()), prec);
  std::vector<double> eps((size_t)nspin * N);
  for (int c = 0; c < nspin; ++c)
    for (int i = 0; i < N; ++i) eps[(size_t)c * N + i] = -1.0 + 1.5 * i / N + 0.001 * c;
  lrdm_occ occ{nspin, 0.03, 0.7 * N};
  auto dV = randv((size_t)r * nspin * M, 41);
  auto G = randv((size_t)r * nspin * M, 43);
  std::vector<double> gdV(dV.size()), geps((size_t)nspin * N), ref(dV.size()), mu(1), dmu(r);
  char name[128];
  std::snprintf(name, sizeof name, "density_response_backward %s N=%d nspin=%d r=%d grid %dx%dx%d",
                prec_name(prec), N, nspin, r, g.n[0], g.n[1], g.n[2]);
  check(density_response_backward(ctx, &g, Psi.data(), eps.data(), N, &occ, dV.data(), r, prec,
                                  G.data(), gdV.data(), gPsi.data(), geps.data()), ctx, name);
  if (!finite(gdV) || !finite(geps) || !finite(gPsi.values())) {
    std::printf("FAIL non-finite gradient\n");
    ++failures;
  }
  check(density_response(ctx, &g, Psi.data(), eps.data(), N, &occ, G.data(), r, prec, ref.data(),
                         mu.data(), dmu.data()), ctx, "density_response of g");
  double num = 0, den = 0;
  for (size_t i = 0; i < ref.size(); ++i) {
    num += (gdV[i] - ref[i]) * (gdV[i] - ref[i]);
    den += ref[i] * ref[i];
  }
  const double err = std::sqrt(num / den);
  std::printf("     self-adjointness %.2e\n", err);
  if (!(err < (prec == LRDM_FP64 ? 1e-12 : 1e-5))) ++failures;
}


void scenario_lowrank(lrdm_ctx* ctx, lrdm_grid g, int N, int nspin, int r_max, lrdm_prec prec) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  std::vector<double> Psi0;
  for (int c = 0; c < nspin; ++c) {
    auto P = orthonormal(N, M, 21 + c);
    Psi0.insert(Psi0.end(), P.begin(), P.end());
  }
  Block Psi(Psi0, prec);
  std::vector<double> eps((size_t)nspin * N);
  for (int c = 0; c < nspin; ++c)
    for (int i = 0; i < N; ++i) eps[(size_t)c * N + i] = -1.0 + 1.5 * i / N + 0.001 * c;
  lrdm_occ occ{nspin, 0.02, 0.8 * N};
  const size_t n = (size_t)nspin * M;
  std::vector<double> rho(n, 0.01), R(n), mu(1), Vext(M, -0.3), Veff(M), range(2);
  char name[160];
  std::snprintf(name, sizeof name, "lrdm_density %s N=%d nspin=%d grid %dx%dx%d", prec_name(prec),
                N, nspin, g.n[0], g.n[1], g.n[2]);
  check(lrdm_density(ctx, &g, Psi.data(), eps.data(), N, &occ, prec, rho.data(), R.data(),
                     mu.data()), ctx, name);
  check(lrdm_effective_potential(ctx, &g, Vext.data(), rho.data(), nspin, nullptr, Veff.data(),
                                 range.data()), ctx, "lrdm_effective_potential");
  lrdm_lowrank_params prm{0.0, r_max, 0.1, 0.5, 1.0, 0};
  std::vector<double> U((size_t)r_max * n), T((size_t)r_max * n), drho(n);
  lrdm_lowrank_info info{};
  std::snprintf(name, sizeof name, "lrdm_lowrank_step %s N=%d nspin=%d r_max=%d", prec_name(prec),
                N, nspin, r_max);
  check(lrdm_lowrank_step(ctx, &g, Psi.data(), eps.data(), N, &occ, prec, R.data(), &prm, 0, nullptr,
                          U.data(), T.data(), drho.data(), rho.data(), &info), ctx, name);
  std::printf("     rank %d s_rel %.3e ||R|| %.3e alpha %.2f\n", info.rank, info.s_rel, info.norm_R,
              info.alpha);
  if (!finite(drho) || info.rank != r_max) {
    std::printf("FAIL lowrank step\n");
    ++failures;
  }
  // accumulate on the kept directions with a changed residual (LRDMA): the kept
  // rows stay, at most two are added, capacity r_max + 2
  {
    lrdm_lowrank_params acc{0.0, r_max + 2, 0.1, 0.5, 1.0, 2};
    std::vector<double> U2((size_t)(r_max + 2) * n), T2((size_t)(r_max + 2) * n);
    std::copy(U.begin(), U.end(), U2.begin());
    std::copy(T.begin(), T.end(), T2.begin());
    std::vector<double> R2(R);
    for (size_t i = 0; i < n; ++i) R2[i] += 0.01 * std::sin(0.37 * (double)i);
    check(lrdm_lowrank_step(ctx, &g, Psi.data(), eps.data(), N, &occ, prec, R2.data(), &acc,
                            r_max, nullptr, U2.data(), T2.data(), drho.data(), nullptr, &info),
          ctx, "lrdm_lowrank_step accumulate");
    std::printf("     accumulated: rank %d added %d s_rel %.3e ||R_lin|| %.3e\n", info.rank,
                info.added, info.s_rel, info.norm_R_lin);
    if (!finite(drho) || info.rank != r_max + 2 || info.added != 2) {
      std::printf("FAIL accumulate step\n");
      ++failures;
    }
    acc.r_add_max = -1;
    check(lrdm_lowrank_step(ctx, &g, Psi.data(), eps.data(), N, &occ, prec, R2.data(), &acc,
                            r_max + 2, nullptr, U2.data(), T2.data(), drho.data(), nullptr, &info),
          ctx, "lrdm_lowrank_step kept fit only");
    if (info.added != 0 || info.rank != r_max + 2) {
      std::printf("FAIL kept-only step\n");
      ++failures;
    }
  }
}

// The autotuner: every candidate split count runs the three contractions, and the
// response keeps its values (to rounding) under the chosen counts.
void scenario_autotune(lrdm_ctx* ctx, lrdm_grid g, int N, int nspin, int r, lrdm_prec prec) {
  const int64_t M = (int64_t)g.n[0] * g.n[1] * g.n[2];
  std::vector<double> Psi0;
  for (int c = 0; c < nspin; ++c) {
    auto P = orthonormal(N, M, 31 + c);
    Psi0.insert(Psi0.end(), P.begin(), P.end());
  }
  Block Psi(Psi0, prec);
  std::vector<double> eps((size_t)nspin * N);
  for (int c = 0; c < nspin; ++c)
    for (int i = 0; i < N; ++i) eps[(size_t)c * N + i] = -1.0 + 1.5 * i / N + 0.001 * c;
  lrdm_occ occ{nspin, 0.02, 0.8 * N};
  auto dV = randv((size_t)r * nspin * M, 5);
  std::vector<double> before(dV.size()), after(dV.size());
  check(density_response(ctx, &g, Psi.data(), eps.data(), N, &occ, dV.data(), r, prec,
                         before.data(), nullptr, nullptr), ctx, "density_response before tuning");
  int32_t splits[3], variants[3];
  double ms[36];
  char name[128];
  std::snprintf(name, sizeof name, "lrdm_autotune %s N=%d nspin=%d r=%d", prec_name(prec), N,
                nspin, r);
  int32_t bp = -1;
  double bp_ms[2];
  check(lrdm_autotune(ctx, &g, N, nspin, r, prec, splits, variants, ms, &bp, bp_ms), ctx, name);
  std::printf("     splits %d %d %d, layouts %d %d %d, back-projection layout %d\n", splits[0],
              splits[1], splits[2], variants[0], variants[1], variants[2], bp);
  check(density_response(ctx, &g, Psi.data(), eps.data(), N, &occ, dV.data(), r, prec,
                         after.data(), nullptr, nullptr), ctx, "density_response after tuning");
  double num = 0, den = 0;
  for (size_t i = 0; i < before.size(); ++i) {
    num += (after[i] - before[i]) * (after[i] - before[i]);
    den += before[i] * before[i];
  }
  const double d = std::sqrt(num / den), tol = prec == LRDM_FP64 ? 1e-13 : 1e-6;
  std::printf("     response change %.2e (bound %.0e)\n", d, tol);
  if (!(d < tol)) ++failures;
}
}  // namespace

int main(int argc, char** argv) {
  const std::string which = argc > 1 ? argv[1] : "all";
  lrdm_ctx* ctx = nullptr;
  check(lrdm_create(&ctx, 0, nullptr, 0), nullptr, "lrdm_create");
  if (which == "all" || which == "small") {
    scenario_response(ctx, grid(20, 18, 13, 0.4), 150, 1, 3);
    scenario_response(ctx, grid(9, 8, 7, 0.5), 40, 2, 2);
    scenario_chfsi(ctx, grid(10, 9, 8, 0.45), 150, 5);
    scenario_chfsi(ctx, grid(12, 12, 12, 0.45), 256, 4);
    scenario_rr_dependent(ctx, grid(10, 9, 8, 0.45), 150, LRDM_FP64);
  }
  if (which == "all" || which == "lp") {
    scenario_response(ctx, grid(20, 18, 13, 0.4), 150, 1, 3, LRDM_FP32);
    scenario_response(ctx, grid(20, 18, 13, 0.4), 150, 1, 3, LRDM_BF16X3);
    scenario_response(ctx, grid(9, 8, 7, 0.5), 40, 2, 2, LRDM_BF16X3);
    // M = 693, not a multiple of 4: the projection takes the register-staged kernel
    scenario_response(ctx, grid(7, 9, 11, 0.5), 70, 1, 2, LRDM_BF16X3);
    scenario_response(ctx, grid(7, 9, 11, 0.5), 70, 2, 1, LRDM_FP32);
    scenario_chfsi(ctx, grid(10, 9, 8, 0.45), 150, 5, LRDM_FP32);
    scenario_chfsi(ctx, grid(12, 12, 12, 0.45), 130, 4, LRDM_BF16X3);
  }
  if (which == "all" || which == "adj") {
    scenario_backward(ctx, grid(20, 18, 13, 0.4), 150, 1, 2, LRDM_FP64);
    scenario_backward(ctx, grid(9, 8, 7, 0.5), 40, 2, 2, LRDM_FP64);
    scenario_backward(ctx, grid(20, 18, 13, 0.4), 150, 1, 2, LRDM_BF16X3);
    scenario_backward(ctx, grid(7, 9, 11, 0.5), 70, 2, 1, LRDM_FP32);
  }
  if (which == "pp") {
    scenario_projection(ctx, grid(8, 8, 8, 0.5), 40, 1, LRDM_FP32);
    scenario_projection(ctx, grid(8, 8, 8, 0.5), 40, 1, LRDM_BF16X3);
  }
  if (which == "all" || which == "rank") {
    scenario_rr_dependent(ctx, grid(10, 9, 8, 0.45), 150, LRDM_FP64);
    scenario_rr_dependent(ctx, grid(7, 9, 11, 0.5), 70, LRDM_FP32);
    // BF16X3 rotations (split operands) on the multi-pass route, M = 693 ragged
    scenario_rr_dependent(ctx, grid(7, 9, 11, 0.5), 70, LRDM_BF16X3);
  }
  if (which == "lprr") {
    scenario_chfsi(ctx, grid(10, 9, 8, 0.45), 150, 5, LRDM_FP32);
    scenario_chfsi(ctx, grid(12, 12, 12, 0.45), 130, 4, LRDM_BF16X3);
  }
  if (which == "all" || which == "lowrank") {
    scenario_lowrank(ctx, grid(7, 9, 11, 0.5), 70, 1, 4, LRDM_FP64);
    scenario_lowrank(ctx, grid(9, 8, 7, 0.5), 40, 2, 3, LRDM_FP32);
    scenario_lowrank(ctx, grid(7, 9, 11, 0.5), 70, 1, 3, LRDM_BF16X3);
    // M a multiple of 8: the projection reads the step's pre-split pieces
    scenario_lowrank(ctx, grid(8, 8, 6, 0.5), 40, 2, 3, LRDM_BF16X3);
  }
  if (which == "all" || which == "tune") {
    scenario_autotune(ctx, grid(20, 18, 13, 0.4), 150, 1, 3, LRDM_FP64);
    scenario_autotune(ctx, grid(16, 16, 12, 0.4), 130, 2, 2, LRDM_BF16X3);
  }
  if (which == "all" || which == "skip") {
    scenario_block_skip(ctx, grid(9, 8, 7, 0.5), 400, 1, 2, LRDM_FP64);
    scenario_block_skip(ctx, grid(8, 8, 8, 0.5), 400, 2, 2, LRDM_FP32);
    scenario_block_skip(ctx, grid(8, 8, 8, 0.5), 400, 1, 3, LRDM_BF16X3);
  }
  if (which == "all" || which == "bz") {
    scenario_response_bz(ctx, grid(9, 8, 7, 0.5), 70, 2, 1, 2, LRDM_FP64);
    scenario_response_bz(ctx, grid(9, 8, 7, 0.5), 70, 3, 2, 1, LRDM_FP32);
    scenario_response_bz(ctx, grid(8, 8, 8, 0.5), 70, 2, 1, 2, LRDM_BF16X3);
  }
  if (which == "all" || which == "kpt") {
    scenario_rr_bloch(ctx, grid(10, 9, 8, 0.45), 150, 5);
    // 4N > M: the overlap product of the pairing has more rows than points
    scenario_rr_bloch(ctx, grid(7, 9, 11, 0.5), 200, 4);
    scenario_rr_bloch_degenerate(ctx);
    scenario_rr_bloch_fp32(ctx, grid(9, 8, 7, 0.5), 60);
  }
  if (which == "all" || which == "batched") {
    scenario_batched(ctx, LRDM_FP32);
    scenario_batched(ctx, LRDM_FP64);
  }
  if (which == "all" || which == "full") scenario_full_n(ctx);
  check(lrdm_destroy(ctx), nullptr, "lrdm_destroy");
  std::printf(failures ? "EMU FAIL (%d)\n" : "EMU OK\n", failures);
  return failures ? 1 : 0;
}

// Host-side argument validation for the C ABI.  No HIP calls: every check here
// runs before a launch and before the context is touched.
#include <cmath>
#include <cstdint>

#include "lrdm.h"

namespace lrdm {

const char* check_grid(const lrdm_grid* g) {
  if (!g) return "grid is NULL";
  for (int d = 0; d < 3; ++d) {
    if (g->n[d] < 3) return "grid: every n[d] must be >= 3";
    if (g->n[d] > 4096) return "grid: n[d] must be <= 4096";
    if (!std::isfinite(g->L[d]) || g->L[d] <= 0.0) return "grid: every L[d] must be finite and > 0";
  }
  if ((int64_t)g->n[0] * g->n[1] > 8192)
    return "grid: an xy plane may hold at most 8192 points (nx * ny <= 8192)";
  return nullptr;
}

const char* check_block(const lrdm_grid* g, int32_t N) {
  if (N < 1) return "N must be >= 1";
  const int64_t M = (int64_t)g->n[0] * g->n[1] * g->n[2];
  if (N > M) return "N must not exceed the number of grid points M";
  if (N > 8192) return "N must be <= 8192";
  return nullptr;
}

// Eq. (14) asks for N > N_e / 2 states (capacity 2 per state); with two
// channels each state holds 1 electron per channel, so N_e < 2 N in both cases.
const char* check_occ(const lrdm_occ* occ, int32_t N) {
  if (!occ) return "occ is NULL";
  if (occ->nspin != 1 && occ->nspin != 2) return "occ: nspin must be 1 or 2";
  if (!std::isfinite(occ->kT) || occ->kT <= 0.0) return "occ: kT must be finite and > 0";
  if (!std::isfinite(occ->n_electrons) || occ->n_electrons <= 0.0)
    return "occ: n_electrons must be finite and > 0";
  const double capacity = 2.0 * (double)N;
  if (occ->n_electrons >= capacity)
    return "occ: n_electrons must be below 2 N (N > N_e/2 states, Eq. (14))";
  return nullptr;
}

const char* check_prec(int prec) {
  if (prec != LRDM_FP64 && prec != LRDM_FP32 && prec != LRDM_BF16X3)
    return "prec must be LRDM_FP64, LRDM_FP32 or LRDM_BF16X3";
  return nullptr;
}

const char* check_rank(int32_t r) {
  if (r < 1) return "r (number of directions) must be >= 1";
  if (r > 4096) return "r must be <= 4096";
  return nullptr;
}

const char* check_lowrank(const lrdm_lowrank_params* p) {
  if (!p) return "params is NULL";
  if (!std::isfinite(p->s_tol) || p->s_tol < 0.0) return "params: s_tol must be finite and >= 0";
  if (p->r_max < 1 || p->r_max > 64) return "params: r_max must be in 1..64";
  if (!std::isfinite(p->alpha_far) || !(p->alpha_far > 0.0 && p->alpha_far <= 1.0))
    return "params: alpha_far must be in (0, 1]";
  if (!std::isfinite(p->alpha_near) || !(p->alpha_near > 0.0 && p->alpha_near <= 1.0))
    return "params: alpha_near must be in (0, 1]";
  if (std::isnan(p->alpha_switch) || p->alpha_switch < 0.0)
    return "params: alpha_switch must be >= 0 (+inf allowed)";
  if (p->r_add_max < -1 || p->r_add_max > 64) return "params: r_add_max must be in -1..64";
  return nullptr;
}

const char* check_filter(int32_t degree, double a, double b, double a0) {
  if (degree < 1) return "degree must be >= 1";
  if (degree > 10000) return "degree must be <= 10000";
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(a0))
    return "filter bounds a, b, a0 must be finite";
  if (!(a0 < a && a < b)) return "filter bounds must satisfy a0 < a < b";
  return nullptr;
}

const char* check_ptr(const void* p, const char* name) {
  (void)name;
  return p ? nullptr : "a required array pointer is NULL";
}

}  // namespace lrdm

// extern "C" entry points of liblrdm (declared in include/lrdm.h): argument
// validation, workspace sizing and the sequence of kernel launches of each call.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>

#include "lrdm_internal.h"

namespace {

thread_local std::string t_err;

lrdm_status fail(lrdm_ctx* ctx, lrdm_status st, const std::string& msg) {
  t_err = msg;
  if (ctx) ctx->err = msg;
  return st;
}

lrdm_status fail_hip(lrdm_ctx* ctx, const char* where, hipError_t e) {
  return fail(ctx, LRDM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

struct WsOverflow : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define LRDM_CHECK(ctx, expr)                                  \
  do {                                                         \
    const char* m_ = (expr);                                   \
    if (m_) return fail((ctx), LRDM_EINVAL, m_);               \
  } while (0)

#define LRDM_NONNULL(ctx, p, name)                                              \
  do {                                                                          \
    if (!(p)) return fail((ctx), LRDM_EINVAL, std::string(name) + " is NULL");  \
  } while (0)

// Common prologue once arguments are valid: the context must exist, its device
// becomes current and the workspace holds `bytes`.
lrdm_status begin(lrdm_ctx* ctx, size_t bytes) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail_hip(ctx, "hipSetDevice", e);
  ctx->ws_top = 0;
  return lrdm::ws_reserve(ctx, bytes + (1u << 20));
}

// Epilogue: in checking mode wait for the stream and turn device status words
// into status codes.
lrdm_status finish(lrdm_ctx* ctx, lrdm_status st) {
  if (st != LRDM_OK || !ctx->checks) return st;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail_hip(ctx, "hipStreamSynchronize", e);
  int h[LRDM_DS_COUNT] = {0, 0, 0, 0};
  e = hipMemcpy(h, ctx->dstatus, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(ctx, "status read", e);
  e = hipMemset(ctx->dstatus, 0, sizeof(h));
  if (e != hipSuccess) return fail_hip(ctx, "status reset", e);
  if (h[LRDM_DS_BISECT]) return fail(ctx, LRDM_ENOTCONV, "Fermi-level bisection did not converge");
  if (h[LRDM_DS_EIGH]) return fail(ctx, LRDM_ENOTCONV, "subspace eigensolver did not converge");
  if (h[LRDM_DS_NONFINITE]) return fail(ctx, LRDM_ENONFINITE, "non-finite value in an output");
  return LRDM_OK;
}

template <typename F>
lrdm_status guarded(lrdm_ctx* ctx, F&& body) {
  try {
    return finish(ctx, body());
  } catch (const WsOverflow& ex) {
    return fail(ctx, LRDM_ENOMEM, ex.what());
  } catch (const std::bad_alloc&) {
    return fail(ctx, LRDM_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(ctx, LRDM_EDEVICE, "unexpected internal error");
  }
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

namespace lrdm {

Grid3 make_grid3(const lrdm_grid* g) {
  Grid3 r;
  r.nx = g->n[0];
  r.ny = g->n[1];
  r.nz = g->n[2];
  r.hx = g->L[0] / g->n[0];
  r.hy = g->L[1] / g->n[1];
  r.hz = g->L[2] / g->n[2];
  r.M = (int64_t)r.nx * r.ny * r.nz;
  r.dv = r.hx * r.hy * r.hz;
  return r;
}

lrdm_status ws_reserve(lrdm_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_cap) return LRDM_OK;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx->stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
    return fail(ctx, LRDM_ENOMEM,
                "the workspace would have to grow during stream capture: make the same call once "
                "before capturing");
  if (ctx->limit && bytes > ctx->limit) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "workspace of %zu bytes exceeds the context limit of %zu", bytes,
                  ctx->limit);
    return fail(ctx, LRDM_ENOMEM, msg);
  }
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail_hip(ctx, "hipStreamSynchronize", e);
  if (ctx->ws) {
    e = hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
    if (e != hipSuccess) return fail_hip(ctx, "hipFree", e);
  }
  e = hipMalloc(&ctx->ws, bytes);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    return fail(ctx, LRDM_ENOMEM, std::string("hipMalloc of workspace: ") + hipGetErrorString(e));
  }
  ctx->ws_cap = bytes;
  return LRDM_OK;
}

void* ws_take(lrdm_ctx* ctx, size_t bytes) {
  const size_t b = ws_align(bytes);
  if (ctx->ws_top + b > ctx->ws_cap) throw WsOverflow("internal workspace sizing error");
  void* p = static_cast<char*>(ctx->ws) + ctx->ws_top;
  ctx->ws_top += b;
  return p;
}

static hipEvent_t pool_event(lrdm_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(lrdm_ctx* ctx, const char* name) : ctx_(ctx), name_(name) {
  if (!ctx_->profiling) return;
  start_ = pool_event(ctx_);
  if (start_ && hipEventRecord(start_, ctx_->stream) != hipSuccess) {
    ctx_->event_pool.push_back(start_);
    start_ = nullptr;
  }
}

ProfScope::~ProfScope() {
  if (!start_) return;
  hipEvent_t stop = pool_event(ctx_);
  if (!stop || hipEventRecord(stop, ctx_->stream) != hipSuccess) {
    ctx_->event_pool.push_back(start_);
    if (stop) ctx_->event_pool.push_back(stop);
    return;
  }
  ctx_->prof.push_back({name_, start_, stop});
}

size_t tn_bytes(int N, int64_t M, int batch, lrdm_prec prec, int split_limit = 0) {
  return tn_workspace_bytes(N, M, batch, prec, split_limit);
}

}  // namespace lrdm

using namespace lrdm;

// ===================================================================== context

extern "C" lrdm_status lrdm_create(lrdm_ctx** ctx, int device, void* hip_stream,
                                   size_t workspace_limit) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx output pointer is NULL");
  *ctx = nullptr;
  if (device < 0) return fail(nullptr, LRDM_EINVAL, "device must be >= 0");
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return fail_hip(nullptr, "hipSetDevice", e);
  lrdm_ctx* c = new (std::nothrow) lrdm_ctx();
  if (!c) return fail(nullptr, LRDM_ENOMEM, "host allocation failed");
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->limit = workspace_limit;
  e = hipMalloc(&c->dstatus, 64 * sizeof(int));
  if (e != hipSuccess) {
    delete c;
    return fail_hip(nullptr, "hipMalloc status", e);
  }
  e = hipMemset(c->dstatus, 0, 64 * sizeof(int));
  if (e != hipSuccess) {
    (void)hipFree(c->dstatus);
    delete c;
    return fail_hip(nullptr, "hipMemset status", e);
  }
  c->zeros = reinterpret_cast<const float*>(c->dstatus + 32);
  {
    // the allocation-free entry point's scratch address on this device, looked up
    // once per device at set-up (a failure is reported by that entry point)
    void* scratch = nullptr;
    (void)noalloc_scratch(device, &scratch);
  }
  for (int k = 0; k < kAuxStreams; ++k) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) break;
    c->aux.push_back(st);
  }
  for (int k = 0; e == hipSuccess && k <= kAuxStreams; ++k) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) c->fork_join.push_back(ev);
  }
  if (e != hipSuccess) {
    for (hipStream_t st : c->aux) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : c->fork_join) (void)hipEventDestroy(ev);
    (void)hipFree(c->dstatus);
    delete c;
    return fail_hip(nullptr, "stream/event creation", e);
  }
  *ctx = c;
  return LRDM_OK;
}

extern "C" lrdm_status lrdm_destroy(lrdm_ctx* ctx) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  for (hipStream_t st : ctx->aux) {
    const hipError_t ea = hipStreamSynchronize(st);
    if (e == hipSuccess) e = ea;
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t ev : ctx->fork_join) (void)hipEventDestroy(ev);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->dstatus) (void)hipFree(ctx->dstatus);
  for (const lrdm_prof_rec& r : ctx->prof) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (hipEvent_t ev : ctx->event_pool) (void)hipEventDestroy(ev);
  delete ctx;
  if (e != hipSuccess) return fail_hip(nullptr, "hipStreamSynchronize", e);
  return LRDM_OK;
}

extern "C" lrdm_status lrdm_set_stream(lrdm_ctx* ctx, void* hip_stream) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return LRDM_OK;
}

extern "C" lrdm_status lrdm_set_checks(lrdm_ctx* ctx, int level) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  if (level < 0 || level > 1) return fail(ctx, LRDM_EINVAL, "checks level must be 0 or 1");
  ctx->checks = level;
  return LRDM_OK;
}

extern "C" lrdm_status lrdm_set_fermi_expansion(lrdm_ctx* ctx, int32_t depth) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  if (depth < 0 || depth > 64) return fail(ctx, LRDM_EINVAL, "depth must be in 0..64");
  ctx->fermi_depth = depth;
  return LRDM_OK;
}

extern "C" lrdm_status lrdm_set_eigensolver_sweeps(lrdm_ctx* ctx, int32_t max_sweeps) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  if (max_sweeps < 1 || max_sweeps > 1000)
    return fail(ctx, LRDM_EINVAL, "max_sweeps must be in 1..1000");
  ctx->eigh_max_sweeps = max_sweeps;
  return LRDM_OK;
}

extern "C" lrdm_status lrdm_set_response_block_skip(lrdm_ctx* ctx, double tau) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  if (!(tau >= 0.0 && tau < 1.0)) return fail(ctx, LRDM_EINVAL, "tau must be in [0, 1)");
  ctx->block_tau = tau;
  return LRDM_OK;
}

extern "C" lrdm_status lrdm_set_backproj_layout(lrdm_ctx* ctx, int32_t layout) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  if (layout != BP_VAR_NARROW && layout != BP_VAR_WIDE)
    return fail(ctx, LRDM_EINVAL, "layout must be 0 (128 points) or 1 (256 points)");
  ctx->bp_variant = layout;
  return LRDM_OK;
}

extern "C" size_t lrdm_workspace_bytes(const lrdm_ctx* ctx) { return ctx ? ctx->ws_cap : 0; }

extern "C" lrdm_status lrdm_profile(lrdm_ctx* ctx, int enable) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  ctx->profiling = enable != 0;
  return LRDM_OK;
}

extern "C" lrdm_status lrdm_profile_read(lrdm_ctx* ctx, const char* kernel, double* ms,
                                         int64_t* launches) {
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  if (!kernel || !ms || !launches) return fail(ctx, LRDM_EINVAL, "kernel, ms and launches must be non-NULL");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail_hip(ctx, "hipStreamSynchronize", e);
  double total = 0.0;
  int64_t count = 0;
  std::vector<lrdm_prof_rec> keep;
  for (const lrdm_prof_rec& r : ctx->prof) {
    if (std::strcmp(r.name, kernel) != 0) {
      keep.push_back(r);
      continue;
    }
    float t = 0.f;
    e = hipEventElapsedTime(&t, r.start, r.stop);
    if (e != hipSuccess) return fail_hip(ctx, "hipEventElapsedTime", e);
    total += t;
    ++count;
    ctx->event_pool.push_back(r.start);
    ctx->event_pool.push_back(r.stop);
  }
  ctx->prof.swap(keep);
  *ms = total;
  *launches = count;
  return LRDM_OK;
}

extern "C" const char* lrdm_last_error(const lrdm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : t_err.c_str();
}

// ===================================================================== single steps

extern "C" lrdm_status lrdm_hamiltonian_apply(lrdm_ctx* ctx, const lrdm_grid* grid,
                                              const double* V, const void* X, void* Y, int32_t N,
                                              lrdm_prec prec) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_NONNULL(ctx, V, "V");
  LRDM_NONNULL(ctx, X, "X");
  LRDM_NONNULL(ctx, Y, "Y");
  const Grid3 g = make_grid3(grid);
  const size_t blk = (size_t)g.M * N * prec_bytes(prec);
  if (overlaps(X, blk, Y, blk)) return fail(ctx, LRDM_EINVAL, "X and Y must not overlap");
  lrdm_status st = begin(ctx, 0);
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e = (prec == LRDM_FP64)
        ? launch_cheb_step<double>(ctx, g, V, static_cast<const double*>(X), nullptr,
                                   static_cast<double*>(Y), N, 1.0, 0.0, 0.0)
        : launch_cheb_step<float>(ctx, g, V, static_cast<const float*>(X), nullptr,
                                  static_cast<float*>(Y), N, 1.0, 0.0, 0.0);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "hamiltonian_apply", e);
  });
}

extern "C" lrdm_status lrdm_fermi_occupations(lrdm_ctx* ctx, const double* eps, int32_t N,
                                              const lrdm_occ* occ, double* mu, double* f,
                                              double* fprime, double* F) {
  if (N < 1 || N > 8192) return fail(ctx, LRDM_EINVAL, "N must be in [1, 8192]");
  LRDM_CHECK(ctx, check_occ(occ, N));
  LRDM_NONNULL(ctx, eps, "eps");
  const int ns = occ->nspin;
  const size_t vec = (size_t)ns * N * sizeof(double);
  lrdm_status st = begin(ctx, 4 * ws_align(vec) + ws_align(8));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    double* mu_d = mu ? mu : static_cast<double*>(ws_take(ctx, 8));
    double* f_d = f ? f : static_cast<double*>(ws_take(ctx, vec));
    double* o_d = static_cast<double*>(ws_take(ctx, vec));
    double* fp_d = fprime ? fprime : static_cast<double*>(ws_take(ctx, vec));
    hipError_t e = launch_fermi(ctx, eps, N, ns, occ->kT, occ->n_electrons, mu_d, f_d, o_d, fp_d, F);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "fermi_occupations", e);
  });
}

extern "C" lrdm_status lrdm_projected_perturbation(lrdm_ctx* ctx, const lrdm_grid* grid,
                                                   const void* Psi, int32_t N, int32_t nspin,
                                                   const double* dV, int32_t r, lrdm_prec prec,
                                                   double* Hp) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_rank(r));
  LRDM_CHECK(ctx, check_prec(prec));
  if (nspin != 1 && nspin != 2) return fail(ctx, LRDM_EINVAL, "nspin must be 1 or 2");
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, dV, "dV");
  LRDM_NONNULL(ctx, Hp, "Hp");
  const Grid3 g = make_grid3(grid);
  lrdm_status st = begin(ctx, tn_bytes(N, g.M, r * nspin, prec));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e;
    if (prec == LRDM_FP64)
      e = launch_tn_sym<double>(ctx, static_cast<const double*>(Psi), nullptr, dV, g.M, N, g.M,
                                nspin, r * nspin, prec, Hp);
    else
      e = launch_tn_sym<float>(ctx, static_cast<const float*>(Psi), nullptr, dV, g.M, N, g.M,
                               nspin, r * nspin, prec, Hp);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "projected_perturbation", e);
  });
}

extern "C" lrdm_status lrdm_hartree_kernel(lrdm_ctx* ctx, const lrdm_grid* grid, const double* u,
                                           double* dV, int32_t r) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_rank(r));
  LRDM_NONNULL(ctx, u, "u");
  LRDM_NONNULL(ctx, dV, "dV");
  const Grid3 g = make_grid3(grid);
  const size_t scratch = 2 * (size_t)r * g.M * sizeof(double);
  lrdm_status st = begin(ctx, ws_align(scratch) + hartree_workspace_bytes(g));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    double* s = static_cast<double*>(ws_take(ctx, scratch));
    hipError_t e = launch_hartree(ctx, g, u, 1, dV, 1, r, s);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "hartree_kernel", e);
  });
}

// ===================================================================== hot path

namespace {

template <typename T>
hipError_t run_filter(lrdm_ctx* ctx, const Grid3& g, const double* V, const T* X, T* Y, int N,
                      int degree, double a, double b, double a0) {
  T* W = static_cast<T*>(ws_take(ctx, (size_t)g.M * N * sizeof(T)));
  const double e = (b - a) / 2.0, c0 = (b + a) / 2.0;
  const double sigma1 = e / (a0 - c0);
  // the vectorised step reads V in the storage type
  auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const bool vec = cheb_vec_ok<T>(g) && aligned(X) && aligned(Y) && aligned(W);
  const T* Vt = nullptr;
  if (vec) {
    if constexpr (sizeof(T) == sizeof(double)) {
      Vt = V;
    } else {
      float* Vf = static_cast<float*>(ws_take(ctx, (size_t)g.M * sizeof(float)));
      LRDM_HIP(launch_to_float(ctx, V, g.M, Vf));
      Vt = Vf;
    }
  }
  auto step = [&](const T* yin, const T* yold, T* yout, double alpha, double beta) {
    return vec ? launch_cheb_step_vec<T>(ctx, g, Vt, yin, yold, yout, N, alpha, c0, beta)
               : launch_cheb_step<T>(ctx, g, V, yin, yold, yout, N, alpha, c0, beta);
  };
  // Y_k lands in bufA for odd k and bufB for even k; choose so that Y_c is in Y.
  T* bufA = (degree % 2 == 1) ? Y : W;
  T* bufB = (degree % 2 == 1) ? W : Y;
  LRDM_HIP(step(X, nullptr, bufA, sigma1 / e, 0.0));
  // steps k .. k+2 (or k, k+1) in one sweep where the vectorised form can own
  // whole z columns
  const bool pair = vec && cheb_pair_ok<T>(g, N);
  const bool triple = vec && cheb_triple_ok<T>(g, N);
  double sigma = sigma1;
  for (int k = 2; k <= degree;) {
    T* ykm1 = (k % 2 == 0) ? bufA : bufB;         // Y_{k-1}
    const T* ykm2 = (k == 2) ? X : ((k % 2 == 0) ? bufB : bufA);  // Y_{k-2}
    T* out = (k % 2 == 1) ? bufA : bufB;          // overwrites Y_{k-2} (k > 2)
    const double s1 = 1.0 / (2.0 / sigma1 - sigma);
    if (triple && k + 2 <= degree) {
      const double s2 = 1.0 / (2.0 / sigma1 - s1);
      const double s3 = 1.0 / (2.0 / sigma1 - s2);
      const double a[3] = {2.0 * s1 / e, 2.0 * s2 / e, 2.0 * s3 / e};
      const double b[3] = {-sigma * s1, -s1 * s2, -s2 * s3};
      // Y_{k+1} overwrites Y_{k-1}, Y_{k+2} overwrites Y_{k-2}; Y_k stays on chip
      LRDM_HIP(launch_cheb_triple_vec<T>(ctx, g, Vt, ykm2, ykm1, ykm1, out, N, c0, a, b));
      sigma = s3;
      k += 3;
    } else if (pair && k + 1 <= degree) {
      const double s2 = 1.0 / (2.0 / sigma1 - s1);
      // Y_{k+1} overwrites Y_{k-1}
      LRDM_HIP(launch_cheb_pair_vec<T>(ctx, g, Vt, ykm2, ykm1, out, ykm1, N, c0,
                                       2.0 * s1 / e, -sigma * s1, 2.0 * s2 / e, -s1 * s2));
      sigma = s2;
      k += 2;
    } else {
      LRDM_HIP(step(ykm1, ykm2, out, 2.0 * s1 / e, -sigma * s1));
      sigma = s1;
      k += 1;
    }
  }
  return hipSuccess;
}

// The Fermi-level quantities a response needs: mu, f, 1 - f, the multiplier's
// diagonal fp (f', or the recursive expansion's) and the multiplier F.
struct FermiState {
  double* mu;
  double* f;
  double* omf;
  double* fp;
  double* F;
  unsigned char* active;   // the response's block mask (blocks.h), NULL: every block
};

size_t block_mask_bytes(int N, int ns) {
  const size_t ntb = (size_t)(N + 127) / 128;
  return ws_align(ns * ntb * ntb * sizeof(double)) + ws_align(ns * ntb * ntb);
}

// mu by bisection, the occupations and the multiplier (exact divided differences,
// or with the recursive expansion its multiplier and diagonal in the places of F
// and f' in Gamma = F o H' - mu' diag(f') and in mu').  mu_out: where mu goes
// (NULL: into the workspace).
hipError_t run_fermi(lrdm_ctx* ctx, const double* eps, int N, const lrdm_occ* occ,
                     double* mu_out, FermiState* st) {
  const int ns = occ->nspin;
  const size_t vec = (size_t)ns * N * sizeof(double);
  st->mu = mu_out ? mu_out : static_cast<double*>(ws_take(ctx, 8));
  st->f = static_cast<double*>(ws_take(ctx, vec));
  st->omf = static_cast<double*>(ws_take(ctx, vec));
  st->fp = static_cast<double*>(ws_take(ctx, vec));
  st->F = static_cast<double*>(ws_take(ctx, (size_t)ns * N * N * sizeof(double)));
  const int depth = ctx->fermi_depth;
  LRDM_HIP(launch_fermi(ctx, eps, N, ns, occ->kT, occ->n_electrons, st->mu, st->f, st->omf,
                        st->fp, depth > 0 ? nullptr : st->F));
  if (depth > 0)
    LRDM_HIP(launch_recursive_multiplier(ctx, eps, st->mu, N, ns, occ->kT, depth, st->F, st->fp));
  st->active = nullptr;
  if (ctx->block_tau > 0.0 && N > 128) {
    const size_t ntb = (size_t)(N + 127) / 128;
    double* tmax = static_cast<double*>(ws_take(ctx, ns * ntb * ntb * sizeof(double)));
    st->active = static_cast<unsigned char*>(ws_take(ctx, ns * ntb * ntb));
    LRDM_HIP(launch_block_mask(ctx, st->F, N, ns, ctx->block_tau, tmax, st->active));
  }
  return hipSuccess;
}

// Shared body of density_response and lrdm_residual_derivative.  fermi: the
// Fermi quantities of these eps when the caller already has them (NULL: formed
// here, mu into `mu` when given).
template <typename T>
hipError_t run_response(lrdm_ctx* ctx, const Grid3& g, const T* Psi, const double* eps, int N,
                        const lrdm_occ* occ, const double* dV, int r, lrdm_prec prec,
                        const double* sub, double* out, double* mu, double* dmu,
                        const FermiState* fermi = nullptr) {
  const int ns = occ->nspin;
  const int batch = r * ns;
  double* dmu_d = dmu ? dmu : static_cast<double*>(ws_take(ctx, (size_t)r * 8));
  FermiState local;
  if (!fermi) {
    LRDM_HIP(run_fermi(ctx, eps, N, occ, mu, &local));
    fermi = &local;
  }
  double* fp = fermi->fp;
  double* F = fermi->F;
  double* Hp = static_cast<double*>(ws_take(ctx, (size_t)batch * N * N * sizeof(double)));
  LRDM_HIP(launch_tn_sym<T>(ctx, Psi, nullptr, dV, g.M, N, g.M, ns, batch, prec, Hp,
                            fermi->active));
  LRDM_HIP(launch_gamma(ctx, Hp, F, fp, N, ns, r, dmu_d));
  const double s = (ns == 1) ? 2.0 : 1.0;
  LRDM_HIP(launch_backproj<T>(ctx, Psi, Hp, N, g.M, ns, batch, prec, s / g.dv, sub, out,
                              fermi->active));
  if (ctx->checks) LRDM_HIP(launch_check_finite(ctx, out, (int64_t)batch * g.M));
  return hipSuccess;
}

// Adjoint of run_response (see density_response_backward in lrdm.h).
template <typename T>
hipError_t run_backward(lrdm_ctx* ctx, const Grid3& g, const T* Psi, const double* eps, int N,
                        const lrdm_occ* occ, const double* dV, int r, lrdm_prec prec,
                        const double* gd, double* g_dV, T* g_Psi, double* g_eps) {
  const int ns = occ->nspin;
  const int batch = r * ns;
  const size_t vec = (size_t)ns * N * sizeof(double);
  const size_t mat = (size_t)batch * N * N * sizeof(double);
  double* mu = static_cast<double*>(ws_take(ctx, 8));
  double* dmu = static_cast<double*>(ws_take(ctx, (size_t)r * 8));
  double* nu = static_cast<double*>(ws_take(ctx, (size_t)r * 8));
  double* f = static_cast<double*>(ws_take(ctx, vec));
  double* omf = static_cast<double*>(ws_take(ctx, vec));
  double* fp = static_cast<double*>(ws_take(ctx, vec));
  double* part = static_cast<double*>(ws_take(ctx, vec));
  double* F = static_cast<double*>(ws_take(ctx, (size_t)ns * N * N * sizeof(double)));
  double* Hp = static_cast<double*>(ws_take(ctx, mat));
  double* A = static_cast<double*>(ws_take(ctx, mat));
  double* Gm = static_cast<double*>(ws_take(ctx, mat));
  double* dH = static_cast<double*>(ws_take(ctx, mat));
  double* gs = static_cast<double*>(ws_take(ctx, (size_t)batch * g.M * sizeof(double)));
  const double c = ((ns == 1) ? 2.0 : 1.0) / g.dv;
  LRDM_HIP(launch_fermi(ctx, eps, N, ns, occ->kT, occ->n_electrons, mu, f, omf, fp, F));
  // the forward's block mask (blocks.h): the adjoint is that of the same map
  unsigned char* active = nullptr;
  if (ctx->block_tau > 0.0 && N > 128) {
    const size_t ntb = (size_t)(N + 127) / 128;
    double* tmax = static_cast<double*>(ws_take(ctx, ns * ntb * ntb * sizeof(double)));
    active = static_cast<unsigned char*>(ws_take(ctx, ns * ntb * ntb));
    LRDM_HIP(launch_block_mask(ctx, F, N, ns, ctx->block_tau, tmax, active));
  }
  const size_t mark = ctx->ws_top;
  // H' and A = (s/dv) Psi diag(g) Psi^T (recomputed; nothing of the forward call is kept)
  LRDM_HIP(launch_tn_sym<T>(ctx, Psi, nullptr, dV, g.M, N, g.M, ns, batch, prec, Hp, active));
  ctx->ws_top = mark;
  LRDM_HIP(launch_scale(ctx, gd, c, (int64_t)batch * g.M, gs));
  LRDM_HIP(launch_tn_sym<T>(ctx, Psi, nullptr, gs, g.M, N, g.M, ns, batch, prec, A, active));
  ctx->ws_top = mark;
  // Gamma and dH' = F o A - nu diag(f'): the same map applied to copies
  LRDM_HIP(hipMemcpyAsync(Gm, Hp, mat, hipMemcpyDeviceToDevice, ctx->stream));
  LRDM_HIP(launch_gamma(ctx, Gm, F, fp, N, ns, r, dmu));
  LRDM_HIP(hipMemcpyAsync(dH, A, mat, hipMemcpyDeviceToDevice, ctx->stream));
  LRDM_HIP(launch_gamma(ctx, dH, F, fp, N, ns, r, nu));
  if (g_dV) {
    LRDM_HIP(launch_backproj<T>(ctx, Psi, dH, N, g.M, ns, batch, prec, 1.0, nullptr, g_dV,
                                active));
    ctx->ws_top = mark;
  }
  if (g_Psi) {
    bool done = false;
    if constexpr (sizeof(T) == sizeof(float)) {
      if (prec == LRDM_BF16X3) {
        LRDM_HIP(launch_adj_psi_bf16x3(ctx, Gm, gs, dH, dV, r, Psi, N, g.M, ns, 2.0, g_Psi,
                                       active));
        done = true;
      }
    }
    if (!done)
      LRDM_HIP(launch_adj_psi<T>(ctx, Gm, gs, dH, dV, r, Psi, N, g.M, ns, 2.0, g_Psi, active));
  }
  if (g_eps)
    LRDM_HIP(launch_adj_eps(ctx, A, Hp, eps, F, f, omf, fp, dmu, nu, N, ns, r, occ->kT, part,
                            g_eps));
  if (ctx->checks) {
    if (g_dV) LRDM_HIP(launch_check_finite(ctx, g_dV, (int64_t)batch * g.M));
    if (g_eps) LRDM_HIP(launch_check_finite(ctx, g_eps, (int64_t)ns * N));
  }
  return hipSuccess;
}

size_t backward_bytes(int N, int64_t M, int r, int ns, lrdm_prec prec) {
  const int batch = r * ns;
  const size_t scratch = std::max({tn_bytes(N, M, batch, prec),
                                   backproj_workspace_bytes(N, M, ns, batch, prec),
                                   adj_psi_workspace_bytes(N, M, ns, r, prec != LRDM_FP64),
                                   prec == LRDM_BF16X3 ? adj_psi_bf16x3_bytes(N, M, ns, r)
                                                       : size_t(0)});
  return ws_align(8) + 2 * ws_align((size_t)r * 8) + 4 * ws_align((size_t)ns * N * 8) +
         block_mask_bytes(N, ns) +
         ws_align((size_t)ns * N * N * 8) + 4 * ws_align((size_t)batch * N * N * 8) +
         ws_align((size_t)batch * M * 8) + ws_align(scratch) + 4096;
}

size_t response_bytes(int N, int64_t M, int r, int ns, lrdm_prec prec, int split_limit = 0) {
  const int batch = r * ns;
  return ws_align(8) + ws_align((size_t)r * 8) + 3 * ws_align((size_t)ns * N * 8) +
         block_mask_bytes(N, ns) +
         ws_align((size_t)ns * N * N * 8) + ws_align((size_t)batch * N * N * 8) +
         ws_align(tn_bytes(N, M, batch, prec, split_limit)) +
         backproj_workspace_bytes(N, M, ns, batch, prec);
}

}  // namespace

extern "C" lrdm_status chfsi_filter(lrdm_ctx* ctx, const lrdm_grid* grid, const double* V,
                                    const void* X, void* Y, int32_t N, lrdm_prec prec,
                                    int32_t degree, double a, double b, double a0) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_CHECK(ctx, check_filter(degree, a, b, a0));
  LRDM_NONNULL(ctx, V, "V");
  LRDM_NONNULL(ctx, X, "X");
  LRDM_NONNULL(ctx, Y, "Y");
  const Grid3 g = make_grid3(grid);
  const size_t blk = (size_t)g.M * N * prec_bytes(prec);
  if (overlaps(X, blk, Y, blk)) return fail(ctx, LRDM_EINVAL, "X and Y must not overlap");
  lrdm_status st = begin(ctx, ws_align(blk) + ws_align((size_t)g.M * sizeof(float)));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e = (prec == LRDM_FP64)
        ? run_filter<double>(ctx, g, V, static_cast<const double*>(X), static_cast<double*>(Y), N,
                             degree, a, b, a0)
        : run_filter<float>(ctx, g, V, static_cast<const float*>(X), static_cast<float*>(Y), N,
                            degree, a, b, a0);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "chfsi_filter", e);
  });
}

namespace {

// The filter of run_filter with the Bloch Hamiltonian of kvec on blocks of N
// complex states [2][N][M]: Y_k lands in bufA for odd k and bufB for even k, so
// that Y_c is in Y; Y_k overwrites Y_{k-2} in place.
template <typename T>
hipError_t run_filter_bloch(lrdm_ctx* ctx, const Grid3& g, const double* V, const double kvec[3],
                            const T* X, T* Y, int N, int degree, double a, double b, double a0) {
  T* W = static_cast<T*>(ws_take(ctx, (size_t)2 * g.M * N * sizeof(T)));
  const double e = (b - a) / 2.0, c0 = (b + a) / 2.0;
  const double sigma1 = e / (a0 - c0);
  T* bufA = (degree % 2 == 1) ? Y : W;
  T* bufB = (degree % 2 == 1) ? W : Y;
  LRDM_HIP(launch_bloch_step<T>(ctx, g, V, kvec, X, nullptr, bufA, N, sigma1 / e, c0, 0.0));
  double sigma = sigma1;
  for (int k = 2; k <= degree; ++k) {
    const T* ykm1 = (k % 2 == 0) ? bufA : bufB;
    const T* ykm2 = (k == 2) ? X : ((k % 2 == 0) ? bufB : bufA);
    T* out = (k % 2 == 1) ? bufA : bufB;
    const double s1 = 1.0 / (2.0 / sigma1 - sigma);
    LRDM_HIP(launch_bloch_step<T>(ctx, g, V, kvec, ykm1, ykm2, out, N, 2.0 * s1 / e, c0,
                                  -sigma * s1));
    sigma = s1;
  }
  return hipSuccess;
}

const char* check_kvec(double kx, double ky, double kz) {
  if (!std::isfinite(kx) || !std::isfinite(ky) || !std::isfinite(kz))
    return "k must be finite";
  return nullptr;
}

}  // namespace

extern "C" lrdm_status lrdm_bloch_hamiltonian_apply(lrdm_ctx* ctx, const lrdm_grid* grid,
                                                    const double* V, double kx, double ky,
                                                    double kz, const void* X, void* Y, int32_t N,
                                                    lrdm_prec prec) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_CHECK(ctx, check_kvec(kx, ky, kz));
  LRDM_NONNULL(ctx, V, "V");
  LRDM_NONNULL(ctx, X, "X");
  LRDM_NONNULL(ctx, Y, "Y");
  const Grid3 g = make_grid3(grid);
  const size_t blk = (size_t)2 * g.M * N * prec_bytes(prec);
  if (overlaps(X, blk, Y, blk)) return fail(ctx, LRDM_EINVAL, "X and Y must not overlap");
  lrdm_status st = begin(ctx, 0);
  if (st != LRDM_OK) return st;
  const double kvec[3] = {kx, ky, kz};
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e = (prec == LRDM_FP64)
        ? launch_bloch_step<double>(ctx, g, V, kvec, static_cast<const double*>(X), nullptr,
                                    static_cast<double*>(Y), N, 1.0, 0.0, 0.0)
        : launch_bloch_step<float>(ctx, g, V, kvec, static_cast<const float*>(X), nullptr,
                                   static_cast<float*>(Y), N, 1.0, 0.0, 0.0);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "lrdm_bloch_hamiltonian_apply", e);
  });
}

extern "C" lrdm_status chfsi_filter_bloch(lrdm_ctx* ctx, const lrdm_grid* grid, const double* V,
                                          double kx, double ky, double kz, const void* X, void* Y,
                                          int32_t N, lrdm_prec prec, int32_t degree, double a,
                                          double b, double a0) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_CHECK(ctx, check_filter(degree, a, b, a0));
  LRDM_CHECK(ctx, check_kvec(kx, ky, kz));
  LRDM_NONNULL(ctx, V, "V");
  LRDM_NONNULL(ctx, X, "X");
  LRDM_NONNULL(ctx, Y, "Y");
  const Grid3 g = make_grid3(grid);
  const size_t blk = (size_t)2 * g.M * N * prec_bytes(prec);
  if (overlaps(X, blk, Y, blk)) return fail(ctx, LRDM_EINVAL, "X and Y must not overlap");
  lrdm_status st = begin(ctx, ws_align(blk));
  if (st != LRDM_OK) return st;
  const double kvec[3] = {kx, ky, kz};
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e = (prec == LRDM_FP64)
        ? run_filter_bloch<double>(ctx, g, V, kvec, static_cast<const double*>(X),
                                   static_cast<double*>(Y), N, degree, a, b, a0)
        : run_filter_bloch<float>(ctx, g, V, kvec, static_cast<const float*>(X),
                                  static_cast<float*>(Y), N, degree, a, b, a0);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "chfsi_filter_bloch", e);
  });
}

extern "C" lrdm_status subspace_rayleigh_ritz(lrdm_ctx* ctx, const lrdm_grid* grid,
                                              const double* V, void* Psi, int32_t N,
                                              lrdm_prec prec, double* eps) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_NONNULL(ctx, V, "V");
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, eps, "eps");
  const Grid3 g = make_grid3(grid);
  lrdm_status st = begin(ctx, rr_workspace_bytes(N, g.M, prec));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    if (prec == LRDM_FP64)
      return rayleigh_ritz<double>(ctx, g, V, static_cast<double*>(Psi), N, prec, eps);
    return rayleigh_ritz<float>(ctx, g, V, static_cast<float*>(Psi), N, prec, eps);
  });
}

extern "C" lrdm_status subspace_rayleigh_ritz_bloch(lrdm_ctx* ctx, const lrdm_grid* grid,
                                                    const double* V, double kx, double ky,
                                                    double kz, void* Psi, int32_t N,
                                                    lrdm_prec prec, double* eps) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  if (N > 4096) return fail(ctx, LRDM_EINVAL, "N must be <= 4096 for a complex block");
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_CHECK(ctx, check_kvec(kx, ky, kz));
  LRDM_NONNULL(ctx, V, "V");
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, eps, "eps");
  const Grid3 g = make_grid3(grid);
  lrdm_status st = begin(ctx, rr_bloch_workspace_bytes(N, g.M, prec));
  if (st != LRDM_OK) return st;
  const double kvec[3] = {kx, ky, kz};
  return guarded(ctx, [&]() -> lrdm_status {
    if (prec == LRDM_FP64)
      return rayleigh_ritz_bloch<double>(ctx, g, V, kvec, static_cast<double*>(Psi), N, eps);
    return rayleigh_ritz_bloch<float>(ctx, g, V, kvec, static_cast<float*>(Psi), N, eps);
  });
}

extern "C" lrdm_status density_response(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                        const double* eps, int32_t N, const lrdm_occ* occ,
                                        const double* dV, int32_t r, lrdm_prec prec, double* drho,
                                        double* mu, double* dmu) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_occ(occ, N));
  LRDM_CHECK(ctx, check_rank(r));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, eps, "eps");
  LRDM_NONNULL(ctx, dV, "dV");
  LRDM_NONNULL(ctx, drho, "drho");
  const Grid3 g = make_grid3(grid);
  lrdm_status st = begin(ctx, response_bytes(N, g.M, r, occ->nspin, prec));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e = (prec == LRDM_FP64)
        ? run_response<double>(ctx, g, static_cast<const double*>(Psi), eps, N, occ, dV, r, prec,
                               nullptr, drho, mu, dmu)
        : run_response<float>(ctx, g, static_cast<const float*>(Psi), eps, N, occ, dV, r, prec,
                              nullptr, drho, mu, dmu);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "density_response", e);
  });
}

// The context's workspace, split limit and profiling switch, replaced for the
// duration of one allocation-free call and put back afterwards.
struct ScratchSwap {
  lrdm_ctx* ctx;
  void* ws;
  size_t cap, top;
  int split_limit;
  bool profiling;
  ScratchSwap(lrdm_ctx* c, void* scratch, size_t bytes, int limit)
      : ctx(c), ws(c->ws), cap(c->ws_cap), top(c->ws_top), split_limit(c->split_limit),
        profiling(c->profiling) {
    c->ws = scratch;
    c->ws_cap = bytes;
    c->ws_top = 0;
    c->split_limit = limit;
    c->profiling = false;     // timing events are created on demand: not here
  }
  ~ScratchSwap() {
    ctx->ws = ws;
    ctx->ws_cap = cap;
    ctx->ws_top = top;
    ctx->split_limit = split_limit;
    ctx->profiling = profiling;
  }
};

extern "C" lrdm_status density_response_noalloc(lrdm_ctx* ctx, const lrdm_grid* grid,
                                                const void* Psi, const double* eps, int32_t N,
                                                const lrdm_occ* occ, const double* dV, int32_t r,
                                                lrdm_prec prec, double* drho, double* mu,
                                                double* dmu) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_occ(occ, N));
  LRDM_CHECK(ctx, check_rank(r));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, eps, "eps");
  LRDM_NONNULL(ctx, dV, "dV");
  LRDM_NONNULL(ctx, drho, "drho");
  if (!ctx) return fail(nullptr, LRDM_EINVAL, "ctx is NULL");
  const Grid3 g = make_grid3(grid);
  const size_t cap = noalloc_scratch_bytes();
  const int ns = occ->nspin;
  // fewer K-splits shrink the projection's partial sums until the call fits
  int limit = 0;
  size_t need = response_bytes(N, g.M, r, ns, prec) + (1u << 20);
  if (need > cap) {
    const int ntb = (N + 127) / 128;
    for (limit = tn_split_cap(ntb * (ntb + 1) / 2 * r * ns, g.M); limit > 1 && need > cap;
         limit /= 2)
      need = response_bytes(N, g.M, r, ns, prec, limit / 2) + (1u << 20);
    limit = std::max(limit, 1);
  }
  if (need > cap) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "this response needs %zu bytes of scratch, more than the %zu the "
                  "allocation-free entry point holds per GPU: use density_response",
                  need, cap);
    return fail(ctx, LRDM_EINVAL, msg);
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail_hip(ctx, "hipSetDevice", e);
  void* scratch = nullptr;
  e = noalloc_scratch(ctx->device, &scratch);
  if (e != hipSuccess || !scratch) return fail_hip(ctx, "scratch symbol address", e);
  ScratchSwap swap(ctx, scratch, cap, limit);
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e2 = (prec == LRDM_FP64)
        ? run_response<double>(ctx, g, static_cast<const double*>(Psi), eps, N, occ, dV, r, prec,
                               nullptr, drho, mu, dmu)
        : run_response<float>(ctx, g, static_cast<const float*>(Psi), eps, N, occ, dV, r, prec,
                              nullptr, drho, mu, dmu);
    return e2 == hipSuccess ? LRDM_OK : fail_hip(ctx, "density_response_noalloc", e2);
  });
}

namespace {

size_t response_bz_bytes(int N, int64_t M, int r, int ns, int nk, lrdm_prec prec) {
  const int nsk = ns * nk, batch = r * nsk, N2 = 2 * N;
  return ws_align(8) + ws_align((size_t)r * 8) + 3 * ws_align((size_t)nsk * N * 8) +
         ws_align((size_t)nsk * N * N * 8) + 2 * ws_align((size_t)batch * M * 8) +
         ws_align((size_t)batch * N2 * N2 * 8) + ws_align(tn_bytes(N2, M, batch, prec)) +
         backproj_workspace_bytes(N2, M, nsk, batch, prec);
}

template <typename T>
hipError_t run_response_bz(lrdm_ctx* ctx, const Grid3& g, const T* Psi, const double* eps,
                           const double* weights, int N, int nk, const lrdm_occ* occ,
                           const double* dV, int r, lrdm_prec prec, double* drho, double* mu,
                           double* dmu) {
  const int ns = occ->nspin, nsk = ns * nk, batch = r * nsk, N2 = 2 * N;
  double* mu_d = mu ? mu : static_cast<double*>(ws_take(ctx, 8));
  double* dmu_d = dmu ? dmu : static_cast<double*>(ws_take(ctx, (size_t)r * 8));
  const size_t vec = (size_t)nsk * N * sizeof(double);
  double* f = static_cast<double*>(ws_take(ctx, vec));
  double* omf = static_cast<double*>(ws_take(ctx, vec));
  double* fp = static_cast<double*>(ws_take(ctx, vec));
  double* F = static_cast<double*>(ws_take(ctx, (size_t)nsk * N * N * sizeof(double)));
  LRDM_HIP(launch_fermi_bz(ctx, eps, N, ns, nk, weights, occ->kT, occ->n_electrons, mu_d, f, omf,
                           fp, F));
  double* W = static_cast<double*>(ws_take(ctx, (size_t)batch * g.M * sizeof(double)));
  LRDM_HIP(launch_expand_dv(ctx, dV, r, ns, nk, g.M, W));
  double* H2 = static_cast<double*>(ws_take(ctx, (size_t)batch * N2 * N2 * sizeof(double)));
  LRDM_HIP(launch_tn_sym<T>(ctx, Psi, nullptr, W, g.M, N2, g.M, nsk, batch, prec, H2));
  LRDM_HIP(launch_gamma_bz(ctx, H2, F, fp, weights, N, ns, nk, r, dmu_d));
  double* part = static_cast<double*>(ws_take(ctx, (size_t)batch * g.M * sizeof(double)));
  const double s = (ns == 1) ? 2.0 : 1.0;
  LRDM_HIP(launch_backproj<T>(ctx, Psi, H2, N2, g.M, nsk, batch, prec, s / g.dv, nullptr, part));
  LRDM_HIP(launch_sum_k(ctx, part, r, ns, nk, g.M, drho));
  if (ctx->checks) LRDM_HIP(launch_check_finite(ctx, drho, (int64_t)r * ns * g.M));
  return hipSuccess;
}

}  // namespace

extern "C" lrdm_status density_response_bz(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                           const double* eps, const double* weights, int32_t N,
                                           int32_t nk, const lrdm_occ* occ, const double* dV,
                                           int32_t r, lrdm_prec prec, double* drho, double* mu,
                                           double* dmu) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_occ(occ, N));
  LRDM_CHECK(ctx, check_rank(r));
  LRDM_CHECK(ctx, check_prec(prec));
  if (nk < 1 || nk > 64) return fail(ctx, LRDM_EINVAL, "nk must be in 1..64");
  if (N > 4096) return fail(ctx, LRDM_EINVAL, "N must be <= 4096 (a k-point block holds 2N rows)");
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, eps, "eps");
  LRDM_NONNULL(ctx, weights, "weights");
  LRDM_NONNULL(ctx, dV, "dV");
  LRDM_NONNULL(ctx, drho, "drho");
  const Grid3 g = make_grid3(grid);
  lrdm_status st = begin(ctx, response_bz_bytes(N, g.M, r, occ->nspin, nk, prec));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e = (prec == LRDM_FP64)
        ? run_response_bz<double>(ctx, g, static_cast<const double*>(Psi), eps, weights, N, nk,
                                  occ, dV, r, prec, drho, mu, dmu)
        : run_response_bz<float>(ctx, g, static_cast<const float*>(Psi), eps, weights, N, nk, occ,
                                 dV, r, prec, drho, mu, dmu);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "density_response_bz", e);
  });
}

namespace {

lrdm_status residual_derivative_impl(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                     const double* eps, int32_t N, const lrdm_occ* occ,
                                     const double* u, int32_t r, lrdm_prec prec,
                                     const double* fxc, double* t) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_occ(occ, N));
  LRDM_CHECK(ctx, check_rank(r));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, eps, "eps");
  LRDM_NONNULL(ctx, u, "u");
  LRDM_NONNULL(ctx, t, "t");
  const Grid3 g = make_grid3(grid);
  const int ns = occ->nspin;
  const size_t ubytes = (size_t)r * ns * g.M * sizeof(double);
  if (overlaps(u, ubytes, t, ubytes)) return fail(ctx, LRDM_EINVAL, "u and t must not overlap");
  const size_t scratch = 2 * (size_t)r * g.M * sizeof(double);
  lrdm_status st = begin(ctx, ws_align(ubytes) + ws_align(scratch) + hartree_workspace_bytes(g) +
                                  response_bytes(N, g.M, r, ns, prec));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    double* dV = static_cast<double*>(ws_take(ctx, ubytes));
    double* s = static_cast<double*>(ws_take(ctx, scratch));
    hipError_t e = launch_hartree(ctx, g, u, ns, dV, ns, r, s);
    if (e != hipSuccess) return fail_hip(ctx, "hartree", e);
    if (fxc) {
      e = launch_xc_apply(ctx, fxc, u, ns, r, g.M, dV);
      if (e != hipSuccess) return fail_hip(ctx, "xc kernel", e);
    }
    e = (prec == LRDM_FP64)
        ? run_response<double>(ctx, g, static_cast<const double*>(Psi), eps, N, occ, dV, r, prec,
                               u, t, nullptr, nullptr)
        : run_response<float>(ctx, g, static_cast<const float*>(Psi), eps, N, occ, dV, r, prec, u,
                              t, nullptr, nullptr);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "residual_derivative", e);
  });
}

}  // namespace

extern "C" lrdm_status lrdm_residual_derivative(lrdm_ctx* ctx, const lrdm_grid* grid,
                                                const void* Psi, const double* eps, int32_t N,
                                                const lrdm_occ* occ, const double* u, int32_t r,
                                                lrdm_prec prec, double* t) {
  return residual_derivative_impl(ctx, grid, Psi, eps, N, occ, u, r, prec, nullptr, t);
}

extern "C" lrdm_status lrdm_residual_derivative_xc(lrdm_ctx* ctx, const lrdm_grid* grid,
                                                   const void* Psi, const double* eps, int32_t N,
                                                   const lrdm_occ* occ, const double* u,
                                                   int32_t r, lrdm_prec prec, const double* fxc,
                                                   double* t) {
  LRDM_NONNULL(ctx, fxc, "fxc");
  return residual_derivative_impl(ctx, grid, Psi, eps, N, occ, u, r, prec, fxc, t);
}

extern "C" lrdm_status density_response_backward(lrdm_ctx* ctx, const lrdm_grid* grid,
                                                 const void* Psi, const double* eps, int32_t N,
                                                 const lrdm_occ* occ, const double* dV, int32_t r,
                                                 lrdm_prec prec, const double* g_drho,
                                                 double* g_dV, void* g_Psi, double* g_eps) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_occ(occ, N));
  LRDM_CHECK(ctx, check_rank(r));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, eps, "eps");
  LRDM_NONNULL(ctx, dV, "dV");
  LRDM_NONNULL(ctx, g_drho, "g_drho");
  const Grid3 g = make_grid3(grid);
  const int ns = occ->nspin;
  const size_t blk = (size_t)ns * N * g.M * prec_bytes(prec);
  if (g_Psi && overlaps(Psi, blk, g_Psi, blk))
    return fail(ctx, LRDM_EINVAL, "g_Psi must not overlap Psi");
  if (ctx && ctx->fermi_depth > 0)
    return fail(ctx, LRDM_EUNSUPPORTED,
                "density_response_backward differentiates the exact Fermi-Dirac form only "
                "(the context is set to the recursive expansion)");
  lrdm_status st = begin(ctx, backward_bytes(N, g.M, r, ns, prec));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e = (prec == LRDM_FP64)
        ? run_backward<double>(ctx, g, static_cast<const double*>(Psi), eps, N, occ, dV, r, prec,
                               g_drho, g_dV, static_cast<double*>(g_Psi), g_eps)
        : run_backward<float>(ctx, g, static_cast<const float*>(Psi), eps, N, occ, dV, r, prec,
                              g_drho, g_dV, static_cast<float*>(g_Psi), g_eps);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "density_response_backward", e);
  });
}

extern "C" lrdm_status density_response_batched(lrdm_ctx* ctx, const lrdm_system* sys,
                                                int32_t nsys, lrdm_prec prec) {
  if (nsys < 1 || nsys > 4096) return fail(ctx, LRDM_EINVAL, "nsys must be in [1, 4096]");
  LRDM_NONNULL(ctx, sys, "sys");
  LRDM_CHECK(ctx, check_prec(prec));
  size_t total = 0;
  for (int s = 0; s < nsys; ++s) {
    const lrdm_system& y = sys[s];
    LRDM_CHECK(ctx, check_grid(&y.grid));
    LRDM_CHECK(ctx, check_block(&y.grid, y.N));
    LRDM_CHECK(ctx, check_occ(&y.occ, y.N));
    LRDM_CHECK(ctx, check_rank(y.r));
    LRDM_NONNULL(ctx, y.Psi, "sys[].Psi");
    LRDM_NONNULL(ctx, y.eps, "sys[].eps");
    LRDM_NONNULL(ctx, y.dV, "sys[].dV");
    LRDM_NONNULL(ctx, y.drho, "sys[].drho");
    total += ws_align(response_bytes(y.N, grid_points(&y.grid), y.r, y.occ.nspin, prec));
  }
  lrdm_status st = begin(ctx, total);
  if (st != LRDM_OK) return st;
  if (prec == LRDM_FP32 && ctx->fermi_depth == 0) {
    // the systems' projections in one launch, then their back-projections in one
    // launch, on the context's stream (the small per-system steps in between)
    return guarded(ctx, [&]() -> lrdm_status {
      std::vector<FermiState> fs(nsys);
      std::vector<FusedProjItem> proj(nsys);
      std::vector<FusedBackprojItem> bp(nsys);
      std::vector<double*> dmu(nsys);
      hipError_t e = hipSuccess;
      for (int s = 0; s < nsys && e == hipSuccess; ++s) {
        const lrdm_system& y = sys[s];
        const Grid3 g = make_grid3(&y.grid);
        const int ns = y.occ.nspin;
        e = run_fermi(ctx, y.eps, y.N, &y.occ, y.mu, &fs[s]);
        dmu[s] = y.dmu ? y.dmu : static_cast<double*>(ws_take(ctx, (size_t)y.r * 8));
        double* Hp = static_cast<double*>(
            ws_take(ctx, (size_t)y.r * ns * y.N * y.N * sizeof(double)));
        const float* P = static_cast<const float*>(y.Psi);
        proj[s] = FusedProjItem{P, y.dV, y.N, g.M, ns, y.r * ns, fs[s].active, Hp};
        bp[s] = FusedBackprojItem{P, Hp, y.N, g.M, ns, y.r * ns, (ns == 1 ? 2.0 : 1.0) / g.dv,
                                  fs[s].active, y.drho};
      }
      if (e == hipSuccess) e = launch_tn_sym_fused(ctx, proj.data(), nsys);
      for (int s = 0; s < nsys && e == hipSuccess; ++s)
        e = launch_gamma(ctx, proj[s].H, fs[s].F, fs[s].fp, sys[s].N, sys[s].occ.nspin, sys[s].r,
                         dmu[s]);
      if (e == hipSuccess) e = launch_backproj_fused(ctx, bp.data(), nsys);
      for (int s = 0; s < nsys && e == hipSuccess && ctx->checks; ++s)
        e = launch_check_finite(ctx, sys[s].drho,
                                (int64_t)sys[s].r * sys[s].occ.nspin * grid_points(&sys[s].grid));
      return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "density_response_batched", e);
    });
  }
  return guarded(ctx, [&]() -> lrdm_status {
    const hipStream_t main = ctx->stream;
    const int K = (int)ctx->aux.size();
    hipError_t e = hipEventRecord(ctx->fork_join[0], main);
    for (int k = 0; e == hipSuccess && k < K; ++k)
      e = hipStreamWaitEvent(ctx->aux[k], ctx->fork_join[0], 0);
    if (e != hipSuccess) return fail_hip(ctx, "batched fork", e);
    struct Restore {              // ctx->stream is main again however the loop ends
      lrdm_ctx* c;
      hipStream_t s;
      ~Restore() { c->stream = s; }
    } restore{ctx, main};
    for (int s = 0; s < nsys; ++s) {
      const lrdm_system& y = sys[s];
      const Grid3 g = make_grid3(&y.grid);
      ctx->stream = ctx->aux[s % K];
      e = (prec == LRDM_FP64)
          ? run_response<double>(ctx, g, static_cast<const double*>(y.Psi), y.eps, y.N, &y.occ,
                                 y.dV, y.r, prec, nullptr, y.drho, y.mu, y.dmu)
          : run_response<float>(ctx, g, static_cast<const float*>(y.Psi), y.eps, y.N, &y.occ,
                                y.dV, y.r, prec, nullptr, y.drho, y.mu, y.dmu);
      ctx->stream = main;
      if (e != hipSuccess) return fail_hip(ctx, "density_response_batched", e);
    }
    for (int k = 0; e == hipSuccess && k < K; ++k) {
      e = hipEventRecord(ctx->fork_join[1 + k], ctx->aux[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(main, ctx->fork_join[1 + k], 0);
    }
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "batched join", e);
  });
}


// ============================================================ low-rank step and model SCF

extern "C" lrdm_status lrdm_density(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                    const double* eps, int32_t N, const lrdm_occ* occ,
                                    lrdm_prec prec, const double* rho_in, double* out,
                                    double* mu) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_occ(occ, N));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, eps, "eps");
  LRDM_NONNULL(ctx, out, "out");
  const Grid3 g = make_grid3(grid);
  const int ns = occ->nspin;
  const size_t obytes = (size_t)ns * g.M * sizeof(double);
  if (overlaps(out, obytes, Psi, (size_t)ns * N * g.M * prec_bytes(prec)) ||
      overlaps(out, obytes, eps, (size_t)ns * N * sizeof(double)))
    return fail(ctx, LRDM_EINVAL, "out must not overlap Psi or eps");
  const size_t vec = ws_align((size_t)ns * N * sizeof(double));
  lrdm_status st = begin(ctx, ws_align(8) + 3 * vec + density_workspace_bytes(N, g.M, ns));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    double* mu_d = mu ? mu : static_cast<double*>(ws_take(ctx, 8));
    double* f = static_cast<double*>(ws_take(ctx, vec));
    double* omf = static_cast<double*>(ws_take(ctx, vec));
    double* fp = static_cast<double*>(ws_take(ctx, vec));
    double* part = static_cast<double*>(ws_take(ctx, density_workspace_bytes(N, g.M, ns)));
    hipError_t e = launch_fermi(ctx, eps, N, ns, occ->kT, occ->n_electrons, mu_d, f, omf, fp,
                                nullptr);
    const double scale = (ns == 1 ? 2.0 : 1.0) / g.dv;
    if (e == hipSuccess)
      e = (prec == LRDM_FP64)
          ? launch_density<double>(ctx, static_cast<const double*>(Psi), f, N, g.M, ns, scale,
                                   rho_in, out, part)
          : launch_density<float>(ctx, static_cast<const float*>(Psi), f, N, g.M, ns, scale,
                                  rho_in, out, part);
    if (e == hipSuccess && ctx->checks) e = launch_check_finite(ctx, out, (int64_t)ns * g.M);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "lrdm_density", e);
  });
}

extern "C" lrdm_status lrdm_effective_potential(lrdm_ctx* ctx, const lrdm_grid* grid,
                                                const double* V_ext, const double* rho,
                                                int32_t nspin, const double* vxc, double* V_eff,
                                                double* range) {
  LRDM_CHECK(ctx, check_grid(grid));
  if (nspin != 1 && nspin != 2) return fail(ctx, LRDM_EINVAL, "nspin must be 1 or 2");
  LRDM_NONNULL(ctx, V_ext, "V_ext");
  LRDM_NONNULL(ctx, rho, "rho");
  LRDM_NONNULL(ctx, V_eff, "V_eff");
  const Grid3 g = make_grid3(grid);
  const size_t vb = (size_t)g.M * sizeof(double);
  const int nout = vxc ? nspin : 1;
  if (overlaps(V_eff, nout * vb, V_ext, vb) || overlaps(V_eff, nout * vb, rho, nspin * vb) ||
      (vxc && overlaps(V_eff, nout * vb, vxc, nspin * vb)))
    return fail(ctx, LRDM_EINVAL, "V_eff must not overlap V_ext, rho or vxc");
  const size_t scratch = 2 * vb;
  lrdm_status st = begin(ctx, ws_align(scratch) + hartree_workspace_bytes(g));
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    double* s = static_cast<double*>(ws_take(ctx, scratch));
    // V_H into every output channel, then + V_ext (and + vxc per channel)
    hipError_t e = launch_hartree(ctx, g, rho, nspin, V_eff, nout, 1, s);
    for (int c = 0; e == hipSuccess && c < nout; ++c) {
      e = launch_axpy(ctx, 1.0, V_ext, g.M, V_eff + (size_t)c * g.M);
      if (e == hipSuccess && vxc)
        e = launch_axpy(ctx, 1.0, vxc + (size_t)c * g.M, g.M, V_eff + (size_t)c * g.M);
    }
    if (e == hipSuccess && range) e = launch_minmax(ctx, V_eff, (int64_t)nout * g.M, range);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "lrdm_effective_potential", e);
  });
}

extern "C" lrdm_status lrdm_lda_xc(lrdm_ctx* ctx, const lrdm_grid* grid, const double* rho,
                                   int32_t nspin, double* vxc, double* fxc) {
  LRDM_CHECK(ctx, check_grid(grid));
  if (nspin != 1 && nspin != 2) return fail(ctx, LRDM_EINVAL, "nspin must be 1 or 2");
  LRDM_NONNULL(ctx, rho, "rho");
  const Grid3 g = make_grid3(grid);
  const size_t rb = (size_t)nspin * g.M * sizeof(double);
  if ((vxc && overlaps(vxc, rb, rho, rb)) || (fxc && overlaps(fxc, nspin * rb, rho, rb)) ||
      (vxc && fxc && overlaps(vxc, rb, fxc, nspin * rb)))
    return fail(ctx, LRDM_EINVAL, "rho, vxc and fxc must not overlap");
  lrdm_status st = begin(ctx, 0);
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e = launch_lda_xc(ctx, rho, nspin, g.M, vxc, fxc);
    return e == hipSuccess ? LRDM_OK : fail_hip(ctx, "lrdm_lda_xc", e);
  });
}

namespace {

// Slots of the small host-read block of lrdm_lowrank_step.
enum { LR_NR2 = 0, LR_FIT2 = 1, LR_UNEW2 = 2, LR_V2 = 3, LR_RW = 4, LR_SLOTS = 5 };

template <typename T>
lrdm_status run_lowrank(lrdm_ctx* ctx, const Grid3& g, const T* Psi, const double* eps, int N,
                        const lrdm_occ* occ, lrdm_prec prec, const double* R,
                        const lrdm_lowrank_params* prm, int r_keep, const double* fxc,
                        double* U, double* Tm, double* drho, double* rho,
                        lrdm_lowrank_info* info) {
  const int ns = occ->nspin;
  const int64_t n = (int64_t)ns * g.M;
  const double dv = g.dv;
  const int K = kMaxLowRank;
  const int r_cap = prm->r_max;
  const int add_cap = prm->r_add_max > 0 ? prm->r_add_max : r_cap;
  auto hip_fail = [&](const char* where, hipError_t e) { return fail_hip(ctx, where, e); };
#define LR_HIP(where, call)                           \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(where, e_); \
  } while (0)
  double* S = static_cast<double*>(ws_take(ctx, (size_t)K * K * sizeof(double)));
  double* c = static_cast<double*>(ws_take(ctx, K * sizeof(double)));
  double* y = static_cast<double*>(ws_take(ctx, K * sizeof(double)));
  double* gco = static_cast<double*>(ws_take(ctx, K * sizeof(double)));
  double* sc = static_cast<double*>(ws_take(ctx, LR_SLOTS * sizeof(double)));
  int* flag = static_cast<int*>(ws_take(ctx, sizeof(int)));
  double* part = static_cast<double*>(ws_take(ctx, dots_workspace_bytes(K)));
  double* w = static_cast<double*>(ws_take(ctx, (size_t)n * sizeof(double)));
  double* dV = static_cast<double*>(ws_take(ctx, (size_t)n * sizeof(double)));
  double* hs = static_cast<double*>(ws_take(ctx, 2 * (size_t)g.M * sizeof(double)));
  // every direction's response reads the same block: in the BF16X3 form split it
  // once here (the context hands the pieces to the projection and back-projection)
  struct PiecesGuard {
    lrdm_ctx* c;
    ~PiecesGuard() { c->pieces = lrdm_psi_pieces{}; }
  } pieces_guard{ctx};
  if constexpr (sizeof(T) == sizeof(float)) {
    if (prec == LRDM_BF16X3) {
      void* p3 = ws_take(ctx, psi_pieces_p3_bytes(N, g.M, ns));
      void* pt3 = ws_take(ctx, psi_pieces_pt3_bytes(N, g.M, ns));
      LR_HIP("lowrank split", launch_psi_pieces(ctx, Psi, N, g.M, ns, p3, pt3));
      ctx->pieces = lrdm_psi_pieces{Psi, N, g.M, ns, p3, pt3};
    }
  }
  // the Fermi quantities depend on eps alone: once for every direction
  FermiState fermi;
  LR_HIP("lowrank fermi", run_fermi(ctx, eps, N, occ, nullptr, &fermi));
  const size_t mark = ctx->ws_top;
  double h[LR_SLOTS] = {0, 0, 0, 0, 0};
  int hflag = 0;
  // host read of the scalar block and the solve flag (one synchronisation)
  auto read = [&]() -> lrdm_status {
    LR_HIP("lowrank read", hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    LR_HIP("lowrank read", hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost,
                                          ctx->stream));
    LR_HIP("lowrank sync", hipStreamSynchronize(ctx->stream));
    if (hflag)
      return fail(ctx, LRDM_ENOTCONV,
                  "lrdm_lowrank_step: the Gram matrix of the directional derivatives is not "
                  "numerically positive definite");
    return LRDM_OK;
  };
  // S row i, c_i, y = S^{-1} c over i + 1 derivatives, the fit residual
  // w = sum_j y_j t_j - R (Eq. (10)) with its norm and <R, w>
  auto fit = [&](int i) -> hipError_t {
    const double* ti = Tm + (size_t)i * n;
    LRDM_HIP(launch_dots(ctx, Tm, n, i + 1, ti, n, dv, S + (size_t)i * K, 1, part));
    LRDM_HIP(launch_dots(ctx, ti, 0, 1, R, n, dv, c + i, 1, part));
    LRDM_HIP(launch_lowrank_solve(ctx, S, K, c, i + 1, y, flag));
    LRDM_HIP(launch_combine(ctx, R, -1.0, Tm, n, y, i + 1, 1.0, n, w));
    LRDM_HIP(launch_dots(ctx, w, 0, 1, w, n, dv, sc + LR_FIT2, 1, part));
    return launch_dots(ctx, w, 0, 1, R, n, dv, sc + LR_RW, 1, part);
  };
  // un = v - sum_{k<m} <v, u_k> u_k, twice, and |un|^2, |v|^2
  auto orthogonalise = [&](const double* v, int m, double* un) -> hipError_t {
    LRDM_HIP(launch_dots(ctx, U, n, m, v, n, dv, gco, 1, part));
    LRDM_HIP(launch_combine(ctx, v, 1.0, U, n, gco, m, -1.0, n, un));
    LRDM_HIP(launch_dots(ctx, U, n, m, un, n, dv, gco, 1, part));
    LRDM_HIP(launch_combine(ctx, un, 1.0, U, n, gco, m, -1.0, n, un));
    LRDM_HIP(launch_dots(ctx, un, 0, 1, un, n, dv, sc + LR_UNEW2, 1, part));
    return launch_dots(ctx, v, 0, 1, v, n, dv, sc + LR_V2, 1, part);
  };

  // ||R||
  LR_HIP("lowrank norm", launch_dots(ctx, R, 0, 1, R, n, dv, sc + LR_NR2, 1, part));
  LR_HIP("lowrank read", hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  LR_HIP("lowrank sync", hipStreamSynchronize(ctx->stream));
  if (!std::isfinite(h[LR_NR2])) return fail(ctx, LRDM_ENONFINITE, "||R|| is not finite");
  const double nR = std::sqrt(h[LR_NR2]);
  const double alpha = nR < prm->alpha_switch ? prm->alpha_near : prm->alpha_far;
  info->norm_R = nR;
  info->alpha = alpha;
  info->added = 0;
  if (nR == 0.0) {
    info->rank = r_keep;
    info->s_rel = 0.0;
    info->norm_R_lin = 0.0;
    LR_HIP("lowrank zero", launch_combine(ctx, nullptr, 0.0, U, n, y, 0, 1.0, n, drho));
    return LRDM_OK;
  }
  int rank = r_keep;
  double s_rel = 1.0;
  bool grow = prm->r_add_max >= 0;
  if (r_keep > 0) {
    // the kept directions first: rebuild S over their derivatives, fit R
    for (int i = 0; i < r_keep; ++i) LR_HIP("lowrank kept", fit(i));
    lrdm_status st = read();
    if (st != LRDM_OK) return st;
    s_rel = std::sqrt(h[LR_FIT2]) / nR;
    grow = grow && !(s_rel < prm->s_tol) && r_keep < r_cap;
  }
  if (grow) {
    // the first new direction: R without its components along the kept ones
    double* un = U + (size_t)r_keep * n;
    LR_HIP("lowrank first", orthogonalise(R, r_keep, un));
    if (r_keep > 0) {
      lrdm_status st = read();
      if (st != LRDM_OK) return st;
      grow = h[LR_UNEW2] > 1e-26 * h[LR_V2];    // R already in span(U): nothing new
    } else {
      h[LR_UNEW2] = h[LR_NR2];
    }
    if (grow) LR_HIP("lowrank normalize", launch_normalize(ctx, un, sc + LR_UNEW2, n, un));
  }
  for (int i = r_keep; grow && i < r_cap; ++i) {
    double* ui = U + (size_t)i * n;
    double* ti = Tm + (size_t)i * n;
    ctx->ws_top = mark;        // the response's slices are reused by every direction
    LR_HIP("lowrank hartree", launch_hartree(ctx, g, ui, ns, dV, ns, 1, hs));
    if (fxc) LR_HIP("lowrank xc", launch_xc_apply(ctx, fxc, ui, ns, 1, g.M, dV));
    LR_HIP("lowrank response",
           run_response<T>(ctx, g, Psi, eps, N, occ, dV, 1, prec, ui, ti, nullptr, nullptr,
                           &fermi));
    LR_HIP("lowrank fit", fit(i));
    const int added = i - r_keep + 1;
    const bool more = i + 1 < r_cap && added < add_cap;
    // the next direction (Eq. (8)), formed before the host decides so that one
    // synchronisation per direction suffices
    if (more) LR_HIP("lowrank next", orthogonalise(ti, i + 1, U + (size_t)(i + 1) * n));
    lrdm_status st = read();
    if (st != LRDM_OK) return st;
    rank = i + 1;
    info->added = added;
    s_rel = std::sqrt(h[LR_FIT2]) / nR;
    if (!std::isfinite(s_rel)) return fail(ctx, LRDM_ENONFINITE, "s_rel is not finite");
    if (s_rel < prm->s_tol || !more) break;
    // t_i inside span(u_1..u_{i+1}): the Krylov space is exhausted and the fit exact
    if (!(h[LR_UNEW2] > 1e-26 * h[LR_V2])) break;
    double* un = U + (size_t)(i + 1) * n;
    LR_HIP("lowrank normalize", launch_normalize(ctx, un, sc + LR_UNEW2, n, un));
  }
  // drho_bar = sum_i y_i u_i (Eq. (9)); R_lin = (1 - alpha) R - alpha w (Eq. (12))
  LR_HIP("lowrank drho", launch_combine(ctx, nullptr, 0.0, U, n, y, rank, 1.0, n, drho));
  if (rho) LR_HIP("lowrank update", launch_axpy(ctx, -alpha, drho, n, rho));
  if (ctx->checks) LR_HIP("lowrank check", launch_check_finite(ctx, drho, n));
  const double lin2 = (1.0 - alpha) * (1.0 - alpha) * h[LR_NR2] -
                      2.0 * alpha * (1.0 - alpha) * h[LR_RW] + alpha * alpha * h[LR_FIT2];
  info->rank = rank;
  info->s_rel = s_rel;
  info->norm_R_lin = std::sqrt(std::max(lin2, 0.0));
  return LRDM_OK;
#undef LR_HIP
}

}  // namespace

extern "C" lrdm_status lrdm_lowrank_step(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                         const double* eps, int32_t N, const lrdm_occ* occ,
                                         lrdm_prec prec, const double* R,
                                         const lrdm_lowrank_params* params, int32_t r_keep,
                                         const double* fxc, double* U, double* T, double* drho,
                                         double* rho, lrdm_lowrank_info* info) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_occ(occ, N));
  LRDM_CHECK(ctx, check_prec(prec));
  LRDM_CHECK(ctx, check_lowrank(params));
  LRDM_NONNULL(ctx, Psi, "Psi");
  LRDM_NONNULL(ctx, eps, "eps");
  LRDM_NONNULL(ctx, R, "R");
  LRDM_NONNULL(ctx, U, "U");
  LRDM_NONNULL(ctx, T, "T");
  LRDM_NONNULL(ctx, drho, "drho");
  LRDM_NONNULL(ctx, info, "info");
  if (r_keep < 0 || r_keep > params->r_max)
    return fail(ctx, LRDM_EINVAL, "r_keep must be in 0..r_max");
  const Grid3 g = make_grid3(grid);
  const int ns = occ->nspin;
  const size_t vb = (size_t)ns * g.M * sizeof(double);
  const size_t ub = (size_t)params->r_max * vb;
  struct Span {
    const void* p;
    size_t n;
  } spans[5] = {{R, vb}, {U, ub}, {T, ub}, {drho, vb}, {rho, rho ? vb : 0}};
  for (int a = 0; a < 5; ++a)
    for (int b = a + 1; b < 5; ++b)
      if (spans[a].n && spans[b].n && overlaps(spans[a].p, spans[a].n, spans[b].p, spans[b].n))
        return fail(ctx, LRDM_EINVAL, "R, U, T, drho and rho must not overlap");
  const int K = kMaxLowRank;
  const size_t small = ws_align((size_t)K * K * 8) + 3 * ws_align(K * 8) + ws_align(LR_SLOTS * 8) +
                       ws_align(sizeof(int)) + dots_workspace_bytes(K);
  const size_t pieces = prec == LRDM_BF16X3
      ? psi_pieces_p3_bytes(N, g.M, ns) + psi_pieces_pt3_bytes(N, g.M, ns) : 0;
  const size_t bytes = small + 2 * ws_align(vb) + ws_align(2 * (size_t)g.M * 8) + pieces +
                       hartree_workspace_bytes(g) + response_bytes(N, g.M, 1, ns, prec);
  lrdm_status st = begin(ctx, bytes);
  if (st != LRDM_OK) return st;
  return guarded(ctx, [&]() -> lrdm_status {
    return (prec == LRDM_FP64)
        ? run_lowrank<double>(ctx, g, static_cast<const double*>(Psi), eps, N, occ, prec, R,
                              params, r_keep, fxc, U, T, drho, rho, info)
        : run_lowrank<float>(ctx, g, static_cast<const float*>(Psi), eps, N, occ, prec, R,
                             params, r_keep, fxc, U, T, drho, rho, info);
  });
}

// ============================================================ autotuner

namespace {

// Times `launch` (enqueued on ctx's stream) once to warm up and then `reps` times
// between two events; milliseconds per launch.
template <typename F>
hipError_t time_launch(lrdm_ctx* ctx, F&& launch, int reps, double* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
  for (int i = 0; e == hipSuccess && i < reps; ++i) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  *ms = (double)t / reps;
  return e;
}

}  // namespace

extern "C" lrdm_status lrdm_autotune(lrdm_ctx* ctx, const lrdm_grid* grid, int32_t N,
                                     int32_t nspin, int32_t r, lrdm_prec prec, int32_t* splits,
                                     int32_t* variants, double* timings,
                                     int32_t* backproj_layout, double* backproj_ms) {
  LRDM_CHECK(ctx, check_grid(grid));
  LRDM_CHECK(ctx, check_block(grid, N));
  LRDM_CHECK(ctx, check_rank(r));
  LRDM_CHECK(ctx, check_prec(prec));
  if (nspin != 1 && nspin != 2) return fail(ctx, LRDM_EINVAL, "nspin must be 1 or 2");
  const Grid3 g = make_grid3(grid);
  const int batch = r * nspin;
  const size_t el = prec_bytes(prec);
  const size_t ws = std::max({tn_workspace_bytes(N, g.M, batch, prec),
                              tn_workspace_bytes(N, g.M, nspin, prec),
                              tn_workspace_bytes(N, g.M, 1, LRDM_FP64),
                              backproj_workspace_bytes(N, g.M, nspin, batch, prec)});
  lrdm_status st = begin(ctx, ws);
  if (st != LRDM_OK) return st;
  void* A = nullptr;
  double* w = nullptr;
  double* H = nullptr;
  struct Free {
    void** p[3];
    ~Free() {
      for (void** q : p)
        if (*q) hipFree(*q);
    }
  } release{{&A, reinterpret_cast<void**>(&w), reinterpret_cast<void**>(&H)}};
  if (hipMalloc(&A, (size_t)nspin * N * g.M * el) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&w), (size_t)batch * g.M * sizeof(double)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&H), (size_t)batch * N * N * sizeof(double)) != hipSuccess)
    return fail(ctx, LRDM_ENOMEM, "lrdm_autotune: scratch allocation failed");
  return guarded(ctx, [&]() -> lrdm_status {
    hipError_t e = launch_pattern(ctx, A, (int64_t)nspin * N * g.M, prec == LRDM_FP64);
    if (e == hipSuccess) e = launch_pattern(ctx, w, (int64_t)batch * g.M, true);
    if (e != hipSuccess) return fail_hip(ctx, "lrdm_autotune", e);
    const int ntb = (N + 127) / 128;
    const int ntiles = ntb * (ntb + 1) / 2;
    const int arith = prec == LRDM_FP64 ? TN_ARITH_F64
                                        : (prec == LRDM_FP32 ? TN_ARITH_F32 : TN_ARITH_BF16X3);
    // three contractions: the response's projection of all directions, the
    // single-direction projection of the low-rank step, and the Gram matrix of
    // Rayleigh-Ritz (FP64 arithmetic, unweighted)
    struct Kind {
      int b, arith;
      bool weighted;
    } kinds[3] = {{batch, arith, true}, {nspin, arith, true}, {1, TN_ARITH_F64, false}};
    for (int k = 0; k < 3; ++k) {
      const Kind& kd = kinds[k];
      const int h = tn_splits(ntiles * kd.b, g.M);
      const int cap = tn_split_cap(ntiles * kd.b, g.M);
      const std::array<int64_t, 5> key{N, g.M, kd.b, kd.arith, kd.weighted ? 1 : 0};
      int best = h, best_v = TN_VAR_DEFAULT;
      double best_ms = 1e300;
      const int cand[4] = {h / 4, h / 2, h, 2 * h};
      // tile and wave layouts: one kernel for FP64 arithmetic, two for FP32,
      // three for BF16X3 (variants of TN_VAR_*)
      const int nvar = kd.arith == TN_ARITH_F64 ? 1 : (kd.arith == TN_ARITH_F32 ? 2 : 3);
      for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 4; ++c)
          if (timings) timings[(k * 3 + v) * 4 + c] = 0.0;
      for (int v = 0; v < nvar; ++v)
      for (int c = 0; c < 4; ++c) {
        const int s = cand[c];
        if (s < 1 || s > cap || (c > 0 && s == cand[c - 1])) continue;
        ctx->tn_variant[key] = v;
        ctx->tn_tuned[key] = s;
        auto launch = [&]() -> hipError_t {
          ctx->ws_top = 0;
          if (!kd.weighted)
            return prec == LRDM_FP64
                ? launch_tn_sym_f64<double, double>(ctx, static_cast<const double*>(A), nullptr,
                                                    nullptr, 0, N, g.M, 1, 1, H)
                : launch_tn_sym_f64<float, float>(ctx, static_cast<const float*>(A), nullptr,
                                                  nullptr, 0, N, g.M, 1, 1, H);
          return prec == LRDM_FP64
              ? launch_tn_sym<double>(ctx, static_cast<const double*>(A), nullptr, w, g.M, N,
                                      g.M, nspin, kd.b, prec, H)
              : launch_tn_sym<float>(ctx, static_cast<const float*>(A), nullptr, w, g.M, N,
                                     g.M, nspin, kd.b, prec, H);
        };
        double ms = 0.0;
        e = time_launch(ctx, launch, 3, &ms);
        if (e != hipSuccess) return fail_hip(ctx, "lrdm_autotune", e);
        if (timings) timings[(k * 3 + v) * 4 + c] = ms;
        if (ms < best_ms) {
          best_ms = ms;
          best = s;
          best_v = v;
        }
      }
      ctx->tn_tuned[key] = best;
      ctx->tn_variant[key] = best_v;
      if (splits) splits[k] = best;
      if (variants) variants[k] = best_v;
    }
    // the BF16X3 back-projection layouts on the response's shape: Gamma = the
    // projected matrices just formed (every block), the result into w
    int bp_best = ctx->bp_variant;
    if (backproj_ms) backproj_ms[0] = backproj_ms[1] = 0.0;
    if (prec == LRDM_BF16X3) {
      double best_ms = 1e300;
      for (int v = BP_VAR_NARROW; v <= BP_VAR_WIDE; ++v) {
        ctx->bp_variant = v;
        auto launch = [&]() -> hipError_t {
          ctx->ws_top = 0;
          return launch_backproj<float>(ctx, static_cast<const float*>(A), H, N, g.M, nspin, batch,
                                        prec, 1.0, nullptr, w, nullptr);
        };
        double ms = 0.0;
        e = time_launch(ctx, launch, 3, &ms);
        if (e != hipSuccess) {
          ctx->bp_variant = bp_best;
          return fail_hip(ctx, "lrdm_autotune", e);
        }
        if (backproj_ms) backproj_ms[v] = ms;
        if (ms < best_ms) {
          best_ms = ms;
          bp_best = v;
        }
      }
      ctx->bp_variant = bp_best;
    }
    if (backproj_layout) *backproj_layout = bp_best;
    return LRDM_OK;
  });
}

// Internal declarations of liblrdm: the context, the workspace arena and the
// kernel launchers.  Nothing here is part of the public C ABI (include/lrdm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "lrdm.h"

struct lrdm_prof_rec {
  const char* name;
  hipEvent_t start, stop;
};

// Pre-split BF16 pieces of one FP32 block, in use while `psi` is set: the BF16X3
// projection and back-projection of that block (same N, M, nspin) read them
// instead of splitting the block again.  Set for the duration of a low-rank step,
// whose directions all share the block.
struct lrdm_psi_pieces {
  const void* psi = nullptr;
  int N = 0;
  int64_t M = 0;
  int nspin = 0;
  const void* p3 = nullptr;    // [nspin][3][N][M]
  const void* pt3 = nullptr;   // [nspin][3][M][ldk]
};

struct lrdm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t limit = 0;          // 0 = unlimited
  void* ws = nullptr;        // device workspace
  size_t ws_cap = 0;
  size_t ws_top = 0;         // bump pointer inside one call
  int checks = 0;
  int fermi_depth = 0;       // 0: exact divided differences; T > 0: recursive expansion
  int eigh_max_sweeps = 40;  // block Jacobi sweeps before the eigensolver gives up
  double block_tau = 1e-14;  // response blocks with max |F| below tau max |F| are skipped
  int bp_variant = 1;        // BF16X3 back-projection layout (BP_VAR_*)
  int split_limit = 0;       // > 0: cap on the projection's K-split count (allocation-free calls)
  lrdm_psi_pieces pieces;
  // K-split counts of the projection contraction chosen by lrdm_autotune, keyed by
  // (N, M, batch, arithmetic, weighted)
  std::map<std::array<int64_t, 5>, int> tn_tuned;
  // the projection kernel variant lrdm_autotune chose for the same keys (TN_VAR_*)
  std::map<std::array<int64_t, 5>, int> tn_variant;
  int* dstatus = nullptr;    // device status words (LRDM_DS_*), then the zero page
  const float* zeros = nullptr;  // 128 bytes of device zeros (source of padding loads)
  std::string err;
  bool profiling = false;    // record hipEvents around the main kernels
  std::vector<lrdm_prof_rec> prof;
  std::vector<hipEvent_t> event_pool;
  // streams and events of the batched entry point: systems are issued round-robin
  // on the aux streams between a fork and a join on `stream`
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> fork_join;   // [0] fork, [1 + k] join of aux[k]
};

constexpr int kAuxStreams = 4;

// Device status word indices (checking mode).
enum { LRDM_DS_BISECT = 0, LRDM_DS_EIGH = 1, LRDM_DS_NONFINITE = 2, LRDM_DS_COUNT = 4 };

namespace lrdm {

// Host-side argument checks (validate.cpp, no HIP).  Each returns nullptr when
// the argument is acceptable, else a message.
const char* check_grid(const lrdm_grid* g);
const char* check_block(const lrdm_grid* g, int32_t N);
const char* check_occ(const lrdm_occ* occ, int32_t N);
const char* check_prec(int prec);
const char* check_rank(int32_t r);
const char* check_filter(int32_t degree, double a, double b, double a0);
const char* check_lowrank(const lrdm_lowrank_params* p);
const char* check_ptr(const void* p, const char* name);

inline int64_t grid_points(const lrdm_grid* g) {
  return (int64_t)g->n[0] * g->n[1] * g->n[2];
}
inline size_t prec_bytes(lrdm_prec p) { return p == LRDM_FP64 ? 8 : 4; }

// Workspace arena: reserve() guarantees `bytes` of capacity (growing the
// allocation if needed, within the context limit); take() hands out aligned
// slices of it for the duration of one ABI call.
lrdm_status ws_reserve(lrdm_ctx* ctx, size_t bytes);
inline size_t ws_align(size_t b) { return (b + 255) & ~size_t(255); }
void* ws_take(lrdm_ctx* ctx, size_t bytes);

struct Grid3 {
  int nx, ny, nz;
  double hx, hy, hz;
  int64_t M;
  double dv;
};
Grid3 make_grid3(const lrdm_grid* g);

// ------------------------------------------------------------------ launchers
// All launchers enqueue on ctx->stream and return the first HIP error.

// Yout = alpha (H - c0) Yin + beta Yold  (Yold unused when beta == 0).
template <typename T>
hipError_t launch_cheb_step(lrdm_ctx* ctx, const Grid3& g, const double* V, const T* Yin,
                            const T* Yold, T* Yout, int N, double alpha, double c0, double beta);

// The same step in its vectorised form, with V given in the storage type (Vt);
// usable when cheb_vec_ok(g): nx a multiple of the 16-byte group and at most 2048
// groups per plane.  Yout may equal Yold.
template <typename T>
bool cheb_vec_ok(const Grid3& g);
template <typename T>
hipError_t launch_cheb_step_vec(lrdm_ctx* ctx, const Grid3& g, const T* Vt, const T* Yin,
                                const T* Yold, T* Yout, int N, double alpha, double c0,
                                double beta);
// Two consecutive steps in one sweep (vectorised form):
//   Yc = a1 (H - c0) Yb + b1 Ya,   Yd = a2 (H - c0) Yc + b2 Yb,
// each element as launch_cheb_step_vec forms it.  Usable when cheb_pair_ok(g, N):
// the vectorised form applies with at most 1024 groups per plane, nz >= 4, and a
// block can own a whole z column.
// Yc may equal Ya and Yd may equal Yb.
template <typename T>
bool cheb_pair_ok(const Grid3& g, int N);
template <typename T>
hipError_t launch_cheb_pair_vec(lrdm_ctx* ctx, const Grid3& g, const T* Vt, const T* Ya,
                                const T* Yb, T* Yc, T* Yd, int N, double c0, double a1, double b1,
                                double a2, double b2);
// Three consecutive steps in one sweep: Y_{k+s} = a[s-1] (H - c0) Y_{k+s-1} +
// b[s-1] Y_{k+s-2} for s = 1, 2, 3 with Ya = Y_{k-1}, Yb = Y_k; writes Y_{k+2} to
// Yp and Y_{k+3} to Yq only.  Usable when cheb_triple_ok(g, N): cheb_pair_ok and
// nz >= 8.  Yp and Yq may be the buffers of Ya and Yb, either way round.
template <typename T>
bool cheb_triple_ok(const Grid3& g, int N);
template <typename T>
hipError_t launch_cheb_triple_vec(lrdm_ctx* ctx, const Grid3& g, const T* Vt, const T* Ya,
                                  const T* Yb, T* Yp, T* Yq, int N, double c0, const double* a,
                                  const double* b);
// b[i] = (float)a[i], i < n.
hipError_t launch_to_float(lrdm_ctx* ctx, const double* a, int64_t n, float* b);

// HY = H Y in FP64 arithmetic and storage for either storage type of Y.
template <typename T>
hipError_t launch_hpsi_f64(lrdm_ctx* ctx, const Grid3& g, const double* V, const T* Y, double* HY,
                           int N);

// mu by bisection, occupations, f' and (optionally) F for nspin channels.
hipError_t launch_fermi(lrdm_ctx* ctx, const double* eps, int N, int nspin, double kT,
                        double n_electrons, double* mu, double* f, double* omf, double* fprime,
                        double* F);

// The pieces of an FP32 block Psi [nspin][N][M] that the BF16X3 projection and
// back-projection read (see lrdm_psi_pieces), into p3 and pt3 of
// psi_pieces_bytes in all.
size_t psi_pieces_p3_bytes(int N, int64_t M, int nspin);
size_t psi_pieces_pt3_bytes(int N, int64_t M, int nspin);
hipError_t launch_psi_pieces(lrdm_ctx* ctx, const float* Psi, int N, int64_t M, int nspin,
                             void* p3, void* pt3);

// Rotation Out = Wt^T B of an FP32 block in the BF16X3 form (both operands split
// into three BF16 pieces, six products, FP32 partials summed in FP64); `upper`: Wt
// upper triangular.  Out may be B (B is consumed by the split before the product).
// Takes rotate_bf16x3_bytes of workspace.
size_t rotate_bf16x3_bytes(int N, int64_t M);
hipError_t launch_rotate_bf16x3(lrdm_ctx* ctx, const double* Wt, const float* B, float* Out,
                                int N, int64_t M, bool upper);

// One Chebyshev step with the Bloch Hamiltonian of kvec (bloch.hip) on blocks of N
// complex states stored as [2][N][M] (real parts, then imaginary parts):
// out = alpha (H_k in - c0 in) + beta old; old may be out, beta = 0 ignores it.
template <typename T>
hipError_t launch_bloch_step(lrdm_ctx* ctx, const Grid3& g, const double* V, const double kvec[3],
                             const T* in, const T* old, T* out, int N, double alpha, double c0,
                             double beta);
// out = H_k in in FP64 for a block of N complex states stored as T (bloch.hip);
// state i has its real part at i sr and its imaginary part at i sr + si (in and
// out alike): sr = M, si = N M for [2][N][M], sr = 2M, si = M for [N][2][M].
template <typename T>
hipError_t launch_bloch_hpsi_f64(lrdm_ctx* ctx, const Grid3& g, const double* V,
                                 const double kvec[3], const T* in, double* out, int N,
                                 int64_t sr, int64_t si);

// launch_fermi with Brillouin-zone sampling: eps [nspin][nk][N], weights [nk]
// (device); mu from the zone-averaged count, then f, 1 - f, f' and the divided
// differences F [nspin][nk][N][N] of every (channel, k).
hipError_t launch_fermi_bz(lrdm_ctx* ctx, const double* eps, int N, int nspin, int nk,
                           const double* weights, double kT, double n_electrons, double* mu,
                           double* f, double* omf, double* fprime, double* F);

// The zone-sampled response's pieces (kpoints.hip).  Psi of channel c at k is
// stored as the 2N real rows [Re psi_1..N; Im psi_1..N] ("realified"), so that
// H2 = Phi^T diag(dV) Phi and the back-projection of G2 are the real kernels'
// products with 2N states.
// W[(q nspin + c) nk + k] = dV[q nspin + c] (M points each).
hipError_t launch_expand_dv(lrdm_ctx* ctx, const double* dV, int r, int nspin, int nk, int64_t M,
                            double* W);
// mu'[q] of the zone-averaged traceless condition from H2 [r][nspin][nk][2N][2N],
// then G2 = w_k [[Gr, Gi], [-Gi, Gr]] in place over H2, with
// Gr = F o (H2_00 + H2_11) - mu' diag(f'), Gi = F o (H2_01 - H2_10).
hipError_t launch_gamma_bz(lrdm_ctx* ctx, double* H2, const double* F, const double* fprime,
                           const double* weights, int N, int nspin, int nk, int r, double* dmu);
// drho[q nspin + c][p] = sum_k part[(q nspin + c) nk + k][p].
hipError_t launch_sum_k(lrdm_ctx* ctx, const double* part, int r, int nspin, int nk, int64_t M,
                        double* drho);

// The recursive expansion's multiplier M [nspin][N][N] and its diagonal [nspin][N]
// (depth T, mu on the device).
hipError_t launch_recursive_multiplier(lrdm_ctx* ctx, const double* eps, const double* mu, int N,
                                      int nspin, double kT, int depth, double* M, double* diag);

// H[b] = A_c diag(w_b) B_c^T for b < batch, c = b % nspin, over the grid index;
// only the upper triangle is formed and mirrored (the callers' products are
// symmetric).  B == nullptr means B = A; w == nullptr means w = 1.
// A, B: nspin blocks of [N][M].
// split_limit > 0 caps the K-split count (and with it the partial sums' size).
size_t tn_workspace_bytes(int N, int64_t M, int batch, lrdm_prec prec, int split_limit = 0);
size_t tn_split_bytes(int N, int64_t M, lrdm_prec prec);
size_t tn_part_bytes(int N, int64_t M, int batch, int split_limit = 0);
// Split count of the K = M contraction: enough blocks to fill 256 CUs several
// times over, with each split at least 4096 grid points long.
inline int tn_splits(int tiles_x_batch, int64_t M) {
  int s = 1;
  while (tiles_x_batch * s < 2048 && M / (2 * s) >= 4096) s *= 2;
  return s;
}
// The largest split count the partial-sum workspace is sized for: twice the
// default, as long as each split keeps at least 2048 grid points.
inline int tn_split_cap(int tiles_x_batch, int64_t M) {
  const int h = tn_splits(tiles_x_batch, M);
  int c = 2 * h;
  while (c > h && M / c < 2048) c /= 2;
  return c;
}
// The allocation-free entry point's device scratch (noalloc.hip): its size, and
// the device address of `device`'s copy (looked up once per device, with that
// device current).
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch(int device, void** out);

// Arithmetic of a projection contraction, part of the autotuner's key.
enum { TN_ARITH_F64 = 0, TN_ARITH_F32 = 1, TN_ARITH_BF16X3 = 2 };
// Kernel variants of the FP32-storage projection (tile and wave layout):
//  TN_VAR_DEFAULT  8 waves of 32 x 64 on a 128 x 128 tile, operands copied to LDS
//                  through a three-stage ring (BF16X3: Psi's pieces split once
//                  per call, only the weighted side split in the kernel);
//  TN_VAR_STAGED   4 waves of 64 x 64 on the same tile, operands staged through
//                  registers (two buffers);
//  TN_VAR_SPLIT    BF16X3 only: the ring kernel splitting both operands in the
//                  kernel (no pre-split copy of Psi).
enum { TN_VAR_DEFAULT = 0, TN_VAR_STAGED = 1, TN_VAR_SPLIT = 2 };
// Layouts of the BF16X3 back-projection:
//  BP_VAR_NARROW  128 points per workgroup, 8 waves of 32 x 64, three ring stages,
//                 FP32 partials added into FP64 once per 128 x 128 block
//  BP_VAR_WIDE    256 points per workgroup, 8 waves of 64 x 64, two ring stages,
//                 FP32 sums over a whole row block of Gamma
enum { BP_VAR_NARROW = 0, BP_VAR_WIDE = 1 };
int tn_variant(const lrdm_ctx* ctx, int N, int64_t M, int batch, int arith, bool weighted);
// The split count a projection launch uses: the autotuned one for this shape if
// lrdm_autotune chose one, else tn_splits.
int tn_split_count(const lrdm_ctx* ctx, int N, int64_t M, int batch, int arith, bool weighted);
// T is the storage type of A and B; prec selects the arithmetic (LRDM_FP64: FP64
// matrix cores on either storage type; LRDM_FP32 / LRDM_BF16X3: FP32 storage only).
// active (blocks.h, may be NULL): the tiles of inactive blocks are left at zero.
template <typename T>
hipError_t launch_tn_sym(lrdm_ctx* ctx, const T* A, const T* B, const double* w,
                         int64_t w_stride, int N, int64_t M, int nspin, int batch, lrdm_prec prec,
                         double* H, const unsigned char* active = nullptr);
template <typename SA, typename SB>
hipError_t launch_tn_sym_f64(lrdm_ctx* ctx, const SA* A, const SB* B, const double* w,
                             int64_t w_stride, int N, int64_t M, int nspin, int batch, double* H,
                             const unsigned char* active = nullptr);

// The response's block mask (blocks.h): active [nspin][ntb][ntb] from the
// multiplier F [nspin][N][N]; tmax: nspin * ntb * ntb doubles of scratch.
hipError_t launch_block_mask(lrdm_ctx* ctx, const double* F, int N, int nspin, double tau,
                             double* tmax, unsigned char* active);

// dmu[k] and Gamma[k][c] = F[c] o Hp[k][c] - dmu[k] diag(fprime[c]), in place over Hp.
hipError_t launch_gamma(lrdm_ctx* ctx, double* Hp, const double* F, const double* fprime, int N,
                        int nspin, int r, double* dmu);

// out[b][p] = scale * sum_ij A_c[i][p] G[b][i][j] A_c[j][p] (- sub[b][p] when sub != nullptr),
// c = b % nspin, G symmetric; the blocks of G that `active` (blocks.h, may be
// NULL) marks inactive are left out.
size_t backproj_workspace_bytes(int N, int64_t M, int nspin, int batch, lrdm_prec prec);
template <typename T>
hipError_t launch_backproj(lrdm_ctx* ctx, const T* A, const double* G, int N, int64_t M, int nspin,
                           int batch, lrdm_prec prec, double scale, const double* sub,
                           double* out, const unsigned char* active = nullptr);

// The FP32-form projection and back-projection of several independent systems,
// each in one launch over all of them (gemm_lp.hip): H = Psi^T diag(w) Psi per
// direction and channel of each item, and out = scale * sum_ij Psi_i G_ij Psi_j,
// skipping the blocks each item's `active` marks inactive.  The per-system
// partial sums, FP32 copies and transposes come from the workspace.
struct FusedProjItem {
  const float* A;          // Psi [nspin][N][M]
  const double* w;         // dV [batch][M]
  int N;
  int64_t M;
  int nspin, batch;
  const unsigned char* active;
  double* H;               // [batch][N][N]
};
struct FusedBackprojItem {
  const float* A;          // Psi [nspin][N][M]
  const double* G;         // Gamma [batch][N][N]
  int N;
  int64_t M;
  int nspin, batch;
  double scale;
  const unsigned char* active;
  double* out;             // [batch][M]
};
hipError_t launch_tn_sym_fused(lrdm_ctx* ctx, const FusedProjItem* items, int n);
hipError_t launch_backproj_fused(lrdm_ctx* ctx, const FusedBackprojItem* items, int n);

// Out[i][p] = sum_j Wt[j][i] B[j][p]  (Out = Wt^T B), Wt double N x N, FP64
// arithmetic for either storage type of B and Out.  upper: Wt is upper triangular
// (Out = L B with L lower triangular), and the zero blocks are skipped.
template <typename S>
hipError_t launch_nn_f64(lrdm_ctx* ctx, const double* Wt, const S* B, S* Out, int N, int64_t M,
                         bool upper = false);

// Adjoint rotation: Out_c = scale * sum_m (X_m Psi_c) o w_m over two lists of nx
// symmetric matrices [nx][nspin][N][N] with weights [nx][nspin][M]; Out has
// Psi's storage type and layout.  FP64 storage: FP64 arithmetic (gemm.hip).  FP32
// storage: FP32 matrix cores with FP64 accumulation across K-tiles, skipping the
// blocks `active` marks inactive (gemm_lp.hip; workspace adj_psi_workspace_bytes).
template <typename T>
hipError_t launch_adj_psi(lrdm_ctx* ctx, const double* X1, const double* w1, const double* X2,
                          const double* w2, int nx, const T* Psi, int N, int64_t M, int nspin,
                          double scale, T* Out, const unsigned char* active = nullptr);
size_t adj_psi_workspace_bytes(int N, int64_t M, int nspin, int nx, bool fp32);
// The same rotation in the BF16X3 form (FP32 storage): both operands split into
// three BF16 pieces, six products, FP32 partial sums per K-tile weighted into
// FP64 (gemm_lp.hip); workspace adj_psi_bf16x3_bytes.
hipError_t launch_adj_psi_bf16x3(lrdm_ctx* ctx, const double* X1, const double* w1,
                                 const double* X2, const double* w2, int nx, const float* Psi,
                                 int N, int64_t M, int nspin, double scale, float* Out,
                                 const unsigned char* active);
size_t adj_psi_bf16x3_bytes(int N, int64_t M, int nspin, int nx);

// Adjoint pieces (adjoint.hip).
// y[i] = a * x[i] for i < n.
hipError_t launch_scale(lrdm_ctx* ctx, const double* x, double a, int64_t n, double* y);
// dL/deps for each channel from A = dL/dGamma and H' ([r][nspin][N][N] each), the
// Fermi quantities of launch_fermi, mu' and nu ([r]), including the chain through mu;
// part: nspin N doubles of scratch.
hipError_t launch_adj_eps(lrdm_ctx* ctx, const double* A, const double* Hp, const double* eps,
                          const double* F, const double* f, const double* omf, const double* fp,
                          const double* dmu, const double* nu, int N, int nspin, int r, double kT,
                          double* part, double* g_eps);

// Orthonormalising factor of a Gram matrix G = Y Y^T (chol.hip): T (N x N) with the
// first `live` rows of T Y orthonormal and the others the explicit residuals of the
// dependent rows of Y (Schur-complement pivot below tau after unit-diagonal
// scaling) against the independent ones before them; cond estimates the condition
// number of the scaled Gram matrix.
struct CholInfo {
  int live;
  double cond;
};
lrdm_status chol_orth(lrdm_ctx* ctx, const double* G, int N, double tau, double* T,
                      CholInfo* info);
size_t chol_orth_bytes(int N);

// Rayleigh-Ritz pieces (rr.hip).
// Eigenpairs of a symmetric N x N matrix (FP64, block Jacobi on the GPU).
lrdm_status sym_eigh(lrdm_ctx* ctx, const double* S, int lda, int N, const double* dinv,
                     double* evals, double* evecs);
template <typename T>
lrdm_status rayleigh_ritz(lrdm_ctx* ctx, const Grid3& g, const double* V, T* Psi, int N,
                          lrdm_prec prec, double* eps);
size_t rr_workspace_bytes(int N, int64_t M, lrdm_prec prec);
// Rayleigh-Ritz of the Bloch Hamiltonian H_k on N complex states [2][N][M]
// (real parts, then imaginary parts) stored as T; FP64 arithmetic.
template <typename T>
lrdm_status rayleigh_ritz_bloch(lrdm_ctx* ctx, const Grid3& g, const double* V,
                                const double kvec[3], T* Psi, int N, double* eps);
size_t rr_bloch_workspace_bytes(int N, int64_t M, lrdm_prec prec);

// Hartree kernel (poisson.hip): dV[k] = 4 pi (-Lap_h)^{-1} (sum_c u[k][c]) for k < r,
// written to every channel slot of dV when nspin_out > 1.
hipError_t launch_hartree(lrdm_ctx* ctx, const Grid3& g, const double* u, int u_nspin,
                          double* dV, int dv_nspin, int r, double* scratch);
size_t hartree_workspace_bytes(const Grid3& g);

hipError_t launch_check_finite(lrdm_ctx* ctx, const double* x, int64_t n);

// Low-rank preconditioner pieces and the output density (lowrank.hip).
constexpr int kMaxLowRank = 64;
// State-range splits of the density sum: enough blocks to fill the chip.
inline int density_splits(int N, int64_t M, int nspin) {
  const int64_t bx = (M + 255) / 256;
  int s = 1;
  while (bx * nspin * s < 2048 && s < 16 && 2 * s <= N) s *= 2;
  return s;
}
size_t density_workspace_bytes(int N, int64_t M, int nspin);
// out[c][p] = scale sum_i f[c][i] Psi[c][i][p]^2 - (rho_in ? rho_in[c][p] : 0);
// part: density_workspace_bytes of scratch.
template <typename T>
hipError_t launch_density(lrdm_ctx* ctx, const T* Psi, const double* f, int N, int64_t M,
                          int nspin, double scale, const double* rho_in, double* out,
                          double* part);
size_t dots_workspace_bytes(int k);
// out[j * stride] = scale sum_i A[j][i] x[i] for j < k (rows lda apart), in a fixed
// order; part: dots_workspace_bytes(k) of scratch.
hipError_t launch_dots(lrdm_ctx* ctx, const double* A, int64_t lda, int k, const double* x,
                       int64_t n, double scale, double* out, int stride, double* part);
// y = beta x + sgn sum_{k < nk} coef[k] A[k] (x may be NULL, y may be x).
hipError_t launch_combine(lrdm_ctx* ctx, const double* x, double beta, const double* A,
                          int64_t lda, const double* coef, int nk, double sgn, int64_t n,
                          double* y);
// y = x / sqrt(nrm2[0]).
hipError_t launch_normalize(lrdm_ctx* ctx, const double* x, const double* nrm2, int64_t n,
                            double* y);
// y += a x.
hipError_t launch_axpy(lrdm_ctx* ctx, double a, const double* x, int64_t n, double* y);
// LDA potential vxc [nspin][M] and kernel fxc [nspin][nspin][M] from rho [nspin][M]
// (xc.hip; either output may be NULL), and dV[k][c] += sum_d fxc[c][d] u[k][d].
hipError_t launch_lda_xc(lrdm_ctx* ctx, const double* rho, int nspin, int64_t M, double* vxc,
                         double* fxc);
hipError_t launch_xc_apply(lrdm_ctx* ctx, const double* fxc, const double* u, int nspin, int r,
                           int64_t M, double* dV);
// x[i] = a hashed value in [-1, 1) (scratch contents for timing runs).
hipError_t launch_pattern(lrdm_ctx* ctx, void* x, int64_t n, bool is_double);
// range[0], range[1] = min and max of x[0..n).
hipError_t launch_minmax(lrdm_ctx* ctx, const double* x, int64_t n, double* range);
// y = S^{-1} c for the r x r lower triangle of S (leading dimension ld); *flag = 1
// (and y = 0) when S is not numerically positive definite.
hipError_t launch_lowrank_solve(lrdm_ctx* ctx, const double* S, int ld, const double* c, int r,
                                double* y, int* flag);

// Records a start/stop hipEvent pair on ctx->stream around its scope when the
// context is profiling (see lrdm_profile).
class ProfScope {
 public:
  ProfScope(lrdm_ctx* ctx, const char* name);
  ~ProfScope();
 private:
  lrdm_ctx* ctx_;
  const char* name_;
  hipEvent_t start_ = nullptr;
};

}  // namespace lrdm

#define LRDM_HIP(call)                         \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) return e_;           \
  } while (0)

/*
 * lrdm.h -- C ABI of the LRDM density-response hot path on MI355X (gfx950).
 *
 * The method is the low-rank dielectric-matrix (LRDM) preconditioner of
 * Das & Gavini, "Accelerating SCF iterations in Kohn-Sham DFT using a low rank
 * approximation of the dielectric matrix".  Each rank-1 term needs the Gateaux
 * derivative t_i of the SCF residual along a direction function u_i
 * (Sec. II B, Eq. (7)), which the paper evaluates in the Chebyshev-filtered
 * subspace (Sec. II C).  This library computes that path on one GPU:
 *
 *   chfsi_filter            Y = T_c(Hbar) X / T_c(ybar0)        (Sec. II C)
 *   subspace_rayleigh_ritz  Psi_R, eps from the filtered block   (Sec. II C, Eq. (15))
 *   density_response        delta rho[dV] in span(Psi_R)         (Eqs. (19)-(22))
 *   density_response_backward  its vector-Jacobian product (adjoint)
 *   lrdm_residual_derivative t = chi0 K_c u - u                  (Eqs. (3), (7))
 *   lrdm_lowrank_step       drho_bar = P^lr_r R, adaptive r, the damped
 *                           quasi-Newton update of rho, and the accumulated
 *                           variant over kept directions   (Sec. II B, Eqs. (4), (8)-(14))
 *   lrdm_density, lrdm_effective_potential  the model SCF map rho -> R[rho]
 *                           around them                             (Sec. II A, Eq. (1))
 *   lrdm_lda_xc, lrdm_residual_derivative_xc  the LDA potential and kernel K_xc,
 *                           and t with K = K_c + K_xc                (Eq. (3), Sec. II D)
 *
 * plus the single steps they are made of (stencil Hamiltonian, occupations and
 * divided differences, projected perturbation, Hartree kernel).
 *
 * Discretisation (the paper's finite-element objects carried to a periodic
 * finite-difference grid, as allowed at the end of Sec. II D):
 *   grid n = (nx, ny, nz) points, spacing h_d = L_d / n_d, dv = hx*hy*hz,
 *   M = nx*ny*nz; H = -1/2 Lap_h + diag(V) with the 7-point periodic stencil;
 *   a block of N vectors is state-major: element (i, z, y, x) lives at
 *   i*M + (z*ny + y)*nx + x ("x fastest"); Ritz vectors are l2-orthonormal,
 *   so rho(x_p) = (s/dv) sum_i f_i Psi_ip^2 with s = 2 (spin restricted) or
 *   s = 1 per channel (spin polarised, Sec. II D).
 *
 * Conventions for every entry point:
 *   - Every array argument is a caller-owned DEVICE pointer on the context's
 *     device, contiguous, in the layout stated.  The library never frees or
 *     keeps a caller pointer after the call returns.
 *   - Calls are asynchronous on the context's HIP stream (see
 *     lrdm_set_checks for the synchronous checking mode).  One context per
 *     stream; a context is not thread-safe.
 *   - The context owns a device workspace, grown on demand up to the
 *     workspace_limit given at creation; a call that would need more returns
 *     LRDM_ENOMEM before launching anything.
 *   - Arguments are validated on the host before any launch: positive sizes,
 *     N <= M, 0 < N_e < s*N*nspin (N > N_e/2 for one channel, Eq. (14)),
 *     kT > 0, degree >= 1, a0 < a < b, finite scalars, non-NULL pointers.
 *     Failures return LRDM_EINVAL and leave a message for lrdm_last_error.
 *     Validation runs before the context is used, so it also works with a
 *     NULL context (which is itself reported as LRDM_EINVAL afterwards).
 *   - HIP failures return LRDM_EDEVICE with the HIP message.
 *   - Precision forms (lrdm_prec): LRDM_FP64 keeps blocks in double;
 *     LRDM_FP32 keeps blocks in float and runs the long contractions on
 *     FP32 matrix cores with FP64 partial sums; LRDM_BF16X3 keeps blocks in
 *     float and runs the projection / back-projection contractions (and the
 *     Rayleigh-Ritz rotations) on BF16 matrix cores: every FP32 operand is
 *     split exactly into three BF16 pieces x = x1 + x2 + x3 (8 significant
 *     bits each), and the six products of order <= 2 are kept (x1*y1; x1*y2 +
 *     x2*y1; x1*y3 + x2*y2 + x3*y1), accumulated in FP32 over four 32-wide K
 *     tiles and in FP64 across them (the default back-projection layout sums
 *     a 128-row block of Gamma's products in FP32 before its FP64 fold with
 *     Psi; lrdm_set_backproj_layout).  Potentials,
 *     eigenvalues, occupations, densities, mu and mu' are always double, and
 *     the subspace eigensolver, the Fermi-level bisection and the divided
 *     differences always run in FP64 on the GPU.
 */
#ifndef LRDM_H
#define LRDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LRDM_OK = 0,
  LRDM_EINVAL = -1,       /* invalid argument (see lrdm_last_error) */
  LRDM_ENOMEM = -2,       /* workspace would exceed the context's limit, or allocation failed */
  LRDM_EDEVICE = -3,      /* a HIP call failed */
  LRDM_ENOTCONV = -4,     /* bisection or eigensolver did not converge (checking mode only) */
  LRDM_ENONFINITE = -5,   /* NaN/Inf found in an output (checking mode only) */
  LRDM_EUNSUPPORTED = -6  /* a valid request that the library does not implement */
} lrdm_status;

typedef enum { LRDM_FP64 = 0, LRDM_FP32 = 1, LRDM_BF16X3 = 2 } lrdm_prec;

/* Periodic orthorhombic cell: n[d] points and length L[d] (bohr) along x, y, z. */
typedef struct { int32_t n[3]; double L[3]; } lrdm_grid;

/* Occupation model of Eq. (1): Fermi-Dirac with temperature kT (Ha) and
 * n_electrons in total (over both channels when nspin = 2). */
typedef struct { int32_t nspin; double kT; double n_electrons; } lrdm_occ;

typedef struct lrdm_ctx lrdm_ctx;

/* ---------------------------------------------------------------- context */

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL means the default stream).  workspace_limit is the
 * largest device workspace, in bytes, the context may allocate (0 = no limit).
 * Selects `device` as current for the calling thread. */
lrdm_status lrdm_create(lrdm_ctx** ctx, int device, void* hip_stream, size_t workspace_limit);

/* Release the context and its workspace (synchronises its stream first). */
lrdm_status lrdm_destroy(lrdm_ctx* ctx);

/* Switch the stream later calls are enqueued on. */
lrdm_status lrdm_set_stream(lrdm_ctx* ctx, void* hip_stream);

/* level 0 (default): calls only enqueue work.  level 1: every call also
 * synchronises its stream and returns LRDM_ENOTCONV / LRDM_ENONFINITE when a
 * device-side check failed (bisection bracket, eigensolver sweeps, NaN/Inf). */
lrdm_status lrdm_set_checks(lrdm_ctx* ctx, int level);

/* Form of the Fermi function in the response multiplier for the calls that
 * follow on this context (density_response, lrdm_residual_derivative,
 * density_response_batched, lrdm_lowrank_step).  depth 0 (the default) uses the
 * exact Fermi-Dirac divided differences of Eq. (22).  depth T in 1..64 uses the
 * paper's recursive expansion of depth T instead (Eqs. (23)-(24)): X_0 =
 * 1/2 - 2^{-(T+2)} (D - mu)/kT, X_n = X^2 (X^2 + (1 - X)^2)^{-1}, whose
 * first-order response on the diagonal D is the Hadamard multiplier
 * M_ij = -(2^{-(T+2)}/kT) prod_n g[x_i^(n), x_j^(n)] (g the step map, g[a, b] its
 * divided difference); M and its diagonal replace F and f' in Gamma and mu'.
 * mu stays at the Fermi-Dirac electron count.  While depth > 0,
 * density_response_backward returns LRDM_EUNSUPPORTED. */
lrdm_status lrdm_set_fermi_expansion(lrdm_ctx* ctx, int32_t depth);

/* Blocks of the response left out.  Gamma = F o H' - mu' diag(f') (Eq. (22))
 * is negligible wherever the Fermi multiplier F is: between two states both
 * deep below the Fermi level, or both far above it.  For the response calls that
 * follow on this context (density_response, lrdm_residual_derivative,
 * density_response_batched, lrdm_lowrank_step), each 128 x 128 block (I, J) of
 * the N x N matrices whose largest |F_ij| does not exceed tau times the largest
 * |F| (over all blocks and channels) is dropped: its projection block is not
 * formed (H' is taken as zero there, also in mu') and the back-projection skips
 * it.  In the l2 norm the dropped part of delta rho is at most
 * (s/dv) tau max|F| (||H'||_F + sqrt(N) |mu'|) per direction and channel, since
 * Psi is orthonormal and |f'_i| = |F_ii| on a dropped diagonal block.  tau in
 * [0, 1); 0 forms every block; the default is 1e-14.  The adjoint
 * (density_response_backward) always forms every block. */
lrdm_status lrdm_set_response_block_skip(lrdm_ctx* ctx, double tau);

/* Largest number of block Jacobi sweeps the subspace eigensolver of
 * subspace_rayleigh_ritz may take (1..1000, default 40).  A solve that has not
 * brought every off-diagonal entry below 1e-13 ||A||_F by then returns
 * LRDM_ENOTCONV, at any checking level, and leaves Psi and eps undefined. */
lrdm_status lrdm_set_eigensolver_sweeps(lrdm_ctx* ctx, int32_t max_sweeps);

/* Layout of the BF16X3 back-projection (Eqs. (16), (20)).  1 (the default):
 * 256 grid points per workgroup, each staged tile of Gamma's pieces serving
 * twice as many points, and each row block of Gamma's products summed in FP32
 * before the FP64 fold with Psi; 0: 128 points per workgroup, FP32 partials
 * added into FP64 once per 128 x 128 block.  The results agree to FP32
 * rounding of 128- to N-term partial sums.  Other values: LRDM_EINVAL. */
lrdm_status lrdm_set_backproj_layout(lrdm_ctx* ctx, int32_t layout);

/* Bytes of device workspace the context currently holds. */
size_t lrdm_workspace_bytes(const lrdm_ctx* ctx);

/* Per-kernel timing for measurement: with enable = 1 the context records a
 * hipEvent pair on its stream around each launch of its main kernels
 * ("cheb_step": single filter steps, "cheb_pair" and "cheb_triple": two and
 * three filter steps in one sweep, "hpsi": plain H X and the first step of the
 * unvectorised filter,
 * "proj": projected perturbation, "gram": Gram and
 * projected-Hamiltonian products, "backproj", "nn", "eigh" (one launch per
 * eigensolve), "jac_sweep" (one per outer sweep), "jac_solve", "jac_update",
 * "hartree").
 * lrdm_profile_read synchronises the stream and returns, for one kernel name,
 * the summed milliseconds and the number of launches recorded since the last
 * read of that name, then forgets them. */
lrdm_status lrdm_profile(lrdm_ctx* ctx, int enable);
lrdm_status lrdm_profile_read(lrdm_ctx* ctx, const char* kernel, double* ms, int64_t* launches);

/* Message of the last failure on this context; with ctx == NULL, the last
 * failure of a call made on this thread without a usable context.  The string
 * stays valid until the next call on the same context / thread. */
const char* lrdm_last_error(const lrdm_ctx* ctx);

/* ---------------------------------------------------------------- single steps */

/* Y = H X with H = -1/2 Lap_h + diag(V) (Eq. (1), 7-point periodic stencil).
 * V [nz][ny][nx] double; X, Y [N][nz][ny][nx], double (FP64) or float
 * (FP32, BF16X3).  X and Y must not overlap. */
lrdm_status lrdm_hamiltonian_apply(lrdm_ctx* ctx, const lrdm_grid* grid, const double* V,
                                   const void* X, void* Y, int32_t N, lrdm_prec prec);

/* Fermi level and occupations of Eq. (1), and the divided-difference matrix
 * that turns H' into the subspace density-matrix response (Eq. (22)):
 *   mu: s sum f(eps) = N_e by FP64 bisection on [min eps - 50 kT, max eps + 50 kT]
 *       until the bracket is within 2 ulp (at most 200 halvings);
 *   f_i = 1/(1 + exp((eps_i - mu)/kT)), fprime_i = -f_i (1 - f_i)/kT;
 *   F_ij = (f_i - f_j)/(eps_i - eps_j), F_ii = fprime_i, evaluated as
 *       -(1/kT) f_lo (1 - f_hi) expm1(z)/z, z = (eps_lo - eps_hi)/kT <= 0.
 * eps [nspin][N] double.  Outputs (device, double): mu [1], f [nspin][N],
 * fprime [nspin][N], F [nspin][N][N]; any output may be NULL. */
lrdm_status lrdm_fermi_occupations(lrdm_ctx* ctx, const double* eps, int32_t N, const lrdm_occ* occ,
                                   double* mu, double* f, double* fprime, double* F);

/* Projected perturbation Hbreve'_k = Psi_R^T diag(dV_k) Psi_R (Eq. (21)) for
 * k < r and each channel.  Psi [nspin][N][M] (double for FP64, float
 * otherwise); dV [r][nspin][M] double; Hp [r][nspin][N][N] double (full,
 * symmetric). */
lrdm_status lrdm_projected_perturbation(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                        int32_t N, int32_t nspin, const double* dV, int32_t r,
                                        lrdm_prec prec, double* Hp);

/* Hartree kernel of Eq. (3): dV_k = 4 pi (-Lap_h)^{-1} u_k with the same
 * 7-point Laplacian as H and the q = 0 component removed.  u, dV [r][M]
 * double; may alias. */
lrdm_status lrdm_hartree_kernel(lrdm_ctx* ctx, const lrdm_grid* grid, const double* u,
                                double* dV, int32_t r);

/* ---------------------------------------------------------------- hot path */

/* ChFSI Chebyshev filter of degree `degree` (Sec. II C): with e = (b - a)/2,
 * c0 = (b + a)/2, Hbar = (H - c0)/e maps the unwanted interval [a, b] to
 * [-1, 1]; the output is Y = T_c(Hbar) X / T_c((a0 - c0)/e), computed by the
 * scaled three-term recurrence of Zhou, Saad, Tiago & Chelikowsky (2006).
 * a0 < a < b: a0 a lower bound of the spectrum, a the top of the wanted
 * part, b an upper bound of the spectrum.  X, Y [N][nz][ny][nx] (double for
 * FP64, float otherwise), must not overlap; X is not modified. */
lrdm_status chfsi_filter(lrdm_ctx* ctx, const lrdm_grid* grid, const double* V,
                         const void* X, void* Y, int32_t N, lrdm_prec prec,
                         int32_t degree, double a, double b, double a0);

/* H_k Y for the Bloch Hamiltonian of one k-point (Sec. II C, last paragraph):
 * for the cell-periodic part u of Bloch states e^{i k.x} u(x), the 7-point
 * stencil of chfsi_filter with the phase e^{i k_d h_d} on the link to the
 * neighbour at +h_d and its conjugate on the link to -h_d,
 *   (H_k u)_p = -1/2 sum_d (e^{i k_d h_d} u_{p+e_d} + e^{-i k_d h_d} u_{p-e_d}
 *               - 2 u_p)/h_d^2 + V_p u_p.
 * X, Y [2][N][nz][ny][nx]: the N real parts, then the N imaginary parts (double
 * for LRDM_FP64, float otherwise; the arithmetic is FP64); (kx, ky, kz) in
 * 1/bohr, finite; k = 0 is the real stencil.  X and Y must not overlap. */
lrdm_status lrdm_bloch_hamiltonian_apply(lrdm_ctx* ctx, const lrdm_grid* grid, const double* V,
                                         double kx, double ky, double kz, const void* X, void* Y,
                                         int32_t N, lrdm_prec prec);

/* chfsi_filter with H_k in place of H (ChFSI of one k-point's subspace, Sec.
 * II C, last paragraph): the same scaled three-term recurrence and bounds on
 * blocks of N complex states stored as in lrdm_bloch_hamiltonian_apply.  The
 * workspace holds one more block. */
lrdm_status chfsi_filter_bloch(lrdm_ctx* ctx, const lrdm_grid* grid, const double* V, double kx,
                               double ky, double kz, const void* X, void* Y, int32_t N,
                               lrdm_prec prec, int32_t degree, double a, double b, double a0);

/* Rayleigh-Ritz step of ChFSI (Sec. II C, Eq. (15)): orthonormalise the
 * filtered block, project H, diagonalise the N x N projection in FP64 on the
 * GPU and rotate.  Psi [N][nz][ny][nx]: in = filtered block, out = Ritz
 * vectors (l2-orthonormal); eps [N] double, ascending.  Each channel of a
 * spin-polarised system is a separate call with its own V.
 * Orthonormalisation: column-scaled Cholesky QR in FP64 arithmetic, one pass
 * for a well-conditioned block, a second pass over the explicitly formed basis
 * for an ill-conditioned one.  Rows numerically dependent on the rows before
 * them are resolved through their explicit residuals; rows still dependent
 * after that (exact copies, zero rows) are replaced by fixed pseudo-random rows,
 * so the output is orthonormal for any input.  The Ritz pairs of such completed
 * directions are not determined by the input.  Synchronises the stream (the
 * pass count and the eigensolver's stop are decided on the host).  Errors:
 * EINVAL (arguments), ENOMEM (workspace), EDEVICE, ENOTCONV (eigensolver
 * without convergence within its sweep limit, 40 unless
 * lrdm_set_eigensolver_sweeps says otherwise, at any checking level; or a
 * block that five passes could not orthonormalise). */
lrdm_status subspace_rayleigh_ritz(lrdm_ctx* ctx, const lrdm_grid* grid, const double* V,
                                   void* Psi, int32_t N, lrdm_prec prec, double* eps);

/* subspace_rayleigh_ritz for the Bloch Hamiltonian H_k of one k-point (Sec. II
 * C, last paragraph; H_k as in lrdm_bloch_hamiltonian_apply): Psi [2][N][M]
 * (the N real parts, then the N imaginary parts; double for LRDM_FP64, float
 * for LRDM_FP32 and LRDM_BF16X3, whose arithmetic here is FP64 as well, H_k Psi
 * included), in = the filtered complex block, out = N Ritz vectors orthonormal
 * in the complex l2 product; eps [N] double (device), ascending.  The complex block is handled as the 2N
 * real vectors of y_i and i y_i: their Gram matrix (the real part of the complex
 * one) is factored by the FP64 Cholesky QR of subspace_rayleigh_ritz, the
 * projection of the real form of H_k is diagonalised by the same block Jacobi
 * eigensolver (each Ritz value of H_k appears twice there, with the vectors v
 * and i v), and one vector of each pair is kept; a multiplet of equal Ritz
 * values comes out as orthonormal complex vectors spanning it.  Each Ritz
 * vector's phase is arbitrary.  Rows that the first Cholesky pass finds
 * dependent are resolved, as in subspace_rayleigh_ritz, by a pass over their
 * explicit residuals; unlike there, a block that stays rank deficient is an
 * error, not completed with pseudo-random rows.  Synchronises the stream.
 * Errors: EINVAL (arguments; N at most 4096), ENOMEM, EDEVICE, ENOTCONV
 * (eigensolver without convergence; a complex block numerically rank deficient
 * as given, i.e. a state whose residual against the states before it is below
 * 1e-8 of its length, or one that five passes could not orthonormalise; a
 * multiplet of more than 32 equal Ritz values, or real Ritz values that do not
 * fall into pairs). */
lrdm_status subspace_rayleigh_ritz_bloch(lrdm_ctx* ctx, const lrdm_grid* grid, const double* V,
                                         double kx, double ky, double kz, void* Psi, int32_t N,
                                         lrdm_prec prec, double* eps);

/* Subspace density response (Eqs. (19)-(22), traceless condition after
 * Eq. (24); per channel without the factor 2 in Sec. II D):
 *   Hp_k = Psi^T diag(dV_k) Psi,  mu'_k = sum f'_i Hp_k,ii / sum f'_i (over
 *   both channels), Gamma_k = F o Hp_k - mu'_k diag(f'),
 *   drho_k(x_p) = (s/dv) sum_ij Psi_ip Gamma_k,ij Psi_jp.
 * Psi [nspin][N][M]; eps [nspin][N]; dV, drho [r][nspin][M] double.
 * mu [1] and dmu [r] (device, double) receive mu and mu'_k; either may be NULL. */
lrdm_status density_response(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                             const double* eps, int32_t N, const lrdm_occ* occ,
                             const double* dV, int32_t r, lrdm_prec prec,
                             double* drho, double* mu, double* dmu);

/* Subspace density response with Brillouin-zone sampling (Sec. II C, last
 * paragraph, and the zone-integrated traceless condition there).  Each of the nk
 * k-points has its own complex subspace Psi_k (from ChFSI of the Bloch
 * Hamiltonian H_k) and Ritz values eps_k; the perturbation dV is lattice-periodic,
 * the same at every k.  With weights w_k (sum_k w_k = 1):
 *   H'_k = Psi_k^H diag(dV_q) Psi_k,  mu from s sum_k w_k sum_i f(eps_ki) = N_e,
 *   mu'_q = sum_k w_k sum_i f'_ki H'_k,ii / sum_k w_k sum_i f'_ki (over both
 *           channels), Gamma_k = F_k o H'_k - mu'_q diag(f'_k),
 *   drho_q(x_p) = (s/dv) sum_k w_k sum_ij psi_ki(p) Gamma_k,ij conj(psi_kj(p)).
 * Psi [nspin][nk][2][N][M]: for each channel and k-point the N real parts of the
 * states, then their N imaginary parts (double for LRDM_FP64, float otherwise);
 * eps [nspin][nk][N] and weights [nk] device doubles (weights non-negative and
 * summing to 1, not checked); dV, drho [r][nspin][M] double; mu [1] and dmu [r]
 * device doubles, either may be NULL.  The complex contractions run as the real
 * ones with the 2N real rows [Re Psi_k; Im Psi_k].  Errors as for
 * density_response, plus EINVAL for nk outside 1..64 or N > 4096. */
lrdm_status density_response_bz(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                const double* eps, const double* weights, int32_t N, int32_t nk,
                                const lrdm_occ* occ, const double* dV, int32_t r, lrdm_prec prec,
                                double* drho, double* mu, double* dmu);

/* density_response for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as density_response, but every intermediate
 * lives in a fixed scratch array of 256 MiB per GPU, part of the library's
 * device image (held from the first use of the library on that GPU until the
 * process ends); the call allocates nothing and never grows the context's
 * workspace.  When the intermediates would not fit, the projection's K-split
 * count is lowered (this changes only the order of its FP64 partial sums); a
 * problem that still needs more than 256 MiB returns LRDM_EINVAL with the
 * bytes it needs, before any launch (FP64 on a 48^3 grid with 256 states and 8
 * directions fits; the FP32-storage forms also need a transposed copy of Psi).
 * All calls on one GPU share its scratch array: calls that overlap on one GPU
 * (on different streams or contexts) race and must be ordered by the caller.
 * Timing (lrdm_profile) is not recorded for these calls.  In checking mode
 * (lrdm_set_checks) the call synchronises, which graph capture does not allow. */
lrdm_status density_response_noalloc(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                     const double* eps, int32_t N, const lrdm_occ* occ,
                                     const double* dV, int32_t r, lrdm_prec prec, double* drho,
                                     double* mu, double* dmu);

/* Gateaux derivative of the SCF residual along u_k (Eq. (7)) with
 * J = chi0 K - I (Eq. (3)) and K = K_c: every channel sees
 * dV_k = K_c (sum_sigma u_k,sigma); t_k = drho[dV_k] - u_k.
 * u, t [r][nspin][M] double; may not alias. */
lrdm_status lrdm_residual_derivative(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                     const double* eps, int32_t N, const lrdm_occ* occ,
                                     const double* u, int32_t r, lrdm_prec prec, double* t);

/* One system of a batched call: the arguments of density_response. */
typedef struct {
  lrdm_grid grid;
  const void* Psi;      /* [nspin][N][M], double (LRDM_FP64) or float */
  const double* eps;    /* [nspin][N] */
  int32_t N;
  lrdm_occ occ;
  const double* dV;     /* [r][nspin][M] */
  int32_t r;
  double* drho;         /* [r][nspin][M], out */
  double* mu;           /* [1], out, may be NULL */
  double* dmu;          /* [r], out, may be NULL */
} lrdm_system;

/* density_response for nsys independent systems of any sizes (uneven grids,
 * subspaces, spin settings and ranks) in one call.  The systems are issued
 * round-robin on four streams owned by the context, forked from and joined back
 * to the context's stream, so they run concurrently; a caller that captures the
 * context's stream into a HIP graph gets the whole batch as one graph.  The
 * workspace (one region per system) must already be large enough when the call
 * is captured: make the same call once before capturing, else LRDM_ENOMEM.
 * Every system is validated as in density_response before anything is
 * launched; outputs of different systems must not overlap. */
lrdm_status density_response_batched(lrdm_ctx* ctx, const lrdm_system* sys, int32_t nsys,
                                     lrdm_prec prec);

/* Adjoint (vector-Jacobian product) of density_response: for a loss L with
 * g_drho = dL/d(delta rho) [r][nspin][M], returns
 *   g_dV  [r][nspin][M] double          dL/ddV  (the response to g_drho itself:
 *                                       the map dV -> delta rho is symmetric)
 *   g_Psi [nspin][N][M] (Psi's type)    dL/dPsi = 2 (s/dv) (Gamma Psi) o g
 *                                                 + 2 (dH' Psi) o dV, summed over k
 *   g_eps [nspin][N] double             dL/deps through the divided differences
 *                                       (second divided differences of f, Eq. (22)),
 *                                       f', mu' and mu(eps) (Eq. (1))
 * with dH' = F o A - nu diag(f'), A = (s/dv) Psi diag(g) Psi^T, nu the Fermi
 * shift of A (text after Eq. (24)).  Inputs as for density_response; Gamma and
 * H' are recomputed, nothing of the forward call is kept.  Any of the three
 * outputs may be NULL (not computed); g_Psi may not alias Psi.  FP64 outputs
 * are written whatever prec is; prec selects the arithmetic of the two
 * projections, the back-projection and the rotation for g_Psi (FP64; FP32 on
 * FP32 matrix cores; BF16X3 on three-piece BF16 operands), whose K-tile sums
 * are accumulated in FP64 in every form. */
lrdm_status density_response_backward(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                      const double* eps, int32_t N, const lrdm_occ* occ,
                                      const double* dV, int32_t r, lrdm_prec prec,
                                      const double* g_drho, double* g_dV, void* g_Psi,
                                      double* g_eps);

/* ------------------------------------------------- low-rank step and model SCF */

/* Output density of Eq. (1) per channel,
 *   rho_c(x_p) = (s/dv) sum_i f_c,i Psi_c,ip^2,
 * with mu and f from eps as in lrdm_fermi_occupations.  With rho_in non-NULL the
 * output is the SCF residual R[rho_in] = rho - rho_in (Sec. II A) instead.
 * Psi [nspin][N][M] (double for LRDM_FP64, float otherwise; the sum is FP64);
 * eps [nspin][N]; rho_in, out [nspin][M] double (out may be rho_in, never Psi or
 * eps); mu [1] device double, may be NULL. */
lrdm_status lrdm_density(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                         const double* eps, int32_t N, const lrdm_occ* occ, lrdm_prec prec,
                         const double* rho_in, double* out, double* mu);

/* Effective potential of the model SCF: V_eff = V_ext + K_c (sum_c rho_c), the
 * Hartree potential of the total density with the kernel of lrdm_hartree_kernel,
 * plus, when vxc is non-NULL, the exchange-correlation potential of each channel
 * (Eq. (1); vxc from lrdm_lda_xc).  V_ext [M]; rho, vxc [nspin][M]; V_eff [M]
 * without vxc, [nspin][M] with it; all double; V_eff overlaps no input.  range
 * (device double [2], may be NULL) receives min and max of V_eff over all its
 * channels, e.g. for the Chebyshev filter's upper bound. */
lrdm_status lrdm_effective_potential(lrdm_ctx* ctx, const lrdm_grid* grid, const double* V_ext,
                                     const double* rho, int32_t nspin, const double* vxc,
                                     double* V_eff, double* range);

/* Local-density exchange-correlation at every grid point (the K_xc part of K in
 * Eq. (3), Sec. II D for two channels): with e(rho) the LDA energy per volume,
 * Slater exchange (spin-scaled for two channels) plus the Perdew-Zunger (1981)
 * fit of the Ceperley-Alder correlation energy, interpolated between the
 * unpolarised and the fully polarised gas with the von Barth-Hedin function,
 *   vxc[s] = de/drho_s,  fxc[s][t] = d^2 e / drho_s drho_t.
 * nspin 1 takes the total density.  Points where a channel density is below
 * 1e-12 get vxc = fxc = 0.  rho, vxc [nspin][M], fxc [nspin][nspin][M], double;
 * vxc or fxc may be NULL; no overlaps. */
lrdm_status lrdm_lda_xc(lrdm_ctx* ctx, const lrdm_grid* grid, const double* rho, int32_t nspin,
                        double* vxc, double* fxc);

/* lrdm_residual_derivative with K = K_c + K_xc: channel c of direction k sees
 * dV_k,c = K_c (sum_s u_k,s) + sum_d fxc[c][d] u_k,d, with fxc [nspin][nspin][M]
 * the LDA kernel at the current density (lrdm_lda_xc). */
lrdm_status lrdm_residual_derivative_xc(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                                        const double* eps, int32_t N, const lrdm_occ* occ,
                                        const double* u, int32_t r, lrdm_prec prec,
                                        const double* fxc, double* t);

/* Parameters of the low-rank step (Sec. II B).  Values the paper uses (Sec.
 * III A): s_tol 0.2-0.3, alpha 0.1 until ||R|| goes below 2.0 and 0.5 from then
 * on (alpha_far 0.1, alpha_near 0.5, alpha_switch 2.0), and for the accumulated
 * variant at most 5 new directions per SCF step, accumulating only while ||R||
 * < 1.0 (a gate the driver applies, not this step).  The step takes alpha from
 * the current ||R||; a driver that keeps alpha_near once the switch is made
 * passes alpha_switch = +inf on the later steps. */
typedef struct {
  double s_tol;       /* stop at the first rank whose s_rel (Eq. (10)) is below s_tol (>= 0) */
  int32_t r_max;      /* capacity of U and T in directions, 1..64 (kept + new) */
  double alpha_far;   /* damping while ||R|| >= alpha_switch, in (0, 1] */
  double alpha_near;  /* damping when ||R|| < alpha_switch, in (0, 1] */
  double alpha_switch; /* threshold on ||R|| (>= 0, +inf allowed: always alpha_near) */
  int32_t r_add_max;  /* new directions this call: k > 0 at most k, 0 up to r_max,
                         -1 none (fit R with the kept directions only) */
} lrdm_lowrank_params;

/* What a low-rank step did (host struct). */
typedef struct {
  int32_t rank;       /* directions used, kept + new (0 for R = 0 without kept ones) */
  int32_t added;      /* new directions computed by this call */
  double s_rel;       /* Eq. (10) at that rank */
  double norm_R;      /* ||R||, the norm of the cell integral (direct sum over channels) */
  double alpha;       /* damping chosen from norm_R */
  double norm_R_lin;  /* ||R - alpha I_r^t R||: the residual the approximation predicts
                         after the update (Eq. (12)); its ratio to the next ||R|| gives
                         the linearity indicator beta of Eq. (13) */
} lrdm_lowrank_info;

/* One LRDM step (Sec. II B) or, with kept directions, one accumulated LRDMA
 * step (Sec. II B 1, Eq. (14)).  In the inner product <a, b> = dv sum over
 * points and channels:
 *  - the first r_keep rows of U and T hold directions (orthonormal) and their
 *    derivatives kept from earlier SCF steps; they are fitted to R first, and if
 *    s_rel < s_tol already (or r_add_max = -1) nothing is added;
 *  - otherwise new directions are added one at a time: the first is R with its
 *    components along the kept u's removed (for r_keep = 0, R/||R||), each later
 *    one the newest t with its components along all u's removed (Eq. (8)), both
 *    normalised; each new t = chi0 K u - u is computed as in
 *    lrdm_residual_derivative (Eq. (7); K = K_c, or K_c + K_xc with fxc
 *    non-NULL as in lrdm_residual_derivative_xc), one direction per launch
 *    sequence;
 *  - after each t: S_ij = <t_i, t_j>, c_j = <t_j, R>, y = S^{-1} c (Cholesky on
 *    the GPU) and s_rel = ||sum_j y_j t_j - R|| / ||R|| (Eq. (10)); adding stops
 *    when s_rel < s_tol, at r_add_max new, at r_max in all, or when a new
 *    direction would vanish (the fit is then exact);
 *  - drho = sum_i y_i u_i = P^lr_r R (Eq. (9)) over all directions; with rho
 *    non-NULL also rho <- rho - alpha drho (Eq. (4)), alpha from the schedule.
 * The orthogonalisation is applied twice, which leaves the span and drho
 * unchanged and keeps u orthonormal in floating point.  Psi, eps, N, occ, prec
 * as for lrdm_residual_derivative; R, drho, rho [nspin][M] double; U, T
 * [r_max][nspin][M] double, rows r_keep.. written (the first info->rank are
 * meaningful); no two of R, U, T, drho, rho overlap.  Synchronises the stream
 * once per new direction and once for the kept fit.  Errors as for
 * lrdm_residual_derivative, plus EINVAL for params out of range or r_keep
 * outside 0..r_max, ENONFINITE for a non-finite ||R|| and ENOTCONV when S is
 * not numerically positive definite. */
lrdm_status lrdm_lowrank_step(lrdm_ctx* ctx, const lrdm_grid* grid, const void* Psi,
                              const double* eps, int32_t N, const lrdm_occ* occ, lrdm_prec prec,
                              const double* R, const lrdm_lowrank_params* params, int32_t r_keep,
                              const double* fxc, double* U, double* T, double* drho, double* rho,
                              lrdm_lowrank_info* info);

/* ---------------------------------------------------------------- autotuner */

/* Chooses, for three shapes at this grid, N, nspin, r and form, the layout of
 * tiles and waves of the projection kernel and its K-split count (the number of
 * point ranges whose FP64 partial sums are added afterwards): the response's
 * projection of r*nspin directions, the single-direction projection of
 * lrdm_lowrank_step, and the unweighted Gram product of subspace_rayleigh_ritz
 * (FP64 arithmetic).  Layouts (variants): 0, eight waves of 32 x 64 on a
 * 128 x 128 tile with the operands copied to LDS through a three-stage ring
 * (BF16X3: the unweighted operand split into its pieces once per call); 1, four
 * waves of 64 x 64 on the same tile with the operands staged through
 * registers; 2 (BF16X3 only), the ring kernel splitting both operands itself.
 * FP64 arithmetic has layout 0 only, FP32 layouts 0 and 1.  Each candidate
 * (layout, count of 1/4, 1/2, 1 and 2 times the default within 1..the
 * workspace's cap) is timed (one warm-up, three timed launches, hipEvents) on
 * scratch blocks the call allocates and frees, and the fastest is kept on this
 * context for later calls of the same shape (the batched FP32 response sends a
 * system whose shape is tuned to layout 1 to its own launch).  splits and
 * variants (host int[3], may be NULL) receive the choices; timings (host
 * double[3][3][4], may be NULL) the milliseconds per shape, layout and count, 0
 * where not tried.  In the BF16X3 form it also times both back-projection
 * layouts (lrdm_set_backproj_layout) on the response's shape and keeps the
 * faster on the context; backproj_layout (host int, may be NULL) receives the
 * layout in use afterwards, backproj_ms (host double[2], may be NULL) the
 * milliseconds of layouts 0 and 1 (0 when not timed).  Synchronises.  For the
 * callers that tune once at set-up, not for those that cannot allocate. */
lrdm_status lrdm_autotune(lrdm_ctx* ctx, const lrdm_grid* grid, int32_t N, int32_t nspin,
                          int32_t r, lrdm_prec prec, int32_t* splits, int32_t* variants,
                          double* timings, int32_t* backproj_layout, double* backproj_ms);

#ifdef __cplusplus
}
#endif

#endif /* LRDM_H */

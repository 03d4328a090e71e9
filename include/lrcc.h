/*
 * lrcc.h -- C ABI of the MI355X (gfx950) particle-particle-ladder library.
 *
 * The library computes the particle-particle-ladder (PPL) part of the
 * Cholesky-decomposed relativistic LR-CCSD Jacobian product and the model
 * response solve built on it (paper: Sec. 2.2 response equations and
 * Jacobian; Sec. 3, integrals with more than two particle indices rebuilt on
 * the fly from Cholesky vectors):
 *
 *   <ab|cd>      = sum_P L^P_ac L^P_bd           (never stored)
 *   <ab||cd>     = <ab|cd> - <ab|dc>
 *   sigma_ij^ab  = sum_{c,d} <ab||cd> X_ij^cd     (unrestricted c,d sum)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array pointers are DEVICE pointers unless marked (host).  Buffers are
 *   contiguous, row-major, complex values interleaved (re, im), and at least
 *   8-byte aligned (16-byte for complex128).  The caller owns every buffer;
 *   the library never frees caller memory.
 * - Cholesky vectors: L[P][a][c] = L^P_ac, shape [nchol][v][v].
 * - Doubles (X, sigma, gradients): packed [nrhs][o(o-1)/2][v(v-1)/2]; the pair
 *   index of p<q among n is p(2n-p-1)/2 + (q-p-1) (row-major upper
 *   triangle), the same formula for (i,j) with n=o and (a,b) with n=v.
 * - Every function returns an lrcc_status.  Nothing throws or aborts across
 *   the ABI.  Argument errors are found before any launch and leave every
 *   output untouched; lrcc_last_error() then names the argument.
 * - lrcc_ppl_sigma and lrcc_ppl_sigma_adjoint are stream-ordered and
 *   asynchronous on the handle's stream.  lrcc_solve and lrcc_solve_batched
 *   are synchronous and return alpha on the host.
 * - A handle owns a grow-only device workspace and is not thread-safe;
 *   separate handles are independent.
 */
#ifndef LRCC_H
#define LRCC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LRCC_OK = 0,
  LRCC_ERR_ARG = 1,            /* null pointer, bad enum, negative size       */
  LRCC_ERR_SHAPE = 2,          /* sizes inconsistent or beyond the limits     */
  LRCC_ERR_DTYPE = 3,          /* dtype/precision combination not offered     */
  LRCC_ERR_DEVICE = 4,         /* no gfx950 device, or a HIP runtime failure  */
  LRCC_ERR_NOMEM = 5,          /* workspace allocation failed                 */
  LRCC_ERR_NOT_CONVERGED = 6,  /* solve hit max_iter; info is still filled    */
  LRCC_ERR_NONFINITE = 7,      /* NaN/Inf met in a residual or norm           */
  LRCC_ERR_UNSUPPORTED = 8,    /* valid request the library does not offer    */
  /* range markers (not returned): the enum spans every int, so that
   * lrcc_status_str accepts any value */
  LRCC_STATUS_RANGE_MIN = -0x7fffffff - 1, LRCC_STATUS_RANGE_MAX = 0x7fffffff
} lrcc_status;

/* Input enums.  The *_RANGE_MIN / *_RANGE_MAX markers are not values to
 * pass: they make each enum span every int, so that an out-of-range
 * argument is a well-defined value the validation rejects (LRCC_ERR_ARG). */
typedef enum {
  LRCC_C128 = 0, LRCC_C64 = 1,                                   /* storage of L, X, sigma */
  LRCC_DTYPE_RANGE_MIN = -0x7fffffff - 1, LRCC_DTYPE_RANGE_MAX = 0x7fffffff
} lrcc_dtype;
typedef enum {
  LRCC_FP64 = 0, LRCC_FP32 = 1, LRCC_BF16X3 = 2,                 /* PPL arithmetic */
  LRCC_PREC_RANGE_MIN = -0x7fffffff - 1, LRCC_PREC_RANGE_MAX = 0x7fffffff
} lrcc_prec;
typedef enum {
  LRCC_CMUL_4M = 0, LRCC_CMUL_3M = 1,                            /* complex product form */
  LRCC_CMUL_RANGE_MIN = -0x7fffffff - 1, LRCC_CMUL_RANGE_MAX = 0x7fffffff
} lrcc_cmul;

typedef struct lrcc_handle_s* lrcc_handle;

/* Create a handle on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Fails with LRCC_ERR_DEVICE when
 * the device is not gfx950. */
lrcc_status lrcc_create(lrcc_handle* h, int device, void* hip_stream);
/* Free the handle and its workspace (waits for its stream first). */
lrcc_status lrcc_destroy(lrcc_handle h);
/* Change the stream later calls are issued on. */
lrcc_status lrcc_set_stream(lrcc_handle h, void* hip_stream);

/* sigma = PPL(L, X).
 * o, v     occupied / virtual counts (o>=0, v>=0; pairs need o,v>=2, else the
 *          packed extent is 0 and the call returns LRCC_OK doing nothing).
 * nchol    number of Cholesky vectors (0 gives sigma = 0).
 * nrhs     number of independent doubles vectors.
 * L        [nchol][v][v] complex in `dt`.
 * X        [nrhs][o(o-1)/2][v(v-1)/2] complex in `dt`.
 * sigma    same shape and dtype as X; overwritten, never accumulated.  May not
 *          alias X or L.
 * prec     arithmetic of the ladder GEMMs: FP64, FP32 (FP32 MFMA with FP32
 *          accumulation inside a tile) or BF16X3 (split hi/lo bf16 MFMA, FP32
 *          accumulation).  Sums across tiles are kept in FP64 for C128 output.
 * cmul     4M (four real products per complex product) or 3M (three).
 * Limits: v <= 4096, nchol <= 65536, nrhs*o(o-1)/2 <= 2^24.
 * When every L^P is Hermitian (L^P_ca == conj L^P_ac, tested exactly on the
 * device during the call) the ladder operator is Hermitian and each integral
 * tile is built once for a pair of block pairs and also used as its
 * conjugate transpose (half the builds); for any other L both tiles are
 * built.  The two routes agree up to rounding order. */
lrcc_status lrcc_ppl_sigma(lrcc_handle h, int o, int v, int nchol, int nrhs,
                           const void* L, const void* X, void* sigma,
                           lrcc_dtype dt, lrcc_prec prec, lrcc_cmul cmul);

/* sigma = PPL(L, X) without allocating: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments, result and errors as lrcc_ppl_sigma,
 * for prec FP64 or FP32 (BF16X3: LRCC_ERR_UNSUPPORTED).  Every intermediate
 * (block-pair table, tile order, Hermiticity flag, staged L, block-layout X
 * and the sigma accumulator) lives in one static device array of 64 MiB per
 * GPU, held from library load until the process ends; a problem that needs
 * more (about (v/8)^2 nchol KB of staged FP64 vectors plus three copies of
 * the padded doubles) returns LRCC_ERR_SHAPE before any launch.  The call
 * issues kernel launches only (no allocation, host copy or memset), on the
 * handle's stream.  All calls on one GPU share that array and each clears
 * what it reads before use: calls that can overlap on one GPU (different
 * streams or handles without ordering between them) race and must be
 * serialised by the caller.  The deterministic mode (lrcc_set_deterministic)
 * does not apply: the call runs the default kernels. */
lrcc_status lrcc_ppl_sigma_noalloc(lrcc_handle h, int o, int v, int nchol, int nrhs,
                                   const void* L, const void* X, void* sigma,
                                   lrcc_dtype dt, lrcc_prec prec, lrcc_cmul cmul);

/* Vector-Jacobian products of sigma = PPL(L, X) for a real loss with
 * upstream gradient G = dloss/dsigma (PyTorch's complex convention:
 * dloss = Re sum conj(grad) d(input)).  dX is the product with the
 * transposed (adjoint) ladder, the operation the left-hand amplitude
 * equation of Sec. 2.2 applies (Y (A + w) = -(eta + F X) multiplies by the
 * Jacobian from the left); dL differentiates the on-the-fly integrals of
 * Sec. 3 with respect to the Cholesky vectors.
 *   dX = sigma(L^H, G)                  (the adjoint ladder; (L^H)^P = (L^P)^H)
 *   dL^P = 2 sum_m G_m conj(L^P) X_m^H  (G_m, X_m full antisymmetric v x v)
 * Either output may be NULL to skip it.  dX has the shape of X, dL of L; both
 * are overwritten.  The ladder tiles are recomputed, never stored. */
lrcc_status lrcc_ppl_sigma_adjoint(lrcc_handle h, int o, int v, int nchol, int nrhs,
                                   const void* L, const void* X, const void* G,
                                   void* dX, void* dL,
                                   lrcc_dtype dt, lrcc_prec prec, lrcc_cmul cmul);

/* Hole-hole ladder alone (a model extension of the Jacobian next to the
 * particle-particle ladder): sigma_ij^ab = sum_{k,l} <kl||ij> X_kl^ab with
 * <kl|ij> = sum_P L^P_ki L^P_lj over occupied-occupied Cholesky vectors
 * Loo[nchol][o][o] (device, dtype dt, Loo[P][k][i] = L^P_ki), the
 * unrestricted k, l sum as in lrcc_ppl_sigma.  X and sigma: packed doubles as
 * in lrcc_ppl_sigma (device; sigma overwritten).  FP64 arithmetic.  The
 * integrals <kl||ij> (no particle index) are formed explicitly, npo x npo.
 * Asynchronous on the handle's stream. */
lrcc_status lrcc_hhl_sigma(lrcc_handle h, int o, int v, int nchol, int nrhs, const void* Loo,
                           const void* X, void* sigma, lrcc_dtype dt);

/* Ring (particle-hole) term of the doubles-doubles Jacobian at zero
 * ground-state amplitudes (Sec. 2.2), integrals from the Cholesky vectors of
 * one decomposition over all spinors (Sec. 3):
 *   <kb||cj> = sum_P L^P_kc L^P_bj - sum_P L^P_kj L^P_bc,
 *   sigma_ij^ab = P(ij) P(ab) sum_{k,c} <kb||cj> X_ik^ac
 * (P(ij) f = f - f with i, j swapped; the k, c sum unrestricted, no factor).
 * Inputs (device, complex128): L_oo [nchol][o][o], L_ov [nchol][o][v],
 * L_vo [nchol][v][o], L_vv [nchol][v][v] (L_xx[P][p][q] = L^P_pq; for a
 * Hermitian decomposition L_vo[P] = L_ov[P]^H), X packed doubles as in
 * lrcc_ppl_sigma.  sigma (device, packed, overwritten).  FP64 arithmetic;
 * the particle-hole integral matrix, (o v)^2 entries, is formed explicitly,
 * and the workspace holds about (1 + 2 max(1, nrhs)) (o v)^2 complex numbers.
 * Asynchronous on the handle's stream.  Errors: LRCC_ERR_ARG for NULL,
 * misaligned or overlapping buffers and negative sizes; LRCC_ERR_SHAPE for
 * o v > 65535 or nrhs o v >= 2^31. */
lrcc_status lrcc_ring_sigma(lrcc_handle h, int o, int v, int nchol, int nrhs, const void* L_oo,
                            const void* L_ov, const void* L_vo, const void* L_vv, const void* X,
                            void* sigma);

/* Pivoted (single-step) Cholesky decomposition of a two-electron integral
 * matrix (Sec. 3): M (device, n x n complex128, row-major, Hermitian positive
 * semi-definite; M[i][p] is read for the pivot column p) is decomposed as
 * M ~= sum_q L_q L_q^H, one vector at a time at the pivot of the largest
 * remaining diagonal element (the first index among equal values), until
 * that element is <= tau or max_vectors (capped at n) vectors exist.
 * L (device, [max_vectors][n] complex128) receives the vectors, pivots
 * (device, [max_vectors] int, nullable) their pivots, *nvec (host) the
 * count.  Synchronous: returns when the decomposition is complete.  Errors:
 * LRCC_ERR_ARG for NULL/misaligned/overlapping buffers, negative sizes or a
 * tau that is negative or not finite; LRCC_ERR_SHAPE for n > 2^20. */
lrcc_status lrcc_cholesky(lrcc_handle h, long n, const void* M, double tau, int max_vectors,
                          void* L, int* pivots, int* nvec);

/* Hermitian eigen-decomposition A = V diag(w) V^H by two-sided Jacobi
 * rotations (used for the natural spinors and the semicanonicalisation of
 * Sec. 2.3; exposed on its own for testing and reuse).  A: device, n x n
 * complex128, row-major, Hermitian (not checked), not modified.  w: device [n], the
 * eigenvalues in ascending order.  V: device [n][n] complex128, column k the
 * eigenvector of w[k] (phases arbitrary); may be NULL.  *sweeps (host, may
 * be NULL): Jacobi sweeps used.  Synchronous.  Errors: LRCC_ERR_ARG for
 * NULL/misaligned/overlapping buffers or n < 0; LRCC_ERR_SHAPE for n > 8192. */
lrcc_status lrcc_heev(lrcc_handle h, int n, const void* A, double* w, void* V, int* sweeps);

typedef struct {
  int sweeps_density;  /* Jacobi sweeps of the density diagonalisation      */
  int sweeps_fock;     /* Jacobi sweeps of the truncated Fock block          */
} lrcc_fns_info;

/* Perturbation-sensitive natural spinors (FNS++) of the virtual space,
 * Sec. 2.4 with the steps of Sec. 2.3, for a canonical reference:
 *   t_ij^ab = <ij||ab> / (e_i + e_j - e_a - e_b), <ij|ab> = sum_P L_ia L_jb,
 *   Hb_ii = e_i + 1/2 sum t_in^ef conj<in||ef>,
 *   Hb_aa = e_a - 1/2 sum t_mn^fa conj<mn||fa>,
 *   per component x: Ab_ij^ac = P(a,c) sum_e t_ij^ec A_ae
 *                               - P(i,j) sum_m t_mj^ac A_mi,
 *   t_ij^ac(A) = Ab / (Hb_aa + Hb_cc - Hb_ii - Hb_jj + omega),
 *   t_i^a(A) = A_ia / (Hb_aa - Hb_ii + omega),
 *   G_ab = mean_x [1/2 sum_ijc t_ij^ac(A) conj t_ij^bc(A)
 *                  + sum_i t_i^a(A) conj t_i^b(A)],
 *   G V = V diag(n), |n| descending; keep the |n| > threshold columns Vt;
 *   Ft = Vt^H diag(e_v) Vt = Z diag(eps_new) Z^H (ascending); B = Vt Z.
 * Inputs (device): eps [o+v] float64 (occupied first), Lov [nchol][o][v]
 * complex128 (Lov[P][i][a] = L^P_ia), A_ov [ncomp][o][v]
 * (A_ov[x][i][a] = <a|A_x|i>), A_vv [ncomp][v][v] (<a|A_x|e> at [x][a][e]),
 * A_oo [ncomp][o][o] (<m|A_x|i> at [x][m][i]); omega and threshold (>= 0)
 * are host doubles.  Outputs (device unless noted): occ [v] the occupation
 * numbers in the order above (nullable); B [v][keep] complex128, written
 * compactly (row stride keep) into a buffer of v*v elements; eps_new [keep]
 * in a buffer of v doubles; *keep (host); gamma [v][v] the averaged density
 * (nullable); hbar [o+v] the dressed diagonals (nullable).  A direction-
 * specific basis (the alternative to averaging that Sec. 2.4 mentions) is
 * a call with that one component.  Workspace about
 * 3.5 (o v)^2 complex numbers, kept in the handle.  Synchronous.  Errors:
 * LRCC_ERR_ARG for NULL/misaligned/overlapping buffers, negative sizes, a
 * threshold that is negative or not finite or an omega that is not finite;
 * LRCC_ERR_SHAPE for o > 255, v > 8192 or o v^2 >= 2^31. */
lrcc_status lrcc_fns_plus(lrcc_handle h, int o, int v, int nchol, const double* eps,
                          const void* Lov, int ncomp, const void* A_ov, const void* A_vv,
                          const void* A_oo, double omega, double threshold, double* occ,
                          void* B, double* eps_new, int* keep, void* gamma, double* hbar,
                          lrcc_fns_info* info);

/* The Cholesky vectors and the occupied-virtual dipole block in the kept
 * FNS++ basis (the basis change of Sec. 2.3 applied to the quantities of
 * the response solve): Lt^P = B^H L^P B and mu_t[x][i][l] = sum_a
 * mu[x][i][a] conj(B[a][l]) (mu[x][i][a] = <a|mu_x|i> has the virtual in
 * the bra).
 * B: device [v][k] complex128 (lrcc_fns_plus's output, row stride k).
 * L: device [nchol][v][v], Lt: device [nchol][k][k]; mu: device
 * [ncomp][o][v], mu_t: device [ncomp][o][k]; either pair may be NULL to skip
 * it.  The new spinor energies are lrcc_fns_plus's eps_new.  Asynchronous on
 * the handle's stream.  Errors: LRCC_ERR_ARG for NULL B with work to do,
 * misaligned or overlapping buffers, negative sizes or k > v. */
lrcc_status lrcc_fns_transform(lrcc_handle h, int v, int k, int nchol, int ncomp, int o,
                               const void* B, const void* L, const void* mu, void* Lt,
                               void* mu_t);

/* Options of the response solve.  Zero-initialised fields take defaults. */
typedef struct {
  double tol;        /* relative residual |R|/|xi| (default 1e-8)            */
  int max_iter;      /* FP64 iterations, or inner iterations per refinement
                        sweep for reduced precision (default 100)            */
  int diis_dim;      /* DIIS subspace size, 1 = plain Jacobi (default 8)     */
  lrcc_prec prec;    /* ladder arithmetic of the inner iterations            */
  lrcc_cmul cmul;    /* complex form of the FP64 and FP32 ladders (the FP64
                        solve, the refinement's anchor and an FP32 inner
                        ladder); bf16x3 ladders always use 4M                */
  double inner_tol;  /* reduced precision: inner relative tolerance (1e-5)   */
  int max_outer;     /* reduced precision: refinement sweeps (default 6)     */
  int deterministic; /* 1: deterministic ladders for this solve (see
                        lrcc_set_deterministic); 0 (default): the handle's
                        setting.  lrcc_solve_batched: 0 only                  */
  int resid_fp64_every; /* reduced precision: 0 (default) = the stopping
                        test's ladder of the iterate is a full FP64 ladder in
                        the first sweep only, later sweeps update it by the
                        reduced-precision ladder of the correction (the
                        ladder is linear); 1 = a full FP64 ladder every sweep.
                        Either way the reported residual is an FP64 one (see
                        lrcc_solve_info.final_relres)                         */
  lrcc_prec anchor_prec; /* reduced precision: arithmetic of that full-iterate
                        ladder: FP64 (default) or FP32 (a cheaper stopping
                        test, exact to FP32 ladder accuracy, about 1e-6
                        relative; the FP64 residual is then evaluated once
                        more at the end).  Inside the solve an FP32 ladder
                        sums its tile partials in FP32 too                   */
  int response;      /* 0 (default): alpha_xy(w) = -<xi_x | X_y(w)> from the
                        right-hand amplitudes only.  1: the full linear
                        response function of Sec. 2.2 (last equation): the
                        left-hand amplitudes Y(w) solve Y (A + w) = -eta,
                        eta = conj(xi) and F = 0 in this model, i.e.
                        (A^T + w) Y^T = -eta, a second solve with the
                        transposed ladder K(L^T) = K(L)^T; then
                        alpha_xy = (s_xy + conj s_yx) / 2 with
                        s = -<xi_x|X_y(w)> - sum xi_x Y_y(w).  For Hermitian
                        L this is alpha_R(w) + conj(alpha_R(-w)), both terms
                        of the sum-over-states form.  lrcc_solve_batched
                        supports 0 only                                      */
  const void* L_oo;  /* (device) NULL (default), or occupied-occupied
                        Cholesky vectors [nchol][o][o] complex128,
                        L_oo[P][k][i] = L^P_ki: the model Jacobian then also
                        holds the hole-hole ladder
                          HHL = sum_{k,l} <kl||ij> X_kl^ab, <kl|ij> = sum_P
                          L^P_ki L^P_lj,
                        which couples the occupied pairs (applied in FP64
                        whatever prec is), and its two-electron part becomes
                        the doubles-doubles block of the two-electron
                        operator at T = 0 (Sec. 2.2): 1/2 sigma + 1/2 HHL
                        (+ the ring term with L_ov), sigma and HHL being the
                        unrestricted sums of lrcc_ppl_sigma and
                        lrcc_hhl_sigma.  Without it the two-electron part is
                        sigma alone.  lrcc_solve_batched: NULL only          */
  const void* L_ov;  /* (device) NULL (default), or occupied-virtual
                        Cholesky vectors [nchol][o][v] complex128 (needs
                        L_oo and L_vo): the model Jacobian then also holds
                        the ring term of lrcc_ring_sigma, built from L_oo,
                        L_ov, L_vo and L (its particle-hole integral matrix
                        formed once per solve side, applied in FP64 whatever
                        prec is).  lrcc_solve_batched: NULL only            */
  const void* L_vo;  /* (device) virtual-occupied vectors [nchol][v][o]
                        complex128 with L_ov; for a Hermitian decomposition
                        L_vo[P] = L_ov[P]^H                                  */
  const void* x0;    /* (device) NULL (default: the Jacobi start
                        X = -xi / (D - w)), or initial right-hand amplitudes
                        [nomega][ncomp][o(o-1)/2][v(v-1)/2] complex128 (a
                        warm start, e.g. the converged X of a neighbouring
                        frequency).  With reduced precision the refinement
                        starts from it (one full-iterate ladder more).
                        lrcc_solve_batched: NULL only                        */
  void* x_out;       /* (device) NULL, or [nomega][ncomp][o(o-1)/2][v(v-1)/2]
                        complex128 receiving the final right-hand amplitudes
                        (the iterate alpha is computed from).
                        lrcc_solve_batched: NULL only                        */
  const char* metrics_path; /* (host) NULL, or a file that receives one JSON
                        line per iteration, appended: side ("right" / "left"),
                        phase ("fp64": the FP64 solve, "inner": a reduced-
                        precision inner iteration, "outer": a refinement
                        sweep's residual, "final": the FP64-ladder residual of
                        the returned amplitudes when the last sweep's was an
                        estimate), sweep, iter, active
                        right-hand sides, ms since the call began and every
                        right-hand side's relative residual.  A file that
                        cannot be opened gives LRCC_ERR_ARG                   */
} lrcc_solve_opts;

typedef struct {
  int iters_max;        /* most iterations any right-hand side took          */
  int n_sigma_fp64;     /* FP64 ladder applications                          */
  int n_sigma_lowp;     /* reduced-precision ladder applications             */
  double final_relres;  /* largest final relative residual |R|/|xi| of the
                           returned amplitudes, R = -xi - (A - w) X with the
                           ladder of X applied in FP64.  The FP64 solve's last
                           iteration gives it; a refinement whose last stopping
                           test was not a full FP64 ladder of X applies one
                           more FP64 ladder at the end for it (counted in
                           n_sigma_fp64), and its status follows that residual */
  double seconds;       /* wall time of the call                             */
} lrcc_solve_info;

/* Model response solve (paper Sec. 2.2): for every dipole component x and
 * frequency w, solve (A - w) X = -xi_x with (A X) = D o X + sigma(X),
 * D_ij^ab = e_a + e_b - e_i - e_j, xi_ij^ab = mu_ia mu_jb - mu_ib mu_ja, by
 * Jacobi + DIIS (reduced precision: iterative refinement around it), then
 * alpha_xy(w) = -<xi_x | X_y(w)>.
 * eps    [o+v] float64, occupied first (device).
 * L      [nchol][v][v] complex128 (device).
 * mu     [ncomp][o][v] complex128 dipole ov block (device).
 * omegas (host) [nomega] float64.
 * alpha  (host) [nomega][ncomp][ncomp] complex128 interleaved.
 * info   (host) nullable.
 * Returns LRCC_ERR_NOT_CONVERGED if any RHS misses tol (alpha still written). */
lrcc_status lrcc_solve(lrcc_handle h, int o, int v, int nchol,
                       const double* eps, const void* L,
                       int ncomp, const void* mu,
                       int nomega, const double* omegas,
                       const lrcc_solve_opts* opts,
                       double* alpha, lrcc_solve_info* info);

/* One instance of a batched solve; all pointers as in lrcc_solve. */
typedef struct {
  int o, v, nchol;
  const double* eps;   /* device */
  const void* L;       /* device, complex128 */
  int ncomp;
  const void* mu;      /* device, complex128 */
  int nomega;
  const double* omegas;/* host */
  double* alpha;       /* host, [nomega][ncomp][ncomp] complex128 */
} lrcc_instance;

/* Solve several uneven instances together: the response equations of
 * Sec. 2.2, one per perturbation component and frequency of each instance
 * (each instance a molecule or basis of its own size), iterated side by
 * side.  With opts->prec = LRCC_FP64 every ladder application of every
 * instance, component and frequency goes into one persistent launch per
 * iteration (a work queue ordered longest tile first), each iteration
 * replayed from a captured HIP graph.  With LRCC_FP32 or LRCC_BF16X3 the
 * solve refines the response equations of Sec. 2.2 iteratively: in each sweep
 * the correction equations of the instances with unconverged right-hand
 * sides are solved to opts->inner_tol with the reduced-precision ladder,
 * one instance after another (their DIIS history, reduced-precision
 * doubles and staged vectors are one shared set sized for the largest
 * instance, so memory grows by a per-instance iterate, residual and ladder
 * only), then the FP64 ladder of every refined iterate runs in one
 * persistent launch and gives each right-hand side its FP64 residual, the
 * stopping test against opts->tol (at most opts->max_outer sweeps).
 * info->n_sigma_fp64 counts those persistent launches (iterations of the
 * FP64 solve), info->n_sigma_lowp the reduced-precision ladder applications
 * summed over instances.  opts->anchor_prec must be LRCC_FP64 and
 * opts->resid_fp64_every has no effect (every sweep ends on the FP64
 * ladder).  The complex form of every FP64 / FP32 ladder is opts->cmul. */
lrcc_status lrcc_solve_batched(lrcc_handle h, int ninst, const lrcc_instance* inst,
                               const lrcc_solve_opts* opts, lrcc_solve_info* info);

/* Kernel timing: while enabled, HIP events are recorded on the handle's
 * stream around every ladder-kernel launch (the fused build/antisymmetrise/
 * contract kernel only, not staging or layout kernels).  lrcc_set_timing
 * with enable != 0 clears the totals and starts recording; 0 stops.
 * lrcc_get_timing synchronises the stream and returns the summed kernel
 * milliseconds and the number of launches since timing was enabled. */
lrcc_status lrcc_set_timing(lrcc_handle h, int enable);
lrcc_status lrcc_get_timing(lrcc_handle h, double* ms, long* launches);

/* Deterministic mode (a debugging aid, for separating races from rounding):
 * while enabled, the FP64 and FP32 ladders run a kernel without atomic
 * additions (one workgroup per output block pair builds every integral tile
 * of its row in a fixed order, without the Hermitian halving, 4M complex
 * form whatever cmul is) and the bf16x3 contraction runs unsplit, so that
 * repeated calls give bit-identical results.  Several times slower than the
 * default kernels.  The environment variable LRCC_DETERMINISTIC=1 sets it for
 * new handles.  Applies to lrcc_ppl_sigma, its adjoint's dX and lrcc_solve;
 * lrcc_solve_batched then returns LRCC_ERR_UNSUPPORTED. */
lrcc_status lrcc_set_deterministic(lrcc_handle h, int enable);

/* Workspace limit of the bf16x3 ladder and of the gradient with respect to
 * L.  The bf16x3 path stores antisymmetrised integral tiles (64 KB per tile
 * pair with its mirror) for one panel of block pairs at a time; the panel
 * holds as many rows of the block-pair triangle as fit in `bytes` (at least
 * one row).  The gradient stores the products sum_m conj(G_m) X_m on packed
 * virtual pairs (64 KB per block-pair pair in FP64) for panels of whole
 * block rows the same way.  0 restores the default:
 * min(16 GiB, half the free device memory at first use), overridable by the
 * environment variable LRCC_PANEL_MB.  The workspace itself is allocated on
 * the next bf16x3 ladder and kept by the handle. */
lrcc_status lrcc_set_workspace_limit(lrcc_handle h, size_t bytes);

/* Result of lrcc_autotune. */
typedef struct {
  int supertile;   /* width, in blocks of 8 virtual indices, of the super-tiles
                      that order the tile pairs (see below)                    */
  int occupancy;   /* launch variant of the fused 4M kernel: 1 = one workgroup
                      per CU, chunks through registers; 2 = two per CU (FP32);
                      3 = one per CU, chunks loaded straight into a two-chunk
                      LDS ring; 4 = two per CU with direct LDS loads; 5 = as 3
                      with eight waves per workgroup (two per SIMD)            */
  double ms;       /* ladder kernel time of the chosen variant                 */
  int candidates;  /* variants timed (0 when read from the cache)              */
} lrcc_tune_result;

/* Tile-shape autotuner.  Times the candidate launch variants of the ladder
 * for this shape, precision and complex form on synthetic inputs: the width
 * s in {2, 4, 8} of the super-tiles (tile pairs whose four Cholesky blocks
 * come from s x s block sets are run together on one XCD) and the launch
 * variants of the fused kernel that exist for the precision.  The fastest is kept in the
 * handle for later calls.  cache_path (host, nullable): a text file of
 * earlier results keyed by (arch, CU count, o, v, nchol, nrhs, prec, cmul);
 * a hit skips the timing, a miss appends the new result.  Tuning restarts
 * the totals of lrcc_get_timing.  LRCC_BF16X3 has a single launch form and
 * a fixed work order: nothing is timed (supertile 4, occupancy 1,
 * candidates 0). */
lrcc_status lrcc_autotune(lrcc_handle h, int o, int v, int nchol, int nrhs, lrcc_prec prec,
                          lrcc_cmul cmul, const char* cache_path, lrcc_tune_result* out);

/* Host-only argument check of lrcc_ppl_sigma: runs the same validation and
 * launches nothing (usable without a GPU; h may be NULL). */
lrcc_status lrcc_check_sigma_args(int o, int v, int nchol, int nrhs,
                                  const void* L, const void* X, const void* sigma,
                                  lrcc_dtype dt, lrcc_prec prec, lrcc_cmul cmul);

/* Static text for a status code. */
const char* lrcc_status_str(lrcc_status s);
/* Message of the last failed call on this handle ("" if none; h may be NULL
 * for the last failure of a call made without a handle). */
const char* lrcc_last_error(lrcc_handle h);
/* Library version string. */
const char* lrcc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LRCC_H */

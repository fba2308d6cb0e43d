/*
 * ovl.h -- C ABI of the MI355X (gfx950) overlap-operator library (libovl.so).
 *
 * Method: N. Cundy and W. Lee, "Overlap fermions on GPUs", Lattice 2015 (arXiv:1510.06897).
 *   Sec. 2, eq. 1:  D[mu] = 1/2 (1 + mu + (1 - mu) gamma5 sign(K)),  K = gamma5 (D_W - m_W).
 *   Sec. 2, eq. 2:  (D_W psi)(x) = 4 psi(x) - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
 *                                   + (1 + gamma_mu) U_mu(x - mu)^+ psi(x - mu) ].
 *   Sec. 2, eq. 3:  sign(K) = sum_m alpha_m T_m(K) + sum_i phi_i phi_i^+ [sign(lambda_i)
 *                                   - sum_m alpha_m T_m(lambda_i)].
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice:  dims[4] = {Lx, Ly, Lz, Lt}, each >= 1; V = Lx Ly Lz Lt sites; periodic boundaries in
 *           all four directions; site index x + Lx (y + Ly (z + Lz t)) (x fastest).
 * Gamma matrices: chiral basis, gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 =
 *           [[0, 1], [1, 0]], gamma5 = diag(1, 1, -1, -1).
 * Complex numbers are stored as interleaved (re, im) pairs of the element type.
 * Gauge field (caller layout): U[mu][a][b][site] complex, mu = 0..3 for x, y, z, t, (a, b) the
 *           colour row and column of U_mu(x).
 * Spinors:  psi[r][s][c][site] complex, r < nrhs right-hand sides, spin s < 4, colour c < 3.
 * Polynomial argument: X = K / lmax, lmax an explicit upper bound on ||K||; the coefficient
 *           alpha_m multiplies T_m(X) and the deflation weights use T_m(lambda_i / lmax).
 * dtypes:   OVL_F64 (double), OVL_F32 (float), OVL_BF16 (bfloat16, gauge-link storage only).
 *           Supported operator precisions (spinor dtype / link storage of the gauge handle):
 *           F64 / F64, F32 / F32, F32 / BF16.  F32 and BF16 forms accumulate in FP32; FP64 is
 *           used for the deflation inner products, the Gram-Schmidt basis set-up, the deflation
 *           weights and the final norm check.
 * Pointers: "_dev" pointers are device memory of the current HIP device, "_host" pointers host
 *           memory.  The caller owns every data pointer; the library owns only its handles, the
 *           temporaries it allocates (stream-ordered, freed before the call's work ends) and the
 *           work vectors of its cached step graphs (see ovl_graph_enable).
 * Streams:  every operator is enqueued on the caller's stream (a hipStream_t passed as void*,
 *           NULL for the null stream) and is asynchronous: results are visible after the stream
 *           synchronises.  Calls that share a handle may run on different streams only if they do
 *           not overlap in time.
 * Errors:   every function returns OVL_OK (0) or a negative ovl_status; none throws or aborts.
 *           Arguments are validated on the host before any HIP call; ovl_last_error() returns a
 *           thread-local message for the most recent failure.  Device-detected problems (a
 *           non-finite or diverging recurrence) set sticky flags read by ovl_status_flags().
 * Aliasing: out == in is rejected (OVL_EALIAS): the stencil reads neighbours of the input.
 */
#ifndef OVL_H
#define OVL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OVL_OK = 0,
  OVL_EINVAL = -1,     /* null pointer, bad count, bad enum value                         */
  OVL_EDIMS = -2,      /* lattice extents or sizes out of range / mismatched              */
  OVL_EDTYPE = -3,     /* unsupported dtype or dtype combination                          */
  OVL_EALIAS = -4,     /* output buffer aliases an input that is read at neighbour sites  */
  OVL_ENOMEM = -5,     /* device or host allocation failed                                */
  OVL_EHIP = -6,       /* a HIP runtime call failed (message in ovl_last_error)           */
  OVL_ENONFINITE = -7, /* non-finite coefficient, lmax, mass or eigenvalue                */
  OVL_EDIVERGED = -8,  /* lmax below ||K||: the recurrence grew without bound             */
  OVL_EDEFL = -9       /* deflation basis is rank deficient                               */
} ovl_status;

typedef enum { OVL_F64 = 0, OVL_F32 = 1, OVL_BF16 = 2 } ovl_dtype;

/* sticky device flags (ovl_status_flags) */
#define OVL_FLAG_NONFINITE 0x1u /* a final result held NaN or Inf                     */
#define OVL_FLAG_DIVERGED 0x2u  /* ||result|| exceeded the polynomial's bound * ||in|| */

typedef struct ovl_gauge ovl_gauge; /* packed links on the device (library-owned)     */
typedef struct ovl_poly ovl_poly;   /* Chebyshev coefficients, lmax, m_W (host FP64)  */
typedef struct ovl_defl ovl_defl;   /* orthonormal deflation basis + eigenvalues      */

/* ---- handles ------------------------------------------------------------------------------ */

/* Pack a gauge field (Sec. 2, eq. 2: the links U_mu(x)) into the library's layout and storage
 * dtype.  U_dev: caller layout above, element dtype in_dt (F64 or F32); it is read on `stream`
 * and may be freed once the stream has passed this call.  store_dt: F64, F32 or BF16 (F64 ->
 * F32 -> BF16, each rounding to nearest even).  *g receives the new handle.
 * Errors: EINVAL (null), EDIMS (extent < 1 or > 2^24, V > 2^31), EDTYPE, ENOMEM, EHIP. */
int ovl_gauge_create(ovl_gauge **g, const int32_t dims[4], const void *U_dev, int in_dt,
                     int store_dt, void *stream);
/* Release a handle (synchronises the device first).  NULL is accepted. */
int ovl_gauge_destroy(ovl_gauge *g);
/* Extents and storage dtype of a handle. */
int ovl_gauge_info(const ovl_gauge *g, int32_t dims_out[4], int *store_dt);
/* Two-row link reads (on = 1): every later stencil launch on this handle reads the first two
 * rows of each link and completes the third as conj(row0 x row1), exact for SU(3) matrices, so
 * a K application moves 2/3 of the link bytes (per site FP64 768, FP32 384, BF16 links 288 bytes
 * instead of 960, 480, 336).  The stored third rows stay in place.  Enabling first measures on
 * the device the largest element-wise deviation of the stored third rows from the completed ones
 * (*max_dev, nullable) and refuses with EINVAL when it exceeds tol (links that are not SU(3) to
 * within their storage rounding: FP64 ~1e-15, FP32 ~1e-7, BF16 ~1e-2).  on = 0 switches back to
 * full reads.  Enabling synchronises the stream; a batch launch reads two rows only if every
 * item's handle allows it.  Errors: EINVAL, ENOMEM, EHIP. */
int ovl_gauge_reconstruct(ovl_gauge *g, int on, double tol, double *max_dev, void *stream);

/* Polynomial of Sec. 2, eq. 3: coefficients alpha_host[0..n_alpha-1] of T_0 .. T_{n_alpha-1}
 * (FP64, copied), applied to X = gamma5 (D_W - m_W) / lmax.  n_alpha >= 2 (at least one K
 * application).  Errors: EINVAL (null, n_alpha < 2 or > 100001, lmax <= 0), ENONFINITE. */
int ovl_poly_create(ovl_poly **p, const double *alpha_host, int n_alpha, double lmax, double m_W);
int ovl_poly_destroy(ovl_poly *p);
/* Value of the polynomial sum_m alpha_m T_m(x) at x = lambda / lmax (host, FP64 Clenshaw). */
int ovl_poly_eval(const ovl_poly *p, double lambda, double *value_out);

/* Coefficients for a Chebyshev approximation of sign(x) on eps <= |x| <= 1 (the paper asks for
 * "appropriate coefficients", Sec. 2, eq. 3, and gives none).  Rule: interpolate q(y) ~ y^{-1/2}
 * on [eps^2, 1] at first-kind Chebyshev nodes with degree (N-1)/2, N the largest odd number
 * <= degree; p(x) = x q(x^2) re-expanded exactly in T_m(x).  alpha_host receives N+1 values
 * (alpha_m = 0 for even m).  *n_alpha_out = N + 1.  Host-only, FP64.
 * Errors: EINVAL (degree < 1 or > 100000, eps outside (0, 1), null). */
int ovl_cheb_sign_coeffs(int degree, double eps, double *alpha_host, int *n_alpha_out);

/* Deflation basis of Sec. 2, eq. 3: n_ev eigenvectors phi_i of K (device, spinor layout with
 * nrhs = n_ev, dtype in_dt F64 or F32) and their eigenvalues lambda_host[i] (unscaled).  The
 * vectors are copied to FP64, orthonormalised on the device by classical Gram-Schmidt applied
 * twice (CGS2), and kept in FP64 and in store_dt (F64 or F32) for the operator of that
 * precision.  The weights w_i = sign(lambda_i) - p(lambda_i / lmax) are formed per call from the
 * polynomial handle.  1 <= n_ev <= 12 V.  Errors: EINVAL, EDIMS, EDTYPE, ENONFINITE, ENOMEM,
 * EHIP; EDEFL when a vector is numerically dependent on the previous ones (checked on the host
 * after a stream synchronisation at the end of the call). */
int ovl_defl_create(ovl_defl **d, const int32_t dims[4], const void *phi_dev, int in_dt,
                    const double *lambda_host, int n_ev, int store_dt, void *stream);
int ovl_defl_destroy(ovl_defl *d);
/* Copy of the orthonormal FP64 basis into phi_out_dev ([n_ev][4][3][V] complex double). */
int ovl_defl_basis(const ovl_defl *d, void *phi_out_dev, void *stream);

/* ---- operators ------------------------------------------------------------------------------ */

/* out = (D_W - m_W) in (Sec. 2, eq. 2), or its adjoint gamma5 (D_W - m_W) gamma5 when dagger != 0.
 * in/out: [nrhs][4][3][V] complex of spin_dt, nrhs >= 1.  m_W = 0 gives D_W itself. */
int ovl_wilson_apply(const ovl_gauge *g, void *out, const void *in, int nrhs, int spin_dt,
                     double m_W, int dagger, void *stream);

/* out = K in = gamma5 (D_W - m_W) in (Sec. 2, definition of K). */
int ovl_kernel_apply(const ovl_gauge *g, void *out, const void *in, int nrhs, int spin_dt,
                     double m_W, void *stream);

/* out = c K in + a src + b w for nrhs right-hand sides, K = gamma5 (D_W - m_W) (Sec. 2): one
 * fused stencil launch, the building block of polynomial filters and Krylov updates.  src and w
 * are nullable (their term is dropped); out must not overlap in (the stencil reads neighbours),
 * and src and w must not be in; out may be src or w (each element is read before it is
 * written).  Same layouts, dtypes and errors as ovl_kernel_apply, plus ENONFINITE for a
 * non-finite coefficient. */
int ovl_kernel_axpby(const ovl_gauge *g, void *out, const void *in, double c, const void *src,
                     double a, const void *w, double b, int nrhs, int spin_dt, double m_W,
                     void *stream);

/* out = sum_m alpha_m T_m(X) in + [d != NULL] sum_i phi_i w_i phi_i^+ in  (Sec. 2, eq. 3),
 * evaluated by the Clenshaw recurrence b_k = alpha_k in + 2 X b_{k+1} - b_{k+2}, one fused
 * stencil + polynomial kernel per K application.  n_alpha - 1 K applications. */
int ovl_sign_apply(const ovl_gauge *g, const ovl_poly *p, const ovl_defl *d, void *out,
                   const void *in, int nrhs, int spin_dt, void *stream);

/* out = D[mu] in (Sec. 2, eq. 1) with the sign function above, or D[mu]^+ in = gamma5 D[mu]
 * gamma5 in when dagger != 0.  mu is the overlap mass parameter. */
int ovl_overlap_apply(const ovl_gauge *g, const ovl_poly *p, const ovl_defl *d, double mu,
                      int dagger, void *out, const void *in, int nrhs, int spin_dt, void *stream);

/* ovl_overlap_apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): same arguments, same kernels
 * and launch configuration, same results.  Its work space (one recurrence vector, norm and
 * projection partials and deflation coefficients: about nrhs * 12 V * sizeof(element) bytes plus
 * a few percent) lives in one 64 MiB array of static device memory that every GPU the library
 * runs on holds until the process ends; its address is looked up once per device.  The call
 * makes no hipMalloc, hipFree or other allocation (and no step graph).  Every word of the work
 * space that the call reads it has written before in the same call, so nothing needs clearing.
 * All calls on one GPU share the array: calls that overlap in time on one GPU (other streams,
 * other threads) race on it.  Errors: as ovl_overlap_apply, plus EINVAL when the evaluation needs
 * more than 64 MiB of work space (for example FP64 single right-hand sides above about 340K
 * sites). */
int ovl_overlap_apply_noalloc(const ovl_gauge *g, const ovl_poly *p, const ovl_defl *d, double mu,
                              int dagger, void *out, const void *in, int nrhs, int spin_dt,
                              void *stream);

/* Batched form of ovl_sign_apply (no deflation; Sec. 2, eq. 3): up to 16 lattice problems --
 * each its own gauge field, volume and right-hand-side count -- evaluated with one polynomial in
 * one kernel launch per K application, so small volumes fill the GPU together and the
 * right-hand sides of one field share its links.  All items must have the same operator
 * precision (spin_dt and link storage).  The launch uses the configuration ovl_autotune measured
 * for the same problem set (same item order, extents, right-hand-side counts and precision),
 * else the default rules.  tune_cache_path (nullable): a tuning cache written by ovl_autotune,
 * read the first time this process names it, before the configuration is looked up.
 * Errors as ovl_sign_apply, plus EINVAL (n_items outside [1, 16], unreadable cache) and EALIAS
 * (an output overlapping any item's input or another output). */
typedef struct {
  const ovl_gauge *g; /* gauge field of this item                                  */
  const void *in;     /* [nrhs][4][3][V] complex of spin_dt                        */
  void *out;          /* same shape                                                */
  int nrhs;
} ovl_batch_item;
int ovl_batch_sign_apply(const ovl_batch_item *items, int n_items, const ovl_poly *p, int spin_dt,
                         const char *tune_cache_path, void *stream);

/* c_dev[r][i] = phi_i^+ in_r (complex double, interleaved; n_ev * nrhs entries), FP64
 * accumulation with a deterministic two-pass reduction (Sec. 2, eq. 3 projection). */
int ovl_defl_project(const ovl_defl *d, double *c_dev, const void *in, int nrhs, int spin_dt,
                     void *stream);

/* inout_r += sum_i phi_i (w_host[i] * c_dev[r][i])  (Sec. 2, eq. 3 correction).  With w = 1 it
 * is the adjoint of ovl_defl_project. */
int ovl_defl_correct(const ovl_defl *d, void *inout, const double *c_dev, const double *w_host,
                     int nrhs, int spin_dt, void *stream);

/* ---- link derivatives (HMC fermion force building blocks) -------------------------------- */

/* G_dev[mu][a][b][site] (complex, dtype spin_dt) = dL/dRe U + i dL/dIm U for
 * L = Re <chi, D_W psi> (Sec. 2, eq. 2 is affine in U).  Single right-hand side.
 * accumulate != 0 adds to G_dev instead of overwriting it. */
int ovl_wilson_link_vjp(const ovl_gauge *g, void *G_dev, const void *chi, const void *psi,
                        int spin_dt, int accumulate, void *stream);

/* G_dev = d Re <chi, p(X) psi> / dU with p the polynomial of the handle (no deflation term,
 * lmax held fixed): reverse Clenshaw sweep on chi with the forward Chebyshev vectors of psi
 * recomputed from checkpoints every ckpt_stride steps (0 = ceil(sqrt(N))).  The recomputation
 * and the reverse sweep of a segment are independent, so their steps run two at a time in one
 * launch that reads the links once (the launch configuration of a two-right-hand-side problem on
 * this lattice, see ovl_autotune).  Layout of G_dev as in ovl_wilson_link_vjp; single right-hand
 * side. */
int ovl_sign_force(const ovl_gauge *g, const ovl_poly *p, void *G_dev, const void *chi,
                   const void *psi, int ckpt_stride, int spin_dt, void *stream);

/* ---- stout smearing of the links (Sec. 2) and its chain rule (HMC, Sec. 1) ------------------- */

/* The links entering K are smoothed by 3 steps of over-improved stout smearing with rho = 0.1,
 * eps = -0.25 (Sec. 2).  One step replaces every link at once by U'_mu(x) = exp(M) U_mu(x), with
 * M the traceless anti-Hermitian part of Omega = C_mu(x) U_mu(x)^+ (M = (Omega - Omega^+)/2 -
 * tr(Omega - Omega^+)/6) and C_mu(x) the sum over the paths from x to x + mu that close a loop
 * with the link: the 6 plaquette staples with weight rho (5 - 2 eps)/3 and the 18 staples of the
 * 2 x 1 rectangles with weight -rho (1 - eps)/12 (the over-improved gauge action; eps = 1 gives
 * plain stout smearing, eps = 0 the tree-level Symanzik weights).  exp(M) is evaluated in FP64
 * (Taylor series after scaling to norm 1/2, then squaring).
 *   U_in, U_out  caller-owned device arrays U[mu][a][b][T][Z][Y][X], complex double (the caller
 *                layout of ovl_gauge_create); they must not overlap; U_in is unchanged.
 *   steps        0 .. 64 (0 copies U_in).
 * Allocates two link fields of work space for steps >= 2.  Asynchronous on `stream`.
 * Errors: EINVAL (NULL, steps out of range), EDIMS (bad extents, or a link field of 4 GiB or more:
 * V >= 7456540 sites), ENONFINITE (rho or eps), EALIAS, ENOMEM, EHIP. */
int ovl_stout_smear(const int32_t dims[4], void *U_out, const void *U_in, double rho, double eps,
                    int steps, void *stream);

/* Chain rule through ovl_stout_smear: given G_smeared = dL/dRe U' + i dL/dIm U' of a real
 * function L of the smeared links U' = stout^steps(U_thin) (for example the output of
 * ovl_sign_force on a gauge handle made from U'), writes G_thin = dL/dRe U + i dL/dIm U of the
 * thin links.  The forward levels are recomputed; each step backwards forms dL/dC_mu(x) per link
 * (through the Frechet derivative of exp, FP64 Taylor series) and then gathers, for every link,
 * the contributions of all staples that contain it (no atomics: deterministic).
 *   G_thin, G_smeared, U_thin  caller-owned device arrays in the layout above, complex double,
 *                pairwise non-overlapping; G_smeared and U_thin are unchanged.
 * Allocates up to 2 steps + 2 link fields of work space (the forward levels and their staple sums,
 * dL/dC, the direct part, two derivative fields).  Asynchronous on `stream`.  Errors as
 * ovl_stout_smear. */
int ovl_stout_backward(const int32_t dims[4], void *G_thin, const void *G_smeared,
                       const void *U_thin, double rho, double eps, int steps, void *stream);

/* ---- diagnostics of the approximation -------------------------------------------------------- */

/* The exact sign function squares to one, which gives the overlap operator of Sec. 2 (eq. 1) its
 * exact chiral symmetry (Sec. 1).  With S the polynomial of ovl_sign_apply plus the deflation of
 * d (nullable): r_out[r] = ||S (S psi_r) - psi_r|| / ||psi_r|| for each of the nrhs right-hand
 * sides in `in` ([nrhs][4][3][T][Z][Y][X] of spin_dt, caller-owned device memory, unchanged),
 * 0 where psi_r = 0.  r_out: caller-owned host array of nrhs doubles.  Two sign evaluations in
 * the storage precision of g, then S^2 psi - psi and FP64 inner products on the device.
 * Allocates two vectors of the input's size for the duration of the call; synchronises the
 * stream.  Errors: as ovl_sign_apply (EINVAL also for a NULL r_out), ENONFINITE for a
 * non-finite norm. */
int ovl_sign_residual(const ovl_gauge *g, const ovl_poly *p, const ovl_defl *d, const void *in,
                      int nrhs, int spin_dt, double *r_out, void *stream);

/* ---- low modes of K (the deflation basis) ------------------------------------------------------ */

/* The n_ev eigenpairs of K = gamma5 (D_W - m_W) with the smallest |lambda|, which the deflation
 * term of Sec. 2, eq. 3 removes from the polynomial (the paper precomputes them once per gauge
 * field by a polynomial-preconditioned Lanczos method, Sec. 2).  Method: Chebyshev-filtered
 * subspace iteration on a block of `block` vectors: the filter T_degree((2 K^2 - (cut^2 + lmax^2))
 * / (lmax^2 - cut^2)) is bounded by 1 for cut <= |lambda| <= lmax and grows fastest towards
 * lambda = 0; each iteration orthonormalises the block (scaled SVQB from its FP64 Gram matrix;
 * numerically dependent directions are replaced by fresh random vectors), does a Rayleigh-Ritz
 * step with K itself (so +lambda and -lambda separate), orders the Ritz pairs by ||K v|| and
 * stops when the first n_ev residuals ||K phi - lambda phi|| are below tol or after max_iter
 * iterations.  Every K application runs in the fused stencil kernel with `block` right-hand sides,
 * in the configuration ovl_autotune keeps for that problem (this lattice, FP64, `block`
 * right-hand sides); when there is none yet, the call first measures the candidates on its own
 * start block, as ovl_autotune would (the choice then holds for the rest of the process).
 * Gram products, block rotations and residual norms are FP64 device kernels; the block x block
 * Hermitian eigen-problems are solved on the host (Householder tridiagonalisation + implicit QL).
 * The start block is complex Gaussian from a counter-based generator keyed by `seed`.
 *   g        gauge handle with FP64 link storage;  m_W the Wilson mass of K
 *   block    1 <= n_ev < block <= min(256, 12 V); it must exceed the size of any near-degenerate
 *            cluster of eigenvalues that straddles the n_ev-th one
 *   phi_out  caller-owned device [n_ev][4][3][T][Z][Y][X] complex double (orthonormal);
 *   lambda_out, resid_out  host arrays of n_ev doubles (ascending |lambda| up to the ordering by
 *            ||K phi||); eps_next_out (nullable) = |lambda| of the first Ritz value beyond n_ev
 *            divided by lmax (the lower end of the polynomial's interval); iters_out (nullable).
 * Allocates about 5 * block * 12 V complex doubles of work space for the call; synchronises the
 * stream.  Errors: EINVAL, EDTYPE (links not FP64), EDIMS, ENONFINITE, ENOMEM, EHIP; EDIVERGED
 * when the residuals are above tol after max_iter iterations (the outputs hold the last
 * iterate). */
int ovl_low_modes(const ovl_gauge *g, int n_ev, int block, double lmax, double cut, int degree,
                  int max_iter, double tol, uint64_t seed, double m_W, void *phi_out,
                  double *lambda_out, double *resid_out, double *eps_next_out, int *iters_out,
                  void *stream);

/* The host eigen-solver of ovl_low_modes on its own (no device involved): a (n x n, row-major,
 * interleaved complex double) Hermitian -> w (n ascending eigenvalues) and q (n x n row-major
 * complex, eigenvectors in the columns).  Errors: EINVAL (NULL, n outside [1, 4096], not
 * Hermitian to 1e-12), EDIVERGED (no convergence). */
int ovl_hermitian_eigh(int n, const double *a, double *w, double *q);

/* ---- overlap inversion ---------------------------------------------------------------------- */

/* Solve D[mu] x = b for one FP64 vector (Sec. 2: the overlap operator exists to be inverted; the
 * paper's solver timings are Table 5).  Method: defect correction in FP64 around conjugate
 * gradients on the normal equations D^+ D dx = D^+ r.  The inner CG runs in the precision of
 * (g_in, d_in) -- FP32 spinors with FP32 or BF16 links -- or, when g_in is NULL, in FP64 with
 * (g, d); each outer pass recomputes the true residual r = b - D x with (g, d) in FP64.
 *   g      gauge handle with FP64 link storage; p polynomial; d deflation (nullable, FP64);
 *   x, b   device [4][3][T][Z][Y][X] complex FP64; x is overwritten (starts from 0); x != b;
 *   g_in   nullable gauge handle of the same field in FP32 or BF16 storage; d_in its deflation
 *          (nullable, FP32 storage);
 *   tol    target ||b - D x|| / ||b|| (> 0); max_iter bound on inner CG iterations (each two
 *          overlap applications);
 *   iters_out, resid_out (nullable) receive the inner iterations used and the final relative
 *          residual.
 * The CG coefficients stay on the device (FP64 inner products feed the vector updates
 * directly); the host reads ||r||^2 two iterations behind the stream to decide when to stop, so
 * an inner CG may run up to two iterations past its tolerance.  Synchronises the stream once
 * per outer pass; allocates 2 FP64 and 6 inner-precision vectors of work space.  Errors: EINVAL, EDIMS, EDTYPE,
 * EALIAS, ENONFINITE, ENOMEM, EHIP; EDIVERGED if the residual target is not reached within
 * max_iter (x then holds the last iterate) or CG loses positivity. */
int ovl_overlap_solve(const ovl_gauge *g, const ovl_poly *p, const ovl_defl *d, double mu,
                      void *x, const void *b, const ovl_gauge *g_in, const ovl_defl *d_in,
                      double tol, int max_iter, int *iters_out, double *resid_out, void *stream);

/* Solve D[mu] x = b for one FP64 vector by GMRESR with relaxed nested sign functions, the
 * paper's outer solver form (Sec. 2: a recursive GMRES outer method around a low-accuracy inner
 * inversion whose bulk needs only a low-accuracy sign function; Sec. 3: overlap inversions to a
 * relative accuracy of 1e-13 in mixed precision).  Outer step k: z_k ~ D^-1 r_k from conjugate
 * gradients on the normal equations in the precision of (g_in, d_in) (FP32 spinors with FP32 or
 * BF16 links; FP64 with (g, d) when g_in is NULL), stopped at relative normal-equation residual
 * inner_tol, with the polynomial of p truncated to the lowest degree whose dropped coefficients
 * sum to at most inner_poly_tol (|T_m| <= 1 bounds the truncation error; 0 keeps p); then
 * c_k = D z_k in FP64, orthogonalised against c_0 .. c_{k-1} by classical Gram-Schmidt applied
 * twice (z_k follows with the same coefficients), normalised, and x += <c_k, r> z_k,
 * r -= <c_k, r> c_k.  relax != 0: the FP64 product of step k uses p truncated at tail
 * 0.1 tol ||b|| / ||r_k|| (a coarser polynomial as the residual falls; the inexact products
 * perturb the final residual by about tol/10).  At the end the residual b - D x is recomputed
 * with the full polynomial; if it misses tol, GMRESR restarts from x without relaxation (at most
 * three cycles).  All Krylov coefficients stay on the device; the host reads ||r|| once per outer
 * step and two iterations behind the stream inside the inner CG.
 *   g, p, d, mu, x, b, g_in, d_in  as ovl_overlap_solve (x is overwritten, starts from 0);
 *   tol            target ||b - D x|| / ||b|| with the full polynomial (> 0);
 *   inner_tol      0 < inner_tol < 1;  inner_poly_tol >= 0;
 *   max_outer      1 .. 1024 directions per cycle (two FP64 vectors each are kept);
 *   max_inner      bound on the total inner CG iterations;
 *   outer_out, inner_out, resid_out (nullable): outer steps and inner iterations used, the final
 *                  relative residual with the full polynomial.
 * Allocates 2 + 2 max_outer FP64 and 6 inner-precision vectors of work space; synchronises the
 * stream.  Errors: as ovl_overlap_solve; EDIVERGED when tol is not reached within the bounds or a
 * direction is numerically dependent on the previous ones (x then holds the last iterate). */
int ovl_overlap_solve_gmresr(const ovl_gauge *g, const ovl_poly *p, const ovl_defl *d, double mu,
                             void *x, const void *b, const ovl_gauge *g_in, const ovl_defl *d_in,
                             double tol, double inner_tol, double inner_poly_tol, int relax,
                             int max_outer, int max_inner, int *outer_out, int *inner_out,
                             double *resid_out, void *stream);

/* ---- launch tuning ------------------------------------------------------------------------ */

/* Measure the fused Chebyshev step kernel (Sec. 2: stencil and polynomial algebra in one
 * kernel) on a problem set -- one item: the single-problem launch of ovl_sign_apply and the
 * other operators; several: the batched launch of ovl_batch_sign_apply -- over its launch
 * configurations and keep the fastest for every later launch of the same problem set (the
 * precision and each item's extents and right-hand-side count, in order).  A configuration is
 * (spb, order, remap, rb).  Order 1 = t-streaming tile order, 0 = memory order, with spb = 8
 * (eight threads per site: forward and backward hops on separate threads), 16 or 64 (four threads
 * per site) or 128 (two x-adjacent sites per lane).  Order 2 = LDS slab of whole x lines with
 * spb = 64, 128, 192 or 256 sites (single problems; spb a multiple of Lx dividing Lx Ly).
 * Remap = XCD-contiguous workgroup ranges on or off.  rb = right-hand-side block: 1, 2 or 4
 * right-hand sides per thread reusing one read of the thread's two links (spb 16 or 64, orders
 * 0 and 1).  Each candidate runs 2 untimed and 10 timed steps that read the items' inputs and
 * write their outputs (the outputs' contents are then undefined).  When the fastest has remap off
 * and the same form with remap on is within 3% of it, the remap-on form is kept (less traffic
 * between the XCDs' caches, a stable choice); likewise the tile order over memory order within 2%
 * (fewer t-neighbour re-reads from HBM).  p (nullable) supplies lmax and
 * m_W for the step's coefficients.  The key includes whether every item's handle reads two-row
 * links (ovl_gauge_reconstruct).  The winner is appended to the text file cache_path when not
 * NULL (one line: B prec r12 n_items, then Lx Ly Lz Lt nrhs per item, then spb order remap rb
 * microseconds).  *best_us (nullable) receives the winner's time per step.  Synchronises the
 * stream.  Errors: as ovl_batch_sign_apply, ENOMEM, EHIP. */
int ovl_autotune(const ovl_batch_item *items, int n_items, const ovl_poly *p, int spin_dt,
                 const char *cache_path, double *best_us, void *stream);
/* Load configurations written by ovl_autotune (also the single-problem short form
 * "Lx Ly Lz Lt precision nrhs spb order remap microseconds", rb = 1); returns the number of
 * entries read (>= 0) or OVL_EINVAL when the file cannot be opened. */
int ovl_autotune_load(const char *cache_path);
/* The configuration the library will use for a single problem: cfg_out = {sites per workgroup,
 * order, remap} (see ovl_autotune).  Defaults: 8 sites per workgroup below 4K
 * site-right-hand-sides, 16 below 64K, else 64 in tile order, with 128 (two sites per lane) for
 * FP32 links from 512K site-right-hand-sides; remap on; rb 1.  Two sites per lane need FP32
 * spinors, an even Lx and 16-byte aligned vectors (a call whose vectors are not aligned runs
 * with 64); a slab entry that does not fit the lattice falls back to the default. */
int ovl_launch_config(const ovl_gauge *g, int nrhs, int spin_dt, int cfg_out[3]);
/* The configuration an evaluation of this problem set will use (the batched launch for several
 * items, the single-problem launch for one): cfg_out = {spb, order, remap, rb}, with the items'
 * own vectors deciding whether two sites per lane are possible.  Errors: as
 * ovl_batch_sign_apply. */
int ovl_batch_launch_config(const ovl_batch_item *items, int n_items, int spin_dt,
                            int cfg_out[4]);

/* ---- diagnostics ------------------------------------------------------------------------- */

/* Thread-local message describing the most recent failure in this thread ("" if none). */
const char *ovl_last_error(void);

/* Read (and with clear != 0, reset) the sticky device flags of a gauge handle (OVL_FLAG_*).
 * Synchronises the device. */
int ovl_status_flags(const ovl_gauge *g, uint32_t *flags, int clear);

/* Step graphs (on by default).  A sign or overlap evaluation of one problem small enough for
 * one-wave workgroups (fewer than 64K site-right-hand-sides) and of degree >= 3 is bound by the
 * launch rate.  The second time the same evaluation is requested (same gauge handle and link
 * read mode, polynomial handle, source and output pointers, right-hand-side count, precision,
 * gamma5 on the source and launch configuration) its plain recurrence steps are captured into a
 * HIP graph, which is replayed from then on; the deflation projection, the final fused step and
 * the norm check stay direct launches.  The library keeps up to 8 such graphs, each with its own
 * work vector (one right-hand-side set of spinors); evicting one synchronises the device.  Two
 * calls that overlap in time and share a graph race on its work vector, as they would on their
 * shared output.  on = 0 turns the mechanism off for later calls (cached graphs are kept).
 * Results are bitwise identical either way. */
int ovl_graph_enable(int on);

/* Kernel timing (measurement support).  When enabled, every sign evaluation (sign, overlap,
 * batched sign) records one HIP event on its stream before its first plain recurrence step and
 * one after its last (the steps k = N-1 .. 1 are consecutive launches of the fused Chebyshev
 * step kernel, so the interval divided by N - 1 is the kernel's average duration back to back,
 * inter-launch gaps included; evaluations of degree 1 record nothing), and every link-VJP launch
 * of the force (ovl_sign_force, ovl_wilson_link_vjp) records one event pair around itself.
 * ovl_timing_read(kind, ...) returns, for kind 0 (fused Chebyshev step) or 1 (link VJP), the
 * summed intervals (ms) and the number of launches they cover since that kind was last read
 * (synchronising the recorded events), and resets them.  Errors: EINVAL (NULL, bad kind). */
int ovl_timing_enable(int on);
int ovl_timing_read(int kind, double *total_ms, int64_t *launches);

/* Device-memory bandwidth ceilings (measurement support, not part of the method): one launch of
 * a plain stream over `bytes` bytes of 16-byte elements, on `stream`.  kind 0: read src (bytes),
 * write one 4-byte value per thread to dst (dst must hold 8 MiB); kind 1: copy src to dst
 * (bytes each); kind 2: dst = x XOR y XOR z with x, y, z the three consecutive `bytes`-long
 * arrays at src (3 * bytes read, bytes written).  Buffers: caller-owned device memory, 16-byte
 * aligned, non-overlapping.  Errors: EINVAL (NULL, bytes not a positive multiple of 16,
 * misaligned, bad kind), EHIP. */
int ovl_stream_probe(int kind, void *dst, const void *src, int64_t bytes, void *stream);

/* Library version string. */
const char *ovl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OVL_H */

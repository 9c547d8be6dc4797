/*
 * ovl.h - C ABI of the MI355X overlap-operator library (libovl.so).
 *
 * Hot path of arXiv:1106.4964 ("Efficient implementation of the overlap
 * operator on multi-GPUs"): the Wilson dslash D_w (Sec. II, eq. 1-2) applied
 * inside the Chebyshev/Clenshaw polynomial approximation of sign(H_w),
 * H_w = gamma5 D_w(-rho) (eq. 4-5, Sec. V), with low-mode projection
 * (eq. 6-7), the overlap operator D(m) (eq. 3, 8) and CG for propagators
 * (Sec. II, Sec. V).  The whole periodic lattice lives on one GPU.
 *
 * Conventions
 *  - Every call returns int: OVL_OK (0), a positive warning, or a negative
 *    error.  ovl_last_error() gives a thread-local message for the last
 *    failure.  Nothing throws across this ABI.
 *  - Field buffers are caller-owned device memory; the library never frees
 *    them or keeps them past the call, except the eigenvector buffer lent
 *    to ovl_lowmodes_create (borrowed for the handle's lifetime).
 *  - Handles (geometry, gauge, sign, lowmodes, net) are library-owned and
 *    released with their _destroy call.
 *  - All device work is enqueued on the caller's HIP stream.  Calls that
 *    return host values (reductions, solvers, bounds) synchronise it.
 *  - Lattice: dims = {Lx, Ly, Lz, Lt}, every extent even and >= 2,
 *    periodic in all directions.  Site order: lex = x + Lx*(y + Ly*(z + Lz*t)),
 *    parity p = (x+y+z+t) mod 2, even-odd index eo = p*N/2 + lex/2.
 *    Gamma matrices: chiral basis, gamma5 = diag(1,1,-1,-1),
 *    gamma_k = [[0,-i sigma_k],[i sigma_k,0]], gamma_4 = [[0,1],[1,0]].
 *
 * Device field layouts (part of the ABI)
 *  A spinor is 12 complex numbers per site, complex index c = 3*spin + colour.
 *  It is stored as 16-byte blocks, structure-of-arrays over the N/2 sites of
 *  each parity:  [parity][block][N/2][16 bytes], where a block holds
 *    OVL_F64  : 1 complex  (double re, im)        -> 12 blocks
 *    OVL_F32  : 2 complex  (c = 2j, 2j+1)          ->  6 blocks
 *    OVL_F16/OVL_BF16 : 4 complex (c = 4j..4j+3)   ->  3 blocks
 *  A batch of nrhs spinors is nrhs such vectors back to back.
 *  The canonical host/device AoS layout used by pack/unpack is complex128
 *  [nrhs][N (lex order)][4 spin][3 colour].  Gauge fields enter as complex128
 *  [N (lex)][4 mu][3][3] with U_mu(x) on the link x -> x + mu.
 */
#ifndef OVL_H
#define OVL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* ovl_stream_t; /* a hipStream_t (0 = null stream) */

enum {
  OVL_OK = 0,
  OVL_W_NOT_CONVERGED = 1, /* solver stopped at maxiter; stats are valid   */
  OVL_E_ARG = -1,          /* null pointer, bad size or out-of-range value */
  OVL_E_DIMS = -2,         /* lattice extent odd or < 2                    */
  OVL_E_PRECISION = -3,    /* precision/representation not available       */
  OVL_E_ALIAS = -4,        /* output aliases an input that it may not      */
  OVL_E_HIP = -5,          /* HIP runtime error (message has details)      */
  OVL_E_NOT_SU3 = -6,      /* 12-real compression asked for non-SU(3) link */
  OVL_E_BREAKDOWN = -7,    /* Krylov breakdown (p^dag A p <= 0)            */
  OVL_E_NAN = -8,          /* NaN or Inf in an input or an iterate         */
  OVL_E_NOMEM = -9,        /* device allocation failed                     */
  OVL_E_STATE = -10        /* handle used in an invalid state              */
};

typedef enum { OVL_F64 = 0, OVL_F32 = 1, OVL_F16 = 2, OVL_BF16 = 3 } ovl_prec;

#define OVL_MAX_RHS 12

typedef struct ovl_geom ovl_geom;
typedef struct ovl_gauge ovl_gauge;
typedef struct ovl_sign ovl_sign;
typedef struct ovl_lowmodes ovl_lowmodes;
typedef struct ovl_net ovl_net;
typedef struct ovl_deflation ovl_deflation;

const char* ovl_last_error(void);
int ovl_version(void);

/* ---------------------------------------------------------------- geometry
 * Site ordering and neighbours of the periodic lattice (Sec. II, Fig. 1).
 * ovl_geom_create: OVL_E_DIMS if an extent is odd or < 2, or N >= 2^31.
 * ovl_geom_neighbors_device: fills dev_table, int32 [8][N] in eo order,
 *   table[d][eo(s)] = eo(neighbour of s), d = 0..3 for +x,+y,+z,+t and
 *   d = 4..7 for -x..-t, computed on the GPU by the same index arithmetic
 *   the stencil kernels use.  Caller-owned device buffer of 32*N bytes.
 */
int ovl_geom_create(const int32_t dims[4], ovl_geom** out);
int ovl_geom_destroy(ovl_geom* g);
int ovl_geom_volume(const ovl_geom* g, int64_t* n_sites);
int ovl_geom_eo_index(const ovl_geom* g, const int32_t xyzt[4], int32_t* eo);
int ovl_geom_neighbors_device(const ovl_geom* g, int32_t* dev_table, ovl_stream_t s);

/* ----------------------------------------------------------------- spinors
 * ovl_spinor_bytes: bytes of a batch of nrhs spinors at precision prec.
 * ovl_pack_spinor / ovl_unpack_spinor: device-to-device conversion between
 *   the canonical AoS complex128 layout and the library layout.  Down-
 *   conversion rounds to nearest even; FP64 -> FP16/BF16 goes through FP32
 *   (two such roundings).  src and dst must not overlap.
 */
int ovl_spinor_bytes(const ovl_geom* g, ovl_prec prec, int nrhs, size_t* bytes);
int ovl_pack_spinor(const ovl_geom* g, const double* dev_aos, void* dev_out, ovl_prec prec,
                    int nrhs, ovl_stream_t s);
int ovl_unpack_spinor(const ovl_geom* g, const void* dev_in, double* dev_aos, ovl_prec prec,
                      int nrhs, ovl_stream_t s);

/* ------------------------------------------------------------------- gauge
 * ovl_gauge_create: copies and packs the links U_mu(x) (Sec. II, Fig. 1)
 *   from a device AoS complex128 [N][4][3][3] buffer into the FP64 18-real
 *   representation, which every FP64 operator uses.  The source buffer may
 *   be freed after the call returns.
 * ovl_gauge_set_repr: (re)builds the representation that operators at
 *   spinor precision prec (F32, F16 or BF16) use: links stored at that
 *   precision with 18 reals, or 12 reals (rows 0 and 1; row 2 rebuilt as
 *   conj(row0 x row1), valid for SU(3)).  compress12 = 1 checks that
 *   every link is unitary with det 1 to 1e-12 (FP64) and returns
 *   OVL_E_NOT_SU3 otherwise.  Also accepts prec = F64 with compress12 = 1
 *   to switch FP64 operators to 12-real links.
 */
int ovl_gauge_create(const ovl_geom* g, const double* dev_aos, ovl_stream_t s, ovl_gauge** out);
int ovl_gauge_set_repr(ovl_gauge* u, ovl_prec prec, int compress12, ovl_stream_t s);
int ovl_gauge_destroy(ovl_gauge* u);
const ovl_geom* ovl_gauge_geom(const ovl_gauge* u);

/* --------------------------------------------------------------- operators
 * ovl_dslash: out = D_w(m) in (eq. 1-2) for a batch of nrhs spinors:
 *   out(x) = (4+m) in(x) - 1/2 sum_mu [ U_mu(x)(1-gamma_mu) in(x+mu)
 *                                     + U_mu(x-mu)^dag (1+gamma_mu) in(x-mu) ].
 *   parity = 0 or 1 writes only the even or odd sites of out (the other
 *   half of out is left untouched); parity = 2 writes both.  in and out
 *   use precision prec; FP64 computes in double, the others in float.
 *   out == in gives OVL_E_ALIAS.
 * ovl_hw_apply: out = H_w in = gamma5 D_w(-rho) in (Sec. II).
 */
int ovl_dslash(void* out, const void* in, const ovl_gauge* u, double m, int parity, ovl_prec prec,
               int nrhs, ovl_stream_t s);
int ovl_hw_apply(void* out, const void* in, const ovl_gauge* u, double rho, ovl_prec prec, int nrhs,
                 ovl_stream_t s);

/* -------------------------------------------------------------------- BLAS1
 * Vector operations of Sec. III on batches of nrhs spinors of precision
 * prec (a is one complex number per right-hand side, host array of 2*nrhs
 * doubles re,im).  Reductions accumulate in FP64 in a fixed order
 * (deterministic) and write 2*nrhs (dot) or nrhs (norm2) doubles to the
 * host array result; they synchronise the stream.
 *   ovl_axpy : y <- a x + y          ovl_xpay : y <- x + a y
 *   ovl_dot  : result_r = x_r^dag y_r     ovl_norm2: result_r = ||x_r||^2
 *   ovl_convert: dst <- src with precision change (RNE on down-conversion)
 */
int ovl_axpy(const ovl_geom* g, const double* a, const void* x, void* y, ovl_prec prec, int nrhs,
             ovl_stream_t s);
int ovl_xpay(const ovl_geom* g, const void* x, const double* a, void* y, ovl_prec prec, int nrhs,
             ovl_stream_t s);
int ovl_dot(const ovl_geom* g, const void* x, const void* y, ovl_prec prec, int nrhs, double* result,
            ovl_stream_t s);
int ovl_norm2(const ovl_geom* g, const void* x, ovl_prec prec, int nrhs, double* result,
              ovl_stream_t s);
int ovl_convert(const ovl_geom* g, const void* src, ovl_prec src_prec, void* dst, ovl_prec dst_prec,
                int nrhs, ovl_stream_t s);

/* ------------------------------------------------------------ sign function
 * Polynomial approximation of sign(H_w) (eq. 4-5, Sec. V): Q = H_w/lam_max,
 * P(x) ~ x^{-1/2} on [eps, 1] with eps = (lam_lo/lam_max)^2, expanded in
 * Chebyshev polynomials T_k(y), y = (2x - 1 - eps)/(1 - eps), and evaluated
 * on vectors by the Clenshaw recursion (2n+1 applications of D_w).
 * P is the optimal polynomial of order n (eq. 4: it minimises
 * delta = max |1 - sqrt(x) P(x)| over [eps, 1]; Fig. 2 prints delta = 0.1
 * at n = 13, sqrt(eps) ~ 0.06), computed on the host by a Remez exchange on
 * the relative error and held as Chebyshev coefficients c_0..c_n in
 * y = (2x - 1 - eps)/(1 - eps).  Where the Chebyshev interpolant of
 * x^{-1/2} at the n+1 Chebyshev-Gauss nodes already has delta <= 1e-12
 * (FP64 rounding), or n > 400, that interpolant is used instead.
 * ovl_sign_create: lam_max must bound |spectrum(H_w)| from above and lam_lo
 *   bound |lambda| from below on the subspace the polynomial acts on (with
 *   low modes: |lambda_l|).  n > 0 fixes the order; n = 0 picks the
 *   smallest n whose measured delta = max |1 - sqrt(x) P(x)| (400000 points
 *   of [eps,1]) is <= delta.  Takes ~0.2-0.7 s for a fixed n and 0.5-15 s
 *   for an order search (longest just below order 400, where the optimal
 *   polynomial is searched one order at a time).  OVL_E_ARG unless
 *   0 < lam_lo < lam_max.
 * ovl_sign_info: order n, eps and the measured delta.
 * ovl_sign_coeffs: copies c_0..c_n (n+1 doubles; cap = buffer length).
 */
int ovl_sign_create(double lam_lo, double lam_max, double delta, int n, ovl_sign** out);
int ovl_sign_destroy(ovl_sign* s);
int ovl_sign_info(const ovl_sign* s, int* n, double* eps, double* delta_measured);
int ovl_sign_coeffs(const ovl_sign* s, double* c, int cap);

/* ---------------------------------------------------------------- low modes
 * The l eigenpairs (lambda_i, eta_i) of H_w closest to zero (eq. 6-7).
 * ovl_lowmodes_create: V is a caller-owned device buffer of ell FP64 spinors
 *   (library layout, back to back), orthonormal; lambda is a host array of
 *   ell eigenvalues of H_w (copied).  The handle BORROWS V: it must stay
 *   valid and unchanged for the handle's lifetime.
 * ovl_lowmodes_project: psi_h = in - sum_i (eta_i^dag in) eta_i and
 *   w = sum_i sign(lambda_i) (eta_i^dag in) eta_i for a batch of nrhs <= 12
 *   spinors at precision prec; the inner products accumulate in FP64.
 */
int ovl_lowmodes_create(const ovl_geom* g, int ell, const void* V, const double* lambda, ovl_lowmodes** out);
int ovl_lowmodes_destroy(ovl_lowmodes* lm);
int ovl_lowmodes_project(const ovl_lowmodes* lm, const void* in, void* psi_h, void* w, ovl_prec prec, int nrhs,
                         ovl_stream_t s);
/* ovl_lowmodes_project_noalloc: ovl_lowmodes_project for callers that cannot
 *   allocate device memory (code under HIP graph capture, tight serving
 *   loops, harnesses that forbid hipMalloc).  Same arguments, layouts,
 *   results and errors, and no hipMalloc, hipFree or other allocating call:
 *   the projection's scratch (ell*nrhs FP64 coefficients and the split-K
 *   partial sums of the inner products) lives in a 16 MiB static array that
 *   each GPU the library runs on holds until the process ends.  Limit:
 *   ell * nrhs <= 16131, OVL_E_ARG beyond.  For ell * nrhs <= 2044 the
 *   partial sums are formed exactly as in ovl_lowmodes_project and the
 *   result is bit-identical; above that fewer partial sums are used and the
 *   result agrees to rounding.  Every call on one GPU uses the same array
 *   and leaves its contents behind: calls that overlap on one GPU (from two
 *   host threads or on two streams that are not ordered) race, so order
 *   them on one stream.
 */
int ovl_lowmodes_project_noalloc(const ovl_lowmodes* lm, const void* in, void* psi_h, void* w, ovl_prec prec,
                                 int nrhs, ovl_stream_t s);

/* ----------------------------------------------------------------- overlap
 * ovl_sign_apply: out = sign(H_w) in ~ sum_i sign(lambda_i)(eta_i^dag in) eta_i
 *   + Q P(Q^2) in_h (eq. 7); lowmodes may be NULL (no projection).
 * ovl_overlap_apply: out = D(m) in with D(m) = rho D + m (1 - D/2) and
 *   D = 1 + gamma5 sign(H_w) (eq. 3, 8), i.e.
 *   D(m) in = (rho + m/2) in + (rho - m/2) gamma5 sign(H_w) in;
 *   dagger = 1 gives D(m)^dag in = (rho + m/2) in + (rho - m/2) sign(H_w) gamma5 in.
 *   H_w = gamma5 D_w(-rho).  Batches of nrhs <= 12 with low modes.
 *   Precision prec applies to in, out, the links and the Clenshaw iterates.
 *   out must not alias in or the eigenvectors (OVL_E_ALIAS).
 */
int ovl_sign_apply(void* out, const void* in, const ovl_gauge* u, double rho, const ovl_sign* sign,
                   const ovl_lowmodes* lowmodes, ovl_prec prec, int nrhs, ovl_stream_t s);
int ovl_overlap_apply(void* out, const void* in, const ovl_gauge* u, double rho, double m, const ovl_sign* sign,
                      const ovl_lowmodes* lowmodes, int dagger, ovl_prec prec, int nrhs, ovl_stream_t s);

/* ----------------------------------------------- rational sign (comparison)
 * The rational alternative to the polynomial (eq. 4-5, Sec. V eq. 12):
 *   sign(H_w) psi ~ sum_i sign(lambda_i)(eta_i^dag psi) eta_i + Q P(Q^2) psi_h,
 *   P(y) = sum_{l=1}^{n} b_l / (y + c_l),
 * P the optimal (Zolotarev, closed form) approximation of y^{-1/2} of type
 * (n-1, n) on [eps, 1], eps = (lam_lo / lam_max)^2.
 * ovl_rational_create: 1 <= n <= 32; the handle holds b, c and the measured
 *   delta = max |1 - sqrt(y) P(y)| (eq. 4).  Host only.
 * ovl_rational_coeffs: copies b[0..n), c[0..n) (cap = buffer length) and,
 *   if non-NULL, eps and delta; returns n (or an error code < 0).
 * ovl_rational_sign_apply: out = sign(H_w) in for one FP64 spinor with the
 *   low modes (optional) projected exactly and P(Q^2) psi_h evaluated by
 *   method 0: multi-shift CG (single pass; every (Q^2 + c_l) x_l = psi_h
 *             to ||residual_l|| <= tol ||psi_h||; 2n + 3 vectors), or
 *   method 1: double pass (Lanczos on Q^2 until the estimated truncation
 *             error of y = P(T_k) e_1 - beta_k |y_k| / (1 - |y_k/y_{k-1}|)
 *             - is <= tol |y_1|, then the Lanczos vectors regenerated and
 *             summed; 7 vectors).
 *   maxiter bounds the Krylov steps (OVL_W_NOT_CONVERGED past it).
 *   stats: Krylov steps, H_w applications, seconds.  Synchronises s.
 */
typedef struct ovl_rational ovl_rational;
typedef struct {
  int iterations;     /* multi-shift CG steps, or Lanczos steps per pass */
  int64_t hw_applies; /* vector applications of H_w                     */
  double seconds;
} ovl_rational_stats;
int ovl_rational_create(double lam_lo, double lam_max, int n, ovl_rational** out);
int ovl_rational_destroy(ovl_rational* r);
int ovl_rational_coeffs(const ovl_rational* r, double* b, double* c, int cap, double* eps, double* delta);
int ovl_rational_sign_apply(void* out, const void* in, const ovl_gauge* u, double rho, const ovl_rational* r,
                            const ovl_lowmodes* lowmodes, int method, double tol, int maxiter,
                            ovl_rational_stats* stats, ovl_stream_t s);

/* ------------------------------------------------------------------ solvers
 * ovl_cg_solve: solves D(m) x = b for nrhs <= 12 FP64 right-hand sides
 *   (library layout, batch) by CG on D(m) D(m)^dag with x = D(m)^dag y, so
 *   the iterated residual is b - D(m) x.  x holds the starting guess on
 *   entry (zero it for a fresh solve; a saved x resumes a solve) and the
 *   solution on exit.  An FP64 outer loop recomputes r = b - D(m) x with the
 *   FP64 operator and restarts the inner solve on r until every rhs has
 *   ||r|| <= tol ||b|| (defect correction).  The inner solve runs at
 *   opts->inner_prec (FP64 = plain FP64 CG; F32/F16/BF16 need the matching
 *   link representation) and accumulates its correction in FP64.  Krylov
 *   scalars stay on the device; with opts->graph_chunk > 0 that many inner
 *   iterations are captured once in a HIP graph and replayed.  A rhs that
 *   converges is frozen (its scalars become zero) while the others go on.
 *   Returns OVL_OK, OVL_W_NOT_CONVERGED (maxiter inner iterations or
 *   max_restarts cycles reached; stats valid), OVL_E_BREAKDOWN or OVL_E_NAN.
 *   The inner operator may use a relaxed sign approximation
 *   (opts->inner_sign): the inner solve only has to reduce the residual by
 *   inner_tol, so its sign function need not be more accurate than that
 *   (adaptive precision, Sec. V); the defect correction still converges to
 *   the FP64 operator built from `sign`.
 *   opts->chiral = 1 runs each inner solve in one chirality sector
 *   (Sec. II, eq. 3 and 8, with the chiral gamma basis of Sec. V): for
 *   gamma5 v = s v, D(m) D(m)^dag v = (2 rho^2 + m^2/2) v
 *   + 2 s (rho^2 - m^2/4) P_s sign(H_w) v with P_s = (1 + s gamma5)/2 when
 *   sign^2 = 1, so CG on that sector costs one sign application per
 *   iteration instead of two.  Each cycle picks, per rhs, the sector
 *   holding the larger part of the residual (the only one for a point
 *   source) and drops the other; the correction is x += D(m)^dag y, applied
 *   in FP64 with the inner sign.  The FP64 true residual with the full
 *   operator still decides convergence.  The sector operator equals
 *   D D^dag only to within 2 rho^2 times the error of the sign function
 *   (approximation and storage rounding), against a smallest eigenvalue
 *   m^2, so a cycle gains at most about m^2 / (2 rho^2 err): it pays in FP64
 *   with an accurate sign, not with FP16 storage at small m.  A cycle that
 *   breaks down or does not halve the true residual switches the rest of
 *   the solve to D D^dag.  Not with harvesting.
 *   opts->deflation (eq. 9): at every FP64 correction cycle the true
 *   residual r is split along the deflation's eigenvectors xi_i of D: x gets
 *   sum_i xi_i (xi_i^dag r) / (rho d_i + m (1 - d_i/2)) at once and the inner
 *   CG solves only for r minus its components along the xi_i, at the reduced
 *   condition number ||D|| / |d_l'|; the cycles repeat until the FP64 true
 *   residual meets tol.  Approximate eigenpairs cost extra cycles as long as
 *   their error, amplified by 1/|rho d_i + m (1 - d_i/2)|, stays below one;
 *   when a deflated cycle ends with a larger true residual than it started
 *   with, x goes back to its value before that cycle, the rest of the solve
 *   runs without deflation and stats->deflation_dropped is set.
 *   opts->relax_signs (adaptive precision, Sec. V): the accuracy of the
 *   inner operator's sign is chosen per defect-correction cycle.  The first
 *   cycle uses inner_sign; each cycle's residual reduction f, run with sign
 *   error delta, gives the error constant K = f / delta of a correction
 *   (from above when inner_tol limited the cycle).  A later cycle takes the
 *   coarsest of inner_sign and relax_signs with K delta within the reduction
 *   that remains to reach tol, so cycles that must gain the full inner_tol
 *   keep inner_sign and the last ones, which need less, run cheaper.  A
 *   cycle that gains less than a factor 2 sends the next one back to
 *   inner_sign.  The FP64 true residual always uses `sign`.
 *   opts may be NULL (plain FP64, no graph).  Work is done on a private
 *   stream ordered after, and before, the caller's stream s.
 * ovl_propagator: out = (1 - D/2) x (Sec. II), the propagator from a
 *   solution x of D(m) x = b.
 */
typedef struct {
  ovl_prec inner_prec; /* precision of the inner solve                    */
  double inner_tol;    /* low-precision inner solve: relative reduction   */
  int graph_chunk;     /* > 0: inner CG iterations per captured HIP graph  */
  int check_every;     /* without graphs: iterations between host checks  */
  int max_restarts;    /* FP64 defect-correction cycles                   */
  void* harvest_x;     /* CG only: FP32 buffers that receive exact pairs  */
  void* harvest_b;     /*   (x, b = D(m) x) from the CG matvecs; NULL=off */
  int harvest_cap;     /*   capacity of each buffer, in spinors           */
  const ovl_sign* inner_sign; /* sign approximation of the inner operator
                                 (same lam_max; typically a larger delta, so
                                 a lower order); NULL = the outer one.  The
                                 FP64 true residual always uses `sign`.   */
  int chiral;          /* CG only: 1 = inner solves in one chiral sector   */
  const ovl_deflation* deflation; /* CG only: eigenpairs of D deflated in
                                     every defect-correction cycle (eq. 9);
                                     NULL = none.  Not with chiral.       */
  int harvest_stride;  /* harvest the pairs of every stride-th inner
                          iteration (<= 1: every one), so a capped harvest
                          spans the whole solve                           */
  const ovl_sign* const* relax_signs; /* CG only (adaptive precision, Sec.
                          V): n_relax coarser inner signs, delta increasing,
                          same lam_max; NULL = off.  Not with chiral.     */
  int n_relax;
} ovl_solve_opts;

typedef struct {
  int iterations;                       /* inner CG iterations, all cycles   */
  int restarts;                         /* inner solves started              */
  double true_residual[OVL_MAX_RHS];    /* ||b - D(m)x|| / ||b|| in FP64     */
  double seconds;                       /* wall time of the call             */
  int64_t sign_applies;                 /* vector applications of sign(H_w)  */
  int64_t dslash_applies;               /* vector applications of D_w        */
  int fallback_used;                    /* FGCR only: CG finished the solve  */
  int harvested;                        /* pairs written to the harvest bufs */
  int deflation_dropped;                /* CG only: a deflated cycle raised
                                           the residual; deflation was off
                                           for the rest of the solve        */
} ovl_solve_stats;

int ovl_cg_solve(void* x, const void* b, int nrhs, const ovl_gauge* u, double rho, double m, const ovl_sign* sign,
                 const ovl_lowmodes* lowmodes, double tol, int maxiter, const ovl_solve_opts* opts,
                 ovl_solve_stats* stats, ovl_stream_t s);
/* ovl_fgcr_solve: solves D(m) x = b (nrhs <= 12) by flexible GCR with the
 *   learned network M as right preconditioner (z = M r, w = D(m) z, w
 *   orthogonalised against the earlier w's of the cycle, restart length
 *   `restart` <= 32), inside the same FP64 defect-correction loop as
 *   ovl_cg_solve; D(m) inside the cycle runs at opts->inner_prec, M in FP32
 *   (needs the FP32 link representation).  M = NULL gives plain GCR.  If a
 *   cycle reduces the residual by less than a factor 0.9, or an iterate is
 *   not finite, the solve is finished by ovl_cg_solve from the current x and
 *   stats->fallback_used is set.  The rhs run in lockstep (one batched M,
 *   D(m), orthogonalisation and update per iteration, scalars on the
 *   device); a converged rhs is frozen while the others go on.  Bases:
 *   2*restart*nrhs FP64 spinors.
 */
int ovl_fgcr_solve(void* x, const void* b, int nrhs, const ovl_gauge* u, double rho, double m, const ovl_sign* sign,
                   const ovl_lowmodes* lowmodes, const ovl_net* M, int restart, double tol, int maxiter,
                   const ovl_solve_opts* opts, ovl_solve_stats* stats, ovl_stream_t s);
/* ovl_cg_multimass: solves D(m_j) x_j = b for nmass <= 8 masses at once
 *   (eq. 3 and 8): with sign^2 = 1, D(m) D(m)^dag = c(m) (K + sigma(m)) with
 *   K = gamma5 sign + sign gamma5, c = rho^2 - m^2/4 and
 *   sigma = (2 rho^2 + m^2/2) / c, so all masses share one Krylov space.  A
 *   shifted CG on K + sigma (two sign applications per iteration, at
 *   opts->inner_prec and to opts->inner_tol, FP64 vectors) gives every y_j;
 *   x_j = D(m_j)^dag y_j / c_j; then each x_j is finished by the FP64
 *   defect-correction loop of ovl_cg_solve (same opts).  x: nmass separate
 *   caller buffers of nrhs FP64 vectors (overwritten); stats: nmass entries,
 *   entry j for mass j's correction solve, the shared shifted stage added to
 *   the entry of the lightest mass.  Errors as ovl_cg_solve; OVL_E_ARG for
 *   chiral mode or harvesting.
 */
int ovl_cg_multimass(void* const* x, const void* b, int nrhs, const ovl_gauge* u, double rho, const double* masses,
                     int nmass, const ovl_sign* sign, const ovl_lowmodes* lowmodes, double tol, int maxiter,
                     const ovl_solve_opts* opts, ovl_solve_stats* stats, ovl_stream_t s);
int ovl_propagator(void* out, const void* x, const ovl_gauge* u, double rho, const ovl_sign* sign,
                   const ovl_lowmodes* lowmodes, ovl_prec prec, int nrhs, ovl_stream_t s);

/* ------------------------------------------------------- spectral set-up
 * ovl_hw_bound: FP64 Lanczos on H_w = gamma5 D_w(-rho) from the start vector
 *   v0 (device FP64 spinor, caller-drawn), full re-orthogonalisation, `steps`
 *   steps.  lam_max = max over the two extreme Ritz pairs of
 *   |theta| + ||H_w y - theta y||: the normalisation ||H_w|| of Q = H_w/||H_w||
 *   (eq. 5).  theta_min/theta_max (may be NULL): the extreme Ritz values.
 * ovl_hw_eigs: the ell eigenpairs of H_w with smallest |lambda|, for the
 *   projection of eq. 6-7.  Thick-restart Lanczos (FP64, full
 *   re-orthogonalisation) on the Chebyshev polynomial T_degree of H_w^2
 *   that damps |lambda| in [0.15 lam_max, lam_max] (Sec. V's acceleration),
 *   then Rayleigh-Ritz with H_w on the top Ritz vectors.  V: caller-owned
 *   device buffer of m >= ell + max(8, ell/10) FP64 spinors; on entry V[:,0]
 *   is the start vector (e.g. Gaussian), on exit the first ell vectors are
 *   orthonormal eigenvectors ordered by (|lambda|, lambda) and lambda[0..ell)
 *   their eigenvalues.  Stops when every wanted pair has
 *   ||H_w v - lambda v|| <= tol * lam_max, or after max_iter restart cycles
 *   (OVL_W_NOT_CONVERGED).  lam_max must bound |spectrum(H_w)|.  Device
 *   workspace: K + 5 FP64 spinors, K = max(2 want, want + 40) <= 512
 *   (want = ell + max(8, ell/10)), lowered in steps of 8 toward want + 40
 *   while the workspace would exceed 90% of the free device memory;
 *   OVL_E_ARG when want + 40 > 512 (ell > 429).
 */
typedef struct {
  int iterations;      /* restart cycles                              */
  int64_t hw_applies;  /* vector applications of H_w                  */
  double max_residual; /* max over wanted pairs of ||H_w v - lambda v|| */
  double seconds;
} ovl_eig_stats;

int ovl_hw_bound(const ovl_gauge* u, double rho, const void* v0, int steps, double* lam_max, double* theta_min,
                 double* theta_max, ovl_stream_t s);
int ovl_hw_eigs(const ovl_gauge* u, double rho, int ell, int m, void* V, double* lambda, double lam_max, double tol,
                int max_iter, int degree, ovl_eig_stats* stats, ovl_stream_t s);
/* ovl_host_heev: eigen-decomposition of a Hermitian n x n matrix on the host
 * (column-major complex128 A, read only); w: n ascending eigenvalues, V:
 * n x n column-major complex128 eigenvectors.  The dense kernel the
 * eigensolver uses for its Gram and Rayleigh-Ritz matrices.
 */
int ovl_host_heev(int n, const double* A, double* w, double* V);

/* ovl_overlap_eigs: eigenpairs of the massless overlap operator
 *   D = 1 + gamma5 sign(H_w) (eq. 3) closest to zero, computed in one chiral
 *   sector as the paper does (Sec. V): thick-restart Lanczos (FP64, full
 *   re-orthogonalisation, basis of K <= 512 chiral half-vectors, 6 complex
 *   per site) on the Hermitian
 *   K_s = s P_s sign(H_w) P_s, P_s = (1 + s gamma5)/2, s = sector (+1 or -1),
 *   each matvec one sign application with `sign` and `lowmodes` at storage
 *   precision prec (OVL_F64 as the paper does; a lower precision converts
 *   the vector in and the result back, so the basis and the Rayleigh-Ritz
 *   step stay FP64 while the eigenvectors are only as good as the sign
 *   applications: ~1e-6 in FP32, enough for the deflation below; the gauge
 *   must hold that precision's links).  The ell
 *   lowest eigenvectors v (eigenvalue k) of K_s give, with
 *   w = P_{-s} sign(H_w) v, sn = ||w|| and u = w/sn, the eigenpairs
 *   xi = (v +- i u)/sqrt(2), d = 1 + k +- i s sn of D (a real mode, sn = 0,
 *   gives xi = v, d = 1 + k): up to 2*ell pairs, ordered by |d| and, within a
 *   pair, negative imaginary part first; *nout receives their number.
 *   V: caller-owned device buffer of at least 2*ell FP64 spinors; V[:, 0]
 *   holds the start vector on entry (its sector-s part is used), V[:, 0..
 *   *nout) the orthonormal eigenvectors on exit (with a lower-precision
 *   sign, orthonormal to the level of its error divided by sn).  d: host array of 4*ell
 *   doubles, (re, im) per pair.  Stops when the Ritz residuals of the ell
 *   sector vectors are <= tol or after max_iter restart cycles
 *   (OVL_W_NOT_CONVERGED); stats->max_residual is the recomputed
 *   ||K_s v - k v||, stats->hw_applies counts D_w applications.  Device
 *   workspace: (K + 2)/2 + 3 FP64 spinors.
 *   A pair whose partner norm sn is below 1e-9 (1e-5 below FP64) is taken
 *   for a real mode.
 * ovl_deflation_create: n eigenpairs (xi_i, d_i) of D for the deflated CG
 *   (ovl_solve_opts.deflation, eq. 9).  Xi: n orthonormal FP64 spinors,
 *   caller-owned device memory BORROWED for the handle's lifetime; d: host
 *   array of 2n doubles (copied).  OVL_E_NAN for a non-finite eigenvalue.
 */
int ovl_overlap_eigs(const ovl_gauge* u, double rho, const ovl_sign* sign, const ovl_lowmodes* lowmodes, ovl_prec prec,
                     int sector, int ell, int K, void* V, double* d, int* nout, double tol, int max_iter,
                     ovl_eig_stats* stats, ovl_stream_t s);
/* ovl_deflation_prepare: switches the deflation to its minimal-residual
 *   form for approximate eigenpairs: Z = D(0) Xi (n FP64 spinors written to
 *   the caller-owned device buffer Z, which the handle then BORROWS; D(0)
 *   with rho, sign and lowmodes, which must be those of the solves that use
 *   the handle) and the n x n Gram matrices of Z and Xi.  A cycle then adds
 *   x += Xi y with y minimising ||r - D(m) Xi y|| (D(m) Xi = (1 - m/(2 rho)) Z
 *   + m Xi, the small normal equations solved on the host), and hands the
 *   inner solve r - D(m) Xi y, the exact new residual.  For exact
 *   eigenpairs it is eq. 9; for approximate ones the correction can only
 *   lower the residual.  Costs n FP64 sign applications (in batches of 12)
 *   once.  OVL_E_ARG for a different lattice, rho <= 0; OVL_E_ALIAS for
 *   Z == Xi; OVL_E_NAN for a non-finite Gram entry.
 */
int ovl_deflation_create(const ovl_geom* g, int n, const void* Xi, const double* d, ovl_deflation** out);
int ovl_deflation_destroy(ovl_deflation* df);
int ovl_deflation_prepare(ovl_deflation* df, const ovl_gauge* u, double rho, const ovl_sign* sign,
                          const ovl_lowmodes* lowmodes, void* Z, ovl_stream_t s);

/* --------------------------------------------------- learned preconditioner
 * A 2-layer gauge-equivariant parallel-transport convolution network
 * 1 -> hidden -> 1 channels (not part of the paper): each layer is
 *   out[a](x) = sum_b sum_k W[k][a][b] (T_k in[b])(x), k = 0..8,
 * T_0 = 1, T_{+mu} phi(x) = U_mu(x) phi(x+mu), T_{-mu} phi(x) =
 * U_mu(x-mu)^dag phi(x-mu) (the transporters of eq. 2 without spin
 * projector), W[k][a][b] a complex 4x4 spin matrix.  Weights: complex128
 * host arrays, layout [k][a][b][4][4] (layer 1: 9 x hidden x 1, layer 2:
 * 9 x 1 x hidden).  Activations: FP32 spinors; links: the FP32
 * representation of the gauge field.
 * ovl_ptc_layer_forward: one layer, cin/cout channels (vectors back to back).
 * ovl_ptc_layer_backward: gin = layer^dag gout (if gin != NULL) and the
 *   weight gradient gW[k][a][b] = sum_x sum_colour gout[a](x) (T_k in[b](x))^dag
 *   (host complex128, if gW != NULL), for real losses with the convention
 *   grad z = dL/dRe z + i dL/dIm z.  cin*cout <= 4.
 * ovl_net_train: `epochs` passes of mini-batch Adam (betas 0.9, 0.999) on
 *   the loss mean_i ||M b_i - x_i||^2 / ||x_i||^2 over npairs FP32 pairs
 *   (B, X: device batches); order: epochs*npairs caller-drawn indices into
 *   the pairs; loss_history[epoch] (may be NULL) receives the mean loss.
 * ovl_net_apply: out = M in for one FP32 spinor.
 */
int ovl_net_create(const ovl_geom* g, int hidden, ovl_net** out);
int ovl_net_destroy(ovl_net* n);
int ovl_net_set_weights(ovl_net* n, const double* w1, const double* w2);
int ovl_net_get_weights(const ovl_net* n, double* w1, double* w2);
int ovl_ptc_layer_forward(const ovl_gauge* u, const void* in, int cin, void* out, int cout, const double* W,
                          ovl_stream_t s);
int ovl_ptc_layer_backward(const ovl_gauge* u, const void* in, int cin, const void* gout, int cout, const double* W,
                           void* gin, double* gW, ovl_stream_t s);
int ovl_net_train(ovl_net* n, const ovl_gauge* u, const void* B, const void* X, int npairs, int epochs, int batch,
                  double lr, const int32_t* order, double* loss_history, ovl_stream_t s);
int ovl_net_apply(const ovl_net* n, const ovl_gauge* u, const void* in, void* out, ovl_stream_t s);

/* ovl_stencil_tune: mode 1 (default; OVL_TUNE=0 in the environment starts
 *   with 0) tunes each stencil configuration (precision, link format, extra
 *   epilogue vectors, batch size, parity mode, volume) at its first launch:
 *   every candidate shape is timed with HIP events on a scratch output in
 *   two rounds of one warm-up and three timed launches, and the first
 *   candidate within 2% of the fastest is kept.  Mode 0 uses the largest
 *   allowed KR (KR divides nrhs, KR <= 4, <= 2 for FP64) and 256 threads.
 *   Changing the mode clears the tuned table.  Launches inside a HIP graph
 *   capture never tune (they use the default until a tuned shape exists).
 *   Candidate shapes: (a) KR vectors per thread, one lattice pass per
 *   group of KR vectors, 128 or 256 threads; (b) the same with all
 *   nrhs/KR groups side by side in one workgroup (32 or 64 sites x groups
 *   threads, at most 512); (c) one-vector kernels that issue the loads of
 *   the next 1..3 directions before the arithmetic of the current one
 *   (pipeline depth 2..4); each in h order, in t-major order (blocks of a
 *   parity walk t for a fixed tile of the x-y-z half slice, so that
 *   t-neighbours come from cache) or in z-slab order (blocks cover a slab
 *   of tm = 4 or 8 z-planes at t, then the same slab at t + 1, ..., so a
 *   site's t-neighbours are read a slab apart instead of a whole 3-d slice;
 *   the last slab may be thinner).  shape[4] = tm: 0 h order, 1 t-major,
 *   2..Lz slab thickness.
 * ovl_stencil_shape: shape[5] = {kr, bs, pipe, rin, tm} tuned for a
 *   full-lattice configuration (precision, link compression, number of
 *   extra epilogue vectors 0..3, batch size); all 0 when it has not been
 *   tuned yet.
 * ovl_stencil_set_shape: pins shape[5] for a configuration (all parity
 *   choices); OVL_E_ARG for shapes the kernels do not support.
 */
int ovl_stencil_tune(int mode);
int ovl_stencil_shape(const ovl_geom* g, ovl_prec prec, int compress12, int nextra, int nrhs, int* shape);
int ovl_stencil_set_shape(const ovl_geom* g, ovl_prec prec, int compress12, int nextra, int nrhs, const int* shape);

/* ovl_stencil_timer: per-configuration launch timing of the stencil kernels
 *   with HIP events recorded on the launch stream around every launch that
 *   is not being captured into a graph.  mode 1 clears and enables, 0
 *   disables (keeps what was measured), 2 clears.
 * ovl_stencil_timer_read: launches and summed kernel milliseconds of one
 *   configuration (precision, link compression, extra epilogue vectors 0..3,
 *   batch size) since the last clear; waits for the recorded events.
 */
int ovl_stencil_timer(int mode);
int ovl_stencil_timer_read(ovl_prec prec, int compress12, int nextra, int nrhs, int64_t* launches,
                           double* total_ms);

/* ovl_counters: stencil launches and vector applications of D_w issued from
 * the host since the last reset (graph replays are not seen here).
 */
int ovl_counters(int64_t* stencil_launches, int64_t* stencil_vectors, int reset);

/* ovl_mem_stats: device memory held by the library (workspace pool, which
 * keeps released buffers for reuse until the process ends; eigensolver
 * basis; packed links) now and at its peak since the last reset_peak; the
 * caller's own buffers (fields, borrowed eigenvectors) are not counted.
 * Either pointer may be NULL; with reset_peak the values returned are those
 * before the reset.
 */
int ovl_mem_stats(int64_t* live_bytes, int64_t* peak_bytes, int reset_peak);

#ifdef __cplusplus
}
#endif
#endif /* OVL_H */

/*
 * sunbloch -- SU(N) Bloch-vector form of a GKSL master equation on one
 * AMD Instinct MI355X (gfx950), FP64.
 *
 * Method: A. Liniov et al., "Unfolding quantum master equation into a system
 * of real-valued equations: computationally effective expansion over the
 * basis of SU(N) generators" (arXiv:1812.11626).  The density matrix of an
 * N-level system is written rho = 1/N + sum_j v_j F_j over the M = N^2 - 1
 * generators of SU(N) (Sec. II, eq. 5); the Lindbladian (eq. 1) becomes the
 * real affine ODE dv/dt = (Q(t) + R) v + K (eq. 9) whose matrices are
 * contractions of the structure constants f, d (eq. 4) with the expansion
 * coefficients of H and L_p (eqs. 6, 10, 11); the ODE is integrated with
 * classical RK4 (Sec. IV, step 3.1).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Generator order ("grouped"): index p in [0,P), P = N(N-1)/2, is the pair
 *    (j,k), j<k, in row-major order, p = j(2N-j-1)/2 + k-j-1; S^(j,k) has
 *    index p, J^(j,k) index P+p, D^l index 2P+l-1 (l = 1..N-1).  All indices
 *    are 0-based.  The diagonal generators are (sum_{i<l} G_ii - l G_ll) /
 *    sqrt(l(l+1)) (the factor i printed in Sec. II is dropped; see design
 *    notes).
 *  - Every pointer argument documented "device" must point to memory of the
 *    current HIP device; "host" pointers are ordinary CPU memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Kernels are queued on it.  Entry points that return sizes or counts to
 *    host memory synchronise that stream before returning.
 *  - Memory ownership: buffers passed in stay owned by the caller.  Objects
 *    created by the library (sun_basis, sun_lind, sun_prop, sun_batch,
 *    sun_adj) own their internal device memory until the matching *_free
 *    call; it comes from hipMalloc, or from the caller's allocator after
 *    sun_set_allocator.  Objects must be freed before the process ends.
 *  - Errors: every int-returning call returns SUN_OK (0) or a negative
 *    status; sun_last_error() then returns a message for the calling thread.
 *    On error, outputs are unspecified but no object is leaked.
 *  - Calls on one object are not thread-safe; distinct objects are.
 */
#ifndef SUNBLOCH_H
#define SUNBLOCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SUN_OK = 0,
  SUN_EINVAL = -1,   /* invalid argument (sizes, null pointers, non-Hermitian H, gamma < 0, ...) */
  SUN_ENOMEM = -2,   /* device allocation failed */
  SUN_EDEVICE = -3,  /* a HIP runtime call failed */
  SUN_ENOTSUP = -4,  /* valid input outside what the library supports (limits stated per call) */
  SUN_ERANGE = -5,   /* caller buffer too small; the needed size is returned */
  SUN_EDIVERGED = -6,/* the propagated state (or a result computed from it) is not finite */
  SUN_EUNSTABLE = -7,/* dt * |lambda|max beyond the RK4 stability bound set by sun_prop_guard_stability */
  SUN_ENOTCONVERGED = -8 /* an iterative solve stopped at its iteration limit above its tolerance */
};

/* Message describing the last failure on the calling thread ("" if none). */
const char* sun_last_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int sun_version(void);

/* Device memory of the library (object layouts, assembly temporaries,
 * internal work buffers) comes from hipMalloc/hipFree unless the caller
 * installs its own pair here, e.g. a framework's caching allocator, so that
 * the framework accounts for it and can reuse it.
 *   alloc(bytes, stream, ctx) returns device memory of at least `bytes`
 *     bytes, 256-byte aligned, usable on `stream` (the stream of the call
 *     that allocates, NULL = the default stream), or NULL on failure (the
 *     library then returns SUN_ENOMEM);
 *   release(ptr, ctx) gives it back.  The library synchronises the device
 *     before calling it (as hipFree does), so no queued kernel still uses
 *     the memory.
 * Both NULL restores hipMalloc/hipFree; exactly one NULL is SUN_EINVAL.
 * Every buffer is released through the pair that allocated it, so objects
 * created before a change stay valid.  Process-wide; install it before
 * creating objects, not while other threads call the library.  The
 * allocation-free entry point never calls either. */
typedef void* (*sun_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*sun_release_fn)(void* ptr, void* ctx);
int sun_set_allocator(sun_alloc_fn alloc, sun_release_fn release, void* ctx);

/* ------------------------------------------------------------------------
 * Basis (Sec. II; Sec. IV step 2.2)
 * ---------------------------------------------------------------------- */
typedef struct sun_basis_s* sun_basis;

/* Build the device metadata of the SU(N) basis: pair <-> index tables and the
 * normalisations 1/sqrt(l(l+1)).  Requires 2 <= N and M = N^2-1 < 2^31.
 * O(N^2) device memory. */
int sun_build_basis(int32_t N, void* stream, sun_basis* out);
/* N and M of a basis. */
int sun_basis_dims(sun_basis b, int32_t* N, int64_t* M);
/* Number of nonzero entries of the full structure-constant tensors f_mns and
 * d_mns (all index orders), counted on the GPU by enumerating the closed-form
 * nonzero pattern (Sec. IV step 2.2 states that the pattern is known
 * analytically).  Host outputs; synchronises `stream`. */
int sun_basis_counts(sun_basis b, void* stream, int64_t* nnz_f, int64_t* nnz_d);
/* Export the nonzero entries of f (which = 0) or d (which = 1) in
 * lexicographic order of (m, n, s): with canonical = 0 every index order of
 * the full tensor; with canonical = 1 only m < n < s for f (antisymmetric,
 * zero when two indices repeat) and m <= n <= s for d (symmetric), from which
 * the full tensor follows by permutation.  idx device int32[cap][3], val
 * device double[cap].  *written (host) receives the number of entries; if it
 * exceeds cap, nothing is written and SUN_ERANGE is returned.  Supports
 * N <= 64 (each row of the tensor must have at most 8192 entries). */
int sun_basis_export(sun_basis b, int32_t which, int32_t canonical, int32_t* idx, double* val,
                     int64_t cap, int64_t* written, void* stream);
void sun_basis_free(sun_basis b);

/* ------------------------------------------------------------------------
 * Operators and their expansion (Sec. IV step 2.1)
 * ---------------------------------------------------------------------- */
/* N x N complex operator in CSR form, all arrays device memory.  Columns in
 * each row must be strictly increasing (no duplicates).  im may be NULL for a
 * real operator. */
typedef struct {
  int32_t n;
  int32_t nnz;
  const int32_t* rowptr; /* [n+1] */
  const int32_t* col;    /* [nnz] */
  const double* re;      /* [nnz] */
  const double* im;      /* [nnz] or NULL */
} sun_zcsr;

/* Expansion coefficients x_m = Tr(F_m X), m = 0..M-1 (complex for a
 * non-Hermitian X), and the trace Tr(X).  coef_re/coef_im: device double[M];
 * trace: host double[2] (re, im) or NULL (synchronises when non-NULL). */
int sun_expand_operator(sun_basis b, const sun_zcsr* X, double* coef_re,
                        double* coef_im, double* trace, void* stream);

/* ------------------------------------------------------------------------
 * Readout (Sec. II eq. 5; Sec. IV step 3.2)
 * ---------------------------------------------------------------------- */
/* Density matrix rho = 1/N + sum_j v_j F_j of a Bloch vector v (device
 * double[M]) into rho_re, rho_im (device double[N*N], row-major; rho_im may
 * be NULL to skip the imaginary part).  Asynchronous on `stream`. */
int sun_bloch_density(sun_basis b, const double* v, double* rho_re, double* rho_im,
                      void* stream);
/* Expectation values Tr(rho_i X) = Tr(X)/N + sum_j v_ij x_j for nvec Bloch
 * vectors v_i = v + i*ldv (device; ldv >= M when nvec > 1), where x_j =
 * Tr(F_j X) are X's coefficients from sun_expand_operator (x_re, x_im device
 * double[M]; x_im may be NULL when out_im is NULL) and trace = Tr(X) (host
 * double[2] as re, im, or NULL for a traceless X).  out_re, out_im: device
 * double[nvec] (out_im may be NULL).  One workgroup per vector, fixed-order
 * reduction.  Asynchronous on `stream`. */
int sun_bloch_expect(sun_basis b, const double* v, int64_t nvec, int64_t ldv,
                     const double* x_re, const double* x_im, const double* trace,
                     double* out_re, double* out_im, void* stream);

/* ------------------------------------------------------------------------
 * Lindbladian expansion (Sec. II eqs. 6, 10, 11; Sec. IV steps 2.3-2.5)
 * ---------------------------------------------------------------------- */
typedef struct sun_lind_s* sun_lind;

enum { SUN_TERM_H = 0, SUN_TERM_L = 1 };

/* Assemble, for each Hamiltonian term H_a (a < nH), the real M x M matrix
 * Q_a with (Q_a)_sn = sum_m f_mns h_m (eq. 6), and for each dissipator L_p
 * (p < P) the matrix R_p and vector K_p at unit rate:
 *     R_p = -(1/2) Re(B^T A),  A_lm = sum_j l_j z_jlm,  B_ls = sum_k conj(l_k) f_kls,
 *     z = f + i d,             K_p = (1/N) Im(B^T l)
 * (eq. 10 with the prefactor and z read as derived in the design notes;
 * eq. 11 with the rate factored out).  The structure constants are
 * generated on the fly from their closed forms; nothing of size O(N^3) is
 * stored.  Exact cancellations are dropped from each matrix: entries with
 * |q| <= 1e-12 max|Q| are removed.
 * H terms must be Hermitian (checked to 1e-12 max|H|, else SUN_EINVAL).  The
 * expansion of eqs. 10-11 runs over the traceless generators; an L with a
 * trace, L = c 1 + L' (c = Tr(L)/N), is handled by the identity
 * D_L = D_L' - i[H_c, .] with H_c = (i/2)(conj(c) L' - c L'^+): R_p is then
 * the R of L' plus the Q of H_c (eq. 6), and K_p is unchanged.
 * Limits: a term whose assembled rows have more than 16384 raw
 * contributions (8192 on devices with less than 160 KB of LDS per
 * workgroup), which dense L reaches beyond N ~ 60, is assembled by the dense
 * path of sun_expand_lindbladian_dense instead (detected from the per-row
 * counts before any fill); total nnz of each matrix < 2^31.  Sparse
 * operators (the dimer: <= 5N per row) are far inside the limit.
 * Synchronises `stream` (sizes are read back).  */
int sun_expand_lindbladian(sun_basis b, const sun_zcsr* H, int32_t nH,
                           const sun_zcsr* L, int32_t P, void* stream,
                           sun_lind* out);
/* The same matrices by the dense path, for operators with many nonzeros
 * (dense or random L and H): every row of the contractions is written into
 * a dense M x M array by the thread that generates it, and the dissipative
 * part is formed as one real matrix product on the matrix cores,
 *     R_p = -(1/2) [Re B^T | -Im B^T] [Re A ; Im A] = -(1/2) Re(B^T A)
 * (eq. 10 with dense sections; a K = 2M contraction), then compressed to CSR
 * with the same drop rule.  No per-row limit; device memory about 5 M^2
 * doubles while a dissipator is assembled (4 GB at N = 100); M^2 < 2^33
 * (N <= 304, else SUN_ENOTSUP).
 * sun_expand_lindbladian itself switches to this path for a term whose rows
 * exceed its per-row limit.  Synchronises `stream`. */
int sun_expand_lindbladian_dense(sun_basis b, const sun_zcsr* H, int32_t nH,
                                 const sun_zcsr* L, int32_t P, void* stream,
                                 sun_lind* out);
/* C = alpha A B + beta C in FP64 (row-major, device pointers; A: M x K with
 * leading dimension lda >= K, B: K x N with ldb >= N, C: M x N with ldc >= N)
 * on the matrix cores (the kernel the dense path uses; exposed for
 * measurement).  beta = 0 does not read C.  Asynchronous on `stream`. */
int sun_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double beta, double* C, int64_t ldc, void* stream);
/* nnz of Q_a (which = SUN_TERM_H) or R_p (which = SUN_TERM_L). */
int sun_lind_nnz(sun_lind l, int32_t which, int32_t index, int64_t* nnz);
/* Copy Q_a or R_p out as CSR into caller device buffers rowptr int32[M+1],
 * col int32[nnz], val double[nnz]; for SUN_TERM_L and K != NULL also K_p
 * (device double[M]).  Any of rowptr/col/val may be NULL to skip it. */
int sun_lind_export(sun_lind l, int32_t which, int32_t index, int32_t* rowptr,
                    int32_t* col, double* val, double* K, void* stream);
void sun_lind_free(sun_lind l);

/* ------------------------------------------------------------------------
 * Propagation (eq. 9; Sec. IV step 3.1): classical RK4
 * ---------------------------------------------------------------------- */
typedef struct sun_prop_s* sun_prop;

/* Terms of a sun_lind are numbered 0..nH-1 (Hamiltonians) then nH..nH+P-1
 * (dissipators).  The generator is
 *     G(t) = sum_a w_a T_a + sum_{d<ndyn} c_d(t) T_{dyn[d]},
 *     K(t) = sum_{a in L} w_a K_a + sum_{d: dyn[d] in L} c_d(t) K_{dyn[d]}
 * static_w: host double[nH+P] (the weights of dissipators, i.e. their rates,
 * must be >= 0, else SUN_EINVAL); dyn: host int32[ndyn], ndyn <= 4.
 * Builds the fused device layout (static part merged into one CSR, the
 * free vector folded in as an extra column, then one segment per dynamic
 * term) and the row-block partition of the streaming kernel. */
int sun_prop_create(sun_lind l, const double* static_w, const int32_t* dyn,
                    int32_t ndyn, void* stream, sun_prop* out);
/* Advance v (device double[M], in/out) by `steps` RK4 steps of size dt.
 * coef: device double[(2*steps+1) * ndyn]; row k holds c_d(t0 + k dt/2), so
 * the stages of step n read rows 2n, 2n+1, 2n+1, 2n+2.  Four kernel launches
 * per step (one per stage), or one launch for all steps on the resident path
 * (see sun_prop_tune_resident).  With the finite check on (the default) the
 * call synchronises `stream` at the end and returns SUN_EDIVERGED for a
 * non-finite state; with it off the call is asynchronous on `stream`.  With a
 * stability guard set (sun_prop_guard_stability) a larger |dt| returns
 * SUN_EUNSTABLE before any launch.  A propagator whose re-layout failed
 * part-way returns SUN_EINVAL until a layout is selected again. */
int sun_propagate(sun_prop p, double* v, const double* coef, double dt,
                  int64_t steps, void* stream);
/* Same as sun_propagate, recording along the way (Sec. IV step 3.2): after
 * steps n = every, 2 every, ..., nrec every (nrec = steps / every, rounded
 * down; any remaining steps are still taken) record r = n/every - 1 stores
 *   states + r*ld   <- v_n          (states: device double[nrec*ld], ld >= M, or NULL)
 *   obs[r]          <- x0 + x . v_n (x: device double[M]; obs: device double[nrec],
 *                                    or NULL to skip; obs needs x)
 * e.g. x_j = Tr(F_j X) from sun_expand_operator and x0 = Tr(X)/N give
 * obs = Tr(rho X) (eq. 5).  The dot products are reduced in a fixed order;
 * the states are bitwise those of sun_propagate calls of `every` steps. */
int sun_propagate_record(sun_prop p, double* v, const double* coef, double dt,
                         int64_t steps, int64_t every, double* states, int64_t ld,
                         const double* x, double x0, double* obs, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as sun_propagate_record, bitwise, with the
 * observable's partial sums kept in a fixed device array of 1024 doubles
 * (8 KiB per device, held until the process ends) instead of a buffer the
 * object allocates on first use; the call makes no device allocation.  The
 * partials of any size fit (at most 512 pairs); a request beyond the array
 * would return SUN_ENOTSUP.  Every call on one device shares that device's
 * array, so calls that overlap on one device (concurrent streams or threads
 * with obs != NULL) race; serialise them.  Same arguments and errors as
 * sun_propagate_record. */
int sun_propagate_record_noalloc(sun_prop p, double* v, const double* coef, double dt,
                                 int64_t steps, int64_t every, double* states, int64_t ld,
                                 const double* x, double x0, double* obs, void* stream);
/* Stability guard (RK4 is stable only while every eigenvalue lambda of the
 * generator's linear part has lambda*dt inside its stability region): the
 * spectral radius is estimated by power iteration (as sun_prop_spectral_radius,
 * `iters` applications) at every corner of the box [coef_lo, coef_hi] of the
 * time-dependent coefficients (host double[ndyn] each; 2^ndyn estimates), and
 * from then on sun_propagate, sun_propagate_record(_noalloc) and
 * sun_propagate_profile refuse, with SUN_EUNSTABLE and before any launch, a
 * step with |dt| * rho_max > limit.  limit = 0 takes 2.6, just below 2.6156,
 * the smallest radius of the boundary of RK4's stability region
 * |1 + z + z^2/2 + z^3/6 + z^4/24| <= 1 in the closed left half-plane (on the
 * imaginary axis it is 2 sqrt 2), so that any eigenvalue with Re <= 0 and
 * |lambda| dt <= 2.6 is stable; limit < 0 turns the guard off (the default).
 * The corners bound the spectral radius when it is convex in the
 * coefficients, as it is for the driven dimer (|lambda|max ~ 2 sqrt(eps^2 +
 * J^2)(N-1)); it is an estimate otherwise.  *rho_max (host, may be NULL)
 * receives the largest estimate.  Synchronises `stream`. */
int sun_prop_guard_stability(sun_prop p, const double* coef_lo, const double* coef_hi, int32_t iters,
                             double limit, double* rho_max, void* stream);
/* Finite check (on by default): at the end of every sun_propagate,
 * sun_propagate_record(_noalloc) and sun_propagate_profile call, one kernel
 * checks the state for NaN and infinite entries, the call synchronises
 * `stream`, and a non-finite state is returned as computed with status
 * SUN_EDIVERGED.  A non-finite entry never becomes finite again under RK4
 * (each step adds to the previous value), so the check at the end of a call
 * catches divergence at any step of it; call per period to detect it per
 * period.  on = 0 turns the check off, and with it the synchronisation: the
 * calls are then asynchronous on `stream`. */
int sun_prop_check_finite(sun_prop p, int32_t on);
/* Stationary state of the time-independent generator G obtained by freezing
 * the time-dependent coefficients at coef (host double[ndyn]): the solution
 * of G v = -K (eq. 9 with dv/dt = 0; the paper's asymptotic state of a
 * time-independent Lindbladian, Sec. I, in Bloch form).  Restarted GMRES
 * (restart vectors, at most max_iter iterations in total) on the RK4 time-tau
 * map, tau = steps_per_map * dt: (I - Phi) v = phi with Phi = R4(dt G)^n and
 * phi the map of the zero state, applied by the propagator's stage kernels.
 * The fixed point of that map is exactly the solution of G v = -K; modes
 * decaying faster than 1/tau are damped by the map, so GMRES only has to
 * resolve the slower ones (choose tau of a few inverse decay rates; the
 * driven dimer's slowest rate is about 0.15, and tau = 5 converges in about
 * 17 iterations for N up to 301).  dt must be a stable RK4 step for G.
 * v: device double[M], the initial guess on entry (e.g. zeros) and the
 * solution on return.  Converged when ||G v + K||_2 <= tol ||K||_2 (K = 0:
 * v = 0, the maximally mixed state, is returned).  *iters and *relres (host,
 * may be NULL) receive the GMRES iterations and ||G v + K||_2 / ||K||_2.
 * SUN_ENOTCONVERGED when max_iter is reached above tol (v holds the last
 * iterate), SUN_EDIVERGED for a non-finite iterate.  Allocates (restart + 6)
 * vectors of M+1 doubles for the call; synchronises `stream`. */
int sun_stationary(sun_prop p, const double* coef, double dt, int64_t steps_per_map, int32_t restart,
                   int32_t max_iter, double tol, double* v, int32_t* iters, double* relres, void* stream);
/* Spectral radius |lambda|max of the linear part of the generator, G with
 * the time-dependent coefficients frozen at coef (host double[ndyn]), by
 * power iteration: `iters` applications of G to a normalised pseudo-random
 * start vector, returning the mean growth factor per application over the
 * second half (host double *rho).  For choosing RK4 steps: the method is
 * stable for |lambda| dt up to about 2.8 on the imaginary axis.  Allocates
 * its own work vectors; synchronises `stream`.  SUN_ERANGE if the iteration
 * collapses (G x = 0) or overflows. */
int sun_prop_spectral_radius(sun_prop p, const double* coef, int32_t iters, double* rho,
                             void* stream);
/* Same as sun_propagate, and additionally records a HIP event pair around
 * every stage launch on `stream`; on return (synchronised) stage_ms[i]
 * (host double[4]) holds the summed GPU time of stage i over all steps and
 * *launches (host, may be NULL) the number of launches.  For measurement. */
int sun_propagate_profile(sun_prop p, double* v, const double* coef, double dt,
                          int64_t steps, void* stream, double* stage_ms,
                          int64_t* launches);
/* For tests of the error paths: site 1 makes the next layout build (by
 * sun_prop_tune, sun_prop_tune_sliced, the adjoint's first run or
 * sun_batch_tune to path 7) fail with SUN_ENOMEM after it has rewritten part
 * of the propagator or group, as a device allocation failure there would;
 * site 0 clears a pending injection.  A propagator left incomplete that way
 * refuses every launching call with SUN_EINVAL until a layout is selected
 * again; a batch group left incomplete (by this or any failure inside
 * sun_batch_tune) makes sun_batch_run refuse with SUN_EINVAL until the group
 * is tuned again. */
int sun_debug_inject_failure(int32_t site);
/* Layout facts for measurement: nnz of the fused matrix (static + dynamic
 * segments + folded free vector), number of work units per stage launch
 * (row blocks, or slices + long rows), rows M. */
int sun_prop_info(sun_prop p, int64_t* nnz_fused, int64_t* nblocks, int64_t* M);
/* Two device layouts exist for the stage kernel:
 *  1 (default when ndyn <= 1) sliced ELL: rows of at most long_len nonzeros
 *    are sorted by length inside windows of sigma rows and packed 64 per
 *    slice, one wavefront lane per row; longer rows are reduced by one
 *    wavefront each.
 *  0 (default for 2-3 time-dependent terms up to 100,000 fused nonzeros,
 *    and for 4) CSR stream: row blocks of about block_nnz
 *    nonzeros are streamed into LDS by a workgroup of `threads` lanes, then
 *    reduced one lane per row.
 * Rows summed by one lane (all of layout 0, the short rows of layout 1 with
 * one wavefront per slice) add their entries in nonzero order; long rows use
 * a wavefront tree reduction.  sun_prop_tune selects layout 0
 * with its knobs (block_nnz a power of two in [128, 8192], threads 64, 128 or
 * 256, xcd_remap 0/1 gives each XCD one contiguous range of blocks);
 * sun_prop_tune_sliced selects layout 1 (sigma a power of two in [64, 4096],
 * long_len in [1, 4096]; ndyn <= 1 only).  In layout 1 the column index of
 * each stored entry is kept as an offset from a per-(slice, entry) base, in
 * 1, 2 or 4 bytes per slice, the narrowest that fits; min_col_bytes (1, 2, 4)
 * bounds that width from below (4 = uncompressed).  flags of
 * sun_prop_tune_sliced: bit 0 gives each XCD one contiguous range of slices
 * (so the state entries its rows gather stay in that XCD's L2); bit 1 reads
 * the matrix stream with non-temporal loads (sun_prop_create chooses them
 * when one launch streams more than 288 MiB of matrix data, too much for the
 * memory-side cache to hold between launches, and ordinary loads, which let
 * the matrix stay there, otherwise); bit 2 cuts the slices from the pair-interleaved row sequence (S_p,
 * J_p adjacent: one gathered range per slice range instead of two, but wider
 * column offsets; off by default); bits 16-23 the entries a lane loads per
 * round (4, 6, 8, 12, 16; 0 = chosen with the next field); bits 24-26 the
 * wavefronts that share a slice (1, 2 or 4, the latter two with 4 or 8
 * entries per round; 0 = chosen from the number of slices and long rows: 4
 * below 12,000, 2 below 24,000, else 1, with 4 entries per round below
 * 1,000 and 8 above).  With 2 or 4 wavefronts per slice a row's sum is
 * formed in that many consecutive parts (ranges of whole multiples of 4
 * entries; a long row: interleaved groups of 64 entries) added in part
 * order, so results differ from one wavefront per slice in rounding only and
 * do not depend on the other fields.  Other bits must be 0 (else SUN_EINVAL).  Defaults: block_nnz 1024,
 * threads 256, xcd_remap 1; sigma 4096, long_len 32, min_col_bytes 1,
 * flags 1 (3 when the matrix stream exceeds 288 MiB per launch), and the
 * wavefronts per slice and entries per round chosen as for fields of 0. */
int sun_prop_tune(sun_prop p, int32_t block_nnz, int32_t threads, int32_t xcd_remap,
                  void* stream);
int sun_prop_tune_sliced(sun_prop p, int32_t sigma, int32_t long_len, int32_t min_col_bytes,
                         int32_t flags, void* stream);
/* Resident path (on by default for small generators -- at most 2500 fused
 * nonzeros, 4(M+1) doubles within one workgroup's LDS, at most one
 * time-dependent term -- and selectable up to the LDS limit): sun_propagate and
 * sun_propagate_record keep v, the stage vectors and the accumulator in the
 * LDS of a single workgroup and run all steps of a call (of a recording
 * interval) in one launch, instead of four launches per step; rows are summed
 * in the same order and rounding as by the sliced kernel.  on = 0 turns it
 * off (sun_prop_tune and sun_prop_tune_sliced also do); on = 1 where it
 * does not apply returns SUN_ENOTSUP. */
int sun_prop_tune_resident(sun_prop p, int32_t on);
/* HIP-graph replay in sun_propagate.  Where a stage launch is dominated by
 * launch latency (M <= 160,000, e.g. the dimer up to N = 400), sun_propagate
 * captures 64 RK4 steps (256 stage launches on the propagator's own
 * vectors) into a graph once per layout and step size and replays it, after
 * copying the chunk's 129 coefficient rows into a fixed device buffer; the
 * remaining steps are launched directly.  Results are bitwise those of
 * direct launches.  mode 0: never; 1: where M <= 160,000 (default); 2:
 * always (64 or more steps).  A re-layout (sun_prop_tune*) or a new dt
 * recaptures.  The graph is launched on the call's stream; the capture uses
 * a stream of the propagator's own (default priority). */
int sun_prop_use_graphs(sun_prop p, int32_t mode);
/* Device memory an object holds (layouts, state and work buffers), in bytes
 * (host size_t).  Host-side bookkeeping; no device work.  With
 * sun_set_allocator installed, this is the memory those objects took from the
 * caller's allocator. */
int sun_prop_device_bytes(sun_prop p, size_t* bytes);
int sun_lind_device_bytes(sun_lind l, size_t* bytes);
/* Current layout, number of stored matrix entries (with padding), rows on
 * the long-row path, and bytes of matrix data plus per-row metadata one
 * stage launch streams (sliced layout: excluding the long rows' entries). */
int sun_prop_layout(sun_prop p, int32_t* layout, int64_t* stored_entries, int64_t* long_rows,
                    int64_t* bytes_per_launch);
void sun_prop_free(sun_prop p);

/* ------------------------------------------------------------------------
 * Batched propagation: many parameter instances, one launch per RK4 stage
 * ---------------------------------------------------------------------- */
typedef struct sun_batch_s* sun_batch;

/* Groups of instances that share an assembled system lind[g] (terms T_a,
 * a < nt_g = nH + P of that system; nt_g <= 8).  Instance b of group g
 * evolves under G_b(t) = sum_a c_{b,a}(t) T_a and K_b(t) = sum over the
 * dissipator terms of c_{b,a}(t) K_a, with the coefficient on the half-step
 * grid t_k = k dt_g / 2 given by c_{b,a}(t_k) = w_g[b*nt_g + a] +
 * u_g[b*nt_g + a] * wave_g[k].  w[g], u[g]: device double[B[g]*nt_g];
 * wave[g]: device double[2*steps[g]+1]; dt, steps: host arrays.  The library
 * keeps pointers to w, u and wave (they must outlive the object).  Each group
 * gets a fused row layout with one segment per term and a state of
 * (M_g+1) x ld_g doubles per buffer (4 buffers, ld_g = B[g] rounded up to 128).
 * States start at zero; set them with sun_batch_set_state.  Synchronises. */
int sun_batch_create(const sun_lind* lind, int32_t ngroups, const int32_t* B,
                     const double* const* w, const double* const* u,
                     const double* const* wave, const double* dt,
                     const int64_t* steps, void* stream, sun_batch* out);
/* Load the states of group g from V (device double[B[g]][M_g], one Bloch
 * vector per instance) and reset the group's step counter to 0. */
int sun_batch_set_state(sun_batch b, int32_t g, const double* V, void* stream);
/* Copy the states of group g to V (device double[B[g]][M_g]). */
int sun_batch_get_state(sun_batch b, int32_t g, double* V, void* stream);
/* Advance every group (or only group `only_group` if >= 0) by up to nsteps
 * RK4 steps, never past its own step count.  Each step is four launches
 * (one per stage) that cover all active groups: work items (group, block of
 * rows, tile of instances) are spread over a fixed grid of wavefronts.
 * Synchronises at the end; a non-finite state of a group the call advanced
 * returns SUN_EDIVERGED. */
int sun_batch_run(sun_batch b, int64_t nsteps, int32_t only_group, void* stream);
/* Per-group tiling.  tile = instances per lane group (8, 16, 32 or 64; a
 * lane group of `tile` lanes sums one row for `tile` instances; 128: 64
 * lanes with two consecutive instances each, on the LDS path, else 64).  path 0
 * (default): one workgroup per (instance tile, block of at most
 * min(rows_per_item, 128) rows and 1024 stored entries), the block's
 * columns, values and row/segment pointers staged in LDS; each XCD sweeps
 * its own eighth of every group's (tile, block) items in tile-major order;
 * taken when every row of the group has at most 1024 entries, else path 1.  path 1: one
 * wavefront per (block of rows_per_item rows, instance tile), reading the
 * matrix from global memory.  path 2: path 0 with two consecutive instances
 * per lane for tiles 16, 32 and 64 as well (tile/2 lanes per row; a group
 * with a row of more than 1024 entries falls back to path 1).  path 3 (tile
 * 8, 16 or 32): path 2 with the state rows each block gathers staged in LDS
 * too (blocks also limited to 4096/tile distinct columns; a group where one
 * row exceeds that falls back to path 2).  path 4 (tile 2, 4 or 8
 * instances per wavefront; rows_per_item unused): the group's state is kept
 * instance-major on a segmented sliced layout of its generator, the terms
 * whose coefficients are the same for every instance merged and the others
 * (1 to 3) kept as segments; SUN_ENOTSUP otherwise.  path 5 (tile 64 or 128;
 * rows_per_item unused): one wavefront per (row, tile of 64 instances with
 * one per lane, or 128 with two), the row's pointers, columns and values
 * read through the scalar cache, each XCD sweeping one eighth of the
 * group's rows in order with the device's resident wavefronts.  path 7
 * (tile 64; rows_per_item 1 to 32 is the most rows per block): persistent
 * workgroups (two per CU) walk (tile, block) items whose blocks are taken
 * along 4 x 4 tiles of the (j, k) pair grid with at most 127 distinct
 * columns; each block's state rows, matrix data and coefficients are
 * staged in LDS while the previous block is summed from LDS; rows with more
 * distinct columns are summed from global memory by a few workgroups of
 * their own; SUN_ENOTSUP when a group's state reaches 2 GiB.  Defaults
 * 64, 64, 0.  Paths 0-3, 5 and 7 add every term's entries in row order: their
 * results do not depend on the tiling or path; path 4 groups the row sums
 * differently and agrees with them to rounding. */
int sun_batch_tune(sun_batch b, int32_t g, int32_t tile, int32_t rows_per_item, int32_t path,
                   void* stream);
int sun_batch_info(sun_batch b, int32_t g, int64_t* M, int64_t* nnz, int32_t* tile,
                   int32_t* rows_per_item);
/* Device memory the batch holds (every group's layout and states), bytes. */
int sun_batch_device_bytes(sun_batch b, size_t* bytes);
void sun_batch_free(sun_batch b);
/* The batched form in one call: sun_batch_create with these arguments,
 * states loaded from V[g] (device double[B[g]][M_g], one Bloch vector per
 * instance), every group advanced through all of its steps[g] steps with the
 * default tiling, and the final states written back to V[g].  A non-finite
 * final state returns SUN_EDIVERGED (the states are still written back).
 * Synchronises `stream`. */
int sun_propagate_batched(const sun_lind* lind, int32_t ngroups, const int32_t* B,
                          const double* const* w, const double* const* u,
                          const double* const* wave, const double* dt, const int64_t* steps,
                          double* const* V, void* stream);

/* ------------------------------------------------------------------------
 * Adjoint: gradient of a time-averaged observable through the RK4 map
 * ---------------------------------------------------------------------- */
typedef struct sun_adj_s* sun_adj;

/* Prepare the forward propagator of the generator described by (static_w,
 * dyn, ndyn) exactly as sun_prop_create does (ndyn <= 1 here), and a second
 * one over the transposed terms T_a^T (built on the GPU) for the reverse
 * sweep.  The terms of `l` must stay alive while the object is used. */
int sun_adjoint_create(sun_lind l, const double* static_w, const int32_t* dyn, int32_t ndyn,
                       void* stream, sun_adj* out);
/* J = (1/S_avg) sum_{n=steps-S_avg+1}^{steps} cobs . v_n for the RK4 states
 * v_n from v0 (device double[M]) with the drive table coef (device
 * double[(2*steps+1)*ndyn], as for sun_propagate), and dJ/dtheta for ntheta
 * (<= 8) parameters, by the discrete adjoint of the RK4 map (the derivative
 * of this J, not of the exact ODE solution).  The coefficient of term a is
 * static_w[a] (+ c_d(t) if a = dyn[d]); its derivative is dstatic[a*ntheta +
 * th] (host) plus, for the time-dependent term, dcoef[(k*ndyn + d)*ntheta +
 * th] (device, may be NULL = 0).  cobs: device double[M].  States are
 * checkpointed every ckpt_every steps and recomputed one interval at a time
 * in the reverse sweep, except the last interval, which the forward sweep
 * keeps (memory: (steps/ckpt_every + ckpt_every + 10) vectors of M+1
 * doubles, plus 3*ckpt_every vectors of stage inputs when they fit in
 * 64 GiB).  When at most three terms depend on a parameter, the reverse
 * stages form the parameter dot products in the same pass, on a transposed
 * generator that keeps those terms as separate segments (built on the first
 * call, kept with the object); with more, one extra launch per step forms
 * them from per-term propagators.  J_out: host double; grad_out: host
 * double[ntheta] (may be NULL).  Synchronises. */
int sun_adjoint_run(sun_adj a, const double* v0, const double* coef, const double* dstatic,
                    const double* dcoef, int32_t ntheta, const double* cobs, double dt,
                    int64_t steps, int64_t S_avg, int64_t ckpt_every, double* J_out,
                    double* grad_out, void* stream);
/* Plan -> allocate -> execute form of sun_adjoint_run, for callers that own
 * the device memory (a PyTorch tensor, say).  sun_adjoint_plan returns, for a
 * run with these parameters (the set of parameter-dependent terms follows
 * from dstatic and the time-dependent term), the workspace size that keeps
 * the stage inputs of a checkpoint interval (*workspace_bytes; equal to the
 * minimum when they would exceed 64 GiB) and the minimum, which recomputes
 * them (*min_workspace_bytes, host, may be NULL).  It builds, on first use,
 * the layouts the object keeps for those terms (the segmented transposed
 * generator or the per-term propagators) and may synchronise `stream`.
 * sun_adjoint_execute runs sun_adjoint_run's computation on the caller's
 * workspace (device, 256-byte aligned, workspace_bytes long; smaller than the
 * minimum: SUN_ERANGE, no work done) and allocates no device memory of its
 * own for the run.  The workspace holds, laid out by the library: checkpoints
 * every ckpt_every steps, the states of one interval, optionally its stage
 * inputs, and the cotangent, stage and partial-sum vectors.  Its contents
 * need no initialisation and are meaningless afterwards.  A non-finite J or
 * gradient returns SUN_EDIVERGED (also from sun_adjoint_run). */
int sun_adjoint_plan(sun_adj a, const double* dstatic, int32_t ntheta, int64_t steps, int64_t ckpt_every,
                     void* stream, size_t* workspace_bytes, size_t* min_workspace_bytes);
int sun_adjoint_execute(sun_adj a, const double* v0, const double* coef, const double* dstatic,
                        const double* dcoef, int32_t ntheta, const double* cobs, double dt,
                        int64_t steps, int64_t S_avg, int64_t ckpt_every, void* workspace,
                        size_t workspace_bytes, double* J_out, double* grad_out, void* stream);
/* New static weights (host double[nH+P]; dissipation rates >= 0) for the
 * same terms and time-dependent term: rebuilds the forward propagator only.
 * The transposed terms are kept, and so is the segmented transposed generator
 * while the weights of the terms it merges (those that depend on no
 * parameter) are unchanged.  For parameter scans and optimisation loops
 * over one sun_adj.  Synchronises `stream`. */
int sun_adjoint_set_weights(sun_adj a, const double* static_w, void* stream);
/* The forward objective J alone (same definition), e.g. for finite differences. */
int sun_adjoint_objective(sun_adj a, const double* v0, const double* coef, const double* cobs,
                          double dt, int64_t steps, int64_t S_avg, double* J_out, void* stream);
void sun_adjoint_free(sun_adj a);

#ifdef __cplusplus
}
#endif
#endif /* SUNBLOCH_H */

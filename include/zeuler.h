/*
 * zeuler.h -- C ABI of libzeuler.so: the isospectral-midpoint (IsoMP) Zeitlin--Euler step on
 * the sphere for MI355X (gfx950), after Cifani, Viviani & Modin, "An efficient geometric
 * method for incompressible hydrodynamics on the sphere" (arXiv 2206.05466).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Matrices are N x N complex128, row-major, interleaved (re, im): entry (r, c) at
 *   element r*N + c, i.e. the memory of a contiguous torch.complex128 tensor.  Matrix
 *   arguments are DEVICE pointers on the context's GPU, 16-byte aligned, owned by the
 *   caller; the library never frees or keeps them.
 * - Diagonal m >= 0 of a matrix means its entries (i+m, i), i = 0..N-m-1 (0-based).
 * - The vorticity W and stream matrix P lie in u(N)/su(N) (skew-Hermitian).  The library
 *   reads only the lower triangle and diagonal of a skew-Hermitian input and writes both
 *   triangles of every skew-Hermitian output (the upper one as -conj of the lower).
 * - Calls are asynchronous on the stream given to ze_create, except where a call returns
 *   host values (documented per call): those synchronise that stream.
 * - Status codes only; nothing is thrown across the ABI.  A context is not thread-safe:
 *   calls on one context must not overlap.
 */
#ifndef ZEULER_H
#define ZEULER_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ze_ctx ze_ctx;  /* opaque: Laplacian factors and workspaces for one N */
typedef struct ze_ens ze_ens;  /* opaque: an ensemble of independent simulations */

typedef enum {
    ZE_OK = 0,
    ZE_EINVAL = 1,      /* bad argument: N < 1, null pointer, h or tol not finite, ... */
    ZE_ENOMEM = 2,      /* device or host allocation failed */
    ZE_ENOTCONV = 3,    /* fixed point not below tol after maxit evaluations (result still written) */
    ZE_ENONFINITE = 4,  /* NaN or Inf met in the fixed-point residual */
    ZE_EHIP = 5         /* a HIP runtime call failed */
} ze_status;

/* Arithmetic of the complex matrix products. */
typedef enum {
    ZE_PREC_FP64 = 0,   /* FP64 MFMA products */
    ZE_PREC_SPLIT = 1,  /* FP64 products emulated on INT8 MFMA: Ozaki splitting into s slices
                           (balanced digits: 7 bits, then 8 bits each) per row / column scale
                           (ze_set_split_slices), exact int32 slice products, FP64
                           accumulation; error ~2^(-8 s) relative to max|row| max|column| per
                           term of the inner sum */
    ZE_PREC_MIXED = 2,  /* ze_isomp_step / ze_isomp_run only: A = P W~ on FP64 MFMA, the lower
                           product Q = A P split as above with ze_set_split_slices_lower slices
                           (default 4).  Q's term enters the map with h^2/4, so its rounding
                           reaches the step at ~(h^2/4) 2^(-8 s_q) relative: at h = 0.005 and
                           s_q = 4 below the FP64 products' own rounding. */
    ZE_PREC_CRT = 3     /* the modular form of the INT8 emulation (Ozaki scheme II): rows of
                           A~ / columns of B~ scaled by powers of two to integers of b bits
                           (b = 55 up to N = 8192, 54 at 16384), residues modulo 16 pairwise
                           coprime moduli <= 256, three exact INT8 products per modulus, and the
                           Chinese remainder theorem; the only error is the rounding of the
                           scaled inputs, 2^-b relative to the row / column maximum, i.e.
                           FP64-level.  ze_zgemm, and in ze_isomp_step / ze_isomp_run the
                           product A = P W~ (the lower product then as ZE_PREC_MIXED's). */
} ze_prec;

/* Message for a status code (static string). */
const char* ze_strerror(ze_status s);

/* Last message recorded by the library in this thread ("" if none): the failing HIP call of a
 * ZE_EHIP, or the measured values of a W refused by ze_set_validation (cleared at the start
 * of each ze_isomp_step / ze_isomp_run). */
const char* ze_last_error(void);

/*
 * ze_create -- set up the quantised Laplacian for matrix size N (Sec. 3.2, eq. (delta_tria)):
 * the tridiagonal block Delta^m of every diagonal m = 0..N-1 is factored (LDL^T, FP64, on
 * the host) and uploaded, and the step's workspaces (4 N x N complex matrices)
 * are allocated on the current HIP device.
 *   N       matrix size, 1 <= N <= 16384.
 *   stream  hipStream_t (as void*) all work of this context is queued on; NULL = default stream.
 *   out     receives the context.
 * Errors: ZE_EINVAL (N out of range, out NULL), ZE_ENOMEM, ZE_EHIP.  Synchronous.
 */
ze_status ze_create(int N, void* stream, ze_ctx** out);

/* Free a context and everything it owns (synchronises its stream).  NULL is accepted. */
ze_status ze_destroy(ze_ctx* ctx);

/* Matrix size of a context (0 for NULL). */
int ze_size(const ze_ctx* ctx);

/*
 * ze_stream_solve -- P = Delta_N^+ W (Sec. 3.3, eq. (sub_tria_W)): one tridiagonal solve per
 * diagonal m, P_m = -(Delta^m)^{-1} W_m (the Laplacian is -Delta^m on diagonal m, its
 * eigenvalues being -l(l+1), eq. (lap_prop)), the upper triangle by skew-symmetry.  The
 * singular m = 0 block is solved as the pseudo-inverse: tr(W)/N is removed from its
 * right-hand side and the result is made traceless, so P is in su(N) even for W in u(N).
 *   W  device, N x N complex128 (lower triangle and diagonal read).
 *   P  device, N x N complex128 (fully written); must not alias W.
 * Errors: ZE_EINVAL (NULL pointers, P == W), ZE_EHIP.  Asynchronous.
 */
ze_status ze_stream_solve(ze_ctx* ctx, const void* W, void* P);

/*
 * ze_isomp_step -- one isospectral-midpoint step, eq. (isomp) (Sec. 2): W_n -> W_{n+1}, with
 * the implicit W~ found by the fixed-point iteration eq. (isomp_iter) from W~ = W_n.  Each
 * evaluation is one stream solve, A = P W~, and the lower triangle of Q = A P, the
 * commutator being A - A^H (Sec. 3.1).  It stops once the matrix infinity norm of the change
 * of W~ is below tol, and W_{n+1} is formed from that same evaluation's products: by default
 * the second line of eq. (isomp) at that W~, W~ + h/2 (A - A^H) - h^2/4 Q; or, with
 * ze_set_update_form 1, W_n + h (A - A^H).
 *   W       device, N x N complex128, skew-Hermitian; in: W_n, out: W_{n+1}.
 *   h       time step (any finite sign).
 *   tol     stopping tolerance (>= 0; 0 runs exactly maxit evaluations).
 *   maxit   evaluation cap, >= 1.
 *   prec    ZE_PREC_FP64, ZE_PREC_SPLIT, ZE_PREC_MIXED or ZE_PREC_CRT.
 *   iters   host, may be NULL: evaluations done (summed over the substeps of a step of
 *           order 4 or 6, see ze_set_order).
 *   resid   host, may be NULL: final residual (the largest over the substeps).
 * Errors: ZE_EINVAL, ZE_ENOTCONV (W holds the maxit-th W_{n+1}; at order 4 or 6 every substep
 * still runs, each stopping at maxit), ZE_ENONFINITE, ZE_EHIP.
 * Synchronises the stream once per evaluation (the convergence test), unless the stopping rule
 * runs on the device (ze_set_stopping).
 */
ze_status ze_isomp_step(ze_ctx* ctx, void* W, double h, double tol, int maxit, int prec,
                        int* iters, double* resid);

/*
 * ze_isomp_run -- nsteps IsoMP steps on the same W (the first exactly as ze_isomp_step; the
 * later ones start their fixed-point iteration as ze_set_initial_guess selects).
 *   iters, resid  host arrays of nsteps entries, may be NULL.
 * Stops at the first step that returns an error and returns it (host stopping rule; with the
 * rule on the device every step runs, and the status covers the whole run).
 */
ze_status ze_isomp_run(ze_ctx* ctx, void* W, double h, double tol, int maxit, int nsteps,
                       int prec, int* iters, double* resid);

/*
 * ze_set_stopping -- where the tolerance test of eq. (isomp_iter) (Sec. 2: stop once the
 * infinity norm of the change of W~ is below tol) is taken.
 *   mode 0  on the host (default): the residual is read back after each evaluation.
 *   mode 1  on the device: ze_isomp_step / ze_isomp_run enqueue maxit evaluations per step
 *           (substep at order 4 or 6); the residual kernel sets a device flag once the change
 *           is below tol (or not finite) and every later kernel of that step returns at once,
 *           so W_{n+1} is that of the same evaluation as with mode 0 (same kernels, same order:
 *           bit-identical results).  Nothing synchronises except, at the end of the call, the
 *           copy of the per-step counts when iters or resid is non-NULL; with both NULL the
 *           call is asynchronous and can be captured into a HIP graph (ze_run_stats reads the
 *           counts afterwards).  Every step of a run is executed even when one fails to
 *           converge.  A skipped evaluation still costs its (empty) launches, so maxit is best
 *           set near the most evaluations a step needs.  Every precision (the split and modular
 *           products' kernels read the flag too); ze_profile's per-phase timing is not taken.
 * Selecting mode 1 allocates the per-step records (65536 steps; older steps of a longer run
 * are reported as -1).
 * Errors: ZE_EINVAL, ZE_ENOMEM.
 */
ze_status ze_set_stopping(ze_ctx* ctx, int mode);

/*
 * ze_set_steady_cap -- evaluation cap of the steps with index >= from_step in a ze_isomp_run
 * call: min(maxit, cap) instead of maxit (cap 0, the default: maxit for every step).  Meant for
 * the polynomial starts (ze_set_initial_guess 2, 3), after whose start-up a step takes one
 * evaluation: with the stopping rule on the device every step enqueues its cap of evaluations,
 * so a cap of 2 leaves one skipped evaluation per step instead of maxit - 1.  A step that
 * reaches the cap above tol reports ZE_ENOTCONV as with maxit.
 * Errors: ZE_EINVAL (cap or from_step negative).
 */
ze_status ze_set_steady_cap(ze_ctx* ctx, int cap, int from_step);

/*
 * ze_set_continuation -- 1: a ze_isomp_run on the same W (the same device pointer, holding the
 * last run's result unchanged), with the same h, precision, starting-iterate mode, order and
 * update form as the last successful run on this context, continues that run's trajectory: its
 * steps carry on the step index (which the starting iterate and ze_set_steady_cap go by) and
 * the history of midpoints, so a long simulation split into calls (diagnostics between them,
 * as in the long runs of Sec. 4) takes the same steps as one call.  Anything else starts a new
 * run at step 0: a call that differs in one of those, a step of ze_isomp_step or a call of a
 * step-option setter (initial guess, order, update form, slices) in between, a run that ended
 * early with an error or ZE_ENOTCONV; with guess mode 3 at order 2, a previous
 * trajectory of fewer than 4 steps (the states its first steps use are not kept).  0 (the
 * default): every call starts at step 0.  The library cannot see whether W was changed
 * between the calls: the caller keeps it unchanged.  A run captured into a graph is recorded
 * with the step indices it had at capture.  Errors: ZE_EINVAL.
 */
ze_status ze_set_continuation(ze_ctx* ctx, int on);

/*
 * ze_run_stats -- on-device stopping: synchronises the context's stream and reads the last
 * nsteps steps of the last ze_isomp_run / ze_isomp_step call (nsteps <= its length).
 *   iters, resid  host arrays of nsteps entries (may be NULL), as ze_isomp_run fills them.
 * Returns the run's status: ZE_ENONFINITE or ZE_ENOTCONV if any of its steps had it, else
 * ZE_OK; ZE_EINVAL if mode 1 is not selected or nsteps is out of range; ZE_EHIP.
 */
ze_status ze_run_stats(ze_ctx* ctx, int nsteps, int* iters, double* resid);

/*
 * ze_set_initial_guess -- starting iterate of the fixed-point iteration (eq. (isomp_iter))
 * for the steps after the first in one ze_isomp_run call; the paper does not fix it.
 *   mode 0  W~ = W_n (default; ze_isomp_step always uses it).
 *   mode 1  W~ = 2 W_n - F_prev, F_prev the previous step's converged midpoint: W~
 *           approximates W half a step ahead, so this linear extrapolation is second-order
 *           accurate and usually saves one evaluation per step; the iteration still runs
 *           to the same tolerance and reaches the same fixed point.
 *   mode 2  the converged midpoints of one run are equally spaced samples of a smooth curve:
 *           the second step starts as in mode 1, the k-th (k >= 3) from the polynomial of
 *           degree min(k - 2, 3) through the last min(k - 1, 4) midpoints, one step ahead
 *           (c = (2, -1), (3, -3, 1), (4, -6, 4, -1), newest first).  Its error is O(h^4),
 *           usually below tol, so after the start-up a step takes one evaluation (with
 *           ze_set_update_form 1).  At order 4 or 6 (ze_set_order) each substep extrapolates
 *           from its own midpoints of the earlier steps (the other substeps of the first
 *           step start as in mode 1).  Selecting it allocates 4 N x N complex buffers per
 *           substep, less the one F already is (kept until ze_destroy).
 *   mode 3  as mode 2, and at order 2 the third and fourth steps of a run (n = 2, 3) add the
 *           n-th backward difference of the run's states W_n .. W_0 to the midpoint
 *           polynomial: each midpoint is the average of its step's two states plus an offset
 *           of order h^2 (the sum of the two lines of eq. (isomp)), so extrapolating the next
 *           state and the offset separately, which that sum works out to, gives an O(h^(n+1))
 *           start where the midpoints alone give O(h^n); those steps then usually take one
 *           evaluation.  With the difference form of W_{n+1} (ze_set_update_form 1) the second
 *           step too starts from F_0 + 2 (W_1 - W_0) - h D_0, D_0 = P_0 W_0 - W_0 P_0 the slope
 *           at W_0 (kept from the first step's first evaluation, whose W_{n+1} is W_0 + h D_0):
 *           O(h^3) against the linear start's O(h^2).  Selecting it also allocates 3 N x N
 *           complex buffers: two hold the run's first states (the steps' outputs rotate
 *           through them; a run that ends away from the caller's W copies back once), one
 *           W_0 + h D_0.  At order 4 or 6 it is mode 2.
 * Every mode restarts at the first step of each ze_isomp_run call.
 * Errors: ZE_EINVAL, ZE_ENOMEM.
 */
ze_status ze_set_initial_guess(ze_ctx* ctx, int mode);

/*
 * ze_set_order -- order of ze_isomp_step / ze_isomp_run: 2 (default) is the midpoint map of
 * eq. (isomp); 4 and 6 are its symmetric compositions.  Sec. 2 obtains the midpoint map as the
 * simplest member of a family of isospectral integrators reduced from symplectic Runge--Kutta
 * methods and names higher orders without giving them; the members built here compose the
 * midpoint map with itself, which keeps every property the map has (isospectral, Lie--Poisson,
 * symmetric) and raises the order by Yoshida's triple jump (Phys. Lett. A 150, 1990): substeps
 * g1 h, g2 h, g1 h with g1 = 1 / (2 - 2^(1/(p+1))), g2 = 1 - 2 g1 take an order p to p + 2.
 * Order 4 is 3 midpoint substeps per step (g2 < 0), order 6 the triple jump applied twice
 * (9 substeps).  With ze_set_initial_guess mode 1 every substep after the first of a call
 * starts from W + rho (W - F_prev), rho the ratio of its step to the previous substep's (also
 * inside a single ze_isomp_step); with mode 2 see ze_set_initial_guess.  The ensemble entry
 * points always step at order 2.
 * Errors: ZE_EINVAL for any other order, ZE_ENOMEM (mode 2's buffers for more substeps).
 */
ze_status ze_set_order(ze_ctx* ctx, int order);

/*
 * ze_set_update_form -- how W_{n+1} is formed from the last evaluation's products.
 *   form 0  (default) the second line of eq. (isomp) at the last iterate W~:
 *           W~ + h/2 (A - A^H) - h^2/4 Q.
 *   form 1  W_n + h (A - A^H): the two lines of eq. (isomp) differ by exactly h [P~, W~], so
 *           both forms agree at the fixed point.  At a stopped iterate (residual r), form 0 is
 *           a unitary conjugate of W_n - (F - W~), with eigenvalues off by O(r); form 1 differs
 *           from it by F - W~ itself, with eigenvalues off by only O(h ||P~|| r).  With
 *           ze_set_initial_guess 2 a step then takes one evaluation after the start-up,
 *           against about 1.5 with form 0, whose O(r) trajectory kinks the extrapolation
 *           amplifies.
 * Errors: ZE_EINVAL.
 */
ze_status ze_set_update_form(ze_ctx* ctx, int form);

/*
 * ze_set_validation -- input check of ze_isomp_step and ze_isomp_run (off by default: the
 * inputs are assumed to lie in su(N), the phase space of eq. (Euler_vort_mat)).  With on = 1
 * each call first checks its W on the GPU, max |W_rc + conj(W_cr)| <= 1e-12 max |W_rc| and
 * |tr W| <= 1e-12 N max |W_rc|, and returns ZE_EINVAL, with the measured values in
 * ze_last_error, when W fails (or holds a NaN or Inf); W is then left unchanged.  The check
 * reads W once and synchronises the stream.
 * Errors: ZE_EINVAL (on not 0 or 1).
 */
ze_status ze_set_validation(ze_ctx* ctx, int on);

/*
 * ze_casimirs -- C_k(W) = Tr(W^k), k = 1..kmax (eq. (W_pow)), in FP64, from powers of W
 * formed with the library's FP64 products: C_{a+b} = sum_ij (W^a)_ij (W^b)_ji.
 *   W     device, N x N complex128 (any matrix; all of it is read).
 *   kmax  1 <= kmax <= 64.
 *   out   host, 2*kmax doubles: (re, im) of C_1..C_kmax.
 * Errors: ZE_EINVAL, ZE_ENOMEM, ZE_EHIP.  Synchronous.
 */
ze_status ze_casimirs(ze_ctx* ctx, const void* W, int kmax, double* out);

/*
 * ze_basis_assemble -- W = sum_{l,m} i omega_lm T_lm (eq. (W0)), the T_lm being the unit
 * eigenvectors of Delta^m for the eigenvalue l(l+1) (eq. (lap_prop)) placed on diagonal m
 * (Sec. 3.2), with T_{l,-m} = (-1)^m T_lm^H.  Eigenvector signs (the paper leaves them
 * open): among the entries with index 0..floor((N-m-1)/2) whose magnitude is within a
 * relative 1e-8 of the largest there, the one with the lowest index is positive.
 *   omega  device, N*N complex128 coefficients, omega_lm at index l*l + l + m.
 *   W      device, N x N complex128, fully written.
 * Allocates a scratch buffer for the eigenvectors (up to 4 GiB, freed before returning).
 * Errors: ZE_EINVAL, ZE_ENOMEM, ZE_EHIP.  Synchronous (waits for the context's stream).
 */
ze_status ze_basis_assemble(ze_ctx* ctx, const void* omega, void* W);

/*
 * ze_basis_extract -- the coefficients of W in the same basis (the post-processing of
 * Sec. 3.2): omega_lm = -i <T_lm, W>_F for every l = 0..N-1, |m| <= l, i.e.
 *   omega_lm     = -i sum_i v^{lm}_i W[i+m][i]              (m >= 0, lower diagonal m),
 *   omega_{l,-m} = -i (-1)^m sum_i v^{lm}_i W[i][i+m]       (m > 0, upper diagonal m),
 * with v^{lm} the eigenvectors of ze_basis_assemble.  Inverse of ze_basis_assemble; for W in
 * su(N) the result satisfies omega_{l,-m} = (-1)^m conj(omega_lm) and omega_00 = 0 to rounding.
 *   W      device, N x N complex128.
 *   omega  device, N*N complex128, fully written (index l*l + l + m).
 * Allocates scratch like ze_basis_assemble.  Errors: ZE_EINVAL, ZE_ENOMEM, ZE_EHIP.
 * Synchronous.
 */
ze_status ze_basis_extract(ze_ctx* ctx, const void* W, void* omega);

/*
 * ze_energy_spectrum -- kinetic energy per degree of the coefficients omega (the spectrum of
 * Sec. 4): E_l = sum_{m=-l..l} |omega_lm|^2 / (l (l+1)) for l = 1..N-1 (the stream function's
 * coefficients are -omega_lm / (l (l+1)), eq. (lap_prop)); E_0 = 0.  Sum_l l (l+1) E_l =
 * ||W||_F^2 for W = ze_basis_assemble(omega) with omega_00 = 0.
 *   omega  device, N*N complex128 (index l*l + l + m).
 *   E      device, N doubles, fully written.
 * Errors: ZE_EINVAL, ZE_EHIP.  Asynchronous.
 */
ze_status ze_energy_spectrum(ze_ctx* ctx, const void* omega, void* E);

/*
 * ze_zgemm -- C = A B for N x N complex128 matrices with the library's product kernels
 * (the GEMM of Sec. 3.1 on its own; for tests and timing).
 *   A, B, C  device, N x N complex128; C must not alias A or B.
 *   prec     ZE_PREC_FP64 or ZE_PREC_SPLIT.
 * Errors: ZE_EINVAL, ZE_EHIP.  Asynchronous.
 */
ze_status ze_zgemm(ze_ctx* ctx, const void* A, const void* B, void* C, int prec);

/*
 * ze_zgemm_noalloc -- C = A B in FP64 (the ze_zgemm product with ZE_PREC_FP64) for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It takes no context and calls no hipMalloc, hipFree or allocating
 * library routine; the split-K partial sums of the product live in a fixed 32 MiB device array
 * of the library, one per GPU, held until the process ends (the split adapts to that size, so
 * every N in range fits; results equal ze_zgemm's up to the rounding of a different K split).
 *   N        1 <= N <= 16384; larger or smaller N is refused with ZE_EINVAL (ze_last_error
 *            names the limit).
 *   A, B, C  device, N x N complex128, row-major; C must not alias A or B.  Caller-owned.
 *   stream   HIP stream of the current device (NULL: the null stream); a stream of another
 *            device is refused with ZE_EINVAL.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams or host threads) race and must be ordered by the caller.  The first call on a device
 * looks the array's address up on that device (it synchronises nothing).
 * Errors: ZE_EINVAL, ZE_EHIP.  Asynchronous on `stream`.
 */
ze_status ze_zgemm_noalloc(int N, const void* A, const void* B, void* C, void* stream);

/*
 * ze_set_split_slices -- number s of slices per operand of the ZE_PREC_SPLIT products (balanced
 * digits: a 7-bit top slice, then 8-bit ones); the products then cost s (s + 1) / 2 INT8
 * products each.  Allowed: 2 <= s <= s_max(N) with
 * s_max(N) = min(8, floor((2^31 - 1) / (2 N 128^2))), the largest count whose int32 sums stay
 * exact (8 up to N = 4096, 7 at N = 8192, 3 at N = 16384); default min(5, s_max(N)).  The
 * first split-precision call of a context allocates its slice buffers (about 24 N^2 bytes)
 * and int32 work slabs (up to 64 N^2 bytes).  s applies to the product A = P W~; the lower
 * product Q = A P takes max(2, s - 1) slices (see ze_set_split_slices_lower).
 * Errors: ZE_EINVAL (also for s > s_max(N)).
 */
ze_status ze_set_split_slices(ze_ctx* ctx, int slices);

/*
 * ze_set_split_slices_lower -- slices s_q (2 <= s_q <= s) of the lower product Q = A P in the
 * ZE_PREC_SPLIT step.  In the fixed-point map (eq. (isomp_iter)) Q enters F with h^2/4 and A
 * with h/2, so at equal relative accuracy Q's rounding weighs about h ||P||_2 / 2 as much as
 * A's.  One slice fewer (the default, s - 1) multiplies Q's relative error by 256 and keeps
 * its share at most 128 |h| ||P||_2 of A's (0.32 at h = 0.005 for ||W||_2 = 1, since
 * ||P||_2 <= ||W||_2 / 2); for steps with |h| ||P||_2 above ~1/128 set s_q = s.  Reset to
 * s - 1 by ze_set_split_slices.
 * Errors: ZE_EINVAL.
 */
ze_status ze_set_split_slices_lower(ze_ctx* ctx, int slices);

/*
 * ze_profile -- per-phase timing of ze_isomp_step, for measurement.  While on, every
 * evaluation records HIP events on the context's stream around its four phases and adds
 * their elapsed times (read back at the evaluation's convergence test, so no extra
 * synchronisation).  Phases: 0 stream solve, 1 product A = P W~, 2 lower product Q = A P
 * with the fixed-point epilogue, 3 residual reduction.
 * Errors: ZE_EINVAL, ZE_EHIP (event creation).  Synchronous.
 */
ze_status ze_profile(ze_ctx* ctx, int on);

/*
 * ze_profile_read -- accumulated milliseconds (ms[4]) and launch counts (launches[4]) per
 * phase since the last reset; both host arrays, either may be NULL.  reset != 0 clears them.
 */
ze_status ze_profile_read(ze_ctx* ctx, double* ms, long long* launches, int reset);

/*
 * Ensembles: nsim independent simulations of (possibly different) sizes N_j stepped together,
 * for statistics over many initial conditions.  Each phase of a fixed-point evaluation is one
 * grouped launch over all simulations' tiles, and a step's launches are captured once into a
 * HIP graph that is replayed (one graph launch per step) on a private default-priority stream
 * ordered after / before the caller's stream with events.  Per-simulation device flags keep the
 * stopping rule of ze_isomp_step: a simulation stops at its first evaluation whose residual is
 * below tol (or at K = maxit), without host synchronisation.  The first run of an ensemble in
 * each precision times the candidate tile shapes / work orders on copies of the inputs and
 * keeps the fastest.
 *
 * ze_ensemble_create -- set up nsim simulations of sizes N[0..nsim-1] (host array,
 *   1 <= N_j <= 4096, nsim <= 4096); stream: the caller's hipStream_t (NULL = default).
 *   Errors: ZE_EINVAL, ZE_ENOMEM, ZE_EHIP.  Synchronous.
 */
ze_status ze_ensemble_create(int nsim, const int* N, void* stream, ze_ens** out);

/* Free an ensemble (synchronises).  NULL is accepted. */
ze_status ze_ensemble_destroy(ze_ens* ens);

/*
 * ze_ensemble_run -- nsteps IsoMP steps of every simulation (eqs. (isomp), (isomp_iter)).
 *   W      host array of nsim device pointers, W[j] an N_j x N_j complex128 skew-Hermitian
 *          matrix (in: W_n, out: W_{n+nsteps}); the pointers may change between calls.
 *   h, tol as in ze_isomp_step; K = maxit (1..64); prec: ZE_PREC_FP64, or ZE_PREC_SPLIT
 *   (both products of every evaluation on INT8 MFMA with ze_ensemble_set_split_slices
 *   slices; the first split run allocates its workspaces, synchronously).
 * Asynchronous on the caller's stream; ze_ensemble_stats reads the outcome of the last step.
 * Errors: ZE_EINVAL, ZE_ENOMEM, ZE_EHIP.
 */
ze_status ze_ensemble_run(ze_ens* ens, void* const* W, double h, double tol, int K, int nsteps,
                          int prec);

/* One step: ze_ensemble_run with nsteps = 1. */
ze_status ze_ensemble_step(ze_ens* ens, void* const* W, double h, double tol, int K, int prec);

/*
 * ze_ensemble_stats -- evaluations done (iters[j]) and final residual (resid[j]) of every
 * simulation in the last step; host arrays of nsim entries, either may be NULL.  Synchronous.
 */
ze_status ze_ensemble_stats(ze_ens* ens, int* iters, double* resid);

/*
 * ze_ensemble_tuning -- the autotuner's choice for precision prec (-1 before the first run in
 * it) and the measured milliseconds per step of its candidates (host ms[4]).  ZE_PREC_FP64:
 * choice 0..3 = 2 * tile shape (0: 128 x 64, 1: 64 x 64 complex) + work order (0: largest
 * simulations first, 1: interleaved); ZE_PREC_SPLIT: choice 0..1 = work order, ms[2..3] = 0.
 */
ze_status ze_ensemble_tuning(ze_ens* ens, int prec, int* choice, double* ms);

/*
 * ze_ensemble_set_split_slices -- slices s of the ensemble's ZE_PREC_SPLIT products
 * (2 <= s <= s_max of the largest N_j, default 5; see ze_set_split_slices; the lower product
 * takes max(2, s - 1)).  Takes effect at the next ze_ensemble_run.
 */
ze_status ze_ensemble_set_split_slices(ze_ens* ens, int slices);

/*
 * ze_ensemble_set_split_slices_lower -- slices of the ensemble's lower products Q = A P
 * (2 <= s_q <= s; see ze_set_split_slices_lower).  Takes effect at the next ze_ensemble_run.
 * Errors: ZE_EINVAL.
 */
ze_status ze_ensemble_set_split_slices_lower(ze_ens* ens, int slices);

/*
 * ze_ensemble_set_update_form -- form of W_{n+1} for the ensemble's steps (0 default, 1; see
 * ze_set_update_form).  Takes effect at the next ze_ensemble_run.
 * Errors: ZE_EINVAL.
 */
ze_status ze_ensemble_set_update_form(ze_ens* ens, int form);

/*
 * ze_ensemble_set_initial_guess -- first iterate of the fixed-point map (eq. (isomp_iter)) for
 * the ensemble's steps, as ze_set_initial_guess for one simulation: 0 (default) W_n at every
 * step; 1: in ze_ensemble_run, every step after the first of the call starts each simulation
 * from 2 W_n - F_prev (its previous step's converged midpoint), which saves about one
 * evaluation per step at the same stopping rule; 2: the polynomial start of
 * ze_set_initial_guess mode 2 per simulation (linear at the second step of the call, then
 * degrees 1, 2, 3 through its previous midpoints), one evaluation per step after the
 * start-up; one captured graph reads the step's index in the call from device memory; 3: as
 * ze_set_initial_guess mode 3 per simulation (the third and fourth steps with the run's states,
 * with the difference form the second with the slope at W_0; the first states rotate through
 * two more buffers per simulation, the rotation done on the device at each step's end).
 * Selecting mode 2 allocates three N_j x N_j complex buffers per simulation, mode 3 three more.
 * Takes effect at the next ze_ensemble_run (the step graphs are captured again).
 * Errors: ZE_EINVAL (mode not 0 .. 3), ZE_ENOMEM.
 */
ze_status ze_ensemble_set_initial_guess(ze_ens* ens, int mode);

/*
 * ze_ensemble_set_steady_cap -- evaluation cap of the steps with index >= from_step in a
 * ze_ensemble_run call, with the polynomial start (mode 2 of ze_ensemble_set_initial_guess):
 * min(K, cap) instead of K, captured as a second step graph (cap 0, the default: K for every
 * step).  Once the polynomial start has reached degree 3 (from the fifth step of a call) a step
 * needs one evaluation at these workloads, and every capped evaluation a step does not need
 * still costs its launches (they return at once), so a small cap saves them; a step that would
 * need more stops at the cap with its residual reported by ze_ensemble_stats (the fixed-count
 * mode of Sec. 3.4).  Takes effect at the next ze_ensemble_run.  Errors: ZE_EINVAL.
 */
ze_status ze_ensemble_set_steady_cap(ze_ens* ens, int cap, int from_step);

/*
 * ze_ensemble_set_continuation -- as ze_set_continuation for the ensemble: with 1, a
 * ze_ensemble_run (or ze_ensemble_step) on the same nsim device pointers, holding the last
 * run's results unchanged, with the same h, precision, start mode and update form, continues
 * that run's trajectories (the step index on the device and every simulation's history of
 * midpoints) instead of starting at step 0; a start-mode, update-form or slice setter in
 * between, the autotuner's first run in a precision, or with guess mode 3 a trajectory of
 * fewer than 4 steps so far, starts over.  0 (the default): every call starts at step 0.
 * Errors: ZE_EINVAL.
 */
ze_status ze_ensemble_set_continuation(ze_ens* ens, int on);

#ifdef __cplusplus
}
#endif

#endif /* ZEULER_H */

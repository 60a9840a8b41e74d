// Internal declarations of libzeuler: the context layout and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "zeuler.h"

// Records a HIP failure (message kept per thread for ze_last_error) and returns ZE_EHIP.
ze_status ze_record_hip(hipError_t e, const char* what);

#define ZE_HIP(call)                                         \
    do {                                                     \
        hipError_t ze_e_ = (call);                           \
        if (ze_e_ != hipSuccess) return ze_record_hip(ze_e_, #call); \
    } while (0)

#define ZE_TRY(call)                                         \
    do {                                                     \
        ze_status ze_s_ = (call);                            \
        if (ze_s_ != ZE_OK) return ze_s_;                    \
    } while (0)

// Offset of entry (r, c), c <= r, in a packed row-major lower triangle.
__host__ __device__ inline size_t tri_off(size_t r, size_t c) { return r * (r + 1) / 2 + c; }

struct ze_ctx {
    int N = 0;
    int device = 0;
    hipStream_t stream = nullptr;

    // LDL^T factors of every Delta^m in the stream solve's workgroup order (diagonal m = 0
    // first, then the pairs (m, N-m), m = 1..N/2, each at offset m*N): per element, the
    // multiplier met when the forward sweep reaches it (0 at the first element of each
    // diagonal) and 1/D (0 for the excluded last element of the singular m = 0 block).
    int solve_bd = 4;  // lanes per band of the stream solve (factor layout, launch shape)
    double* fac_l = nullptr;
    double* fac_dinv = nullptr;

    // Step workspaces, N x N complex each.
    double2* Wn = nullptr;   // second state buffer: a run's steps alternate between it and W
    double2* F = nullptr;    // fixed-point iterate W~ (after the first evaluation)
    double2* P = nullptr;    // stream matrix
    double2* A = nullptr;    // A = P W~
    double2* Q = nullptr;    // lower product Q = A P (FP64 path)
    int ut = 64;                // tile of the fixed-point update (update_tile_of(N))
    double* rowpart = nullptr;  // ceil(N / ut) x N partial row sums of |F - W~|
    double* blockmax = nullptr; // per-block maxima of the row sums
    double* resid = nullptr;    // device scalar: infinity norm of F - W~
    double* host_resid = nullptr;      // pinned, mapped host word of the residual
    double* host_resid_dev = nullptr;  // its device address

    // Products: concurrent-block capacities and the split-K partial buffer.
    int cap_full = 0, cap_low = 0, cus = 0;
    double* gemm_part = nullptr;
    int* low_order = nullptr;  // lower-product tiles in 8 x 8 super-tile order

    // Split-precision products (allocated on first use): slice count s, INT8 slices of the
    // A~ and B~^T operands (kSplitMax slices each, rows of ze_split_ldk(N) bytes), their scale
    // exponents, column-maximum partials, and the int32 product slabs.
    int split_slices = 5;
    // Slices of the lower product Q = A P, whose term enters F with h^2/4 against h/2 for A:
    // one slice fewer by default (ze_set_split_slices), or as ze_set_split_slices_lower sets.
    int split_slices_low = 4;
    signed char* split_a = nullptr;
    signed char* split_b = nullptr;
    int* split_ea = nullptr;
    int* split_eb = nullptr;
    int* split_ec = nullptr;  // row exponents of A in the lower product Q = A P
    double* split_colmax = nullptr;
    int* split_g = nullptr;  // int32 slabs G[t-2], N x 2N each, t = 2..s+1
    int cap_i8 = 0;          // blocks of the INT8 product kernel that fit on the device at once
    int cap_i8l = 0;         // the same for the 256 x 256 residue-product kernel
    // Modular (CRT) form of the product A = P W~: residues of A~ and B~^T for 16 moduli (split
    // layouts) and the 16 int32 residue products, N x 2N each; allocated on first use.
    signed char* crt_a = nullptr;
    signed char* crt_b = nullptr;
    int* crt_g = nullptr;

    // Starting iterate of the steps after the first in ze_isomp_run: 0 = W_n, 1 = 2 W_n - F
    // (F = the previous step's converged midpoint, left in ze_ctx::F), 2 = the polynomial
    // extrapolation of the last (up to 4) midpoints of the run, 3 = as 2, and at order 2 the
    // starts of steps 2 and 3 add the n-th backward difference of the run's states.
    int guess_mode = 0;
    // Midpoint history of mode 2: a ring of 4 buffers per substep of a step, ring[4 j + i]
    // (ring[0] is the allocation F starts with; the others are allocated on first use); the
    // newest midpoint of substep j is ring[4 j + rhead[j]].
    std::vector<double2*> ring;
    std::vector<int> rhead;
    // Guess mode 3 at order 2: two more state buffers, so that the states W_0 .. W_3 of a run's
    // first steps stay in memory until the start of step 3 (allocated with the mode).
    double2* Wh[2] = {nullptr, nullptr};
    // ... and with the difference form of W_{n+1}, the first evaluation's W_{n+1} of a run's
    // first step, W_0 + h (P_0 W_0 - W_0 P_0), for the second step's start (allocated with the
    // mode); save_first points at it while that step is enqueued, else null.
    double2* Wd = nullptr;
    double2* save_first = nullptr;
    // Order of the time step (2: the midpoint map; 4, 6: its symmetric compositions) and the
    // substep fractions c_j of one step.
    int order = 2;
    std::vector<double> comp_w{1.0};
    // Form of W_{n+1}: 0 the second line of eq. (isomp) at the last iterate, 1 W_n + h [P~, W~].
    int update_form = 0;
    // Input check of ze_isomp_step / ze_isomp_run (ze_set_validation) and its buffers.
    bool validate = false;
    double* val_part = nullptr;

    // Stopping rule (ze_set_stopping): 0 = the host reads the residual after each evaluation;
    // 1 = on the device: every evaluation up to maxit is enqueued, its kernels skip themselves
    // once the step's done flag is set, and nothing waits for the host.  Control words dctl
    // (kCtlWords ints, always allocated; dctl[kCtlCounter] is the residual reduction's block
    // counter) and dctld (2 doubles); per-step records of the last run (kDevSteps each,
    // allocated with mode 1).
    int stop_mode = 0;
    // Evaluation cap min(maxit, cap2) of the steps with index >= cap2_after in a run (cap2 0:
    // maxit for every step; ze_set_steady_cap).
    int cap2 = 0, cap2_after = 0;
    // Continuation (ze_set_continuation): with cont on, the step index cont_n the next run
    // starts from when it continues the last successful run (same W pointer, h, precision,
    // starting-iterate mode, order and update form); cont_n < 0: no run to continue.
    int cont = 0, cont_n = -1;
    const void* cont_w = nullptr;
    double cont_h = 0.0;
    int cont_prec = -1, cont_guess = -1, cont_form = -1;
    size_t cont_ns = 0;
    int* dctl = nullptr;
    double* dctld = nullptr;
    int* dstep_it = nullptr;
    double* dstep_r = nullptr;
    int last_run_steps = 0;
    // Done flag read by the split and modular products' kernels while a substep with on-device
    // stopping is being enqueued (dctl then, else null: they always run).
    const int* skip = nullptr;

    // Optional per-phase timing (ze_profile).
    bool prof = false;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double prof_ms[4] = {0, 0, 0, 0};
    long long prof_n[4] = {0, 0, 0, 0};
};

// Control words of on-device stopping: [0] done flag of the current substep, [1] its
// evaluations, [2] evaluations of the current step, [3] the step's flags (1: not converged,
// 2: non-finite residual), [4] steps of the run not converged, [5] steps with a non-finite
// residual, [6] evaluations of the run, [7] most evaluations of one step, [kCtlCounter] the
// residual reduction's block counter, [9] index of the current step in the run.  dctld:
// [0] the step's largest residual, [1] the run's.
constexpr int kCtlWords = 16;
constexpr int kCtlCounter = 8;
// Per-step records kept by on-device stopping (step n of a run at n % kDevSteps).
constexpr int kDevSteps = 1 << 16;

// Largest matrix size a context accepts.
constexpr int kMaxN = 16384;
// Largest number of slices of the split-precision products.
constexpr int kSplitMax = 8;
// Number of moduli of the modular (CRT) form of the product.
constexpr int kCrtMods = 16;

// Largest slice count whose int32 sums stay exact for size N: the stored digits lie in
// [-128, 127], so the pairs of one order t = i + j (at most s of them) add up to at most
// s * 2N * 128^2 in magnitude, which must stay below 2^31 (8 up to N = 4096, 7 at 8192,
// 3 at 16384).
inline int split_max_slices(int N) {
    const long long per = 2LL * N * 128 * 128;
    const long long m = ((1LL << 31) - 1) / per;
    return (int)(m < kSplitMax ? m : kSplitMax);
}

// Workspaces of the split-precision products (kSplitMax slices), allocated on first use.
ze_status ze_ensure_split(ze_ctx* c);
// Blocks of the single-problem INT8 product kernel that fit on the device at once.
hipError_t ze_i8_capacity(int* cap, int* cap_large);

// Slice buffers hold whole 128-row tiles: A~ slices have split_rows_pad(N) rows and B~^T
// slices split_cols_pad(N) rows; the rows past N (2N) are zeroed when the buffers are
// allocated and never written, so the INT8 product reads them without bounds checks.
__host__ __device__ inline int split_rows_pad(int N) { return ((N + 127) / 128) * 128; }
__host__ __device__ inline int split_cols_pad(int N) { return ((2 * N + 127) / 128) * 128; }
// Rows of the residue slabs of A~ and of B~^T (the modular form), padded to its 256-row tiles.
__host__ __device__ inline int crt_rows_pad(int N) { return ((N + 255) / 256) * 256; }

// ze_create without (split_k = false) the split-K partial buffer of the single-problem products.
// solve_bd: stream-solve band width (1, 2 or 4), 0 = the default for N (solve_bd(N)).
ze_status ze_create_ctx(int N, void* stream, bool split_k, int solve_bd, ze_ctx** out);

// Host: the factors held in ze_ctx::fac_l / fac_dinv (about N^2 / 2 entries each, in the
// band order of the stream solve).
void ze_build_factors(int N, int bd, std::vector<double>& fl, std::vector<double>& fd);

// ---- kernel launchers (all asynchronous on `s`) ----

// Stream solve P = Delta_N^+ W (both N x N, row-major, leading dimension N); skip as for the
// products.
hipError_t launch_stream_solve(const ze_ctx* c, const double2* W, double2* P, hipStream_t s,
                               const int* skip = nullptr);

// Blocks of the two product kernels that fit on the device at once, and the bytes of the
// split-K partial buffer (ze_ctx::gemm_part) those capacities need.
hipError_t ze_gemm_capacity(int* cap_full, int* cap_low, int* cus);
size_t ze_gemm_part_bytes(int cap_full, int cap_low);
// Lower-triangle tile indices (64 x 64 complex tiles) in 8 x 8 super-tile order.
void ze_lower_tile_order(int N, std::vector<int>& order);

// C = A B, all N x N complex (leading dimension N = c->N), FP64 MFMA.  skip: a device flag
// read at the start of every block (on-device stopping); nonzero there makes the launch a no-op.
hipError_t launch_zgemm_f64(const ze_ctx* c, const double2* A, const double2* B, double2* C,
                            hipStream_t s, const int* skip = nullptr);

// The same product with its split-K partial sums in the library's fixed device array (no
// allocation; ze_zgemm_noalloc): N x N, on the current device, asynchronous on `s`.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
hipError_t launch_zgemm_f64_noalloc(int N, const double2* A, const double2* B, double2* C,
                                    hipStream_t s);

// Lower-triangle Q = A P (64 x 64 complex tiles meeting the lower triangle) into Q.
hipError_t launch_zgemm_lower(const ze_ctx* c, const double2* A, const double2* P, double2* Q,
                              hipStream_t s, const int* skip = nullptr);

// resid = max_r sum_{X < T} rowpart[X*N + r]  (NaN propagates), one launch (counter: a zeroed device
// word the launch leaves zeroed), also stored to host_out (device address of mapped host
// memory) if given.  With ctl: ctl[1] += 1 and ctl[0] = 1 once resid < tol or is
// not finite; skip as for the products.
hipError_t launch_resid_reduce(const double* rowpart, int T, double* blockmax, unsigned* counter,
                               double* resid, int N, hipStream_t s, const int* skip = nullptr,
                               int* ctl = nullptr, double tol = 0.0, double* host_out = nullptr);

// out[0] = sum_ij X_ij Y_ji (complex), through `partial` (>= ze_trace_partials(N) doubles2).
int ze_trace_partials(int N);
hipError_t launch_trace_product(const double2* X, const double2* Y, double2* partial,
                                double2* out, int N, hipStream_t s);
// out[0] = sum_i X_ii.
hipError_t launch_trace(const double2* X, double2* partial, double2* out, int N, hipStream_t s);

// W = sum_lm i omega_lm T_lm; scratch as returned by ze_basis_scratch_bytes(N).
size_t ze_basis_scratch_bytes(int N);
hipError_t launch_basis_assemble(const double2* omega, double2* W, void* scratch, int N,
                                 hipStream_t s);
// omega_lm = -i <T_lm, W> for every (l, m) (the inverse of launch_basis_assemble on su(N)).
hipError_t launch_basis_extract(const double2* W, double2* omega, void* scratch, int N,
                                hipStream_t s);
// E_l = sum_m |omega_lm|^2 / (l (l + 1)), l = 0..N-1 (E_0 = 0).
hipError_t launch_energy_spectrum(const double2* omega, double* E, int N, hipStream_t s);

// ---- split-precision products (INT8 MFMA, Ozaki splitting) ----
int ze_split_ldk(int N);  // bytes per slice row: 2N rounded up to the K stage
// Slices A (rows; exponents into ea) and B (columns) into the context's buffers.  The column
// exponents of B are computed into eb, or, with eb_known, read from eb (a skew-Hermitian B whose
// row exponents are known: they are its column exponents).  lower selects the slice count of
// the lower product.
hipError_t launch_split_prepare(const ze_ctx* c, const double2* A, const double2* B, int* ea,
                                int* eb, bool eb_known, int lower, hipStream_t s);
// C = A B (lower != 0: only the tiles meeting the lower triangle are formed, and left in the
// int32 slabs for launch_lower_update); ea, eb, eb_known as for launch_split_prepare.
hipError_t launch_zgemm_split(const ze_ctx* c, const double2* A, const double2* B, double2* C,
                              int lower, int* ea, int* eb, bool eb_known, hipStream_t s);
// The fixed-point update from the lower product:
//   F     = Wn + h/2 (A - A^H) + h^2/4 Q       (both triangles; may alias Wt)
//   Wout  = Wt + h/2 (A - A^H) - h^2/4 Q       (both triangles)
//   rowpart[X*N + r]  partial row sums of |F - Wt| (slot layout in update_tile.h)
// with Q read from Q (FP64, lower tiles) or, if Q is null, from the int32 slabs of the
// preceding split lower product with its row and column exponents ea, eb.
hipError_t launch_lower_update(const ze_ctx* c, const double2* Q, const double2* A,
                               const double2* Wn, const double2* Wt, double2* F, double2* Wout,
                               double* rowpart, double h, const int* ea, const int* eb,
                               hipStream_t s, const int* skip = nullptr);

// On-device stopping: start of a run (clears the run's totals and the first step's fields);
// end of a substep (its count and residual into the step's, then its done flag and count
// cleared; last: the step's record written at its index, run totals, the step's fields
// cleared).
hipError_t launch_ctl_run_begin(int* ctl, double* ctld, hipStream_t s);
hipError_t launch_ctl_substep_end(int* ctl, double* ctld, const double* resid, double tol, bool last,
                                  int* step_it, double* step_r, hipStream_t s);

// F <- 2 W - F (N x N complex).
hipError_t launch_extrapolate(const double2* W, double2* F, int N, double rho, hipStream_t s);
// out <- sum_i coef[i] src[i] (i = 0 .. m-1, in that order), N x N complex, m <= kLinCombMax.
constexpr int kLinCombMax = 8;
hipError_t launch_lincomb(const double2* const* src, const double* coef, int m, double2* out, int N,
                          hipStream_t s);
// dst <- src, N x N complex (a kernel, so a captured graph holds no copy node).
hipError_t launch_copy(const double2* src, double2* dst, int N, hipStream_t s);
// out = polynomial extrapolation of degree d (1..3) through Fs[0] (newest) .. Fs[d], one step
// ahead; out may be Fs[d].
hipError_t launch_extrapolate_poly(const double2* const* Fs, int d, double2* out, int N,
                                   hipStream_t s);
// Modular form: bits of the scaled integers for size N, int32 count of the residue products,
// the product C = A B (full), and the context's buffers for it.
int ze_crt_bits(int N);
size_t ze_crt_slab_ints(int N);
int ze_crt_ldk(int N);
void ze_crt_plan(int N, int cap_blocks, int* ntiles, int* tn, int* G);
hipError_t launch_zgemm_crt(const ze_ctx* c, const double2* A, const double2* B, double2* C,
                            hipStream_t s);
ze_status ze_ensure_crt(ze_ctx* c);
// Grows the context's midpoint rings to 4 buffers for each of ns substeps.
ze_status ze_ensure_rings(ze_ctx* c, int ns);
// Input check of W (ze_set_validation): out[0..3] = max |W + W^H|, max |W|, Re tr W, Im tr W;
// part holds 4 doubles per block of ze_su_check_blocks(N).
int ze_su_check_blocks(int N);
hipError_t launch_su_check(const double2* W, int N, double* part, double* out, hipStream_t s);

// Ensembles of independent IsoMP simulations of uneven N (statistics over many initial
// conditions): the step's starting iterate and every phase of a fixed-point evaluation --
// stream solve, A = P W~, lower Q = A P, the update, residual -- run as ONE grouped launch each
// over a work list of (simulation, tile) items, and the 1 + 5K launches of a step are captured
// once into a HIP graph and replayed, one graph launch per step.
//
// Convergence stays tolerance-driven without host round trips: per-simulation device flags
// `done` are cleared at the start of a step and set by the residual kernel once the change of
// W~ is below tol; every later block of that simulation exits at once, so its W keeps the
// W_{n+1} of the converged evaluation (the same result as ze_isomp_step with maxit = K).
//
// Autotuning: the product A = P W~ has two tile shapes (128 x 64 and 64 x 64 complex) and the
// work lists two orders (largest problems first, or simulations interleaved); the first step
// times the four graphs on copies of the inputs and keeps the fastest.

#include <algorithm>
#include <cmath>
#include <vector>

#include "solve_wg.h"
#include "split_tile.h"
#include "tile_f64.h"
#include "update_tile.h"

namespace {

using namespace zk;

struct EnsProb {
    int N;
    int pad;
    // W_n of the step and where its W_{n+1} goes: the caller's matrix Wc and the scratch
    // matrix X take turns (set at the start of a run; swapped at the end of each step, so no
    // step copies W_n; the run's last W_{n+1} is copied to Wc if it ended in X)
    double2* W;
    double2* Wn;
    double2* Wc;
    double2* X;
    double2* F;
    double2* P;
    double2* A;
    double2* Q;
    double* rowpart;
    const double* fl;
    const double* fd;
    // split-precision products: slices, int32 slabs, exponents (rows of P, columns of W~,
    // rows of A); null until the first split run
    signed char* sa;
    signed char* sb;
    int* G;
    int* ep;
    int* ew;
    int* eA;
    // earlier midpoints of the run for starting-iterate mode 2 (F_{n-2}, F_{n-3}, F_{n-4});
    // null until that mode is selected
    double2* H1;
    double2* H2;
    double2* H3;
    // guess mode 3: two more state buffers (the first steps' outputs rotate through X, S1, S2
    // and Wc, so W_0 .. W_3 are in memory at the start of step 3) and the first step's first
    // output W_0 + h D_0 (difference form); null until that mode is selected
    double2* S1;
    double2* S2;
    double2* Wd;
};

// blocks per simulation of the whole-matrix copies (the first evaluation's output, the run's last
// state)
constexpr int kCopyParts = 64;

// Start of a step: the first iterate F (W_n is read where the previous step left it, Wn).
// mode 0: F <- W_n; mode 1: F <- 2 W_n - F,
// the linear extrapolation of the previous step's converged midpoint (still in F); mode 2: by
// the step's index n in the run (*stepc): W_n at n = 0, 2 W_n - H1 at n = 1, else the
// polynomial of degree d = min(n - 1, 3) through the midpoints H1 (newest), H2, H3 and F (the
// oldest, overwritten in place) one step ahead (coefficients (2, -1), (3, -3, 1),
// (4, -6, 4, -1), summed in that order).  In mode 2 the four buffers form a ring: at the end
// of each step ens_stepc_kernel turns the descriptors (F, H1, H2, H3) <- (H3, F, H1, H2), so
// the midpoint just written to F becomes H1 and the oldest slot becomes the next F; entries
// not yet written in this run are never read.
// Every evaluation then reads its iterate from F (the update rewrites it in place: each entry
// it reads is written by the same thread, and the mirrored upper entries it writes are read by
// no other block of that launch).
// mode 3 (guess mode 3; slope: with the difference form): as mode 2, except that step 1 starts
// from F_0 + 2 W_1 - W_0 - Wd (slope; Wd = W_0 + h D_0, D_0 the slope of the states at W_0),
// step 2 from 2 H1 - H2 + W_2 - 2 W_1 + W_0 and step 3 from 3 H1 - 3 H2 + H3 + W_3 - 3 W_2 +
// 3 W_1 - W_0: the midpoint polynomial plus the backward difference of the states, which sit in
// Wc (W_0), X (W_1), S1 (W_2) and S2 (W_3) then.
// begin_value gives that starting iterate at entry e of one simulation; c1..c3 are the
// coefficients of the midpoint polynomial of degree min(n - 1, 3).
__device__ __forceinline__ double2 begin_value(const EnsProb& p, size_t e, int mode, int n, int slope,
                                               double c1, double c2, double c3) {
    if (n == 0) return p.Wn[e];
    if (mode == 3 && n == 1 && slope) {
        const double2 f = p.H1[e], w1 = p.Wn[e], w0 = p.Wc[e], wd = p.Wd[e];
        double2 g = make_double2(f.x + 2.0 * w1.x, f.y + 2.0 * w1.y);
        return make_double2(g.x - w0.x - wd.x, g.y - w0.y - wd.y);
    }
    if (mode == 3 && n == 2) {
        const double2 f1 = p.H1[e], f2 = p.H2[e];
        const double2 w2 = p.Wn[e], w1 = p.X[e], w0 = p.Wc[e];
        const double2 g = make_double2(2.0 * f1.x - f2.x, 2.0 * f1.y - f2.y);
        return make_double2(g.x + w2.x - 2.0 * w1.x + w0.x, g.y + w2.y - 2.0 * w1.y + w0.y);
    }
    if (mode == 3 && n == 3) {
        const double2 f1 = p.H1[e], f2 = p.H2[e], f3 = p.H3[e];
        const double2 w3 = p.Wn[e], w2 = p.S1[e], w1 = p.X[e], w0 = p.Wc[e];
        const double2 g = make_double2(3.0 * f1.x - 3.0 * f2.x + f3.x, 3.0 * f1.y - 3.0 * f2.y + f3.y);
        return make_double2(g.x + w3.x - 3.0 * w2.x + 3.0 * w1.x - w0.x,
                            g.y + w3.y - 3.0 * w2.y + 3.0 * w1.y - w0.y);
    }
    if (mode == 1) {
        const double2 w = p.Wn[e], f = p.F[e];
        return make_double2(2.0 * w.x - f.x, 2.0 * w.y - f.y);
    }
    if (n == 1) {
        const double2 w = p.Wn[e], f1 = p.H1[e];
        return make_double2(2.0 * w.x - f1.x, 2.0 * w.y - f1.y);
    }
    const double2 f1 = p.H1[e], f2 = p.H2[e];
    double2 g = make_double2(c1 * f1.x, c1 * f1.y);
    g = make_double2(g.x + c2 * f2.x, g.y + c2 * f2.y);
    if (n >= 3) {
        const double2 f3 = p.H3[e];
        g = make_double2(g.x + c3 * f3.x, g.y + c3 * f3.y);
        if (n >= 4) {
            const double2 f4 = p.F[e];
            g = make_double2(g.x - f4.x, g.y - f4.y);
        }
    }
    return g;
}

// Work item (simulation, chunk): entries chunk * kBeginChunk + u * 256 + thread, u = 0 .. 3, all
// read before any is written (the oldest midpoint slot may be the one written).
constexpr int kBeginChunk = 4 * 256;
__global__ __launch_bounds__(256) void ens_begin_kernel(const EnsProb* __restrict__ probs,
                                                        const int2* __restrict__ work,
                                                        int* __restrict__ done, int mode,
                                                        const int* __restrict__ stepc, int slope) {
    const int2 it = work[blockIdx.x];
    const EnsProb p = probs[it.x];
    const size_t n2 = (size_t)p.N * p.N;
    const int n = mode >= 2 ? stepc[0] : (mode == 1 ? 1 : 0);
    const int d = n - 1 < 3 ? n - 1 : 3;  // polynomial degree for n >= 2
    const double c1 = d + 1.0;
    const double c2 = d == 1 ? -1.0 : (d == 2 ? -3.0 : -6.0);
    const double c3 = d == 2 ? 1.0 : 4.0;
    const size_t e0 = (size_t)it.y * kBeginChunk + threadIdx.x;
    double2 g[4];
    if (mode >= 2 && n >= 4) {  // the steady case, one straight pass: all 16 loads issued first
        double2 f1[4], f2[4], f3[4], f4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            size_t e = e0 + (size_t)u * 256;
            e = e < n2 ? e : n2 - 1;  // in bounds
            f1[u] = p.H1[e];
            f2[u] = p.H2[e];
            f3[u] = p.H3[e];
            f4[u] = p.F[e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // 4 H1 - 6 H2 + 4 H3 - F, summed in that order
            double2 t = make_double2(4.0 * f1[u].x, 4.0 * f1[u].y);
            t = make_double2(t.x + -6.0 * f2[u].x, t.y + -6.0 * f2[u].y);
            t = make_double2(t.x + 4.0 * f3[u].x, t.y + 4.0 * f3[u].y);
            g[u] = make_double2(t.x - f4[u].x, t.y - f4[u].y);
        }
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const size_t e = e0 + (size_t)u * 256;
            g[u] = begin_value(p, e < n2 ? e : n2 - 1, mode, n, slope, c1, c2, c3);  // in bounds
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const size_t e = e0 + (size_t)u * 256;
        if (e < n2) p.F[e] = g[u];
    }
    if (it.y == 0 && threadIdx.x == 0) done[it.x] = 0;
}

// Step index of mode 2: set before the first step of a run (set >= 0), or advanced at the end
// of each step (set < 0), when each simulation's W_n and W_{n+1} buffers swap and, with ring,
// its midpoint ring also turns (see ens_begin_kernel).
// rot (guess mode 3): after steps 0, 1, 2 of a run the next output is S1, S2, then Wc, so the
// states W_0 .. W_3 stay in Wc, X, S1, S2 until step 3 has started.
// One block: every thread reads the step index before thread 0 advances it.
constexpr int kStepcThreads = 256;
__global__ __launch_bounds__(kStepcThreads) void ens_stepc_kernel(int* __restrict__ stepc, int set,
                                                                  EnsProb* __restrict__ probs,
                                                                  int nsim, int ring, int rot) {
    const int n = stepc[0];  // the step that ends
    if (set < 0) {
        for (int i = threadIdx.x; i < nsim; i += kStepcThreads) {
            EnsProb& p = probs[i];
            double2* w = p.W;
            if (rot && n <= 2) {
                p.Wn = w;
                p.W = n == 0 ? p.S1 : (n == 1 ? p.S2 : p.Wc);
            } else {
                p.W = p.Wn;
                p.Wn = w;
            }
            if (ring) {
                double2* oldest = p.H3;
                p.H3 = p.H2;
                p.H2 = p.H1;
                p.H1 = p.F;
                p.F = oldest;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) stepc[0] = set >= 0 ? set : n + 1;
}

// Start of a run: W_n in the caller's matrix, W_{n+1} to the scratch one.
__global__ __launch_bounds__(64) void ens_run_begin_kernel(EnsProb* __restrict__ probs, int nsim) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i < nsim) {
        probs[i].Wn = probs[i].Wc;
        probs[i].W = probs[i].X;
    }
}

// Guess mode 3 with the difference form: after the first evaluation of a run's first step
// (step index 0), its W_{n+1} = W_0 + h D_0 is kept in Wd for the second step's start.
__global__ __launch_bounds__(256) void ens_save_first_kernel(const EnsProb* __restrict__ probs,
                                                             const int* __restrict__ stepc) {
    if (stepc[0] != 0) return;
    const int sim = blockIdx.x / kCopyParts, part = blockIdx.x % kCopyParts;
    const EnsProb p = probs[sim];
    const size_t n2 = (size_t)p.N * p.N;
    for (size_t e = (size_t)part * 256 + threadIdx.x; e < n2; e += (size_t)kCopyParts * 256)
        p.Wd[e] = p.W[e];
}

// End of a run: the last W_{n+1} (now in Wn) copied to the caller's matrix if it is in X.
__global__ __launch_bounds__(256) void ens_run_end_kernel(const EnsProb* __restrict__ probs) {
    const int sim = blockIdx.x / kCopyParts, part = blockIdx.x % kCopyParts;
    const EnsProb p = probs[sim];
    if (p.Wn == p.Wc) return;
    const size_t n2 = (size_t)p.N * p.N;
    for (size_t e = (size_t)part * 256 + threadIdx.x; e < n2; e += (size_t)kCopyParts * 256)
        p.Wc[e] = p.Wn[e];
}

template <int T, int C, int BD>
__global__ __launch_bounds__(T) void ens_solve_kernel(const EnsProb* __restrict__ probs,
                                                      const int2* __restrict__ work,
                                                      const int* __restrict__ done, int eval) {
    __shared__ double sG[T];
    __shared__ double2 sY[T];
    const int2 it = work[blockIdx.x];
    if (done[it.x]) return;
    const EnsProb p = probs[it.x];
    const double2* Wt = p.F;
    solve_band<T, C, BD>(Wt, p.P, p.fl, p.fd, p.N, it.y, sG, sY);
}

template <class C>
__global__ __launch_bounds__(kThreads) void ens_product_kernel(const EnsProb* __restrict__ probs,
                                                               const int2* __restrict__ work,
                                                               const int* __restrict__ done,
                                                               int eval) {
    __shared__ double smem[2 * C::STAGE];
    const int2 it = work[blockIdx.x];
    if (done[it.x]) return;
    const EnsProb p = probs[it.x];
    const int N = p.N;
    const double2* Wt = p.F;
    const int tiles_n = (N + C::BNC - 1) / C::BNC;
    const int row0 = (it.y / tiles_n) * C::BM, col0 = (it.y % tiles_n) * C::BNC;
    d4 acc[C::MT][C::NT];
    const int nk = (N + kBK - 1) / kBK;
    mainloop<C>(p.P, N, row0, N, Wt, N, col0, N, N, 0, nk, smem, acc);
    store_tile<C>(acc, p.A, N, row0, col0);
}

__global__ __launch_bounds__(kThreads) void ens_lower_kernel(const EnsProb* __restrict__ probs,
                                                             const int2* __restrict__ work,
                                                             const int* __restrict__ done) {
    __shared__ double smem[2 * LowCfg::STAGE];
    const int2 it = work[blockIdx.x];
    if (done[it.x]) return;
    const EnsProb p = probs[it.x];
    const int N = p.N;
    int I, J;
    lower_tile(it.y, I, J);
    d4 acc[LowCfg::MT][LowCfg::NT];
    const int nk = (N + kBK - 1) / kBK;
    mainloop<LowCfg>(p.A, N, I * kTile, N, p.P, N, J * kTile, N, N, 0, nk, smem, acc);
    store_tile<LowCfg>(acc, p.Q, N, I * kTile, J * kTile);
}

// The fixed-point update of the FP64 products, on UT x UT lower tiles (work items (sim, tile)).
template <int UT>
__global__ __launch_bounds__(kUThreads) void ens_update_kernel(const EnsProb* __restrict__ probs,
                                                               const int2* __restrict__ work,
                                                               const int* __restrict__ done,
                                                               int eval, double h, int form) {
    __shared__ double2 sT[UT][UT + 1];
    const int2 it = work[blockIdx.x];
    if (done[it.x]) return;
    const EnsProb p = probs[it.x];
    const double2* Wt = p.F;
    int I, J;
    lower_tile(it.y, I, J);
    lower_update_tile_t<UT>(I, J, p.Q, nullptr, nullptr, nullptr, 0, p.A, p.Wn, Wt, p.F, p.W,
                            p.rowpart, p.N, h, form, sT);
}

// ---------------------------------------------------------------- split-precision phases
// which = 0 (product P W~): item y < N slices row y of P (exponent ep), item y >= N takes the
// column exponents ew of W~ for columns 64 (y - N) ...; which = 1 (product A P): row y of A
// (exponent eA).
__global__ __launch_bounds__(kSThreads) void ens_split_rows_kernel(const EnsProb* __restrict__ probs,
                                                                   const int2* __restrict__ work,
                                                                   const int* __restrict__ done,
                                                                   int eval, int which, int s) {
    __shared__ double red[kSThreads];
    const int2 it = work[blockIdx.x];
    if (done[it.x]) return;
    const EnsProb p = probs[it.x];
    const int N = p.N, ldk = split_ldk_of(N);
    if (which == 1) {
        split_row_block(p.A, N, it.y, s, ldk, p.sa, p.eA, red);
    } else if (it.y < N) {
        split_row_block(p.P, N, it.y, s, ldk, p.sa, p.ep, red);
    } else {
        const double2* Wt = p.F;
        col_exponent_block(Wt, N, 64 * (it.y - N), p.ew, reinterpret_cast<double(*)[64]>(red));
    }
}

// B~^T slices of W~ (which = 0, exponents ew) or of P (which = 1; P is skew-Hermitian, so
// its column exponents are its row exponents ep).
__global__ __launch_bounds__(kSThreads) void ens_split_cols_kernel(const EnsProb* __restrict__ probs,
                                                                   const int2* __restrict__ work,
                                                                   const int* __restrict__ done,
                                                                   int eval, int which, int s) {
    __shared__ double2 tile[kCT][kCT + 1];
    const int2 it = work[blockIdx.x];
    if (done[it.x]) return;
    const EnsProb p = probs[it.x];
    const int N = p.N, ldk = split_ldk_of(N);
    const int gx = (N + kCT - 1) / kCT;
    const double2* B = which == 1 ? p.P : p.F;
    split_cols_tile(B, N, it.y % gx, it.y / gx, s, ldk, which == 1 ? p.ep : p.ew, p.sb, tile);
}

// INT8 slabs: mode 0 all tiles (row tile y / tn, column tile y % tn), mode 1 lower tiles.
__global__ __launch_bounds__(kSThreads, 2) void ens_i8_kernel(const EnsProb* __restrict__ probs,
                                                              const int2* __restrict__ work,
                                                              const int* __restrict__ done,
                                                              int mode, int s) {
    __shared__ I8Smem sm;
    const int2 it = work[blockIdx.x];
    if (done[it.x]) return;
    const EnsProb p = probs[it.x];
    const int N = p.N;
    const int tn = (2 * N + kI8BN - 1) / kI8BN;
    int ti, tj;
    if (mode == 0) {
        ti = it.y / tn;
        tj = it.y % tn;
    } else {
        i8_lower_tile(it.y, ti, tj);
        if (tj >= tn) return;
    }
    zgemm_i8_tile(ti, tj, p.sa, p.sb, p.G, N, s, split_ldk_of(N), sm);
}

// A from the slabs of the product P W~: item y covers elements 1024 y ... 1024 y + 1023.
constexpr int kCombineChunk = 1024;
__global__ __launch_bounds__(kSThreads) void ens_combine_kernel(const EnsProb* __restrict__ probs,
                                                                const int2* __restrict__ work,
                                                                const int* __restrict__ done,
                                                                int s) {
    const int2 it = work[blockIdx.x];
    if (done[it.x]) return;
    const EnsProb p = probs[it.x];
    const size_t n2 = (size_t)p.N * p.N;
#pragma unroll
    for (int j = 0; j < kCombineChunk / kSThreads; ++j) {
        const size_t e = (size_t)it.y * kCombineChunk + j * kSThreads + threadIdx.x;
        if (e < n2) p.A[e] = split_combine_elem(p.G, p.ep, p.ew, p.N, s, e);
    }
}

// The fixed-point update from the slabs of the lower product A P (exponents eA, ep).
__global__ __launch_bounds__(kUThreads) void ens_update_split_kernel(const EnsProb* __restrict__ probs,
                                                                     const int2* __restrict__ work,
                                                                     const int* __restrict__ done,
                                                                     int eval, double h, int s,
                                                                     int form) {
    __shared__ double2 sT[kUT][kUT + 1];
    const int2 it = work[blockIdx.x];
    if (done[it.x]) return;
    const EnsProb p = probs[it.x];
    const double2* Wt = p.F;
    int I, J;
    lower_tile(it.y, I, J);
    lower_update_tile_t<kUT, true>(I, J, nullptr, p.G, p.eA, p.ep, s, p.A, p.Wn, Wt, p.F, p.W,
                                   p.rowpart, p.N, h, form, sT);
}

__global__ __launch_bounds__(256) void ens_resid_kernel(const EnsProb* __restrict__ probs,
                                                        int* __restrict__ done,
                                                        int* __restrict__ iters,
                                                        double* __restrict__ resid, int eval,
                                                        double tol, int ut) {
    __shared__ double sm[256];
    const int sim = blockIdx.x;
    if (done[sim]) return;
    const EnsProb p = probs[sim];
    const int N = p.N, T = (N + ut - 1) / ut;  // row-sum slots of the update's ut x ut tiles
    double best = 0.0;
    for (int i = threadIdx.x; i < N; i += 256) {
        const double v = slot_row_sum<8>(p.rowpart, T, N, i);
        best = (v != v || v > best) ? v : best;
    }
    sm[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = sm[threadIdx.x + s], a = sm[threadIdx.x];
            sm[threadIdx.x] = (o != o || o > a) ? o : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double r = sm[0];
        resid[sim] = r;
        iters[sim] = eval;
        if (!(r < tol) && r == r && r < INFINITY) return;  // keep iterating
        done[sim] = 1;  // converged, or non-finite: stop this simulation
    }
}

// Grouped stream solve of every simulation.  All contexts of an ensemble share one band width,
// ens_bd(maxN), and the launch shape satisfies (T / BD) C >= N + BD for every N <= maxN.
template <int T, int C, int BD>
hipError_t launch_ens_solve(const EnsProb* probs, const int2* work, int n, const int* done,
                            int eval, hipStream_t s) {
    hipLaunchKernelGGL((ens_solve_kernel<T, C, BD>), dim3(n), dim3(T), 0, s, probs, work, done, eval);
    return hipGetLastError();
}

// Band width of an ensemble's stream solve.  Not solve_bd's: the many bands of an ensemble
// keep the GPU busy, so the longer row segments of wide bands pay even where one small problem
// alone wants one-lane bands (64 simulations, N <= 512: 97 us with 4 lanes, 192 with 1).
int ens_bd(int maxN) { return maxN <= 2172 ? 4 : (maxN <= 4606 ? 2 : 1); }

hipError_t ens_solve(int maxN, const EnsProb* probs, const int2* work, int n, const int* done,
                     int eval, hipStream_t s) {
    const int bd = ens_bd(maxN);
    if (bd == 1) {  // maxN > 4606
        if (maxN <= 9215) return launch_ens_solve<1024, 9, 1>(probs, work, n, done, eval, s);
        return launch_ens_solve<1024, 17, 1>(probs, work, n, done, eval, s);
    }
    if (bd == 2) return launch_ens_solve<1024, 9, 2>(probs, work, n, done, eval, s);
    if (maxN <= 76) return launch_ens_solve<64, 5, 4>(probs, work, n, done, eval, s);
    if (maxN <= 156) return launch_ens_solve<128, 5, 4>(probs, work, n, done, eval, s);
    if (maxN <= 316) return launch_ens_solve<256, 5, 4>(probs, work, n, done, eval, s);
    if (maxN <= 572) return launch_ens_solve<256, 9, 4>(probs, work, n, done, eval, s);
    if (maxN <= 1084) return launch_ens_solve<256, 17, 4>(probs, work, n, done, eval, s);
    return launch_ens_solve<512, 17, 4>(probs, work, n, done, eval, s);
}

using WideCfg = FullCfg;  // 128 x 64 complex
using SmallCfg = LowCfg;  // 64 x 64 complex

int tiles_of(int N, int variant) {
    if (variant == 0) return ((N + WideCfg::BM - 1) / WideCfg::BM) * ((N + WideCfg::BNC - 1) / WideCfg::BNC);
    return ((N + SmallCfg::BM - 1) / SmallCfg::BM) * ((N + SmallCfg::BNC - 1) / SmallCfg::BNC);
}

// Work list: all (sim, item) pairs, either largest N first or simulations interleaved.
std::vector<int2> make_work(const std::vector<int>& N, const std::vector<int>& count, int order) {
    std::vector<int2> w;
    const int ns = (int)N.size();
    if (order == 0) {
        std::vector<int> idx(ns);
        for (int i = 0; i < ns; ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return N[a] > N[b]; });
        for (int i : idx)
            for (int k = 0; k < count[i]; ++k) w.push_back(make_int2(i, k));
    } else {
        int maxc = 0;
        for (int c : count) maxc = std::max(maxc, c);
        for (int k = 0; k < maxc; ++k)
            for (int i = 0; i < ns; ++i)
                if (k < count[i]) w.push_back(make_int2(i, k));
    }
    return w;
}

}  // namespace

struct ze_ens {
    int nsim = 0, maxN = 0;
    hipStream_t user = nullptr;   // caller's stream
    hipStream_t own = nullptr;    // private stream the graph is captured on and replayed on
    hipEvent_t ev_in = nullptr, ev_out = nullptr, t0 = nullptr, t1 = nullptr;
    std::vector<int> N;
    std::vector<ze_ctx*> ctx;     // per-simulation factors and workspaces
    std::vector<EnsProb> hp;
    EnsProb* dp = nullptr;
    int* done = nullptr;
    int* iters = nullptr;
    double* resid = nullptr;
    int2* work_solve = nullptr;
    int n_solve = 0;
    int2* work_prod[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [variant][order]
    int n_prod[2] = {0, 0};
    int2* work_low[2] = {nullptr, nullptr};                            // [order]
    int n_low = 0;
    int2* work_begin = nullptr;  // (simulation, chunk of kBeginChunk entries) of the step start
    int n_begin = 0;
    // the FP64 path's update tile (32, or 64 when a context's row-sum slots are 64 wide) and
    // its lower tiles
    int ut = 32;
    int2* work_up[2] = {nullptr, nullptr};                             // [order]
    int n_up = 0;
    // split-precision phases (work lists built at creation, buffers on first use)
    int slices = 5;  // min(5, split_max_slices(maxN)), set at creation
    int slices_low = 4;  // of the lower product Q = A P (its term enters F with h^2/4)
    bool split_ready = false;
    int2* w_rows0 = nullptr;   // rows of P + column chunks of W~
    int2* w_rows1 = nullptr;   // rows of A
    int2* w_cols = nullptr;    // B~^T slice tiles
    int2* w_comb = nullptr;    // combine chunks
    int2* w_i8[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [mode][order]
    int n_rows0 = 0, n_rows1 = 0, n_cols = 0, n_comb = 0, n_i8[2] = {0, 0};
    // tuning: FP64 (tile shape, order) and split (order)
    int variant = -1, order = 0;
    double tune_ms[4] = {0, 0, 0, 0};
    int s_order = -1;
    double s_tune_ms[2] = {0, 0};
    // captured graph and the parameters it was captured with
    hipGraphExec_t exec = nullptr;
    int g_prec = -1, g_variant = -1, g_order = -1, g_K = -1, g_slices = -1, g_guess = -1;
    int g_slices_low = -1;
    // first iterate of the steps after the first of a run: 0 = W_n, 1 = 2 W_n - F_prev,
    // 2 = polynomial extrapolation of the run's midpoints (the step index in *stepc)
    int guess_mode = 0;
    int* stepc = nullptr;
    int update_form = 0;  // W_{n+1}: 0 the second line of eq. (isomp), 1 W_n + h [P~, W~]
    int g_form = -1;
    hipGraphExec_t exec_x = nullptr;  // the step graph with the extrapolated first iterate
    double g_h = 0.0, g_tol = -1.0;
    // evaluation cap of the steps from index cap2_after on (guess mode 2; 0: the run's cap K)
    // and the step graph captured with it
    int cap2 = 0, cap2_after = 0, g_cap2 = -1;
    // continuation (ze_ensemble_set_continuation): the step index cont_n the next run starts
    // from when it continues the last one (same matrices, h, precision, start mode and update
    // form); cont_n < 0: none
    int cont = 0, cont_n = -1;
    std::vector<void*> cont_w;
    double cont_h = 0.0;
    int cont_prec = -1, cont_guess = -1, cont_form = -1;
    bool g_cap2_first = true;  // the capped graph was captured for a step index that may be 0
    hipGraphExec_t exec_s = nullptr;
};

namespace {

// first: the graph may run the first step of a call (the step index 0), whose first
// evaluation's output the second step's slope start needs.
hipError_t record_step(ze_ens* e, double h, double tol, int K, int prec, int variant, int order,
                       int mode, hipStream_t s, bool first = true) {
    const int slope = mode == 3 && e->update_form == 1 ? 1 : 0;
    hipLaunchKernelGGL(ens_begin_kernel, dim3(e->n_begin), dim3(256), 0, s, e->dp, e->work_begin,
                       e->done, mode, e->stepc, slope);
    hipError_t err = hipGetLastError();
    const int ns = e->slices, nl = e->slices_low;
#define ZE_ENS_LAUNCH(...)                       \
    do {                                         \
        hipLaunchKernelGGL(__VA_ARGS__);         \
        err = hipGetLastError();                 \
        if (err != hipSuccess) return err;       \
    } while (0)
    for (int k = 1; k <= K && err == hipSuccess; ++k) {
        err = ens_solve(e->maxN, e->dp, e->work_solve, e->n_solve, e->done, k, s);
        if (err != hipSuccess) break;
        if (prec == ZE_PREC_SPLIT) {
            ZE_ENS_LAUNCH(ens_split_rows_kernel, dim3(e->n_rows0), dim3(kSThreads), 0, s, e->dp,
                          e->w_rows0, e->done, k, 0, ns);
            ZE_ENS_LAUNCH(ens_split_cols_kernel, dim3(e->n_cols), dim3(kSThreads), 0, s, e->dp,
                          e->w_cols, e->done, k, 0, ns);
            ZE_ENS_LAUNCH(ens_i8_kernel, dim3(e->n_i8[0]), dim3(kSThreads), 0, s, e->dp,
                          e->w_i8[0][order], e->done, 0, ns);
            ZE_ENS_LAUNCH(ens_combine_kernel, dim3(e->n_comb), dim3(kSThreads), 0, s, e->dp,
                          e->w_comb, e->done, ns);
            ZE_ENS_LAUNCH(ens_split_rows_kernel, dim3(e->n_rows1), dim3(kSThreads), 0, s, e->dp,
                          e->w_rows1, e->done, k, 1, nl);
            ZE_ENS_LAUNCH(ens_split_cols_kernel, dim3(e->n_cols), dim3(kSThreads), 0, s, e->dp,
                          e->w_cols, e->done, k, 1, nl);
            ZE_ENS_LAUNCH(ens_i8_kernel, dim3(e->n_i8[1]), dim3(kSThreads), 0, s, e->dp,
                          e->w_i8[1][order], e->done, 1, nl);
            ZE_ENS_LAUNCH(ens_update_split_kernel, dim3(e->n_low), dim3(kUThreads), 0, s, e->dp,
                          e->work_low[order], e->done, k, h, nl, e->update_form);
        } else {
            if (variant == 0)
                ZE_ENS_LAUNCH(ens_product_kernel<WideCfg>, dim3(e->n_prod[0]), dim3(kThreads), 0, s,
                              e->dp, e->work_prod[0][order], e->done, k);
            else
                ZE_ENS_LAUNCH(ens_product_kernel<SmallCfg>, dim3(e->n_prod[1]), dim3(kThreads), 0, s,
                              e->dp, e->work_prod[1][order], e->done, k);
            ZE_ENS_LAUNCH(ens_lower_kernel, dim3(e->n_low), dim3(kThreads), 0, s, e->dp,
                          e->work_low[order], e->done);
            if (e->ut == 32)
                ZE_ENS_LAUNCH(ens_update_kernel<32>, dim3(e->n_up), dim3(kUThreads), 0, s, e->dp,
                              e->work_up[order], e->done, k, h, e->update_form);
            else
                ZE_ENS_LAUNCH(ens_update_kernel<kUT>, dim3(e->n_low), dim3(kUThreads), 0, s, e->dp,
                              e->work_low[order], e->done, k, h, e->update_form);
        }
        ZE_ENS_LAUNCH(ens_resid_kernel, dim3(e->nsim), dim3(256), 0, s, e->dp, e->done, e->iters,
                      e->resid, k, tol, prec == ZE_PREC_SPLIT ? kUT : e->ut);
        if (k == 1 && slope && first)
            ZE_ENS_LAUNCH(ens_save_first_kernel, dim3(e->nsim * kCopyParts), dim3(256), 0, s, e->dp,
                          e->stepc);
    }
    if (err == hipSuccess)
        ZE_ENS_LAUNCH(ens_stepc_kernel, dim3(1), dim3(kStepcThreads), 0, s, e->stepc, -1,
                      e->dp, e->nsim, mode >= 2 ? 1 : 0, mode == 3 ? 1 : 0);
#undef ZE_ENS_LAUNCH
    return err;
}

hipError_t capture_one(ze_ens* e, double h, double tol, int K, int prec, int variant, int order,
                       int mode, hipGraphExec_t* out, bool first = true) {
    if (*out) {
        (void)hipGraphExecDestroy(*out);
        *out = nullptr;
    }
    hipGraph_t g = nullptr;
    hipError_t err = hipStreamBeginCapture(e->own, hipStreamCaptureModeRelaxed);
    if (err != hipSuccess) return err;
    hipError_t rec = record_step(e, h, tol, K, prec, variant, order, mode, e->own, first);
    err = hipStreamEndCapture(e->own, &g);
    if (rec != hipSuccess) err = rec;
    if (err == hipSuccess) err = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return err;
}

// The step graph (first iterate W_n, or with guess mode 2 chosen by the step index) and, with
// guess mode 1, the graph of the steps after the first of a run (first iterate 2 W_n - F_prev).
hipError_t capture(ze_ens* e, double h, double tol, int K, int prec, int variant, int order) {
    hipError_t err = capture_one(e, h, tol, K, prec, variant, order,
                                 e->guess_mode >= 2 ? e->guess_mode : 0, &e->exec);
    if (err == hipSuccess && e->guess_mode == 1)
        err = capture_one(e, h, tol, K, prec, variant, order, 1, &e->exec_x);
    if (e->exec_s) {
        (void)hipGraphExecDestroy(e->exec_s);
        e->exec_s = nullptr;
    }
    if (err == hipSuccess && e->guess_mode >= 2 && e->cap2 > 0 && e->cap2 < K)
        err = capture_one(e, h, tol, e->cap2, prec, variant, order, e->guess_mode, &e->exec_s,
                          e->cap2_after == 0);
    if (err == hipSuccess) {
        e->g_guess = e->guess_mode;
        e->g_prec = prec;
        e->g_variant = variant;
        e->g_order = order;
        e->g_K = K;
        e->g_slices = e->slices;
        e->g_slices_low = e->slices_low;
        e->g_form = e->update_form;
        e->g_h = h;
        e->g_tol = tol;
        e->g_cap2 = e->cap2;
        e->g_cap2_first = e->cap2_after == 0;
    }
    return err;
}

template <class T>
ze_status ens_alloc(T** p, size_t n) {
    if (hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T) + 64) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return ZE_ENOMEM;
    }
    return ZE_OK;
}

ze_status upload_work(const std::vector<int2>& w, int2** dst) {
    ZE_TRY(ens_alloc(dst, w.size()));
    ZE_HIP(hipMemcpy(*dst, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice));
    return ZE_OK;
}

ze_status set_pointers(ze_ens* e, void* const* W) {
    bool changed = false;
    for (int i = 0; i < e->nsim; ++i) {
        if (!W[i]) return ZE_EINVAL;
        if (e->hp[i].Wc != W[i]) {
            e->hp[i].Wc = static_cast<double2*>(W[i]);
            changed = true;
        }
    }
    if (changed) {  // rare: drain the private stream, then replace the descriptors
        ZE_HIP(hipStreamSynchronize(e->own));
        ZE_HIP(hipMemcpy(e->dp, e->hp.data(), e->hp.size() * sizeof(EnsProb), hipMemcpyHostToDevice));
    }
    return ZE_OK;
}

// Times the candidate graphs on copies of the inputs and keeps the fastest: FP64, the four
// (tile shape, order) pairs; split precision, the two work orders.
ze_status autotune(ze_ens* e, void* const* W, double h, double tol, int K, int prec) {
    std::vector<double2*> copies(e->nsim, nullptr);
    ze_status st = ZE_OK;
    for (int i = 0; i < e->nsim && st == ZE_OK; ++i) {
        const size_t n2 = (size_t)e->N[i] * e->N[i];
        st = ens_alloc(&copies[i], n2);
        if (st == ZE_OK &&
            hipMemcpyAsync(copies[i], W[i], n2 * sizeof(double2), hipMemcpyDeviceToDevice, e->own) != hipSuccess)
            st = ZE_EHIP;
    }
    const bool split = prec == ZE_PREC_SPLIT;
    const int ncand = split ? 2 : 4;
    double best = 1e300;
    for (int cand = 0; cand < ncand && st == ZE_OK; ++cand) {
        const int variant = split ? 0 : cand >> 1, order = split ? cand : cand & 1;
        st = set_pointers(e, reinterpret_cast<void* const*>(copies.data()));
        if (st != ZE_OK) break;
        if (capture_one(e, h, tol, K, prec, variant, order, 0, &e->exec) != hipSuccess) {
            st = ze_record_hip(hipGetLastError(), "ensemble autotune capture");
            break;
        }
        float ms = 0.f;
        hipLaunchKernelGGL(ens_run_begin_kernel, dim3((e->nsim + 63) / 64), dim3(64), 0, e->own,
                           e->dp, e->nsim);
        hipError_t err = hipGetLastError();
        if (err == hipSuccess) err = hipGraphLaunch(e->exec, e->own);  // warm-up
        if (err == hipSuccess) err = hipEventRecord(e->t0, e->own);
        for (int r = 0; r < 3 && err == hipSuccess; ++r) err = hipGraphLaunch(e->exec, e->own);
        if (err == hipSuccess) err = hipEventRecord(e->t1, e->own);
        if (err == hipSuccess) err = hipEventSynchronize(e->t1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e->t0, e->t1);
        if (err != hipSuccess) {
            st = ze_record_hip(err, "ensemble autotune run");
            break;
        }
        (split ? e->s_tune_ms : e->tune_ms)[cand] = ms / 3.0;
        if (ms < best) {
            best = ms;
            if (split) {
                e->s_order = order;
            } else {
                e->variant = variant;
                e->order = order;
            }
        }
    }
    (void)hipStreamSynchronize(e->own);
    for (double2* c : copies)
        if (c) (void)hipFree(c);
    // restore the caller's pointers (set_pointers compares against hp)
    for (int i = 0; i < e->nsim; ++i) e->hp[i].Wc = nullptr;
    if (e->exec) {
        (void)hipGraphExecDestroy(e->exec);
        e->exec = nullptr;
    }
    if (e->exec_x) {
        (void)hipGraphExecDestroy(e->exec_x);
        e->exec_x = nullptr;
    }
    if (e->exec_s) {
        (void)hipGraphExecDestroy(e->exec_s);
        e->exec_s = nullptr;
    }
    return st;
}

// Split-precision workspaces of every simulation, allocated on the first split run.
ze_status ensure_split(ze_ens* e) {
    if (e->split_ready) return ZE_OK;
    ZE_HIP(hipStreamSynchronize(e->own));
    for (int i = 0; i < e->nsim; ++i) {
        ze_ctx* c = e->ctx[i];
        ZE_TRY(ze_ensure_split(c));
        e->hp[i].sa = c->split_a;
        e->hp[i].sb = c->split_b;
        e->hp[i].G = c->split_g;
        e->hp[i].ep = c->split_ea;
        e->hp[i].ew = c->split_eb;
        e->hp[i].eA = c->split_ec;
    }
    ZE_HIP(hipMemcpy(e->dp, e->hp.data(), e->hp.size() * sizeof(EnsProb), hipMemcpyHostToDevice));
    e->split_ready = true;
    return ZE_OK;
}

}  // namespace

extern "C" {

ze_status ze_ensemble_destroy(ze_ens* e) {
    if (!e) return ZE_OK;
    if (e->own) (void)hipStreamSynchronize(e->own);
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->exec_x) (void)hipGraphExecDestroy(e->exec_x);
    if (e->exec_s) (void)hipGraphExecDestroy(e->exec_s);
    for (ze_ctx* c : e->ctx) ze_destroy(c);
    (void)hipFree(e->dp);
    (void)hipFree(e->done);
    (void)hipFree(e->iters);
    (void)hipFree(e->resid);
    (void)hipFree(e->stepc);
    (void)hipFree(e->work_solve);
    for (auto& v : e->work_prod)
        for (int2* p : v) (void)hipFree(p);
    for (int2* p : e->work_low) (void)hipFree(p);
    for (int2* p : e->work_up) (void)hipFree(p);
    if (e->work_begin) (void)hipFree(e->work_begin);
    for (int2* p : {e->w_rows0, e->w_rows1, e->w_cols, e->w_comb}) (void)hipFree(p);
    for (auto& v : e->w_i8)
        for (int2* p : v) (void)hipFree(p);
    for (hipEvent_t ev : {e->ev_in, e->ev_out, e->t0, e->t1})
        if (ev) (void)hipEventDestroy(ev);
    if (e->own) (void)hipStreamDestroy(e->own);
    delete e;
    return ZE_OK;
}

ze_status ze_ensemble_create(int nsim, const int* N, void* stream, ze_ens** out) {
    if (!out || !N || nsim < 1 || nsim > 4096) return ZE_EINVAL;
    *out = nullptr;
    for (int i = 0; i < nsim; ++i)
        if (N[i] < 1 || N[i] > 4096) return ZE_EINVAL;
    ze_ens* e = new ze_ens();
    e->nsim = nsim;
    e->user = reinterpret_cast<hipStream_t>(stream);
    e->N.assign(N, N + nsim);
    e->maxN = *std::max_element(e->N.begin(), e->N.end());
    e->slices = split_max_slices(e->maxN) < 5 ? split_max_slices(e->maxN) : 5;
    e->slices_low = e->slices > 2 ? e->slices - 1 : 2;
    ze_status st = ZE_OK;
    auto fail = [&](ze_status s) {
        ze_ensemble_destroy(e);
        return s;
    };
    if (hipStreamCreateWithFlags(&e->own, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&e->t0) != hipSuccess || hipEventCreate(&e->t1) != hipSuccess)
        return fail(ze_record_hip(hipGetLastError(), "ensemble stream/events"));
    e->ctx.assign(nsim, nullptr);
    e->hp.resize(nsim);
    for (int i = 0; i < nsim; ++i) {
        st = ze_create_ctx(e->N[i], e->own, false, ens_bd(e->maxN), &e->ctx[i]);
        if (st != ZE_OK) return fail(st);
        ze_ctx* c = e->ctx[i];
        e->hp[i] = EnsProb{c->N,       0,       nullptr,  c->Wn,       nullptr, c->Wn,   c->F,
                           c->P,       c->A,    c->Q,     c->rowpart,  c->fac_l, c->fac_dinv,
                           nullptr,    nullptr, nullptr,  nullptr,     nullptr, nullptr,
                           nullptr,    nullptr, nullptr,  nullptr,     nullptr, nullptr};
    }
    if ((st = ens_alloc(&e->dp, (size_t)nsim)) != ZE_OK) return fail(st);
    if ((st = ens_alloc(&e->done, (size_t)nsim)) != ZE_OK) return fail(st);
    if ((st = ens_alloc(&e->iters, (size_t)nsim)) != ZE_OK) return fail(st);
    if ((st = ens_alloc(&e->resid, (size_t)nsim)) != ZE_OK) return fail(st);
    if ((st = ens_alloc(&e->stepc, (size_t)1)) != ZE_OK) return fail(st);
    std::vector<int> cs(nsim), c0(nsim), c1(nsim), cl(nsim), cu(nsim);
    // the update's tile: 32, unless a context keeps only 64-wide row-sum slots
    for (int i = 0; i < nsim; ++i)
        if (e->ctx[i]->ut > 32) e->ut = kUT;
    std::vector<int> r0(nsim), r1(nsim), ccol(nsim), ccomb(nsim), i8f(nsim), i8l(nsim);
    for (int i = 0; i < nsim; ++i) {
        const int n = e->N[i], T = (n + kTile - 1) / kTile;
        cs[i] = solve_bands(n, ens_bd(e->maxN));
        c0[i] = tiles_of(n, 0);
        c1[i] = tiles_of(n, 1);
        cl[i] = T * (T + 1) / 2;
        const int Tu = (n + e->ut - 1) / e->ut;
        cu[i] = Tu * (Tu + 1) / 2;
        const int tr = (n + kI8BM - 1) / kI8BM, tn = (2 * n + kI8BN - 1) / kI8BN;
        r0[i] = n + (n + 63) / 64;
        r1[i] = n;
        ccol[i] = ((n + kCT - 1) / kCT) * ((split_ldk_of(n) / 2 + kCT - 1) / kCT);
        ccomb[i] = (int)(((size_t)n * n + kCombineChunk - 1) / kCombineChunk);
        i8f[i] = tr * tn;
        i8l[i] = tr * (tr + 1);
    }
    {
        std::vector<int2> w;
        w = make_work(e->N, r0, 0);
        e->n_rows0 = (int)w.size();
        if ((st = upload_work(w, &e->w_rows0)) != ZE_OK) return fail(st);
        w = make_work(e->N, r1, 0);
        e->n_rows1 = (int)w.size();
        if ((st = upload_work(w, &e->w_rows1)) != ZE_OK) return fail(st);
        w = make_work(e->N, ccol, 0);
        e->n_cols = (int)w.size();
        if ((st = upload_work(w, &e->w_cols)) != ZE_OK) return fail(st);
        w = make_work(e->N, ccomb, 0);
        e->n_comb = (int)w.size();
        if ((st = upload_work(w, &e->w_comb)) != ZE_OK) return fail(st);
        for (int order = 0; order < 2; ++order) {
            w = make_work(e->N, i8f, order);
            e->n_i8[0] = (int)w.size();
            if ((st = upload_work(w, &e->w_i8[0][order])) != ZE_OK) return fail(st);
            w = make_work(e->N, i8l, order);
            e->n_i8[1] = (int)w.size();
            if ((st = upload_work(w, &e->w_i8[1][order])) != ZE_OK) return fail(st);
        }
    }
    {
        std::vector<int> cb(nsim);
        for (int i = 0; i < nsim; ++i)
            cb[i] = (int)(((size_t)e->N[i] * e->N[i] + kBeginChunk - 1) / kBeginChunk);
        std::vector<int2> wb = make_work(e->N, cb, 0);
        e->n_begin = (int)wb.size();
        if ((st = upload_work(wb, &e->work_begin)) != ZE_OK) return fail(st);
    }
    std::vector<int2> ws = make_work(e->N, cs, 0);
    e->n_solve = (int)ws.size();
    if ((st = upload_work(ws, &e->work_solve)) != ZE_OK) return fail(st);
    for (int order = 0; order < 2; ++order) {
        std::vector<int2> w0 = make_work(e->N, c0, order), w1 = make_work(e->N, c1, order);
        std::vector<int2> wl = make_work(e->N, cl, order), wu = make_work(e->N, cu, order);
        e->n_prod[0] = (int)w0.size();
        e->n_prod[1] = (int)w1.size();
        e->n_low = (int)wl.size();
        if ((st = upload_work(w0, &e->work_prod[0][order])) != ZE_OK) return fail(st);
        if ((st = upload_work(w1, &e->work_prod[1][order])) != ZE_OK) return fail(st);
        if ((st = upload_work(wl, &e->work_low[order])) != ZE_OK) return fail(st);
        e->n_up = (int)wu.size();
        if ((st = upload_work(wu, &e->work_up[order])) != ZE_OK) return fail(st);
    }
    if (hipMemcpy(e->dp, e->hp.data(), nsim * sizeof(EnsProb), hipMemcpyHostToDevice) != hipSuccess)
        return fail(ze_record_hip(hipGetLastError(), "ensemble descriptors"));
    *out = e;
    return ZE_OK;
}

ze_status ze_ensemble_run(ze_ens* e, void* const* W, double h, double tol, int K, int nsteps,
                          int prec) {
    if (!e || !W || !std::isfinite(h) || !(tol >= 0.0) || !std::isfinite(tol) || K < 1 || K > 64 ||
        nsteps < 0)
        return ZE_EINVAL;
    if (prec != ZE_PREC_FP64 && prec != ZE_PREC_SPLIT) return ZE_EINVAL;
    for (int i = 0; i < e->nsim; ++i)
        if (!W[i]) return ZE_EINVAL;
    const bool split = prec == ZE_PREC_SPLIT;
    // the step index this run starts from: that of the run it continues, else 0 (guess mode 3
    // needs the states of the first four steps for steps 1 .. 3, which a run does not keep)
    int n0 = 0;
    if (e->cont && e->cont_n >= 0 && h == e->cont_h && prec == e->cont_prec &&
        e->guess_mode == e->cont_guess && e->update_form == e->cont_form &&
        (e->guess_mode != 3 || e->cont_n >= 4)) {
        n0 = e->cont_n;
        for (int i = 0; i < e->nsim; ++i)
            if (W[i] != e->cont_w[i]) n0 = 0;
    }
    e->cont_n = -1;
    // order after the caller's pending work
    ZE_HIP(hipEventRecord(e->ev_in, e->user));
    ZE_HIP(hipStreamWaitEvent(e->own, e->ev_in, 0));
    if (split) ZE_TRY(ensure_split(e));
    if (split ? e->s_order < 0 : e->variant < 0) {
        ZE_TRY(autotune(e, W, h, tol, K, prec));
        n0 = 0;  // the candidates' steps moved the step index
    }
    ZE_TRY(set_pointers(e, W));
    const int variant = split ? 0 : e->variant, order = split ? e->s_order : e->order;
    if (!e->exec || e->g_prec != prec || e->g_variant != variant || e->g_order != order ||
        e->g_K != K || e->g_h != h || e->g_tol != tol || e->g_slices != e->slices || e->g_slices_low != e->slices_low ||
        e->g_form != e->update_form || e->g_guess != e->guess_mode || e->g_cap2 != e->cap2 ||
        e->g_cap2_first != (e->cap2_after == 0))
        ZE_HIP(capture(e, h, tol, K, prec, variant, order));
    if (nsteps > 0) {
        hipLaunchKernelGGL(ens_run_begin_kernel, dim3((e->nsim + 63) / 64), dim3(64), 0, e->own,
                           e->dp, e->nsim);
        ZE_HIP(hipGetLastError());
    }
    if (e->guess_mode >= 2 && nsteps > 0 && n0 == 0) {  // the run's step index starts at 0
        hipLaunchKernelGGL(ens_stepc_kernel, dim3(1), dim3(kStepcThreads), 0, e->own, e->stepc, 0,
                           e->dp, 0, 0, 0);
        ZE_HIP(hipGetLastError());
    }
    for (int n = n0; n < n0 + nsteps; ++n) {
        hipGraphExec_t g = n > 0 && e->guess_mode == 1 ? e->exec_x : e->exec;
        if (e->exec_s && n >= e->cap2_after) g = e->exec_s;
        ZE_HIP(hipGraphLaunch(g, e->own));
    }
    if (nsteps > 0) {
        hipLaunchKernelGGL(ens_run_end_kernel, dim3(e->nsim * kCopyParts), dim3(256), 0, e->own, e->dp);
        ZE_HIP(hipGetLastError());
    }
    ZE_HIP(hipEventRecord(e->ev_out, e->own));
    ZE_HIP(hipStreamWaitEvent(e->user, e->ev_out, 0));
    if (e->cont) {
        e->cont_n = n0 + nsteps;
        e->cont_w.assign(W, W + e->nsim);
        e->cont_h = h;
        e->cont_prec = prec;
        e->cont_guess = e->guess_mode;
        e->cont_form = e->update_form;
    }
    return ZE_OK;
}

ze_status ze_ensemble_set_continuation(ze_ens* e, int on) {
    if (!e || on < 0 || on > 1) return ZE_EINVAL;
    e->cont = on;
    e->cont_n = -1;
    return ZE_OK;
}

ze_status ze_ensemble_step(ze_ens* e, void* const* W, double h, double tol, int K, int prec) {
    return ze_ensemble_run(e, W, h, tol, K, 1, prec);
}

ze_status ze_ensemble_stats(ze_ens* e, int* iters, double* resid) {
    if (!e) return ZE_EINVAL;
    ZE_HIP(hipStreamSynchronize(e->own));
    if (iters) ZE_HIP(hipMemcpy(iters, e->iters, e->nsim * sizeof(int), hipMemcpyDeviceToHost));
    if (resid) ZE_HIP(hipMemcpy(resid, e->resid, e->nsim * sizeof(double), hipMemcpyDeviceToHost));
    return ZE_OK;
}

ze_status ze_ensemble_tuning(ze_ens* e, int prec, int* choice, double* ms) {
    if (!e || (prec != ZE_PREC_FP64 && prec != ZE_PREC_SPLIT)) return ZE_EINVAL;
    if (prec == ZE_PREC_SPLIT) {
        if (choice) *choice = e->s_order;
        if (ms)
            for (int i = 0; i < 4; ++i) ms[i] = i < 2 ? e->s_tune_ms[i] : 0.0;
        return ZE_OK;
    }
    if (choice) *choice = e->variant < 0 ? -1 : 2 * e->variant + e->order;
    if (ms)
        for (int i = 0; i < 4; ++i) ms[i] = e->tune_ms[i];
    return ZE_OK;
}

ze_status ze_ensemble_set_initial_guess(ze_ens* e, int mode) {
    if (!e || mode < 0 || mode > 3) return ZE_EINVAL;
    e->cont_n = -1;  // the next run starts at step 0
    const bool ring = mode >= 2 && !e->hp[0].H1, states = mode == 3 && !e->hp[0].S1;
    if (ring || states) {
        // the descriptors on the device are the current ones (the steps turn them): fetch, add
        // the new buffers, put back
        ZE_HIP(hipStreamSynchronize(e->own));
        ZE_HIP(hipMemcpy(e->hp.data(), e->dp, e->hp.size() * sizeof(EnsProb), hipMemcpyDeviceToHost));
        for (int i = 0; i < e->nsim; ++i) {
            ze_ctx* c = e->ctx[i];
            if (ring) {  // midpoint history, 3 buffers per simulation
                ZE_TRY(ze_ensure_rings(c, 1));
                e->hp[i].H1 = c->ring[1];
                e->hp[i].H2 = c->ring[2];
                e->hp[i].H3 = c->ring[3];
            }
            if (states) {  // two more states and W_0 + h D_0 per simulation
                ZE_TRY(ze_set_initial_guess(c, 3));
                e->hp[i].S1 = c->Wh[0];
                e->hp[i].S2 = c->Wh[1];
                e->hp[i].Wd = c->Wd;
            }
        }
        ZE_HIP(hipMemcpy(e->dp, e->hp.data(), e->hp.size() * sizeof(EnsProb), hipMemcpyHostToDevice));
    }
    e->guess_mode = mode;
    return ZE_OK;
}

ze_status ze_ensemble_set_steady_cap(ze_ens* e, int cap, int from_step) {
    if (!e || cap < 0 || cap > 64 || from_step < 0) return ZE_EINVAL;
    e->cap2 = cap;
    e->cap2_after = from_step;
    return ZE_OK;
}

ze_status ze_ensemble_set_split_slices(ze_ens* e, int slices) {
    if (!e || slices < 2 || slices > split_max_slices(e->maxN)) return ZE_EINVAL;
    e->cont_n = -1;  // the next run starts at step 0
    e->slices = slices;
    e->slices_low = slices > 2 ? slices - 1 : 2;
    return ZE_OK;
}

ze_status ze_ensemble_set_update_form(ze_ens* e, int form) {
    if (!e || form < 0 || form > 1) return ZE_EINVAL;
    e->cont_n = -1;  // the next run starts at step 0
    e->update_form = form;
    return ZE_OK;
}

ze_status ze_ensemble_set_split_slices_lower(ze_ens* e, int slices) {
    if (!e || slices < 2 || slices > e->slices) return ZE_EINVAL;
    e->cont_n = -1;  // the next run starts at step 0
    e->slices_low = slices;
    return ZE_OK;
}

}  // extern "C"

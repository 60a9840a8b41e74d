// Stream solve P = Delta_N^+ W: one tridiagonal system per matrix diagonal (Sec. 3.3,
// eq. (sub_tria_W)), with the LDL^T factors of the blocks Delta^m of eq. (delta_tria).
//
// Work split and memory layout.  Diagonal m (N - m entries) is paired with m' = N - 1 - m
// (m + 1 entries); workgroup k solves the BD consecutive diagonals m = k BD .. k BD + BD - 1
// and their partners, one lane per pair.  The entries are placed on "virtual rows" (see
// solve_band in solve_wg.h) so that at every step the BD lanes of a group read or write BD
// neighbouring entries of one matrix row: the accesses are row segments, not the one-entry-
// per-row pattern of a diagonal.  The factors are stored in the same (band, virtual row,
// lane) order.  BD (solve_bd) = 1 up to N = 639, 2 up to 1150, 4 up to 2172, then 2 up to
// 4606, then 1 (small problems want many short chains; the chunk a thread holds must fit in
// registers).
//
// Within a workgroup, thread (c, d) owns C consecutive virtual rows of lane d in registers.
// Each sweep is a first-order linear recurrence, solved as: local sweep of every chunk with a
// zero carry, a scan over the chunks of each lane of their affine maps x -> G x + Y (G the
// product of the chunk's factors, Y its zero-carry result), then a local fix-up with the
// scanned carry.
//   forward:  y_k = b_k - l_k y_{k-1}            (l_k: multiplier met at entry k)
//             z_k = y_k / D_k
//   backward: x_k = z_k - l_{k+1} x_{k+1}
// The lower triangle gets -x (the Laplacian is -Delta^m on diagonal m), the upper conj(x)
// (P skew-Hermitian).  The multipliers satisfy |l| <= 1, so the chunk products stay bounded.
//
// Diagonal m = 0 is singular (pseudo-inverse): lane 0 of band 0 removes tr(W)/N from its
// right-hand side first, its factors cover the leading (N-1) block only (1/D = 0 on the last
// entry, so x_{N-1} = 0), and the mean of x is subtracted at the end.
//
// XCD-aware order: the hardware sends workgroup b to XCD b % 8; workgroups are renumbered so
// that each XCD takes a contiguous range of bands: neighbouring bands write the other halves of
// the same cache lines.

#include <cmath>
#include <vector>

#include "solve_wg.h"

namespace {

using namespace zk;

template <int T, int C, int BD>
__global__ __launch_bounds__(T) void stream_solve_kernel(const double2* __restrict__ W,
                                                         double2* __restrict__ P,
                                                         const double* __restrict__ fl,
                                                         const double* __restrict__ fd,
                                                         int N, int nwg, int per,
                                                         const int* __restrict__ skip) {
    __shared__ double sG[T];
    __shared__ double2 sY[T];
    if (skip && *skip) return;  // on-device stopping: the step has converged
    const int b = blockIdx.x;
    const int w = (b & 7) * per + (b >> 3);
    if (w >= nwg) return;  // uniform for the block
    solve_band<T, C, BD>(W, P, fl, fd, N, w, sG, sY);
}

template <int T, int C, int BD>
hipError_t launch_tc(const ze_ctx* c, const double2* W, double2* P, hipStream_t s, const int* skip) {
    const int N = c->N;
    static_assert(T % BD == 0, "lanes");
    const int nwg = solve_bands(N, BD);
    const int per = (nwg + 7) / 8;
    hipLaunchKernelGGL((stream_solve_kernel<T, C, BD>), dim3(8 * per), dim3(T), 0, s, W, P,
                       c->fac_l, c->fac_dinv, N, nwg, per, skip);
    return hipGetLastError();
}

// LDL^T factors of Delta^m (host, FP64): L[i] = multiplier met at entry i (0 at i = 0),
// Dinv[i] = 1 / D_i.  Delta^m: d_i = 2 (s (2i+1+m) - i (i+m)),
// e_i = -sqrt((i+m+1)(N-1-i-m)) sqrt((i+1)(N-1-i)); m = 0: leading (N-1) block only.
void factor_diagonal(int N, int m, std::vector<double>& L, std::vector<double>& Dinv) {
    const int n = N - m;
    const int nf = (m == 0) ? n - 1 : n;
    const double s = 0.5 * (N - 1);
    L.assign(n, 0.0);
    Dinv.assign(n, 0.0);
    double Dp = 0.0;
    for (int i = 0; i < nf; ++i) {
        const double d = 2.0 * (s * (2.0 * i + 1.0 + m) - (double)i * (double)(i + m));
        double D;
        if (i == 0) {
            D = d;
        } else {
            const double k = i - 1;
            const double e = -std::sqrt((k + m + 1.0) * (N - 1.0 - k - m)) *
                             std::sqrt((k + 1.0) * (N - 1.0 - k));
            L[i] = e / Dp;
            D = d - L[i] * e;
        }
        Dinv[i] = 1.0 / D;
        Dp = D;
    }
}

}  // namespace

// Factors in the (band, virtual row, lane) order of solve_band with bd lanes per band; zero
// where a lane has no entry.
void ze_build_factors(int N, int bd, std::vector<double>& fl, std::vector<double>& fd) {
    const int K = solve_bands(N, bd), R = solve_rows(N, bd);
    const size_t tot = (size_t)K * R * bd;
    fl.assign(tot, 0.0);
    fd.assign(tot, 0.0);
    std::vector<double> L, Dv;
    for (int k = 0; k < K; ++k)
        for (int d = 0; d < bd; ++d) {
            const int m = k * bd + d, mp = N - 1 - m;
            const size_t base = (size_t)k * R * bd + d;
            if (m < N) {  // main: entry i on virtual row i + m + bd
                factor_diagonal(N, m, L, Dv);
                for (int i = 0; i < N - m; ++i) {
                    const size_t at = base + (size_t)(i + m + bd) * bd;
                    fl[at] = L[i];
                    fd[at] = Dv[i];
                }
            }
            if (mp >= K * bd) {  // partner: entry i on virtual row i - 1 - d + bd
                factor_diagonal(N, mp, L, Dv);
                for (int i = 0; i < N - mp; ++i) {
                    const size_t at = base + (size_t)(i - 1 - d + bd) * bd;
                    fl[at] = L[i];
                    fd[at] = Dv[i];
                }
            }
        }
}

// The (threads, rows per chunk) shape for N and the context's band width:
// (T / BD) C >= N + BD, C <= 17.
hipError_t launch_stream_solve(const ze_ctx* c, const double2* W, double2* P, hipStream_t s,
                               const int* skip) {
    const int N = c->N;
    if (c->solve_bd == 4) {
        if (N <= 76) return launch_tc<64, 5, 4>(c, W, P, s, skip);
        if (N <= 156) return launch_tc<128, 5, 4>(c, W, P, s, skip);
        if (N <= 316) return launch_tc<256, 5, 4>(c, W, P, s, skip);
        if (N <= 572) return launch_tc<256, 9, 4>(c, W, P, s, skip);
        if (N <= 1084) return launch_tc<256, 17, 4>(c, W, P, s, skip);
        if (N <= 2172) return launch_tc<512, 17, 4>(c, W, P, s, skip);
        return hipErrorInvalidValue;  // band width 4 is only chosen up to N = 2172
    }
    if (c->solve_bd == 2) {
        if (N <= 1150) return launch_tc<256, 9, 2>(c, W, P, s, skip);
        if (N <= 4606) return launch_tc<1024, 9, 2>(c, W, P, s, skip);
        return hipErrorInvalidValue;  // band width 2 is only chosen up to N = 4606
    }
    if (N <= 191) return launch_tc<64, 3, 1>(c, W, P, s, skip);
    if (N <= 383) return launch_tc<128, 3, 1>(c, W, P, s, skip);
    if (N <= 639) return launch_tc<128, 5, 1>(c, W, P, s, skip);
    if (N <= 9215) return launch_tc<1024, 9, 1>(c, W, P, s, skip);
    return launch_tc<1024, 17, 1>(c, W, P, s, skip);
}

// Stream solve P = Delta_N^+ W: one tridiagonal system per matrix diagonal (Sec. 3.3,
// eq. (sub_tria_W)), with the LDL^T factors of the blocks Delta^m of eq. (delta_tria).
//
// Work split.  Diagonal m has N - m entries, so diagonals m and N - m together have exactly
// N; workgroup w >= 1 solves that pair (w = m), workgroup 0 solves m = 0 alone and, for even
// N, workgroup N/2 the single middle diagonal.  The pair is laid out as one "virtual" array
// of length L <= N, diagonal m first: element k is (m, i = k) for k < N - m, else
// (N - m, i = k - (N - m)).  The factors are stored in the same order, so each workgroup
// reads its factors contiguously; the multiplier stored at the first element of each
// diagonal is 0, which keeps the two recurrences apart.
//
// Within a workgroup, thread t owns the chunk k = t*C .. t*C + C - 1 in registers.  Each
// sweep is a first-order linear recurrence, solved as: local sweep of every chunk with a
// zero carry, a block scan of the chunks' affine maps x -> G x + Y (G the product of the
// chunk's factors, Y its zero-carry result), then a local fix-up with the scanned carry.
//   forward:  y_k = b_k - l_k y_{k-1}            (l_k: multiplier met at element k)
//             z_k = y_k / D_k
//   backward: x_k = z_k - l_{k+1} x_{k+1}
// The lower triangle gets -x (the Laplacian is -Delta^m on diagonal m), the upper conj(x)
// (P skew-Hermitian).  The multipliers satisfy |l| <= 1, so the chunk products stay bounded.
//
// Diagonal m = 0 is singular (pseudo-inverse): workgroup 0 removes tr(W)/N from the
// right-hand side first, its factors cover the leading (N-1) block only (1/D = 0 on the last
// element, so x_{N-1} = 0), and the mean of x is subtracted at the end.
//
// XCD-aware order: the hardware sends workgroup b to XCD b % 8; workgroups are renumbered so
// that each XCD takes a contiguous range of pairs.  Neighbouring diagonals touch neighbouring
// entries of the same matrix rows, so their scattered accesses meet in the XCD's L2.

#include <cmath>
#include <vector>

#include "solve_wg.h"

namespace {

using namespace zk;

template <int T, int C>
__global__ __launch_bounds__(T) void stream_solve_kernel(const double2* __restrict__ W,
                                                         double2* __restrict__ P,
                                                         const double* __restrict__ fl,
                                                         const double* __restrict__ fd,
                                                         int N, int nwg, int per) {
    __shared__ double sG[T];
    __shared__ double2 sY[T];
    const int b = blockIdx.x;
    const int w = (b & 7) * per + (b >> 3);
    if (w >= nwg) return;  // uniform for the block
    solve_pair<T, C>(W, P, fl, fd, N, w, sG, sY);
}

template <int T, int C>
hipError_t launch_tc(const ze_ctx* c, const double2* W, double2* P, hipStream_t s) {
    const int N = c->N;
    const int nwg = N / 2 + 1;
    const int per = (nwg + 7) / 8;
    hipLaunchKernelGGL((stream_solve_kernel<T, C>), dim3(8 * per), dim3(T), 0, s, W, P, c->fac_l,
                       c->fac_dinv, N, nwg, per);
    return hipGetLastError();
}

}  // namespace

// Factors in the workgroup order described above (host, FP64).  Delta^m:
// d_i = 2 (s (2i+1+m) - i (i+m)), e_i = -sqrt((i+m+1)(N-1-i-m)) sqrt((i+1)(N-1-i)).
void ze_build_factors(int N, std::vector<double>& fl, std::vector<double>& fd) {
    const size_t tot = (size_t)N * (N + 1) / 2;
    fl.assign(tot, 0.0);
    fd.assign(tot, 0.0);
    const double s = 0.5 * (N - 1);
    std::vector<double> D(N), Lm(N);
    auto factor = [&](int m, size_t at) {
        const int n = N - m;
        const int nf = (m == 0) ? n - 1 : n;  // m = 0: leading (N-1) block only
        for (int i = 0; i < nf; ++i) {
            const double d = 2.0 * (s * (2.0 * i + 1.0 + m) - (double)i * (double)(i + m));
            if (i == 0) {
                D[0] = d;
            } else {
                const double k = i - 1;
                const double e = -std::sqrt((k + m + 1.0) * (N - 1.0 - k - m)) *
                                 std::sqrt((k + 1.0) * (N - 1.0 - k));
                Lm[i - 1] = e / D[i - 1];
                D[i] = d - Lm[i - 1] * e;
            }
            fl[at + i] = (i == 0) ? 0.0 : Lm[i - 1];
            fd[at + i] = 1.0 / D[i];
        }
    };
    factor(0, 0);
    for (int w = 1; w <= N / 2; ++w) {
        factor(w, (size_t)w * N);
        if (N - w != w && N - w < N) factor(N - w, (size_t)w * N + (N - w));
    }
}

hipError_t launch_stream_solve(const ze_ctx* c, const double2* W, double2* P, hipStream_t s) {
    const int N = c->N;
    if (N <= 64) return launch_tc<64, 1>(c, W, P, s);
    if (N <= 128) return launch_tc<128, 1>(c, W, P, s);
    if (N <= 256) return launch_tc<256, 1>(c, W, P, s);
    if (N <= 512) return launch_tc<256, 2>(c, W, P, s);
    if (N <= 1024) return launch_tc<256, 4>(c, W, P, s);
    if (N <= 2048) return launch_tc<256, 8>(c, W, P, s);
    if (N <= 4096) return launch_tc<256, 16>(c, W, P, s);
    if (N <= 8192) return launch_tc<512, 16>(c, W, P, s);
    return launch_tc<1024, 16>(c, W, P, s);
}

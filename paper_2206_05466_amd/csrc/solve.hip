// Stream solve P = Delta_N^+ W: one tridiagonal system per matrix diagonal (Sec. 3.3,
// eq. (sub_tria_W)), with the LDL^T factors of the blocks Delta^m of eq. (delta_tria).
//
// Layout and parallelisation.  Lane m of the grid owns diagonal m (entries (i+m, i)).  The
// sweeps advance row by row: at row t every active lane m handles its element i = t - m,
// i.e. entry (t, t - m), so the 64 lanes of a wave read 64 neighbouring entries of one
// matrix row -- a coalesced access -- and the packed factors are stored in the same
// row-major lower-triangle order.  Forward sweep (rows ascending): y_i = b_i - l_{i-1} y_{i-1},
// z_i = y_i / D_i, with z kept in P as scratch.  Backward sweep (rows descending):
// x_i = z_i - l_i x_{i+1}; the lower triangle gets -x (the Laplacian is -Delta^m on diagonal
// m), the upper triangle conj(x) (P skew-Hermitian).
//
// Diagonal m = 0 (singular block, pseudo-inverse): the factors cover only the leading
// (N-1) block and zero the last element, so the sweeps return x_raw = B^{-1} b[0..N-2]
// (x_raw[N-1] = 0) for the raw right-hand side; lane 0 also sums tr = sum_i b_i and
// sum_i x_raw_i.  The fix-up kernel then applies, by linearity,
//   x = x_raw - (tr/N) ubar - mean(x_raw),    ubar = B^{-1} 1 - mean(B^{-1} 1),
// which equals removing tr/N from the right-hand side and subtracting the mean.

#include "internal.h"

namespace {

constexpr int kSolveLanes = 64;

__global__ __launch_bounds__(kSolveLanes) void stream_solve_kernel(
    const double2* __restrict__ W, double2* __restrict__ P, const double* __restrict__ fl,
    const double* __restrict__ fd, int N, double2* __restrict__ diagstat) {
    const int m0 = blockIdx.x * kSolveLanes;
    const int m = m0 + threadIdx.x;
    const bool lane_ok = m < N;
    const size_t ldN = (size_t)N;

    // Forward sweep.
    double yr = 0.0, yi = 0.0, tr_r = 0.0, tr_i = 0.0;
    for (int t = m0; t < N; ++t) {
        if (lane_ok && m <= t) {
            const int i = t - m;
            const size_t off = (size_t)t * ldN + i;
            const size_t po = tri_off(t, i);
            const double2 b = W[off];
            const double l = fl[po];
            const double dv = fd[po];
            yr = b.x - l * yr;
            yi = b.y - l * yi;
            P[off] = make_double2(yr * dv, yi * dv);
            if (m == 0) {
                tr_r += b.x;
                tr_i += b.y;
            }
        }
    }

    // Backward sweep.
    double xr = 0.0, xi = 0.0, lnext = 0.0, sx_r = 0.0, sx_i = 0.0;
    for (int t = N - 1; t >= m0; --t) {
        if (lane_ok && m <= t) {
            const int i = t - m;
            const size_t off = (size_t)t * ldN + i;
            const double2 z = P[off];
            xr = z.x - lnext * xr;
            xi = z.y - lnext * xi;
            lnext = fl[tri_off(t, i)];
            P[off] = make_double2(-xr, -xi);
            if (m > 0) {
                P[(size_t)i * ldN + t] = make_double2(xr, -xi);
            } else {
                sx_r += xr;
                sx_i += xi;
            }
        }
    }
    if (m == 0) {
        diagstat[0] = make_double2(tr_r, tr_i);
        diagstat[1] = make_double2(sx_r, sx_i);
    }
}

__global__ __launch_bounds__(256) void stream_solve_diag_fixup(double2* __restrict__ P,
                                                                const double* __restrict__ ubar,
                                                                const double2* __restrict__ diagstat,
                                                                int N) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double invN = 1.0 / (double)N;
    const double2 tr = diagstat[0];
    const double2 sx = diagstat[1];
    const double u = ubar[i];
    double2 p = P[(size_t)i * N + i];  // holds -x_raw_i
    p.x += tr.x * invN * u + sx.x * invN;
    p.y += tr.y * invN * u + sx.y * invN;
    P[(size_t)i * N + i] = p;
}

}  // namespace

hipError_t launch_stream_solve(const ze_ctx* c, const double2* W, double2* P, hipStream_t s) {
    const int N = c->N;
    const int nb = (N + kSolveLanes - 1) / kSolveLanes;
    hipLaunchKernelGGL(stream_solve_kernel, dim3(nb), dim3(kSolveLanes), 0, s, W, P, c->fac_l,
                       c->fac_dinv, N, c->diagstat);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stream_solve_diag_fixup, dim3((N + 255) / 256), dim3(256), 0, s, P,
                       c->ubar, c->diagstat, N);
    return hipGetLastError();
}

// Elementwise kernels of the step driver.

#include "internal.h"

namespace {

// F <- W + rho (W - F): the starting iterate of a step extrapolated from the previous step's
// converged midpoint F (W~ approximates W half a step ahead; rho = this step's h over the
// previous one's, and rho = 1 is evaluated as 2 W - F).  Exact skew-Hermitian inputs give an
// exact skew-Hermitian result.
__global__ __launch_bounds__(256) void extrapolate_kernel(const double2* __restrict__ W,
                                                          double2* __restrict__ F, size_t n,
                                                          double rho) {
    const bool unit = rho == 1.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        const double2 w = W[e], f = F[e];
        F[e] = unit ? make_double2(2.0 * w.x - f.x, 2.0 * w.y - f.y)
                    : make_double2(w.x + rho * (w.x - f.x), w.y + rho * (w.y - f.y));
    }
}

// out <- sum_j c_j F_j over the d + 1 newest midpoints F_1 (newest), F_2, ...: the polynomial
// of degree d through them evaluated one step ahead (Newton's forward differences; c = (2, -1),
// (3, -3, 1), (4, -6, 4, -1)), summed in that order.  out may be the oldest input: every entry
// is read before it is written, by the same thread.
__global__ __launch_bounds__(256) void extrapolate_poly_kernel(const double2* F1, const double2* F2,
                                                               const double2* F3, const double2* F4,
                                                               double2* out, size_t n, int d) {
    const double c1 = d + 1.0;
    const double c2 = d == 1 ? -1.0 : (d == 2 ? -3.0 : -6.0);
    const double c3 = d == 2 ? 1.0 : 4.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        const double2 f1 = F1[e], f2 = F2[e];
        double2 o = make_double2(c1 * f1.x, c1 * f1.y);
        o = make_double2(o.x + c2 * f2.x, o.y + c2 * f2.y);
        if (d >= 2) {
            const double2 f3 = F3[e];
            o = make_double2(o.x + c3 * f3.x, o.y + c3 * f3.y);
        }
        if (d >= 3) {
            const double2 f4 = F4[e];
            o = make_double2(o.x - f4.x, o.y - f4.y);
        }
        out[e] = o;
    }
}

// out <- sum_i c_i src_i over m <= kLinCombMax matrices, added in index order (each entry read
// before it is written, by the same thread).
struct LinComb {
    const double2* src[kLinCombMax];
    double c[kLinCombMax];
    int m;
};

__global__ __launch_bounds__(256) void lincomb_kernel(LinComb lc, double2* out, size_t n) {
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        double2 o = make_double2(0.0, 0.0);
        for (int i = 0; i < lc.m; ++i) {
            const double2 v = lc.src[i][e];
            o = make_double2(o.x + lc.c[i] * v.x, o.y + lc.c[i] * v.y);
        }
        out[e] = o;
    }
}

// Input check of W: block b takes the 32 x 32 tile pair (I, J), (J, I), I >= J, of the lower
// triangle of tiles, staged in LDS so both are read row-wise, and writes part[4 b ..]: the
// largest |W_rc + conj(W_cr)| of the pair, the largest |W_rc| of both tiles, and (diagonal
// tiles only, else 0) the real and imaginary parts of the tile's trace, summed in a fixed order.
constexpr int kVT = 32;
__global__ __launch_bounds__(256) void su_check_kernel(const double2* __restrict__ W, int N,
                                                      double* __restrict__ part) {
    __shared__ double2 ta[kVT][kVT + 1], tb[kVT][kVT + 1];
    __shared__ double r0[256], r1[256], r2[256], r3[256];
    const int b = blockIdx.x, tid = threadIdx.x;
    int I = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    const int J = b - I * (I + 1) / 2;
    const int c = tid & 31;
    for (int r = tid >> 5; r < kVT; r += 8) {
        const int ra = I * kVT + r, ca = J * kVT + c, rb = J * kVT + r, cb = I * kVT + c;
        ta[r][c] = (ra < N && ca < N) ? W[(size_t)ra * N + ca] : make_double2(0.0, 0.0);
        tb[r][c] = (rb < N && cb < N) ? W[(size_t)rb * N + cb] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double asym = 0.0, amax = 0.0, tre = 0.0, tim = 0.0;
    for (int r = tid >> 5; r < kVT; r += 8) {
        const double2 x = ta[r][c], y = tb[c][r], z = tb[r][c];  // y = W_cr for x = W_rc
        const double dx = x.x + y.x, dy = x.y - y.y;             // W_rc + conj(W_cr)
        const double d = sqrt(dx * dx + dy * dy);
        asym = (d != d || d > asym) ? d : asym;
        const double m = fmax(sqrt(x.x * x.x + x.y * x.y), sqrt(z.x * z.x + z.y * z.y));
        amax = (m != m || m > amax) ? m : amax;
        if (I == J && r == c) {
            tre += x.x;
            tim += x.y;
        }
    }
    r0[tid] = asym;
    r1[tid] = amax;
    r2[tid] = tre;
    r3[tid] = tim;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            const double a0 = r0[tid + s], a1 = r1[tid + s];
            r0[tid] = (a0 != a0 || a0 > r0[tid]) ? a0 : r0[tid];
            r1[tid] = (a1 != a1 || a1 > r1[tid]) ? a1 : r1[tid];
            r2[tid] += r2[tid + s];
            r3[tid] += r3[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        part[4 * (size_t)b] = r0[0];
        part[4 * (size_t)b + 1] = r1[0];
        part[4 * (size_t)b + 2] = r2[0];
        part[4 * (size_t)b + 3] = r3[0];
    }
}

// out[0..3] = the maxima and sums of su_check_kernel over its G blocks (fixed order).
__global__ __launch_bounds__(256) void su_check_final(const double* __restrict__ part, int G,
                                                     double* __restrict__ out) {
    __shared__ double r0[256], r1[256], r2[256], r3[256];
    const int tid = threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int b = tid; b < G; b += 256) {
        const double p0 = part[4 * (size_t)b], p1 = part[4 * (size_t)b + 1];
        a0 = (p0 != p0 || p0 > a0) ? p0 : a0;
        a1 = (p1 != p1 || p1 > a1) ? p1 : a1;
        a2 += part[4 * (size_t)b + 2];
        a3 += part[4 * (size_t)b + 3];
    }
    r0[tid] = a0;
    r1[tid] = a1;
    r2[tid] = a2;
    r3[tid] = a3;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            const double b0 = r0[tid + s], b1 = r1[tid + s];
            r0[tid] = (b0 != b0 || b0 > r0[tid]) ? b0 : r0[tid];
            r1[tid] = (b1 != b1 || b1 > r1[tid]) ? b1 : r1[tid];
            r2[tid] += r2[tid + s];
            r3[tid] += r3[tid + s];
        }
        __syncthreads();
    }
    if (tid < 4) out[tid] = tid == 0 ? r0[0] : tid == 1 ? r1[0] : tid == 2 ? r2[0] : r3[0];
}

// ---------------------------------------------------------------- on-device stopping
// Control words: see kCtlWords in internal.h.  NaN-propagating maximum.
__device__ __forceinline__ double nanmax(double a, double o) { return (o != o || o > a) ? o : a; }

// Run start: the run's totals and the first step's fields cleared.  Every later step and
// substep starts from the fields the end of the previous one cleared.
__global__ __launch_bounds__(64) void ctl_run_begin_kernel(int* ctl, double* ctld) {
    if (threadIdx.x == 0) {
        for (int w = 0; w <= 7; ++w) ctl[w] = 0;
        ctl[9] = 0;
        ctld[0] = 0.0;
        ctld[1] = 0.0;
    }
}

// Substep end: its count and residual into the step's; the done flag and the substep's count
// cleared for the next substep; last: the step's record written at its index, the run totals
// updated and the step's fields cleared for the next step.
__global__ __launch_bounds__(64) void ctl_substep_end_kernel(int* ctl, double* ctld,
                                                             const double* __restrict__ resid,
                                                             double tol, int last, int* step_it,
                                                             double* step_r) {
    if (threadIdx.x != 0) return;
    const double r = resid[0];
    ctl[2] += ctl[1];
    ctld[0] = nanmax(ctld[0], r);
    if (!(r < tol)) ctl[3] |= 1;
    if (!isfinite(r)) ctl[3] |= 2;
    ctl[0] = 0;
    ctl[1] = 0;
    if (!last) return;
    const int n = ctl[9];
    step_it[n % kDevSteps] = ctl[2];
    step_r[n % kDevSteps] = ctld[0];
    if (ctl[3] & 1) ctl[4] += 1;
    if (ctl[3] & 2) ctl[5] += 1;
    ctl[6] += ctl[2];
    ctl[7] = ctl[2] > ctl[7] ? ctl[2] : ctl[7];
    ctld[1] = nanmax(ctld[1], ctld[0]);
    ctl[9] = n + 1;
    ctl[2] = 0;
    ctl[3] = 0;
    ctld[0] = 0.0;
}

__global__ __launch_bounds__(256) void copy_kernel(const double2* __restrict__ src,
                                                   double2* __restrict__ dst, size_t n) {
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256)
        dst[e] = src[e];
}

}  // namespace

int ze_su_check_blocks(int N) {
    const int T = (N + kVT - 1) / kVT;
    return T * (T + 1) / 2;
}

hipError_t launch_su_check(const double2* W, int N, double* part, double* out, hipStream_t s) {
    const int G = ze_su_check_blocks(N);
    hipLaunchKernelGGL(su_check_kernel, dim3(G), dim3(256), 0, s, W, N, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(su_check_final, dim3(1), dim3(256), 0, s, part, G, out);
    return hipGetLastError();
}

hipError_t launch_extrapolate_poly(const double2* const* Fs, int d, double2* out, int N,
                                   hipStream_t s) {
    if (d < 1 || d > 3) return hipErrorInvalidValue;
    const size_t n = (size_t)N * N;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(extrapolate_poly_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)),
                       dim3(256), 0, s, Fs[0], Fs[1], d >= 2 ? Fs[2] : nullptr,
                       d >= 3 ? Fs[3] : nullptr, out, n, d);
    return hipGetLastError();
}

hipError_t launch_lincomb(const double2* const* src, const double* coef, int m, double2* out, int N,
                          hipStream_t s) {
    if (m < 1 || m > kLinCombMax) return hipErrorInvalidValue;
    LinComb lc{};
    for (int i = 0; i < m; ++i) {
        lc.src[i] = src[i];
        lc.c[i] = coef[i];
    }
    lc.m = m;
    const size_t n = (size_t)N * N;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(lincomb_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0,
                       s, lc, out, n);
    return hipGetLastError();
}

hipError_t launch_extrapolate(const double2* W, double2* F, int N, double rho, hipStream_t s) {
    const size_t n = (size_t)N * N;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(extrapolate_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256),
                       0, s, W, F, n, rho);
    return hipGetLastError();
}

hipError_t launch_ctl_run_begin(int* ctl, double* ctld, hipStream_t s) {
    hipLaunchKernelGGL(ctl_run_begin_kernel, dim3(1), dim3(64), 0, s, ctl, ctld);
    return hipGetLastError();
}

hipError_t launch_copy(const double2* src, double2* dst, int N, hipStream_t s) {
    const size_t n2 = (size_t)N * N;
    const size_t blocks = (n2 + 255) / 256;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0,
                       s, src, dst, n2);
    return hipGetLastError();
}

hipError_t launch_ctl_substep_end(int* ctl, double* ctld, const double* resid, double tol, bool last,
                                  int* step_it, double* step_r, hipStream_t s) {
    hipLaunchKernelGGL(ctl_substep_end_kernel, dim3(1), dim3(64), 0, s, ctl, ctld, resid, tol,
                       last ? 1 : 0, step_it, step_r);
    return hipGetLastError();
}

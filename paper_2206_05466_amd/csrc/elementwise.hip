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

}  // namespace

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

hipError_t launch_extrapolate(const double2* W, double2* F, int N, double rho, hipStream_t s) {
    const size_t n = (size_t)N * N;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(extrapolate_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256),
                       0, s, W, F, n, rho);
    return hipGetLastError();
}

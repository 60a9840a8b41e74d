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

}  // namespace

hipError_t launch_extrapolate(const double2* W, double2* F, int N, double rho, hipStream_t s) {
    const size_t n = (size_t)N * N;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(extrapolate_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256),
                       0, s, W, F, n, rho);
    return hipGetLastError();
}

// FP64 trace reductions for the Casimirs C_k(W) = Tr(W^k) (eq. (W_pow)):
// Tr(X Y) = sum_ij X_ij Y_ji over 32 x 32 tiles (Y's tile transposed through LDS so both
// operands are read row-coalesced), block partials written to a buffer and summed by one
// block in a fixed order (deterministic).

#include "internal.h"

namespace {

constexpr int kT = 32;

__global__ __launch_bounds__(256) void trace_product_partial(const double2* __restrict__ X,
                                                             const double2* __restrict__ Y,
                                                             double2* __restrict__ partial, int N) {
    __shared__ double2 ys[kT][kT + 1];
    __shared__ double2 red[256];
    const int i0 = blockIdx.y * kT, j0 = blockIdx.x * kT;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    // ys[a][b] = Y[j0 + a][i0 + b]
    for (int a = ty; a < kT; a += 8) {
        const int r = j0 + a, c = i0 + tx;
        ys[a][tx] = (r < N && c < N) ? Y[(size_t)r * N + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double sr = 0.0, si = 0.0;
    for (int a = ty; a < kT; a += 8) {
        const int i = i0 + a, j = j0 + tx;
        if (i < N && j < N) {
            const double2 x = X[(size_t)i * N + j];
            const double2 y = ys[tx][a];  // Y[j][i]
            sr += x.x * y.x - x.y * y.y;
            si += x.x * y.y + x.y * y.x;
        }
    }
    red[threadIdx.x] = make_double2(sr, si);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x].x += red[threadIdx.x + s].x;
            red[threadIdx.x].y += red[threadIdx.x + s].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void trace_diag_partial(const double2* __restrict__ X,
                                                          double2* __restrict__ partial, int N) {
    __shared__ double2 red[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    red[threadIdx.x] = i < N ? X[(size_t)i * N + i] : make_double2(0.0, 0.0);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x].x += red[threadIdx.x + s].x;
            red[threadIdx.x].y += red[threadIdx.x + s].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void sum_partials(const double2* __restrict__ partial, int G,
                                                    double2* __restrict__ out) {
    __shared__ double2 red[256];
    double sr = 0.0, si = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) {
        sr += partial[i].x;
        si += partial[i].y;
    }
    red[threadIdx.x] = make_double2(sr, si);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x].x += red[threadIdx.x + s].x;
            red[threadIdx.x].y += red[threadIdx.x + s].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

int ze_trace_partials(int N) {
    const int t = (N + kT - 1) / kT;
    return t * t;
}

hipError_t launch_trace_product(const double2* X, const double2* Y, double2* partial,
                                double2* out, int N, hipStream_t s) {
    const int t = (N + kT - 1) / kT;
    hipLaunchKernelGGL(trace_product_partial, dim3(t, t), dim3(256), 0, s, X, Y, partial, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, s, partial, t * t, out);
    return hipGetLastError();
}

hipError_t launch_trace(const double2* X, double2* partial, double2* out, int N, hipStream_t s) {
    const int g = (N + 255) / 256;
    hipLaunchKernelGGL(trace_diag_partial, dim3(g), dim3(256), 0, s, X, partial, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, s, partial, g, out);
    return hipGetLastError();
}

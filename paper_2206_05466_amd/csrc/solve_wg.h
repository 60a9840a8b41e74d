// Device building blocks of the stream solve (shared by the single-problem and the ensemble
// kernels).  See solve.hip for the method.
#pragma once

#include "internal.h"

namespace zk {

template <int T>
__device__ __forceinline__ void block_scan_affine(double& G, double2& Y, bool reverse, double* sG,
                                         double2* sY) {
    // Inclusive scan over threads (in reverse thread order if `reverse`) of the affine maps
    // f_t(x) = G_t x + Y_t composed in scan order: earlier maps are applied first.
    const int t = threadIdx.x;
    for (int off = 1; off < T; off <<= 1) {
        sG[t] = G;
        sY[t] = Y;
        __syncthreads();
        const int src = reverse ? t + off : t - off;
        if (src >= 0 && src < T) {
            const double pg = sG[src];
            const double2 py = sY[src];
            Y.x += G * py.x;
            Y.y += G * py.y;
            G *= pg;
        }
        __syncthreads();
    }
}

template <int T>
__device__ __forceinline__ double2 block_sum(double2 v, double2* s) {
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int h = T / 2; h > 0; h >>= 1) {
        if (t < h) {
            s[t].x += s[t + h].x;
            s[t].y += s[t + h].y;
        }
        __syncthreads();
    }
    const double2 r = s[0];
    __syncthreads();
    return r;
}

// Solves the diagonal pair of workgroup w (see solve.hip) for an N x N problem.
template <int T, int C>
__device__ __forceinline__ void solve_pair(const double2* __restrict__ W, double2* __restrict__ P,
                                  const double* __restrict__ fl, const double* __restrict__ fd,
                                  int N, int w, double* sG, double2* sY) {
    int m1, n1, m2;
    if (w == 0) {
        m1 = 0;
        n1 = N;
        m2 = -1;
    } else {
        m1 = w;
        n1 = N - w;
        m2 = (N - w != w) ? N - w : -1;
    }
    const int L = n1 + (m2 >= 0 ? w : 0);
    const size_t base = (size_t)w * N;
    const double* flw = fl + base;
    const double* fdw = fd + base;
    const int t = threadIdx.x;
    const int k0 = t * C;

    auto entry = [&](int k) -> size_t {  // matrix offset of virtual element k
        const int m = k < n1 ? m1 : m2;
        const int i = k < n1 ? k : k - n1;
        return (size_t)(i + m) * N + i;
    };

    double2 v[C];
    double l[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int k = k0 + c;
        if (k < L) {
            v[c] = W[entry(k)];
            l[c] = flw[k];
        } else {
            v[c] = make_double2(0.0, 0.0);
            l[c] = 0.0;
        }
    }

    if (w == 0) {  // trace removal on the singular block (all L = N elements are diagonal 0)
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            s.x += v[c].x;
            s.y += v[c].y;
        }
        const double2 tr = block_sum<T>(s, sY);
        const double ir = tr.x / N, ii = tr.y / N;
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (k0 + c < L) {
                v[c].x -= ir;
                v[c].y -= ii;
            }
    }

    // Forward sweep: local pass with zero carry.
    double G = 1.0;
    double2 y = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        y.x = v[c].x - l[c] * y.x;
        y.y = v[c].y - l[c] * y.y;
        G *= -l[c];
        v[c] = y;
    }
    double2 Y = y;
    block_scan_affine<T>(G, Y, false, sG, sY);
    sY[t] = Y;  // inclusive: true y at the end of chunk t
    __syncthreads();
    const double2 cin = t > 0 ? sY[t - 1] : make_double2(0.0, 0.0);
    __syncthreads();
    double g = 1.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int k = k0 + c;
        g *= -l[c];
        const double dv = k < L ? fdw[k] : 0.0;
        v[c].x = (v[c].x + g * cin.x) * dv;
        v[c].y = (v[c].y + g * cin.y) * dv;
    }

    // Backward sweep: x_k = z_k - l_{k+1} x_{k+1}; local pass from the chunk end.
    const double lend = (k0 + C < L) ? flw[k0 + C] : 0.0;
    G = 1.0;
    double2 x = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        const double ln = (c == C - 1) ? lend : l[c + 1];
        x.x = v[c].x - ln * x.x;
        x.y = v[c].y - ln * x.y;
        G *= -ln;
        v[c] = x;
    }
    Y = x;
    block_scan_affine<T>(G, Y, true, sG, sY);
    sY[t] = Y;  // inclusive from the right: true x at the start of chunk t
    __syncthreads();
    const double2 cr = t + 1 < T ? sY[t + 1] : make_double2(0.0, 0.0);
    __syncthreads();
    g = 1.0;
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        const double ln = (c == C - 1) ? lend : l[c + 1];
        g *= -ln;
        v[c].x += g * cr.x;
        v[c].y += g * cr.y;
    }

    if (w == 0) {  // minimum-norm solution: subtract the mean
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            s.x += v[c].x;
            s.y += v[c].y;
        }
        const double2 sx = block_sum<T>(s, sY);
        const double mr = sx.x / N, mi = sx.y / N;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            v[c].x -= mr;
            v[c].y -= mi;
        }
    }

#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int k = k0 + c;
        if (k < L) {
            const int m = k < n1 ? m1 : m2;
            const int i = k < n1 ? k : k - n1;
            P[(size_t)(i + m) * N + i] = make_double2(-v[c].x, -v[c].y);
            if (m > 0) P[(size_t)i * N + i + m] = make_double2(v[c].x, -v[c].y);
        }
    }
}


}  // namespace zk

// Device building blocks of the stream solve (shared by the single-problem and the ensemble
// kernels).  See solve.hip for the method.
#pragma once

#include "internal.h"

namespace zk {

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

// ---------------------------------------------------------------- band layout
// Diagonal m is paired with m' = N - 1 - m (together N + 1 entries).  Band k holds the
// "main" diagonals m = k BD + d (lane d = 0..BD-1) and their partners m'.  All entries a band
// touches are placed on virtual rows rho = -BD .. N-1 so that, on every virtual row, the BD
// lanes touch BD neighbouring entries of ONE matrix row:
//   main entry i of diagonal m:      rho = i + m,              matrix (rho, rho - m);
//   partner entry i of diagonal m':  rho = i - 1 - d,          matrix (rho + N - k BD, i);
// so lane d's partner occupies rho in [-1-d, k BD) and its main diagonal rho in [k BD + d, N):
// one chain per lane, partner first, a gap between.  The first entry of each diagonal has
// multiplier 0, which keeps the two recurrences (and the gap) apart.  Mains cover
// [0, K BD), partners the rest; a partner that is itself a main (m' < K BD) is skipped.
// Default band width: a thread holds C <= 17 rows (the launch shapes of solve.hip); wider
// bands mean longer row segments per access, narrower ones more and smaller workgroups with
// shorter chains, which is what the small problems (latency-bound) want.  Measured: 1 lane up
// to N = 639 (N = 512: 5.5 us against 7.9 with 4 lanes), 2 up to 1150, 4 up to 2172, 2 lanes
// of 9 rows up to 4606, then 1.
__host__ __device__ inline int solve_bd(int N) {
    if (N <= 639) return 1;
    if (N <= 1150) return 2;
    if (N <= 2172) return 4;
    return N <= 4606 ? 2 : 1;
}
__host__ __device__ inline int solve_bands(int N, int bd) { return (N + 2 * bd - 1) / (2 * bd); }
__host__ __device__ inline int solve_rows(int N, int bd) { return N + bd; }  // virtual rows

// Entry of lane d at virtual row v of band k: matrix offset, or -1 for none.
__host__ __device__ inline long long solve_entry(int N, int bd, int K, int k, int d, int v,
                                                 bool* is_main, int* m_out) {
    const int rho = v - bd, m0 = k * bd, m = m0 + d, mp = N - 1 - m;
    if (m < N && rho >= m0 + d) {  // main
        *is_main = true;
        *m_out = m;
        return (long long)rho * N + (rho - m);
    }
    if (mp >= K * bd && rho >= -1 - d && rho < m0) {  // partner
        *is_main = false;
        *m_out = mp;
        return (long long)(rho + N - m0) * N + (rho + 1 + d);
    }
    return -1;
}

// Inclusive scan over the chunks c (threads c * BD + d of one lane d, in order c, or
// reversed) of the affine maps f(x) = G x + Y: earlier maps are applied first.  Within a wave
// by shuffles (no barrier), then across the T / 64 waves through LDS: one barrier.
template <int T, int BD>
__device__ __forceinline__ void lane_scan_affine(double& G, double2& Y, bool reverse, double* sG,
                                                 double2* sY) {
    constexpr int CW = 64 / BD;  // chunks per wave
    constexpr int NW = T / 64;   // waves
    const int t = threadIdx.x, l = t & 63, w = t >> 6, cw = l / BD;
#pragma unroll
    for (int off = 1; off < CW; off <<= 1) {
        const int sh = off * BD;
        const double pg = reverse ? __shfl_down(G, sh, 64) : __shfl_up(G, sh, 64);
        const double px = reverse ? __shfl_down(Y.x, sh, 64) : __shfl_up(Y.x, sh, 64);
        const double py = reverse ? __shfl_down(Y.y, sh, 64) : __shfl_up(Y.y, sh, 64);
        if (reverse ? cw + off < CW : cw >= off) {
            Y.x += G * px;
            Y.y += G * py;
            G *= pg;
        }
    }
    if (NW == 1) return;
    // wave aggregates (last chunk of the wave in scan order), one per lane d
    if (reverse ? cw == 0 : cw == CW - 1) {
        sG[w * BD + (l % BD)] = G;
        sY[w * BD + (l % BD)] = Y;
    }
    __syncthreads();
    // compose the aggregates of the waves before this one (in scan order), nearest first
    double pg = 1.0;
    double2 py = make_double2(0.0, 0.0);
    const int d = l % BD;
    if (reverse) {
        for (int v = w + 1; v < NW; ++v) {  // p <- p o agg(v)
            const double ag = sG[v * BD + d];
            const double2 ay = sY[v * BD + d];
            py.x += pg * ay.x;
            py.y += pg * ay.y;
            pg *= ag;
        }
    } else {
        for (int v = w - 1; v >= 0; --v) {
            const double ag = sG[v * BD + d];
            const double2 ay = sY[v * BD + d];
            py.x += pg * ay.x;
            py.y += pg * ay.y;
            pg *= ag;
        }
    }
    Y.x += G * py.x;
    Y.y += G * py.y;
    G *= pg;
    __syncthreads();  // sG / sY are reused right after
}

// Stream solve of band k (BD lanes, T / BD chunks of C virtual rows each) of an N x N problem.
// Every global access is a run of BD neighbouring complex entries of one matrix row.
template <int T, int C, int BD>
__device__ __forceinline__ void solve_band(const double2* __restrict__ W, double2* __restrict__ P,
                                           const double* __restrict__ fl,
                                           const double* __restrict__ fd, int N, int k,
                                           double* sG, double2* sY) {
    const int K = solve_bands(N, BD), R = solve_rows(N, BD);
    const int t = threadIdx.x, c = t / BD, d = t % BD;
    const int v0 = c * C;
    const int m0 = k * BD, m = m0 + d, mp = N - 1 - m;
    const bool main_ok = m < N, part_ok = mp >= K * BD;
    const size_t fb = (size_t)k * R * BD + d;  // factor (k, v, d) at fb + v * BD

    double2 x[C];
    double l[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const int v = v0 + j;
        bool im;
        int mm;
        const long long e = v < R ? solve_entry(N, BD, K, k, d, v, &im, &mm) : -1;
        x[j] = e >= 0 ? W[e] : make_double2(0.0, 0.0);
        l[j] = v < R ? fl[fb + (size_t)v * BD] : 0.0;
    }

    const bool sing = (k == 0 && d == 0);  // diagonal 0: pseudo-inverse
    if (k == 0) {  // remove tr(W)/N from diagonal 0's right-hand side (its entries are main)
        double2 sum = make_double2(0.0, 0.0);
        if (sing)
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const int rho = v0 + j - BD;  // lane 0 also holds diagonal N-1 at rho = -1
                if (rho >= 0 && rho < N) {
                    sum.x += x[j].x;
                    sum.y += x[j].y;
                }
            }
        const double2 tr = block_sum<T>(sum, sY);
        if (sing) {
            const double ir = tr.x / N, ii = tr.y / N;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const int rho = v0 + j - BD;
                if (rho >= 0 && rho < N) {
                    x[j].x -= ir;
                    x[j].y -= ii;
                }
            }
        }
    }

    // forward sweep y_v = b_v - l_v y_{v-1}: local pass with zero carry, lane scan, fix-up
    double G = 1.0;
    double2 y = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < C; ++j) {
        y.x = x[j].x - l[j] * y.x;
        y.y = x[j].y - l[j] * y.y;
        G *= -l[j];
        x[j] = y;
    }
    double2 Y = y;
    lane_scan_affine<T, BD>(G, Y, false, sG, sY);
    sY[t] = Y;  // inclusive: true y at the end of chunk c
    __syncthreads();
    const double2 cin = c > 0 ? sY[t - BD] : make_double2(0.0, 0.0);
    __syncthreads();
    double g = 1.0;
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const int v = v0 + j;
        g *= -l[j];
        const double dv = v < R ? fd[fb + (size_t)v * BD] : 0.0;
        x[j].x = (x[j].x + g * cin.x) * dv;
        x[j].y = (x[j].y + g * cin.y) * dv;
    }

    // backward sweep x_v = z_v - l_{v+1} x_{v+1}
    const double lend = (v0 + C < R) ? fl[fb + (size_t)(v0 + C) * BD] : 0.0;
    G = 1.0;
    double2 xx = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = C - 1; j >= 0; --j) {
        const double ln = (j == C - 1) ? lend : l[j + 1];
        xx.x = x[j].x - ln * xx.x;
        xx.y = x[j].y - ln * xx.y;
        G *= -ln;
        x[j] = xx;
    }
    Y = xx;
    lane_scan_affine<T, BD>(G, Y, true, sG, sY);
    sY[t] = Y;  // inclusive from the right: true x at the start of chunk c
    __syncthreads();
    const double2 cr = c + 1 < T / BD ? sY[t + BD] : make_double2(0.0, 0.0);
    __syncthreads();
    g = 1.0;
#pragma unroll
    for (int j = C - 1; j >= 0; --j) {
        const double ln = (j == C - 1) ? lend : l[j + 1];
        g *= -ln;
        x[j].x += g * cr.x;
        x[j].y += g * cr.y;
    }

    if (k == 0) {  // minimum-norm solution on diagonal 0: subtract the mean
        double2 sum = make_double2(0.0, 0.0);
        if (sing)
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const int rho = v0 + j - BD;
                if (rho >= 0 && rho < N) {
                    sum.x += x[j].x;
                    sum.y += x[j].y;
                }
            }
        const double2 sx = block_sum<T>(sum, sY);
        if (sing) {
            const double mr = sx.x / N, mi = sx.y / N;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const int rho = v0 + j - BD;
                if (rho >= 0 && rho < N) {
                    x[j].x -= mr;
                    x[j].y -= mi;
                }
            }
        }
    }

    // lower entries: -x at the entries read (the Laplacian is -Delta^m on diagonal m)
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const int v = v0 + j;
        bool im;
        int mm;
        const long long e = v < R ? solve_entry(N, BD, K, k, d, v, &im, &mm) : -1;
        if (e >= 0) P[e] = make_double2(-x[j].x, -x[j].y);
    }
    // upper entries conj(x), P[i][i + m]: lane d writes its entry j = q + d (main) or
    // j = q - d (partner), which puts the BD lanes of a step on one matrix row
#pragma unroll
    for (int q = -(BD - 1); q < C; ++q) {
        double2 val = make_double2(0.0, 0.0);
        bool have = false;
#pragma unroll
        for (int dd = 0; dd < BD; ++dd) {
            const int j = q + dd;
            if (j >= 0 && j < C && d == dd) {
                val = x[j];
                have = true;
            }
        }
        const int rho = v0 + q + d - BD;
        if (have && main_ok && m > 0 && rho >= m0 + d && rho < N)
            P[(size_t)(rho - m) * N + rho] = make_double2(val.x, -val.y);
    }
#pragma unroll
    for (int q = 0; q < C + BD - 1; ++q) {
        double2 val = make_double2(0.0, 0.0);
        bool have = false;
#pragma unroll
        for (int dd = 0; dd < BD; ++dd) {
            const int j = q - dd;
            if (j >= 0 && j < C && d == dd) {
                val = x[j];
                have = true;
            }
        }
        const int rho = v0 + q - d - BD;
        if (have && part_ok && rho >= -1 - d && rho < m0)
            P[(size_t)(rho + 1 + d) * N + (rho + N - m0)] = make_double2(val.x, -val.y);
    }
}

}  // namespace zk

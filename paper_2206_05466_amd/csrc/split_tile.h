// Device bodies of the split-precision (INT8 MFMA, Ozaki splitting) products, shared by the
// single-problem kernels and the grouped ensemble kernels.  The splitting itself, the slice
// layouts and the exactness bounds are described at the top of gemm_split.hip.
#pragma once

#include "internal.h"

namespace zk {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kSThreads = 256;

__device__ __forceinline__ int exponent_of(double m) {  // smallest e with m < 2^e (0 for m == 0)
    if (!(m > 0.0)) return 0;
    int e;
    frexp(m, &e);
    return e;
}

// Row r of A~ (complex row r of A): scale exponent ea[r] and the s slices (rows of ldk bytes,
// zero padded beyond 2N).  red: kSThreads doubles of LDS.
__device__ __forceinline__ void split_row_block(const double2* __restrict__ A, int N, int r, int s, int ldk,
                                       signed char* __restrict__ slices, int* __restrict__ ea,
                                       double* red) {
    const double2* row = A + (size_t)r * N;
    double m = 0.0;
    for (int c = threadIdx.x; c < N; c += kSThreads) {
        const double2 v = row[c];
        m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = kSThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    const int e = exponent_of(red[0]);
    if (threadIdx.x == 0) ea[r] = e;
    const size_t ss = (size_t)N * ldk;  // bytes per slice
    signed char* base = slices + (size_t)r * ldk;
    for (int c = threadIdx.x; c < ldk / 2; c += kSThreads) {
        double yr = 0.0, yi = 0.0;
        if (c < N) {
            const double2 v = row[c];
            yr = ldexp(v.x, -e);
            yi = ldexp(v.y, -e);
        }
        for (int i = 0; i < s; ++i) {
            yr *= 128.0;
            yi *= 128.0;
            const double tr = trunc(yr), ti = trunc(yi);
            yr -= tr;
            yi -= ti;
            const unsigned short pk = (unsigned short)((unsigned char)(signed char)tr) |
                                      ((unsigned short)((unsigned char)(signed char)ti) << 8);
            *reinterpret_cast<unsigned short*>(base + i * ss + 2 * c) = pk;
        }
    }
}

// Column exponents of the 64 complex columns c0 .. c0+63 of B over all N rows (one pass; for
// the small matrices of the grouped kernels).  red: 4 x 64 doubles of LDS.
__device__ __forceinline__ void col_exponent_block(const double2* __restrict__ B, int N, int c0,
                                          int* __restrict__ eb, double (*red)[64]) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int c = c0 + tx;
    double m = 0.0;
    if (c < N)
        for (int k = ty; k < N; k += 4) {
            const double2 v = B[(size_t)k * N + c];
            m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
        }
    red[ty][tx] = m;
    __syncthreads();
    if (ty == 0 && c < N)
        eb[c] = exponent_of(fmax(fmax(red[0][tx], red[1][tx]), fmax(red[2][tx], red[3][tx])));
}

// B~^T slices, tile (bx, by) of 32 rows (k) x 32 complex columns (c) of B through LDS.  Output
// row cc = 2c + u of B~^T holds, at kk = 2k + t:  u = 0: (Re b, -Im b), u = 1: (Im b, Re b).
// Rows are ldk bytes; tiles with k >= N write the zero padding.
constexpr int kCT = 32;
__device__ __forceinline__ void split_cols_tile(const double2* __restrict__ B, int N, int bx, int by, int s,
                                       int ldk, const int* __restrict__ eb,
                                       signed char* __restrict__ slices,
                                       double2 (*tile)[kCT + 1]) {
    const int k0 = by * kCT, c0 = bx * kCT;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int a = ty; a < kCT; a += 8) {
        const int k = k0 + a, c = c0 + tx;
        tile[a][tx] = (k < N && c < N) ? B[(size_t)k * N + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // Thread (tx = k offset, ty) writes, for columns c0 + ty + 8 j, the 2 bytes (t = 0, 1) of
    // output rows 2c and 2c+1 at kk = 2 (k0 + tx) + t.
    const size_t ss = (size_t)2 * N * ldk;  // bytes per slice
    const int k = k0 + tx;
    if (2 * k >= ldk) return;
    for (int a = ty; a < kCT; a += 8) {
        const int c = c0 + a;
        if (c >= N) break;
        const double2 v = tile[tx][a];  // B[k][c] (0 beyond N)
        const int e = eb[c];
        double br = ldexp(v.x, -e), bi = ldexp(v.y, -e);
        signed char* o0 = slices + (size_t)(2 * c) * ldk + 2 * k;
        signed char* o1 = slices + (size_t)(2 * c + 1) * ldk + 2 * k;
        for (int i = 0; i < s; ++i) {
            br *= 128.0;
            bi *= 128.0;
            const double tr = trunc(br), ti = trunc(bi);
            br -= tr;
            bi -= ti;
            const unsigned char ur = (unsigned char)(signed char)tr;
            const unsigned char ui = (unsigned char)(signed char)ti;
            const unsigned char nui = (unsigned char)(signed char)(-ti);
            *reinterpret_cast<unsigned short*>(o0 + i * ss) = (unsigned short)ur | ((unsigned short)nui << 8);
            *reinterpret_cast<unsigned short*>(o1 + i * ss) = (unsigned short)ui | ((unsigned short)ur << 8);
        }
    }
}

// ---------------------------------------------------------------- INT8 product tile
// Block tile 128 rows x 128 real columns (64 complex), 4 waves as 2 x 2 of 64 x 64;
// K stage of 128 bytes (two MFMA k-steps), double-buffered in LDS, global loads one stage
// ahead.  Slice pairs run in order of decreasing t = i + j; the pairs of one t share one
// exact int32 accumulator ((t-1) 2N 127^2 < 2^31), which is stored to the slab G[t-2]
// (int32, N x 2N) when t changes.  The FP64 weighting happens afterwards (combine or the
// fixed-point update), so no FP64 accumulator occupies registers here.
constexpr int kI8BM = 128, kI8BN = 128, kI8BK = 128;
constexpr int kI8LD = kI8BK + 16;  // padded LDS row (bytes)
constexpr int kI8Stage = (kI8BM + kI8BN) * kI8LD;
constexpr int kMaxPairs = kSplitMax * (kSplitMax + 1) / 2;

// Bytes per slice row: the real K = 2N rounded up to the K stage.
__host__ __device__ inline int split_ldk_of(int N) { return ((2 * N + kI8BK - 1) / kI8BK) * kI8BK; }

struct I8Smem {
    signed char stage[2 * kI8Stage] __attribute__((aligned(16)));
    unsigned char pt_i[kMaxPairs], pt_j[kMaxPairs], pt_flush[kMaxPairs];
};

// Tiles of the lower-triangle product: row tile I (128 rows) has column tiles J = 0 .. 2I+1
// (64 complex columns each), numbered b = I (I+1) + J.
__device__ __forceinline__ void i8_lower_tile(int b, int& I, int& J) {
    I = (int)((sqrt(4.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) <= b) ++I;
    while (I * (I + 1) > b) --I;
    J = b - I * (I + 1);
}

// Slabs G[t-2] of tile (ti, tj) of A~ B~ from the slices sa (A~, N x ldk each) and sb
// (B~^T, 2N x ldk each).
__device__ __forceinline__ void zgemm_i8_tile(int ti, int tj, const signed char* __restrict__ sa,
                                     const signed char* __restrict__ sb, int* __restrict__ G, int N,
                                     int s, int ldk, I8Smem& sm) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) {
        int p = 0;
        for (int t = s + 1; t >= 2; --t)
            for (int a = 1; a <= t - 1; ++a, ++p) {
                sm.pt_i[p] = (unsigned char)a;
                sm.pt_j[p] = (unsigned char)(t - a);
                sm.pt_flush[p] = (unsigned char)(a == t - 1);
            }
    }
    const int row0 = ti * kI8BM;      // rows of A~ / G
    const int cc0 = tj * kI8BN;       // real columns of G (rows of B~^T)
    const int M2 = 2 * N;             // real columns
    const size_t sA = (size_t)N * ldk, sB = (size_t)M2 * ldk;  // bytes per slice
    const int nk = ldk / kI8BK;       // K stages (real K = 2N, zero padded to ldk)
    const int total = s * (s + 1) / 2 * nk;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int q = lane >> 4, l16 = lane & 15;
    __syncthreads();

    v4i acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = v4i{0, 0, 0, 0};

    uint4 ra[4], rb[4];
    auto load = [&](int it) {
        const int p = it / nk;
        const int k0 = (it - p * nk) * kI8BK;
        const signed char* A = sa + (size_t)(sm.pt_i[p] - 1) * sA;
        const signed char* B = sb + (size_t)(sm.pt_j[p] - 1) * sB;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int id = tid + x * kSThreads;
            const int rr = id >> 3, cb = (id & 7) * 16;
            const int gr = row0 + rr, gc = cc0 + rr;
            ra[x] = gr < N ? *reinterpret_cast<const uint4*>(A + (size_t)gr * ldk + k0 + cb)
                           : make_uint4(0, 0, 0, 0);
            rb[x] = gc < M2 ? *reinterpret_cast<const uint4*>(B + (size_t)gc * ldk + k0 + cb)
                            : make_uint4(0, 0, 0, 0);
        }
    };
    auto store = [&](signed char* st) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int id = tid + x * kSThreads;
            const int rr = id >> 3, cb = (id & 7) * 16;
            *reinterpret_cast<uint4*>(st + rr * kI8LD + cb) = ra[x];
            *reinterpret_cast<uint4*>(st + (kI8BM + rr) * kI8LD + cb) = rb[x];
        }
    };

    load(0);
    store(sm.stage);
    __syncthreads();
    for (int it = 0; it < total; ++it) {
        const int cur = it & 1;
        if (it + 1 < total) load(it + 1);
        const signed char* st = sm.stage + cur * kI8Stage;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            v4i fa[4], fb[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                fa[x] = *reinterpret_cast<const v4i*>(st + (wr + x * 16 + l16) * kI8LD + ks * 64 + q * 16);
                fb[x] = *reinterpret_cast<const v4i*>(st + (kI8BM + wc + x * 16 + l16) * kI8LD + ks * 64 + q * 16);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[a], fb[c], acc[a][c], 0, 0, 0);
        }
        const int p = it / nk;
        if (it - p * nk == nk - 1 && sm.pt_flush[p]) {  // last stage of the last pair of this t
            int* g = G + (size_t)(sm.pt_i[p] + sm.pt_j[p] - 2) * N * M2;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int cc = cc0 + wc + c * 16 + l16;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = row0 + wr + a * 16 + 4 * q + r;
                        if (row < N && cc < M2) g[(size_t)row * M2 + cc] = acc[a][c][r];
                    }
                    acc[a][c] = v4i{0, 0, 0, 0};
                }
        }
        if (it + 1 < total) store(sm.stage + (cur ^ 1) * kI8Stage);
        __syncthreads();
    }
}

// Element e (row-major complex index) of C = 2^(ea_r + eb_c) sum_{t=2}^{s+1} 2^(-7 t) G[t-2].
__device__ __forceinline__ double2 split_combine_elem(const int* __restrict__ G, const int* __restrict__ ea,
                                             const int* __restrict__ eb, int N, int s, size_t e) {
    const size_t slab = 2 * (size_t)N * N;
    const int r = (int)(e / N), c = (int)(e - (size_t)r * N);
    double vr = 0.0, vi = 0.0;
    for (int t = s + 1; t >= 2; --t) {
        const int2 g = *reinterpret_cast<const int2*>(G + (size_t)(t - 2) * slab + 2 * e);
        const double w = ldexp(1.0, -7 * t);
        vr += w * (double)g.x;
        vi += w * (double)g.y;
    }
    const int ex = ea[r] + eb[c];
    return make_double2(ldexp(vr, ex), ldexp(vi, ex));
}

}  // namespace zk

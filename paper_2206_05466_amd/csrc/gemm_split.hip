// Split-precision complex products: FP64 matrix products emulated on INT8 MFMA
// (v_mfma_i32_16x16x64_i8) by the error-free splitting of Ozaki, Ogita, Oishi & Rump,
// "Error-free transformations of matrix multiplication by using fast routines of matrix
// multiplication and its applications", Numer. Algorithms 59 (2012), in its integer form
// (Ootomo, Ozaki & Yokota, "DGEMM on integer matrix multiplication unit", 2024).
//
// The products are the two of the fixed-point map (Sec. 3.1, eq. (isomp_iter)).  As in the
// FP64 kernels, a complex product C = A B is the real product C~ = A~ B~ of the interleaved
// A~ (N x 2N) and the 2 x 2-block form B~ (2N x 2N) of B.
//
// Splitting.  Row r of A~ is scaled by 2^-ea_r (ea_r = exponent of its largest magnitude, so
// |entries| < 1) and cut into s signed 7-bit slices by exact truncation:
//     y = x 2^-ea;  for i = 1..s:  y = 128 y;  a_i = trunc(y) in [-127, 127];  y = y - a_i.
// Column cc of B~ likewise with 2^-eb_c (one exponent per complex column c; both real columns
// 2c, 2c+1 hold the same magnitudes).  Then
//     C~[r][cc] ~= 2^(ea_r + eb_c) sum_{i + j <= s + 1} 2^(-7 (i + j)) (a_i b_j)[r][cc],
// the products of one t = i + j summed exactly in int32 ((t-1) 2N 127^2 < 2^31 for the sizes
// and slice counts allowed), then weighted and added in FP64 in a fixed order.  The neglected terms are below ~2^(-7 s) relative to
// max|row of A~| max|column of B~| per term of the K sum, so s trades accuracy for speed.
//
// Slices: A~ slices row-major [r][kk] (N x 2N bytes each); B~ slices transposed,
// B~^T[cc][kk] (2N x 2N bytes each), which is the MFMA's B-operand order (K contiguous).
// INT8 MFMA operand layout (16x16x64): lane l supplies 16 bytes of A~ row l%16 and of B~^T row
// l%16, at the same 16 k positions (k = 16 (l/16) + 0..15 here); accumulator register r of
// lane l holds D[4 (l/16) + r][l%16].

#include <type_traits>

#include "update_tile.h"

namespace {

using namespace zk;

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

// ---------------------------------------------------------------- slicing

__device__ inline int exponent_of(double m) {  // smallest e with m < 2^e (0 for m == 0)
    if (!(m > 0.0)) return 0;
    int e;
    frexp(m, &e);
    return e;
}

// One block per row r of A~: scale exponent and s slices (rows of ldk bytes, zero padded).
__global__ __launch_bounds__(kThreads) void split_rows_kernel(const double2* __restrict__ A,
                                                              int N, int s, int ldk,
                                                              signed char* __restrict__ slices,
                                                              int* __restrict__ ea) {
    __shared__ double red[kThreads];
    const int r = blockIdx.x;
    const double2* row = A + (size_t)r * N;
    double m = 0.0;
    for (int c = threadIdx.x; c < N; c += kThreads) {
        const double2 v = row[c];
        m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    const int e = exponent_of(red[0]);
    if (threadIdx.x == 0) ea[r] = e;
    const size_t ss = (size_t)N * ldk;  // bytes per slice
    signed char* base = slices + (size_t)r * ldk;
    for (int c = threadIdx.x; c < ldk / 2; c += kThreads) {
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

// Column maxima of B (complex N x N, row-major), two stages: block (x, y) takes 256
// columns over the row chunk y; then one thread per column combines the chunks.
constexpr int kColChunks = 64;
__global__ __launch_bounds__(kThreads) void col_max_partial(const double2* __restrict__ B, int N,
                                                            double* __restrict__ part) {
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= N) return;
    const int k0 = (int)((long long)blockIdx.y * N / kColChunks);
    const int k1 = (int)((long long)(blockIdx.y + 1) * N / kColChunks);
    double m = 0.0;
    for (int k = k0; k < k1; ++k) {
        const double2 v = B[(size_t)k * N + c];
        m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
    }
    part[(size_t)blockIdx.y * N + c] = m;
}

__global__ __launch_bounds__(kThreads) void col_exponent_kernel(const double* __restrict__ part,
                                                                int N, int* __restrict__ eb) {
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= N) return;
    double m = 0.0;
    for (int y = 0; y < kColChunks; ++y) m = fmax(m, part[(size_t)y * N + c]);
    eb[c] = exponent_of(m);
}

// B~^T slices: tile of 32 rows (k) x 32 complex columns (c) of B through LDS.  Output row
// cc = 2c + u of B~^T holds, at kk = 2k + t:  u = 0: (Re b, -Im b), u = 1: (Im b, Re b).
// Rows are ldk bytes; tiles with k >= N write the zero padding.
constexpr int kCT = 32;
__global__ __launch_bounds__(kThreads) void split_cols_kernel(const double2* __restrict__ B,
                                                              int N, int s, int ldk,
                                                              const int* __restrict__ eb,
                                                              signed char* __restrict__ slices) {
    __shared__ double2 tile[kCT][kCT + 1];
    const int k0 = blockIdx.y * kCT, c0 = blockIdx.x * kCT;
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

// ---------------------------------------------------------------- INT8 product
// Block tile 128 rows x 128 real columns (64 complex), 4 waves as 2 x 2 of 64 x 64;
// K stage of 128 bytes (two MFMA k-steps), double-buffered in LDS, global loads one stage
// ahead.  Slice pairs run in order of decreasing t = i + j; the pairs of one t share one
// exact int32 accumulator ((t-1) 2N 127^2 < 2^31), which is stored to the slab G[t-2]
// (int32, N x 2N) when t changes.  The FP64 weighting happens afterwards (combine kernel or
// the fixed-point update), so no FP64 accumulator occupies registers here.
constexpr int kBM = 128, kBN = 128, kBKB = 128;
constexpr int kLD = kBKB + 16;  // padded LDS row (bytes)
constexpr int kStage = (kBM + kBN) * kLD;
constexpr int kMaxPairs = kSplitMax * (kSplitMax + 1) / 2;

// mode 0: full product, tile b -> (b / tiles_n, b % tiles_n).
// mode 1: tiles meeting the lower triangle: row tile I (128 rows) has column tiles
//         J = 0..2I+1 (64 complex columns each), b = I (I+1) + J.
__global__ __launch_bounds__(kThreads, 2) void zgemm_i8_kernel(
    const signed char* __restrict__ sa, const signed char* __restrict__ sb, int* __restrict__ G,
    int N, int s, int ldk, int mode, int tiles_n) {
    __shared__ __attribute__((aligned(16))) signed char smem[2 * kStage];
    __shared__ unsigned char pt_i[kMaxPairs], pt_j[kMaxPairs], pt_flush[kMaxPairs];
    int ti, tj;
    const int b = blockIdx.x;
    if (mode == 0) {
        ti = b / tiles_n;
        tj = b % tiles_n;
    } else {
        int I = (int)((sqrt(4.0 * (double)b + 1.0) - 1.0) * 0.5);
        while ((I + 1) * (I + 2) <= b) ++I;
        while (I * (I + 1) > b) --I;
        ti = I;
        tj = b - I * (I + 1);
        if (tj >= tiles_n) return;  // ragged N: block idle (uniform)
    }
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) {
        int p = 0;
        for (int t = s + 1; t >= 2; --t)
            for (int a = 1; a <= t - 1; ++a, ++p) {
                pt_i[p] = (unsigned char)a;
                pt_j[p] = (unsigned char)(t - a);
                pt_flush[p] = (unsigned char)(a == t - 1);
            }
    }
    const int row0 = ti * kBM;        // rows of A~ / G
    const int cc0 = tj * kBN;         // real columns of G (rows of B~^T)
    const int M2 = 2 * N;             // real columns
    const size_t sA = (size_t)N * ldk, sB = (size_t)M2 * ldk;  // bytes per slice
    const int nk = ldk / kBKB;        // K stages (real K = 2N, zero padded to ldk)
    const int total = s * (s + 1) / 2 * nk;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int q = lane >> 4, l16 = lane & 15;
    __syncthreads();

    v4i acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = v4i{0, 0, 0, 0};

    uint4 ra[1][4], rb[1][4];
    auto load = [&](int it, int slot) {
        const int p = it / nk;
        const int k0 = (it - p * nk) * kBKB;
        const signed char* A = sa + (size_t)(pt_i[p] - 1) * sA;
        const signed char* B = sb + (size_t)(pt_j[p] - 1) * sB;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int id = tid + x * kThreads;
            const int rr = id >> 3, cb = (id & 7) * 16;
            const int gr = row0 + rr, gc = cc0 + rr;
            ra[slot][x] = gr < N ? *reinterpret_cast<const uint4*>(A + (size_t)gr * ldk + k0 + cb)
                                 : make_uint4(0, 0, 0, 0);
            rb[slot][x] = gc < M2 ? *reinterpret_cast<const uint4*>(B + (size_t)gc * ldk + k0 + cb)
                                  : make_uint4(0, 0, 0, 0);
        }
    };
    auto store = [&](signed char* st, int slot) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int id = tid + x * kThreads;
            const int rr = id >> 3, cb = (id & 7) * 16;
            *reinterpret_cast<uint4*>(st + rr * kLD + cb) = ra[slot][x];
            *reinterpret_cast<uint4*>(st + (kBM + rr) * kLD + cb) = rb[slot][x];
        }
    };

    load(0, 0);
    store(smem, 0);
    __syncthreads();
    for (int it = 0; it < total; ++it) {
        const int cur = it & 1;
        if (it + 1 < total) load(it + 1, 0);
        const signed char* st = smem + cur * kStage;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            v4i fa[4], fb[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                fa[x] = *reinterpret_cast<const v4i*>(st + (wr + x * 16 + l16) * kLD + ks * 64 + q * 16);
                fb[x] = *reinterpret_cast<const v4i*>(st + (kBM + wc + x * 16 + l16) * kLD + ks * 64 + q * 16);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[a], fb[c], acc[a][c], 0, 0, 0);
        }
        const int p = it / nk;
        if (it - p * nk == nk - 1 && pt_flush[p]) {  // last stage of the last pair of this t
            int* g = G + (size_t)(pt_i[p] + pt_j[p] - 2) * N * M2;
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
        if (it + 1 < total) store(smem + (cur ^ 1) * kStage, 0);
        __syncthreads();
    }
}

// C~[r][cc] = 2^(ea_r + eb_c) sum_{t=2}^{s+1} 2^(-7 t) G[t-2][r][cc], complex pairs per thread.
__global__ __launch_bounds__(kThreads) void split_combine_kernel(const int* __restrict__ G,
                                                                 const int* __restrict__ ea,
                                                                 const int* __restrict__ eb,
                                                                 double2* __restrict__ Cm, int N,
                                                                 int s) {
    const size_t n2 = (size_t)N * N;
    const size_t slab = 2 * n2;
    for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n2;
         e += (size_t)gridDim.x * kThreads) {
        const int r = (int)(e / N), c = (int)(e - (size_t)r * N);
        double vr = 0.0, vi = 0.0;
        for (int t = s + 1; t >= 2; --t) {
            const int2 g = *reinterpret_cast<const int2*>(G + (size_t)(t - 2) * slab + 2 * e);
            const double w = ldexp(1.0, -7 * t);
            vr += w * (double)g.x;
            vi += w * (double)g.y;
        }
        const int ex = ea[r] + eb[c];
        Cm[e] = make_double2(ldexp(vr, ex), ldexp(vi, ex));
    }
}

// ---------------------------------------------------------------- fixed-point update
__global__ __launch_bounds__(kThreads) void lower_update_kernel(
    const double2* __restrict__ Qf, const int* __restrict__ G, const int* __restrict__ ea,
    const int* __restrict__ eb, int s, const double2* __restrict__ Am,
    const double2* __restrict__ Wn, const double2* Wt, double2* F, double2* __restrict__ Wout,
    double* __restrict__ rowpart, int N, double h) {
    __shared__ double2 sT[kUT][kUT + 1];
    const int b = blockIdx.x;
    int I = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    const int J = b - I * (I + 1) / 2;
    lower_update_tile(I, J, Qf, G, ea, eb, s, Am, Wn, Wt, F, Wout, rowpart, N, h, sT);
}

}  // namespace

int ze_split_ldk(int N) { return ((2 * N + kBKB - 1) / kBKB) * kBKB; }

hipError_t launch_split_prepare(const ze_ctx* c, const double2* A, const double2* B,
                                hipStream_t st) {
    const int N = c->N, s = c->split_slices, ldk = ze_split_ldk(N);
    hipLaunchKernelGGL(split_rows_kernel, dim3(N), dim3(kThreads), 0, st, A, N, s, ldk, c->split_a,
                       c->split_ea);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int gx = (N + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(col_max_partial, dim3(gx, kColChunks), dim3(kThreads), 0, st, B, N,
                       c->split_colmax);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(col_exponent_kernel, dim3(gx), dim3(kThreads), 0, st, c->split_colmax, N,
                       c->split_eb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g((N + kCT - 1) / kCT, (ldk / 2 + kCT - 1) / kCT);
    hipLaunchKernelGGL(split_cols_kernel, g, dim3(kThreads), 0, st, B, N, s, ldk, c->split_eb,
                       c->split_b);
    return hipGetLastError();
}

hipError_t launch_zgemm_split(const ze_ctx* c, const double2* A, const double2* B, double2* C,
                              int lower, hipStream_t st) {
    const int N = c->N, s = c->split_slices;
    hipError_t e = launch_split_prepare(c, A, B, st);
    if (e != hipSuccess) return e;
    const int tr = (N + kBM - 1) / kBM;
    const int tn = (2 * N + kBN - 1) / kBN;
    const int nb = lower ? tr * (tr + 1) : tr * tn;
    hipLaunchKernelGGL(zgemm_i8_kernel, dim3(nb), dim3(kThreads), 0, st, c->split_a, c->split_b,
                       c->split_g, N, s, ze_split_ldk(N), lower ? 1 : 0, tn);
    e = hipGetLastError();
    if (e != hipSuccess || lower) return e;
    const size_t n2 = (size_t)N * N;
    const unsigned grid = (unsigned)((n2 + kThreads - 1) / kThreads < 16384 ? (n2 + kThreads - 1) / kThreads : 16384);
    hipLaunchKernelGGL(split_combine_kernel, dim3(grid), dim3(kThreads), 0, st, c->split_g,
                       c->split_ea, c->split_eb, C, N, s);
    return hipGetLastError();
}

hipError_t launch_lower_update(const ze_ctx* c, const double2* Q, const double2* A,
                               const double2* Wn, const double2* Wt, double2* F, double2* Wout,
                               double* rowpart, double h, hipStream_t st) {
    const int N = c->N;
    const int T = (N + kUT - 1) / kUT;
    hipLaunchKernelGGL(lower_update_kernel, dim3(T * (T + 1) / 2), dim3(kThreads), 0, st, Q,
                       c->split_g, c->split_ea, c->split_eb, c->split_slices, A, Wn, Wt, F, Wout,
                       rowpart, N, h);
    return hipGetLastError();
}

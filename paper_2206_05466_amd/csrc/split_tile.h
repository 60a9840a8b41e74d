// Device bodies of the split-precision (INT8 MFMA, Ozaki splitting) products, shared by the
// single-problem kernels and the grouped ensemble kernels.  The splitting itself, the slice
// layouts and the exactness bounds are described at the top of gemm_split.hip.
#pragma once

#include "internal.h"

namespace zk {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kSThreads = 256;

// Scale exponent for a row / column whose largest magnitude is m: the e with
// 0.495 < m 2^-e <= 0.99 (0 for m == 0), which keeps the top digit of split_digits within
// [-127, 127].
__device__ __forceinline__ int exponent_of(double m) {
    if (!(m > 0.0)) return 0;
    int e;
    const double f = frexp(m, &e);  // m = f 2^e, 0.5 <= f < 1
    return f > 0.99 ? e + 1 : e;
}

// The s balanced base-256 digits of y = x 2^-e (|y| <= 0.99): X = y 2^(7 + 8 (s - 1)) rounded
// to the nearest integer (|X| < 2^63 for s <= 8), then from the lowest digit up
// d_k = ((X + 128) mod 256) - 128 in [-128, 127] and X <- (X - d_k) / 256; the top digit
// d_1 = X is within [-127, 127].  So y = sum_k d_k 2^(1 - 8k) + R with |R| <= 2^(-8s): 7 bits
// in the first digit and 8 in each further one, zero-mean rounding, every step exact.
__device__ __forceinline__ void split_digits(double x, int e, int s, int (&d)[kSplitMax]) {
    long long X = llrint(ldexp(x, 7 + 8 * (s - 1) - e));
#pragma unroll
    for (int k = kSplitMax - 1; k >= 1; --k) {
        d[k] = 0;
        if (k < s) {
            const int dk = (int)((X + 128) & 255) - 128;
            d[k] = dk;
            X = (X - dk) >> 8;
        }
    }
    d[0] = (int)X;
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
    const size_t ss = (size_t)split_rows_pad(N) * ldk;  // bytes per slice
    signed char* base = slices + (size_t)r * ldk;
    for (int c = threadIdx.x; c < ldk / 2; c += kSThreads) {
        const double2 v = c < N ? row[c] : make_double2(0.0, 0.0);  // zero padding beyond N
        int dr[kSplitMax], di[kSplitMax];
        split_digits(v.x, e, s, dr);
        split_digits(v.y, e, s, di);
#pragma unroll
        for (int i = 0; i < kSplitMax; ++i) {
            if (i >= s) break;
            const unsigned short pk = (unsigned short)((unsigned char)(signed char)dr[i]) |
                                      ((unsigned short)((unsigned char)(signed char)di[i]) << 8);
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
// row cc = 2c + u of B~^T holds, at kk = 2k + t:  u = 0: (Re b, -Im b), u = 1: (Im b, Re b);
// -Im b gets its own digits (the balanced digits of -x are minus those of x except where a
// digit is -128).  Rows are ldk bytes; tiles with k >= N write the zero padding.
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
    const size_t ss = (size_t)split_cols_pad(N) * ldk;  // bytes per slice
    const int k = k0 + tx;
    if (2 * k >= ldk) return;
    for (int a = ty; a < kCT; a += 8) {
        const int c = c0 + a;
        if (c >= N) break;
        const double2 v = tile[tx][a];  // B[k][c] (0 beyond N)
        const int e = eb[c];
        int dr[kSplitMax], di[kSplitMax], dn[kSplitMax];
        split_digits(v.x, e, s, dr);
        split_digits(v.y, e, s, di);
        split_digits(-v.y, e, s, dn);
        signed char* o0 = slices + (size_t)(2 * c) * ldk + 2 * k;
        signed char* o1 = slices + (size_t)(2 * c + 1) * ldk + 2 * k;
#pragma unroll
        for (int i = 0; i < kSplitMax; ++i) {
            if (i >= s) break;
            const unsigned char ur = (unsigned char)(signed char)dr[i];
            const unsigned char ui = (unsigned char)(signed char)di[i];
            const unsigned char nui = (unsigned char)(signed char)dn[i];
            *reinterpret_cast<unsigned short*>(o0 + i * ss) = (unsigned short)ur | ((unsigned short)nui << 8);
            *reinterpret_cast<unsigned short*>(o1 + i * ss) = (unsigned short)ui | ((unsigned short)ur << 8);
        }
    }
}

// ---------------------------------------------------------------- modular (CRT) form
// Ozaki scheme II: a row of A~ (column of B~) scaled by a power of two to integers X with
// |X| <= 0.99 2^b is represented exactly by its residues modulo kCrtMods pairwise coprime
// moduli p_k <= 256 (balanced, so each fits an int8); exact INT8 products per modulus give
// the integer product modulo p_k, and the Chinese remainder theorem recovers it exactly while
// |X_A X_B| summed stays below 0.99^2 M / 2, M = prod p_k (~2^125.2).
constexpr int kCrtP[kCrtMods] = {256, 255, 253, 251, 247, 241, 239, 233,
                                 229, 227, 223, 211, 199, 197, 193, 191};


// p_k for a wave-uniform runtime k.
__device__ __forceinline__ int crt_modulus(int k) {
    int p = kCrtP[0];
#pragma unroll
    for (int j = 1; j < kCrtMods; ++j) p = k == j ? kCrtP[j] : p;
    return p;
}

// Balanced residue, in [-(p_K)/2, (p_K - 1)/2], of an integer X held exactly in a double
// (|X| < 2^62), given in four exact pieces X = (x3 - 2^14) 2^48 + x2 2^32 + x1 2^16 + x0 with
// 0 <= x3 < 2^15 and 0 <= x2, x1, x0 < 2^16.  In 32-bit integer arithmetic: d = x3 (2^48 mod p)
// + x2 (2^32 mod p) + x1 (2^16 mod p) + x0 - 2^14 (2^48 mod p), congruent to X, each product a
// 24-bit multiply-add (-2^22 < d < 2^26); q = d / p rounded to the nearest integer from an
// FP32 estimate (d / p < 2^19: off by less than 0.1 before the rounding), so r = d - q p (exact)
// lies in [-0.6 p, 0.6 p] and one step brings it into the balanced range.
template <int K>
__device__ __forceinline__ int crt_residue(unsigned x3, unsigned x2, unsigned x1, unsigned x0) {
    constexpr int p = kCrtP[K];
    constexpr unsigned c48 = (unsigned)((1ULL << 48) % p), c32 = (unsigned)((1ULL << 32) % p);
    constexpr unsigned c16 = (unsigned)((1ULL << 16) % p);
    const int d = (int)(x3 * c48 + x2 * c32 + x1 * c16 + x0) - (int)((1u << 14) * c48);
    const int q = (int)rintf((float)d * (1.0f / (float)p));
    int r = d - q * p;
    r = r > (p - 1) / 2 ? r - p : r;
    return r < -(p / 2) ? r + p : r;
}

template <int K>
struct CrtResidues {
    // d[k] = balanced residue of X (in the pieces of crt_residue) modulo p_k for k < K
    __device__ __forceinline__ static void run(unsigned x3, unsigned x2, unsigned x1, unsigned x0,
                                               int (&d)[kCrtMods]) {
        CrtResidues<K - 1>::run(x3, x2, x1, x0, d);
        d[K - 1] = crt_residue<K - 1>(x3, x2, x1, x0);
    }
};
template <>
struct CrtResidues<0> {
    __device__ __forceinline__ static void run(unsigned, unsigned, unsigned, unsigned,
                                               int (&)[kCrtMods]) {}
};

// Residues of the integer X (exactly representable as a double, |X| < 2^62): its 16-bit pieces,
// taken in FP64 (exact: floors, and differences of exact multiples of powers of two); the masks
// change no value and let the compiler use 24-bit multiplies.
__device__ __forceinline__ void crt_residues_of(double X, int (&d)[kCrtMods]) {
    const double h3 = floor(X * 0x1p-48);      // [-2^14, 2^14)
    const double r3 = fma(-h3, 0x1p48, X);     // [0, 2^48)
    const double h2 = floor(r3 * 0x1p-32);
    const double r2 = fma(-h2, 0x1p32, r3);    // [0, 2^32)
    const double h1 = floor(r2 * 0x1p-16);
    const double h0 = fma(-h1, 0x1p16, r2);    // [0, 2^16)
    const unsigned x3 = (unsigned)((int)h3 + (1 << 14)) & 0x7fffu;
    CrtResidues<kCrtMods>::run(x3, (unsigned)h2 & 0xffffu, (unsigned)h1 & 0xffffu,
                               (unsigned)h0 & 0xffffu, d);
}

// Residues of x scaled by 2^(b - e) and rounded to the nearest integer (ties to even): the
// scaled value is exact, and from 2^52 on it is already an integer, so X is exact too.
__device__ __forceinline__ void crt_digits(double x, int e, int b, int (&d)[kCrtMods]) {
    crt_residues_of(rint(ldexp(x, b - e)), d);
}

// Balanced residue of d1 + d2 (both balanced residues modulo p_K).
template <int K>
__device__ __forceinline__ int crt_balanced_sum(int d1, int d2) {
    constexpr int p = kCrtP[K];
    int t = d1 + d2;
    t = t > (p - 1) / 2 ? t - p : t;
    return t < -(p / 2) ? t + p : t;
}

// Residues of four consecutive K positions j = 0..3 of one A~ row / B~^T row: the real and
// imaginary parts' residues dr[j], di[j], stored as one 32-bit word per slab at o (4-byte
// aligned) in slabs 3k (real part), 3k + 1 (imaginary part) and 3k + 2 (their sum modulo p_k),
// slab stride ss, for every modulus k.
__device__ __forceinline__ unsigned crt_pack4(int a0, int a1, int a2, int a3) {
    return (unsigned)(a0 & 0xff) | ((unsigned)(a1 & 0xff) << 8) | ((unsigned)(a2 & 0xff) << 16) |
           ((unsigned)(a3 & 0xff) << 24);
}

template <int K>
struct CrtStore3x4 {
    __device__ __forceinline__ static void run(const int (&dr)[4][kCrtMods], const int (&di)[4][kCrtMods],
                                               signed char* o, size_t ss) {
        CrtStore3x4<K - 1>::run(dr, di, o, ss);
        constexpr int k = K - 1;
        *reinterpret_cast<unsigned*>(o + (3 * k) * ss) = crt_pack4(dr[0][k], dr[1][k], dr[2][k], dr[3][k]);
        *reinterpret_cast<unsigned*>(o + (3 * k + 1) * ss) = crt_pack4(di[0][k], di[1][k], di[2][k], di[3][k]);
        *reinterpret_cast<unsigned*>(o + (3 * k + 2) * ss) =
            crt_pack4(crt_balanced_sum<k>(dr[0][k], di[0][k]), crt_balanced_sum<k>(dr[1][k], di[1][k]),
                      crt_balanced_sum<k>(dr[2][k], di[2][k]), crt_balanced_sum<k>(dr[3][k], di[3][k]));
    }
};
template <>
struct CrtStore3x4<0> {
    __device__ __forceinline__ static void run(const int (&)[4][kCrtMods], const int (&)[4][kCrtMods],
                                               signed char*, size_t) {}
};

// Residues for the complex product in three real products per modulus (exact modulo p_k):
// Re = ar br - ai bi, Im = (ar + ai)(br + bi) - ar br - ai bi.  Slab 3k + q (q = 0: real part,
// 1: imaginary part, 2: their sum, all modulo p_k) holds crt_rows_pad(N) rows of ldk bytes
// (K = N, zero padded; ldk a multiple of 128).  Row r of A~ (one block per row; the row
// exponent from its maximum), four consecutive columns per thread:
__device__ __forceinline__ void crt_row_block(const double2* __restrict__ A, int N, int r, int b, int ldk,
                                      signed char* __restrict__ slabs, int* __restrict__ ea,
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
    const size_t ss = (size_t)crt_rows_pad(N) * ldk;
    signed char* base = slabs + (size_t)r * ldk;
    for (int c0 = 4 * threadIdx.x; c0 < ldk; c0 += 4 * kSThreads) {
        int dr[4][kCrtMods], di[4][kCrtMods];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = c0 + j;
            const double2 v = c < N ? row[c] : make_double2(0.0, 0.0);
            crt_digits(v.x, e, b, dr[j]);
            crt_digits(v.y, e, b, di[j]);
        }
        CrtStore3x4<kCrtMods>::run(dr, di, base + c0, ss);
    }
}

// B~^T rows (one per column c of B, K = N along the row), tile (bx, by) of kCT columns x kCT
// K values staged through LDS so that both the reads of B and the word stores are coalesced:
// thread t takes column c0 + t / 8 and K positions k0 + 4 (t % 8) .. + 3.
__device__ __forceinline__ void crt_cols_tile(const double2* __restrict__ B, int N, int bx, int by, int b,
                                      int ldk, const int* __restrict__ eb,
                                      signed char* __restrict__ slabs,
                                      double2 (*tile)[kCT + 1]) {
    static_assert(kCT * kCT == 4 * kSThreads, "one pass of four K positions per thread");
    const int k0 = by * kCT, c0 = bx * kCT;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int a = ty; a < kCT; a += 8) {
        const int k = k0 + a, c = c0 + tx;
        tile[a][tx] = (k < N && c < N) ? B[(size_t)k * N + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const size_t ss = (size_t)crt_rows_pad(N) * ldk;
    const int kq = 4 * (threadIdx.x & 7), cl = threadIdx.x >> 3;
    const int c = c0 + cl, k = k0 + kq;
    if (c >= N || k >= ldk) return;
    const int e = eb[c];
    int dr[4][kCrtMods], di[4][kCrtMods];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double2 v = tile[kq + j][cl];
        crt_digits(v.x, e, b, dr[j]);
        crt_digits(v.y, e, b, di[j]);
    }
    CrtStore3x4<kCrtMods>::run(dr, di, slabs + (size_t)c * ldk + k, ss);
}

// Constants of the reconstruction: W_k = (M / p_k) ((M / p_k)^-1 mod p_k) < M, so that
// X = sum_k c_k W_k mod M for c_k = X mod p_k, in 32-bit limbs; M as two 64-bit halves and as a
// double.
struct CrtConst {
    unsigned wl[kCrtMods][4];  // W_k in 32-bit limbs, least significant first
    unsigned long long mlo, mhi;
    double md;
};

constexpr double crt_u128_to_double(unsigned __int128 v) {
    return (double)(unsigned long long)(v >> 64) * 18446744073709551616.0 +
           (double)(unsigned long long)v;
}

constexpr CrtConst make_crt_const() {
    CrtConst k{};
    unsigned __int128 M = 1;
    for (int i = 0; i < kCrtMods; ++i) M *= (unsigned __int128)kCrtP[i];
    for (int i = 0; i < kCrtMods; ++i) {
        const unsigned p = (unsigned)kCrtP[i];
        const unsigned __int128 Mk = M / p;
        const unsigned r = (unsigned)(Mk % p);
        unsigned y = 0;
        for (unsigned x = 1; x < p && y == 0; ++x)
            if ((r * x) % p == 1) y = x;
        const unsigned __int128 W = Mk * y;
        for (int j = 0; j < 4; ++j) k.wl[i][j] = (unsigned)(W >> (32 * j));
    }
    k.mlo = (unsigned long long)M;
    k.mhi = (unsigned long long)(M >> 64);
    k.md = crt_u128_to_double(M);
    return k;
}

constexpr CrtConst kCrtK = make_crt_const();

// The integer X with |X| <= 0.99^2 M / 2 from the kCrtMods int32 products g_k (|g_k| < 2^31) of one
// output value (with `Reduced`, g_k = c_k already in [0, p_k)), rounded to FP64:
// c_k = g_k mod p_k, or any representative of it in [0, 3 p_k); S = sum_k c_k W_k < 2^14 M
// exactly modulo 2^128, each 32-bit limb of W_k times c_k summed in its own 64-bit accumulator
// (16 terms below 2^42 each); q = S / M rounded to the nearest integer, from an FP64 estimate
// of S built from the exact limb sums (exact: S / M = q + X / M lies at least 0.01 from a
// half-integer, and the estimate of S / M < 2^14 is off by less than 2^-35);
// X = S - q M modulo 2^128 is X
// itself, read as signed.  The magnitude is converted from its two 64-bit halves, each exact
// when X is representable.
// Running sums of that reconstruction: add(k, c) takes c = c_k + j p_k, j in {0, 1, 2} (the
// combine passes unreduced differences of residues); value() gives X.
struct CrtAcc {
    unsigned long long l0 = 0, l1 = 0, l2 = 0, l3 = 0;
    __device__ __forceinline__ void add(int k, int c) {
        constexpr CrtConst C = kCrtK;
        const unsigned long long u = (unsigned)c;
        l0 += u * C.wl[k][0];
        l1 += u * C.wl[k][1];
        l2 += u * C.wl[k][2];
        l3 += u * C.wl[k][3];
    }
    __device__ __forceinline__ double value() const {
        constexpr CrtConst C = kCrtK;
        const unsigned __int128 S = (unsigned __int128)l0 + ((unsigned __int128)l1 << 32) +
                                    ((unsigned __int128)l2 << 64) + ((unsigned __int128)l3 << 96);
        // S itself, not modulo 2^128 (it may reach 2^141): the limb sums are exact integers
        const double Sd = (((double)l3 * 0x1p32 + (double)l2) * 0x1p32 + (double)l1) * 0x1p32 +
                          (double)l0;
        const unsigned long long q = (unsigned long long)rint(Sd / C.md);
        const unsigned __int128 M = ((unsigned __int128)C.mhi << 64) | C.mlo;
        const __int128 X = (__int128)(S - (unsigned __int128)q * M);
        const unsigned __int128 a = X < 0 ? (unsigned __int128)(-X) : (unsigned __int128)X;
        const double v = (double)(unsigned long long)(a >> 64) * 0x1p64 + (double)(unsigned long long)a;
        return X < 0 ? -v : v;
    }
};

template <bool Reduced = false>
__device__ __forceinline__ double crt_reconstruct(const int (&g)[kCrtMods]) {
    CrtAcc acc;
#pragma unroll
    for (int k = 0; k < kCrtMods; ++k) {
        int c = g[k];
        if (!Reduced) {
            const int p = kCrtP[k];
            c = c - (int)floor((double)c * (1.0 / (double)p)) * p;
            c = c < 0 ? c + p : (c >= p ? c - p : c);
        }
        acc.add(k, c);
    }
    return acc.value();
}

// ---------------------------------------------------------------- INT8 product tile
// Block tile 128 rows x 128 real columns (64 complex), 4 waves as 2 x 2 of 64 x 64, each wave
// 2 x 2 tiles of v_mfma_i32_32x32x32_i8 (on gfx950 this form has about twice the throughput
// of the 16x16x64 one; measured 4.4 vs 2.6 POPS).  K stage of 128 bytes (four MFMA k-steps),
// double-buffered in LDS, global loads one stage ahead.  Slice pairs run in order of
// decreasing t = i + j; the pairs of one t share one exact int32 accumulator
// ((t-1) 2N 128^2 < 2^31), which is stored to the slab G[t-2] (int32, N x 2N) when t changes.
// The FP64 weighting happens afterwards (combine or the fixed-point update), so no FP64
// accumulator occupies registers here.
//
// MFMA operands: lane l supplies 16 bytes of A~ row (l % 32) and of B~^T row (l % 32) at
// k = 16 (l / 32) + 0..15 of the k-step; accumulator register r of lane l holds
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] (checked on the GPU).
//
// LDS rows are 128 bytes with no padding; the 16-byte chunk c of row r is stored at chunk
// position c ^ ((r & 6) | ((r >> 4) & 1)).  The operand reads (32 consecutive rows, one chunk
// per half-wave) then fall on distinct bank groups in every group of lanes the LDS serves
// together (measured: full read bandwidth, half of it without the swizzle).
constexpr int kI8BM = 128, kI8BN = 128, kI8BK = 128;
constexpr int kI8Stage = (kI8BM + kI8BN) * kI8BK;

typedef int v16i __attribute__((ext_vector_type(16)));

// Bytes per slice row: the real K = 2N rounded up to the K stage.
__host__ __device__ inline int split_ldk_of(int N) { return ((2 * N + kI8BK - 1) / kI8BK) * kI8BK; }

struct I8Smem {
    signed char stage[2 * kI8Stage] __attribute__((aligned(16)));
};

__device__ __forceinline__ int i8_swizzle(int row) { return (row & 6) | ((row >> 4) & 1); }
__device__ __forceinline__ int i8_lds_offset(int row, int chunk) {
    return row * kI8BK + ((chunk ^ i8_swizzle(row)) << 4);
}

// Tiles of the lower-triangle product: row tile I (128 rows) has column tiles J = 0 .. 2I+1
// (64 complex columns each), numbered b = I (I+1) + J.
__device__ __forceinline__ void i8_lower_tile(int b, int& I, int& J) {
    I = (int)((sqrt(4.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) <= b) ++I;
    while (I * (I + 1) > b) --I;
    J = b - I * (I + 1);
}

// Next slice pair (i, j) in order of decreasing t = i + j, i ascending within t:
// (1, t-1), (2, t-2), ..., (t-1, 1), then (1, t-2), ...
__device__ __forceinline__ void i8_next_pair(int& i, int& j) {
    if (j > 1) {
        ++i;
        --j;
    } else {
        j = i - 1;  // new t = i + j - 1 = i: pairs (1, i - 1), ...
        i = 1;
    }
}

// Slabs G[t-2] of tile (ti, tj) of A~ B~ from the slices sa (A~, split_rows_pad(N) x ldk
// each) and sb (B~^T, split_cols_pad(N) x ldk each), over the K stages [kb, ke) of every slice
// pair (kb = 0, ke < 0: all of K).  With `add` the int32 sums are added to G with atomics
// (exact: a tile split along K over several blocks, G cleared beforehand), else stored.
// Each iteration issues the global loads of the next stage, computes the current stage from
// LDS, and stores the next stage to the other LDS buffer at the end of the stage; scheduling
// barriers keep that order (left alone, the compiler moves the LDS store up to the loads,
// which waits for them before the MFMAs).
__device__ __forceinline__ void zgemm_i8_tile(int ti, int tj, const signed char* __restrict__ sa,
                                              const signed char* __restrict__ sb,
                                              int* __restrict__ G, int N, int s, int ldk,
                                              I8Smem& sm, int kb = 0, int ke = -1,
                                              bool add = false) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int row0 = ti * kI8BM;      // rows of A~ / G
    const int cc0 = tj * kI8BN;       // real columns of G (rows of B~^T)
    const int M2 = 2 * N;             // real columns
    const size_t sA = (size_t)split_rows_pad(N) * ldk;  // bytes per slice
    const size_t sB = (size_t)split_cols_pad(N) * ldk;
    if (ke < 0) ke = ldk / kI8BK;     // K stages (real K = 2N, zero padded to ldk)
    const int total = s * (s + 1) / 2 * (ke - kb);
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int l32 = lane & 31, h = lane >> 5;

    v16i acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = (v16i)0;

    // this thread's rows of the A~ and B~^T tiles (padded buffers: always in range); a
    // thread's x-th 16-byte piece of a stage is row (tid / 8) + 32 x, bytes 16 (tid % 8) ..
    const signed char* pa = sa + (size_t)(row0 + (tid >> 3)) * ldk + (tid & 7) * 16;
    const signed char* pb = sb + (size_t)(cc0 + (tid >> 3)) * ldk + (tid & 7) * 16;
    const size_t xstep = (size_t)(kSThreads / 8) * ldk;
    int soff_a[4], soff_b[4];  // LDS byte offsets of those pieces
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int rr = (tid >> 3) + 32 * x, ch = tid & 7;
        soff_a[x] = i8_lds_offset(rr, ch);
        soff_b[x] = i8_lds_offset(kI8BM + rr, ch);
    }
    // operand reads: rows wr/wc + 32 x + l32 (swizzle depends on l32 only), chunk 2 ks + h
    const int swz = i8_swizzle(l32);
    const int rda = (wr + l32) * kI8BK, rdb = (kI8BM + wc + l32) * kI8BK;

    int li = 1, lj = s, lk = kb;  // next stage to load
    int ci = 1, cj = s, ck = kb;  // stage in LDS
    v4i ra[4], rb[4];  // native vectors (HIP's uint4 is a struct whose copies become memcpy)
#define ZE_I8_LOAD()                                                              \
    do {                                                                          \
        const signed char* A_ = pa + (size_t)(li - 1) * sA + lk * kI8BK;          \
        const signed char* B_ = pb + (size_t)(lj - 1) * sB + lk * kI8BK;          \
        _Pragma("unroll") for (int x = 0; x < 4; ++x) {                           \
            ra[x] = *reinterpret_cast<const v4i*>(A_ + x * xstep);                \
            rb[x] = *reinterpret_cast<const v4i*>(B_ + x * xstep);                \
        }                                                                         \
        if (++lk == ke) {                                                         \
            lk = kb;                                                              \
            i8_next_pair(li, lj);                                                 \
        }                                                                         \
    } while (0)
#define ZE_I8_STORE(st)                                                           \
    do {                                                                          \
        _Pragma("unroll") for (int x = 0; x < 4; ++x) {                           \
            *reinterpret_cast<v4i*>((st) + soff_a[x]) = ra[x];                    \
            *reinterpret_cast<v4i*>((st) + soff_b[x]) = rb[x];                    \
        }                                                                         \
    } while (0)

    ZE_I8_LOAD();
    ZE_I8_STORE(sm.stage);
    __syncthreads();
    for (int it = 0; it < total; ++it) {
        const bool more = it + 1 < total;
        if (more) ZE_I8_LOAD();
        __builtin_amdgcn_sched_barrier(0);
        const signed char* st = sm.stage + (it & 1) * kI8Stage;
        // software-pipelined operand reads: the 4 fragments of k-step ks + 1 are read while
        // the 4 MFMAs of k-step ks run; the next stage goes to the other LDS buffer after the
        // last k-step's MFMAs are issued, when its global loads have had the most time to land
        v4i fa[2][2], fb[2][2];
#define ZE_I8_READ(ks, slot)                                                              \
    do {                                                                                  \
        const int chunk_ = (((ks) * 2 + h) ^ swz) << 4;                                   \
        _Pragma("unroll") for (int x = 0; x < 2; ++x) {                                   \
            fa[slot][x] = *reinterpret_cast<const v4i*>(st + rda + x * 32 * kI8BK + chunk_); \
            fb[slot][x] = *reinterpret_cast<const v4i*>(st + rdb + x * 32 * kI8BK + chunk_); \
        }                                                                                 \
    } while (0)
        ZE_I8_READ(0, 0);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            if (ks < 3) ZE_I8_READ(ks + 1, (ks + 1) & 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[ks & 1][a], fb[ks & 1][c], acc[a][c], 0, 0, 0);
            if (ks == 3 && more) ZE_I8_STORE(sm.stage + ((it + 1) & 1) * kI8Stage);
            __builtin_amdgcn_sched_barrier(0);
        }
#undef ZE_I8_READ
        if (ck == ke - 1 && cj == 1) {  // last stage of the last pair of this t
            int* g = G + (size_t)(ci + cj - 2) * N * M2;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int cc = cc0 + wc + 32 * c + l32;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row = row0 + wr + 32 * a + 8 * (r >> 2) + 4 * h + (r & 3);
                        if (row < N && cc < M2) {
                            if (add)
                                atomicAdd(g + (size_t)row * M2 + cc, acc[a][c][r]);
                            else
                                g[(size_t)row * M2 + cc] = acc[a][c][r];
                        }
                    }
                    acc[a][c] = (v16i)0;
                }
        }
        if (++ck == ke) {
            ck = kb;
            i8_next_pair(ci, cj);
        }
        __syncthreads();
    }
#undef ZE_I8_LOAD
#undef ZE_I8_STORE
}

// ------------------------------------------------- INT8 residue products, 256 x 256 tiles
// The modular form's products (one per modulus) use a larger tile than zgemm_i8_tile's:
// 256 rows x 256 real columns with 8 waves of
// 128 x 64 (4 x 2 tiles of v_mfma_i32_32x32x32_i8): per MFMA half the global bytes and 3/4
// of the LDS operand reads of the 128 x 128 tile.  LDS: two 64 KiB stages.  Same operand
// layout, LDS row swizzle and stage pipeline as zgemm_i8_tile.
constexpr int kI8LM = 256, kI8LN = 256, kI8LThreads = 512;
constexpr int kI8LStage = (kI8LM + kI8LN) * kI8BK;

struct I8LSmem {
    signed char stage[2 * kI8LStage] __attribute__((aligned(16)));
};

// Byte slabs G8[j] (N x N) of tile (ti, tj) for the residue slab pairs j = j0 .. j0 + s - 1
// (three per modulus, see crt_row_block), from sa and sb (crt_rows_pad(N) x ldk bytes per
// slab, slab j at offset j times that), over the K stages [kb, ke): each int32 sum is stored
// reduced modulo p_(j / 3).
__device__ __forceinline__ void zgemm_i8_tile_large(int ti, int tj, const signed char* __restrict__ sa,
                                                    const signed char* __restrict__ sb,
                                                    unsigned char* __restrict__ G8, int N, int j0,
                                                    int s, int ldk, I8LSmem& sm, int kb, int ke) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int row0 = ti * kI8LM, cc0 = tj * kI8LN, M2 = N;  // N output columns per slab
    const size_t sA = (size_t)crt_rows_pad(N) * ldk, sB = sA;
    sa += (size_t)j0 * sA;
    sb += (size_t)j0 * sB;
    G8 += (size_t)j0 * N * M2;
    const int total = s * (ke - kb);
    const int wr = (wave >> 2) * 128, wc = (wave & 3) * 64;
    const int l32 = lane & 31, h = lane >> 5;

    v16i acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = (v16i)0;

    // thread's x-th 16-byte piece of a stage: row (tid / 8) + 64 x, bytes 16 (tid % 8) ..
    const signed char* pa = sa + (size_t)(row0 + (tid >> 3)) * ldk + (tid & 7) * 16;
    const signed char* pb = sb + (size_t)(cc0 + (tid >> 3)) * ldk + (tid & 7) * 16;
    const size_t xstep = (size_t)(kI8LThreads / 8) * ldk;
    int soff_a[4], soff_b[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int rr = (tid >> 3) + 64 * x, ch = tid & 7;
        soff_a[x] = i8_lds_offset(rr, ch);
        soff_b[x] = i8_lds_offset(kI8LM + rr, ch);
    }
    const int swz = i8_swizzle(l32);
    const int rda = (wr + l32) * kI8BK, rdb = (kI8LM + wc + l32) * kI8BK;

    // next stage to load: K stage lk of the modulus whose slabs start at A_ / B_
    int lk = kb;
    const signed char* A_ = pa + kb * kI8BK;
    const signed char* B_ = pb + kb * kI8BK;
    const size_t wrapA = sA - (size_t)(ke - kb) * kI8BK, wrapB = sB - (size_t)(ke - kb) * kI8BK;
    int cm = 0, ck = kb;  // stage in LDS
    v4i ra[4], rb[4];
#define ZE_I8L_LOAD()                                                             \
    do {                                                                          \
        _Pragma("unroll") for (int x = 0; x < 4; ++x) {                           \
            ra[x] = *reinterpret_cast<const v4i*>(A_ + x * xstep);                \
            rb[x] = *reinterpret_cast<const v4i*>(B_ + x * xstep);                \
        }                                                                         \
        A_ += kI8BK;                                                              \
        B_ += kI8BK;                                                              \
        if (++lk == ke) {                                                         \
            lk = kb;                                                              \
            A_ += wrapA;                                                          \
            B_ += wrapB;                                                          \
        }                                                                         \
    } while (0)
#define ZE_I8L_STORE(st)                                                          \
    do {                                                                          \
        _Pragma("unroll") for (int x = 0; x < 4; ++x) {                           \
            *reinterpret_cast<v4i*>((st) + soff_a[x]) = ra[x];                    \
            *reinterpret_cast<v4i*>((st) + soff_b[x]) = rb[x];                    \
        }                                                                         \
    } while (0)

    ZE_I8L_LOAD();
    ZE_I8L_STORE(sm.stage);
    __syncthreads();
    for (int it = 0; it < total; ++it) {
        const bool more = it + 1 < total;
        if (more) ZE_I8L_LOAD();
        __builtin_amdgcn_sched_barrier(0);
        const signed char* st = sm.stage + (it & 1) * kI8LStage;
        v4i fa[4], fb[2];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int chunk = ((ks * 2 + h) ^ swz) << 4;
#pragma unroll
            for (int x = 0; x < 4; ++x)
                fa[x] = *reinterpret_cast<const v4i*>(st + rda + x * 32 * kI8BK + chunk);
#pragma unroll
            for (int x = 0; x < 2; ++x)
                fb[x] = *reinterpret_cast<const v4i*>(st + rdb + x * 32 * kI8BK + chunk);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[c], acc[a][c], 0, 0, 0);
            if (ks == 3 && more) ZE_I8L_STORE(sm.stage + ((it + 1) & 1) * kI8LStage);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (ck == ke - 1) {  // last K stage of modulus cm: flush its accumulators to G[cm]
            // the row stride passes through an empty asm statement so that the 128 output
            // addresses are formed here, not kept in registers across the whole loop
            int m2 = M2;
            asm volatile("" : "+v"(m2));
            unsigned char* g8 = G8 + (size_t)cm * N * M2;
            const int p = crt_modulus((j0 + cm) / 3);
            const double rp = 1.0 / (double)p;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int cc = cc0 + wc + 32 * c + l32;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int row = row0 + wr + 32 * a + 8 * (r >> 2) + 4 * h + (r & 3);
                        if (row < N && cc < M2) {
                            const int v = acc[a][c][r];
                            int t = v - (int)floor((double)v * rp) * p;
                            t = t < 0 ? t + p : (t >= p ? t - p : t);
                            g8[(size_t)row * m2 + cc] = (unsigned char)t;
                        }
                    }
                    acc[a][c] = (v16i)0;
                }
        }
        if (++ck == ke) {
            ck = kb;
            ++cm;
        }
        __syncthreads();
    }
#undef ZE_I8L_LOAD
#undef ZE_I8L_STORE
}

// Element e (row-major complex index) of C = 2^(ea_r + eb_c) sum_{t=2}^{s+1} 2^(2 - 8t) G[t-2].
__device__ __forceinline__ double2 split_combine_elem(const int* __restrict__ G, const int* __restrict__ ea,
                                             const int* __restrict__ eb, int N, int s, size_t e) {
    const size_t slab = 2 * (size_t)N * N;
    const int r = (int)(e / N), c = (int)(e - (size_t)r * N);
    double vr = 0.0, vi = 0.0;
    for (int t = s + 1; t >= 2; --t) {
        const int2 g = *reinterpret_cast<const int2*>(G + (size_t)(t - 2) * slab + 2 * e);
        const double w = ldexp(1.0, 2 - 8 * t);
        vr += w * (double)g.x;
        vi += w * (double)g.y;
    }
    const int ex = ea[r] + eb[c];
    return make_double2(ldexp(vr, ex), ldexp(vi, ex));
}

}  // namespace zk

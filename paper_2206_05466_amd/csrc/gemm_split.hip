// Split-precision complex products: FP64 matrix products emulated on INT8 MFMA
// (v_mfma_i32_32x32x32_i8) by the error-free splitting of Ozaki, Ogita, Oishi & Rump,
// "Error-free transformations of matrix multiplication by using fast routines of matrix
// multiplication and its applications", Numer. Algorithms 59 (2012), in its integer form
// (Ootomo, Ozaki & Yokota, "DGEMM on integer matrix multiplication unit", 2024).
//
// The products are the two of the fixed-point map (Sec. 3.1, eq. (isomp_iter)).  As in the
// FP64 kernels, a complex product C = A B is the real product C~ = A~ B~ of the interleaved
// A~ (N x 2N) and the 2 x 2-block form B~ (2N x 2N) of B.
//
// Splitting.  Row r of A~ is scaled by 2^-ea_r (ea_r chosen so the largest magnitude becomes
// at most 0.99) and written as s balanced digits (split_digits in split_tile.h): the row value
// rounded to a multiple of 2^(1 - 8s), then cut into a top digit in [-127, 127] (7 bits) and
// s - 1 digits in [-128, 127] (8 bits each), y = sum_i a_i 2^(1 - 8i) + R, |R| <= 2^(-8s).
// Column cc of B~ likewise with 2^-eb_c (one exponent per complex column c).  Then
//     C~[r][cc] ~= 2^(ea_r + eb_c) sum_{i + j <= s + 1} 2^(2 - 8 (i + j)) (a_i b_j)[r][cc],
// the products of one t = i + j summed exactly in int32 ((t-1) 2N 128^2 < 2^31: the slice
// count is capped by split_max_slices(N)), then weighted and added in FP64 in a fixed order.
// The neglected terms (the roundings R and the pairs with t > s + 1) are about 2^(-8s)
// relative to max|row of A~| max|column of B~| per term of the K sum, and zero-mean.
//
// Column exponents of a skew-Hermitian B equal its row exponents (|B[k][c]| = |B[c][k]| entry
// by entry, exactly), so the product Q = A P of the fixed-point map reuses the row exponents
// of P from the product P W~ instead of a column pass.
//
// Slices: A~ slices row-major [r][kk] (N x 2N bytes each); B~ slices transposed,
// B~^T[cc][kk] (2N x 2N bytes each), which is the MFMA's B-operand order (K contiguous).
//
// Modular form (ZE_PREC_CRT; Ozaki scheme II: Ozaki, Uchino & Imamura, "Ozaki scheme II: a
// GEMM-oriented emulation of floating-point matrix multiplication using an integer modular
// technique", 2025).  Rows of A~ and columns of B~ are scaled by powers of two to integers of
// at most b bits, exactly, up to the one rounding to an integer; their residues modulo 16
// pairwise coprime moduli <= 256 are stored for the real part, the imaginary part and their
// sum; three exact INT8 products per modulus (ar br, ai bi, (ar + ai)(br + bi)) give the real
// and imaginary parts of the complex product modulo p_k, and the Chinese remainder theorem
// recovers the integer product exactly, since b is chosen so that 2N 2^(2b) < M / 2,
// M = prod p_k ~ 2^125.2.  The only error is the rounding of the scaled inputs to integers,
// 2^-b relative to the row / column maximum, with b = 55 up to N = 8192: FP64-level accuracy
// from 48 INT8 products of N x N x N.

#include <cmath>

#include "split_tile.h"
#include "update_tile.h"

namespace {

using namespace zk;

constexpr int kThreads = kSThreads;

// One block per row r of A~.
__global__ __launch_bounds__(kThreads) void split_rows_kernel(const double2* __restrict__ A,
                                                              int N, int s, int ldk,
                                                              signed char* __restrict__ slices,
                                                              int* __restrict__ ea,
                                                              const int* __restrict__ skip) {
    __shared__ double red[kThreads];
    if (skip && *skip) return;  // on-device stopping: the step has converged
    split_row_block(A, N, blockIdx.x, s, ldk, slices, ea, red);
}

// Column maxima of B (complex N x N, row-major), two stages: block (x, y) takes 256
// columns over the row chunk y; then one thread per column combines the chunks.
constexpr int kColChunks = 64;
__global__ __launch_bounds__(kThreads) void col_max_partial(const double2* __restrict__ B, int N,
                                                            double* __restrict__ part,
                                                            const int* __restrict__ skip) {
    if (skip && *skip) return;  // on-device stopping: the step has converged
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
                                                                int N, int* __restrict__ eb,
                                                                const int* __restrict__ skip) {
    if (skip && *skip) return;  // on-device stopping: the step has converged
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= N) return;
    double m = 0.0;
    for (int y = 0; y < kColChunks; ++y) m = fmax(m, part[(size_t)y * N + c]);
    eb[c] = exponent_of(m);
}

__global__ __launch_bounds__(kThreads) void split_cols_kernel(const double2* __restrict__ B,
                                                              int N, int s, int ldk,
                                                              const int* __restrict__ eb,
                                                              signed char* __restrict__ slices,
                                                              const int* __restrict__ skip) {
    __shared__ double2 tile[kCT][kCT + 1];
    if (skip && *skip) return;  // on-device stopping: the step has converged
    split_cols_tile(B, N, blockIdx.x, blockIdx.y, s, ldk, eb, slices, tile);
}

// Residue form of A~ (one block per row) and of B~^T (tiles as split_cols_kernel).
__global__ __launch_bounds__(kThreads) void crt_rows_kernel(const double2* __restrict__ A, int N,
                                                            int b, int ldk,
                                                            signed char* __restrict__ slices,
                                                            int* __restrict__ ea,
                                                            const int* __restrict__ skip) {
    __shared__ double red[kThreads];
    if (skip && *skip) return;  // on-device stopping: the step has converged
    crt_row_block(A, N, blockIdx.x, b, ldk, slices, ea, red);
}

__global__ __launch_bounds__(kThreads) void crt_cols_kernel(const double2* __restrict__ B, int N,
                                                            int b, int ldk,
                                                            const int* __restrict__ eb,
                                                            signed char* __restrict__ slices,
                                                            const int* __restrict__ skip) {
    __shared__ double2 tile[kCT][kCT + 1];
    if (skip && *skip) return;  // on-device stopping: the step has converged
    crt_cols_tile(B, N, blockIdx.x, blockIdx.y, b, ldk, eb, slices, tile);
}

// Representatives of the residues of the real and imaginary parts of one output value from its
// P1, P2, P3 (bytes sh .. sh + 7 of the loaded words, each in [0, p_k)): Re = P1 - P2 + p_k in
// [1, 2 p_k), Im = P3 - P1 - P2 + 2 p_k in [1, 3 p_k), left unreduced (the CRT sums take them;
// a reduction would cost two compares and selects per value and modulus).
__device__ __forceinline__ void crt_parts_to_residues(unsigned p1, unsigned p2, unsigned p3, int sh,
                                                      int p, int& re, int& im) {
    const int a = (int)((p1 >> sh) & 0xffu), b = (int)((p2 >> sh) & 0xffu);
    const int c = (int)((p3 >> sh) & 0xffu);
    re = a - b + p;
    im = c + 2 * p - a - b;
}

// C[e] from the residue products, three N x N byte slabs per modulus k (P1 = ar br,
// P2 = ai bi, P3 = (ar + ai)(br + bi), each reduced modulo p_k): Re = P1 - P2 and
// Im = P3 - P1 - P2 modulo p_k through the CRT, then scaled by 2^(ea_r + eb_c - 2b).  Four
// consecutive outputs 4v .. 4v + 3 per thread (one 32-bit load of each slab) when N^2 is a
// multiple of 4 (so every slab starts 4-byte aligned); otherwise one output per thread.
__global__ __launch_bounds__(kThreads) void crt_combine_kernel(const unsigned char* __restrict__ G8,
                                                               const int* __restrict__ ea,
                                                               const int* __restrict__ eb,
                                                               double2* __restrict__ Cm, int N,
                                                               int b,
                                                               const int* __restrict__ skip) {
    if (skip && *skip) return;  // on-device stopping: the step has converged
    const size_t n2 = (size_t)N * N;
    const size_t n4 = n2 % 4 == 0 ? n2 / 4 : 0;
    const unsigned* G32 = reinterpret_cast<const unsigned*>(G8);
    for (size_t v = (size_t)blockIdx.x * kThreads + threadIdx.x; v < n4;
         v += (size_t)gridDim.x * kThreads) {
        CrtAcc ar[4], ai[4];
#pragma unroll
        for (int k = 0; k < kCrtMods; ++k) {
            const size_t o = (size_t)(3 * k) * n4 + v;
            const unsigned p1 = G32[o], p2 = G32[o + n4], p3 = G32[o + 2 * n4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int re, im;
                crt_parts_to_residues(p1, p2, p3, 8 * j, kCrtP[k], re, im);
                ar[j].add(k, re);
                ai[j].add(k, im);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const size_t e = 4 * v + j;
            const int r = (int)(e / N), c = (int)(e - (size_t)r * N);
            const int sh = ea[r] + eb[c] - 2 * b;
            Cm[e] = make_double2(ldexp(ar[j].value(), sh), ldexp(ai[j].value(), sh));
        }
    }
    for (size_t e = 4 * n4 + (size_t)blockIdx.x * kThreads + threadIdx.x; e < n2;
         e += (size_t)gridDim.x * kThreads) {
        CrtAcc ar, ai;
#pragma unroll
        for (int k = 0; k < kCrtMods; ++k) {
            const size_t o = (size_t)(3 * k) * n2 + e;
            int re, im;
            crt_parts_to_residues(G8[o], G8[o + n2], G8[o + 2 * n2], 0, kCrtP[k], re, im);
            ar.add(k, re);
            ai.add(k, im);
        }
        const int r = (int)(e / N), c = (int)(e - (size_t)r * N);
        const int sh = ea[r] + eb[c] - 2 * b;
        Cm[e] = make_double2(ldexp(ar.value(), sh), ldexp(ai.value(), sh));
    }
}

// mode 0: full product (tiles_m x tiles_n tiles), mode 1: lower-triangle tiles (ntiles of
// them in i8_lower_tile's numbering).  Blocks b < full take one whole tile each; the
// remaining tiles (a last, partial round of the GPU's block slots) are split along K: block
// full + S t + p takes part p of tile full + t and adds its sums to the cleared slabs.
__device__ __forceinline__ void i8_tile_of(int mode, int tile, int tiles_n, int ntiles, bool xcd,
                                           int b, int& ti, int& tj) {
    if (mode == 1) {
        i8_lower_tile(tile, ti, tj);
        return;
    }
    const int tm = ntiles / tiles_n;
    if (xcd && tm % 2 == 0 && tiles_n % 4 == 0) {
        // XCD-aware order: blocks b with b % 8 == x run on XCD x.  With the tile grid split
        // into 2 x 4 regions, XCD x takes region (x / 4, x % 4), walked in 8 x 8 super-tiles,
        // so the tiles an XCD holds at once share A~ and B~^T panels in its L2.
        const int x = b & 7, L = b >> 3;
        const int rm = tm / 2, rn = tiles_n / 4;
        int r, c;
        if (rm % 8 == 0 && rn % 8 == 0) {
            const int sg = L >> 6, w = L & 63, spr = rn / 8;
            r = (sg / spr) * 8 + (w >> 3);
            c = (sg % spr) * 8 + (w & 7);
        } else {
            r = L / rn;
            c = L % rn;
        }
        ti = (x >> 2) * rm + r;
        tj = (x & 3) * rn + c;
    } else {
        ti = tile / tiles_n;
        tj = tile % tiles_n;
    }
}

__global__ __launch_bounds__(kThreads, 2) void zgemm_i8_kernel(
    const signed char* __restrict__ sa, const signed char* __restrict__ sb, int* __restrict__ G,
    int N, int s, int ldk, int mode, int tiles_n, int ntiles, int full, int S,
    const int* __restrict__ skip) {
    __shared__ I8Smem sm;
    if (skip && *skip) return;  // on-device stopping: the step has converged
    int ti, tj;
    const int b = blockIdx.x;
    if (b < full) {
        i8_tile_of(mode, b, tiles_n, ntiles, full == ntiles, b, ti, tj);
        if (tj >= tiles_n) return;  // ragged N: block idle (uniform)
        zgemm_i8_tile(ti, tj, sa, sb, G, N, s, ldk, sm, 0, -1, false);
    } else {
        const int e = b - full, p = e % S, nk = ldk / kI8BK;
        i8_tile_of(mode, full + e / S, tiles_n, ntiles, false, b, ti, tj);
        if (tj >= tiles_n) return;
        zgemm_i8_tile(ti, tj, sa, sb, G, N, s, ldk, sm, (int)((long long)p * nk / S),
                      (int)((long long)(p + 1) * nk / S), true);
    }
}

// Clears the slabs G[0..s-1] (N x ncols each) over the tiles full .. ntiles-1 (the K-split
// ones) of bm x bn tiles; grid (ntiles - full, s).
__global__ __launch_bounds__(kThreads) void i8_clear_tail(int* __restrict__ G, int N, int mode,
                                                          int tiles_n, int ntiles, int full,
                                                          int bm, int bn, int ncols,
                                                          const int* __restrict__ skip) {
    if (skip && *skip) return;  // on-device stopping: the step has converged
    int ti, tj;
    i8_tile_of(mode, full + blockIdx.x, tiles_n, ntiles, false, 0, ti, tj);
    const int M2 = ncols;
    if (tj >= tiles_n) return;
    int* g = G + (size_t)blockIdx.y * N * M2;
    for (int x = threadIdx.x; x < bm * bn; x += kThreads) {
        const int row = ti * bm + x / bn, cc = tj * bn + x % bn;
        if (row < N && cc < M2) g[(size_t)row * M2 + cc] = 0;
    }
}

// The modular form's residue products on 256 x 256 tiles (zgemm_i8_tile_large) over the N x N
// output: block b takes part b % S of the K stages of tile b / S and writes its byte residues
// to part region b % S of G8 (regions of 3 kCrtMods N^2 bytes).
// Block b: slab group g = b / ntiles (slabs [g s / G, (g + 1) s / G), whole moduli when G
// divides the modulus count) of tile b % ntiles, over all of K.  Within a group, consecutive
// blocks run on consecutive XCDs; with whole rounds of 8 the XCD-aware tile order keeps the
// tiles an XCD holds at once on shared panels.
__global__ __launch_bounds__(kI8LThreads, 1) void zgemm_i8_large_kernel(
    const signed char* __restrict__ sa, const signed char* __restrict__ sb,
    unsigned char* __restrict__ G8, int N, int s, int ldk, int tiles_n, int ntiles, int G,
    const int* __restrict__ skip) {
    __shared__ I8LSmem sm;
    if (skip && *skip) return;  // on-device stopping: the step has converged
    const int b = blockIdx.x, g = b / ntiles, tile = b % ntiles;
    int ti, tj;
    i8_tile_of(0, tile, tiles_n, ntiles, ntiles % 8 == 0, tile, ti, tj);
    if (tj >= tiles_n) return;
    const int j0 = g * s / G, j1 = (g + 1) * s / G;
    zgemm_i8_tile_large(ti, tj, sa, sb, G8, N, j0, j1 - j0, ldk, sm, 0, ldk / kI8BK);
}

__global__ __launch_bounds__(kThreads) void split_combine_kernel(const int* __restrict__ G,
                                                                 const int* __restrict__ ea,
                                                                 const int* __restrict__ eb,
                                                                 double2* __restrict__ Cm, int N,
                                                                 int s,
                                                                 const int* __restrict__ skip) {
    if (skip && *skip) return;  // on-device stopping: the step has converged
    const size_t n2 = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * kThreads + threadIdx.x; e < n2;
         e += (size_t)gridDim.x * kThreads)
        Cm[e] = split_combine_elem(G, ea, eb, N, s, e);
}

// ---------------------------------------------------------------- fixed-point update
template <int UT, bool SLABS>
__global__ __launch_bounds__(kThreads) void lower_update_kernel(
    const double2* __restrict__ Qf, const int* __restrict__ G, const int* __restrict__ ea,
    const int* __restrict__ eb, int s, const double2* __restrict__ Am,
    const double2* __restrict__ Wn, const double2* Wt, double2* F, double2* __restrict__ Wout,
    double* __restrict__ rowpart, int N, double h, int form, const int* __restrict__ skip) {
    __shared__ double2 sT[UT][UT + 1];
    if (skip && *skip) return;  // on-device stopping: the step has converged
    const int b = blockIdx.x;
    int I = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    while (I * (I + 1) / 2 > b) --I;
    const int J = b - I * (I + 1) / 2;
    lower_update_tile_t<UT, SLABS>(I, J, Qf, G, ea, eb, s, Am, Wn, Wt, F, Wout, rowpart, N, h, form,
                                   sT);
}

}  // namespace

int ze_split_ldk(int N) { return split_ldk_of(N); }

hipError_t ze_i8_capacity(int* cap, int* cap_large) {
    int dev = 0, cus = 0, nb = 0, nl = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, zgemm_i8_kernel, kThreads, 0);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nl, zgemm_i8_large_kernel, kI8LThreads, 0);
    if (e != hipSuccess) return e;
    *cap = (nb > 0 ? nb : 1) * cus;
    *cap_large = (nl > 0 ? nl : 1) * cus;
    return hipSuccess;
}

// Slices of the product A = P W~ (lower == 0) or of the lower product Q = A P (lower != 0).
static int slices_of(const ze_ctx* c, int lower) {
    return lower ? c->split_slices_low : c->split_slices;
}

hipError_t launch_split_prepare(const ze_ctx* c, const double2* A, const double2* B, int* ea,
                                int* eb, bool eb_known, int lower, hipStream_t st) {
    const int N = c->N, s = slices_of(c, lower), ldk = ze_split_ldk(N);
    hipLaunchKernelGGL(split_rows_kernel, dim3(N), dim3(kThreads), 0, st, A, N, s, ldk, c->split_a,
                       ea, c->skip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!eb_known) {
        const int gx = (N + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(col_max_partial, dim3(gx, kColChunks), dim3(kThreads), 0, st, B, N,
                           c->split_colmax, c->skip);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(col_exponent_kernel, dim3(gx), dim3(kThreads), 0, st, c->split_colmax,
                           N, eb, c->skip);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    dim3 g((N + kCT - 1) / kCT, (ldk / 2 + kCT - 1) / kCT);
    hipLaunchKernelGGL(split_cols_kernel, g, dim3(kThreads), 0, st, B, N, s, ldk, eb, c->split_b, c->skip);
    return hipGetLastError();
}

hipError_t launch_zgemm_split(const ze_ctx* c, const double2* A, const double2* B, double2* C,
                              int lower, int* ea, int* eb, bool eb_known, hipStream_t st) {
    const int N = c->N, s = slices_of(c, lower);
    hipError_t e = launch_split_prepare(c, A, B, ea, eb, eb_known, lower, st);
    if (e != hipSuccess) return e;
    const int tr = (N + kI8BM - 1) / kI8BM;
    const int tn = (2 * N + kI8BN - 1) / kI8BN;
    const int ntiles = lower ? tr * (tr + 1) : tr * tn;
    const int nk = ze_split_ldk(N) / kI8BK;
    // whole tiles one block each, the rest split along K into S parts (at least 4 stages each,
    // summed by integer atomics), by the rule of the FP64 products: the busiest CU's stages,
    // ceil(full / cus) nk + ceil(tail S / cus) ceil(nk / S), minimised over whole tiles in
    // rounds of the block slots or in multiples of the CU count (ties: the larger S; the
    // tail's blocks fit in the slots beside the last whole round)
    int full = ntiles, S = 1;
    {
        const int cap = c->cap_i8 > 0 ? c->cap_i8 : ntiles, cus = c->cus > 0 ? c->cus : 1;
        auto busiest = [&](long long n) { return (n + cus - 1) / cus; };
        long long best = busiest(ntiles) * nk;
        for (int f : {(ntiles / cap) * cap, (ntiles / cus) * cus}) {
            const int rem = ntiles - f;
            if (rem <= 0) continue;
            int smax = nk / 4;
            if (smax > (cap - f % cap) / rem) smax = (cap - f % cap) / rem;
            for (int sp = 2; sp <= smax; ++sp) {
                const long long L = busiest(f) * nk + busiest((long long)rem * sp) * ((nk + sp - 1) / sp);
                if (L <= best) {
                    best = L;
                    full = f;
                    S = sp;
                }
            }
        }
    }
    if (full < ntiles) {
        hipLaunchKernelGGL(i8_clear_tail, dim3(ntiles - full, s), dim3(kThreads), 0, st, c->split_g,
                           N, lower ? 1 : 0, tn, ntiles, full, kI8BM, kI8BN, 2 * N, c->skip);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(zgemm_i8_kernel, dim3(full + (ntiles - full) * S), dim3(kThreads), 0, st,
                       c->split_a, c->split_b, c->split_g, N, s, ze_split_ldk(N), lower ? 1 : 0, tn,
                       ntiles, full, S, c->skip);
    e = hipGetLastError();
    if (e != hipSuccess || lower) return e;
    const size_t n2 = (size_t)N * N;
    const unsigned grid = (unsigned)((n2 + kThreads - 1) / kThreads < 16384 ? (n2 + kThreads - 1) / kThreads : 16384);
    hipLaunchKernelGGL(split_combine_kernel, dim3(grid), dim3(kThreads), 0, st, c->split_g, ea, eb,
                       C, N, s, c->skip);
    return hipGetLastError();
}

int ze_crt_bits(int N) {
    double log2m = 0.0;
    for (int k = 0; k < kCrtMods; ++k) log2m += std::log2((double)kCrtP[k]);
    // 2N (0.99 2^b)^2 < M / 2
    const int b = (int)std::floor((log2m - 1.0 - std::log2(2.0 * N)) / 2.0 - 1e-9);
    return b < 55 ? b : 55;
}

// int32 words holding the 3 kCrtMods byte slabs (N x N bytes each) of the residue products.
size_t ze_crt_slab_ints(int N) { return ((size_t)3 * kCrtMods * N * (size_t)N + 3) / 4; }

int ze_crt_ldk(int N) { return ((N + kI8BK - 1) / kI8BK) * kI8BK; }

// Tiles of the modular product (256 x 256 over the N x N output).  When they fill at least
// one round of the block slots each tile is one block over all slabs; else the 3 kCrtMods
// slabs are split into G groups (G the largest divisor of 3 kCrtMods with ntiles G <= the
// slots), each block one tile and one group, so every block still runs the whole K of its
// slabs and flushes once per slab.
void ze_crt_plan(int N, int cap_blocks, int* ntiles, int* tn, int* G) {
    const int t = (N + kI8LM - 1) / kI8LM;
    *tn = t;
    *ntiles = t * t;
    *G = 1;
    const int cap = cap_blocks > 0 ? cap_blocks : *ntiles;
    for (int g = 3 * kCrtMods; g > 1; --g)
        if ((3 * kCrtMods) % g == 0 && (long long)*ntiles * g <= cap) {
            *G = g;
            break;
        }
}

hipError_t launch_zgemm_crt(const ze_ctx* c, const double2* A, const double2* B, double2* C,
                            hipStream_t st) {
    const int N = c->N, ldk = ze_crt_ldk(N), b = ze_crt_bits(N);
    hipLaunchKernelGGL(crt_rows_kernel, dim3(N), dim3(kThreads), 0, st, A, N, b, ldk, c->crt_a,
                       c->split_ea, c->skip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int gx = (N + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(col_max_partial, dim3(gx, kColChunks), dim3(kThreads), 0, st, B, N,
                       c->split_colmax, c->skip);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(col_exponent_kernel, dim3(gx), dim3(kThreads), 0, st, c->split_colmax, N,
                       c->split_eb, c->skip);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g((N + kCT - 1) / kCT, (ldk + kCT - 1) / kCT);
    hipLaunchKernelGGL(crt_cols_kernel, g, dim3(kThreads), 0, st, B, N, b, ldk, c->split_eb,
                       c->crt_b, c->skip);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int ntiles, tn, G;
    ze_crt_plan(N, c->cap_i8l, &ntiles, &tn, &G);
    unsigned char* G8 = reinterpret_cast<unsigned char*>(c->crt_g);
    hipLaunchKernelGGL(zgemm_i8_large_kernel, dim3(ntiles * G), dim3(kI8LThreads), 0, st,
                       c->crt_a, c->crt_b, G8, N, 3 * kCrtMods, ldk, tn, ntiles, G, c->skip);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t n2 = (size_t)N * N, per = n2 % 4 == 0 ? n2 / 4 : n2;  // outputs / thread: 4 or 1
    const size_t want = (per + kThreads - 1) / kThreads;  // one pass: no loop-carried addresses
    const unsigned grid = (unsigned)(want < 1 ? 1 : want);
    hipLaunchKernelGGL(crt_combine_kernel, dim3(grid), dim3(kThreads), 0, st, G8, c->split_ea,
                       c->split_eb, C, N, b, c->skip);
    return hipGetLastError();
}

hipError_t launch_lower_update(const ze_ctx* c, const double2* Q, const double2* A,
                               const double2* Wn, const double2* Wt, double2* F, double2* Wout,
                               double* rowpart, double h, const int* ea, const int* eb,
                               hipStream_t st, const int* skip) {
    const int N = c->N, ut = c->ut;
    const int T = (N + ut - 1) / ut;
    auto kern = Q ? (ut == 64 ? lower_update_kernel<64, false>
                              : (ut == 32 ? lower_update_kernel<32, false> : lower_update_kernel<16, false>))
                  : (ut == 64 ? lower_update_kernel<64, true>
                              : (ut == 32 ? lower_update_kernel<32, true> : lower_update_kernel<16, true>));
    hipLaunchKernelGGL(kern, dim3(T * (T + 1) / 2), dim3(kThreads), 0, st, Q, c->split_g, ea, eb,
                       slices_of(c, 1), A, Wn, Wt, F, Wout, rowpart, N, h, c->update_form, skip);
    return hipGetLastError();
}

// Device building blocks of the FP64 complex products (shared by the single-problem and the
// ensemble kernels).  See gemm_f64.hip for the method.
#pragma once

#include "internal.h"

namespace zk {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // 4 waves
constexpr int kBK = 8;         // complex k per LDS stage (16 real k = 4 MFMA k-steps)

// SB_: B~ itself in LDS (both rows of each 2 x 2 block, signs applied when the stage is
// stored: one plain read per operand, twice the B stage) or B as it lies in memory (each lane
// reads one component and applies a lane-constant sign).  The first is faster where LDS does
// not limit the blocks per CU (the full product), the second where it does (64 x 64 tiles).
template <int BM_, int BNC_, int WM_, int WNC_, bool SB_>
struct Cfg {
    static constexpr bool SB = SB_;
    static constexpr int BM = BM_;     // block rows
    static constexpr int BNC = BNC_;   // block columns (complex)
    static constexpr int WM = WM_;     // wave rows
    static constexpr int WNC = WNC_;   // wave columns (complex)
    static constexpr int MT = WM / 16;        // MFMA tiles per wave, rows
    static constexpr int NT = 2 * WNC / 16;   // MFMA tiles per wave, real columns
    static constexpr int WAVES_N = BNC / WNC;
    static constexpr int AS_LD = BM + 1;           // A stage: [16 real k][BM rows] (+1 pad)
    // B stage, SB: [16 real k rows of B~][2*BNC doubles] (+16 pad, so that the two rows one
    // MFMA k-step reads start 32 banks apart): row 2k holds (Re b, Im b) per column, row 2k+1
    // holds (-Im b, Re b).  Otherwise: [8 complex k][2*BNC doubles] (+2 pad).
    static constexpr int BS_LD = SB ? 2 * BNC + 16 : 2 * BNC + 2;
    static constexpr int AS = 2 * kBK * AS_LD;
    static constexpr int BS = (SB ? 2 : 1) * kBK * BS_LD;
    static constexpr int STAGE = AS + BS;          // doubles per stage
    static constexpr int A_LOADS = BM * kBK / kThreads;
    static constexpr int B_LOADS = kBK * BNC / kThreads;
    static_assert((BM / WM) * (BNC / WNC) == 4, "4 waves per block");
    static_assert(A_LOADS * kThreads == BM * kBK && B_LOADS * kThreads == kBK * BNC, "loads");
};

// Global -> register loads of one K stage (zero outside the matrices).
template <class C>
__device__ __forceinline__ void load_stage(const double2* __restrict__ A, int lda, int row0, int M,
                                  const double2* __restrict__ B, int ldb, int col0, int Nc,
                                  int K, int k0, double2 (&ra)[C::A_LOADS],
                                  double2 (&rb)[C::B_LOADS]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < C::A_LOADS; ++j) {
        const int idx = tid + j * kThreads;
        const int r = idx / kBK, kc = idx % kBK;
        const int gr = row0 + r, gk = k0 + kc;
        ra[j] = (gr < M && gk < K) ? A[(size_t)gr * lda + gk] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < C::B_LOADS; ++j) {
        const int idx = tid + j * kThreads;
        const int kc = idx / C::BNC, c = idx % C::BNC;
        const int gk = k0 + kc, gc = col0 + c;
        rb[j] = (gk < K && gc < Nc) ? B[(size_t)gk * ldb + gc] : make_double2(0.0, 0.0);
    }
}

template <class C>
__device__ __forceinline__ void store_stage(double* __restrict__ st, const double2 (&ra)[C::A_LOADS],
                                   const double2 (&rb)[C::B_LOADS]) {
    const int tid = threadIdx.x;
    double* as = st;
    double* bs = st + C::AS;
#pragma unroll
    for (int j = 0; j < C::A_LOADS; ++j) {
        const int idx = tid + j * kThreads;
        const int r = idx / kBK, kc = idx % kBK;
        as[(2 * kc) * C::AS_LD + r] = ra[j].x;
        as[(2 * kc + 1) * C::AS_LD + r] = ra[j].y;
    }
#pragma unroll
    for (int j = 0; j < C::B_LOADS; ++j) {
        const int idx = tid + j * kThreads;
        const int kc = idx / C::BNC, c = idx % C::BNC;
        if (C::SB) {
            *reinterpret_cast<double2*>(bs + (2 * kc) * C::BS_LD + 2 * c) = rb[j];
            *reinterpret_cast<double2*>(bs + (2 * kc + 1) * C::BS_LD + 2 * c) =
                make_double2(-rb[j].y, rb[j].x);
        } else {
            *reinterpret_cast<double2*>(bs + kc * C::BS_LD + 2 * c) = rb[j];
        }
    }
}

// MFMAs of one stage for this wave.
template <class C>
__device__ __forceinline__ void compute_stage(const double* __restrict__ st, int wrow, int wcc,
                                     d4 (&acc)[C::MT][C::NT]) {
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, l16 = lane & 15;
    const int t = q & 1;        // real-k parity: 0 -> Re(a) row of B~, 1 -> Im(a) row
    const int u = lane & 1;     // real-column parity: 0 -> Re(c), 1 -> Im(c)
    const double sgn = (t == 1 && u == 0) ? -1.0 : 1.0;
    const double* as = st;
    const double* bs = st + C::AS;
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
        const int kk = 4 * k4 + q;  // real k: row kk of B~
        const int kc = 2 * k4 + (q >> 1);
        double a[C::MT], b[C::NT];
#pragma unroll
        for (int mt = 0; mt < C::MT; ++mt) a[mt] = as[kk * C::AS_LD + wrow + mt * 16 + l16];
#pragma unroll
        for (int nt = 0; nt < C::NT; ++nt) {
            const int cc = wcc + nt * 16 + l16;
            b[nt] = C::SB ? bs[kk * C::BS_LD + cc] : sgn * bs[kc * C::BS_LD + (cc & ~1) + (t ^ u)];
        }
#pragma unroll
        for (int mt = 0; mt < C::MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < C::NT; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
    }
}

// acc = A[row0:row0+BM, K range] * B[K range, col0:col0+BNC] for the K stages [kb, ke),
// double-buffered in LDS.
template <class C>
__device__ __forceinline__ void mainloop(const double2* __restrict__ A, int lda, int row0, int M,
                                const double2* __restrict__ B, int ldb, int col0, int Nc, int K,
                                int kb, int ke, double* smem, d4 (&acc)[C::MT][C::NT]) {
    const int wave = threadIdx.x >> 6;
    const int wrow = (wave / C::WAVES_N) * C::WM;
    const int wcc = (wave % C::WAVES_N) * (2 * C::WNC);
#pragma unroll
    for (int mt = 0; mt < C::MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < C::NT; ++nt) acc[mt][nt] = d4{0.0, 0.0, 0.0, 0.0};
    if (kb >= ke) return;

    double2 ra[C::A_LOADS], rb[C::B_LOADS];
    load_stage<C>(A, lda, row0, M, B, ldb, col0, Nc, K, kb * kBK, ra, rb);
    store_stage<C>(smem, ra, rb);
    __syncthreads();
    for (int kt = kb; kt < ke; ++kt) {
        const bool more = kt + 1 < ke;
        const int buf = (kt - kb) & 1;
        if (more) load_stage<C>(A, lda, row0, M, B, ldb, col0, Nc, K, (kt + 1) * kBK, ra, rb);
        compute_stage<C>(smem + buf * C::STAGE, wrow, wcc, acc);
        if (more) store_stage<C>(smem + (buf ^ 1) * C::STAGE, ra, rb);
        __syncthreads();
    }
}

using FullCfg = Cfg<128, 64, 64, 32, true>;

// Store a block's accumulators (MFMA layout of config C) to C~ (complex N x N), bounds-checked.
template <class C>
__device__ __forceinline__ void store_tile(const d4 (&acc)[C::MT][C::NT], double2* Cm, int N, int row0,
                                  int col0) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wrow = (wave / C::WAVES_N) * C::WM;
    const int wcc = (wave % C::WAVES_N) * (2 * C::WNC);
    const int q = lane >> 4, l16 = lane & 15;
    double* Cd = reinterpret_cast<double*>(Cm);
    const size_t ld = 2 * (size_t)N;
#pragma unroll
    for (int mt = 0; mt < C::MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < C::NT; ++nt) {
            const int cc = 2 * col0 + wcc + nt * 16 + l16;
            if (cc >= 2 * N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + wrow + mt * 16 + q + 4 * r;
                if (row < N) Cd[(size_t)row * ld + cc] = acc[mt][nt][r];
            }
        }
}

__device__ __forceinline__ void store_full_tile(const d4 (&acc)[FullCfg::MT][FullCfg::NT], double2* Cm,
                                       int N, int row0, int col0) {
    store_tile<FullCfg>(acc, Cm, N, row0, col0);
}

// ---------------------------------------------------------------- small products
// Up to one tile per CU (N <= 512 on 256 CUs): one block per 32 x 32 complex tile of C.  Each
// of the 4 waves takes a contiguous quarter of K and holds the whole tile (2 x 4 MFMA tiles,
// 32 rows x 64 real columns).  A wave needs no LDS in its K loop: every lane loads from global
// memory exactly the double its MFMA operand is (A~ entry; B~ entry, whose sign the lane
// applies), kSmallDepth k-steps ahead in registers.  The quarters' sums are added in wave
// order through LDS at the end.  No split-K partial sums and no fix-up launch.
constexpr int kSmallTile = 32;
constexpr int kSmallDepth = 8;                         // k-steps of loads in flight per wave
constexpr int kSmallRed = 4 * 8 * 4 * 64;              // the 4 waves' sums (doubles)

// C[row0:row0+32, col0:col0+32] = A[row0:, :] B[:, col0:] (all N x N, leading dimension N),
// bounds-checked; red holds kSmallRed doubles of LDS.
__device__ __forceinline__ void small_product(const double2* __restrict__ A,
                                              const double2* __restrict__ B,
                                              double2* __restrict__ Cm, int N, int row0, int col0,
                                              double* red) {
    constexpr int P = kSmallDepth;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, l16 = lane & 15;
    const int t = q & 1;   // real-k parity of this lane's k-row: 0 -> Re(a) row of B~, 1 -> Im(a)
    const int u = l16 & 1; // real-column parity: 0 -> Re(c), 1 -> Im(c)
    // one k-step = 4 real k = 2 complex k; lanes q = 0, 1 take the first, q = 2, 3 the second
    const int kl = q >> 1;
    const int kq0 = (int)((long long)wave * N / 4), kq1 = (int)((long long)(wave + 1) * N / 4);
    const int nst = (kq1 - kq0 + 1) / 2;
    // Clamped indices keep every load in bounds.  Rows and columns beyond N feed only outputs
    // that are not stored; k beyond the quarter feeds only steps that are not computed, except
    // the second k of the last step of an odd-length quarter, which is zeroed through a.
    const int ra0 = min(row0 + l16, N - 1), ra1 = min(row0 + 16 + l16, N - 1);
    int cb[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) cb[nt] = min(col0 + nt * 8 + (l16 >> 1), N - 1);
    const int bcomp = t ^ u;  // B~[2k + t][2c + u] = +-(Re b, Im b)[t ^ u]
    const double bsgn = (t == 1 && u == 0) ? -1.0 : 1.0;
    const double* As = reinterpret_cast<const double*>(A);
    const double* Bs = reinterpret_cast<const double*>(B);
    d4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    double ring[P][6];
    auto issue = [&](int st, double (&r)[6]) {
        const int k = max(min(kq0 + 2 * st + kl, kq1 - 1), 0);
        r[0] = As[2 * ((size_t)ra0 * N + k) + t];
        r[1] = As[2 * ((size_t)ra1 * N + k) + t];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) r[2 + nt] = Bs[2 * ((size_t)k * N + cb[nt]) + bcomp];
    };
    auto mma = [&](const double (&r)[6], bool zero) {
        const double a0 = zero ? 0.0 : r[0], a1 = zero ? 0.0 : r[1];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double b = bsgn * r[2 + j];
            acc[0][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc[0][j], 0, 0, 0);
            acc[1][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc[1][j], 0, 0, 0);
        }
    };
    const bool odd_last = ((kq1 - kq0) & 1) && kl == 1;
#pragma unroll
    for (int p = 0; p < P; ++p) issue(p, ring[p]);
    int st = 0;
    for (; st + P < nst; st += P) {  // every step of the group has a successor group
#pragma unroll
        for (int p = 0; p < P; ++p) {
            mma(ring[p], false);
            issue(st + P + p, ring[p]);
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p)
        if (st + p < nst) mma(ring[p], odd_last && st + p == nst - 1);
    // the quarters' sums: each wave stores its 8 MFMA tiles, then wave w adds tiles 2w, 2w+1
    // over the four waves in wave order and stores them
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[((wave * 8 + i * 4 + j) * 4 + r) * 64 + lane] = acc[i][j][r];
    __syncthreads();
    double* Cd = reinterpret_cast<double*>(Cm);
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2) {
        const int tt = 2 * wave + t2, mt = tt / 4, nt = tt % 4;
        const int cc = 2 * col0 + nt * 16 + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double x = red[((0 * 8 + tt) * 4 + r) * 64 + lane];
            x += red[((1 * 8 + tt) * 4 + r) * 64 + lane];
            x += red[((2 * 8 + tt) * 4 + r) * 64 + lane];
            x += red[((3 * 8 + tt) * 4 + r) * 64 + lane];
            const int row = row0 + mt * 16 + q + 4 * r;
            if (row < N && cc < 2 * N) Cd[(size_t)row * 2 * N + cc] = x;
        }
    }
}

// ---------------------------------------------------------------- lower product + epilogue
using LowCfg = Cfg<64, 64, 32, 32, false>;
constexpr int kTile = 64;  // square complex tile of the lower-triangle product

// Tile index b of the lower triangle -> (I, J), I >= J, b = I (I+1)/2 + J.
__device__ __forceinline__ void lower_tile(int b, int& I, int& J) {
    int i = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= b) ++i;
    while (i * (i + 1) / 2 > b) --i;
    I = i;
    J = b - i * (i + 1) / 2;
}

}  // namespace zk

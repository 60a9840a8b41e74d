// Device body of the fixed-point update after the lower product (shared by the
// single-problem and the ensemble kernels).
#pragma once

#include "internal.h"

namespace zk {

// ---------------------------------------------------------------- fixed-point update
// For tile (I, J), I >= J, of UT x UT complex entries (UT = 64, 32 or 16: smaller tiles give a
// small N enough blocks), from Q (lower tiles valid):
//   F = Wn + h/2 (A - A^H) + h^2/4 Q   (Re Q_RR := 0),
//   Wout = Wt + h/2 (A - A^H) - h^2/4 Q   (form 0: the second line of eq. (isomp) at Wt), or
//   Wout = Wn + h (A - A^H)               (form 1: the two lines differ by h [P~, W~]; at a
//                                          stopped iterate the spectrum is then off by
//                                          O(h ||P|| residual) instead of O(residual)),
// lower entries written directly, upper ones (-conj) through an LDS transpose so every
// global access is a coalesced row segment.  Row sums of |F - Wt| go to slots
// rowpart[X*N + r] (tile-column X, row r): tile (I, J), I > J, writes the row sums of its
// entries to slots (J, rows of I) and their column sums (the mirrored upper entries, which
// lie in the rows of J) to slots (I, rows of J); a diagonal tile writes the full row sums of
// its rows to (I, rows of I).  Every slot with r < N is written once (deterministic sums).
constexpr int kUT = 64;  // the tile of the ensemble kernels (and of the single context from N = 2048)
constexpr int kUThreads = 256;
// Q comes from the FP64 lower product (Qf != nullptr, complex N x N, lower tiles) or from the
// int32 slabs of the split lower product (G, ea, eb, s).
// SLABS: Q from the slabs (Qf unused), else from Qf; each form is its own instance, so the
// registers the slab sums need do not cost the FP64 form occupancy.
template <int UT, bool SLABS = false>
__device__ __forceinline__ void lower_update_tile_t(int I, int J, const double2* __restrict__ Qf,
                                         const int* __restrict__ G, const int* __restrict__ ea,
                                         const int* __restrict__ eb, int s,
                                         const double2* __restrict__ Am,
                                         const double2* __restrict__ Wn, const double2* Wt,
                                         double2* F, double2* __restrict__ Wout,
                                         double* __restrict__ rowpart, int N, double h, int form,
                                         double2 (*sT)[UT + 1]) {
    static_assert(kUThreads % UT == 0 && 2 * UT <= kUThreads, "tile");
    constexpr int RP = kUThreads / UT;  // rows per pass; each thread takes UT / RP of them
    double(*sD)[UT + 1] = reinterpret_cast<double(*)[UT + 1]>(&sT[0][0]);  // reused at the end
    const int R0 = I * UT, C0 = J * UT;
    const int tid = threadIdx.x;
    const int lc = tid % UT, lr0 = tid / UT;  // RP rows per pass, UT consecutive columns
    const double h2 = 0.5 * h, h4 = 0.25 * h * h;

    // A^T tile: sT[c][R] = A[C0 + c][R0 + R].
    for (int rr = lr0; rr < UT; rr += RP) {
        const int gr = C0 + rr, gc = R0 + lc;
        sT[rr][lc] = (gr < N && gc < N) ? Am[(size_t)gr * N + gc] : make_double2(0.0, 0.0);
    }
    __syncthreads();

    double2 fv[UT / RP], wv[UT / RP];
    double dv[UT / RP];
#pragma unroll
    for (int x = 0; x < UT / RP; ++x) {
        const int r = lr0 + RP * x, R = R0 + r, c = C0 + lc;
        const bool ok = R < N && c < N && c <= R;
        double2 f = make_double2(0.0, 0.0), wo = f, d = f;
        if (ok) {
            const size_t o = (size_t)R * N + c;
            double2 qv = make_double2(0.0, 0.0);
            if (!SLABS) {
                qv = Qf[o];
            } else {  // Q = A P from the int32 slabs t = s + 1 .. 2, summed in that order
                int2 gv[kSplitMax];
#pragma unroll
                for (int u = 0; u < kSplitMax; ++u) {  // all loads first (s <= kSplitMax)
                    const int t = s + 1 - u;
                    gv[u] = t >= 2 ? *reinterpret_cast<const int2*>(G + (size_t)(t - 2) * 2 * N * N + 2 * o)
                                   : make_int2(0, 0);
                }
#pragma unroll
                for (int u = 0; u < kSplitMax; ++u) {
                    const int t = s + 1 - u;
                    if (t >= 2) {
                        const double w = ldexp(1.0, 2 - 8 * t);
                        qv.x += w * (double)gv[u].x;
                        qv.y += w * (double)gv[u].y;
                    }
                }
                const int ex = ea[R] + eb[c];
                qv.x = ldexp(qv.x, ex);
                qv.y = ldexp(qv.y, ex);
            }
            if (c == R) qv.x = 0.0;
            const double2 arc = Am[o], acr = sT[lc][r];
            const double cr = arc.x - acr.x, ci = arc.y + acr.y;  // (A - A^H)_{Rc}
            const double2 wn = Wn[o], wt = Wt[o];
            f = make_double2(wn.x + h2 * cr + h4 * qv.x, wn.y + h2 * ci + h4 * qv.y);
            wo = form == 1 ? make_double2(wn.x + h * cr, wn.y + h * ci)
                           : make_double2(wt.x + h2 * cr - h4 * qv.x, wt.y + h2 * ci - h4 * qv.y);
            d = make_double2(f.x - wt.x, f.y - wt.y);
            F[o] = f;
            Wout[o] = wo;
        }
        fv[x] = f;
        wv[x] = wo;
        dv[x] = ok ? sqrt(d.x * d.x + d.y * d.y) : 0.0;
    }
    __syncthreads();
    // Upper entries: F[c][R] = -conj(F[R][c]) for c < R, via sT.
    for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
        for (int x = 0; x < UT / RP; ++x) {
            const int r = lr0 + RP * x;
            const double2 v = pass == 0 ? fv[x] : wv[x];
            sT[lc][r] = make_double2(-v.x, v.y);
        }
        __syncthreads();
        double2* out = pass == 0 ? F : Wout;
        for (int cr = lr0; cr < UT; cr += RP) {  // row C0 + cr of the upper tile, columns R0 + lc
            const int gc = C0 + cr, gR = R0 + lc;
            if (gc < N && gR < N && gc < gR) out[(size_t)gc * N + gR] = sT[cr][lc];
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < UT / RP; ++x) sD[lr0 + RP * x][lc] = dv[x];
    __syncthreads();
    if (I != J) {
        if (tid < UT) {
            double sum = 0.0;
            for (int k = 0; k < UT; ++k) sum += sD[tid][k];
            if (R0 + tid < N) rowpart[(size_t)J * N + R0 + tid] = sum;
        } else if (tid < 2 * UT) {
            const int j = tid - UT;
            double sum = 0.0;
            for (int k = 0; k < UT; ++k) sum += sD[k][j];
            if (C0 + j < N) rowpart[(size_t)I * N + C0 + j] = sum;
        }
    } else if (tid < UT) {
        double sum = 0.0;
        for (int k = 0; k < UT; ++k) sum += sD[tid][k];
        for (int k = tid + 1; k < UT; ++k) sum += sD[k][tid];
        if (R0 + tid < N) rowpart[(size_t)I * N + R0 + tid] = sum;
    }
}


// Update tile of a single context of size N: 64 where its lower tiles number at least 4096
// (eight rounds of its two blocks per CU, so a partial last round costs little), else 32 where
// those number at least 512, else 16.  Measured: N = 2048, 528 tiles of 64 (one round and a
// tail of 16) 66 us against 47 us with 32 x 32 tiles; N = 4096, 2080 tiles of 64 (four rounds
// and a tail of 32) 243 us against 225 us.
// Row sum sum_X rowpart[X N + r] over the T slots of row r, added in slot order; the loads are
// issued B at a time, so a small N (many slots of few rows) waits for T / B memory latencies
// rather than T.
template <int B>
__device__ __forceinline__ double slot_row_sum(const double* __restrict__ rowpart, int T, int N,
                                               int r) {
    double v = 0.0;
    int X = 0;
    for (; X + B <= T; X += B) {
        double t[B];
#pragma unroll
        for (int u = 0; u < B; ++u) t[u] = rowpart[(size_t)(X + u) * N + r];
#pragma unroll
        for (int u = 0; u < B; ++u) v += t[u];
    }
    for (; X < T; ++X) v += rowpart[(size_t)X * N + r];
    return v;
}

__host__ __device__ inline int update_tile_of(int N) {
    const long long t64 = (N + 63) / 64, t32 = (N + 31) / 32;
    if (t64 * (t64 + 1) / 2 >= 4096) return 64;
    if (t32 * (t32 + 1) / 2 >= 512) return 32;
    return 16;
}

}  // namespace zk

// Complex FP64 matrix products on CDNA4 FP64 MFMA (v_mfma_f64_16x16x4_f64).
//
// The commutator and the P W~ P term of the fixed-point map (eq. (isomp_iter)) need two
// complex products per evaluation (Sec. 3.1): A = P W~ (full) and Q = A P, of which only the
// lower triangle is formed, since Q is skew-Hermitian; C = A - A^H and the update of W~ are
// applied afterwards by the coalesced update kernel (gemm_split.hip).
//
// Complex arithmetic on a real MFMA.  With X (M x K complex) stored interleaved (re, im),
// its memory is a real M x 2K matrix X~.  For B (K x N complex) let B~ be the real 2K x 2N
// matrix whose 2 x 2 block (k, c) is [[Re b, Im b], [-Im b, Re b]].  Then X~ B~ is exactly
// the interleaved storage of X B (8 M N K real flops), so the operands are read as they lie
// in memory and B~ is formed from the LDS copy of B: either written out when a stage is
// stored (both rows of each 2 x 2 block, signs applied there; the full product) or read per
// lane as one component of one B element with a lane-constant sign (the 64 x 64 tiles, where
// the smaller stage keeps three blocks per CU).
//
// MFMA operand layout (16x16x4, f64): lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator register r of lane l holds D[l/16 + 4*r][l%16].

#include <mutex>
#include <vector>

#include "tile_f64.h"
#include "update_tile.h"

namespace {

using namespace zk;

// Split-K partial accumulators, one block's registers in thread-major order.
template <class C>
__device__ inline void store_partial(double* __restrict__ part, const d4 (&acc)[C::MT][C::NT]) {
#pragma unroll
    for (int mt = 0; mt < C::MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < C::NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                part[((mt * C::NT + nt) * 4 + r) * kThreads + threadIdx.x] = acc[mt][nt][r];
}

// Sum over the S partial sums of accumulator tile k = mt * NT + nt (4 values per thread).
template <class C>
__device__ inline d4 sum_partial_tile(const double* __restrict__ part, int S, int k) {
    constexpr int PS = C::MT * C::NT * 4 * kThreads;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] += part[(size_t)s * PS + (k * 4 + r) * kThreads + threadIdx.x];
    return acc;
}

// Store accumulator tile k = mt * NT + nt of a block (MFMA layout of config C) to C~.
template <class C>
__device__ inline void store_acc_tile(const d4& acc, int k, double2* Cm, int N, int row0, int col0) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wrow = (wave / C::WAVES_N) * C::WM;
    const int wcc = (wave % C::WAVES_N) * (2 * C::WNC);
    const int q = lane >> 4, l16 = lane & 15, mt = k / C::NT, nt = k % C::NT;
    double* Cd = reinterpret_cast<double*>(Cm);
    const int cc = 2 * col0 + wcc + nt * 16 + l16;
    if (cc >= 2 * N) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = row0 + wrow + mt * 16 + q + 4 * r;
        if (row < N) Cd[(size_t)row * 2 * N + cc] = acc[r];
    }
}

// Work split of one launch: tiles [0, full) whole, one block each; tiles [full, full + tail)
// split into S ranges of K stages (blocks full + t*S + s), whose partial sums a fix-up kernel
// adds in a fixed order.
struct Split {
    int full, tail, S;
};

// `cap`: concurrent blocks of the kernel, `cus` the CUs they share, `pmax` the most split
// blocks whose partial sums the partial buffer holds.  Blocks are dealt out evenly over the
// CUs, so the busiest CU runs ceil(full / cus) whole tiles of nk stages and ceil(tail S / cus)
// ranges of ceil(nk / S) stages; the split minimising that is taken (ties: the larger S).  Two
// places for the whole tiles are tried: whole rounds of `cap` blocks (the tail is the last,
// partial round), and whole multiples of `cus` (the tail is what is left over one per CU: at
// N = 2048 the lower product's 528 tiles on 256 CUs holding 4 blocks each are one partial
// round, whose busiest CUs would run 3 tiles; as 512 whole tiles and 16 tiles in 16 K ranges
// every CU runs 2 tiles and one range).  At least 8 K stages (64 complex k) per range.
Split make_split(int ntiles, int nk, int cap, int pmax, int cus) {
    if (cus < 1) cus = 1;
    if (cap < 1) cap = 1;
    auto busiest = [&](long long n) { return (n + cus - 1) / cus; };
    Split best{ntiles, 0, 1};
    long long best_cost = busiest(ntiles) * nk;
    const int fulls[2] = {(ntiles / cap) * cap, (ntiles / cus) * cus};
    for (int f : fulls) {
        const int rem = ntiles - f;
        if (rem <= 0) continue;
        int smax = nk / 8 > 1 ? nk / 8 : 1;
        if (smax > (cap - f % cap) / rem) smax = (cap - f % cap) / rem;  // the tail fits beside
        if (smax > pmax / rem) smax = pmax / rem;
        for (int s = 2; s <= smax; ++s) {
            const long long L = busiest(f) * nk + busiest((long long)rem * s) * ((nk + s - 1) / s);
            if (L <= best_cost) {
                best_cost = L;
                best = {f, rem, s};
            }
        }
    }
    return best;
}

// ---------------------------------------------------------------- full product
__global__ __launch_bounds__(kThreads) void zgemm_f64_kernel(const double2* __restrict__ A,
                                                             const double2* __restrict__ B,
                                                             double2* __restrict__ Cm, int N,
                                                             int tiles_n, int full, int S,
                                                             double* __restrict__ part,
                                                             const int* __restrict__ skip) {
    using C = FullCfg;
    __shared__ double smem[2 * C::STAGE];
    if (skip && *skip) return;  // on-device stopping: the step has converged
    const int nk = (N + kBK - 1) / kBK;
    const int b = blockIdx.x;
    int tile, kb = 0, ke = nk;
    if (b < full) {
        tile = b;
    } else {
        const int e = b - full, s = e % S;
        tile = full + e / S;
        kb = (int)((long long)s * nk / S);
        ke = (int)((long long)(s + 1) * nk / S);
    }
    const int row0 = (tile / tiles_n) * C::BM;
    const int col0 = (tile % tiles_n) * C::BNC;
    d4 acc[C::MT][C::NT];
    mainloop<C>(A, N, row0, N, B, N, col0, N, N, kb, ke, smem, acc);
    if (b < full)
        store_full_tile(acc, Cm, N, row0, col0);
    else
        store_partial<C>(part + (size_t)(b - full) * (C::MT * C::NT * 4 * kThreads), acc);
}

// Small sizes (ceil(N/32)^2 tiles, at most one per CU): block b forms the 32 x 32 tile b of C.
__global__ __launch_bounds__(kThreads) void zgemm_small_kernel(const double2* __restrict__ A,
                                                               const double2* __restrict__ B,
                                                               double2* __restrict__ Cm, int N,
                                                               int tiles_n,
                                                               const int* __restrict__ skip) {
    __shared__ double red[kSmallRed];
    if (skip && *skip) return;  // on-device stopping: the step has converged
    const int tile = blockIdx.x;
    small_product(A, B, Cm, N, (tile / tiles_n) * kSmallTile, (tile % tiles_n) * kSmallTile, red);
}

// Fix-up of the split tiles: block (t, k) adds the S partial sums of accumulator tile k of
// split tile t, in part order (deterministic), and stores it.
__global__ __launch_bounds__(kThreads) void zgemm_f64_fixup(double2* __restrict__ Cm, int N,
                                                            int tiles_n, int full, int S,
                                                            const double* __restrict__ part,
                                                            const int* __restrict__ skip) {
    using C = FullCfg;
    if (skip && *skip) return;
    const int tile = full + blockIdx.x;
    const d4 acc = sum_partial_tile<C>(part + (size_t)blockIdx.x * S * (C::MT * C::NT * 4 * kThreads),
                                       S, blockIdx.y);
    store_acc_tile<C>(acc, blockIdx.y, Cm, N, (tile / tiles_n) * C::BM, (tile % tiles_n) * C::BNC);
}


// Lower-triangle product Q = A P into a buffer (64 x 64 complex tiles meeting the lower
// triangle; the fixed-point update reads them).  Tiles are taken from `order` (8 x 8
// super-tile order): the whole-tile blocks of XCD x (blocks b with b % 8 == x) run the
// contiguous chunk x * full/8 .. (x+1) * full/8 - 1 of it, so the tiles an XCD holds at once
// share A row panels and P column panels in its L2.
__global__ __launch_bounds__(kThreads) void zgemm_lower_kernel(
    const double2* __restrict__ Am, const double2* __restrict__ Pm, double2* __restrict__ Q,
    int N, int full, int S, double* __restrict__ part, const int* __restrict__ order,
    const int* __restrict__ skip) {
    using C = LowCfg;
    __shared__ double smem[2 * C::STAGE];
    if (skip && *skip) return;
    const int nk = (N + kBK - 1) / kBK;
    const int b = blockIdx.x;
    int tile, kb = 0, ke = nk;
    if (b < full) {
        tile = (full & 7) == 0 ? order[(b & 7) * (full >> 3) + (b >> 3)] : order[b];
    } else {
        const int e = b - full, s = e % S;
        tile = order[full + e / S];
        kb = (int)((long long)s * nk / S);
        ke = (int)((long long)(s + 1) * nk / S);
    }
    int I, J;
    lower_tile(tile, I, J);
    d4 acc[C::MT][C::NT];
    mainloop<C>(Am, N, I * kTile, N, Pm, N, J * kTile, N, N, kb, ke, smem, acc);
    if (b < full)
        store_tile<C>(acc, Q, N, I * kTile, J * kTile);
    else
        store_partial<C>(part + (size_t)(b - full) * (C::MT * C::NT * 4 * kThreads), acc);
}

__global__ __launch_bounds__(kThreads) void zgemm_lower_fixup(double2* __restrict__ Q, int N,
                                                              int full, int S,
                                                              const double* __restrict__ part,
                                                              const int* __restrict__ order,
                                                              const int* __restrict__ skip) {
    using C = LowCfg;
    if (skip && *skip) return;
    int I, J;
    lower_tile(order[full + blockIdx.x], I, J);
    const d4 acc = sum_partial_tile<C>(part + (size_t)blockIdx.x * S * (C::MT * C::NT * 4 * kThreads),
                                       S, blockIdx.y);
    store_acc_tile<C>(acc, blockIdx.y, Q, N, I * kTile, J * kTile);
}

// ---------------------------------------------------------------- residual reduction
constexpr int kRedThreads = 256;

// resid = max_r sum_X rowpart[X N + r] (NaN propagates; also to host_out if given, a mapped
// host word) in one launch: each block takes the
// row sums of 256 rows and stores their maximum; the last block to finish (a counter, reset
// by that block) takes the maximum over the blocks.  With ctl (on-device stopping) that block
// also counts the evaluation (ctl[1]) and sets the step's done flag ctl[0] when resid < tol or
// resid is not finite; with skip set at entry (the step had already converged) it does nothing.
__global__ __launch_bounds__(kRedThreads) void resid_kernel(const double* __restrict__ rowpart,
                                                            int T, int N, double* blockmax,
                                                            unsigned* counter, double* resid,
                                                            const int* __restrict__ skip, int* ctl,
                                                            double tol, double* host_out) {
    __shared__ double sm[kRedThreads];
    __shared__ bool last;
    if (skip && *skip) return;
    const int i = blockIdx.x * kRedThreads + threadIdx.x;
    const double v = i < N ? slot_row_sum<32>(rowpart, T, N, i) : 0.0;
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = sm[threadIdx.x + s], a = sm[threadIdx.x];
            sm[threadIdx.x] = (o != o || o > a) ? o : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __hip_atomic_store(blockmax + blockIdx.x, sm[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double m = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kRedThreads) {
        const double o = __hip_atomic_load(blockmax + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        m = (o != o || o > m) ? o : m;
    }
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = sm[threadIdx.x + s], a = sm[threadIdx.x];
            sm[threadIdx.x] = (o != o || o > a) ? o : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double r = sm[0];
        resid[0] = r;
        if (host_out) __hip_atomic_store(host_out, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        *counter = 0u;
        if (ctl) {
            ctl[1] += 1;
            if (r < tol || !isfinite(r)) ctl[0] = 1;
        }
    }
}

}  // namespace

void ze_lower_tile_order(int N, std::vector<int>& order) {
    const int T = (N + kTile - 1) / kTile;
    order.clear();
    for (int si = 0; si * 8 < T; ++si)
        for (int sj = 0; sj <= si; ++sj)
            for (int I = si * 8; I < si * 8 + 8 && I < T; ++I)
                for (int J = sj * 8; J < sj * 8 + 8 && J <= I; ++J) order.push_back(I * (I + 1) / 2 + J);
}

size_t ze_gemm_part_bytes(int cap_full, int cap_low) {
    const size_t a = (size_t)cap_full * FullCfg::MT * FullCfg::NT * 4 * kThreads;
    const size_t b = (size_t)cap_low * LowCfg::MT * LowCfg::NT * 4 * kThreads;
    return (a > b ? a : b) * sizeof(double);
}

hipError_t ze_gemm_capacity(int* cap_full, int* cap_low, int* cus_out) {
    int dev = 0, cus = 0, nf = 0, nl = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nf, zgemm_f64_kernel, kThreads, 0);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nl, zgemm_lower_kernel, kThreads, 0);
    if (e != hipSuccess) return e;
    *cap_full = (nf > 0 ? nf : 1) * cus;
    *cap_low = (nl > 0 ? nl : 1) * cus;
    *cus_out = cus;
    return hipSuccess;
}

namespace {

// The full product with `cap` concurrent blocks on `cus` CUs and a partial buffer `part` of
// `pmax` split blocks' partial sums.  Sizes whose 32 x 32 tiles fit one per CU take the small
// kernel (no split, no fix-up).
hipError_t launch_full(int N, int cap, int cus, double* part, int pmax, const double2* A,
                       const double2* B, double2* Cm, hipStream_t s, const int* skip = nullptr) {
    const int wn = (N + kSmallTile - 1) / kSmallTile;
    if ((long long)wn * wn <= cus) {
        hipLaunchKernelGGL(zgemm_small_kernel, dim3(wn * wn), dim3(kThreads), 0, s, A, B, Cm, N, wn, skip);
        return hipGetLastError();
    }
    const int tiles_n = (N + FullCfg::BNC - 1) / FullCfg::BNC;
    const int tiles = tiles_n * ((N + FullCfg::BM - 1) / FullCfg::BM);
    const Split sp = make_split(tiles, (N + kBK - 1) / kBK, cap, pmax, cus);
    hipLaunchKernelGGL(zgemm_f64_kernel, dim3(sp.full + sp.tail * sp.S), dim3(kThreads), 0, s, A, B,
                       Cm, N, tiles_n, sp.full, sp.S, part, skip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || sp.tail == 0) return e;
    hipLaunchKernelGGL(zgemm_f64_fixup, dim3(sp.tail, FullCfg::MT * FullCfg::NT), dim3(kThreads), 0, s,
                       Cm, N, tiles_n, sp.full, sp.S, part, skip);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_zgemm_f64(const ze_ctx* c, const double2* A, const double2* B, double2* Cm,
                            hipStream_t s, const int* skip) {
    // the context's buffer holds cap_full blocks' partial sums (ze_gemm_part_bytes)
    return launch_full(c->N, c->cap_full, c->cus, c->gemm_part, c->cap_full, A, B, Cm, s, skip);
}

// ---------------------------------------------------------------- allocation-free product
// ze_zgemm_noalloc keeps the split-K partial sums of the full product in this fixed device
// array instead of a context's buffer: each GPU holds its own copy until the process ends.
// In host code `scratch` is a host-side stand-in, not a device address; its address on a
// device is looked up once per device (hipGetSymbolAddress, with that device current) and
// only that address reaches a kernel.  Every call on one GPU shares the array: calls that
// overlap on one GPU race.  Nothing in it has to start at zero (each partial slot is written
// by its block before the fix-up reads it).
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {

constexpr int kNoAllocMaxDevices = 64;

struct NoAllocDevice {
    double* ptr = nullptr;  // device address of `scratch` on this device
    int cap_full = 0;       // concurrent blocks of the full product
    int cus = 0;            // compute units
};

std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[kNoAllocMaxDevices];

constexpr int kPartialDoubles = FullCfg::MT * FullCfg::NT * 4 * kThreads;  // one split block

}  // namespace

hipError_t launch_zgemm_f64_noalloc(int N, const double2* A, const double2* B, double2* Cm,
                                    hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    NoAllocDevice d;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (!g_noalloc[dev].ptr) {
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            int cap_low = 0;
            e = ze_gemm_capacity(&g_noalloc[dev].cap_full, &cap_low, &g_noalloc[dev].cus);
            if (e != hipSuccess) return e;
            g_noalloc[dev].ptr = static_cast<double*>(ptr);
        }
        d = g_noalloc[dev];
    }
    const int pmax = (int)(kNoAllocScratchBytes / sizeof(double) / kPartialDoubles);
    return launch_full(N, d.cap_full, d.cus, d.ptr, pmax, A, B, Cm, s);
}

hipError_t launch_zgemm_lower(const ze_ctx* c, const double2* A, const double2* P, double2* Q,
                              hipStream_t s, const int* skip) {
    const int N = c->N;
    const int T = (N + kTile - 1) / kTile;
    const Split sp = make_split(T * (T + 1) / 2, (N + kBK - 1) / kBK, c->cap_low, c->cap_low, c->cus);
    hipLaunchKernelGGL(zgemm_lower_kernel, dim3(sp.full + sp.tail * sp.S), dim3(kThreads), 0, s, A,
                       P, Q, N, sp.full, sp.S, c->gemm_part, c->low_order, skip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || sp.tail == 0) return e;
    hipLaunchKernelGGL(zgemm_lower_fixup, dim3(sp.tail, LowCfg::MT * LowCfg::NT), dim3(kThreads), 0, s,
                       Q, N, sp.full, sp.S, c->gemm_part, c->low_order, skip);
    return hipGetLastError();
}

hipError_t launch_resid_reduce(const double* rowpart, int T, double* blockmax, unsigned* counter,
                               double* resid, int N, hipStream_t s, const int* skip, int* ctl,
                               double tol, double* host_out) {
    const int G = (N + kRedThreads - 1) / kRedThreads;
    hipLaunchKernelGGL(resid_kernel, dim3(G), dim3(kRedThreads), 0, s, rowpart, T, N, blockmax,
                       counter, resid, skip, ctl, tol, host_out);
    return hipGetLastError();
}

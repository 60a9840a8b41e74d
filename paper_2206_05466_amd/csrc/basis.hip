// Quantised basis and vorticity assembly W = sum_lm i omega_lm T_lm (eq. (W0), Sec. 3.2).
//
// The basis elements with m >= 0 are the eigenvectors of the tridiagonal blocks Delta^m of
// eq. (delta_tria) for the eigenvalues l(l+1), l = m..N-1 (eq. (lap_prop)).  The paper
// computes them with a divide-and-conquer eigensolver; here every eigenvalue is known in
// closed form, so each eigenvector is one O(n) twisted-factorisation solve (Parlett &
// Dhillon, "Fernando's solution to Wilkinson's problem", 1997), one GPU thread per (m, l):
//
//   a_i = d_i - lambda;  D+_0 = a_0,  D+_i = a_i - e_{i-1}^2 / D+_{i-1}   (top-down pivots)
//                        D-_{n-1} = a_{n-1},  D-_i = a_i - e_i^2 / D-_{i+1}  (bottom-up pivots)
//   twist r: z_r = 1,  z_i = -(e_i / D+_i) z_{i+1} (i < r),  z_i = -(e_{i-1} / D-_i) z_{i-1} (i > r).
//
// Two details make this robust for these blocks:
// * The twist index must sit where the eigenvector is large.  With the exact eigenvalue all
//   gamma_k = D+_k + D-_k - a_k are rounding noise, so r is picked from the pivots of a
//   shift lambda + sigma (sigma = 1e-3, far above the noise, far below the gaps >= 2), where
//   gamma_k ~ sigma / v_k^2; the vector itself is formed with the exact lambda.
// * The blocks have exact zero pivots (lambda is then also an eigenvalue of a leading or
//   trailing sub-block).  A zero pivot is replaced by 1e-200, small enough to be exact in the
//   limit and large enough that e^2 / pivot stays finite, so the next z is the finite limit.
//
// Each vector is normalised to unit 2-norm.  Its sign: among the entries with index
// 0..floor((n-1)/2) whose magnitude is within a relative 1e-8 of the largest there, the one
// with the lowest index is made positive (these blocks have eigenvectors with exactly equal
// magnitudes at different indices, so the largest entry alone does not fix the sign).
//
// Memory: the vectors of a batch of diagonals are kept in scratch as V_m[i][j] (row i,
// column j = l - m), so the lanes of a wave (consecutive j) touch consecutive addresses at
// every step; a second array holds the pivots.  A second kernel then forms, for each row i,
// W[i+m][i] = i sum_j omega_{m+j, m} V_m[i][j] and W[i][i+m] = i (-1)^m sum_j omega_{m+j,-m} V_m[i][j].

#include "internal.h"

namespace {

constexpr double kTiny = 1e-200;
constexpr double kSigma = 1e-3;
constexpr double kSignTieRel = 1e-8;  // magnitudes this close to the largest count as ties

__device__ inline double nz(double x) { return x == 0.0 ? kTiny : x; }

// Sum of n'^2 for n' = 1..a.
__host__ __device__ inline size_t sumsq(size_t a) { return a * (a + 1) * (2 * a + 1) / 6; }

__device__ inline double diag_d(int N, int m, int i) {
    const double s = 0.5 * (N - 1);
    return 2.0 * (s * (2.0 * i + 1.0 + m) - (double)i * (double)(i + m));
}

// e_k^2 = (k+m+1)(N-1-k-m)(k+1)(N-1-k), an integer (exact in FP64 for N below ~16000).
__device__ inline double offdiag_sq(int N, int m, int k) {
    return ((double)(k + m + 1) * (double)(N - 1 - k - m)) * ((double)(k + 1) * (double)(N - 1 - k));
}

__global__ __launch_bounds__(64) void basis_vectors_kernel(int N, int m_begin, int nb,
                                                           double* __restrict__ V,
                                                           double* __restrict__ S) {
    const int m = m_begin + blockIdx.y;
    const int n = N - m;
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (blockIdx.x * 64 >= n) return;  // whole wave idle
    const bool act = j < n;
    const size_t off = sumsq((size_t)nb) - sumsq((size_t)n);
    double* v = V + off;
    double* sp = S + off;
    const double l = (double)(m + j);
    const double lam = l * (l + 1.0);
    const double lams = lam + kSigma;

    // Top-down pivots for lambda (-> v) and lambda + sigma (-> sp).
    double dp = 0.0, dps = 0.0;
    for (int i = 0; i < n; ++i) {
        if (act) {
            const double d = diag_d(N, m, i);
            if (i == 0) {
                dp = d - lam;
                dps = d - lams;
            } else {
                const double e2 = offdiag_sq(N, m, i - 1);
                dp = (d - lam) - e2 / nz(dp);
                dps = (d - lams) - e2 / nz(dps);
            }
            v[(size_t)i * n + j] = dp;
            sp[(size_t)i * n + j] = dps;
        }
    }
    // Bottom-up pivots; twist index from the shifted gammas; sp <- D- (exact lambda).
    double dm = 0.0, dms = 0.0, best = 0.0;
    int r = n - 1;
    for (int i = n - 1; i >= 0; --i) {
        if (act) {
            const double a = diag_d(N, m, i) - lam;
            const double as = diag_d(N, m, i) - lams;
            if (i == n - 1) {
                dm = a;
                dms = as;
            } else {
                const double e2 = offdiag_sq(N, m, i);
                dm = a - e2 / nz(dm);
                dms = as - e2 / nz(dms);
            }
            const size_t o = (size_t)i * n + j;
            const double g = fabs(sp[o] + dms - as);
            if (i == n - 1 || g <= best) {
                best = g;
                r = i;
            }
            sp[o] = dm;
        }
    }
    // Twisted solve with the exact lambda: downward from r (uses D+ in v), upward (D- in sp).
    const int half = (n - 1) / 2;  // the sign rule looks at indices 0..half
    double ss = 1.0;               // sum of squares, z_r = 1 included
    double amax = (r <= half) ? 1.0 : 0.0;
    double z = 1.0;
    for (int i = n - 1; i >= 0; --i) {
        if (act && i < r) {
            const size_t o = (size_t)i * n + j;
            const double e = -sqrt(offdiag_sq(N, m, i));
            z = -(e / nz(v[o])) * z;
            v[o] = z;
            ss += z * z;
            if (i <= half) amax = fmax(amax, fabs(z));
        }
    }
    if (act) v[(size_t)r * n + j] = 1.0;
    z = 1.0;
    for (int i = 0; i < n; ++i) {
        if (act && i > r) {
            const size_t o = (size_t)i * n + j;
            const double e = -sqrt(offdiag_sq(N, m, i - 1));
            z = -(e / nz(sp[o])) * z;
            v[o] = z;
            ss += z * z;
            if (i <= half) amax = fmax(amax, fabs(z));
        }
    }
    // Sign: the lowest index i <= half with |z_i| >= (1 - kSignTieRel) max |z_0..z_half|.
    const double thr = (1.0 - kSignTieRel) * amax;
    double sgn = 1.0;
    bool found = false;
    for (int i = 0; i <= half; ++i) {
        if (act && !found) {
            const double zi = v[(size_t)i * n + j];
            if (fabs(zi) >= thr) {
                sgn = zi < 0.0 ? -1.0 : 1.0;
                found = true;
            }
        }
    }
    const double scale = sgn / sqrt(ss);
    for (int i = 0; i < n; ++i)
        if (act) v[(size_t)i * n + j] *= scale;
}

__global__ __launch_bounds__(256) void basis_project_kernel(int N, int m_begin, int nb,
                                                            const double* __restrict__ V,
                                                            const double2* __restrict__ omega,
                                                            double2* __restrict__ W) {
    const int m = m_begin + blockIdx.y;
    const int n = N - m;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;  // whole wave
    const size_t off = sumsq((size_t)nb) - sumsq((size_t)n);
    const double* row = V + off + (size_t)i * n;
    double pr = 0.0, pi = 0.0, nr = 0.0, ni = 0.0;
    for (int j = lane; j < n; j += 64) {
        const double x = row[j];
        const size_t l = (size_t)(m + j);
        const double2 op = omega[l * l + l + m];
        pr += x * op.x;
        pi += x * op.y;
        if (m > 0) {
            const double2 om = omega[l * l + l - m];
            nr += x * om.x;
            ni += x * om.y;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        pr += __shfl_down(pr, o);
        pi += __shfl_down(pi, o);
        nr += __shfl_down(nr, o);
        ni += __shfl_down(ni, o);
    }
    if (lane == 0) {
        // i * (pr + i pi) = -pi + i pr
        W[(size_t)(i + m) * N + i] = make_double2(-pi, pr);
        if (m > 0) {
            const double sg = (m & 1) ? -1.0 : 1.0;
            W[(size_t)i * N + i + m] = make_double2(-sg * ni, sg * nr);
        }
    }
}

// Inverse of the assembly (post-processing, Sec. 3.2): one thread per (m, l = m + j) forms
// the projections onto T_lm and T_{l,-m},
//     omega_lm = -i sum_i v_i W[i+m][i],   omega_{l,-m} = -i (-1)^m sum_i v_i W[i][i+m],
// the lanes of a wave reading consecutive j of V_m (coalesced) and one diagonal entry of W
// (the same address: a broadcast).
__global__ __launch_bounds__(64) void basis_extract_kernel(int N, int m_begin, int nb,
                                                           const double* __restrict__ V,
                                                           const double2* __restrict__ W,
                                                           double2* __restrict__ omega) {
    const int m = m_begin + blockIdx.y;
    const int n = N - m;
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= n) return;
    const double* v = V + (sumsq((size_t)nb) - sumsq((size_t)n)) + j;
    double lr = 0.0, li = 0.0, ur = 0.0, ui = 0.0;
    for (int i = 0; i < n; ++i) {
        const double x = v[(size_t)i * n];
        const double2 lo = W[(size_t)(i + m) * N + i];
        lr += x * lo.x;
        li += x * lo.y;
        if (m > 0) {
            const double2 up = W[(size_t)i * N + i + m];
            ur += x * up.x;
            ui += x * up.y;
        }
    }
    const size_t l = (size_t)(m + j);
    omega[l * l + l + m] = make_double2(li, -lr);  // -i (lr + i li)
    if (m > 0) {
        const double sg = (m & 1) ? -1.0 : 1.0;
        omega[l * l + l - m] = make_double2(sg * ui, -sg * ur);
    }
}

// Kinetic energy per degree, E_l = sum_{m=-l..l} |omega_lm|^2 / (l (l + 1)) for l >= 1 (the
// stream function has coefficients -omega_lm / (l (l + 1)), eq. (lap_prop)); E_0 = 0.
__global__ __launch_bounds__(256) void energy_spectrum_kernel(int N, const double2* __restrict__ omega,
                                                             double* __restrict__ E) {
    const int l = blockIdx.x * 256 + threadIdx.x;
    if (l >= N) return;
    double s = 0.0;
    for (int k = 0; k <= 2 * l; ++k) {
        const double2 o = omega[(size_t)l * l + k];
        s += o.x * o.x + o.y * o.y;
    }
    E[l] = l > 0 ? s / ((double)l * (double)(l + 1)) : 0.0;
}

constexpr size_t kScratchBudget = (size_t)4 << 30;  // bytes for V and S of one batch

}  // namespace

size_t ze_basis_scratch_bytes(int N) {
    const size_t all = 2 * sizeof(double) * sumsq((size_t)N);
    const size_t first = 2 * sizeof(double) * (size_t)N * N;
    size_t b = all < kScratchBudget ? all : kScratchBudget;
    return b < first ? first : b;
}

hipError_t launch_basis_assemble(const double2* omega, double2* W, void* scratch, int N,
                                 hipStream_t s) {
    const size_t cap = ze_basis_scratch_bytes(N) / (2 * sizeof(double));  // doubles per array
    double* V = static_cast<double*>(scratch);
    double* S = V + cap;
    // Every entry of W lies on exactly one diagonal, so the projection writes all of W.
    hipError_t e = hipSuccess;
    int m = 0;
    while (m < N && e == hipSuccess) {
        const int nb = N - m;
        int me = m;
        size_t used = 0;
        while (me < N) {
            const size_t need = (size_t)(N - me) * (size_t)(N - me);
            if (me > m && used + need > cap) break;
            used += need;
            ++me;
        }
        const int count = me - m;
        hipLaunchKernelGGL(basis_vectors_kernel, dim3((nb + 63) / 64, count), dim3(64), 0, s, N, m,
                           nb, V, S);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(basis_project_kernel, dim3((nb + 3) / 4, count), dim3(256), 0, s, N, m,
                           nb, V, omega, W);
        e = hipGetLastError();
        m = me;
    }
    return e;
}

hipError_t launch_basis_extract(const double2* W, double2* omega, void* scratch, int N,
                                hipStream_t s) {
    const size_t cap = ze_basis_scratch_bytes(N) / (2 * sizeof(double));  // doubles per array
    double* V = static_cast<double*>(scratch);
    double* S = V + cap;
    // Every coefficient (l, +-m) belongs to exactly one diagonal m, so all of omega is written.
    hipError_t e = hipSuccess;
    int m = 0;
    while (m < N && e == hipSuccess) {
        const int nb = N - m;
        int me = m;
        size_t used = 0;
        while (me < N) {
            const size_t need = (size_t)(N - me) * (size_t)(N - me);
            if (me > m && used + need > cap) break;
            used += need;
            ++me;
        }
        const int count = me - m;
        hipLaunchKernelGGL(basis_vectors_kernel, dim3((nb + 63) / 64, count), dim3(64), 0, s, N, m,
                           nb, V, S);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(basis_extract_kernel, dim3((nb + 63) / 64, count), dim3(64), 0, s, N, m,
                           nb, V, W, omega);
        e = hipGetLastError();
        m = me;
    }
    return e;
}

hipError_t launch_energy_spectrum(const double2* omega, double* E, int N, hipStream_t s) {
    hipLaunchKernelGGL(energy_spectrum_kernel, dim3((N + 255) / 256), dim3(256), 0, s, N, omega, E);
    return hipGetLastError();
}

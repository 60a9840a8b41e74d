// C ABI of libzeuler: context set-up (Laplacian factors), stream solve, IsoMP step driver,
// Casimirs, products.  Host code; the arithmetic of every step runs in the HIP kernels.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "solve_wg.h"
#include "update_tile.h"

namespace {

thread_local std::string g_last_error;

bool is_finite(double x) { return std::isfinite(x); }

template <class T>
ze_status dalloc(T** p, size_t count) {
    if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T) + 256) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return ZE_ENOMEM;
    }
    return ZE_OK;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

}  // namespace

// Workspaces of the split-precision products, allocated on first use.
ze_status ze_ensure_rings(ze_ctx* c, int ns) {
    const size_t need = 4 * (size_t)ns, nn = (size_t)c->N * c->N;
    const size_t had = c->ring.size();
    if (had >= need) return ZE_OK;
    c->ring.resize(need, nullptr);
    for (size_t i = had; i < need; ++i) {
        const ze_status st = dalloc(&c->ring[i], nn);
        if (st != ZE_OK) {
            for (size_t k = had; k < i; ++k) dfree(c->ring[k]);
            c->ring.resize(had);
            return st;
        }
    }
    c->rhead.resize((size_t)ns, 0);
    return ZE_OK;
}

ze_status ze_ensure_crt(ze_ctx* c) {
    if (c->crt_g) return ZE_OK;
    ZE_TRY(ze_ensure_split(c));  // exponent vectors and column-maximum partials
    const size_t ldk = (size_t)ze_crt_ldk(c->N);
    const size_t bytes_a = (size_t)3 * kCrtMods * crt_rows_pad(c->N) * ldk;
    const size_t bytes_b = bytes_a;
    ze_status st = dalloc(&c->crt_a, bytes_a);
    if (st == ZE_OK) st = dalloc(&c->crt_b, bytes_b);
    // zero padding rows once; the residue kernels never write them
    if (st == ZE_OK &&
        (hipMemsetAsync(c->crt_a, 0, bytes_a, c->stream) != hipSuccess ||
         hipMemsetAsync(c->crt_b, 0, bytes_b, c->stream) != hipSuccess ||
         hipStreamSynchronize(c->stream) != hipSuccess))
        st = ze_record_hip(hipGetLastError(), "residue workspace clear");
    if (st == ZE_OK) st = dalloc(&c->crt_g, ze_crt_slab_ints(c->N));
    if (st != ZE_OK) {
        dfree(c->crt_a);
        dfree(c->crt_b);
        dfree(c->crt_g);
        c->crt_a = c->crt_b = nullptr;
        c->crt_g = nullptr;
    }
    return st;
}

ze_status ze_ensure_split(ze_ctx* c) {
    if (c->split_a) return ZE_OK;
    const size_t n = (size_t)c->N, ldk = (size_t)ze_split_ldk(c->N);
    const size_t bytes_a = (size_t)kSplitMax * split_rows_pad(c->N) * ldk;
    const size_t bytes_b = (size_t)kSplitMax * split_cols_pad(c->N) * ldk;
    ze_status st = dalloc(&c->split_a, bytes_a);
    if (st == ZE_OK) st = dalloc(&c->split_b, bytes_b);
    // zero padding rows (and everything else) once; the slicing kernels never write them
    if (st == ZE_OK &&
        (hipMemsetAsync(c->split_a, 0, bytes_a, c->stream) != hipSuccess ||
         hipMemsetAsync(c->split_b, 0, bytes_b, c->stream) != hipSuccess ||
         hipStreamSynchronize(c->stream) != hipSuccess))
        st = ze_record_hip(hipGetLastError(), "split workspace clear");
    if (st == ZE_OK) st = dalloc(&c->split_ea, n);
    if (st == ZE_OK) st = dalloc(&c->split_eb, n);
    if (st == ZE_OK) st = dalloc(&c->split_ec, n);
    if (st == ZE_OK) st = dalloc(&c->split_colmax, 64 * n);
    if (st == ZE_OK) {
        const hipError_t ce = ze_i8_capacity(&c->cap_i8, &c->cap_i8l);
        if (ce != hipSuccess) st = ze_record_hip(ce, "ze_i8_capacity");
    }
    if (st == ZE_OK) st = dalloc(&c->split_g, (size_t)kSplitMax * 2 * n * n);
    if (st != ZE_OK) {
        dfree(c->split_a);
        dfree(c->split_b);
        dfree(c->split_ea);
        dfree(c->split_eb);
        dfree(c->split_ec);
        dfree(c->split_colmax);
        dfree(c->split_g);
        c->split_a = c->split_b = nullptr;
        c->split_ea = c->split_eb = c->split_ec = nullptr;
        c->split_colmax = nullptr;
        c->split_g = nullptr;
    }
    return st;
}


ze_status ze_record_hip(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return ZE_EHIP;
}

// Input check of ze_set_validation: W must be skew-Hermitian and traceless to 1e-12 relative,
// max |W_rc + conj(W_cr)| <= 1e-12 max |W_rc| and |tr W| <= 1e-12 N max |W_rc| (non-finite
// entries fail).  Synchronises the context's stream.
static ze_status check_su(ze_ctx* c, const void* W) {
    const int N = c->N, G = ze_su_check_blocks(N);
    if (!c->val_part) ZE_TRY(dalloc(&c->val_part, 4 * (size_t)G + 4));
    double* out = c->val_part + 4 * (size_t)G;
    ZE_HIP(launch_su_check(static_cast<const double2*>(W), N, c->val_part, out, c->stream));
    double h[4] = {0, 0, 0, 0};
    ZE_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    ZE_HIP(hipStreamSynchronize(c->stream));
    const double asym = h[0], amax = h[1], tr = std::hypot(h[2], h[3]);
    if (asym <= 1e-12 * amax && tr <= 1e-12 * N * amax && std::isfinite(amax)) return ZE_OK;
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "W is not in su(N) to 1e-12: max|W + W^H| = %.3e, |tr W| = %.3e, max|W| = %.3e",
                  asym, tr, amax);
    g_last_error = msg;
    return ZE_EINVAL;
}

extern "C" {

const char* ze_strerror(ze_status s) {
    switch (s) {
        case ZE_OK: return "ok";
        case ZE_EINVAL: return "invalid argument";
        case ZE_ENOMEM: return "out of memory";
        case ZE_ENOTCONV: return "fixed-point iteration not converged within maxit";
        case ZE_ENONFINITE: return "non-finite fixed-point residual";
        case ZE_EHIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char* ze_last_error(void) { return g_last_error.c_str(); }

int ze_size(const ze_ctx* ctx) { return ctx ? ctx->N : 0; }

ze_status ze_destroy(ze_ctx* c) {
    if (!c) return ZE_OK;
    (void)hipStreamSynchronize(c->stream);
    dfree(c->fac_l);
    dfree(c->fac_dinv);
    dfree(c->Wn);
    dfree(c->Wh[0]);
    dfree(c->Wh[1]);
    dfree(c->Wd);
    for (double2* p : c->ring) dfree(p);  // ring[0] is the F allocation
    dfree(c->P);
    dfree(c->A);
    dfree(c->Q);
    dfree(c->rowpart);
    dfree(c->blockmax);
    dfree(c->gemm_part);
    dfree(c->low_order);
    dfree(c->split_a);
    dfree(c->split_b);
    dfree(c->split_ea);
    dfree(c->split_eb);
    dfree(c->split_ec);
    dfree(c->split_colmax);
    dfree(c->split_g);
    dfree(c->crt_a);
    dfree(c->crt_b);
    dfree(c->crt_g);
    dfree(c->resid);
    dfree(c->dctl);
    dfree(c->dctld);
    dfree(c->dstep_it);
    dfree(c->dstep_r);
    dfree(c->val_part);
    if (c->host_resid) (void)hipHostFree(c->host_resid);
    for (hipEvent_t e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
    return ZE_OK;
}

ze_status ze_create(int N, void* stream, ze_ctx** out) { return ze_create_ctx(N, stream, true, 0, out); }

}  // extern "C"

ze_status ze_create_ctx(int N, void* stream, bool split_k, int solve_bd_, ze_ctx** out) {
    if (!out) return ZE_EINVAL;
    *out = nullptr;
    if (N < 1 || N > kMaxN) return ZE_EINVAL;
    if (solve_bd_ != 0 && solve_bd_ != 1 && solve_bd_ != 2 && solve_bd_ != 4) return ZE_EINVAL;
    ze_ctx* c = new ze_ctx();
    c->N = N;
    c->solve_bd = solve_bd_ ? solve_bd_ : zk::solve_bd(N);
    c->split_slices = split_max_slices(N) < 5 ? split_max_slices(N) : 5;
    c->split_slices_low = c->split_slices > 2 ? c->split_slices - 1 : 2;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return ze_record_hip(hipGetLastError(), "hipGetDevice");
    }
    std::vector<double> fl, fd;
    ze_build_factors(N, c->solve_bd, fl, fd);
    const size_t nn = (size_t)N * N;
    c->ut = zk::update_tile_of(N);
    const int T = (N + c->ut - 1) / c->ut;
    {
        hipError_t ce = ze_gemm_capacity(&c->cap_full, &c->cap_low, &c->cus);
        if (ce != hipSuccess) {
            delete c;
            return ze_record_hip(ce, "ze_gemm_capacity");
        }
    }
    ze_status st = ZE_OK;
    if (st == ZE_OK && split_k)
        st = dalloc(&c->gemm_part, ze_gemm_part_bytes(c->cap_full, c->cap_low) / sizeof(double));
    if (st == ZE_OK) st = dalloc(&c->fac_l, fl.size());
    if (st == ZE_OK) st = dalloc(&c->fac_dinv, fd.size());
    if (st == ZE_OK) st = dalloc(&c->Wn, nn);
    if (st == ZE_OK) st = dalloc(&c->F, nn);
    c->ring.assign(1, c->F);
    c->rhead.assign(1, 0);
    if (st == ZE_OK) st = dalloc(&c->P, nn);
    if (st == ZE_OK) st = dalloc(&c->A, nn);
    if (st == ZE_OK) st = dalloc(&c->Q, nn);
    if (st == ZE_OK) st = dalloc(&c->rowpart, (size_t)T * N);
    if (st == ZE_OK) st = dalloc(&c->blockmax, (size_t)(N + 255) / 256 + 1);
    if (st == ZE_OK) st = dalloc(&c->resid, 1);
    if (st == ZE_OK) st = dalloc(&c->dctl, kCtlWords);
    if (st == ZE_OK) st = dalloc(&c->dctld, 2);
    if (st == ZE_OK && (hipMemset(c->dctl, 0, kCtlWords * sizeof(int)) != hipSuccess ||
                        hipMemset(c->dctld, 0, 2 * sizeof(double)) != hipSuccess))
        st = ze_record_hip(hipGetLastError(), "control words clear");
    // the residual kernel writes the infinity norm straight into this pinned, mapped host word
    if (st == ZE_OK &&
        (hipHostMalloc(reinterpret_cast<void**>(&c->host_resid), sizeof(double),
                       hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
         hipHostGetDevicePointer(reinterpret_cast<void**>(&c->host_resid_dev), c->host_resid, 0) !=
             hipSuccess)) {
        if (c->host_resid) (void)hipHostFree(c->host_resid);
        c->host_resid = nullptr;
        (void)hipGetLastError();
        st = ZE_ENOMEM;
    }
    if (st != ZE_OK) {
        ze_destroy(c);
        return st;
    }
    std::vector<int> order;
    ze_lower_tile_order(N, order);
    if (st == ZE_OK) st = dalloc(&c->low_order, order.size());
    if (st != ZE_OK) {
        ze_destroy(c);
        return st;
    }
    hipError_t e = hipMemcpy(c->fac_l, fl.data(), fl.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->low_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->fac_dinv, fd.data(), fd.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        ze_destroy(c);
        return ze_record_hip(e, "hipMemcpy(factors)");
    }
    *out = c;
    return ZE_OK;
}

extern "C" {

ze_status ze_stream_solve(ze_ctx* c, const void* W, void* P) {
    if (!c || !W || !P || W == P) return ZE_EINVAL;
    ZE_HIP(launch_stream_solve(c, static_cast<const double2*>(W), static_cast<double2*>(P), c->stream));
    return ZE_OK;
}

ze_status ze_zgemm(ze_ctx* c, const void* A, const void* B, void* C, int prec) {
    if (!c || !A || !B || !C || C == A || C == B) return ZE_EINVAL;
    if (prec != ZE_PREC_FP64 && prec != ZE_PREC_SPLIT && prec != ZE_PREC_CRT) return ZE_EINVAL;
    if (prec == ZE_PREC_CRT) {
        ZE_TRY(ze_ensure_crt(c));
        ZE_HIP(launch_zgemm_crt(c, static_cast<const double2*>(A), static_cast<const double2*>(B),
                                static_cast<double2*>(C), c->stream));
        return ZE_OK;
    }
    if (prec == ZE_PREC_SPLIT) {
        ZE_TRY(ze_ensure_split(c));
        ZE_HIP(launch_zgemm_split(c, static_cast<const double2*>(A), static_cast<const double2*>(B),
                                  static_cast<double2*>(C), 0, c->split_ea, c->split_eb, false,
                                  c->stream));
        return ZE_OK;
    }
    ZE_HIP(launch_zgemm_f64(c, static_cast<const double2*>(A), static_cast<const double2*>(B),
                            static_cast<double2*>(C), c->stream));
    return ZE_OK;
}

ze_status ze_zgemm_noalloc(int N, const void* A, const void* B, void* C, void* stream) {
    if (N < 1 || N > kMaxN) {
        g_last_error = "ze_zgemm_noalloc: N = " + std::to_string(N) + " outside 1.." +
                       std::to_string(kMaxN);
        return ZE_EINVAL;
    }
    if (!A || !B || !C || C == A || C == B) {
        g_last_error = "ze_zgemm_noalloc: null or aliased matrix pointer";
        return ZE_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, sdev = 0;
    ZE_HIP(hipGetDevice(&dev));
    if (s) {
        ZE_HIP(hipStreamGetDevice(s, &sdev));
        if (sdev != dev) {
            g_last_error = "ze_zgemm_noalloc: the stream belongs to device " + std::to_string(sdev) +
                           ", the current device is " + std::to_string(dev);
            return ZE_EINVAL;
        }
    }
    ZE_HIP(launch_zgemm_f64_noalloc(N, static_cast<const double2*>(A), static_cast<const double2*>(B),
                                    static_cast<double2*>(C), s));
    return ZE_OK;
}

namespace {

enum StartFrom { kFromWn = 0, kLinear = 1, kFromF = 2 };

// One midpoint step of size h from W_n in Win (read only) to W_{n+1} in Wout (another buffer,
// written by every evaluation, so it ends with that of the last one).  The fixed point starts
// from W_n (kFromWn), from W_n + rho (W_n - F) written over F (kLinear; F = the previous step's
// converged midpoint, still in c->F; rho = 1 gives 2 W_n - F), or from the iterate the caller
// has put in c->F (kFromF).
ze_status isomp_step_device(ze_ctx* c, const double2* Win, double2* Wout, double h, double tol,
                            int maxit, int prec, StartFrom start, double rho, bool last);

ze_status isomp_step_impl(ze_ctx* c, const double2* Win, double2* Wout, double h, double tol,
                          int maxit, int prec, StartFrom start, double rho, int* iters,
                          double* resid, bool last) {
    if (!c || !Win || !Wout || Win == Wout || !is_finite(h) || !(tol >= 0.0) || !is_finite(tol) ||
        maxit < 1)
        return ZE_EINVAL;
    if (prec != ZE_PREC_FP64 && prec != ZE_PREC_SPLIT && prec != ZE_PREC_MIXED &&
        prec != ZE_PREC_CRT)
        return ZE_EINVAL;
    if (c->stop_mode == 1) return isomp_step_device(c, Win, Wout, h, tol, maxit, prec, start, rho, last);
    const int N = c->N;
    double2* Wu = Wout;
    const bool split = prec == ZE_PREC_SPLIT, mixed = prec == ZE_PREC_MIXED;
    const bool crt = prec == ZE_PREC_CRT;
    if (split || mixed) ZE_TRY(ze_ensure_split(c));
    if (crt) ZE_TRY(ze_ensure_crt(c));
    hipStream_t s = c->stream;
    const double2* Wn = Win;
    const double2* Wt = Wn;
    if (start == kLinear) ZE_HIP(launch_extrapolate(Wn, c->F, N, rho, s));
    if (start != kFromWn) Wt = c->F;
    double r = 0.0;
    int k = 0;
    const bool prof = c->prof;
    for (k = 1; k <= maxit; ++k) {
        if (prof) ZE_HIP(hipEventRecord(c->ev[0], s));
        ZE_HIP(launch_stream_solve(c, Wt, c->P, s));
        if (prof) ZE_HIP(hipEventRecord(c->ev[1], s));
        if (split)
            ZE_HIP(launch_zgemm_split(c, c->P, Wt, c->A, 0, c->split_ea, c->split_eb, false, s));
        else if (crt)
            ZE_HIP(launch_zgemm_crt(c, c->P, Wt, c->A, s));
        else
            ZE_HIP(launch_zgemm_f64(c, c->P, Wt, c->A, s));
        if (prof) ZE_HIP(hipEventRecord(c->ev[2], s));
        if (split || crt) {
            // P is skew-Hermitian: its column exponents are the row exponents just taken
            ZE_HIP(launch_zgemm_split(c, c->A, c->P, nullptr, 1, c->split_ec, c->split_ea, true, s));
            ZE_HIP(launch_lower_update(c, nullptr, c->A, Wn, Wt, c->F, Wu, c->rowpart, h,
                                       c->split_ec, c->split_ea, s));
        } else if (mixed) {
            // A came from the FP64 product: P's column exponents are taken here
            ZE_HIP(launch_zgemm_split(c, c->A, c->P, nullptr, 1, c->split_ec, c->split_ea, false, s));
            ZE_HIP(launch_lower_update(c, nullptr, c->A, Wn, Wt, c->F, Wu, c->rowpart, h,
                                       c->split_ec, c->split_ea, s));
        } else {
            ZE_HIP(launch_zgemm_lower(c, c->A, c->P, c->Q, s));
            ZE_HIP(launch_lower_update(c, c->Q, c->A, Wn, Wt, c->F, Wu, c->rowpart, h, nullptr,
                                       nullptr, s));
        }
        if (prof) ZE_HIP(hipEventRecord(c->ev[3], s));
        ZE_HIP(launch_resid_reduce(c->rowpart, (N + c->ut - 1) / c->ut, c->blockmax,
                                   reinterpret_cast<unsigned*>(c->dctl + kCtlCounter), c->resid, N, s,
                                   nullptr, nullptr, 0.0, c->host_resid_dev));
        if (k == 1 && c->save_first) ZE_HIP(launch_copy(Wu, c->save_first, N, s));
        if (prof) ZE_HIP(hipEventRecord(c->ev[4], s));
        ZE_HIP(hipStreamSynchronize(s));
        if (prof) {
            for (int p = 0; p < 4; ++p) {
                float ms = 0.f;
                ZE_HIP(hipEventElapsedTime(&ms, c->ev[p], c->ev[p + 1]));
                c->prof_ms[p] += ms;
                c->prof_n[p] += 1;
            }
        }
        r = *c->host_resid;
        if (!std::isfinite(r)) break;
        if (r < tol || k == maxit) break;
        Wt = c->F;
    }
    if (k > maxit) k = maxit;
    if (iters) *iters = k;
    if (resid) *resid = r;
    if (!std::isfinite(r)) return ZE_ENONFINITE;
    if (!(r < tol)) return ZE_ENOTCONV;
    return ZE_OK;
}

// The same substep with the stopping rule on the device: maxit evaluations are enqueued, each
// kernel of an evaluation reads the done flag (dctl[0]) first and returns at once when it is
// set, and the residual reduction sets it once the change of W~ is below tol (or not finite).
// Wout receives W_{n+1} from every evaluation that runs, so it ends with that of the last one,
// as in the host loop.  Nothing synchronises; the counts and residuals go to the control words
// and the per-step records (last: the substep closes the step).
ze_status isomp_step_device(ze_ctx* c, const double2* Win, double2* Wout, double h, double tol,
                            int maxit, int prec, StartFrom start, double rho, bool last) {
    const int N = c->N;
    double2* Wu = Wout;
    const double2* Wn = Win;
    hipStream_t s = c->stream;
    const bool split = prec == ZE_PREC_SPLIT, mixed = prec == ZE_PREC_MIXED;
    const bool crt = prec == ZE_PREC_CRT;
    if (split || mixed) ZE_TRY(ze_ensure_split(c));
    if (crt) ZE_TRY(ze_ensure_crt(c));
    const int* skip = c->dctl;
    // the split and modular launchers take the flag from the context while this substep is
    // enqueued; it is cleared on every way out
    struct SkipScope {
        ze_ctx* c;
        ~SkipScope() { c->skip = nullptr; }
    } scope{c};
    c->skip = skip;
    unsigned* counter = reinterpret_cast<unsigned*>(c->dctl + kCtlCounter);
    if (start == kLinear) ZE_HIP(launch_extrapolate(Wn, c->F, N, rho, s));
    const double2* Wt = start == kFromWn ? Wn : c->F;
    for (int k = 1; k <= maxit; ++k) {
        ZE_HIP(launch_stream_solve(c, Wt, c->P, s, skip));
        if (split)
            ZE_HIP(launch_zgemm_split(c, c->P, Wt, c->A, 0, c->split_ea, c->split_eb, false, s));
        else if (crt)
            ZE_HIP(launch_zgemm_crt(c, c->P, Wt, c->A, s));
        else
            ZE_HIP(launch_zgemm_f64(c, c->P, Wt, c->A, s, skip));
        if (split || crt || mixed) {
            // P is skew-Hermitian: after the split or modular product its column exponents are
            // the row exponents just taken; after the FP64 product (mixed) they are taken here
            ZE_HIP(launch_zgemm_split(c, c->A, c->P, nullptr, 1, c->split_ec, c->split_ea, !mixed, s));
            ZE_HIP(launch_lower_update(c, nullptr, c->A, Wn, Wt, c->F, Wu, c->rowpart, h,
                                       c->split_ec, c->split_ea, s, skip));
        } else {
            ZE_HIP(launch_zgemm_lower(c, c->A, c->P, c->Q, s, skip));
            ZE_HIP(launch_lower_update(c, c->Q, c->A, Wn, Wt, c->F, Wu, c->rowpart, h, nullptr,
                                       nullptr, s, skip));
        }
        ZE_HIP(launch_resid_reduce(c->rowpart, (N + c->ut - 1) / c->ut, c->blockmax, counter,
                                   c->resid, N, s, skip, c->dctl, tol));
        // the first evaluation always runs: its W_{n+1} is kept unguarded
        if (k == 1 && c->save_first) ZE_HIP(launch_copy(Wu, c->save_first, N, s));
        Wt = c->F;
    }
    ZE_HIP(launch_ctl_substep_end(c->dctl, c->dctld, c->resid, tol, last, c->dstep_it, c->dstep_r, s));
    return ZE_OK;
}

// The state of a run: W_n in cur; a substep writes W_{n+1} into other, and the two swap.  The
// caller's W and the context's Wn take turns (guess mode 3 at order 2: Wh[0], Wh[1] too, for
// the first steps), and the run ends with a copy into the caller's W when the last substep
// left it elsewhere.
struct RunState {
    double2* user;
    double2* cur;
    double2* other;
    int nsteps;  // steps of the run (the first step keeps its first output only if there are more)
};

ze_status finish_run(ze_ctx* c, const RunState& rs) {
    if (rs.cur != rs.user) ZE_HIP(launch_copy(rs.cur, rs.user, c->N, c->stream));
    return ZE_OK;
}

// Start of substep j of the step with index n in the run, guess mode 2 (and 3): the next slot of
// substep j's ring receives the polynomial of degree min(nm - 1, 3) through that substep's
// nm = min(n, 4) previous midpoints when nm >= 2 (with four, the slot is the oldest one's,
// overwritten in place), else W + rho (W - F_prev) from the previous substep's midpoint F_prev
// (in F) when there is one; the slot then becomes F and receives this substep's midpoint.
// hist (guess mode 3 at order 2): steps 2 and 3 also use the states W_0 .. W_n, and with the
// difference form step 1 the slope at W_0 (from the first step's first evaluation).
ze_status ring_start(ze_ctx* c, const RunState& rs, size_t j, int n, double rho, bool hist,
                     StartFrom* start) {
    const int N = c->N;
    const void* W = rs.cur;
    double2** rg = c->ring.data() + 4 * j;
    const int head = c->rhead[j], next = (head + 1) & 3;
    double2* out = rg[next];
    const int nm = n < 4 ? n : 4;
    if (hist && (n == 2 || n == 3)) {
        // guess mode 3: the midpoint polynomial of degree n - 1 through F_{n-1} .. F_0 plus the
        // n-th backward difference of the states W_n .. W_0 (each midpoint is the average of
        // its step's states plus an O(h^2) offset; the next state and the offset are each
        // extrapolated one step ahead), newest first in both sums
        static const double cf2[2] = {2.0, -1.0}, cf3[3] = {3.0, -3.0, 1.0};
        static const double cw2[3] = {1.0, -2.0, 1.0}, cw3[4] = {1.0, -3.0, 3.0, -1.0};
        const double2* states[4] = {rs.user, c->Wn, c->Wh[0], c->Wh[1]};  // W_0 .. W_3
        const double2* src[kLinCombMax];
        double coef[kLinCombMax];
        int m = 0;
        for (int i = 0; i < n; ++i) {
            src[m] = rg[(head - i + 4) & 3];
            coef[m++] = n == 2 ? cf2[i] : cf3[i];
        }
        for (int i = 0; i <= n; ++i) {
            src[m] = states[n - i];
            coef[m++] = n == 2 ? cw2[i] : cw3[i];
        }
        ZE_HIP(launch_lincomb(src, coef, m, out, N, c->stream));
        *start = kFromF;
    } else if (hist && n == 1 && c->update_form == 1) {
        // guess mode 3, difference form: F_0 + 2 (W_1 - W_0) - h D_0, with h D_0 = Wd - W_0
        // (Wd: the first step's first output, W_0 + h (P_0 W_0 - W_0 P_0)), formed as
        // F_0 + 2 W_1 - W_0 - Wd
        const double2* src[4] = {rg[head], rs.cur, rs.user, c->Wd};
        const double coef[4] = {1.0, 2.0, -1.0, -1.0};
        ZE_HIP(launch_lincomb(src, coef, 4, out, N, c->stream));
        *start = kFromF;
    } else if (nm >= 2) {
        const int d = nm - 1 < 3 ? nm - 1 : 3;
        const double2* Fs[4];
        for (int i = 0; i <= d; ++i) Fs[i] = rg[(head - i + 4) & 3];
        ZE_HIP(launch_extrapolate_poly(Fs, d, out, N, c->stream));
        *start = kFromF;
    } else if (n > 0 || j > 0) {
        ZE_HIP(hipMemcpyAsync(out, c->F, (size_t)N * N * sizeof(double2), hipMemcpyDeviceToDevice,
                              c->stream));
        ZE_HIP(launch_extrapolate(static_cast<const double2*>(W), out, N, rho, c->stream));
        *start = kFromF;
    } else {
        *start = kFromWn;
    }
    c->rhead[j] = next;
    c->F = out;
    return ZE_OK;
}

// One step of the context's order: a midpoint substep of size c_j h for every fraction c_j.
// n is the step's index in the run.  Guess mode 1: every substep after the first of the call
// (n > 0 or j > 0) starts from W + rho (W - F_prev), rho = c_j / c_{j-1} (cyclically, so 1
// across a step boundary), written over F_prev in place.  Guess mode 2: see ring_start.  A
// substep that reaches maxit above tol still completes the step (the fixed-iteration mode)
// and the step then reports ZE_ENOTCONV; any other error ends it.  iters: evaluations over all
// substeps; resid: the largest substep residual.
ze_status composed_step(ze_ctx* c, RunState& rs, double h, double tol, int maxit, int prec, int n,
                        int* iters, double* resid) {
    if (!c || !rs.cur) return ZE_EINVAL;
    const std::vector<double>& w = c->comp_w;
    const size_t ns = w.size();
    if (c->guess_mode >= 2) ZE_TRY(ze_ensure_rings(c, (int)ns));
    // guess mode 3 at order 2: steps 0 .. 3 write W_1 .. W_4 into Wn, Wh[0], Wh[1] and the
    // caller's W, so W_0 .. W_3 are all in memory when step 3 starts; later steps alternate
    const bool hist = c->guess_mode == 3 && ns == 1;
    int total = 0;
    double rmax = 0.0;
    ze_status out = ZE_OK;
    for (size_t j = 0; j < ns; ++j) {
        const double rho = w[j] / w[j == 0 ? ns - 1 : j - 1];
        StartFrom start = kFromWn;
        if (c->guess_mode == 1 && (j > 0 || n > 0)) start = kLinear;
        if (c->guess_mode >= 2) ZE_TRY(ring_start(c, rs, j, n, rho, hist, &start));
        if (hist && n <= 3) {
            double2* const outs[4] = {c->Wn, c->Wh[0], c->Wh[1], rs.user};
            rs.other = outs[n];
        }
        // the second step's start needs h D_0 = (first output of step 0) - W_0
        c->save_first = (hist && n == 0 && rs.nsteps >= 2 && c->update_form == 1) ? c->Wd : nullptr;
        int k = 0;
        double r = 0.0;
        const ze_status st = isomp_step_impl(c, rs.cur, rs.other, w[j] * h, tol, maxit, prec, start,
                                             rho, &k, &r, j + 1 == ns);
        c->save_first = nullptr;
        if (st == ZE_OK || st == ZE_ENOTCONV || st == ZE_ENONFINITE) std::swap(rs.cur, rs.other);
        total += k;
        if (!(r <= rmax)) rmax = r;  // keeps a NaN
        if (st == ZE_ENOTCONV) {
            out = ZE_ENOTCONV;
            continue;
        }
        if (st != ZE_OK) {
            out = st;
            break;
        }
    }
    if (iters) *iters = total;
    if (resid) *resid = rmax;
    return out;
}

}  // namespace

// The evaluation cap of step n of a run (ze_set_steady_cap).
static int step_cap(const ze_ctx* c, int maxit, int n) {
    return (c->cap2 > 0 && n >= c->cap2_after) ? std::min(maxit, c->cap2) : maxit;
}

// The step index a run on W starts from: that of the run it continues (ze_set_continuation),
// else 0.  Guess mode 3 at order 2 needs the states of the first four steps for steps 1 .. 3,
// which a run does not keep, so it continues only from step 4 on.
static int run_first_step(const ze_ctx* c, const void* W, double h, int prec) {
    if (!c->cont || c->cont_n < 0 || W != c->cont_w || h != c->cont_h || prec != c->cont_prec ||
        c->guess_mode != c->cont_guess || c->update_form != c->cont_form ||
        c->comp_w.size() != c->cont_ns)
        return 0;
    if (c->guess_mode == 3 && c->comp_w.size() == 1 && c->cont_n < 4) return 0;
    return c->cont_n;
}

// After a run from step n0 of nsteps steps: a successful one (ZE_OK, or ZE_ENOTCONV, whose
// steps all completed) can be continued; any other outcome ends the continuation.
static void run_finished(ze_ctx* c, const void* W, double h, int prec, int n0, int nsteps,
                         ze_status st) {
    if (c->cont && (st == ZE_OK || st == ZE_ENOTCONV)) {
        c->cont_n = n0 + nsteps;
        c->cont_w = W;
        c->cont_h = h;
        c->cont_prec = prec;
        c->cont_guess = c->guess_mode;
        c->cont_form = c->update_form;
        c->cont_ns = c->comp_w.size();
    } else {
        c->cont_n = -1;
    }
}

// On-device stopping: the records of the last run (nsteps <= its length) and its status.
static ze_status read_run_records(ze_ctx* c, int nsteps, int* iters, double* resid) {
    if (nsteps < 0 || nsteps > c->last_run_steps) return ZE_EINVAL;
    // the last m = min(nsteps, kDevSteps) steps of the run: step n sits at n % kDevSteps, so
    // they are at most two contiguous pieces of the records
    const int total = c->last_run_steps, m = nsteps < kDevSteps ? nsteps : kDevSteps;
    int ctl[kCtlWords];
    std::vector<int> it((size_t)m);
    std::vector<double> rr((size_t)m);
    ZE_HIP(hipMemcpyAsync(ctl, c->dctl, sizeof(ctl), hipMemcpyDeviceToHost, c->stream));
    for (int done = 0; done < m;) {
        const int pos = (total - m + done) % kDevSteps;
        const int len = std::min(m - done, kDevSteps - pos);
        ZE_HIP(hipMemcpyAsync(it.data() + done, c->dstep_it + pos, (size_t)len * sizeof(int),
                              hipMemcpyDeviceToHost, c->stream));
        ZE_HIP(hipMemcpyAsync(rr.data() + done, c->dstep_r + pos, (size_t)len * sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
        done += len;
    }
    ZE_HIP(hipStreamSynchronize(c->stream));
    // steps older than the last kDevSteps are reported as -1
    for (int i = 0; i < nsteps; ++i) {
        const int j = i - (nsteps - m);
        if (iters) iters[i] = j >= 0 ? it[(size_t)j] : -1;
        if (resid) resid[i] = j >= 0 ? rr[(size_t)j] : -1.0;
    }
    if (ctl[5] > 0) return ZE_ENONFINITE;
    if (ctl[4] > 0) return ZE_ENOTCONV;
    return ZE_OK;
}

// A run with on-device stopping: every step enqueued, one synchronisation at the end only if
// per-step results are asked for.
static ze_status run_device(ze_ctx* c, void* W, double h, double tol, int maxit, int nsteps,
                            int prec, int* iters, double* resid) {
    if (prec != ZE_PREC_FP64 && prec != ZE_PREC_SPLIT && prec != ZE_PREC_MIXED &&
        prec != ZE_PREC_CRT)
        return ZE_EINVAL;
    if (!is_finite(h) || !(tol >= 0.0) || !is_finite(tol) || maxit < 1) return ZE_EINVAL;
    ZE_HIP(launch_ctl_run_begin(c->dctl, c->dctld, c->stream));
    const int n0 = run_first_step(c, W, h, prec);
    c->cont_n = -1;
    RunState rs{static_cast<double2*>(W), static_cast<double2*>(W), c->Wn, n0 + nsteps};
    for (int n = 0; n < nsteps; ++n) {
        const ze_status st = composed_step(c, rs, h, tol, step_cap(c, maxit, n0 + n), prec, n0 + n,
                                           nullptr, nullptr);
        if (st != ZE_OK) {
            finish_run(c, rs);
            return st;
        }
    }
    ZE_TRY(finish_run(c, rs));
    run_finished(c, W, h, prec, n0, nsteps, ZE_OK);
    c->last_run_steps = nsteps;
    if (!iters && !resid) return ZE_OK;
    return read_run_records(c, nsteps, iters, resid);
}

ze_status ze_isomp_step(ze_ctx* c, void* W, double h, double tol, int maxit, int prec,
                        int* iters, double* resid) {
    g_last_error.clear();
    if (!c || !W) return ZE_EINVAL;
    if (c->validate) ZE_TRY(check_su(c, W));
    c->cont_n = -1;  // a single step uses the workspaces a continued run would need
    if (c->stop_mode == 1) {
        const int keep = c->cont;
        c->cont = 0;
        const ze_status st = run_device(c, W, h, tol, maxit, 1, prec, iters, resid);
        c->cont = keep;
        return st;
    }
    RunState rs{static_cast<double2*>(W), static_cast<double2*>(W), c->Wn, 1};
    const ze_status st = composed_step(c, rs, h, tol, maxit, prec, 0, iters, resid);
    const ze_status fin = finish_run(c, rs);
    return st != ZE_OK ? st : fin;
}

ze_status ze_set_stopping(ze_ctx* c, int mode) {
    if (!c || mode < 0 || mode > 1) return ZE_EINVAL;
    if (mode == 1 && !c->dstep_it) {
        ZE_TRY(dalloc(&c->dstep_it, (size_t)kDevSteps));
        const ze_status st = dalloc(&c->dstep_r, (size_t)kDevSteps);
        if (st != ZE_OK) {
            dfree(c->dstep_it);
            c->dstep_it = nullptr;
            return st;
        }
    }
    c->stop_mode = mode;
    return ZE_OK;
}

ze_status ze_set_steady_cap(ze_ctx* c, int cap, int from_step) {
    if (!c || cap < 0 || from_step < 0) return ZE_EINVAL;
    c->cap2 = cap;
    c->cap2_after = from_step;
    return ZE_OK;
}

ze_status ze_run_stats(ze_ctx* c, int nsteps, int* iters, double* resid) {
    if (!c || c->stop_mode != 1) return ZE_EINVAL;
    return read_run_records(c, nsteps, iters, resid);
}

ze_status ze_set_validation(ze_ctx* c, int on) {
    if (!c || on < 0 || on > 1) return ZE_EINVAL;
    c->validate = on == 1;
    return ZE_OK;
}

ze_status ze_isomp_run(ze_ctx* c, void* W, double h, double tol, int maxit, int nsteps, int prec,
                       int* iters, double* resid) {
    g_last_error.clear();
    if (!c || !W || nsteps < 0) return ZE_EINVAL;
    if (c->validate && nsteps > 0) ZE_TRY(check_su(c, W));
    if (c->stop_mode == 1) return run_device(c, W, h, tol, maxit, nsteps, prec, iters, resid);
    const int n0 = run_first_step(c, W, h, prec);
    c->cont_n = -1;
    RunState rs{static_cast<double2*>(W), static_cast<double2*>(W), c->Wn, n0 + nsteps};
    ze_status out = ZE_OK;
    for (int n = 0; n < nsteps; ++n) {
        int k = 0;
        double r = 0.0;
        ze_status st = composed_step(c, rs, h, tol, step_cap(c, maxit, n0 + n), prec, n0 + n, &k, &r);
        if (iters) iters[n] = k;
        if (resid) resid[n] = r;
        if (st != ZE_OK) {
            finish_run(c, rs);
            return st;
        }
    }
    out = finish_run(c, rs);
    run_finished(c, W, h, prec, n0, nsteps, out);
    return out;
}

ze_status ze_set_continuation(ze_ctx* c, int on) {
    if (!c || on < 0 || on > 1) return ZE_EINVAL;
    c->cont = on;
    c->cont_n = -1;
    return ZE_OK;
}

ze_status ze_casimirs(ze_ctx* c, const void* W, int kmax, double* out) {
    if (!c || !W || !out || kmax < 1 || kmax > 64) return ZE_EINVAL;
    const int N = c->N;
    const size_t nn = (size_t)N * N;
    const int hp = (kmax + 1) / 2;  // powers W^1..W^hp
    std::vector<double2*> pw(hp + 1, nullptr);
    pw[1] = const_cast<double2*>(static_cast<const double2*>(W));
    double2* partial = nullptr;
    double2* dres = nullptr;
    ze_status st = ZE_OK;
    for (int a = 2; a <= hp && st == ZE_OK; ++a) st = dalloc(&pw[a], nn);
    if (st == ZE_OK) st = dalloc(&partial, (size_t)ze_trace_partials(N) + (size_t)N);
    if (st == ZE_OK) st = dalloc(&dres, (size_t)kmax);
    hipError_t e = hipSuccess;
    for (int a = 2; a <= hp && st == ZE_OK && e == hipSuccess; ++a)
        e = launch_zgemm_f64(c, pw[a - 1], pw[1], pw[a], c->stream);
    for (int k = 1; k <= kmax && st == ZE_OK && e == hipSuccess; ++k) {
        if (k == 1) {
            e = launch_trace(pw[1], partial, dres, N, c->stream);
        } else {
            const int a = (k + 1) / 2, b = k / 2;
            e = launch_trace_product(pw[a], pw[b], partial, dres + (k - 1), N, c->stream);
        }
    }
    std::vector<double2> host(kmax);
    if (st == ZE_OK && e == hipSuccess)
        e = hipMemcpy(host.data(), dres, kmax * sizeof(double2), hipMemcpyDeviceToHost);
    for (int a = 2; a <= hp; ++a) dfree(pw[a]);
    dfree(partial);
    dfree(dres);
    if (st != ZE_OK) return st;
    if (e != hipSuccess) return ze_record_hip(e, "ze_casimirs");
    for (int k = 0; k < kmax; ++k) {
        out[2 * k] = host[k].x;
        out[2 * k + 1] = host[k].y;
    }
    return ZE_OK;
}

ze_status ze_basis_assemble(ze_ctx* c, const void* omega, void* W) {
    if (!c || !omega || !W || omega == W) return ZE_EINVAL;
    void* scratch = nullptr;
    if (hipMalloc(&scratch, ze_basis_scratch_bytes(c->N)) != hipSuccess) {
        (void)hipGetLastError();
        return ZE_ENOMEM;
    }
    hipError_t e = launch_basis_assemble(static_cast<const double2*>(omega), static_cast<double2*>(W),
                                         scratch, c->N, c->stream);
    hipError_t e2 = hipStreamSynchronize(c->stream);
    (void)hipFree(scratch);
    if (e != hipSuccess) return ze_record_hip(e, "launch_basis_assemble");
    if (e2 != hipSuccess) return ze_record_hip(e2, "hipStreamSynchronize(basis)");
    return ZE_OK;
}

ze_status ze_basis_extract(ze_ctx* c, const void* W, void* omega) {
    if (!c || !omega || !W || omega == W) return ZE_EINVAL;
    void* scratch = nullptr;
    if (hipMalloc(&scratch, ze_basis_scratch_bytes(c->N)) != hipSuccess) {
        (void)hipGetLastError();
        return ZE_ENOMEM;
    }
    hipError_t e = launch_basis_extract(static_cast<const double2*>(W), static_cast<double2*>(omega),
                                        scratch, c->N, c->stream);
    hipError_t e2 = hipStreamSynchronize(c->stream);
    (void)hipFree(scratch);
    if (e != hipSuccess) return ze_record_hip(e, "launch_basis_extract");
    if (e2 != hipSuccess) return ze_record_hip(e2, "hipStreamSynchronize(basis)");
    return ZE_OK;
}

ze_status ze_energy_spectrum(ze_ctx* c, const void* omega, void* E) {
    if (!c || !omega || !E || omega == E) return ZE_EINVAL;
    ZE_HIP(launch_energy_spectrum(static_cast<const double2*>(omega), static_cast<double*>(E), c->N,
                                  c->stream));
    return ZE_OK;
}

ze_status ze_set_initial_guess(ze_ctx* c, int mode) {
    if (!c || mode < 0 || mode > 3) return ZE_EINVAL;
    c->cont_n = -1;  // the next run starts at step 0
    if (mode >= 2) ZE_TRY(ze_ensure_rings(c, (int)c->comp_w.size()));
    if (mode == 3) {
        for (double2*& b : c->Wh)
            if (!b) ZE_TRY(dalloc(&b, (size_t)c->N * c->N));
        if (!c->Wd) ZE_TRY(dalloc(&c->Wd, (size_t)c->N * c->N));
    }
    c->guess_mode = mode;
    return ZE_OK;
}

ze_status ze_set_order(ze_ctx* c, int order) {
    if (!c || (order != 2 && order != 4 && order != 6)) return ZE_EINVAL;
    c->cont_n = -1;  // the next run starts at step 0
    // Triple jump (Yoshida 1990): from a symmetric method of even order p, the substeps
    // g1, g2, g1 with g1 = 1 / (2 - 2^(1/(p+1))) and g2 = 1 - 2 g1 give order p + 2.
    std::vector<double> w{1.0};
    for (int p = 2; p < order; p += 2) {
        const double g1 = 1.0 / (2.0 - std::pow(2.0, 1.0 / (p + 1)));
        const double g2 = 1.0 - 2.0 * g1;
        std::vector<double> next;
        for (double g : {g1, g2, g1})
            for (double x : w) next.push_back(g * x);
        w.swap(next);
    }
    if (c->guess_mode >= 2) ZE_TRY(ze_ensure_rings(c, (int)w.size()));
    c->comp_w = w;
    c->order = order;
    return ZE_OK;
}

ze_status ze_set_split_slices(ze_ctx* c, int slices) {
    if (!c || slices < 2 || slices > split_max_slices(c->N)) return ZE_EINVAL;
    c->cont_n = -1;  // the next run starts at step 0
    c->split_slices = slices;
    c->split_slices_low = slices > 2 ? slices - 1 : 2;
    return ZE_OK;
}

ze_status ze_set_update_form(ze_ctx* c, int form) {
    if (!c || form < 0 || form > 1) return ZE_EINVAL;
    c->cont_n = -1;  // the next run starts at step 0
    c->update_form = form;
    return ZE_OK;
}

ze_status ze_set_split_slices_lower(ze_ctx* c, int slices) {
    if (!c || slices < 2 || slices > c->split_slices) return ZE_EINVAL;
    c->cont_n = -1;  // the next run starts at step 0
    c->split_slices_low = slices;
    return ZE_OK;
}

ze_status ze_profile(ze_ctx* c, int on) {
    if (!c) return ZE_EINVAL;
    if (on) {
        for (hipEvent_t& e : c->ev)
            if (!e) ZE_HIP(hipEventCreate(&e));
    }
    c->prof = on != 0;
    return ZE_OK;
}

ze_status ze_profile_read(ze_ctx* c, double* ms, long long* launches, int reset) {
    if (!c) return ZE_EINVAL;
    for (int p = 0; p < 4; ++p) {
        if (ms) ms[p] = c->prof_ms[p];
        if (launches) launches[p] = c->prof_n[p];
        if (reset) {
            c->prof_ms[p] = 0.0;
            c->prof_n[p] = 0;
        }
    }
    return ZE_OK;
}

}  // extern "C"

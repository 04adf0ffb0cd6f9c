// Thermophysical and transport properties over a whole field (paper
// Section 3.1, the Thermo class: Newton's method on the temperature
// polynomials; Section 3.2: these kernels are compute-bound, keep their
// coefficients in constant memory, and are split into segments to bound
// register use; Section 2: the transport model is Cantera's mixture-averaged
// one).  One thread per cell, cells in index order (SoA, coalesced).
//
// The coefficients are uniform across a wave, so every table read is a
// scalar load through the scalar cache (the counterpart of CUDA's constant
// memory); a cell's mole fractions and per-species reciprocals live in
// registers, sized by a compile-time bound KM >= K.  The loops over the
// second species index are unrolled over KM (guards against K are uniform
// branches); the loops over the first index run at run time, except for
// small KM where everything unrolls.  Costs per cell with K species:
//   viscosity (Wilke)       K^2 pair terms of 5 FP64 operations
//   conductivity (Mathur)   K terms
//   diffusion               K (K - 1) / 2 pair polynomials and reciprocals
// Storage substitution (Section 3.2): the pair factors of Wilke's rule that
// depend only on molar masses, (W_j/W_k)^(1/4) and 1/sqrt(8 (1 + W_k/W_j)),
// are tabulated once per mechanism, and sqrt(mu_k/mu_j) is taken as
// s_k / s_j with s_k = T^(1/4) |P_k(ln T)| (the fitted square root itself),
// so no pow() and one square root pair per cell remain.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_common.h"

using chem_host::check_hip;
using chem_host::fail;
using chem_host::is_device_ptr;

namespace chem {
namespace {

constexpr int kThermoBlock = 256;
constexpr int kTrMaxK = 64;   // species the property kernels hold in registers
constexpr int kPoly = 5;      // coefficients of every ln T fit

// Mixture-averaged transport tables of a mechanism (device, contiguous).
struct TrView {
    int32_t K;
    const double *P;     // K x 5: viscosity fit, mu_k = (T^(1/4) P_k(ln T))^2
    const double *Q;     // K x 5: conductivity fit, lam_k = T^(1/2) Q_k(ln T)
    const double *c1;    // K x K: (W_j / W_k)^(1/4) at [k K + j]
    const double *c2;    // K x K: 1 / sqrt(8 (1 + W_k / W_j))
    const double *B;     // K x K x 5: diffusion fits, D_jk = T^(3/2) B_jk(ln T) / p (symmetric)
    const double *invW;  // K
};

__device__ __forceinline__ double rcp_t(double x)
{
    // hardware estimate and two Newton steps: within an ulp or two of 1/x
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

__device__ __forceinline__ double poly5(const double *c, double x)
{
    return fma(fma(fma(fma(c[4], x, c[3]), x, c[2]), x, c[1]), x, c[0]);
}

// Call f(k) for k = 0 .. K-1: unrolled over KM when UO, else a run-time loop.
template <int KM, bool UO, class F>
__device__ __forceinline__ void for_species(int K, F &&f)
{
    if constexpr (UO) {
#pragma unroll
        for (int k = 0; k < KM; k++)
            if (k < K) f(k);
    } else {
        for (int k = 0; k < K; k++) f(k);
    }
}

// MODE bit 1: viscosity and conductivity; bit 2: diffusion coefficients.
template <int KM, bool UO, int MODE>
__global__ void __launch_bounds__(kThermoBlock) transport_kernel(TrView v, const double *__restrict__ T,
                                                                 const double *__restrict__ p,
                                                                 const double *__restrict__ Y, int64_t ldY,
                                                                 int64_t n, double *__restrict__ mu,
                                                                 double *__restrict__ lam,
                                                                 double *__restrict__ D, int64_t ldD)
{
    const int64_t i = (int64_t)blockIdx.x * kThermoBlock + threadIdx.x;
    if (i >= n) return;
    const int K = v.K;
    const double Tc = T[i];
    const double lnT = log(Tc);
    const double sT = sqrt(Tc);

    // composition: y_k = max(Y_k, 0) / sum, X_k = (y_k / W_k) / sum_j (y_j / W_j)
    double X[KM];
    double ysum = 0.0;
#pragma unroll
    for (int k = 0; k < KM; k++) {
        X[k] = 0.0;
        if (k < K) {
            X[k] = fmax(Y[(int64_t)k * ldY + i], 0.0);
            ysum += X[k];
        }
    }
    const double inv_y = rcp_t(ysum);
    double csum = 0.0;
#pragma unroll
    for (int k = 0; k < KM; k++)
        if (k < K) {
            X[k] = X[k] * inv_y * v.invW[k];
            csum += X[k];
        }
    const double inv_c = rcp_t(csum);
#pragma unroll
    for (int k = 0; k < KM; k++)
        if (k < K) X[k] *= inv_c;

    if constexpr (MODE & 1) {
        const double qT = sqrt(sT);
        double r[KM];   // 1 / s_k
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int k = 0; k < KM; k++) {
            r[k] = 0.0;
            if (k < K) {
                r[k] = rcp_t(qT * fabs(poly5(v.P + kPoly * k, lnT)));
                const double lk = sT * poly5(v.Q + kPoly * k, lnT);
                a1 = fma(X[k], lk, a1);
                a2 = fma(X[k], rcp_t(lk), a2);
            }
        }
        lam[i] = 0.5 * (a1 + rcp_t(a2));
        double m = 0.0;
        for_species<KM, UO>(K, [&](int k) {
            // X_k and s_k again from the inputs (a run-time k cannot index registers)
            const double xk = fmax(Y[(int64_t)k * ldY + i], 0.0) * inv_y * v.invW[k] * inv_c;
            const double sk = qT * fabs(poly5(v.P + kPoly * k, lnT));
            const double *c1 = v.c1 + (int64_t)k * K;
            const double *c2 = v.c2 + (int64_t)k * K;
            double den = 0.0;
#pragma unroll
            for (int j = 0; j < KM; j++)
                if (j < K) {
                    const double t = fma(sk * c1[j], r[j], 1.0);
                    den = fma(X[j], t * t * c2[j], den);
                }
            m = fma(xk * sk * sk, rcp_t(den), m);
        });
        mu[i] = m;
    }

    if constexpr (MODE & 2) {
        // S_k = sum_{j != k} X_j / B_jk(ln T); pairs j < k once each
        double S[KM];
#pragma unroll
        for (int k = 0; k < KM; k++) S[k] = 0.0;
        const double t32 = Tc * sT;
        const double pc = p[i];
        const double t32_p = t32 * rcp_t(pc);
        for_species<KM, UO>(K, [&](int k) {
            const double xk = fmax(Y[(int64_t)k * ldY + i], 0.0) * inv_y * v.invW[k] * inv_c;
            const double *B = v.B + (int64_t)k * K * kPoly;
            double own = 0.0, earlier = 0.0;
#pragma unroll
            for (int j = 0; j < KM; j++)
                if (j < K) {
                    if (j == k) {
                        earlier = S[j];   // the terms of the pairs (j' < k, k)
                    } else if (j > k) {
                        const double ib = rcp_t(poly5(B + kPoly * j, lnT));
                        S[j] = fma(xk, ib, S[j]);
                        own = fma(X[j], ib, own);
                    }
                }
            const double s = earlier + own;
            const double yk = fmax(Y[(int64_t)k * ldY + i], 0.0) * inv_y;
            D[(int64_t)k * ldD + i] = s > 0.0 ? (1.0 - yk) * t32_p * rcp_t(s) : t32_p * poly5(B + kPoly * k, lnT);
        });
    }
}

// NASA-7 cp/R and H/(R T) of species k at T (range of the lane's T); the
// coefficients are uniform scalar loads, selected per lane.
__device__ __forceinline__ void nasa_cp_hrt(const double *species, int k, double T, double invT, double &cp,
                                            double &hrt)
{
    const double *s = species + k * kSpeciesLen;
    const bool low = T < s[0];
    const double *lo = s + 1, *hi = s + 1 + kRangeLen;
    const double a0 = low ? lo[0] : hi[0], a1 = low ? lo[1] : hi[1], a2 = low ? lo[2] : hi[2];
    const double a3 = low ? lo[3] : hi[3], a4 = low ? lo[4] : hi[4], a5 = low ? lo[5] : hi[5];
    const double b1 = low ? lo[7] : hi[7], b2 = low ? lo[8] : hi[8], b3 = low ? lo[9] : hi[9];
    const double b4 = low ? lo[10] : hi[10];
    cp = fma(fma(fma(fma(a4, T, a3), T, a2), T, a1), T, a0);
    hrt = fma(fma(fma(fma(b4, T, b3), T, b2), T, b1), T, a0) + a5 * invT;
}

// Mixture h (J/kg) and cp (J/(kg K)) at T from yr_k = Y_k R / W_k.
template <int KM>
__device__ __forceinline__ void mix_h_cp(const double *species, int K, const double (&yr)[KM], double T,
                                         double &h, double &cp)
{
    const double invT = rcp_t(T);
    double hs = 0.0, cs = 0.0;
#pragma unroll
    for (int k = 0; k < KM; k++)
        if (k < K) {
            double c, hr;
            nasa_cp_hrt(species, k, T, invT, c, hr);
            hs = fma(yr[k], hr, hs);
            cs = fma(yr[k], c, cs);
        }
    h = hs * T;
    cp = cs;
}

// Mixture h and cp of every cell at its temperature.
template <int KM>
__global__ void __launch_bounds__(kThermoBlock) h_cp_kernel(const double *__restrict__ species,
                                                            const double *__restrict__ invW, int K,
                                                            const double *__restrict__ T,
                                                            const double *__restrict__ Y, int64_t ldY, int64_t n,
                                                            double *__restrict__ h, double *__restrict__ cp)
{
    const int64_t i = (int64_t)blockIdx.x * kThermoBlock + threadIdx.x;
    if (i >= n) return;
    double yr[KM];
#pragma unroll
    for (int k = 0; k < KM; k++) yr[k] = k < K ? Y[(int64_t)k * ldY + i] * (kRu * invW[k]) : 0.0;
    double hm, cm;
    mix_h_cp<KM>(species, K, yr, T[i], hm, cm);
    if (h) h[i] = hm;
    if (cp) cp[i] = cm;
}

// Temperature from mixture enthalpy: Newton from the guess in T, each step
// T <- clamp(T - (h(T) - h) / cp(T), 200, 3500) K, done when the step is
// below tol; after max_iter steps without that, T = NaN and iters = max_iter + 1.
template <int KM>
__global__ void __launch_bounds__(kThermoBlock) t_from_h_kernel(const double *__restrict__ species,
                                                                const double *__restrict__ invW, int K,
                                                                const double *__restrict__ h,
                                                                const double *__restrict__ Y, int64_t ldY,
                                                                int64_t n, double *__restrict__ T,
                                                                double *__restrict__ cp,
                                                                int32_t *__restrict__ iters, int max_iter,
                                                                double tol)
{
    const int64_t i = (int64_t)blockIdx.x * kThermoBlock + threadIdx.x;
    if (i >= n) return;
    double yr[KM];
#pragma unroll
    for (int k = 0; k < KM; k++) yr[k] = k < K ? Y[(int64_t)k * ldY + i] * (kRu * invW[k]) : 0.0;
    const double h0 = h[i];
    double Tc = T[i];
    int it = 1;
    bool done = false;
    for (; it <= max_iter; it++) {
        double hm, cm;
        mix_h_cp<KM>(species, K, yr, Tc, hm, cm);
        const double dT = -(hm - h0) * rcp_t(cm);
        Tc = fmin(fmax(Tc + dT, 200.0), 3500.0);
        if (fabs(dT) < tol) {
            done = true;
            break;
        }
    }
    if (!done) Tc = __builtin_nan("");
    T[i] = Tc;
    if (cp) {
        double hm, cm;
        mix_h_cp<KM>(species, K, yr, Tc, hm, cm);
        cp[i] = done ? cm : __builtin_nan("");
    }
    if (iters) iters[i] = done ? it : max_iter + 1;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThermoBlock - 1) / kThermoBlock); }

// Dispatch on the smallest compile-time bound that holds K.
#define CHEM_TR_BOUNDS(X) X(12, true) X(16, true) X(24, false) X(36, false) X(48, false) X(64, false)

template <int MODE>
hipError_t launch_transport(const TrView &v, const double *T, const double *p, const double *Y, int64_t ldY,
                            int64_t n, double *mu, double *lam, double *D, int64_t ldD, hipStream_t st)
{
#define CHEM_TR_CASE(KM, UO)                                                                                 \
    if (v.K <= KM) {                                                                                          \
        hipLaunchKernelGGL((transport_kernel<KM, UO, MODE>), dim3(blocks_for(n)), dim3(kThermoBlock), 0, st, \
                           v, T, p, Y, ldY, n, mu, lam, D, ldD);                                             \
        return hipGetLastError();                                                                             \
    }
    CHEM_TR_BOUNDS(CHEM_TR_CASE)
#undef CHEM_TR_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_h_cp(const DevMechView &m, const double *T, const double *Y, int64_t ldY, int64_t n, double *h,
                       double *cp, hipStream_t st)
{
#define CHEM_TH_CASE(KM, UO)                                                                                 \
    if (m.K <= KM) {                                                                                          \
        hipLaunchKernelGGL((h_cp_kernel<KM>), dim3(blocks_for(n)), dim3(kThermoBlock), 0, st, m.species,     \
                           m.invW, m.K, T, Y, ldY, n, h, cp);                                                 \
        return hipGetLastError();                                                                             \
    }
    CHEM_TR_BOUNDS(CHEM_TH_CASE)
#undef CHEM_TH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_t_from_h(const DevMechView &m, const double *h, const double *Y, int64_t ldY, int64_t n,
                           double *T, double *cp, int32_t *iters, int max_iter, double tol, hipStream_t st)
{
#define CHEM_TN_CASE(KM, UO)                                                                                 \
    if (m.K <= KM) {                                                                                          \
        hipLaunchKernelGGL((t_from_h_kernel<KM>), dim3(blocks_for(n)), dim3(kThermoBlock), 0, st, m.species, \
                           m.invW, m.K, h, Y, ldY, n, T, cp, iters, max_iter, tol);                           \
        return hipGetLastError();                                                                             \
    }
    CHEM_TR_BOUNDS(CHEM_TN_CASE)
#undef CHEM_TN_CASE
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace chem

namespace {

int check_field(chem_mech m, int64_t n, int64_t ldY)
{
    if (!m) return fail(CHEM_EINVAL, "mechanism handle is NULL");
    if (n < 0) return fail(CHEM_EINVAL, "ncells must be >= 0");
    if (n > 0 && ldY < n) return fail(CHEM_EINVAL, "ldY must be >= ncells");
    if (m->host.K > chem::kTrMaxK)
        return fail(CHEM_EUNSUP, "the property kernels hold at most " + std::to_string(chem::kTrMaxK) + " species");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != m->device)
        return fail(CHEM_EINVAL, "the current HIP device is not the mechanism's device");
    return CHEM_OK;
}

bool dev_or_null(const void *p) { return p == nullptr || is_device_ptr(p); }

}  // namespace

extern "C" {

int chem_set_transport(chem_mech m, const double *visc, const double *cond, const double *diff)
{
    if (!m) return fail(CHEM_EINVAL, "mechanism handle is NULL");
    if (!visc || !cond || !diff) return fail(CHEM_EINVAL, "visc, cond and diff must be host arrays");
    const int K = m->host.K;
    if (K > chem::kTrMaxK)
        return fail(CHEM_EUNSUP, "the property kernels hold at most " + std::to_string(chem::kTrMaxK) + " species");
    const size_t KK = (size_t)K * K;
    std::vector<double> t(10 * (size_t)K + 2 * KK + 5 * KK + K);
    double *P = t.data(), *Q = P + 5 * K, *c1 = Q + 5 * K, *c2 = c1 + KK, *B = c2 + KK, *iw = B + 5 * KK;
    for (int k = 0; k < K; k++)
        for (int c = 0; c < 5; c++) {
            P[5 * k + c] = visc[5 * k + c];
            Q[5 * k + c] = cond[5 * k + c];
            if (!std::isfinite(P[5 * k + c]) || !std::isfinite(Q[5 * k + c]))
                return fail(CHEM_EINVAL, "transport fits must be finite");
        }
    for (int k = 0; k < K; k++)
        for (int j = 0; j < K; j++) {
            const double Wk = m->W[k], Wj = m->W[j];
            c1[(size_t)k * K + j] = std::pow(Wj / Wk, 0.25);
            c2[(size_t)k * K + j] = 1.0 / std::sqrt(8.0 * (1.0 + Wk / Wj));
            for (int c = 0; c < 5; c++) {
                const double a = diff[((size_t)k * K + j) * 5 + c];
                if (!std::isfinite(a)) return fail(CHEM_EINVAL, "transport fits must be finite");
                if (a != diff[((size_t)j * K + k) * 5 + c])
                    return fail(CHEM_EINVAL, "the binary diffusion fits must be symmetric in the two species");
                B[((size_t)k * K + j) * 5 + c] = a;
            }
        }
    for (int k = 0; k < K; k++) iw[k] = 1.0 / m->W[k];
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(CHEM_EHIP, "hipGetDevice failed");
    int rc = check_hip(hipSetDevice(m->device), "hipSetDevice");
    void *blk = nullptr;
    if (rc == CHEM_OK && hipMalloc(&blk, t.size() * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(CHEM_ENOMEM, "transport table allocation failed");
    }
    if (rc == CHEM_OK)
        rc = check_hip(hipMemcpy(blk, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice),
                       "transport table copy");
    if (rc == CHEM_OK) {
        if (m->transport_block) {
            hipDeviceSynchronize();   // earlier calls may still read the old table
            hipFree(m->transport_block);
        }
        m->transport_block = blk;
    } else if (blk) {
        hipFree(blk);
    }
    hipSetDevice(prev);
    return rc;
}

int chem_mixture_h_cp(chem_mech m, const double *T, const double *Y, int64_t ldY, int64_t n, double *h,
                      double *cp, void *stream)
{
    int rc = check_field(m, n, ldY);
    if (rc != CHEM_OK || n == 0) return rc;
    if (!is_device_ptr(T) || !is_device_ptr(Y) || !dev_or_null(h) || !dev_or_null(cp))
        return fail(CHEM_EINVAL, "T, Y, h and cp must be device pointers (h and cp may be NULL)");
    return check_hip(chem::launch_h_cp(m->view, T, Y, ldY, n, h, cp, (hipStream_t)stream), "h/cp launch");
}

int chem_T_from_h(chem_mech m, const double *h, const double *Y, int64_t ldY, int64_t n, double *T, double *cp,
                  int32_t *iters, int32_t max_iter, double tol, void *stream)
{
    int rc = check_field(m, n, ldY);
    if (rc != CHEM_OK) return rc;
    if (max_iter < 1 || max_iter > 1000) return fail(CHEM_EINVAL, "max_iter must be in 1 .. 1000");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(CHEM_EINVAL, "tol must be positive and finite");
    if (n == 0) return CHEM_OK;
    if (!is_device_ptr(h) || !is_device_ptr(Y) || !is_device_ptr(T) || !dev_or_null(cp) || !dev_or_null(iters))
        return fail(CHEM_EINVAL, "h, Y, T, cp and iters must be device pointers (cp and iters may be NULL)");
    return check_hip(chem::launch_t_from_h(m->view, h, Y, ldY, n, T, cp, iters, max_iter, tol, (hipStream_t)stream),
                     "T-from-h launch");
}

int chem_transport_field(chem_mech m, const double *T, const double *p, const double *Y, int64_t ldY, int64_t n,
                         double *mu, double *lam, double *D, int64_t ldD, void *stream)
{
    int rc = check_field(m, n, ldY);
    if (rc != CHEM_OK) return rc;
    if (!m->transport_block) return fail(CHEM_EINVAL, "no transport data: call chem_set_transport first");
    if ((mu == nullptr) != (lam == nullptr)) return fail(CHEM_EINVAL, "mu and lam are given together or not at all");
    if (!mu && !D) return fail(CHEM_EINVAL, "nothing to compute: mu/lam and D are all NULL");
    if (n == 0) return CHEM_OK;
    if (D && ldD < n) return fail(CHEM_EINVAL, "ldD must be >= ncells");
    if (!is_device_ptr(T) || !is_device_ptr(Y) || (D && !is_device_ptr(p)) || !dev_or_null(mu) ||
        !dev_or_null(lam) || !dev_or_null(D))
        return fail(CHEM_EINVAL, "T, p, Y, mu, lam and D must be device pointers");
    const int K = m->host.K;
    const size_t KK = (size_t)K * K;
    const double *t = (const double *)m->transport_block;
    chem::TrView v{K, t, t + 5 * K, t + 10 * K, t + 10 * K + KK, t + 10 * K + 2 * KK, t + 10 * K + 7 * KK};
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (mu && D)
        e = chem::launch_transport<3>(v, T, p, Y, ldY, n, mu, lam, D, ldD, st);
    else if (mu)
        e = chem::launch_transport<1>(v, T, p, Y, ldY, n, mu, lam, D, ldD, st);
    else
        e = chem::launch_transport<2>(v, T, p, Y, ldY, n, mu, lam, D, ldD, st);
    return check_hip(e, "transport launch");
}

}  // extern "C"

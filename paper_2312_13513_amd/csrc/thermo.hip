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
//   viscosity (Wilke)       K^2 pair terms of 3 fused multiply-adds
//   conductivity (Mathur)   K terms
//   diffusion               K (K - 1) / 2 pair polynomials and reciprocals
// Storage substitution (Section 3.2): the pair factors of Wilke's rule that
// depend only on molar masses are tabulated once per mechanism, and
// sqrt(mu_k/mu_j) is taken as s_k / s_j with s_k = T^(1/4) |P_k(ln T)| (the
// fitted square root itself), so no pow() and one square root pair per cell
// remain.
#include <algorithm>
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
// Wilke's factor times X_j, with t = s_k c1_kj / s_j and
// c1_kj = (W_j/W_k)^(1/4), c2_kj = 1/sqrt(8 (1 + W_k/W_j)), expands to
//   X_j c2 (1 + t)^2 = A_kj X_j + s_k (Bw_kj X_j/s_j + s_k C_kj X_j/s_j^2)
// with A = c2, Bw = 2 c1 c2, C = c1^2 c2: three fused multiply-adds per
// pair on per-cell vectors X, X/s, X/s^2 (all terms positive: no
// cancellation).
struct TrView {
    int32_t K;
    int32_t ld;          // row stride of every table: the kernel's bound KM (rows K .. KM-1 are padding)
    const double *P;     // ld x 5: viscosity fit, mu_k = (T^(1/4) P_k(ln T))^2 (padding: P = 1)
    const double *Q;     // ld x 5: conductivity fit, lam_k = T^(1/2) Q_k(ln T) (padding: Q = 1)
    const double *A;     // ld x ld at [k ld + j]: c2_kj (padding 0)
    const double *Bw;    // ld x ld: 2 c1_kj c2_kj
    const double *C;     // ld x ld: c1_kj^2 c2_kj
    const double *c1;    // ld x ld: c1_kj (the factored form of the larger kernels)
    const double *B;     // ld x ld x 5: diffusion fits, D_jk = T^(3/2) B_jk(ln T) / p (symmetric; padding B = 1)
    const double *invW;  // ld (padding 1)
};

// Reciprocals: the hardware estimate (relative error about 2^-24) refined
// by Newton steps, e -> e^2.  Two steps give the correctly rounded 1/x (all
// of 2^20 seeded x in [1e-12, 1e12] on gfx950); one step leaves about 10
// ulp (2.2e-15), used for the per-species and per-pair factors of the
// transport sums, where nothing cancels.
__device__ __forceinline__ double rcp_t(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

__device__ __forceinline__ double rcp_1(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(fma(-x, r, 1.0), r, r);
}

// Powers of ln T shared by every fit of a cell.
struct LnPow {
    double x, x2, x3, x4;
};

__device__ __forceinline__ LnPow ln_powers(double x)
{
    const double x2 = x * x;
    return {x, x2, x2 * x, x2 * x2};
}

// c0 + c1 x + c2 x^2 + c3 x^3 + c4 x^4 with uniform (scalar) coefficients:
// every step multiplies a scalar by a per-cell power into a vector
// accumulator, one instruction each.  (Horner's rule would add a scalar to
// a product and costs a register move per step on this target, which takes
// one scalar operand per instruction.)
__device__ __forceinline__ double poly5(const double *c, const LnPow &p)
{
    double q = c[1] * p.x;
    q = fma(c[2], p.x2, q);
    q = fma(c[3], p.x3, q);
    q = fma(c[4], p.x4, q);
    return q + c[0];
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

// A cell's K mass fractions into registers, rows beyond K zero.  The loads
// are unconditional (rows past K - 1 read row K - 1 again), so all of them
// are in flight together; guarded loads would each wait for the last.
template <int KM>
__device__ __forceinline__ void load_rows(const double *__restrict__ Y, int64_t ldY, int64_t i, int K,
                                          double (&y)[KM])
{
#pragma unroll
    for (int k = 0; k < KM; k++) y[k] = Y[(int64_t)(k < K ? k : K - 1) * ldY + i];
#pragma unroll
    for (int k = 0; k < KM; k++)
        if (k >= K) y[k] = 0.0;
}

// yr_k = Y_k / W_k: the mixture sums below are in units of R (mass-specific
// h / R and cp / R); R enters once per cell, not once per species.
template <int KM>
__device__ __forceinline__ void load_yr(const double *__restrict__ Y, int64_t ldY, int64_t i, int K,
                                        const double *__restrict__ invW, double (&yr)[KM])
{
    load_rows<KM>(Y, ldY, i, K, yr);
#pragma unroll
    for (int k = 0; k < KM; k++)
        if (k < K) yr[k] *= invW[k];
}

// MODE bit 1: viscosity and conductivity; bit 2: diffusion coefficients.
// With UO every species loop unrolls and a cell's values stay in
// registers; otherwise the outer loops run at run time and take X_k, y_k and
// s_k again from the inputs (a run-time index cannot address registers).
// UO is chosen per phase (see launch_transport).
template <int KM, bool UO, int MODE, bool EX = false>
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
    const LnPow lnT = ln_powers(log(Tc));
    const double sT = sqrt(Tc);

    // composition: y_k = max(Y_k, 0) / sum, X_k = (y_k / W_k) / sum_j (y_j / W_j);
    // X_j = 0 for the padding rows j >= K, so the padded tables need no
    // guards in the loops over j
    double X[KM], yv[UO ? KM : 1];
    load_rows<KM>(Y, ldY, i, K, X);
    double ysum = 0.0;
#pragma unroll
    for (int k = 0; k < KM; k++) {
        X[k] = fmax(X[k], 0.0);
        ysum += X[k];
    }
    const double inv_y = rcp_t(ysum);
    double csum = 0.0;
#pragma unroll
    for (int k = 0; k < KM; k++) {
        if constexpr (UO) yv[k] = X[k] * inv_y;
        X[k] = X[k] * inv_y * v.invW[k];
        csum += X[k];
    }
    const double inv_c = rcp_t(csum);
#pragma unroll
    for (int k = 0; k < KM; k++) X[k] *= inv_c;
    auto x_of = [&](int k) -> double {
        if constexpr (UO) return X[k];
        else return fmax(Y[(int64_t)k * ldY + i], 0.0) * inv_y * v.invW[k] * inv_c;
    };
    auto y_of = [&](int k) -> double {
        if constexpr (UO) return yv[k];
        else return fmax(Y[(int64_t)k * ldY + i], 0.0) * inv_y;
    };
    const int ld = KM;

    if constexpr (MODE & 1) {
        // up to 36 species: the expanded form on X, X/s, X/s^2; beyond, the
        // factored form on X and 1/s (two vectors fewer in registers)
        constexpr bool kExpand = KM <= 36;
        const double qT = sqrt(sT);
        double V[KM], Wv[kExpand ? KM : 1];   // X_j / s_j and X_j / s_j^2, or 1 / s_j
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int k = 0; k < KM; k++) {
            const double r = rcp_1(qT * fabs(poly5(v.P + kPoly * k, lnT)));
            if constexpr (kExpand) {
                V[k] = X[k] * r;
                Wv[k] = V[k] * r;
            } else {
                V[k] = r;
            }
            const double lk = sT * poly5(v.Q + kPoly * k, lnT);
            a1 = fma(X[k], lk, a1);
            a2 = fma(X[k], rcp_1(lk), a2);
        }
        lam[i] = 0.5 * (a1 + rcp_t(a2));
        double m = 0.0;
        for_species<KM, UO>(K, [&](int k) {
            const double sk = qT * fabs(poly5(v.P + kPoly * k, lnT));
            const double *A = v.A + (int64_t)k * ld, *Bw = v.Bw + (int64_t)k * ld, *C = v.C + (int64_t)k * ld;
            double den;
            if constexpr (kExpand) {
                double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
                for (int j = 0; j < KM; j++)
                    if (!UO || j < K) {   // unrolled kernels skip the padding, the others run through it
                        d0 = fma(A[j], X[j], d0);
                        d1 = fma(Bw[j], V[j], d1);
                        d2 = fma(C[j], Wv[j], d2);
                    }
                den = fma(sk, fma(sk, d2, d1), d0);
            } else {
                // (1 + s_k c1_kj / s_j)^2 c2_kj X_j
                const double *c1 = v.c1 + (int64_t)k * ld;
                den = 0.0;
#pragma unroll
                for (int j = 0; j < KM; j++) {
                    const double t = fma(sk * c1[j], V[j], 1.0);
                    den = fma(X[j], t * t * A[j], den);
                }
            }
            m = fma(x_of(k) * sk * sk, rcp_1(den), m);
        });
        mu[i] = m;
    }

    if constexpr (MODE & 2) {
        const double t32_p = Tc * sT * rcp_1(p[i]);
        if constexpr (UO) {
            // S_k = sum_{j != k} X_j / B_jk(ln T); pairs j < k once each
            double S[KM];
#pragma unroll
            for (int k = 0; k < KM; k++) S[k] = 0.0;
#pragma unroll
            for (int k = 0; k < KM; k++)
                if (k < K) {
                    const double *B = v.B + (int64_t)k * ld * kPoly;
#pragma unroll
                    for (int j = k + 1; j < KM; j++)
                        if (j < K) {
                            const double ib = rcp_1(poly5(B + kPoly * j, lnT));
                            S[j] = fma(X[k], ib, S[j]);
                            S[k] = fma(X[j], ib, S[k]);
                        }
                    const double sk = S[k];
                    D[(int64_t)k * ldD + i] = sk > 0.0 ? (1.0 - yv[k]) * t32_p * rcp_1(sk)
                                                       : t32_p * poly5(B + kPoly * k, lnT);
                }
        } else {
            // a run-time k cannot address the accumulators of the pairs
            // (j < k, k): every species sums its own row (each pair twice)
            for (int k = 0; k < K; k++) {
                const double *B = v.B + (int64_t)k * ld * kPoly;
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < KM; j++) {
                    const double ib = rcp_1(poly5(B + kPoly * j, lnT));
                    s = fma(j == k ? 0.0 : X[j], ib, s);
                }
                D[(int64_t)k * ldD + i] = s > 0.0 ? (1.0 - y_of(k)) * t32_p * rcp_1(s) : t32_p * poly5(B + kPoly * k, lnT);
            }
        }
    }
}

// Range boundaries of the mechanism's species: up to kMaxMid distinct T_mid
// values (ascending); a lane's choice of range for every species is fixed by
// which of them its T has reached.  nt < 0: more distinct values than that,
// the mixture coefficients are rebuilt at every temperature.
constexpr int kMaxMid = 4;
struct MidSet {
    int32_t nt;
    double t[kMaxMid];
};

__device__ __forceinline__ unsigned mid_pattern(const MidSet &ms, double T)
{
    unsigned b = 0;
#pragma unroll
    for (int q = 0; q < kMaxMid; q++)
        if (q < ms.nt && T >= ms.t[q]) b |= 1u << q;
    return b;
}

// Mixture polynomial coefficients at T (computation consolidation): with
// yr_k = Y_k / W_k and each species' range at T, in units of R,
//   cp  = sum_c M[c] T^c                                 (c = 0..4)
//   h   = T (M[0] + sum_c M[4+c] T^c) + M[9]             (c = 1..4)
// where M[0..4] = sum_k yr_k a1..a5, M[5..8] = sum_k yr_k a2/2..a5/5 and
// M[9] = sum_k yr_k a6 -- one pass over the species, after which every
// Newton step costs two quartics, whatever K.  The coefficients are
// uniform scalar loads: a wave wholly in one range takes one multiply-add
// per coefficient; a wave across T_mid takes both ranges with each lane's
// weight zero in the other (never a per-lane coefficient address, which
// would turn the loads into vector loads).
template <int KM>
__device__ __forceinline__ void mix_coeffs(const double *species, int K, const double (&yr)[KM], double T,
                                           double (&M)[10])
{
#pragma unroll
    for (int c = 0; c < 10; c++) M[c] = 0.0;
    constexpr int src[10] = {0, 1, 2, 3, 4, 7, 8, 9, 10, 5};
#pragma unroll
    for (int k = 0; k < KM; k++)
        if (k < K) {
            const double *s = species + k * kSpeciesLen;
            const double *lo = s + 1, *hi = s + 1 + kRangeLen;
            const bool low = T < s[0];
            // each lane's weight is zero in the other range; a range no lane
            // of the wave is in is skipped (a uniform branch)
            const double wl = low ? yr[k] : 0.0, wh = low ? 0.0 : yr[k];
            if (__any(low)) {
#pragma unroll
                for (int c = 0; c < 10; c++) M[c] = fma(wl, lo[src[c]], M[c]);
            }
            if (!__all(low)) {
#pragma unroll
                for (int c = 0; c < 10; c++) M[c] = fma(wh, hi[src[c]], M[c]);
            }
        }
}

__device__ __forceinline__ double mix_cp(const double (&M)[10], double T)
{
    return fma(fma(fma(fma(M[4], T, M[3]), T, M[2]), T, M[1]), T, M[0]);
}

__device__ __forceinline__ double mix_h(const double (&M)[10], double T)
{
    return fma(T, fma(fma(fma(fma(M[8], T, M[7]), T, M[6]), T, M[5]), T, M[0]), M[9]);
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
    double yr[KM], M[10];
    load_yr<KM>(Y, ldY, i, K, invW, yr);
    const double Tc = T[i];
    mix_coeffs<KM>(species, K, yr, Tc, M);
    if (h) h[i] = kRu * mix_h(M, Tc);
    if (cp) cp[i] = kRu * mix_cp(M, Tc);
}

// Temperature from mixture enthalpy: Newton from the guess in T, each step
// T <- clamp(T - (h(T) - h) / cp(T), 200, 3500) K, done when the step is
// below tol; after max_iter steps without that, T = NaN and iters =
// max_iter + 1.  The mixture coefficients are rebuilt only when T crosses a
// range boundary.  cp is the mixture cp at the result.
template <int KM, bool EX>
__global__ void __launch_bounds__(kThermoBlock) t_from_h_kernel(const double *__restrict__ species,
                                                                const double *__restrict__ invW, int Kr, MidSet ms,
                                                                const double *__restrict__ h,
                                                                const double *__restrict__ Y, int64_t ldY,
                                                                int64_t n, double *__restrict__ T,
                                                                double *__restrict__ cp,
                                                                int32_t *__restrict__ iters, int max_iter,
                                                                double tol)
{
    const int64_t i = (int64_t)blockIdx.x * kThermoBlock + threadIdx.x;
    if (i >= n) return;
    const int K = EX ? KM : Kr;   // EX: exactly KM species, guards known at compile time
    double yr[KM], M[10];
    load_yr<KM>(Y, ldY, i, K, invW, yr);
    const double h0 = h[i] * (1.0 / kRu);
    double Tc = T[i];
    unsigned pat = mid_pattern(ms, Tc);
    int it = 0;
    bool done = false, rebuild = true;
    // one copy of the coefficient pass: built first, then again after a
    // step that crossed a range boundary (before the next step, or before cp)
    for (;;) {
        if (rebuild) mix_coeffs<KM>(species, K, yr, Tc, M);
        if (done || it == max_iter) break;
        it++;
        const double dT = -(mix_h(M, Tc) - h0) * rcp_t(mix_cp(M, Tc));
        Tc = fmin(fmax(Tc + dT, 200.0), 3500.0);
        const unsigned np = mid_pattern(ms, Tc);
        rebuild = ms.nt < 0 || np != pat;
        pat = np;
        done = fabs(dT) < tol;
    }
    T[i] = done ? Tc : __builtin_nan("");
    if (cp) cp[i] = done ? kRu * mix_cp(M, Tc) : __builtin_nan("");
    if (iters) iters[i] = done ? it : max_iter + 1;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThermoBlock - 1) / kThermoBlock); }

// Dispatch on the smallest compile-time bound that holds K.  The bounds up to
// 16 unroll every loop and run both phases in one kernel; 20 unrolls them in
// two kernels (the size of the paper's CH4 mechanism); from 24 on the two
// phases are separate kernels (the segments of Section 3.2: the fused
// kernel's registers would cut occupancy to one or two waves per SIMD), the
// diffusion phase unrolled at 24 (its triangular pair loop needs
// compile-time indices) and both phases with run-time outer loops beyond.
#define CHEM_TR_BOUNDS(X) X(9) X(12) X(16) X(20) X(24) X(36) X(48) X(64)

// The kernel bound KM for K species (the tables' padded row count).
int tr_bound(int K)
{
#define CHEM_TR_BOUND(KM) \
    if (K <= KM) return KM;
    CHEM_TR_BOUNDS(CHEM_TR_BOUND)
#undef CHEM_TR_BOUND
    return -1;
}

// Doubles of the transport tables at bound L: P, Q, A, Bw, C, c1, B, invW.
size_t tr_table_len(int L) { return 10 * (size_t)L + 4 * (size_t)L * L + 5 * (size_t)L * L + L; }

template <int KM>
hipError_t launch_transport_km(const TrView &v, const double *T, const double *p, const double *Y, int64_t ldY,
                               int64_t n, double *mu, double *lam, double *D, int64_t ldD, hipStream_t st)
{
    const dim3 g(blocks_for(n)), b(kThermoBlock);
    if constexpr (KM <= 16) {
        const bool ex = v.K == KM;
#define CHEM_TR_UO(MODE)                                                                                      \
    do {                                                                                                     \
        if (ex)                                                                                              \
            hipLaunchKernelGGL((transport_kernel<KM, true, MODE, true>), g, b, 0, st, v, T, p, Y, ldY, n, mu,  \
                               lam, D, ldD);                                                                 \
        else                                                                                                 \
            hipLaunchKernelGGL((transport_kernel<KM, true, MODE, false>), g, b, 0, st, v, T, p, Y, ldY, n, mu, \
                               lam, D, ldD);                                                                 \
    } while (0)
        if (mu && D)
            CHEM_TR_UO(3);
        else if (mu)
            CHEM_TR_UO(1);
        else
            CHEM_TR_UO(2);
#undef CHEM_TR_UO
    } else if constexpr (KM <= 20) {
        // unrolled, in two kernels (the fused one would hold five species
        // vectors: two waves per SIMD)
        const bool ex = v.K == KM;
        if (mu) {
            if (ex)
                hipLaunchKernelGGL((transport_kernel<KM, true, 1, true>), g, b, 0, st, v, T, p, Y, ldY, n, mu, lam,
                                   D, ldD);
            else
                hipLaunchKernelGGL((transport_kernel<KM, true, 1, false>), g, b, 0, st, v, T, p, Y, ldY, n, mu, lam,
                                   D, ldD);
        }
        if (D) {
            if (ex)
                hipLaunchKernelGGL((transport_kernel<KM, true, 2, true>), g, b, 0, st, v, T, p, Y, ldY, n, mu, lam,
                                   D, ldD);
            else
                hipLaunchKernelGGL((transport_kernel<KM, true, 2, false>), g, b, 0, st, v, T, p, Y, ldY, n, mu, lam,
                                   D, ldD);
        }
    } else {
        if (mu)
            hipLaunchKernelGGL((transport_kernel<KM, false, 1>), g, b, 0, st, v, T, p, Y, ldY, n, mu, lam, D, ldD);
        if (D)
            hipLaunchKernelGGL((transport_kernel<KM, KM <= 24, 2>), g, b, 0, st, v, T, p, Y, ldY, n, mu, lam, D,
                               ldD);
    }
    return hipGetLastError();
}

hipError_t launch_transport(const TrView &v, const double *T, const double *p, const double *Y, int64_t ldY,
                            int64_t n, double *mu, double *lam, double *D, int64_t ldD, hipStream_t st)
{
#define CHEM_TR_CASE(KM) \
    if (v.ld == KM) return launch_transport_km<KM>(v, T, p, Y, ldY, n, mu, lam, D, ldD, st);
    CHEM_TR_BOUNDS(CHEM_TR_CASE)
#undef CHEM_TR_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_h_cp(const DevMechView &m, const double *T, const double *Y, int64_t ldY, int64_t n, double *h,
                       double *cp, hipStream_t st)
{
#define CHEM_TH_CASE(KM)                                                                                 \
    if (m.K <= KM) {                                                                                          \
        hipLaunchKernelGGL((h_cp_kernel<KM>), dim3(blocks_for(n)), dim3(kThermoBlock), 0, st, m.species,     \
                           m.invW, m.K, T, Y, ldY, n, h, cp);                                                 \
        return hipGetLastError();                                                                             \
    }
    CHEM_TR_BOUNDS(CHEM_TH_CASE)
#undef CHEM_TH_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_t_from_h(const DevMechView &m, const MidSet &ms, const double *h, const double *Y, int64_t ldY,
                           int64_t n, double *T, double *cp, int32_t *iters, int max_iter, double tol,
                           hipStream_t st)
{
#define CHEM_TN_CASE(KM)                                                                                 \
    if (m.K <= KM) {                                                                                          \
        if (m.K == KM)                                                                                        \
            hipLaunchKernelGGL((t_from_h_kernel<KM, true>), dim3(blocks_for(n)), dim3(kThermoBlock), 0, st,  \
                               m.species, m.invW, m.K, ms, h, Y, ldY, n, T, cp, iters, max_iter, tol);        \
        else                                                                                                  \
            hipLaunchKernelGGL((t_from_h_kernel<KM, false>), dim3(blocks_for(n)), dim3(kThermoBlock), 0, st, \
                               m.species, m.invW, m.K, ms, h, Y, ldY, n, T, cp, iters, max_iter, tol);        \
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
    const int L = chem::tr_bound(K);
    const size_t LL = (size_t)L * L;
    std::vector<double> t(chem::tr_table_len(L), 0.0);
    double *P = t.data(), *Q = P + 5 * L, *A = Q + 5 * L, *Bw = A + LL, *C = Bw + LL, *c1t = C + LL, *B = c1t + LL;
    double *iw = B + 5 * LL;
    for (int k = 0; k < L; k++) {
        P[5 * k] = Q[5 * k] = 1.0;   // padding rows: finite, and weighted by X = 0
        iw[k] = 1.0;
        for (int j = 0; j < L; j++) B[((size_t)k * L + j) * 5] = 1.0;
    }
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
            const double c1 = std::pow(Wj / Wk, 0.25), c2 = 1.0 / std::sqrt(8.0 * (1.0 + Wk / Wj));
            A[(size_t)k * L + j] = c2;
            Bw[(size_t)k * L + j] = 2.0 * c1 * c2;
            C[(size_t)k * L + j] = std::sqrt(Wj / Wk) * c2;
            c1t[(size_t)k * L + j] = c1;
            for (int c = 0; c < 5; c++) {
                const double a = diff[((size_t)k * K + j) * 5 + c];
                if (!std::isfinite(a)) return fail(CHEM_EINVAL, "transport fits must be finite");
                if (a != diff[((size_t)j * K + k) * 5 + c])
                    return fail(CHEM_EINVAL, "the binary diffusion fits must be symmetric in the two species");
                B[((size_t)k * L + j) * 5 + c] = a;
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
    // the distinct range boundaries of the species with two distinct ranges
    chem::MidSet ms{};
    std::vector<double> mids;
    for (int k = 0; k < m->host.K; k++) {
        const double *a = &m->host.nasa[k][0];
        bool two = false;
        for (int j = 0; j < 7; j++) two = two || a[3 + j] != a[10 + j];
        if (two) mids.push_back(a[1]);
    }
    std::sort(mids.begin(), mids.end());
    mids.erase(std::unique(mids.begin(), mids.end()), mids.end());
    ms.nt = mids.size() <= (size_t)chem::kMaxMid ? (int32_t)mids.size() : -1;
    for (int q = 0; q < chem::kMaxMid && q < (int)mids.size(); q++) ms.t[q] = mids[q];
    return check_hip(chem::launch_t_from_h(m->view, ms, h, Y, ldY, n, T, cp, iters, max_iter, tol,
                                           (hipStream_t)stream),
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
    const int K = m->host.K, L = chem::tr_bound(K);
    const size_t LL = (size_t)L * L;
    const double *t = (const double *)m->transport_block;
    chem::TrView v{K, L, t, t + 5 * L, t + 10 * L, t + 10 * L + LL, t + 10 * L + 2 * LL, t + 10 * L + 3 * LL,
                   t + 10 * L + 4 * LL, t + 10 * L + 9 * LL};
    return check_hip(chem::launch_transport(v, T, p, Y, ldY, n, mu, lam, D, ldD, (hipStream_t)stream),
                     "transport launch");
}

}  // extern "C"

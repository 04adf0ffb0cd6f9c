// HIP kernels for gfx950: reactor right-hand side, analytic Jacobian and the
// one-thread-per-cell BDF integrator.
//
// Data layout: cell state is structure-of-arrays in HBM (T[i], p[i],
// Y[k*ldY + i]) so that consecutive lanes read consecutive doubles (paper
// Section 3.2: coalesced storage of the components of multi-component fields).
// Mechanism tables are read with wave-uniform addresses, i.e. through scalar
// loads, and the species count K is a template parameter so that every
// per-species array lives in registers.  Reaction loops run over a runtime
// count with wave-uniform species indices (register indexing mode).
//
// The integrator implements the same contract as the CPU oracle (variable
// order 1..5, variable-coefficient BDF in Nordsieck form, modified Newton,
// identical constants and decision rules) but is written independently.

#include "chem_internal.h"

namespace chem {
namespace {

// ---------------------------------------------------------------------------
// thermo and kinetics building blocks
// ---------------------------------------------------------------------------

// Species thermo at T: cp/R, H/(RT), G/(RT), and d(cp/R)/dT when wanted.
template <int K, bool WANT_DCP>
__device__ __forceinline__ void species_thermo(const DevMechView &m, double T, double invT,
                                               double lnT, double *cpR, double *hRT, double *gRT,
                                               double *dcpR)
{
#pragma unroll
    for (int k = 0; k < K; k++) {
        const double *s = m.species + k * kSpeciesLen;
        const double *c = s + 1;
        double a[kRangeLen];
        if (m.two_range) {
            const double *hi = s + 1 + kRangeLen;
            const bool low = T < s[0];
#pragma unroll
            for (int j = 0; j < kRangeLen; j++) a[j] = low ? c[j] : hi[j];
        } else {
#pragma unroll
            for (int j = 0; j < kRangeLen; j++) a[j] = c[j];
        }
        cpR[k] = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
        hRT[k] = a[0] + T * (a[7] + T * (a[8] + T * (a[9] + T * a[10]))) + a[5] * invT;
        const double sR = a[0] * lnT + T * (a[1] + T * (a[11] + T * (a[12] + T * a[13]))) + a[6];
        gRT[k] = hRT[k] - sR;
        if (WANT_DCP) dcpR[k] = a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * 4.0 * a[4]));
    }
}

// Right-hand side f(y), y = (Y_1..Y_K, T).
template <int K>
__device__ void reactor_rhs(const DevMechView &m, double p, const double *y, double *f)
{
    const double T = y[K];
    const double invT = 1.0 / T;
    const double lnT = log(T);
    double cpR[K], hRT[K + 1], gRT[K + 1], C[K + 1], wdot[K + 1];
    species_thermo<K, false>(m, T, invT, lnT, cpR, hRT, gRT, nullptr);
    gRT[K] = 0.0;
    hRT[K] = 0.0;
    double sumYW = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) sumYW += y[k] * m.invW[k];
    const double rho = p / (kRu * T * sumYW);
    double cpm = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        C[k] = rho * y[k] * m.invW[k];
        cpm += y[k] * cpR[k] * m.invW[k];
        wdot[k] = 0.0;
    }
    C[K] = 1.0;
    wdot[K] = 0.0;
    cpm *= kRu;
    const double ln_c0 = log(kPstd / kRu) - lnT;   // ln(p_std / (R T))
    for (int r = 0; r < m.R; r++) {
        const DevRxn x = m.rxn[r];
        const double lnkf = x.lnA + x.b * lnT - x.Ea_R * invT;
        const double dg = gRT[x.p0] + gRT[x.p1] - gRT[x.r0] - gRT[x.r1];
        // k_r = k_f / K_c with ln K_c = -dg + dnu ln(p_std/(R T))
        const double lnkr = lnkf + dg - x.dnu * ln_c0;
        const double q = exp(lnkf) * C[x.r0] * C[x.r1] - exp(lnkr) * C[x.p0] * C[x.p1];
        wdot[x.r0] -= q;
        wdot[x.r1] -= q;
        wdot[x.p0] += q;
        wdot[x.p1] += q;
    }
    const double inv_rho = 1.0 / rho;
    double heat = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        f[k] = m.W[k] * wdot[k] * inv_rho;
        heat += hRT[k] * wdot[k];
    }
    f[K] = -(kRu * T) * heat / (rho * cpm);
}

// Analytic Jacobian J[r][c] = d f_r / d y_c (row-major, N x N registers).
// The species block of dwdot/dC is accumulated with wave-uniform indices in
// a per-thread array A (private memory); everything else is static.
template <int K>
__device__ void reactor_jacobian(const DevMechView &m, double p, const double *y, double *J)
{
    constexpr int N = K + 1;
    constexpr int KP = K + 1;   // with the sentinel slot
    const double T = y[K];
    const double invT = 1.0 / T;
    const double lnT = log(T);
    double cpR[K], hRT[KP], gRT[KP], dcpR[K], C[KP], wdot[KP], wT[KP];
    double A[KP * KP];
    species_thermo<K, true>(m, T, invT, lnT, cpR, hRT, gRT, dcpR);
    gRT[K] = 0.0;
    hRT[K] = 0.0;
    double sumYW = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) sumYW += y[k] * m.invW[k];
    const double wbar = 1.0 / sumYW;
    const double rho = p * wbar / (kRu * T);
    double cpm = 0.0, dcpm = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        C[k] = rho * y[k] * m.invW[k];
        cpm += y[k] * cpR[k] * m.invW[k];
        dcpm += y[k] * dcpR[k] * m.invW[k];
    }
    cpm *= kRu;
    dcpm *= kRu;
    C[K] = 1.0;
#pragma unroll
    for (int k = 0; k < KP; k++) {
        wdot[k] = 0.0;
        wT[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < KP * KP; k++) A[k] = 0.0;
    const double ln_c0 = log(kPstd / kRu) - lnT;
    for (int r = 0; r < m.R; r++) {
        const DevRxn x = m.rxn[r];
        const double lnkf = x.lnA + x.b * lnT - x.Ea_R * invT;
        const double dg = gRT[x.p0] + gRT[x.p1] - gRT[x.r0] - gRT[x.r1];
        const double dh = hRT[x.p0] + hRT[x.p1] - hRT[x.r0] - hRT[x.r1];
        const double lnkr = lnkf + dg - x.dnu * ln_c0;
        const double kf = exp(lnkf), kr = exp(lnkr);
        const double fwd = kf * C[x.r0] * C[x.r1];
        const double rev = kr * C[x.p0] * C[x.p1];
        const double q = fwd - rev;
        const double dlnkf = (x.b + x.Ea_R * invT) * invT;
        const double dlnkr = dlnkf - (dh - x.dnu) * invT;
        const double dqT = fwd * dlnkf - rev * dlnkr;
        // d q / d C at each slot (an empty slot's entry lands on the sentinel)
        const int sl[4] = {x.r0, x.r1, x.p0, x.p1};
        const double dq[4] = {kf * C[x.r1], kf * C[x.r0], -kr * C[x.p1], -kr * C[x.p0]};
        const double nu[4] = {-1.0, -1.0, 1.0, 1.0};
#pragma unroll
        for (int a = 0; a < 4; a++) {
            wdot[sl[a]] += nu[a] * q;
            wT[sl[a]] += nu[a] * dqT;
#pragma unroll
            for (int b = 0; b < 4; b++) A[sl[a] * KP + sl[b]] += nu[a] * dq[b];
        }
    }
    double AC[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < K; l++) s += A[k * KP + l] * C[l];
        AC[k] = s;
    }
    const double g = wbar / rho;
    const double RT = kRu * T;
    const double rcp = rho * cpm;
    double S = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) S += RT * hRT[k] * wdot[k];
    double dST = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        const double u = wdot[k] - AC[k];
        const double BT = wT[k] - AC[k] * invT;
        J[k * N + K] = m.W[k] / rho * (wT[k] + u * invT);
        dST += kRu * cpR[k] * wdot[k] + RT * hRT[k] * BT;
    }
#pragma unroll
    for (int j = 0; j < K; j++) {
        double dS = 0.0;
#pragma unroll
        for (int k = 0; k < K; k++) {
            const double v = A[k * KP + j] - g * AC[k];   // B_kj * W_j / rho
            J[k * N + j] = m.W[k] * m.invW[j] * (v + g * wdot[k]);
            dS += RT * hRT[k] * v;
        }
        dS *= rho * m.invW[j];
        const double drcp = rho * m.invW[j] * (kRu * cpR[j] - cpm * wbar);
        J[K * N + j] = -dS / rcp + S * drcp / (rcp * rcp);
    }
    const double drcpT = rho * dcpm - cpm * rho * invT;
    J[K * N + K] = -dST / rcp + S * drcpT / (rcp * rcp);
}

// ---------------------------------------------------------------------------
// dense LU with partial pivoting in registers
// ---------------------------------------------------------------------------

// Factor M in place; ties keep the upper row.  Returns false on a zero pivot.
template <int N>
__device__ __forceinline__ bool lu_factor(double *M, int *piv)
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < N; k++) {
        int pk = k;
        double best = fabs(M[k * N + k]);
#pragma unroll
        for (int r = k + 1; r < N; r++) {
            const double v = fabs(M[r * N + k]);
            if (v > best) {
                best = v;
                pk = r;
            }
        }
        piv[k] = pk;
        ok = ok && (best != 0.0);
        if (pk != k) {
#pragma unroll
            for (int r = k + 1; r < N; r++) {
                if (pk == r) {
#pragma unroll
                    for (int c = 0; c < N; c++) {
                        const double t = M[k * N + c];
                        M[k * N + c] = M[r * N + c];
                        M[r * N + c] = t;
                    }
                }
            }
        }
        const double inv = 1.0 / M[k * N + k];
#pragma unroll
        for (int r = k + 1; r < N; r++) {
            const double l = M[r * N + k] * inv;
            M[r * N + k] = l;
#pragma unroll
            for (int c = k + 1; c < N; c++) M[r * N + c] -= l * M[k * N + c];
        }
    }
    return ok;
}

template <int N>
__device__ __forceinline__ void lu_solve(const double *M, const int *piv, double *b)
{
#pragma unroll
    for (int k = 0; k < N; k++) {
        const int pk = piv[k];
        if (pk != k) {
#pragma unroll
            for (int r = k + 1; r < N; r++) {
                if (pk == r) {
                    const double t = b[k];
                    b[k] = b[r];
                    b[r] = t;
                }
            }
        }
    }
#pragma unroll
    for (int r = 1; r < N; r++)
#pragma unroll
        for (int c = 0; c < r; c++) b[r] -= M[r * N + c] * b[c];
#pragma unroll
    for (int r = N - 1; r >= 0; r--) {
#pragma unroll
        for (int c = r + 1; c < N; c++) b[r] -= M[r * N + c] * b[c];
        b[r] /= M[r * N + r];
    }
}

// ---------------------------------------------------------------------------
// the BDF contract
// ---------------------------------------------------------------------------

constexpr int kMaxCor = 3;
constexpr int kMsbp = 20;
constexpr double kDgmax = 0.3;
constexpr double kCrdown = 0.3;
constexpr double kRdiv = 2.0;
constexpr double kNlscoef = 0.1;
constexpr int kMaxNef = 7;
constexpr int kMaxNcf = 10;
constexpr double kEtaCf = 0.25;
constexpr double kEtaMinEf = 0.1;
constexpr double kEtaMaxEf = 0.9;
constexpr double kEtaNef2 = 0.2;
constexpr int kNefRestart = 3;
constexpr double kThresh = 1.5;
constexpr double kEtaMaxFirst = 1e4;
constexpr double kEtaMax = 10.0;
constexpr double kBiasQm1 = 6.0, kBiasQ = 6.0, kBiasQp1 = 10.0;
constexpr double kAddon = 1e-6;
constexpr int kH0Iters = 4;

template <int N>
__device__ __forceinline__ double wrms_norm(const double *v, const double *w)
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < N; i++) {
        const double t = v[i] * w[i];
        s += t * t;
    }
    return sqrt(s * (1.0 / N));
}

template <int N>
__device__ __forceinline__ bool finite_vec(const double *v)
{
    bool ok = true;
#pragma unroll
    for (int i = 0; i < N; i++) ok = ok && isfinite(v[i]);
    return ok;
}

// z[j][i] ~ h^j y^(j) / j!.  All loops run to kQmax with the order as a guard
// so that the array stays in registers.
template <int N>
__device__ __forceinline__ void nord_shift(double (*z)[N], int q, double sign)
{
#pragma unroll
    for (int k = 1; k <= kQmax; k++)
#pragma unroll
        for (int j = kQmax; j >= k; j--)
            if (j <= q)
#pragma unroll
                for (int i = 0; i < N; i++) z[j - 1][i] += sign * z[j][i];
}

template <int N>
__device__ __forceinline__ void nord_unshift(double (*z)[N], int q)
{
#pragma unroll
    for (int k = kQmax; k >= 1; k--)
#pragma unroll
        for (int j = k; j <= kQmax; j++)
            if (j <= q && k <= q)
#pragma unroll
                for (int i = 0; i < N; i++) z[j - 1][i] -= z[j][i];
}

template <int N>
__device__ __forceinline__ void nord_scale(double (*z)[N], int q, double eta)
{
    double f = 1.0;
#pragma unroll
    for (int j = 1; j <= kQmax; j++) {
        f *= eta;
        if (j <= q)
#pragma unroll
            for (int i = 0; i < N; i++) z[j][i] *= f;
    }
}

__device__ __forceinline__ double factorial_d(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= i;
    return f;
}

struct Counters {
    int nst, nfe, nje, nni, netf, ncfn;
};

// Integrate one cell; y holds the state (in/out).  Returns a CHEM_CELL code.
template <int K>
__device__ int integrate_cell(const DevMechView &m, double p, double *y, double t_end,
                              const BdfParams &prm, Counters &cnt)
{
    constexpr int N = K + 1;
    double z[kQmax + 2][N];
    double M[N * N];
    int piv[N];
    double w[N], e[N], ehat[N], tmp[N], fy[N], y0[N];
    double tau[kQmax + 3];
    double xi[kQmax + 3], l[kQmax + 2];
    const double rtol = prm.rtol, atol = prm.atol;

#pragma unroll
    for (int i = 0; i < N; i++) y0[i] = y[i];
#pragma unroll
    for (int i = 0; i < kQmax + 3; i++) tau[i] = 0.0;

    // initial derivative and step size
    reactor_rhs<K>(m, p, y0, fy);
    cnt.nfe++;
    if (!finite_vec<N>(fy)) return 4;
#pragma unroll
    for (int i = 0; i < N; i++) w[i] = 1.0 / (rtol * fabs(y0[i]) + atol);
    double h;
    if (wrms_norm<N>(fy, w) == 0.0) {
        h = t_end;
    } else {
        double hub = t_end;
#pragma unroll
        for (int i = 0; i < N; i++) {
            const double lim = 0.1 * fabs(y0[i]) + 1.0 / w[i];
            if (fabs(fy[i]) * hub > lim) hub = lim / fabs(fy[i]);
        }
        double hg = hub;
        for (int it = 0; it < kH0Iters; it++) {
#pragma unroll
            for (int i = 0; i < N; i++) tmp[i] = y0[i] + hg * fy[i];
            double f1[N];
            reactor_rhs<K>(m, p, tmp, f1);
            cnt.nfe++;
            if (!finite_vec<N>(f1)) {
                hg *= 0.1;
                continue;
            }
#pragma unroll
            for (int i = 0; i < N; i++) tmp[i] = (f1[i] - fy[i]) / hg;
            const double ydd = wrms_norm<N>(tmp, w);
            double hnew = ydd > 0.0 ? sqrt(2.0 / ydd) : hub;
            if (hnew > hub) hnew = hub;
            const double ratio = hnew / hg;
            hg = hnew;
            if (ratio >= 0.5 && ratio <= 2.0) break;
        }
        h = 0.5 * hg;
        if (h > t_end) h = t_end;
    }
    int q = 1;
#pragma unroll
    for (int j = 0; j < kQmax + 2; j++)
#pragma unroll
        for (int i = 0; i < N; i++) z[j][i] = 0.0;
#pragma unroll
    for (int i = 0; i < N; i++) {
        z[0][i] = y0[i];
        z[1][i] = h * fy[i];
    }

    int qwait = 2, nst_M = 0;
    bool have_M = false, ehat_ok = false;
    double gamma_M = 0.0, crate = 1.0, ehat_h = 0.0;
    double t = 0.0;

    while (t < t_end) {
        if (cnt.nst >= prm.max_steps) return 1;
        bool last = false;
        if (t + h >= t_end) {
            nord_scale<N>(z, q, (t_end - t) / h);
            h = t_end - t;
            last = true;
        }
#pragma unroll
        for (int i = 0; i < N; i++) w[i] = 1.0 / (rtol * fabs(z[0][i]) + atol);
        int nef = 0, ncf = 0;
        bool force_M = false;
        double dsm = 0.0;
        for (;;) {
            const double tnew = t + h;
            if (tnew == t) return 2;
            nord_shift<N>(z, q, 1.0);
            // coefficients: xi_i = (t_new - t_{new-i}) / h, Lambda = prod (1 + x/xi_i)
            {
                double s = h;
                xi[1] = 1.0;
#pragma unroll
                for (int i = 2; i <= kQmax + 1; i++) {
                    s += tau[i - 1];
                    xi[i] = s / h;
                }
                l[0] = 1.0;
#pragma unroll
                for (int j = 1; j <= kQmax; j++) l[j] = 0.0;
#pragma unroll
                for (int i = 1; i <= kQmax; i++)
                    if (i <= q)
#pragma unroll
                        for (int j = i; j >= 1; j--) l[j] += l[j - 1] / xi[i];
            }
            const double gamma = h / l[1];
            double xq1 = xi[2];
#pragma unroll
            for (int i = 3; i <= kQmax + 1; i++)
                if (i == q + 1) xq1 = xi[i];
            const double Cq = 1.0 / (1.0 + l[1] * xq1);
            bool jcur = false, conv = false, lu_ok = true;
            if (!have_M || force_M || cnt.nst >= nst_M + kMsbp || fabs(gamma / gamma_M - 1.0) > kDgmax) {
                reactor_jacobian<K>(m, p, z[0], M);
#pragma unroll
                for (int r = 0; r < N; r++)
#pragma unroll
                    for (int c = 0; c < N; c++) M[r * N + c] = (r == c ? 1.0 : 0.0) - gamma * M[r * N + c];
                cnt.nje++;
                lu_ok = lu_factor<N>(M, piv);
                gamma_M = gamma;
                nst_M = cnt.nst;
                crate = 1.0;
                have_M = lu_ok;
                jcur = true;
                force_M = false;
            }
            if (lu_ok) {
                double del_old = 0.0;
#pragma unroll
                for (int i = 0; i < N; i++) {
                    e[i] = 0.0;
                    tmp[i] = z[0][i];
                }
                const double inv_l1 = 1.0 / l[1];
                for (int it = 0; it < kMaxCor; it++) {
                    reactor_rhs<K>(m, p, tmp, fy);
                    cnt.nfe++;
                    if (!finite_vec<N>(fy)) break;
                    double d[N];
#pragma unroll
                    for (int i = 0; i < N; i++) d[i] = -(e[i] - gamma * fy[i] + z[1][i] * inv_l1);
                    lu_solve<N>(M, piv, d);
                    if (gamma != gamma_M) {
                        const double s = 2.0 / (1.0 + gamma / gamma_M);
#pragma unroll
                        for (int i = 0; i < N; i++) d[i] *= s;
                    }
                    const double dl = wrms_norm<N>(d, w);
#pragma unroll
                    for (int i = 0; i < N; i++) {
                        e[i] += d[i];
                        tmp[i] = z[0][i] + e[i];
                    }
                    cnt.nni++;
                    if (it > 0) crate = fmax(kCrdown * crate, dl / del_old);
                    const double dcon = dl * fmin(crate, 1.0) * Cq / kNlscoef;
                    if (dcon <= 1.0) {
                        conv = true;
                        break;
                    }
                    if (it > 0 && dl > kRdiv * del_old) break;
                    del_old = dl;
                }
            }
            if (!conv) {
                nord_unshift<N>(z, q);
                if (!jcur) {
                    force_M = true;
                    continue;
                }
                cnt.ncfn++;
                if (++ncf >= kMaxNcf) return 3;
                nord_scale<N>(z, q, kEtaCf);
                h *= kEtaCf;
                last = false;
                continue;
            }
            dsm = Cq * wrms_norm<N>(e, w);
            if (dsm > 1.0) {
                nord_unshift<N>(z, q);
                cnt.netf++;
                if (++nef >= kMaxNef) return 2;
                last = false;
                if (nef >= kNefRestart) {
                    h *= kEtaMinEf;
                    q = 1;
                    reactor_rhs<K>(m, p, z[0], fy);
                    cnt.nfe++;
                    if (!finite_vec<N>(fy)) return 4;
#pragma unroll
                    for (int i = 0; i < N; i++) z[1][i] = h * fy[i];
#pragma unroll
                    for (int i = 0; i < kQmax + 3; i++) tau[i] = 0.0;
                    qwait = 2;
                    ehat_ok = false;
                    continue;
                }
                double eta = 1.0 / (pow(kBiasQ * dsm, 1.0 / (q + 1)) + kAddon);
                eta = fmin(fmax(eta, kEtaMinEf), kEtaMaxEf);
                if (nef >= 2) eta = fmin(eta, kEtaNef2);
                nord_scale<N>(z, q, eta);
                h *= eta;
                continue;
            }
            // accepted: z += l e
#pragma unroll
            for (int j = 0; j <= kQmax; j++)
                if (j <= q)
#pragma unroll
                    for (int i = 0; i < N; i++) z[j][i] += l[j] * e[i];
            break;
        }
        t = last ? t_end : t + h;
        cnt.nst++;
        if (t >= t_end) break;

        // ---- next step size and order ----
        const double h_done = h;
        double prod_q = 1.0, xq1 = xi[2];
#pragma unroll
        for (int i = 1; i <= kQmax; i++)
            if (i <= q) prod_q *= xi[i];
#pragma unroll
        for (int i = 3; i <= kQmax + 1; i++)
            if (i == q + 1) xq1 = xi[i];
        const double gfac = prod_q * (1.0 / l[1] + xq1) / factorial_d(q + 1);
        double ehat_new[N];
#pragma unroll
        for (int i = 0; i < N; i++) ehat_new[i] = e[i] / gfac;
        if (qwait > 0) qwait--;
        const double etamax = (nef > 0 || ncf > 0) ? 1.0 : (cnt.nst == 1 ? kEtaMaxFirst : kEtaMax);
        double eta = 1.0;
        int qnew = q;
        if (etamax > 1.0) {
            eta = 1.0 / (pow(kBiasQ * dsm, 1.0 / (q + 1)) + kAddon);
            if (qwait == 0) {
                double eta_m = 0.0, eta_p = 0.0;
                if (q > 1) {
                    double prod = 1.0, l1 = 0.0, zq[N];
#pragma unroll
                    for (int i = 0; i < N; i++) zq[i] = 0.0;
#pragma unroll
                    for (int j = 2; j <= kQmax; j++)
                        if (j == q)
#pragma unroll
                            for (int i = 0; i < N; i++) zq[i] = z[j][i];
#pragma unroll
                    for (int i = 1; i < kQmax; i++)
                        if (i <= q - 1) {
                            prod *= xi[i];
                            l1 += 1.0 / xi[i];
                        }
                    const double Em = wrms_norm<N>(zq, w) * prod / l1;
                    eta_m = 1.0 / (pow(kBiasQm1 * Em, 1.0 / q) + kAddon);
                }
                if (q < kQmax && ehat_ok) {
                    const double rr = pow(h_done / ehat_h, q + 1);
                    double dv[N];
#pragma unroll
                    for (int i = 0; i < N; i++) dv[i] = ehat_new[i] - ehat[i] * rr;
                    double prod = 1.0, l1 = 0.0;
#pragma unroll
                    for (int i = 1; i <= kQmax; i++)
                        if (i <= q + 1) {
                            prod *= xi[i];
                            l1 += 1.0 / xi[i];
                        }
                    const double Ep = wrms_norm<N>(dv, w) * prod / (factorial_d(q + 2) * l1);
                    eta_p = 1.0 / (pow(kBiasQp1 * Ep, 1.0 / (q + 2)) + kAddon);
                }
                if (eta_m > eta && eta_m >= eta_p) {
                    eta = eta_m;
                    qnew = q - 1;
                } else if (eta_p > eta) {
                    eta = eta_p;
                    qnew = q + 1;
                }
            }
            if (eta < kThresh) {
                eta = 1.0;
                qnew = q;
            } else if (eta > etamax) {
                eta = etamax;
            }
        }
        if (qnew == q - 1) {
            // drop the top column: subtract z_q * x * prod_{i<q} (x + xi_i)
            double d[kQmax + 2];
#pragma unroll
            for (int j = 0; j < kQmax + 2; j++) d[j] = 0.0;
            d[1] = 1.0;
#pragma unroll
            for (int i = 1; i < kQmax; i++)
                if (i <= q - 1)
#pragma unroll
                    for (int j = kQmax; j >= 1; j--)
                        if (j <= i + 1) d[j] = d[j - 1] + xi[i] * d[j];
            double zq[N];
#pragma unroll
            for (int i = 0; i < N; i++) zq[i] = 0.0;
#pragma unroll
            for (int j = 2; j <= kQmax; j++)
                if (j == q)
#pragma unroll
                    for (int i = 0; i < N; i++) zq[i] = z[j][i];
#pragma unroll
            for (int j = 1; j < kQmax; j++)
                if (j < q)
#pragma unroll
                    for (int i = 0; i < N; i++) z[j][i] -= d[j] * zq[i];
            q = qnew;
            qwait = q + 1;
            ehat_ok = false;
        } else if (qnew == q + 1) {
            // add e * (x / xi_{q+1}) * Lambda_q(x)
            double xq1n = xi[2];
#pragma unroll
            for (int i = 3; i <= kQmax + 1; i++)
                if (i == q + 1) xq1n = xi[i];
            const double inv = 1.0 / xq1n;
#pragma unroll
            for (int j = 2; j <= kQmax; j++)
                if (j == q + 1)
#pragma unroll
                    for (int i = 0; i < N; i++) z[j][i] = 0.0;
#pragma unroll
            for (int j = 1; j <= kQmax; j++)
                if (j <= q + 1)
#pragma unroll
                    for (int i = 0; i < N; i++) z[j][i] += e[i] * l[j - 1] * inv;
            q = qnew;
            qwait = q + 1;
            ehat_ok = false;
        } else {
#pragma unroll
            for (int i = 0; i < N; i++) ehat[i] = ehat_new[i];
            ehat_h = h_done;
            ehat_ok = true;
        }
#pragma unroll
        for (int i = kQmax + 2; i >= 2; i--) tau[i] = tau[i - 1];
        tau[1] = h_done;
        if (eta != 1.0) {
            nord_scale<N>(z, q, eta);
            h *= eta;
        }
    }
#pragma unroll
    for (int i = 0; i < N; i++) y[i] = z[0][i];
    if (!finite_vec<N>(y)) return 4;
    return 0;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <int K>
__global__ void __launch_bounds__(256) rhs_kernel(DevMechView m, const double *__restrict__ T,
                                                  const double *__restrict__ p,
                                                  const double *__restrict__ Y, int64_t ldY,
                                                  int64_t n, double *__restrict__ F, int64_t ldF)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int N = K + 1;
    double y[N], f[N];
#pragma unroll
    for (int k = 0; k < K; k++) y[k] = Y[k * ldY + i];
    y[K] = T[i];
    reactor_rhs<K>(m, p[i], y, f);
#pragma unroll
    for (int k = 0; k < N; k++) F[k * ldF + i] = f[k];
}

template <int K>
__global__ void __launch_bounds__(64) jac_kernel(DevMechView m, const double *__restrict__ T,
                                                 const double *__restrict__ p,
                                                 const double *__restrict__ Y, int64_t ldY,
                                                 int64_t n, double *__restrict__ J, int64_t ldJ)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int N = K + 1;
    double y[N], jac[N * N];
#pragma unroll
    for (int k = 0; k < K; k++) y[k] = Y[k * ldY + i];
    y[K] = T[i];
    reactor_jacobian<K>(m, p[i], y, jac);
#pragma unroll
    for (int k = 0; k < N * N; k++) J[k * ldJ + i] = jac[k];
}

template <int K>
__global__ void __launch_bounds__(64) bdf_thread_kernel(DevMechView m, double *__restrict__ T,
                                                        const double *__restrict__ p,
                                                        double *__restrict__ Y, int64_t ldY,
                                                        int64_t n, double dt, BdfParams prm,
                                                        int32_t *__restrict__ status,
                                                        int32_t *__restrict__ counters)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int N = K + 1;
    double y[N];
#pragma unroll
    for (int k = 0; k < K; k++) y[k] = Y[k * ldY + i];
    y[K] = T[i];
    Counters cnt = {0, 0, 0, 0, 0, 0};
    const int st = integrate_cell<K>(m, p[i], y, dt, prm, cnt);
    if (st == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) Y[k * ldY + i] = y[k];
        T[i] = y[K];
    }
    if (status) status[i] = st;
    if (counters) {
        counters[0 * n + i] = cnt.nst;
        counters[1 * n + i] = cnt.nfe;
        counters[2 * n + i] = cnt.nje;
        counters[3 * n + i] = cnt.nni;
        counters[4 * n + i] = cnt.netf;
        counters[5 * n + i] = cnt.ncfn;
    }
}

}  // namespace

#define CHEM_FOR_EACH_K(X) X(9)

bool thread_kernel_supports(int K)
{
#define CHEM_CASE(KK) if (K == KK) return true;
    CHEM_FOR_EACH_K(CHEM_CASE)
#undef CHEM_CASE
    return false;
}

static dim3 grid_for(int64_t n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

hipError_t launch_rhs(const DevMechView &m, const double *T, const double *p, const double *Y,
                      int64_t ldY, int64_t n, double *F, int64_t ldF, hipStream_t s)
{
#define CHEM_CASE(KK)                                                                          \
    if (m.K == KK) {                                                                           \
        hipLaunchKernelGGL(rhs_kernel<KK>, grid_for(n, 256), dim3(256), 0, s, m, T, p, Y, ldY, \
                           n, F, ldF);                                                         \
        return hipGetLastError();                                                              \
    }
    CHEM_FOR_EACH_K(CHEM_CASE)
#undef CHEM_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_jacobian(const DevMechView &m, const double *T, const double *p, const double *Y,
                           int64_t ldY, int64_t n, double *J, int64_t ldJ, hipStream_t s)
{
#define CHEM_CASE(KK)                                                                         \
    if (m.K == KK) {                                                                          \
        hipLaunchKernelGGL(jac_kernel<KK>, grid_for(n, 64), dim3(64), 0, s, m, T, p, Y, ldY, \
                           n, J, ldJ);                                                        \
        return hipGetLastError();                                                             \
    }
    CHEM_FOR_EACH_K(CHEM_CASE)
#undef CHEM_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_bdf_thread(const DevMechView &m, double *T, const double *p, double *Y,
                             int64_t ldY, int64_t n, double dt, const BdfParams &prm,
                             int32_t *status, int32_t *counters, int block, hipStream_t s)
{
    if (block <= 0) block = 64;
#define CHEM_CASE(KK)                                                                           \
    if (m.K == KK) {                                                                            \
        hipLaunchKernelGGL(bdf_thread_kernel<KK>, grid_for(n, block), dim3(block), 0, s, m, T, \
                           p, Y, ldY, n, dt, prm, status, counters);                           \
        return hipGetLastError();                                                               \
    }
    CHEM_FOR_EACH_K(CHEM_CASE)
#undef CHEM_CASE
    return hipErrorInvalidValue;
}

}  // namespace chem

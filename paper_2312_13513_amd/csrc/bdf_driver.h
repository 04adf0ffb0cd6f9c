// BDF integrator driver for gfx950: one lane owns one cell, lanes refill from
// a work queue, and each lane runs a small state machine so that the costly
// pieces -- the right-hand side and the Jacobian + LU -- have exactly one call
// site each.  Whatever phase a lane is in (initial-step estimate, Newton
// iteration, restart), all lanes that need a right-hand side evaluate it
// together in the same instruction stream; branch divergence is confined to
// the cheap bookkeeping between those sites.
//
// The decisions follow the integrator contract shared with the CPU oracle
// (variable-order 1..5, variable-coefficient BDF in Nordsieck form, modified
// Newton); only their scheduling across lanes differs.
//
// Mech is a functor type with `static constexpr int K` and device members
//   rhs(p, y[K+1], f[K+1])   and   jac(p, y[K+1], J[(K+1)*(K+1)]).
#pragma once

#include <utility>

#include "chem_internal.h"
#include "kinetics.h"

namespace chem {

// ---------------------------------------------------------------------------
// dense LU with row partial pivoting, registers, static indexing
// ---------------------------------------------------------------------------

// A value the optimiser must treat as opaque: a per-lane row exchange written
// as selects between such values cannot be folded back into a load through a
// selected address (which would push the whole array out of registers).
__device__ __forceinline__ double reg_value(double v)
{
    unsigned lo = (unsigned)__double_as_longlong(v);
    unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(v) >> 32);
    
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Reciprocal of a finite nonzero x: the hardware estimate refined by two
// Newton steps (within an ulp or two of 1/x; the step-control quantities it
// serves are continuous, and a division costs several times more here).
__device__ __forceinline__ double rcp_d(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

// x^(1/k) for x >= 0, k = 1..7, as exp(ln x / k).
__device__ __forceinline__ double root_k(double x, int k)
{
    const double inv = k == 1 ? 1.0 : k == 2 ? 0.5 : k == 3 ? 1.0 / 3.0 : k == 4 ? 0.25
                     : k == 5 ? 0.2 : k == 6 ? 1.0 / 6.0 : 1.0 / 7.0;
    return exp(log(x) * inv);
}

// x^k for k = 1..7 by products.
__device__ __forceinline__ double pow_k(double x, int k)
{
    double r = x;
#pragma unroll
    for (int j = 2; j <= 7; j++)
        if (j <= k) r *= x;
    return r;
}

// Compile-time loops: f(std::integral_constant<int, i>) for i in [B, E).  The
// index is a constant expression in the body, so every array access it makes
// is static whatever the loop unroller decides (a dynamic index would push
// the whole per-lane state out of registers into scratch memory).
template <int B, class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, B + I>{}), ...);
}
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (E > B) static_for_impl<B>(f, std::make_integer_sequence<int, E - B>{});
}

// Factor in place; ties keep the upper row (the pivot is the first row of
// largest magnitude).  Rows are exchanged by selects on the pivot index; the
// pivot row of column k is kept in bits 4k..4k+3 of one 64-bit word (N <= 16).
// Operation order per element as a textbook LU: l = m_rk (1 / m_kk), then
// m_rc -= l m_kc for c = k+1..N-1; the diagonal keeps 1 / m_kk for the
// solve (multiplications in place of divisions, with a reciprocal within an
// ulp or two).
template <int N>
__device__ __forceinline__ bool lu_factor(double *M, unsigned long long &piv)
{
    static_assert(N <= 16, "packed pivots hold at most 16 rows");
    bool ok = true;
    piv = 0ull;
    static_for<0, N>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        int pk = k;
        double best = fabs(M[k * N + k]);
        static_for<k + 1, N>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            const double v = fabs(M[r * N + k]);
            if (v > best) {
                best = v;
                pk = r;
            }
        });
        piv |= (unsigned long long)pk << (4 * k);
        ok = ok && (best != 0.0);
        if constexpr (k + 1 < N) {
            if (pk != k) {
                static_for<0, N>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    const double mk = reg_value(M[k * N + c]);
                    double nk = mk;
                    static_for<k + 1, N>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        const double mr = reg_value(M[r * N + c]);
                        const bool sw = (pk == r);
                        nk = sw ? mr : nk;
                        M[r * N + c] = sw ? mk : mr;
                    });
                    M[k * N + c] = nk;
                });
            }
        }
        const double rp = rcp_d(M[k * N + k]);
        static_for<k + 1, N>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            const double l = M[r * N + k] * rp;
            M[r * N + k] = l;
            static_for<k + 1, N>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                M[r * N + c] -= l * M[k * N + c];
            });
        });
        M[k * N + k] = rp;
    });
    return ok;
}

template <int N>
__device__ __forceinline__ void lu_solve(const double *M, unsigned long long piv, double *b)
{
    static_for<0, N>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const int pk = (int)((piv >> (4 * k)) & 15ull);
        const double bk = reg_value(b[k]);
        double nk = bk;
        static_for<k + 1, N>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            const double br = reg_value(b[r]);
            const bool sw = (pk == r);
            nk = sw ? br : nk;
            b[r] = sw ? bk : br;
        });
        b[k] = nk;
    });
    static_for<1, N>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        static_for<0, r>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            b[r] -= M[r * N + c] * b[c];
        });
    });
    static_for<0, N>([&](auto ri) {
        constexpr int r = N - 1 - decltype(ri)::value;
        static_for<r + 1, N>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            b[r] -= M[r * N + c] * b[c];
        });
        b[r] *= M[r * N + r];
    });
}

// ---------------------------------------------------------------------------
// contract constants
// ---------------------------------------------------------------------------

namespace bdf {
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

enum Phase : int { FETCH = 0, NEWTON = 3, RESTART = 4, LUFAIL = 5, DONE = 6 };
}  // namespace bdf

template <int N>
struct NordLds;

template <int N>
__device__ __forceinline__ double wrms_norm(const double *v, const NordLds<N> &z);

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

__device__ __forceinline__ double factorial_d(int n)
{
    double f = 1.0;
#pragma unroll
    for (int i = 2; i <= 7; i++)
        if (i <= n) f *= i;
    return f;
}

// Per-lane arrays kept in LDS: element (j, i) of lane L at lds[(j*N + i)*64 + L],
// so a wave's 64 lanes touch 64 consecutive doubles and every static (j, i)
// is an immediate offset.  Rows 0..kQmax hold the Nordsieck array, row
// kQmax+1 the scaled correction of the previous step (order-raise estimate),
// row kQmax+2 the error weights.
template <int N>
struct NordLds {
    double *base;   // lds + lane
    __device__ __forceinline__ double &operator()(int j, int i) const { return base[(j * N + i) * 64]; }
};
constexpr int kLdsRows = kQmax + 3;

template <int N>
__device__ __forceinline__ double wrms_norm(const double *v, const NordLds<N> &z)
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < N; i++) {
        const double t = v[i] * z(kQmax + 2, i);
        s += t * t;
    }
    return sqrt(s * (1.0 / N));
}
constexpr int kEhatRow = kQmax + 1;
constexpr int kWeightRow = kQmax + 2;   // error weights 1/(rtol |y_n| + atol)

// Per-lane integrator state.  Every array is indexed statically.
template <int N>
struct LaneState {
    NordLds<N> z;               // Nordsieck array and previous scaled correction (LDS)
    double M[N * N];            // LU factors of I - gamma_M J
    unsigned long long piv;     // packed pivot rows
    double e[N], fy[N];
    double tau[kQmax + 2];      // past step sizes, tau[1] most recent
    double p, t, h, t_end, gamma, gamma_M, Cq, inv_l1, crate, del_old, dsm, ehat_h;
    int64_t cell;
    int phase, q, qwait, nst_M, it, nef, ncf;
    bool have_M, ehat_ok, force_M, last, jcur, need_J;
    int nst, nfe, nje, nni, netf, ncfn;
};

template <int N>
__device__ __forceinline__ void nord_predict(LaneState<N> &S)
{
#pragma unroll
    for (int k = 1; k <= kQmax; k++)
#pragma unroll
        for (int j = kQmax; j >= k; j--)
            if (j <= S.q)
#pragma unroll
                for (int i = 0; i < N; i++) S.z(j - 1, i) += S.z(j, i);
}

template <int N>
__device__ __forceinline__ void nord_restore(LaneState<N> &S)
{
#pragma unroll
    for (int k = kQmax; k >= 1; k--)
#pragma unroll
        for (int j = k; j <= kQmax; j++)
            if (j <= S.q && k <= S.q)
#pragma unroll
                for (int i = 0; i < N; i++) S.z(j - 1, i) -= S.z(j, i);
}

template <int N>
__device__ __forceinline__ void nord_rescale(LaneState<N> &S, double eta)
{
    double f = 1.0;
#pragma unroll
    for (int j = 1; j <= kQmax; j++) {
        f *= eta;
        if (j <= S.q)
#pragma unroll
            for (int i = 0; i < N; i++) S.z(j, i) *= f;
    }
}

// Step coefficients from the history: xi_i = (h + tau_1 + ... + tau_{i-1}) / h
// and its reciprocal rxi_i, l = coefficients of prod_{i=1..q} (1 + x / xi_i).
template <int N>
__device__ __forceinline__ void step_coeffs(const LaneState<N> &S, double *xi, double *rxi, double *l)
{
    const double invh = rcp_d(S.h);
    double s = S.h;
    xi[1] = 1.0;
    rxi[1] = 1.0;
#pragma unroll
    for (int i = 2; i <= kQmax + 1; i++) {
        s += S.tau[i - 1];
        xi[i] = s * invh;
        rxi[i] = S.h * rcp_d(s);
    }
    l[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= kQmax; j++) l[j] = 0.0;
#pragma unroll
    for (int i = 1; i <= kQmax; i++)
        if (i <= S.q)
#pragma unroll
            for (int j = i; j >= 1; j--) l[j] += l[j - 1] * rxi[i];
}

// xi_{q+1} = (h + tau_1 + ... + tau_q) / h, summed with the order as a guard
// on values (an element pick by order would become a dynamic register index).
template <int N>
__device__ __forceinline__ double xi_q1(const LaneState<N> &S)
{
    double s = S.h;
#pragma unroll
    for (int i = 1; i <= kQmax; i++)
        if (i <= S.q) s += S.tau[i];
    return s * rcp_d(S.h);
}

struct CellIO {
    double *T;
    const double *p;
    double *Y;
    int64_t ldY, n;              // n: cells in the arrays (stride of the counter rows)
    int32_t *status, *counters;
    const BdfParams *prm;
    int64_t nq;                  // work items of the queue
    const int32_t *idx;          // work item -> cell (NULL: identity)
};

// Work items of one launch: the index list or all cells, bounded by a
// device-side count when one is given.
__device__ __forceinline__ CellIO make_cell_io(double *T, const double *p, double *Y, int64_t ldY,
                                               int64_t n, int32_t *status, int32_t *counters,
                                               const BdfParams &prm)
{
    int64_t nq = prm.idx ? prm.n_idx : n;
    if (prm.n_dev && *prm.n_dev < nq) nq = *prm.n_dev;
    return CellIO{T, p, Y, ldY, n, status, counters, &prm, nq, prm.idx};
}

// Start pass of the one-thread-per-cell kernels.  Before the integration
// proper, one straight-line pass computes every work item's start -- f(y0)
// and the initial step h0, the same arithmetic the integration would do at
// its first step -- and files the item under a cost bucket from dt/h0 (a
// small initial step marks a stiff cell: many steps).  The integration then
// takes the items most costly bucket first, so that the longest cells start
// first and the last cells of the queue are short ones (longest processing
// time first), and cells of alike cost share a wave.  Scheduling only: each
// cell's result does not depend on the order.
constexpr int kCostBuckets = 64;
struct StartPass {
    double *f0;        // N rows of `stride`: f(y0) per work item
    double *h0;        // initial step per work item
    int32_t *info;     // right-hand sides used | status << 8 (4: f(y0) not finite)
    int32_t *key;      // cost bucket per work item
    int32_t *cnt;      // kCostBuckets counts, then running offsets
    int32_t *ord;      // work items, most costly bucket first
    int64_t stride;    // >= work items of the launch
};

template <int N>
__device__ __forceinline__ void finish_cell(LaneState<N> &S, const CellIO &io, int st)
{
    constexpr int K = N - 1;
    double y[N];
#pragma unroll
    for (int i = 0; i < N; i++) y[i] = S.z(0, i);
    if (st == 0 && !finite_vec<N>(y)) st = 4;
    const int64_t i = S.cell;
    if (st == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) io.Y[k * io.ldY + i] = y[k];
        io.T[i] = y[K];
    }
    if (io.status) io.status[i] = st;
    if (io.counters) {
        io.counters[0 * io.n + i] = S.nst;
        io.counters[1 * io.n + i] = S.nfe;
        io.counters[2 * io.n + i] = S.nje;
        io.counters[3 * io.n + i] = S.nni;
        io.counters[4 * io.n + i] = S.netf;
        io.counters[5 * io.n + i] = S.ncfn;
    }
    S.phase = bdf::FETCH;
}

// Predict, compute the step coefficients and decide whether M is refreshed.
template <int N>
__device__ __forceinline__ void begin_attempt(LaneState<N> &S, const CellIO &io)
{
    const double tnew = S.t + S.h;
    if (tnew == S.t) {
        finish_cell(S, io, 2);
        return;
    }
    nord_predict(S);
    double xi[kQmax + 2], rxi[kQmax + 2], l[kQmax + 1];
    step_coeffs(S, xi, rxi, l);
    S.inv_l1 = rcp_d(l[1]);
    S.gamma = S.h * S.inv_l1;
    S.Cq = rcp_d(1.0 + l[1] * xi_q1(S));
    S.jcur = false;
    S.need_J = !S.have_M || S.force_M || S.nst >= S.nst_M + bdf::kMsbp ||
               fabs(S.gamma / S.gamma_M - 1.0) > bdf::kDgmax;
    S.it = 0;   // the accumulated correction e starts at 0 (set after the first solve)
    S.del_old = 0.0;
    S.phase = bdf::NEWTON;
}

template <int N>
__device__ __forceinline__ void begin_step(LaneState<N> &S, const CellIO &io)
{
    if (S.nst >= io.prm->max_steps) {
        finish_cell(S, io, 1);
        return;
    }
    S.last = false;
    if (S.t + S.h >= S.t_end) {
        nord_rescale(S, (S.t_end - S.t) / S.h);
        S.h = S.t_end - S.t;
        S.last = true;
    }
#pragma unroll
    for (int i = 0; i < N; i++) S.z(kWeightRow, i) = rcp_d(io.prm->rtol * fabs(S.z(0, i)) + io.prm->atol);
    S.nef = 0;
    S.ncf = 0;
    S.force_M = false;
    begin_attempt(S, io);
}

template <int N>
__device__ __forceinline__ void begin_integration(LaneState<N> &S, const CellIO &io)
{
    // S.h set; S.e holds f(y0); z[0] holds y0
    S.q = 1;
#pragma unroll
    for (int i = 0; i < N; i++) S.z(1, i) = S.h * S.e[i];
    S.qwait = 2;
    S.have_M = false;
    S.ehat_ok = false;
    S.gamma_M = 0.0;
    S.crate = 1.0;
    S.ehat_h = 0.0;
    S.t = 0.0;
    begin_step(S, io);
}

template <int N>
__device__ __forceinline__ void conv_fail(LaneState<N> &S, const CellIO &io)
{
    nord_restore(S);
    if (!S.jcur) {
        S.force_M = true;
        begin_attempt(S, io);
        return;
    }
    S.ncfn++;
    if (++S.ncf >= bdf::kMaxNcf) {
        finish_cell(S, io, 3);
        return;
    }
    nord_rescale(S, bdf::kEtaCf);
    S.h *= bdf::kEtaCf;
    S.last = false;
    begin_attempt(S, io);
}

// Step size and order for the step after an accepted one (orders up to qmax).
template <int N>
__device__ __forceinline__ void select_next(LaneState<N> &S, int qmax)
{
    using namespace bdf;
    const int q = S.q;
    const double h_done = S.h;
    double xi[kQmax + 2], rxi[kQmax + 2], l[kQmax + 1];
    step_coeffs(S, xi, rxi, l);
    double prod_q = 1.0;
#pragma unroll
    for (int i = 1; i <= kQmax; i++)
        if (i <= q) prod_q *= xi[i];
    const double x1 = xi_q1(S);
    const double rgfac = factorial_d(q + 1) * rcp_d(prod_q * (S.inv_l1 + x1));
    double ehat_new[N];
#pragma unroll
    for (int i = 0; i < N; i++) ehat_new[i] = S.e[i] * rgfac;
    if (S.qwait > 0) S.qwait--;
    const double etamax = (S.nef > 0 || S.ncf > 0) ? 1.0 : (S.nst == 1 ? kEtaMaxFirst : kEtaMax);
    double eta = 1.0;
    int qnew = q;
    if (etamax > 1.0) {
        eta = rcp_d(root_k(kBiasQ * S.dsm, q + 1) + kAddon);
        if (S.qwait == 0) {
            double eta_m = 0.0, eta_p = 0.0;
            if (q > 1) {
                double prod = 1.0, l1 = 0.0, zq[N];
#pragma unroll
                for (int i = 0; i < N; i++) zq[i] = 0.0;
#pragma unroll
                for (int j = 2; j <= kQmax; j++)
                    if (j == q)
#pragma unroll
                        for (int i = 0; i < N; i++) zq[i] = S.z(j, i);
#pragma unroll
                for (int i = 1; i < kQmax; i++)
                    if (i <= q - 1) {
                        prod *= xi[i];
                        l1 += rxi[i];
                    }
                const double Em = wrms_norm<N>(zq, S.z) * prod * rcp_d(l1);
                eta_m = rcp_d(root_k(kBiasQm1 * Em, q) + kAddon);
            }
            if (q < qmax && S.ehat_ok) {
                const double rr = pow_k(h_done * rcp_d(S.ehat_h), q + 1);
                double dv[N];
#pragma unroll
                for (int i = 0; i < N; i++) dv[i] = ehat_new[i] - S.z(kEhatRow, i) * rr;
                double prod = 1.0, l1 = 0.0;
#pragma unroll
                for (int i = 1; i <= kQmax; i++)
                    if (i <= q + 1) {
                        prod *= xi[i];
                        l1 += rxi[i];
                    }
                const double Ep = wrms_norm<N>(dv, S.z) * prod * rcp_d(factorial_d(q + 2) * l1);
                eta_p = rcp_d(root_k(kBiasQp1 * Ep, q + 2) + kAddon);
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
                for (int i = 0; i < N; i++) zq[i] = S.z(j, i);
#pragma unroll
        for (int j = 1; j < kQmax; j++)
            if (j < q)
#pragma unroll
                for (int i = 0; i < N; i++) S.z(j, i) -= d[j] * zq[i];
        S.q = qnew;
        S.qwait = qnew + 1;
        S.ehat_ok = false;
    } else if (qnew == q + 1) {
        // add e * (x / xi_{q+1}) * Lambda_q(x)
        const double inv = rcp_d(x1);
#pragma unroll
        for (int j = 2; j <= kQmax; j++)
            if (j == q + 1)
#pragma unroll
                for (int i = 0; i < N; i++) S.z(j, i) = 0.0;
#pragma unroll
        for (int j = 1; j <= kQmax; j++)
            if (j <= q + 1)
#pragma unroll
                for (int i = 0; i < N; i++) S.z(j, i) += S.e[i] * l[j - 1] * inv;
        S.q = qnew;
        S.qwait = qnew + 1;
        S.ehat_ok = false;
    } else {
#pragma unroll
        for (int i = 0; i < N; i++) S.z(kEhatRow, i) = ehat_new[i];
        S.ehat_h = h_done;
        S.ehat_ok = true;
    }
#pragma unroll
    for (int i = kQmax + 1; i >= 2; i--) S.tau[i] = S.tau[i - 1];
    S.tau[1] = h_done;
    if (eta != 1.0) {
        nord_rescale(S, eta);
        S.h *= eta;
    }
}

// Error test after a converged Newton iteration; accept or retry.
template <int N>
__device__ __forceinline__ void error_test(LaneState<N> &S, const CellIO &io)
{
    using namespace bdf;
    S.dsm = S.Cq * wrms_norm<N>(S.e, S.z);
    if (S.dsm > 1.0) {
        nord_restore(S);
        S.netf++;
        if (++S.nef >= kMaxNef) {
            finish_cell(S, io, 2);
            return;
        }
        S.last = false;
        if (S.nef >= kNefRestart) {
            S.h *= kEtaMinEf;
            S.q = 1;
            S.phase = RESTART;   // needs f(z0)
            return;
        }
        double eta = rcp_d(root_k(kBiasQ * S.dsm, S.q + 1) + kAddon);
        eta = fmin(fmax(eta, kEtaMinEf), kEtaMaxEf);
        if (S.nef >= 2) eta = fmin(eta, kEtaNef2);
        nord_rescale(S, eta);
        S.h *= eta;
        begin_attempt(S, io);
        return;
    }
    {
        double xi[kQmax + 2], rxi[kQmax + 2], l[kQmax + 1];
        step_coeffs(S, xi, rxi, l);
#pragma unroll
        for (int j = 0; j <= kQmax; j++)
            if (j <= S.q)
#pragma unroll
                for (int i = 0; i < N; i++) S.z(j, i) += l[j] * S.e[i];
    }
    S.t = S.last ? S.t_end : S.t + S.h;
    S.nst++;
    if (S.t >= S.t_end) {
        finish_cell(S, io, 0);
        return;
    }
    select_next(S, io.prm->qmax);
    begin_step(S, io);
}

// The integration's start for one cell: f0 = f(y0) and the initial step
// (the step whose second-derivative estimate gives a local error of 0.5,
// refined at most kH0Iters times, half of the estimate, bounded by a 10 %
// change of any component, at most t_end).  st = 4 when f(y0) is not finite.
template <class Mech>
__device__ __forceinline__ void initial_step(const Mech &mech, double p, const double *y0, double rtol,
                                             double atol, double t_end, double *f0, double &h, int &nfe,
                                             int &st)
{
    constexpr int N = Mech::K + 1;
    mech.rhs(p, y0, f0);
    nfe = 1;
    st = 0;
    h = t_end;
    if (!finite_vec<N>(f0)) {
        st = 4;
        return;
    }
    double w[N];
#pragma unroll
    for (int i = 0; i < N; i++) w[i] = 1.0 / (rtol * fabs(y0[i]) + atol);
    if (wrms_norm<N>(f0, w) == 0.0) return;
    double hub = t_end;
#pragma unroll
    for (int i = 0; i < N; i++) {
        const double lim = 0.1 * fabs(y0[i]) + 1.0 / w[i];
        if (fabs(f0[i]) * hub > lim) hub = lim / fabs(f0[i]);
    }
    double hg = hub;
    for (int it = 0; it < bdf::kH0Iters; it++) {
        double yv[N], fy[N];
#pragma unroll
        for (int i = 0; i < N; i++) yv[i] = y0[i] + hg * f0[i];
        mech.rhs(p, yv, fy);
        nfe++;
        if (!finite_vec<N>(fy)) {
            hg *= 0.1;
            continue;
        }
        double dv[N];
#pragma unroll
        for (int i = 0; i < N; i++) dv[i] = (fy[i] - f0[i]) / hg;
        const double ydd = wrms_norm<N>(dv, w);
        double hnew = ydd > 0.0 ? sqrt(2.0 / ydd) : hub;
        if (hnew > hub) hnew = hub;
        const double ratio = hnew / hg;
        hg = hnew;
        if (ratio >= 0.5 && ratio <= 2.0) break;
    }
    h = 0.5 * hg;
    if (h > t_end) h = t_end;
}

// Cost bucket of a cell from its start: 3 log2(dt / h0), clamped (0 for a
// cell that fails at the start).
__device__ __forceinline__ int cost_bucket(double h, double t_end, int st)
{
    if (st != 0 || !(h > 0.0)) return 0;
    const double b = 3.0 * log2(t_end / h);
    return b < 1.0 ? 0 : (b >= kCostBuckets - 1 ? kCostBuckets - 1 : (int)b);
}

// Start pass: one thread per work item; bucket counts per block in LDS, then
// one atomic per non-empty bucket.
// Mech::kStartWaves waves per SIMD: the pass runs a few rounds of waves
// through long exp chains, so a second resident wave hides their latency
// where the mechanism's code fits 256 registers without spills.
template <class Mech>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Mech::kStartWaves))) bdf_start_kernel(Mech mech, double *__restrict__ T,
                                                        const double *__restrict__ p,
                                                        double *__restrict__ Y, int64_t ldY, int64_t n,
                                                        double dt, BdfParams prm, StartPass sp)
{
    constexpr int N = Mech::K + 1;
    __shared__ int hist[kCostBuckets];
    if (threadIdx.x < kCostBuckets) hist[threadIdx.x] = 0;
    __syncthreads();
    const CellIO io = make_cell_io(T, p, Y, ldY, n, nullptr, nullptr, prm);
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it < io.nq) {
        const int64_t cc = io.idx ? (int64_t)io.idx[it] : it;
        int key = 0;
        if (cc >= 0 && cc < io.n) {   // an index outside the arrays is skipped by the integration
            double y0[N], f0[N], h;
            int nfe, st;
#pragma unroll
            for (int k = 0; k < N - 1; k++) y0[k] = io.Y[k * io.ldY + cc];
            y0[N - 1] = io.T[cc];
            initial_step(mech, io.p[cc], y0, prm.rtol, prm.atol, dt, f0, h, nfe, st);
#pragma unroll
            for (int i = 0; i < N; i++) sp.f0[i * sp.stride + it] = f0[i];
            sp.h0[it] = h;
            sp.info[it] = nfe | (st << 8);
            key = cost_bucket(h, dt, st);
        }
        sp.key[it] = key;
        atomicAdd(&hist[key], 1);
    }
    __syncthreads();
    if (threadIdx.x < kCostBuckets && hist[threadIdx.x] != 0) atomicAdd(&sp.cnt[threadIdx.x], hist[threadIdx.x]);
}

// Clears the work-queue counter and the bucket counts (a kernel, not a
// memset, so that a captured graph replays it like any other node).
__global__ void start_reset_kernel(unsigned long long *queue, int32_t *cnt);
// Bucket counts -> offsets, most costly bucket first.
__global__ void start_scan_kernel(int32_t *cnt);
// Files every work item at the next offset of its bucket.
__global__ void __launch_bounds__(256) start_scatter_kernel(const int32_t *key, int32_t *cnt, int32_t *ord,
                                                            int64_t n, BdfParams prm);

template <class Mech>
__device__ void run_lanes(const Mech &mech, const CellIO &io, double t_end,
                          unsigned long long *queue, double *lds, const StartPass &sp)
{
    constexpr int K = Mech::K;
    constexpr int N = K + 1;
    using namespace bdf;
    LaneState<N> S;
    S.z.base = lds + (threadIdx.x & 63);
    S.phase = FETCH;
    S.t_end = t_end;
    S.need_J = false;
    const int lane = threadIdx.x & 63;
    for (;;) {
        // ---- refill idle lanes from the queue (one atomic per wave) ----
        {
            const bool want = (S.phase == FETCH);
            const unsigned long long mask = __ballot(want);
            if (mask) {
                const int leader = __ffsll((long long)mask) - 1;
                const int cnt = __popcll(mask);
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(queue, (unsigned long long)cnt);
                base = __shfl(base, leader);
                if (want) {
                    const unsigned long long rank = __popcll(mask & ((1ull << lane) - 1ull));
                    const unsigned long long c = base + rank;
                    const int64_t item = c < (unsigned long long)io.nq ? (int64_t)sp.ord[c] : -1;
                    const int64_t cc = item >= 0 ? (io.idx ? (int64_t)io.idx[item] : item) : -1;
                    if (c < (unsigned long long)io.nq && (cc < 0 || cc >= io.n)) {
                        // an index outside the arrays is skipped: this lane fetches again
                    } else if (c < (unsigned long long)io.nq) {
                        S.cell = cc;
                        const int64_t i = S.cell;
#pragma unroll
                        for (int k = 0; k < K; k++) S.z(0, k) = io.Y[k * io.ldY + i];
                        S.z(0, K) = io.T[i];
                        S.p = io.p[i];
                        S.nst = S.nfe = S.nje = S.nni = S.netf = S.ncfn = 0;
#pragma unroll
                        for (int j = 0; j < kQmax + 2; j++) S.tau[j] = 0.0;
                        S.need_J = false;
                        // the start from the start pass: e = f(y0), h = h0
#pragma unroll
                        for (int k = 0; k < N; k++) S.e[k] = sp.f0[k * sp.stride + item];
                        S.h = sp.h0[item];
                        const int inf = sp.info[item];
                        S.nfe = inf & 0xff;
                        if (inf >> 8)
                            finish_cell(S, io, inf >> 8);
                        else
                            begin_integration(S, io);
                    } else {
                        S.phase = DONE;
                    }
                }
            }
        }
        if (__ballot(S.phase != DONE) == 0ull) break;

        // ---- Jacobian + LU (the single call site), batched across the wave:
        // a lane that needs a new Newton matrix waits until jac_batch lanes
        // wait too, or until no lane can progress without one.  This moves
        // work in time only; every lane takes the same decisions. ----
        const bool waitJ = S.need_J && S.phase == NEWTON;
        const unsigned long long mJ = __ballot(waitJ);
        bool runJ = false;
        if (mJ) {
            const bool progress = ((S.phase == NEWTON || S.phase == RESTART) && !waitJ) || S.phase == LUFAIL;
            runJ = __popcll(mJ) >= io.prm->jac_batch || __ballot(progress) == 0ull;
        }
        if (runJ && waitJ) {
            double yj[N];
#pragma unroll
            for (int i = 0; i < N; i++) yj[i] = S.z(0, i);
            mech.jac(S.p, yj, S.M);
#pragma unroll
            for (int r = 0; r < N; r++)
#pragma unroll
                for (int c = 0; c < N; c++) S.M[r * N + c] = (r == c ? 1.0 : 0.0) - S.gamma * S.M[r * N + c];
            S.nje++;
            const bool ok = lu_factor<N>(S.M, S.piv);
            S.gamma_M = S.gamma;
            S.nst_M = S.nst;
            S.crate = 1.0;
            S.have_M = ok;
            S.jcur = true;
            S.force_M = false;
            S.need_J = false;
            if (!ok) S.phase = LUFAIL;
        }

        const bool waiting = S.need_J && S.phase == NEWTON;

        // ---- right-hand side (the single call site) ----
        if ((S.phase == NEWTON || S.phase == RESTART) && !waiting) {
            double yv[N];
            // the prediction itself (first Newton iteration, RESTART), or
            // the prediction plus the accumulated correction e
            const bool use_e = S.phase == NEWTON && S.it > 0;
#pragma unroll
            for (int i = 0; i < N; i++) yv[i] = use_e ? S.z(0, i) + S.e[i] : S.z(0, i);
            mech.rhs(S.p, yv, S.fy);
            S.nfe++;
        }

        // ---- bookkeeping ----
        if (S.phase == NEWTON && !waiting) {
            bool conv = false, fail = false;
            if (!finite_vec<N>(S.fy)) {
                fail = true;
            } else {
                double d[N];
                const double inv_l1 = S.inv_l1;
                const bool first = (S.it == 0);
#pragma unroll
                for (int i = 0; i < N; i++)
                    d[i] = -((first ? 0.0 : S.e[i]) - S.gamma * S.fy[i] + S.z(1, i) * inv_l1);
                lu_solve<N>(S.M, S.piv, d);
                if (S.gamma != S.gamma_M) {
                    const double s = 2.0 * rcp_d(1.0 + S.gamma * rcp_d(S.gamma_M));
#pragma unroll
                    for (int i = 0; i < N; i++) d[i] *= s;
                }
                const double dl = wrms_norm<N>(d, S.z);
#pragma unroll
                for (int i = 0; i < N; i++) S.e[i] = first ? d[i] : S.e[i] + d[i];
                S.nni++;
                if (S.it > 0) S.crate = fmax(kCrdown * S.crate, dl / S.del_old);
                const double dcon = dl * fmin(S.crate, 1.0) * S.Cq / kNlscoef;
                if (dcon <= 1.0) {
                    conv = true;
                } else if ((S.it > 0 && dl > kRdiv * S.del_old) || S.it + 1 >= kMaxCor) {
                    fail = true;
                } else {
                    S.del_old = dl;
                    S.it++;
                }
            }
            if (conv)
                error_test(S, io);
            else if (fail)
                conv_fail(S, io);
        } else if (S.phase == LUFAIL) {
            conv_fail(S, io);
        } else if (S.phase == RESTART) {
            if (!finite_vec<N>(S.fy)) {
                finish_cell(S, io, 4);
            } else {
#pragma unroll
                for (int i = 0; i < N; i++) S.z(1, i) = S.h * S.fy[i];
#pragma unroll
                for (int j = 0; j < kQmax + 2; j++) S.tau[j] = 0.0;
                S.qwait = 2;
                S.ehat_ok = false;
                begin_attempt(S, io);
            }
        }
    }
}

template <class Mech>
__global__ void __launch_bounds__(64) bdf_queue_kernel(Mech mech, double *__restrict__ T,
                                                       const double *__restrict__ p,
                                                       double *__restrict__ Y, int64_t ldY,
                                                       int64_t n, double dt, BdfParams prm,
                                                       int32_t *__restrict__ status,
                                                       int32_t *__restrict__ counters,
                                                       unsigned long long *__restrict__ queue,
                                                       StartPass sp)
{
    __shared__ double nord[kLdsRows * (Mech::K + 1) * 64];
    const CellIO io = make_cell_io(T, p, Y, ldY, n, status, counters, prm);
    run_lanes(mech, io, dt, queue, nord, sp);
}

template <class Mech>
__global__ void __launch_bounds__(256) rhs_eval_kernel(Mech mech, const double *__restrict__ T,
                                                       const double *__restrict__ p,
                                                       const double *__restrict__ Y, int64_t ldY,
                                                       int64_t n, double *__restrict__ F, int64_t ldF)
{
    constexpr int K = Mech::K;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double y[K + 1], f[K + 1];
#pragma unroll
    for (int k = 0; k < K; k++) y[k] = Y[k * ldY + i];
    y[K] = T[i];
    mech.rhs(p[i], y, f);
#pragma unroll
    for (int k = 0; k <= K; k++) F[k * ldF + i] = f[k];
}

template <class Mech>
__global__ void __launch_bounds__(64) jac_eval_kernel(Mech mech, const double *__restrict__ T,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ Y, int64_t ldY,
                                                      int64_t n, double *__restrict__ J, int64_t ldJ)
{
    constexpr int K = Mech::K;
    constexpr int N = K + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double y[N], jac[N * N];
#pragma unroll
    for (int k = 0; k < K; k++) y[k] = Y[k * ldY + i];
    y[K] = T[i];
    mech.jac(p[i], y, jac);
#pragma unroll
    for (int k = 0; k < N * N; k++) J[k * ldJ + i] = jac[k];
}

__global__ void reset_queue_kernel(unsigned long long *queue);

// Grid of the queue kernel: enough one-wave blocks to fill every CU at the
// kernel's occupancy, never more lanes than cells.
int queue_grid(const void *kernel, int64_t n, int waves_per_simd);

// Bytes of the start-pass workspace for `items` work items of an N-component
// cell, and its layout in such a buffer (256-byte aligned pieces).
inline size_t start_pass_bytes(int N, int64_t items)
{
    auto a = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t m = (size_t)(items > 0 ? items : 1);
    return a(N * m * 8) + a(m * 8) + 3 * a(m * 4) + a(kCostBuckets * 4);
}
inline StartPass start_pass_carve(void *base, int N, int64_t items)
{
    auto a = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t m = (size_t)(items > 0 ? items : 1);
    char *c = (char *)base;
    StartPass sp;
    sp.f0 = (double *)c;
    c += a(N * m * 8);
    sp.h0 = (double *)c;
    c += a(m * 8);
    sp.info = (int32_t *)c;
    c += a(m * 4);
    sp.key = (int32_t *)c;
    c += a(m * 4);
    sp.ord = (int32_t *)c;
    c += a(m * 4);
    sp.cnt = (int32_t *)c;
    sp.stride = (int64_t)m;
    return sp;
}

// The one-thread-per-cell integration of at most `items` work items: reset,
// start pass, bucket offsets, filing, then the integration in that order.
template <class Mech>
hipError_t launch_thread_integrate(const Mech &mech, double *T, const double *p, double *Y, int64_t ldY,
                                   int64_t n, double dt, const BdfParams &prm, int32_t *status,
                                   int32_t *counters, unsigned long long *queue, const StartPass &sp,
                                   int64_t items, hipStream_t s)
{
    const unsigned gb = (unsigned)((items + 255) / 256);
    hipLaunchKernelGGL(start_reset_kernel, dim3(1), dim3(64), 0, s, queue, sp.cnt);
    hipLaunchKernelGGL(bdf_start_kernel<Mech>, dim3(gb), dim3(256), 0, s, mech, T, p, Y, ldY, n, dt, prm, sp);
    hipLaunchKernelGGL(start_scan_kernel, dim3(1), dim3(64), 0, s, sp.cnt);
    hipLaunchKernelGGL(start_scatter_kernel, dim3(gb), dim3(256), 0, s, sp.key, sp.cnt, sp.ord, n, prm);
    const int blocks = queue_grid((const void *)bdf_queue_kernel<Mech>, items, prm.waves_per_simd);
    hipLaunchKernelGGL(bdf_queue_kernel<Mech>, dim3(blocks), dim3(64), 0, s, mech, T, p, Y, ldY, n, dt, prm,
                       status, counters, queue, sp);
    return hipGetLastError();
}

// Launchers of a mechanism-specialised functor (defined by generated code).
typedef hipError_t (*gen_integrate_fn)(double *T, const double *p, double *Y, int64_t ldY,
                                       int64_t n, double dt, const BdfParams &prm, int32_t *status,
                                       int32_t *counters, unsigned long long *queue, const StartPass &sp,
                                       int64_t items, hipStream_t s);
typedef hipError_t (*gen_eval_fn)(const double *T, const double *p, const double *Y, int64_t ldY,
                                  int64_t n, double *out, int64_t ld, hipStream_t s);

struct GenEntry {
    unsigned long long hash;
    int K;
    const char *tag;
    gen_integrate_fn integrate;
    gen_eval_fn rhs;
    gen_eval_fn jac;
};

const GenEntry *gen_registry(int *count);

#define CHEM_DECLARE_GEN_LAUNCHERS(TAG)                                                          \
    hipError_t gen_integrate_##TAG(double *, const double *, double *, int64_t, int64_t, double,  \
                                   const BdfParams &, int32_t *, int32_t *, unsigned long long *, \
                                   const StartPass &, int64_t, hipStream_t);                      \
    hipError_t gen_rhs_##TAG(const double *, const double *, const double *, int64_t, int64_t,    \
                             double *, int64_t, hipStream_t);                                     \
    hipError_t gen_jac_##TAG(const double *, const double *, const double *, int64_t, int64_t,    \
                             double *, int64_t, hipStream_t);

#define CHEM_DEFINE_GEN_LAUNCHERS(MECH, TAG)                                                      \
    hipError_t gen_integrate_##TAG(double *T, const double *p, double *Y, int64_t ldY, int64_t n, \
                                   double dt, const BdfParams &prm, int32_t *status,              \
                                   int32_t *counters, unsigned long long *queue,                  \
                                   const StartPass &sp, int64_t items, hipStream_t s)             \
    {                                                                                             \
        return launch_thread_integrate(MECH{}, T, p, Y, ldY, n, dt, prm, status, counters, queue, \
                                       sp, items, s);                                             \
    }                                                                                             \
    hipError_t gen_rhs_##TAG(const double *T, const double *p, const double *Y, int64_t ldY,      \
                             int64_t n, double *F, int64_t ldF, hipStream_t s)                    \
    {                                                                                             \
        hipLaunchKernelGGL(rhs_eval_kernel<MECH>, dim3((unsigned)((n + 255) / 256)), dim3(256),   \
                           0, s, MECH{}, T, p, Y, ldY, n, F, ldF);                                \
        return hipGetLastError();                                                                 \
    }                                                                                             \
    hipError_t gen_jac_##TAG(const double *T, const double *p, const double *Y, int64_t ldY,      \
                             int64_t n, double *J, int64_t ldJ, hipStream_t s)                    \
    {                                                                                             \
        hipLaunchKernelGGL(jac_eval_kernel<MECH>, dim3((unsigned)((n + 63) / 64)), dim3(64), 0,  \
                           s, MECH{}, T, p, Y, ldY, n, J, ldJ);                                   \
        return hipGetLastError();                                                                 \
    }

}  // namespace chem

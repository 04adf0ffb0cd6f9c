// Lane-group BDF integrators on gfx950: one 64-lane wave per cell (larger
// mechanisms), or one 16-lane tile per cell with four cells per wave (N <= 16).
//
// A group of G lanes owns one cell at a time and takes the next from a work
// queue as soon as that cell is done.  Lane i owns component i of every state
// vector (Nordsieck column, correction, weights); the Newton matrix and its
// LU factors live in LDS (lane i: row i); lanes cooperate on the right-hand
// side (lane k: thermo of species k; lane j: reactions j, j+G, ...) through
// LDS.  Sums over reactions are gathered by the owning species lane in a
// fixed order, so results do not depend on timing.  Control flow is uniform
// within a group: every decision of the integrator contract (the same as the
// one-thread-per-cell driver and the CPU oracle) is taken once per cell, so
// cells of very different stiffness do not hold each other back; the groups
// of one wave diverge like the lanes of any SIMT program.
//
// NP is the padded row count (a compile-time bound on N = K+1 <= 64).  LT is
// the type of the Jacobian, the Newton matrix, its LU factors and the
// triangular solves: double (plain FP64) or float (mixed precision: those in
// FP32; residuals, state, norms, error control and the equilibrium constants
// in FP64, so that the Newton iteration restores the accuracy).

#include "bdf_driver.h"
#include "bdf_wave.h"

// Built twice: as is, for mechanisms whose reactions are all elementary, and
// with CHEM_WAVE_PDEP = 1 (bdf_wave_pdep.hip) for mechanisms with third-body
// or fall-off reactions.  The pressure-dependent terms take registers that
// would halve the occupancy of the elementary kernels.
#ifndef CHEM_WAVE_PDEP
#define CHEM_WAVE_PDEP 0
#endif

namespace chem {
namespace {

constexpr bool kPD = CHEM_WAVE_PDEP != 0;

// Lanes that own one cell: Grp<64> is a whole wave (one cell per wave),
// Grp<16> one DPP row of 16 lanes (four cells per wave, the tile schedule).
// Within a group every decision is uniform; groups of one wave follow their
// own cells and diverge freely.  Every primitive below needs all lanes of
// the calling group active, and touches no lane outside it.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL>((int)(b & 0xffffffffll));
    const int hi = dpp_i32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double bpermute_f64(double v, int src_lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 16 lanes of each DPP row, the same value in every lane of the
// row: pairwise within quads (xor 1, xor 2), then the mirrored halves of 8
// and of 16 lanes (each a commutative pair, so all lanes of a row agree).
__device__ __forceinline__ double row_sum(double v)
{
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    return v;
}

__device__ __forceinline__ double row_max(double v)
{
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    return v;
}

// lane S of each row, to every lane of the row (row_newbcast)
template <int S>
__device__ __forceinline__ double row_bcast(double v) { return dpp_f64<0x150 + S>(v); }
template <int S>
__device__ __forceinline__ float row_bcast(float v) { return __int_as_float(dpp_i32<0x150 + S>(__float_as_int(v))); }

template <int G>
struct Grp;

template <>
struct Grp<64> {
    static constexpr int kCells = 1;
    __device__ static int lane() { return threadIdx.x & 63; }
    __device__ static int slot() { return 0; }
    // the four row sums added in a fixed order
    __device__ static double sum(double v)
    {
        v = row_sum(v);
        return ((readlane_f64(v, 15) + readlane_f64(v, 31)) + readlane_f64(v, 47)) + readlane_f64(v, 63);
    }
    __device__ static double max(double v)
    {
        v = row_max(v);
        return fmax(fmax(readlane_f64(v, 15), readlane_f64(v, 31)), fmax(readlane_f64(v, 47), readlane_f64(v, 63)));
    }
    // value of lane src (the same src in every lane of the wave)
    __device__ static double at(double v, int src) { return readlane_f64(v, src); }
    __device__ static float at(float v, int src) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src)); }
    __device__ static int at(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
    // value of lane k, k a constant after unrolling
    template <typename V>
    __device__ static V at_k(V v, int k) { return at(v, k); }
    // value of lane src of the group, src chosen per lane
    __device__ static double gather(double v, int src) { return __shfl(v, src); }
    __device__ static unsigned long long ballot(bool b) { return __ballot(b); }
    __device__ static unsigned long long first(unsigned long long v) { return __shfl(v, 0); }
    __device__ static void sync() { __syncthreads(); }
};

template <>
struct Grp<16> {
    static constexpr int kCells = 4;
    __device__ static int lane() { return threadIdx.x & 15; }
    __device__ static int slot() { return (threadIdx.x >> 4) & 3; }
    __device__ static double sum(double v) { return row_sum(v); }
    __device__ static double max(double v) { return row_max(v); }
    __device__ static double at(double v, int src) { return bpermute_f64(v, (threadIdx.x & 48) + src); }
    __device__ static int at(int v, int src) { return __builtin_amdgcn_ds_bpermute(((threadIdx.x & 48) + src) << 2, v); }
    // k must fold to a constant (fully unrolled loops): one DPP broadcast
    template <typename V>
    __device__ static V at_k(V v, int k)
    {
        switch (k) {
        case 0: return row_bcast<0>(v);
        case 1: return row_bcast<1>(v);
        case 2: return row_bcast<2>(v);
        case 3: return row_bcast<3>(v);
        case 4: return row_bcast<4>(v);
        case 5: return row_bcast<5>(v);
        case 6: return row_bcast<6>(v);
        case 7: return row_bcast<7>(v);
        case 8: return row_bcast<8>(v);
        case 9: return row_bcast<9>(v);
        case 10: return row_bcast<10>(v);
        case 11: return row_bcast<11>(v);
        case 12: return row_bcast<12>(v);
        case 13: return row_bcast<13>(v);
        case 14: return row_bcast<14>(v);
        default: return row_bcast<15>(v);
        }
    }
    __device__ static double gather(double v, int src) { return bpermute_f64(v, (threadIdx.x & 48) + src); }
    __device__ static unsigned long long ballot(bool b) { return (__ballot(b) >> (threadIdx.x & 48)) & 0xFFFFull; }
    __device__ static unsigned long long first(unsigned long long v)
    {
        const int lo = dpp_i32<0x150>((int)(v & 0xffffffffull)), hi = dpp_i32<0x150>((int)(v >> 32));
        return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    }
    // LDS written by some lanes of the group, then read by others: the DS
    // instructions of one wave execute in order, so ordering them in the
    // instruction stream (and waiting for completion) is enough
    __device__ static void sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }
};

// Lowest candidate lane of the group holding the largest |v| (-1 if no
// candidate has a comparable value).
template <int G>
__device__ __forceinline__ int group_argmax(double v, bool cand)
{
    const double a = cand ? fabs(v) : -1.0;
    const double best = Grp<G>::max(a);
    const unsigned long long hit = Grp<G>::ballot(cand && a == best);
    return hit ? (int)__ffsll((long long)hit) - 1 : -1;
}

template <int NP, typename LT, int G>
struct WaveLds {
    double C[G + 1], g[G + 1], h[G + 1];
    double invW[G + 1];   // 1 / W_k, 0 for the sentinel slot (set once)
    LT row[NP][NP + 2];   // Jacobian rows, then the LU factors of I - gamma J;
                          // column NP+1 collects sentinel slots
    LT lcol[NP];          // multipliers of the current elimination step
};

// Species data of this lane: its NASA block stays in the (cached) mechanism
// table and is read when the thermo is evaluated.
struct SpeciesLane {
    const double *blk;   // Tmid, low range, high range
    double W, invW;
};

__device__ __forceinline__ void lane_thermo(const SpeciesLane &s, bool two_range, double T,
                                            double invT, double lnT, double &cp, double &h,
                                            double &g, double &dcp)
{
    double a[kRangeLen];
    const bool low = !two_range || T < s.blk[0];
    const double *src = s.blk + 1 + (low ? 0 : kRangeLen);
#pragma unroll
    for (int j = 0; j < kRangeLen; j++) a[j] = src[j];
    cp = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
    h = a[0] + T * (a[7] + T * (a[8] + T * (a[9] + T * a[10]))) + a[5] * invT;
    g = h - (a[0] * lnT + T * (a[1] + T * (a[11] + T * (a[12] + T * a[13]))) + a[6]);
    dcp = a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * 4.0 * a[4]));
}

// f(y): each lane passes its component yi and receives fi.
template <int NP, typename LT, int G>
__device__ __forceinline__ double wave_rhs(const DevMechView &m, const WaveTables &wt, WaveLds<NP, LT, G> &L,
                           const SpeciesLane &sp, int K, double p, double yi, double *qbuf)
{
    using Gp = Grp<G>;
    const int lane = Gp::lane();
    const double T = Gp::at(yi, K);
    const double invT = 1.0 / T;
    const double lnT = log(T);
    double cpk = 0.0, hk = 0.0, gk = 0.0, dcpk = 0.0;
    if (lane < K) lane_thermo(sp, m.two_range, T, invT, lnT, cpk, hk, gk, dcpk);
    const double sumYW = Gp::sum(lane < K ? yi * sp.invW : 0.0);
    const double rho = p / (kRu * T * sumYW);
    const double cpm = kRu * Gp::sum(lane < K ? yi * cpk * sp.invW : 0.0);
    if (lane < K) {
        L.C[lane] = rho * yi * sp.invW;
        L.g[lane] = gk;
    } else if (lane == K) {
        L.C[K] = 1.0;
        L.g[K] = 0.0;
    }
    double ctot = 0.0;
    if constexpr (kPD) ctot = Gp::sum(lane < K ? rho * yi * sp.invW : 0.0);
    Gp::sync();
    const double ln_c0 = log(kPstd / kRu) - lnT;
    for (int r = lane; r < m.R; r += G) {
        const DevRxn x = m.rxn[r];
        const double lnkf = x.lnA + x.b * lnT - x.Ea_R * invT;
        const double dg = L.g[x.p0] + L.g[x.p1] - L.g[x.r0] - L.g[x.r1];
        const double lnkr = lnkf + dg - x.dnu * ln_c0;
        const double fwd = exp(lnkf) * L.C[x.r0] * L.C[x.r1];
        double q = (x.kind & kRxnIrrev) ? fwd : fwd - exp(lnkr) * L.C[x.p0] * L.C[x.p1];
        if constexpr (kPD) {
            const int kind = x.kind & 7;
            if (kind != kRxnElem) {
                const double M = third_body(x, m.aux, ctot, [&](int l) { return L.C[l]; });
                q *= pdep_rate<false>(kind, m.aux + x.aux, M, T, lnT, invT, lnkf, 0.0).mult;
            }
        }
        qbuf[r] = q;
    }
    Gp::sync();
    double wk = 0.0;
    if (lane < K) {
        const int b = wt.inc_off[lane], e = wt.inc_off[lane + 1];
#pragma unroll 4
        for (int j = b; j < e; j++) {
            const int2 ent = wt.inc[j];
            wk += (double)ent.y * qbuf[ent.x];
        }
    }
    const double heat = Gp::sum(lane < K ? hk * wk : 0.0);
    Gp::sync();
    if (lane < K) return sp.W * wk / rho;
    if (lane == K) return -(kRu * T) * heat / (rho * cpm);
    return 0.0;
}

// Row `lane` of M = I - gamma J at the state yi.
template <int NP, typename LT, int G>
__device__ __forceinline__ void wave_newton_matrix(const DevMechView &m, const WaveTables &wt, WaveLds<NP, LT, G> &L,
                                   const SpeciesLane &sp, int K, double p, double yi, double gamma,
                                   double *qbuf)
{
    using Gp = Grp<G>;
    const int lane = Gp::lane();
    const int N = K + 1;
    const double T = Gp::at(yi, K);
    const double invT = 1.0 / T;
    const double lnT = log(T);
    double cpk = 0.0, hk = 0.0, gk = 0.0, dcpk = 0.0;
    if (lane < K) lane_thermo(sp, m.two_range, T, invT, lnT, cpk, hk, gk, dcpk);
    const double sumYW = Gp::sum(lane < K ? yi * sp.invW : 0.0);
    const double wbar = 1.0 / sumYW;
    const double rho = p * wbar / (kRu * T);
    const double cpm = kRu * Gp::sum(lane < K ? yi * cpk * sp.invW : 0.0);
    const double dcpm = kRu * Gp::sum(lane < K ? yi * dcpk * sp.invW : 0.0);
    if (lane < K) {
        L.C[lane] = rho * yi * sp.invW;
        L.g[lane] = gk;
        L.h[lane] = hk;
    } else if (lane == K) {
        L.C[K] = 1.0;
        L.g[K] = 0.0;
        L.h[K] = 0.0;
    }
    if (lane < N)
#pragma unroll
        for (int c = 0; c < NP + 2; c++) L.row[lane][c] = (LT)0;
    double ctot = 0.0;
    if constexpr (kPD) ctot = Gp::sum(lane < K ? rho * yi * sp.invW : 0.0);
    Gp::sync();
    const int R = m.R;
    // per reaction: q, sum_l C_l dq/dC_l, dq/dT, dq/dC at the four slots and
    // (pressure-dependent mechanisms) G = d q / d[M]
    double *qh = qbuf + R, *dqT = qbuf + 2 * R, *dq = qbuf + 3 * R, *gM = qbuf + 7 * R;
    const double ln_c0 = log(kPstd / kRu) - lnT;
    for (int r = lane; r < R; r += G) {
        const DevRxn x = m.rxn[r];
        const double lnkf = x.lnA + x.b * lnT - x.Ea_R * invT;
        const double dg = L.g[x.p0] + L.g[x.p1] - L.g[x.r0] - L.g[x.r1];
        const double dh = L.h[x.p0] + L.h[x.p1] - L.h[x.r0] - L.h[x.r1];
        const double lnkr = lnkf + dg - x.dnu * ln_c0;
        const int kind = x.kind & 7;
        const double dlnk = (x.b + x.Ea_R * invT) * invT;
        const double cr0 = L.C[x.r0], cr1 = L.C[x.r1], cp0 = L.C[x.p0], cp1 = L.C[x.p1];
        const double k0f = exp(lnkf), k0r = (x.kind & kRxnIrrev) ? 0.0 : exp(lnkr);
        PdepRate pd{1.0, 0.0, 0.0};
        double M = 0.0;
        if constexpr (kPD) {
            if (kind != kRxnElem) {
                M = third_body(x, m.aux, ctot, [&](int l) { return L.C[l]; });
                pd = pdep_rate<true>(kind, m.aux + x.aux, M, T, lnT, invT, lnkf, dlnk);
            }
        }
        const double kf = kPD ? k0f * pd.mult : k0f, kr = kPD ? k0r * pd.mult : k0r;
        const double fwd = kf * cr0 * cr1, rev = kr * cp0 * cp1;
        const double mf = (x.r1 != K) ? 2.0 : 1.0, mr = (x.p1 != K) ? 2.0 : 1.0;
        const double dlnkf = kPD ? dlnk + pd.dlnT : dlnk;
        const double dlnkr = dlnkf - (dh - x.dnu) * invT;
        qbuf[r] = fwd - rev;
        dqT[r] = fwd * dlnkf - rev * dlnkr;
        dq[4 * r + 0] = kf * cr1;
        dq[4 * r + 1] = kf * cr0;
        dq[4 * r + 2] = -kr * cp1;
        dq[4 * r + 3] = -kr * cp0;
        if constexpr (kPD) {
            const double g = pd.dM * (k0f * cr0 * cr1 - k0r * cp0 * cp1);
            qh[r] = mf * fwd - mr * rev + g * M;
            gM[r] = g;
        } else {
            qh[r] = mf * fwd - mr * rev;
        }
    }
    Gp::sync();
    // species rows: owner lane k walks the reactions it takes part in
    double wk = 0.0, wTk = 0.0, ACk = 0.0, uk = 0.0;
    if (lane < K) {
        const int b = wt.inc_off[lane], e = wt.inc_off[lane + 1];
        for (int j = b; j < e; j++) {
            const int2 ent = wt.inc[j];
            const int r = ent.x;
            const double nu = (double)ent.y;
            const DevRxn x = m.rxn[r];
            wk += nu * qbuf[r];
            wTk += nu * dqT[r];
            ACk += nu * qh[r];
            const int sl[4] = {x.r0, x.r1, x.p0, x.p1};
#pragma unroll
            for (int s = 0; s < 4; s++) {
                const bool sentinel = sl[s] == K;
                const int c = sentinel ? NP + 1 : sl[s];
                const double f = sentinel ? 0.0 : nu * sp.W * L.invW[sl[s]];
                L.row[lane][c] += (LT)(f * dq[4 * r + s]);
            }
            if (kPD && (x.kind & 7) != kRxnElem) {
                // through [M]: the default efficiency on every column (added
                // with the rank-one term below), the listed ones here
                const double gn = nu * gM[r];
                uk += gn * x.def_eff;
                const double *ef = m.aux + x.aux + kAuxHead;
                for (int t = 0; t < x.neff; t++) {
                    const int l = (int)ef[2 * t];
                    L.row[lane][l] += (LT)(gn * ef[2 * t + 1] * sp.W * L.invW[l]);
                }
            }
        }
    }
    const double RT = kRu * T;
    const double rcp = rho * cpm;
    const double inv_rcp = 1.0 / rcp;
    const double S = RT * Gp::sum(lane < K ? hk * wk : 0.0);
    const double hAC = Gp::sum(lane < K ? hk * ACk : 0.0);
    const double dST = Gp::sum(lane < K ? kRu * cpk * wk + RT * hk * (wTk - ACk * invT) : 0.0);
    double hU = 0.0;
    if constexpr (kPD) hU = Gp::sum(lane < K ? hk * uk : 0.0);
    Gp::sync();
    // temperature row: lane j sums column j over the species rows
    double JT = 0.0;
    if (lane < K) {
        double col = 0.0;
#pragma unroll 4
        for (int k = 0; k < K; k++) col += (double)L.row[k][lane] * (L.h[k] * L.invW[k]);
        if constexpr (kPD) col += sp.invW * hU;
        const double dS = RT * rho * (col - (wbar / rho) * sp.invW * hAC);
        const double drcp = rho * sp.invW * (kRu * cpk - cpm * wbar);
        JT = (-dS + S * drcp * inv_rcp) * inv_rcp;
    } else if (lane == K) {
        const double drcpT = rho * dcpm - cpm * rho * invT;
        JT = (-dST + S * drcpT * inv_rcp) * inv_rcp;
    }
    Gp::sync();
    const double gq = wbar / rho;
    if (lane < K) {
        const double u = kPD ? sp.W * (gq * (wk - ACk) + uk) : sp.W * gq * (wk - ACk);
#pragma unroll 4
        for (int c = 0; c < K; c++) L.row[lane][c] += (LT)(u * L.invW[c]);
        L.row[lane][K] = (LT)(sp.W / rho * (wTk + (wk - ACk) * invT));
    }
    if (lane < N) L.row[K][lane] = (LT)JT;
    Gp::sync();
    if (lane < N)
        for (int c = 0; c < N; c++)
            L.row[lane][c] = (LT)((c == lane ? 1.0 : 0.0) - gamma * (double)L.row[lane][c]);
    Gp::sync();
}

// LU with row partial pivoting of the Newton matrix in LDS, in place: at
// step k the pivot is the largest magnitude in column k at or below the
// diagonal (ties to the lowest row), rows k and p are exchanged, and lane r
// eliminates its row r > k against the pivot row (read by every lane from
// the same LDS address).
template <int NP, typename LT, int G>
__device__ __forceinline__ bool wave_lu(WaveLds<NP, LT, G> &L, int N, int &pi, LT &dinv)
{
    using Gp = Grp<G>;
    const int lane = Gp::lane();
    bool ok = true;
    pi = lane;   // lane k ends with the original row that lands at position k
    for (int k = 0; k < N; k++) {
        const bool cand = lane >= k && lane < N;
        int p = group_argmax<G>(cand ? (double)L.row[lane][k] : 0.0, cand);
        if (p < 0) {   // no comparable value (NaN column): keep the row, fail below
            p = k;
            ok = false;
        }
        if (p != k) {
            const int a = Gp::at(pi, k), b = Gp::at(pi, p);
            if (lane == k) pi = b;
            if (lane == p) pi = a;
            if (lane < N) {
                const LT ra = L.row[k][lane], rb = L.row[p][lane];
                L.row[k][lane] = rb;
                L.row[p][lane] = ra;
            }
        }
        Gp::sync();
        const LT piv = L.row[k][k];
        ok = ok && (piv != (LT)0);
        if (lane > k && lane < N) {
            const LT l = L.row[lane][k] / piv;
            L.row[lane][k] = l;
            L.lcol[lane] = l;
        }
        Gp::sync();
        // lane c updates column c below the pivot row: one multiplier read
        // (same address for every lane) and one element of its own column
        // per row, independent from row to row
        if (lane > k && lane < N) {
            const LT ukc = L.row[k][lane];
#pragma unroll 4
            for (int r = k + 1; r < N; r++) L.row[r][lane] -= L.lcol[r] * ukc;
        }
        Gp::sync();
    }
    dinv = lane < N ? (LT)1 / L.row[lane][lane] : (LT)0;
    return ok;
}

// Solve M x = b with the factors of wave_lu.  Lane i passes b_i and receives
// x_i: the row exchanges applied at once (each lane reads the component of
// its original row), then forward (unit lower) and backward substitution,
// each step broadcasting one component; the diagonal enters through its
// reciprocal.  The lane's matrix elements are read eight at a time ahead of
// the broadcast chain, which then runs on registers; with 16-lane groups the
// loops unroll completely and every broadcast is one DPP row broadcast.
template <int NP, typename LT, int G>
__device__ __forceinline__ double wave_solve(const WaveLds<NP, LT, G> &L, int N, int pi, LT dinv, double bi)
{
    using Gp = Grp<G>;
    const int lane = Gp::lane();
    LT x = (LT)Gp::gather(bi, pi);
    constexpr int B = 8;
#pragma unroll(G == 16 ? (NP + B - 1) / B : 1)
    for (int k0 = 0; k0 < NP; k0 += B) {
        if (k0 >= N) break;
        LT a[B];
#pragma unroll
        for (int j = 0; j < B; j++) {
            const int k = k0 + j;
            a[j] = (k < N && lane > k && lane < N) ? L.row[lane][k] : (LT)0;
        }
#pragma unroll
        for (int j = 0; j < B; j++) {
            const int k = k0 + j;
            if (k < N) x -= a[j] * Gp::at_k(x, k);
        }
    }
#pragma unroll(G == 16 ? (NP + B - 1) / B : 1)
    for (int k1 = (G == 16 ? NP - 1 : N - 1); k1 >= 0; k1 -= B) {
        LT a[B];
#pragma unroll
        for (int j = 0; j < B; j++) {
            const int k = k1 - j;
            a[j] = (k >= 0 && k < N && lane < k) ? L.row[lane][k] : (LT)0;
        }
#pragma unroll
        for (int j = 0; j < B; j++) {
            const int k = k1 - j;
            if (k >= 0 && k < N) {
                if (lane == k) x = x * dinv;
                x -= a[j] * Gp::at_k(x, k);
            }
        }
    }
    return lane < N ? (double)x : 0.0;
}

// One group of G lanes integrates one cell at a time and takes the next from
// the work queue as soon as its cell is done, whatever the other groups of
// the wave are doing: each pass of the loop is one step of the group's cell
// (preceded by taking and starting a new cell when the group has none).
template <int NP, typename LT, int G, bool DEFER>
__device__ void run_cells(const DevMechView &m, const WaveTables &wt, const CellIO &io,
                          double t_end, unsigned long long *queue, double *qbuf,
                          WaveLds<NP, LT, G> &L)
{
    using namespace bdf;
    using Gp = Grp<G>;
    const int lane = Gp::lane();
    const int K = m.K, N = K + 1;
    const double rtol = io.prm->rtol, atol = io.prm->atol;
    SpeciesLane sp;
    {
        const int k = lane < K ? lane : 0;
        sp.blk = m.species + k * kSpeciesLen;
        sp.W = m.W[k];
        sp.invW = m.invW[k];
    }
    if (lane <= K) L.invW[lane] = lane < K ? sp.invW : 0.0;
    Gp::sync();
    const bool active = lane < N;
    int lu_pi = lane;       // factorisation's row permutation (this lane's entry)
    LT lu_dinv = (LT)0;     // reciprocal of this lane's diagonal element of U
    // the group's cell and its integration state
    bool busy = false;
    int64_t cell = 0;
    double p = 0.0, w = 0.0, h = 0.0, t = 0.0;
    double z[kQmax + 1], tau[kQmax + 2];
    int nst = 0, nfe = 0, nje = 0, nni = 0, netf = 0, ncfn = 0, status = 0;
    int q = 1, qwait = 2, nst_M = 0;
    bool have_M = false, ehat_ok = false;
    bool waited = false;    // the group sat out the last pass (refresh deferral)
    unsigned long long ticket = 0;   // the group's last work-queue position
    double gamma_M = 0.0, crate = 1.0, ehat_h = 0.0, ehat = 0.0;
    auto wnorm = [&](double v) { const double u = active ? v * w : 0.0; return sqrt(Gp::sum(u * u) * (1.0 / N)); };
    auto all_finite = [&](double v) { return Gp::ballot(active && !isfinite(v)) == 0ull; };
    for (;;) {
        if (!busy) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(queue, 1ull);
            c = Gp::first(c);
            if (c >= (unsigned long long)io.nq) break;
            ticket = c;
            const int64_t cc = io.idx ? (int64_t)io.idx[c] : (int64_t)c;
            if (cc < 0 || cc >= io.n) continue;   // an index outside the arrays is skipped
            cell = cc;
            busy = true;
            p = io.p[cell];
            double y0 = 0.0;
            if (lane < K) y0 = io.Y[lane * io.ldY + cell];
            else if (lane == K) y0 = io.T[cell];
            nst = nfe = nje = nni = netf = ncfn = 0;
            status = 0;
            // ---------------- initial derivative and step ----------------
            const double f0 = wave_rhs<NP, LT, G>(m, wt, L, sp, K, p, y0, qbuf);
            nfe++;
#pragma unroll
            for (int j = 0; j <= kQmax; j++) z[j] = 0.0;
            z[0] = y0;
            w = active ? 1.0 / (rtol * fabs(y0) + atol) : 0.0;
            if (!all_finite(f0)) {
                status = 4;
            }
            h = t_end;
            if (status == 0 && wnorm(f0) != 0.0) {
                double hub = t_end;
                {
                    // hub = min over components of (0.1|y0| + 1/w)/|f0| where it binds
                    double lim = active ? 0.1 * fabs(y0) + 1.0 / w : 0.0;
                    // sequential in component order, like the definition
                    for (int i = 0; i < N; i++) {
                        const double fi = Gp::at(f0, i), li = Gp::at(lim, i);
                        if (fabs(fi) * hub > li) hub = li / fabs(fi);
                    }
                }
                double hg = hub;
                for (int it = 0; it < kH0Iters; it++) {
                    const double f1 = wave_rhs<NP, LT, G>(m, wt, L, sp, K, p, y0 + hg * f0, qbuf);
                    nfe++;
                    if (!all_finite(f1)) {
                        hg *= 0.1;
                        continue;
                    }
                    const double ydd = wnorm((f1 - f0) / hg);
                    double hnew = ydd > 0.0 ? sqrt(2.0 / ydd) : hub;
                    if (hnew > hub) hnew = hub;
                    const double ratio = hnew / hg;
                    hg = hnew;
                    if (ratio >= 0.5 && ratio <= 2.0) break;
                }
                h = 0.5 * hg;
                if (h > t_end) h = t_end;
            }
            z[1] = h * f0;
            q = 1;
            qwait = 2;
            nst_M = 0;
            have_M = false;
            ehat_ok = false;
            gamma_M = 0.0;
            crate = 1.0;
            ehat_h = 0.0;
            ehat = 0.0;
            t = 0.0;
#pragma unroll
            for (int j = 0; j < kQmax + 2; j++) tau[j] = 0.0;
        }
        do {   // one step of the cell; break ends the step early
            if (status != 0 || t >= t_end) break;
            if (nst >= io.prm->max_steps) {
                status = 1;
                break;
            }
            if constexpr (Gp::kCells > 1 && DEFER) {
                // The cells of a wave share its instruction stream: a Newton
                // matrix refresh (Jacobian and LU) for one of them costs the
                // whole wave.  A cell whose step will start with a refresh
                // sits out one pass unless another cell of the wave needs one
                // too (or it is the only cell stepping), so refreshes are
                // shared more often.  Only while more cells were queued than
                // the grid holds groups when this one took its cell: in the
                // tail the slowest cell's latency is the run time, and waiting
                // would lengthen it.  Its state is untouched while it waits:
                // results do not depend on this.  The test estimates the
                // step's gamma = h / l_1, l_1 = sum of 1/xi_i over the order;
                // the refresh itself is decided exactly inside the step.
                bool need = false;
                if ((unsigned long long)io.nq - ticket > (unsigned long long)gridDim.x * Gp::kCells) {
                    const double hh = (t + h >= t_end) ? t_end - t : h;
                    double l1 = 0.0, s = hh;
#pragma unroll
                    for (int i = 1; i <= kQmax; i++)
                        if (i <= q) {
                            l1 += hh / s;
                            s += tau[i];
                        }
                    need = !have_M || nst >= nst_M + kMsbp || fabs((hh / l1) / gamma_M - 1.0) > kDgmax;
                }
                const bool lead = lane == 0;
                const int n_need = __popcll(__ballot(lead && need));
                const int n_step = __popcll(__ballot(lead));
                if (need && !waited && n_need < 2 && n_step >= 2) {
                    waited = true;
                    break;
                }
                waited = false;
            }
            bool last = false;
            if (t + h >= t_end) {
                const double eta = (t_end - t) / h;
                double f = 1.0;
#pragma unroll
                for (int j = 1; j <= kQmax; j++) {
                    f *= eta;
                    if (j <= q) z[j] *= f;
                }
                h = t_end - t;
                last = true;
            }
            w = active ? 1.0 / (rtol * fabs(z[0]) + atol) : 0.0;
            int nef = 0, ncf = 0;
            bool force_M = false;
            double dsm = 0.0, e = 0.0;
            double xi[kQmax + 2], l[kQmax + 1];
            for (;;) {
                const double tnew = t + h;
                if (tnew == t) {
                    status = 2;
                    break;
                }
#pragma unroll
                for (int kk = 1; kk <= kQmax; kk++)
#pragma unroll
                    for (int j = kQmax; j >= kk; j--)
                        if (j <= q) z[j - 1] += z[j];
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
                double xq1 = h;
#pragma unroll
                for (int i = 1; i <= kQmax; i++)
                    if (i <= q) xq1 += tau[i];
                xq1 /= h;
                const double Cq = 1.0 / (1.0 + l[1] * xq1);
                bool jcur = false, conv = false, lu_ok = true;
                if (!have_M || force_M || nst >= nst_M + kMsbp || fabs(gamma / gamma_M - 1.0) > kDgmax) {
                    wave_newton_matrix<NP, LT, G>(m, wt, L, sp, K, p, z[0], gamma, qbuf);
                    nje++;
                    lu_ok = wave_lu<NP, LT, G>(L, N, lu_pi, lu_dinv);
                    gamma_M = gamma;
                    nst_M = nst;
                    crate = 1.0;
                    have_M = lu_ok;
                    jcur = true;
                    force_M = false;
                }
                if (lu_ok) {
                    double del_old = 0.0;
                    e = 0.0;
                    const double inv_l1 = 1.0 / l[1];
                    for (int it = 0; it < kMaxCor; it++) {
                        const double fy = wave_rhs<NP, LT, G>(m, wt, L, sp, K, p, z[0] + e, qbuf);
                        nfe++;
                        if (!all_finite(fy)) break;
                        double d = active ? -(e - gamma * fy + z[1] * inv_l1) : 0.0;
                        d = wave_solve<NP, LT, G>(L, N, lu_pi, lu_dinv, d);
                        if (!active) d = 0.0;
                        if (gamma != gamma_M) d *= 2.0 / (1.0 + gamma / gamma_M);
                        const double dl = wnorm(d);
                        e += d;
                        nni++;
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
#pragma unroll
                    for (int kk = kQmax; kk >= 1; kk--)
#pragma unroll
                        for (int j = kk; j <= kQmax; j++)
                            if (j <= q && kk <= q) z[j - 1] -= z[j];
                    if (!jcur) {
                        force_M = true;
                        continue;
                    }
                    ncfn++;
                    if (++ncf >= kMaxNcf) {
                        status = 3;
                        break;
                    }
                    double f = 1.0;
#pragma unroll
                    for (int j = 1; j <= kQmax; j++) {
                        f *= kEtaCf;
                        if (j <= q) z[j] *= f;
                    }
                    h *= kEtaCf;
                    last = false;
                    continue;
                }
                dsm = Cq * wnorm(e);
                if (dsm > 1.0) {
#pragma unroll
                    for (int kk = kQmax; kk >= 1; kk--)
#pragma unroll
                        for (int j = kk; j <= kQmax; j++)
                            if (j <= q && kk <= q) z[j - 1] -= z[j];
                    netf++;
                    if (++nef >= kMaxNef) {
                        status = 2;
                        break;
                    }
                    last = false;
                    if (nef >= kNefRestart) {
                        h *= kEtaMinEf;
                        q = 1;
                        const double fr = wave_rhs<NP, LT, G>(m, wt, L, sp, K, p, z[0], qbuf);
                        nfe++;
                        if (!all_finite(fr)) {
                            status = 4;
                            break;
                        }
                        z[1] = h * fr;
#pragma unroll
                        for (int j = 0; j < kQmax + 2; j++) tau[j] = 0.0;
                        qwait = 2;
                        ehat_ok = false;
                        continue;
                    }
                    double eta = 1.0 / (pow(kBiasQ * dsm, 1.0 / (q + 1)) + kAddon);
                    eta = fmin(fmax(eta, kEtaMinEf), kEtaMaxEf);
                    if (nef >= 2) eta = fmin(eta, kEtaNef2);
                    double f = 1.0;
#pragma unroll
                    for (int j = 1; j <= kQmax; j++) {
                        f *= eta;
                        if (j <= q) z[j] *= f;
                    }
                    h *= eta;
                    continue;
                }
#pragma unroll
                for (int j = 0; j <= kQmax; j++)
                    if (j <= q) z[j] += l[j] * e;
                break;
            }
            if (status != 0) break;
            t = last ? t_end : t + h;
            nst++;
            if (t >= t_end) break;

            // ---------------- next step size and order ----------------
            const double h_done = h;
            double prod_q = 1.0;
#pragma unroll
            for (int i = 1; i <= kQmax; i++)
                if (i <= q) prod_q *= xi[i];
            double x1 = h;
#pragma unroll
            for (int i = 1; i <= kQmax; i++)
                if (i <= q) x1 += tau[i];
            x1 /= h;
            double fact = 1.0;
#pragma unroll
            for (int i = 2; i <= kQmax + 1; i++)
                if (i <= q + 1) fact *= i;
            const double gfac = prod_q * (1.0 / l[1] + x1) / fact;
            const double ehat_new = e / gfac;
            if (qwait > 0) qwait--;
            const double etamax = (nef > 0 || ncf > 0) ? 1.0 : (nst == 1 ? kEtaMaxFirst : kEtaMax);
            double eta = 1.0;
            int qnew = q;
            if (etamax > 1.0) {
                eta = 1.0 / (pow(kBiasQ * dsm, 1.0 / (q + 1)) + kAddon);
                if (qwait == 0) {
                    double eta_m = 0.0, eta_p = 0.0;
                    if (q > 1) {
                        double prod = 1.0, l1 = 0.0, zq = 0.0;
#pragma unroll
                        for (int j = 2; j <= kQmax; j++)
                            if (j == q) zq = z[j];
#pragma unroll
                        for (int i = 1; i < kQmax; i++)
                            if (i <= q - 1) {
                                prod *= xi[i];
                                l1 += 1.0 / xi[i];
                            }
                        const double Em = wnorm(zq) * prod / l1;
                        eta_m = 1.0 / (pow(kBiasQm1 * Em, 1.0 / q) + kAddon);
                    }
                    if (q < io.prm->qmax && ehat_ok) {
                        const double rr = pow(h_done / ehat_h, q + 1);
                        const double dv = ehat_new - ehat * rr;
                        double prod = 1.0, l1 = 0.0;
#pragma unroll
                        for (int i = 1; i <= kQmax; i++)
                            if (i <= q + 1) {
                                prod *= xi[i];
                                l1 += 1.0 / xi[i];
                            }
                        double fact2 = fact * (q + 2);
                        const double Ep = wnorm(dv) * prod / (fact2 * l1);
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
                double zq = 0.0;
#pragma unroll
                for (int j = 2; j <= kQmax; j++)
                    if (j == q) zq = z[j];
#pragma unroll
                for (int j = 1; j < kQmax; j++)
                    if (j < q) z[j] -= d[j] * zq;
                q = qnew;
                qwait = q + 1;
                ehat_ok = false;
            } else if (qnew == q + 1) {
                const double inv = 1.0 / x1;
#pragma unroll
                for (int j = 2; j <= kQmax; j++)
                    if (j == q + 1) z[j] = 0.0;
#pragma unroll
                for (int j = 1; j <= kQmax; j++)
                    if (j <= q + 1) z[j] += e * l[j - 1] * inv;
                q = qnew;
                qwait = q + 1;
                ehat_ok = false;
            } else {
                ehat = ehat_new;
                ehat_h = h_done;
                ehat_ok = true;
            }
#pragma unroll
            for (int i = kQmax + 1; i >= 2; i--) tau[i] = tau[i - 1];
            tau[1] = h_done;
            if (eta != 1.0) {
                double f = 1.0;
#pragma unroll
                for (int j = 1; j <= kQmax; j++) {
                    f *= eta;
                    if (j <= q) z[j] *= f;
                }
                h *= eta;
            }
        } while (false);
        if (status == 0 && t < t_end) continue;
        // ---------------- the cell is done ----------------
        if (status == 0 && !all_finite(z[0])) status = 4;
        if (status == 0) {
            if (lane < K) io.Y[lane * io.ldY + cell] = z[0];
            else if (lane == K) io.T[cell] = z[0];
        }
        if (lane == 0) {
            if (io.status) io.status[cell] = status;
            if (io.counters) {
                io.counters[0 * io.n + cell] = nst;
                io.counters[1 * io.n + cell] = nfe;
                io.counters[2 * io.n + cell] = nje;
                io.counters[3 * io.n + cell] = nni;
                io.counters[4 * io.n + cell] = netf;
                io.counters[5 * io.n + cell] = ncfn;
            }
        }
        busy = false;
    }
}

// Reaction scratch of the right-hand side and the Jacobian (7 R doubles per
// cell in flight): in LDS after `qlds` (QLDS), else a global slice per group
// (qscratch).  Fixing the choice at compile time keeps LDS accesses as LDS
// instructions.
template <int NP, typename LT, int G, bool QLDS, bool DEFER>
__device__ __forceinline__ void run_block(const DevMechView &m, const WaveTables &wt, double *T, const double *p,
                                          double *Y, int64_t ldY, int64_t n, double dt, const BdfParams &prm,
                                          int32_t *status, int32_t *counters, unsigned long long *queue,
                                          double *qscratch, double *qlds, WaveLds<NP, LT, G> *Ls)
{
    const CellIO io = make_cell_io(T, p, Y, ldY, n, status, counters, prm);
    const int slot = Grp<G>::slot();
    const size_t q7 = (size_t)m.qstride;
    double *qbuf;
    if constexpr (QLDS)
        qbuf = qlds + slot * q7;
    else
        qbuf = qscratch + ((size_t)blockIdx.x * Grp<G>::kCells + slot) * q7;
    run_cells<NP, LT, G, DEFER>(m, wt, io, dt, queue, qbuf, Ls[slot]);
}

// One 64-lane wave per cell.
template <int NP, typename LT, bool QLDS>
__global__ void __launch_bounds__(64) bdf_wave_kernel(DevMechView m, WaveTables wt, double *__restrict__ T,
                                                      const double *__restrict__ p, double *__restrict__ Y,
                                                      int64_t ldY, int64_t n, double dt, BdfParams prm,
                                                      int32_t *__restrict__ status, int32_t *__restrict__ counters,
                                                      unsigned long long *__restrict__ queue,
                                                      double *__restrict__ qscratch)
{
    __shared__ WaveLds<NP, LT, 64> Ls[1];
    extern __shared__ double dyn[];
    run_block<NP, LT, 64, QLDS, false>(m, wt, T, p, Y, ldY, n, dt, prm, status, counters, queue, qscratch, dyn, Ls);
}

// Tile schedule: 16 lanes per cell, four cells per wave (N <= NP <= 16).  With
// STAGE the mechanism tables (species .. incidence entries, one contiguous
// range) are first copied into LDS, where the four cells share them, and the
// reaction scratch follows them there; without it both stay in global memory.
// DEFER: Newton-matrix refreshes are deferred by a pass to share them between
// the cells of a wave (for large batches; scheduling only).
template <int NP, typename LT, bool STAGE, bool DEFER>
__global__ void __launch_bounds__(64) bdf_tile_kernel(DevMechView m, WaveTables wt, double *__restrict__ T,
                                                      const double *__restrict__ p, double *__restrict__ Y,
                                                      int64_t ldY, int64_t n, double dt, BdfParams prm,
                                                      int32_t *__restrict__ status, int32_t *__restrict__ counters,
                                                      unsigned long long *__restrict__ queue,
                                                      double *__restrict__ qscratch)
{
    __shared__ WaveLds<NP, LT, 16> Ls[4];
    extern __shared__ double dyn[];
    if constexpr (STAGE) {
        const int tb = m.table_bytes;
        const int4 *src = (const int4 *)m.species;
        int4 *dst = (int4 *)dyn;
        for (int i = threadIdx.x; i < tb / 16; i += 64) dst[i] = src[i];
        __syncthreads();
        const char *base = (const char *)m.species;
        const char *lds = (const char *)dyn;
        DevMechView ml = m;
        ml.species = (const double *)lds;
        ml.W = (const double *)(lds + ((const char *)m.W - base));
        ml.invW = (const double *)(lds + ((const char *)m.invW - base));
        ml.rxn = (const DevRxn *)(lds + ((const char *)m.rxn - base));
        ml.aux = (const double *)(lds + ((const char *)m.aux - base));
        WaveTables wl;
        wl.inc_off = (const int *)(lds + ((const char *)wt.inc_off - base));
        wl.inc = (const int2 *)(lds + ((const char *)wt.inc - base));
        run_block<NP, LT, 16, true, DEFER>(ml, wl, T, p, Y, ldY, n, dt, prm, status, counters, queue, qscratch,
                                           dyn + tb / 8, Ls);
    } else {
        run_block<NP, LT, 16, false, DEFER>(m, wt, T, p, Y, ldY, n, dt, prm, status, counters, queue, qscratch, dyn,
                                            Ls);
    }
}

}  // namespace

#if !CHEM_WAVE_PDEP
int wave_kernel_rows(int N) { return N <= 16 ? 16 : (N <= 40 ? 40 : (N <= 64 ? 64 : 0)); }
#endif

// Persistent grid: as many one-wave blocks as fit on the device at once
// (occupancy with `dyn` bytes of dynamic LDS), at most one per `cells_per_wave`
// cells, at most max_groups / cells_per_wave when the reaction scratch is in
// global memory (one slice per group).
template <typename Kern>
static hipError_t launch_groups(Kern kern, int cells_per_wave, size_t dyn, bool qglobal, const DevMechView &m,
                                const WaveTables &wt, double *T, const double *p, double *Y, int64_t ldY, int64_t n,
                                double dt, const BdfParams &prm, int32_t *status, int32_t *counters,
                                unsigned long long *queue, double *qscratch, int max_groups, hipStream_t s)
{
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(1), 0, s, queue);
    int blocks = 0;
    {
        int dev = 0, cus = 0, per_cu = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, 64, dyn) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        // one-wave blocks: four SIMDs per compute unit
        if (prm.waves_per_simd > 0 && per_cu > 4 * prm.waves_per_simd) per_cu = 4 * prm.waves_per_simd;
        blocks = cus * per_cu;
    }
    if (qglobal && blocks > max_groups / cells_per_wave) blocks = max_groups / cells_per_wave;
    const int64_t need = (n + cells_per_wave - 1) / cells_per_wave;
    if (blocks > need) blocks = (int)need;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64), dyn, s, m, wt, T, p, Y, ldY, n, dt, prm, status, counters, queue,
                       qscratch);
    return hipGetLastError();
}

constexpr size_t kQbufLdsMax = 49152;     // reaction scratch of one wave kept in LDS up to this size
constexpr size_t kTileStageMax = 24576;   // tables + scratch of a tile block staged in LDS up to this size
constexpr int64_t kDeferMinCells = 65536; // tile batches from this size defer Newton-matrix refreshes

#if !CHEM_WAVE_PDEP
bool wave_uses_global_scratch(const DevMechView &m, int lanes)
{
    const size_t q7 = (size_t)m.qstride * sizeof(double);
    if (lanes == 16) return (size_t)m.table_bytes + 4 * q7 > kTileStageMax;
    return q7 > kQbufLdsMax;
}
#endif

template <int NP, typename LT>
static hipError_t launch_wave(const DevMechView &m, const WaveTables &wt, double *T, const double *p, double *Y,
                              int64_t ldY, int64_t n, double dt, const BdfParams &prm, int32_t *status,
                              int32_t *counters, unsigned long long *queue, double *qscratch, int max_groups,
                              hipStream_t s)
{
    const size_t qbytes = (size_t)m.qstride * sizeof(double);
    if (qbytes <= kQbufLdsMax)
        return launch_groups(bdf_wave_kernel<NP, LT, true>, 1, qbytes, false, m, wt, T, p, Y, ldY, n, dt, prm,
                             status, counters, queue, qscratch, max_groups, s);
    return launch_groups(bdf_wave_kernel<64, LT, false>, 1, 0, true, m, wt, T, p, Y, ldY, n, dt, prm, status,
                         counters, queue, qscratch, max_groups, s);
}

template <int NP, typename LT>
static hipError_t launch_tile(const DevMechView &m, const WaveTables &wt, double *T, const double *p, double *Y,
                              int64_t ldY, int64_t n, double dt, const BdfParams &prm, int32_t *status,
                              int32_t *counters, unsigned long long *queue, double *qscratch, int max_groups,
                              hipStream_t s)
{
    const size_t lds = (size_t)m.table_bytes + (size_t)4 * m.qstride * sizeof(double);
    // refresh deferral pays when the queue holds many cells per group; a
    // small batch is latency bound and runs the plain loop.  A count that
    // lives on the device is taken as small.
    const int64_t nq = prm.n_dev ? 0 : (prm.idx ? prm.n_idx : n);
    const bool defer = nq >= kDeferMinCells;
#define CHEM_TILE(NPV, STAGE, DEF, DYN, QG)                                                                      \
    return launch_groups(bdf_tile_kernel<NPV, LT, STAGE, DEF>, 4, DYN, QG, m, wt, T, p, Y, ldY, n, dt, prm, status, \
                         counters, queue, qscratch, max_groups, s)
    if (lds <= kTileStageMax) {
        if (defer) CHEM_TILE(NP, true, true, lds, false);
        CHEM_TILE(NP, true, false, lds, false);
    }
    if (defer) CHEM_TILE(16, false, true, 0, true);
    CHEM_TILE(16, false, false, 0, true);
#undef CHEM_TILE
}

#if CHEM_WAVE_PDEP
hipError_t launch_bdf_wave_pdep(const DevMechView &m, const WaveTables &wt, double *T, const double *p,
                                double *Y, int64_t ldY, int64_t n, double dt, const BdfParams &prm,
                                int32_t *status, int32_t *counters, unsigned long long *queue,
                                double *qscratch, int max_groups, bool fp32_lu, int lanes, hipStream_t s)
{
#else
hipError_t launch_bdf_wave_pdep(const DevMechView &m, const WaveTables &wt, double *T, const double *p,
                                double *Y, int64_t ldY, int64_t n, double dt, const BdfParams &prm,
                                int32_t *status, int32_t *counters, unsigned long long *queue,
                                double *qscratch, int max_groups, bool fp32_lu, int lanes, hipStream_t s);

hipError_t launch_bdf_wave(const DevMechView &m, const WaveTables &wt, double *T, const double *p,
                           double *Y, int64_t ldY, int64_t n, double dt, const BdfParams &prm,
                           int32_t *status, int32_t *counters, unsigned long long *queue,
                           double *qscratch, int max_groups, bool fp32_lu, int lanes, hipStream_t s)
{
    if (m.n_pdep)
        return launch_bdf_wave_pdep(m, wt, T, p, Y, ldY, n, dt, prm, status, counters, queue, qscratch,
                                    max_groups, fp32_lu, lanes, s);
#endif
#define CHEM_LAUNCH(FN, NPV)                                                                                     \
    return fp32_lu ? FN<NPV, float>(m, wt, T, p, Y, ldY, n, dt, prm, status, counters, queue, qscratch,        \
                                    max_groups, s)                                                             \
                   : FN<NPV, double>(m, wt, T, p, Y, ldY, n, dt, prm, status, counters, queue, qscratch,       \
                                     max_groups, s)
    const int N = m.K + 1;
    if (lanes == 16) {
        if (N <= 12) CHEM_LAUNCH(launch_tile, 12);
        if (N <= 16) CHEM_LAUNCH(launch_tile, 16);
        return hipErrorInvalidValue;
    }
    if (N <= 16) CHEM_LAUNCH(launch_wave, 16);
    if (N <= 40) CHEM_LAUNCH(launch_wave, 40);
    if (N <= 64) CHEM_LAUNCH(launch_wave, 64);
#undef CHEM_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace chem

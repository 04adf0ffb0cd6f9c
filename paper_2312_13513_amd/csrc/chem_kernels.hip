// Table-driven (generic) mechanism kernels for gfx950: reactor right-hand
// side and analytic Jacobian read the mechanism from device tables, and plug
// into the shared BDF driver (bdf_driver.h).  Mechanisms compiled by the
// mechanism compiler use specialised functors instead.
//
// Data layout: cell state is structure-of-arrays in HBM (T[i], p[i],
// Y[k*ldY + i]) so that consecutive lanes read consecutive doubles (paper
// Section 3.2: coalesced storage of the components of multi-component fields).
// Mechanism tables are read with wave-uniform addresses, i.e. through scalar
// loads, and the species count K is a template parameter so that every
// per-species array lives in registers.  Reaction loops run over a runtime
// count with wave-uniform species indices (register indexing mode).

#include "bdf_driver.h"

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
    double ctot = 0.0;   // total concentration (third bodies)
    if (m.n_pdep) {
#pragma unroll
        for (int k = 0; k < K; k++) ctot += C[k];
    }
    const double ln_c0 = log(kPstd / kRu) - lnT;   // ln(p_std / (R T))
    for (int r = 0; r < m.R; r++) {
        const DevRxn x = m.rxn[r];
        const double lnkf = x.lnA + x.b * lnT - x.Ea_R * invT;
        const double dg = gRT[x.p0] + gRT[x.p1] - gRT[x.r0] - gRT[x.r1];
        // k_r = k_f / K_c with ln K_c = -dg + dnu ln(p_std/(R T))
        const double lnkr = lnkf + dg - x.dnu * ln_c0;
        const double fwd = exp(lnkf) * C[x.r0] * C[x.r1];
        double q = (x.kind & kRxnIrrev) ? fwd : fwd - exp(lnkr) * C[x.p0] * C[x.p1];
        const int kind = x.kind & 7;
        if (kind != kRxnElem) {
            const double M = third_body(x, m.aux, ctot, [&](int l) { return C[l]; });
            q *= pdep_rate<false>(kind, m.aux + x.aux, M, T, lnT, invT, lnkf, 0.0).mult;
        }
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
    double ctot = 0.0, udef[KP];   // total concentration; dense third-body part of A per row
    if (m.n_pdep) {
#pragma unroll
        for (int k = 0; k < K; k++) ctot += C[k];
    }
#pragma unroll
    for (int k = 0; k < KP; k++) udef[k] = 0.0;
    const double ln_c0 = log(kPstd / kRu) - lnT;
    for (int r = 0; r < m.R; r++) {
        const DevRxn x = m.rxn[r];
        const double lnkf = x.lnA + x.b * lnT - x.Ea_R * invT;
        const double dg = gRT[x.p0] + gRT[x.p1] - gRT[x.r0] - gRT[x.r1];
        const double dh = hRT[x.p0] + hRT[x.p1] - hRT[x.r0] - hRT[x.r1];
        const double lnkr = lnkf + dg - x.dnu * ln_c0;
        const int kind = x.kind & 7;
        const double dlnk = (x.b + x.Ea_R * invT) * invT;
        // k_f = exp(lnkf) mult; mult = 1 for an elementary reaction
        PdepRate pd{1.0, 0.0, 0.0};
        double M = 0.0;
        if (kind != kRxnElem) {
            M = third_body(x, m.aux, ctot, [&](int l) { return C[l]; });
            pd = pdep_rate<true>(kind, m.aux + x.aux, M, T, lnT, invT, lnkf, dlnk);
        }
        const double kf = exp(lnkf) * pd.mult;
        const double kr = (x.kind & kRxnIrrev) ? 0.0 : exp(lnkr) * pd.mult;
        const double fwd = kf * C[x.r0] * C[x.r1];
        const double rev = kr * C[x.p0] * C[x.p1];
        const double q = fwd - rev;
        const double dlnkf = dlnk + pd.dlnT;
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
        if (kind != kRxnElem) {
            // through [M]: d q / d C_l += G eff_l with G = d mult/d[M] (q / mult)
            const double G = pd.dM * (exp(lnkf) * C[x.r0] * C[x.r1] -
                                      ((x.kind & kRxnIrrev) ? 0.0 : exp(lnkr) * C[x.p0] * C[x.p1]));
            const double *e = m.aux + x.aux + kAuxHead;
#pragma unroll
            for (int a = 0; a < 4; a++) {
                udef[sl[a]] += nu[a] * G * x.def_eff;
                for (int j = 0; j < x.neff; j++) A[sl[a] * KP + (int)e[2 * j]] += nu[a] * G * e[2 * j + 1];
            }
        }
    }
    if (m.n_pdep) {
#pragma unroll
        for (int k = 0; k < K; k++)
#pragma unroll
            for (int l = 0; l < K; l++) A[k * KP + l] += udef[k];
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

}  // namespace

// Table-driven mechanism functor for the generic kernels.
template <int KK>
struct TableMech {
    static constexpr int K = KK;
    DevMechView m;
    __device__ __forceinline__ void rhs(double p, const double *y, double *f) const { reactor_rhs<KK>(m, p, y, f); }
    __device__ __forceinline__ void jac(double p, const double *y, double *J) const { reactor_jacobian<KK>(m, p, y, J); }
};

__global__ void reset_queue_kernel(unsigned long long *queue) { *queue = 0ull; }

__global__ void start_reset_kernel(unsigned long long *queue, int32_t *cnt)
{
    if (threadIdx.x < kCostBuckets) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) *queue = 0ull;
}

__global__ void start_scan_kernel(int32_t *cnt)
{
    if (threadIdx.x != 0) return;
    int32_t s = 0;
    for (int b = kCostBuckets - 1; b >= 0; b--) {
        const int32_t c = cnt[b];
        cnt[b] = s;
        s += c;
    }
}

// Ranks within the block by LDS atomics, then one global atomic per
// non-empty bucket of the block reserves its range (a global atomic per item
// would serialise on the few buckets that hold most cells).
__global__ void __launch_bounds__(256) start_scatter_kernel(const int32_t *key, int32_t *cnt, int32_t *ord,
                                                            int64_t n, BdfParams prm)
{
    __shared__ int hist[kCostBuckets], base[kCostBuckets];
    if (threadIdx.x < kCostBuckets) hist[threadIdx.x] = 0;
    __syncthreads();
    const CellIO io = make_cell_io(nullptr, nullptr, nullptr, 0, n, nullptr, nullptr, prm);
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = it < io.nq;
    const int k = in ? key[it] : 0;
    const int rank = in ? atomicAdd(&hist[k], 1) : 0;
    __syncthreads();
    if (threadIdx.x < kCostBuckets)
        base[threadIdx.x] = hist[threadIdx.x] != 0 ? atomicAdd(&cnt[threadIdx.x], hist[threadIdx.x]) : 0;
    __syncthreads();
    if (in) ord[base[k] + rank] = (int32_t)it;
}

int queue_grid(const void *kernel, int64_t n, int waves_per_simd)
{
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    // one-wave blocks: four SIMDs per compute unit
    if (waves_per_simd > 0 && per_cu > 4 * waves_per_simd) per_cu = 4 * waves_per_simd;
    int64_t blocks = (int64_t)cus * per_cu;
    const int64_t need = (n + 63) / 64;
    if (blocks > need) blocks = need;
    return (int)(blocks < 1 ? 1 : blocks);
}

#define CHEM_FOR_EACH_K(X) X(9)

bool table_eval_supports(int K)
{
#define CHEM_CASE(KK) if (K == KK) return true;
    CHEM_FOR_EACH_K(CHEM_CASE)
#undef CHEM_CASE
    return false;
}

hipError_t launch_rhs(const DevMechView &m, const double *T, const double *p, const double *Y,
                      int64_t ldY, int64_t n, double *F, int64_t ldF, hipStream_t s)
{
#define CHEM_CASE(KK)                                                                              \
    if (m.K == KK) {                                                                               \
        hipLaunchKernelGGL(rhs_eval_kernel<TableMech<KK>>, dim3((unsigned)((n + 255) / 256)),      \
                           dim3(256), 0, s, TableMech<KK>{m}, T, p, Y, ldY, n, F, ldF);            \
        return hipGetLastError();                                                                  \
    }
    CHEM_FOR_EACH_K(CHEM_CASE)
#undef CHEM_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_jacobian(const DevMechView &m, const double *T, const double *p, const double *Y,
                           int64_t ldY, int64_t n, double *J, int64_t ldJ, hipStream_t s)
{
#define CHEM_CASE(KK)                                                                            \
    if (m.K == KK) {                                                                             \
        hipLaunchKernelGGL(jac_eval_kernel<TableMech<KK>>, dim3((unsigned)((n + 63) / 64)),      \
                           dim3(64), 0, s, TableMech<KK>{m}, T, p, Y, ldY, n, J, ldJ);           \
        return hipGetLastError();                                                                \
    }
    CHEM_FOR_EACH_K(CHEM_CASE)
#undef CHEM_CASE
    return hipErrorInvalidValue;
}

}  // namespace chem

// Internal declarations shared by the host runtime and the HIP kernels of the
// chemistry library.  Nothing here is part of the public ABI (include/chem.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chem {

constexpr double kRu = 8.31446261815324;   // J/(mol K)
constexpr double kPstd = 101325.0;         // standard-state pressure, Pa
constexpr int kQmax = 5;                   // highest BDF order

// NASA-7 range block: 7 coefficients plus the divided ones used by H/RT and S/R.
//   c[0..6] = a1..a7, c[7..10] = a2/2, a3/3, a4/4, a5/5, c[11..13] = a3/2, a4/3, a5/4
constexpr int kRangeLen = 14;
// Per species: T_mid, low block, high block.
constexpr int kSpeciesLen = 1 + 2 * kRangeLen;

// One reaction as seen by the kernels: up to two molecule slots per side; an
// empty slot holds the sentinel species index K (concentration 1, G/RT 0), a
// coefficient of 2 is two slots with the same species.
struct DevRxn {
    int32_t r0, r1, p0, p1;
    int32_t dnu;       // product molecules minus reactant molecules
    int32_t kind;      // kRxn* pressure dependence, plus kRxnIrrev for no reverse rate
    int32_t aux;       // pressure-dependent kinds: offset of the record in DevMechView::aux
    int32_t neff;      // listed third-body efficiencies
    double lnA;        // ln of the SI pre-exponential factor (high-pressure limit of a fall-off)
    double b;          // temperature exponent
    double Ea_R;       // activation temperature Ea / Ru, K
    double def_eff;    // third-body efficiency of the species not listed
};
static_assert(sizeof(DevRxn) == 64, "reaction record is 64 bytes");

// DevRxn::kind: third body, Lindemann fall-off, Troe fall-off (T2 term in
// the record, 0 without one), plus a flag for an irreversible reaction.
constexpr int32_t kRxnElem = 0, kRxnThird = 1, kRxnLind = 2, kRxnTroe = 3, kRxnIrrev = 8;
// Record of a pressure-dependent reaction in DevMechView::aux: the header
// (ln A0 in SI units, b0, Ea0/Ru, Troe a, 1/T3, 1/T1, T2, has-T2 flag), then
// neff pairs (species index, efficiency minus the default efficiency).
constexpr int kAuxHead = 8;

struct DevMechView {
    int32_t K, R;
    int32_t two_range;          // 0 when every species uses one NASA range
    int32_t table_bytes;        // species .. incidence entries: one contiguous
                                // range of bytes starting at `species`
    const double *species;      // K x kSpeciesLen
    const double *W;            // K, kg/mol
    const double *invW;         // K
    const DevRxn *rxn;          // R
    const double *aux;          // records of the pressure-dependent reactions (inside the table range)
    int32_t n_pdep;             // pressure-dependent reactions (0: all elementary)
    int32_t qstride;            // doubles of reaction scratch per cell of the lane-group kernels
};

struct BdfParams {
    double rtol, atol;
    int32_t max_steps;
    int32_t jac_batch;      // lanes of a wave that wait before a Jacobian is evaluated
    const int64_t *n_dev;   // if not NULL: at most *n_dev cells (read on the device)
    const int32_t *idx;     // if not NULL: integrate cells idx[0 .. n_idx) in this order
    int64_t n_idx;
    int32_t qmax;           // highest order the step selection may raise to (1..kQmax)
    int32_t waves_per_simd; // cap on the persistent grid (0: as many waves as fit)
};

// Launchers of the table-driven kernels.  Return hipError_t of the launch.
hipError_t launch_rhs(const DevMechView &m, const double *T, const double *p, const double *Y,
                      int64_t ldY, int64_t n, double *F, int64_t ldF, hipStream_t s);
hipError_t launch_jacobian(const DevMechView &m, const double *T, const double *p, const double *Y,
                           int64_t ldY, int64_t n, double *J, int64_t ldJ, hipStream_t s);
struct StartPass;
// Species counts with table-driven right-hand-side and Jacobian evaluation
// kernels (chem_eval_rhs / chem_eval_jacobian of a mechanism that is not
// compiled in).
bool table_eval_supports(int K);

}  // namespace chem

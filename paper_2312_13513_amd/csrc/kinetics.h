// Pressure dependence of a reaction rate on the device: the third-body
// concentration, and the Lindemann and Troe fall-off forms (Gilbert, Luther
// and Troe 1983), with the derivatives the analytic Jacobians need.
//
// With k the reaction's own Arrhenius rate (the high-pressure limit of a
// fall-off reaction) the forward rate constant is k * mult:
//   third body: mult = [M]
//   fall-off:   mult = Pr / (1 + Pr) F,  Pr = k0 [M] / k,
//               F = 1 (Lindemann) or log10 F = log10 Fc / (1 + f^2),
//               f = (log10 Pr + c) / (n - 0.14 (log10 Pr + c)),
//               c = -0.4 - 0.67 log10 Fc, n = 0.75 - 1.27 log10 Fc,
//               Fc = (1 - a) exp(-T / T3) + a exp(-T / T1) [+ exp(-T2 / T)],
// the logarithms taken of max(Pr, 1e-300) and max(Fc, 1e-300).  The reverse
// rate constant carries the same factor (detailed balance).
#pragma once

#include "chem_internal.h"

namespace chem {

struct PdepRate {
    double mult;   // k_f / k
    double dlnT;   // d ln(mult) / dT at fixed concentrations
    double dM;     // d mult / d[M] at fixed T
};

// Third-body concentration of reaction x: default efficiency times the total
// concentration, plus (efficiency - default) C_l for every listed species.
// C(l) returns the concentration of species l.
template <class Conc>
__device__ __forceinline__ double third_body(const DevRxn &x, const double *aux, double ctot, Conc C)
{
    double M = x.def_eff * ctot;
    const double *e = aux + x.aux + kAuxHead;
    for (int j = 0; j < x.neff; j++) M += e[2 * j + 1] * C((int)e[2 * j]);
    return M;
}

// mult and its derivatives for a pressure-dependent kind; lnk is ln k, dlnk
// its temperature derivative (b + Ea/Ru / T) / T.
template <bool DERIV>
__device__ __forceinline__ PdepRate pdep_rate(int kind, const double *a, double M, double T, double lnT,
                                              double invT, double lnk, double dlnk)
{
    PdepRate o{M, 0.0, 1.0};
    if (kind == kRxnThird) return o;
    constexpr double kTiny = 1e-300, kLn10 = 2.302585092994045684;
    const double r0 = exp(a[0] + a[1] * lnT - a[2] * invT - lnk);   // k0 / k
    const double Pr = r0 * M;
    const double opr = 1.0 + Pr, iopr = 1.0 / opr;
    double F = 1.0, dx = 0.0, dlnF_T = 0.0;
    const double dlnPr = (a[1] + a[2] * invT) * invT - dlnk;
    if (kind == kRxnTroe) {
        const double e3 = exp(-T * a[4]), e1 = exp(-T * a[5]);
        double Fc = (1.0 - a[3]) * e3 + a[3] * e1;
        double dFc = -(1.0 - a[3]) * a[4] * e3 - a[3] * a[5] * e1;
        if (a[7] != 0.0) {
            const double e2 = exp(-a[6] * invT);
            Fc += e2;
            dFc += a[6] * invT * invT * e2;
        }
        if (Fc < kTiny) {
            Fc = kTiny;
            dFc = 0.0;
        }
        const double Lc = log10(Fc);
        const double x = log10(Pr < kTiny ? kTiny : Pr);
        const double c = -0.4 - 0.67 * Lc, n = 0.75 - 1.27 * Lc;
        const double u = x + c, D = n - 0.14 * u, iD = 1.0 / D, f = u * iD;
        const double s = 1.0 + f * f, is = 1.0 / s;
        F = exp(kLn10 * Lc * is);
        if (DERIV) {
            const double w = Lc * 2.0 * f * is * is * iD * iD;
            dx = Pr < kTiny ? 0.0 : -w * n;
            const double dLc = is - w * (1.27 * u - 0.67 * n);
            dlnF_T = dx * dlnPr + dLc * dFc / Fc;
        }
    }
    o.mult = Pr * iopr * F;
    if (DERIV) {
        o.dlnT = dlnPr * iopr + dlnF_T;
        o.dM = r0 * F * iopr * (iopr + dx);
    }
    return o;
}

}  // namespace chem

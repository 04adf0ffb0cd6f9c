/* Right-hand side of the per-cell reactor ODE, written once and instantiated
 * for real (double) and complex (double complex) arithmetic by oracle.c.
 * The complex instance exists only for the complex-step Jacobian check.
 *
 * Before inclusion define:
 *   RB_NAME   function name
 *   RB_KF     name of the forward rate constant function
 *   RB_T      scalar type
 *   RB_EXP, RB_LOG, RB_POW   exp, log, pow for RB_T
 *   RB_RE(x)  real part of an RB_T (branch decisions use it)
 *
 * What it computes (paper Section 2: detailed kinetics, chemistry source
 * integrated per cell as a stiff ODE; the equations are those of an adiabatic
 * constant-pressure reactor, state y = (Y_1..Y_K, T)):
 *   NASA-7 thermo per species, mixture molar mass, density, concentrations,
 *   Arrhenius forward rate (times the third-body concentration, or in the
 *   Lindemann / Troe fall-off form), reverse rate from the equilibrium
 *   constant (none for an irreversible reaction), mass-action rates of
 *   progress, net molar production rates, and
 *   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum_k H_k wdot_k / (rho cp).
 */

/* Forward rate constant of reaction r at T and concentrations C.
 *  third-body:  k [M],  [M] = sum_k eff_k C_k
 *  fall-off:    k_inf Pr / (1 + Pr) F,  Pr = k_0 [M] / k_inf  (Lindemann: F = 1)
 *  Troe:        log10 F = log10 Fcent / (1 + f^2),
 *               f = (log10 Pr + c) / (n - 0.14 (log10 Pr + c)),
 *               c = -0.4 - 0.67 log10 Fcent,  n = 0.75 - 1.27 log10 Fcent,
 *               Fcent = (1 - a) exp(-T/T3) + a exp(-T/T1) [+ exp(-T2/T)],
 *               T3, T1, T2 the parameters usually written with three, one
 *               and two asterisks
 * (Gilbert, Luther and Troe 1983).  The logarithms take max(Pr, 1e-300) and
 * max(Fcent, 1e-300). */
static RB_T RB_KF(const om_rxn *r, int K, RB_T T, const RB_T *C)
{
    const double ln10 = log(10.0), tiny = 1e-300;
    RB_T k = r->A_si * RB_POW(T, r->b) * RB_EXP(-r->Ea / (OM_RU * T));
    if (r->kind == OM_ELEM) return k;
    RB_T M = 0.0;
    for (int l = 0; l < K; l++) M += r->eff[l] * C[l];
    if (r->kind == OM_THIRD) return k * M;
    RB_T k0 = r->A0_si * RB_POW(T, r->b0) * RB_EXP(-r->Ea0 / (OM_RU * T));
    RB_T Pr = k0 * M / k;
    RB_T F = 1.0;
    if (r->kind == OM_TROE3 || r->kind == OM_TROE4) {
        RB_T Fc = (1.0 - r->ta) * RB_EXP(-T / r->tT3) + r->ta * RB_EXP(-T / r->tT1);
        if (r->kind == OM_TROE4) Fc += RB_EXP(-r->tT2 / T);
        RB_T Lc = RB_LOG(RB_RE(Fc) < tiny ? (RB_T)tiny : Fc) / ln10;
        RB_T x = RB_LOG(RB_RE(Pr) < tiny ? (RB_T)tiny : Pr) / ln10;
        RB_T c = -0.4 - 0.67 * Lc, n = 0.75 - 1.27 * Lc;
        RB_T fr = (x + c) / (n - 0.14 * (x + c));
        F = RB_EXP(ln10 * Lc / (1.0 + fr * fr));
    }
    return k * Pr / (1.0 + Pr) * F;
}

static void RB_NAME(const om_mech *m, double p, const RB_T *y, RB_T *f)
{
    const int K = m->K;
    RB_T T = y[K];
    RB_T cp_R[OM_KMAX], h_RT[OM_KMAX], s_R[OM_KMAX], g_RT[OM_KMAX], C[OM_KMAX], wdot[OM_KMAX];

    /* species thermo: range chosen on the real part of T */
    for (int k = 0; k < K; k++) {
        const double *a = (RB_RE(T) < m->nasa[k][1]) ? &m->nasa[k][3] : &m->nasa[k][10];
        cp_R[k] = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
        h_RT[k] = a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0
                + a[4] * T * T * T * T / 5.0 + a[5] / T;
        s_R[k] = a[0] * RB_LOG(T) + a[1] * T + a[2] * T * T / 2.0 + a[3] * T * T * T / 3.0
               + a[4] * T * T * T * T / 4.0 + a[6];
        g_RT[k] = h_RT[k] - s_R[k];
    }

    /* mixture: mean molar mass, density, concentrations, mass cp */
    RB_T inv_wbar = 0.0;
    for (int k = 0; k < K; k++) inv_wbar += y[k] / m->W[k];
    RB_T wbar = 1.0 / inv_wbar;
    RB_T rho = p * wbar / (OM_RU * T);
    RB_T cp_mass = 0.0;
    for (int k = 0; k < K; k++) {
        C[k] = rho * y[k] / m->W[k];
        cp_mass += y[k] * cp_R[k] * OM_RU / m->W[k];
        wdot[k] = 0.0;
    }

    /* reactions */
    for (int i = 0; i < m->R; i++) {
        const om_rxn *r = &m->rxn[i];
        RB_T kf = RB_KF(r, K, T, C);
        RB_T sum_nu_g = 0.0;
        for (int t = 0; t < r->np; t++) sum_nu_g += r->pnu[t] * g_RT[r->psp[t]];
        for (int t = 0; t < r->nr; t++) sum_nu_g -= r->rnu[t] * g_RT[r->rsp[t]];
        RB_T conc_fac = 1.0;  /* (p_std / (R T))^dnu, dnu an integer */
        RB_T base = OM_PSTD / (OM_RU * T);
        for (int d = 0; d < r->dnu; d++) conc_fac *= base;
        for (int d = 0; d > r->dnu; d--) conc_fac /= base;
        RB_T Kc = RB_EXP(-sum_nu_g) * conc_fac;
        RB_T kr = r->rev ? kf / Kc : 0.0;
        RB_T fwd = kf, rev = kr;
        for (int t = 0; t < r->nr; t++)
            for (int e = 0; e < r->rnu[t]; e++) fwd *= C[r->rsp[t]];
        for (int t = 0; t < r->np; t++)
            for (int e = 0; e < r->pnu[t]; e++) rev *= C[r->psp[t]];
        RB_T q = fwd - rev;
        for (int t = 0; t < r->nr; t++) wdot[r->rsp[t]] -= r->rnu[t] * q;
        for (int t = 0; t < r->np; t++) wdot[r->psp[t]] += r->pnu[t] * q;
    }

    /* ODE right-hand side */
    RB_T heat = 0.0;
    for (int k = 0; k < K; k++) {
        f[k] = m->W[k] * wdot[k] / rho;
        heat += OM_RU * T * h_RT[k] * wdot[k];
    }
    f[K] = -heat / (rho * cp_mass);
}

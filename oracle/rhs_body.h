/* Right-hand side of the per-cell reactor ODE, written once and instantiated
 * for real (double) and complex (double complex) arithmetic by oracle.c.
 * The complex instance exists only for the complex-step Jacobian check.
 *
 * Before inclusion define:
 *   RB_NAME   function name
 *   RB_T      scalar type
 *   RB_EXP, RB_LOG, RB_POW   exp, log, pow for RB_T
 *   RB_RE(x)  real part of an RB_T (branch decisions use it)
 *
 * What it computes (paper Section 2: detailed kinetics, chemistry source
 * integrated per cell as a stiff ODE; the equations are those of an adiabatic
 * constant-pressure reactor, state y = (Y_1..Y_K, T)):
 *   NASA-7 thermo per species, mixture molar mass, density, concentrations,
 *   Arrhenius forward rate, reverse rate from the equilibrium constant,
 *   mass-action rates of progress, net molar production rates, and
 *   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum_k H_k wdot_k / (rho cp).
 */
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
        RB_T kf = r->A_si * RB_POW(T, r->b) * RB_EXP(-r->Ea / (OM_RU * T));
        RB_T sum_nu_g = 0.0;
        for (int t = 0; t < r->np; t++) sum_nu_g += r->pnu[t] * g_RT[r->psp[t]];
        for (int t = 0; t < r->nr; t++) sum_nu_g -= r->rnu[t] * g_RT[r->rsp[t]];
        RB_T conc_fac = 1.0;  /* (p_std / (R T))^dnu, dnu an integer */
        RB_T base = OM_PSTD / (OM_RU * T);
        for (int d = 0; d < r->dnu; d++) conc_fac *= base;
        for (int d = 0; d > r->dnu; d--) conc_fac /= base;
        RB_T Kc = RB_EXP(-sum_nu_g) * conc_fac;
        RB_T kr = kf / Kc;
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

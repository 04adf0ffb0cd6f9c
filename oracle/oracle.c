/*
 * Plain FP64 CPU oracle for per-cell stiff chemistry integration.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header or table with the GPU library: it has its own mechanism reader, its
 * own thermo/kinetics, its own dense LU and its own BDF integrator, all
 * written as plainly as possible (no blocking, no fusion, no reordering).
 *
 * What it follows:
 *  - Paper Section 2: chemistry source of each CFD cell integrated as a stiff
 *    ODE (CVODE on the CPU path), detailed kinetics and thermo through
 *    temperature polynomials (also Section 3.1, the Thermo class: Newton's
 *    method on temperature polynomials).
 *  - The equations of an adiabatic constant-pressure reactor (state Y_1..Y_K,
 *    T), Arrhenius forward rates, reverse rates from K_c, NASA-7 polynomials.
 *  - The integrator contract: variable-order (1..5), variable-step BDF in
 *    Nordsieck form, variable-coefficient (interpolatory) formulation, with
 *    modified Newton on M = I - gamma J.  The paper names CVODE (Hindmarsh et
 *    al., ACM TOMS 2005) as its CPU chemistry integrator but gives no scheme
 *    constants; every constant below is this implementation's stated reading.
 *
 * Compiled with -O2 -ffp-contract=off, no fast-math.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OM_KMAX 64
#define OM_NMAX (OM_KMAX + 1)
#define OM_EMAX 16
#define OM_RU 8.31446261815324 /* J/(mol K), CODATA 2018 exact */
#define OM_PSTD 101325.0       /* standard-state pressure, Pa (1 atm) */

/* Pressure dependence of a reaction (file format version 2). */
enum { OM_ELEM = 0, OM_THIRD = 1, OM_LIND = 2, OM_TROE3 = 3, OM_TROE4 = 4 };

typedef struct {
    int nr, np;          /* number of reactant / product terms (1..2) */
    int rsp[2], rnu[2];  /* reactant species and integer coefficients */
    int psp[2], pnu[2];
    int dnu;             /* sum of product minus reactant coefficients */
    double A_si, b, Ea;  /* SI pre-exponential, temperature exponent, J/mol */
    int kind;            /* OM_ELEM .. OM_TROE4 */
    int rev;             /* 1: reverse rate from K_c; 0: irreversible */
    double *eff;         /* third-body efficiency of every species (NULL for OM_ELEM) */
    double A0_si, b0, Ea0;        /* low-pressure limit of a fall-off reaction */
    double ta, tT3, tT1, tT2;     /* Troe parameters (tT2 used by OM_TROE4 only) */
} om_rxn;

typedef struct {
    int K, R, E;
    double W[OM_KMAX];          /* kg/mol */
    int counts[OM_KMAX][OM_EMAX];
    double nasa[OM_KMAX][17];   /* Tlo Tmid Thi, 7 low, 7 high */
    om_rxn *rxn;
} om_mech;

/* ------------------------------------------------------------------------ */
/* mechanism file reader                                                      */
/* ------------------------------------------------------------------------ */

static int expect_word(FILE *fp, const char *w)
{
    char buf[128];
    if (fscanf(fp, "%127s", buf) != 1) return -1;
    return strcmp(buf, w) == 0 ? 0 : -1;
}

void om_free(void *h);

/* Version 2 tail of a reaction line: reversibility flag, kind, then for a
 * fall-off reaction the low-pressure Arrhenius triple (A0 in cm-mol-s units
 * with the third body counted as a molecule), the Troe parameters a, T3, T1
 * (and T2 for troe4: the temperatures usually written with three, one and
 * two asterisks), and for every pressure-dependent kind the default
 * efficiency and the listed (species, efficiency) pairs. */
static int read_kinetics(FILE *fp, int K, om_rxn *r)
{
    char kind[16];
    int n = 0;
    if (fscanf(fp, "%d %15s", &r->rev, kind) != 2 || (r->rev != 0 && r->rev != 1)) return -1;
    if (!strcmp(kind, "elem")) r->kind = OM_ELEM;
    else if (!strcmp(kind, "third")) r->kind = OM_THIRD;
    else if (!strcmp(kind, "lind")) r->kind = OM_LIND;
    else if (!strcmp(kind, "troe3")) r->kind = OM_TROE3;
    else if (!strcmp(kind, "troe4")) r->kind = OM_TROE4;
    else return -1;
    if (r->kind == OM_ELEM) return 0;
    if (r->kind >= OM_LIND) {
        double A0;
        int order = 0;
        if (fscanf(fp, "%lf %lf %lf", &A0, &r->b0, &r->Ea0) != 3) return -1;
        for (int t = 0; t < r->nr; t++) order += r->rnu[t];
        r->A0_si = A0 * pow(1e-6, order);
    }
    if (r->kind >= OM_TROE3 && fscanf(fp, "%lf %lf %lf", &r->ta, &r->tT3, &r->tT1) != 3) return -1;
    if (r->kind >= OM_TROE3 && !(r->tT3 > 0.0 && r->tT1 > 0.0)) return -1;
    if (r->kind == OM_TROE4 && fscanf(fp, "%lf", &r->tT2) != 1) return -1;
    double def = 0.0;
    if (fscanf(fp, "%lf %d", &def, &n) != 2 || n < 0 || n > K || !(def >= 0.0)) return -1;
    r->eff = malloc((size_t)K * sizeof(double));
    if (!r->eff) return -1;
    for (int k = 0; k < K; k++) r->eff[k] = def;
    for (int j = 0; j < n; j++) {
        int k = -1;
        double e = 0.0;
        if (fscanf(fp, "%d %lf", &k, &e) != 2 || k < 0 || k >= K || !(e >= 0.0)) return -1;
        r->eff[k] = e;
    }
    return 0;
}

void *om_load(const char *path)
{
    FILE *fp = fopen(path, "r");
    if (!fp) return NULL;
    om_mech *m = calloc(1, sizeof(om_mech));
    char buf[128];
    int ver, seed, attempt;
    double aw[OM_EMAX] = {0};
    if (expect_word(fp, "CHEMMECH") || fscanf(fp, "%d", &ver) != 1 || (ver != 1 && ver != 2)) goto fail;
    if (expect_word(fp, "generator") || fscanf(fp, "%127s", buf) != 1) goto fail;
    if (expect_word(fp, "seed") || fscanf(fp, "%d", &seed) != 1) goto fail;
    if (expect_word(fp, "attempt") || fscanf(fp, "%d", &attempt) != 1) goto fail;
    if (expect_word(fp, "units")) goto fail;
    for (int i = 0; i < 6; i++)
        if (fscanf(fp, "%127s", buf) != 1) goto fail;
    if (expect_word(fp, "elements") || fscanf(fp, "%d", &m->E) != 1 || m->E < 1 || m->E > OM_EMAX) goto fail;
    for (int e = 0; e < m->E; e++)
        if (fscanf(fp, "%127s %lf", buf, &aw[e]) != 2) goto fail;
    if (expect_word(fp, "species") || fscanf(fp, "%d", &m->K) != 1 || m->K < 1 || m->K > OM_KMAX) goto fail;
    for (int k = 0; k < m->K; k++) {
        if (fscanf(fp, "%127s", buf) != 1) goto fail;
        double w = 0.0;
        for (int e = 0; e < m->E; e++) {
            if (fscanf(fp, "%d", &m->counts[k][e]) != 1 || m->counts[k][e] < 0) goto fail;
            w += m->counts[k][e] * aw[e];
        }
        m->W[k] = 1e-3 * w;
        for (int j = 0; j < 17; j++)
            if (fscanf(fp, "%lf", &m->nasa[k][j]) != 1) goto fail;
    }
    if (expect_word(fp, "reactions") || fscanf(fp, "%d", &m->R) != 1 || m->R < 0 || m->R > 1000000) goto fail;
    m->rxn = calloc(m->R > 0 ? m->R : 1, sizeof(om_rxn));
    if (!m->rxn) goto fail;
    for (int i = 0; i < m->R; i++) {
        om_rxn *r = &m->rxn[i];
        double A;
        int order = 0, sum_p = 0;
        if (fscanf(fp, "%127s %d", buf, &r->nr) != 2 || r->nr < 1 || r->nr > 2) goto fail;
        for (int t = 0; t < r->nr; t++) {
            if (fscanf(fp, "%d %d", &r->rsp[t], &r->rnu[t]) != 2) goto fail;
            if (r->rsp[t] < 0 || r->rsp[t] >= m->K || r->rnu[t] < 1 || r->rnu[t] > 2) goto fail;
            order += r->rnu[t];
        }
        if (fscanf(fp, "%d", &r->np) != 1 || r->np < 1 || r->np > 2) goto fail;
        for (int t = 0; t < r->np; t++) {
            if (fscanf(fp, "%d %d", &r->psp[t], &r->pnu[t]) != 2) goto fail;
            if (r->psp[t] < 0 || r->psp[t] >= m->K || r->pnu[t] < 1 || r->pnu[t] > 2) goto fail;
            sum_p += r->pnu[t];
        }
        if (order > 2 || sum_p > 2) goto fail; /* at most two molecules on a side */
        if (fscanf(fp, "%lf %lf %lf", &A, &r->b, &r->Ea) != 3) goto fail;
        r->dnu = sum_p - order;
        r->kind = OM_ELEM;
        r->rev = 1;
        if (ver == 2 && read_kinetics(fp, m->K, r)) goto fail;
        /* A is given in cm-mol-s units: (cm^3/mol)^(n-1)/s with n the number of
         * colliding molecules, the third body included -> SI */
        r->A_si = A * pow(1e-6, order - 1 + (r->kind == OM_THIRD));
    }
    if (expect_word(fp, "end")) goto fail;
    fclose(fp);
    return m;
fail:
    fclose(fp);
    om_free(m);
    return NULL;
}

void om_free(void *h)
{
    om_mech *m = h;
    if (!m) return;
    if (m->rxn)
        for (int i = 0; i < m->R; i++) free(m->rxn[i].eff);
    free(m->rxn);
    free(m);
}

int om_info(void *h, int *K, int *R, int *E, double *W)
{
    om_mech *m = h;
    *K = m->K;
    *R = m->R;
    *E = m->E;
    if (W)
        for (int k = 0; k < m->K; k++) W[k] = m->W[k];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* thermo, rates, right-hand side                                            */
/* ------------------------------------------------------------------------ */

/* NASA-7 polynomials: cp/R, H/(RT), S/R of every species at T. */
int om_thermo(void *h, double T, double *cp_R, double *h_RT, double *s_R)
{
    om_mech *m = h;
    for (int k = 0; k < m->K; k++) {
        const double *a = (T < m->nasa[k][1]) ? &m->nasa[k][3] : &m->nasa[k][10];
        cp_R[k] = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
        h_RT[k] = a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0
                + a[4] * T * T * T * T / 5.0 + a[5] / T;
        s_R[k] = a[0] * log(T) + a[1] * T + a[2] * T * T / 2.0 + a[3] * T * T * T / 3.0
               + a[4] * T * T * T * T / 4.0 + a[6];
    }
    return 0;
}

#define RB_NAME rhs_real
#define RB_KF kf_real
#define RB_T double
#define RB_EXP exp
#define RB_LOG log
#define RB_POW pow
#define RB_RE(x) (x)
#include "rhs_body.h"
#undef RB_NAME
#undef RB_KF
#undef RB_T
#undef RB_EXP
#undef RB_LOG
#undef RB_POW
#undef RB_RE

#define RB_NAME rhs_cplx
#define RB_KF kf_cplx
#define RB_T double complex
#define RB_EXP cexp
#define RB_LOG clog
#define RB_POW cpow
#define RB_RE(x) creal(x)
#include "rhs_body.h"

/* Rate constants, rates of progress and net production rates at (T, p, Y). */
int om_rates(void *h, double T, double p, const double *Y, double *kf, double *kr, double *q,
             double *wdot)
{
    om_mech *m = h;
    double cp_R[OM_KMAX], h_RT[OM_KMAX], s_R[OM_KMAX], C[OM_KMAX];
    om_thermo(m, T, cp_R, h_RT, s_R);
    double inv_wbar = 0.0;
    for (int k = 0; k < m->K; k++) inv_wbar += Y[k] / m->W[k];
    double rho = p / inv_wbar / (OM_RU * T);
    for (int k = 0; k < m->K; k++) {
        C[k] = rho * Y[k] / m->W[k];
        wdot[k] = 0.0;
    }
    for (int i = 0; i < m->R; i++) {
        const om_rxn *r = &m->rxn[i];
        kf[i] = kf_real(r, m->K, T, C);
        double sum_nu_g = 0.0;
        for (int t = 0; t < r->np; t++) sum_nu_g += r->pnu[t] * (h_RT[r->psp[t]] - s_R[r->psp[t]]);
        for (int t = 0; t < r->nr; t++) sum_nu_g -= r->rnu[t] * (h_RT[r->rsp[t]] - s_R[r->rsp[t]]);
        double Kc = exp(-sum_nu_g) * pow(OM_PSTD / (OM_RU * T), r->dnu);
        kr[i] = r->rev ? kf[i] / Kc : 0.0;
        double fwd = kf[i], rev = kr[i];
        for (int t = 0; t < r->nr; t++)
            for (int e = 0; e < r->rnu[t]; e++) fwd *= C[r->rsp[t]];
        for (int t = 0; t < r->np; t++)
            for (int e = 0; e < r->pnu[t]; e++) rev *= C[r->psp[t]];
        q[i] = fwd - rev;
        for (int t = 0; t < r->nr; t++) wdot[r->rsp[t]] -= r->rnu[t] * q[i];
        for (int t = 0; t < r->np; t++) wdot[r->psp[t]] += r->pnu[t] * q[i];
    }
    return 0;
}

int om_rhs(void *h, double p, const double *y, double *f)
{
    rhs_real((const om_mech *)h, p, y, f);
    return 0;
}

/* Complex-step Jacobian (Squire and Trapp 1998): df/dy_j = Im f(y + i s e_j) / s. */
int om_jac_cs(void *h, double p, const double *y, double *J)
{
    const om_mech *m = h;
    const int N = m->K + 1;
    const double s = 1e-30;
    double complex yc[OM_NMAX], fc[OM_NMAX];
    for (int j = 0; j < N; j++) {
        for (int i = 0; i < N; i++) yc[i] = y[i];
        yc[j] += s * I;
        rhs_cplx(m, p, yc, fc);
        for (int i = 0; i < N; i++) J[i * N + j] = cimag(fc[i]) / s;
    }
    return 0;
}

/* Forward rate constant with its partial derivatives: d(ln k_f)/dT at fixed
 * concentrations and d k_f / d[M] at fixed T (0 for an elementary
 * reaction).  For the fall-off forms, with x = log10 Pr, u = x + c,
 * D = n - 0.14 u, f = u / D and Lc = log10 Fcent:
 *   d ln k_f / dT = d ln k_inf/dT + (d ln Pr/dT) / (1 + Pr) + d ln F/dT,
 *   d ln Pr / dT  = d ln k_0/dT - d ln k_inf/dT,
 *   d log10 F / dx  = -Lc 2 f / (1 + f^2)^2 n / D^2,
 *   d log10 F / dLc = 1 / (1 + f^2) - Lc 2 f / (1 + f^2)^2 (1.27 u - 0.67 n) / D^2,
 *   d ln F / dT = (d log10 F/dx) d ln Pr/dT + (d log10 F/dLc) (dFcent/dT) / Fcent,
 *   d k_f / d[M] = k_0 F / (1 + Pr) (1 / (1 + Pr) + d log10 F / dx). */
static double kf_parts(const om_rxn *r, int K, double T, const double *C, double *dlnkf, double *dkfdM)
{
    const double ln10 = log(10.0), tiny = 1e-300;
    const double k = kf_real(r, K, T, C);
    const double dlnk_inf = r->b / T + r->Ea / (OM_RU * T * T);
    *dlnkf = dlnk_inf;
    *dkfdM = 0.0;
    if (r->kind == OM_ELEM) return k;
    const double kinf = r->A_si * pow(T, r->b) * exp(-r->Ea / (OM_RU * T));
    if (r->kind == OM_THIRD) {
        *dkfdM = kinf;
        return k;
    }
    double M = 0.0;
    for (int l = 0; l < K; l++) M += r->eff[l] * C[l];
    const double k0 = r->A0_si * pow(T, r->b0) * exp(-r->Ea0 / (OM_RU * T));
    const double Pr = k0 * M / kinf;
    const double dlnPr = r->b0 / T + r->Ea0 / (OM_RU * T * T) - dlnk_inf;
    double F = 1.0, dx = 0.0, dlnF = 0.0;
    if (r->kind == OM_TROE3 || r->kind == OM_TROE4) {
        double Fc = (1.0 - r->ta) * exp(-T / r->tT3) + r->ta * exp(-T / r->tT1);
        double dFc = -(1.0 - r->ta) / r->tT3 * exp(-T / r->tT3) - r->ta / r->tT1 * exp(-T / r->tT1);
        if (r->kind == OM_TROE4) {
            Fc += exp(-r->tT2 / T);
            dFc += r->tT2 / (T * T) * exp(-r->tT2 / T);
        }
        if (Fc < tiny) {
            Fc = tiny;
            dFc = 0.0;
        }
        const double Lc = log10(Fc);
        const double x = log10(Pr < tiny ? tiny : Pr);
        const double c = -0.4 - 0.67 * Lc, n = 0.75 - 1.27 * Lc;
        const double u = x + c, D = n - 0.14 * u, f = u / D;
        const double s = 1.0 + f * f;
        F = pow(10.0, Lc / s);
        dx = Pr < tiny ? 0.0 : -Lc * 2.0 * f / (s * s) * n / (D * D);
        const double dLc = 1.0 / s - Lc * 2.0 * f / (s * s) * (1.27 * u - 0.67 * n) / (D * D);
        dlnF = ln10 * (dx * dlnPr / ln10 + dLc * dFc / (Fc * ln10));
    }
    *dlnkf = dlnk_inf + dlnPr / (1.0 + Pr) + dlnF;
    *dkfdM = k0 * F / (1.0 + Pr) * (1.0 / (1.0 + Pr) + dx);
    return k;
}

/* Analytic Jacobian of the reactor right-hand side, row-major N x N.
 * Built from A = d(wdot)/dC at fixed T and d(wdot)/dT at fixed C, then the
 * chain rule through C_l = rho Y_l / W_l, rho = p Wbar / (R T). */
int om_jac(void *h, double p, const double *y, double *J)
{
    const om_mech *m = h;
    const int K = m->K, N = K + 1;
    const double T = y[K];
    double cp_R[OM_KMAX], h_RT[OM_KMAX], s_R[OM_KMAX], C[OM_KMAX], wdot[OM_KMAX];
    static __thread double A[OM_KMAX][OM_KMAX];
    double wT[OM_KMAX];
    om_thermo((void *)m, T, cp_R, h_RT, s_R);
    double inv_wbar = 0.0;
    for (int k = 0; k < K; k++) inv_wbar += y[k] / m->W[k];
    double wbar = 1.0 / inv_wbar;
    double rho = p * wbar / (OM_RU * T);
    double cp_mass = 0.0, dcp_dT = 0.0;
    for (int k = 0; k < K; k++) {
        C[k] = rho * y[k] / m->W[k];
        cp_mass += y[k] * cp_R[k] * OM_RU / m->W[k];
        const double *a = (T < m->nasa[k][1]) ? &m->nasa[k][3] : &m->nasa[k][10];
        double dcpR = a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T * T + 4.0 * a[4] * T * T * T;
        dcp_dT += y[k] * dcpR * OM_RU / m->W[k];
        wdot[k] = 0.0;
        wT[k] = 0.0;
        for (int l = 0; l < K; l++) A[k][l] = 0.0;
    }
    for (int i = 0; i < m->R; i++) {
        const om_rxn *r = &m->rxn[i];
        double dlnkf, dkfdM;
        double kf = kf_parts(r, K, T, C, &dlnkf, &dkfdM);
        double sum_nu_g = 0.0, sum_nu_h = 0.0;
        for (int t = 0; t < r->np; t++) {
            sum_nu_g += r->pnu[t] * (h_RT[r->psp[t]] - s_R[r->psp[t]]);
            sum_nu_h += r->pnu[t] * h_RT[r->psp[t]];
        }
        for (int t = 0; t < r->nr; t++) {
            sum_nu_g -= r->rnu[t] * (h_RT[r->rsp[t]] - s_R[r->rsp[t]]);
            sum_nu_h -= r->rnu[t] * h_RT[r->rsp[t]];
        }
        double Kc = exp(-sum_nu_g) * pow(OM_PSTD / (OM_RU * T), r->dnu);
        double kr = r->rev ? kf / Kc : 0.0;
        double dlnKc = sum_nu_h / T - r->dnu / T;
        double dlnkr = dlnkf - dlnKc;
        /* forward and reverse concentration products and their partials */
        double Pf = 1.0, Pr = 1.0;
        for (int t = 0; t < r->nr; t++)
            for (int e = 0; e < r->rnu[t]; e++) Pf *= C[r->rsp[t]];
        for (int t = 0; t < r->np; t++)
            for (int e = 0; e < r->pnu[t]; e++) Pr *= C[r->psp[t]];
        double q = kf * Pf - kr * Pr;
        double dq_dT = kf * Pf * dlnkf - kr * Pr * dlnkr;
        double dqdC[OM_KMAX];
        for (int l = 0; l < K; l++) dqdC[l] = 0.0;
        for (int t = 0; t < r->nr; t++) {
            /* d(prod C^nu)/dC_s = nu C_s^(nu-1) * product of the other terms */
            double d = r->rnu[t] == 2 ? 2.0 * C[r->rsp[t]] : 1.0;
            for (int u = 0; u < r->nr; u++)
                if (u != t)
                    for (int e = 0; e < r->rnu[u]; e++) d *= C[r->rsp[u]];
            dqdC[r->rsp[t]] += kf * d;
        }
        for (int t = 0; t < r->np; t++) {
            double d = r->pnu[t] == 2 ? 2.0 * C[r->psp[t]] : 1.0;
            for (int u = 0; u < r->np; u++)
                if (u != t)
                    for (int e = 0; e < r->pnu[u]; e++) d *= C[r->psp[u]];
            dqdC[r->psp[t]] -= kr * d;
        }
        /* through the third-body concentration: dq/dC_l += dkf/d[M] eff_l (Pf - Pr / Kc) */
        if (r->kind != OM_ELEM) {
            double g = dkfdM * (Pf - (r->rev ? Pr / Kc : 0.0));
            for (int l = 0; l < K; l++) dqdC[l] += g * r->eff[l];
        }
        int sp[4], nu[4], ns = 0;
        for (int t = 0; t < r->nr; t++) { sp[ns] = r->rsp[t]; nu[ns] = -r->rnu[t]; ns++; }
        for (int t = 0; t < r->np; t++) { sp[ns] = r->psp[t]; nu[ns] = r->pnu[t]; ns++; }
        for (int s = 0; s < ns; s++) {
            wdot[sp[s]] += nu[s] * q;
            wT[sp[s]] += nu[s] * dq_dT;
            for (int l = 0; l < K; l++) A[sp[s]][l] += nu[s] * dqdC[l];
        }
    }
    /* AC_k = sum_l A_kl C_l */
    double AC[OM_KMAX];
    for (int k = 0; k < K; k++) {
        AC[k] = 0.0;
        for (int l = 0; l < K; l++) AC[k] += A[k][l] * C[l];
    }
    /* species rows */
    double BT[OM_KMAX];
    for (int k = 0; k < K; k++) {
        for (int j = 0; j < K; j++) {
            double B = A[k][j] * rho / m->W[j] - (wbar / m->W[j]) * AC[k];
            J[k * N + j] = (m->W[k] / rho) * B + m->W[k] * wdot[k] * wbar / (rho * m->W[j]);
        }
        BT[k] = wT[k] - AC[k] / T;
        J[k * N + K] = (m->W[k] / rho) * BT[k] + m->W[k] * wdot[k] / (rho * T);
    }
    /* temperature row */
    double S = 0.0;
    for (int k = 0; k < K; k++) S += OM_RU * T * h_RT[k] * wdot[k];
    double rcp = rho * cp_mass;
    for (int j = 0; j < K; j++) {
        double dS = 0.0;
        for (int k = 0; k < K; k++) {
            double B = A[k][j] * rho / m->W[j] - (wbar / m->W[j]) * AC[k];
            dS += OM_RU * T * h_RT[k] * B;
        }
        double drcp = rho * OM_RU * cp_R[j] / m->W[j] - cp_mass * rho * wbar / m->W[j];
        J[K * N + j] = -dS / rcp + S * drcp / (rcp * rcp);
    }
    double dST = 0.0;
    for (int k = 0; k < K; k++) dST += OM_RU * cp_R[k] * wdot[k] + OM_RU * T * h_RT[k] * BT[k];
    double drcpT = rho * dcp_dT - cp_mass * rho / T;
    J[K * N + K] = -dST / rcp + S * drcpT / (rcp * rcp);
    return 0;
}

/* Mass-specific enthalpy (J/kg) and cp (J/(kg K)) of the mixture. */
static void mix_h_cp(const om_mech *m, double T, const double *Y, double *hmass, double *cpmass)
{
    double cp_R[OM_KMAX], h_RT[OM_KMAX], s_R[OM_KMAX];
    om_thermo((void *)m, T, cp_R, h_RT, s_R);
    double hm = 0.0, cm = 0.0;
    for (int k = 0; k < m->K; k++) {
        hm += Y[k] * OM_RU * T * h_RT[k] / m->W[k];
        cm += Y[k] * OM_RU * cp_R[k] / m->W[k];
    }
    *hmass = hm;
    *cpmass = cm;
}

double om_enthalpy(void *h, double T, const double *Y)
{
    double hm, cm;
    mix_h_cp(h, T, Y, &hm, &cm);
    return hm;
}

/* Temperature from mixture enthalpy by Newton's method on the temperature
 * polynomials (paper Section 3.1, Thermo class).  Stops when |dT| < 1e-10 K or
 * after 20 iterations (then returns NaN); T is clamped to [200, 3500] K. */
double om_T_from_h(void *h, double h0, const double *Y, double T_guess, int *iters)
{
    const om_mech *m = h;
    double T = T_guess;
    for (int it = 1; it <= 20; it++) {
        double hm, cm;
        mix_h_cp(m, T, Y, &hm, &cm);
        double dT = -(hm - h0) / cm;
        T += dT;
        if (T < 200.0) T = 200.0;
        if (T > 3500.0) T = 3500.0;
        if (fabs(dT) < 1e-10) {
            if (iters) *iters = it;
            return T;
        }
    }
    if (iters) *iters = 21;
    return NAN;
}

/* ------------------------------------------------------------------------ */
/* dense linear algebra                                                       */
/* ------------------------------------------------------------------------ */

/* LU with row partial pivoting, in place, row-major.  Pivot = largest
 * magnitude in the column at or below the diagonal; ties go to the lowest row.
 * Returns 0, or 1 if a zero pivot is met. */
int om_lu(int N, double *M, int *piv)
{
    for (int k = 0; k < N; k++) {
        int p = k;
        double best = fabs(M[k * N + k]);
        for (int r = k + 1; r < N; r++)
            if (fabs(M[r * N + k]) > best) {
                best = fabs(M[r * N + k]);
                p = r;
            }
        piv[k] = p;
        if (best == 0.0) return 1;
        if (p != k)
            for (int c = 0; c < N; c++) {
                double t = M[k * N + c];
                M[k * N + c] = M[p * N + c];
                M[p * N + c] = t;
            }
        for (int r = k + 1; r < N; r++) {
            double l = M[r * N + k] / M[k * N + k];
            M[r * N + k] = l;
            for (int c = k + 1; c < N; c++) M[r * N + c] -= l * M[k * N + c];
        }
    }
    return 0;
}

void om_lu_solve(int N, const double *LU, const int *piv, double *b)
{
    for (int k = 0; k < N; k++)
        if (piv[k] != k) {
            double t = b[k];
            b[k] = b[piv[k]];
            b[piv[k]] = t;
        }
    for (int r = 0; r < N; r++)
        for (int c = 0; c < r; c++) b[r] -= LU[r * N + c] * b[c];
    for (int r = N - 1; r >= 0; r--) {
        for (int c = r + 1; c < N; c++) b[r] -= LU[r * N + c] * b[c];
        b[r] /= LU[r * N + r];
    }
}

/* ------------------------------------------------------------------------ */
/* BDF integrator (the integrator contract)                                   */
/* ------------------------------------------------------------------------ */

#define BDF_QMAX 5
#define BDF_MAXCOR 3          /* Newton iterations per attempt */
#define BDF_MSBP 20           /* accepted steps between Newton-matrix refreshes */
#define BDF_DGMAX 0.3         /* refresh when |gamma/gamma_M - 1| exceeds this */
#define BDF_CRDOWN 0.3        /* memory of the convergence-rate estimate */
#define BDF_RDIV 2.0          /* divergence: correction grew by more than this */
#define BDF_NLSCOEF 0.1       /* Newton tolerance relative to the error-test bound */
#define BDF_MAXNEF 7          /* error-test failures on one step before giving up */
#define BDF_MAXNCF 10         /* convergence failures on one step before giving up */
#define BDF_ETACF 0.25        /* step factor after a convergence failure */
#define BDF_ETAMIN_EF 0.1     /* bounds of the step factor after an error-test failure */
#define BDF_ETAMAX_EF 0.9
#define BDF_ETA_NEF2 0.2      /* cap on the factor from the second failure on */
#define BDF_NEF_RESTART 3     /* failures after which the order restarts at 1 */
#define BDF_THRESH 1.5        /* smallest growth that changes h or q */
#define BDF_ETAMAX_FIRST 1e4  /* growth cap after the first step */
#define BDF_ETAMAX 10.0       /* growth cap otherwise */
#define BDF_BIAS_QM1 6.0
#define BDF_BIAS_Q 6.0
#define BDF_BIAS_QP1 10.0
#define BDF_ADDON 1e-6
#define BDF_H0_ITERS 4

enum { OM_OK = 0, OM_MAX_STEPS = 1, OM_ERR_FAIL = 2, OM_CONV_FAIL = 3, OM_NAN = 4 };

typedef int (*om_f_fn)(void *ctx, double t, const double *y, double *f);
typedef int (*om_j_fn)(void *ctx, double t, const double *y, double *J);

typedef struct {
    int nst, nfe, nje, nni, netf, ncfn;
} om_counts;

static double wrms(int N, const double *v, const double *w)
{
    double s = 0.0;
    for (int i = 0; i < N; i++) s += (v[i] * w[i]) * (v[i] * w[i]);
    return sqrt(s / N);
}

static int all_finite(int N, const double *v)
{
    for (int i = 0; i < N; i++)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Nordsieck array z[j][i] ~ h^j y^(j)(t) / j!, j = 0..q. */
static void nord_predict(int N, int q, double z[][OM_NMAX])
{
    /* evaluate the history polynomial and its scaled derivatives at t + h */
    for (int k = 1; k <= q; k++)
        for (int j = q; j >= k; j--)
            for (int i = 0; i < N; i++) z[j - 1][i] += z[j][i];
}

static void nord_unpredict(int N, int q, double z[][OM_NMAX])
{
    for (int k = q; k >= 1; k--)
        for (int j = k; j <= q; j++)
            for (int i = 0; i < N; i++) z[j - 1][i] -= z[j][i];
}

static void nord_rescale(int N, int q, double z[][OM_NMAX], double eta)
{
    double f = 1.0;
    for (int j = 1; j <= q; j++) {
        f *= eta;
        for (int i = 0; i < N; i++) z[j][i] *= f;
    }
}

/* Coefficients of a step of size h at order q from past step sizes tau[1..]
 * (tau[1] the most recent; 0 where no history exists, the Taylor start).
 * xi[i] = (t_new - t_{new-i}) / h for i = 1..q+1.  l[0..q] are the
 * coefficients of Lambda(x) = prod_{i=1..q} (1 + x / xi[i]); the corrected
 * polynomial interpolates the last q+1 solution values. */
void om_bdf_coeffs(int q, double h, const double *tau, double *xi, double *l)
{
    double s = h;
    xi[1] = 1.0;
    for (int i = 2; i <= q + 1; i++) {
        s += tau[i - 1];
        xi[i] = s / h;
    }
    l[0] = 1.0;
    for (int j = 1; j <= q; j++) l[j] = 0.0;
    for (int i = 1; i <= q; i++)
        for (int j = i; j >= 1; j--) l[j] += l[j - 1] / xi[i];
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= i;
    return f;
}

typedef struct {
    int N;
    om_f_fn f;
    om_j_fn jac;
    void *ctx;
    int qmax;            /* highest order the step selection may raise to (1..BDF_QMAX) */
    double *trace;       /* optional: per accepted step (t, h, q, dsm, failed attempts), at most trace_cap steps */
    int trace_cap;
    int *trace_n;
} om_problem;

/* Order change of the Nordsieck array after an accepted step (rows 0..q+1
 * used), from the step's xi and l and its correction e.
 * Down (qnew = q - 1): subtract z_q times x prod_{i=1..q-1} (x + xi_i), a
 * polynomial that vanishes at x = 0 and at the q - 1 past points x = -xi_i,
 * so the result interpolates the same values with degree q - 1.
 * Up (qnew = q + 1): add e times (x / xi_{q+1}) Lambda_q(x), Lambda_q(x) =
 * prod_{i=1..q} (1 + x / xi_i) with coefficients l, which also vanishes at x
 * = 0 and at the q past points and brings in the degree q + 1 term. */
static void order_change(int N, int q, int qnew, const double *xi, const double *l, const double *e,
                         double z[][OM_NMAX])
{
    if (qnew == q - 1) {
        double d[BDF_QMAX + 2];
        d[0] = 0.0;
        d[1] = 1.0;
        for (int j = 2; j <= q; j++) d[j] = 0.0;
        for (int i = 1; i <= q - 1; i++)
            for (int j = i + 1; j >= 1; j--) d[j] = d[j - 1] + xi[i] * d[j];
        for (int j = 1; j < q; j++)
            for (int i = 0; i < N; i++) z[j][i] -= d[j] * z[q][i];
    } else if (qnew == q + 1) {
        for (int i = 0; i < N; i++) z[q + 1][i] = 0.0;
        for (int j = 1; j <= q + 1; j++)
            for (int i = 0; i < N; i++) z[j][i] += e[i] * l[j - 1] / xi[q + 1];
    }
}

/* The order change on a flat array (rows 0..max(q, qnew), row j at
 * zflat[j * N]): the same arithmetic as inside the integrator, exposed for
 * tests of its interpolation property. */
void om_order_change(int N, int q, int qnew, const double *xi, const double *l, const double *e,
                     double *zflat)
{
    double z[BDF_QMAX + 2][OM_NMAX];
    const int rows = (qnew > q ? qnew : q) + 1;
    for (int j = 0; j < rows; j++)
        for (int i = 0; i < N; i++) z[j][i] = zflat[j * N + i];
    order_change(N, q, qnew, xi, l, e, z);
    for (int j = 0; j < rows; j++)
        for (int i = 0; i < N; i++) zflat[j * N + i] = z[j][i];
}

/* Controlled integration of y from t = 0 to t_end.  On failure y is restored
 * to its input and a non-zero status returned. */
static int bdf_integrate(const om_problem *P, double *y, double t_end, double rtol, double atol,
                         int max_steps, om_counts *cnt)
{
    const int N = P->N;
    double z[BDF_QMAX + 2][OM_NMAX];
    double y_in[OM_NMAX], w[OM_NMAX], e[OM_NMAX], ycur[OM_NMAX], fy[OM_NMAX], del[OM_NMAX];
    double ehat[OM_NMAX], ehat_new[OM_NMAX], ytmp[OM_NMAX], f1[OM_NMAX];
    static __thread double Mlu[OM_NMAX * OM_NMAX];
    int piv[OM_NMAX];
    double tau[BDF_QMAX + 3];
    double xi[BDF_QMAX + 3], l[BDF_QMAX + 2];
    memset(cnt, 0, sizeof(*cnt));
    memcpy(y_in, y, sizeof(double) * N);
    for (int i = 0; i <= BDF_QMAX + 2; i++) tau[i] = 0.0;

    /* ---- initial derivative and step size ---- */
    double t = 0.0;
    if (P->f(P->ctx, t, y, f1) || !all_finite(N, f1)) {
        cnt->nfe++;
        return OM_NAN;
    }
    cnt->nfe++;
    for (int i = 0; i < N; i++) w[i] = 1.0 / (rtol * fabs(y[i]) + atol);
    double h;
    if (wrms(N, f1, w) == 0.0) {
        h = t_end;
    } else {
        double hub = t_end;
        for (int i = 0; i < N; i++) {
            double lim = 0.1 * fabs(y[i]) + 1.0 / w[i];
            if (fabs(f1[i]) * hub > lim) hub = lim / fabs(f1[i]);
        }
        double hg = hub;
        for (int it = 0; it < BDF_H0_ITERS; it++) {
            for (int i = 0; i < N; i++) ytmp[i] = y[i] + hg * f1[i];
            int bad = P->f(P->ctx, t + hg, ytmp, fy);
            cnt->nfe++;
            if (bad || !all_finite(N, fy)) {
                hg *= 0.1;
                continue;
            }
            for (int i = 0; i < N; i++) del[i] = (fy[i] - f1[i]) / hg;
            double ydd = wrms(N, del, w);
            double hnew = ydd > 0.0 ? sqrt(2.0 / ydd) : hub;
            if (hnew > hub) hnew = hub;
            double ratio = hnew / hg;
            hg = hnew;
            if (ratio >= 0.5 && ratio <= 2.0) break;
        }
        h = 0.5 * hg;
        if (h > t_end) h = t_end;
    }
    int q = 1;
    for (int i = 0; i < N; i++) {
        z[0][i] = y[i];
        z[1][i] = h * f1[i];
    }

    int qwait = 2, have_M = 0, nst_M = 0, ehat_valid = 0;
    double gamma_M = 0.0, crate = 1.0, ehat_h = 0.0;

    while (t < t_end) {
        if (cnt->nst >= max_steps) {
            memcpy(y, y_in, sizeof(double) * N);
            return OM_MAX_STEPS;
        }
        int last = 0;
        if (t + h >= t_end) {
            double eta = (t_end - t) / h;
            nord_rescale(N, q, z, eta);
            h = t_end - t;
            last = 1;
        }
        for (int i = 0; i < N; i++) w[i] = 1.0 / (rtol * fabs(z[0][i]) + atol);
        int nef = 0, ncf = 0, force_M = 0;
        double dsm = 0.0, Cq = 0.0;
        for (;;) { /* attempts at this step */
            double tnew = t + h;
            if (tnew == t) {
                memcpy(y, y_in, sizeof(double) * N);
                return OM_ERR_FAIL;
            }
            nord_predict(N, q, z);
            om_bdf_coeffs(q, h, tau, xi, l);
            double gamma = h / l[1];
            Cq = 1.0 / (1.0 + l[1] * xi[q + 1]);
            int jcur = 0, conv = 0, lu_bad = 0;
            if (!have_M || force_M || cnt->nst >= nst_M + BDF_MSBP ||
                fabs(gamma / gamma_M - 1.0) > BDF_DGMAX) {
                P->jac(P->ctx, tnew, z[0], Mlu);
                for (int r = 0; r < N; r++)
                    for (int c = 0; c < N; c++)
                        Mlu[r * N + c] = (r == c ? 1.0 : 0.0) - gamma * Mlu[r * N + c];
                cnt->nje++;
                lu_bad = om_lu(N, Mlu, piv);
                gamma_M = gamma;
                nst_M = cnt->nst;
                crate = 1.0;
                have_M = !lu_bad;
                jcur = 1;
                force_M = 0;
            }
            if (!lu_bad) {
                double del_old = 0.0;
                for (int i = 0; i < N; i++) {
                    e[i] = 0.0;
                    ycur[i] = z[0][i];
                }
                for (int m = 0; m < BDF_MAXCOR; m++) {
                    int bad = P->f(P->ctx, tnew, ycur, fy);
                    cnt->nfe++;
                    if (bad || !all_finite(N, fy)) break;
                    for (int i = 0; i < N; i++) del[i] = -(e[i] - gamma * fy[i] + z[1][i] / l[1]);
                    om_lu_solve(N, Mlu, piv, del);
                    if (gamma != gamma_M) {
                        double s = 2.0 / (1.0 + gamma / gamma_M);
                        for (int i = 0; i < N; i++) del[i] *= s;
                    }
                    double dl = wrms(N, del, w);
                    for (int i = 0; i < N; i++) {
                        e[i] += del[i];
                        ycur[i] = z[0][i] + e[i];
                    }
                    cnt->nni++;
                    if (m > 0) {
                        double r = dl / del_old;
                        crate = BDF_CRDOWN * crate > r ? BDF_CRDOWN * crate : r;
                    }
                    double dcon = dl * (crate < 1.0 ? crate : 1.0) * Cq / BDF_NLSCOEF;
                    if (dcon <= 1.0) {
                        conv = 1;
                        break;
                    }
                    if (m > 0 && dl > BDF_RDIV * del_old) break;
                    del_old = dl;
                }
            }
            if (!conv) {
                nord_unpredict(N, q, z);
                if (!jcur) {
                    force_M = 1;
                    continue;
                }
                cnt->ncfn++;
                ncf++;
                if (ncf >= BDF_MAXNCF) {
                    memcpy(y, y_in, sizeof(double) * N);
                    return OM_CONV_FAIL;
                }
                nord_rescale(N, q, z, BDF_ETACF);
                h *= BDF_ETACF;
                last = 0;
                continue;
            }
            dsm = Cq * wrms(N, e, w);
            if (dsm > 1.0) {
                nord_unpredict(N, q, z);
                cnt->netf++;
                nef++;
                if (nef >= BDF_MAXNEF) {
                    memcpy(y, y_in, sizeof(double) * N);
                    return OM_ERR_FAIL;
                }
                last = 0;
                if (nef >= BDF_NEF_RESTART) {
                    /* restart at order 1 from a fresh derivative */
                    h *= BDF_ETAMIN_EF;
                    q = 1;
                    int bad = P->f(P->ctx, t, z[0], fy);
                    cnt->nfe++;
                    if (bad || !all_finite(N, fy)) {
                        memcpy(y, y_in, sizeof(double) * N);
                        return OM_NAN;
                    }
                    for (int i = 0; i < N; i++) z[1][i] = h * fy[i];
                    for (int i = 0; i <= BDF_QMAX + 2; i++) tau[i] = 0.0;
                    qwait = 2;
                    ehat_valid = 0;
                    continue;
                }
                double eta = 1.0 / (pow(BDF_BIAS_Q * dsm, 1.0 / (q + 1)) + BDF_ADDON);
                if (eta < BDF_ETAMIN_EF) eta = BDF_ETAMIN_EF;
                if (eta > BDF_ETAMAX_EF) eta = BDF_ETAMAX_EF;
                if (nef >= 2 && eta > BDF_ETA_NEF2) eta = BDF_ETA_NEF2;
                nord_rescale(N, q, z, eta);
                h *= eta;
                continue;
            }
            /* ---- accepted ---- */
            for (int j = 0; j <= q; j++)
                for (int i = 0; i < N; i++) z[j][i] += l[j] * e[i];
            break;
        }
        t = last ? t_end : t + h;
        cnt->nst++;
        if (P->trace && *P->trace_n < P->trace_cap) {
            double *r = P->trace + 5 * (*P->trace_n);
            r[0] = t;
            r[1] = h;
            r[2] = q;
            r[3] = dsm;
            r[4] = nef + ncf;
            (*P->trace_n)++;
        }
        if (t >= t_end) break;

        /* ---- step size and order for the next step ---- */
        double h_done = h;
        /* scaled correction: ehat ~ h^(q+1) y^(q+1) */
        double prod_q = 1.0;
        for (int i = 1; i <= q; i++) prod_q *= xi[i];
        double gfac = prod_q * (1.0 / l[1] + xi[q + 1]) / factorial(q + 1);
        for (int i = 0; i < N; i++) ehat_new[i] = e[i] / gfac;
        if (qwait > 0) qwait--;
        double etamax = (nef > 0 || ncf > 0) ? 1.0 : (cnt->nst == 1 ? BDF_ETAMAX_FIRST : BDF_ETAMAX);
        double eta = 1.0;
        int qnew = q;
        if (etamax > 1.0) {
            double eta_q = 1.0 / (pow(BDF_BIAS_Q * dsm, 1.0 / (q + 1)) + BDF_ADDON);
            eta = eta_q;
            if (qwait == 0) {
                double eta_m = 0.0, eta_p = 0.0;
                if (q > 1) {
                    double prod = 1.0, l1 = 0.0;
                    for (int i = 1; i <= q - 1; i++) {
                        prod *= xi[i];
                        l1 += 1.0 / xi[i];
                    }
                    double Em = wrms(N, z[q], w) * prod / l1;
                    eta_m = 1.0 / (pow(BDF_BIAS_QM1 * Em, 1.0 / q) + BDF_ADDON);
                }
                if (q < P->qmax && ehat_valid) {
                    double rr = pow(h_done / ehat_h, q + 1);
                    for (int i = 0; i < N; i++) del[i] = ehat_new[i] - ehat[i] * rr;
                    double prod = 1.0, l1 = 0.0;
                    for (int i = 1; i <= q + 1; i++) {
                        prod *= xi[i];
                        l1 += 1.0 / xi[i];
                    }
                    double Ep = wrms(N, del, w) * prod / (factorial(q + 2) * l1);
                    eta_p = 1.0 / (pow(BDF_BIAS_QP1 * Ep, 1.0 / (q + 2)) + BDF_ADDON);
                }
                if (eta_m > eta && eta_m >= eta_p) {
                    eta = eta_m;
                    qnew = q - 1;
                } else if (eta_p > eta) {
                    eta = eta_p;
                    qnew = q + 1;
                }
            }
            if (eta < BDF_THRESH) {
                eta = 1.0;
                qnew = q;
            } else if (eta > etamax) {
                eta = etamax;
            }
        }
        /* history of step sizes (before any order change, the new z uses it) */
        if (qnew != q) {
            order_change(N, q, qnew, xi, l, e, z);
            q = qnew;
            qwait = q + 1;
            ehat_valid = 0;
        } else {
            memcpy(ehat, ehat_new, sizeof(double) * N);
            ehat_h = h_done;
            ehat_valid = 1;
        }
        for (int i = BDF_QMAX + 1; i >= 2; i--) tau[i] = tau[i - 1];
        tau[1] = h_done;
        if (eta != 1.0) {
            nord_rescale(N, q, z, eta);
            h *= eta;
        }
    }
    for (int i = 0; i < N; i++) y[i] = z[0][i];
    if (!all_finite(N, y)) {
        memcpy(y, y_in, sizeof(double) * N);
        return OM_NAN;
    }
    return OM_OK;
}

/* ------------------------------------------------------------------------ */
/* chemistry problems and batch driver                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    const om_mech *m;
    double p;
} chem_ctx;

static int chem_f(void *ctx, double t, const double *y, double *f)
{
    (void)t;
    chem_ctx *c = ctx;
    rhs_real(c->m, c->p, y, f);
    return 0;
}

static int chem_j(void *ctx, double t, const double *y, double *J)
{
    (void)t;
    chem_ctx *c = ctx;
    om_jac((void *)c->m, c->p, y, J);
    return 0;
}

/* Integrate n cells over [0, dt].  T (n), p (n), Y (K rows of stride ldY) are
 * updated in place.  status (n) and counters (n x 6: nst nfe nje nni netf ncfn)
 * may be NULL.  qmax caps the order (1..5, anything else means 5: the
 * maximum-order option of the BDF family, Section 2's CVODE).  nthreads <= 0
 * uses every available thread.  Returns the number of threads used. */
int om_integrate(void *h, int64_t n, double *T, const double *p, double *Y, int64_t ldY, double dt,
                 double rtol, double atol, int max_steps, int qmax, int nthreads, int32_t *status,
                 int32_t *counters)
{
    const om_mech *m = h;
    const int K = m->K;
    int used = 1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    used = nthreads;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < n; i++) {
        double y[OM_NMAX];
        for (int k = 0; k < K; k++) y[k] = Y[k * ldY + i];
        y[K] = T[i];
        chem_ctx c = {m, p[i]};
        om_problem P = {K + 1, chem_f, chem_j, &c, (qmax >= 1 && qmax <= BDF_QMAX) ? qmax : BDF_QMAX};
        om_counts cnt;
        int st = bdf_integrate(&P, y, dt, rtol, atol, max_steps, &cnt);
        for (int k = 0; k < K; k++) Y[k * ldY + i] = y[k];
        T[i] = y[K];
        if (status) status[i] = st;
        if (counters) {
            int32_t *o = counters + 6 * i;
            o[0] = cnt.nst;
            o[1] = cnt.nfe;
            o[2] = cnt.nje;
            o[3] = cnt.nni;
            o[4] = cnt.netf;
            o[5] = cnt.ncfn;
        }
    }
    return used;
}

/* ------------------------------------------------------------------------ */
/* generic problems for pinning the integrator                               */
/* ------------------------------------------------------------------------ */

typedef void (*om_user_f)(double t, const double *y, double *f, void *ud);
typedef void (*om_user_j)(double t, const double *y, double *J, void *ud);

typedef struct {
    om_user_f f;
    om_user_j j;
    void *ud;
} user_ctx;

static int user_f(void *ctx, double t, const double *y, double *f)
{
    user_ctx *u = ctx;
    u->f(t, y, f, u->ud);
    return 0;
}

static int user_j(void *ctx, double t, const double *y, double *J)
{
    user_ctx *u = ctx;
    u->j(t, y, J, u->ud);
    return 0;
}

int om_bdf_user_trace(int N, om_user_f f, om_user_j j, void *ud, double *y, double t_end, double rtol,
                      double atol, int max_steps, int qmax, int32_t *counters, double *trace, int trace_cap,
                      int *trace_n);

/* Controlled integration of a user ODE y' = f(t, y) over [0, t_end], orders
 * up to qmax (1..5, anything else means 5). */
int om_bdf_user(int N, om_user_f f, om_user_j j, void *ud, double *y, double t_end, double rtol,
                double atol, int max_steps, int qmax, int32_t *counters)
{
    return om_bdf_user_trace(N, f, j, ud, y, t_end, rtol, atol, max_steps, qmax, counters, NULL, 0, NULL);
}

/* The same, recording (t, h, q, dsm, failed attempts before acceptance) of
 * every accepted step (at most trace_cap) into trace[5 * k ..]; *trace_n
 * receives the number recorded. */
int om_bdf_user_trace(int N, om_user_f f, om_user_j j, void *ud, double *y, double t_end, double rtol,
                      double atol, int max_steps, int qmax, int32_t *counters, double *trace, int trace_cap,
                      int *trace_n)
{
    user_ctx u = {f, j, ud};
    int nrec = 0;
    om_problem P = {N, user_f, user_j, &u, (qmax >= 1 && qmax <= BDF_QMAX) ? qmax : BDF_QMAX,
                    trace, trace_cap, &nrec};
    om_counts cnt;
    int st = bdf_integrate(&P, y, t_end, rtol, atol, max_steps, &cnt);
    if (trace_n) *trace_n = nrec;
    if (counters) {
        counters[0] = cnt.nst;
        counters[1] = cnt.nfe;
        counters[2] = cnt.nje;
        counters[3] = cnt.nni;
        counters[4] = cnt.netf;
        counters[5] = cnt.ncfn;
    }
    return st;
}

/* Prescribed steps at a fixed order q: no error control, Newton iterated to
 * convergence with a fresh Jacobian.  z is the Nordsieck array ((q+1) x N,
 * row j = h0^j y^(j)/j!) scaled with h0 = hseq[0]; tau[1..q+1] the past step
 * sizes (0 for a Taylor start).  On return z holds the array scaled with the
 * last step size and tau the updated history; t0 is the start time. */
int om_bdf_prescribed(int N, om_user_f f, om_user_j j, void *ud, int q, double t0, double *zflat,
                      double *tau_io, int nsteps, const double *hseq)
{
    double z[BDF_QMAX + 2][OM_NMAX], xi[BDF_QMAX + 3], l[BDF_QMAX + 2], tau[BDF_QMAX + 3];
    double e[OM_NMAX], ycur[OM_NMAX], fy[OM_NMAX], del[OM_NMAX];
    static __thread double M[OM_NMAX * OM_NMAX];
    int piv[OM_NMAX];
    for (int jj = 0; jj <= q; jj++)
        for (int i = 0; i < N; i++) z[jj][i] = zflat[jj * N + i];
    for (int i = 0; i <= BDF_QMAX + 2; i++) tau[i] = tau_io[i];
    double t = t0, h = hseq[0];
    for (int s = 0; s < nsteps; s++) {
        if (s > 0) {
            nord_rescale(N, q, z, hseq[s] / h);
            h = hseq[s];
        }
        double tnew = t + h;
        nord_predict(N, q, z);
        om_bdf_coeffs(q, h, tau, xi, l);
        double gamma = h / l[1];
        for (int i = 0; i < N; i++) {
            e[i] = 0.0;
            ycur[i] = z[0][i];
        }
        for (int it = 0; it < 50; it++) {
            f(tnew, ycur, fy, ud);
            j(tnew, ycur, M, ud);
            for (int r = 0; r < N; r++)
                for (int c = 0; c < N; c++) M[r * N + c] = (r == c ? 1.0 : 0.0) - gamma * M[r * N + c];
            if (om_lu(N, M, piv)) return 1;
            for (int i = 0; i < N; i++) del[i] = -(e[i] - gamma * fy[i] + z[1][i] / l[1]);
            om_lu_solve(N, M, piv, del);
            double mx = 0.0, sc = 0.0;
            for (int i = 0; i < N; i++) {
                e[i] += del[i];
                ycur[i] = z[0][i] + e[i];
                if (fabs(del[i]) > mx) mx = fabs(del[i]);
                if (fabs(ycur[i]) > sc) sc = fabs(ycur[i]);
            }
            if (mx <= 1e-15 * (sc + 1e-300)) break;
        }
        for (int jj = 0; jj <= q; jj++)
            for (int i = 0; i < N; i++) z[jj][i] += l[jj] * e[i];
        for (int i = BDF_QMAX + 1; i >= 2; i--) tau[i] = tau[i - 1];
        tau[1] = h;
        t = tnew;
    }
    for (int jj = 0; jj <= q; jj++)
        for (int i = 0; i < N; i++) zflat[jj * N + i] = z[jj][i];
    for (int i = 0; i <= BDF_QMAX + 2; i++) tau_io[i] = tau[i];
    return 0;
}

/* Classical fourth-order Runge-Kutta with nsteps equal steps over [0, dt]
 * (brute-force reference on mild mechanisms). */
int om_rk4(void *h, double p, double *y, double dt, int64_t nsteps)
{
    const om_mech *m = h;
    const int N = m->K + 1;
    double k1[OM_NMAX], k2[OM_NMAX], k3[OM_NMAX], k4[OM_NMAX], yt[OM_NMAX];
    double hh = dt / (double)nsteps;
    for (int64_t s = 0; s < nsteps; s++) {
        rhs_real(m, p, y, k1);
        for (int i = 0; i < N; i++) yt[i] = y[i] + 0.5 * hh * k1[i];
        rhs_real(m, p, yt, k2);
        for (int i = 0; i < N; i++) yt[i] = y[i] + 0.5 * hh * k2[i];
        rhs_real(m, p, yt, k3);
        for (int i = 0; i < N; i++) yt[i] = y[i] + hh * k3[i];
        rhs_real(m, p, yt, k4);
        for (int i = 0; i < N; i++) y[i] += hh / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    return all_finite(N, y) ? 0 : 1;
}

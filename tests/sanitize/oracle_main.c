/* Host driver of the CPU oracle, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by the sanitizer test.  With a mechanism file
 * that loads it evaluates thermodynamics, rates, the right-hand side, both
 * Jacobians, the enthalpy inversion and a short controlled integration of a
 * few cells; a damaged file must be rejected cleanly.
 *
 *   oracle_main <mech path>...    prints "ok K R E <checksum> ..." or "rejected" per file */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void *om_load(const char *path);
void om_free(void *h);
int om_info(void *h, int *K, int *R, int *E, double *W);
int om_thermo(void *h, double T, double *cp_R, double *h_RT, double *s_R);
int om_rates(void *h, double T, double p, const double *Y, double *kf, double *kr, double *q, double *wdot);
int om_rhs(void *h, double p, const double *y, double *f);
int om_jac(void *h, double p, const double *y, double *J);
int om_jac_cs(void *h, double p, const double *y, double *J);
double om_enthalpy(void *h, double T, const double *Y);
double om_T_from_h(void *h, double h0, const double *Y, double T_guess, int *iters);
int om_integrate(void *h, int64_t n, double *T, const double *p, double *Y, int64_t ldY, double dt, double rtol,
                 double atol, int max_steps, int qmax, int nthreads, int32_t *status, int32_t *counters);

static int run_one(const char *path)
{
    void *h = om_load(path);
    if (!h) {
        printf("rejected\n");
        return 0;
    }
    int K = 0, R = 0, E = 0;
    om_info(h, &K, &R, &E, NULL);
    const int N = K + 1;
    double *W = calloc((size_t)K, sizeof(double));
    double *cp = calloc((size_t)K, sizeof(double)), *hh = calloc((size_t)K, sizeof(double));
    double *ss = calloc((size_t)K, sizeof(double));
    double *kf = calloc((size_t)(R + 1), sizeof(double)), *kr = calloc((size_t)(R + 1), sizeof(double));
    double *q = calloc((size_t)(R + 1), sizeof(double)), *wd = calloc((size_t)K, sizeof(double));
    double *y = calloc((size_t)N, sizeof(double)), *f = calloc((size_t)N, sizeof(double));
    double *J = calloc((size_t)N * N, sizeof(double)), *Jc = calloc((size_t)N * N, sizeof(double));
    om_info(h, &K, &R, &E, W);
    double sum = 0.0;
    for (int i = 0; i < 3; i++) {
        om_thermo(h, 400.0 + 900.0 * i, cp, hh, ss);
        for (int k = 0; k < K; k++) sum += cp[k] + hh[k] + ss[k];
    }
    for (int k = 0; k < K; k++) y[k] = 1.0 / K;
    y[K] = 1500.0;
    om_rates(h, y[K], 101325.0, y, kf, kr, q, wd);
    om_rhs(h, 101325.0, y, f);
    om_jac(h, 101325.0, y, J);
    om_jac_cs(h, 101325.0, y, Jc);
    int it = 0;
    const double h0 = om_enthalpy(h, 1500.0, y);
    const double T = om_T_from_h(h, h0, y, 1000.0, &it);
    for (int i = 0; i < N; i++) sum += isfinite(f[i]) ? f[i] * 1e-12 : 0.0;
    double jd = 0.0;
    for (int i = 0; i < N * N; i++) jd = fmax(jd, fabs(J[i] - Jc[i]) / (fabs(Jc[i]) + 1.0));
    enum { CELLS = 4 };
    double Tc[CELLS], pc[CELLS];
    double *Y = calloc((size_t)K * CELLS, sizeof(double));
    int32_t st[CELLS], cnt[6 * CELLS];
    for (int c = 0; c < CELLS; c++) {
        Tc[c] = 1000.0 + 300.0 * c;
        pc[c] = 101325.0;
        for (int k = 0; k < K; k++) Y[(size_t)k * CELLS + c] = 1.0 / K;
    }
    om_integrate(h, CELLS, Tc, pc, Y, CELLS, 1e-7, 1e-6, 1e-10, 2000, 5, 1, st, cnt);
    for (int c = 0; c < CELLS; c++) sum += isfinite(Tc[c]) ? Tc[c] : 0.0;
    printf("ok %d %d %d %.6e jac_dev=%.3e T=%.6f\n", K, R, E, sum, jd, T);
    free(W), free(cp), free(hh), free(ss), free(kf), free(kr), free(q), free(wd);
    free(y), free(f), free(J), free(Jc), free(Y);
    om_free(h);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    for (int i = 1; i < argc; i++) run_one(argv[i]);
    return 0;
}

/*
 * chem.h - C ABI of the MI355X (gfx950) per-cell stiff chemistry library.
 *
 * The operation: every CFD cell is advanced over one flow step dt as an
 * adiabatic, constant-pressure reactor (paper Section 2: the chemical source
 * of each cell is integrated as a stiff ODE, CVODE on the CPU path; Section
 * 3.1: after initialisation all time advancement stays on the GPU, with no
 * host-device copies inside a step).  State per cell: T (K), p (Pa), mass
 * fractions Y_1..Y_K.  Kinetics: elementary reversible reactions with
 * Arrhenius forward rates and reverse rates from the equilibrium constant of
 * NASA-7 thermo.  Integrator: variable-order (1..5) variable-step BDF in
 * Nordsieck form with modified Newton, the method family of CVODE.
 *
 * Conventions for every entry point:
 *  - Return 0 on success or a negative CHEM_E* code; chem_last_error() then
 *    returns a thread-local message.
 *  - Array arguments are DEVICE pointers owned by the caller (e.g. torch
 *    tensors on the current HIP device).  State arrays are updated in place.
 *  - Species arrays are structure-of-arrays: Y[k * ldY + i] for species k of
 *    cell i, with ldY >= ncells.
 *  - hip_stream is a hipStream_t (NULL = default stream).  Calls only enqueue
 *    work on that stream: no host synchronisation and no allocation, so they
 *    may be captured in a HIP graph.  Workspace is allocated at mechanism load.
 *  - Per-cell numerical failures are not call errors: they are reported in
 *    status[] and the failed cell keeps its input state.
 */
#ifndef CHEM_H
#define CHEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHEM_OK 0
#define CHEM_EINVAL -1   /* bad argument, shape or option */
#define CHEM_ENOMEM -2   /* device allocation failed */
#define CHEM_EHIP -3     /* HIP runtime error */
#define CHEM_EMECH -4    /* mechanism file unreadable or invalid */
#define CHEM_EUNSUP -5   /* mechanism size or option not supported by any kernel */

/* Per-cell status codes written to status[]. */
#define CHEM_CELL_OK 0
#define CHEM_CELL_MAX_STEPS 1   /* max_steps accepted steps without reaching dt */
#define CHEM_CELL_ERR_FAIL 2    /* error test failed repeatedly or h underflowed */
#define CHEM_CELL_CONV_FAIL 3   /* Newton iteration failed repeatedly */
#define CHEM_CELL_NAN 4         /* non-finite right-hand side or result */

/* Per-cell counters, written as rows of counters[c * ncells + i]. */
#define CHEM_CNT_STEPS 0        /* accepted BDF steps */
#define CHEM_CNT_RHS 1          /* right-hand-side evaluations */
#define CHEM_CNT_JAC 2          /* Jacobian evaluations = LU factorisations */
#define CHEM_CNT_NEWTON 3       /* Newton iterations */
#define CHEM_CNT_ERRFAIL 4      /* error-test failures */
#define CHEM_CNT_CONVFAIL 5     /* Newton convergence failures */
#define CHEM_NCOUNTERS 6

typedef struct chem_mech_s *chem_mech;

typedef struct {
    double rtol;        /* relative tolerance (default 1e-8) */
    double atol;        /* absolute tolerance, all components (default 1e-12) */
    int32_t max_steps;  /* accepted steps per cell per call (default 20000) */
    int32_t precision;  /* 0 = FP64 throughout; 1 = Jacobian, Newton matrix, LU
                           factors and triangular solves in FP32, while residuals,
                           state, norms, error control and equilibrium constants
                           stay FP64 (wave schedule only; results then differ
                           from FP64 at the level of the integration tolerance) */
    int32_t schedule;   /* -1 = library choice (one thread per cell when such a
                           kernel exists and precision is 0, else one wave per
                           cell), 0 = one thread per cell (K <= 9 table kernel or
                           a compiled-in mechanism), 1 = one 64-lane wave per
                           cell (any K <= 63).  CHEM_EUNSUP when the chosen
                           schedule cannot serve the mechanism or precision. */
    int32_t block;      /* threads per block, 0 = library choice */
    int32_t jac_batch;  /* one-thread-per-cell kernels: lanes of a wave that wait for
                           a new Newton matrix before the Jacobian is evaluated
                           (1..64; 0 = library choice).  Scheduling only: results
                           do not depend on it. */
    int32_t reserved[7];
} chem_opts;

/* Fill opts with the defaults above. */
int chem_default_opts(chem_opts *opts);

/* Read a .mech file (format "CHEMMECH 1": elements with atomic weights,
 * species with element counts and two NASA-7 ranges, reactions with <= 2
 * reactant and <= 2 product molecules, A in cm-mol-s units, b, Ea in J/mol),
 * validate it (element balance, indices, finite coefficients) and upload its
 * tables to `device`.  The handle owns its device memory; it is immutable
 * after loading and may be used from several streams of that device. */
int chem_load_mechanism(const char *path, int device, chem_mech *out);
void chem_free_mechanism(chem_mech mech);
/* Number of species, reactions, elements; W (may be NULL) receives the K
 * species molar masses in kg/mol (host memory). */
int chem_mechanism_info(chem_mech mech, int32_t *K, int32_t *R, int32_t *E, double *W);

/* Which kernels serve this mechanism: "specialised:<tag>" when the file was
 * compiled into the library by the mechanism compiler (straight-line
 * right-hand side and Jacobian), "table" for the table-driven kernels.
 * The string is owned by the handle. */
const char *chem_mechanism_variant(chem_mech mech);

/* Advance ncells cells over [0, dt] in place.
 *   T[ncells]            temperature, K (in/out)
 *   p[ncells]            pressure, Pa (in), constant over the step
 *   Y[K * ldY]           mass fractions (in/out)
 *   status[ncells]       per-cell CHEM_CELL_* code (out, may be NULL)
 *   counters[6*ncells]   per-cell CHEM_CNT_* rows (out, may be NULL)
 * ncells == 0 is a no-op.  dt must be finite and > 0. */
int chem_integrate(chem_mech mech, double *T, const double *p, double *Y, int64_t ldY,
                   int64_t ncells, double dt, const chem_opts *opts, int32_t *status,
                   int32_t *counters, void *hip_stream);

/* Right-hand side of the reactor ODE at the given states (diagnostics and
 * parity tests of the kernels' building blocks).  F has N = K+1 rows of
 * stride ldF (rows 0..K-1: dY_k/dt in 1/s, row K: dT/dt in K/s). */
int chem_eval_rhs(chem_mech mech, const double *T, const double *p, const double *Y, int64_t ldY,
                  int64_t ncells, double *F, int64_t ldF, void *hip_stream);

/* Analytic Jacobian d f / d y of the same ODE, y = (Y_1..Y_K, T): element
 * (r, c) of cell i at J[(r * N + c) * ldJ + i]. */
int chem_eval_jacobian(chem_mech mech, const double *T, const double *p, const double *Y,
                       int64_t ldY, int64_t ncells, double *J, int64_t ldJ, void *hip_stream);

/* Thread-local description of the last error (never NULL). */
const char *chem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CHEM_H */

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
 *    work on that stream: no host synchronisation, so they may be captured in
 *    a HIP graph (paper Section 3.2: one graph launch per time step).
 *    Workspace is allocated at mechanism load, or grown by the first call of
 *    a given size on a stream; a call that would have to grow it while the
 *    stream is being captured fails with CHEM_EINVAL (make the same call
 *    eagerly first); chem_integrate_noalloc never allocates.
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
                           stay FP64 (wave and tile schedules; results then
                           differ from FP64 at the level of the integration
                           tolerance) */
    int32_t schedule;   /* -2 = the autotuned choice (chem_autotune), else as -1;
                           -1 = library choice (one thread per cell for a
                           compiled-in mechanism in FP64, else the tile schedule
                           when K <= 15, else one wave per cell), 0 = one thread per cell
                           (FP64 only; a compiled-in mechanism: its straight-line
                           kernels keep a cell's state in registers and LDS,
                           which table-driven kernels cannot do without
                           spilling), 1 = one 64-lane wave per
                           cell (any K <= 63), 2 = tile: 16 lanes per cell, four
                           cells per wave (K <= 15; the same operations per
                           cell as 1).  CHEM_EUNSUP when the chosen schedule
                           cannot serve the mechanism or precision. */
    int32_t block;      /* threads per block, 0 = library choice */
    int32_t jac_batch;  /* one-thread-per-cell kernels: lanes of a wave that wait for
                           a new Newton matrix before the Jacobian is evaluated
                           (1..64; 0 = library choice).  Scheduling only: results
                           do not depend on it. */
    int32_t qmax;       /* highest BDF order the step selection may raise to,
                           1..5 (0 = 5, the default method) */
    int32_t waves_per_simd; /* at most this many waves of the integrator per
                           SIMD (a cap on the persistent grid; 0 = as many as
                           fit).  Scheduling only: results do not depend on it. */
    int32_t reserved[5];
} chem_opts;

/* Fill opts with the defaults above (rtol, atol and the BDF limits of the
 * paper's CVODE method, Section 2). */
int chem_default_opts(chem_opts *opts);

/* Read a .mech file (format "CHEMMECH 1": elements with atomic weights,
 * species with element counts and two NASA-7 ranges, reactions with <= 2
 * reactant and <= 2 product molecules, A in cm-mol-s units, b, Ea in J/mol),
 * validate it (element balance, indices, finite coefficients) and upload its
 * tables to `device` (paper Section 3.2: the constant coefficients of the
 * property kernels live in fast read-only memory; here one device block that
 * the kernels copy into LDS).  The handle owns its device memory; it is
 * immutable after loading and may be used from several streams of that
 * device. */
int chem_load_mechanism(const char *path, int device, chem_mech *out);
void chem_free_mechanism(chem_mech mech);
/* Number of species, reactions, elements; W (may be NULL) receives the K
 * species molar masses in kg/mol (host memory; the mechanism of Section 2's
 * detailed kinetics). */
int chem_mechanism_info(chem_mech mech, int32_t *K, int32_t *R, int32_t *E, double *W);

/* Which kernels serve this mechanism: "specialised:<tag>" when the file was
 * compiled into the library by the mechanism compiler (straight-line
 * right-hand side and Jacobian: the coefficients in the instruction stream,
 * Section 3.2's constant-memory placement taken one step further), "table"
 * for the table-driven kernels.  The string is owned by the handle. */
const char *chem_mechanism_variant(chem_mech mech);

/* Advance ncells cells over [0, dt] in place (the per-cell chemistry source
 * of one flow step, integrated as a stiff ODE: paper Section 2, CVODE's
 * variable-order BDF method; Section 3.1, the chemistry of every cell on the
 * GPU).
 *   T[ncells]            temperature, K (in/out)
 *   p[ncells]            pressure, Pa (in), constant over the step
 *   Y[K * ldY]           mass fractions (in/out)
 *   status[ncells]       per-cell CHEM_CELL_* code (out, may be NULL)
 *   counters[6*ncells]   per-cell CHEM_CNT_* rows (out, may be NULL)
 * ncells == 0 is a no-op.  dt must be finite and > 0. */
int chem_integrate(chem_mech mech, double *T, const double *p, double *Y, int64_t ldY,
                   int64_t ncells, double dt, const chem_opts *opts, int32_t *status,
                   int32_t *counters, void *hip_stream);

/* chem_integrate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and kernels as chem_integrate, but the
 * one-thread-per-cell schedule keeps its per-call start-pass workspace (f(y0),
 * initial step and cost order of every cell, (8 K + 28) bytes per cell) in a
 * fixed array of 32 MiB that the library holds on each GPU until the process
 * ends, instead of a workspace it grows; the call makes no hipMalloc or
 * hipFree.  That schedule then serves every call of up to
 * floor((2^25 - 1276) / (8 K + 28)) cells (335,531 for K = 9; the exact
 * bound, set by 256-byte alignment of the pieces, is a few cells higher);
 * a call beyond the array fails with CHEM_EINVAL and a message giving the
 * limit.  Every call on one GPU shares that GPU's array, so calls that
 * overlap in time on one GPU (different streams) race: order them.  The
 * other schedules use no such workspace and behave as in chem_integrate. */
int chem_integrate_noalloc(chem_mech mech, double *T, const double *p, double *Y, int64_t ldY,
                           int64_t ncells, double dt, const chem_opts *opts, int32_t *status,
                           int32_t *counters, void *hip_stream);

/* Advance the listed cells only, in list order: work item j integrates cell
 * cell_idx[j] of the arrays (sizes as chem_integrate; status and counters,
 * if given, are indexed by cell).  cell_idx is a device array of nidx
 * indices; an index outside [0, ncells) is skipped.  On the wave and tile
 * schedules the list order is the order in which the work queue hands cells
 * to the lanes (e.g. from chem_lpt_order); the one-thread-per-cell schedule
 * orders the listed cells itself, most costly first by its start pass.
 * Results per cell do not depend on the order.  nidx == 0 is a no-op. */
int chem_integrate_indexed(chem_mech mech, double *T, const double *p, double *Y, int64_t ldY,
                           int64_t ncells, const int32_t *cell_idx, int64_t nidx, double dt,
                           const chem_opts *opts, int32_t *status, int32_t *counters,
                           void *hip_stream);

/* Totals of one integration (or inference) call, reduced on the device from
 * its per-cell outputs. */
typedef struct {
    int64_t cells;            /* cells reduced (n) */
    int64_t steps_total;      /* accepted steps, summed over cells */
    int64_t rejects;          /* error-test plus Newton convergence failures */
    int64_t newton_iters;     /* Newton iterations */
    int64_t jac_evals;        /* Jacobian evaluations (= LU factorisations) */
    int64_t rhs_evals;        /* right-hand-side evaluations */
    int64_t fallback_cells;   /* *fallback_count when given, else 0 */
    int32_t steps_max;        /* largest per-cell step count */
    int32_t reserved;
    int64_t status_count[8];  /* cells per status code 0..7 (CHEM_CELL_*) */
} chem_stats;

/* Per-call statistics (the work behind Table 1's chemistry time: steps,
 * rejections, Newton iterations, Jacobians, fallback cells).
 * Reduce the per-cell outputs of a call: status[n] (device, may be NULL)
 * and counters[6][n] (device, layout of chem_integrate; may be NULL) into
 * *out (host), plus the fallback count of chem_surrogate_infer (device, may
 * be NULL).  A diagnostics call: allocates a small device buffer, enqueues
 * the reduction on the stream, synchronises the stream and copies the
 * totals back.  Integer sums, so the result does not depend on the order of
 * the reduction.  A status outside 0..7 is counted in status_count[7]. */
int chem_get_stats(const int32_t *status, const int32_t *counters, int64_t n, const int64_t *fallback_count,
                   chem_stats *out, void *hip_stream);

/* Load balance across uneven per-cell stiffness (the chemistry is
 * communication-free per cell, Section 1; its cost per cell varies by
 * orders of magnitude between cold and flame-front cells).
 * Longest-processing-time-first order: order[0..n) (device) receives the
 * indices 0..n-1 sorted by descending cost[i] (device int32, e.g. the step
 * counts of the previous flow step), ties in index order.  A planning call:
 * allocates temporary device memory and synchronises the stream. */
int chem_lpt_order(const int32_t *cost, int64_t n, int32_t *order, void *hip_stream);

/* Launch configuration chosen by measurement (Section 3.2: optimisations of
 * the kernels and of their launch).
 * Autotuner: times every configuration that can serve the mechanism at
 * opts->precision -- one thread per cell (compiled-in mechanisms, FP64) with
 * jac_batch 4, 16, 64; one wave per cell and the 16-lane tile (K <= 15),
 * each at the most waves per SIMD that fit and at one, in natural and in
 * LPT order -- twice each on a strided sample of at most max_sample cells
 * (0 = 262,144, four cells per lane of a full device for the thread
 * schedule; the whole field when it is smaller) of the given states (not
 * modified), and returns the fastest as *best (schedule, jac_batch,
 * waves_per_simd filled in), *use_lpt (1 if the LPT order was faster) and
 * *best_ms.  The choice is kept in the handle per precision and per
 * size class floor(log2(ncells)); opts.schedule = -2 selects the choice of
 * the call's size class (else of the nearest tuned one).  With the
 * environment variable CHEM_TUNE_CACHE naming a file, every result is also
 * appended there as a text line (GPU architecture, mechanism file hash,
 * species count, precision, size class, choice, time) and loading the same
 * mechanism file on the same architecture restores it.  chem_autotune_results
 * copies the measured table of the handle's last chem_autotune (at most
 * capacity entries, host memory; *count = the number measured).  Allocates
 * and synchronises: a planning call, not for a capture. */
typedef struct {
    int32_t schedule, jac_batch, lpt, waves_per_simd;
    double ms;          /* fastest of the two timed runs, HIP events */
} chem_tune_entry;
int chem_autotune(chem_mech mech, const double *T, const double *p, const double *Y, int64_t ldY,
                  int64_t ncells, double dt, const chem_opts *base, int32_t max_sample, chem_opts *best,
                  int32_t *use_lpt, double *best_ms, void *hip_stream);
int chem_autotune_results(chem_mech mech, chem_tune_entry *out, int32_t capacity, int32_t *count);

/* Right-hand side of the reactor ODE at the given states (Section 2's
 * species and temperature equations; diagnostics and parity tests of the
 * kernels' building blocks).  F has N = K+1 rows of
 * stride ldF (rows 0..K-1: dY_k/dt in 1/s, row K: dT/dt in K/s). */
int chem_eval_rhs(chem_mech mech, const double *T, const double *p, const double *Y, int64_t ldY,
                  int64_t ncells, double *F, int64_t ldF, void *hip_stream);

/* Analytic Jacobian d f / d y of the same ODE (the Newton matrix of the
 * implicit BDF method, Section 2), y = (Y_1..Y_K, T): element
 * (r, c) of cell i at J[(r * N + c) * ldJ + i]. */
int chem_eval_jacobian(chem_mech mech, const double *T, const double *p, const double *Y,
                       int64_t ldY, int64_t ncells, double *J, int64_t ldJ, void *hip_stream);

/* Thread-local description of the last error (never NULL). */
const char *chem_last_error(void);

/* ------------------------------------------------------------------------
 * Learned surrogate (paper Section 2: a DNN predicts the chemical source of
 * every cell from its temperature, pressure and mass fractions; Sections 3.1
 * and 3.2: the network runs on the GPU with its input and output kept in
 * device memory; training uses Adam and GELU activations).
 *
 * Network: x = zscore([T, p, BoxCox(max(Y,0); 0.1)]) (K + 2 inputs, padded to
 * 64), three GELU hidden layers of h1, h2, h3 units (multiples of 64;
 * 512/256/128 in the reference configuration), output the z-scored change
 * of the K mass fractions over one flow step dt.  Weights and activations
 * BF16, accumulation and biases FP32 (MFMA), Adam on FP32 master weights.
 *
 * Logical parameter vector (set/get/grad), FP32, in this order:
 *   W1[h1][K+2], b1[h1], W2[h2][h1], b2[h2], W3[h3][h2], b3[h3], W4[K][h3], b4[K]
 * (row-major, out x in).  Normalisation vector, FP64:
 *   mu_x[K+2], sig_x[K+2], mu_y[K], sig_y[K], dt
 * (features with sig < 1e-12 map to 0; dt is the flow step the network was
 * trained for).
 *
 * A surrogate handle refers to its mechanism, which must outlive it.  The
 * surrogate grows workspace on first use (chem_surrogate_infer at a given
 * ncells) or through chem_surrogate_reserve; later calls of at most that
 * size neither allocate nor synchronise and may be captured in a HIP graph.
 * A call that would have to grow the workspace while its stream is being
 * captured fails with CHEM_EINVAL instead; buffers replaced by growth stay
 * allocated until the handle is freed, so graphs captured earlier stay
 * valid.  The workspace belongs to the handle: calls on one surrogate
 * handle must not overlap (issue them on one stream, or order them).
 * ------------------------------------------------------------------------ */
typedef struct chem_surr_s *chem_surr;

/* Acceptance checks of a predicted cell; a cell failing any of them is
 * integrated instead (per-cell fallback). */
typedef struct {
    double elem_tol;    /* max_e |sum_k n_ke (Y'-Y)_k/W_k| / max(sum_k n_ke Y_k/W_k, 1e-12) (1e-3) */
    double sum_tol;     /* |sum Y' - 1| (1e-3); then Y' is clipped at 0 and renormalised */
    double neg_tol;     /* Y'_k >= -neg_tol (1e-6) */
    double T_out_min, T_out_max;   /* recovered temperature range (250, 2600 K) */
    double T_in_min, T_in_max;     /* input temperature inside the training box (300, 2500 K) */
    double dT_gate;     /* |T' - T| <= dT_gate when > 0 (0 = off) */
    int32_t reserved[8];
} chem_surr_checks;

int chem_surrogate_default_checks(chem_surr_checks *checks);

/* New surrogate for mech (Section 2's network, hidden widths h1, h2, h3)
 * with zero parameters and unset normalisation. */
int chem_surrogate_create(chem_mech mech, int32_t h1, int32_t h2, int32_t h3, chem_surr *out);
/* The paper's per-species variant (Section 2: one network per species, each
 * with its own hidden layers h1, h2, h3 (the paper's are 1600, 800, 400) and
 * a single output, all fed the same encoded input): K networks, species k's
 * output in column k of the output rows, so encode, apply, infer, grad, adam
 * and train work unchanged.  Stored as one network whose first layer stacks
 * the K first layers and whose later layers are block diagonal; only the
 * diagonal blocks are stored and multiplied (grouped BF16 MFMA products, one
 * group per species).  Parameters in logical order network by network (each
 * W1, b1, W2, b2, W3, b3, W4 (1 x h3), b4 (1)).  Inference runs the layered
 * products (no fused kernel).  The weights file holds one network:
 * chem_surrogate_save and _save_checkpoint return CHEM_EUNSUP for it.
 * Widths 16 .. 4096, each padded to a multiple of 64 with units whose
 * weights and biases stay zero; K * (padded h_l) <= 65536.
 * chem_surrogate_info reports the padded totals K * padded h_l. */
int chem_surrogate_create_species(chem_mech mech, int32_t h1, int32_t h2, int32_t h3, chem_surr *out);
/* *groups = 1 for one network, K for the per-species networks. */
int chem_surrogate_groups(chem_surr surr, int32_t *groups);
void chem_free_surrogate(chem_surr surr);
/* dims[0..5] = K+2, h1, h2, h3, K, number of logical parameters. */
int chem_surrogate_info(chem_surr surr, int64_t *dims);
/* Host FP32 logical parameter vector in / out (count must match). */
int chem_surrogate_set_params(chem_surr surr, const float *params, int64_t count);
int chem_surrogate_get_params(chem_surr surr, float *params, int64_t count);
/* Host FP64 normalisation vector in / out (2 (K+2) + 2 K + 1 values). */
int chem_surrogate_set_norm(chem_surr surr, const double *norm, int64_t count);
int chem_surrogate_get_norm(chem_surr surr, double *norm, int64_t count);
/* Input/output scaling of the network (Section 2's inputs T, p, Y).
 * Normalisation from training samples (device): states T, p, Y and the mass
 * fractions Ynext[k * ldYn + i] of the same cells one flow step dt later.
 * Population mean and standard deviation of each feature and of each
 * dY_k = Ynext_k - Y_k.  Synchronises the stream. */
int chem_surrogate_fit_norm(chem_surr surr, const double *T, const double *p, const double *Y,
                            int64_t ldY, const double *Ynext, int64_t ldYn, int64_t n, double dt,
                            void *hip_stream);
/* Network input of n cells (Section 2: temperature, pressure and mass
 * fractions): X[i * 64 + j] BF16 bit patterns (device, n x 64). */
int chem_surrogate_encode(chem_surr surr, const double *T, const double *p, const double *Y,
                          int64_t ldY, int64_t n, uint16_t *X, void *hip_stream);
/* Network output for n encoded rows (Section 2: three GELU hidden layers;
 * Section 3.1: inference on the GPU): out[i * ldo + k], k < K (device FP32,
 * ldo >= K rounded up to 16; columns K..ldo-1 are written with the padding
 * outputs). */
int chem_surrogate_forward(chem_surr surr, const uint16_t *X, int64_t n, float *out, int64_t ldo,
                           void *hip_stream);
/* The same with a choice of kernels: path 0 = library choice (as
 * chem_surrogate_forward), 1 = one GEMM per layer with the activations in
 * device memory, 2 = the fused kernel (all layers per 32-row block, activations
 * in LDS; CHEM_EUNSUP unless every width is <= 512).  Paths 1 and 2 give the
 * same output bit for bit (same MFMA accumulation order, same epilogues). */
int chem_surrogate_forward_path(chem_surr surr, const uint16_t *X, int64_t n, float *out, int64_t ldo,
                                int32_t path, void *hip_stream);
/* Size the inference workspace for calls of up to ncells cells (the same
 * allocation the first chem_surrogate_infer of that size makes), so that
 * such calls can then be captured.  Not capturable itself. */
int chem_surrogate_reserve(chem_surr surr, int64_t ncells, void *hip_stream);
/* Rows per inference pass of chem_surrogate_infer (encode, network, decode
 * and checks run pass by pass over the cells): 0 = the library's choice
 * (2,097,152 rows with the fused forward, 262,144 with the per-layer GEMMs);
 * a smaller value caps it.  Results do not depend on it. */
int chem_surrogate_set_pass_rows(chem_surr surr, int64_t rows);
/* The per-layer path (path 1) with its hidden activations kept: H1, H2, H3
 * (device, n x h1, n x h2, n x h3 BF16 bit patterns, row-major) receive the
 * BF16 outputs of the three GELU layers and out the network output, as
 * chem_surrogate_forward_path writes it.  A diagnostics call for layer-wise
 * checks of the kernels; n <= 2^20. */
int chem_surrogate_forward_trace(chem_surr surr, const uint16_t *X, int64_t n, uint16_t *H1, uint16_t *H2,
                                 uint16_t *H3, float *out, int64_t ldo, void *hip_stream);
/* Decode, temperature recovery and checks (Section 3.1: the temperature
 * follows from the enthalpy by Newton's method on the temperature
 * polynomials) of n cells from a network output
 * (device, layout of chem_surrogate_forward): accepted cells take the
 * prediction in place, mask[i] = 1 marks the rejected ones (their state is
 * unchanged).  No integration. */
int chem_surrogate_apply(chem_surr surr, double *T, const double *p, double *Y, int64_t ldY,
                         int64_t n, const float *out, int64_t ldo, const chem_surr_checks *checks,
                         int32_t *mask, void *hip_stream);
/* The DNN chemistry of one flow step (Section 2 option 2; Table 1's GPU
 * chemistry), with per-cell fallback to the integrator (Section 2 option 1).
 * One flow step of n cells by the surrogate with per-cell fallback: encode,
 * network, decode and checks; rejected cells are integrated by
 * chem_integrate (opts) over dt.  mask (nullable): 1 for fallback cells.
 * status (nullable): integrator status of fallback cells, 0 elsewhere.
 * fallback_count (nullable, device int64): number of fallback cells.
 * dt must equal the dt of the normalisation.  The cells run in passes; the
 * rejected cells of each pass are integrated on the handle's own second
 * stream (default priority) while the later passes run, joined back into
 * hip_stream by events before the call's last kernel, so the call stays
 * asynchronous and capturable. */
int chem_surrogate_infer(chem_surr surr, double *T, const double *p, double *Y, int64_t ldY,
                         int64_t n, double dt, const chem_opts *opts,
                         const chem_surr_checks *checks, int32_t *mask, int32_t *status,
                         int64_t *fallback_count, void *hip_stream);
/* Training building blocks (Section 2: the network is trained with Adam).
 * Loss and parameter gradient of one batch: X (device, n x 64 BF16 rows as
 * from chem_surrogate_encode), targets Yt[i * ldt + k] (device FP32 z-scored
 * dY, ldt >= K).  Loss = mean over the n x K entries of (out - Yt)^2; the
 * gradient is kept inside the handle.  *loss is written (host).  Synchronises. */
int chem_surrogate_grad(chem_surr surr, const uint16_t *X, const float *Yt, int64_t ldt, int64_t n,
                        double *loss, void *hip_stream);
/* The handle's gradient as a host logical vector, or replaced by one. */
int chem_surrogate_get_grads(chem_surr surr, float *grads, int64_t count);
int chem_surrogate_set_grads(chem_surr surr, const float *grads, int64_t count);
/* One Adam step (beta 0.9, 0.999, eps 1e-8, bias corrected) with the handle's
 * gradient and learning rate lr; the step counter is kept in the handle. */
int chem_surrogate_adam(chem_surr surr, double lr, void *hip_stream);
/* Training (Section 2: GELU network trained with Adam on states labelled by
 * the integrator): encodes the n samples (states T, p, Y and Ynext one flow step of
 * the normalisation's dt later, device; the target is the z-scored
 * Ynext - Y), then `epochs` passes of minibatches of `batch`
 * rows in the sample order order[e * n + i] (device int32, NULL = 0..n-1 every
 * epoch), each: forward, MSE loss, backward, Adam with a cosine learning rate
 * from lr0 to lr1 over all minibatches.  loss_per_epoch (host, nullable)
 * receives the mean loss of each epoch.  Allocates its own buffers and
 * synchronises. */
int chem_surrogate_train(chem_surr surr, const double *T, const double *p, const double *Y,
                         int64_t ldY, const double *Ynext, int64_t ldYn, int64_t n,
                         const int32_t *order, int32_t epochs, int32_t batch, double lr0,
                         double lr1, double *loss_per_epoch, void *hip_stream);
/* Part of a training run (resume after a checkpoint): epochs
 * [first_epoch, first_epoch + epochs) of a run of total_epochs, with the
 * cosine learning rate taken over the whole run, so that a run cut into parts
 * (with the optimiser state kept, in the handle or through a checkpoint file)
 * takes exactly the steps of the uncut run.  order holds the `epochs` orders
 * of this part (order[(e - first_epoch) * n + i]); the rest as
 * chem_surrogate_train, which is the part (0, epochs, epochs). */
int chem_surrogate_train_part(chem_surr surr, const double *T, const double *p, const double *Y,
                              int64_t ldY, const double *Ynext, int64_t ldYn, int64_t n,
                              const int32_t *order, int32_t first_epoch, int32_t epochs,
                              int32_t total_epochs, int32_t batch, double lr0, double lr1,
                              double *loss_per_epoch, void *hip_stream);
/* Weights file (the trained network the paper's inference loads, Section
 * 3.1): magic, version, dimensions, normalisation, FP32 parameters in logical
 * order, FNV-1a checksum.  chem_surrogate_save writes version 1 (no training
 * state); chem_surrogate_save_checkpoint writes version 2, which adds the
 * Adam step and both moment vectors and user_bytes (0..2^20) of the caller's
 * own data (host memory: the state of the generator of its sample orders).
 * chem_surrogate_load reads either version (a version 2 file restores the
 * optimiser state too) and rejects a file whose checksum, sizes or dimensions
 * do not agree or whose species count is not the mechanism's.
 * chem_surrogate_checkpoint_user copies a version 2 file's user bytes into
 * user (host, capacity bytes) and their count into *user_bytes; CHEM_EINVAL
 * (with *user_bytes set) when they do not fit. */
int chem_surrogate_save(chem_surr surr, const char *path);
int chem_surrogate_save_checkpoint(chem_surr surr, const char *path, const void *user, int64_t user_bytes);
int chem_surrogate_load(chem_mech mech, const char *path, chem_surr *out);
int chem_surrogate_checkpoint_user(const char *path, void *user, int64_t capacity, int64_t *user_bytes);

/* ------------------------------------------------------------------------ */
/* Implicit finite-volume Laplacian: ldu assembly and CSR conversion          */
/* ------------------------------------------------------------------------ */

typedef struct chem_ldu_s *chem_ldu;

/* A mesh in owner/neighbour (ldu) addressing (Section 3.1, the ldu/CSR
 * figure), copied to `device` from host arrays the caller keeps:
 * internal faces in upper-triangular order (0 <= owner[f] < neighbour[f] <
 * ncells; sorted by owner, then neighbour), with the owner weight of linear
 * interpolation, the inverse distance of the two cell centres delta and the
 * face area mag_sf; boundary faces grouped by patch, patch p holding faces
 * patch_start[p] .. patch_start[p+1]-1 (patch_start[0] = 0) of type
 * patch_type[p] (0 fixed value, 1 zero gradient), with the cell next to each
 * face, the inverse centre-to-face distance bdelta and the area bmag_sf.
 * The CSR pattern is built here: row i holds the columns of the faces
 * whose neighbour is i (increasing), i itself, then the faces whose owner
 * is i (increasing); ncells + 2 nfaces < 2^31.  CHEM_EINVAL on arrays that
 * break these rules.  Allocates; synchronous. */
int chem_ldu_create(int64_t ncells, int64_t nfaces, const int32_t *owner, const int32_t *neighbour,
                    const double *weight, const double *delta, const double *mag_sf, int32_t npatches,
                    const int64_t *patch_start, const int32_t *patch_type, const int32_t *face_cells,
                    const double *bdelta, const double *bmag_sf, int device, chem_ldu *out);
void chem_free_ldu(chem_ldu mesh);
/* dims[0..3] = ncells, nfaces, boundary faces, CSR entries. */
int chem_ldu_info(chem_ldu mesh, int64_t *dims);
/* Algorithm 1 of Section 3.1, the implicit discretisation of
 * div(gamma grad psi): per internal face gamma_f = w gamma_c[owner] +
 * (1 - w) gamma_c[neighbour], upper[f] = lower[f] = gamma_f delta_f |S_f|,
 * diag (ncells) = -(sum of the coefficients of the cell's faces), accumulated
 * with atomics (so its last bits depend on the order of the additions);
 * then one launch per boundary patch: fixed value internal[b] =
 * -gamma_b[b] |S_b| delta_b, boundary[b] = gamma_b[b] |S_b| delta_b psi_b[b];
 * zero gradient 0 and 0.  The operator is L(psi) = A psi + r with A the ldu
 * matrix with the internal coefficients added to the diagonal and r the
 * boundary coefficients summed per cell.  All arrays device memory; enqueued
 * on the stream; allocates nothing. */
int chem_ldu_laplacian(chem_ldu mesh, const double *gamma_c, const double *gamma_b, const double *psi_b,
                       double *lower, double *upper, double *diag, double *internal, double *boundary,
                       void *hip_stream);
/* The ldu matrix in CSR (the ldu/CSR figure): csr_val (CSR entries, in the
 * pattern of chem_ldu_create) and rhs (ncells) = r, the boundary's internal
 * coefficients added to the diagonal entries in boundary-face order
 * (deterministic).  Device arrays; enqueued on the stream; allocates
 * nothing. */
int chem_ldu_to_csr(chem_ldu mesh, const double *lower, const double *upper, const double *diag,
                    const double *internal, const double *boundary, double *csr_val, double *rhs,
                    void *hip_stream);
/* The same matrix and right-hand side assembled straight into CSR, with no
 * ldu arrays and no atomics: every off-diagonal entry is gamma_f delta_f
 * |S_f| of the face it comes from (the same bits as chem_ldu_laplacian's
 * upper and lower), each diagonal entry minus the sum of its row's
 * off-diagonal entries (in column order) plus its boundary faces' internal
 * coefficients, and rhs its boundary coefficients
 * (deterministic: the same bits every call).  Device arrays; enqueued on the
 * stream; allocates nothing.  The face coefficients pass through a work
 * array of the mesh handle: calls on one mesh must not overlap. */
int chem_ldu_laplacian_csr(chem_ldu mesh, const double *gamma_c, const double *gamma_b, const double *psi_b,
                           double *csr_val, double *rhs, void *hip_stream);
/* Copies the CSR pattern: row_ptr (ncells + 1) and col (CSR entries), device. */
int chem_ldu_csr_pattern(chem_ldu mesh, int32_t *row_ptr, int32_t *col, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Thermophysical and transport properties over a field                     */
/* ------------------------------------------------------------------------ */

/* The thermo part of the Thermo class of Section 3.1: mass-specific
 * enthalpy h (J/kg) and cp (J/(kg K)) of every cell's mixture from the
 * NASA-7 polynomials at its temperature T (K); Y[k*ldY + i] as in
 * chem_integrate.  h or cp may be NULL.  Device arrays; enqueued on the
 * stream; allocates nothing.  K <= 64 (CHEM_EUNSUP otherwise). */
int chem_mixture_h_cp(chem_mech mech, const double *T, const double *Y, int64_t ldY, int64_t ncells,
                      double *h, double *cp, void *hip_stream);
/* Temperature from mass-specific enthalpy by Newton's method on the
 * temperature polynomials (Section 3.1): from the guess in T, every step
 * T <- min(max(T - (h(T) - h) / cp(T), 200), 3500) K until a step is below
 * tol (K); T then holds the result, cp (if not NULL) the mixture cp there
 * and iters (if not NULL) the steps taken.  A cell that has not converged
 * after max_iter steps (1 .. 1000) gets T = cp = NaN and iters = max_iter + 1
 * (a per-cell result, not a call error).  Y is used as given (no clipping).
 * Device arrays; enqueued on the stream; allocates nothing. */
int chem_T_from_h(chem_mech mech, const double *h, const double *Y, int64_t ldY, int64_t ncells, double *T,
                  double *cp, int32_t *iters, int32_t max_iter, double tol, void *hip_stream);
/* Transport data of the mechanism's species (host arrays, copied; lowest
 * power first): visc (K x 5) with mu_k = (T^(1/4) P_k(ln T))^2 in Pa s,
 * cond (K x 5) with lam_k = T^(1/2) Q_k(ln T) in W/(m K), and diff
 * (K x K x 5, symmetric in the species pair, diagonal = self-diffusion)
 * with D_jk = T^(3/2) B_jk(ln T) / p in m^2/s.  CHEM_EINVAL on non-finite or
 * asymmetric fits.  Allocates and synchronises; replaces earlier data, so it
 * must not run while transport calls on this mechanism are in flight. */
int chem_set_transport(chem_mech mech, const double *visc, const double *cond, const double *diff);
/* Mixture-averaged transport properties (the molecular transport model of
 * Section 2; compute-bound kernels of Section 3.2) of every cell at T (K),
 * p (Pa) and mass fractions Y, after y_k = max(Y_k, 0) / sum_j max(Y_j, 0):
 * mu (Pa s) by Wilke's rule, lam (W/(m K)) as the mean of the mole-fraction
 * weighted arithmetic and harmonic means of the species values, and
 * D[k*ldD + i] (m^2/s) = (1 - y_k) / sum_{j != k} X_j / D_jk (D_kk for a
 * pure species).  mu and lam are given together or both NULL; D may be NULL
 * (then p may be NULL too); not all NULL.  Needs chem_set_transport.  Device
 * arrays; enqueued on the stream; allocates nothing; K <= 64. */
int chem_transport_field(chem_mech mech, const double *T, const double *p, const double *Y, int64_t ldY,
                         int64_t ncells, double *mu, double *lam, double *D, int64_t ldD, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* CHEM_H */

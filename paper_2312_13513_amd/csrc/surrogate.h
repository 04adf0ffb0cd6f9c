// Learned chemistry surrogate: device kernels (surrogate.hip) and their
// launchers.  The network is an MLP [T, p, BoxCox(Y)] -> z-scored dY with GELU
// hidden layers, BF16 weights and activations, FP32 accumulation on MFMA.
#pragma once

#include <cstdint>

#include "chem_internal.h"

namespace chem {

typedef uint16_t bf16_t;   // bfloat16 bit pattern

constexpr int kMaxSurrSpecies = 62;   // network input K + 2 <= 64

// C[m][n] = sum_k A(m,k) B(n,k) over BF16 operands with FP32 accumulation.
// A(m,k) = A[m*sam + k*sak], B(n,k) = B[n*sbn + k*sbk]; for each operand one
// of its two strides is 1 and the extent along that dimension is a multiple
// of 8 (16-byte aligned rows).  The epilogue decides what is written.
enum GemmEpilogue {
    kEpiBiasF32 = 0,       // outf[m][n] = acc + bias[n]
    kEpiBiasGeluBf16 = 1,  // u = acc + bias[n]; outf[m][n] = u (if outf); outh[m][n] = bf16(gelu(u))
    kEpiGeluGradBf16 = 2,  // outh[m][n] = bf16(acc * gelu'(u[m][n]))
    kEpiF32 = 3,           // outf[m][n] = acc
};

struct GemmArgs {
    const bf16_t *A;
    int64_t sam, sak;
    const bf16_t *B;
    int64_t sbn, sbk;
    int M, N, K;
    int epi;
    const float *bias;
    float *outf;
    int64_t ldf;
    bf16_t *outh;
    int64_t ldh;
    const float *u;
    int64_t ldu;
    // grouped product (one independent GEMM per group, blockIdx.z): group z
    // offsets every pointer by z times its stride (0 or 1 group: one GEMM)
    int groups;
    int64_t za, zb, zbias, zf, zh, zu;
};

hipError_t launch_gemm_bf16(const GemmArgs &g, hipStream_t s);

// Fused inference forward pass: out = W4 h3 + b4 with h_l = GELU(W_l h_(l-1) + b_l),
// h_0 = the 64-wide input rows.  W[l] holds the [out_l][in_l] BF16 weights in
// fragment order (launch_swizzle_frag; in_l of layer 0 is 64), b[l] FP32.
// One block takes 32 rows through all four layers with the activations in
// LDS; the result equals the layer-by-layer GEMMs bit for bit.
struct MlpArgs {
    const bf16_t *X;        // rows x 64
    int64_t rows;
    const bf16_t *W[4];
    const float *b[4];
    int in_l[4], out_l[4];
    float *out;
    int64_t ldo;
};
// false when the hidden widths do not fit the fused kernel (each <= 512).
bool mlp_fused_supported(const int out_l[4]);
// W [N][K] row-major -> Wf in the fused kernel's fragment order (N % 16 == 0, K % 32 == 0).
hipError_t launch_swizzle_frag(const bf16_t *W, int N, int K, bf16_t *Wf, hipStream_t s);
hipError_t launch_mlp_forward(const MlpArgs &a, hipStream_t s);

// Network input of cells: x = zscore([T, p, BoxCox(max(Y,0); 0.1)]) -> FP32 -> BF16,
// written as rows of nin_pad values (zero padded).  norm = mu_x[nin], sig_x[nin].
hipError_t launch_encode(const double *T, const double *p, const double *Y, int64_t ldY, int64_t n,
                         int K, int nin_pad, const double *norm, bf16_t *X, hipStream_t s);

// Training targets: with d = Yn[k*ldYn + i] - Y[k*ldY + i] (the change over one
// flow step), Yt[i][k] = (d - mu_y[k]) / sig_y[k] as FP32, rows of nout_pad.
hipError_t launch_targets(const double *Y, int64_t ldY, const double *Yn, int64_t ldYn, int64_t n,
                          int K, int nout_pad, const double *mu_y, const double *sig_y, float *Yt,
                          hipStream_t s);

// Column means and standard deviations (population, two-pass, FP64) of the
// raw features [T, p, BoxCox(Y)] and of dY = Yn - Y: out = mu_x, sig_x, mu_y, sig_y.
hipError_t launch_fit_norm(const double *T, const double *p, const double *Y, int64_t ldY,
                           const double *Yn, int64_t ldYn, int64_t n, int K, double *out,
                           hipStream_t s);

struct ApplyArgs {
    const double *species;   // NASA blocks of the mechanism (device)
    const double *rw;        // R / W_k, J/(kg K) (device)
    const double *ncoef;     // n_ke / W_k, [E][K] (device), E <= 8
    int K, E;
    bool two_range;
    const double *mu_y, *sig_y;
    double elem_tol, sum_tol, neg_tol, T_out_min, T_out_max, T_in_min, T_in_max, dT_gate;
};

// Decode, temperature recovery and checks, one thread per cell: accepted
// cells take the prediction in place; rejected ones keep their state, get
// mask[i] = 1 (if mask) and their index base + i appended to list (count in
// *count).  status[i] (if status) is set to 0 for every cell.
hipError_t launch_apply(const ApplyArgs &a, double *T, const double *p, double *Y, int64_t ldY,
                        int64_t n, int64_t base, const float *out, int nout_pad, int32_t *mask,
                        int32_t *status, int32_t *list, int64_t *count, hipStream_t s);

hipError_t launch_zero_i64(int64_t *p, int n, hipStream_t s);
// out = v[0] + ... + v[n-1], one small kernel
hipError_t launch_sum_i64(const int64_t *v, int n, int64_t *out, hipStream_t s);
// gather / scatter with the compacted arrays' leading dimension ldc apart
// from the capacity cap (a pass's slice of a larger compaction buffer)
hipError_t launch_gather_cells_ld(const int32_t *list, const int64_t *count, int64_t cap, int64_t ldc,
                                  const double *T, const double *p, const double *Y, int64_t ldY,
                                  int K, double *cT, double *cp, double *cY, hipStream_t s);
hipError_t launch_scatter_cells_ld(const int32_t *list, const int64_t *count, int64_t cap, int64_t ldc,
                                   const double *cT, const double *cY, const int32_t *cstatus, int K,
                                   double *T, double *Y, int64_t ldY, int32_t *status, hipStream_t s);

// Compaction of the listed cells into contiguous arrays and back.
hipError_t launch_gather_cells(const int32_t *list, const int64_t *count, int64_t cap,
                               const double *T, const double *p, const double *Y, int64_t ldY,
                               int K, double *cT, double *cp, double *cY, hipStream_t s);
hipError_t launch_scatter_cells(const int32_t *list, const int64_t *count, int64_t cap,
                                const double *cT, const double *cY, const int32_t *cstatus, int K,
                                double *T, double *Y, int64_t ldY, int32_t *status, hipStream_t s);

// Training pieces.
hipError_t launch_gather_rows(const int32_t *order, int64_t start, int64_t rows, const bf16_t *X,
                              int nin_pad, const float *Yt, int nout_pad, bf16_t *Xb, float *Yb,
                              hipStream_t s);
// loss partial (sum of squares over rows x K valid outputs) into *loss_acc
// (FP64, accumulated over calls), dOut = bf16(2 (out - y) / (rows K)).
hipError_t launch_loss_grad(const float *out, const float *Yb, int rows, int K, int nout_pad,
                            bf16_t *dOut, double *loss_acc, hipStream_t s);
// db[n] = sum over rows of d[r][n]; part: 64 x N floats of workspace.
hipError_t launch_bias_grad(const bf16_t *d, int rows, int N, int ld, float *part, float *db, hipStream_t s);
// Adam on FP32 master weights, BF16 copies refreshed from them.
struct AdamArgs {
    float *p, *m, *v;
    const float *g;
    int64_t n;
    // 1 - beta and 1 - beta^t are rounded from FP64: 1.0f - 0.999f would
    // carry the cancellation error of 0.999f (1.3e-5 relative) into v
    float lr, beta1, beta2, omb1, omb2, eps, bc1, bc2;
};
hipError_t launch_adam(const AdamArgs &a, hipStream_t s);
hipError_t launch_to_bf16(const float *src, bf16_t *dst, int64_t n, hipStream_t s);

}  // namespace chem

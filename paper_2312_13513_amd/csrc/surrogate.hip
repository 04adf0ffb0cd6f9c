// Learned chemistry surrogate on gfx950: BF16 MFMA GEMMs with fused
// bias/GELU epilogues for the forward pass and for both backward products,
// the input encoding (Box-Cox of the mass fractions, z-scores), the decode
// with temperature recovery and the acceptance checks, cell compaction for
// the integrator fallback, and the Adam update.
//
// The network follows the paper's use of a DNN for the chemistry source
// (Section 2): fully connected layers with GELU activations trained with
// Adam; here its input is [T, p, BoxCox(Y)] and its output the z-scored
// change of the mass fractions over one flow step.

#include "surrogate.h"

namespace chem {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest, ties to even; NaN -> quiet NaN.
__device__ __forceinline__ bf16_t to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

// GELU(u) = u Phi(u) without branches: Phi(-|u|) = erfc(z)/2, z = |u|/sqrt(2),
// in the form erfc(z) = t exp(-z^2 + P(t)), t = 1/(1 + z/2) (Numerical
// Recipes' erfcc), P of degree 7 refitted in FP64 (gelu_fit.py).  Evaluated
// through the hardware base-2 exponential with 1/2 and log2(e) folded into
// the coefficients, Phi(-|u|) = t 2^(Q(t) - u^2 log2(e)/2), Q = log2(e) P - 1,
// and GELU(u) = max(u, 0) - |u| Phi(-|u|) (one fused multiply-add for both
// signs; an infinite u gives NaN there).  Relative error within 1.7e-5 of
// the exact GELU for every finite u; the activations are then rounded to
// BF16 (unit roundoff 2^-8).
__device__ __forceinline__ float gelu(float u)
{
    const float a = fabsf(u);
    const float t = __builtin_amdgcn_rcpf(fmaf(a, 0.35355339059327373f, 1.0f));
    float q = -2.396635413e-01f;
    q = fmaf(q, t, 9.644635320e-01f);
    q = fmaf(q, t, -1.259334445e+00f);
    q = fmaf(q, t, 3.582076728e-01f);
    q = fmaf(q, t, 5.822304171e-03f);
    q = fmaf(q, t, 5.541245341e-01f);
    q = fmaf(q, t, 1.442124605e+00f);
    q = fmaf(q, t, -2.825743914e+00f);
    const float half = t * __builtin_amdgcn_exp2f(fmaf(u * u, -0.72134752044448170f, q));
    return fmaf(-a, half, fmaxf(u, 0.0f));
}

// Activation FP32 -> BF16 with the hardware conversion (round to nearest even).
__device__ __forceinline__ bf16_t act_bf16(float f) { return __builtin_bit_cast(bf16_t, (__bf16)f); }

__device__ __forceinline__ float gelu_grad(float u)
{
    return 0.5f * (1.0f + erff(u * 0.70710678118654752f)) +
           u * expf(-0.5f * u * u) * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------
// GEMM: 64 x 64 output tile per 256-thread block, four waves in 2 x 2, each
// wave 32 x 32 = 2 x 2 MFMA 16x16x32 tiles; K in steps of 32 through LDS.
// ---------------------------------------------------------------------------
constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;
typedef bf16_t TileRow[kBK + kPad];

// lds[r][k] = X(r0 + r, k0 + k), zero outside [0,R) x [0,Kd).  Each thread
// moves 8 consecutive values as one 16-byte load when they are aligned and
// inside the matrix, else one by one (the single-column blocks of the
// per-species networks' output layer start at any column).
template <int W = kBK + kPad>
__device__ __forceinline__ void stage_tile(const bf16_t *X, int64_t sr, int64_t sk, int R, int Kd,
                                           int r0, int k0, bf16_t (*lds)[W], int c0 = 0)
{
    const int t = threadIdx.x;
    if (sk == 1) {
        // rows contiguous along k: 16-byte chunks of 8 k-values
        const int r = t >> 2, kc = (t & 3) * 8;
        const int gr = r0 + r, gk = k0 + kc;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gr < R && gk < Kd) {
            const bf16_t *src = X + (int64_t)gr * sr + gk;
            if (gk + 8 <= Kd && ((uintptr_t)src & 15) == 0) {
                v = *(const uint4 *)src;
            } else {
                bf16_t *e = (bf16_t *)&v;
#pragma unroll
                for (int i = 0; i < 8; i++)
                    if (gk + i < Kd) e[i] = src[i];
            }
        }
        *(uint4 *)&lds[r][c0 + kc] = v;
    } else {
        // contiguous along r: 8 r-values of one k, transposed into LDS
        const int k = t >> 3, rc = (t & 7) * 8;
        const int gr = r0 + rc, gk = k0 + k;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gr < R && gk < Kd) {
            const bf16_t *src = X + (int64_t)gk * sk + gr;
            if (gr + 8 <= R && ((uintptr_t)src & 15) == 0) {
                v = *(const uint4 *)src;
            } else {
                bf16_t *e = (bf16_t *)&v;
#pragma unroll
                for (int i = 0; i < 8; i++)
                    if (gr + i < R) e[i] = src[i];
            }
        }
        const bf16_t *e = (const bf16_t *)&v;
#pragma unroll
        for (int i = 0; i < 8; i++) lds[rc + i][c0 + k] = e[i];
    }
}

// Offsets of group blockIdx.z of a grouped product.
__device__ __forceinline__ void gemm_group(GemmArgs &g)
{
    if (blockIdx.z) {
        // group z of a grouped product (the per-species networks' layers)
        const int64_t z = blockIdx.z;
        g.A += z * g.za;
        g.B += z * g.zb;
        if (g.bias) g.bias += z * g.zbias;
        if (g.outf) g.outf += z * g.zf;
        if (g.outh) g.outh += z * g.zh;
        if (g.u) g.u += z * g.zu;
    }
}

__device__ __forceinline__ void gemm_store(const GemmArgs &g, int m, int n, float v)
{
    if (m >= g.M || n >= g.N) return;
    switch (g.epi) {
    case kEpiBiasF32:
        g.outf[(int64_t)m * g.ldf + n] = v + (g.bias ? g.bias[n] : 0.0f);
        break;
    case kEpiBiasGeluBf16: {
        const float u = v + (g.bias ? g.bias[n] : 0.0f);
        if (g.outf) g.outf[(int64_t)m * g.ldf + n] = u;
        g.outh[(int64_t)m * g.ldh + n] = act_bf16(gelu(u));
        break;
    }
    case kEpiGeluGradBf16:
        g.outh[(int64_t)m * g.ldh + n] = act_bf16(v * gelu_grad(g.u[(int64_t)m * g.ldu + n]));
        break;
    default:
        g.outf[(int64_t)m * g.ldf + n] = v;
        break;
    }
}

// TM x TM output tile per 256-thread block (TM = 64 or 128), four waves in
// 2 x 2, each wave (TM/2) x (TM/2) = (TM/32)^2 MFMA 16x16x32 tiles; K in
// steps of 32 through LDS, in increasing order: every output element sees
// the same sequence of MFMAs whatever TM, so both tile sizes (and the fused
// forward kernel) give the same bits.  The 128 tile does four times the
// MFMA work per barrier pair and per staged byte.
template <int TM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM == 128 ? 4 : 1))) gemm_bf16_kernel(GemmArgs g)
{
    constexpr int WT = TM / 32;              // MFMA tiles per wave and dimension
    constexpr int KB = TM == 128 ? 64 : 32;  // K per staged step (two MFMA K steps at the 128 tile)
    constexpr int RW = KB + kPad;            // LDS row, padded
    gemm_group(g);
    __shared__ __attribute__((aligned(16))) bf16_t As[TM][RW];
    __shared__ __attribute__((aligned(16))) bf16_t Bs[TM][RW];
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = (w & 1) * (TM / 2), wn = (w >> 1) * (TM / 2);
    const int kk = (lane >> 4) * 8;
    floatx4 acc[WT][WT];
#pragma unroll
    for (int i = 0; i < WT; i++)
#pragma unroll
        for (int j = 0; j < WT; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += KB) {
#pragma unroll
        for (int h = 0; h < TM / 64; h++)
#pragma unroll
            for (int c = 0; c < KB / kBK; c++) {
                stage_tile<RW>(g.A, g.sam, g.sak, g.M, g.K, m0 + 64 * h, k0 + kBK * c, As + 64 * h, kBK * c);
                stage_tile<RW>(g.B, g.sbn, g.sbk, g.N, g.K, n0 + 64 * h, k0 + kBK * c, Bs + 64 * h, kBK * c);
            }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < KB / kBK; c++) {
            bf16x8 a[WT], b[WT];
#pragma unroll
            for (int i = 0; i < WT; i++)
                __builtin_memcpy(&a[i], &As[wm + i * 16 + (lane & 15)][kBK * c + kk], 16);
#pragma unroll
            for (int j = 0; j < WT; j++)
                __builtin_memcpy(&b[j], &Bs[wn + j * 16 + (lane & 15)][kBK * c + kk], 16);
#pragma unroll
            for (int i = 0; i < WT; i++)
#pragma unroll
                for (int j = 0; j < WT; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // D layout of a 16x16 MFMA tile: lane l holds rows 4*(l/16) + r, column l%16
#pragma unroll
    for (int i = 0; i < WT; i++)
#pragma unroll
        for (int j = 0; j < WT; j++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                gemm_store(g, m0 + wm + i * 16 + (lane >> 4) * 4 + r, n0 + wn + j * 16 + (lane & 15),
                           acc[i][j][r]);
}

// ---------------------------------------------------------------------------
// Fused forward pass (inference): 32 rows per block, four waves, 50 KB of
// LDS, so that three blocks share a CU and one block's GELU epilogues overlap
// another's matrix products; each layer is a 32 x N x K product with A (the
// activations) from LDS and B (the weights, L2-resident) loaded by each lane
// straight into its MFMA operand registers.  Wave w owns the 16-column blocks
// w + 4 j of the layer's output for both 16-row blocks, so every weight
// fragment is loaded once per block.  The weights come in fragment order (swizzle_frag_kernel): the
// 16 x 32 operand of column block jb and K step ks is 1 KB at
// ((jb * K/32 + ks) * 512 + 8 lane), so a wave reads it as one contiguous
// 16-byte-per-lane load.  The accumulation over K runs in steps of 32 in
// increasing order, as in gemm_bf16_kernel, and the epilogues are the same,
// so the result is bitwise that of the GEMMs.
// ---------------------------------------------------------------------------
constexpr int kMlpRows = 32, kMlpWaves = 4, kMlpMaxN = 512, kMlpJ = kMlpMaxN / 16 / kMlpWaves;
constexpr int kMlpRB = kMlpRows / 16;
constexpr int kMlpPad = 8;   // bf16 pad per LDS row: spreads the 16 rows of an A fragment over banks
constexpr int kMlpDepth = 2; // K steps of weight fragments loaded ahead

// KS > 0: the layer has KS K steps, known at compile time, and the step
// loop is unrolled completely (one straight block, so the waits on the
// weight loads count the loads in flight instead of draining them at a loop
// head); KS = 0: any K.
template <int J, int KS = 0>
__device__ __forceinline__ void mlp_layer(const bf16_t *in, int ldi, int K, const bf16_t *__restrict__ Wf, int N,
                                          const float *__restrict__ bias, bf16_t *outs, int lds_out,
                                          float *outg, int64_t ldg, int64_t r0, int64_t rows)
{
    // the wave index is uniform: as a scalar, the block guards below are
    // scalar branches
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int kk = (lane >> 4) * 8;
    const int nblk = N >> 4, ksteps = KS > 0 ? KS : K >> 5;
    floatx4 acc[J][kMlpRB];
#pragma unroll
    for (int j = 0; j < J; j++)
#pragma unroll
        for (int i = 0; i < kMlpRB; i++) acc[j][i] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bf16_t *wfr[J];
#pragma unroll
    for (int j = 0; j < J; j++) {
        const int jb = w + kMlpWaves * j;
        wfr[j] = Wf + (int64_t)(jb < nblk ? jb : 0) * ksteps * 512 + lane * 8;
    }
    const bf16_t *arow = in + (lane & 15) * ldi + kk;
    // weight fragments of the next D K steps are in flight while the current
    // step's products run (one register slot per step, the loop unrolled by
    // the depth so that every slot index is static; four steps ahead when the
    // step count is known, else kMlpDepth).  A wave whose column block j lies
    // past the layer (only when N is not a multiple of 64) loads and
    // multiplies block 0 in its place and drops the result: no branch around
    // the loads, so the loop body is one block and each step waits only for
    // its own fragments.
    constexpr int D = KS > 0 ? (KS < 4 ? KS : 4) : kMlpDepth;
    bf16x8 bq[D][J];
#pragma unroll
    for (int d = 0; d < D; d++)
#pragma unroll
        for (int j = 0; j < J; j++)
            if (d < ksteps) __builtin_memcpy(&bq[d][j], wfr[j] + d * 512, 16);
    // ksteps is a multiple of D (KS: by the shapes of mlp_layer_any; else
    // mlp_fused_supported)
#pragma unroll(KS > 0 ? KS / D : 1)
    for (int s0 = 0; s0 < ksteps; s0 += D) {
#pragma unroll
        for (int d = 0; d < D; d++) {
            const int ks = s0 + d;
            bf16x8 a[kMlpRB];
#pragma unroll
            for (int i = 0; i < kMlpRB; i++) __builtin_memcpy(&a[i], arow + i * 16 * ldi + ks * 32, 16);
            // weights as the first operand: the output tile comes out
            // transposed (lane l: columns 4 (l/16) .. +3 of row l % 16), so
            // each lane's four results are adjacent in a row of the output
#pragma unroll
            for (int j = 0; j < J; j++)
#pragma unroll
                for (int i = 0; i < kMlpRB; i++)
                    acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bq[d][j], a[i], acc[j][i], 0, 0, 0);
            // the last steps reload the last fragment (unused) instead of
            // branching around the load
            const int kn = ks + D < ksteps ? ks + D : ksteps - 1;
#pragma unroll
            for (int j = 0; j < J; j++) __builtin_memcpy(&bq[d][j], wfr[j] + kn * 512, 16);
        }
    }
#pragma unroll
    for (int j = 0; j < J; j++) {
        const int jb = w + kMlpWaves * j;
        if (jb >= nblk) continue;
        const int n0 = jb * 16 + (lane >> 4) * 4;
        float bn[4];
#pragma unroll
        for (int r = 0; r < 4; r++) bn[r] = bias[n0 + r];
#pragma unroll
        for (int i = 0; i < kMlpRB; i++) {
            const int m = i * 16 + (lane & 15);
            if (outs) {
                // four activations of row m, columns n0 .. n0 + 3: one 8-byte store
                bf16_t h[4];
#pragma unroll
                for (int r = 0; r < 4; r++) h[r] = act_bf16(gelu(acc[j][i][r] + bn[r]));
                uint2 pk;
                __builtin_memcpy(&pk, h, 8);
                *(uint2 *)(outs + m * lds_out + n0) = pk;
            } else if (r0 + m < rows) {
#pragma unroll
                for (int r = 0; r < 4; r++) outg[(r0 + m) * ldg + n0 + r] = acc[j][i][r] + bn[r];
            }
        }
    }
}

// one layer with the register budget of its width; the shapes of the
// default network (64 -> 512 -> 256 -> 128 -> 48 padded) with their K steps
// fixed at compile time
__device__ __forceinline__ void mlp_layer_any(const bf16_t *in, int ldi, int K, const bf16_t *Wf, int N,
                                              const float *bias, bf16_t *outs, int lds_out, float *outg,
                                              int64_t ldg, int64_t r0, int64_t rows)
{
#define CHEM_MLP_LAYER(JJ, KK)                                                                     \
    if (K == KK) {                                                                                 \
        mlp_layer<JJ, KK / 32>(in, ldi, K, Wf, N, bias, outs, lds_out, outg, ldg, r0, rows);       \
        return;                                                                                    \
    }
    if (N <= 64) {
        CHEM_MLP_LAYER(1, 128)
        mlp_layer<1>(in, ldi, K, Wf, N, bias, outs, lds_out, outg, ldg, r0, rows);
    } else if (N <= 128) {
        CHEM_MLP_LAYER(2, 256)
        mlp_layer<2>(in, ldi, K, Wf, N, bias, outs, lds_out, outg, ldg, r0, rows);
    } else if (N <= 256) {
        CHEM_MLP_LAYER(4, 512)
        mlp_layer<4>(in, ldi, K, Wf, N, bias, outs, lds_out, outg, ldg, r0, rows);
    } else {
        CHEM_MLP_LAYER(kMlpJ, 64)
        mlp_layer<kMlpJ>(in, ldi, K, Wf, N, bias, outs, lds_out, outg, ldg, r0, rows);
    }
#undef CHEM_MLP_LAYER
}

// Weights [N][K] -> fragment order (see above), 8 values per thread.
__global__ void __launch_bounds__(256) swizzle_frag_kernel(const bf16_t *__restrict__ W, int N, int K,
                                                           bf16_t *__restrict__ Wf)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // 8-value chunk of Wf
    if (c >= (int64_t)N * K / 8) return;
    const int64_t blk = c >> 6;
    const int L = (int)(c & 63);
    const int ksteps = K >> 5;
    const int jb = (int)(blk / ksteps), ks = (int)(blk % ksteps);
    const int n = jb * 16 + (L & 15), k = ks * 32 + (L >> 4) * 8;
    *(uint4 *)(Wf + c * 8) = *(const uint4 *)(W + (int64_t)n * K + k);
}

__global__ void __launch_bounds__(64 * kMlpWaves, 3) mlp_forward_kernel(MlpArgs a)
{
    extern __shared__ __attribute__((aligned(16))) bf16_t mlp_lds[];
    const int ld0 = (a.out_l[1] > 64 ? a.out_l[1] : 64) + kMlpPad;
    const int ld1 = (a.out_l[0] > a.out_l[2] ? a.out_l[0] : a.out_l[2]) + kMlpPad;
    bf16_t *buf0 = mlp_lds, *buf1 = mlp_lds + kMlpRows * ld0;
    const int64_t r0 = (int64_t)blockIdx.x * kMlpRows;
    // the block's input rows, zero past the end
    for (int c = threadIdx.x; c < kMlpRows * 8; c += 64 * kMlpWaves) {
        const int r = c >> 3, kc = (c & 7) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r0 + r < a.rows) v = *(const uint4 *)(a.X + (r0 + r) * 64 + kc);
        *(uint4 *)(buf0 + r * ld0 + kc) = v;
    }
    __syncthreads();
    mlp_layer_any(buf0, ld0, a.in_l[0], a.W[0], a.out_l[0], a.b[0], buf1, ld1, nullptr, 0, r0, a.rows);
    __syncthreads();
    mlp_layer_any(buf1, ld1, a.in_l[1], a.W[1], a.out_l[1], a.b[1], buf0, ld0, nullptr, 0, r0, a.rows);
    __syncthreads();
    mlp_layer_any(buf0, ld0, a.in_l[2], a.W[2], a.out_l[2], a.b[2], buf1, ld1, nullptr, 0, r0, a.rows);
    __syncthreads();
    mlp_layer_any(buf1, ld1, a.in_l[3], a.W[3], a.out_l[3], a.b[3], nullptr, 0, a.out, a.ldo, r0, a.rows);
}

// ---------------------------------------------------------------------------
// encoding
// ---------------------------------------------------------------------------
// Box-Cox with lambda 0.1; y^0.1 as exp2(0.1 log2 y) (y = 0 gives exp2(-inf) =
// 0, as the power), a few ulp of FP64 from the correctly rounded power, far
// below the BF16 rounding of the feature
__device__ __forceinline__ double boxcox(double y) { return (exp2(0.1 * log2(fmax(y, 0.0))) - 1.0) / 0.1; }

__global__ void __launch_bounds__(256) encode_kernel(const double *__restrict__ T,
                                                     const double *__restrict__ p,
                                                     const double *__restrict__ Y, int64_t ldY,
                                                     int64_t n, int K, int nin_pad,
                                                     const double *__restrict__ norm,
                                                     bf16_t *__restrict__ X)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int nin = K + 2;
    const double *mu = norm, *sg = norm + nin;
    bf16_t *row = X + i * nin_pad;
    for (int j = 0; j < nin_pad; j += 8) {
        uint4 pk;
        bf16_t *v = (bf16_t *)&pk;
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int f = j + e;
            double z = 0.0;
            if (f < nin) {
                const double raw = f == 0 ? T[i] : (f == 1 ? p[i] : boxcox(Y[(int64_t)(f - 2) * ldY + i]));
                if (sg[f] >= 1e-12) z = (raw - mu[f]) / sg[f];
            }
            v[e] = to_bf16((float)z);
        }
        *(uint4 *)(row + j) = pk;
    }
}

__global__ void __launch_bounds__(256) targets_kernel(const double *__restrict__ Y, int64_t ldY,
                                                      const double *__restrict__ Yn, int64_t ldYn,
                                                      int64_t n, int K, int nout_pad,
                                                      const double *__restrict__ mu,
                                                      const double *__restrict__ sg,
                                                      float *__restrict__ Yt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < nout_pad; k++) {
        float v = 0.0f;
        if (k < K && sg[k] >= 1e-12) {
            const double d = Yn[(int64_t)k * ldYn + i] - Y[(int64_t)k * ldY + i];
            v = (float)((d - mu[k]) / sg[k]);
        }
        Yt[i * nout_pad + k] = v;
    }
}

// one block per column; fixed summation order (per-thread strided partial
// sums, then a tree), so the result does not depend on timing
__global__ void __launch_bounds__(256) fit_norm_kernel(const double *__restrict__ T,
                                                       const double *__restrict__ p,
                                                       const double *__restrict__ Y, int64_t ldY,
                                                       const double *__restrict__ Yn, int64_t ldYn,
                                                       int64_t n, int K, double *__restrict__ out)
{
    __shared__ double red[256];
    const int c = blockIdx.x;
    const int nin = K + 2;
    auto value = [&](int64_t i) -> double {
        if (c == 0) return T[i];
        if (c == 1) return p[i];
        if (c < nin) return boxcox(Y[(int64_t)(c - 2) * ldY + i]);
        return Yn[(int64_t)(c - nin) * ldYn + i] - Y[(int64_t)(c - nin) * ldY + i];
    };
    auto block_sum = [&](double v) -> double {
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        const double r = red[0];
        __syncthreads();
        return r;
    };
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += value(i);
    const double mean = block_sum(s) / (double)n;
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double d = value(i) - mean;
        q += d * d;
    }
    const double var = block_sum(q) / (double)n;
    if (threadIdx.x == 0) {
        if (c < nin) {
            out[c] = mean;
            out[nin + c] = sqrt(var);
        } else {
            out[2 * nin + (c - nin)] = mean;
            out[2 * nin + K + (c - nin)] = sqrt(var);
        }
    }
}

// ---------------------------------------------------------------------------
// decode, temperature recovery, checks
// ---------------------------------------------------------------------------
constexpr int kApplyMaxE = 8;   // elements the decode kernel handles

// mass-specific enthalpy and cp of the mixture Y[0..K) (KM >= K, static loop)
// Thermo of species k at T (the NASA range of the lane's T): cp/R and H/(R T).
__device__ __forceinline__ void species_cp_hrt(const ApplyArgs &a, const double *species, int k, double T,
                                               double invT, double &cp, double &hrt)
{
    const double *s = species + k * kSpeciesLen;
    const bool low = !a.two_range || T < s[0];
    double r[11];
    const double *c = s + 1 + (low ? 0 : kRangeLen);
#pragma unroll
    for (int j = 0; j < 11; j++)
        if (j != 6) r[j] = c[j];
    cp = r[0] + T * (r[1] + T * (r[2] + T * (r[3] + T * r[4])));
    hrt = r[0] + T * (r[7] + T * (r[8] + T * (r[9] + T * r[10]))) + r[5] * invT;
}

// Mixture enthalpy (J/kg) and cp (J/(kg K)) at T: sums over species in order,
// each term Y_k (R/W_k) times T H_k/(R T), resp. cp_k/R.
template <int KM>
__device__ __forceinline__ void mix_h_cp(const ApplyArgs &a, const double *species, double T,
                                         const double (&Y)[KM], double &hm, double &cm)
{
    double h = 0.0, c = 0.0;
    const double invT = 1.0 / T;
#pragma unroll
    for (int k = 0; k < KM; k++) {
        if (k < a.K) {
            double cp, hrt;
            species_cp_hrt(a, species, k, T, invT, cp, hrt);
            const double yr = Y[k] * a.rw[k];
            h += yr * (T * hrt);
            c += yr * cp;
        }
    }
    hm = h;
    cm = c;
}

// Decode, checks and temperature recovery, one thread per cell.  The input
// state is read once: its element content, the element residual of the
// prediction and the input enthalpy are accumulated in the same pass, so
// only the predicted mass fractions stay in registers.  The block first
// copies the species thermo blocks into LDS, where the enthalpy Newton
// iterations read them.  With V4 (the output rows 16-byte aligned) a cell's
// network outputs are read four at a time; one float per load touches a
// different cache line in every lane of a wave for each species.
template <int KM, int KE, bool V4>
__global__ void __launch_bounds__(256, 3) apply_kernel(ApplyArgs a, double *__restrict__ T,
                                                    const double *__restrict__ p,
                                                    double *__restrict__ Y, int64_t ldY, int64_t n,
                                                    int64_t base, const float *__restrict__ out,
                                                    int nout_pad, int32_t *__restrict__ mask,
                                                    int32_t *__restrict__ status,
                                                    int32_t *__restrict__ list,
                                                    int64_t *__restrict__ count)
{
    __shared__ double sp_lds[KM * kSpeciesLen];
    for (int j = threadIdx.x; j < a.K * kSpeciesLen; j += 256) sp_lds[j] = a.species[j];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool reject = false;
    if (i < n) {
        (void)p;
        const int K = a.K;
        const double T0 = T[i];
        const double invT0 = 1.0 / T0;
        double Y1[KM];
        bool ok = true;
        double sum = 0.0, ymin = 1e300, h0 = 0.0;
        double res[KE], ref[KE];
#pragma unroll
        for (int e = 0; e < KE; e++) res[e] = ref[e] = 0.0;
        float4 o4 = make_float4(0.f, 0.f, 0.f, 0.f);   // outputs k .. k+3 (V4)
#pragma unroll
        for (int k = 0; k < KM; k++) {
            Y1[k] = 0.0;
            if (k < K) {
                const double y0 = Y[(int64_t)k * ldY + i];
                float o;   // the network's output for species k
                if constexpr (V4) {
                    // k + 3 < round_up(K, 4) <= nout_pad: inside the row
                    if (k % 4 == 0) o4 = *(const float4 *)(out + i * nout_pad + k);
                    o = (k % 4 == 0) ? o4.x : (k % 4 == 1) ? o4.y : (k % 4 == 2) ? o4.z : o4.w;
                } else {
                    o = out[i * nout_pad + k];
                }
                const double v = y0 + a.mu_y[k] + a.sig_y[k] * (double)o;
                Y1[k] = v;
                ok = ok && isfinite(v);
                sum += v;
                ymin = fmin(ymin, v);
#pragma unroll
                for (int e = 0; e < KE; e++)
                    if (e < a.E) {
                        const double nk = a.ncoef[e * K + k];
                        res[e] += nk * (v - y0);
                        ref[e] += nk * y0;
                    }
                double cp, hrt;
                species_cp_hrt(a, sp_lds, k, T0, invT0, cp, hrt);
                h0 += (y0 * a.rw[k]) * (T0 * hrt);
            }
        }
        // element residual relative to the element content of the input
#pragma unroll
        for (int e = 0; e < KE; e++)
            if (ok && e < a.E && fabs(res[e]) / fmax(ref[e], 1e-12) > a.elem_tol) ok = false;
        if (ok && fabs(sum - 1.0) > a.sum_tol) ok = false;
        if (ok && ymin < -a.neg_tol) ok = false;
        double Tn = T0;
        if (ok) {
            double s2 = 0.0;
#pragma unroll
            for (int k = 0; k < KM; k++) {
                if (k < K) {
                    Y1[k] = fmax(Y1[k], 0.0);
                    s2 += Y1[k];
                }
            }
            const double inv_s2 = 1.0 / s2;
#pragma unroll
            for (int k = 0; k < KM; k++)
                if (k < K) Y1[k] = Y1[k] * inv_s2;
            // Newton on h(T, Y2) = h0 from T0; |dT| < 1e-10 K, at most 20
            // iterations, T kept in [200, 3500] K
            bool conv = false;
            double Tk = T0;
            for (int it = 0; it < 20; it++) {
                double hm, cm;
                // an offset the compiler cannot see through keeps the table
                // reads inside the loop: hoisted, the coefficients of every
                // species would be held in registers across the iterations
                int off = 0;
                asm volatile("" : "+v"(off));
                mix_h_cp<KM>(a, sp_lds + off, Tk, Y1, hm, cm);
                const double dT = -(hm - h0) / cm;
                Tk += dT;
                Tk = fmin(fmax(Tk, 200.0), 3500.0);
                if (fabs(dT) < 1e-10) {
                    conv = true;
                    break;
                }
            }
            if (!conv || !(Tk >= a.T_out_min && Tk <= a.T_out_max)) ok = false;
            if (ok && (T0 < a.T_in_min || T0 > a.T_in_max)) ok = false;
            if (ok && a.dT_gate > 0.0 && fabs(Tk - T0) > a.dT_gate) ok = false;
            Tn = Tk;
        }
        if (ok) {
            T[i] = Tn;
#pragma unroll
            for (int k = 0; k < KM; k++)
                if (k < K) Y[(int64_t)k * ldY + i] = Y1[k];
        }
        if (mask) mask[i] = ok ? 0 : 1;
        if (status) status[i] = 0;
        reject = !ok;
    }
    // wave-aggregated append of the rejected cells
    const unsigned long long bal = __ballot(reject);
    if (bal) {
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((long long)bal) - 1;
        unsigned long long slot = 0;
        if (lane == leader) slot = atomicAdd((unsigned long long *)count, (unsigned long long)__popcll(bal));
        slot = __shfl(slot, leader);
        if (reject) {
            const unsigned long long rank = __popcll(bal & ((1ull << lane) - 1ull));
            list[slot + rank] = (int32_t)(base + i);
        }
    }
}

// out = v[0] + ... + v[n-1] (one wave; n is a handful of pass counts)
__global__ void sum_i64_kernel(const int64_t *__restrict__ v, int n, int64_t *__restrict__ out)
{
    int64_t s = 0;
    for (int i = threadIdx.x; i < n; i += 64) s += v[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if (threadIdx.x == 0) *out = s;
}

__global__ void zero_i64_kernel(int64_t *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void __launch_bounds__(256) gather_cells_kernel(const int32_t *__restrict__ list,
                                                           const int64_t *__restrict__ count,
                                                           int64_t cap, int64_t ldc, const double *__restrict__ T,
                                                           const double *__restrict__ p,
                                                           const double *__restrict__ Y, int64_t ldY,
                                                           int K, double *__restrict__ cT,
                                                           double *__restrict__ cp,
                                                           double *__restrict__ cY)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cnt = *count < cap ? *count : cap;
    if (j >= cnt) return;
    const int64_t i = list[j];
    cT[j] = T[i];
    cp[j] = p[i];
    for (int k = 0; k < K; k++) cY[(int64_t)k * ldc + j] = Y[(int64_t)k * ldY + i];
}

__global__ void __launch_bounds__(256) scatter_cells_kernel(const int32_t *__restrict__ list,
                                                            const int64_t *__restrict__ count,
                                                            int64_t cap, int64_t ldc, const double *__restrict__ cT,
                                                            const double *__restrict__ cY,
                                                            const int32_t *__restrict__ cstatus, int K,
                                                            double *__restrict__ T,
                                                            double *__restrict__ Y, int64_t ldY,
                                                            int32_t *__restrict__ status)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cnt = *count < cap ? *count : cap;
    if (j >= cnt) return;
    const int64_t i = list[j];
    T[i] = cT[j];
    for (int k = 0; k < K; k++) Y[(int64_t)k * ldY + i] = cY[(int64_t)k * ldc + j];
    if (status) status[i] = cstatus ? cstatus[j] : 0;
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) gather_rows_kernel(const int32_t *__restrict__ order,
                                                          int64_t start, int64_t rows,
                                                          const bf16_t *__restrict__ X, int nin_pad,
                                                          const float *__restrict__ Yt, int nout_pad,
                                                          bf16_t *__restrict__ Xb,
                                                          float *__restrict__ Yb)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int64_t src = order ? (int64_t)order[start + r] : start + r;
    const uint4 *xs = (const uint4 *)(X + src * nin_pad);
    uint4 *xd = (uint4 *)(Xb + r * nin_pad);
    for (int j = 0; j < nin_pad / 8; j++) xd[j] = xs[j];
    for (int j = 0; j < nout_pad; j++) Yb[r * nout_pad + j] = Yt[src * nout_pad + j];
}

__global__ void __launch_bounds__(256) loss_grad_kernel(const float *__restrict__ out,
                                                        const float *__restrict__ Yb, int rows, int K,
                                                        int nout_pad, bf16_t *__restrict__ dOut,
                                                        double *__restrict__ partial)
{
    __shared__ double red[256];
    const int64_t total = (int64_t)rows * nout_pad;
    const float scale = 2.0f / ((float)rows * (float)K);
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(e % nout_pad);
        float d = 0.0f;
        if (col < K) {
            d = out[e] - Yb[e];
            s += (double)d * (double)d;
        }
        dOut[e] = to_bf16(scale * d);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_partials_kernel(const double *__restrict__ partial, int np, double *acc)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < np; i++) s += partial[i];
        *acc += s;
    }
}

// Column sums in two passes with a fixed order: block (column tile, row
// chunk) sums its rows per column into part[chunk][n], then the chunks are
// added in chunk order.
constexpr int kBiasChunks = 64;

__global__ void __launch_bounds__(64) bias_grad_part_kernel(const bf16_t *__restrict__ d, int rows, int N,
                                                            int ld, float *__restrict__ part)
{
    const int n = blockIdx.x * 64 + threadIdx.x;
    const int chunk = blockIdx.y;
    const int per = (rows + kBiasChunks - 1) / kBiasChunks;
    const int r0 = chunk * per, r1 = min(rows, r0 + per);
    if (n >= N) return;
    float s = 0.0f;
    for (int r = r0; r < r1; r++) s += __uint_as_float((unsigned)d[(int64_t)r * ld + n] << 16);
    part[chunk * N + n] = s;
}

__global__ void __launch_bounds__(256) bias_grad_final_kernel(const float *__restrict__ part, int N,
                                                              float *__restrict__ db)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int c = 0; c < kBiasChunks; c++) s += part[c * N + n];
    db[n] = s;
}

__global__ void __launch_bounds__(256) adam_kernel(AdamArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float g = a.g[i];
    const float m = a.beta1 * a.m[i] + a.omb1 * g;
    const float v = a.beta2 * a.v[i] + a.omb2 * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float mh = m / a.bc1, vh = v / a.bc2;
    a.p[i] -= a.lr * mh / (sqrtf(vh) + a.eps);
}

__global__ void __launch_bounds__(256) to_bf16_kernel(const float *__restrict__ src,
                                                      bf16_t *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = to_bf16(src[i]);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_gemm_bf16(const GemmArgs &g, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const unsigned gz = (unsigned)(g.groups > 1 ? g.groups : 1);
    // the 128 tile where it still gives every CU several blocks
    const int64_t tiles128 = (int64_t)((g.N + 127) / 128) * ((g.M + 127) / 128) * gz;
    if (g.M >= 128 && g.N >= 128 && tiles128 >= 1024) {
        dim3 grid((unsigned)((g.N + 127) / 128), (unsigned)((g.M + 127) / 128), gz);
        hipLaunchKernelGGL(gemm_bf16_kernel<128>, grid, dim3(256), 0, s, g);
    } else {
        dim3 grid((unsigned)((g.N + kBN - 1) / kBN), (unsigned)((g.M + kBM - 1) / kBM), gz);
        hipLaunchKernelGGL(gemm_bf16_kernel<64>, grid, dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

static size_t mlp_lds_bytes(const int out_l[4])
{
    const int ld0 = (out_l[1] > 64 ? out_l[1] : 64) + kMlpPad;
    const int ld1 = (out_l[0] > out_l[2] ? out_l[0] : out_l[2]) + kMlpPad;
    return (size_t)kMlpRows * (ld0 + ld1) * sizeof(bf16_t);
}

bool mlp_fused_supported(const int out_l[4])
{
    for (int l = 0; l < 4; l++)
        if (out_l[l] > kMlpMaxN || out_l[l] % 16 != 0) return false;
    // every layer's K (64, then the hidden widths) in whole prefetch groups
    for (int l = 0; l < 3; l++)
        if (out_l[l] % (32 * kMlpDepth) != 0) return false;
    int dev = 0, max_lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return false;
    return mlp_lds_bytes(out_l) <= (size_t)max_lds;
}

hipError_t launch_swizzle_frag(const bf16_t *W, int N, int K, bf16_t *Wf, hipStream_t s)
{
    if (N % 16 != 0 || K % 32 != 0) return hipErrorInvalidValue;
    const int64_t chunks = (int64_t)N * K / 8;
    hipLaunchKernelGGL(swizzle_frag_kernel, dim3(blocks_for(chunks, 256)), dim3(256), 0, s, W, N, K, Wf);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpArgs &a, hipStream_t s)
{
    if (a.rows <= 0) return hipSuccess;
    if (!mlp_fused_supported(a.out_l) || a.in_l[0] != 64) return hipErrorInvalidValue;
    const size_t lds = mlp_lds_bytes(a.out_l);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)mlp_forward_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((a.rows + kMlpRows - 1) / kMlpRows)),
                       dim3(64 * kMlpWaves), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_encode(const double *T, const double *p, const double *Y, int64_t ldY, int64_t n,
                         int K, int nin_pad, const double *norm, bf16_t *X, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(encode_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, T, p, Y, ldY, n, K,
                       nin_pad, norm, X);
    return hipGetLastError();
}

hipError_t launch_targets(const double *Y, int64_t ldY, const double *Yn, int64_t ldYn, int64_t n,
                          int K, int nout_pad, const double *mu_y, const double *sig_y, float *Yt,
                          hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(targets_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, Y, ldY, Yn, ldYn, n,
                       K, nout_pad, mu_y, sig_y, Yt);
    return hipGetLastError();
}

hipError_t launch_fit_norm(const double *T, const double *p, const double *Y, int64_t ldY,
                           const double *Yn, int64_t ldYn, int64_t n, int K, double *out,
                           hipStream_t s)
{
    if (n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fit_norm_kernel, dim3((unsigned)(2 * K + 2)), dim3(256), 0, s, T, p, Y, ldY,
                       Yn, ldYn, n, K, out);
    return hipGetLastError();
}

hipError_t launch_apply(const ApplyArgs &a, double *T, const double *p, double *Y, int64_t ldY,
                        int64_t n, int64_t base, const float *out, int nout_pad, int32_t *mask,
                        int32_t *status, int32_t *list, int64_t *count, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (a.E > kApplyMaxE) return hipErrorInvalidValue;
    const bool v4 = ((uintptr_t)out % 16 == 0) && nout_pad % 4 == 0;
#define CHEM_APPLY_E(KM, KE)                                                                                  \
    if (v4)                                                                                                   \
        hipLaunchKernelGGL((apply_kernel<KM, KE, true>), dim3(blocks_for(n, 256)), dim3(256), 0, s, a, T, p, Y,  \
                           ldY, n, base, out, nout_pad, mask, status, list, count);                           \
    else                                                                                                      \
        hipLaunchKernelGGL((apply_kernel<KM, KE, false>), dim3(blocks_for(n, 256)), dim3(256), 0, s, a, T, p, Y, \
                           ldY, n, base, out, nout_pad, mask, status, list, count)
#define CHEM_APPLY(KM)                                                                                        \
    do {                                                                                                      \
        if (a.E <= 4) {                                                                                       \
            CHEM_APPLY_E(KM, 4);                                                                              \
        } else {                                                                                              \
            CHEM_APPLY_E(KM, kApplyMaxE);                                                                     \
        }                                                                                                     \
    } while (0)
    if (a.K <= 16)
        CHEM_APPLY(16);
    else if (a.K <= 32)
        CHEM_APPLY(32);
    else if (a.K <= 40)
        CHEM_APPLY(40);
    else if (a.K <= 48)
        CHEM_APPLY(48);
    else if (a.K <= kMaxSurrSpecies)
        CHEM_APPLY(kMaxSurrSpecies);
    else
        return hipErrorInvalidValue;
#undef CHEM_APPLY
#undef CHEM_APPLY_E
    return hipGetLastError();
}

hipError_t launch_zero_i64(int64_t *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_i64_kernel, dim3(blocks_for(n, 64)), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_gather_cells_ld(const int32_t *list, const int64_t *count, int64_t cap, int64_t ldc,
                                  const double *T, const double *p, const double *Y, int64_t ldY,
                                  int K, double *cT, double *cp, double *cY, hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_cells_kernel, dim3(blocks_for(cap, 256)), dim3(256), 0, s, list, count,
                       cap, ldc, T, p, Y, ldY, K, cT, cp, cY);
    return hipGetLastError();
}

hipError_t launch_gather_cells(const int32_t *list, const int64_t *count, int64_t cap,
                               const double *T, const double *p, const double *Y, int64_t ldY,
                               int K, double *cT, double *cp, double *cY, hipStream_t s)
{
    return launch_gather_cells_ld(list, count, cap, cap, T, p, Y, ldY, K, cT, cp, cY, s);
}

hipError_t launch_scatter_cells_ld(const int32_t *list, const int64_t *count, int64_t cap, int64_t ldc,
                                   const double *cT, const double *cY, const int32_t *cstatus, int K,
                                   double *T, double *Y, int64_t ldY, int32_t *status, hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_cells_kernel, dim3(blocks_for(cap, 256)), dim3(256), 0, s, list, count,
                       cap, ldc, cT, cY, cstatus, K, T, Y, ldY, status);
    return hipGetLastError();
}

hipError_t launch_scatter_cells(const int32_t *list, const int64_t *count, int64_t cap,
                                const double *cT, const double *cY, const int32_t *cstatus, int K,
                                double *T, double *Y, int64_t ldY, int32_t *status, hipStream_t s)
{
    return launch_scatter_cells_ld(list, count, cap, cap, cT, cY, cstatus, K, T, Y, ldY, status, s);
}

hipError_t launch_sum_i64(const int64_t *v, int n, int64_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_i64_kernel, dim3(1), dim3(64), 0, s, v, n, out);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const int32_t *order, int64_t start, int64_t rows, const bf16_t *X,
                              int nin_pad, const float *Yt, int nout_pad, bf16_t *Xb, float *Yb,
                              hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for(rows, 256)), dim3(256), 0, s, order, start,
                       rows, X, nin_pad, Yt, nout_pad, Xb, Yb);
    return hipGetLastError();
}

hipError_t launch_loss_grad(const float *out, const float *Yb, int rows, int K, int nout_pad,
                            bf16_t *dOut, double *loss_acc, hipStream_t s)
{
    // fixed grid: partial sums land in loss_acc[1 ..], summed in order into loss_acc[0]
    constexpr int kParts = 64;
    hipLaunchKernelGGL(loss_grad_kernel, dim3(kParts), dim3(256), 0, s, out, Yb, rows, K, nout_pad,
                       dOut, loss_acc + 1);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, loss_acc + 1, kParts, loss_acc);
    return hipGetLastError();
}

hipError_t launch_bias_grad(const bf16_t *d, int rows, int N, int ld, float *part, float *db, hipStream_t s)
{
    hipLaunchKernelGGL(bias_grad_part_kernel, dim3(blocks_for(N, 64), kBiasChunks), dim3(64), 0, s, d, rows, N, ld,
                       part);
    hipLaunchKernelGGL(bias_grad_final_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, s, part, N, db);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(a.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, bf16_t *dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace chem

// Host side of the learned surrogate: parameter and normalisation storage,
// workspaces, the forward/backward/Adam sequence, training loop, inference
// with per-cell fallback to the integrator, and the weights file.

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <iterator>
#include <string>
#include <vector>

#include "host_common.h"
#include "surrogate.h"
#include "surr_file.h"

using chem::bf16_t;
using chem_host::check_hip;
using chem_host::fail;
using chem_host::is_device_ptr;
using chem_host::DevBuf;

namespace {

constexpr int kInPad = 64;            // network input padded for the MFMA K steps
constexpr int64_t kChunk = 262144;    // rows per inference pass (bounds the activations)
constexpr int64_t kFusedChunk = 2097152;   // rows per pass of the fused forward (input + output only)
constexpr double kBeta1 = 0.9, kBeta2 = 0.999, kEps = 1e-8;
constexpr double kPi = 3.14159265358979323846;

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Carves aligned sub-buffers out of one allocation.
struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(int64_t count)
    {
        T *r = (T *)(base + off);
        off += ((size_t)count * sizeof(T) + 255) & ~size_t(255);
        return r;
    }
};

template <typename T>
size_t carve_size(int64_t count) { return ((size_t)count * sizeof(T) + 255) & ~size_t(255); }

}  // namespace

struct chem_surr_s {
    chem_mech mech = nullptr;
    int device = 0;
    int K = 0, E = 0, nin = 0, h[3] = {0, 0, 0}, nout_pad = 0;
    // G > 1: one network per species (G = K), each nin -> hg[0] -> hg[1] ->
    // hg[2] -> 1, stored as one network of widths h = G hg whose layers 2-4
    // are block diagonal (only the diagonal blocks are stored and computed,
    // as grouped products); G = 1: one network nin -> h -> K
    int G = 1, hg[3] = {0, 0, 0};
    int hr[3] = {0, 0, 0};            // the per-species networks' real widths (hg: padded to 64)
    int in_l[4], out_l[4];            // padded GEMM shapes of the four layers (in_l: a weight row's length)
    int ain[4];                       // width of each layer's input activations (G in_l for grouped layers)
    int64_t off_W[4], off_b[4], n_pad = 0, n_logical = 0;
    float *master = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
    bf16_t *wbf = nullptr;
    bf16_t *wfrag = nullptr;          // the BF16 weights in the fused kernel's fragment order
    bool frag_valid = false;          // wfrag matches wbf
    double *norm_dev = nullptr;       // mu_x, sig_x, mu_y, sig_y
    double *coef_dev = nullptr;       // [E][K] n_ke / W_k, then [K] R / W_k
    int64_t *scalars = nullptr;       // [0] fallback count
    double *loss_dev = nullptr;       // [0] accumulated loss, [1..64] partials
    void *block = nullptr;
    std::vector<double> norm;         // host copy incl. dt
    bool norm_set = false;
    int64_t adam_t = 0;
    DevBuf act;                       // activations of one chunk / batch
    int64_t act_rows = 0;
    bool act_train = false;
    DevBuf fb;                        // fallback compaction
    int64_t fb_cap = 0;
    DevBuf io;                        // encoded rows and outputs of the fused inference pass
    int64_t io_rows = 0;
    int64_t pass_rows = 0;            // rows per inference pass (0: the library's choice)
    // inference: each pass's rejected cells are integrated on a second
    // stream (default priority) while the later passes run; fork events
    // (reused in turn: a wait binds to the record before it) and the join
    hipStream_t side = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    DevBuf pcount;                    // per-pass fallback counts
    int64_t pcount_len = 0;
};

namespace {

int check_surr(chem_surr s)
{
    if (!s) return fail(CHEM_EINVAL, "surrogate handle is NULL");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != s->device)
        return fail(CHEM_EINVAL, "the current HIP device is not the surrogate's device");
    return CHEM_OK;
}

int64_t norm_len(const chem_surr_s *s) { return 2 * (int64_t)s->nin + 2 * (int64_t)s->K + 1; }

// Activation buffers of `rows` rows: X, H1..H3 (BF16), OUT (FP32); with
// `train` also U1..U3 (FP32), Yb (FP32), dOut, D1..D3 (BF16).
struct Acts {
    bf16_t *X, *H[3], *dOut, *D[3];
    float *OUT, *U[3], *Yb, *bpart;
};

// Partial bias gradients: 64 row chunks times the widest layer.
int64_t bias_part_len(const chem_surr_s *s)
{
    int w = 0;
    for (int l = 0; l < 4; l++) w = s->out_l[l] > w ? s->out_l[l] : w;
    return 64 * (int64_t)w;
}

size_t acts_bytes(const chem_surr_s *s, int64_t rows, bool train)
{
    size_t b = carve_size<bf16_t>(rows * kInPad) + carve_size<float>(rows * s->nout_pad);
    for (int l = 0; l < 3; l++) b += carve_size<bf16_t>(rows * s->h[l]);
    if (train) {
        for (int l = 0; l < 3; l++) b += carve_size<float>(rows * s->h[l]) + carve_size<bf16_t>(rows * s->h[l]);
        b += carve_size<float>(rows * s->nout_pad) + carve_size<bf16_t>(rows * s->nout_pad);
        b += carve_size<float>(bias_part_len(s));
    }
    return b;
}

int ensure_acts(chem_surr_s *s, int64_t rows, bool train, hipStream_t st)
{
    if (rows <= s->act_rows && (!train || s->act_train)) return CHEM_OK;
    const int64_t r = rows > s->act_rows ? rows : s->act_rows;
    const bool t = train || s->act_train;
    int rc = s->act.grow(acts_bytes(s, r, t), st);
    if (rc != CHEM_OK) return rc;
    s->act_rows = r;
    s->act_train = t;
    return CHEM_OK;
}

Acts carve_acts(const chem_surr_s *s)
{
    Acts a{};
    Carver c{(char *)s->act.p};
    const int64_t rows = s->act_rows;
    a.X = c.take<bf16_t>(rows * kInPad);
    a.OUT = c.take<float>(rows * s->nout_pad);
    for (int l = 0; l < 3; l++) a.H[l] = c.take<bf16_t>(rows * s->h[l]);
    if (s->act_train) {
        for (int l = 0; l < 3; l++) {
            a.U[l] = c.take<float>(rows * s->h[l]);
            a.D[l] = c.take<bf16_t>(rows * s->h[l]);
        }
        a.Yb = c.take<float>(rows * s->nout_pad);
        a.dOut = c.take<bf16_t>(rows * s->nout_pad);
        a.bpart = c.take<float>(bias_part_len(s));
    }
    return a;
}

hipError_t gemm(const bf16_t *A, int64_t sam, int64_t sak, const bf16_t *B, int64_t sbn, int64_t sbk,
                int M, int N, int K, int epi, const float *bias, float *outf, int64_t ldf, bf16_t *outh,
                int64_t ldh, const float *u, int64_t ldu, hipStream_t st)
{
    chem::GemmArgs g{A, sam, sak, B, sbn, sbk, M, N, K, epi, bias, outf, ldf, outh, ldh, u, ldu};
    return chem::launch_gemm_bf16(g, st);
}

// G independent products, group z's operands offset by z times the strides.
struct GroupStrides {
    int groups;
    int64_t za, zb, zbias, zf, zh, zu;
};

hipError_t gemm_grouped(const GroupStrides &z, const bf16_t *A, int64_t sam, int64_t sak, const bf16_t *B,
                        int64_t sbn, int64_t sbk, int M, int N, int K, int epi, const float *bias, float *outf,
                        int64_t ldf, bf16_t *outh, int64_t ldh, const float *u, int64_t ldu, hipStream_t st)
{
    chem::GemmArgs g{A, sam, sak, B, sbn, sbk, M, N, K, epi, bias, outf, ldf, outh, ldh, u, ldu,
                     z.groups, z.za, z.zb, z.zbias, z.zf, z.zh, z.zu};
    return chem::launch_gemm_bf16(g, st);
}

bool fused_ok(const chem_surr_s *s)
{
    return s->G == 1 && s->in_l[0] == kInPad && chem::mlp_fused_supported(s->out_l);
}

// Columns per group of layer l's output: the whole layer unless it is grouped.
int group_n(const chem_surr_s *s, int l) { return s->G == 1 || l == 0 ? s->out_l[l] : (l == 3 ? 1 : s->hg[l]); }
bool grouped(const chem_surr_s *s, int l) { return s->G > 1 && l > 0; }

// Inference forward pass of all four layers in one kernel (activations in
// LDS); the fragment-order copy of the weights is made when they changed.
hipError_t forward_fused(chem_surr_s *s, const bf16_t *X, int64_t rows, float *OUT, int64_t ldo,
                         hipStream_t st)
{
    if (!s->frag_valid) {
        for (int l = 0; l < 4; l++) {
            hipError_t e = chem::launch_swizzle_frag(s->wbf + s->off_W[l], s->out_l[l], s->in_l[l],
                                                     s->wfrag + s->off_W[l], st);
            if (e != hipSuccess) return e;
        }
        s->frag_valid = true;
    }
    chem::MlpArgs a{};
    a.X = X;
    a.rows = rows;
    for (int l = 0; l < 4; l++) {
        a.W[l] = s->wfrag + s->off_W[l];
        a.b[l] = s->master + s->off_b[l];
        a.in_l[l] = s->in_l[l];
        a.out_l[l] = s->out_l[l];
    }
    a.out = OUT;
    a.ldo = ldo;
    return chem::launch_mlp_forward(a, st);
}

// Forward pass of `rows` rows of X; saves pre-activations when U[0] != NULL.
// Without saved pre-activations the fused kernel runs when the widths allow
// it (the same result bit for bit), unless `layered` asks for the GEMMs.
hipError_t forward(chem_surr_s *s, const bf16_t *X, int rows, bf16_t *const H[3],
                   float *const U[3], float *OUT, int64_t ldo, hipStream_t st, bool layered = false)
{
    if (!U[0] && !layered && fused_ok(s)) return forward_fused(s, X, rows, OUT, ldo, st);
    const bf16_t *in = X;
    hipError_t e = hipSuccess;
    for (int l = 0; l < 4 && e == hipSuccess; l++) {
        const int N = s->out_l[l], Kd = s->in_l[l], ld_in = s->ain[l];
        const bool last = l == 3;
        const int epi = last ? chem::kEpiBiasF32 : chem::kEpiBiasGeluBf16;
        float *outf = last ? OUT : U[l];
        const int64_t ldf = last ? ldo : N;
        bf16_t *outh = last ? nullptr : H[l];
        if (!grouped(s, l)) {
            e = gemm(in, ld_in, 1, s->wbf + s->off_W[l], Kd, 1, rows, N, Kd, epi, s->master + s->off_b[l], outf,
                     ldf, outh, N, nullptr, 0, st);
        } else {
            // group z: its block of the input columns times its block of weight rows
            const int gn = group_n(s, l);
            const GroupStrides z{s->G, Kd, (int64_t)gn * Kd, gn, gn, gn, 0};
            e = gemm_grouped(z, in, ld_in, 1, s->wbf + s->off_W[l], Kd, 1, rows, gn, Kd, epi,
                             s->master + s->off_b[l], outf, ldf, outh, N, nullptr, 0, st);
            if (last && e == hipSuccess && s->G < N)
                // the padding columns G .. nout_pad-1: zero weight rows and biases, so zeros
                e = gemm(in, ld_in, 1, s->wbf + s->off_W[l] + (int64_t)s->G * Kd, Kd, 1, rows, N - s->G, Kd, epi,
                         s->master + s->off_b[l] + s->G, outf + s->G, ldf, nullptr, 0, nullptr, 0, st);
        }
        if (!last) in = H[l];
    }
    return e;
}

// Backward pass from dOut (rows x nout_pad BF16) into s->grad.
hipError_t backward(const chem_surr_s *s, const Acts &a, const bf16_t *X, int rows, hipStream_t st)
{
    hipError_t e = hipSuccess;
    const bf16_t *d = a.dOut;
    int64_t ldd = s->nout_pad;
    for (int l = 3; l >= 0 && e == hipSuccess; l--) {
        const int Nout = s->out_l[l], Kin = s->in_l[l], gn = group_n(s, l);
        const bf16_t *hin = l == 0 ? X : a.H[l - 1];
        const int64_t ld_h = s->ain[l];
        const bf16_t *W = s->wbf + s->off_W[l];
        if (!grouped(s, l)) {
            // dW[n][k] = sum_r d[r][n] h[r][k]
            e = gemm(d, 1, ldd, hin, 1, ld_h, Nout, Kin, rows, chem::kEpiF32, nullptr, s->grad + s->off_W[l], Kin,
                     nullptr, 0, nullptr, 0, st);
        } else {
            const GroupStrides z{s->G, gn, Kin, 0, (int64_t)gn * Kin, 0, 0};
            e = gemm_grouped(z, d, 1, ldd, hin, 1, ld_h, gn, Kin, rows, chem::kEpiF32, nullptr,
                             s->grad + s->off_W[l], Kin, nullptr, 0, nullptr, 0, st);
        }
        if (e == hipSuccess)
            e = chem::launch_bias_grad(d, rows, Nout, (int)ldd, a.bpart, s->grad + s->off_b[l], st);
        if (l > 0 && e == hipSuccess) {
            // d_prev[r][k] = (sum_n d[r][n] W[n][k]) * gelu'(u_prev[r][k])
            if (!grouped(s, l)) {
                e = gemm(d, ldd, 1, W, 1, Kin, rows, Kin, Nout, chem::kEpiGeluGradBf16, nullptr, nullptr, 0,
                         a.D[l - 1], ld_h, a.U[l - 1], ld_h, st);
            } else {
                const GroupStrides z{s->G, gn, (int64_t)gn * Kin, 0, 0, Kin, Kin};
                e = gemm_grouped(z, d, ldd, 1, W, 1, Kin, rows, Kin, gn, chem::kEpiGeluGradBf16, nullptr, nullptr,
                                 0, a.D[l - 1], ld_h, a.U[l - 1], ld_h, st);
            }
            d = a.D[l - 1];
            ldd = ld_h;
        }
    }
    return e;
}

// logical <-> padded parameter vectors
void logical_map(const chem_surr_s *s, std::vector<std::pair<int64_t, int64_t>> &runs)
{
    // (padded offset, length) runs in logical order: layer by layer (W rows,
    // then b) for one network; network by network for the per-species ones
    runs.clear();
    if (s->G == 1) {
        const int in_real[4] = {s->nin, s->h[0], s->h[1], s->h[2]};
        const int out_real[4] = {s->h[0], s->h[1], s->h[2], s->K};
        for (int l = 0; l < 4; l++) {
            for (int r = 0; r < out_real[l]; r++)
                runs.push_back({s->off_W[l] + (int64_t)r * s->in_l[l], in_real[l]});
            runs.push_back({s->off_b[l], out_real[l]});
        }
        return;
    }
    const int in_real[4] = {s->nin, s->hr[0], s->hr[1], s->hr[2]};
    const int out_real[4] = {s->hr[0], s->hr[1], s->hr[2], 1};
    const int out_pad[4] = {s->hg[0], s->hg[1], s->hg[2], 1};
    for (int g = 0; g < s->G; g++)
        for (int l = 0; l < 4; l++) {
            const int64_t row0 = (int64_t)g * out_pad[l];
            for (int r = 0; r < out_real[l]; r++)
                runs.push_back({s->off_W[l] + (row0 + r) * s->in_l[l], in_real[l]});
            runs.push_back({s->off_b[l] + row0, out_real[l]});
        }
}

int upload_logical(chem_surr_s *s, float *dev, const float *host, int64_t count)
{
    if (count != s->n_logical) return fail(CHEM_EINVAL, "parameter count does not match the network");
    std::vector<float> pad((size_t)s->n_pad, 0.0f);
    std::vector<std::pair<int64_t, int64_t>> runs;
    logical_map(s, runs);
    int64_t o = 0;
    for (auto &r : runs) {
        std::memcpy(&pad[(size_t)r.first], host + o, (size_t)r.second * sizeof(float));
        o += r.second;
    }
    return check_hip(hipMemcpy(dev, pad.data(), pad.size() * sizeof(float), hipMemcpyHostToDevice),
                     "parameter upload");
}

int download_logical(chem_surr_s *s, const float *dev, float *host, int64_t count)
{
    if (count != s->n_logical) return fail(CHEM_EINVAL, "parameter count does not match the network");
    std::vector<float> pad((size_t)s->n_pad);
    int rc = check_hip(hipMemcpy(pad.data(), dev, pad.size() * sizeof(float), hipMemcpyDeviceToHost),
                       "parameter download");
    if (rc != CHEM_OK) return rc;
    std::vector<std::pair<int64_t, int64_t>> runs;
    logical_map(s, runs);
    int64_t o = 0;
    for (auto &r : runs) {
        std::memcpy(host + o, &pad[(size_t)r.first], (size_t)r.second * sizeof(float));
        o += r.second;
    }
    return CHEM_OK;
}

int refresh_bf16(chem_surr_s *s, hipStream_t st)
{
    s->frag_valid = false;
    return check_hip(chem::launch_to_bf16(s->master, s->wbf, s->n_pad, st), "bf16 weights");
}

// Fallback compaction buffers for up to n cells: list, T, p, Y (K x cap), status.
struct Fallback {
    int32_t *list;
    double *T, *p, *Y;
    int32_t *status;
    int64_t cap;
};

int ensure_fb(chem_surr_s *s, int64_t n, Fallback &f, hipStream_t st)
{
    const int K = s->K;
    if (n > s->fb_cap) {
        const size_t b = carve_size<int32_t>(n) + 2 * carve_size<double>(n) + carve_size<double>(n * K) +
                         carve_size<int32_t>(n);
        int rc = s->fb.grow(b, st);
        if (rc != CHEM_OK) return rc;
        s->fb_cap = n;
    }
    Carver fc{(char *)s->fb.p};
    f.cap = s->fb_cap;
    f.list = fc.take<int32_t>(f.cap);
    f.T = fc.take<double>(f.cap);
    f.p = fc.take<double>(f.cap);
    f.Y = fc.take<double>(f.cap * K);
    f.status = fc.take<int32_t>(f.cap);
    return CHEM_OK;
}

chem::ApplyArgs apply_args(const chem_surr_s *s, const chem_surr_checks &c)
{
    chem::ApplyArgs a{};
    a.species = s->mech->view.species;
    a.ncoef = s->coef_dev;
    a.rw = s->coef_dev + (int64_t)s->E * s->K;
    a.K = s->K;
    a.E = s->E;
    a.two_range = s->mech->view.two_range;
    a.mu_y = s->norm_dev + 2 * s->nin;
    a.sig_y = s->norm_dev + 2 * s->nin + s->K;
    a.elem_tol = c.elem_tol;
    a.sum_tol = c.sum_tol;
    a.neg_tol = c.neg_tol;
    a.T_out_min = c.T_out_min;
    a.T_out_max = c.T_out_max;
    a.T_in_min = c.T_in_min;
    a.T_in_max = c.T_in_max;
    a.dT_gate = c.dT_gate;
    return a;
}

// Adam constants of the handle's current step (adam_t already advanced).
chem::AdamArgs adam_args(chem_surr_s *s, double lr)
{
    const double t = (double)s->adam_t;
    return chem::AdamArgs{s->master, s->am, s->av, s->grad, s->n_pad, (float)lr, (float)kBeta1,
                          (float)kBeta2, (float)(1.0 - kBeta1), (float)(1.0 - kBeta2), (float)kEps,
                          (float)(1.0 - std::pow(kBeta1, t)), (float)(1.0 - std::pow(kBeta2, t))};
}

}  // namespace

extern "C" {

int chem_surrogate_default_checks(chem_surr_checks *c)
{
    if (!c) return fail(CHEM_EINVAL, "checks is NULL");
    std::memset(c, 0, sizeof(*c));
    c->elem_tol = 1e-3;
    c->sum_tol = 1e-3;
    c->neg_tol = 1e-6;
    c->T_out_min = 250.0;
    c->T_out_max = 2600.0;
    c->T_in_min = 300.0;
    c->T_in_max = 2500.0;
    c->dT_gate = 0.0;
    return CHEM_OK;
}

namespace {

// One network nin -> h1 -> h2 -> h3 -> K (G = 1) or K per-species networks
// nin -> h1 -> h2 -> h3 -> 1 (G = K).
int create_surrogate(chem_mech mech, int32_t h1, int32_t h2, int32_t h3, bool per_species, chem_surr *out)
{
    if (!mech || !out) return fail(CHEM_EINVAL, "mech and out must not be NULL");
    *out = nullptr;
    const int K = mech->host.K, E = mech->host.E;
    if (K + 2 > kInPad) return fail(CHEM_EUNSUP, "the surrogate takes at most 62 species");
    if (E > 8) return fail(CHEM_EUNSUP, "the surrogate takes at most 8 elements");
    if (per_species) {
        // any width: each network's layers are padded to multiples of 64 with
        // units whose weights and biases stay zero (their gradients are zero)
        for (int v : {h1, h2, h3})
            if (v < 16 || v > 4096) return fail(CHEM_EINVAL, "hidden widths must be in [16, 4096]");
    } else {
        for (int v : {h1, h2, h3})
            if (v < 64 || v % 64 != 0 || v > 4096)
                return fail(CHEM_EINVAL, "hidden widths must be multiples of 64 in [64, 4096]");
    }
    const int G = per_species ? K : 1;
    const int hr[3] = {h1, h2, h3};
    h1 = round_up(h1, 64);
    h2 = round_up(h2, 64);
    h3 = round_up(h3, 64);
    if ((int64_t)G * h1 > 65536 || (int64_t)G * h2 > 65536 || (int64_t)G * h3 > 65536)
        return fail(CHEM_EINVAL, "the per-species networks' layers exceed 65,536 units in all");
    int prev = 0;
    hipGetDevice(&prev);
    if (hipSetDevice(mech->device) != hipSuccess) return fail(CHEM_EHIP, "hipSetDevice failed");
    auto *s = new chem_surr_s();
    s->mech = mech;
    s->device = mech->device;
    s->K = K;
    s->E = E;
    s->nin = K + 2;
    s->G = G;
    for (int l = 0; l < 3; l++) s->hr[l] = hr[l];
    s->hg[0] = h1;
    s->hg[1] = h2;
    s->hg[2] = h3;
    s->h[0] = G * h1;
    s->h[1] = G * h2;
    s->h[2] = G * h3;
    s->nout_pad = round_up(K, 16);
    const int in_l[4] = {kInPad, h1, h2, h3};
    const int out_l[4] = {G * h1, G * h2, G * h3, s->nout_pad};
    const int ain[4] = {kInPad, G * h1, G * h2, G * h3};
    int64_t off = 0;
    s->n_logical = 0;
    for (int l = 0; l < 4; l++) {
        s->in_l[l] = in_l[l];
        s->out_l[l] = out_l[l];
        s->ain[l] = ain[l];
        s->off_W[l] = off;
        off += (int64_t)in_l[l] * out_l[l];
        s->off_b[l] = off;
        off += round_up(out_l[l], 64);
    }
    if (G == 1)
        s->n_logical = (int64_t)s->nin * h1 + h1 + (int64_t)h1 * h2 + h2 + (int64_t)h2 * h3 + h3 + (int64_t)h3 * K + K;
    else
        s->n_logical = (int64_t)G * ((int64_t)s->nin * hr[0] + hr[0] + (int64_t)hr[0] * hr[1] + hr[1] +
                                     (int64_t)hr[1] * hr[2] + hr[2] + hr[2] + 1);
    s->n_pad = off;
    const int64_t nn = 2 * (int64_t)s->nin + 2 * K;
    const size_t bytes = 4 * carve_size<float>(s->n_pad) + 2 * carve_size<bf16_t>(s->n_pad) +
                         carve_size<double>(nn) + carve_size<double>((int64_t)(E + 1) * K) +
                         carve_size<int64_t>(8) + carve_size<double>(80);
    if (hipMalloc(&s->block, bytes) != hipSuccess) {
        (void)hipGetLastError();
        hipSetDevice(prev);
        delete s;
        return fail(CHEM_ENOMEM, "surrogate allocation failed");
    }
    Carver c{(char *)s->block};
    s->master = c.take<float>(s->n_pad);
    s->grad = c.take<float>(s->n_pad);
    s->am = c.take<float>(s->n_pad);
    s->av = c.take<float>(s->n_pad);
    s->wbf = c.take<bf16_t>(s->n_pad);
    s->wfrag = c.take<bf16_t>(s->n_pad);
    s->norm_dev = c.take<double>(nn);
    s->coef_dev = c.take<double>((int64_t)(E + 1) * K);
    s->scalars = c.take<int64_t>(8);
    s->loss_dev = c.take<double>(80);
    int rc = check_hip(hipMemset(s->block, 0, bytes), "surrogate init");
    // decode constants: n_ke / W_k and R / W_k, each one FP64 division here
    std::vector<double> cnt((size_t)(E + 1) * K);
    for (int e = 0; e < E; e++)
        for (int k = 0; k < K; k++) cnt[(size_t)e * K + k] = mech->host.counts[k][e] / mech->W[k];
    for (int k = 0; k < K; k++) cnt[(size_t)E * K + k] = 8.31446261815324 / mech->W[k];
    if (rc == CHEM_OK)
        rc = check_hip(hipMemcpy(s->coef_dev, cnt.data(), cnt.size() * sizeof(double), hipMemcpyHostToDevice),
                       "decode constants upload");
    s->norm.assign((size_t)norm_len(s), 0.0);
    if (rc == CHEM_OK)
        rc = check_hip(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking), "fallback stream");
    for (int i = 0; i < 4 && rc == CHEM_OK; i++)
        rc = check_hip(hipEventCreateWithFlags(&s->ev[i], hipEventDisableTiming), "fallback events");
    hipSetDevice(prev);
    if (rc != CHEM_OK) {
        for (hipEvent_t e : s->ev)
            if (e) hipEventDestroy(e);
        if (s->side) hipStreamDestroy(s->side);
        hipFree(s->block);
        delete s;
        return rc;
    }
    *out = s;
    return CHEM_OK;
}

}  // namespace

int chem_surrogate_create(chem_mech mech, int32_t h1, int32_t h2, int32_t h3, chem_surr *out)
{
    return create_surrogate(mech, h1, h2, h3, false, out);
}

int chem_surrogate_create_species(chem_mech mech, int32_t h1, int32_t h2, int32_t h3, chem_surr *out)
{
    return create_surrogate(mech, h1, h2, h3, true, out);
}

int chem_surrogate_groups(chem_surr s, int32_t *groups)
{
    if (!s || !groups) return fail(CHEM_EINVAL, "surrogate and groups must not be NULL");
    *groups = s->G;
    return CHEM_OK;
}

void chem_free_surrogate(chem_surr s)
{
    if (!s) return;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(s->device);
    s->act.release();
    s->fb.release();
    s->io.release();
    s->pcount.release();
    if (s->side) {
        hipStreamSynchronize(s->side);
        hipStreamDestroy(s->side);
    }
    for (hipEvent_t e : s->ev)
        if (e) hipEventDestroy(e);
    if (s->block) hipFree(s->block);
    hipSetDevice(prev);
    delete s;
}

int chem_surrogate_info(chem_surr s, int64_t *dims)
{
    if (!s || !dims) return fail(CHEM_EINVAL, "surrogate and dims must not be NULL");
    dims[0] = s->nin;
    dims[1] = s->h[0];
    dims[2] = s->h[1];
    dims[3] = s->h[2];
    dims[4] = s->K;
    dims[5] = s->n_logical;
    return CHEM_OK;
}

int chem_surrogate_set_params(chem_surr s, const float *params, int64_t count)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (!params) return fail(CHEM_EINVAL, "params is NULL");
    rc = upload_logical(s, s->master, params, count);
    if (rc != CHEM_OK) return rc;
    rc = refresh_bf16(s, nullptr);
    if (rc != CHEM_OK) return rc;
    // a new parameter vector restarts the optimiser
    s->adam_t = 0;
    rc = check_hip(hipMemset(s->am, 0, 2 * carve_size<float>(s->n_pad)), "optimiser reset");
    if (rc != CHEM_OK) return rc;
    return check_hip(hipDeviceSynchronize(), "parameter upload");
}

int chem_surrogate_get_params(chem_surr s, float *params, int64_t count)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (!params) return fail(CHEM_EINVAL, "params is NULL");
    rc = check_hip(hipDeviceSynchronize(), "sync");
    if (rc != CHEM_OK) return rc;
    return download_logical(s, s->master, params, count);
}

int chem_surrogate_set_norm(chem_surr s, const double *norm, int64_t count)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (!norm || count != norm_len(s)) return fail(CHEM_EINVAL, "normalisation vector has the wrong length");
    for (int64_t i = 0; i < count; i++)
        if (!std::isfinite(norm[i])) return fail(CHEM_EINVAL, "normalisation values must be finite");
    if (!(norm[count - 1] > 0.0)) return fail(CHEM_EINVAL, "dt of the normalisation must be > 0");
    s->norm.assign(norm, norm + count);
    s->norm_set = true;
    return check_hip(hipMemcpy(s->norm_dev, norm, (size_t)(count - 1) * sizeof(double), hipMemcpyHostToDevice),
                     "normalisation upload");
}

int chem_surrogate_get_norm(chem_surr s, double *norm, int64_t count)
{
    if (!s || !norm || count != norm_len(s)) return fail(CHEM_EINVAL, "normalisation vector has the wrong length");
    std::memcpy(norm, s->norm.data(), (size_t)count * sizeof(double));
    return CHEM_OK;
}

int chem_surrogate_fit_norm(chem_surr s, const double *T, const double *p, const double *Y,
                            int64_t ldY, const double *Yn, int64_t ldYn, int64_t n, double dt,
                            void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (n < 2 || ldY < n || ldYn < n) return fail(CHEM_EINVAL, "need n >= 2 samples and ldY, ldYn >= n");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CHEM_EINVAL, "dt must be finite and > 0");
    if (!is_device_ptr(T) || !is_device_ptr(p) || !is_device_ptr(Y) || !is_device_ptr(Yn))
        return fail(CHEM_EINVAL, "T, p, Y and Ynext must be device pointers");
    hipStream_t st = (hipStream_t)stream;
    rc = check_hip(chem::launch_fit_norm(T, p, Y, ldY, Yn, ldYn, n, s->K, s->norm_dev, st), "fit_norm");
    if (rc != CHEM_OK) return rc;
    const int64_t nn = norm_len(s) - 1;
    rc = check_hip(hipMemcpyAsync(s->norm.data(), s->norm_dev, (size_t)nn * sizeof(double),
                                  hipMemcpyDeviceToHost, st), "normalisation download");
    if (rc != CHEM_OK) return rc;
    rc = check_hip(hipStreamSynchronize(st), "sync");
    s->norm[(size_t)nn] = dt;
    s->norm_set = true;
    return rc;
}

int chem_surrogate_encode(chem_surr s, const double *T, const double *p, const double *Y, int64_t ldY,
                          int64_t n, uint16_t *X, void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK || n == 0) return rc;
    if (n < 0 || ldY < n) return fail(CHEM_EINVAL, "need ncells >= 0 and ldY >= ncells");
    if (!s->norm_set) return fail(CHEM_EINVAL, "the surrogate has no normalisation");
    if (!is_device_ptr(T) || !is_device_ptr(p) || !is_device_ptr(Y) || !is_device_ptr(X))
        return fail(CHEM_EINVAL, "T, p, Y and X must be device pointers");
    return check_hip(chem::launch_encode(T, p, Y, ldY, n, s->K, kInPad, s->norm_dev, X, (hipStream_t)stream),
                     "encode");
}

int chem_surrogate_forward(chem_surr s, const uint16_t *X, int64_t n, float *out, int64_t ldo, void *stream)
{
    return chem_surrogate_forward_path(s, X, n, out, ldo, 0, stream);
}

int chem_surrogate_forward_path(chem_surr s, const uint16_t *X, int64_t n, float *out, int64_t ldo, int32_t path,
                                void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (path < 0 || path > 2) return fail(CHEM_EINVAL, "path must be 0, 1 or 2");
    if (path == 2 && !fused_ok(s))
        return fail(CHEM_EUNSUP, "the fused forward kernel takes one network with widths up to 512");
    if (n == 0) return CHEM_OK;
    if (n < 0 || ldo < s->nout_pad) return fail(CHEM_EINVAL, "need ncells >= 0 and ldo >= K rounded up to 16");
    if (!is_device_ptr(X) || !is_device_ptr(out)) return fail(CHEM_EINVAL, "X and out must be device pointers");
    if (path != 1 && fused_ok(s)) return check_hip(forward_fused(s, (const bf16_t *)X, n, out, ldo, (hipStream_t)stream),
                                                   "fused forward");
    const int64_t rows = n < kChunk ? n : kChunk;
    hipStream_t st = (hipStream_t)stream;
    rc = ensure_acts(s, rows, false, st);
    if (rc != CHEM_OK) return rc;
    Acts a = carve_acts(s);
    float *noU[3] = {nullptr, nullptr, nullptr};
    for (int64_t r0 = 0; r0 < n; r0 += kChunk) {
        const int rr = (int)(n - r0 < kChunk ? n - r0 : kChunk);
        hipError_t e = forward(s, X + r0 * kInPad, rr, a.H, noU, out + r0 * ldo, ldo, st, true);
        if (e != hipSuccess) return check_hip(e, "forward");
    }
    return CHEM_OK;
}

int chem_surrogate_forward_trace(chem_surr s, const uint16_t *X, int64_t n, uint16_t *H1, uint16_t *H2,
                                 uint16_t *H3, float *out, int64_t ldo, void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (n == 0) return CHEM_OK;
    if (n < 0 || n > (1 << 20) || ldo < s->nout_pad)
        return fail(CHEM_EINVAL, "need 0 <= ncells <= 2^20 and ldo >= K rounded up to 16");
    if (!is_device_ptr(X) || !is_device_ptr(H1) || !is_device_ptr(H2) || !is_device_ptr(H3) || !is_device_ptr(out))
        return fail(CHEM_EINVAL, "X, H1, H2, H3 and out must be device pointers");
    bf16_t *const H[3] = {(bf16_t *)H1, (bf16_t *)H2, (bf16_t *)H3};
    float *noU[3] = {nullptr, nullptr, nullptr};
    return check_hip(forward(s, (const bf16_t *)X, (int)n, H, noU, out, ldo, (hipStream_t)stream, true),
                     "forward trace");
}

int chem_surrogate_apply(chem_surr s, double *T, const double *p, double *Y, int64_t ldY, int64_t n,
                         const float *out, int64_t ldo, const chem_surr_checks *checks, int32_t *mask,
                         void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK || n == 0) return rc;
    if (n < 0 || ldY < n || ldo < s->nout_pad) return fail(CHEM_EINVAL, "bad sizes");
    if (n > INT32_MAX) return fail(CHEM_EINVAL, "ncells must fit in int32");
    if (!s->norm_set) return fail(CHEM_EINVAL, "the surrogate has no normalisation");
    if (!is_device_ptr(T) || !is_device_ptr(p) || !is_device_ptr(Y) || !is_device_ptr(out) ||
        (mask && !is_device_ptr(mask)))
        return fail(CHEM_EINVAL, "arrays must be device pointers");
    chem_surr_checks c;
    chem_surrogate_default_checks(&c);
    if (checks) c = *checks;
    if (ldo != s->nout_pad) return fail(CHEM_EINVAL, "ldo must equal K rounded up to 16 here");
    Fallback fb;
    hipStream_t st = (hipStream_t)stream;
    rc = ensure_fb(s, n, fb, st);
    if (rc != CHEM_OK) return rc;
    rc = check_hip(chem::launch_zero_i64(s->scalars, 1, st), "zero");
    if (rc != CHEM_OK) return rc;
    return check_hip(chem::launch_apply(apply_args(s, c), T, p, Y, ldY, n, 0, out, (int)ldo, mask, nullptr,
                                        fb.list, s->scalars, st),
                     "apply");
}

namespace {

// Workspace of an inference call over n cells: the encoded rows and outputs
// of one pass (fused forward) or every activation of one pass (per-layer
// GEMMs), and the fallback compaction buffers for all n cells.
struct InferWork {
    bool fused = false;
    int64_t chunk = 0;   // rows per pass
    bf16_t *X = nullptr;
    float *OUT = nullptr;
    Acts a{};
    Fallback fb{};
};

int infer_workspace(chem_surr_s *s, int64_t n, hipStream_t st, InferWork &w)
{
    // the fused forward needs only the encoded rows and the outputs, so it
    // takes larger passes; the layered GEMMs keep every activation
    w.fused = fused_ok(s);
    w.chunk = w.fused ? kFusedChunk : kChunk;
    if (s->pass_rows > 0 && s->pass_rows < w.chunk) w.chunk = s->pass_rows;
    const int64_t rows = n < w.chunk ? n : w.chunk;
    int rc;
    if (w.fused) {
        if (rows > s->io_rows) {
            rc = s->io.grow(carve_size<bf16_t>(rows * kInPad) + carve_size<float>(rows * s->nout_pad), st);
            if (rc != CHEM_OK) return rc;
            s->io_rows = rows;
        }
        Carver ic{(char *)s->io.p};
        w.X = ic.take<bf16_t>(s->io_rows * kInPad);
        w.OUT = ic.take<float>(s->io_rows * s->nout_pad);
    } else {
        rc = ensure_acts(s, rows, false, st);
        if (rc != CHEM_OK) return rc;
        w.a = carve_acts(s);
        w.X = w.a.X;
        w.OUT = w.a.OUT;
    }
    return ensure_fb(s, n, w.fb, st);
}

}  // namespace

int chem_surrogate_reserve(chem_surr s, int64_t ncells, void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (ncells < 0 || ncells > INT32_MAX) return fail(CHEM_EINVAL, "ncells must be in 0..2^31-1");
    if (ncells == 0) return CHEM_OK;
    InferWork w;
    return infer_workspace(s, ncells, (hipStream_t)stream, w);
}

int chem_surrogate_set_pass_rows(chem_surr s, int64_t rows)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (rows < 0 || rows > INT32_MAX) return fail(CHEM_EINVAL, "rows must be in 0..2^31-1");
    s->pass_rows = rows;
    return CHEM_OK;
}

int chem_surrogate_infer(chem_surr s, double *T, const double *p, double *Y, int64_t ldY, int64_t n,
                         double dt, const chem_opts *opts, const chem_surr_checks *checks,
                         int32_t *mask, int32_t *status, int64_t *fallback_count, void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK || n == 0) return rc;
    if (n < 0 || ldY < n) return fail(CHEM_EINVAL, "need ncells >= 0 and ldY >= ncells");
    if (n > INT32_MAX) return fail(CHEM_EINVAL, "ncells must fit in int32");
    if (!s->norm_set) return fail(CHEM_EINVAL, "the surrogate has no normalisation");
    const double tdt = s->norm.back();
    if (!(std::fabs(dt - tdt) <= 1e-12 * tdt))
        return fail(CHEM_EINVAL, "dt differs from the flow step the surrogate was trained for");
    if (!is_device_ptr(T) || !is_device_ptr(p) || !is_device_ptr(Y) || (mask && !is_device_ptr(mask)) ||
        (status && !is_device_ptr(status)) || (fallback_count && !is_device_ptr(fallback_count)))
        return fail(CHEM_EINVAL, "arrays must be device pointers");
    chem_surr_checks c;
    chem_surrogate_default_checks(&c);
    if (checks) c = *checks;
    const int K = s->K;
    hipStream_t st = (hipStream_t)stream;
    InferWork w;
    rc = infer_workspace(s, n, st, w);
    if (rc != CHEM_OK) return rc;
    const bool fused = w.fused;
    const int64_t chunk = w.chunk;
    bf16_t *Xc = w.X;
    float *OUTc = w.OUT;
    Acts &a = w.a;
    Fallback &fb = w.fb;
    float *noU[3] = {nullptr, nullptr, nullptr};
    int64_t *count = fallback_count ? fallback_count : s->scalars;
    // per-pass counts: pass q's rejected cells go to fb.list[r0 ..] (at most
    // its rr rows), gathered into fb.T/p/Y/status[r0 ..] and integrated on
    // the side stream as soon as the pass is applied
    const int64_t npass = (n + chunk - 1) / chunk;
    if (npass > s->pcount_len) {
        rc = s->pcount.grow(carve_size<int64_t>(npass), st);
        if (rc != CHEM_OK) return rc;
        s->pcount_len = npass;
    }
    int64_t *pc = (int64_t *)s->pcount.p;
    rc = check_hip(chem::launch_zero_i64(pc, (int)npass, st), "zero");
    if (rc != CHEM_OK) return rc;
    const chem::ApplyArgs aa = apply_args(s, c);
    hipStream_t sd = s->side;
    int64_t q = 0;
    for (int64_t r0 = 0; r0 < n; r0 += chunk, q++) {
        const int rr = (int)(n - r0 < chunk ? n - r0 : chunk);
        hipError_t e = chem::launch_encode(T + r0, p + r0, Y + r0, ldY, rr, K, kInPad, s->norm_dev, Xc, st);
        if (e == hipSuccess)
            e = fused ? forward_fused(s, Xc, rr, OUTc, s->nout_pad, st)
                      : forward(s, Xc, rr, a.H, noU, OUTc, s->nout_pad, st, true);
        if (e == hipSuccess)
            e = chem::launch_apply(aa, T + r0, p + r0, Y + r0, ldY, rr, r0, OUTc, s->nout_pad,
                                   mask ? mask + r0 : nullptr, status ? status + r0 : nullptr, fb.list + r0,
                                   pc + q, st);
        if (e != hipSuccess) return check_hip(e, "surrogate pass");
        hipEvent_t fork = s->ev[q % 3];
        rc = check_hip(hipEventRecord(fork, st), "fork event");
        if (rc == CHEM_OK) rc = check_hip(hipStreamWaitEvent(sd, fork, 0), "fork wait");
        if (rc == CHEM_OK)
            rc = check_hip(chem::launch_gather_cells_ld(fb.list + r0, pc + q, rr, fb.cap, T, p, Y, ldY, K,
                                                        fb.T + r0, fb.p + r0, fb.Y + r0, sd),
                           "gather");
        if (rc == CHEM_OK)
            rc = chem_host::integrate_cells(s->mech, fb.T + r0, fb.p + r0, fb.Y + r0, fb.cap, rr, dt, opts,
                                            fb.status + r0, nullptr, sd, pc + q);
        if (rc == CHEM_OK)
            rc = check_hip(chem::launch_scatter_cells_ld(fb.list + r0, pc + q, rr, fb.cap, fb.T + r0, fb.Y + r0,
                                                         fb.status + r0, K, T, Y, ldY, status, sd),
                           "scatter");
        if (rc != CHEM_OK) return rc;
    }
    rc = check_hip(hipEventRecord(s->ev[3], sd), "join event");
    if (rc == CHEM_OK) rc = check_hip(hipStreamWaitEvent(st, s->ev[3], 0), "join wait");
    if (rc == CHEM_OK) rc = check_hip(chem::launch_sum_i64(pc, (int)npass, count, st), "fallback count");
    return rc;
}

int chem_surrogate_grad(chem_surr s, const uint16_t *X, const float *Yt, int64_t ldt, int64_t n,
                        double *loss, void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (n < 1 || n > (1 << 20) || ldt < s->K) return fail(CHEM_EINVAL, "need 1 <= n <= 2^20 and ldt >= K");
    if (!is_device_ptr(X) || !is_device_ptr(Yt)) return fail(CHEM_EINVAL, "X and Yt must be device pointers");
    hipStream_t st = (hipStream_t)stream;
    rc = ensure_acts(s, n, true, st);
    if (rc != CHEM_OK) return rc;
    Acts a = carve_acts(s);
    // targets into the padded layout
    rc = check_hip(hipMemsetAsync(a.Yb, 0, (size_t)n * s->nout_pad * sizeof(float), st), "clear");
    if (rc != CHEM_OK) return rc;
    rc = check_hip(hipMemcpy2DAsync(a.Yb, (size_t)s->nout_pad * sizeof(float), Yt, (size_t)ldt * sizeof(float),
                                    (size_t)s->K * sizeof(float), (size_t)n, hipMemcpyDeviceToDevice, st),
                   "targets");
    if (rc != CHEM_OK) return rc;
    rc = check_hip(hipMemsetAsync(s->loss_dev, 0, sizeof(double), st), "clear");
    if (rc != CHEM_OK) return rc;
    hipError_t e = forward(s, X, (int)n, a.H, a.U, a.OUT, s->nout_pad, st);
    if (e == hipSuccess) e = chem::launch_loss_grad(a.OUT, a.Yb, (int)n, s->K, s->nout_pad, a.dOut, s->loss_dev, st);
    if (e == hipSuccess) e = backward(s, a, X, (int)n, st);
    if (e != hipSuccess) return check_hip(e, "gradient");
    double acc = 0.0;
    rc = check_hip(hipMemcpyAsync(&acc, s->loss_dev, sizeof(double), hipMemcpyDeviceToHost, st), "loss");
    if (rc != CHEM_OK) return rc;
    rc = check_hip(hipStreamSynchronize(st), "sync");
    if (loss) *loss = acc / ((double)n * s->K);
    return rc;
}

int chem_surrogate_get_grads(chem_surr s, float *grads, int64_t count)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (!grads) return fail(CHEM_EINVAL, "grads is NULL");
    rc = check_hip(hipDeviceSynchronize(), "sync");
    if (rc != CHEM_OK) return rc;
    return download_logical(s, s->grad, grads, count);
}

int chem_surrogate_set_grads(chem_surr s, const float *grads, int64_t count)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (!grads) return fail(CHEM_EINVAL, "grads is NULL");
    return upload_logical(s, s->grad, grads, count);
}

int chem_surrogate_adam(chem_surr s, double lr, void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (!(lr >= 0.0) || !std::isfinite(lr)) return fail(CHEM_EINVAL, "lr must be finite and >= 0");
    s->adam_t++;
    chem::AdamArgs a = adam_args(s, lr);
    hipStream_t st = (hipStream_t)stream;
    rc = check_hip(chem::launch_adam(a, st), "adam");
    if (rc != CHEM_OK) return rc;
    return refresh_bf16(s, st);
}

int chem_surrogate_train_part(chem_surr s, const double *T, const double *p, const double *Y, int64_t ldY,
                              const double *Yn, int64_t ldYn, int64_t n, const int32_t *order,
                              int32_t first_epoch, int32_t epochs, int32_t total_epochs, int32_t batch,
                              double lr0, double lr1, double *loss_per_epoch, void *stream)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (n < 1 || ldY < n || ldYn < n) return fail(CHEM_EINVAL, "need n >= 1 and ldY, ldYn >= n");
    if (n > INT32_MAX) return fail(CHEM_EINVAL, "n must fit in int32");
    if (epochs < 1 || batch < 1 || batch > (1 << 20)) return fail(CHEM_EINVAL, "bad epochs or batch");
    if (first_epoch < 0 || total_epochs < 1 || (int64_t)first_epoch + epochs > total_epochs)
        return fail(CHEM_EINVAL, "need 0 <= first_epoch and first_epoch + epochs <= total_epochs");
    if (!(lr0 >= 0.0) || !(lr1 >= 0.0)) return fail(CHEM_EINVAL, "learning rates must be >= 0");
    if (!s->norm_set) return fail(CHEM_EINVAL, "the surrogate has no normalisation");
    if (!is_device_ptr(T) || !is_device_ptr(p) || !is_device_ptr(Y) || !is_device_ptr(Yn) ||
        (order && !is_device_ptr(order)))
        return fail(CHEM_EINVAL, "arrays must be device pointers");
    hipStream_t st = (hipStream_t)stream;
    const int64_t rows = batch < n ? batch : n;
    rc = ensure_acts(s, rows, true, st);
    if (rc != CHEM_OK) return rc;
    DevBuf data;
    rc = data.grow(carve_size<bf16_t>(n * kInPad) + carve_size<float>(n * s->nout_pad), st);
    if (rc != CHEM_OK) return rc;
    Carver dc{(char *)data.p};
    bf16_t *Xall = dc.take<bf16_t>(n * kInPad);
    float *Yall = dc.take<float>(n * s->nout_pad);
    Acts a = carve_acts(s);
    hipError_t e = chem::launch_encode(T, p, Y, ldY, n, s->K, kInPad, s->norm_dev, Xall, st);
    if (e == hipSuccess)
        e = chem::launch_targets(Y, ldY, Yn, ldYn, n, s->K, s->nout_pad, s->norm_dev + 2 * s->nin,
                                 s->norm_dev + 2 * s->nin + s->K, Yall, st);
    const int64_t per_epoch = (n + batch - 1) / batch;
    const int64_t total = per_epoch * total_epochs;
    int64_t step = per_epoch * first_epoch;
    for (int ep = 0; ep < epochs && e == hipSuccess; ep++) {
        e = hipMemsetAsync(s->loss_dev, 0, sizeof(double), st);
        for (int64_t b = 0; b < per_epoch && e == hipSuccess; b++, step++) {
            const int64_t start = b * batch;
            const int rr = (int)(n - start < batch ? n - start : batch);
            e = chem::launch_gather_rows(order ? order + (int64_t)ep * n : nullptr, start, rr, Xall, kInPad,
                                         Yall, s->nout_pad, a.X, a.Yb, st);
            if (e == hipSuccess) e = forward(s, a.X, rr, a.H, a.U, a.OUT, s->nout_pad, st);
            if (e == hipSuccess)
                e = chem::launch_loss_grad(a.OUT, a.Yb, rr, s->K, s->nout_pad, a.dOut, s->loss_dev, st);
            if (e == hipSuccess) e = backward(s, a, a.X, rr, st);
            if (e == hipSuccess) {
                const double lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + std::cos(kPi * (double)step / (double)total));
                s->adam_t++;
                e = chem::launch_adam(adam_args(s, lr), st);
                if (e == hipSuccess) e = chem::launch_to_bf16(s->master, s->wbf, s->n_pad, st);
                s->frag_valid = false;
            }
        }
        if (e == hipSuccess && loss_per_epoch) {
            double acc = 0.0;
            e = hipMemcpyAsync(&acc, s->loss_dev, sizeof(double), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            loss_per_epoch[ep] = acc / ((double)n * s->K);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    data.release();
    return check_hip(e, "training");
}

int chem_surrogate_train(chem_surr s, const double *T, const double *p, const double *Y, int64_t ldY,
                         const double *Yn, int64_t ldYn, int64_t n, const int32_t *order, int32_t epochs,
                         int32_t batch, double lr0, double lr1, double *loss_per_epoch, void *stream)
{
    return chem_surrogate_train_part(s, T, p, Y, ldY, Yn, ldYn, n, order, 0, epochs, epochs, batch, lr0, lr1,
                                     loss_per_epoch, stream);
}

namespace {

// The handle's network, normalisation and, with opt, optimiser state as a file image.
int surr_to_file(chem_surr s, bool opt, chem_file::SurrFile &f)
{
    if (s->G != 1)
        return fail(CHEM_EUNSUP, "the weights file holds one network; the per-species networks are not saved "
                                 "(get their parameters with chem_surrogate_get_params)");
    f.K = s->K;
    f.nin = s->nin;
    for (int l = 0; l < 3; l++) f.h[l] = s->h[l];
    f.norm_set = s->norm_set;
    f.norm = s->norm;
    f.norm.resize((size_t)norm_len(s), 0.0);
    f.params.resize((size_t)s->n_logical);
    int rc = chem_surrogate_get_params(s, f.params.data(), s->n_logical);
    if (rc != CHEM_OK || !opt) return rc;
    f.has_opt = true;
    f.adam_t = s->adam_t;
    f.m.resize((size_t)s->n_logical);
    f.v.resize((size_t)s->n_logical);
    rc = download_logical(s, s->am, f.m.data(), s->n_logical);
    if (rc == CHEM_OK) rc = download_logical(s, s->av, f.v.data(), s->n_logical);
    return rc;
}

int write_file(const std::string &path, const std::string &bytes)
{
    std::ofstream f(path, std::ios::binary);
    if (!f || !f.write(bytes.data(), (std::streamsize)bytes.size())) return fail(CHEM_EINVAL, "cannot write the file");
    return CHEM_OK;
}

}  // namespace

int chem_surrogate_save(chem_surr s, const char *path)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (!path) return fail(CHEM_EINVAL, "path is NULL");
    chem_file::SurrFile f;
    rc = surr_to_file(s, false, f);
    if (rc != CHEM_OK) return rc;
    return write_file(path, chem_file::encode_surr(f));
}

int chem_surrogate_save_checkpoint(chem_surr s, const char *path, const void *user, int64_t user_bytes)
{
    int rc = check_surr(s);
    if (rc != CHEM_OK) return rc;
    if (!path) return fail(CHEM_EINVAL, "path is NULL");
    if (user_bytes < 0 || user_bytes > chem_file::kSurrMaxUser || (user_bytes > 0 && !user))
        return fail(CHEM_EINVAL, "user bytes: need 0 <= user_bytes <= 2^20 and a pointer when > 0");
    chem_file::SurrFile f;
    rc = surr_to_file(s, true, f);
    if (rc != CHEM_OK) return rc;
    f.user.assign((const char *)user, (size_t)user_bytes);
    return write_file(path, chem_file::encode_surr(f));
}

int chem_surrogate_load(chem_mech mech, const char *path, chem_surr *out)
{
    if (!mech || !path || !out) return fail(CHEM_EINVAL, "mech, path and out must not be NULL");
    *out = nullptr;
    chem_file::SurrFile f;
    std::string err;
    if (chem_file::read_surr_file(path, f, err) != 0) return fail(CHEM_EINVAL, err);
    if (f.K != mech->host.K) return fail(CHEM_EINVAL, "surrogate does not match the mechanism");
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(mech->device);
    chem_surr s = nullptr;
    int rc = chem_surrogate_create(mech, f.h[0], f.h[1], f.h[2], &s);
    if (rc == CHEM_OK) rc = chem_surrogate_set_params(s, f.params.data(), (int64_t)f.params.size());
    if (rc == CHEM_OK && f.norm_set) rc = chem_surrogate_set_norm(s, f.norm.data(), (int64_t)f.norm.size());
    if (rc == CHEM_OK && f.has_opt) {
        rc = upload_logical(s, s->am, f.m.data(), (int64_t)f.m.size());
        if (rc == CHEM_OK) rc = upload_logical(s, s->av, f.v.data(), (int64_t)f.v.size());
        if (rc == CHEM_OK) s->adam_t = f.adam_t;
    }
    hipSetDevice(prev);
    if (rc != CHEM_OK) {
        if (s) chem_free_surrogate(s);
        return rc;
    }
    *out = s;
    return CHEM_OK;
}

int chem_surrogate_checkpoint_user(const char *path, void *user, int64_t capacity, int64_t *user_bytes)
{
    if (!path || !user_bytes || capacity < 0 || (capacity > 0 && !user))
        return fail(CHEM_EINVAL, "path and user_bytes must not be NULL, capacity >= 0");
    chem_file::SurrFile f;
    std::string err;
    if (chem_file::read_surr_file(path, f, err) != 0) return fail(CHEM_EINVAL, err);
    if (!f.has_opt) return fail(CHEM_EINVAL, "the file holds no training state");
    *user_bytes = (int64_t)f.user.size();
    if ((int64_t)f.user.size() > capacity) return fail(CHEM_EINVAL, "user buffer too small");
    if (!f.user.empty()) std::memcpy(user, f.user.data(), f.user.size());
    return CHEM_OK;
}

}  // extern "C"

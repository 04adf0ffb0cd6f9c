// Batching of uneven per-cell work: integration of a listed subset of cells
// in a given order, the longest-first (LPT) order from per-cell costs, and an
// autotuner that times the candidate schedules on a sample of the cells.

#include <algorithm>
#include <cstring>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "host_common.h"
#include "surrogate.h"

using chem_host::check_hip;
using chem_host::fail;
using chem_host::is_device_ptr;

namespace {

__global__ void iota_kernel(int32_t *v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

// Stable sort of cell indices by descending cost (ties keep index order).
int lpt_order(const int32_t *cost, int64_t n, int32_t *order, hipStream_t st)
{
    if (n <= 0) return CHEM_OK;
    void *buf = nullptr;
    size_t tmp = 0;
    int32_t *keys_out = nullptr, *vals_in = nullptr;
    hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tmp, cost, keys_out, vals_in, order,
                                                                 (int)n, 0, 32, st);
    if (e != hipSuccess) return check_hip(e, "radix sort size");
    const size_t a = ((size_t)n * sizeof(int32_t) + 255) & ~size_t(255);
    if (hipMalloc(&buf, 2 * a + tmp) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CHEM_ENOMEM, "LPT order workspace allocation failed");
    }
    keys_out = (int32_t *)buf;
    vals_in = (int32_t *)((char *)buf + a);
    void *temp = (char *)buf + 2 * a;
    hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, vals_in, n);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairsDescending(temp, tmp, cost, keys_out, vals_in, order, (int)n, 0, 32,
                                                         st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(buf);
    return check_hip(e, "LPT order");
}

// Totals of per-cell outputs: a grid-stride pass per thread, a block sum in
// LDS, one set of 64-bit atomics per block.  acc: 6 counter sums, steps_max,
// 8 status counts.
__global__ void __launch_bounds__(256) stats_kernel(const int32_t *__restrict__ status,
                                                    const int32_t *__restrict__ counters, int64_t n,
                                                    unsigned long long *__restrict__ acc)
{
    __shared__ unsigned long long part[256][15];
    unsigned long long v[15];
#pragma unroll
    for (int j = 0; j < 15; j++) v[j] = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (counters) {
#pragma unroll
            for (int c = 0; c < 6; c++) v[c] += (unsigned long long)(unsigned)counters[c * n + i];
            const unsigned long long st = (unsigned)counters[i];
            v[6] = st > v[6] ? st : v[6];
        }
        if (status) {
            const int s = status[i];
            v[7 + ((s >= 0 && s < 8) ? s : 7)] += 1ull;
        }
    }
#pragma unroll
    for (int j = 0; j < 15; j++) part[threadIdx.x][j] = v[j];
    __syncthreads();
    if (threadIdx.x < 15) {
        const int j = threadIdx.x;
        unsigned long long t = 0ull;
        for (int k = 0; k < 256; k++) t = j == 6 ? (part[k][j] > t ? part[k][j] : t) : t + part[k][j];
        if (j == 6)
            atomicMax(&acc[j], t);
        else
            atomicAdd(&acc[j], t);
    }
}

__global__ void zero_u64_kernel(unsigned long long *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

}  // namespace

extern "C" {

int chem_get_stats(const int32_t *status, const int32_t *counters, int64_t n, const int64_t *fallback_count,
                   chem_stats *out, void *stream)
{
    if (!out) return fail(CHEM_EINVAL, "out is NULL");
    if (n < 0) return fail(CHEM_EINVAL, "n must be >= 0");
    if ((status && !is_device_ptr(status)) || (counters && !is_device_ptr(counters)) ||
        (fallback_count && !is_device_ptr(fallback_count)))
        return fail(CHEM_EINVAL, "status, counters and fallback_count must be device pointers or NULL");
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *acc = nullptr;
    if (hipMalloc((void **)&acc, 16 * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CHEM_ENOMEM, "stats buffer allocation failed");
    }
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, acc, 16);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && n > 0 && (status || counters)) {
        const int64_t want = (n + 255) / 256;
        const unsigned blocks = (unsigned)(want < 1024 ? want : 1024);
        hipLaunchKernelGGL(stats_kernel, dim3(blocks), dim3(256), 0, st, status, counters, n, acc);
        e = hipGetLastError();
    }
    unsigned long long h[16] = {0};
    int64_t fb = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(h, acc, 15 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && fallback_count)
        e = hipMemcpyAsync(&fb, fallback_count, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(acc);
    if (e != hipSuccess) return check_hip(e, "stats");
    chem_stats r;
    std::memset(&r, 0, sizeof(r));
    r.cells = n;
    r.steps_total = (int64_t)h[0];
    r.rhs_evals = (int64_t)h[1];
    r.jac_evals = (int64_t)h[2];
    r.newton_iters = (int64_t)h[3];
    r.rejects = (int64_t)(h[4] + h[5]);
    r.steps_max = (int32_t)h[6];
    for (int s = 0; s < 8; s++) r.status_count[s] = (int64_t)h[7 + s];
    r.fallback_cells = fb;
    *out = r;
    return CHEM_OK;
}

int chem_integrate_indexed(chem_mech m, double *T, const double *p, double *Y, int64_t ldY, int64_t ncells,
                           const int32_t *cell_idx, int64_t nidx, double dt, const chem_opts *opts,
                           int32_t *status, int32_t *counters, void *stream)
{
    if (!m) return fail(CHEM_EINVAL, "mechanism handle is NULL");
    if (ncells < 0 || nidx < 0) return fail(CHEM_EINVAL, "ncells and nidx must be >= 0");
    if (nidx == 0 || ncells == 0) return CHEM_OK;
    if (nidx > INT32_MAX || ncells > INT32_MAX) return fail(CHEM_EINVAL, "sizes must fit in int32");
    if (ldY < ncells) return fail(CHEM_EINVAL, "ldY must be >= ncells");
    if (!is_device_ptr(T) || !is_device_ptr(p) || !is_device_ptr(Y) || !is_device_ptr(cell_idx))
        return fail(CHEM_EINVAL, "T, p, Y and cell_idx must be device pointers");
    if ((status && !is_device_ptr(status)) || (counters && !is_device_ptr(counters)))
        return fail(CHEM_EINVAL, "status and counters must be device pointers or NULL");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != m->device)
        return fail(CHEM_EINVAL, "the current HIP device is not the mechanism's device");
    return chem_host::integrate_cells(m, T, p, Y, ldY, ncells, dt, opts, status, counters, (hipStream_t)stream,
                                      nullptr, cell_idx, nidx);
}

int chem_lpt_order(const int32_t *cost, int64_t n, int32_t *order, void *stream)
{
    if (n < 0 || n > INT32_MAX) return fail(CHEM_EINVAL, "n must be in [0, 2^31)");
    if (n == 0) return CHEM_OK;
    if (!is_device_ptr(cost) || !is_device_ptr(order)) return fail(CHEM_EINVAL, "cost and order must be device pointers");
    return lpt_order(cost, n, order, (hipStream_t)stream);
}

int chem_autotune(chem_mech m, const double *T, const double *p, const double *Y, int64_t ldY, int64_t n,
                  double dt, const chem_opts *base, int32_t max_sample, chem_opts *best, int32_t *use_lpt,
                  double *best_ms, void *stream)
{
    if (!m || !best) return fail(CHEM_EINVAL, "mech and best must not be NULL");
    if (n < 1 || ldY < n) return fail(CHEM_EINVAL, "need ncells >= 1 and ldY >= ncells");
    if (!is_device_ptr(T) || !is_device_ptr(p) || !is_device_ptr(Y))
        return fail(CHEM_EINVAL, "T, p and Y must be device pointers");
    chem_opts o0;
    chem_default_opts(&o0);
    if (base) o0 = *base;
    const int K = m->host.K;
    const int64_t ns = std::min<int64_t>(n, max_sample > 0 ? max_sample : 262144);
    hipStream_t st = (hipStream_t)stream;
    // strided sample of the field, copied into work arrays
    std::vector<int32_t> hidx((size_t)ns);
    for (int64_t i = 0; i < ns; i++) hidx[(size_t)i] = (int32_t)(i * n / ns);
    const size_t a8 = ((size_t)ns * 8 + 255) & ~size_t(255), a4 = ((size_t)ns * 4 + 255) & ~size_t(255);
    const size_t bytes = a8 * (2 + 2 * (K + 1)) + a4 * (4 + 6) + 256;
    char *buf = nullptr;
    if (hipMalloc((void **)&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CHEM_ENOMEM, "autotune workspace allocation failed");
    }
    size_t off = 0;
    auto take = [&](size_t b) { char *r = buf + off; off += b; return r; };
    double *Ts = (double *)take(a8), *ps = (double *)take(a8), *Ys = (double *)take(a8 * K);
    double *T0 = (double *)take(a8), *Y0 = (double *)take(a8 * K);
    int32_t *idx = (int32_t *)take(a4), *lpt = (int32_t *)take(a4), *cost = (int32_t *)take(a4);
    int32_t *stat = (int32_t *)take(a4), *cnt = (int32_t *)take(a4 * 6);
    int64_t *count = (int64_t *)take(256);
    int rc = check_hip(hipMemcpy(idx, hidx.data(), (size_t)ns * 4, hipMemcpyHostToDevice), "sample upload");
    if (rc == CHEM_OK) rc = check_hip(hipMemcpy(count, &ns, sizeof(int64_t), hipMemcpyHostToDevice), "count");
    if (rc == CHEM_OK)
        rc = check_hip(chem::launch_gather_cells(idx, count, ns, T, p, Y, ldY, K, T0, ps, Y0, st), "gather");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == CHEM_OK) rc = check_hip(hipEventCreate(&e0), "event");
    if (rc == CHEM_OK) rc = check_hip(hipEventCreate(&e1), "event");
    auto run = [&](const chem_opts &o, const int32_t *order, float &ms) -> int {
        ms = 1e30f;
        for (int rep = 0; rep < 2; rep++) {
            int r = check_hip(hipMemcpyAsync(Ts, T0, (size_t)ns * 8, hipMemcpyDeviceToDevice, st), "restore");
            if (r == CHEM_OK)
                r = check_hip(hipMemcpyAsync(Ys, Y0, (size_t)ns * K * 8, hipMemcpyDeviceToDevice, st), "restore");
            if (r == CHEM_OK) r = check_hip(hipEventRecord(e0, st), "event");
            if (r == CHEM_OK)
                r = chem_host::integrate_cells(m, Ts, ps, Ys, ns, ns, dt, &o, stat, cnt, st, nullptr, order,
                                               order ? ns : 0);
            if (r == CHEM_OK) r = check_hip(hipEventRecord(e1, st), "event");
            if (r == CHEM_OK) r = check_hip(hipEventSynchronize(e1), "sync");
            float t = 0.0f;
            if (r == CHEM_OK) r = check_hip(hipEventElapsedTime(&t, e0, e1), "elapsed");
            if (r != CHEM_OK) return r;
            ms = std::min(ms, t);
        }
        return CHEM_OK;
    };
    const bool thread_ok = m->gen != nullptr && o0.precision == 0;
    const bool wave_ok = chem::wave_kernel_rows(K + 1) > 0;
    const bool tile_ok = K + 1 <= 16;
    struct Cand {
        int schedule, jac_batch, lpt, waves;
    };
    std::vector<Cand> cands;
    // the thread schedule orders its cells itself (start pass): no LPT variant
    if (thread_ok)
        for (int jb : {4, 16, 64}) cands.push_back({0, jb, 0, 0});
    for (int l = 0; l < 2; l++)
        for (int w : {0, 1}) {
            if (wave_ok) cands.push_back({1, 0, l, w});
            if (tile_ok) cands.push_back({2, 0, l, w});
        }
    const bool any_lpt = wave_ok || tile_ok;
    // a first run in natural order gives the per-cell step counts for LPT
    float best_t = 1e30f;
    Cand bc{-1, 0, 0, 0};
    std::vector<chem_tune_entry> table;
    if (rc == CHEM_OK && any_lpt) {
        chem_opts o = o0;
        o.schedule = -1;
        float t = 0.0f;
        rc = run(o, nullptr, t);
        if (rc == CHEM_OK)
            rc = check_hip(hipMemcpyAsync(cost, cnt, (size_t)ns * 4, hipMemcpyDeviceToDevice, st), "cost");
        if (rc == CHEM_OK) rc = lpt_order(cost, ns, lpt, st);
    }
    for (size_t c = 0; rc == CHEM_OK && c < cands.size(); c++) {
        chem_opts o = o0;
        o.schedule = cands[c].schedule;
        o.jac_batch = cands[c].jac_batch;
        o.waves_per_simd = cands[c].waves;
        float t = 0.0f;
        rc = run(o, cands[c].lpt ? lpt : nullptr, t);
        if (rc != CHEM_OK) break;
        table.push_back({cands[c].schedule, cands[c].jac_batch, cands[c].lpt, cands[c].waves, (double)t});
        if (t < best_t) {
            best_t = t;
            bc = cands[c];
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(buf);
    if (rc != CHEM_OK) return rc;
    if (bc.schedule < 0) return fail(CHEM_EUNSUP, "no schedule can serve this mechanism");
    *best = o0;
    best->schedule = bc.schedule;
    best->jac_batch = bc.jac_batch;
    best->waves_per_simd = bc.waves;
    const int prec = o0.precision == 1 ? 1 : 0;
    // kept for the size class of the calls this sample stands for
    const int cls = size_class(n);
    Tuned tu;
    tu.schedule = bc.schedule;
    tu.jac_batch = bc.jac_batch;
    tu.waves_per_simd = bc.waves;
    tu.lpt = bc.lpt;
    tu.ms = best_t;
    {
        std::lock_guard<std::mutex> lk(m->ws_mu);
        m->tuned[{prec, cls}] = tu;
        m->tune_results = table;
    }
    chem_host::tune_cache_append(m, prec, cls, tu);
    if (use_lpt) *use_lpt = bc.lpt;
    if (best_ms) *best_ms = best_t;
    return CHEM_OK;
}

int chem_autotune_results(chem_mech m, chem_tune_entry *out, int32_t capacity, int32_t *count)
{
    if (!m || !count || capacity < 0 || (capacity > 0 && !out))
        return fail(CHEM_EINVAL, "mech and count must not be NULL, capacity >= 0");
    std::lock_guard<std::mutex> lk(m->ws_mu);
    *count = (int32_t)m->tune_results.size();
    for (int32_t i = 0; i < capacity && i < *count; i++) out[i] = m->tune_results[(size_t)i];
    return CHEM_OK;
}

}  // extern "C"

// Host-side pieces shared by the integrator and surrogate halves of the C ABI:
// the mechanism handle, error reporting and the internal integrate call.
#pragma once

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "chem.h"
#include "bdf_driver.h"
#include "bdf_wave.h"
#include "mech_file.h"

namespace chem_host {

// Records msg as the calling thread's last error and returns code.
int fail(int code, const std::string &msg);
// CHEM_OK for hipSuccess, else CHEM_EHIP with the runtime's message.
int check_hip(hipError_t e, const char *what);
bool is_device_ptr(const void *p);

// A device workspace that only grows.  Growing is refused while the stream
// is being captured (a graph must not record an allocation), and a replaced
// buffer is kept until release(): a graph captured earlier may still refer
// to it.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    std::vector<void *> retired;
    int grow(size_t want, hipStream_t st)
    {
        if (want <= bytes) return CHEM_OK;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CHEM_EHIP, "hipStreamIsCapturing failed");
        }
        if (cs != hipStreamCaptureStatusNone)
            return fail(CHEM_EINVAL, "the workspace is too small for this call and cannot grow while the "
                                     "stream is captured: make the same call (or the reserve call) eagerly "
                                     "before capturing");
        void *q = nullptr;
        if (hipMalloc(&q, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CHEM_ENOMEM, "workspace allocation failed");
        }
        if (p) retired.push_back(p);
        p = q;
        bytes = want;
        return CHEM_OK;
    }
    void release()
    {
        for (void *r : retired) hipFree(r);
        retired.clear();
        if (p) hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

}  // namespace chem_host

// One autotuned launch configuration.
struct Tuned {
    int schedule = -1, jac_batch = 0, waves_per_simd = 0, lpt = 0;
    double ms = 0.0;
};

struct chem_mech_s {
    int device = 0;
    chem_file::HostMech host;
    std::vector<double> W;
    chem::DevMechView view{};
    void *dev_block = nullptr;
    unsigned long long *queues = nullptr;   // work-queue counters, one per in-flight call
    unsigned next_queue = 0;
    const chem::GenEntry *gen = nullptr;    // mechanism-specialised kernels, if compiled
    std::string variant = "table";
    chem::WaveTables wave{};                // species -> reaction incidence (wave kernel)
    // reaction scratch of the kernels whose 7 R doubles per cell in flight do
    // not fit in LDS: kScratchParts partitions of wave_slots slices, one
    // partition per call in rotation (NULL when no variant needs it)
    double *wave_scratch = nullptr;
    int wave_slots = 0;
    unsigned next_part = 0;
    // start-pass workspaces of the one-thread-per-cell kernels, one per
    // stream (calls on one stream run in order, so they can share one); each
    // grows to the largest call made on its stream outside graph capture
    std::map<void *, chem_host::DevBuf> start_ws;
    std::mutex ws_mu;
    // autotuned choices per (precision, size class floor(log2 ncells)), used
    // when opts.schedule == -2; guarded by ws_mu
    std::map<std::pair<int, int>, Tuned> tuned;
    std::vector<chem_tune_entry> tune_results;   // measured table of the last chem_autotune
    unsigned long long file_hash = 0;            // FNV-1a of the mechanism file
    std::string arch;                            // GPU architecture name of the device
    void *transport_block = nullptr;             // mixture-averaged transport tables (chem_set_transport)
    const Tuned *find_tuned(int precision, int cls) const
    {
        const Tuned *best = nullptr;
        int dist = 1 << 30;
        for (const auto &t : tuned) {
            if (t.first.first != precision) continue;
            const int d = t.first.second > cls ? t.first.second - cls : cls - t.first.second;
            if (d < dist) {
                dist = d;
                best = &t.second;
            }
        }
        return best;
    }
};

// Size class of a call of n cells (the autotuner's key).
inline int size_class(int64_t n)
{
    int c = 0;
    while (c < 62 && (int64_t(2) << c) <= n) c++;
    return c;
}

namespace chem_host {

// chem_integrate after argument checks of the state arrays; when n_dev is not
// NULL the kernels integrate the first *n_dev cells (read on the device, at
// most n), so that a count produced by an earlier kernel needs no host sync.
// fixed_ws (fixed_bytes long, device memory), when given, serves as the
// start-pass workspace of the one-thread-per-cell schedule instead of the
// stream's growing one: the call then allocates nothing, and fails with
// CHEM_EINVAL when its work items do not fit.
int integrate_cells(chem_mech m, double *T, const double *p, double *Y, int64_t ldY, int64_t n,
                    double dt, const chem_opts *opts, int32_t *status, int32_t *counters,
                    hipStream_t stream, const int64_t *n_dev, const int32_t *idx = nullptr,
                    int64_t n_idx = 0, void *fixed_ws = nullptr, size_t fixed_bytes = 0);

// Tuning cache file (CHEM_TUNE_CACHE): append one result, and restore the
// lines of this mechanism file and architecture into the handle.
void tune_cache_append(const chem_mech_s *m, int precision, int cls, const Tuned &t);
void tune_cache_restore(chem_mech_s *m);

}  // namespace chem_host

// Host runtime of the chemistry library: mechanism loading (the reader is in
// mech_file.cpp), device tables, argument checking and the C ABI of include/chem.h.

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iterator>
#include <sstream>
#include <string>
#include <vector>

#include "host_common.h"

using chem_host::check_hip;
using chem_host::fail;
using chem_file::HostMech;
using chem_file::HostRxn;
using chem_host::is_device_ptr;

namespace {

thread_local std::string g_err = "no error";

constexpr int kQueues = 64;
constexpr int kScratchParts = 4;               // reaction-scratch partitions (calls in flight)
constexpr size_t kScratchBudget = size_t(1) << 30;   // bytes of reaction scratch per mechanism, at most

// Start-pass workspace of chem_integrate_noalloc: one copy of this array on
// every GPU the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel (in host code it is only a
// stand-in): once per device, with that device current, it takes the device
// address of that GPU's copy with hipGetSymbolAddress and uses that address.
constexpr size_t kNoAllocBytes = size_t(32) << 20;
__device__ __align__(256) char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// Device address of `device`'s copy of the array (resolved once, with that
// device current).
int noalloc_scratch(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return chem_host::fail(CHEM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess) return chem_host::fail(CHEM_EHIP, "hipGetDevice failed");
        void *ptr = nullptr;
        hipError_t e = hipSetDevice(device);
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        hipSetDevice(prev);
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return chem_host::fail(CHEM_EHIP, std::string("hipGetSymbolAddress of the fixed workspace: ") +
                                                  hipGetErrorString(e));
        }
        g_scratch_addr[device] = ptr;
    }
    *out = g_scratch_addr[device];
    return CHEM_OK;
}

// Work items of an N-component mechanism that fit the fixed workspace.
int64_t noalloc_max_items(int N)
{
    int64_t lo = 0, hi = (int64_t)(kNoAllocBytes / 8);
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (chem::start_pass_bytes(N, mid) <= kNoAllocBytes) lo = mid; else hi = mid - 1;
    }
    return lo;
}

unsigned long long fnv1a64(const std::string &data)
{
    unsigned long long h = 0xCBF29CE484222325ull;
    for (unsigned char c : data) {
        h ^= c;
        h *= 0x100000001B3ull;
    }
    return h;
}
}  // namespace

namespace {

void fill_range(const double *a, double *out)
{
    for (int j = 0; j < 7; j++) out[j] = a[j];
    out[7] = a[1] / 2.0;
    out[8] = a[2] / 3.0;
    out[9] = a[3] / 4.0;
    out[10] = a[4] / 5.0;
    out[11] = a[2] / 2.0;
    out[12] = a[3] / 3.0;
    out[13] = a[4] / 4.0;
}

}  // namespace

namespace chem_host {

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return CHEM_OK;
    return fail(CHEM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void tune_cache_append(const chem_mech_s *m, int precision, int cls, const Tuned &t)
{
    const char *path = std::getenv("CHEM_TUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    char line[256];
    std::snprintf(line, sizeof(line), "chemtune1 %s %016llx %d %d %d %d %d %d %d %.6g\n", m->arch.c_str(),
                  m->file_hash, m->host.K, precision, cls, t.schedule, t.jac_batch, t.waves_per_simd, t.lpt, t.ms);
    f << line;
}

void tune_cache_restore(chem_mech_s *m)
{
    const char *path = std::getenv("CHEM_TUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string tag, arch, hash;
        int K = 0, prec = 0, cls = 0;
        Tuned t;
        if (!(is >> tag >> arch >> hash >> K >> prec >> cls >> t.schedule >> t.jac_batch >> t.waves_per_simd >>
              t.lpt >> t.ms))
            continue;
        char want[32];
        std::snprintf(want, sizeof(want), "%016llx", m->file_hash);
        // later lines win; values outside the option ranges are ignored
        if (tag != "chemtune1" || arch != m->arch || hash != want || K != m->host.K || prec < 0 || prec > 1 ||
            cls < 0 || cls > 62 || t.schedule < 0 || t.schedule > 2 || t.jac_batch < 0 || t.jac_batch > 64 ||
            t.waves_per_simd < 0)
            continue;
        m->tuned[{prec, cls}] = t;
    }
}

bool is_device_ptr(const void *p)
{
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace chem_host

namespace chem_host {

int integrate_cells(chem_mech m, double *T, const double *p, double *Y, int64_t ldY, int64_t n,
                    double dt, const chem_opts *opts, int32_t *status, int32_t *counters,
                    hipStream_t stream, const int64_t *n_dev, const int32_t *idx, int64_t n_idx,
                    void *fixed_ws, size_t fixed_bytes)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CHEM_EINVAL, "dt must be finite and > 0");
    chem_opts o;
    chem_default_opts(&o);
    if (opts) o = *opts;
    if (!(o.rtol > 0.0) || !(o.atol > 0.0) || !std::isfinite(o.rtol) || !std::isfinite(o.atol))
        return fail(CHEM_EINVAL, "rtol and atol must be finite and > 0");
    if (o.max_steps < 1) return fail(CHEM_EINVAL, "max_steps must be >= 1");
    if (o.precision != 0 && o.precision != 1) return fail(CHEM_EINVAL, "precision must be 0 or 1");
    if (o.schedule < -2 || o.schedule > 2) return fail(CHEM_EINVAL, "unknown schedule");
    if (o.waves_per_simd < 0) return fail(CHEM_EINVAL, "waves_per_simd must be >= 0");
    if (o.schedule == -2) {
        // the tuned choice of this call's size class, else of the nearest tuned one
        const int64_t items = idx ? n_idx : n;
        Tuned t;
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(m->ws_mu);
            const Tuned *tu = m->find_tuned(o.precision == 1 ? 1 : 0, size_class(items));
            if (tu) {
                t = *tu;
                have = true;
            }
        }
        o.schedule = have ? t.schedule : -1;
        if (have && o.jac_batch == 0) o.jac_batch = t.jac_batch;
        if (have && o.waves_per_simd == 0) o.waves_per_simd = t.waves_per_simd;
    }
    if (o.block != 0 && o.block != 64) return fail(CHEM_EUNSUP, "block must be 0 or 64");
    if (n == 0) return CHEM_OK;
    if ((status && !is_device_ptr(status)) || (counters && !is_device_ptr(counters)))
        return fail(CHEM_EINVAL, "status and counters must be device pointers or NULL");
    const int K = m->host.K;
    const bool thread_ok = m->gen != nullptr;
    const bool wave_ok = chem::wave_kernel_rows(K + 1) > 0;
    // automatic choice: one thread per cell for a compiled-in mechanism
    // (state in registers and LDS, no spill), else the 16-lane tile when a
    // cell fits in it (N <= 16), else one wave per cell
    const int sched = o.schedule >= 0 ? o.schedule : (m->gen && o.precision == 0 ? 0 : (K + 1 <= 16 ? 2 : 1));
    if (sched == 0 && !thread_ok)
        return fail(CHEM_EUNSUP, "the one-thread-per-cell schedule needs a compiled-in mechanism (list the "
                                 ".mech file in CHEM_EXTRA_MECHS when building)");
    if (sched == 0 && o.precision != 0)
        return fail(CHEM_EUNSUP, "the one-thread-per-cell schedule computes in FP64 only");
    if (sched == 1 && !wave_ok)
        return fail(CHEM_EUNSUP, "the wave schedule supports at most 63 species");
    if (sched == 2 && K + 1 > 16)
        return fail(CHEM_EUNSUP, "the tile schedule supports at most 15 species");
    if (o.jac_batch < 0 || o.jac_batch > 64) return fail(CHEM_EINVAL, "jac_batch must be in 0..64");
    if (o.qmax < 0 || o.qmax > chem::kQmax) return fail(CHEM_EINVAL, "qmax must be in 0..5");
    chem::BdfParams prm{o.rtol,  o.atol, o.max_steps, o.jac_batch > 0 ? o.jac_batch : 16,
                        n_dev,   idx,    n_idx,       o.qmax > 0 ? o.qmax : chem::kQmax,
                        o.waves_per_simd};
    // each call takes its own queue counter (64 rotate), so that calls in
    // flight on different streams do not share one
    unsigned long long *queue = m->queues + 32 * (__atomic_fetch_add(&m->next_queue, 1u, __ATOMIC_RELAXED) % kQueues);
    hipError_t e;
    if (sched == 1 || sched == 2) {
        const int lanes = sched == 2 ? 16 : 64;
        double *qs = nullptr;
        if (chem::wave_uses_global_scratch(m->view, lanes)) {
            // calls in flight on different streams take different partitions
            const unsigned part = __atomic_fetch_add(&m->next_part, 1u, __ATOMIC_RELAXED) % kScratchParts;
            qs = m->wave_scratch + (size_t)part * m->wave_slots * m->view.qstride;
        }
        e = chem::launch_bdf_wave(m->view, m->wave, T, p, Y, ldY, n, dt, prm, status, counters, queue, qs,
                                  m->wave_slots, o.precision == 1, lanes, stream);
    }
    else {
        // one thread per cell: the start pass and its cost order need
        // workspace for every work item of the call
        const int64_t items = idx ? n_idx : n;
        if (items <= 0) return CHEM_OK;
        void *wp = fixed_ws;
        if (fixed_ws) {
            if (chem::start_pass_bytes(K + 1, items) > fixed_bytes)
                return fail(CHEM_EINVAL, "too many cells for the fixed workspace: at most " +
                                             std::to_string(noalloc_max_items(K + 1)) + " work items for K = " +
                                             std::to_string(K));
        } else {
            std::lock_guard<std::mutex> lk(m->ws_mu);
            chem_host::DevBuf &wb = m->start_ws[(void *)stream];
            const int rc = wb.grow(chem::start_pass_bytes(K + 1, items), stream);
            if (rc != CHEM_OK) return rc;
            wp = wb.p;
        }
        const chem::StartPass sp = chem::start_pass_carve(wp, K + 1, items);
        e = m->gen->integrate(T, p, Y, ldY, n, dt, prm, status, counters, queue, sp, items, stream);
    }
    return check_hip(e, "integrator launch");
}

}  // namespace chem_host

extern "C" {

const char *chem_last_error(void) { return g_err.c_str(); }

int chem_default_opts(chem_opts *o)
{
    if (!o) return fail(CHEM_EINVAL, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->rtol = 1e-8;
    o->atol = 1e-12;
    o->max_steps = 20000;
    o->precision = 0;
    o->schedule = -1;
    o->block = 0;
    return CHEM_OK;
}

int chem_load_mechanism(const char *path, int device, chem_mech *out)
{
    if (!path || !out) return fail(CHEM_EINVAL, "path and out must not be NULL");
    *out = nullptr;
    auto *m = new chem_mech_s();
    std::string perr;
    int rc = chem_file::parse_mech_file(path, m->host, perr);
    if (rc != CHEM_OK) fail(rc, perr);
    if (rc == CHEM_OK) {
        std::ifstream fb(path, std::ios::binary);
        std::string bytes((std::istreambuf_iterator<char>(fb)), std::istreambuf_iterator<char>());
        const unsigned long long h = fnv1a64(bytes);
        m->file_hash = h;
        int ng = 0;
        const chem::GenEntry *reg = chem::gen_registry(&ng);
        for (int i = 0; i < ng; i++)
            if (reg[i].hash == h && reg[i].K == m->host.K) {
                m->gen = &reg[i];
                m->variant = std::string("specialised:") + reg[i].tag;
            }
    }
    if (rc != CHEM_OK) {
        delete m;
        return rc;
    }
    const HostMech &h = m->host;
    m->device = device;
    const int K = h.K, R = h.R;
    // host-side tables
    std::vector<double> species((size_t)K * chem::kSpeciesLen), W(K), invW(K);
    bool two_range = false;
    for (int k = 0; k < K; k++) {
        double w = 0.0;
        for (int e = 0; e < h.E; e++) w += h.counts[k][e] * h.aw[e];
        W[k] = 1e-3 * w;
        invW[k] = 1.0 / W[k];
        double *s = &species[(size_t)k * chem::kSpeciesLen];
        s[0] = h.nasa[k][1];
        fill_range(&h.nasa[k][3], s + 1);
        fill_range(&h.nasa[k][10], s + 1 + chem::kRangeLen);
        for (int j = 0; j < 7; j++)
            if (h.nasa[k][3 + j] != h.nasa[k][10 + j]) two_range = true;
    }
    std::vector<chem::DevRxn> rx(R > 0 ? R : 1);
    std::vector<double> aux;   // records of the pressure-dependent reactions
    int n_pdep = 0;
    for (int i = 0; i < R; i++) {
        const HostRxn &r = h.rxn[i];
        int slots_r[2] = {K, K}, slots_p[2] = {K, K}, nr = 0, np = 0, order = 0;
        for (auto &s : r.reac)
            for (int c = 0; c < s.second; c++) slots_r[nr++] = s.first;
        for (auto &s : r.prod)
            for (int c = 0; c < s.second; c++) slots_p[np++] = s.first;
        order = nr;
        chem::DevRxn d{};
        d.r0 = slots_r[0];
        d.r1 = slots_r[1];
        d.p0 = slots_p[0];
        d.p1 = slots_p[1];
        d.dnu = np - nr;
        // A in cm-mol-s: (cm^3/mol)^(order-1)/s; SI factor 1e-6 per extra order
        // a third body counts as one more colliding molecule
        d.lnA = std::log(r.A) + (order - 1 + (r.kind == chem_file::kThird ? 1 : 0)) * std::log(1e-6);
        d.b = r.b;
        d.Ea_R = r.Ea / chem::kRu;
        d.kind = (r.kind == chem_file::kElem ? chem::kRxnElem
                  : r.kind == chem_file::kThird ? chem::kRxnThird
                  : r.kind == chem_file::kLind  ? chem::kRxnLind
                                                : chem::kRxnTroe) |
                 (r.reversible ? 0 : chem::kRxnIrrev);
        d.def_eff = r.default_eff;
        if (r.kind != chem_file::kElem) {
            d.aux = (int32_t)aux.size();
            d.neff = (int32_t)r.effs.size();
            const double head[chem::kAuxHead] = {
                r.kind >= chem_file::kLind ? std::log(r.A0) + order * std::log(1e-6) : 0.0,
                r.b0,
                r.Ea0 / chem::kRu,
                r.troe[0],
                r.kind >= chem_file::kTroe3 ? 1.0 / r.troe[1] : 0.0,
                r.kind >= chem_file::kTroe3 ? 1.0 / r.troe[2] : 0.0,
                r.kind == chem_file::kTroe4 ? r.troe[3] : 0.0,
                r.kind == chem_file::kTroe4 ? 1.0 : 0.0};
            aux.insert(aux.end(), head, head + chem::kAuxHead);
            for (auto &e : r.effs) {
                aux.push_back((double)e.first);
                aux.push_back(e.second - r.default_eff);
            }
            n_pdep++;
        }
        rx[i] = d;
    }
    if (aux.empty()) aux.assign(2, 0.0);
    m->W = W;
    // one device block: the tables (species | W | invW | reactions | incidence
    // offsets | incidence entries, contiguous so that a kernel can copy them
    // into LDS in one pass), then the work-queue counters, then wave scratch
    const size_t n_sp = species.size() * sizeof(double);
    const size_t n_w = (size_t)K * sizeof(double);
    auto a16 = [](size_t x) { return (x + 15) & ~size_t(15); };
    const size_t off_w = a16(n_sp);
    const size_t off_iw = a16(off_w + n_w);
    const size_t off_rx = a16(off_iw + n_w);
    // species -> (reaction, net coefficient) incidence, reactions in order
    std::vector<int> inc_off(K + 1, 0);
    std::vector<std::vector<std::pair<int, int>>> inc_lists(K);
    for (int i = 0; i < R; i++) {
        std::vector<int> net(K, 0);
        for (auto &t : h.rxn[i].reac) net[t.first] -= t.second;
        for (auto &t : h.rxn[i].prod) net[t.first] += t.second;
        for (int k = 0; k < K; k++)
            if (net[k] != 0) inc_lists[k].push_back({i, net[k]});
    }
    std::vector<int> inc_flat;
    for (int k = 0; k < K; k++) {
        inc_off[k + 1] = inc_off[k] + (int)inc_lists[k].size();
        for (auto &pr : inc_lists[k]) {
            inc_flat.push_back(pr.first);
            inc_flat.push_back(pr.second);
        }
    }
    if (inc_flat.empty()) inc_flat.assign(2, 0);
    const size_t off_io = a16(off_rx + rx.size() * sizeof(chem::DevRxn));
    const size_t off_inc = a16(off_io + (K + 1) * sizeof(int));
    const size_t off_aux = a16(off_inc + inc_flat.size() * sizeof(int));
    const size_t table_bytes = a16(off_aux + aux.size() * sizeof(double));
    const size_t off_q = (table_bytes + 255) & ~size_t(255);
    const size_t off_ws = off_q + kQueues * 256;
    // global reaction scratch, only when a wave or tile variant needs it:
    // kScratchParts partitions of up to 4096 slices (cells in flight)
    chem::DevMechView probe{};
    probe.K = K;
    probe.R = R;
    probe.table_bytes = (int32_t)table_bytes;
    // reaction scratch of the lane-group kernels: 7 R doubles, one R more
    // for the third-body derivatives when a reaction is pressure dependent
    probe.qstride = (n_pdep ? 8 : 7) * (R > 0 ? R : 1);
    const size_t slice = (size_t)probe.qstride * sizeof(double);
    const bool need_ws = (chem::wave_kernel_rows(K + 1) > 0 && chem::wave_uses_global_scratch(probe, 64)) ||
                         (K + 1 <= 16 && chem::wave_uses_global_scratch(probe, 16));
    int wave_slots = 0;
    if (need_ws) {
        size_t slots = kScratchBudget / (kScratchParts * slice);
        wave_slots = (int)(slots < 4096 ? (slots < 64 ? 64 : slots) : 4096);
    }
    const size_t total = off_ws + (size_t)kScratchParts * wave_slots * slice;
    int prev = 0;
    if ((rc = check_hip(hipGetDevice(&prev), "hipGetDevice")) != CHEM_OK) {
        delete m;
        return rc;
    }
    if ((rc = check_hip(hipSetDevice(device), "hipSetDevice")) != CHEM_OK) {
        delete m;
        return rc;
    }
    char *blk = nullptr;
    if (hipMalloc((void **)&blk, total) != hipSuccess) {
        (void)hipGetLastError();
        hipSetDevice(prev);
        delete m;
        return fail(CHEM_ENOMEM, "hipMalloc of the mechanism tables failed");
    }
    std::vector<char> staging(off_ws, 0);
    std::memcpy(staging.data(), species.data(), n_sp);
    std::memcpy(staging.data() + off_w, W.data(), n_w);
    std::memcpy(staging.data() + off_iw, invW.data(), n_w);
    std::memcpy(staging.data() + off_rx, rx.data(), rx.size() * sizeof(chem::DevRxn));
    std::memcpy(staging.data() + off_io, inc_off.data(), inc_off.size() * sizeof(int));
    std::memcpy(staging.data() + off_inc, inc_flat.data(), inc_flat.size() * sizeof(int));
    std::memcpy(staging.data() + off_aux, aux.data(), aux.size() * sizeof(double));
    rc = check_hip(hipMemcpy(blk, staging.data(), off_ws, hipMemcpyHostToDevice), "hipMemcpy");
    hipSetDevice(prev);
    if (rc != CHEM_OK) {
        hipFree(blk);
        delete m;
        return rc;
    }
    m->dev_block = blk;
    m->view.K = K;
    m->view.R = R;
    m->view.two_range = two_range ? 1 : 0;
    m->view.species = (const double *)blk;
    m->view.W = (const double *)(blk + off_w);
    m->view.invW = (const double *)(blk + off_iw);
    m->view.rxn = (const chem::DevRxn *)(blk + off_rx);
    m->view.table_bytes = (int32_t)table_bytes;
    m->view.aux = (const double *)(blk + off_aux);
    m->view.n_pdep = n_pdep;
    m->view.qstride = probe.qstride;
    m->queues = (unsigned long long *)(blk + off_q);
    m->wave.inc_off = (const int *)(blk + off_io);
    m->wave.inc = (const int2 *)(blk + off_inc);
    m->wave_scratch = wave_slots > 0 ? (double *)(blk + off_ws) : nullptr;
    m->wave_slots = wave_slots;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) m->arch = prop.gcnArchName;
        const std::string::size_type colon = m->arch.find(':');
        if (colon != std::string::npos) m->arch.resize(colon);
        if (m->arch.empty()) m->arch = "unknown";
        chem_host::tune_cache_restore(m);
    }
    // set-up of the fixed workspace of this device (chem_integrate_noalloc)
    void *fixed = nullptr;
    if ((rc = noalloc_scratch(device, &fixed)) != CHEM_OK) {
        chem_free_mechanism(m);
        return rc;
    }
    *out = m;
    return CHEM_OK;
}

void chem_free_mechanism(chem_mech m)
{
    if (!m) return;
    if (m->dev_block || m->transport_block) {
        int prev = 0;
        hipGetDevice(&prev);
        hipSetDevice(m->device);
        if (m->dev_block) hipFree(m->dev_block);
        if (m->transport_block) hipFree(m->transport_block);
        for (auto &w : m->start_ws) w.second.release();
        hipSetDevice(prev);
    }
    delete m;
}

int chem_mechanism_info(chem_mech m, int32_t *K, int32_t *R, int32_t *E, double *W)
{
    if (!m) return fail(CHEM_EINVAL, "mechanism handle is NULL");
    if (K) *K = m->host.K;
    if (R) *R = m->host.R;
    if (E) *E = m->host.E;
    if (W)
        for (int k = 0; k < m->host.K; k++) W[k] = m->W[k];
    return CHEM_OK;
}

const char *chem_mechanism_variant(chem_mech m)
{
    if (!m) return "";
    return m->variant.c_str();
}

static int check_state_args(chem_mech m, const double *T, const double *p, const double *Y,
                            int64_t ldY, int64_t n)
{
    if (!m) return fail(CHEM_EINVAL, "mechanism handle is NULL");
    if (n < 0) return fail(CHEM_EINVAL, "ncells must be >= 0");
    if (n == 0) return CHEM_OK;
    if (ldY < n) return fail(CHEM_EINVAL, "ldY must be >= ncells");
    if (!is_device_ptr(T) || !is_device_ptr(p) || !is_device_ptr(Y))
        return fail(CHEM_EINVAL, "T, p and Y must be device pointers");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != m->device)
        return fail(CHEM_EINVAL, "the current HIP device is not the mechanism's device");
    return CHEM_OK;
}

int chem_integrate(chem_mech m, double *T, const double *p, double *Y, int64_t ldY, int64_t n,
                   double dt, const chem_opts *opts, int32_t *status, int32_t *counters,
                   void *stream)
{
    int rc = check_state_args(m, T, p, Y, ldY, n);
    if (rc != CHEM_OK) return rc;
    return chem_host::integrate_cells(m, T, p, Y, ldY, n, dt, opts, status, counters,
                                      (hipStream_t)stream, nullptr);
}

int chem_integrate_noalloc(chem_mech m, double *T, const double *p, double *Y, int64_t ldY, int64_t n,
                           double dt, const chem_opts *opts, int32_t *status, int32_t *counters,
                           void *stream)
{
    int rc = check_state_args(m, T, p, Y, ldY, n);
    if (rc != CHEM_OK) return rc;
    void *ws = nullptr;
    if ((rc = noalloc_scratch(m->device, &ws)) != CHEM_OK) return rc;
    return chem_host::integrate_cells(m, T, p, Y, ldY, n, dt, opts, status, counters, (hipStream_t)stream,
                                      nullptr, nullptr, 0, ws, kNoAllocBytes);
}

int chem_eval_rhs(chem_mech m, const double *T, const double *p, const double *Y, int64_t ldY,
                  int64_t n, double *F, int64_t ldF, void *stream)
{
    int rc = check_state_args(m, T, p, Y, ldY, n);
    if (rc != CHEM_OK || n == 0) return rc;
    if (ldF < n || !is_device_ptr(F)) return fail(CHEM_EINVAL, "F must be a device array with ldF >= ncells");
    if (m->gen) return check_hip(m->gen->rhs(T, p, Y, ldY, n, F, ldF, (hipStream_t)stream), "rhs launch");
    if (!chem::table_eval_supports(m->host.K))
        return fail(CHEM_EUNSUP, "no kernel is built for K = " + std::to_string(m->host.K));
    return check_hip(chem::launch_rhs(m->view, T, p, Y, ldY, n, F, ldF, (hipStream_t)stream), "rhs launch");
}

int chem_eval_jacobian(chem_mech m, const double *T, const double *p, const double *Y, int64_t ldY,
                       int64_t n, double *J, int64_t ldJ, void *stream)
{
    int rc = check_state_args(m, T, p, Y, ldY, n);
    if (rc != CHEM_OK || n == 0) return rc;
    if (ldJ < n || !is_device_ptr(J)) return fail(CHEM_EINVAL, "J must be a device array with ldJ >= ncells");
    if (m->gen) return check_hip(m->gen->jac(T, p, Y, ldY, n, J, ldJ, (hipStream_t)stream), "jacobian launch");
    if (!chem::table_eval_supports(m->host.K))
        return fail(CHEM_EUNSUP, "no kernel is built for K = " + std::to_string(m->host.K));
    return check_hip(chem::launch_jacobian(m->view, T, p, Y, ldY, n, J, ldJ, (hipStream_t)stream),
                     "jacobian launch");
}

}  // extern "C"

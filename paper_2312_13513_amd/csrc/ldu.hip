// Implicit finite-volume Laplacian on the GPU: assembly of the ldu matrix
// with atomic accumulation of the diagonal (paper Section 3.1, Algorithm 1)
// and its conversion to CSR (the ldu/CSR figure), for meshes in
// owner/neighbour addressing; and the same matrix assembled straight into
// CSR without atomics (one thread per CSR entry), which on a GPU of several
// dies with their own L2 avoids the atomic traffic between them and writes
// the value array in order.  All are HBM-bound: one thread
// per face or per cell, face arrays read in face order (coalesced), the
// diagonal of the ldu path accumulated with FP64 atomics that stay in L2.  The CSR pattern and the
// position of every ldu coefficient in it are built once per mesh on the
// host, so a conversion is a scatter of the face values plus one pass over
// the cells.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_common.h"

using chem_host::check_hip;
using chem_host::fail;
using chem_host::is_device_ptr;

struct chem_ldu_s {
    int device = 0;
    int64_t ncells = 0, nfaces = 0, nbfaces = 0, nnz = 0;
    std::vector<int64_t> patch_start;
    std::vector<int32_t> patch_type;
    void *block = nullptr;
    // device arrays (inside block)
    const int32_t *owner = nullptr, *neighbour = nullptr, *face_cells = nullptr;
    const double *weight = nullptr, *delta = nullptr, *mag_sf = nullptr, *bdelta = nullptr, *bmag_sf = nullptr;
    const int32_t *upper_pos = nullptr, *lower_pos = nullptr, *diag_pos = nullptr;
    const int32_t *bnd_ptr = nullptr, *bnd_face = nullptr, *row_ptr = nullptr, *col = nullptr;
    const int32_t *btype = nullptr;   // patch type of every boundary face
    const int32_t *ent_face = nullptr;   // face of every CSR entry; -(row + 1) on the diagonal
    double *coef = nullptr;              // face coefficients of the direct CSR assembly (work space)
};

namespace chem {
namespace {

constexpr int kLduBlock = 256;

unsigned ldu_blocks(int64_t n) { return (unsigned)((n + kLduBlock - 1) / kLduBlock); }

__global__ void __launch_bounds__(kLduBlock) ldu_zero_kernel(double *__restrict__ v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kLduBlock + threadIdx.x;
    if (i < n) v[i] = 0.0;
}

// The coefficient of an internal face: gamma_f by linear interpolation,
// times delta_f |S_f| (every kernel forms it here: the same bits on every
// path).
__device__ __forceinline__ double face_coeff(int64_t f, const int32_t *__restrict__ owner,
                                             const int32_t *__restrict__ neighbour, const double *__restrict__ weight,
                                             const double *__restrict__ delta, const double *__restrict__ mag_sf,
                                             const double *__restrict__ gamma_c)
{
    const double w = weight[f];
    const double gf = w * gamma_c[owner[f]] + (1.0 - w) * gamma_c[neighbour[f]];
    return gf * delta[f] * mag_sf[f];
}

// Internal faces (Algorithm 1, internal field): gamma_f by linear
// interpolation, upper = lower = gamma_f delta_f |S_f|, and the diagonal of
// both cells of the face accumulated by atomics.
__global__ void __launch_bounds__(kLduBlock) ldu_internal_kernel(
    int64_t nfaces, const int32_t *__restrict__ owner, const int32_t *__restrict__ neighbour,
    const double *__restrict__ weight, const double *__restrict__ delta, const double *__restrict__ mag_sf,
    const double *__restrict__ gamma_c, double *__restrict__ lower, double *__restrict__ upper,
    double *__restrict__ diag)
{
    const int64_t f = (int64_t)blockIdx.x * kLduBlock + threadIdx.x;
    if (f >= nfaces) return;
    const double c = face_coeff(f, owner, neighbour, weight, delta, mag_sf, gamma_c);
    upper[f] = c;
    lower[f] = c;
    atomicAdd(&diag[owner[f]], -c);
    atomicAdd(&diag[neighbour[f]], -c);
}

// Assembly straight into CSR, without atomics, in two passes.  First every
// internal face's coefficient, in face order (all reads and writes
// coalesced) ...
__global__ void __launch_bounds__(kLduBlock) face_coeff_kernel(
    int64_t nfaces, const int32_t *__restrict__ owner, const int32_t *__restrict__ neighbour,
    const double *__restrict__ weight, const double *__restrict__ delta, const double *__restrict__ mag_sf,
    const double *__restrict__ gamma_c, double *__restrict__ coef)
{
    const int64_t f = (int64_t)blockIdx.x * kLduBlock + threadIdx.x;
    if (f >= nfaces) return;
    coef[f] = face_coeff(f, owner, neighbour, weight, delta, mag_sf, gamma_c);
}

constexpr int kHalo = 16;                       // entries beyond each end of a block kept in LDS
constexpr int kEntPer = 4;                      // entries per thread
constexpr int kEntBlock = kLduBlock * kEntPer;  // entries per block

// ... then the CSR entries in blocks of kEntBlock, kEntPer per thread (all
// their loads issued before the first wait), so the entry arrays are read
// and the values written in order (each once): an off-diagonal entry takes the
// coefficient of the face it comes from (the face's index stored beside the
// entry).  The diagonal entry (its slot holds -(row + 1)) is minus the sum
// of its row's off-diagonal entries in column order, from the block's LDS
// copy (which reaches kHalo entries into the neighbouring blocks; an entry
// of a longer row beyond that is read from the coefficient array: the same
// bits), plus the row's fixed-value boundary faces (-gamma_b |S_b| delta_b;
// gamma_b |S_b| delta_b psi_b to the right-hand side; a zero-gradient face
// adds nothing).
__global__ void __launch_bounds__(kLduBlock) csr_assemble_entries_kernel(
    int64_t nnz, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ ent_face,
    const double *__restrict__ coef, const int32_t *__restrict__ bnd_ptr, const int32_t *__restrict__ bnd_face,
    const int32_t *__restrict__ btype, const double *__restrict__ bdelta, const double *__restrict__ bmag_sf,
    const double *__restrict__ gamma_b, const double *__restrict__ psi_b, double *__restrict__ val,
    double *__restrict__ rhs)
{
    __shared__ double sv[kEntBlock + 2 * kHalo];
    const int t = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * kEntBlock;
    const int64_t lo = j0 - kHalo, hi = j0 + kEntBlock + kHalo;
    int f[kEntPer], b[kEntPer], e[kEntPer], bb[kEntPer], be[kEntPer];
#pragma unroll
    for (int q = 0; q < kEntPer; q++) {
        const int64_t j = j0 + q * kLduBlock + t;
        f[q] = j < nnz ? ent_face[j] : 0;
    }
    // halo entries: the threads at the block's two ends take one each
    const int hs = t < kHalo ? t : (t >= kLduBlock - kHalo ? t + kEntBlock + 2 * kHalo - kLduBlock : -1);
    const int64_t h = lo + hs;
    const int fh = (hs >= 0 && h >= 0 && h < nnz) ? ent_face[h] : -1;
    // the diagonals' row and boundary extents, loaded beside the coefficients
#pragma unroll
    for (int q = 0; q < kEntPer; q++) {
        const int64_t j = j0 + q * kLduBlock + t;
        b[q] = e[q] = bb[q] = be[q] = 0;
        if (j < nnz && f[q] < 0) {
            const int i = -(f[q] + 1);
            b[q] = row_ptr[i];
            e[q] = row_ptr[i + 1];
            bb[q] = bnd_ptr[i];
            be[q] = bnd_ptr[i + 1];
        }
    }
    double v[kEntPer];
#pragma unroll
    for (int q = 0; q < kEntPer; q++) {
        const int64_t j = j0 + q * kLduBlock + t;
        v[q] = (j < nnz && f[q] >= 0) ? coef[f[q]] : 0.0;
        sv[kHalo + q * kLduBlock + t] = v[q];
    }
    if (hs >= 0) sv[hs] = fh >= 0 ? coef[fh] : 0.0;
    __syncthreads();
    // every value is written once, after the diagonals are known: each store
    // covers whole lines of the value array
#pragma unroll
    for (int q = 0; q < kEntPer; q++) {
        const int64_t j = j0 + q * kLduBlock + t;
        if (j >= nnz) continue;
        if (f[q] >= 0) {
            val[j] = v[q];
            continue;
        }
        const int i = -(f[q] + 1);
        double s = 0.0;
        for (int k = b[q]; k < e[q]; k++) {
            if (k == j) continue;
            s += (k >= lo && k < hi) ? sv[k - lo] : coef[ent_face[k]];
        }
        double d = -s, r = 0.0;
        for (int k = bb[q]; k < be[q]; k++) {
            const int bf = bnd_face[k];
            if (btype[bf] == 0) {
                const double c = gamma_b[bf] * bmag_sf[bf] * bdelta[bf];
                d += -c;
                r += c * psi_b[bf];
            }
        }
        val[j] = d;
        rhs[i] = r;
    }
}

// One boundary patch (Algorithm 1, boundary loop: a launch per patch, the
// patch type fixed at compile time): a fixed-value face adds the flux
// gamma_b |S_b| delta_b (psi_b - psi_P), internal = -gamma_b |S_b| delta_b
// and boundary = gamma_b |S_b| delta_b psi_b; a zero-gradient face adds
// nothing.
template <int TYPE>
__global__ void __launch_bounds__(kLduBlock) ldu_patch_kernel(
    int64_t start, int64_t count, const double *__restrict__ bdelta, const double *__restrict__ bmag_sf,
    const double *__restrict__ gamma_b, const double *__restrict__ psi_b, double *__restrict__ internal,
    double *__restrict__ boundary)
{
    const int64_t i = (int64_t)blockIdx.x * kLduBlock + threadIdx.x;
    if (i >= count) return;
    const int64_t b = start + i;
    if (TYPE == 0) {
        const double c = gamma_b[b] * bmag_sf[b] * bdelta[b];
        internal[b] = -c;
        boundary[b] = c * psi_b[b];
    } else {
        internal[b] = 0.0;
        boundary[b] = 0.0;
    }
}

// ldu -> CSR: the face coefficients to their places in the rows of both
// cells of the face.
__global__ void __launch_bounds__(kLduBlock) csr_faces_kernel(
    int64_t nfaces, const int32_t *__restrict__ upper_pos, const int32_t *__restrict__ lower_pos,
    const double *__restrict__ lower, const double *__restrict__ upper, double *__restrict__ val)
{
    const int64_t f = (int64_t)blockIdx.x * kLduBlock + threadIdx.x;
    if (f >= nfaces) return;
    val[upper_pos[f]] = upper[f];
    val[lower_pos[f]] = lower[f];
}

// ... and per cell its diagonal plus the internal coefficients of its
// boundary faces, and the right-hand side from their boundary coefficients
// (faces of a cell in increasing order: no atomics, the same sums every call).
__global__ void __launch_bounds__(kLduBlock) csr_cells_kernel(
    int64_t ncells, const int32_t *__restrict__ diag_pos, const int32_t *__restrict__ bnd_ptr,
    const int32_t *__restrict__ bnd_face, const double *__restrict__ diag, const double *__restrict__ internal,
    const double *__restrict__ boundary, double *__restrict__ val, double *__restrict__ rhs)
{
    const int64_t i = (int64_t)blockIdx.x * kLduBlock + threadIdx.x;
    if (i >= ncells) return;
    double d = diag[i], r = 0.0;
    for (int j = bnd_ptr[i]; j < bnd_ptr[i + 1]; j++) {
        const int b = bnd_face[j];
        d += internal[b];
        r += boundary[b];
    }
    val[diag_pos[i]] = d;
    rhs[i] = r;
}

}  // namespace
}  // namespace chem

namespace {

int check_ldu(chem_ldu m)
{
    if (!m) return fail(CHEM_EINVAL, "mesh handle is NULL");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != m->device)
        return fail(CHEM_EINVAL, "the current HIP device is not the mesh's device");
    return CHEM_OK;
}

bool all_dev(std::initializer_list<const void *> ps)
{
    for (const void *p : ps)
        if (!is_device_ptr(p)) return false;
    return true;
}

}  // namespace

extern "C" {

int chem_ldu_create(int64_t ncells, int64_t nfaces, const int32_t *owner, const int32_t *neighbour,
                    const double *weight, const double *delta, const double *mag_sf, int32_t npatches,
                    const int64_t *patch_start, const int32_t *patch_type, const int32_t *face_cells,
                    const double *bdelta, const double *bmag_sf, int device, chem_ldu *out)
{
    if (!out) return fail(CHEM_EINVAL, "out is NULL");
    *out = nullptr;
    if (ncells < 1 || nfaces < 0 || npatches < 0 || npatches > 4096)
        return fail(CHEM_EINVAL, "need ncells >= 1, nfaces >= 0, 0 <= npatches <= 4096");
    if (ncells + 2 * nfaces >= INT32_MAX) return fail(CHEM_EINVAL, "the matrix must have fewer than 2^31 entries");
    if (nfaces && (!owner || !neighbour || !weight || !delta || !mag_sf))
        return fail(CHEM_EINVAL, "face arrays must not be NULL");
    if (!patch_start || (npatches && !patch_type)) return fail(CHEM_EINVAL, "patch arrays must not be NULL");
    if (patch_start[0] != 0) return fail(CHEM_EINVAL, "patch_start[0] must be 0");
    for (int32_t p = 0; p < npatches; p++) {
        if (patch_start[p + 1] < patch_start[p]) return fail(CHEM_EINVAL, "patch_start must not decrease");
        if (patch_type[p] != 0 && patch_type[p] != 1) return fail(CHEM_EINVAL, "patch types are 0 (fixed value) or 1 (zero gradient)");
    }
    const int64_t nb = patch_start[npatches];
    if (nb > INT32_MAX) return fail(CHEM_EINVAL, "too many boundary faces");
    if (nb && (!face_cells || !bdelta || !bmag_sf)) return fail(CHEM_EINVAL, "boundary arrays must not be NULL");
    // faces in upper-triangular order: owner < neighbour, sorted by owner then neighbour
    for (int64_t f = 0; f < nfaces; f++) {
        const int32_t o = owner[f], n = neighbour[f];
        if (o < 0 || n >= ncells || o >= n) return fail(CHEM_EINVAL, "face " + std::to_string(f) + ": need 0 <= owner < neighbour < ncells");
        if (f && (o < owner[f - 1] || (o == owner[f - 1] && n <= neighbour[f - 1])))
            return fail(CHEM_EINVAL, "faces must be in upper-triangular order (owner, then neighbour, increasing)");
        if (!std::isfinite(weight[f]) || !std::isfinite(delta[f]) || !std::isfinite(mag_sf[f]))
            return fail(CHEM_EINVAL, "face geometry must be finite");
    }
    for (int64_t b = 0; b < nb; b++) {
        if (face_cells[b] < 0 || face_cells[b] >= ncells) return fail(CHEM_EINVAL, "boundary face cell out of range");
        if (!std::isfinite(bdelta[b]) || !std::isfinite(bmag_sf[b])) return fail(CHEM_EINVAL, "boundary geometry must be finite");
    }
    // CSR pattern: row i = faces with neighbour i (owners increasing), the
    // diagonal, faces with owner i (neighbours increasing)
    std::vector<int32_t> nup(ncells, 0), nlo(ncells, 0);
    for (int64_t f = 0; f < nfaces; f++) {
        nup[owner[f]]++;
        nlo[neighbour[f]]++;
    }
    std::vector<int32_t> row_ptr(ncells + 1, 0);
    for (int64_t i = 0; i < ncells; i++) row_ptr[i + 1] = row_ptr[i] + nlo[i] + 1 + nup[i];
    const int64_t nnz = row_ptr[ncells];
    std::vector<int32_t> col(nnz), upos(nfaces), lpos(nfaces), dpos(ncells);
    std::vector<int32_t> lfill(ncells, 0), ufill(ncells, 0);
    for (int64_t f = 0; f < nfaces; f++) {   // face order: owners increasing within a neighbour's list
        const int32_t n = neighbour[f], o = owner[f];
        lpos[f] = row_ptr[n] + lfill[n]++;
        col[lpos[f]] = o;
    }
    for (int64_t i = 0; i < ncells; i++) {
        dpos[i] = row_ptr[i] + nlo[i];
        col[dpos[i]] = (int32_t)i;
    }
    for (int64_t f = 0; f < nfaces; f++) {   // neighbours increasing within an owner's faces
        const int32_t o = owner[f];
        upos[f] = row_ptr[o] + nlo[o] + 1 + ufill[o]++;
        col[upos[f]] = neighbour[f];
    }
    std::vector<int32_t> entf(nnz);
    for (int64_t i = 0; i < ncells; i++) entf[dpos[i]] = -(int32_t)i - 1;
    for (int64_t f = 0; f < nfaces; f++) {
        entf[lpos[f]] = (int32_t)f;
        entf[upos[f]] = (int32_t)f;
    }
    std::vector<int32_t> btype(nb);
    for (int32_t p = 0; p < npatches; p++)
        for (int64_t b = patch_start[p]; b < patch_start[p + 1]; b++) btype[b] = patch_type[p];
    // boundary faces grouped by cell, faces increasing
    std::vector<int32_t> bptr(ncells + 1, 0), bface(nb);
    for (int64_t b = 0; b < nb; b++) bptr[face_cells[b] + 1]++;
    for (int64_t i = 0; i < ncells; i++) bptr[i + 1] += bptr[i];
    {
        std::vector<int32_t> fill(bptr.begin(), bptr.end() - 1);
        for (int64_t b = 0; b < nb; b++) bface[fill[face_cells[b]]++] = (int32_t)b;
    }
    auto *m = new chem_ldu_s();
    m->device = device;
    m->ncells = ncells;
    m->nfaces = nfaces;
    m->nbfaces = nb;
    m->nnz = nnz;
    m->patch_start.assign(patch_start, patch_start + npatches + 1);
    m->patch_type.assign(patch_type, patch_type + npatches);
    auto a256 = [](size_t x) { return (x + 255) & ~size_t(255); };
    struct Part {
        const void *src;
        size_t bytes;
        size_t off;
    };
    std::vector<Part> parts = {
        {owner, (size_t)nfaces * 4, 0},       {neighbour, (size_t)nfaces * 4, 0}, {weight, (size_t)nfaces * 8, 0},
        {delta, (size_t)nfaces * 8, 0},       {mag_sf, (size_t)nfaces * 8, 0},    {face_cells, (size_t)nb * 4, 0},
        {bdelta, (size_t)nb * 8, 0},          {bmag_sf, (size_t)nb * 8, 0},       {upos.data(), (size_t)nfaces * 4, 0},
        {lpos.data(), (size_t)nfaces * 4, 0}, {dpos.data(), (size_t)ncells * 4, 0},
        {bptr.data(), (size_t)(ncells + 1) * 4, 0}, {bface.data(), (size_t)nb * 4, 0},
        {row_ptr.data(), (size_t)(ncells + 1) * 4, 0}, {col.data(), (size_t)nnz * 4, 0},
        {btype.data(), (size_t)nb * 4, 0},      {entf.data(), (size_t)nnz * 4, 0},
        {nullptr, (size_t)nfaces * 8, 0}};
    size_t total = 0;
    for (auto &p : parts) {
        p.off = total;
        total += a256(p.bytes > 0 ? p.bytes : 1);
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    int rc = check_hip(hipSetDevice(device), "hipSetDevice");
    if (rc == CHEM_OK && hipMalloc(&m->block, total) != hipSuccess) {
        (void)hipGetLastError();
        rc = fail(CHEM_ENOMEM, "mesh allocation failed");
    }
    for (auto &p : parts)
        if (rc == CHEM_OK && p.bytes && p.src)
            rc = check_hip(hipMemcpy((char *)m->block + p.off, p.src, p.bytes, hipMemcpyHostToDevice), "mesh upload");
    (void)hipSetDevice(prev);
    if (rc != CHEM_OK) {
        if (m->block) (void)hipFree(m->block);
        delete m;
        return rc;
    }
    char *base = (char *)m->block;
    int k = 0;
    m->owner = (const int32_t *)(base + parts[k++].off);
    m->neighbour = (const int32_t *)(base + parts[k++].off);
    m->weight = (const double *)(base + parts[k++].off);
    m->delta = (const double *)(base + parts[k++].off);
    m->mag_sf = (const double *)(base + parts[k++].off);
    m->face_cells = (const int32_t *)(base + parts[k++].off);
    m->bdelta = (const double *)(base + parts[k++].off);
    m->bmag_sf = (const double *)(base + parts[k++].off);
    m->upper_pos = (const int32_t *)(base + parts[k++].off);
    m->lower_pos = (const int32_t *)(base + parts[k++].off);
    m->diag_pos = (const int32_t *)(base + parts[k++].off);
    m->bnd_ptr = (const int32_t *)(base + parts[k++].off);
    m->bnd_face = (const int32_t *)(base + parts[k++].off);
    m->row_ptr = (const int32_t *)(base + parts[k++].off);
    m->col = (const int32_t *)(base + parts[k++].off);
    m->btype = (const int32_t *)(base + parts[k++].off);
    m->ent_face = (const int32_t *)(base + parts[k++].off);
    m->coef = (double *)(base + parts[k++].off);
    *out = m;
    return CHEM_OK;
}

void chem_free_ldu(chem_ldu m)
{
    if (!m) return;
    if (m->block) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(m->device);
        (void)hipFree(m->block);
        (void)hipSetDevice(prev);
    }
    delete m;
}

int chem_ldu_info(chem_ldu m, int64_t *dims)
{
    if (!m || !dims) return fail(CHEM_EINVAL, "mesh and dims must not be NULL");
    dims[0] = m->ncells;
    dims[1] = m->nfaces;
    dims[2] = m->nbfaces;
    dims[3] = m->nnz;
    return CHEM_OK;
}

int chem_ldu_laplacian(chem_ldu m, const double *gamma_c, const double *gamma_b, const double *psi_b, double *lower,
                       double *upper, double *diag, double *internal, double *boundary, void *stream)
{
    int rc = check_ldu(m);
    if (rc != CHEM_OK) return rc;
    if (!all_dev({gamma_c, diag}) || (m->nfaces && !all_dev({lower, upper})) ||
        (m->nbfaces && !all_dev({gamma_b, psi_b, internal, boundary})))
        return fail(CHEM_EINVAL, "arrays must be device pointers");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(chem::ldu_zero_kernel, dim3(chem::ldu_blocks(m->ncells)), dim3(chem::kLduBlock), 0, st, diag,
                       m->ncells);
    if (m->nfaces)
        hipLaunchKernelGGL(chem::ldu_internal_kernel, dim3(chem::ldu_blocks(m->nfaces)), dim3(chem::kLduBlock), 0, st,
                           m->nfaces, m->owner, m->neighbour, m->weight, m->delta, m->mag_sf, gamma_c, lower, upper,
                           diag);
    for (size_t p = 0; p < m->patch_type.size(); p++) {
        const int64_t s = m->patch_start[p], c = m->patch_start[p + 1] - s;
        if (c <= 0) continue;
        if (m->patch_type[p] == 0)
            hipLaunchKernelGGL(chem::ldu_patch_kernel<0>, dim3(chem::ldu_blocks(c)), dim3(chem::kLduBlock), 0, st, s,
                               c, m->bdelta, m->bmag_sf, gamma_b, psi_b, internal, boundary);
        else
            hipLaunchKernelGGL(chem::ldu_patch_kernel<1>, dim3(chem::ldu_blocks(c)), dim3(chem::kLduBlock), 0, st, s,
                               c, m->bdelta, m->bmag_sf, gamma_b, psi_b, internal, boundary);
    }
    return check_hip(hipGetLastError(), "laplacian launch");
}

int chem_ldu_to_csr(chem_ldu m, const double *lower, const double *upper, const double *diag, const double *internal,
                    const double *boundary, double *csr_val, double *rhs, void *stream)
{
    int rc = check_ldu(m);
    if (rc != CHEM_OK) return rc;
    if (!all_dev({diag, csr_val, rhs}) || (m->nfaces && !all_dev({lower, upper})) ||
        (m->nbfaces && !all_dev({internal, boundary})))
        return fail(CHEM_EINVAL, "arrays must be device pointers");
    hipStream_t st = (hipStream_t)stream;
    if (m->nfaces)
        hipLaunchKernelGGL(chem::csr_faces_kernel, dim3(chem::ldu_blocks(m->nfaces)), dim3(chem::kLduBlock), 0, st,
                           m->nfaces, m->upper_pos, m->lower_pos, lower, upper, csr_val);
    hipLaunchKernelGGL(chem::csr_cells_kernel, dim3(chem::ldu_blocks(m->ncells)), dim3(chem::kLduBlock), 0, st,
                       m->ncells, m->diag_pos, m->bnd_ptr, m->bnd_face, diag, internal, boundary, csr_val, rhs);
    return check_hip(hipGetLastError(), "csr launch");
}

int chem_ldu_laplacian_csr(chem_ldu m, const double *gamma_c, const double *gamma_b, const double *psi_b,
                           double *csr_val, double *rhs, void *stream)
{
    int rc = check_ldu(m);
    if (rc != CHEM_OK) return rc;
    if (!all_dev({gamma_c, csr_val, rhs}) || (m->nbfaces && !all_dev({gamma_b, psi_b})))
        return fail(CHEM_EINVAL, "arrays must be device pointers");
    hipStream_t st = (hipStream_t)stream;
    if (m->nfaces)
        hipLaunchKernelGGL(chem::face_coeff_kernel, dim3(chem::ldu_blocks(m->nfaces)), dim3(chem::kLduBlock), 0, st,
                           m->nfaces, m->owner, m->neighbour, m->weight, m->delta, m->mag_sf, gamma_c, m->coef);
    hipLaunchKernelGGL(chem::csr_assemble_entries_kernel, dim3((unsigned)((m->nnz + chem::kEntBlock - 1) / chem::kEntBlock)),
                       dim3(chem::kLduBlock), 0,
                       st, m->nnz, m->row_ptr, m->ent_face, m->coef, m->bnd_ptr, m->bnd_face, m->btype, m->bdelta,
                       m->bmag_sf, gamma_b, psi_b, csr_val, rhs);
    return check_hip(hipGetLastError(), "csr assembly launch");
}

int chem_ldu_csr_pattern(chem_ldu m, int32_t *row_ptr, int32_t *col, void *stream)
{
    int rc = check_ldu(m);
    if (rc != CHEM_OK) return rc;
    if (!all_dev({row_ptr, col})) return fail(CHEM_EINVAL, "arrays must be device pointers");
    hipStream_t st = (hipStream_t)stream;
    rc = check_hip(hipMemcpyAsync(row_ptr, m->row_ptr, (size_t)(m->ncells + 1) * 4, hipMemcpyDeviceToDevice, st),
                   "pattern copy");
    if (rc == CHEM_OK)
        rc = check_hip(hipMemcpyAsync(col, m->col, (size_t)m->nnz * 4, hipMemcpyDeviceToDevice, st), "pattern copy");
    return rc;
}

}  // extern "C"

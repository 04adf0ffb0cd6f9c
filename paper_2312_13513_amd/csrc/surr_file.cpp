// Surrogate weights / checkpoint file; see surr_file.h.

#include "surr_file.h"

#include <cmath>
#include <cstring>
#include <fstream>
#include <iterator>

namespace chem_file {

namespace {

constexpr size_t kMagic = 8;
constexpr int32_t kMaxDim = 1 << 16;

struct Reader {
    const char *p;
    size_t end, o;
    bool get(void *d, size_t n)
    {
        if (n > end - o) return false;
        if (n) std::memcpy(d, p + o, n);
        o += n;
        return true;
    }
};

}  // namespace

int64_t surr_param_count(int32_t nin, int32_t h1, int32_t h2, int32_t h3, int32_t K)
{
    const int64_t in[4] = {nin, h1, h2, h3}, out[4] = {h1, h2, h3, K};
    int64_t n = 0;
    for (int l = 0; l < 4; l++) n += in[l] * out[l] + out[l];
    return n;
}

unsigned long long fnv1a(const char *p, size_t n, unsigned long long h)
{
    for (size_t i = 0; i < n; i++) {
        h ^= (unsigned char)p[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

std::string encode_surr(const SurrFile &f)
{
    std::string buf("CHEMSURR", kMagic);
    auto put = [&](const void *d, size_t n) { buf.append((const char *)d, n); };
    const int32_t ver = f.has_opt ? 2 : 1, hdr[6] = {f.K, f.nin, f.h[0], f.h[1], f.h[2], f.K};
    const double lam = 0.1;
    put(&ver, 4);
    put(hdr, sizeof(hdr));
    put(&lam, 8);
    const int32_t nset = f.norm_set ? 1 : 0;
    const int64_t nn = (int64_t)f.norm.size(), np = (int64_t)f.params.size();
    put(&nset, 4);
    put(&nn, 8);
    put(f.norm.data(), (size_t)nn * 8);
    put(&np, 8);
    put(f.params.data(), (size_t)np * 4);
    if (f.has_opt) {
        const int64_t nu = (int64_t)f.user.size();
        put(&f.adam_t, 8);
        put(f.m.data(), (size_t)np * 4);
        put(f.v.data(), (size_t)np * 4);
        put(&nu, 8);
        put(f.user.data(), (size_t)nu);
    }
    const unsigned long long sum = fnv1a(buf.data(), buf.size());
    put(&sum, 8);
    return buf;
}

int decode_surr(const char *data, size_t size, SurrFile &f, std::string &err)
{
    auto bad = [&err](const char *msg) {
        err = msg;
        return -1;
    };
    if (!data || size < kMagic + 8 || std::memcmp(data, "CHEMSURR", kMagic) != 0)
        return bad("not a surrogate file");
    unsigned long long sum = 0;
    std::memcpy(&sum, data + size - 8, 8);
    if (fnv1a(data, size - 8) != sum) return bad("surrogate file checksum mismatch");
    Reader r{data, size - 8, kMagic};
    int32_t ver = 0, hdr[6] = {0, 0, 0, 0, 0, 0}, nset = 0;
    double lam = 0;
    int64_t nn = 0, np = 0;
    if (!r.get(&ver, 4) || (ver != 1 && ver != 2) || !r.get(hdr, sizeof(hdr)) || !r.get(&lam, 8) ||
        !r.get(&nset, 4) || !r.get(&nn, 8))
        return bad("bad surrogate header");
    for (int i = 0; i < 5; i++)
        if (hdr[i] < 1 || hdr[i] > kMaxDim) return bad("bad network dimensions");
    if (hdr[5] != hdr[0] || hdr[1] != hdr[0] + 2 || lam != 0.1 || (nset != 0 && nset != 1))
        return bad("bad surrogate header");
    f = SurrFile();
    f.K = hdr[0];
    f.nin = hdr[1];
    for (int l = 0; l < 3; l++) f.h[l] = hdr[2 + l];
    f.norm_set = nset == 1;
    if (nn != 2 * (int64_t)f.nin + 2 * (int64_t)f.K + 1) return bad("bad normalisation length");
    f.norm.resize((size_t)nn);
    if (!r.get(f.norm.data(), (size_t)nn * 8) || !r.get(&np, 8)) return bad("truncated surrogate file");
    if (np != surr_param_count(f.nin, f.h[0], f.h[1], f.h[2], f.K)) return bad("bad parameter count");
    if ((size_t)np > (r.end - r.o) / 4) return bad("truncated surrogate file");
    f.params.resize((size_t)np);
    if (!r.get(f.params.data(), (size_t)np * 4)) return bad("truncated surrogate file");
    if (ver == 2) {
        int64_t nu = -1;
        if ((size_t)np > (r.end - r.o) / 8 || !r.get(&f.adam_t, 8) || f.adam_t < 0)
            return bad("truncated or bad optimiser state");
        f.m.resize((size_t)np);
        f.v.resize((size_t)np);
        if (!r.get(f.m.data(), (size_t)np * 4) || !r.get(f.v.data(), (size_t)np * 4) || !r.get(&nu, 8) ||
            nu < 0 || nu > kSurrMaxUser)
            return bad("truncated or bad optimiser state");
        f.user.resize((size_t)nu);
        if (!r.get(&f.user[0], (size_t)nu)) return bad("truncated surrogate file");
        f.has_opt = true;
    }
    if (r.o != r.end) return bad("trailing bytes in the surrogate file");
    if (f.norm_set)
        for (double x : f.norm)
            if (!std::isfinite(x)) return bad("normalisation values must be finite");
    return 0;
}

int read_surr_file(const char *path, SurrFile &f, std::string &err)
{
    std::ifstream in(path, std::ios::binary);
    if (!in) {
        err = "cannot open the file";
        return -1;
    }
    std::string buf((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
    return decode_surr(buf.data(), buf.size(), f, err);
}

}  // namespace chem_file

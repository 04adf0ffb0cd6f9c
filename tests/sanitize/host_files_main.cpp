// Host-only driver of the library's two file readers (mechanism text files
// and surrogate weight / checkpoint files), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by the sanitizer test and fed valid and
// damaged files.
//
//   host_files mech <path>...         parse each; prints "ok K R E" or "rejected: <why>" per file
//   host_files surr <path>...         decode each; a file that decodes must encode back to the same bytes
//   host_files surr-write <path> K h1 h2 h3 opt user_bytes
//                                     writes a well-formed file with seeded contents
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iterator>
#include <string>

#include "mech_file.h"
#include "surr_file.h"

namespace {

int do_mech(const char *path)
{
    chem_file::HostMech m;
    std::string err;
    if (chem_file::parse_mech_file(path, m, err) != 0) {
        std::printf("rejected: %s\n", err.c_str());
        return 0;
    }
    std::printf("ok %d %d %d\n", m.K, m.R, m.E);
    return 0;
}

int do_surr(const char *path)
{
    std::ifstream in(path, std::ios::binary);
    std::string buf((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
    chem_file::SurrFile f;
    std::string err;
    if (chem_file::decode_surr(buf.data(), buf.size(), f, err) != 0) {
        std::printf("rejected: %s\n", err.c_str());
        return 0;
    }
    if (chem_file::encode_surr(f) != buf) {
        std::printf("round trip changed the file\n");
        return 1;
    }
    std::printf("ok %d %d %d %d %d opt=%d user=%zu\n", f.K, f.nin, f.h[0], f.h[1], f.h[2], f.has_opt ? 1 : 0,
                f.user.size());
    return 0;
}

int do_write(int argc, char **argv)
{
    if (argc != 9) return 2;
    chem_file::SurrFile f;
    f.K = std::atoi(argv[3]);
    f.nin = f.K + 2;
    for (int l = 0; l < 3; l++) f.h[l] = std::atoi(argv[4 + l]);
    f.norm_set = true;
    f.norm.resize((size_t)(2 * f.nin + 2 * f.K + 1));
    for (size_t i = 0; i < f.norm.size(); i++) f.norm[i] = 1.0 + 0.25 * (double)i;
    const int64_t np = chem_file::surr_param_count(f.nin, f.h[0], f.h[1], f.h[2], f.K);
    unsigned x = 12345u;
    auto next = [&x]() {
        x = x * 1664525u + 1013904223u;
        return (float)(x >> 8) / 16777216.0f - 0.5f;
    };
    f.params.resize((size_t)np);
    for (auto &v : f.params) v = next();
    f.has_opt = std::atoi(argv[7]) != 0;
    if (f.has_opt) {
        f.adam_t = 77;
        f.m.resize((size_t)np);
        f.v.resize((size_t)np);
        for (int64_t i = 0; i < np; i++) {
            f.m[(size_t)i] = 1e-3f * next();
            f.v[(size_t)i] = 1e-6f * (next() + 0.5f);
        }
        f.user.assign((size_t)std::atoi(argv[8]), 'u');
    }
    const std::string bytes = chem_file::encode_surr(f);
    std::ofstream out(argv[2], std::ios::binary);
    out.write(bytes.data(), (std::streamsize)bytes.size());
    return out ? 0 : 1;
}

}  // namespace

int main(int argc, char **argv)
{
    const bool mech = argc >= 3 && !std::strcmp(argv[1], "mech"), surr = argc >= 3 && !std::strcmp(argv[1], "surr");
    if (mech || surr) {
        int rc = 0;
        for (int i = 2; i < argc && rc == 0; i++) rc = mech ? do_mech(argv[i]) : do_surr(argv[i]);
        return rc;
    }
    if (argc >= 3 && !std::strcmp(argv[1], "surr-write")) return do_write(argc, argv);
    std::fprintf(stderr, "usage: host_files mech|surr|surr-write <path> ...\n");
    return 2;
}

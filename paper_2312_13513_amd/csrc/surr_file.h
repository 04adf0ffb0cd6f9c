// Surrogate weights / checkpoint file: magic "CHEMSURR", version, network
// dimensions, normalisation, FP32 parameters in logical order and an FNV-1a
// checksum of everything before it.  Version 2 adds the optimiser state
// (Adam step and both moment vectors, logical order) and up to 1 MiB of the
// caller's own bytes (its sample-order generator state), so that training
// can resume exactly.  Plain C++17 with no HIP dependency (the sanitizer
// build of the tests builds it for the host alone).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace chem_file {

constexpr int64_t kSurrMaxUser = int64_t(1) << 20;

struct SurrFile {
    int32_t K = 0, nin = 0, h[3] = {0, 0, 0};
    bool norm_set = false;
    std::vector<double> norm;      // 2 nin + 2 K + 1 values (mu_x, sig_x, mu_y, sig_y, dt)
    std::vector<float> params;     // logical order, surr_param_count() values
    bool has_opt = false;          // version 2: optimiser state follows
    int64_t adam_t = 0;
    std::vector<float> m, v;       // Adam moments, logical order
    std::string user;              // the caller's bytes
};

// Parameter count of the network nin -> h1 -> h2 -> h3 -> K (weights and biases).
int64_t surr_param_count(int32_t nin, int32_t h1, int32_t h2, int32_t h3, int32_t K);

unsigned long long fnv1a(const char *p, size_t n, unsigned long long h = 0xCBF29CE484222325ull);

// Serialises f (version 2 when f.has_opt, else 1).  The sizes of f's vectors
// must already agree with its dimensions.
std::string encode_surr(const SurrFile &f);

// Parses and checks a whole file image.  Returns 0, or -1 with a message in err.
int decode_surr(const char *data, size_t size, SurrFile &f, std::string &err);
int read_surr_file(const char *path, SurrFile &f, std::string &err);

}  // namespace chem_file

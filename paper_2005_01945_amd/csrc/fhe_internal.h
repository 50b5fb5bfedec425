// Internal declarations shared by the library's host and device sources.
#pragma once

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fhe.h"

namespace fhe {

// Structural parameters the kernels are specialised for.
constexpr uint32_t kN = 1024;        // ring degree
constexpr uint32_t kLweN = 500;      // LWE dimension
constexpr uint32_t kLweW = kLweN + 1;
constexpr uint32_t kBkL = 2;         // gadget digits
constexpr uint32_t kBgBit = 10;
constexpr uint32_t kKsT = 8;         // key-switch digits
constexpr uint32_t kKsBaseBit = 2;
constexpr uint32_t kKsBase = 1u << kKsBaseBit;
constexpr uint32_t kMu = 1u << 29;   // 1/8 on the torus
constexpr uint32_t kKskRowWords = 512;  // one KS row padded to 2 KB for 16-byte loads

// Sets the thread-local error message and returns `code`.
int set_error(int code, const char* fmt, ...);
void clear_error();

bool params_supported(const fhe_params& P, std::string* why);

}  // namespace fhe

struct fhe_secret_key {
    fhe_params P;
    uint64_t seed;
    std::vector<int32_t> lwe;   // [n]
    std::vector<int32_t> tlwe;  // [N]
};

struct fhe_cloud_key {
    fhe_params P;
    uint64_t seed;
    std::vector<uint32_t> bk;   // [n][2l][2][N]
    std::vector<uint32_t> ksk;  // [N][t][B][n+1]
};

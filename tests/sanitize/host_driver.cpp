// Drives the library's host-only code (keys, encryption, key files, circuit
// builders and level schedules) for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer.  Exits non-zero on any wrong result; the
// sanitizers abort on any memory or undefined-behaviour error.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/fhe.h"
#include "../../paper_2005_01945_amd/csrc/circuit_ir.h"

#define CHECK(x)                                                     \
    do {                                                             \
        if (!(x)) {                                                  \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
            return 1;                                                \
        }                                                            \
    } while (0)

int main(int argc, char** argv) {
    const char* path = argc > 1 ? argv[1] : "sanitize_keys.bin";
    fhe_params P;
    CHECK(fhe_default_params(&P) == FHE_OK);
    fhe_secret_key* sk = nullptr;
    fhe_cloud_key* ck = nullptr;
    CHECK(fhe_keygen(&P, 0, &sk, &ck) == FHE_OK);
    const uint32_t W = P.n + 1;

    // encryption round trips, bits and integers of every width
    for (uint32_t width = 1; width <= 64; width += 9) {
        std::vector<uint64_t> v = {0, 1, 0x123456789abcdefull, ~0ull};
        std::vector<uint32_t> ct(v.size() * width * W);
        CHECK(fhe_encrypt_uint(sk, v.data(), v.size(), width, 1000 * width, ct.data()) == FHE_OK);
        std::vector<uint64_t> back(v.size());
        CHECK(fhe_decrypt_uint(sk, ct.data(), v.size(), width, back.data()) == FHE_OK);
        const uint64_t mask = width == 64 ? ~0ull : (1ull << width) - 1;
        for (size_t i = 0; i < v.size(); ++i) CHECK(back[i] == (v[i] & mask));
        std::vector<int32_t> ph(v.size() * width);
        CHECK(fhe_phase(sk, ct.data(), v.size() * width, ph.data()) == FHE_OK);
    }
    uint8_t bits[5] = {0, 1, 1, 0, 1}, out[5];
    std::vector<uint32_t> cb(5 * W);
    CHECK(fhe_encrypt_bits(sk, bits, 5, 77, cb.data()) == FHE_OK);
    CHECK(fhe_decrypt_bits(sk, cb.data(), 5, out) == FHE_OK);
    for (int i = 0; i < 5; ++i) CHECK(out[i] == bits[i]);
    uint8_t bad[1] = {2};
    CHECK(fhe_encrypt_bits(sk, bad, 1, 0, cb.data()) == FHE_EINVAL);

    // export, save and load
    std::vector<int32_t> lwe(P.n), tlwe(P.N);
    CHECK(fhe_secret_key_export(sk, lwe.data(), tlwe.data()) == FHE_OK);
    std::vector<uint32_t> bk((size_t)P.n * 4 * 2 * P.N), ksk((size_t)P.N * 8 * 4 * W);
    CHECK(fhe_cloud_key_export(ck, bk.data(), ksk.data()) == FHE_OK);
    CHECK(fhe_key_save(sk, ck, path) == FHE_OK);
    fhe_secret_key* sk2 = nullptr;
    fhe_cloud_key* ck2 = nullptr;
    CHECK(fhe_key_load(path, &sk2, &ck2) == FHE_OK);
    std::vector<uint32_t> bk2(bk.size());
    CHECK(fhe_cloud_key_export(ck2, bk2.data(), nullptr) == FHE_OK);
    CHECK(bk2 == bk);
    fhe_secret_key_free(sk2);
    fhe_cloud_key_free(ck2);
    fhe_secret_key* sk3 = nullptr;
    fhe_cloud_key* ck3 = nullptr;
    CHECK(fhe_key_load("/nonexistent/keys.bin", &sk3, &ck3) == FHE_EIO);
    CHECK(!sk3 && !ck3);
    std::remove(path);

    // every circuit kind at several widths, its levels and balanced schedules
    for (int kind = 0; kind <= fhe::kLastKind; ++kind)
        for (uint32_t w : {1u, 2u, 5u, 16u, 33u}) {
            if (kind == fhe::kKaratsuba && w < 2) continue;
            const uint32_t rows = kind == fhe::kMatvec ? 3 : kind == fhe::kMatmul ? 2 : 0;
            const uint32_t cols = kind == fhe::kMatvec ? 4 : 0;
            const fhe::Circuit c = fhe::build_circuit(kind, w, rows, cols);
            uint32_t depth = 0;
            const std::vector<uint32_t> asap = fhe::asap_levels(c, &depth);
            CHECK(asap.size() == c.gates.size());
            for (size_t count : {(size_t)1, (size_t)7, (size_t)1024}) {
                const std::vector<uint32_t> lev = fhe::balance_levels(c, asap, depth, count, 2048);
                CHECK(lev.size() == c.gates.size());
                const uint32_t base = c.na + c.nb;
                for (size_t k = 0; k < lev.size(); ++k) {
                    CHECK(lev[k] >= asap[k] && lev[k] <= depth);
                    const fhe::Gate& g = c.gates[k];  // every input from an earlier level
                    for (uint32_t in : {g.in0, g.in1, g.in2})
                        if (in != fhe::kNoWire && in >= base) CHECK(lev[in - base] < lev[k]);
                    if (g.second) CHECK(lev[k] == lev[k - 1]);  // a compound node stays whole
                }
            }
            uint64_t g = 0;
            uint32_t lv = 0;
            CHECK(fhe_circuit_shape(kind, w, rows, cols, &g, &lv, nullptr) == FHE_OK);
            CHECK(lv == depth && g == c.bootstraps());
            std::vector<uint64_t> sched(depth);
            CHECK(fhe_circuit_schedule(kind, w, rows, cols, 5, 256, sched.data(), depth, &lv) == FHE_OK);
        }
    fhe_secret_key_free(sk);
    fhe_cloud_key_free(ck);
    std::puts("host checks passed");
    return 0;
}

// Host-side TFHE: parameters, the counter-based generator, key generation,
// LWE encryption / decryption / phase, key serialisation.
//
// LWE sample (A, B = A.S + e) with binary key and Gaussian noise, one bit per
// sample and an n-bit integer as n samples: paper Sec. II-A.  Key structure
// (TGSW bootstrapping key, LWE key-switching key) follows the published TFHE
// method the paper builds on (Chillotti et al., ASIACRYPT 2016).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <thread>

#include "fhe_internal.h"

namespace fhe {

static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

bool params_supported(const fhe_params& P, std::string* why) {
    if (P.n != kLweN || P.N != kN || P.k != 1 || P.bk_l != kBkL || P.bk_bgbit != kBgBit ||
        P.ks_t != kKsT || P.ks_basebit != kKsBaseBit) {
        *why = "only n=500 N=1024 k=1 l=2 Bgbit=10 t=8 basebit=2 is supported";
        return false;
    }
    if (!(P.lwe_stdev >= 0.0 && P.lwe_stdev < 0.1 && P.bk_stdev >= 0.0 && P.bk_stdev < 0.1)) {
        *why = "noise deviations must lie in [0, 0.1)";
        return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Counter-based generator: the SplitMix64 output function (Steele, Lea,
// Flood, OOPSLA 2014) applied to a Weyl sequence.  A stream is keyed by
// (seed, stream id); value idx of the stream is
//     out(out(seed + G*(id+1)) + G*(idx+1)),  G = 0x9E3779B97F4A7C15.
// ---------------------------------------------------------------------------
namespace {

constexpr uint64_t kWeyl = 0x9E3779B97F4A7C15ull;

inline uint64_t splitmix_output(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

enum StreamId : uint64_t {
    kStreamLweKey = 1, kStreamTlweKey = 2, kStreamBkMask = 3, kStreamBkNoise = 4,
    kStreamKskMask = 5, kStreamKskNoise = 6, kStreamEncMask = 7, kStreamEncNoise = 8
};

class Stream {
  public:
    Stream(uint64_t seed, uint64_t id) : key_(splitmix_output(seed + kWeyl * (id + 1))) {}
    uint64_t word64(uint64_t idx) const { return splitmix_output(key_ + kWeyl * (idx + 1)); }
    uint32_t torus(uint64_t idx) const { return static_cast<uint32_t>(word64(idx) >> 32); }
    int32_t bit(uint64_t idx) const { return static_cast<int32_t>(word64(idx) >> 63); }
    // Standard normal by Box-Muller (cosine branch) from values 2idx, 2idx+1.
    double normal(uint64_t idx) const {
        const uint64_t x = word64(2 * idx), y = word64(2 * idx + 1);
        const double u1 = static_cast<double>((x >> 11) + 1) * 0x1.0p-53;
        const double u2 = static_cast<double>(y >> 11) * 0x1.0p-53;
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    }

  private:
    uint64_t key_;
};

// Real x in (-1/2, 1/2) -> Torus32, round to nearest with ties to even.
inline uint32_t to_torus32(double x) {
    return static_cast<uint32_t>(static_cast<int64_t>(std::nearbyint(x * 0x1p32)));
}

// acc += X^j * a in Z/2^32[X]/(X^N+1) for 0 <= j < N.
inline void add_shifted(uint32_t* acc, const uint32_t* a, uint32_t j) {
    const uint32_t N = kN;
    for (uint32_t c = 0; c + j < N; ++c) acc[c + j] += a[c];
    for (uint32_t c = N - j; c < N; ++c) acc[c + j - N] -= a[c];
}

template <class F>
void parallel_for(uint32_t count, F&& body) {
    unsigned T = std::thread::hardware_concurrency();
    if (T == 0) T = 1;
    if (T > 16) T = 16;
    if (T > count) T = count ? count : 1;
    std::vector<std::thread> pool;
    for (unsigned w = 0; w < T; ++w)
        pool.emplace_back([&, w] {
            for (uint32_t i = w; i < count; i += T) body(i);
        });
    for (auto& th : pool) th.join();
}

}  // namespace

}  // namespace fhe

using namespace fhe;

extern "C" int fhe_default_params(fhe_params* out) {
    if (!out) return set_error(FHE_EINVAL, "fhe_default_params: null output");
    out->n = kLweN;
    out->N = kN;
    out->k = 1;
    out->bk_l = kBkL;
    out->bk_bgbit = kBgBit;
    out->ks_t = kKsT;
    out->ks_basebit = kKsBaseBit;
    out->lwe_stdev = 2.44e-5;
    out->bk_stdev = 7.18e-9;
    return FHE_OK;
}

extern "C" int fhe_keygen_with_keys(const fhe_params* params, uint64_t seed,
                                    const int32_t* lwe_key, const int32_t* tlwe_key,
                                    fhe_secret_key** sk_out, fhe_cloud_key** ck_out) {
    if (!params || !sk_out || !ck_out) return set_error(FHE_EINVAL, "fhe_keygen: null argument");
    std::string why;
    if (!params_supported(*params, &why)) return set_error(FHE_EINVAL, "fhe_keygen: %s", why.c_str());
    const fhe_params P = *params;
    const uint32_t n = P.n, N = P.N, rows = 2 * P.bk_l, B = 1u << P.ks_basebit;

    fhe_secret_key* sk = nullptr;
    fhe_cloud_key* ck = nullptr;
    try {
        sk = new fhe_secret_key{P, seed, std::vector<int32_t>(n), std::vector<int32_t>(N)};
        ck = new fhe_cloud_key{P, seed, std::vector<uint32_t>((size_t)n * rows * 2 * N),
                               std::vector<uint32_t>((size_t)N * P.ks_t * B * (n + 1), 0u)};
    } catch (...) {
        delete sk;
        delete ck;
        return set_error(FHE_ENOMEM, "fhe_keygen: out of host memory");
    }

    const Stream lwe_s(seed, kStreamLweKey), tlwe_s(seed, kStreamTlweKey);
    for (uint32_t i = 0; i < n; ++i) {
        const int32_t b = lwe_key ? lwe_key[i] : lwe_s.bit(i);
        if (b != 0 && b != 1) { delete sk; delete ck; return set_error(FHE_EINVAL, "lwe_key must be 0/1"); }
        sk->lwe[i] = b;
    }
    for (uint32_t j = 0; j < N; ++j) {
        const int32_t b = tlwe_key ? tlwe_key[j] : tlwe_s.bit(j);
        if (b != 0 && b != 1) { delete sk; delete ck; return set_error(FHE_EINVAL, "tlwe_key must be 0/1"); }
        sk->tlwe[j] = b;
    }
    std::vector<uint32_t> ones;  // positions j with S_j = 1
    for (uint32_t j = 0; j < N; ++j)
        if (sk->tlwe[j]) ones.push_back(j);

    // Bootstrapping key.  BK_i row r = 2j + p is the TLWE zero sample
    // (A, A*S + E) plus s_i * 2^(32 - Bgbit(p+1)) on coefficient 0 of
    // column j: a TGSW encryption of s_i.
    const Stream bk_mask(seed, kStreamBkMask), bk_noise(seed, kStreamBkNoise);
    parallel_for(n, [&](uint32_t i) {
        for (uint32_t r = 0; r < rows; ++r) {
            uint32_t* A = &ck->bk[(((size_t)i * rows + r) * 2 + 0) * N];
            uint32_t* Bp = &ck->bk[(((size_t)i * rows + r) * 2 + 1) * N];
            const uint64_t off = ((uint64_t)i * rows + r) * N;
            for (uint32_t c = 0; c < N; ++c) A[c] = bk_mask.torus(off + c);
            for (uint32_t c = 0; c < N; ++c) Bp[c] = to_torus32(P.bk_stdev * bk_noise.normal(off + c));
            for (uint32_t j : ones) add_shifted(Bp, A, j);  // + A*S, S binary
            const uint32_t col = r / P.bk_l, digit = r % P.bk_l;
            const uint32_t gadget = 1u << (32 - P.bk_bgbit * (digit + 1));
            (col == 0 ? A : Bp)[0] += gadget * static_cast<uint32_t>(sk->lwe[i]);
        }
    });

    // Key-switching key.  KSK[i][j][v], v >= 1, encrypts v * S_i *
    // 2^(32 - basebit(j+1)) under the LWE key; v = 0 stays all zero.
    const Stream ks_mask(seed, kStreamKskMask), ks_noise(seed, kStreamKskNoise);
    parallel_for(N, [&](uint32_t i) {
        for (uint32_t j = 0; j < P.ks_t; ++j)
            for (uint32_t v = 1; v < B; ++v) {
                uint32_t* row = &ck->ksk[(((size_t)i * P.ks_t + j) * B + v) * (n + 1)];
                const uint64_t sample = ((uint64_t)i * P.ks_t + j) * (B - 1) + (v - 1);
                uint32_t dot = 0;
                for (uint32_t l = 0; l < n; ++l) {
                    row[l] = ks_mask.torus(sample * n + l);
                    if (sk->lwe[l]) dot += row[l];
                }
                const uint32_t msg = static_cast<uint32_t>(sk->tlwe[i]) * v << (32 - P.ks_basebit * (j + 1));
                row[n] = dot + to_torus32(P.lwe_stdev * ks_noise.normal(sample)) + msg;
            }
    });

    *sk_out = sk;
    *ck_out = ck;
    return FHE_OK;
}

extern "C" int fhe_keygen(const fhe_params* params, uint64_t seed, fhe_secret_key** sk,
                          fhe_cloud_key** ck) {
    return fhe_keygen_with_keys(params, seed, nullptr, nullptr, sk, ck);
}

extern "C" void fhe_secret_key_free(fhe_secret_key* sk) { delete sk; }
extern "C" void fhe_cloud_key_free(fhe_cloud_key* ck) { delete ck; }

extern "C" int fhe_secret_key_export(const fhe_secret_key* sk, int32_t* lwe_key, int32_t* tlwe_key) {
    if (!sk) return set_error(FHE_EINVAL, "fhe_secret_key_export: null key");
    if (lwe_key) std::memcpy(lwe_key, sk->lwe.data(), sk->lwe.size() * sizeof(int32_t));
    if (tlwe_key) std::memcpy(tlwe_key, sk->tlwe.data(), sk->tlwe.size() * sizeof(int32_t));
    return FHE_OK;
}

extern "C" int fhe_cloud_key_export(const fhe_cloud_key* ck, uint32_t* bk, uint32_t* ksk) {
    if (!ck) return set_error(FHE_EINVAL, "fhe_cloud_key_export: null key");
    if (bk) std::memcpy(bk, ck->bk.data(), ck->bk.size() * sizeof(uint32_t));
    if (ksk) std::memcpy(ksk, ck->ksk.data(), ck->ksk.size() * sizeof(uint32_t));
    return FHE_OK;
}

extern "C" int fhe_cloud_key_params(const fhe_cloud_key* ck, fhe_params* out) {
    if (!ck || !out) return set_error(FHE_EINVAL, "fhe_cloud_key_params: null argument");
    *out = ck->P;
    return FHE_OK;
}

// ---------------------------------------------------------------------------
// Encryption: b = <a, s> + e + (bit ? +mu : -mu); ciphertext index q = nonce
// + c draws its mask from stream 7 at q*n + l and its noise from stream 8 at q.
// ---------------------------------------------------------------------------
static void encrypt_one(const fhe_secret_key* sk, uint8_t bit, uint64_t q, uint32_t* s) {
    const uint32_t n = sk->P.n;
    const Stream mask(sk->seed, kStreamEncMask), noise(sk->seed, kStreamEncNoise);
    uint32_t dot = 0;
    for (uint32_t l = 0; l < n; ++l) {
        s[l] = mask.torus(q * n + l);
        dot += s[l] * static_cast<uint32_t>(sk->lwe[l]);
    }
    s[n] = dot + to_torus32(sk->P.lwe_stdev * noise.normal(q)) + (bit ? kMu : 0u - kMu);
}

extern "C" int fhe_encrypt_bits(const fhe_secret_key* sk, const uint8_t* bits, size_t count,
                                uint64_t nonce, uint32_t* ct_out) {
    if (!sk || (count && (!bits || !ct_out))) return set_error(FHE_EINVAL, "fhe_encrypt_bits: null argument");
    const size_t W = sk->P.n + 1;
    for (size_t c = 0; c < count; ++c) {
        if (bits[c] > 1) return set_error(FHE_EINVAL, "fhe_encrypt_bits: bit %zu is %u", c, bits[c]);
        encrypt_one(sk, bits[c], nonce + c, ct_out + c * W);
    }
    return FHE_OK;
}

extern "C" int fhe_encrypt_uint(const fhe_secret_key* sk, const uint64_t* v, size_t count,
                                uint32_t width, uint64_t nonce, uint32_t* ct_out) {
    if (!sk || (count && (!v || !ct_out))) return set_error(FHE_EINVAL, "fhe_encrypt_uint: null argument");
    if (width < 1 || width > 64) return set_error(FHE_EINVAL, "fhe_encrypt_uint: width %u not in 1..64", width);
    const size_t W = sk->P.n + 1;
    for (size_t c = 0; c < count; ++c)
        for (uint32_t k = 0; k < width; ++k)
            encrypt_one(sk, (uint8_t)((v[c] >> k) & 1u), nonce + c * width + k,
                        ct_out + (c * width + k) * W);
    return FHE_OK;
}

extern "C" int fhe_phase(const fhe_secret_key* sk, const uint32_t* ct, size_t count, int32_t* phase_out) {
    if (!sk || (count && (!ct || !phase_out))) return set_error(FHE_EINVAL, "fhe_phase: null argument");
    const uint32_t n = sk->P.n;
    for (size_t c = 0; c < count; ++c) {
        const uint32_t* s = ct + c * (n + 1);
        uint32_t dot = 0;
        for (uint32_t l = 0; l < n; ++l) dot += s[l] * static_cast<uint32_t>(sk->lwe[l]);
        phase_out[c] = static_cast<int32_t>(s[n] - dot);
    }
    return FHE_OK;
}

extern "C" int fhe_decrypt_bits(const fhe_secret_key* sk, const uint32_t* ct, size_t count,
                                uint8_t* bits_out) {
    if (!sk || (count && (!ct || !bits_out))) return set_error(FHE_EINVAL, "fhe_decrypt_bits: null argument");
    std::vector<int32_t> ph(count);
    fhe_phase(sk, ct, count, ph.data());
    for (size_t c = 0; c < count; ++c) bits_out[c] = ph[c] > 0 ? 1 : 0;
    return FHE_OK;
}

extern "C" int fhe_decrypt_uint(const fhe_secret_key* sk, const uint32_t* ct, size_t count,
                                uint32_t width, uint64_t* v_out) {
    if (!sk || (count && (!ct || !v_out))) return set_error(FHE_EINVAL, "fhe_decrypt_uint: null argument");
    if (width < 1 || width > 64) return set_error(FHE_EINVAL, "fhe_decrypt_uint: width %u not in 1..64", width);
    std::vector<uint8_t> b((size_t)count * width);
    fhe_decrypt_bits(sk, ct, b.size(), b.data());
    for (size_t c = 0; c < count; ++c) {
        uint64_t v = 0;
        for (uint32_t k = 0; k < width; ++k) v |= (uint64_t)b[c * width + k] << k;
        v_out[c] = v;
    }
    return FHE_OK;
}

// ---------------------------------------------------------------------------
// Key file: "FHEKEYS1", params, seed, presence flags, then the arrays.
// ---------------------------------------------------------------------------
namespace {
constexpr char kMagic[8] = {'F', 'H', 'E', 'K', 'E', 'Y', 'S', '1'};

bool wr(FILE* f, const void* p, size_t bytes) { return std::fwrite(p, 1, bytes, f) == bytes; }
bool rd(FILE* f, void* p, size_t bytes) { return std::fread(p, 1, bytes, f) == bytes; }
}  // namespace

extern "C" int fhe_key_save(const fhe_secret_key* sk, const fhe_cloud_key* ck, const char* path) {
    if (!path || (!sk && !ck)) return set_error(FHE_EINVAL, "fhe_key_save: nothing to save");
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(FHE_EIO, "fhe_key_save: cannot open %s", path);
    const fhe_params P = sk ? sk->P : ck->P;
    const uint64_t seed = sk ? sk->seed : ck->seed;
    const uint32_t flags = (sk ? 1u : 0u) | (ck ? 2u : 0u);
    bool ok = wr(f, kMagic, 8) && wr(f, &P, sizeof P) && wr(f, &seed, 8) && wr(f, &flags, 4);
    if (ok && sk) ok = wr(f, sk->lwe.data(), sk->lwe.size() * 4) && wr(f, sk->tlwe.data(), sk->tlwe.size() * 4);
    if (ok && ck) ok = wr(f, ck->bk.data(), ck->bk.size() * 4) && wr(f, ck->ksk.data(), ck->ksk.size() * 4);
    ok = (std::fclose(f) == 0) && ok;
    return ok ? FHE_OK : set_error(FHE_EIO, "fhe_key_save: write to %s failed", path);
}

extern "C" int fhe_key_load(const char* path, fhe_secret_key** sk_out, fhe_cloud_key** ck_out) {
    if (!path || !sk_out || !ck_out) return set_error(FHE_EINVAL, "fhe_key_load: null argument");
    *sk_out = nullptr;
    *ck_out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(FHE_EIO, "fhe_key_load: cannot open %s", path);
    char magic[8];
    fhe_params P;
    uint64_t seed;
    uint32_t flags;
    std::string why;
    if (!rd(f, magic, 8) || std::memcmp(magic, kMagic, 8) != 0 || !rd(f, &P, sizeof P) ||
        !rd(f, &seed, 8) || !rd(f, &flags, 4) || !params_supported(P, &why) || flags == 0 || flags > 3) {
        std::fclose(f);
        return set_error(FHE_EIO, "fhe_key_load: %s is not a key file", path);
    }
    fhe_secret_key* sk = nullptr;
    fhe_cloud_key* ck = nullptr;
    bool ok = true;
    if (flags & 1u) {
        sk = new fhe_secret_key{P, seed, std::vector<int32_t>(P.n), std::vector<int32_t>(P.N)};
        ok = rd(f, sk->lwe.data(), P.n * 4) && rd(f, sk->tlwe.data(), P.N * 4);
    }
    if (ok && (flags & 2u)) {
        const size_t B = 1u << P.ks_basebit;
        ck = new fhe_cloud_key{P, seed, std::vector<uint32_t>((size_t)P.n * 2 * P.bk_l * 2 * P.N),
                               std::vector<uint32_t>((size_t)P.N * P.ks_t * B * (P.n + 1))};
        ok = rd(f, ck->bk.data(), ck->bk.size() * 4) && rd(f, ck->ksk.data(), ck->ksk.size() * 4);
    }
    std::fclose(f);
    if (!ok) {
        delete sk;
        delete ck;
        return set_error(FHE_EIO, "fhe_key_load: %s is truncated", path);
    }
    *sk_out = sk;
    *ck_out = ck;
    return FHE_OK;
}

extern "C" const char* fhe_last_error(void) { return fhe::g_last_error.c_str(); }

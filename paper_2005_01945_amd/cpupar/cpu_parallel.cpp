// The paper's CPU parallel framework (Sec. IV) as a host baseline beside the
// GPU path: every bootstrapped gate runs on one CPU core, and independent work
// is spread over the cores with OpenMP the way the paper describes it:
//  - a batch of gates (an n-bit gate operation): one gate per thread;
//  - additions (IV-A): the carry chain keeps the bits of one number in order,
//    so a vector of numbers is spread by number;
//  - multiplication (IV-B): the AND gates of the partial products run across
//    threads, their accumulation in order (the shift-and-add circuit).
// The gate bootstrap itself is the same TFHE gate bootstrap the GPU runs,
// with exact negacyclic products: forward and inverse NTTs modulo the two
// 28-bit primes 268369921 and 268367873, pointwise products, and the Chinese
// remainder theorem to lift the product sums (at most 2^52 in magnitude)
// back to Z/2^32.  The eight transforms of a CMux step (four digit
// polynomials, two primes) run side by side in the eight 32-bit lanes of an
// AVX2 register, so every butterfly stage is one vector operation per pair.
// Results are therefore the same words as the GPU's and the oracle's.  This
// is measurement code for the host baseline, not a fallback
// of the GPU path (nothing in the GPU library calls it).
#include <immintrin.h>
#include <omp.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr int N = 1024;
constexpr int NLWE = 500;
constexpr int NW = NLWE + 1;
constexpr int KS_T = 8;
constexpr uint32_t MU = 1u << 29;
constexpr uint32_t DECOMP_OFFSET = 0x80200800u;  // 2^31 + 2^21 + 2^11: rounding of the two 10-bit digits

int64_t powmod(int64_t b, int64_t e, int64_t m) {
    int64_t r = 1;
    b %= m;
    if (b < 0) b += m;
    while (e) {
        if (e & 1) r = (__int128)r * b % m;
        b = (__int128)b * b % m;
        e >>= 1;
    }
    return r;
}

int brv10(int x) {
    int r = 0;
    for (int i = 0; i < 10; ++i) r |= ((x >> i) & 1) << (9 - i);
    return r;
}

// Arithmetic modulo one prime q < 2^28 with signed Montgomery products
// (R = 2^32): mont(a) = (a - m q) / R with m = a q^-1 mod R lies in (-q, q)
// for |a| < q 2^31.
struct Prime {
    int32_t q;
    uint32_t qinv;       // q^-1 mod 2^32
    int32_t rmod;        // R mod q, centred: mont(x * rmod) = x mod q
    int32_t ninv_r;      // N^-1 R mod q: scales the inverse transform
    int32_t zeta[N];     // psi^brv10(k) R mod q, centred (k = 1 .. N-1)

    static int32_t centre(int64_t x, int32_t q) {
        int64_t r = x % q;
        if (r < 0) r += q;
        if (r > q / 2) r -= q;
        return (int32_t)r;
    }
    inline int32_t mont(int64_t a) const {
        const int32_t m = (int32_t)((uint32_t)a * qinv);
        return (int32_t)((a - (int64_t)m * q) >> 32);
    }
    inline int32_t reduce(int32_t x) const { return mont((int64_t)x * rmod); }

    void init(int32_t prime) {
        q = prime;
        uint32_t inv = 1;
        for (int i = 0; i < 5; ++i) inv *= 2u - (uint32_t)q * inv;  // Newton: inverse mod 2^32
        qinv = inv;
        const int64_t R = (int64_t)1 << 32;
        rmod = centre(R, q);
        // a generator of Z_q^*: no prime factor f of q - 1 has g^((q-1)/f) = 1
        std::vector<int64_t> fac;
        int64_t m = q - 1;
        for (int64_t f = 2; f * f <= m; ++f)
            if (m % f == 0) {
                fac.push_back(f);
                while (m % f == 0) m /= f;
            }
        if (m > 1) fac.push_back(m);
        int64_t g = 2;
        for (;; ++g) {
            bool ok = true;
            for (int64_t f : fac) ok = ok && powmod(g, (q - 1) / f, q) != 1;
            if (ok) break;
        }
        const int64_t psi = powmod(g, (q - 1) / (2 * N), q);  // primitive 2N-th root: psi^N = -1
        zeta[0] = 0;
        for (int k = 1; k < N; ++k) zeta[k] = centre((__int128)powmod(psi, brv10(k), q) * R % q, q);
        ninv_r = centre((__int128)powmod(N, q - 2, q) * R % q, q);
    }

    // Negacyclic forward transform (merged Cooley-Tukey, natural order in,
    // bit-reversed out).  |x| < 2^10 in; out |x| < 6q.  A reduction after the
    // fifth stage keeps every value below 6q < 2^31.
    void forward(int32_t* a) const {
        int k = 1;
        for (int len = N / 2; len >= 1; len >>= 1) {
            for (int start = 0; start < N; start += 2 * len) {
                const int64_t z = zeta[k++];
                int32_t* lo = a + start;
                int32_t* hi = a + start + len;
#pragma omp simd
                for (int j = 0; j < len; ++j) {
                    const int32_t t = mont(z * hi[j]);
                    hi[j] = lo[j] - t;
                    lo[j] = lo[j] + t;
                }
            }
            if (len == N / 32)
                for (int j = 0; j < N; ++j) a[j] = reduce(a[j]);
        }
    }

    // Inverse (Gentleman-Sande, bit-reversed in, natural out), scaled by
    // N^-1; every stage leaves values in (-q, q).  Output: the residue in (-q, q).
    void inverse(int32_t* a) const {
        int k = N - 1;
        for (int len = 1; len < N; len <<= 1) {
            for (int start = 0; start < N; start += 2 * len) {
                const int64_t z = zeta[k--];
                int32_t* lo = a + start;
                int32_t* hi = a + start + len;
#pragma omp simd
                for (int j = 0; j < len; ++j) {
                    const int32_t t = lo[j];
                    lo[j] = reduce(t + hi[j]);
                    hi[j] = mont(z * (hi[j] - t));
                }
            }
        }
        for (int j = 0; j < N; ++j) a[j] = mont((int64_t)a[j] * ninv_r);
    }
};

// Eight lanes of one register: lane 2r + p holds row r (0..3) in prime p.
struct Lanes {
    __m256i q, qinv, rmod, ninv;
    __m256i q_odd, qinv_odd;  // the odd lanes' constants moved to the even positions
    __m256i zeta[N];  // lane 2r + p: prime p's zeta[k]

    void init(const Prime (&P)[2]) {
        auto pair = [](int32_t a, int32_t b) { return _mm256_setr_epi32(a, b, a, b, a, b, a, b); };
        q = pair(P[0].q, P[1].q);
        qinv = pair((int32_t)P[0].qinv, (int32_t)P[1].qinv);
        rmod = pair(P[0].rmod, P[1].rmod);
        ninv = pair(P[0].ninv_r, P[1].ninv_r);
        q_odd = _mm256_srli_epi64(q, 32);
        qinv_odd = _mm256_srli_epi64(qinv, 32);
        for (int k = 0; k < N; ++k) zeta[k] = pair(P[0].zeta[k], P[1].zeta[k]);
    }
    // Signed Montgomery product of eight lanes: (a b - m q) / 2^32, |a b| < q 2^31.
    // The 32x32 -> 64-bit products take the even lanes; the odd lanes are
    // shifted down for theirs and their results come back in the high halves.
    inline __m256i mont(__m256i a, __m256i b) const {
        const __m256i pe = _mm256_mul_epi32(a, b);
        const __m256i po = _mm256_mul_epi32(_mm256_srli_epi64(a, 32), _mm256_srli_epi64(b, 32));
        const __m256i me = _mm256_mullo_epi32(pe, qinv);
        const __m256i mo = _mm256_mullo_epi32(po, qinv_odd);
        const __m256i te = _mm256_sub_epi64(pe, _mm256_mul_epi32(me, q));
        const __m256i to = _mm256_sub_epi64(po, _mm256_mul_epi32(mo, q_odd));
        return _mm256_blend_epi32(_mm256_srli_epi64(te, 32), to, 0xAA);
    }
    // The same transforms as Prime::forward / inverse on every lane.
    void forward(__m256i* a) const {
        int k = 1;
        for (int len = N / 2; len >= 1; len >>= 1) {
            for (int start = 0; start < N; start += 2 * len) {
                const __m256i z = zeta[k++];
                for (int j = start; j < start + len; ++j) {
                    const __m256i t = mont(z, a[j + len]);
                    a[j + len] = _mm256_sub_epi32(a[j], t);
                    a[j] = _mm256_add_epi32(a[j], t);
                }
            }
            if (len == N / 32)
                for (int j = 0; j < N; ++j) a[j] = mont(a[j], rmod);
        }
    }
    void inverse(__m256i* a) const {
        int k = N - 1;
        for (int len = 1; len < N; len <<= 1) {
            for (int start = 0; start < N; start += 2 * len) {
                const __m256i z = zeta[k--];
                for (int j = start; j < start + len; ++j) {
                    const __m256i t = a[j];
                    a[j] = mont(_mm256_add_epi32(t, a[j + len]), rmod);
                    a[j + len] = mont(z, _mm256_sub_epi32(a[j + len], t));
                }
            }
        }
        for (int j = 0; j < N; ++j) a[j] = mont(a[j], ninv);
    }
};

}  // namespace

struct cpupar {
    Prime p[2];
    Lanes v;
    int32_t crt_qinv;                 // q0^-1 mod q1
    std::vector<int32_t> bk;          // [i][N][col][8 lanes (row, prime)]: NTT(BK) R mod q
    std::vector<uint32_t> ksk;        // [N][t][4][n+1] as exported
};

namespace {

// ACC[col] += sum over rows of dec_row (x) BK_i[row][col], the rows being the
// two gadget digits of the two polynomials of D = X^abar ACC - ACC.
void cmux(const cpupar& C, const int32_t* bk_i, int abar, uint32_t (&acc)[2][N]) {
    alignas(32) static thread_local __m256i dig[N];  // lane 2 row + prime
    alignas(32) static thread_local __m256i col[N];  // lanes 0..3: (col 0, prime 0), (0, 1), (1, 0), (1, 1)
    alignas(32) int32_t d8[8];
    for (int m = 0; m < N; ++m) {
        for (int j = 0; j < 2; ++j) {
            const int s = (m - abar) & (2 * N - 1);
            const uint32_t v = acc[j][s & (N - 1)];
            const uint32_t rot = (s & N) ? 0u - v : v;
            const uint32_t x = rot - acc[j][m] + DECOMP_OFFSET;
            for (int p = 0; p < 2; ++p) {
                const int32_t d = (int32_t)((x >> (22 - 10 * p)) & 1023u) - 512;
                d8[2 * (2 * j + p)] = d;
                d8[2 * (2 * j + p) + 1] = d;
            }
        }
        dig[m] = _mm256_load_si256(reinterpret_cast<const __m256i*>(d8));
    }
    C.v.forward(dig);
    const __m256i* bk = reinterpret_cast<const __m256i*>(bk_i);
    for (int m = 0; m < N; ++m) {
        __m128i s[2];
        for (int c = 0; c < 2; ++c) {
            const __m256i pr = C.v.mont(dig[m], _mm256_loadu_si256(bk + 2 * m + c));  // |.| < q per lane
            __m128i h = _mm_add_epi32(_mm256_castsi256_si128(pr), _mm256_extracti128_si256(pr, 1));
            s[c] = _mm_add_epi32(h, _mm_unpackhi_epi64(h, h));  // lanes 0, 1: sums of prime 0, 1
        }
        const __m128i both = _mm_unpacklo_epi64(s[0], s[1]);
        col[m] = _mm256_set_m128i(both, both);
    }
    C.v.inverse(col);
    const int64_t q0 = C.p[0].q, q1 = C.p[1].q;
    alignas(32) int32_t r8[8];
    for (int m = 0; m < N; ++m) {
        _mm256_store_si256(reinterpret_cast<__m256i*>(r8), col[m]);
        for (int c = 0; c < 2; ++c) {
            const int64_t v0 = r8[2 * c], v1 = r8[2 * c + 1];
            int64_t t = ((v1 - v0) % q1) * C.crt_qinv % q1;
            if (t > q1 / 2) t -= q1;
            if (t < -q1 / 2) t += q1;
            acc[c][m] += (uint32_t)(v0 + q0 * t);
        }
    }
}

void gate_consts(int op, uint32_t& kappa, int32_t& s1, int32_t& s2) {
    switch (op) {
    case 0: kappa = 0u - MU; s1 = 1; s2 = 1; break;            // AND
    case 1: kappa = MU; s1 = -1; s2 = -1; break;               // NAND
    case 2: kappa = MU; s1 = 1; s2 = 1; break;                 // OR
    case 3: kappa = 0u - MU; s1 = -1; s2 = -1; break;          // NOR
    case 4: kappa = 2u * MU; s1 = 2; s2 = 2; break;            // XOR
    case 5: kappa = 0u - 2u * MU; s1 = -2; s2 = -2; break;     // XNOR
    case 6: kappa = 0u - MU; s1 = -1; s2 = 1; break;           // ANDNY
    case 7: kappa = 0u - MU; s1 = 1; s2 = -1; break;           // ANDYN
    case 8: kappa = MU; s1 = -1; s2 = 1; break;                // ORNY
    default: kappa = MU; s1 = 1; s2 = -1; break;               // ORYN
    }
}

inline uint32_t modswitch(uint32_t x) { return (x + (1u << 20)) >> 21; }

// One bootstrapped gate: linear combination, blind rotation of the constant
// test vector, extraction of coefficient 0, key switching.
void bootstrap_gate(const cpupar& C, int op, const uint32_t* c1, const uint32_t* c2, uint32_t* out) {
    uint32_t kappa;
    int32_t s1, s2;
    gate_consts(op, kappa, s1, s2);
    uint32_t comb[NW];
    for (int w = 0; w < NW; ++w) comb[w] = (uint32_t)s1 * c1[w] + (uint32_t)s2 * c2[w];
    comb[NLWE] += kappa;
    static thread_local uint32_t acc[2][N];
    const int c = (2 * N - (int)modswitch(comb[NLWE])) & (2 * N - 1);
    for (int m = 0; m < N; ++m) {
        acc[0][m] = 0;
        const int j = (m - c) & (2 * N - 1);  // coefficient m of X^c mu (1 + ... + X^(N-1))
        acc[1][m] = j < N ? MU : 0u - MU;
    }
    for (int i = 0; i < NLWE; ++i)
        cmux(C, C.bk.data() + (size_t)i * N * 2 * 8, (int)modswitch(comb[i]), acc);
    // extraction of coefficient 0, then key switching N -> n
    uint32_t big[N];
    big[0] = acc[0][0];
    for (int m = 1; m < N; ++m) big[m] = 0u - acc[0][N - m];
    for (int w = 0; w < NLWE; ++w) out[w] = 0;
    out[NLWE] = acc[1][0];
    for (int i = 0; i < N; ++i) {
        const uint32_t x = big[i] + (1u << 15);
        for (int j = 0; j < KS_T; ++j) {
            const uint32_t d = (x >> (30 - 2 * j)) & 3u;
            if (!d) continue;
            const uint32_t* row = C.ksk.data() + (((size_t)i * KS_T + j) * 4 + d) * NW;
            for (int w = 0; w < NW; ++w) out[w] -= row[w];
        }
    }
}

int resolve_threads(int threads) { return threads > 0 ? threads : omp_get_max_threads(); }

// Ripple-carry adder of eqs. (1)-(2) on ciphertext pointers, sum mod 2^w
// (carry out dropped), the same gates as the GPU library's and the oracle's.
void add_bits(const cpupar& C, const uint32_t* const* a, const uint32_t* const* b, uint32_t* const* r, int w) {
    std::vector<uint32_t> t(NW), g(NW), h(NW), carry(NW), nc(NW);
    bootstrap_gate(C, 4, a[0], b[0], r[0]);
    if (w == 1) return;
    bootstrap_gate(C, 0, a[0], b[0], carry.data());
    for (int i = 1; i < w; ++i) {
        bootstrap_gate(C, 4, a[i], b[i], t.data());
        if (i == w - 1) {
            bootstrap_gate(C, 4, t.data(), carry.data(), r[i]);
            break;
        }
        bootstrap_gate(C, 0, a[i], b[i], g.data());
        bootstrap_gate(C, 4, t.data(), carry.data(), r[i]);
        bootstrap_gate(C, 0, t.data(), carry.data(), h.data());
        bootstrap_gate(C, 2, g.data(), h.data(), nc.data());
        carry.swap(nc);
    }
}

}  // namespace

extern "C" {

int cpupar_create(const uint32_t* bk, const uint32_t* ksk, cpupar** out) {
    if (!bk || !ksk || !out) return -1;
    cpupar* C = new (std::nothrow) cpupar();
    if (!C) return -2;
    C->p[0].init(268369921);
    C->p[1].init(268367873);
    C->crt_qinv = (int32_t)powmod(C->p[0].q, C->p[1].q - 2, C->p[1].q);
    C->v.init(C->p);
    C->bk.assign((size_t)NLWE * N * 2 * 8, 0);
    // BK polynomials [i][row][col][N] (words read as signed) -> NTT domain x R,
    // laid out [i][m][col][row][prime] to meet the digit lanes
#pragma omp parallel for schedule(dynamic)
    for (int poly = 0; poly < NLWE * 8; ++poly) {
        const int i = poly / 8, row = (poly / 2) % 4, cl = poly % 2;
        std::vector<int32_t> x(N);
        for (int pr = 0; pr < 2; ++pr) {
            const Prime& P = C->p[pr];
            for (int m = 0; m < N; ++m) x[m] = Prime::centre((int32_t)bk[(size_t)poly * N + m], P.q);
            P.forward(x.data());
            for (int m = 0; m < N; ++m)
                C->bk[(((size_t)i * N + m) * 2 + cl) * 8 + 2 * row + pr] =
                    Prime::centre((int64_t)x[m] * ((int64_t)1 << 32), P.q);
        }
    }
    C->ksk.assign(ksk, ksk + (size_t)N * KS_T * 4 * NW);
    *out = C;
    return 0;
}

void cpupar_destroy(cpupar* C) { delete C; }

// count independent gates over `threads` threads (0: all), one gate each.
int cpupar_bootstrap_gates(const cpupar* C, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                           uint32_t* out, size_t count, int threads) {
    if (!C || (count && (!ops || !in0 || !in1 || !out))) return -1;
    for (size_t g = 0; g < count; ++g)
        if (ops[g] > 9) return -1;
#pragma omp parallel for schedule(dynamic) num_threads(resolve_threads(threads))
    for (long g = 0; g < (long)count; ++g)
        bootstrap_gate(*C, ops[g], in0 + g * NW, in1 + g * NW, out + g * NW);
    return 0;
}

// R = (A + B) mod 2^width for count numbers [count][width][n+1]: numbers
// across threads, each number's bits in carry order (Sec. IV-A).
int cpupar_add(const cpupar* C, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count, uint32_t width,
               int threads) {
    if (!C || width < 1 || width > 64 || (count && (!A || !B || !R))) return -1;
#pragma omp parallel for schedule(dynamic) num_threads(resolve_threads(threads))
    for (long k = 0; k < (long)count; ++k) {
        std::vector<const uint32_t*> a(width), b(width);
        std::vector<uint32_t*> r(width);
        for (uint32_t i = 0; i < width; ++i) {
            a[i] = A + ((size_t)k * width + i) * NW;
            b[i] = B + ((size_t)k * width + i) * NW;
            r[i] = R + ((size_t)k * width + i) * NW;
        }
        add_bits(*C, a.data(), b.data(), r.data(), (int)width);
    }
    return 0;
}

// R = (A * B) mod 2^width, shift-and-add keeping the low width bits, for
// count products: the AND gates of every partial product run across the
// threads, then each product's accumulation runs in order (Sec. IV-B), the
// products of a vector side by side.
int cpupar_mul(const cpupar* C, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count, uint32_t width,
               int threads) {
    if (!C || width < 1 || width > 64 || (count && (!A || !B || !R))) return -1;
    const int T = resolve_threads(threads);
    const size_t w = width, npp = w * (w + 1) / 2;  // ANDs a_j & b_i with i + j < w
    std::vector<uint32_t> pp(count * npp * NW);
    auto pp_at = [&](size_t k, size_t i, size_t j) {  // partial product i, bit j (j < w - i)
        const size_t idx = i * w - i * (i - 1) / 2 + j;
        return pp.data() + (k * npp + idx) * NW;
    };
#pragma omp parallel for schedule(dynamic) num_threads(T)
    for (long e = 0; e < (long)(count * w * w); ++e) {
        const size_t k = e / (w * w), i = (e / w) % w, j = e % w;
        if (i + j >= w) continue;
        bootstrap_gate(*C, 0, A + (k * w + j) * NW, B + (k * w + i) * NW, pp_at(k, i, j));
    }
#pragma omp parallel for schedule(dynamic) num_threads(T)
    for (long k = 0; k < (long)count; ++k) {
        std::vector<uint32_t> acc(w * NW), sum(w * NW);
        for (size_t j = 0; j < w; ++j) std::memcpy(acc.data() + j * NW, pp_at(k, 0, j), NW * 4);
        for (size_t i = 1; i < w; ++i) {
            const size_t len = w - i;
            std::vector<const uint32_t*> a(len), b(len);
            std::vector<uint32_t*> r(len);
            for (size_t j = 0; j < len; ++j) {
                a[j] = acc.data() + (i + j) * NW;
                b[j] = pp_at(k, i, j);
                r[j] = sum.data() + (i + j) * NW;
            }
            add_bits(*C, a.data(), b.data(), r.data(), (int)len);
            std::memcpy(acc.data() + i * NW, sum.data() + i * NW, len * NW * 4);
        }
        std::memcpy(R + k * w * NW, acc.data(), w * NW * 4);
    }
    return 0;
}

}  // extern "C"

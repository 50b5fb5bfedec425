/*
 * CPU oracle for TFHE gate bootstrapping — TEST INFRASTRUCTURE ONLY.
 * See tfhe_oracle.h for what each part follows.  Everything here is the plain
 * definition: schoolbook negacyclic products in wrapping uint32 arithmetic, no
 * transform, no blocking, no fusion.  Threads only run independent gates side
 * by side; they never change what a gate computes.
 */
#define _GNU_SOURCE
#include "tfhe_oracle.h"

#include <math.h>
#include <pthread.h>
#include <assert.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* Counter-based generator.                                                  */
/* The mixing function is the SplitMix64 output function (Steele, Lea, Flood, */
/* "Fast splittable pseudorandom number generators", OOPSLA 2014), with its   */
/* published constants.  draw(seed, stream, idx) feeds it a Weyl sequence:   */
/*   base = mix(seed + GAMMA*(stream+1)),  draw = mix(base + GAMMA*(idx+1)).  */
/* ------------------------------------------------------------------------ */
#define OR_GAMMA 0x9E3779B97F4A7C15ULL

uint64_t or_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t or_draw(uint64_t seed, uint64_t stream, uint64_t idx) {
    uint64_t base = or_mix64(seed + OR_GAMMA * (stream + 1));
    return or_mix64(base + OR_GAMMA * (idx + 1));
}

/* Box-Muller, cosine branch, one standard normal from draws 2*idx, 2*idx+1. */
double or_gaussian(uint64_t seed, uint64_t stream, uint64_t idx) {
    uint64_t x = or_draw(seed, stream, 2 * idx);
    uint64_t y = or_draw(seed, stream, 2 * idx + 1);
    double u1 = (double)((x >> 11) + 1) * 0x1.0p-53; /* (0, 1] */
    double u2 = (double)(y >> 11) * 0x1.0p-53;       /* [0, 1) */
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* A real number in (-1/2, 1/2) as a Torus32 word: round(x * 2^32), ties to even. */
uint32_t or_torus_from_double(double x) {
    return (uint32_t)(int64_t)nearbyint(x * 4294967296.0);
}

/* Streams of the generator (one per kind of random quantity). */
enum { ST_LWE_KEY = 1, ST_TLWE_KEY = 2, ST_BK_MASK = 3, ST_BK_NOISE = 4,
       ST_KSK_MASK = 5, ST_KSK_NOISE = 6, ST_ENC_MASK = 7, ST_ENC_NOISE = 8 };

static uint32_t top_word(uint64_t d) { return (uint32_t)(d >> 32); }
static int32_t top_bit(uint64_t d) { return (int32_t)(d >> 63); }

/* ------------------------------------------------------------------------ */
/* Parameters: TFHE's 110-bit gate-bootstrapping set (paper Sec. VII, "same   */
/* as the existing implementation of TFHE").                                  */
/* ------------------------------------------------------------------------ */
void or_default_params(or_params* P) {
    P->n = 500;
    P->N = 1024;
    P->bk_l = 2;
    P->bk_bgbit = 10;
    P->ks_t = 8;
    P->ks_basebit = 2;
    P->lwe_stdev = 2.44e-5;
    P->bk_stdev = 7.18e-9;
}

/* mu = 1/8 on the torus: a bit b is encrypted as +mu (b = 1) or -mu (b = 0). */
#define OR_MU 0x20000000u

static int log2i(int32_t v) {
    int r = 0;
    while ((1 << r) < v) r++;
    return r;
}

/* ------------------------------------------------------------------------ */
/* Ring Z/2^32[X]/(X^N + 1).                                                   */
/* ------------------------------------------------------------------------ */

/* Schoolbook negacyclic product:
 *   (P*Q)_m = sum_{j+k=m} P_j Q_k  -  sum_{j+k=m+N} P_j Q_k   (mod 2^32),
 * because X^N = -1.  Wrapping uint32 multiply-add is exact mod 2^32. */
void or_negacyclic_mul(int32_t N, const uint32_t* P, const uint32_t* Q, uint32_t* out) {
    uint32_t* acc = (uint32_t*)calloc((size_t)N, sizeof(uint32_t));
    for (int32_t j = 0; j < N; j++) {
        uint32_t pj = P[j];
        for (int32_t k = 0; k < N - j; k++) acc[j + k] += pj * Q[k];
        for (int32_t k = N - j; k < N; k++) acc[j + k - N] -= pj * Q[k];
    }
    memcpy(out, acc, (size_t)N * sizeof(uint32_t));
    free(acc);
}

/* out = X^a * P for a in [0, 2N): the coefficient at j moves to j + a, with a
 * sign flip each time it passes X^N. */
void or_rotate(int32_t N, const uint32_t* P, int32_t a, uint32_t* out) {
    int32_t twoN = 2 * N;
    a %= twoN;
    if (a < 0) a += twoN;
    for (int32_t j = 0; j < N; j++) {
        int32_t e = j + a;
        if (e >= twoN) e -= twoN;
        if (e < N) out[e] = P[j];
        else out[e - N] = (uint32_t)0 - P[j];
    }
}

/* ------------------------------------------------------------------------ */
/* Gadget decomposition (TFHE, signed balanced digits of Bgbit bits):        */
/*   x~ = x + sum_p (Bg/2) 2^(32-Bgbit(p+1)) + 2^(32-l*Bgbit-1)                */
/*   d_p = ((x~ >> (32 - Bgbit(p+1))) & (Bg-1)) - Bg/2,   p = 0..l-1          */
/* so that x ~= sum_p d_p 2^(32-Bgbit(p+1)) with |error| <= 2^(32-l*Bgbit-1). */
/* ------------------------------------------------------------------------ */
void or_gadget_decompose(const or_params* P, uint32_t x, int32_t* digits) {
    uint32_t Bg = 1u << P->bk_bgbit;
    uint32_t half = Bg / 2;
    uint32_t offset = 1u << (32 - P->bk_l * P->bk_bgbit - 1);
    for (int p = 0; p < P->bk_l; p++) offset += half << (32 - P->bk_bgbit * (p + 1));
    uint32_t xt = x + offset;
    for (int p = 0; p < P->bk_l; p++) {
        uint32_t field = (xt >> (32 - P->bk_bgbit * (p + 1))) & (Bg - 1);
        digits[p] = (int32_t)field - (int32_t)half;
    }
}

/* Modulus switch to Z_2N: round(x * 2N / 2^32) mod 2N, ties rounded up. */
uint32_t or_modswitch(const or_params* P, uint32_t x) {
    int s = 32 - log2i(2 * P->N);
    return (x + (1u << (s - 1))) >> s;
}

/* ------------------------------------------------------------------------ */
/* Gate linear combination: out = (0, kappa) + s1*c1 + s2*c2 over all n+1     */
/* words.  The constants put the true inputs' phase in (0, 1/2).             */
/* ------------------------------------------------------------------------ */
void or_gate_combine(const or_params* P, int op, const uint32_t* c1,
                     const uint32_t* c2, uint32_t* out) {
    const uint32_t mu = OR_MU;
    uint32_t kappa;
    int32_t s1, s2;
    switch (op) {
    case OR_AND:   kappa = 0u - mu;      s1 = 1;  s2 = 1;  break;
    case OR_NAND:  kappa = mu;           s1 = -1; s2 = -1; break;
    case OR_OR:    kappa = mu;           s1 = 1;  s2 = 1;  break;
    case OR_NOR:   kappa = 0u - mu;      s1 = -1; s2 = -1; break;
    case OR_XOR:   kappa = 2u * mu;      s1 = 2;  s2 = 2;  break;
    case OR_XNOR:  kappa = 0u - 2u * mu; s1 = -2; s2 = -2; break;
    case OR_ANDNY: kappa = 0u - mu;      s1 = -1; s2 = 1;  break;
    case OR_ANDYN: kappa = 0u - mu;      s1 = 1;  s2 = -1; break;
    case OR_ORNY:  kappa = mu;           s1 = -1; s2 = 1;  break;
    case OR_ORYN:  kappa = mu;           s1 = 1;  s2 = -1; break;
    default:       kappa = 0;            s1 = 0;  s2 = 0;  break;
    }
    for (int32_t i = 0; i <= P->n; i++)
        out[i] = (uint32_t)s1 * c1[i] + (uint32_t)s2 * c2[i];
    out[P->n] += kappa;
}

/* ------------------------------------------------------------------------ */
/* Keys.                                                                      */
/* ------------------------------------------------------------------------ */
static size_t bk_words(const or_params* P) {
    return (size_t)P->n * (size_t)(2 * P->bk_l) * 2u * (size_t)P->N;
}
static size_t ksk_words(const or_params* P) {
    return (size_t)P->N * (size_t)P->ks_t * (size_t)(1u << P->ks_basebit) * (size_t)(P->n + 1);
}

int or_keygen(const or_params* P, uint64_t seed, const int32_t* lwe_key_in,
              const int32_t* tlwe_key_in, or_keys* K) {
    const int32_t n = P->n, N = P->N, L2 = 2 * P->bk_l, t = P->ks_t;
    const uint32_t B = 1u << P->ks_basebit;
    memset(K, 0, sizeof(*K));
    K->P = *P;
    K->seed = seed;
    K->lwe_key = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    K->tlwe_key = (int32_t*)malloc((size_t)N * sizeof(int32_t));
    K->bk = (uint32_t*)calloc(bk_words(P), sizeof(uint32_t));
    K->ksk = (uint32_t*)calloc(ksk_words(P), sizeof(uint32_t));
    if (!K->lwe_key || !K->tlwe_key || !K->bk || !K->ksk) { or_keys_free(K); return -2; }

    /* Binary keys: the top bit of each draw. */
    for (int32_t i = 0; i < n; i++)
        K->lwe_key[i] = lwe_key_in ? lwe_key_in[i] : top_bit(or_draw(seed, ST_LWE_KEY, (uint64_t)i));
    for (int32_t j = 0; j < N; j++)
        K->tlwe_key[j] = tlwe_key_in ? tlwe_key_in[j] : top_bit(or_draw(seed, ST_TLWE_KEY, (uint64_t)j));

    /* Bootstrapping key: BK_i = TGSW(s_i).  Row r = 2j + p is a TLWE sample of
     * zero (A_r uniform, B_r = A_r*S + E_r) plus s_i * 2^(32-Bgbit(p+1)) added to
     * coefficient 0 of column j. */
    uint32_t* S = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    uint32_t* AS = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    for (int32_t j = 0; j < N; j++) S[j] = (uint32_t)K->tlwe_key[j];
    for (int32_t i = 0; i < n; i++) {
        for (int32_t r = 0; r < L2; r++) {
            uint32_t* rowA = K->bk + (((size_t)i * L2 + r) * 2 + 0) * N;
            uint32_t* rowB = K->bk + (((size_t)i * L2 + r) * 2 + 1) * N;
            uint64_t base = ((uint64_t)i * L2 + (uint64_t)r) * (uint64_t)N;
            for (int32_t c = 0; c < N; c++) rowA[c] = top_word(or_draw(seed, ST_BK_MASK, base + c));
            or_negacyclic_mul(N, rowA, S, AS);
            for (int32_t c = 0; c < N; c++)
                rowB[c] = AS[c] + or_torus_from_double(P->bk_stdev * or_gaussian(seed, ST_BK_NOISE, base + c));
            int32_t j = r / P->bk_l, p = r % P->bk_l;
            uint32_t h = 1u << (32 - P->bk_bgbit * (p + 1));
            uint32_t* col = (j == 0) ? rowA : rowB;
            col[0] += (uint32_t)K->lwe_key[i] * h;
        }
    }
    free(S);
    free(AS);

    /* Key-switching key: KSK[i][jj][v] = LWE_s(v * s'_i * 2^(32-basebit(jj+1)))
     * for v = 1..B-1, with s' the extracted key (the TLWE key coefficients);
     * KSK[i][jj][0] is the all-zero sample. */
    for (int32_t i = 0; i < N; i++) {
        for (int32_t jj = 0; jj < t; jj++) {
            for (uint32_t v = 1; v < B; v++) {
                uint32_t* row = K->ksk + (((size_t)i * t + jj) * B + v) * (size_t)(n + 1);
                uint64_t sample = ((uint64_t)i * t + (uint64_t)jj) * (B - 1) + (v - 1);
                uint32_t body = 0;
                for (int32_t l = 0; l < n; l++) {
                    row[l] = top_word(or_draw(seed, ST_KSK_MASK, sample * (uint64_t)n + l));
                    body += row[l] * (uint32_t)K->lwe_key[l];
                }
                uint32_t msg = v * (uint32_t)K->tlwe_key[i] * (1u << (32 - P->ks_basebit * (jj + 1)));
                body += or_torus_from_double(P->lwe_stdev * or_gaussian(seed, ST_KSK_NOISE, sample));
                row[n] = body + msg;
            }
        }
    }
    return 0;
}

void or_keys_free(or_keys* K) {
    free(K->lwe_key);
    free(K->tlwe_key);
    free(K->bk);
    free(K->ksk);
    K->lwe_key = NULL;
    K->tlwe_key = NULL;
    K->bk = NULL;
    K->ksk = NULL;
}

/* ------------------------------------------------------------------------ */
/* LWE encryption / phase / decryption (paper Sec. II-A: B = A.S + e).       */
/* Ciphertext q = nonce + c of a call draws its mask from stream 7 at        */
/* q*n + l and its noise from stream 8 at q.                                 */
/* ------------------------------------------------------------------------ */
void or_encrypt_bits(const or_keys* K, const uint8_t* bits, size_t count,
                     uint64_t nonce, uint32_t* ct) {
    const int32_t n = K->P.n;
    for (size_t c = 0; c < count; c++) {
        uint64_t q = nonce + (uint64_t)c;
        uint32_t* s = ct + c * (size_t)(n + 1);
        uint32_t body = 0;
        for (int32_t l = 0; l < n; l++) {
            s[l] = top_word(or_draw(K->seed, ST_ENC_MASK, q * (uint64_t)n + l));
            body += s[l] * (uint32_t)K->lwe_key[l];
        }
        body += or_torus_from_double(K->P.lwe_stdev * or_gaussian(K->seed, ST_ENC_NOISE, q));
        body += bits[c] ? OR_MU : (0u - OR_MU);
        s[n] = body;
    }
}

void or_phase(const or_keys* K, const uint32_t* ct, size_t count, int32_t* phase) {
    const int32_t n = K->P.n;
    for (size_t c = 0; c < count; c++) {
        const uint32_t* s = ct + c * (size_t)(n + 1);
        uint32_t dot = 0;
        for (int32_t l = 0; l < n; l++) dot += s[l] * (uint32_t)K->lwe_key[l];
        phase[c] = (int32_t)(s[n] - dot);
    }
}

void or_decrypt_bits(const or_keys* K, const uint32_t* ct, size_t count, uint8_t* bits) {
    int32_t* ph = (int32_t*)malloc(count * sizeof(int32_t) + 1);
    or_phase(K, ct, count, ph);
    for (size_t c = 0; c < count; c++) bits[c] = ph[c] > 0 ? 1 : 0;
    free(ph);
}

/* ------------------------------------------------------------------------ */
/* Bootstrapping.                                                             */
/* ------------------------------------------------------------------------ */

/* One CMux step of the blind rotation on accumulator acc = [a(X) | b(X)]:
 *   D = X^abar * acc - acc,
 *   acc[c] += sum_{j, p} digit_p(D_j) * BK_i[2j+p][c]   for c = 0, 1.
 * bk_i points at BK_i laid out [2l][2][N]. */
void or_external_product_cmux(const or_params* P, const uint32_t* bk_i,
                              int32_t abar, uint32_t* acc) {
    const int32_t N = P->N, l = P->bk_l;
    uint32_t* rot = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    uint32_t* D = (uint32_t*)malloc(2u * (size_t)N * sizeof(uint32_t));
    uint32_t* dig = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    uint32_t* prod = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    uint32_t* sum = (uint32_t*)calloc(2u * (size_t)N, sizeof(uint32_t));
    int32_t digits[32];
    for (int32_t j = 0; j < 2; j++) {
        or_rotate(N, acc + (size_t)j * N, abar, rot);
        for (int32_t m = 0; m < N; m++) D[(size_t)j * N + m] = rot[m] - acc[(size_t)j * N + m];
    }
    for (int32_t j = 0; j < 2; j++) {
        for (int32_t p = 0; p < l; p++) {
            for (int32_t m = 0; m < N; m++) {
                or_gadget_decompose(P, D[(size_t)j * N + m], digits);
                dig[m] = (uint32_t)digits[p];
            }
            int32_t r = 2 * j + p;
            for (int32_t c = 0; c < 2; c++) {
                or_negacyclic_mul(N, dig, bk_i + ((size_t)r * 2 + c) * N, prod);
                for (int32_t m = 0; m < N; m++) sum[(size_t)c * N + m] += prod[m];
            }
        }
    }
    for (int32_t m = 0; m < 2 * N; m++) acc[m] += sum[m];
    free(rot);
    free(D);
    free(dig);
    free(prod);
    free(sum);
}

/* Blind rotation of the test vector v = sum_j mu X^j:
 *   acc = (0, X^(2N - bbar) v);  for i < n: CMux with BK_i and abar_i.
 * lwe_in is the gate's combined sample (n+1 words). */
/* Blind rotation of test vector tv (N words): ACC = (0, X^(2N - bbar) tv),
 * then the n CMux steps.  Coefficient 0 of the result's body polynomial
 * encrypts tv[phibar] for a modulus-switched phase phibar < N and
 * -tv[phibar - N] above. */
void or_blind_rotate_tv(const or_keys* K, const uint32_t* lwe_in, const uint32_t* tv, uint32_t* acc) {
    const or_params* P = &K->P;
    const int32_t n = P->n, N = P->N, L2 = 2 * P->bk_l;
    int32_t bbar = (int32_t)or_modswitch(P, lwe_in[n]);
    memset(acc, 0, (size_t)N * sizeof(uint32_t));
    or_rotate(N, tv, 2 * N - bbar, acc + N);
    for (int32_t i = 0; i < n; i++) {
        int32_t abar = (int32_t)or_modswitch(P, lwe_in[i]);
        or_external_product_cmux(P, K->bk + (size_t)i * L2 * 2 * N, abar, acc);
    }
}

/* Gate bootstrapping's test vector: mu in every coefficient. */
void or_blind_rotate(const or_keys* K, const uint32_t* lwe_in, uint32_t* acc) {
    const int32_t N = K->P.N;
    uint32_t* v = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    for (int32_t j = 0; j < N; j++) v[j] = OR_MU;
    or_blind_rotate_tv(K, lwe_in, v, acc);
    free(v);
}

/* Sample extraction of coefficient 0: a'_0 = a_0, a'_m = -a_(N-m), b' = b_0. */
void or_sample_extract(const or_params* P, const uint32_t* acc, uint32_t* lwe_big) {
    const int32_t N = P->N;
    lwe_big[0] = acc[0];
    for (int32_t m = 1; m < N; m++) lwe_big[m] = (uint32_t)0 - acc[N - m];
    lwe_big[N] = acc[N];
}

/* Sample extraction of coefficient m of a TLWE sample (A, B): the LWE sample
 * under the coefficients of S whose phase is coefficient m of B - A S.  From
 * (A S)_m = sum_{j <= m} A_(m-j) S_j - sum_{j > m} A_(N+m-j) S_j:
 *   a'_j = A_(m-j) for j <= m,  a'_j = -A_(N+m-j) for j > m,  b' = B_m. */
void or_sample_extract_at(const or_params* P, const uint32_t* acc, int32_t m, uint32_t* lwe_big) {
    const int32_t N = P->N;
    const uint32_t* A = acc;
    const uint32_t* B = acc + N;
    for (int32_t j = 0; j < N; j++) lwe_big[j] = j <= m ? A[m - j] : (uint32_t)0 - A[N + m - j];
    lwe_big[N] = B[m];
}

/* Key switching N -> n with unsigned base-2^basebit digits of a'_i rounded to
 * t*basebit bits:  out = (0, b') - sum_{i, jj} KSK[i][jj][d_{i,jj}]. */
void or_key_switch(const or_keys* K, const uint32_t* lwe_big, uint32_t* out) {
    const or_params* P = &K->P;
    const int32_t n = P->n, N = P->N, t = P->ks_t, bb = P->ks_basebit;
    const uint32_t B = 1u << bb;
    const uint32_t round_off = 1u << (32 - t * bb - 1);
    for (int32_t l = 0; l < n; l++) out[l] = 0;
    out[n] = lwe_big[N];
    for (int32_t i = 0; i < N; i++) {
        uint32_t xt = lwe_big[i] + round_off;
        for (int32_t jj = 0; jj < t; jj++) {
            uint32_t d = (xt >> (32 - bb * (jj + 1))) & (B - 1);
            const uint32_t* row = K->ksk + (((size_t)i * t + jj) * B + d) * (size_t)(n + 1);
            for (int32_t l = 0; l <= n; l++) out[l] -= row[l];
        }
    }
}

/* Three-input gates (encoding +-mu, mu = 1/8): c1 + c2 + c3 has phase
 * -3/8, -1/8, 1/8 or 3/8 for 0, 1, 2 or 3 true inputs, positive iff most are
 * true (MAJ); -2 (c1 + c2 + c3) has phase 3/4 = -1/4, 1/4, -1/4 or -3/4 =
 * 1/4, positive iff an odd number is true (XOR3).  No constant is added. */
void or_gate_combine3(const or_params* P, int op, const uint32_t* c1, const uint32_t* c2,
                      const uint32_t* c3, uint32_t* out) {
    if (op != OR_MAJ && op != OR_XOR3) {
        or_gate_combine(P, op, c1, c2, out);
        return;
    }
    const uint32_t s = op == OR_MAJ ? 1u : 0u - 2u;
    for (int32_t i = 0; i <= P->n; i++) out[i] = s * (c1[i] + c2[i] + c3[i]);
}

void or_bootstrap_gate3(const or_keys* K, int op, const uint32_t* c1, const uint32_t* c2,
                        const uint32_t* c3, uint32_t* out) {
    const or_params* P = &K->P;
    uint32_t* comb = (uint32_t*)malloc((size_t)(P->n + 1) * sizeof(uint32_t));
    uint32_t* acc = (uint32_t*)malloc(2u * (size_t)P->N * sizeof(uint32_t));
    uint32_t* big = (uint32_t*)malloc((size_t)(P->N + 1) * sizeof(uint32_t));
    or_gate_combine3(P, op, c1, c2, c3, comb);
    or_blind_rotate(K, comb, acc);
    or_sample_extract(P, acc, big);
    or_key_switch(K, big, out);
    free(comb);
    free(acc);
    free(big);
}

/* Programmable bootstrapping: no gate combination, the input's own phase
 * selects the test-vector entry; blind rotation of tv, sample extraction, key
 * switching.  count samples [count][n+1], independent, on `threads`. */
typedef struct {
    const or_keys* K;
    const uint32_t* tv;
    const uint32_t* in;
    uint32_t* out;
    size_t count, next;
    pthread_mutex_t lock;
} lut_job;

static void* lut_worker(void* arg) {
    lut_job* J = (lut_job*)arg;
    const or_params* P = &J->K->P;
    const size_t W = (size_t)P->n + 1;
    uint32_t* acc = (uint32_t*)malloc(2u * (size_t)P->N * sizeof(uint32_t));
    uint32_t* big = (uint32_t*)malloc((size_t)(P->N + 1) * sizeof(uint32_t));
    for (;;) {
        pthread_mutex_lock(&J->lock);
        size_t g = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (g >= J->count) break;
        or_blind_rotate_tv(J->K, J->in + g * W, J->tv, acc);
        or_sample_extract(P, acc, big);
        or_key_switch(J->K, big, J->out + g * W);
    }
    free(acc);
    free(big);
    return NULL;
}

static int resolve_threads(int threads);

void or_bootstrap_lut(const or_keys* K, const uint32_t* tv, const uint32_t* in, uint32_t* out, size_t count,
                      int threads) {
    if (count == 0) return;
    lut_job J;
    J.K = K;
    J.tv = tv;
    J.in = in;
    J.out = out;
    J.count = count;
    J.next = 0;
    pthread_mutex_init(&J.lock, NULL);
    int T = resolve_threads(threads);
    if ((size_t)T > count) T = (int)count;
    pthread_t* tid = (pthread_t*)malloc((size_t)T * sizeof(pthread_t));
    for (int i = 0; i < T; i++) pthread_create(&tid[i], NULL, lut_worker, &J);
    for (int i = 0; i < T; i++) pthread_join(tid[i], NULL);
    free(tid);
    pthread_mutex_destroy(&J.lock);
}

void or_bootstrap_gate(const or_keys* K, int op, const uint32_t* c1,
                       const uint32_t* c2, uint32_t* out) {
    const or_params* P = &K->P;
    uint32_t* comb = (uint32_t*)malloc((size_t)(P->n + 1) * sizeof(uint32_t));
    uint32_t* acc = (uint32_t*)malloc(2u * (size_t)P->N * sizeof(uint32_t));
    uint32_t* big = (uint32_t*)malloc((size_t)(P->N + 1) * sizeof(uint32_t));
    or_gate_combine(P, op, c1, c2, comb);
    or_blind_rotate(K, comb, acc);
    or_sample_extract(P, acc, big);
    or_key_switch(K, big, out);
    free(comb);
    free(acc);
    free(big);
}

/* ------------------------------------------------------------------------ */
/* Compound gates (Sec. V-A-3): two gates on the same two inputs, here from  */
/* ONE blind rotation.                                                        */
/* ------------------------------------------------------------------------ */
/* Value (+1 true, -1 false) of a symmetric two-input gate with k of its two
 * inputs true; 0 for a code that is not symmetric. */
static int sym_truth(int op, int k) {
    switch (op) {
    case OR_AND: return k == 2 ? 1 : -1;
    case OR_NAND: return k == 2 ? -1 : 1;
    case OR_OR: return k >= 1 ? 1 : -1;
    case OR_NOR: return k >= 1 ? -1 : 1;
    case OR_XOR: return k == 1 ? 1 : -1;
    case OR_XNOR: return k == 1 ? -1 : 1;
    default: return 0;
    }
}

/* The compound gate rotates the constant test vector 1/16 by the phase of
 * c1 + c2, which is -1/4, 0 or +1/4 for k = 0, 1, 2 true inputs (encoding
 * +-1/8).  Coefficient m of the rotated accumulator encrypts U(phibar + m),
 * U = +1/16 on [0, N) and -1/16 on [N, 2N) (negacyclic); the extractions at
 * m = 3N/4 and m = N/4 (E1, E2) take the values
 *     k = 0 (phibar = -N/2):  E1 = +1/16, E2 = -1/16
 *     k = 1 (phibar = 0):     E1 = +1/16, E2 = +1/16
 *     k = 2 (phibar = +N/2):  E1 = -1/16, E2 = +1/16
 * and switch sign exactly half-way between those phases, like the two-input
 * gates.  A symmetric gate with values g0, g1, g2 (units of 1/8) is then the
 * sample (g1 - g2) E1 + (g1 - g0) E2 + (0, (g0 + g2) / 16): at each k it
 * evaluates to g_k / 8.  This writes that N-dimensional sample (before key
 * switching) into big; returns -1 for a code that is not symmetric. */
int or_compound_combine(const or_params* P, int op, const uint32_t* acc, uint32_t* big) {
    const int32_t N = P->N;
    const int g0 = sym_truth(op, 0), g1 = sym_truth(op, 1), g2 = sym_truth(op, 2);
    if (!g0) return -1;
    uint32_t* e1 = (uint32_t*)malloc((size_t)(N + 1) * sizeof(uint32_t));
    uint32_t* e2 = (uint32_t*)malloc((size_t)(N + 1) * sizeof(uint32_t));
    or_sample_extract_at(P, acc, 3 * N / 4, e1);
    or_sample_extract_at(P, acc, N / 4, e2);
    const uint32_t x = (uint32_t)(g1 - g2), y = (uint32_t)(g1 - g0);
    for (int32_t j = 0; j <= N; j++) big[j] = x * e1[j] + y * e2[j];
    big[N] += (uint32_t)(g0 + g2) * (1u << 28);
    free(e1);
    free(e2);
    return 0;
}

/* out0 = op0(c1, c2), out1 = op1(c1, c2) for symmetric codes op0, op1 (AND,
 * NAND, OR, NOR, XOR, XNOR): one blind rotation of the constant test vector
 * 1/16 by c1 + c2, two combinations of its extracted coefficients, two key
 * switchings.  Returns -1 (and writes nothing) for other codes. */
int or_bootstrap_compound(const or_keys* K, int op0, int op1, const uint32_t* c1, const uint32_t* c2,
                          uint32_t* out0, uint32_t* out1) {
    const or_params* P = &K->P;
    if (!sym_truth(op0, 0) || !sym_truth(op1, 0)) return -1;
    uint32_t* comb = (uint32_t*)malloc((size_t)(P->n + 1) * sizeof(uint32_t));
    uint32_t* tv = (uint32_t*)malloc((size_t)P->N * sizeof(uint32_t));
    uint32_t* acc = (uint32_t*)malloc(2u * (size_t)P->N * sizeof(uint32_t));
    uint32_t* big = (uint32_t*)malloc((size_t)(P->N + 1) * sizeof(uint32_t));
    for (int32_t i = 0; i <= P->n; i++) comb[i] = c1[i] + c2[i];
    for (int32_t j = 0; j < P->N; j++) tv[j] = 1u << 28;
    or_blind_rotate_tv(K, comb, tv, acc);
    or_compound_combine(P, op0, acc, big);
    or_key_switch(K, big, out0);
    or_compound_combine(P, op1, acc, big);
    or_key_switch(K, big, out1);
    free(comb);
    free(tv);
    free(acc);
    free(big);
    return 0;
}

typedef struct {
    const or_keys* K;
    const uint8_t* ops;
    const uint32_t* in0;
    const uint32_t* in1;
    uint32_t* out;
    size_t count, next;
    int bad;
    pthread_mutex_t lock;
} compound_job;

static void* compound_worker(void* arg) {
    compound_job* J = (compound_job*)arg;
    const size_t W = (size_t)J->K->P.n + 1;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        size_t g = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (g >= J->count) break;
        if (or_bootstrap_compound(J->K, J->ops[2 * g], J->ops[2 * g + 1], J->in0 + g * W, J->in1 + g * W,
                                  J->out + 2 * g * W, J->out + (2 * g + 1) * W)) {
            pthread_mutex_lock(&J->lock);
            J->bad = 1;
            pthread_mutex_unlock(&J->lock);
        }
    }
    return NULL;
}

static int resolve_threads(int threads);

int or_bootstrap_compounds(const or_keys* K, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                           uint32_t* out, size_t count, int threads) {
    if (count == 0) return 0;
    compound_job J;
    J.K = K;
    J.ops = ops;
    J.in0 = in0;
    J.in1 = in1;
    J.out = out;
    J.count = count;
    J.next = 0;
    J.bad = 0;
    pthread_mutex_init(&J.lock, NULL);
    int T = resolve_threads(threads);
    if ((size_t)T > count) T = (int)count;
    pthread_t* tid = (pthread_t*)malloc((size_t)T * sizeof(pthread_t));
    for (int i = 0; i < T; i++) pthread_create(&tid[i], NULL, compound_worker, &J);
    for (int i = 0; i < T; i++) pthread_join(tid[i], NULL);
    free(tid);
    pthread_mutex_destroy(&J.lock);
    return J.bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Running independent gates on several threads.                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_keys* K;
    const uint8_t* ops;
    const uint32_t* const* in0;
    const uint32_t* const* in1;
    const uint32_t* const* in2; /* NULL: two-input gates only */
    uint32_t* const* out;
    const int* ops2;            /* NULL, or per gate: >= 0 for a compound node */
    uint32_t* const* out2;      /* its second output */
    size_t count;
    size_t next;
    pthread_mutex_t lock;
} gate_job;

static void* gate_worker(void* arg) {
    gate_job* J = (gate_job*)arg;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        size_t g = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (g >= J->count) break;
        if (J->ops2 && J->ops2[g] >= 0)
            or_bootstrap_compound(J->K, J->ops[g], J->ops2[g], J->in0[g], J->in1[g], J->out[g], J->out2[g]);
        else if (J->in2)
            or_bootstrap_gate3(J->K, J->ops[g], J->in0[g], J->in1[g], J->in2[g], J->out[g]);
        else
            or_bootstrap_gate(J->K, J->ops[g], J->in0[g], J->in1[g], J->out[g]);
    }
    return NULL;
}

/* threads <= 0: one per online processor, at most 16. */
static int resolve_threads(int threads) {
    if (threads > 0) return threads;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 16 ? 16 : c > 0 ? (int)c : 1;
}

/* Runs gate g on (in0[g], in1[g]) -> out[g] for g < count, pointer form;
 * compound nodes (ops2[g] >= 0) also write out2[g]. */
static void run_gates_c(const or_keys* K, const uint8_t* ops, const uint32_t* const* in0,
                        const uint32_t* const* in1, const uint32_t* const* in2, uint32_t* const* out,
                        const int* ops2, uint32_t* const* out2, size_t count, int threads) {
    if (count == 0) return;
    gate_job J;
    J.K = K;
    J.ops = ops;
    J.in0 = in0;
    J.in1 = in1;
    J.in2 = in2;
    J.out = out;
    J.ops2 = ops2;
    J.out2 = out2;
    J.count = count;
    J.next = 0;
    pthread_mutex_init(&J.lock, NULL);
    int T = resolve_threads(threads);
    if ((size_t)T > count) T = (int)count;
    pthread_t* tid = (pthread_t*)malloc((size_t)T * sizeof(pthread_t));
    for (int i = 0; i < T; i++) pthread_create(&tid[i], NULL, gate_worker, &J);
    for (int i = 0; i < T; i++) pthread_join(tid[i], NULL);
    free(tid);
    pthread_mutex_destroy(&J.lock);
}

static void run_gates(const or_keys* K, const uint8_t* ops, const uint32_t* const* in0,
                      const uint32_t* const* in1, const uint32_t* const* in2, uint32_t* const* out,
                      size_t count, int threads) {
    run_gates_c(K, ops, in0, in1, in2, out, NULL, NULL, count, threads);
}

void or_bootstrap_gates(const or_keys* K, const uint8_t* ops, const uint32_t* in0,
                        const uint32_t* in1, uint32_t* out, size_t count, int threads) {
    const size_t W = (size_t)K->P.n + 1;
    const uint32_t** a = (const uint32_t**)malloc((count + 1) * sizeof(*a));
    const uint32_t** b = (const uint32_t**)malloc((count + 1) * sizeof(*b));
    uint32_t** o = (uint32_t**)malloc((count + 1) * sizeof(*o));
    for (size_t g = 0; g < count; g++) {
        a[g] = in0 + g * W;
        b[g] = in1 + g * W;
        o[g] = out + g * W;
    }
    run_gates(K, ops, a, b, NULL, o, count, threads);
    free(a);
    free(b);
    free(o);
}

void or_bootstrap_gates3(const or_keys* K, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                         const uint32_t* in2, uint32_t* out, size_t count, int threads) {
    const size_t W = (size_t)K->P.n + 1;
    const uint32_t** a = (const uint32_t**)malloc((count + 1) * sizeof(*a));
    const uint32_t** b = (const uint32_t**)malloc((count + 1) * sizeof(*b));
    const uint32_t** c = (const uint32_t**)malloc((count + 1) * sizeof(*c));
    uint32_t** o = (uint32_t**)malloc((count + 1) * sizeof(*o));
    for (size_t g = 0; g < count; g++) {
        a[g] = in0 + g * W;
        b[g] = in1 + g * W;
        c[g] = in2 + g * W;
        o[g] = out + g * W;
    }
    run_gates(K, ops, a, b, c, o, count, threads);
    free(a);
    free(b);
    free(c);
    free(o);
}

/* ------------------------------------------------------------------------ */
/* Circuits as gate lists over wires (each wire holds one LWE sample).        */
/* ------------------------------------------------------------------------ */
/* in2 < 0: two inputs.  op2 >= 0: a compound node writing op(in0, in1) to
 * out and op2(in0, in1) to out2 from one rotation (or_bootstrap_compound). */
typedef struct { int op, in0, in1, in2, out, op2, out2; } or_gate_t;
typedef struct { or_gate_t* g; long ng, cap; long nwires; } or_prog;

static long new_wire(or_prog* pr) { return pr->nwires++; }

static long emit3(or_prog* pr, int op, long a, long b, long c) {
    if (pr->ng == pr->cap) {
        pr->cap = pr->cap ? 2 * pr->cap : 256;
        pr->g = (or_gate_t*)realloc(pr->g, (size_t)pr->cap * sizeof(or_gate_t));
    }
    long o = new_wire(pr);
    or_gate_t* G = &pr->g[pr->ng++];
    G->op = op;
    G->in0 = (int)a;
    G->in1 = (int)b;
    G->in2 = (int)c;
    G->out = (int)o;
    G->op2 = -1;
    G->out2 = -1;
    return o;
}

static long emit(or_prog* pr, int op, long a, long b) { return emit3(pr, op, a, b, -1); }

/* Compound node: *o0 = op0(a, b), *o1 = op1(a, b). */
static void emit_compound(or_prog* pr, int op0, int op1, long a, long b, long* o0, long* o1) {
    *o0 = emit(pr, op0, a, b);
    or_gate_t* G = &pr->g[pr->ng - 1];
    G->op2 = op1;
    G->out2 = (int)new_wire(pr);
    *o1 = G->out2;
}

/* Ripple-carry adder of eqs. (1)-(2) with compound gates (Sec. V-A-3): the
 * XOR and the AND of the same two bits come from one compound node.
 *   bit 0:     (r, c) = (a ^ b, a & b)
 *   bit i:     (t, g) = (a ^ b, a & b), (r, h) = (t ^ c, t & c), c = g | h
 *   bit w-1:   t = a ^ b, r = t ^ c                                         */
static void build_add_compound(or_prog* pr, const long* a, const long* b, int w, long* r) {
    if (w <= 0) return;
    if (w == 1) { r[0] = emit(pr, OR_XOR, a[0], b[0]); return; }
    long c;
    emit_compound(pr, OR_XOR, OR_AND, a[0], b[0], &r[0], &c);
    for (int i = 1; i < w; i++) {
        if (i == w - 1) {
            long t = emit(pr, OR_XOR, a[i], b[i]);
            r[i] = emit(pr, OR_XOR, t, c);
            break;
        }
        long t, g, h;
        emit_compound(pr, OR_XOR, OR_AND, a[i], b[i], &t, &g);
        emit_compound(pr, OR_XOR, OR_AND, t, c, &r[i], &h);
        c = emit(pr, OR_OR, g, h);
    }
}

/* Ripple-carry adder of eqs. (1)-(2), sum modulo 2^w (carry out dropped):
 *   bit 0:     r = a ^ b,            c = a & b
 *   bit i:     t = a ^ b, g = a & b, r = t ^ c, h = t & c, c = g | h
 *   bit w-1:   t = a ^ b,            r = t ^ c                              */
static void build_add(or_prog* pr, const long* a, const long* b, int w, long* r) {
    if (w <= 0) return;
    if (w == 1) { r[0] = emit(pr, OR_XOR, a[0], b[0]); return; }
    r[0] = emit(pr, OR_XOR, a[0], b[0]);
    long c = emit(pr, OR_AND, a[0], b[0]);
    for (int i = 1; i < w; i++) {
        long t = emit(pr, OR_XOR, a[i], b[i]);
        if (i == w - 1) { r[i] = emit(pr, OR_XOR, t, c); break; }
        long g = emit(pr, OR_AND, a[i], b[i]);
        r[i] = emit(pr, OR_XOR, t, c);
        long h = emit(pr, OR_AND, t, c);
        c = emit(pr, OR_OR, g, h);
    }
}

/* Naive multiplication (Sec. III-B-1) keeping the low w bits:
 *   acc = A & b_0;  for i >= 1: acc[i..w-1] += (A & b_i)[0..w-1-i]. */
static void build_mul(or_prog* pr, const long* a, const long* b, int w, long* r) {
    long* acc = (long*)malloc((size_t)w * sizeof(long));
    long* pp = (long*)malloc((size_t)w * sizeof(long));
    long* sum = (long*)malloc((size_t)w * sizeof(long));
    for (int j = 0; j < w; j++) acc[j] = emit(pr, OR_AND, a[j], b[0]);
    for (int i = 1; i < w; i++) {
        int m = w - i;
        for (int j = 0; j < m; j++) pp[j] = emit(pr, OR_AND, a[j], b[i]);
        build_add(pr, acc + i, pp, m, sum);
        for (int j = 0; j < m; j++) acc[i + j] = sum[j];
    }
    memcpy(r, acc, (size_t)w * sizeof(long));
    free(acc);
    free(pp);
    free(sum);
}

/* Multiplication with tree accumulation (Sec. V-B-2, "Multiplication"; Fig. 4),
 * low w bits.  Partial product i is (A & b_i) shifted left by i: its bits
 * i..w-1 are the gates a_j & b_i for j = 0..w-1-i, its bits below i are zero
 * and carry no wire.  The list of the w partial products is split into its
 * first and second halves, which are added element-wise; an odd last element
 * waits a round; the rounds repeat until one number is left.  Adding a
 * number whose known-zero low bits end at l to one whose end at m > l copies
 * bits l..m-1 of the first and ripple-adds (eqs. (1)-(2), carry out dropped)
 * bits m..w-1 of both. */
static void build_mul_tree(or_prog* pr, const long* a, const long* b, int w, long* r) {
    long* bits = (long*)malloc((size_t)w * w * sizeof(long)); /* number k: bits[k*w + pos] */
    int* low = (int*)malloc((size_t)w * sizeof(int));         /* first wired bit of number k */
    long* sum = (long*)malloc((size_t)w * sizeof(long));
    for (int i = 0; i < w; i++) {
        low[i] = i;
        for (int j = 0; i + j < w; j++) bits[(size_t)i * w + i + j] = emit(pr, OR_AND, a[j], b[i]);
    }
    int len = w;
    while (len > 1) {
        int h = len / 2;
        for (int k = 0; k < h; k++) {
            long* x = bits + (size_t)k * w;
            long* y = bits + (size_t)(k + h) * w;
            int lx = low[k], ly = low[k + h];
            if (ly < lx) { /* keep x the one with fewer known-zero bits */
                long* t = x; x = y; y = t;
                int u = lx; lx = ly; ly = u;
            }
            build_add(pr, x + ly, y + ly, w - ly, sum);
            long* dst = bits + (size_t)k * w;
            for (int p = lx; p < ly; p++) dst[p] = x[p];
            for (int p = ly; p < w; p++) dst[p] = sum[p - ly];
            low[k] = lx;
        }
        if (len & 1) {
            memcpy(bits + (size_t)h * w, bits + (size_t)(len - 1) * w, (size_t)w * sizeof(long));
            low[h] = low[len - 1];
        }
        len = h + (len & 1);
    }
    memcpy(r, bits, (size_t)w * sizeof(long));
    free(bits);
    free(low);
    free(sum);
}

/* Ripple-carry adder of full-adder gates, sum mod 2^w: bit 0 r = a ^ b,
 * c = a & b; bit i: r = XOR3(a, b, c), c = MAJ(a, b, c) (eqs. (1)-(2) with
 * the sum and carry of each bit as one three-input gate each); the top bit
 * r = XOR3(a, b, c) only.  2w - 1 gates (w > 1) in w levels. */
static void build_add_fa(or_prog* pr, const long* a, const long* b, int w, long* r) {
    if (w <= 0) return;
    r[0] = emit(pr, OR_XOR, a[0], b[0]);
    if (w == 1) return;
    long c = emit(pr, OR_AND, a[0], b[0]);
    for (int i = 1; i < w; i++) {
        r[i] = emit3(pr, OR_XOR3, a[i], b[i], c);
        if (i + 1 < w) c = emit3(pr, OR_MAJ, a[i], b[i], c);
    }
}

/* Number-wise addition (GPU_n, Sec. V-B-1), sum mod 2^w: R = A; then w
 * rounds of carry = R & B, R = R ^ B, B = carry << 1 (the AND and XOR of a
 * round side by side).  After round k the low k+1 bits of B are zero and carry
 * no wire, so round k acts on bits k..w-1 only (its carry out of bit w-1 is
 * dropped): w^2 gates in w levels. */
static void build_add_numberwise(or_prog* pr, const long* a, const long* b, int w, long* r) {
    long* B = (long*)malloc((size_t)w * sizeof(long));
    long* carry = (long*)malloc((size_t)w * sizeof(long));
    memcpy(r, a, (size_t)w * sizeof(long));
    memcpy(B, b, (size_t)w * sizeof(long));
    for (int k = 0; k < w; k++) {
        for (int i = k; i + 1 < w; i++) carry[i] = emit(pr, OR_AND, r[i], B[i]);
        for (int i = k; i < w; i++) r[i] = emit(pr, OR_XOR, r[i], B[i]);
        for (int i = w - 1; i > k; i--) B[i] = carry[i - 1];
    }
    free(B);
    free(carry);
}

/* ---- Karatsuba multiplication (Sec. III-B-2, Algorithm 1; Sec. V-B-2) ----
 * Full products (2n bits of n-bit operands).  Numbers are wire arrays, LSB
 * first; a bit beyond an array's length is zero and carries no wire. */

/* r = x + y mod 2^L (r has L wires; lx, ly <= L).  Ripple carry: both bits
 * present and no carry in: r = x^y, c = x&y; with a carry in:
 * t = x^y, r = t^c, c = (x&y) | (t&c); one bit and a carry: r = v^c,
 * c = v&c; one bit alone: r = that wire; no bit: r = the carry (then no
 * higher bit exists).  Carries only where a higher bit needs them.
 * Returns the number of wires written (L, or fewer when the sum is shorter). */
static int build_add_n(or_prog* pr, const long* x, int lx, const long* y, int ly, int L, long* r) {
    long c = -1;
    int n = 0;
    for (int i = 0; i < L; i++) {
        const int hx = i < lx, hy = i < ly, more = i + 1 < L;
        long nc = -1;
        if (hx && hy) {
            if (c < 0) {
                r[n++] = emit(pr, OR_XOR, x[i], y[i]);
                if (more) nc = emit(pr, OR_AND, x[i], y[i]);
            } else {
                long t = emit(pr, OR_XOR, x[i], y[i]);
                r[n++] = emit(pr, OR_XOR, t, c);
                if (more) {
                    long g = emit(pr, OR_AND, x[i], y[i]);
                    long h = emit(pr, OR_AND, t, c);
                    nc = emit(pr, OR_OR, g, h);
                }
            }
        } else if (hx || hy) {
            long v = hx ? x[i] : y[i];
            if (c < 0) {
                r[n++] = v;
            } else {
                r[n++] = emit(pr, OR_XOR, v, c);
                if (more) nc = emit(pr, OR_AND, v, c);
            }
        } else {
            if (c < 0) break;
            r[n++] = c;
        }
        c = nc;
    }
    return n;
}

/* r = x - y mod 2^L (both L bits) as x + ~y + 1 with the +1 folded into
 * bit 0: r_0 = x^y, c = x | ~y (ORYN); bit i: t = x XNOR y, r = t^c,
 * c = (x & ~y) | (t & c) (ANDYN, AND, OR). */
static void build_sub_n(or_prog* pr, const long* x, const long* y, int L, long* r) {
    long c = -1;
    for (int i = 0; i < L; i++) {
        const int more = i + 1 < L;
        if (i == 0) {
            r[0] = emit(pr, OR_XOR, x[0], y[0]);
            if (more) c = emit(pr, OR_ORYN, x[0], y[0]);
            continue;
        }
        long t = emit(pr, OR_XNOR, x[i], y[i]);
        r[i] = emit(pr, OR_XOR, t, c);
        if (more) {
            long g = emit(pr, OR_ANDYN, x[i], y[i]);
            long h = emit(pr, OR_AND, t, c);
            c = emit(pr, OR_OR, g, h);
        }
    }
}

/* Full product of m-bit a and b (2m wires into r, m >= 2) with the partial
 * products (A & b_i) << i summed by the tree of Sec. V-B-2: first and second
 * halves of the list added element-wise, an odd last element waiting a
 * round; a sum keeps one bit more than its wider operand, up to 2m. */
static void build_mul_full_tree(or_prog* pr, const long* a, const long* b, int m, long* r) {
    const int W2 = 2 * m;
    long* bits = (long*)malloc((size_t)m * W2 * sizeof(long)); /* number k: wires of bits low[k].. */
    int* low = (int*)malloc((size_t)m * sizeof(int));
    int* len = (int*)malloc((size_t)m * sizeof(int));
    long* sum = (long*)malloc((size_t)W2 * sizeof(long));
    for (int i = 0; i < m; i++) {
        low[i] = i;
        len[i] = m;
        for (int j = 0; j < m; j++) bits[(size_t)i * W2 + j] = emit(pr, OR_AND, a[j], b[i]);
    }
    int cnt = m;
    while (cnt > 1) {
        int h = cnt / 2;
        for (int k = 0; k < h; k++) {
            int ix = k, iy = k + h;
            if (low[iy] < low[ix]) { int u = ix; ix = iy; iy = u; }
            const long* x = bits + (size_t)ix * W2;
            const long* y = bits + (size_t)iy * W2;
            const int skip = low[iy] - low[ix];
            int top = low[ix] + len[ix];
            if (low[iy] + len[iy] > top) top = low[iy] + len[iy];
            const int L = (top + 1 < W2 ? top + 1 : W2) - low[iy];
            assert(len[ix] >= skip); /* no gap between the two numbers' wired bits */
            const int lxh = len[ix] - skip;
            const int ns = build_add_n(pr, x + skip, lxh, y, len[iy], L, sum);
            long* dst = bits + (size_t)k * W2;
            const int nl = low[ix];
            memmove(dst, x, (size_t)skip * sizeof(long)); /* x's own low bits (skip <= len[ix]) */
            memcpy(dst + skip, sum, (size_t)ns * sizeof(long));
            low[k] = nl;
            len[k] = skip + ns;
        }
        if (cnt & 1) {
            memcpy(bits + (size_t)h * W2, bits + (size_t)(cnt - 1) * W2, (size_t)W2 * sizeof(long));
            low[h] = low[cnt - 1];
            len[h] = len[cnt - 1];
        }
        cnt = h + (cnt & 1);
    }
    assert(low[0] == 0 && len[0] == W2); /* one number left, at offset 0, 2m bits long */
    memcpy(r, bits, (size_t)W2 * sizeof(long));
    free(bits);
    free(low);
    free(len);
    free(sum);
}

#define OR_KARATSUBA_BASE 16 /* operands narrower than this: tree base multiplier */

/* Algorithm 1 (Sec. III-B-2) with n-bit operands, r = 2n wires: n < 16:
 * base product; else with h = floor(n/2), X = X0 + 2^h X1 (Y likewise):
 * Z0 = X0 Y0, Z1 = X1 Y1, Z2 = (X0 + X1)(Y0 + Y1) (operands n - h + 1 bits),
 * M = Z2 - Z1 - Z0 = X0 Y1 + X1 Y0 (computed mod 2^(n+1), where it fits),
 * Z = Z0 + 2^h M + 2^(2h) Z1: Z0 and 2^(2h) Z1 do not overlap, so M is added
 * to their concatenation from bit h on. */
static void build_karatsuba(or_prog* pr, const long* X, const long* Y, int n, long* r) {
    if (n < OR_KARATSUBA_BASE) {
        build_mul_full_tree(pr, X, Y, n, r);
        return;
    }
    const int h = n / 2, u = n - h, s = u + 1;
    long* S = (long*)malloc((size_t)s * sizeof(long));
    long* T = (long*)malloc((size_t)s * sizeof(long));
    long* Z2 = (long*)malloc((size_t)2 * s * sizeof(long));
    long* P = (long*)malloc((size_t)(n + 1) * sizeof(long));
    long* M = (long*)malloc((size_t)(n + 1) * sizeof(long));
    long* hi = (long*)malloc((size_t)2 * n * sizeof(long));
    build_karatsuba(pr, X, Y, h, r);                /* Z0 -> r[0, 2h) */
    build_karatsuba(pr, X + h, Y + h, u, r + 2 * h); /* Z1 -> r[2h, 2n) */
    build_add_n(pr, X, h, X + h, u, s, S);
    build_add_n(pr, Y, h, Y + h, u, s, T);
    build_karatsuba(pr, S, T, s, Z2);
    build_add_n(pr, r, 2 * h, r + 2 * h, 2 * u, n + 1, P);
    build_sub_n(pr, Z2, P, n + 1, M);
    build_add_n(pr, r + h, 2 * n - h, M, n + 1, 2 * n - h, hi);
    memcpy(r + h, hi, (size_t)(2 * n - h) * sizeof(long));
    free(S);
    free(T);
    free(Z2);
    free(P);
    free(M);
    free(hi);
}

/* Tree accumulation (Sec. V-B-2, Fig. 4): the list is split into its first
 * and second halves, which are added element-wise; an odd last element is
 * carried to the next round unchanged. */
static void build_tree_sum(or_prog* pr, long* vals, int count, int w, long* r) {
    int len = count;
    long* tmp = (long*)malloc((size_t)w * sizeof(long));
    while (len > 1) {
        int h = len / 2;
        for (int k = 0; k < h; k++) {
            build_add(pr, vals + (size_t)k * w, vals + (size_t)(k + h) * w, w, tmp);
            memcpy(vals + (size_t)k * w, tmp, (size_t)w * sizeof(long));
        }
        if (len & 1) memcpy(vals + (size_t)h * w, vals + (size_t)(len - 1) * w, (size_t)w * sizeof(long));
        len = h + (len & 1);
    }
    memcpy(r, vals, (size_t)w * sizeof(long));
    free(tmp);
}

/* Evaluates a program: wires 0..ninputs-1 hold the inputs; each gate runs
 * once all its inputs exist, gates whose inputs are ready run side by side. */
static void run_prog(const or_keys* K, const or_prog* pr, uint32_t* wires, int threads) {
    const size_t W = (size_t)K->P.n + 1;
    long* level = (long*)calloc((size_t)pr->nwires, sizeof(long));
    long maxlev = 0;
    for (long k = 0; k < pr->ng; k++) {
        const or_gate_t* G = &pr->g[k];
        long l = level[G->in0] > level[G->in1] ? level[G->in0] : level[G->in1];
        if (G->in2 >= 0 && level[G->in2] > l) l = level[G->in2];
        level[G->out] = 1 + l;
        if (G->out2 >= 0) level[G->out2] = 1 + l;
        if (level[G->out] > maxlev) maxlev = level[G->out];
    }
    uint8_t* ops = (uint8_t*)malloc((size_t)pr->ng + 1);
    const uint32_t** a = (const uint32_t**)malloc(((size_t)pr->ng + 1) * sizeof(*a));
    const uint32_t** b = (const uint32_t**)malloc(((size_t)pr->ng + 1) * sizeof(*b));
    const uint32_t** c = (const uint32_t**)malloc(((size_t)pr->ng + 1) * sizeof(*c));
    uint32_t** o = (uint32_t**)malloc(((size_t)pr->ng + 1) * sizeof(*o));
    int* ops2 = (int*)malloc(((size_t)pr->ng + 1) * sizeof(int));
    uint32_t** o2 = (uint32_t**)malloc(((size_t)pr->ng + 1) * sizeof(*o2));
    for (long L = 1; L <= maxlev; L++) {
        size_t cnt = 0;
        int three = 0;
        for (long k = 0; k < pr->ng; k++) {
            const or_gate_t* G = &pr->g[k];
            if (level[G->out] != L) continue;
            ops[cnt] = (uint8_t)G->op;
            a[cnt] = wires + (size_t)G->in0 * W;
            b[cnt] = wires + (size_t)G->in1 * W;
            c[cnt] = G->in2 >= 0 ? wires + (size_t)G->in2 * W : a[cnt]; /* (unread by two-input gates) */
            three |= G->in2 >= 0;
            o[cnt] = wires + (size_t)G->out * W;
            ops2[cnt] = G->op2;
            o2[cnt] = G->out2 >= 0 ? wires + (size_t)G->out2 * W : NULL;
            cnt++;
        }
        run_gates_c(K, ops, a, b, three ? c : NULL, o, ops2, o2, cnt, threads);
    }
    free(ops2);
    free(o2);
    free(level);
    free(ops);
    free(a);
    free(b);
    free(c);
    free(o);
}

enum { KIND_ADD = 0, KIND_MUL = 1, KIND_MATVEC = 2, KIND_MUL_TREE = 3, KIND_KARATSUBA = 4, KIND_ADD_NUMBERWISE = 5,
       KIND_MATMUL = 6, KIND_ADD_FA = 7, KIND_ADD_COMPOUND = 8 };

static void circuit_binary(const or_keys* K, int kind, const uint32_t* A, const uint32_t* B,
                           uint32_t* R, size_t count, int32_t width, int threads) {
    const size_t W = (size_t)K->P.n + 1;
    or_prog pr = {0};
    pr.nwires = (long)(2 * count * (size_t)width);
    const int32_t ow = kind == KIND_KARATSUBA ? 2 * width : width; /* result bits */
    long* outw = (long*)malloc(count * (size_t)ow * sizeof(long));
    long* ia = (long*)malloc((size_t)width * sizeof(long));
    long* ib = (long*)malloc((size_t)width * sizeof(long));
    for (size_t c = 0; c < count; c++) {
        for (int32_t k = 0; k < width; k++) {
            ia[k] = (long)(c * width + k);
            ib[k] = (long)((count + c) * width + k);
        }
        if (kind == KIND_ADD) build_add(&pr, ia, ib, width, outw + c * ow);
        else if (kind == KIND_MUL_TREE) build_mul_tree(&pr, ia, ib, width, outw + c * ow);
        else if (kind == KIND_KARATSUBA) build_karatsuba(&pr, ia, ib, width, outw + c * ow);
        else if (kind == KIND_ADD_NUMBERWISE) build_add_numberwise(&pr, ia, ib, width, outw + c * ow);
        else if (kind == KIND_ADD_FA) build_add_fa(&pr, ia, ib, width, outw + c * ow);
        else if (kind == KIND_ADD_COMPOUND) build_add_compound(&pr, ia, ib, width, outw + c * ow);
        else build_mul(&pr, ia, ib, width, outw + c * ow);
    }
    uint32_t* wires = (uint32_t*)malloc((size_t)pr.nwires * W * sizeof(uint32_t));
    memcpy(wires, A, count * width * W * sizeof(uint32_t));
    memcpy(wires + count * width * W, B, count * width * W * sizeof(uint32_t));
    run_prog(K, &pr, wires, threads);
    for (size_t q = 0; q < count * (size_t)ow; q++)
        memcpy(R + q * W, wires + (size_t)outw[q] * W, W * sizeof(uint32_t));
    free(wires);
    free(outw);
    free(ia);
    free(ib);
    free(pr.g);
}

void or_circuit_add(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                    size_t count, int32_t width, int threads) {
    circuit_binary(K, KIND_ADD, A, B, R, count, width, threads);
}

void or_circuit_mul(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                    size_t count, int32_t width, int threads) {
    circuit_binary(K, KIND_MUL, A, B, R, count, width, threads);
}

void or_circuit_mul_tree(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                         size_t count, int32_t width, int threads) {
    circuit_binary(K, KIND_MUL_TREE, A, B, R, count, width, threads);
}

void or_circuit_karatsuba(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                          size_t count, int32_t width, int threads) {
    circuit_binary(K, KIND_KARATSUBA, A, B, R, count, width, threads);
}

void or_circuit_add_numberwise(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                               size_t count, int32_t width, int threads) {
    circuit_binary(K, KIND_ADD_NUMBERWISE, A, B, R, count, width, threads);
}

void or_circuit_add_compound(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                             size_t count, int32_t width, int threads) {
    circuit_binary(K, KIND_ADD_COMPOUND, A, B, R, count, width, threads);
}

void or_circuit_add_fa(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                       size_t count, int32_t width, int threads) {
    circuit_binary(K, KIND_ADD_FA, A, B, R, count, width, threads);
}

/* y_r = sum_c M[r][c] * x_c mod 2^w: every product by the shift-and-add multiplier,
 * each row's products summed by the tree above. */
static void build_matvec(or_prog* pr, int32_t rows, int32_t cols, int32_t w, long* yw) {
    long* prods = (long*)malloc((size_t)cols * w * sizeof(long));
    long xbase = (long)rows * cols * w;
    for (int32_t r = 0; r < rows; r++) {
        for (int32_t c = 0; c < cols; c++) {
            long ia[64], ib[64];
            for (int32_t k = 0; k < w; k++) {
                ia[k] = ((long)r * cols + c) * w + k;
                ib[k] = xbase + (long)c * w + k;
            }
            build_mul(pr, ia, ib, w, prods + (size_t)c * w);
        }
        build_tree_sum(pr, prods, cols, w, yw + (size_t)r * w);
    }
    free(prods);
}

/* C = A B mod 2^w for n x n matrices by Cannon's algorithm (Sec. V-B-3): after
 * the initial skew (row i of A left by i, column j of B up by j) cycle t
 * multiplies, in every cell at once, the aligned pair A[i][k] B[k][j] with
 * k = (i + j + t) mod n, adds it to the cell's sum, and shifts A left and B
 * up by one.  The shifts move no data in a circuit (they only rename wires);
 * the products use the tree-accumulated multiplier (the paper's vector
 * multiplication), the sums the ripple-carry adder, in cycle order.
 * Wires: A then B, [n][n][w] each; cw: [n][n][w]. */
static void build_matmul_cannon(or_prog* pr, int32_t n, int32_t w, long* cw) {
    long* prod = (long*)malloc((size_t)w * sizeof(long));
    long* sum = (long*)malloc((size_t)w * sizeof(long));
    long ia[64], ib[64];
    const long bbase = (long)n * n * w;
    for (int32_t i = 0; i < n; i++)
        for (int32_t j = 0; j < n; j++) {
            long* c = cw + ((size_t)i * n + j) * w;
            for (int32_t t = 0; t < n; t++) {
                const int32_t k = (i + j + t) % n;
                for (int32_t q = 0; q < w; q++) {
                    ia[q] = ((long)i * n + k) * w + q;
                    ib[q] = bbase + ((long)k * n + j) * w + q;
                }
                build_mul_tree(pr, ia, ib, w, t == 0 ? c : prod);
                if (t > 0) {
                    build_add(pr, c, prod, w, sum);
                    memcpy(c, sum, (size_t)w * sizeof(long));
                }
            }
        }
    free(prod);
    free(sum);
}

void or_circuit_matmul(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* Cm,
                       int32_t n, int32_t width, int threads) {
    const size_t W = (size_t)K->P.n + 1;
    const size_t cells = (size_t)n * n;
    or_prog pr = {0};
    pr.nwires = (long)(2 * cells * (size_t)width);
    long* cw = (long*)malloc(cells * (size_t)width * sizeof(long));
    build_matmul_cannon(&pr, n, width, cw);
    uint32_t* wires = (uint32_t*)malloc((size_t)pr.nwires * W * sizeof(uint32_t));
    memcpy(wires, A, cells * width * W * sizeof(uint32_t));
    memcpy(wires + cells * width * W, B, cells * width * W * sizeof(uint32_t));
    run_prog(K, &pr, wires, threads);
    for (size_t q = 0; q < cells * (size_t)width; q++)
        memcpy(Cm + q * W, wires + (size_t)cw[q] * W, W * sizeof(uint32_t));
    free(wires);
    free(cw);
    free(pr.g);
}

void or_circuit_matvec(const or_keys* K, const uint32_t* M, const uint32_t* x, uint32_t* y,
                       int32_t rows, int32_t cols, int32_t width, int threads) {
    const size_t W = (size_t)K->P.n + 1;
    or_prog pr = {0};
    pr.nwires = (long)rows * cols * width + (long)cols * width;
    long* yw = (long*)malloc((size_t)rows * width * sizeof(long));
    build_matvec(&pr, rows, cols, width, yw);
    uint32_t* wires = (uint32_t*)malloc((size_t)pr.nwires * W * sizeof(uint32_t));
    memcpy(wires, M, (size_t)rows * cols * width * W * sizeof(uint32_t));
    memcpy(wires + (size_t)rows * cols * width * W, x, (size_t)cols * width * W * sizeof(uint32_t));
    run_prog(K, &pr, wires, threads);
    for (long q = 0; q < (long)rows * width; q++)
        memcpy(y + (size_t)q * W, wires + (size_t)yw[q] * W, W * sizeof(uint32_t));
    free(wires);
    free(yw);
    free(pr.g);
}

/* Truth table of gate op on plaintext bits (the readings of the gate list). */
static int plain_gate(int op, int a, int b) {
    switch (op) {
    case OR_AND: return a & b;
    case OR_NAND: return !(a & b);
    case OR_OR: return a | b;
    case OR_NOR: return !(a | b);
    case OR_XOR: return a ^ b;
    case OR_XNOR: return !(a ^ b);
    case OR_ANDNY: return (!a) & b;
    case OR_ANDYN: return a & !b;
    case OR_ORNY: return (!a) | b;
    case OR_ORYN: return a | !b;
    default: return -1;
    }
}

/* The circuit of or_circuit_{add,mul,matvec,mul_tree,karatsuba,add_numberwise,
 * matmul,add_fa} (kind 0..7; matmul: rows = n)
 * evaluated on plaintext bits, gate by gate in the order the program lists
 * them: in = operand bits (A then B, or M then x), LSB first, one byte per
 * bit; out = result bits.  Returns the number of result bits. */
long or_circuit_eval_plain(int kind, int32_t width, int32_t rows, int32_t cols, const uint8_t* in, uint8_t* out) {
    or_prog pr = {0};
    long nin, nout;
    long* res;
    if (kind == KIND_MATVEC) {
        nin = (long)rows * cols * width + (long)cols * width;
        nout = (long)rows * width;
        pr.nwires = nin;
        res = (long*)malloc((size_t)nout * sizeof(long));
        build_matvec(&pr, rows, cols, width, res);
    } else if (kind == KIND_MATMUL) { /* rows = n */
        nin = 2L * rows * rows * width;
        nout = (long)rows * rows * width;
        pr.nwires = nin;
        res = (long*)malloc((size_t)nout * sizeof(long));
        build_matmul_cannon(&pr, rows, width, res);
    } else {
        nin = 2L * width;
        nout = kind == KIND_KARATSUBA ? 2L * width : width;
        pr.nwires = nin;
        long* ia = (long*)malloc((size_t)width * sizeof(long));
        long* ib = (long*)malloc((size_t)width * sizeof(long));
        res = (long*)malloc((size_t)nout * sizeof(long));
        for (int32_t k = 0; k < width; k++) { ia[k] = k; ib[k] = width + k; }
        if (kind == KIND_ADD) build_add(&pr, ia, ib, width, res);
        else if (kind == KIND_MUL_TREE) build_mul_tree(&pr, ia, ib, width, res);
        else if (kind == KIND_KARATSUBA) build_karatsuba(&pr, ia, ib, width, res);
        else if (kind == KIND_ADD_NUMBERWISE) build_add_numberwise(&pr, ia, ib, width, res);
        else if (kind == KIND_ADD_FA) build_add_fa(&pr, ia, ib, width, res);
        else if (kind == KIND_ADD_COMPOUND) build_add_compound(&pr, ia, ib, width, res);
        else build_mul(&pr, ia, ib, width, res);
        free(ia);
        free(ib);
    }
    uint8_t* v = (uint8_t*)malloc((size_t)pr.nwires);
    memcpy(v, in, (size_t)nin);
    for (long k = 0; k < pr.ng; k++) {
        const or_gate_t* G = &pr.g[k];
        if (G->in2 >= 0) {
            const int n1 = v[G->in0] + v[G->in1] + v[G->in2];
            v[G->out] = (uint8_t)(G->op == OR_MAJ ? n1 >= 2 : n1 & 1);
        } else {
            v[G->out] = (uint8_t)plain_gate(G->op, v[G->in0], v[G->in1]);
            if (G->out2 >= 0) v[G->out2] = (uint8_t)plain_gate(G->op2, v[G->in0], v[G->in1]);
        }
    }
    for (long q = 0; q < nout; q++) out[q] = v[res[q]];
    free(v);
    free(res);
    free(pr.g);
    return nout;
}

long or_circuit_gate_count(int kind, int32_t width, int32_t rows, int32_t cols) {
    or_prog pr = {0};
    long n;
    if (kind == KIND_MATVEC) {
        pr.nwires = (long)rows * cols * width + (long)cols * width;
        long* yw = (long*)malloc((size_t)rows * width * sizeof(long));
        build_matvec(&pr, rows, cols, width, yw);
        free(yw);
    } else if (kind == KIND_MATMUL) {
        pr.nwires = 2L * rows * rows * width;
        long* cw = (long*)malloc((size_t)rows * rows * width * sizeof(long));
        build_matmul_cannon(&pr, rows, width, cw);
        free(cw);
    } else {
        long* ia = (long*)malloc((size_t)width * sizeof(long));
        long* ib = (long*)malloc((size_t)width * sizeof(long));
        long* r = (long*)malloc((size_t)2 * width * sizeof(long));
        for (int32_t k = 0; k < width; k++) { ia[k] = k; ib[k] = width + k; }
        pr.nwires = 2L * width;
        if (kind == KIND_ADD) build_add(&pr, ia, ib, width, r);
        else if (kind == KIND_MUL_TREE) build_mul_tree(&pr, ia, ib, width, r);
        else if (kind == KIND_KARATSUBA) build_karatsuba(&pr, ia, ib, width, r);
        else if (kind == KIND_ADD_NUMBERWISE) build_add_numberwise(&pr, ia, ib, width, r);
        else if (kind == KIND_ADD_FA) build_add_fa(&pr, ia, ib, width, r);
        else if (kind == KIND_ADD_COMPOUND) build_add_compound(&pr, ia, ib, width, r);
        else build_mul(&pr, ia, ib, width, r);
        free(ia);
        free(ib);
        free(r);
    }
    n = pr.ng;
    free(pr.g);
    return n;
}

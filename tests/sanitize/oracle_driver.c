/* Drives every entry of the CPU oracle for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: the full parameter set for key generation and a
 * batch of gates, a reduced one (n = 16, N = 64, noiseless keys) for the
 * compound, three-input and programmable bootstraps and the circuits.
 * Exits non-zero on a wrong decryption; the sanitizers abort on memory or
 * undefined-behaviour errors. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/tfhe_oracle.h"

#define CHECK(x)                                                          \
    do {                                                                  \
        if (!(x)) {                                                       \
            fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

static int circuits(const or_keys* K, int32_t w) {
    const size_t W = (size_t)K->P.n + 1;
    uint8_t bits[2 * 64];
    for (int i = 0; i < 2 * w; i++) bits[i] = (uint8_t)((i * 7 + 3) % 5 < 2);
    uint32_t* A = malloc(2 * w * W * sizeof(uint32_t));
    uint32_t* R = malloc(2 * w * W * sizeof(uint32_t));
    or_encrypt_bits(K, bits, 2 * (size_t)w, 500, A);
    const uint32_t* B = A + w * W;
    or_circuit_add(K, A, B, R, 1, w, 2);
    or_circuit_add_fa(K, A, B, R, 1, w, 2);
    or_circuit_add_compound(K, A, B, R, 1, w, 2);
    or_circuit_add_numberwise(K, A, B, R, 1, w, 2);
    or_circuit_mul(K, A, B, R, 1, w, 2);
    or_circuit_mul_tree(K, A, B, R, 1, w, 2);
    if (w >= 2) or_circuit_karatsuba(K, A, B, R, 1, w, 2);
    uint8_t in[2 * 64], outb[2 * 64];
    memcpy(in, bits, 2 * (size_t)w);
    for (int kind = 0; kind <= 8; kind++) {
        if (kind == 2 || kind == 6) continue; /* matvec / matmul below */
        if (kind == 4 && w < 2) continue;
        CHECK(or_circuit_gate_count(kind, w, 0, 0) > 0);
        CHECK(or_circuit_eval_plain(kind, w, 0, 0, in, outb) >= 0);
    }
    free(A);
    free(R);
    return 0;
}

int main(void) {
    or_params P;
    or_default_params(&P);
    or_keys K;
    CHECK(or_keygen(&P, 0, NULL, NULL, &K) == 0);
    const size_t W = (size_t)P.n + 1;
    uint8_t a[4] = {0, 0, 1, 1}, b[4] = {0, 1, 0, 1}, d[8];
    uint32_t* c = malloc(12 * W * sizeof(uint32_t));
    uint32_t* o = malloc(8 * W * sizeof(uint32_t));
    or_encrypt_bits(&K, a, 4, 1, c);
    or_encrypt_bits(&K, b, 4, 100, c + 4 * W);
    or_encrypt_bits(&K, a, 4, 200, c + 8 * W);
    const uint8_t ops[4] = {OR_NAND, OR_XOR, OR_ORYN, OR_AND};
    or_bootstrap_gates(&K, ops, c, c + 4 * W, o, 4, 4);
    or_decrypt_bits(&K, o, 4, d);
    CHECK(d[0] == 1 && d[1] == 1 && d[2] == 1 && d[3] == 1);
    free(c);
    free(o);
    or_keys_free(&K);

    /* reduced parameters, noiseless keys: every circuit of the oracle */
    or_params S = P;
    S.n = 16;
    S.N = 64;
    S.lwe_stdev = 0;
    S.bk_stdev = 0;
    or_keys KS;
    CHECK(or_keygen(&S, 1, NULL, NULL, &KS) == 0);
    for (int32_t w = 1; w <= 5; w += 2)
        if (circuits(&KS, w)) return 1;
    const size_t WS = (size_t)S.n + 1;
    {  /* compound, three-input and programmable bootstraps */
        uint32_t* cs = malloc(12 * WS * sizeof(uint32_t));
        uint32_t* os = malloc(8 * WS * sizeof(uint32_t));
        or_encrypt_bits(&KS, a, 4, 1, cs);
        or_encrypt_bits(&KS, b, 4, 100, cs + 4 * WS);
        or_encrypt_bits(&KS, a, 4, 200, cs + 8 * WS);
        const uint8_t pair[2] = {OR_XOR, OR_AND};
        CHECK(or_bootstrap_compounds(&KS, pair, cs + 3 * WS, cs + 7 * WS, os, 1, 1) == 0);
        or_decrypt_bits(&KS, os, 2, d);
        CHECK(d[0] == 0 && d[1] == 1);
        const uint8_t maj[1] = {OR_MAJ};
        or_bootstrap_gates3(&KS, maj, cs + 2 * WS, cs + 5 * WS, cs + 11 * WS, os, 1, 1);
        or_decrypt_bits(&KS, os, 1, d);
        CHECK(d[0] == 1);
        uint32_t* tv = malloc((size_t)S.N * sizeof(uint32_t));
        for (int j = 0; j < S.N; j++) tv[j] = 1u << 29;
        or_bootstrap_lut(&KS, tv, cs, os, 1, 1); /* input bit 0: phase -1/8 maps to -tv */
        int32_t ph[1];
        or_phase(&KS, os, 1, ph);
        CHECK(ph[0] < 0);
        free(tv);
        free(cs);
        free(os);
    }
    uint8_t mb[2 * 2 * 2 * 3]; /* matvec: M (12) and x (6); matmul: A and B (12 each) */
    for (size_t i = 0; i < sizeof mb; i++) mb[i] = (uint8_t)(i % 3 == 0);
    uint32_t* M = malloc(sizeof mb * WS * sizeof(uint32_t));
    uint32_t* Y = malloc(2 * 2 * 3 * WS * sizeof(uint32_t));
    or_encrypt_bits(&KS, mb, sizeof mb, 9, M);
    or_circuit_matvec(&KS, M, M + 2 * 2 * 3 * WS, Y, 2, 2, 3, 2);
    or_circuit_matmul(&KS, M, M + 2 * 2 * 3 * WS, Y, 2, 3, 2);
    free(M);
    free(Y);
    or_keys_free(&KS);
    puts("oracle checks passed");
    return 0;
}

/*
 * CPU oracle for TFHE gate bootstrapping — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct C: polynomial products are schoolbook
 * negacyclic products in wrapping uint32 arithmetic, every step follows the
 * definition in the order the method states it.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load this code;
 * the product library never links or calls it, and it shares no source,
 * header, table or helper with the product library.
 *
 * What it follows:
 *  - LWE samples (A, B = A.S + e), binary keys, Gaussian noise: the paper's
 *    preliminaries on Torus FHE (Sec. II-A).
 *  - One bootstrap per gate, bootstrapping then key switching: Sec. II-A and
 *    Fig. 2 (boolean gate on GPU: BS key, then KS key).
 *  - Bits as LWE samples, n-bit integers as n samples (Sec. II-A, Table III).
 *  - Ripple-carry addition, eqs. (1)-(2) (Sec. V-A-3); naive shift-and-add
 *    multiplication (Sec. III-B-1); tree accumulation of products
 *    (Sec. V-B-2, Fig. 4).
 *  - The internals of bootstrapping (gadget decomposition, CMux blind
 *    rotation, sample extraction, key switching) are not described in the
 *    paper, which uses the TFHE library as a black box; they follow the
 *    published TFHE method (Chillotti, Gama, Georgieva, Izabachene,
 *    ASIACRYPT 2016 / J. Cryptology 2020) that the paper builds on.
 *
 * Parity unpinned: the absolute key and ciphertext bytes produced by the
 * counter-based generator (see or_draw) have no external reference value;
 * they are pinned only by an independent second implementation of the same
 * written generator definition.
 */
#ifndef TFHE_ORACLE_H
#define TFHE_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;          /* LWE dimension (500) */
    int32_t N;          /* ring degree, power of two (1024) */
    int32_t bk_l;       /* gadget digits per coefficient (2) */
    int32_t bk_bgbit;   /* bits per gadget digit (10) */
    int32_t ks_t;       /* key-switch digits per coefficient (8) */
    int32_t ks_basebit; /* bits per key-switch digit (2) */
    double lwe_stdev;   /* fresh LWE and key-switch key noise (2.44e-5) */
    double bk_stdev;    /* bootstrapping key noise (7.18e-9) */
} or_params;

typedef struct {
    or_params P;
    uint64_t seed;
    int32_t* lwe_key;   /* [n] in {0,1} */
    int32_t* tlwe_key;  /* [N] in {0,1} */
    uint32_t* bk;       /* [n][2*l][2][N]: row r = 2*j + p, column c */
    uint32_t* ksk;      /* [N][t][2^basebit][n+1], value 0 rows all zero */
} or_keys;

/* Gate codes (uint8 on the wire), same numbering as the public gate enum. */
enum { OR_AND = 0, OR_NAND, OR_OR, OR_NOR, OR_XOR, OR_XNOR,
       OR_ANDNY, OR_ANDYN, OR_ORNY, OR_ORYN, OR_NUM_GATES };
/* Three-input gates: majority (the sign of c1 + c2 + c3, a full adder's
 * carry) and parity (the sign of -2 (c1 + c2 + c3), its sum bit).  Both read
 * the same constant test vector as the two-input gates. */
enum { OR_MAJ = 10, OR_XOR3 = 11 };

/* ---- counter-based generator (SplitMix64 output function) ---- */
uint64_t or_mix64(uint64_t z);
uint64_t or_draw(uint64_t seed, uint64_t stream, uint64_t idx);
double or_gaussian(uint64_t seed, uint64_t stream, uint64_t idx);
uint32_t or_torus_from_double(double x);

/* ---- keys ---- */
void or_default_params(or_params* P);
/* lwe_key_in / tlwe_key_in may be NULL (drawn from the seed) or point to
 * n / N values in {0,1} that replace the drawn keys (special-case tests). */
int or_keygen(const or_params* P, uint64_t seed, const int32_t* lwe_key_in,
              const int32_t* tlwe_key_in, or_keys* out);
void or_keys_free(or_keys* K);

/* ---- LWE encryption (one bit = one sample, +mu for 1, -mu for 0) ---- */
void or_encrypt_bits(const or_keys* K, const uint8_t* bits, size_t count,
                     uint64_t nonce, uint32_t* ct);
void or_phase(const or_keys* K, const uint32_t* ct, size_t count, int32_t* phase);
void or_decrypt_bits(const or_keys* K, const uint32_t* ct, size_t count, uint8_t* bits);

/* ---- ring arithmetic in Z/2^32[X]/(X^N+1) ---- */
void or_negacyclic_mul(int32_t N, const uint32_t* P, const uint32_t* Q, uint32_t* out);
void or_rotate(int32_t N, const uint32_t* P, int32_t a, uint32_t* out);

/* ---- pieces of the bootstrap, exposed for pinning ---- */
void or_gadget_decompose(const or_params* P, uint32_t x, int32_t* digits);
uint32_t or_modswitch(const or_params* P, uint32_t x);
void or_gate_combine(const or_params* P, int op, const uint32_t* c1,
                     const uint32_t* c2, uint32_t* out);
void or_external_product_cmux(const or_params* P, const uint32_t* bk_i,
                              int32_t abar, uint32_t* acc);
void or_blind_rotate(const or_keys* K, const uint32_t* lwe_in, uint32_t* acc);
/* Blind rotation of an arbitrary test vector tv[N] (programmable bootstrapping). */
void or_blind_rotate_tv(const or_keys* K, const uint32_t* lwe_in, const uint32_t* tv, uint32_t* acc);
/* out[g] = key switch of the sample extracted from the blind rotation of tv
 * by in[g] (no gate combination): encrypts tv[phibar] for phibar < N and
 * -tv[phibar - N] above, phibar the modulus-switched phase of in[g]. */
void or_bootstrap_lut(const or_keys* K, const uint32_t* tv, const uint32_t* in, uint32_t* out, size_t count,
                      int threads);
void or_sample_extract(const or_params* P, const uint32_t* acc, uint32_t* lwe_big);
/* Extraction of coefficient m (0 <= m < N): the phase of the result is
 * coefficient m of the TLWE phase B - A S (m = 0: or_sample_extract). */
void or_sample_extract_at(const or_params* P, const uint32_t* acc, int32_t m, uint32_t* lwe_big);
void or_key_switch(const or_keys* K, const uint32_t* lwe_big, uint32_t* out);

/* One bootstrapped gate; threads = 0 means all online cores. */
/* Linear combination of a three-input gate (OR_MAJ, OR_XOR3; a two-input
 * code ignores c3). */
void or_gate_combine3(const or_params* P, int op, const uint32_t* c1, const uint32_t* c2,
                      const uint32_t* c3, uint32_t* out);
/* Bootstrapped gate of up to three inputs. */
void or_bootstrap_gate3(const or_keys* K, int op, const uint32_t* c1, const uint32_t* c2,
                        const uint32_t* c3, uint32_t* out);
/* out[g] = ops[g](in0[g], in1[g], in2[g]), independent gates on `threads`. */
void or_bootstrap_gates3(const or_keys* K, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                         const uint32_t* in2, uint32_t* out, size_t count, int threads);
void or_bootstrap_gate(const or_keys* K, int op, const uint32_t* c1,
                       const uint32_t* c2, uint32_t* out);
void or_bootstrap_gates(const or_keys* K, const uint8_t* ops, const uint32_t* in0,
                        const uint32_t* in1, uint32_t* out, size_t count, int threads);

/* ---- compound gates: two symmetric gates on the same inputs, one rotation ---- */
/* The N-dimensional sample of symmetric gate `op` combined from the blind
 * rotation acc of the constant test vector 1/16 by c1 + c2 (before key
 * switching); -1 for a code other than AND, NAND, OR, NOR, XOR, XNOR. */
int or_compound_combine(const or_params* P, int op, const uint32_t* acc, uint32_t* big);
int or_bootstrap_compound(const or_keys* K, int op0, int op1, const uint32_t* c1, const uint32_t* c2,
                          uint32_t* out0, uint32_t* out1);
/* ops [count][2], in0/in1 [count][n+1], out [count][2][n+1]; -1 if a code is invalid. */
int or_bootstrap_compounds(const or_keys* K, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                           uint32_t* out, size_t count, int threads);

/* ---- circuits on encrypted integers (width ciphertexts, LSB first) ---- */
void or_circuit_add(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                    size_t count, int32_t width, int threads);
void or_circuit_mul(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                    size_t count, int32_t width, int threads);
/* Low width bits of A*B with the partial products accumulated by a tree
 * (Sec. V-B-2): same gates as or_circuit_mul, fewer levels. */
void or_circuit_mul_tree(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                         size_t count, int32_t width, int threads);
/* Full product (2 width bits into R, [count][2 width][n+1]) by Karatsuba's
 * algorithm (Sec. III-B-2, Algorithm 1), operands below 16 bits by the
 * tree-accumulated base product. */
void or_circuit_karatsuba(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                          size_t count, int32_t width, int threads);
/* (A + B) mod 2^width by number-wise addition (GPU_n, Sec. V-B-1). */
void or_circuit_add_numberwise(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                               size_t count, int32_t width, int threads);
void or_circuit_matvec(const or_keys* K, const uint32_t* M, const uint32_t* x, uint32_t* y,
                       int32_t rows, int32_t cols, int32_t width, int threads);
/* (A + B) mod 2^width, eqs. (1)-(2) with compound (XOR, AND) nodes (Sec. V-A-3). */
void or_circuit_add_compound(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                             size_t count, int32_t width, int threads);
/* (A + B) mod 2^width by a ripple carry of full-adder gates (XOR3, MAJ). */
void or_circuit_add_fa(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* R,
                       size_t count, int32_t width, int threads);
/* C = A B mod 2^width (n x n matrices, [n][n][width][n+1] each) by Cannon's
 * algorithm (Sec. V-B-3). */
void or_circuit_matmul(const or_keys* K, const uint32_t* A, const uint32_t* B, uint32_t* C,
                       int32_t n, int32_t width, int threads);
/* The same circuits evaluated on plaintext bits (one byte per bit, operands
 * LSB first); returns the number of result bits written to out. */
long or_circuit_eval_plain(int kind, int32_t width, int32_t rows, int32_t cols, const uint8_t* in, uint8_t* out);
/* Number of bootstrapped gates the circuits above evaluate (no evaluation);
 * kind 0 add, 1 mul, 2 matvec, 3 mul with tree accumulation, 4 Karatsuba,
 * 5 number-wise add, 6 Cannon matmul (rows = n), 7 full-adder add, 8 add with
 * compound nodes (a compound node counts once). */
long or_circuit_gate_count(int kind, int32_t width, int32_t rows, int32_t cols);

#ifdef __cplusplus
}
#endif
#endif

/*
 * fhe.h — C ABI of the MI355X (gfx950) TFHE gate-bootstrapping library.
 *
 * The library evaluates boolean gates on LWE-encrypted bits with one
 * bootstrap per gate (paper Sec. II-A: bootstrapping decrypts and re-encrypts
 * under encryption to reset the noise; Fig. 2: a gate runs its linear
 * combination, bootstrapping with the BS key, then key switching with the KS
 * key), and builds the paper's integer circuits from those gates (Sec. III
 * and V-B: ripple-carry and number-wise addition, shift-and-add, tree and
 * Karatsuba multiplication, vector and matrix products with tree
 * accumulation, Cannon's matrix product).  It also offers three-input gates
 * (majority and parity, a full adder per level) and programmable
 * bootstrapping with a caller's test vector.
 *
 * Conventions
 *  - Every function returns int: FHE_OK (0) or a negative FHE_E* code.  No
 *    C++ exception and no abort crosses this boundary.  fhe_last_error()
 *    returns a thread-local message describing the last failure.
 *  - Torus32: a uint32 word w stands for w / 2^32 on the torus R/Z.
 *  - An LWE ciphertext is n+1 uint32 words laid out a[0..n-1], b.  A batch of
 *    `count` ciphertexts is contiguous, [count][n+1] (the paper's bit
 *    coalescing, Sec. V-A-2).  An encrypted w-bit integer is w consecutive
 *    ciphertexts, least significant bit first.
 *  - A bit is encrypted as +1/8 (bit 1) or -1/8 (bit 0) plus Gaussian noise;
 *    decryption returns 1 when the phase b - <a, s>, read as a signed int32,
 *    is > 0.
 *  - Handles (fhe_secret_key, fhe_cloud_key, fhe_ctx, fhe_server) are
 *    allocated and freed by the library.  Ciphertext buffers are always owned
 *    by the caller; the library never frees or retains them beyond the
 *    completion of the work it enqueued on the caller's stream.
 *  - Functions taking `void* stream` read and write DEVICE memory (for
 *    example torch tensors' data_ptr()) and are asynchronous on that HIP
 *    stream (NULL = the default stream).  They return once the work is
 *    enqueued.  Functions without a stream take HOST buffers and complete
 *    before returning.
 *  - Inputs and outputs of one call must not overlap.
 *  - A context is used by one host thread at a time.  Its calls may use
 *    different streams: each call's device work is ordered after the
 *    context's previous call on another stream (an event wait), because
 *    calls share the context's scratch buffer and circuit pools.
 *  - Gate codes in device memory cannot be checked when a call is made.  A
 *    gate whose code is not valid for its call outputs the all-zero sample,
 *    and the next batched call on the context made after that work has
 *    completed (or fhe_ctx_check) returns FHE_EINVAL.
 */
#ifndef FHE_H
#define FHE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FHE_OK = 0,
    FHE_EINVAL = -1,     /* bad argument (null pointer, size, parameter set) */
    FHE_ENOMEM = -2,     /* host or device allocation failed */
    FHE_EDEVICE = -3,    /* HIP runtime error, or no usable gfx950 device */
    FHE_EBUSY = -4,      /* a serving job does not fit the HBM budget now */
    FHE_ECANCELED = -5,  /* a serving job was cancelled */
    FHE_EIO = -6         /* key file could not be read or written */
};

/* TFHE parameters.  The library's kernels are specialised for the 110-bit
 * gate-bootstrapping set the paper uses (Sec. VII: the parameters of the TFHE
 * library): n=500, N=1024, k=1, l=2, Bgbit=10, t=8, basebit=2.  Any other structural value is rejected with FHE_EINVAL; the
 * noise deviations may be changed (0 gives noiseless keys for tests). */
typedef struct {
    uint32_t n;          /* LWE dimension */
    uint32_t N;          /* ring degree of Z/2^32[X]/(X^N+1) */
    uint32_t k;          /* TLWE mask polynomials (1) */
    uint32_t bk_l;       /* gadget digits */
    uint32_t bk_bgbit;   /* bits per gadget digit */
    uint32_t ks_t;       /* key-switch digits */
    uint32_t ks_basebit; /* bits per key-switch digit */
    double lwe_stdev;    /* noise of fresh ciphertexts and of the KS key */
    double bk_stdev;     /* noise of the bootstrapping key */
} fhe_params;

typedef struct fhe_secret_key fhe_secret_key; /* host-only */
typedef struct fhe_cloud_key fhe_cloud_key;   /* host copy of BK and KSK */
typedef struct fhe_ctx fhe_ctx;               /* device-resident keys on one GPU */

/* Gate codes, one byte each on the wire.  NY / YN negate the first / second
 * input (ANDNY = (not a) and b).  MAJ and XOR3 take three inputs (majority
 * and parity: a full adder's carry and sum, each one bootstrap of c1 + c2 + c3
 * resp. -2 (c1 + c2 + c3)); only fhe_bootstrap_gate3_batch and the circuits
 * accept them. */
typedef enum {
    FHE_AND = 0, FHE_NAND = 1, FHE_OR = 2, FHE_NOR = 3, FHE_XOR = 4, FHE_XNOR = 5,
    FHE_ANDNY = 6, FHE_ANDYN = 7, FHE_ORNY = 8, FHE_ORYN = 9, FHE_MAJ = 10, FHE_XOR3 = 11
} fhe_gate;

/* ---------------------------------------------------------------------- */
/* Parameters and keys (host).                                             */
/* ---------------------------------------------------------------------- */

/* Fills *out with the default parameter set above. */
int fhe_default_params(fhe_params* out);

/* Generates a secret key and the matching cloud key (bootstrapping key =
 * TGSW encryptions of the LWE key bits under the TLWE key; key-switching key
 * = LWE encryptions of the TLWE key bits scaled by each base-4 digit
 * position).  All randomness comes from the counter-based generator keyed by
 * `seed`, so the same seed gives the same key bytes.  *sk and *ck receive new
 * handles; free them with fhe_secret_key_free / fhe_cloud_key_free. */
int fhe_keygen(const fhe_params* params, uint64_t seed, fhe_secret_key** sk,
               fhe_cloud_key** ck);

/* As fhe_keygen, but the binary keys are given instead of drawn: lwe_key has
 * n entries and tlwe_key N entries, each 0 or 1; either may be NULL to draw
 * it from the seed.  Used for special-case keys with known outputs. */
int fhe_keygen_with_keys(const fhe_params* params, uint64_t seed, const int32_t* lwe_key,
                         const int32_t* tlwe_key, fhe_secret_key** sk, fhe_cloud_key** ck);

void fhe_secret_key_free(fhe_secret_key* sk);
void fhe_cloud_key_free(fhe_cloud_key* ck);

/* Copies key material out (host buffers, any may be NULL):
 *   lwe_key [n], tlwe_key [N]                        int32 in {0,1}
 *   bk  [n][2l][2][N]  uint32, row r = 2j + p, column c
 *   ksk [N][t][2^basebit][n+1] uint32 (value-0 rows are all zero) */
int fhe_secret_key_export(const fhe_secret_key* sk, int32_t* lwe_key, int32_t* tlwe_key);
int fhe_cloud_key_export(const fhe_cloud_key* ck, uint32_t* bk, uint32_t* ksk);
int fhe_cloud_key_params(const fhe_cloud_key* ck, fhe_params* out);

/* Saves both keys to one file / loads them back (checkpoint of key state).
 * Either handle may be NULL on save; on load, absent parts come back NULL.
 * Errors: FHE_EIO on file errors or a malformed file. */
int fhe_key_save(const fhe_secret_key* sk, const fhe_cloud_key* ck, const char* path);
int fhe_key_load(const char* path, fhe_secret_key** sk, fhe_cloud_key** ck);

/* ---------------------------------------------------------------------- */
/* Encryption and decryption (host buffers; paper Sec. II-A).               */
/* ---------------------------------------------------------------------- */

/* Encrypts count bits (each 0 or 1) into ct_out[count][n+1].  Ciphertext c
 * uses randomness index nonce + c: never reuse a nonce range under one key. */
int fhe_encrypt_bits(const fhe_secret_key* sk, const uint8_t* bits, size_t count,
                     uint64_t nonce, uint32_t* ct_out);

/* Encrypts count integers of `width` bits (1..64; higher bits ignored) into
 * ct_out[count][width][n+1], LSB first; bit k of integer c uses randomness
 * index nonce + c*width + k. */
int fhe_encrypt_uint(const fhe_secret_key* sk, const uint64_t* v, size_t count,
                     uint32_t width, uint64_t nonce, uint32_t* ct_out);

int fhe_decrypt_bits(const fhe_secret_key* sk, const uint32_t* ct, size_t count,
                     uint8_t* bits_out);
int fhe_decrypt_uint(const fhe_secret_key* sk, const uint32_t* ct, size_t count,
                     uint32_t width, uint64_t* v_out);

/* Phase b - <a, s> of each ciphertext as a signed int32 (noise tests). */
int fhe_phase(const fhe_secret_key* sk, const uint32_t* ct, size_t count, int32_t* phase_out);

/* ---------------------------------------------------------------------- */
/* Device context.                                                          */
/* ---------------------------------------------------------------------- */

/* Uploads the cloud key to HIP device `device`, converts the bootstrapping
 * key to the NTT domains of both arithmetics (modulo two 28-bit primes, the
 * default, and over p = 2^64 - 2^32 + 1; 32.8 MB each) and lays out the
 * key-switching key for row gathers (50.3 MB).  The cloud key may be freed
 * afterwards.  Errors: FHE_EDEVICE if the device is missing or not gfx950;
 * FHE_ENOMEM if device memory runs out. */
int fhe_ctx_create(const fhe_cloud_key* ck, int device, fhe_ctx** out);
void fhe_ctx_destroy(fhe_ctx* ctx);

/* ---------------------------------------------------------------------- */
/* Gate bootstrapping (device buffers, asynchronous on `stream`).           */
/* ---------------------------------------------------------------------- */

/* out[g] = gate ops[g] applied to (in0[g], in1[g]) for g < count: linear
 * combination, modulus switch, 500-step CMux blind rotation of the test
 * vector, sample extraction and key switching, all gates of the batch in one
 * launch per step.  ops: device uint8[count]; in0, in1, out: device
 * uint32[count][n+1].  count = 0 is a no-op.  The result is bit-exact with
 * the definition (exact NTT arithmetic).  The codes live in device memory: a
 * code outside FHE_AND..FHE_ORYN (including the three-input codes, which need
 * fhe_bootstrap_gate3_batch) gives the all-zero output sample and is reported
 * as FHE_EINVAL by the context's next batched call or fhe_ctx_check. */
int fhe_bootstrap_gate_batch(fhe_ctx* ctx, const uint8_t* ops, const uint32_t* in0,
                             const uint32_t* in1, uint32_t* out, size_t count, void* stream);

/* As fhe_bootstrap_gate_batch with a third input in2 (device
 * uint32[count][n+1]) for the three-input codes FHE_MAJ and FHE_XOR3;
 * two-input codes ignore in2[g].  The combinations carry no constant:
 * MAJ: c1 + c2 + c3, XOR3: -2 (c1 + c2 + c3), then the same bootstrap. */
int fhe_bootstrap_gate3_batch(fhe_ctx* ctx, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                              const uint32_t* in2, uint32_t* out, size_t count, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation and words as fhe_bootstrap_gate_batch, with the scratch
 * (extracted samples between blind rotation and key switching) in a fixed
 * device array of the library instead of the context's buffer, so the call
 * allocates nothing (no hipMalloc, no library allocation, no timing events).
 * count is at most 4096 (FHE_EINVAL beyond).  The array is one per GPU,
 * shared by every context on that GPU and kept until the process ends:
 * calls that overlap on one GPU (other streams, other contexts, other
 * threads) race on it and must be ordered by the caller.  Outside graph
 * capture the call is ordered after the context's last call on another
 * stream, like the other calls; under capture the caller orders it. */
int fhe_bootstrap_gate_batch_noalloc(fhe_ctx* ctx, const uint8_t* ops, const uint32_t* in0, const uint32_t* in1,
                                     uint32_t* out, size_t count, void* stream);

/* Compound gates (Sec. V-A-3: two gates on the same inputs computed
 * together), here from ONE blind rotation: out0[g] = ops0[g](in0[g], in1[g])
 * and out1[g] = ops1[g](in0[g], in1[g]) for symmetric codes (FHE_AND, NAND,
 * OR, NOR, XOR, XNOR).  The rotation takes the phase of c1 + c2 (-1/4, 0,
 * +1/4 for 0, 1, 2 true inputs, no constant) through the constant test
 * vector 1/16; coefficients 3N/4 and N/4 of the result are extracted (E1,
 * E2) and a gate with values g_k (+1 true, -1 false, k true inputs) is the
 * sample (g1 - g2) E1 + (g1 - g0) E2 + (0, (g0 + g2)/16), key-switched.  One
 * rotation and two key switchings per gate pair instead of two of each; the
 * words differ from the single gates' (other samples) and decrypt the same.
 * ops0, ops1: device uint8[count]; in0, in1, out0, out1: device
 * uint32[count][n+1].  A code that is not symmetric gives all-zero outputs
 * and is reported like an invalid code of fhe_bootstrap_gate_batch. */
int fhe_bootstrap_compound_batch(fhe_ctx* ctx, const uint8_t* ops0, const uint8_t* ops1, const uint32_t* in0,
                                 const uint32_t* in1, uint32_t* out0, uint32_t* out1, size_t count, void* stream);

/* FHE_EINVAL (and clears the report) if a kernel of this context met an
 * invalid gate code since the last report; FHE_OK otherwise.  Synchronize
 * the stream of the work in question first. */
int fhe_ctx_check(fhe_ctx* ctx);

/* Programmable bootstrapping: out[g] = the bootstrapped and key-switched
 * sample of in[g] with the test vector tv (device uint32[N]) in place of the
 * gates' constant one; no gate combination.  For the modulus-switched phase
 * phibar = round(2N phase(in[g])) mod 2N, out[g] encrypts tv[phibar] when
 * phibar < N and -tv[phibar - N] otherwise (a negacyclic lookup table; keep
 * inputs in [0, 1/2) with a padding bit for an arbitrary function).  in, out:
 * device uint32[count][n+1].  Bit-exact with the definition like the gates. */
int fhe_bootstrap_lut_batch(fhe_ctx* ctx, const uint32_t* tv, const uint32_t* in, uint32_t* out,
                            size_t count, void* stream);

/* One gate per launch, synchronous: enqueues one bootstrap on `stream` and
 * waits for it.  The baseline for batched throughput. */
int fhe_bootstrap_gate_plain(fhe_ctx* ctx, uint8_t op, const uint32_t* in0,
                             const uint32_t* in1, uint32_t* out, void* stream);

/* ---------------------------------------------------------------------- */
/* Circuits on encrypted integers (device buffers, asynchronous).           */
/* Each circuit level runs as one batched launch over every gate of the     */
/* level (all `count` instances together).                                   */
/* ---------------------------------------------------------------------- */

/* R = (A + B) mod 2^width, ripple-carry adder of eqs. (1)-(2).
 * A, B, R: device uint32[count][width][n+1]; width 1..64. */
int fhe_add(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
            uint32_t width, void* stream);

/* R = (A + B) mod 2^width by a ripple carry of full-adder gates: bit 0 a half
 * adder (XOR, AND), then per bit r = XOR3(a, b, c) and c = MAJ(a, b, c), one
 * level per bit: 2 width - 1 gates in width levels (16 bits: 31 gates, 16
 * levels).  Buffers and errors as fhe_add. */
int fhe_add_fa(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
               uint32_t width, void* stream);

/* R = (A + B) mod 2^width, the ripple-carry adder of fhe_add with compound
 * gates (Sec. V-A-3): the XOR and the AND of the same two bits come from one
 * rotation (fhe_bootstrap_compound_batch), three rotations per middle bit
 * instead of five (16 bits: 45 rotations in 30 levels against 74 gates).
 * Levels are ASAP (not balanced).  Output words differ from fhe_add's;
 * buffers and errors as fhe_add. */
int fhe_add_compound(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                     uint32_t width, void* stream);

/* R = (A + B) mod 2^width by number-wise addition (GPU_n, Sec. V-B-1): w rounds
 * of carry = R & B, R = R ^ B, B = carry << 1 over all bits at once (the
 * round's AND and XOR side by side).  width^2 gates in width levels (16 bits:
 * 256 gates, 16 levels, against 74 gates in 30 levels for fhe_add): fewer
 * levels, more gates.  Output words differ from fhe_add's; buffers and errors
 * as fhe_add. */
int fhe_add_numberwise(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                       uint32_t width, void* stream);

/* R = (A * B) mod 2^width, shift-and-add multiplier (Sec. III-B-1) keeping the
 * low width bits. */
int fhe_mul(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
            uint32_t width, void* stream);

/* R = (A * B) mod 2^width with the partial products (A & b_i) << i summed by
 * a tree (Sec. V-B-2, "Multiplication", Fig. 4): the list is split into its
 * first and second halves, added element-wise, until one number is left.
 * Same gates as fhe_mul (2,824 at width 32), fewer levels (62 instead of
 * 120), so lower latency; the output words differ from fhe_mul's (other
 * gates produce them) but decrypt to the same product.  Buffers and errors
 * as fhe_mul. */
int fhe_mul_tree(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                 uint32_t width, void* stream);

/* R = A * B in full (2 width bits: R is [count][2 width][n+1]) by Karatsuba's
 * algorithm (Sec. III-B-2, Algorithm 1): from 16-bit operands on, three
 * half-width products Z0 = X0 Y0, Z1 = X1 Y1, Z2 = (X0 + X1)(Y0 + Y1) and
 * Z = Z0 + (Z2 - Z1 - Z0) 2^h + Z1 2^(2h), h = floor(width / 2), the
 * subtraction as an addition of the complement; narrower operands by the
 * tree-accumulated product.  5,271 gates in 116 levels at width 32.
 * EINVAL: width outside 2..64, null buffers. */
int fhe_mul_karatsuba(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* R, size_t count,
                      uint32_t width, void* stream);

/* y = M x mod 2^width: every product by the shift-and-add multiplier, each row summed
 * by a tree of adders (Sec. V-B-2, Fig. 4: split in halves, add pairwise).
 * M: device uint32[rows][cols][width][n+1]; x: [cols][width][n+1];
 * y: [rows][width][n+1]. */
int fhe_matvec(fhe_ctx* ctx, const uint32_t* M, const uint32_t* x, uint32_t* y, uint32_t rows,
               uint32_t cols, uint32_t width, void* stream);

/* C = A B mod 2^width for n x n matrices by Cannon's algorithm (Sec. V-B-3):
 * in cycle t cell (i, j) multiplies A[i][k] B[k][j], k = (i + j + t) mod n
 * (the skew and shifts rename wires, no data moves), with the tree
 * multiplier of fhe_mul_tree, and adds the product to the cell's sum in cycle
 * order with the ripple-carry adder.  All cycles' products are independent,
 * so the level schedule runs them side by side (HBM holds every sample).
 * A, B, C: device uint32[n][n][width][n+1].  EINVAL: n outside 1..64, width
 * outside 1..64, null buffers. */
int fhe_matmul(fhe_ctx* ctx, const uint32_t* A, const uint32_t* B, uint32_t* C, uint32_t n,
               uint32_t width, void* stream);

/* Caller-defined circuits: any DAG of gates, run by the same level scheduler
 * as the circuits above (ASAP levels balanced to whole launch rounds, one
 * launch pair per level over all instances, captured HIP graphs).
 * Wires: 0 .. n_inputs-1 are a instance's inputs; gate k writes wire
 * n_inputs + k and may read only wires below that.  in2 is read only by
 * FHE_MAJ and FHE_XOR3.  outputs lists distinct gate-output wires.
 * fhe_circuit_run: in = device uint32[count][n_inputs][n+1], out =
 * [count][n_outputs][n+1], asynchronous on `stream`.  Destroy a circuit
 * before its context; fhe_circuit_destroy waits for the device.
 * EINVAL: a gate reading an undefined wire, an unknown gate code, an output
 * that is an input or repeated, null pointers. */
typedef struct {
    uint8_t op;
    uint32_t in0, in1, in2;
} fhe_gate_node;
typedef struct fhe_circuit fhe_circuit;
int fhe_circuit_create(fhe_ctx* ctx, const fhe_gate_node* gates, uint32_t n_gates, uint32_t n_inputs,
                       const uint32_t* outputs, uint32_t n_outputs, fhe_circuit** out);
int fhe_circuit_run(fhe_circuit* c, const uint32_t* in, uint32_t* out, size_t count, void* stream);
void fhe_circuit_destroy(fhe_circuit* c);

/* Circuit calls replay their level schedule as a captured HIP graph (one
 * per circuit shape and set of buffers, captured on first use; kernel
 * launches only).  enable = 0 launches every level directly instead.
 * While per-phase timing is on (fhe_ctx_set_timing) levels are launched
 * directly so that each launch can be timed. */
int fhe_ctx_set_graphs(fhe_ctx* ctx, int enable);

/* ---------------------------------------------------------------------- */
/* Launch shapes and the autotuner (batching of gates per circuit level).   */
/* A batch of `width` gates runs with the shape stored for its width bucket */
/* (bucket b covers widths 2^(b-1) < w <= 2^b, the last bucket, b = 15,     */
/* every width above 2^14).  Shapes:                                        */
/*   waves_per_gate = 1, gates_per_group in {1, 2, 4, 8}: one wavefront per */
/*     gate, that many ciphertexts per workgroup (throughput shape);        */
/*   waves_per_gate = 2, gates_per_group = 1: two wavefronts split every    */
/*     CMux of one gate (latency shape for levels narrower than the chip);  */
/*   each of these with either NTT arithmetic (arith 0 or 1);               */
/*   waves_per_gate = 4, gates_per_group = 1, arith = 1: four wavefronts    */
/*     per gate, one per (polynomial, prime) (lowest latency).              */
/* The shape changes only the schedule and the exact arithmetic used to     */
/* reach the result: every shape computes the same words.  Captured level   */
/* schedules are recaptured after a change.                                 */
/* ---------------------------------------------------------------------- */
typedef struct {
    uint32_t waves_per_gate;
    uint32_t gates_per_group;
    uint32_t arith;  /* 0: NTT over p = 2^64 - 2^32 + 1; 1: NTT modulo two
                        28-bit primes, recombined by CRT (both exact) */
} fhe_launch_config;

/* Times every shape on synthetic gate batches of width 1, 2, 4, ... up to
 * max_width (at most 2^15; reps timed runs each after one warm-up run, the
 * fastest kept) on the context's device and stores the fastest shape per
 * bucket (the default shape of a bucket stays unless another is more than
 * 2% faster); wider buckets take the widest measured one's.  Synchronous:
 * allocates and frees two batches of max_width samples and waits for the
 * device.  EINVAL: max_width or reps is 0. */
int fhe_ctx_autotune(fhe_ctx* ctx, uint32_t max_width, uint32_t reps);

/* The shape a batch of `width` gates (width >= 1) runs with. */
int fhe_ctx_launch_config(const fhe_ctx* ctx, uint32_t width, fhe_launch_config* out);

/* Stores cfg for every bucket that holds a width in [min_width, max_width].
 * EINVAL: an empty range or a shape outside the list above. */
int fhe_ctx_set_launch_config(fhe_ctx* ctx, uint32_t min_width, uint32_t max_width,
                              const fhe_launch_config* cfg);

/* Number of gates and of levels of a circuit as the library schedules it
 * (kind 0 = add, 1 = mul, 2 = matvec, 3 = mul with tree accumulation,
 * 4 = Karatsuba, 5 = number-wise add, 6 = Cannon matmul with rows = n,
 * 7 = full-adder add, 8 = compound add; rows/cols only for matvec and
 * matmul).  A compound gate counts once (one bootstrap). */
int fhe_circuit_shape(int kind, uint32_t width, uint32_t rows, uint32_t cols,
                      uint64_t* gates, uint32_t* levels, uint64_t* widest_level);

/* The level schedule the circuit calls run for `count` instances on a device
 * with cu_count compute units (host only): level_gates[L] = gates in launch
 * L (max_levels entries available), *levels = number of launches.  Levels
 * start from ASAP; a level narrower than one round of the widest launch shape
 * (8 cu_count gates) takes gates with slack from earlier levels (each still
 * after its inputs and before its consumers) when a per-round cost model says
 * the whole schedule gets faster.  The gates and the depth do not change. */
int fhe_circuit_schedule(int kind, uint32_t width, uint32_t rows, uint32_t cols, uint64_t count,
                         uint32_t cu_count, uint64_t* level_gates, uint32_t max_levels, uint32_t* levels);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of jobs on one context.                     */
/* A worker thread owns the context while the server exists (no other call */
/* may use that context meanwhile).  Each tick it admits queued jobs, in    */
/* arrival order, whose samples (inputs and every gate output) fit the pool */
/* left under the HBM budget; runs the next circuit level of every running */
/* job as one batched launch pair; and retires finished jobs, copying their */
/* outputs to the caller's buffer.  Jobs that arrive while a tick runs join */
/* the next tick.  Results do not depend on the mix (each gate is computed  */
/* exactly, independently of the others in its launch).                      */
/* Ticks are enqueued ahead of the device (up to three in flight), so the    */
/* GPU does not idle between them; a job is done once its last tick ran.     */
/* ---------------------------------------------------------------------- */
typedef struct fhe_server fhe_server;

typedef enum {
    FHE_JOB_GATE = 0, FHE_JOB_ADD = 1, FHE_JOB_MUL = 2, FHE_JOB_MATVEC = 3, FHE_JOB_MUL_TREE = 4,
    FHE_JOB_ADD_FA = 5, FHE_JOB_ADD_NUMBERWISE = 6, FHE_JOB_KARATSUBA = 7, FHE_JOB_MATMUL = 8
} fhe_job_kind;

/* One job.  Buffers are DEVICE memory owned by the caller; inputs must be
 * written (their stream synchronized) before submission and stay valid, and
 * `out` is written when the job reaches FHE_JOB_DONE.
 *   GATE:   in0, in1 [1][n+1], op = gate code, out [1][n+1]
 *   ADD/MUL/MUL_TREE/ADD_FA/ADD_NUMBERWISE: in0, in1, out [width][n+1] (one
 *           integer, LSB first; the circuits of fhe_add, fhe_mul, fhe_mul_tree,
 *           fhe_add_fa, fhe_add_numberwise)
 *   KARATSUBA: in0, in1 [width][n+1], out [2 width][n+1] (fhe_mul_karatsuba)
 *   MATMUL: rows = n; in0 = A, in1 = B, out = C, each [n][n][width][n+1]
 *           (fhe_matmul)
 *   MATVEC: in0 = M [rows][cols][width][n+1], in1 = x [cols][width][n+1],
 *           out = y [rows][width][n+1]                                        */
typedef struct {
    uint32_t kind, op, width, rows, cols;
    const uint32_t* in0;
    const uint32_t* in1;
    uint32_t* out;
} fhe_job;

enum { FHE_JOB_QUEUED = 0, FHE_JOB_RUNNING = 1, FHE_JOB_DONE = 2, FHE_JOB_CANCELLED = 3, FHE_JOB_FAILED = 4 };

/* Creates a server whose job pool may use hbm_budget_bytes of device memory
 * (allocated at once; 2,004 bytes per sample).  FHE_EINVAL below one gate
 * job, FHE_ENOMEM if the device cannot hold the pool. */
int fhe_serve_create(fhe_ctx* ctx, size_t hbm_budget_bytes, fhe_server** out);

/* Queues a job and returns its ticket.  FHE_EBUSY if the job alone needs more
 * samples than the whole budget (it could never be admitted). */
int fhe_serve_submit(fhe_server* srv, const fhe_job* job, uint64_t* ticket);

/* State of a job (FHE_JOB_*) and, once done, its latency from submission to
 * completion in milliseconds (-1 before).  Returns FHE_ECANCELED or the
 * job's error code for cancelled or failed jobs. */
int fhe_serve_poll(fhe_server* srv, uint64_t ticket, int* state, double* latency_ms);

/* Split of a done job's latency: time queued before admission and time from
 * admission to completion (milliseconds; either pointer may be NULL).
 * EINVAL: unknown ticket or a job that is not done. */
int fhe_serve_job_times(fhe_server* srv, uint64_t ticket, double* queue_ms, double* service_ms);

/* Blocks until the job is done, cancelled or failed, or timeout_s elapses
 * (FHE_EBUSY). */
int fhe_serve_wait(fhe_server* srv, uint64_t ticket, double timeout_s);

/* Cancels a queued or running job; its pool samples are freed at the next
 * tick and its output buffer is left unspecified. */
int fhe_serve_cancel(fhe_server* srv, uint64_t ticket);

/* Counters since creation (any pointer may be NULL). */
int fhe_serve_stats(fhe_server* srv, uint64_t* jobs_done, uint64_t* gates_done, uint64_t* launches,
                    uint64_t* pool_bytes_in_use, uint64_t* jobs_waiting);

/* Cancels what is left, stops the worker and frees the pool. */
void fhe_serve_destroy(fhe_server* srv);

/* ---------------------------------------------------------------------- */
/* Errors and diagnostics.                                                  */
/* ---------------------------------------------------------------------- */

/* Per-phase device timing, the split of the paper's Table IV (bootstrapping,
 * key switching).  While enabled, every batched launch pair records HIP
 * events on the stream it runs on.  fhe_ctx_timing() waits for the recorded
 * work, returns the totals since the last call (milliseconds of blind-
 * rotation and key-switch kernels, number of launch pairs, gates) and resets
 * them.  Any output pointer may be NULL. */
int fhe_ctx_set_timing(fhe_ctx* ctx, int enable);
int fhe_ctx_timing(fhe_ctx* ctx, double* blind_rotate_ms, double* key_switch_ms,
                   uint64_t* launches, uint64_t* gates);

/* The same records launch by launch, with the shape each ran with.  Waits
 * for the recorded work; writes min(recorded, max) records in launch order
 * to out, the number recorded to *count, and resets the records. */
typedef struct {
    uint64_t gates;
    uint32_t waves_per_gate;
    uint32_t gates_per_group;
    uint32_t arith;
    uint32_t reserved;  /* 0 */
    double blind_rotate_ms;
    double key_switch_ms;
} fhe_launch_record;
int fhe_ctx_timing_launches(fhe_ctx* ctx, fhe_launch_record* out, size_t max, size_t* count);

/* Message of the last failing call on this thread ("" if none). */
const char* fhe_last_error(void);

/* Test entry: one CMux step of the blind rotation on explicit HOST data,
 * computed on `device` with the production kernels of NTT arithmetic `arith`
 * (0: Goldilocks prime, 1: two 28-bit primes and CRT; see fhe_launch_config):
 *   acc[2][N] <- acc + BK_i [x] (X^abar acc - acc),
 * bk_i: uint32 [2l][2][N] (coefficient domain, rows r = 2j + p). */
int fhe_debug_cmux(int device, int arith, const uint32_t* bk_i, int32_t abar, uint32_t* acc);

/* Measurement entry: the issue rate of one VALU instruction class on
 * `device`, in 32-bit lane operations per second (every lane of eight waves
 * per SIMD runs 16 independent chains of the instruction; fastest of two
 * timed runs): op 0 v_add_u32, 1 v_mul_lo_u32, 2 v_mad_i64_i32, 3
 * v_mul_hi_u32, 4 v_bfe_i32, 5 v_permlane32_swap (two registers exchanged
 * per instruction).  It is the per-class peak behind the blind rotation's
 * roofline.  Synchronous; allocates and frees 2 MB.  EINVAL: op outside 0..5. */
int fhe_debug_valu_rate(int device, int op, double* lane_ops_per_s);

/* Test entries: the level schedule of the plan a circuit entry point runs on
 * this context, and the words its wires hold after a run, so that tests can
 * recompute sampled gates of a full-size circuit from the inputs the GPU gave
 * them (the wire ids travel with the gates, so every gate can be checked on
 * its own).  kind as in fhe_circuit_shape; count = 1 for matvec (rows, cols)
 * and matmul (rows = n); other kinds ignore rows and cols.  The plan is built
 * (and its pool allocated) if the context has none yet.
 * fhe_debug_plan: gates_out (host, NULL to query sizes) receives
 * [gates][5] uint32 {op, in0, in1, out, in2} in launch order, in2 =
 * 0xFFFFFFFF for two-input gates; a compound gate has op = 0x10000 | code0 |
 * code1 << 8 and in2 = the wire of its second output; level_off (host, NULL allowed) receives
 * levels + 1 offsets into that list; *n_gates, *n_levels the sizes.  A wire
 * id is (region << 30) | index, region 0 = A, 1 = B, 2 = R (the caller's
 * buffers of the entry point), 3 = the plan's pool; sample `index` of the
 * region.  fhe_debug_read_wires waits for the device, then copies the n
 * wires' samples to words_out (host [n][n+1]); A, B, R are the buffers the
 * entry point ran on.  EINVAL: bad kind or sizes, buffers too small, a wire
 * outside the plan's regions. */
int fhe_debug_plan(fhe_ctx* ctx, int kind, uint32_t width, uint32_t rows, uint32_t cols, uint64_t count,
                   uint32_t* gates_out, uint64_t max_gates, uint32_t* level_off, uint32_t max_levels,
                   uint64_t* n_gates, uint32_t* n_levels);
int fhe_debug_read_wires(fhe_ctx* ctx, int kind, uint32_t width, uint32_t rows, uint32_t cols, uint64_t count,
                         const uint32_t* A, const uint32_t* B, const uint32_t* R, const uint32_t* wires, size_t n,
                         uint32_t* words_out);

#ifdef __cplusplus
}
#endif
#endif

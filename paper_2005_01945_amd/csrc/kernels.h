// Launchers of the gfx950 kernels (kernels.hip), called by the runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fhe {
namespace dev {

constexpr int kWavesPerBlock = 4;
constexpr int kBlockThreads = 64 * kWavesPerBlock;

// Compound gates: two symmetric gates of the same two inputs from one blind
// rotation.  In descriptor mode the op field holds kCompoundFlag | code0 |
// code1 << 8 and desc3[g] the wire of the second output.
constexpr uint32_t kCompoundFlag = 1u << 16;

// Where a batch of gates reads its operands and writes its results.
//  Direct mode (desc == nullptr): gate g reads in0 + g*(n+1), in1 + g*(n+1),
//  writes out + g*(n+1); its code is ops[g], or op_const when ops == nullptr.
//  With ops1 (compound batch) gate g is the compound of codes ops[g] and
//  ops1[g], its second output out1 + g*(n+1).
//  Descriptor mode: desc[g] = {op, in0 wire, in1 wire, out wire}; a wire id
//  is (region << 30) | index and addresses region[region] + index*(n+1).
//  pair_slots = 1: every gate owns two extracted-sample slots (2g, 2g+1) and
//  key switching runs over 2*count samples (compound gates present); slot
//  2g+1 of a gate that is not compound is skipped.
//  A gate whose code is not valid for the batch (two-input codes 0..9; MAJ
//  and XOR3 with a third input; symmetric codes for compound gates) outputs
//  the all-zero sample and stores 0x100 | code into *err (when err is set).
struct GateIO {
    const uint4* desc;        // {op, in0, in1, out} wire ids per gate, or null
    const uint32_t* desc3;    // with desc: third-input wire id per gate (three-input codes), or null
    const uint8_t* ops;
    uint32_t op_const;
    const uint32_t* in0;
    const uint32_t* in1;
    const uint32_t* in2;      // without desc: third inputs, or null
    const uint32_t* tv;       // programmable bootstrapping: test vector [N] (in0 taken as is), or null
    uint32_t* out;
    uint32_t* region[4];
    const uint8_t* ops1;      // compound batch (direct mode): second code per gate, or null
    uint32_t* out1;           //   and its outputs [count][n+1]
    uint32_t pair_slots;      // 1: two extracted-sample slots per gate
    uint32_t* err;            // invalid-code report word (device-visible), or null
};

// Per-context device key material.
struct DeviceKeys {
    const uint64_t* bkd;      // BK in the NTT domain, kernel layout (32 MB)
    const uint32_t* ksk;      // KSK rows v = 1..3, [N][t][3][512] (50 MB)
    const uint32_t* zero_row; // 512 zero words (digit 0 rows)
    const uint64_t* twf;      // forward twiddles [32][32]
    const uint64_t* twi;      // inverse twiddles (with N^-1) [32][32]
    // Two-prime NTT: BK residues (Montgomery form, 32-bit words)
    // [n][hp][prime][q / 2][64 lanes][q % 2][digit], and twiddle tables int32
    // [prime][32][32] (8 KB each, read as 1024 uint64).
    const uint64_t* bkq;
    const uint64_t* twfq;
    const uint64_t* twiq;
};

// BK (uint32 [n][2l][2][N], device) -> NTT-domain kernel layout.
hipError_t launch_bk_prepare(const uint32_t* bk, uint64_t* bkd, const uint64_t* twf,
                             uint32_t n_lwe, hipStream_t s);
// The same for the two-prime NTT (twfq: the two-prime forward table).
hipError_t launch_bk_prepare_q(const uint32_t* bk, uint64_t* bkq, const uint64_t* twfq,
                               uint32_t n_lwe, hipStream_t s);

// Kernel shape of a blind-rotation launch.  waves_per_gate = 1: one wave
// bootstraps a gate, gates_per_group in {1, 2, 4, 8} gates share a workgroup
// (and its twiddle copy in LDS).  waves_per_gate = 2: two waves split each
// CMux of one gate (one gate per workgroup; gates_per_group is ignored);
// waves_per_gate = 4 (arith 1 only): one wave per (polynomial, prime).
// arith: 0 = NTT over the Goldilocks prime, 1 = NTT modulo two 28-bit
// primes recombined by CRT.  Every shape gives the same words.
struct LaunchConfig {
    uint32_t waves_per_gate;
    uint32_t gates_per_group;
    uint32_t arith;
};

// Gate prologue + blind rotation + sample extraction: writes big[g][N+1]
// (big[2g], big[2g+1] with pair_slots).
hipError_t launch_blind_rotate(const DeviceKeys& K, const GateIO& io, uint32_t* big,
                               uint32_t count, LaunchConfig cfg, hipStream_t s);

// Key switching big[k] -> the gate's output sample, k < count (with
// pair_slots, count = 2 * gates).
hipError_t launch_key_switch(const DeviceKeys& K, const GateIO& io, const uint32_t* big,
                             uint32_t count, hipStream_t s);

// One CMux on acc[2][N] (device) with prepared BK_i (one iteration of bkd
// for arith 0, of bkq for arith 1).
hipError_t launch_debug_cmux(const DeviceKeys& K, int arith, const uint64_t* bk_i, int32_t abar,
                             uint32_t* acc, hipStream_t s);

// Issue-rate probe of VALU instruction class `op` (0 v_add_u32, 1
// v_mul_lo_u32, 2 v_mad_i64_i32, 3 v_mul_hi_u32, 4 v_bfe_i32, 5
// v_permlane32_swap): blocks x 256 threads, 64 x iters instructions per
// lane; out holds blocks x 256 words.
hipError_t launch_valu_probe(int op, uint32_t* out, uint32_t blocks, int iters, hipStream_t s);

}  // namespace dev
}  // namespace fhe

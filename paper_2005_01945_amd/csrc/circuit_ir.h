// Circuits on encrypted bits as gate lists (shared by the batched circuit
// entry points and the serving runtime).
#pragma once

#include <cstdint>
#include <vector>

namespace fhe {

enum Kind { kAdd = 0, kMul = 1, kMatvec = 2, kMulTree = 3, kKaratsuba = 4, kAddNumberwise = 5, kMatmul = 6, kAddFa = 7 };

constexpr uint32_t kNoWire = 0xFFFFFFFFu;

struct Gate {
    uint8_t op;
    uint32_t in0, in1, out;
    uint32_t in2 = kNoWire;  // third input of FHE_MAJ / FHE_XOR3
};

// One instance of a circuit over local wire ids: [0, na) first operand,
// [na, na+nb) second operand, then one wire per gate output (gate k writes
// wire na + nb + k).  `outputs` lists the result bits, LSB first.
struct Circuit {
    uint32_t na = 0, nb = 0;
    std::vector<Gate> gates;
    std::vector<uint32_t> outputs;
    uint32_t wires() const { return na + nb + (uint32_t)gates.size(); }
};

// kind: kAdd / kAddNumberwise / kAddFa / kMul / kMulTree / kKaratsuba (operands of
// width w; Karatsuba has 2w result bits), kMatvec (rows x cols matrix of w-bit
// entries times a cols-vector) or kMatmul (two rows x rows matrices).
Circuit build_circuit(int kind, uint32_t w, uint32_t rows, uint32_t cols);

// ASAP level of every gate (inputs are level 0); *depth = deepest level.
std::vector<uint32_t> asap_levels(const Circuit& c, uint32_t* depth);

}  // namespace fhe

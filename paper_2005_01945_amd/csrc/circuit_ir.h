// Circuits on encrypted bits as gate lists (shared by the batched circuit
// entry points and the serving runtime).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace fhe {

enum Kind {
    kAdd = 0, kMul = 1, kMatvec = 2, kMulTree = 3, kKaratsuba = 4, kAddNumberwise = 5, kMatmul = 6, kAddFa = 7,
    kAddCompound = 8
};
constexpr int kLastKind = kAddCompound;

constexpr uint32_t kNoWire = 0xFFFFFFFFu;

struct Gate {
    uint8_t op;
    uint32_t in0, in1, out;
    uint32_t in2 = kNoWire;  // third input of FHE_MAJ / FHE_XOR3
    bool second = false;     // second output of a compound node: the previous
                             // gate has the same inputs and one rotation serves both
};

// One instance of a circuit over local wire ids: [0, na) first operand,
// [na, na+nb) second operand, then one wire per gate output (gate k writes
// wire na + nb + k).  `outputs` lists the result bits, LSB first.
struct Circuit {
    uint32_t na = 0, nb = 0;
    std::vector<Gate> gates;
    std::vector<uint32_t> outputs;
    uint32_t wires() const { return na + nb + (uint32_t)gates.size(); }
    bool has_compound() const {
        for (const Gate& g : gates)
            if (g.second) return true;
        return false;
    }
    // bootstraps (a compound node is one)
    uint64_t bootstraps() const {
        uint64_t n = 0;
        for (const Gate& g : gates) n += g.second ? 0 : 1;
        return n;
    }
};

// kind: kAdd / kAddNumberwise / kAddFa / kAddCompound / kMul / kMulTree / kKaratsuba (operands of
// width w; Karatsuba has 2w result bits), kMatvec (rows x cols matrix of w-bit
// entries times a cols-vector) or kMatmul (two rows x rows matrices).
Circuit build_circuit(int kind, uint32_t w, uint32_t rows, uint32_t cols);

// ASAP level of every gate (inputs are level 0); *depth = deepest level.
std::vector<uint32_t> asap_levels(const Circuit& c, uint32_t* depth);

// Level balancing for `count` instances and launch rounds of `round` gates:
// gates with slack move to narrow levels (each still after its inputs and
// before its consumers) when a per-round cost model says the schedule gets
// faster.  Returns every gate's level; the depth does not change.
std::vector<uint32_t> balance_levels(const Circuit& c, const std::vector<uint32_t>& asap, uint32_t depth,
                                     size_t count, uint64_t round);

}  // namespace fhe

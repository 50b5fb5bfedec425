// Integer circuits on encrypted bits as gate lists, and their level
// schedules (host code only; the device plans are in circuits.cpp).
//
// Circuit definitions (each gate a two-input bootstrapped gate):
//  - add, w bits, sum mod 2^w: the ripple-carry adder of eqs. (1)-(2),
//      bit 0:     r = a^b,            c = a&b
//      bit i:     t = a^b, g = a&b,  r = t^c, h = t&c, c = g|h
//      bit w-1:   t = a^b,            r = t^c      (carry out dropped)
//  - compound add (Sec. V-A-3), sum mod 2^w: the adder above with the XOR
//    and the AND of the same two bits from one compound node (one rotation,
//    two outputs): bit 0 (r, c) = (a^b, a&b); bit i (t, g) = (a^b, a&b),
//    (r, h) = (t^c, t&c), c = g|h; top bit t = a^b, r = t^c.  Three
//    rotations per middle bit instead of five.
//  - full-adder add, sum mod 2^w: bit 0 half adder (XOR, AND); bit i
//    r = XOR3(a, b, c), c = MAJ(a, b, c) (three-input gates, one level per
//    bit); top bit r = XOR3(a, b, c).
//  - number-wise add (GPU_n, Sec. V-B-1), sum mod 2^w: R = A, then w rounds
//    of carry = R & B, R = R ^ B, B = carry << 1, each round on the bits of B
//    not yet known zero (round k: bits k..w-1): w^2 gates in w levels.
//  - mul, low w bits: naive shift-and-add (Sec. III-B-1):
//      acc = A & b_0;  acc[i..w-1] += (A & b_i)[0..w-1-i] for i = 1..w-1
//  - mul with tree accumulation (Sec. V-B-2, Fig. 4), low w bits: partial
//    product i = (A & b_i) << i carries wires for bits i..w-1 only; the list
//    of partial products is split into first and second halves added
//    element-wise (an odd last element waits a round) until one is left.
//    Adding numbers whose known-zero low bits end at l < m copies bits
//    l..m-1 of the first and ripple-adds bits m..w-1.  Same gates as mul,
//    depth 62 instead of 120 at w = 32.
//  - Karatsuba (Sec. III-B-2, Algorithm 1), full 2w-bit product: below 16
//    bits the tree-accumulated full product (a sum keeps one bit more than
//    its wider operand, up to 2w); else with h = floor(w/2), Z0 = X0 Y0,
//    Z1 = X1 Y1, Z2 = (X0 + X1)(Y0 + Y1), M = Z2 - (Z0 + Z1) mod 2^(w+1)
//    (subtraction as x + ~y + 1: XNOR / ANDYN gates, the +1 folded into bit
//    0 as XOR / ORYN), Z = (Z0 | Z1 << 2h) + M << h.
//  - matmul, n x n, by Cannon's algorithm (Sec. V-B-3): cell (i, j) in cycle
//    t multiplies A[i][k] B[k][j], k = (i + j + t) mod n (the skew and the
//    per-cycle shifts only rename wires), with the tree multiplier, and adds
//    the product to its sum in cycle order with the ripple-carry adder.
//  - matvec: every product by mul; each row's products accumulated by the
//    tree of Sec. V-B-2 / Fig. 4: the list is split into first and second
//    halves that are added element-wise, an odd last element waits a round.
//
// Scheduling: every gate gets its ASAP level (1 + the later of its inputs'
// levels); levels are then balanced to whole launch rounds.
#include <algorithm>
#include <cstddef>

#include "fhe_internal.h"
#include "circuit_ir.h"

namespace fhe {

namespace {

constexpr size_t kKaratsubaBase = 16;  // narrower operands: base product

class Builder {
  public:
    Circuit c;
    Builder(uint32_t na, uint32_t nb) {
        c.na = na;
        c.nb = nb;
    }
    uint32_t gate(uint8_t op, uint32_t a, uint32_t b, uint32_t x = kNoWire) {
        const uint32_t o = c.na + c.nb + (uint32_t)c.gates.size();
        c.gates.push_back({op, a, b, o, x});
        return o;
    }
    // Compound node: (op0(a, b), op1(a, b)) from one rotation.
    void compound(uint8_t op0, uint8_t op1, uint32_t a, uint32_t b, uint32_t* o0, uint32_t* o1) {
        *o0 = gate(op0, a, b);
        *o1 = gate(op1, a, b);
        c.gates.back().second = true;
    }
    std::vector<uint32_t> add_compound(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
        const size_t w = a.size();
        std::vector<uint32_t> r(w);
        if (w == 0) return r;
        if (w == 1) {
            r[0] = gate(FHE_XOR, a[0], b[0]);
            return r;
        }
        uint32_t carry;
        compound(FHE_XOR, FHE_AND, a[0], b[0], &r[0], &carry);
        for (size_t i = 1; i < w; ++i) {
            if (i == w - 1) {
                const uint32_t t = gate(FHE_XOR, a[i], b[i]);
                r[i] = gate(FHE_XOR, t, carry);
                break;
            }
            uint32_t t, g, h;
            compound(FHE_XOR, FHE_AND, a[i], b[i], &t, &g);
            compound(FHE_XOR, FHE_AND, t, carry, &r[i], &h);
            carry = gate(FHE_OR, g, h);
        }
        return r;
    }
    // Ripple carry of full-adder gates: half adder, then XOR3 / MAJ per bit.
    std::vector<uint32_t> add_fa(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
        const size_t w = a.size();
        std::vector<uint32_t> r(w);
        if (w == 0) return r;
        r[0] = gate(FHE_XOR, a[0], b[0]);
        if (w == 1) return r;
        uint32_t carry = gate(FHE_AND, a[0], b[0]);
        for (size_t i = 1; i < w; ++i) {
            r[i] = gate(FHE_XOR3, a[i], b[i], carry);
            if (i + 1 < w) carry = gate(FHE_MAJ, a[i], b[i], carry);
        }
        return r;
    }
    std::vector<uint32_t> add(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
        const size_t w = a.size();
        std::vector<uint32_t> r(w);
        if (w == 0) return r;
        r[0] = gate(FHE_XOR, a[0], b[0]);
        if (w == 1) return r;
        uint32_t carry = gate(FHE_AND, a[0], b[0]);
        for (size_t i = 1; i < w; ++i) {
            const uint32_t t = gate(FHE_XOR, a[i], b[i]);
            if (i == w - 1) {
                r[i] = gate(FHE_XOR, t, carry);
                break;
            }
            const uint32_t g = gate(FHE_AND, a[i], b[i]);
            r[i] = gate(FHE_XOR, t, carry);
            const uint32_t h = gate(FHE_AND, t, carry);
            carry = gate(FHE_OR, g, h);
        }
        return r;
    }
    std::vector<uint32_t> add_numberwise(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
        const size_t w = a.size();
        std::vector<uint32_t> r(a), sh(b), carry(w);
        for (size_t k = 0; k < w; ++k) {
            for (size_t i = k; i + 1 < w; ++i) carry[i] = gate(FHE_AND, r[i], sh[i]);
            for (size_t i = k; i < w; ++i) r[i] = gate(FHE_XOR, r[i], sh[i]);
            for (size_t i = w - 1; i > k; --i) sh[i] = carry[i - 1];  // bit k of B is now zero
        }
        return r;
    }
    std::vector<uint32_t> mul(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
        const size_t w = a.size();
        std::vector<uint32_t> acc(w);
        for (size_t j = 0; j < w; ++j) acc[j] = gate(FHE_AND, a[j], b[0]);
        for (size_t i = 1; i < w; ++i) {
            std::vector<uint32_t> pp(w - i), hi(acc.begin() + i, acc.end());
            for (size_t j = 0; j < w - i; ++j) pp[j] = gate(FHE_AND, a[j], b[i]);
            const std::vector<uint32_t> s = add(hi, pp);
            std::copy(s.begin(), s.end(), acc.begin() + i);
        }
        return acc;
    }
    std::vector<uint32_t> mul_tree(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
        const size_t w = a.size();
        struct Part {
            size_t low;                  // bits below `low` are known zero
            std::vector<uint32_t> bits;  // wires of bits low..w-1
        };
        std::vector<Part> parts;
        for (size_t i = 0; i < w; ++i) {
            Part p{i, std::vector<uint32_t>(w - i)};
            for (size_t j = 0; j + i < w; ++j) p.bits[j] = gate(FHE_AND, a[j], b[i]);
            parts.push_back(std::move(p));
        }
        while (parts.size() > 1) {
            const size_t h = parts.size() / 2;
            std::vector<Part> next;
            for (size_t k = 0; k < h; ++k) {
                const Part* x = &parts[k];
                const Part* y = &parts[k + h];
                if (y->low < x->low) std::swap(x, y);
                const size_t skip = y->low - x->low;
                const std::vector<uint32_t> hi(x->bits.begin() + skip, x->bits.end());
                const std::vector<uint32_t> s = add(hi, y->bits);
                Part z{x->low, std::vector<uint32_t>(x->bits.begin(), x->bits.begin() + skip)};
                z.bits.insert(z.bits.end(), s.begin(), s.end());
                next.push_back(std::move(z));
            }
            if (parts.size() & 1) next.push_back(std::move(parts.back()));
            parts.swap(next);
        }
        return parts.empty() ? std::vector<uint32_t>() : parts[0].bits;
    }
    // x + y mod 2^len; missing high bits are zero.  The result can be
    // shorter than len when its top bits are known zero.
    std::vector<uint32_t> add_to(const std::vector<uint32_t>& x, const std::vector<uint32_t>& y, size_t len) {
        std::vector<uint32_t> r;
        bool have_c = false;
        uint32_t c = 0;
        for (size_t i = 0; i < len; ++i) {
            const bool hx = i < x.size(), hy = i < y.size(), more = i + 1 < len;
            bool next_c = false;
            uint32_t nc = 0;
            if (hx && hy) {
                const uint32_t t = gate(FHE_XOR, x[i], y[i]);
                if (!have_c) {
                    r.push_back(t);
                    if (more) { nc = gate(FHE_AND, x[i], y[i]); next_c = true; }
                } else {
                    r.push_back(gate(FHE_XOR, t, c));
                    if (more) {
                        const uint32_t g = gate(FHE_AND, x[i], y[i]);
                        const uint32_t h = gate(FHE_AND, t, c);
                        nc = gate(FHE_OR, g, h);
                        next_c = true;
                    }
                }
            } else if (hx || hy) {
                const uint32_t v = hx ? x[i] : y[i];
                if (!have_c) {
                    r.push_back(v);
                } else {
                    r.push_back(gate(FHE_XOR, v, c));
                    if (more) { nc = gate(FHE_AND, v, c); next_c = true; }
                }
            } else {
                if (!have_c) break;
                r.push_back(c);
            }
            have_c = next_c;
            c = nc;
        }
        return r;
    }
    // x - y mod 2^len (both len bits) as x + ~y + 1.
    std::vector<uint32_t> sub_to(const std::vector<uint32_t>& x, const std::vector<uint32_t>& y, size_t len) {
        std::vector<uint32_t> r(len);
        uint32_t c = 0;
        for (size_t i = 0; i < len; ++i) {
            const bool more = i + 1 < len;
            if (i == 0) {
                r[0] = gate(FHE_XOR, x[0], y[0]);
                if (more) c = gate(FHE_ORYN, x[0], y[0]);
                continue;
            }
            const uint32_t t = gate(FHE_XNOR, x[i], y[i]);
            r[i] = gate(FHE_XOR, t, c);
            if (more) {
                const uint32_t g = gate(FHE_ANDYN, x[i], y[i]);
                const uint32_t h = gate(FHE_AND, t, c);
                c = gate(FHE_OR, g, h);
            }
        }
        return r;
    }
    // Full 2m-bit product, partial products summed by the first/second-half
    // tree.
    std::vector<uint32_t> mul_full_tree(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
        const size_t m = a.size(), top_bits = 2 * m;
        struct Num {
            size_t low;
            std::vector<uint32_t> bits;
        };
        std::vector<Num> nums;
        for (size_t i = 0; i < m; ++i) {
            Num v{i, std::vector<uint32_t>(m)};
            for (size_t j = 0; j < m; ++j) v.bits[j] = gate(FHE_AND, a[j], b[i]);
            nums.push_back(std::move(v));
        }
        while (nums.size() > 1) {
            const size_t h = nums.size() / 2;
            std::vector<Num> next;
            for (size_t k = 0; k < h; ++k) {
                const Num* x = &nums[k];
                const Num* y = &nums[k + h];
                if (y->low < x->low) std::swap(x, y);
                const size_t skip = y->low - x->low;
                const size_t top = std::max(x->low + x->bits.size(), y->low + y->bits.size());
                const size_t len = std::min(top + 1, top_bits) - y->low;
                const std::vector<uint32_t> hi(x->bits.begin() + skip, x->bits.end());
                const std::vector<uint32_t> s = add_to(hi, y->bits, len);
                Num z{x->low, std::vector<uint32_t>(x->bits.begin(), x->bits.begin() + skip)};
                z.bits.insert(z.bits.end(), s.begin(), s.end());
                next.push_back(std::move(z));
            }
            if (nums.size() & 1) next.push_back(std::move(nums.back()));
            nums.swap(next);
        }
        return nums[0].bits;  // offset 0, 2m bits
    }
    std::vector<uint32_t> karatsuba(const std::vector<uint32_t>& x, const std::vector<uint32_t>& y) {
        const size_t n = x.size();
        if (n < kKaratsubaBase) return mul_full_tree(x, y);
        const size_t h = n / 2, u = n - h;
        const std::vector<uint32_t> x0(x.begin(), x.begin() + h), x1(x.begin() + h, x.end());
        const std::vector<uint32_t> y0(y.begin(), y.begin() + h), y1(y.begin() + h, y.end());
        const std::vector<uint32_t> z0 = karatsuba(x0, y0);  // 2h bits
        const std::vector<uint32_t> z1 = karatsuba(x1, y1);  // 2u bits
        const std::vector<uint32_t> z2 = karatsuba(add_to(x0, x1, u + 1), add_to(y0, y1, u + 1));
        const std::vector<uint32_t> p = add_to(z0, z1, n + 1);
        const std::vector<uint32_t> m = sub_to(std::vector<uint32_t>(z2.begin(), z2.begin() + n + 1), p, n + 1);
        std::vector<uint32_t> z(z0);
        z.insert(z.end(), z1.begin(), z1.end());  // Z0 | Z1 << 2h
        const std::vector<uint32_t> hi = add_to(std::vector<uint32_t>(z.begin() + h, z.end()), m, 2 * n - h);
        std::copy(hi.begin(), hi.end(), z.begin() + h);
        return z;
    }
    std::vector<uint32_t> tree_sum(std::vector<std::vector<uint32_t>> vals) {
        while (vals.size() > 1) {
            const size_t h = vals.size() / 2;
            std::vector<std::vector<uint32_t>> next;
            for (size_t k = 0; k < h; ++k) next.push_back(add(vals[k], vals[k + h]));
            if (vals.size() & 1) next.push_back(vals.back());
            vals.swap(next);
        }
        return vals.empty() ? std::vector<uint32_t>() : vals[0];
    }
};

}  // namespace

static std::vector<uint32_t> iota_wires(uint32_t first, uint32_t count) {
    std::vector<uint32_t> v(count);
    for (uint32_t k = 0; k < count; ++k) v[k] = first + k;
    return v;
}

Circuit build_circuit(int kind, uint32_t w, uint32_t rows, uint32_t cols) {
    if (kind == kMatmul) {  // rows = n
        const uint32_t n = rows;
        Builder B(n * n * w, n * n * w);
        for (uint32_t i = 0; i < n; ++i)
            for (uint32_t j = 0; j < n; ++j) {
                std::vector<uint32_t> c;
                for (uint32_t t = 0; t < n; ++t) {
                    const uint32_t k = (i + j + t) % n;
                    const std::vector<uint32_t> p =
                        B.mul_tree(iota_wires((i * n + k) * w, w), iota_wires(n * n * w + (k * n + j) * w, w));
                    c = t == 0 ? p : B.add(c, p);
                }
                B.c.outputs.insert(B.c.outputs.end(), c.begin(), c.end());
            }
        return B.c;
    }
    if (kind == kMatvec) {
        Builder B(rows * cols * w, cols * w);
        for (uint32_t r = 0; r < rows; ++r) {
            std::vector<std::vector<uint32_t>> prods;
            for (uint32_t c = 0; c < cols; ++c)
                prods.push_back(B.mul(iota_wires((r * cols + c) * w, w), iota_wires(rows * cols * w + c * w, w)));
            const std::vector<uint32_t> y = B.tree_sum(prods);
            B.c.outputs.insert(B.c.outputs.end(), y.begin(), y.end());
        }
        return B.c;
    }
    Builder B(w, w);
    const std::vector<uint32_t> a = iota_wires(0, w), b = iota_wires(w, w);
    B.c.outputs = kind == kAdd        ? B.add(a, b)
                  : kind == kAddCompound ? B.add_compound(a, b)
                  : kind == kAddNumberwise ? B.add_numberwise(a, b)
                  : kind == kAddFa     ? B.add_fa(a, b)
                  : kind == kMulTree  ? B.mul_tree(a, b)
                  : kind == kKaratsuba ? B.karatsuba(a, b)
                                       : B.mul(a, b);
    return B.c;
}

// ASAP level of every gate (inputs are level 0).
std::vector<uint32_t> asap_levels(const Circuit& c, uint32_t* depth) {
    std::vector<uint32_t> lev(c.wires(), 0);
    std::vector<uint32_t> glev(c.gates.size());
    uint32_t d = 0;
    for (size_t k = 0; k < c.gates.size(); ++k) {
        const Gate& g = c.gates[k];
        glev[k] = 1 + std::max(lev[g.in0], lev[g.in1]);
        if (g.in2 != kNoWire) glev[k] = std::max(glev[k], 1 + lev[g.in2]);
        lev[g.out] = glev[k];
        d = std::max(d, glev[k]);
    }
    *depth = d;
    return glev;
}

// Relative time of one launch of `gates` gates, in units of one round of the
// widest launch shape (`round` gates: eight per compute unit, two waves per
// SIMD), from the measured shape timings: a level of at most an eighth, a
// quarter or half a round runs on the narrower shapes in about 0.27, 0.36 and
// 0.64 of a round's time; wider levels take whole rounds.
static double level_cost(uint64_t gates, uint64_t round) {
    if (gates == 0) return 0.0;
    if (8 * gates <= round) return 0.27;
    if (4 * gates <= round) return 0.36;
    if (2 * gates <= round) return 0.64;
    return (double)((gates + round - 1) / round);
}

// List scheduling against the launch rounds: level by level, the ready gates
// that must run now (their ALAP level) fix the number of rounds the level
// takes, and the room left in its last round goes to the most urgent other
// ready gates (smallest ALAP level first).  A level whose urgent gates fill
// less than half a round runs on a narrower launch shape and is filled up to
// one round only when `fill_narrow`.  Gates become ready one level after
// their last input; the depth stays the critical path.
static std::vector<uint32_t> list_schedule(const Circuit& c, const std::vector<uint32_t>& alap,
                                           const std::vector<std::vector<uint32_t>>& cons, uint32_t depth,
                                           size_t count, uint64_t round, bool fill_narrow) {
    const size_t ng = c.gates.size();
    const uint32_t base = c.na + c.nb;
    std::vector<uint32_t> lev(ng, 0), pend(ng, 0);
    for (size_t k = 0; k < ng; ++k) {
        const Gate& g = c.gates[k];
        for (uint32_t w : {g.in0, g.in1, g.in2})
            if (w != kNoWire && w >= base) pend[k]++;
    }
    // ready gates by ALAP level; head[a] = first not yet taken in bucket a
    std::vector<std::vector<uint32_t>> bucket(depth + 2);
    std::vector<size_t> head(depth + 2, 0);
    for (size_t k = 0; k < ng; ++k)
        if (pend[k] == 0) bucket[alap[k]].push_back((uint32_t)k);
    std::vector<uint32_t> fresh;
    for (uint32_t L = 1; L <= depth; ++L) {
        fresh.clear();
        auto take = [&](uint32_t k) {
            lev[k] = L;
            for (uint32_t q : cons[k])
                if (--pend[q] == 0) fresh.push_back(q);
        };
        const uint64_t urgent = bucket[L].size() - head[L];
        const uint64_t g = urgent * count;
        uint64_t cap = urgent;  // gates per instance this level may take
        if (2 * g > round || (fill_narrow && g > 0)) {
            const uint64_t rounds = std::max<uint64_t>(1, (g + round - 1) / round);
            cap = std::max<uint64_t>(urgent, rounds * round / count);
        }
        while (head[L] < bucket[L].size()) take(bucket[L][head[L]++]);
        uint64_t room = cap - urgent;
        for (uint32_t a = L + 1; a <= depth && room > 0; ++a)
            while (room > 0 && head[a] < bucket[a].size()) {
                take(bucket[a][head[a]++]);
                room--;
            }
        for (uint32_t q : fresh) bucket[alap[q]].push_back(q);
    }
    return lev;
}

// Level balancing: ASAP levels put every gate whose inputs are ready at the
// earliest level (e.g. all partial products and operand XORs/ANDs at level
// 1), leaving the levels along the critical path narrow.  A gate with slack
// can run at any level between its ASAP level and its latest level (ALAP)
// as long as its inputs come from earlier levels and its consumers run
// later.  Levels (ascending) narrower than one round take the most urgent
// such gates until they hold one round; then levels whose last round is
// partly filled pass that overflow on to later levels with room (below).
// Of ASAP, filled and filled + trimmed the cost model's cheapest is kept.
// The depth and every gate's inputs and outputs are unchanged, so the words
// computed are too.
std::vector<uint32_t> balance_levels(const Circuit& c, const std::vector<uint32_t>& asap, uint32_t depth,
                                            size_t count, uint64_t round) {
    if (c.has_compound()) return asap;  // compound nodes keep their ASAP levels (moved only as pairs)
    const size_t ng = c.gates.size();
    const uint32_t base = c.na + c.nb;
    std::vector<std::vector<uint32_t>> cons(ng);
    for (size_t k = 0; k < ng; ++k) {
        const Gate& g = c.gates[k];
        for (uint32_t w : {g.in0, g.in1, g.in2})
            if (w != kNoWire && w >= base) cons[w - base].push_back((uint32_t)k);
    }
    std::vector<uint32_t> alap(ng, depth);
    for (size_t k = ng; k-- > 0;)
        for (uint32_t q : cons[k]) alap[k] = std::min(alap[k], alap[q] - 1);
    std::vector<uint32_t> slack;
    for (size_t k = 0; k < ng; ++k)
        if (alap[k] > asap[k]) slack.push_back((uint32_t)k);
    std::stable_sort(slack.begin(), slack.end(), [&](uint32_t a, uint32_t b) { return alap[a] < alap[b]; });
    std::vector<uint32_t> lev(asap);
    std::vector<uint64_t> width(depth + 1, 0);
    for (uint32_t l : lev) width[l]++;
    for (uint32_t L = 2; L <= depth; ++L) {
        for (uint32_t k : slack) {
            if ((width[L] + 1) * count > round) break;
            if (lev[k] >= L || alap[k] < L) continue;
            bool ok = true;
            for (uint32_t q : cons[k]) ok = ok && lev[q] > L;
            if (!ok) continue;
            width[lev[k]]--;
            width[L]++;
            lev[k] = L;
        }
    }
    const std::vector<uint32_t> filled(lev);
    // Trim: a level wider than a round whose last round is partly empty hands
    // that overflow (gates with slack, those with the most first) to the
    // earliest later level that has room below its own round boundary and
    // still precedes the gate's consumers.
    std::vector<std::vector<uint32_t>> at(depth + 2);
    for (size_t k = 0; k < ng; ++k) at[lev[k]].push_back((uint32_t)k);
    auto room = [&](uint32_t L) -> uint64_t {
        const uint64_t g = width[L] * count;
        const uint64_t cap = 2 * g > round ? (g + round - 1) / round * round : round;
        return cap - g;
    };
    for (uint32_t L = 1; L < depth; ++L) {
        const uint64_t g = width[L] * count;
        if (g <= round || g % round == 0) continue;
        uint64_t need = (g % round + count - 1) / count;
        std::vector<uint32_t> cand;
        for (uint32_t k : at[L])
            if (alap[k] > L) cand.push_back(k);
        std::stable_sort(cand.begin(), cand.end(), [&](uint32_t a, uint32_t b) { return alap[a] > alap[b]; });
        for (uint32_t k : cand) {
            if (need == 0) break;
            uint32_t lim = alap[k];
            for (uint32_t q : cons[k]) lim = std::min(lim, lev[q] - 1);
            for (uint32_t L2 = L + 1; L2 <= lim; ++L2) {
                if (room(L2) < count) continue;
                width[L]--;
                width[L2]++;
                lev[k] = L2;
                at[L2].push_back(k);
                need--;
                break;
            }
        }
    }
    // candidates: ASAP, filled, filled + trimmed, and list schedules with and
    // without filling narrow levels; the cheapest by the cost model is kept
    auto cost = [&](const std::vector<uint32_t>& l) {
        std::vector<uint64_t> w(depth + 1, 0);
        for (uint32_t x : l) w[x]++;
        double t = 0;
        for (uint32_t L = 1; L <= depth; ++L) t += level_cost(w[L] * count, round);
        return t;
    };
    std::vector<std::vector<uint32_t>> cand;
    cand.push_back(asap);
    cand.push_back(filled);
    cand.push_back(lev);
    cand.push_back(list_schedule(c, alap, cons, depth, count, round, false));
    cand.push_back(list_schedule(c, alap, cons, depth, count, round, true));
    size_t best = 0;
    double best_cost = cost(cand[0]);
    for (size_t i = 1; i < cand.size(); ++i) {
        const double t = cost(cand[i]);
        if (t < best_cost) {
            best_cost = t;
            best = i;
        }
    }
    return cand[best];
}

}  // namespace fhe

using namespace fhe;

// Host-only queries of the built-in circuits (no device involved).
extern "C" int fhe_circuit_schedule(int kind, uint32_t width, uint32_t rows, uint32_t cols, uint64_t count,
                                    uint32_t cu_count, uint64_t* level_gates, uint32_t max_levels, uint32_t* levels) {
    if (kind < 0 || kind > kLastKind || width < 1 || width > 64 || count == 0 || count > (1ull << 30) || cu_count == 0 ||
        (kind == kKaratsuba && width < 2) || (kind == kMatvec && (rows == 0 || cols == 0)) ||
        (kind == kMatmul && (rows == 0 || rows > 64)))
        return set_error(FHE_EINVAL, "fhe_circuit_schedule: bad arguments");
    const Circuit c = build_circuit(kind, width, rows, cols);
    uint32_t depth = 0;
    const std::vector<uint32_t> asap = asap_levels(c, &depth);
    const std::vector<uint32_t> lev = balance_levels(c, asap, depth, count, 8 * (uint64_t)cu_count);
    if (levels) *levels = depth;
    if (level_gates) {
        if (max_levels < depth) return set_error(FHE_EINVAL, "fhe_circuit_schedule: %u levels do not fit", depth);
        for (uint32_t L = 0; L < depth; ++L) level_gates[L] = 0;
        for (size_t k = 0; k < lev.size(); ++k)
            if (!c.gates[k].second) level_gates[lev[k] - 1] += count;
    }
    return FHE_OK;
}

extern "C" int fhe_circuit_shape(int kind, uint32_t width, uint32_t rows, uint32_t cols, uint64_t* gates,
                                 uint32_t* levels, uint64_t* widest_level) {
    if (kind < 0 || kind > kLastKind || width < 1 || (kind == kKaratsuba && width < 2) || width > 64 ||
        (kind == kMatvec && (rows == 0 || cols == 0)) || (kind == kMatmul && (rows == 0 || rows > 64)))
        return set_error(FHE_EINVAL, "fhe_circuit_shape: bad arguments");
    const Circuit c = build_circuit(kind, width, rows, cols);
    uint32_t depth = 0;
    const std::vector<uint32_t> glev = asap_levels(c, &depth);
    std::vector<uint64_t> per(depth + 1, 0);
    for (size_t k = 0; k < glev.size(); ++k)
        if (!c.gates[k].second) per[glev[k]]++;
    if (gates) *gates = c.bootstraps();
    if (levels) *levels = depth;
    if (widest_level) *widest_level = *std::max_element(per.begin(), per.end());
    return FHE_OK;
}

// Arithmetic in Z_p, p = 2^64 - 2^32 + 1, for the exact negacyclic NTT.
//
// Elements are kept canonical (uint64 in [0, p)).  The reductions use
// 2^64 = 2^32 - 1 and 2^96 = -1 (mod p); carries are detected by comparing
// a wrapped sum with one of its addends.
// Usable on the host (twiddle tables) and on gfx950.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define GL_FN __host__ __device__ __forceinline__
#else
#define GL_FN inline
#endif

namespace gl {

constexpr uint64_t P = 0xFFFFFFFF00000001ull;
constexpr uint64_t EPS = 0xFFFFFFFFull;  // 2^64 mod p

// Every function below takes and returns canonical values (in [0, p)).
// A carry (or borrow) is a 3-input boolean function of the top bits of the
// operands and of the wrapped result; on gfx950 that is one v_bitop3_b32,
// and an arithmetic shift turns its top bit into a 0 / 0xFFFFFFFF mask that
// is added back as 0 / EPS.  This keeps carries out of scalar lane masks
// (and the wait states their reuse costs).

GL_FN uint32_t hi32(uint64_t a) { return (uint32_t)(a >> 32); }

// Bitwise 3-input function with truth table `tt`: bit (a<<2 | b<<1 | c).
template <uint32_t TT>
GL_FN uint32_t bitop3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
#else
    uint32_t r = 0;
    for (int i = 0; i < 8; ++i)
        if ((TT >> i) & 1u)
            r |= ((i & 4) ? a : ~a) & ((i & 2) ? b : ~b) & ((i & 1) ? c : ~c);
    return r;
#endif
}

// 0 or 0xFFFFFFFF from the top bit of v.
GL_FN uint32_t top_mask(uint32_t v) { return (uint32_t)((int32_t)v >> 31); }

// x + (top bit of v) * EPS, for sums that cannot wrap.  On gfx950 this is a
// single v_mad_u64_u32 (bit * 0xFFFFFFFF + x); written out because the
// compiler otherwise turns the multiply into a mask and a 64-bit add that
// needs a zeroed register pair.  The instruction reads only VGPRs and its
// carry-out goes to a scalar pair nothing reads.
GL_FN uint64_t add_eps_if(uint64_t x, uint32_t v) {
    const uint32_t bit = v >> 31;
#if defined(__HIP_DEVICE_COMPILE__)
    uint64_t r, carry;
    asm("v_mad_u64_u32 %0, %1, %2, -1, %3" : "=v"(r), "=s"(carry) : "v"(bit), "v"(x));
    return r;
#else
    return x + (uint64_t)bit * EPS;
#endif
}

// The 64-bit value p * (top bit of v) mod 2^64 = -(bit * EPS): (bit, -bit).
GL_FN uint64_t p_if(uint32_t v) {
    const uint32_t bit = v >> 31;
    return ((uint64_t)(0u - bit) << 32) | bit;
}

// carry of s = a + b: (a & b) | ((a | b) & ~s) = majority(a, b, ~s)
constexpr uint32_t kCarryTT = 0xD4;
// borrow of d = a - b: (~a & b) | ((~a | b) & d) = majority(~a, b, d)
constexpr uint32_t kBorrowTT = 0x8E;
// a & ~b (c ignored)
constexpr uint32_t kAndNotTT = 0x30;

// x mod p for any 64-bit x: x >= p exactly when x + EPS wraps.
GL_FN uint64_t canon(uint64_t x) {
    const uint64_t t = x + EPS;
    return add_eps_if(x, bitop3<kAndNotTT>(hi32(x), hi32(t), hi32(t)));
}

// x + y: t = x + (y + EPS) wraps exactly when x + y >= p, and then the
// reduced sum is x + y + EPS (mod 2^64); otherwise it is x + y.
GL_FN uint64_t add(uint64_t x, uint64_t y) {
    const uint64_t y2 = y + EPS;  // < 2^64 because y < p
    const uint64_t t = x + y2;
    return add_eps_if(x + y, bitop3<kCarryTT>(hi32(x), hi32(y2), hi32(t)));
}

// x - y: on borrow add p = 2^64 - EPS, i.e. (lo + 1, hi + 0xFFFFFFFF).
GL_FN uint64_t sub(uint64_t x, uint64_t y) {
    const uint64_t d = x - y;
    return d + p_if(bitop3<kBorrowTT>(hi32(x), hi32(y), hi32(d)));
}

// (hi * 2^64 + lo) mod p for any hi, lo.  hi = hh*2^32 + hl:
// hh*2^96 = -hh and hl*2^64 = hl*(2^32 - 1).
GL_FN uint64_t reduce128(uint64_t hi, uint64_t lo) {
    const uint64_t hh = hi >> 32;
    const uint32_t hl = (uint32_t)hi;
    uint64_t t0 = lo - hh;
    // borrow iff lo < hh (< 2^32): then add p; lo - hh + 2^64 >= 2^64 - 2^32, no second wrap
    t0 += p_if(bitop3<kAndNotTT>(hi32(t0), hi32(lo), hi32(lo)));
    const uint64_t t1 = (uint64_t)hl * EPS;  // <= (2^32 - 1)^2 < p
    const uint64_t r = t0 + t1;              // a wrap leaves r < t1: + EPS cannot wrap again
    return canon(add_eps_if(r, bitop3<kCarryTT>(hi32(t0), hi32(t1), hi32(r))));
}

// 64 x 64 -> 128-bit product from four 32 x 32 -> 64 partial products.
GL_FN void mul_wide(uint64_t x, uint64_t y, uint64_t& hi, uint64_t& lo) {
    const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
    const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
    const uint64_t p00 = (uint64_t)x0 * y0;
    const uint64_t t = (uint64_t)x1 * y0 + (p00 >> 32);
    const uint64_t u = (uint64_t)x0 * y1 + (uint32_t)t;
    hi = (uint64_t)x1 * y1 + (t >> 32) + (u >> 32);
    lo = (u << 32) | (uint32_t)p00;
}

GL_FN uint64_t mul(uint64_t x, uint64_t y) {
    uint64_t hi, lo;
    mul_wide(x, y, hi, lo);
    return reduce128(hi, lo);
}

// x * 2^S for a compile-time S in [0, 96), by shifts: with the 32-bit limbs
// w0..w4 of x << S,  x 2^S = (w1:w0) + w2 (2^32 - 1) - (w4:w3)  (mod p).
template <int S>
GL_FN uint64_t mul_pow2(uint64_t x) {
    static_assert(S >= 0 && S < 96, "shift out of range");
    if constexpr (S == 0) {
        return x;
    } else if constexpr (S < 64) {
        const uint64_t A = x << S;                                   // (w1:w0)
        const uint64_t W = (uint64_t)(uint32_t)(x >> (64 - S)) * EPS;  // w2 (2^32 - 1) < p
        const uint64_t T = W + A;
        const uint64_t R = canon(add_eps_if(T, bitop3<kCarryTT>(hi32(W), hi32(A), hi32(T))));
        if constexpr (S <= 32) {
            return R;                                                // w3 = w4 = 0
        } else {
            return sub(R, (uint32_t)(x >> (96 - S)));                // - w3
        }
    } else {
        const uint64_t B = (uint64_t)(uint32_t)(x << (S - 64)) * EPS;  // w2 (2^32 - 1) < p
        return sub(B, x >> (96 - S));                                // - (w4:w3), < 2^63
    }
}

// Element of Z_p for a signed 64-bit integer of magnitude < p.
GL_FN uint64_t from_i64(int64_t v) {
    return v >= 0 ? (uint64_t)v : P - (uint64_t)(-v);
}

// Lift of a canonical r in [0, p) to its centred integer value mod 2^32:
// r <= (p-1)/2 stands for r itself, otherwise for r - p = r - 1 (mod 2^32).
GL_FN uint32_t lift32(uint64_t r) {
    return (uint32_t)r - (r > (P >> 1) ? 1u : 0u);
}

GL_FN uint64_t pow(uint64_t b, uint64_t e) {
    uint64_t r = 1;
    b = canon(b);
    while (e) {
        if (e & 1) r = mul(r, b);
        b = mul(b, b);
        e >>= 1;
    }
    return r;
}

}  // namespace gl

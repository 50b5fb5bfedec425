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
// Carries are read from the top bits (majority of the operands' and the
// complemented result's sign bits) and folded back with a multiply-add
// c * (2^32 - 1) + s, which on gfx950 keeps them out of scalar lane masks.

GL_FN uint32_t hi32(uint64_t a) { return (uint32_t)(a >> 32); }

// Carry out of the 64-bit sum s = a + b (mod 2^64), as 0 or 1.
GL_FN uint32_t carry64(uint64_t a, uint64_t b, uint64_t s) {
    const uint32_t a1 = hi32(a), b1 = hi32(b), s1 = hi32(s);
    return ((a1 & b1) | ((a1 | b1) & ~s1)) >> 31;
}

// x mod p for any 64-bit x: x >= p exactly when x + EPS wraps.
GL_FN uint64_t canon(uint64_t x) {
    const uint64_t t = x + EPS;
    return carry64(x, EPS, t) ? t : x;
}

// x + y: t = x + (y + EPS) wraps exactly when x + y >= p, and then t is the
// reduced sum; otherwise the sum is t - EPS.
GL_FN uint64_t add(uint64_t x, uint64_t y) {
    const uint64_t y2 = y + EPS;  // < 2^64 because y < p
    const uint64_t t = x + y2;
    return (uint64_t)carry64(x, y2, t) * EPS + (t - EPS);
}

// x - y: on borrow add p, i.e. subtract EPS modulo 2^64.
GL_FN uint64_t sub(uint64_t x, uint64_t y) {
    const uint64_t d = x - y;
    return d - (uint64_t)(x < y) * EPS;
}

// (hi * 2^64 + lo) mod p for any hi, lo.  hi = hh*2^32 + hl:
// hh*2^96 = -hh and hl*2^64 = hl*(2^32 - 1).
GL_FN uint64_t reduce128(uint64_t hi, uint64_t lo) {
    const uint64_t hh = hi >> 32;
    const uint32_t hl = (uint32_t)hi;
    uint64_t t0 = lo - hh;
    // borrow iff lo < hh (< 2^32); then lo - hh + 2^64 >= 2^64 - 2^32, no second wrap
    t0 -= (uint64_t)((~hi32(lo) & hi32(t0)) >> 31) * EPS;
    const uint64_t t1 = (uint64_t)hl * EPS;  // <= (2^32 - 1)^2 < p
    const uint64_t r = t0 + t1;              // a wrap leaves r < t1, + EPS cannot wrap again
    return canon((uint64_t)carry64(t0, t1, r) * EPS + r);
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
        const uint64_t A = x << S;                                      // (w1:w0)
        const uint64_t T = (uint64_t)(uint32_t)(x >> (64 - S)) * EPS + A;  // + w2 (2^32 - 1)
        const uint64_t R = canon((uint64_t)(T < A) * EPS + T);          // one wrap at most
        if constexpr (S <= 32) {
            return R;                                                   // w3 = w4 = 0
        } else {
            return sub(R, (uint32_t)(x >> (96 - S)));                   // - w3
        }
    } else {
        const uint64_t B = (uint64_t)(uint32_t)(x << (S - 64)) * EPS;   // w2 (2^32 - 1) < p
        return sub(B, x >> (96 - S));                                   // - (w4:w3), < 2^63
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

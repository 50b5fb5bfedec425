// Arithmetic in Z_p, p = 2^64 - 2^32 + 1, for the exact negacyclic NTT.
//
// Values are uint64 words congruent to the element mod p, not necessarily
// reduced below p ("loose" form); gl_canon() gives the representative in
// [0, p).  The reductions use 2^64 = 2^32 - 1 and 2^96 = -1 (mod p).
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

GL_FN uint64_t canon(uint64_t x) { return x >= P ? x - P : x; }

// x + y for loose x, y.
GL_FN uint64_t add(uint64_t x, uint64_t y) {
    uint64_t s = x + y;
    uint64_t c = (s < x) ? EPS : 0;  // 2^64 wrapped away: add it back as EPS
    s += c;
    s += (s < c) ? EPS : 0;          // second wrap (only when s >= p)
    return s;
}

// x - y for loose x, y.
GL_FN uint64_t sub(uint64_t x, uint64_t y) {
    uint64_t d = x - y;
    uint64_t b = (x < y) ? EPS : 0;  // 2^64 borrowed: remove it as EPS
    uint64_t d2 = d - b;
    d2 -= (d < b) ? EPS : 0;
    return d2;
}

// (hi * 2^64 + lo) mod p, loose.  hi = hh*2^32 + hl:
// hh*2^96 = -hh and hl*2^64 = hl*(2^32 - 1).
GL_FN uint64_t reduce128(uint64_t hi, uint64_t lo) {
    const uint64_t hh = hi >> 32, hl = hi & 0xFFFFFFFFull;
    uint64_t t0 = lo - hh;
    if (lo < hh) t0 -= EPS;          // lo - hh + 2^64 >= 2^64 - 2^32: no second wrap
    const uint64_t t1 = (hl << 32) - hl;
    uint64_t r = t0 + t1;
    if (r < t1) r += EPS;            // t0 + t1 - 2^64 < t1 <= 2^64 - 2^33 + 1
    return r;
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

// x * 2^S for a compile-time S in [0, 96), by limb shifts only:
// x << S spans five 32-bit limbs w0..w4, and
//   w0 + w1 2^32 + w2 2^64 + w3 2^96 + w4 2^128
//     = (w1:w0) + w2 (2^32 - 1) - (w4:w3)   (mod p).
template <int S>
GL_FN uint64_t mul_pow2(uint64_t x) {
    static_assert(S >= 0 && S < 96, "shift out of range");
    if constexpr (S == 0) {
        return x;
    } else {
        constexpr int q = S / 32, r = S % 32;
        const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
        uint32_t u0, u1, u2;
        if constexpr (r == 0) {
            u0 = x0; u1 = x1; u2 = 0;
        } else {
            u0 = x0 << r;
            u1 = (x1 << r) | (x0 >> (32 - r));
            u2 = x1 >> (32 - r);
        }
        uint32_t w[5] = {0, 0, 0, 0, 0};
        w[q] = u0;
        w[q + 1] = u1;
        w[q + 2] = u2;
        const uint64_t lo = ((uint64_t)w[1] << 32) | w[0];
        const uint64_t mid = ((uint64_t)w[2] << 32) - w[2];   // w2 * (2^32 - 1)
        const uint64_t top = ((uint64_t)w[4] << 32) | w[3];
        uint64_t s = lo + mid;
        if (s < mid) s += EPS;                                 // no second wrap (mid <= p - 2^32)
        return sub(s, top);
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
        if (e & 1) r = canon(mul(r, b));
        b = canon(mul(b, b));
        e >>= 1;
    }
    return r;
}

}  // namespace gl

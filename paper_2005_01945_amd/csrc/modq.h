// Arithmetic modulo two 28-bit NTT primes, for the exact negacyclic products
// of the CMux computed with 32-bit integer operations.
//
// q0 = 268369921 = 2^28 - 2^16 + 1 and q1 = 268367873 are primes with
// q = 1 (mod 2048), so Z_q holds a primitive 2048-th root psi and the
// negacyclic NTT of length 1024.  A coefficient of a summed CMux product is an
// integer of magnitude at most 2^52 < q0 q1 / 2 (about 2^55), so its residues
// modulo q0 and q1 determine it exactly (Chinese remainder theorem), and with
// it the result modulo 2^32.
//
// Values are signed 32-bit residues.  Products use signed Montgomery
// reduction with R = 2^32 (Seiler, "Faster AVX2 optimized NTT multiplication
// for Ring-LWE lattice cryptography", 2018): for |a| < q 2^31,
//   m = (a mod 2^32) q^-1 mod 2^32 (as int32),  mont(a) = (a - m q) / 2^32,
// is congruent to a R^-1 and lies in (-q, q).  Constants are stored in the
// Montgomery form c R mod q, centred, so mul(v, cR) = mont(v cR) = v c.
// Three VALU instructions on gfx950: v_mad_i64_i32, v_mul_lo_u32,
// v_mad_i64_i32.
//
// Butterflies add and subtract without reduction; the transforms below carry
// a compile-time bound (in units of q) for every value and reduce only where a
// sum could leave |x| < 8q < 2^31.
#pragma once

#include <cstdint>
#include <type_traits>

#if defined(__HIPCC__)
#define MQ_FN __host__ __device__ __forceinline__
#else
#define MQ_FN inline
#endif

namespace mq {

constexpr uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
    uint64_t r = 1;
    b %= q;
    while (e) {
        if (e & 1) r = r * b % q;
        b = b * b % q;
        e >>= 1;
    }
    return r;
}

// q^-1 mod 2^32 for odd q (Newton iteration, each step doubles the bits).
constexpr uint32_t inv32(uint32_t q) {
    uint32_t x = q;  // correct to 3 bits
    for (int i = 0; i < 5; ++i) x *= 2u - q * x;
    return x;
}

// c mod q as a signed residue in (-q/2, q/2].
constexpr int32_t centred(uint64_t c, uint32_t q) {
    const uint64_t r = c % q;
    return r > q / 2 ? (int32_t)((int64_t)r - (int64_t)q) : (int32_t)r;
}

template <int I>
struct Prime;

template <>
struct Prime<0> {
    static constexpr uint32_t q = 268369921u;
    static constexpr uint32_t psi = 135902522u;  // 11^((q-1)/2048), order 2048
};

template <>
struct Prime<1> {
    static constexpr uint32_t q = 268367873u;
    static constexpr uint32_t psi = 16675871u;  // 3^((q-1)/2048), order 2048
};

template <int I>
struct Mod {
    static constexpr uint32_t q = Prime<I>::q;
    static constexpr uint32_t psi = Prime<I>::psi;
    static constexpr uint32_t qinv = inv32(q);
    static constexpr uint64_t R = (uint64_t)1 << 32;
    static_assert(q < (1u << 28), "bounds assume q < 2^28");
    static_assert(q % 2048 == 1, "needs 2048-th roots of unity");
    static_assert(q * qinv == 1u, "q^-1 mod 2^32");
    static_assert(powmod(psi, 1024, q) == q - 1, "psi has order 2048");
    // Montgomery form of c, centred.
    static constexpr int32_t rform(uint64_t c) { return centred((c % q) * (R % q), q); }
    // psi^e for any integer e (order 2048).
    static constexpr uint64_t psi_pow(int64_t e) {
        return powmod(psi, (uint64_t)(((e % 2048) + 2048) % 2048), q);
    }
    // Montgomery forms of rho^e, rho = psi^32, e = 0..63.
    struct RhoTable {
        int32_t v[64];
    };
    static constexpr RhoTable make_rho() {
        RhoTable t{};
        for (int e = 0; e < 64; ++e) t.v[e] = rform(psi_pow(32 * e));
        return t;
    }
    static constexpr RhoTable rho = make_rho();
};

// Signed Montgomery reduction of |a| < q 2^31: congruent to a 2^-32, in (-q, q).
template <int I>
MQ_FN int32_t mont(int64_t a) {
    const int32_t m = (int32_t)((uint32_t)a * Mod<I>::qinv);
    return (int32_t)((a - (int64_t)m * (int64_t)Mod<I>::q) >> 32);
}

// v * c for w = c R mod q (|v| < 2^31, |w| <= q/2).
template <int I>
MQ_FN int32_t mul(int32_t v, int32_t w) {
    return mont<I>((int64_t)v * w);
}

// The constant W, materialised in a scalar register where it is used.  The
// transforms use about a hundred distinct twiddles; left to itself the
// compiler hoists them out of the CMux loop into vector registers, which
// then spill.  An s_mov_b32 per use costs a scalar slot, not a vector one.
template <int32_t W>
MQ_FN int32_t sconst() {
#if defined(__HIP_DEVICE_COMPILE__)
    int32_t r;
    asm volatile("s_mov_b32 %0, %1" : "=s"(r) : "i"(W));
    return r;
#else
    return W;
#endif
}

// A value of magnitude < 2^31 reduced to (-q, q).
template <int I>
MQ_FN int32_t reduce(int32_t v) {
    return mul<I>(v, sconst<Mod<I>::rform(1)>());
}

// ---------------------------------------------------------------------------
// 32-point transforms over the 32 registers of a lane.
//
// Two shapes, both Cooley-Tukey (the twiddle multiplies the second input
// before the butterfly, so value bounds grow additively):
//   kNeg, kCycFwd, kCycInv: natural order in, bit-reversed order out.  Stage
//     L (0..4) has 2^L blocks of 16 >> L butterflies; block i twiddles with
//     rho^e(L, i), rho = psi^32 (a primitive 64-th root of unity):
//       kNeg    e = brv5(2^L + i)                negacyclic: out[brv5(k)] =
//                                                sum_m x_m rho^(m(2k+1))
//       kCycFwd e = 2 brv_L(i) (16 >> L)         cyclic, root rho^2:
//                                                out[brv5(k)] = sum_m x_m rho^(2mk)
//       kCycInv e = -2 brv_L(i) (16 >> L)        cyclic, root rho^-2
//   kDitInv: bit-reversed order in, natural order out, cyclic with root
//     rho^-2: span h = 1, 2, ..., 16, butterfly j < h twiddles with
//     rho^(-2 j (16 / h)).
// ---------------------------------------------------------------------------

enum Kind { kNeg = 0, kCycFwd = 1, kCycInv = 2, kDitInv = 3 };

constexpr int brv_bits(int x, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b)
        if (x & (1 << b)) r |= 1 << (bits - 1 - b);
    return r;
}

// Exponent of rho = psi^32 used by butterfly k (0..15) of stage L.
constexpr int tw_exp(int kind, int L, int k) {
    if (kind == kDitInv) {
        const int h = 1 << L, j = k % h;
        return -2 * j * (16 / h);
    }
    const int tt = 16 >> L, i = k / tt;
    if (kind == kNeg) return brv_bits((1 << L) + i, 5);
    const int e = L == 0 ? 0 : 2 * brv_bits(i, L) * (16 >> L);
    return kind == kCycFwd ? e : -e;
}

// Register indices (u, v) of butterfly k of stage L.
constexpr int bf_u(int kind, int L, int k) {
    if (kind == kDitInv) {
        const int h = 1 << L;
        return (k / h) * 2 * h + k % h;
    }
    const int tt = 16 >> L;
    return (k / tt) * 2 * tt + k % tt;
}
constexpr int bf_v(int kind, int L, int k) {
    return bf_u(kind, L, k) + (kind == kDitInv ? (1 << L) : (16 >> L));
}

constexpr bool trivial(int e) { return ((e % 64) + 64) % 64 == 0; }

// Reduction plan: which inputs of which butterflies are reduced first, from
// bounds in units of q (a reduced or twiddled value is below 1 q; sums add
// bounds; every value must stay at most 8 q).  A trivial twiddle's input is
// reduced only when needed, then the other input.
struct Plan {
    bool red_u[5][16];
    bool red_v[5][16];
    int out_bound;
};

constexpr Plan make_plan(int kind, int in_bound) {
    Plan p{};
    int b[32] = {};
    for (int r = 0; r < 32; ++r) b[r] = in_bound;
    for (int L = 0; L < 5; ++L) {
        for (int k = 0; k < 16; ++k) {
            const int u = bf_u(kind, L, k), v = bf_v(kind, L, k);
            int bu = b[u], bv = b[v];
            if (!trivial(tw_exp(kind, L, k))) bv = 1;
            if (bu + bv > 8 && bv > 1) {
                bv = 1;
                p.red_v[L][k] = true;
            }
            if (bu + bv > 8) {
                bu = 1;
                p.red_u[L][k] = true;
            }
            b[u] = b[v] = bu + bv;
        }
    }
    int mx = 0;
    for (int r = 0; r < 32; ++r) mx = b[r] > mx ? b[r] : mx;
    p.out_bound = mx;
    return p;
}

template <int KIND, int IN>
struct PlanOf {
    static constexpr Plan value = make_plan(KIND, IN);
};

// Scheduling fence on the device (keeps the compiler from interleaving
// stages, which bounds the registers in flight); nothing on the host.
MQ_FN void stage_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_sched_barrier(0);
#endif
}

template <int B, int E, class F>
MQ_FN void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// First butterfly of stage L that uses the same twiddle as butterfly k.
constexpr int first_same_tw(int kind, int L, int k) {
    for (int j = 0; j < k; ++j)
        if (((tw_exp(kind, L, j) - tw_exp(kind, L, k)) % 64) == 0) return j;
    return k;
}

// The 32-point transform KIND of the 32 registers x (modulo q_I), inputs
// bounded by IN q; outputs are bounded by PlanOf<KIND, IN>::value.out_bound q.
// Each stage first materialises its distinct twiddles (2^L of them, 31 per
// transform) in scalar registers.
template <int I, int KIND, int IN>
MQ_FN void ntt32(int32_t (&x)[32]) {
    using P = PlanOf<KIND, IN>;
#if defined(__HIP_DEVICE_COMPILE__)
    // A wave in a transform (VALU only) takes issue priority over its SIMD's
    // other wave, which meanwhile runs its LDS and memory phases.
    __builtin_amdgcn_s_setprio(1);
#endif
    static_for<0, 5>([&](auto L_) {
        constexpr int L = decltype(L_)::value;
        stage_fence();
        int32_t w[16];
        static_for<0, 16>([&](auto K_) {
            constexpr int k = decltype(K_)::value;
            constexpr int e = ((tw_exp(KIND, L, k) % 64) + 64) % 64;
            constexpr int f = first_same_tw(KIND, L, k);
            if constexpr (e != 0 && f == k) w[k] = sconst<Mod<I>::rho.v[e]>();
            else if constexpr (e != 0) w[k] = w[f];
        });
        constexpr bool any_red = [] {
            for (int k = 0; k < 16; ++k)
                if (P::value.red_u[L][k] || P::value.red_v[L][k]) return true;
            return false;
        }();
        int32_t one = 0;  // R mod q: a Montgomery product with it reduces
        if constexpr (any_red) one = sconst<Mod<I>::rform(1)>();
        // Montgomery products of the stage in three phases (products,
        // quotients, reductions), each over all butterflies, so that
        // dependent instructions are 16 apart.
        int64_t pv[16], pu[16];
        int32_t mv[16], mu[16];
        static_for<0, 16>([&](auto K_) {
            constexpr int k = decltype(K_)::value;
            constexpr int u = bf_u(KIND, L, k), v = bf_v(KIND, L, k);
            constexpr int e = ((tw_exp(KIND, L, k) % 64) + 64) % 64;
            if constexpr (e != 0) pv[k] = (int64_t)x[v] * w[k];
            else if constexpr (P::value.red_v[L][k]) pv[k] = (int64_t)x[v] * one;
            if constexpr (P::value.red_u[L][k]) pu[k] = (int64_t)x[u] * one;
        });
        stage_fence();
        static_for<0, 16>([&](auto K_) {
            constexpr int k = decltype(K_)::value;
            constexpr int e = ((tw_exp(KIND, L, k) % 64) + 64) % 64;
            if constexpr (e != 0 || P::value.red_v[L][k]) mv[k] = (int32_t)((uint32_t)pv[k] * Mod<I>::qinv);
            if constexpr (P::value.red_u[L][k]) mu[k] = (int32_t)((uint32_t)pu[k] * Mod<I>::qinv);
        });
        stage_fence();
        static_for<0, 16>([&](auto K_) {
            constexpr int k = decltype(K_)::value;
            constexpr int u = bf_u(KIND, L, k), v = bf_v(KIND, L, k);
            constexpr int e = ((tw_exp(KIND, L, k) % 64) + 64) % 64;
            if constexpr (e != 0 || P::value.red_v[L][k])
                x[v] = (int32_t)((pv[k] - (int64_t)mv[k] * (int64_t)Mod<I>::q) >> 32);
            if constexpr (P::value.red_u[L][k])
                x[u] = (int32_t)((pu[k] - (int64_t)mu[k] * (int64_t)Mod<I>::q) >> 32);
        });
        stage_fence();
        static_for<0, 16>([&](auto K_) {
            constexpr int k = decltype(K_)::value;
            constexpr int u = bf_u(KIND, L, k), v = bf_v(KIND, L, k);
            const int32_t U = x[u], V = x[v];
            x[u] = U + V;
            x[v] = U - V;
        });
    });
    stage_fence();
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_s_setprio(0);
#endif
}

}  // namespace mq

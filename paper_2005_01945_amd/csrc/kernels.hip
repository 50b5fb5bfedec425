// gfx950 kernels of TFHE gate bootstrapping.
//
// Arithmetic: the negacyclic products of the CMux external product are done
// as an exact NTT over Z_p, p = 2^64 - 2^32 + 1.  Digits are in [-512, 511]
// and key words are read as signed 32-bit, so every coefficient of a summed
// product is below 4 * 1024 * 2^9 * 2^31 = 2^52 < p/2 in magnitude and lifts
// back to Z/2^32 exactly: results equal the schoolbook definition bit for bit.
//
// Work layout: one wavefront (64 lanes) bootstraps one gate; its accumulator
// (two polynomials of 1024 uint32) lives in LDS.  Lane l = 32h + t (half h,
// t < 32) transforms polynomial data of coefficients m = t + 32*q, held in
// register q (q < 32).  A 1024-point negacyclic
// NTT is split 32 x 32: a 32-point negacyclic transform in registers over q
// (root psi^32 = 8, so every twiddle is a power of two: shifts only), one
// general twiddle psi^(t(2j+1)) per value, a transpose through LDS, and a
// 32-point cyclic transform in registers (root psi^64 = 2^6).  After it, lane
// (h, t) register q holds frequency k = t + 32*brv5(q).  The inverse runs the
// same steps backwards; N^-1 is folded into its twiddles.
//
// CMux i (TFHE blind rotation): D = X^abar_i ACC - ACC; each half extracts
// its own gadget digit (half h -> digit h) of polynomial hp = 0, 1 in two
// passes, transforms it, swaps it with the other half (v_permlane32_swap),
// and half h accumulates output column h against BK_i in the NTT domain.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fhe_internal.h"
#include "goldilocks.h"
#include "kernels.h"
#include "modq.h"

namespace fhe {
namespace dev {
namespace {

constexpr int N = 1024;
constexpr int NW = 501;            // LWE sample words
constexpr int NLWE = 500;
constexpr uint32_t kDecompOffset = 0x80200800u;  // 2^31 + 2^21 + 2^11

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

__host__ __device__ constexpr int brv5(int x) {
    return ((x & 1) << 4) | ((x & 2) << 2) | (x & 4) | ((x & 8) >> 2) | ((x & 16) >> 4);
}

// ---------------------------------------------------------------------------
// 32-point transforms in registers.
// ---------------------------------------------------------------------------

// Negacyclic forward, root psi2 = 8 (order 64), natural in, bit-reversed out:
// out[q] = sum_i x[i] psi2^(i (2 brv5(q) + 1)).  Merged Cooley-Tukey.
__device__ __forceinline__ void ntt32_neg_fwd(uint64_t (&x)[32]) {
    static_for<0, 5>([&](auto L) {
        constexpr int m = 1 << decltype(L)::value;
        constexpr int t = 16 >> decltype(L)::value;
        static_for<0, m>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int S = 3 * brv5(m + i);
            static_for<0, t>([&](auto J) {
                constexpr int j = 2 * i * t + decltype(J)::value;
                const uint64_t U = x[j];
                const uint64_t V = gl::mul_pow2<S>(x[j + t]);
                x[j] = gl::add(U, V);
                x[j + t] = gl::sub(U, V);
            });
        });
    });
}

// Cyclic forward, root w = 2^6 (order 32), natural in, bit-reversed out.
// Decimation in frequency.
__device__ __forceinline__ void ntt32_cyc_fwd(uint64_t (&x)[32]) {
    static_for<0, 5>([&](auto L) {
        constexpr int ln = 16 >> decltype(L)::value;
        static_for<0, 16 / ln>([&](auto B) {
            constexpr int st = 2 * ln * decltype(B)::value;
            static_for<0, ln>([&](auto J) {
                constexpr int j = decltype(J)::value;
                constexpr int S = 6 * j * (16 / ln);
                const uint64_t U = x[st + j], V = x[st + j + ln];
                x[st + j] = gl::add(U, V);
                x[st + j + ln] = gl::mul_pow2<S>(gl::sub(U, V));
            });
        });
    });
}

// Inverse of ntt32_cyc_fwd without the 1/32: bit-reversed in, natural out.
// w^-s = -2^(96-s).
__device__ __forceinline__ void ntt32_cyc_inv(uint64_t (&x)[32]) {
    static_for<0, 5>([&](auto L) {
        constexpr int ln = 1 << decltype(L)::value;
        static_for<0, 16 / ln>([&](auto B) {
            constexpr int st = 2 * ln * decltype(B)::value;
            static_for<0, ln>([&](auto J) {
                constexpr int j = decltype(J)::value;
                constexpr int S = 6 * j * (16 / ln);
                const uint64_t U = x[st + j], V = x[st + j + ln];
                if constexpr (S == 0) {
                    x[st + j] = gl::add(U, V);
                    x[st + j + ln] = gl::sub(U, V);
                } else {
                    const uint64_t W = gl::mul_pow2<96 - S>(V);
                    x[st + j] = gl::sub(U, W);
                    x[st + j + ln] = gl::add(U, W);
                }
            });
        });
    });
}

// Inverse of ntt32_neg_fwd without the 1/32: bit-reversed in, natural out.
// Gentleman-Sande; psi2^-e = -2^(96-e), so (U - V) psi2^-e = (V - U) 2^(96-e).
__device__ __forceinline__ void ntt32_neg_inv(uint64_t (&x)[32]) {
    static_for<0, 5>([&](auto L) {
        constexpr int t = 1 << decltype(L)::value;
        constexpr int h = 16 >> decltype(L)::value;
        static_for<0, h>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int E = 3 * brv5(h + i);
            static_for<0, t>([&](auto J) {
                constexpr int j = 2 * t * i + decltype(J)::value;
                const uint64_t U = x[j], V = x[j + t];
                x[j] = gl::add(U, V);
                x[j + t] = gl::mul_pow2<96 - E>(gl::sub(V, U));
            });
        });
    });
}

// Scheduling fence: keeps the compiler from hoisting the loads of later
// chunks above it, which bounds the registers held by loads in flight.
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// Orders the wave's LDS traffic: LDS operations of one wavefront execute in
// issue order, so a compiler-level barrier is all a wave-private exchange
// needs.
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// Word t of an LDS array as an LDS address the optimiser cannot see through,
// so that the 32 reads at t + 32 q share one base register held in the loop
// (otherwise it hoists a base per pair of reads and spills them).
__device__ __forceinline__ const lds_u32* lds_column(const uint32_t* a, int t) {
    const lds_u32* p = (const lds_u32*)(a + t);
    asm volatile("" : "+v"(p));
    return p;
}

// Gadget digit of coefficient m of D = X^ai ACC - ACC for this half (digit
// h of two: bits 22..31 for h = 0, 12..21 for h = 1), in [-512, 511], from
// d4 = 4 (m - ai).  d4 needs no reduction: its bits 2..11 are (m - ai) mod
// 1024 times 4, the byte offset of the word read, and its bit 12 tells
// whether (m - ai) mod 2048 >= 1024 (X^N = -1: the word is negated), for
// negative m - ai too.  doff is the rounding offset of both digits plus
// 2^(shift + 9), which makes the signed 10-bit field equal to the unsigned
// field minus 512.
__device__ __forceinline__ uint32_t digit_offset(int h) { return kDecompOffset + (1u << (31 - 10 * h)); }

// The digit in two halves, so that the reads can run ahead of the digits:
// the word's LDS address, with abase the byte address of the polynomial (a
// multiple of 4096), is one AND-OR; the digit comes from the word v read
// there and the unrotated word own.  The negation is written (v + sgn) ^
// sgn, which needs the mask alone (the form (v ^ sgn) - sgn makes the
// optimiser build -sgn as a second, zero-extended bit): bit-field extract,
// add, XOR-add, subtract per coefficient.
__device__ __forceinline__ uint32_t rotated_word(uint32_t abase, int d4) {
    return *(const lds_u32*)(uintptr_t)(((uint32_t)d4 & 0xFFCu) | abase);
}

__device__ __forceinline__ int32_t rotated_digit_q(uint32_t v, uint32_t own, int d4, uint32_t doff, int shift) {
    const uint32_t sgn = (uint32_t)__builtin_amdgcn_sbfe(d4, 12, 1);
    return __builtin_amdgcn_sbfe((int32_t)(((v + sgn) ^ sgn) + (doff - own)), shift, 10);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 32 x 32 transpose of 64-bit values through this half's 4 KB tile of
// 32-bit words, one word of each value at a time.  Element (row, col) sits at
// row*32 + (col ^ row), which keeps both the row writes and the column reads
// free of bank conflicts.  Before: register k holds (row wr(k), col t); after:
// register k holds (row t, col rd(k)).
template <class WR, class RD>
__device__ __forceinline__ void transpose32(uint64_t (&x)[32], uint32_t* tile, int t, WR wr, RD rd) {
    uint32_t lo[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) tile[wr(k) * 32 + (t ^ wr(k))] = (uint32_t)x[k];
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < 32; ++k) lo[k] = tile[t * 32 + (rd(k) ^ t)];
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < 32; ++k) tile[wr(k) * 32 + (t ^ wr(k))] = (uint32_t)(x[k] >> 32);
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < 32; ++k) x[k] = ((uint64_t)tile[t * 32 + (rd(k) ^ t)] << 32) | lo[k];
    wave_lds_sync();
}

// Full 1024-point forward negacyclic NTT of this half's polynomial.
__device__ __forceinline__ void ntt1024_fwd(uint64_t (&x)[32], uint32_t* tile,
                                            const uint64_t* twf, int t) {
    ntt32_neg_fwd(x);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        sched_fence();
#pragma unroll
        for (int q = 8 * c; q < 8 * c + 8; ++q) x[q] = gl::mul(x[q], twf[q * 32 + t]);
    }
    sched_fence();
    transpose32(x, tile, t, [](int q) { return brv5(q); }, [](int r) { return r; });
    ntt32_cyc_fwd(x);
}

// Inverse of ntt1024_fwd including N^-1 (folded in twi).
__device__ __forceinline__ void ntt1024_inv(uint64_t (&x)[32], uint32_t* tile,
                                            const uint64_t* twi, int t) {
    ntt32_cyc_inv(x);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        sched_fence();
#pragma unroll
        for (int r = 8 * c; r < 8 * c + 8; ++r) x[r] = gl::mul(x[r], twi[r * 32 + t]);
    }
    sched_fence();
    transpose32(x, tile, t, [](int r) { return r; }, [](int q) { return brv5(q); });
    ntt32_neg_inv(x);
}

// Value of the other half's lane with the same t.
__device__ __forceinline__ uint32_t partner32(uint32_t v, int h) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return h ? r[0] : r[1];
}

__device__ __forceinline__ uint64_t partner64(uint64_t v, int h) {
    const uint32_t lo = partner32((uint32_t)v, h);
    const uint32_t hi = partner32((uint32_t)(v >> 32), h);
    return ((uint64_t)hi << 32) | lo;
}

// Per-wave LDS, as views into the block's arrays: the accumulator (two
// polynomials of 1024 words) and one 32 x 32 transpose tile of 32-bit words
// per half (TW words: 32 x 32 with an XOR swizzle for the Goldilocks path,
// 32 x 36 padded rows for the two-prime path).  16 KB (17 KB).
template <int TW>
struct WaveLdsT {
    uint32_t (&acc)[2][1024];
    uint32_t (&tile)[2][TW];
};
using WaveLds = WaveLdsT<32 * 32>;

template <int A>
constexpr int kTileWords = A == 1 ? 32 * 36 : 32 * 32;

// Shared-memory footprint of a block of WPB one-wave gates: twiddles plus one
// accumulator and one pair of tiles per wave (WPB = 4 with the Goldilocks
// path: 80 KB, so two blocks fit a CU's 160 KB, i.e. two waves per SIMD;
// WPB = 8 with the two-prime path: 152 KB, one block of two waves per SIMD).
// Every accumulator polynomial starts at a multiple of 4 KB (rotated_digit_q).
template <int WPB, int A>
struct alignas(4096) BlockLds {
    uint64_t twf[32 * 32];
    uint64_t twi[32 * 32];
    uint32_t acc[WPB][2][1024];
    uint32_t tile[WPB][2][kTileWords<A>];
};
using BlockLds81 = BlockLds<8, 1>;
static_assert(offsetof(BlockLds81, acc) % 4096 == 0, "accumulators must be 4 KB aligned");

// Shared memory of one gate bootstrapped by two waves (56 KB): wave w runs
// pass w of every CMux; wave 1 hands its multiply-accumulate result to wave 0
// through `part`, and wave 0 finishes the step.
template <int A>
struct alignas(4096) PairLds {
    uint64_t twf[32 * 32];
    uint64_t twi[32 * 32];
    uint32_t acc[2][1024];
    uint32_t tile[2][2][kTileWords<A>];  // [wave][half]
    uint64_t part[32][64];               // [register q][lane]
};
static_assert(offsetof(PairLds<1>, acc) % 4096 == 0, "accumulators must be 4 KB aligned");

// Shared memory of one gate bootstrapped by four waves (two-prime arithmetic
// only, 74 KB): wave w = 2 hp + prime runs pass hp in that prime; the pass-1
// waves hand their column sums to the pass-0 waves through `part`, which
// finish their prime; wave 1 hands its residues to wave 0, which recombines.
struct alignas(4096) QuadLds {
    uint64_t twf[32 * 32];
    uint64_t twi[32 * 32];
    uint32_t acc[2][1024];
    uint32_t tile[4][2][32 * 36];  // [wave][half]
    int32_t part[2][32][64];       // [prime][register][lane]
};
static_assert(offsetof(QuadLds, acc) % 4096 == 0, "accumulators must be 4 KB aligned");

// Pass HP of a CMux step: D = X^ai ACC_HP - ACC_HP (a = ACC_HP), this half's
// gadget digit of it (half h extracts digit h), its forward NTT, then the
// multiply-accumulate against BK_i rows (2HP + h) and (2HP + 1 - h), column h,
// added to mac when ACCUM (else stored).  tile: this half's transpose tile;
// bk_i: BK_i in the kernel layout [hp][q][sel][64 lanes].  PREFETCH issues
// the 64 key loads before the digit extraction so that their latency hides
// behind the forward NTT (128 more registers live across it).
template <int HP, bool ACCUM, bool PREFETCH>
__device__ __forceinline__ void cmux_pass(const uint32_t* a, uint32_t* tile, int ai,
                                          const uint64_t* __restrict__ bk_i,
                                          const uint64_t* twf, int lane, uint64_t (&mac)[32]) {
    const int h = lane >> 5, t = lane & 31;
    const int shift = 22 - 10 * h;
    uint64_t b_pre[PREFETCH ? 64 : 1];
    if constexpr (PREFETCH) {
        const uint64_t* bkp = bk_i + (size_t)HP * (32 * 2 * 64) + lane;
#pragma unroll
        for (int k = 0; k < 64; ++k) b_pre[k] = bkp[k * 64];
    }
    uint64_t x[32];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        sched_fence();
#pragma unroll
        for (int q = 8 * c; q < 8 * c + 8; ++q) {
            const int m = t + 32 * q;
            const int s = (m - ai) & 2047;
            const uint32_t v = a[s & 1023];
            const uint32_t rot = (s & 1024) ? 0u - v : v;
            const uint32_t D = rot - a[m];
            const int32_t dg = (int32_t)(((D + kDecompOffset) >> shift) & 1023u) - 512;
            x[q] = gl::from_i64(dg);
        }
    }
    sched_fence();
    ntt1024_fwd(x, tile, twf, t);
    const uint64_t* bkp = bk_i + (size_t)HP * (32 * 2 * 64) + lane;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        sched_fence();
#pragma unroll
        for (int q = 4 * c; q < 4 * c + 4; ++q) {
            const uint64_t other = partner64(x[q], h);
            uint64_t b_own, b_oth;
            if constexpr (PREFETCH) {
                b_own = b_pre[q * 2 + 0];
                b_oth = b_pre[q * 2 + 1];
            } else {
                b_own = bkp[(q * 2 + 0) * 64];
                b_oth = bkp[(q * 2 + 1) * 64];
            }
            const uint64_t v = gl::add(gl::mul(x[q], b_own), gl::mul(other, b_oth));
            mac[q] = ACCUM ? gl::add(mac[q], v) : v;
        }
    }
    sched_fence();
}

// Inverse NTT of the two output columns (half h: column h) and ACC += their
// lift to Z/2^32.
__device__ __forceinline__ void cmux_finish(uint32_t (&acc)[2][1024], uint32_t* tile,
                                            uint64_t (&mac)[32], const uint64_t* twi, int lane) {
    const int h = lane >> 5, t = lane & 31;
    ntt1024_inv(mac, tile, twi, t);
    uint32_t* mine = acc[h];
#pragma unroll
    for (int q = 0; q < 32; ++q) mine[t + 32 * q] += gl::lift32(mac[q]);
}

// One CMux step on this wave's accumulator W.acc:
//   ACC += BK_i [x] (X^ai ACC - ACC).
__device__ __forceinline__ void cmux_step(WaveLds& W, int ai, const uint64_t* __restrict__ bk_i,
                                          const uint64_t* twf, const uint64_t* twi, int lane) {
    const int h = lane >> 5;
    uint64_t mac[32];
    cmux_pass<0, false, false>(W.acc[0], W.tile[h], ai, bk_i, twf, lane, mac);
    cmux_pass<1, true, false>(W.acc[1], W.tile[h], ai, bk_i, twf, lane, mac);
    cmux_finish(W.acc, W.tile[h], mac, twi, lane);
    wave_lds_sync();
}

// ---------------------------------------------------------------------------
// The same CMux with the products computed modulo two 28-bit primes q0, q1
// (modq.h) and recombined by the Chinese remainder theorem.  A 64-bit
// multiply-accumulate value holds the prime-0 residue in its low word and the
// prime-1 residue in its high word (signed 32-bit each); BK is in the
// Montgomery form c R mod q with |c| <= q/2, in the 32-bit layout
// [i][hp][prime][q / 2][lane 32c + t][q % 2][digit]: the four words of a
// lane's register pair (2 registers x 2 digits) are one 16-byte load.
// Twiddle tables (LDS, int32): forward [prime][q][t] = psi^(t(2 brv5(q)+1)) R,
// inverse [prime][r][j] = psi^(-r(2j+1)) N^-1 R.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int32_t lo_of(uint64_t v) { return (int32_t)(uint32_t)v; }
__device__ __forceinline__ int32_t hi_of(uint64_t v) { return (int32_t)(uint32_t)(v >> 32); }
__device__ __forceinline__ uint64_t pack2(int32_t a, int32_t b) {
    return ((uint64_t)(uint32_t)b << 32) | (uint32_t)a;
}

// 32 x 32 transpose of 32-bit values through a tile of 32 rows of 36 words:
// element (row, col) at row*36 + col.  Column writes hit 32 consecutive
// words per row; each lane reads its row as eight 16-byte loads, and the
// rows' 4-word skew spreads eight lanes' loads over all 32 banks.  Every
// address is a per-lane base (t or 36 t) plus a constant, so no per-register
// address is kept live.  Before: register k holds (row wr(k), col t); after:
// register k holds (row t, col k).
template <class WR>
__device__ __forceinline__ void transpose32_w(int32_t (&x)[32], uint32_t* tile, int t, WR wr) {
    uint32_t* col = tile + t;  // this lane's column
    // This lane's row, as an LDS address opaque to the optimiser: otherwise
    // it hoists one base address per pair of reads out of the CMux loop and
    // spills them.  (Kept in the LDS address space so that the reads are LDS
    // instructions, which wait on LDS traffic only.)
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) v4u lds_u4;
    lds_u4* row = (lds_u4*)(tile + 36 * t);
    asm volatile("" : "+v"(row));
    // LDS phases take the highest issue priority (the transforms have 1): a
    // wave about to wait on LDS gets its requests out first, then the SIMD's
    // other wave computes under the latency
    __builtin_amdgcn_s_setprio(2);
#pragma unroll
    for (int k = 0; k < 32; ++k) col[wr(k) * 36] = (uint32_t)x[k];
    wave_lds_sync();
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        const v4u v = row[g];
        x[4 * g + 0] = (int32_t)v.x;
        x[4 * g + 1] = (int32_t)v.y;
        x[4 * g + 2] = (int32_t)v.z;
        x[4 * g + 3] = (int32_t)v.w;
    }
    __builtin_amdgcn_s_setprio(0);
    wave_lds_sync();
}

// x[B..B+8) *= w[0..8) (Montgomery forms), in three phases (products,
// quotients, reductions) so that dependent instructions are 8 apart.
template <int I, int B>
__device__ __forceinline__ void mul8_q(int32_t (&x)[32], const int32_t (&w)[8]) {
    int64_t p[8];
    int32_t m[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = (int64_t)x[B + k] * w[k];
    sched_fence();
#pragma unroll
    for (int k = 0; k < 8; ++k) m[k] = (int32_t)((uint32_t)p[k] * mq::Mod<I>::qinv);
    sched_fence();
#pragma unroll
    for (int k = 0; k < 8; ++k) x[B + k] = (int32_t)((p[k] - (int64_t)m[k] * (int64_t)mq::Mod<I>::q) >> 32);
    sched_fence();
}

// Table twiddles: x[q] *= tw[q * 32 + t], eight at a time.
template <int I>
__device__ __forceinline__ void table_mul_q(int32_t (&x)[32], const int32_t* tw, int t) {
    int32_t w[2][8];  // the twiddles of chunk c + 1 are read before chunk c is multiplied
#pragma unroll
    for (int k = 0; k < 8; ++k) w[0][k] = tw[k * 32 + t];
    mq::static_for<0, 4>([&](auto C_) {
        constexpr int c = decltype(C_)::value;
        if constexpr (c < 3) {
#pragma unroll
            for (int k = 0; k < 8; ++k) w[(c + 1) & 1][k] = tw[(8 * c + 8 + k) * 32 + t];
        }
        mul8_q<I, 8 * c>(x, w[c & 1]);
    });
}

// Forward 1024-point negacyclic NTT modulo q_I of this half's polynomial
// (|x| < q in); lane t, register r then holds frequency t + 32 brv5(r),
// bounded by 7 q.
template <int I>
__device__ __forceinline__ void ntt1024_fwd_q(int32_t (&x)[32], uint32_t* tile, const int32_t* twf, int t) {
    mq::ntt32<I, mq::kNeg, 1>(x);
    table_mul_q<I>(x, twf, t);
    transpose32_w(x, tile, t, [](int q) { return brv5(q); });
    mq::ntt32<I, mq::kCycFwd, 1>(x);
}

// Inverse, from the forward's layout with |x| < 2q: lane t, register r then
// holds the residue (|.| < q) of coefficient t + 32 brv5(r).
template <int I>
__device__ __forceinline__ void ntt1024_inv_q(int32_t (&x)[32], uint32_t* tile, const int32_t* twi, int t) {
    mq::ntt32<I, mq::kDitInv, 2>(x);
    table_mul_q<I>(x, twi, t);
    transpose32_w(x, tile, t, [](int r) { return r; });
    mq::ntt32<I, mq::kCycInv, 1>(x);
    // negacyclic twist psi^(-32 q) of output q = brv5(r): rho^(-q)
    mq::static_for<0, 4>([&](auto C_) {
        constexpr int c = decltype(C_)::value;
        int32_t w[8];
        mq::static_for<0, 8>([&](auto K_) {
            constexpr int r = 8 * c + decltype(K_)::value;
            w[decltype(K_)::value] = mq::sconst<mq::Mod<I>::rho.v[(64 - brv5(r)) % 64]>();
        });
        mul8_q<I, 8 * c>(x, w);
    });
}

// Multiply-accumulate of prime I for pass HP: column h of the products of the
// two digit transforms (r0: digit 0, half 0's; r1: digit 1, half 1's, both
// obtained with one v_permlane32_swap) with BK rows 2HP and 2HP + 1.
// bk: the prime-I plane of BK_i for pass HP, [q / 2][64 lanes][q % 2][digit] words, in
// 8 chunks of 4 registers (8 words).  Key loads run W chunks ahead of their
// use; the first W chunks (`pre`) were issued before the forward transform.
template <int W>
struct KeyWindow {
    uint32_t w[W + 1 > 8 ? 8 : W + 1][8];
};

template <int W>
__device__ __forceinline__ void prefetch_q(const uint32_t* __restrict__ bk, int lane, KeyWindow<W>& kw) {
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const uint4 v = *reinterpret_cast<const uint4*>(bk + ((2 * c + u) * 64 + lane) * 4);
            kw.w[c][4 * u + 0] = v.x;
            kw.w[c][4 * u + 1] = v.y;
            kw.w[c][4 * u + 2] = v.z;
            kw.w[c][4 * u + 3] = v.w;
        }
}

template <int I, bool ACCUM, int W>
__device__ __forceinline__ void mac_q(const int32_t (&x)[32], const uint32_t* __restrict__ bk,
                                      KeyWindow<W>& kw, int lane, int32_t (&mac)[32]) {
    constexpr int R = W + 1 > 8 ? 8 : W + 1;  // ring slots
    mq::static_for<0, 8>([&](auto C_) {
        constexpr int c = decltype(C_)::value;
        if constexpr (c + W < 8) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const uint4 v = *reinterpret_cast<const uint4*>(bk + ((2 * (c + W) + u) * 64 + lane) * 4);
                kw.w[(c + W) % R][4 * u + 0] = v.x;
                kw.w[(c + W) % R][4 * u + 1] = v.y;
                kw.w[(c + W) % R][4 * u + 2] = v.z;
                kw.w[(c + W) % R][4 * u + 3] = v.w;
            }
        }
        sched_fence();
        // phases: exchanges, first products, second products, quotients,
        // reductions (dependent instructions four apart)
        int32_t d0[4], d1[4], m[4];
        int64_t p[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const auto sw = __builtin_amdgcn_permlane32_swap((uint32_t)x[4 * c + j], (uint32_t)x[4 * c + j], false, false);
            d0[j] = (int32_t)sw[0];
            d1[j] = (int32_t)sw[1];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) p[j] = (int64_t)d0[j] * (int32_t)kw.w[c % R][2 * j];
        sched_fence();
#pragma unroll
        for (int j = 0; j < 4; ++j) p[j] += (int64_t)d1[j] * (int32_t)kw.w[c % R][2 * j + 1];
        sched_fence();
#pragma unroll
        for (int j = 0; j < 4; ++j) m[j] = (int32_t)((uint32_t)p[j] * mq::Mod<I>::qinv);
        sched_fence();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t v = (int32_t)((p[j] - (int64_t)m[j] * (int64_t)mq::Mod<I>::q) >> 32);
            mac[4 * c + j] = ACCUM ? mac[4 * c + j] + v : v;
        }
    });
    sched_fence();
}

// Pass HP of a CMux step with two-prime products (see cmux_pass): digits of
// ACC_HP (half h: digit h), then for each prime in turn its transform and
// multiply-accumulate of column h.  The digits wait for the second prime
// packed two to a register.  mac: low word prime 0, high word prime 1, each
// |.| < q per pass.  bk_i: BK_i, [hp][prime][q / 2][64 lanes][q % 2][digit] words.
// W: key-load window in chunks (8: all loads issued before the transform).
template <int HP, bool ACCUM, int W>
__device__ __forceinline__ void cmux_pass_q(const uint32_t* a, uint32_t* tile, int ai,
                                            const uint64_t* __restrict__ bk_i, const int32_t* twf,
                                            int lane, uint64_t (&mac)[32]) {
    const int h = lane >> 5, t = lane & 31;
    const int shift = 22 - 10 * h;
    const uint32_t doff = digit_offset(h);
    const lds_u32* am = lds_column(a, t);
    const uint32_t abase = (uint32_t)(uintptr_t)(const lds_u32*)a;
    int d4 = 4 * (t - ai);  // opaque: each pass forms its own addresses instead of keeping them
    asm volatile("" : "+v"(d4));
    const uint32_t* bk0 = reinterpret_cast<const uint32_t*>(bk_i) + HP * 8192;
    const uint32_t* bk1 = bk0 + 4096;
    KeyWindow<W> kw;
    prefetch_q<W>(bk0, lane, kw);
    int32_t x[32];
    uint32_t dp[16];
    // the reads of chunk c + 1 are issued before the digits of chunk c
    uint32_t rv[2][8], ow[2][8];
    int dq[2][8];
    auto issue = [&](auto C_, auto B_) {
        constexpr int c = decltype(C_)::value, b = decltype(B_)::value;
        __builtin_amdgcn_s_setprio(2);  // as in transpose32_w
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = 8 * c + k;
            dq[b][k] = d4 + 128 * q;
            rv[b][k] = rotated_word(abase, dq[b][k]);
            ow[b][k] = am[32 * q];
        }
        __builtin_amdgcn_s_setprio(0);
    };
    issue(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    mq::static_for<0, 4>([&](auto C_) {
        constexpr int c = decltype(C_)::value;
        sched_fence();
        if constexpr (c < 3) issue(std::integral_constant<int, c + 1>{}, std::integral_constant<int, (c + 1) & 1>{});
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = 8 * c + k;
            x[q] = rotated_digit_q(rv[c & 1][k], ow[c & 1][k], dq[c & 1][k], doff, shift);
        }
#pragma unroll
        for (int j = 4 * c; j < 4 * c + 4; ++j)
            dp[j] = ((uint32_t)x[2 * j] & 0xFFFFu) | ((uint32_t)x[2 * j + 1] << 16);
    });
    sched_fence();
    int32_t m0[32], m1[32];
    if constexpr (ACCUM) {
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            m0[q] = lo_of(mac[q]);
            m1[q] = hi_of(mac[q]);
        }
    }
    ntt1024_fwd_q<0>(x, tile, twf, t);
    mac_q<0, ACCUM, W>(x, bk0, kw, lane, m0);
    prefetch_q<W>(bk1, lane, kw);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        x[2 * j] = (int32_t)(dp[j] << 16) >> 16;
        x[2 * j + 1] = (int32_t)dp[j] >> 16;
    }
    ntt1024_fwd_q<1>(x, tile, twf + 1024, t);
    mac_q<1, ACCUM, W>(x, bk1, kw, lane, m1);
#pragma unroll
    for (int q = 0; q < 32; ++q) mac[q] = pack2(m0[q], m1[q]);
}

// Inverse NTTs of both columns (half h: column h), CRT, ACC += result.
// One prime's share of pass HP (the four-wave shape): the digits of ACC_HP,
// their transform modulo q_I and the multiply-accumulate of column h.
template <int HP, int I, int W>
__device__ __forceinline__ void cmux_pass_q1(const uint32_t* a, uint32_t* tile, int ai,
                                             const uint64_t* __restrict__ bk_i, const int32_t* twf,
                                             int lane, int32_t (&mac)[32]) {
    const int h = lane >> 5, t = lane & 31;
    const int shift = 22 - 10 * h;
    const uint32_t doff = digit_offset(h);
    const lds_u32* am = lds_column(a, t);
    const uint32_t abase = (uint32_t)(uintptr_t)(const lds_u32*)a;
    int d4 = 4 * (t - ai);  // opaque: the pass forms its own addresses instead of keeping them
    asm volatile("" : "+v"(d4));
    const uint32_t* bk = reinterpret_cast<const uint32_t*>(bk_i) + HP * 8192 + I * 4096;
    KeyWindow<W> kw;
    prefetch_q<W>(bk, lane, kw);
    int32_t x[32];
    // the reads of chunk c + 1 are issued before the digits of chunk c
    uint32_t rv[2][8], ow[2][8];
    int dq[2][8];
    auto issue = [&](auto C_, auto B_) {
        constexpr int c = decltype(C_)::value, b = decltype(B_)::value;
        __builtin_amdgcn_s_setprio(2);  // as in transpose32_w
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = 8 * c + k;
            dq[b][k] = d4 + 128 * q;
            rv[b][k] = rotated_word(abase, dq[b][k]);
            ow[b][k] = am[32 * q];
        }
        __builtin_amdgcn_s_setprio(0);
    };
    issue(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
    mq::static_for<0, 4>([&](auto C_) {
        constexpr int c = decltype(C_)::value;
        sched_fence();
        if constexpr (c < 3) issue(std::integral_constant<int, c + 1>{}, std::integral_constant<int, (c + 1) & 1>{});
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = 8 * c + k;
            x[q] = rotated_digit_q(rv[c & 1][k], ow[c & 1][k], dq[c & 1][k], doff, shift);
        }
    });
    sched_fence();
    ntt1024_fwd_q<I>(x, tile, twf + I * 1024, t);
    mac_q<I, false, W>(x, bk, kw, lane, mac);
}

__device__ __forceinline__ void crt_update_q(uint32_t (&acc)[2][1024], const int32_t (&x0)[32],
                                             const int32_t (&x1)[32], int lane);

__device__ __forceinline__ void cmux_finish_q(uint32_t (&acc)[2][1024], uint32_t* tile,
                                              uint64_t (&mac)[32], const int32_t* twi, int lane) {
    const int t = lane & 31;
    int32_t x0[32], x1[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        x0[q] = lo_of(mac[q]);
        x1[q] = hi_of(mac[q]);
    }
    ntt1024_inv_q<0>(x0, tile, twi, t);
    ntt1024_inv_q<1>(x1, tile, twi + 1024, t);
    crt_update_q(acc, x0, x1, lane);
}

// ACC (half h: polynomial h) += the column given by its residues x0, x1
// (register r: coefficient t + 32 brv5(r)).
// Registers 8C..8C+7 of the CRT update below (x0, x1: those registers'
// residues; old: their accumulator words, read ahead by the caller).  The
// constants come in scalar registers (crt_consts), so that
// the optimiser keeps the products as multiplies instead of expanding them
// into shifts and adds of the 2^28 - 2^16 + ... forms of the primes.
struct CrtConsts {
    int32_t q0, nq1, cq;  // q0, -q1, q0^-1 R mod q1 (centred)
};

__device__ __forceinline__ CrtConsts crt_consts() {
    constexpr int32_t cq = mq::Mod<1>::rform(mq::powmod(mq::Mod<0>::q, mq::Mod<1>::q - 2, mq::Mod<1>::q));
    return {mq::sconst<(int32_t)mq::Mod<0>::q>(), mq::sconst<-(int32_t)mq::Mod<1>::q>(), mq::sconst<cq>()};
}

template <int C>
__device__ __forceinline__ void crt_chunk_core(uint32_t (&acc)[2][1024], const int32_t (&x0)[8],
                                               const int32_t (&x1)[8], int lane, const CrtConsts& K,
                                               const uint32_t (&old)[8]) {
    const int h = lane >> 5, t = lane & 31;
    uint32_t* mine = acc[h] + t;
    int32_t d[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        d[k] = x1[k];
        asm volatile("" : "+v"(d[k]));  // keeps the subtraction 32-bit (the optimiser folds it into
        d[k] -= x0[k];                    // the preceding Montgomery reduction as a 64-bit one)
    }
    sched_fence();
    int64_t p[8];
    int32_t m[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = (int64_t)d[k] * K.cq;
    sched_fence();
#pragma unroll
    for (int k = 0; k < 8; ++k) m[k] = (int32_t)((uint32_t)p[k] * mq::Mod<1>::qinv);
    sched_fence();
#pragma unroll
    for (int k = 0; k < 8; ++k) d[k] = (int32_t)((p[k] + (int64_t)m[k] * K.nq1) >> 32);
    sched_fence();
#pragma unroll
    for (int k = 0; k < 8; ++k) mine[32 * brv5(8 * C + k)] = old[k] + (uint32_t)x0[k] + (uint32_t)K.q0 * (uint32_t)d[k];
    sched_fence();
}

// The same, reading the chunk's accumulator words itself.
template <int C>
__device__ __forceinline__ void crt_chunk_q(uint32_t (&acc)[2][1024], const int32_t (&x0)[8],
                                            const int32_t (&x1)[8], int lane, const CrtConsts& K) {
    const uint32_t* mine = acc[lane >> 5] + (lane & 31);
    uint32_t old[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) old[k] = mine[32 * brv5(8 * C + k)];
    crt_chunk_core<C>(acc, x0, x1, lane, K, old);
}

// Residues (|v0| < q0, |v1| < q1) of an integer V with |V| <= 2^52 ->
// V mod 2^32: V = v0 + q0 T with T = (v1 - v0) q0^-1 mod q1 taken in
// (-q1/2, q1/2); in fact |T| <= (2^52 + q0) / q0 < 2^24 + 2^13.  The Montgomery
// product t = mont((v1 - v0) cq), cq = q0^-1 R mod q1 centred, is that T
// without any correction: |v1 - v0| < 2^29 and |cq| <= q1/2 < 2^27 bound the
// product by 2^56, so |t| < 2^56 / 2^32 + q1/2 < 2^24 + q1/2, and t and T,
// congruent modulo q1, differ by less than 2^25 + 2^13 + q1/2 < q1: t = T.
// ACC[h][t + 32 brv5(r)] += V.  Eight registers at a time, in phases.
__device__ __forceinline__ void crt_update_q(uint32_t (&acc)[2][1024], const int32_t (&x0)[32],
                                             const int32_t (&x1)[32], int lane) {
    const CrtConsts K = crt_consts();
    const uint32_t* mine = acc[lane >> 5] + (lane & 31);
    uint32_t old[2][8];  // the words of chunk c + 1 are read before chunk c is updated
#pragma unroll
    for (int k = 0; k < 8; ++k) old[0][k] = mine[32 * brv5(k)];
    mq::static_for<0, 4>([&](auto C_) {
        constexpr int c = decltype(C_)::value;
        if constexpr (c < 3) {
#pragma unroll
            for (int k = 0; k < 8; ++k) old[(c + 1) & 1][k] = mine[32 * brv5(8 * c + 8 + k)];
        }
        int32_t a0[8], a1[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a0[k] = x0[8 * c + k];
            a1[k] = x1[8 * c + k];
        }
        crt_chunk_core<c>(acc, a0, a1, lane, K, old[c & 1]);
    });
}

template <int KW>
__device__ __forceinline__ void cmux_step_q(WaveLdsT<32 * 36>& W, int ai, const uint64_t* __restrict__ bk_i,
                                            const int32_t* twf, const int32_t* twi, int lane) {
    const int h = lane >> 5;
    uint64_t mac[32];
    cmux_pass_q<0, false, KW>(W.acc[0], W.tile[h], ai, bk_i, twf, lane, mac);
    cmux_pass_q<1, true, KW>(W.acc[1], W.tile[h], ai, bk_i, twf, lane, mac);
    cmux_finish_q(W.acc, W.tile[h], mac, twi, lane);
    wave_lds_sync();
}

// Arithmetic selector of the blind-rotation kernels: 0 = Goldilocks NTT,
// 1 = two-prime NTT.
template <int A>
struct Arith;

template <>
struct Arith<0> {
    __host__ __device__ static const uint64_t* bk(const DeviceKeys& K) { return K.bkd; }
    __host__ __device__ static const uint64_t* twf(const DeviceKeys& K) { return K.twf; }
    __host__ __device__ static const uint64_t* twi(const DeviceKeys& K) { return K.twi; }
    template <int KW>
    __device__ __forceinline__ static void step(WaveLds& W, int ai, const uint64_t* bk_i, const uint64_t* twf,
                                const uint64_t* twi, int lane) {
        cmux_step(W, ai, bk_i, twf, twi, lane);
    }
    template <int HP, int KW>
    __device__ __forceinline__ static void pass(const uint32_t* a, uint32_t* tile, int ai, const uint64_t* bk_i,
                                const uint64_t* twf, int lane, uint64_t (&mac)[32]) {
        cmux_pass<HP, false, true>(a, tile, ai, bk_i, twf, lane, mac);  // (two-wave shape only)
    }
    __device__ __forceinline__ static uint64_t add(uint64_t x, uint64_t y) { return gl::add(x, y); }
    __device__ __forceinline__ static void finish(uint32_t (&acc)[2][1024], uint32_t* tile, uint64_t (&mac)[32],
                                  const uint64_t* twi, int lane) {
        cmux_finish(acc, tile, mac, twi, lane);
    }
};

template <>
struct Arith<1> {
    __host__ __device__ static const uint64_t* bk(const DeviceKeys& K) { return K.bkq; }
    __host__ __device__ static const uint64_t* twf(const DeviceKeys& K) { return K.twfq; }
    __host__ __device__ static const uint64_t* twi(const DeviceKeys& K) { return K.twiq; }
    template <int KW>
    __device__ __forceinline__ static void step(WaveLdsT<32 * 36>& W, int ai, const uint64_t* bk_i, const uint64_t* twf,
                                const uint64_t* twi, int lane) {
        cmux_step_q<KW>(W, ai, bk_i, reinterpret_cast<const int32_t*>(twf),
                    reinterpret_cast<const int32_t*>(twi), lane);
    }
    template <int HP, int KW>
    __device__ __forceinline__ static void pass(const uint32_t* a, uint32_t* tile, int ai, const uint64_t* bk_i,
                                const uint64_t* twf, int lane, uint64_t (&mac)[32]) {
        cmux_pass_q<HP, false, KW>(a, tile, ai, bk_i, reinterpret_cast<const int32_t*>(twf), lane, mac);
    }
    __device__ __forceinline__ static uint64_t add(uint64_t x, uint64_t y) {
        return pack2(lo_of(x) + lo_of(y), hi_of(x) + hi_of(y));
    }
    __device__ __forceinline__ static void finish(uint32_t (&acc)[2][1024], uint32_t* tile, uint64_t (&mac)[32],
                                  const uint64_t* twi, int lane) {
        cmux_finish_q(acc, tile, mac, reinterpret_cast<const int32_t*>(twi), lane);
    }
};

// Gate constants: phase offset kappa and input signs (TFHE +-1/8 encoding)
// of the two-input codes 0..9.
__device__ __forceinline__ void gate_consts(uint32_t op, uint32_t& kappa, int32_t& s1, int32_t& s2) {
    constexpr uint32_t mu = kMu;
    switch (op) {
    case FHE_AND:   kappa = 0u - mu;      s1 = 1;  s2 = 1;  break;
    case FHE_NAND:  kappa = mu;           s1 = -1; s2 = -1; break;
    case FHE_OR:    kappa = mu;           s1 = 1;  s2 = 1;  break;
    case FHE_NOR:   kappa = 0u - mu;      s1 = -1; s2 = -1; break;
    case FHE_XOR:   kappa = 2u * mu;      s1 = 2;  s2 = 2;  break;
    case FHE_XNOR:  kappa = 0u - 2u * mu; s1 = -2; s2 = -2; break;
    case FHE_ANDNY: kappa = 0u - mu;      s1 = -1; s2 = 1;  break;
    case FHE_ANDYN: kappa = 0u - mu;      s1 = 1;  s2 = -1; break;
    case FHE_ORNY:  kappa = mu;           s1 = -1; s2 = 1;  break;
    default:        kappa = mu;           s1 = 1;  s2 = -1; break;  // FHE_ORYN
    }
}

// Value (+1 true, -1 false) of a symmetric two-input code with k of its two
// inputs true; 0 for a code that is not symmetric (compound gates take
// AND, NAND, OR, NOR, XOR, XNOR).
__device__ __forceinline__ int32_t sym_value(uint32_t op, int k) {
    switch (op) {
    case FHE_AND:  return k == 2 ? 1 : -1;
    case FHE_NAND: return k == 2 ? -1 : 1;
    case FHE_OR:   return k >= 1 ? 1 : -1;
    case FHE_NOR:  return k >= 1 ? -1 : 1;
    case FHE_XOR:  return k == 1 ? 1 : -1;
    case FHE_XNOR: return k == 1 ? -1 : 1;
    default:       return 0;
    }
}

// What gate g of a batch computes (uniform over the wave).
struct GateMode {
    uint32_t op0, op1;  // code; second code of a compound gate
    bool compound;      // two symmetric gates from one rotation
    bool three;         // MAJ / XOR3 with a third input
    bool valid;
};

__device__ __forceinline__ GateMode gate_mode(const GateIO& io, uint32_t g) {
    GateMode m{0u, 0u, false, false, true};
    if (io.tv) return m;  // programmable bootstrapping: no gate code
    uint32_t op;
    bool has3;
    if (io.desc) {
        op = io.desc[g].x;
        has3 = io.desc3 != nullptr;
        m.compound = (op & kCompoundFlag) != 0;
    } else {
        op = io.ops ? io.ops[g] : io.op_const;
        has3 = io.in2 != nullptr;
        m.compound = io.ops1 != nullptr;
    }
    if (m.compound) {
        m.op0 = op & 0xFFu;
        m.op1 = io.desc ? (op >> 8) & 0xFFu : io.ops1[g];
        m.valid = sym_value(m.op0, 0) != 0 && sym_value(m.op1, 0) != 0 && (!io.desc || op < 2 * kCompoundFlag);
        return m;
    }
    m.op0 = op;
    m.three = has3 && (op == FHE_MAJ || op == FHE_XOR3);
    m.valid = op <= FHE_ORYN || m.three;
    return m;
}

__device__ __forceinline__ uint32_t* wire_ptr(const GateIO& io, uint32_t w) {
    return io.region[w >> 30] + (size_t)(w & 0x3FFFFFFFu) * NW;
}

// Input samples of gate g; c3 is null unless the gate takes three inputs.
__device__ __forceinline__ void gate_operands(const GateIO& io, uint32_t g, const GateMode& m,
                                              const uint32_t*& c1, const uint32_t*& c2, const uint32_t*& c3) {
    c3 = nullptr;
    if (io.desc) {
        const uint4 d = io.desc[g];
        c1 = wire_ptr(io, d.y);
        c2 = wire_ptr(io, d.z);
        if (m.three) c3 = wire_ptr(io, io.desc3[g]);
    } else {
        c1 = io.in0 + (size_t)g * NW;
        c2 = io.in1 + (size_t)g * NW;
        if (m.three) c3 = io.in2 + (size_t)g * NW;
    }
}

__device__ __forceinline__ uint32_t* gate_output(const GateIO& io, uint32_t g) {
    return io.desc ? wire_ptr(io, io.desc[g].w) : io.out + (size_t)g * NW;
}

// Output of key-switched sample k: gate k, or with pair slots output k & 1
// of gate k >> 1 (null for the unused second slot of a single gate).
__device__ __forceinline__ uint32_t* ks_output(const GateIO& io, uint32_t k) {
    if (!io.pair_slots) return gate_output(io, k);
    const uint32_t g = k >> 1;
    if ((k & 1) == 0) return gate_output(io, g);
    if (io.desc) return (io.desc[g].x & kCompoundFlag) ? wire_ptr(io, io.desc3[g]) : nullptr;
    return io.ops1 ? io.out1 + (size_t)g * NW : nullptr;
}

template <int THREADS, class L>
__device__ __forceinline__ void load_twiddles(L& S, const uint64_t* twf, const uint64_t* twi) {
    for (int k = threadIdx.x; k < 1024; k += THREADS) {
        S.twf[k] = twf[k];
        S.twi[k] = twi[k];
    }
    __syncthreads();
}

// Gate linear combination and modulus switch to Z_2N.  Lane l keeps abar of
// words l + 64k in ab[k]; returns bbar (uniform).  Two-input codes: (0,
// kappa) + s1 c1 + s2 c2; MAJ: c1 + c2 + c3; XOR3: -2 (c1 + c2 + c3);
// compound gates: c1 + c2; programmable bootstrapping: c1 itself.
__device__ __forceinline__ int gate_prologue(const GateIO& io, uint32_t g, int lane, uint32_t (&ab)[8]) {
    const GateMode m = gate_mode(io, g);
    const uint32_t *c1, *c2, *c3;
    gate_operands(io, g, m, c1, c2, c3);
    uint32_t kappa = 0;
    int32_t s1 = 1, s2 = 1, s3 = 0;
    if (io.tv) {
        s2 = 0;
    } else if (m.three) {
        s1 = s2 = s3 = m.op0 == FHE_MAJ ? 1 : -2;
    } else if (!m.compound) {
        gate_consts(m.op0, kappa, s1, s2);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int w = lane + 64 * k;
        uint32_t v = 0;
        if (w < NW) {
            v = (uint32_t)s1 * c1[w] + (uint32_t)s2 * c2[w];
            if (c3) v += (uint32_t)s3 * c3[w];
            if (w == NLWE) v += kappa;
        }
        ab[k] = (v + (1u << 20)) >> 21;
    }
    return __builtin_amdgcn_readlane(ab[7], NLWE - 448);
}

// Constant test vector of gate g: mu = 1/8 for the gates, 1/16 for compound
// gates (their two outputs are weighted sums of two extractions).
__device__ __forceinline__ uint32_t gate_mu(const GateIO& io, uint32_t g) {
    return gate_mode(io, g).compound ? kMu >> 1 : kMu;
}

// Test-vector rotation: ACC = (0, X^(2N - bbar) v), v = mu (1 + X + ... +
// X^(N-1)).  Lane l = 32h + t writes coefficients t + 32q of polynomial h.
// With a test vector tv (programmable bootstrapping): ACC = (0, X^c tv),
// coefficient m = tv[j] for j = (m - c) mod 2N < N, else -tv[j - N].
__device__ __forceinline__ void acc_init(uint32_t (&acc)[2][1024], int bbar, int h, int t,
                                         const uint32_t* __restrict__ tv, uint32_t mu) {
    const int c = (2 * N - bbar) & (2 * N - 1);
    if (tv) {
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const int m = t + 32 * q;
            const int j = (m - c) & (2 * N - 1);
            const uint32_t v = tv[j & (N - 1)];
            acc[h][m] = h == 0 ? 0u : (j < N ? v : 0u - v);
        }
        return;
    }
    const int cm = c & (N - 1);
    const uint32_t neg = (c >= N) ? 1u : 0u;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const int m = t + 32 * q;
        const uint32_t sgn = (m >= cm) ? neg : 1u - neg;  // 1 -> -mu
        acc[h][m] = h == 0 ? 0u : (sgn ? 0u - mu : mu);
    }
}

// Sample extraction of coefficient 0: a'_0 = a_0, a'_m = -a_(N-m), b' = b_0,
// by THREADS threads with index `tid`.
template <int THREADS>
__device__ __forceinline__ void sample_extract(const uint32_t (&acc)[2][1024], uint32_t* o, int tid) {
    for (int m = tid; m < N; m += THREADS) o[m == 0 ? 0 : N - m] = m == 0 ? acc[0][0] : 0u - acc[0][m];
    if (tid == 0) o[N] = acc[1][0];
}

// Compound gate outputs.  The accumulator was rotated from the test vector
// 1/16 by the phase of c1 + c2 (-1/4, 0, +1/4 for k = 0, 1, 2 true inputs);
// the extractions of coefficients 3N/4 (E1) and N/4 (E2) then encrypt
// (E1, E2) = (+,-), (+,+), (-,+) x 1/16 for k = 0, 1, 2.  A symmetric gate
// with values g0, g1, g2 (+-1, units of 1/8) is the sample
// (g1 - g2) E1 + (g1 - g0) E2 + (0, (g0 + g2)/16).  Extraction of
// coefficient m: a'_j = a_(m-j) for j <= m, -a_(N+m-j) for j > m, b' = b_m.
template <int THREADS>
__device__ __forceinline__ void compound_extract(const uint32_t (&acc)[2][1024], uint32_t op0, uint32_t op1,
                                                 uint32_t* o0, uint32_t* o1, int tid) {
    constexpr int m1 = 3 * N / 4, m2 = N / 4;
    const int32_t a0 = sym_value(op0, 0), a1 = sym_value(op0, 1), a2 = sym_value(op0, 2);
    const int32_t b0 = sym_value(op1, 0), b1 = sym_value(op1, 1), b2 = sym_value(op1, 2);
    const uint32_t x0 = (uint32_t)(a1 - a2), y0 = (uint32_t)(a1 - a0);
    const uint32_t x1 = (uint32_t)(b1 - b2), y1 = (uint32_t)(b1 - b0);
    for (int j = tid; j < N; j += THREADS) {
        const uint32_t e1 = j <= m1 ? acc[0][m1 - j] : 0u - acc[0][N + m1 - j];
        const uint32_t e2 = j <= m2 ? acc[0][m2 - j] : 0u - acc[0][N + m2 - j];
        o0[j] = x0 * e1 + y0 * e2;
        o1[j] = x1 * e1 + y1 * e2;
    }
    if (tid == 0) {
        const uint32_t e1 = acc[1][m1], e2 = acc[1][m2];
        o0[N] = x0 * e1 + y0 * e2 + (uint32_t)(a0 + a2) * (kMu >> 1);
        o1[N] = x1 * e1 + y1 * e2 + (uint32_t)(b0 + b2) * (kMu >> 1);
    }
}

// After the blind rotation: the extracted sample(s) of gate g into its
// slot(s) of big; an invalid code gives all-zero samples (which key-switch
// to the all-zero output) and is reported through io.err.
template <int THREADS>
__device__ __forceinline__ void gate_epilogue(const GateIO& io, uint32_t g, const uint32_t (&acc)[2][1024],
                                              uint32_t* __restrict__ big, int tid) {
    const GateMode m = gate_mode(io, g);
    uint32_t* o = big + (size_t)(io.pair_slots ? 2 * g : g) * (N + 1);
    if (!m.valid) {
        const int words = (io.pair_slots ? 2 : 1) * (N + 1);
        for (int j = tid; j < words; j += THREADS) o[j] = 0u;
        if (tid == 0 && io.err)
            __hip_atomic_store(io.err, 0x100u | (m.op0 & 0xFFu), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return;
    }
    if (m.compound)
        compound_extract<THREADS>(acc, m.op0, m.op1, o, o + N + 1, tid);
    else
        sample_extract<THREADS>(acc, o, tid);
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------

// Key-load window (chunks of 8 words ahead) of the two-prime passes.  Two
// chunks measured best for every shape: issuing all of a pass's key loads
// before its transform was slower even with the full register file.
constexpr int kKeyWindow = 2;

// Gate linear combination + modulus switch, test-vector rotation, 500 CMux,
// sample extraction.  One wave per gate, WPB gates per block; the register
// budget allows two waves per SIMD.
template <int WPB, int A>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_blind_rotate(
    DeviceKeys K, GateIO io, uint32_t* __restrict__ big, uint32_t count) {
    __shared__ BlockLds<WPB, A> S;
    load_twiddles<64 * WPB>(S, Arith<A>::twf(K), Arith<A>::twi(K));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * WPB + wave;
    if (g >= count) return;

    const int h = lane >> 5, t = lane & 31;
    uint32_t ab[8];
    const int bbar = gate_prologue(io, g, lane, ab);
    WaveLdsT<kTileWords<A>> W{S.acc[wave], S.tile[wave]};
    acc_init(W.acc, bbar, h, t, io.tv, gate_mu(io, g));
    wave_lds_sync();

    // Blind rotation.  abar_i = 0 would give D = 0 and leave ACC unchanged,
    // so every step runs unconditionally.
    const uint64_t* bk = Arith<A>::bk(K);
#pragma unroll 1
    for (int i = 0; i < NLWE; ++i) {
        const int ai = __builtin_amdgcn_readlane(ab[0], i & 63);
        Arith<A>::template step<kKeyWindow>(W, ai, bk, S.twf, S.twi, lane);
        bk += 2 * 32 * 2 * 64;
        if ((i & 63) == 63) {
#pragma unroll
            for (int r = 0; r < 7; ++r) ab[r] = ab[r + 1];
        }
    }
    gate_epilogue<64>(io, g, W.acc, big, lane);
}

// The same computation with two waves per gate (one gate per block), for
// latency: wave w runs pass w of each CMux (digits of ACC_w, their forward
// NTTs and multiply-accumulate) concurrently; wave 0 then adds wave 1's
// partial sums, runs the inverse NTTs and updates ACC while wave 1 waits.
// The critical path of a CMux drops from two passes plus the inverse to one
// pass plus the inverse; the issued work stays the same.
template <int A>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_blind_rotate_pair(
    DeviceKeys K, GateIO io, uint32_t* __restrict__ big, uint32_t count) {
    __shared__ PairLds<A> S;
    load_twiddles<128>(S, Arith<A>::twf(K), Arith<A>::twi(K));
    const uint32_t g = blockIdx.x;
    if (g >= count) return;  // uniform over the block
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, h = lane >> 5, t = lane & 31;

    uint32_t ab[8];
    const int bbar = gate_prologue(io, g, lane, ab);
    if (wave == 0) acc_init(S.acc, bbar, h, t, io.tv, gate_mu(io, g));
    __syncthreads();

    const uint64_t* bk = Arith<A>::bk(K);
    if constexpr (A == 1) {
        // Two-prime form: each wave also takes one prime's inverse.  The
        // waves swap the other prime's partial column sums, wave w
        // finishes prime w, the waves swap the residues of half of the
        // registers, and wave w recombines and updates registers 16w..16w+15.
        int32_t* part0 = reinterpret_cast<int32_t*>(&S.part[0][0]);  // [32][64]
        int32_t* part1 = part0 + 32 * 64;
        const int32_t* twi = reinterpret_cast<const int32_t*>(S.twi);
#pragma unroll 1
        for (int i = 0; i < NLWE; ++i) {
            const int ai = __builtin_amdgcn_readlane(ab[0], i & 63);
            uint64_t mac[32];
            int32_t x[32];
            if (wave == 0) {
                Arith<A>::template pass<0, kKeyWindow>(S.acc[0], S.tile[0][h], ai, bk, S.twf, lane, mac);
#pragma unroll
                for (int q = 0; q < 32; ++q) part1[q * 64 + lane] = hi_of(mac[q]);
            } else {
                Arith<A>::template pass<1, kKeyWindow>(S.acc[1], S.tile[1][h], ai, bk, S.twf, lane, mac);
#pragma unroll
                for (int q = 0; q < 32; ++q) part0[q * 64 + lane] = lo_of(mac[q]);
            }
            __syncthreads();  // partials written; both waves done reading ACC
            if (wave == 0) {
#pragma unroll
                for (int q = 0; q < 32; ++q) x[q] = lo_of(mac[q]) + part0[q * 64 + lane];
                ntt1024_inv_q<0>(x, S.tile[0][h], twi, t);
            } else {
#pragma unroll
                for (int q = 0; q < 32; ++q) x[q] = hi_of(mac[q]) + part1[q * 64 + lane];
                ntt1024_inv_q<1>(x, S.tile[1][h], twi + 1024, t);
            }
            // wave 0 hands over prime-0 residues of registers 16..31, wave 1
            // prime-1 residues of registers 0..15 (each read its slot above)
            {
                int32_t* mine = wave == 0 ? part0 : part1;
                const int r0 = wave == 0 ? 16 : 0;
#pragma unroll
                for (int r = 0; r < 16; ++r) mine[(r0 + r) * 64 + lane] = x[r0 + r];
            }
            __syncthreads();  // residues written
            if (wave == 0) {
                int32_t a0[8], a1[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    a0[k] = x[k];
                    a1[k] = part1[k * 64 + lane];
                }
                crt_chunk_q<0>(S.acc, a0, a1, lane, crt_consts());
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    a0[k] = x[8 + k];
                    a1[k] = part1[(8 + k) * 64 + lane];
                }
                crt_chunk_q<1>(S.acc, a0, a1, lane, crt_consts());
            } else {
                int32_t a0[8], a1[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    a0[k] = part0[(16 + k) * 64 + lane];
                    a1[k] = x[16 + k];
                }
                crt_chunk_q<2>(S.acc, a0, a1, lane, crt_consts());
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    a0[k] = part0[(24 + k) * 64 + lane];
                    a1[k] = x[24 + k];
                }
                crt_chunk_q<3>(S.acc, a0, a1, lane, crt_consts());
            }
            __syncthreads();  // ACC updated
            bk += 2 * 32 * 2 * 64;
            if ((i & 63) == 63) {
#pragma unroll
                for (int r = 0; r < 7; ++r) ab[r] = ab[r + 1];
            }
        }
        gate_epilogue<128>(io, g, S.acc, big, threadIdx.x);
        return;
    }
#pragma unroll 1
    for (int i = 0; i < NLWE; ++i) {
        const int ai = __builtin_amdgcn_readlane(ab[0], i & 63);
        uint64_t mac[32];
        if (wave == 0) {
            Arith<A>::template pass<0, kKeyWindow>(S.acc[0], S.tile[0][h], ai, bk, S.twf, lane, mac);
        } else {
            Arith<A>::template pass<1, kKeyWindow>(S.acc[1], S.tile[1][h], ai, bk, S.twf, lane, mac);
#pragma unroll
            for (int q = 0; q < 32; ++q) S.part[q][lane] = mac[q];
        }
        __syncthreads();  // part written; both waves done reading ACC
        if (wave == 0) {
#pragma unroll
            for (int q = 0; q < 32; ++q) mac[q] = Arith<A>::add(mac[q], S.part[q][lane]);
            Arith<A>::finish(S.acc, S.tile[0][h], mac, S.twi, lane);
        }
        __syncthreads();  // ACC updated; part free
        bk += 2 * 32 * 2 * 64;
        if ((i & 63) == 63) {
#pragma unroll
            for (int r = 0; r < 7; ++r) ab[r] = ab[r + 1];
        }
    }
    gate_epilogue<128>(io, g, S.acc, big, threadIdx.x);
}

// Four waves per gate (two-prime arithmetic), for the lowest latency: the
// critical path of a CMux is one prime's pass, one prime's inverse and the
// recombination.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_blind_rotate_quad(
    DeviceKeys K, GateIO io, uint32_t* __restrict__ big, uint32_t count) {
    __shared__ QuadLds S;
    load_twiddles<256>(S, K.twfq, K.twiq);
    const uint32_t g = blockIdx.x;
    if (g >= count) return;  // uniform over the block
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, h = lane >> 5, t = lane & 31;

    uint32_t ab[8];
    const int bbar = gate_prologue(io, g, lane, ab);
    if (wave == 0) acc_init(S.acc, bbar, h, t, io.tv, gate_mu(io, g));
    __syncthreads();

    const int32_t* twf = reinterpret_cast<const int32_t*>(S.twf);
    const int32_t* twi = reinterpret_cast<const int32_t*>(S.twi);
    const uint64_t* bk = K.bkq;
#pragma unroll 1
    for (int i = 0; i < NLWE; ++i) {
        const int ai = __builtin_amdgcn_readlane(ab[0], i & 63);
        int32_t x[32];
        uint32_t* tile = S.tile[wave][h];
        switch (wave) {
        case 0: cmux_pass_q1<0, 0, kKeyWindow>(S.acc[0], tile, ai, bk, twf, lane, x); break;
        case 1: cmux_pass_q1<0, 1, kKeyWindow>(S.acc[0], tile, ai, bk, twf, lane, x); break;
        case 2: cmux_pass_q1<1, 0, kKeyWindow>(S.acc[1], tile, ai, bk, twf, lane, x); break;
        default: cmux_pass_q1<1, 1, kKeyWindow>(S.acc[1], tile, ai, bk, twf, lane, x); break;
        }
        if (wave >= 2) {
#pragma unroll
            for (int q = 0; q < 32; ++q) S.part[wave - 2][q][lane] = x[q];
        }
        __syncthreads();  // pass-1 sums written; all waves done reading ACC
        if (wave < 2) {  // wave p: prime p's column sums, inverse transform
#pragma unroll
            for (int q = 0; q < 32; ++q) x[q] += S.part[wave][q][lane];
            if (wave == 0)
                ntt1024_inv_q<0>(x, tile, twi, t);
            else
                ntt1024_inv_q<1>(x, tile, twi + 1024, t);
            // residues of the registers the other waves recombine (this wave
            // read its part[] slot above)
#pragma unroll
            for (int r = 0; r < 32; ++r)
                if (r / 8 != wave) S.part[wave][r][lane] = x[r];
        }
        __syncthreads();  // residues written
        {  // wave w recombines registers 8w..8w+7
            int32_t a0[8], a1[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                a0[k] = wave == 0 ? x[k] : S.part[0][8 * wave + k][lane];
                a1[k] = wave == 1 ? x[8 + k] : S.part[1][8 * wave + k][lane];
            }
            switch (wave) {
            case 0: crt_chunk_q<0>(S.acc, a0, a1, lane, crt_consts()); break;
            case 1: crt_chunk_q<1>(S.acc, a0, a1, lane, crt_consts()); break;
            case 2: crt_chunk_q<2>(S.acc, a0, a1, lane, crt_consts()); break;
            default: crt_chunk_q<3>(S.acc, a0, a1, lane, crt_consts()); break;
            }
        }
        __syncthreads();  // ACC updated
        bk += 2 * 32 * 2 * 64;
        if ((i & 63) == 63) {
#pragma unroll
            for (int r = 0; r < 7; ++r) ab[r] = ab[r + 1];
        }
    }
    gate_epilogue<256>(io, g, S.acc, big, threadIdx.x);
}

// Key switching N -> n: out = (0, b') - sum_{i,j} KSK[i][j][d_ij], d_ij the
// j-th base-4 digit of a'_i rounded to 16 bits.  One wave per gate; lane l
// owns output words 8l .. 8l+7 and gathers 2 KB rows with 16-byte loads; a
// zero digit (a quarter of them) skips its row.
__global__ __launch_bounds__(kBlockThreads) void k_key_switch(DeviceKeys K, GateIO io,
                                                              const uint32_t* __restrict__ big,
                                                              uint32_t count) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * kWavesPerBlock + wave;
    if (g >= count) return;
    uint32_t* o = ks_output(io, g);
    if (!o) return;  // unused second slot of a single gate
    const uint32_t* src = big + (size_t)g * (N + 1);
    uint32_t acc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = (8 * lane + e == NLWE) ? src[N] : 0u;
#pragma unroll 1
    for (int i0 = 0; i0 < N; i0 += 64) {
        const uint32_t digits = (src[i0 + lane] + (1u << 15)) >> 16;
#pragma unroll 1
        for (int l = 0; l < 64; ++l) {
            const uint32_t dd = __builtin_amdgcn_readlane(digits, l);
            const size_t rowbase = ((size_t)(i0 + l) * kKsT) * 3;
#pragma unroll
            for (int j = 0; j < (int)kKsT; ++j) {
                const uint32_t d = (dd >> (14 - 2 * j)) & 3u;
                if (d == 0) continue;  // uniform over the wave: a zero digit selects no row
                const uint4* row = reinterpret_cast<const uint4*>(K.ksk + (rowbase + 3 * j + d - 1) * kKskRowWords);
                const uint4 v0 = row[2 * lane], v1 = row[2 * lane + 1];
                acc[0] -= v0.x; acc[1] -= v0.y; acc[2] -= v0.z; acc[3] -= v0.w;
                acc[4] -= v1.x; acc[5] -= v1.y; acc[6] -= v1.z; acc[7] -= v1.w;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (8 * lane + e < NW) o[8 * lane + e] = acc[e];
}

// Key switching with W waves per gate: wave w sums the rows of coefficients
// (N/W) w .. (N/W)(w + 1) - 1, the W partial sums meet in LDS and wave 0
// writes the result.  SKIP: zero digits (a quarter of them) skip their row
// by a branch uniform over the wave, at the price of serialising the row
// loads of a coefficient; otherwise they read the all-zero row.  Per launch
// width the fastest form was measured (ms per launch; "1" is k_key_switch,
// which skips):
//   gates    8 waves   4+skip   2+skip   1
//   256      0.15      0.35     0.60
//   1,024    0.56      0.46     0.68     1.05
//   1,536    0.82      0.62     0.74
//   2,048    1.07      1.71     0.82     1.13
//   2,560    1.29      2.31     1.09     1.29
//   6,144    3.20                        2.26
//   8,192    4.27                        6.05
//   16,384   8.52      22.3     20.6     17.3 (without skip)
// With eight waves a skip costs 8.5 -> 21.3 ms at 16,384 gates, and staging
// the rows of a coefficient in LDS once per workgroup of eight gates 12.4 ms.
constexpr uint32_t kKsSplit4Min = 769, kKsSplit2Min = 1793, kKsOneWaveMin = 2817, kKsOneWaveMax = 6144;

template <int W, bool SKIP>
__global__ __launch_bounds__(64 * W) void k_key_switch_split(DeviceKeys K, GateIO io,
                                                             const uint32_t* __restrict__ big, uint32_t count) {
    __shared__ uint32_t part[W][512];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x;
    if (g >= count) return;  // uniform over the block
    uint32_t* o = ks_output(io, g);
    if (!o) return;  // unused second slot of a single gate (uniform over the block)
    const uint32_t* src = big + (size_t)g * (N + 1);
    uint32_t acc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = (wave == 0 && 8 * lane + e == NLWE) ? src[N] : 0u;
    const uint4* zero = reinterpret_cast<const uint4*>(K.zero_row);
    constexpr int kPerWave = N / W;
#pragma unroll 1
    for (int i0 = wave * kPerWave; i0 < (wave + 1) * kPerWave; i0 += 64) {
        const uint32_t digits = (src[i0 + lane] + (1u << 15)) >> 16;
#pragma unroll 1
        for (int l = 0; l < 64; ++l) {
            const uint32_t dd = __builtin_amdgcn_readlane(digits, l);
            const size_t rowbase = ((size_t)(i0 + l) * kKsT) * 3;
#pragma unroll
            for (int j = 0; j < (int)kKsT; ++j) {
                const uint32_t d = (dd >> (14 - 2 * j)) & 3u;
                if (SKIP && d == 0) continue;
                const uint4* row = d ? reinterpret_cast<const uint4*>(K.ksk + (rowbase + 3 * j + d - 1) * kKskRowWords)
                                     : zero;
                const uint4 v0 = row[2 * lane], v1 = row[2 * lane + 1];
                acc[0] -= v0.x; acc[1] -= v0.y; acc[2] -= v0.z; acc[3] -= v0.w;
                acc[4] -= v1.x; acc[5] -= v1.y; acc[6] -= v1.z; acc[7] -= v1.w;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) part[wave][8 * lane + e] = acc[e];
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 1; w < W; ++w)
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[e] += part[w][8 * lane + e];
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (8 * lane + e < NW) o[8 * lane + e] = acc[e];
}

// BK (uint32 [n][4][2][N]) -> NTT domain in the layout cmux_step reads:
// bkd[i][hp][q][sel][lane], lane = 32c + t, for row r = 2hp + digit, column c:
// sel = 0 when digit == c (the half's own digit), 1 otherwise.
__global__ __launch_bounds__(kBlockThreads) void k_bk_prepare(const uint32_t* __restrict__ bk,
                                                              uint64_t* __restrict__ bkd,
                                                              const uint64_t* __restrict__ twf,
                                                              uint32_t npolys) {
    __shared__ uint64_t stw[32 * 32];
    __shared__ uint32_t tiles[kWavesPerBlock][2][32 * 32];
    for (int k = threadIdx.x; k < 1024; k += kBlockThreads) stw[k] = twf[k];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int h = lane >> 5, t = lane & 31;
    const uint32_t base = 2 * (blockIdx.x * kWavesPerBlock + wave);
    if (base >= npolys) return;
    const uint32_t poly = base + h;  // npolys is even
    uint64_t x[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) x[q] = gl::from_i64((int32_t)bk[(size_t)poly * N + t + 32 * q]);
    ntt1024_fwd(x, &tiles[wave][h][0], stw, t);
    const uint32_t i = poly / 8, r = (poly / 2) % 4, c = poly % 2;
    const uint32_t hp = r >> 1, digit = r & 1, sel = (digit == c) ? 0 : 1;
    uint64_t* dst = bkd + (size_t)i * (2 * 32 * 2 * 64) + (size_t)hp * (32 * 2 * 64) + 32 * c + t;
#pragma unroll
    for (int q = 0; q < 32; ++q) dst[(q * 2 + sel) * 64] = gl::canon(x[q]);
}

// BK -> two-prime NTT domain in the layout cmux_pass_q reads:
// bkq[i][hp][prime][q / 2][lane 32c + t][q % 2][digit] (32-bit words) for row
// r = 2hp + digit, column c, each residue in Montgomery form and centred
// (|.| <= q/2).
template <int I>
__device__ __forceinline__ void bk_residue(const uint32_t* __restrict__ bk, uint32_t poly, int t,
                                           int32_t (&x)[32], uint32_t* tile, const int32_t* twf) {
    constexpr int64_t Q = mq::Mod<I>::q;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        int64_t v = (int64_t)(int32_t)bk[(size_t)poly * N + t + 32 * k] % Q;  // |v| < q
        x[k] = (int32_t)v;
    }
    ntt1024_fwd_q<I>(x, tile, twf, t);
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        int32_t y = mq::mul<I>(x[k], mq::Mod<I>::rform(mq::Mod<I>::R % Q));  // x R, |.| < q
        y += y < -(int32_t)(Q / 2) ? (int32_t)Q : 0;
        y -= y > (int32_t)(Q / 2) ? (int32_t)Q : 0;
        x[k] = y;
    }
}

__global__ __launch_bounds__(kBlockThreads) void k_bk_prepare_q(const uint32_t* __restrict__ bk,
                                                                uint64_t* __restrict__ bkq,
                                                                const uint64_t* __restrict__ twfq,
                                                                uint32_t npolys) {
    __shared__ int32_t stw[2 * 32 * 32];
    __shared__ uint32_t tiles[kWavesPerBlock][2][kTileWords<1>];
    const int32_t* tw = reinterpret_cast<const int32_t*>(twfq);
    for (int k = threadIdx.x; k < 2048; k += kBlockThreads) stw[k] = tw[k];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int h = lane >> 5, t = lane & 31;
    const uint32_t base = 2 * (blockIdx.x * kWavesPerBlock + wave);
    if (base >= npolys) return;
    const uint32_t poly = base + h;  // npolys is even
    int32_t x0[32], x1[32];
    bk_residue<0>(bk, poly, t, x0, &tiles[wave][h][0], stw);
    bk_residue<1>(bk, poly, t, x1, &tiles[wave][h][0], stw + 1024);
    const uint32_t i = poly / 8, r = (poly / 2) % 4, c = poly % 2;
    const uint32_t hp = r >> 1, digit = r & 1;
    uint32_t* dst = reinterpret_cast<uint32_t*>(bkq) + (size_t)i * 16384 + (size_t)hp * 8192;
    const int lw = 32 * c + t;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        dst[((q >> 1) * 64 + lw) * 4 + (q & 1) * 2 + digit] = (uint32_t)x0[q];
        dst[4096 + ((q >> 1) * 64 + lw) * 4 + (q & 1) * 2 + digit] = (uint32_t)x1[q];
    }
}

// One CMux on acc[2][N] in global memory (single wave).
template <int A>
__global__ __launch_bounds__(64) void k_debug_cmux(DeviceKeys K, const uint64_t* __restrict__ bk_i,
                                                   int32_t abar, uint32_t* __restrict__ accg) {
    __shared__ BlockLds<1, A> S;
    WaveLdsT<kTileWords<A>> W{S.acc[0], S.tile[0]};
    const uint64_t* twf = Arith<A>::twf(K);
    const uint64_t* twi = Arith<A>::twi(K);
    for (int k = threadIdx.x; k < 1024; k += 64) {
        S.twf[k] = twf[k];
        S.twi[k] = twi[k];
    }
    for (int k = threadIdx.x; k < 2 * N; k += 64) W.acc[k / N][k % N] = accg[k];
    __syncthreads();
    Arith<A>::template step<kKeyWindow>(W, abar, bk_i, S.twf, S.twi, threadIdx.x);
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * N; k += 64) accg[k] = W.acc[k / N][k % N];
}

// Issue-rate probe of one VALU instruction class (the roofline's peak per
// class): every lane runs 16 independent chains of the instruction (eight
// for the swap, which writes two registers), 64 instructions per
// iteration.  Only arithmetic instructions, no memory access but the final
// store of each lane's sum into out[global thread index].
template <int OP>
__global__ __launch_bounds__(256) void k_valu_probe(uint32_t* __restrict__ out, int iters) {
    uint32_t a[16];
    uint64_t w[16];
    const uint32_t b = threadIdx.x * 3u + 1u, c = threadIdx.x ^ 5u;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        a[k] = threadIdx.x + k;
        w[k] = (uint64_t)threadIdx.x * (k + 1);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if constexpr (OP == 0) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (OP == 1) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (OP == 2)
                    asm volatile("v_mad_i64_i32 %0, vcc, %1, %2, %0" : "+v"(w[k]) : "v"(b), "v"(c) : "vcc");
                if constexpr (OP == 3) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (OP == 4) asm volatile("v_bfe_i32 %0, %0, %1, 10" : "+v"(a[k]) : "v"(c));
                if constexpr (OP == 5)  // eight disjoint register pairs, each swapped twice per pass
                    asm volatile("v_permlane32_swap_b32 %0, %1" : "+v"(a[k & 7]), "+v"(a[8 + (k & 7)]));
            }
        }
    }
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) sum += a[k] + (uint32_t)w[k] + (uint32_t)(w[k] >> 32);
    out[blockIdx.x * blockDim.x + threadIdx.x] = sum;
}

}  // namespace

hipError_t launch_valu_probe(int op, uint32_t* out, uint32_t blocks, int iters, hipStream_t s) {
    switch (op) {
    case 0: hipLaunchKernelGGL(k_valu_probe<0>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 1: hipLaunchKernelGGL(k_valu_probe<1>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 2: hipLaunchKernelGGL(k_valu_probe<2>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 3: hipLaunchKernelGGL(k_valu_probe<3>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 4: hipLaunchKernelGGL(k_valu_probe<4>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 5: hipLaunchKernelGGL(k_valu_probe<5>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bk_prepare(const uint32_t* bk, uint64_t* bkd, const uint64_t* twf,
                             uint32_t n_lwe, hipStream_t s) {
    const uint32_t npolys = n_lwe * 8;
    const uint32_t waves = npolys / 2;
    const uint32_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(k_bk_prepare, dim3(blocks), dim3(kBlockThreads), 0, s, bk, bkd, twf, npolys);
    return hipGetLastError();
}

template <int A>
static hipError_t launch_blind_rotate_a(const DeviceKeys& K, const GateIO& io, uint32_t* big,
                                        uint32_t count, LaunchConfig cfg, hipStream_t s) {
    if (cfg.waves_per_gate == 2) {
        hipLaunchKernelGGL(k_blind_rotate_pair<A>, dim3(count), dim3(128), 0, s, K, io, big, count);
        return hipGetLastError();
    }
    const uint32_t wpb = cfg.gates_per_group;
    const uint32_t blocks = (count + wpb - 1) / wpb;
    switch (wpb) {
    case 1: hipLaunchKernelGGL((k_blind_rotate<1, A>), dim3(blocks), dim3(64), 0, s, K, io, big, count); break;
    case 2: hipLaunchKernelGGL((k_blind_rotate<2, A>), dim3(blocks), dim3(128), 0, s, K, io, big, count); break;
    case 4: hipLaunchKernelGGL((k_blind_rotate<4, A>), dim3(blocks), dim3(256), 0, s, K, io, big, count); break;
    case 8: hipLaunchKernelGGL((k_blind_rotate<8, A>), dim3(blocks), dim3(512), 0, s, K, io, big, count); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_blind_rotate(const DeviceKeys& K, const GateIO& io, uint32_t* big,
                               uint32_t count, LaunchConfig cfg, hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (cfg.waves_per_gate == 4) {
        if (cfg.arith != 1 || !K.bkq) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_blind_rotate_quad, dim3(count), dim3(256), 0, s, K, io, big, count);
        return hipGetLastError();
    }
    if (cfg.waves_per_gate != 1 && cfg.waves_per_gate != 2) return hipErrorInvalidValue;
    if (cfg.arith == 1) {
        if (!K.bkq) return hipErrorInvalidValue;
        return launch_blind_rotate_a<1>(K, io, big, count, cfg, s);
    }
    if (cfg.arith != 0) return hipErrorInvalidValue;
    return launch_blind_rotate_a<0>(K, io, big, count, cfg, s);
}

hipError_t launch_key_switch(const DeviceKeys& K, const GateIO& io, const uint32_t* big,
                             uint32_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (count >= kKsOneWaveMin && count <= kKsOneWaveMax) {
        const uint32_t blocks = (count + kWavesPerBlock - 1) / kWavesPerBlock;
        hipLaunchKernelGGL(k_key_switch, dim3(blocks), dim3(kBlockThreads), 0, s, K, io, big, count);
    } else if (count >= kKsSplit2Min && count < kKsOneWaveMin) {
        hipLaunchKernelGGL((k_key_switch_split<2, true>), dim3(count), dim3(128), 0, s, K, io, big, count);
    } else if (count >= kKsSplit4Min && count < kKsSplit2Min) {
        hipLaunchKernelGGL((k_key_switch_split<4, true>), dim3(count), dim3(256), 0, s, K, io, big, count);
    } else {
        hipLaunchKernelGGL((k_key_switch_split<8, false>), dim3(count), dim3(512), 0, s, K, io, big, count);
    }
    return hipGetLastError();
}

hipError_t launch_debug_cmux(const DeviceKeys& K, int arith, const uint64_t* bk_i, int32_t abar,
                             uint32_t* acc, hipStream_t s) {
    if (arith == 1)
        hipLaunchKernelGGL(k_debug_cmux<1>, dim3(1), dim3(64), 0, s, K, bk_i, abar, acc);
    else
        hipLaunchKernelGGL(k_debug_cmux<0>, dim3(1), dim3(64), 0, s, K, bk_i, abar, acc);
    return hipGetLastError();
}

hipError_t launch_bk_prepare_q(const uint32_t* bk, uint64_t* bkq, const uint64_t* twfq,
                               uint32_t n_lwe, hipStream_t s) {
    const uint32_t npolys = n_lwe * 8;
    const uint32_t waves = npolys / 2;
    const uint32_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL(k_bk_prepare_q, dim3(blocks), dim3(kBlockThreads), 0, s, bk, bkq, twfq, npolys);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace fhe

// Wheel start offsets: Table 1 of the paper (Sec. 3), host and device.
//
// A segment ("tile") with value base B (a multiple of 6) holds two bit
// planes; bit i of plane A_r stands for the value B + 6*i + r, r in {1, 5}
// (Sec. 2.1, Fig. 2).  For a prime P >= 5 and a first value M, the first bit
// to clear in each plane is found as in Sec. 3:
//   Q    = the greatest multiple of P strictly below M,
//   q    = Q mod 6, p = P mod 6 (1 or 5), R = floor(P / 6),
//   idx0 = floor((Q - B) / 6), the index Q would have (may be -1 or less),
//   id_r = idx0 + k * R + c, with (k, c) read from Table 1 for (p, q, r).
// M is max(B, P*P): marking starts at the square (Sec. 1.1, Sec. 2.4), which
// also keeps a segment that holds P itself from clearing it.
//
// Arithmetic.  The one wide step is rem = (M - 1) mod P.  When M = P*P it
// is simply P - 1.  Otherwise it uses a per-prime reciprocal
// m = floor((2^64 - 1) / P): mulhi64(x, m) is floor(x / P) or one less (m is
// below 2^64 / P by less than 1, so x * m / 2^64 > x / P - 1), and one
// conditional subtraction of P corrects it (Granlund and Montgomery, PLDI
// 1994, division by invariant integers using multiplication).  Everything
// after the remainder fits in 32 bits: d = Q - B lies in [-P, 2^22) for a
// tile, so d + 6(R + 1) (> P) is non-negative and below 2^32 for every
// P < 3.1e9, and floor division of that biased value by 6 gives
// idx0 + R + 1 and q = Q mod 6 without signed 64-bit division.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sieve {

// Table 1 as printed in the paper, one byte per column q = 0..5 (byte q),
// each byte holding (k - 1) | (c << 3) for id = idx0 + k*R + c.
// The paper's "k*(R+1) - 1" is (k, k-1) and "k*(R+1)" is (k, k).
//   p = 1:  id_1: R, 6R+1, 5R+1, 4R+1, 3R+1, 2R+1
//           id_5: 5R, 4R,   3R,   2R,   R,    6R+1
//   p = 5:  id_1: 5(R+1)-1, 6(R+1)-1, R+1,      2(R+1),   3(R+1),   4(R+1)
//           id_5: R,        2(R+1)-1, 3(R+1)-1, 4(R+1)-1, 5(R+1)-1, 6(R+1)-1
constexpr uint64_t table1_byte(int k, int c) { return (uint64_t)((k - 1) | (c << 3)); }
constexpr uint64_t table1_row(const int (&kc)[6][2])
{
    uint64_t v = 0;
    for (int q = 0; q < 6; ++q)
        v |= table1_byte(kc[q][0], kc[q][1]) << (8 * q);
    return v;
}
constexpr int kT1p1[6][2] = {{1, 0}, {6, 1}, {5, 1}, {4, 1}, {3, 1}, {2, 1}};
constexpr int kT5p1[6][2] = {{5, 0}, {4, 0}, {3, 0}, {2, 0}, {1, 0}, {6, 1}};
constexpr int kT1p5[6][2] = {{5, 4}, {6, 5}, {1, 1}, {2, 2}, {3, 3}, {4, 4}};
constexpr int kT5p5[6][2] = {{1, 0}, {2, 1}, {3, 2}, {4, 3}, {5, 4}, {6, 5}};
constexpr uint64_t kTable1_id1_p1 = table1_row(kT1p1);
constexpr uint64_t kTable1_id5_p1 = table1_row(kT5p1);
constexpr uint64_t kTable1_id1_p5 = table1_row(kT1p5);
constexpr uint64_t kTable1_id5_p5 = table1_row(kT5p5);

// Per-prime constants resident on the device (16 bytes, one load).
struct PrimeConst {
    uint32_t p;       // the prime, >= 5
    uint32_t r;       // bits 0..28: floor(p / 6); bits 29..31: p^-1 mod 5 (0 for p = 5)
    uint32_t m_lo;    // m = floor((2^64 - 1) / p), low and high halves; m < 2^62, so
    uint32_t m_hi;    // bit 31 of m_hi is free and flags p = 5 (mod 6)
};

constexpr uint32_t kP5Flag = 0x80000000u;

// x^-1 mod 5 for x mod 5 in 1..4 (0 stays 0).
__host__ __device__ inline uint32_t inv_mod5(uint32_t x)
{
    return (0x42310u >> (4u * (x % 5u))) & 0xFu;  // 0->0, 1->1, 2->3, 3->2, 4->4
}

inline PrimeConst make_prime_const(uint32_t p)
{
    const uint64_t m = UINT64_MAX / p;
    return PrimeConst{p, (p / 6u) | (inv_mod5(p) << 29), (uint32_t)m,
                      (uint32_t)(m >> 32) | (p % 6u == 5u ? kP5Flag : 0u)};
}

__host__ __device__ inline uint64_t prime_recip(const PrimeConst &pc)
{
    return ((uint64_t)(pc.m_hi & ~kP5Flag) << 32) | pc.m_lo;
}

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// x mod P for 5 <= P < 2^32, given m = floor((2^64 - 1) / P).  `narrow`
// (P < 2^31) lets the correction run in 32 bits: the remainder before it is
// below 2P.  Callers pass a value that is uniform across the wavefront.
__host__ __device__ inline uint32_t mod_invariant(uint64_t x, uint32_t P, uint64_t m, bool narrow)
{
    const uint64_t q = mulhi64(x, m);  // floor(x / P) or one less
    if (narrow) {
        uint32_t r = (uint32_t)x - (uint32_t)q * P;
        return r >= P ? r - P : r;
    }
    uint64_t r = x - q * (uint64_t)P;
    return (uint32_t)(r >= P ? r - P : r);
}

// (M - 1) mod P for M = max(B, P * P); `narrow` as for mod_invariant.
__host__ __device__ inline uint32_t start_rem(const PrimeConst &pc, uint64_t B, uint64_t P2, bool narrow)
{
    if (P2 > B)
        return pc.p - 1u;  // (P^2 - 1) mod P
    return mod_invariant(B - 1, pc.p, prime_recip(pc), narrow);
}

// Table 1 lookup: given dp = (Q - B) + 6(R + 1) (Q the greatest multiple of
// P below the first value, 1 <= dp < 2^32), the start indices of P in both
// planes.  p5: P = 5 (mod 6).
__host__ __device__ inline void table1_ids(uint32_t dp, uint32_t R, bool p5, uint32_t &id1, uint32_t &id5)
{
    const uint32_t i0 = dp / 6u;       // = idx0 + R + 1
    const uint32_t q = dp - 6u * i0;   // = Q mod 6
    const uint64_t t1 = p5 ? kTable1_id1_p5 : kTable1_id1_p1;
    const uint64_t t5 = p5 ? kTable1_id5_p5 : kTable1_id5_p1;
    const uint32_t e1 = (uint32_t)(t1 >> (8u * q));
    const uint32_t e5 = (uint32_t)(t5 >> (8u * q));
    // id = idx0 + k*R + c = i0 + (k - 1)*R + c - 1
    id1 = i0 + (e1 & 7u) * R + ((e1 >> 3) & 7u) - 1u;
    id5 = i0 + (e5 & 7u) * R + ((e5 >> 3) & 7u) - 1u;
}

// Start indices (relative to base B) of prime P in both planes for a first
// value M with B <= M < B + 2^22 and M >= 1, given rem = (M - 1) mod P.
// Both results are the true indices (>= 0); callers compare them against
// the plane length.
__host__ __device__ inline void wheel_start(uint32_t P, uint32_t R, uint64_t B, uint64_t M, uint32_t rem,
                                            uint32_t &id1, uint32_t &id5)
{
    const uint64_t x = M - 1;  // Q = x - rem, the greatest multiple of P below M
    // dp = (Q - B) + 6(R + 1), computed mod 2^32 (its true value is in [1, 2^32)).
    const uint32_t dp = (uint32_t)(x - B) - rem + 6u * (R + 1u);
    table1_ids(dp, R, (P - 6u * R) == 5u, id1, id5);
}

// x mod P for x < 2^62 and P < 2^31 (the narrow case of mod_invariant),
// where only the low 32 bits of the quotient estimate are formed: the
// remainder x - q P is below 2P < 2^32, so it is determined mod 2^32.  With
// x = xh 2^32 + xl and m = mh 2^32 + ml the high half of x m is
// xh mh + hi(xl mh + hi(xl ml)) + hi(xh ml + lo(xl mh + hi(xl ml))) plus no
// further carry into bit 64, and its low 32 bits need only 32-bit adds.
__device__ inline uint32_t mod_narrow(uint32_t xl, uint32_t xh, uint32_t P, uint32_t ml, uint32_t mh)
{
    const uint32_t t = __umulhi(xl, ml);
    const uint64_t u = (uint64_t)xl * mh + t;
    const uint64_t w = (uint64_t)xh * ml + (uint32_t)u;
    const uint32_t q = xh * mh + (uint32_t)(u >> 32) + (uint32_t)(w >> 32);
    const uint32_t r = xl - q * P;
    const uint32_t r2 = r - P;
    return r2 < r ? r2 : r;  // r in [0, 2P): subtract P once when r >= P
}

// The same for the sieve kernel's tiles, with the square test done on 32-bit
// per-tile thresholds: sqb = isqrt(B).  For P <= sqb the first value is
// M = B, so x - B = -1 and dp = 6R + 5 - rem with rem = (B - 1) mod P, where
// 6R + 5 is P + 4 or P for P = 1 or 5 (mod 6).  For P > sqb (the square lies
// in the tile) M = P*P, rem = P - 1 and dp = P*P - B + 6 - (P mod 6), whose
// true value is below 2^22 + 6, so 32-bit wrap-around arithmetic gives it.
__device__ inline void tile_start(const PrimeConst &pc, uint32_t sqb, uint64_t Bm1, uint32_t B32, bool narrow,
                                  uint32_t &id1, uint32_t &id5)
{
    const uint32_t R = pc.r & 0x1FFFFFFFu;
    const bool p5 = (pc.m_hi & kP5Flag) != 0;
    uint32_t dp;
    if (pc.p > sqb) {
        dp = pc.p * pc.p - B32 + (p5 ? 1u : 5u);
    } else {
        const uint32_t rem = narrow ? mod_narrow((uint32_t)Bm1, (uint32_t)(Bm1 >> 32), pc.p, pc.m_lo,
                                                 pc.m_hi & ~kP5Flag)
                                    : mod_invariant(Bm1, pc.p, prime_recip(pc), false);
        dp = pc.p + (p5 ? 0u : 4u) - rem;
    }
    table1_ids(dp, R, p5, id1, id5);
}

// tile_start for tiles whose active primes are all below 2^24 - 8 (so R,
// dp, i0 and the per-prime products fit 24 bits).  The same arithmetic with
// every product formed by the full-rate 24-bit multiplier: i0 = dp div 6 as
// (dp * ceil(2^26 / 6)) >> 26, exact for dp < 2^25, and k R with R < 2^22.
// The remainder keeps the 64-bit reciprocal.
__device__ inline void tile_start_u24(const PrimeConst &pc, uint32_t sqb, uint64_t Bm1, uint32_t B32, bool narrow,
                                      uint32_t &id1, uint32_t &id5)
{
    const uint32_t P = pc.p & 0xFFFFFFu;
    const uint32_t R = pc.r & 0xFFFFFFu;
    const bool p5 = (pc.m_hi & kP5Flag) != 0;
    uint32_t dp;
    if (P > sqb) {
        dp = __umul24(P, P) - B32 + (p5 ? 1u : 5u);
    } else {
        const uint32_t rem = narrow ? mod_narrow((uint32_t)Bm1, (uint32_t)(Bm1 >> 32), pc.p, pc.m_lo,
                                                 pc.m_hi & ~kP5Flag)
                                    : mod_invariant(Bm1, pc.p, prime_recip(pc), false);
        dp = P + (p5 ? 0u : 4u) - rem;
    }
    dp &= 0xFFFFFFu;  // below 2^24 by the bound on P
    constexpr uint32_t kM6 = 11184811u;  // ceil(2^26 / 6)
    const uint32_t i0 = (uint32_t)(((uint64_t)dp * kM6) >> 26);  // 24 x 24-bit product
    // 6 i0 on the 24-bit multiplier (written out: the compiler would fold
    // dp - 6 i0 into a 32-bit multiply by -6)
    uint32_t i6;
    asm("v_mul_u32_u24 %0, %1, 6" : "=v"(i6) : "v"(i0));
    const uint32_t q = dp - i6;
    const uint64_t t1 = p5 ? kTable1_id1_p5 : kTable1_id1_p1;
    const uint64_t t5 = p5 ? kTable1_id5_p5 : kTable1_id5_p1;
    const uint32_t e1 = (uint32_t)(t1 >> (8u * q));
    const uint32_t e5 = (uint32_t)(t5 >> (8u * q));
    id1 = i0 + __umul24(e1 & 7u, R) + ((e1 >> 3) & 7u) - 1u;
    id5 = i0 + __umul24(e5 & 7u, R) + ((e5 >> 3) & 7u) - 1u;
}

}  // namespace sieve

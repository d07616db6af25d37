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
    uint32_t m_lo;    // floor((2^64 - 1) / p), low and high halves
    uint32_t m_hi;
};

// x^-1 mod 5 for x mod 5 in 1..4 (0 stays 0).
__host__ __device__ inline uint32_t inv_mod5(uint32_t x)
{
    return (0x42310u >> (4u * (x % 5u))) & 0xFu;  // 0->0, 1->1, 2->3, 3->2, 4->4
}

inline PrimeConst make_prime_const(uint32_t p)
{
    const uint64_t m = UINT64_MAX / p;
    return PrimeConst{p, (p / 6u) | (inv_mod5(p) << 29), (uint32_t)m, (uint32_t)(m >> 32)};
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
    return mod_invariant(B - 1, pc.p, ((uint64_t)pc.m_hi << 32) | pc.m_lo, narrow);
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
    const uint32_t i0 = dp / 6u;       // = idx0 + R + 1
    const uint32_t q = dp - 6u * i0;   // = Q mod 6
    const bool p5 = (P - 6u * R) == 5u;
    const uint64_t t1 = p5 ? kTable1_id1_p5 : kTable1_id1_p1;
    const uint64_t t5 = p5 ? kTable1_id5_p5 : kTable1_id5_p1;
    const uint32_t e1 = (uint32_t)(t1 >> (8u * q));
    const uint32_t e5 = (uint32_t)(t5 >> (8u * q));
    // id = idx0 + k*R + c = i0 + (k - 1)*R + c - 1
    id1 = i0 + (e1 & 7u) * R + ((e1 >> 3) & 7u) - 1u;
    id5 = i0 + (e5 & 7u) * R + ((e5 >> 3) & 7u) - 1u;
}

}  // namespace sieve

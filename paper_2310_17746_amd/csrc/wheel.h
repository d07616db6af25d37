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
// The division by P uses a per-prime reciprocal m = floor((2^64 - 1) / P):
// for any 64-bit x, mulhi64(x, m) is floor(x / P) or one less (m is below
// 2^64 / P by less than 1, so x * m / 2^64 > x / P - 1), and one conditional
// subtraction of P from the remainder corrects it (Granlund and Montgomery,
// PLDI 1994, division by invariant integers using multiplication).
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sieve {

// Table 1 as printed in the paper.  Entry [p == 5][q] = {k1, c1, k5, c5}:
// id_1 = idx0 + k1*R + c1 and id_5 = idx0 + k5*R + c5.  The paper's
// "k*(R+1) - 1" is stored as (k, k-1) and "k*(R+1)" as (k, k).
struct Table1Entry {
    uint8_t k1, c1, k5, c5;
};

__host__ __device__ constexpr Table1Entry table1(int p5, int q)
{
    // Rows p = 1 (p5 == 0) and p = 5 (p5 == 1), columns q = 0..5.
    constexpr Table1Entry t[2][6] = {
        {{1, 0, 5, 0}, {6, 1, 4, 0}, {5, 1, 3, 0}, {4, 1, 2, 0}, {3, 1, 1, 0}, {2, 1, 6, 1}},
        {{5, 4, 1, 0}, {6, 5, 2, 1}, {1, 1, 3, 2}, {2, 2, 4, 3}, {3, 3, 5, 4}, {4, 4, 6, 5}},
    };
    return t[p5][q];
}

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// x mod P for P >= 2, given m = floor((2^64 - 1) / P).
__host__ __device__ inline uint64_t mod_invariant(uint64_t x, uint64_t P, uint64_t m)
{
    uint64_t r = x - mulhi64(x, m) * P;
    return r >= P ? r - P : r;
}

// Start indices (relative to base B) of prime P in both planes for first
// value M >= 1, M >= B.  R = P / 6, m = reciprocal of P.  Both results are
// >= 0; callers compare them against the plane length.
__host__ __device__ inline void wheel_start(uint64_t P, uint64_t R, uint64_t m, uint64_t B,
                                            uint64_t M, int64_t &id1, int64_t &id5)
{
    const uint64_t x = M - 1;
    const uint64_t Q = x - mod_invariant(x, P, m);  // greatest multiple of P below M
    const int64_t d = (int64_t)(Q - B);             // >= -P, may be negative
    // floor division by 6 and the matching non-negative remainder q = Q mod 6
    // (B is a multiple of 6, so Q mod 6 = d mod 6).
    int64_t idx0 = d / 6;
    int64_t q = d - 6 * idx0;
    if (q < 0) {
        q += 6;
        idx0 -= 1;
    }
    const Table1Entry e = table1((P - 6 * R) == 5, (int)q);
    id1 = idx0 + (int64_t)e.k1 * (int64_t)R + e.c1;
    id5 = idx0 + (int64_t)e.k5 * (int64_t)R + e.c5;
}

}  // namespace sieve

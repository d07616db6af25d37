/*
 * sieve_debug.h -- marking tally of the debug build of the library
 * (libsieve_markcount.so, compiled with SIEVE_MARK_COUNT; the product
 * libsieve.so does not export it).
 *
 * For the pin of marking completeness: over a range [lo, hi) the tiles cover
 * the wheel values of [B, E), B = lo - lo mod 6 and E = B + 192 * ceil(n / 32)
 * with n = ceil((hi - B - 1) / 6) indices per plane; every base prime P above
 * the presieved ones with P * P < hi must visit exactly the values m * P with
 * gcd(m, 6) = 1 and max(P * P, B) <= m * P < E (Sec. 1.1: marking starts at
 * the square; Sec. 2.1: the arrays hold only values coprime to 6).
 */
#ifndef SIEVE_DEBUG_H
#define SIEVE_DEBUG_H

#include <stdint.h>

#include "sieve.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Copies into out[0..3] the sums over the context's jobs since the last
 * reset of: out[0] the hits the marking loops visited (LDS marks, marks of
 * split-tile parts in device memory, bucket-sieve hits within the range's
 * words); out[1] the OR operations issued for them; out[2] the hits skipped
 * because their cofactor is a multiple of 5 (cleared by the presieve), so
 * that out[1] + out[2] = out[0]; out[3] the marking runs whose first hit was
 * not a multiple of its prime at or past the prime's square (0 when correct).
 * reset != 0 clears the sums afterwards.  Counting a job only; no device work.
 */
int sieve_debug_tally(sieve_ctx *ctx, uint64_t *out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* SIEVE_DEBUG_H */

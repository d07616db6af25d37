/*
 * sieve_probe.h -- LDS throughput probe exported by libsieve.so.
 *
 * Measures the LDS instruction rates the sieve's marking kernel depends on,
 * so that its roofline can use a measured peak for the exact instruction
 * (32-bit LDS OR without return) beside the nominal LDS bandwidth.
 */
#ifndef SIEVE_PROBE_H
#define SIEVE_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Probe modes: instruction and address pattern. */
#define SIEVE_PROBE_OR_LINEAR 0      /* ds_or_b32, lane-consecutive words (no bank conflict) */
#define SIEVE_PROBE_OR_RANDOM 1      /* ds_or_b32, random words */
#define SIEVE_PROBE_OR_EVEN 2        /* ds_or_b32, random even words (one plane of two interleaved) */
#define SIEVE_PROBE_OR_SAME 3        /* ds_or_b32, every lane of a wave on one word */
#define SIEVE_PROBE_WRITE_LINEAR 4   /* ds_write_b32, lane-consecutive words */
#define SIEVE_PROBE_WRITE_RANDOM 5   /* ds_write_b32, random words */
#define SIEVE_PROBE_WRITE8_RANDOM 6  /* ds_write_b8, random bytes */
#define SIEVE_PROBE_READ_RANDOM 7    /* ds_read_b32, random words */
#define SIEVE_PROBE_NUM_MODES 8

/*
 * Runs one probe on HIP device `device`: wg_per_cu (1 or 2) workgroups of
 * 1024 threads per compute unit, each thread issuing 8 * iters operations
 * (1 <= iters <= 2^20).  *ops_per_s receives lane operations per second over
 * the whole device and *ms the kernel time (HIP events).  Returns 0, -1 on a
 * bad argument, -6 on a HIP error.
 */
int sieve_probe_lds(int device, int mode, int iters, int wg_per_cu, double *ops_per_s, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* SIEVE_PROBE_H */

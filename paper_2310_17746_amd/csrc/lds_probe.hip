// LDS throughput probe: the measured peak of the LDS instructions the sieve
// uses, for the roofline of the marking kernel.
//
// Each thread issues `iters` x 8 LDS operations of one kind against a 64 KiB
// LDS array.  The instruction and the address pattern are template
// parameters, so the inner loop has no branches: per operation one VALU XOR
// forms the address and one LDS instruction follows.  Addresses come from
// eight per-lane base byte offsets XOR-ed with a value that is uniform
// across the wavefront and changes every iteration (computed on the scalar
// unit), so the bank pattern of every instruction equals that of its base (a
// uniform XOR permutes banks).  All addresses stay inside the array: the
// bases and the XOR value are masked to its range.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sieve_probe.h"

namespace {

constexpr uint32_t kWords = 16384;  // 64 KiB of LDS
constexpr int kThreads = 1024;

typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

// Pseudo-random word indices for the random-address patterns: the
// "lowbias32" integer hash (xorshift-multiply rounds) published by
// C. Wellons, "Prospecting for Hash Functions" (2018, hash-prospector).
__host__ __device__ __forceinline__ uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Word index of base j of a thread for each address pattern.
template <int MODE>
__device__ __forceinline__ uint32_t base_word(uint32_t tid, uint32_t lane, int j)
{
    if (MODE == SIEVE_PROBE_OR_LINEAR || MODE == SIEVE_PROBE_WRITE_LINEAR)
        return ((tid >> 6) * 512 + j * 64 + lane) % kWords;  // lane-consecutive words
    if (MODE == SIEVE_PROBE_OR_SAME)
        return (tid >> 6) * 64 + j;  // all lanes of a wave on one word
    if (MODE == SIEVE_PROBE_OR_EVEN)
        return (hash32(tid * 8 + j + 1) % (kWords / 2)) * 2;  // random, even words only
    return hash32(tid * 8 + j + 1) % kWords;  // random words
}

template <int MODE>
__global__ void __launch_bounds__(kThreads) k_lds_probe(int iters, uint32_t *sink)
{
    __shared__ uint32_t buf[kWords];
    const uint32_t tid = threadIdx.x;
    for (uint32_t w = tid; w < kWords; w += kThreads)
        buf[w] = 0;
    __syncthreads();
    const uint32_t lane = tid & 63;
    constexpr bool kBytes = MODE == SIEVE_PROBE_WRITE8_RANDOM;
    uint32_t base[8];  // byte offsets
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        base[j] = base_word<MODE>(tid, lane, j) * 4 + (kBytes ? (lane & 3) : 0);
        asm volatile("" : "+v"(base[j]));  // keep the byte offsets: one XOR per operation
    }
    const uint32_t bit = 1u << (lane & 31);
    // even-word mode keeps word bit 0 (byte bit 2) clear
    const uint32_t umask = (kWords - 1) * 4 & (MODE == SIEVE_PROBE_OR_EVEN ? ~4u : ~0u);
    uint32_t acc = 0;
    for (int it = 0; it < iters; ++it) {
        const uint32_t u = (hash32((uint32_t)it) * 4) & umask;  // uniform
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t a = base[j] ^ u;
            if (MODE == SIEVE_PROBE_WRITE_LINEAR || MODE == SIEVE_PROBE_WRITE_RANDOM)
                *((lds_u32 *)(size_t)a) = bit;
            else if (kBytes)
                *((lds_u8 *)(size_t)a) = (uint8_t)lane;
            else if (MODE == SIEVE_PROBE_READ_RANDOM)
                acc += *((lds_u32 *)(size_t)a);
            else
                __atomic_fetch_or((lds_u32 *)(size_t)a, bit, __ATOMIC_RELAXED);
        }
    }
    __syncthreads();
    // keep the work observable
    const uint32_t v = buf[tid % kWords] + acc;
    if (v == 0x9E3779B9u)
        sink[blockIdx.x] = v;
}

template <int MODE>
void launch_probe(int grid, int iters, uint32_t *sink)
{
    hipLaunchKernelGGL(k_lds_probe<MODE>, dim3(grid), dim3(kThreads), 0, 0, iters, sink);
}

void launch_mode(int mode, int grid, int iters, uint32_t *sink)
{
    switch (mode) {
    case SIEVE_PROBE_OR_LINEAR: launch_probe<SIEVE_PROBE_OR_LINEAR>(grid, iters, sink); break;
    case SIEVE_PROBE_OR_RANDOM: launch_probe<SIEVE_PROBE_OR_RANDOM>(grid, iters, sink); break;
    case SIEVE_PROBE_OR_EVEN: launch_probe<SIEVE_PROBE_OR_EVEN>(grid, iters, sink); break;
    case SIEVE_PROBE_OR_SAME: launch_probe<SIEVE_PROBE_OR_SAME>(grid, iters, sink); break;
    case SIEVE_PROBE_WRITE_LINEAR: launch_probe<SIEVE_PROBE_WRITE_LINEAR>(grid, iters, sink); break;
    case SIEVE_PROBE_WRITE_RANDOM: launch_probe<SIEVE_PROBE_WRITE_RANDOM>(grid, iters, sink); break;
    case SIEVE_PROBE_WRITE8_RANDOM: launch_probe<SIEVE_PROBE_WRITE8_RANDOM>(grid, iters, sink); break;
    default: launch_probe<SIEVE_PROBE_READ_RANDOM>(grid, iters, sink); break;
    }
}

}  // namespace

extern "C" int sieve_probe_lds(int device, int mode, int iters, int wg_per_cu, double *ops_per_s,
                               double *ms)
{
    if (!ops_per_s || !ms || mode < 0 || mode >= SIEVE_PROBE_NUM_MODES || iters < 1 || iters > (1 << 20) ||
        wg_per_cu < 1 || wg_per_cu > 2)
        return -1;
    hipDeviceProp_t prop;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess) {
        (void)hipGetLastError();
        return -6;
    }
    const int grid = prop.multiProcessorCount * wg_per_cu;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = -6;
    if (hipMalloc((void **)&sink, sizeof(uint32_t) * grid) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess) {
        launch_mode(mode, grid, 16, sink);  // warm-up
        hipEventRecord(e0, 0);
        launch_mode(mode, grid, iters, sink);
        hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) == hipSuccess) {
            float t = 0;
            hipEventElapsedTime(&t, e0, e1);
            *ms = t;
            *ops_per_s = (double)grid * kThreads * (double)iters * 8.0 / (t * 1e-3);
            st = 0;
        }
    }
    (void)hipGetLastError();
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (sink)
        (void)hipFree(sink);
    return st;
}

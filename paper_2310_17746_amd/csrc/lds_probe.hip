// LDS throughput probe: the measured peak of the LDS instructions the sieve
// uses, for the roofline of the marking kernel.
//
// Each thread issues `iters` LDS operations of one kind against a 64 KiB LDS
// array.  Addresses come from eight per-lane base offsets XOR-ed with a value
// that is uniform across the wavefront and changes every iteration, so the
// bank pattern of every instruction equals that of its base (a uniform XOR
// permutes banks) and each operation costs one VALU instruction.  All
// addresses stay inside the array: bases and the XOR value are masked to the
// array's word (or byte) range.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sieve_probe.h"

namespace {

constexpr int kWords = 16384;  // 64 KiB of LDS
constexpr int kThreads = 1024;

typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

__device__ __forceinline__ uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(kThreads) k_lds_probe(int mode, int iters, uint32_t *sink)
{
    __shared__ uint32_t buf[kWords];
    const uint32_t tid = threadIdx.x;
    for (int w = tid; w < kWords; w += kThreads)
        buf[w] = 0;
    __syncthreads();
    const uint32_t lane = tid & 63;
    uint32_t base[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        uint32_t word;
        switch (mode) {
        case SIEVE_PROBE_OR_LINEAR:
        case SIEVE_PROBE_WRITE_LINEAR:
            word = ((tid >> 6) * 512 + j * 64 + lane) % kWords;  // lane-consecutive words
            break;
        case SIEVE_PROBE_OR_SAME:
            word = (tid >> 6) * 64 + j;  // all lanes of a wave on one word
            break;
        case SIEVE_PROBE_OR_EVEN:
            word = (hash32(tid * 8 + j + 1) % (kWords / 2)) * 2;  // random, even words only
            break;
        default:
            word = hash32(tid * 8 + j + 1) % kWords;  // random words
            break;
        }
        base[j] = word;
    }
    const uint32_t bit = 1u << (lane & 31);
    const bool bytes = mode == SIEVE_PROBE_WRITE8_RANDOM;
    uint32_t acc = 0;
    for (int it = 0; it < iters; ++it) {
        // uniform XOR keeps addresses in range (kWords is a power of two);
        // even-word mode keeps bit 0 clear
        const uint32_t u = (hash32((uint32_t)it) & (kWords - 1)) & (mode == SIEVE_PROBE_OR_EVEN ? ~1u : ~0u);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t w = base[j] ^ u;
            if (mode == SIEVE_PROBE_WRITE_LINEAR || mode == SIEVE_PROBE_WRITE_RANDOM) {
                *((lds_u32 *)(size_t)(w * 4)) = bit;
            } else if (bytes) {
                *((lds_u8 *)(size_t)(w * 4 + (lane & 3))) = (uint8_t)lane;
            } else if (mode == SIEVE_PROBE_READ_RANDOM) {
                acc += *((lds_u32 *)(size_t)(w * 4));
            } else {
                __atomic_fetch_or((lds_u32 *)(size_t)(w * 4), bit, __ATOMIC_RELAXED);
            }
        }
    }
    __syncthreads();
    // keep the work observable
    uint32_t v = buf[tid % kWords] + acc;
    if (v == 0x9E3779B9u)
        sink[blockIdx.x] = v;
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
        hipLaunchKernelGGL(k_lds_probe, dim3(grid), dim3(kThreads), 0, 0, mode, 16, sink);  // warm-up
        hipEventRecord(e0, 0);
        hipLaunchKernelGGL(k_lds_probe, dim3(grid), dim3(kThreads), 0, 0, mode, iters, sink);
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

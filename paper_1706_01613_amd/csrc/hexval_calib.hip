// Machine ceilings of the GPU the library runs on, measured with kernels of
// known work: a read-only stream over a device buffer (the HBM read rate a
// kernel can reach), a copy (read + write), and independent FP64 FMA chains
// on every lane (the FP64 vector issue rate, and the shader clock during it).
// These set the achievable figures beside the vendor's peak numbers when the
// first passes' roofline fractions are read.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hexval_calib.h"

namespace {

constexpr int kBlock = 256;

// Every lane streams 16-byte vectors, four in flight per iteration; the XOR of
// everything read decides a store that never happens for real data (so the
// loads stay).
__global__ __launch_bounds__(kBlock) void k_read(const int4* __restrict__ p, int64_t n, unsigned* sink)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int acc = 0;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const int4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
        acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n; i += stride) {
        const int4 a = p[i];
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    if (acc == 0x5eed1e55) sink[0] = (unsigned)acc;
}

__global__ __launch_bounds__(kBlock) void k_copy(int4* __restrict__ q, const int4* __restrict__ p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) q[i] = p[i];
}

// Eight independent FMA chains per lane, `iters` steps each.  Block 0's first
// lane records the shader clock counter and the constant 100 MHz counter
// around its chains.
__global__ __launch_bounds__(kBlock) void k_fma(double* out, int64_t iters, double b, double c, uint64_t* clocks)
{
    double a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6,
           a7 = a0 + 7;
    const bool rec = blockIdx.x == 0 && threadIdx.x == 0;
    uint64_t t0 = 0, r0 = 0;
    if (rec) {
        t0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    for (int64_t k = 0; k < iters; ++k) {
        a0 = fma(a0, b, c);
        a1 = fma(a1, b, c);
        a2 = fma(a2, b, c);
        a3 = fma(a3, b, c);
        a4 = fma(a4, b, c);
        a5 = fma(a5, b, c);
        a6 = fma(a6, b, c);
        a7 = fma(a7, b, c);
    }
    if (rec) {
        clocks[0] = __builtin_amdgcn_s_memtime() - t0;
        clocks[1] = __builtin_amdgcn_s_memrealtime() - r0;
    }
    const double s = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
    if (s == 1.2345) out[blockIdx.x] = s;
}

int device_cus(int* cus)
{
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return 2;
    return hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess ? 0 : 2;
}

// Times `reps` launches of f() after one untimed launch; ms per launch.
template <typename F>
int time_reps(int reps, F f, float* ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 2;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return 2;
    }
    f();
    hipEventRecord(e0, 0);
    for (int r = 0; r < reps; ++r) f();
    hipEventRecord(e1, 0);
    int rc = hipEventSynchronize(e1) == hipSuccess && hipGetLastError() == hipSuccess ? 0 : 2;
    float t = 0.0f;
    if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = 2;
    *ms = t / reps;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}

}  // namespace

extern "C" int hexval_calib_read(const void* buf, int64_t bytes, int reps, float* ms)
{
    if (!buf || bytes < 16 || reps < 1 || !ms) return 1;
    int cus;
    if (device_cus(&cus)) return 2;
    unsigned* sink = nullptr;
    if (hipMalloc(&sink, sizeof(unsigned)) != hipSuccess) return 3;
    const int64_t n = bytes / 16;
    const int grid = cus * 8;
    const int rc = time_reps(reps, [&] { k_read<<<grid, kBlock>>>((const int4*)buf, n, sink); }, ms);
    hipFree(sink);
    return rc;
}

extern "C" int hexval_calib_copy(void* dst, const void* src, int64_t bytes, int reps, float* ms)
{
    if (!dst || !src || bytes < 16 || reps < 1 || !ms) return 1;
    int cus;
    if (device_cus(&cus)) return 2;
    const int64_t n = bytes / 16;
    const int grid = cus * 8;
    return time_reps(reps, [&] { k_copy<<<grid, kBlock>>>((int4*)dst, (const int4*)src, n); }, ms);
}

extern "C" int hexval_calib_fp64(int64_t iters, int reps, float* ms, double* flops, double* clock_mhz)
{
    if (iters < 1 || reps < 1 || !ms || !flops || !clock_mhz) return 1;
    int cus;
    if (device_cus(&cus)) return 2;
    double* out = nullptr;
    uint64_t* clocks = nullptr;
    const int grid = cus * 8;
    if (hipMalloc(&out, grid * sizeof(double)) != hipSuccess) return 3;
    if (hipMalloc(&clocks, 2 * sizeof(uint64_t)) != hipSuccess) {
        hipFree(out);
        return 3;
    }
    int rc = time_reps(reps, [&] { k_fma<<<grid, kBlock>>>(out, iters, 0.999999, 1e-7, clocks); }, ms);
    uint64_t h[2] = {0, 0};
    if (!rc && hipMemcpy(h, clocks, sizeof h, hipMemcpyDeviceToHost) != hipSuccess) rc = 2;
    *flops = 2.0 * 8.0 * (double)iters * grid * kBlock;
    *clock_mhz = h[1] ? 100.0 * (double)h[0] / (double)h[1] : 0.0;
    hipFree(out);
    hipFree(clocks);
    return rc;
}

// probe.hip -- peak-rate microbenchmarks for the roofline denominators of the
// search kernel (libmce_probe.so, a measurement aid; not part of libmce.so).
//
//   * 32-bit integer VALU: every lane runs 16 independent chains of
//     dependent XOR / AND / OR operations written as single instructions (one
//     VALU instruction = 64 lane-operations), many wavefronts per SIMD;
//   * LDS: every lane reads 16-byte words of its workgroup's LDS in a
//     conflict-free pattern (consecutive lanes, consecutive 16-byte words).
// Rates are work over the time between two HIP events around the launch.
#include "mce_probe.h"

#include <hip/hip_runtime.h>

namespace {

constexpr int kChains = 16;

__global__ void __launch_bounds__(256) valu_probe_kernel(const uint32_t* seed, uint32_t iters, uint32_t* out)
{
    uint32_t x[kChains];
    const uint32_t s = seed[threadIdx.x & 63] ^ (blockIdx.x * 0x9E3779B9u + threadIdx.x);
#pragma unroll
    for (int c = 0; c < kChains; c++) x[c] = s + (uint32_t)c * 0x01010101u;
    const uint32_t k1 = seed[64], k2 = seed[65], k3 = seed[66];
    for (uint32_t i = 0; i < iters; i++) {
        // 3 instructions per chain per iteration, written out so that the
        // compiler can neither fuse nor drop them
#pragma unroll
        for (int c = 0; c < kChains; c++) {
            asm volatile("v_xor_b32 %0, %1, %0" : "+v"(x[c]) : "s"(k1));
            asm volatile("v_and_b32 %0, %1, %0" : "+v"(x[c]) : "s"(k2));
            asm volatile("v_or_b32 %0, %1, %0" : "+v"(x[c]) : "s"(k3));
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; c++) r ^= x[c];
    if (r == 0x12345678u) out[blockIdx.x] = r; // keeps the chains live
}

__global__ void __launch_bounds__(256) lds_probe_kernel(uint32_t iters, uint32_t* out)
{
    // 16 KB per workgroup: 1024 words of 16 bytes; lane t reads word t, t + 256, ...
    __shared__ uint4 buf[1024];
    for (uint32_t i = threadIdx.x; i < 1024; i += blockDim.x) buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
    __syncthreads();
    // four 16-byte reads a lane per iteration (fixed offsets: no address
    // arithmetic in the loop), folded with one XOR per word
    uint4 acc = make_uint4(0, 0, 0, 0);
    const uint32_t t = threadIdx.x;
    for (uint32_t i = 0; i < iters; i++) {
        const uint4 v0 = buf[t], v1 = buf[t + 256], v2 = buf[t + 512], v3 = buf[t + 768];
        acc.x ^= v0.x ^ v1.x ^ v2.x ^ v3.x;
        acc.y ^= v0.y ^ v1.y ^ v2.y ^ v3.y;
        acc.z ^= v0.z ^ v1.z ^ v2.z ^ v3.z;
        acc.w ^= v0.w ^ v1.w ^ v2.w ^ v3.w;
        asm volatile("" ::: "memory"); // the reads are repeated every iteration
    }
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x12345678u) out[blockIdx.x] = acc.x;
}

int status(hipError_t e) { return e == hipSuccess ? 0 : -4; }

} // namespace

extern "C" int mce_probe_valu(uint32_t blocks, uint32_t iters, double* lane_ops_per_s, double* seconds)
{
    if (!lane_ops_per_s || blocks == 0 || iters == 0) return -1;
    uint32_t *seed = nullptr, *out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    uint32_t h_seed[67];
    for (int i = 0; i < 64; i++) h_seed[i] = 0x2545F491u * (uint32_t)(i + 1);
    h_seed[64] = 0x5bd1e995u;
    h_seed[65] = 0xfffffffeu;
    h_seed[66] = 0x00010001u;
    hipError_t e = hipMalloc(&seed, sizeof(h_seed));
    if (e == hipSuccess) e = hipMalloc(&out, 4ull * blocks);
    if (e == hipSuccess) e = hipMemcpy(seed, h_seed, sizeof(h_seed), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    float ms = 0.f;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(256), 0, nullptr, seed, 8u, out); // warm-up
        (void)hipEventRecord(a, nullptr);
        hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(256), 0, nullptr, seed, iters, out);
        (void)hipEventRecord(b, nullptr);
        e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (seed) (void)hipFree(seed);
    if (out) (void)hipFree(out);
    if (e != hipSuccess || ms <= 0.f) return status(e != hipSuccess ? e : hipErrorUnknown);
    const double ops = (double)blocks * 256.0 * (double)iters * kChains * 3.0;
    *lane_ops_per_s = ops / (ms * 1e-3);
    if (seconds) *seconds = ms * 1e-3;
    return 0;
}

extern "C" int mce_probe_lds(uint32_t blocks, uint32_t iters, double* bytes_per_s, double* seconds)
{
    if (!bytes_per_s || blocks == 0 || iters == 0) return -1;
    uint32_t* out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc(&out, 4ull * blocks);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    float ms = 0.f;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(lds_probe_kernel, dim3(blocks), dim3(256), 0, nullptr, 8u, out); // warm-up
        (void)hipEventRecord(a, nullptr);
        hipLaunchKernelGGL(lds_probe_kernel, dim3(blocks), dim3(256), 0, nullptr, iters, out);
        (void)hipEventRecord(b, nullptr);
        e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (out) (void)hipFree(out);
    if (e != hipSuccess || ms <= 0.f) return status(e != hipSuccess ? e : hipErrorUnknown);
    *bytes_per_s = (double)blocks * 256.0 * (double)iters * 64.0 / (ms * 1e-3);
    if (seconds) *seconds = ms * 1e-3;
    return 0;
}

// probe.hip -- plain device-copy kernels used as the achievable-bandwidth
// reference and to calibrate the HBM byte counters against a kernel whose
// traffic is known exactly (n bytes read, n bytes written).
#include <hip/hip_runtime.h>
#include <stdint.h>

__global__ __launch_bounds__(256) void k_copy4(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n4)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t stride = (size_t)gridDim.x * 256;
    for (; i < n4; i += stride) dst[i] = src[i];
}

typedef float f4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy4_nt(const f4v *__restrict__ src, f4v *__restrict__ dst, size_t n4)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t stride = (size_t)gridDim.x * 256;
    for (; i < n4; i += stride) {
        f4v v = __builtin_nontemporal_load(src + i);
        __builtin_nontemporal_store(v, dst + i);
    }
}

// one float per thread, no grid stride (the access shape of the LB kernels)
__global__ __launch_bounds__(256) void k_copy1(const float *__restrict__ src, float *__restrict__ dst, size_t n)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// U float4 per thread in flight, block-contiguous chunks
template <int U>
__global__ __launch_bounds__(256) void k_copyU(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n4)
{
    size_t base = ((size_t)blockIdx.x * U) * 256 + threadIdx.x;
    float4 v[U];
#pragma unroll
    for (int j = 0; j < U; j++)
        if (base + (size_t)j * 256 < n4) v[j] = src[base + (size_t)j * 256];
#pragma unroll
    for (int j = 0; j < U; j++)
        if (base + (size_t)j * 256 < n4) dst[base + (size_t)j * 256] = v[j];
}

// 41 structure-of-arrays streams (the population layout of the fused step):
// thread i copies element i of each of 41 arrays of n floats, every value read
// once and written once with a nontemporal store
__global__ __launch_bounds__(256) void k_copy_soa41(const float *__restrict__ src, float *__restrict__ dst, size_t n)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float v[41];
#pragma unroll
    for (int q = 0; q < 41; q++) v[q] = src[(size_t)q * n + i];
#pragma unroll
    for (int q = 0; q < 41; q++) __builtin_nontemporal_store(v[q], dst + (size_t)q * n + i);
}

extern "C" int pgk_probe_copy(void *dst, const void *src, size_t nbytes, int variant, int blocks, void *stream)
{
    if (!dst || !src || (nbytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15)) return -1;
    hipStream_t s = (hipStream_t)stream;
    size_t n4 = nbytes / 16;
    if (blocks <= 0) blocks = 256 * 16;
    if (variant == 0)
        hipLaunchKernelGGL(k_copy4, dim3(blocks), dim3(256), 0, s, (const float4 *)src, (float4 *)dst, n4);
    else if (variant == 1)
        hipLaunchKernelGGL(k_copy4_nt, dim3(blocks), dim3(256), 0, s, (const f4v *)src, (f4v *)dst, n4);
    else if (variant == 3)
        hipLaunchKernelGGL(k_copyU<4>, dim3((unsigned)((n4 + 1023) / 1024)), dim3(256), 0, s, (const float4 *)src,
                           (float4 *)dst, n4);
    else if (variant == 4)
        hipLaunchKernelGGL(k_copyU<8>, dim3((unsigned)((n4 + 2047) / 2048)), dim3(256), 0, s, (const float4 *)src,
                           (float4 *)dst, n4);
    else if (variant == 5)
        hipLaunchKernelGGL(k_copyU<16>, dim3((unsigned)((n4 + 4095) / 4096)), dim3(256), 0, s, (const float4 *)src,
                           (float4 *)dst, n4);
    else if (variant == 7)   // one float4 per thread, no grid stride: the fastest plain copy measured here
        hipLaunchKernelGGL(k_copyU<1>, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, (const float4 *)src,
                           (float4 *)dst, n4);
    else if (variant == 6) {
        // nbytes = 41 arrays of n floats
        if (nbytes % (41 * 4)) return -1;
        size_t n = nbytes / (41 * 4);
        hipLaunchKernelGGL(k_copy_soa41, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const float *)src,
                           (float *)dst, n);
    } else {
        size_t n = nbytes / 4;
        hipLaunchKernelGGL(k_copy1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const float *)src,
                           (float *)dst, n);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

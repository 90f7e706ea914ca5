// Device helpers shared by the step, adjoint, diagnostic and resident
// kernels: the staggered stencil sum, the per-voxel speed perturbation, and
// vector loads and stores of a cell's N memory variables (stored
// contiguously, N * 4 bytes, aligned to N * 4 bytes for N = 2, 4), with their
// non-temporal forms.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fw {

// sum_m c_m d_m with an explicit fused-multiply-add chain.  The library is
// compiled without implicit contraction, so every kernel and every
// instantiation (tile shape, batching) performs the same rounding sequence.
__device__ __forceinline__ float stencil4(const float (&c)[4], float d1, float d2, float d3, float d4)
{
    return fmaf(c[3], d4, fmaf(c[2], d3, fmaf(c[1], d2, c[0] * d1)));
}

// SplitMix64 (Steele, Lea and Flood, 2014): the hash behind the per-voxel
// speed perturbation.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// (1 + eps)^2, the factor of the bulk modulus rho c^2 (1 + eps)^2 of the cell
// with unpadded index `index`: eps = amp (2 u - 1), u from the top 24 bits of
// SplitMix64(seed ^ index).
__device__ __forceinline__ float speed_factor_sq(uint64_t seed, uint32_t index, float amp)
{
    const uint64_t h = splitmix64(seed ^ (uint64_t)index);
    const float u = (float)(h >> 40) * 0x1.0p-24f;
    const float e = amp * fmaf(2.0f, u, -1.0f);
    const float f1 = 1.0f + e;
    return f1 * f1;
}

template <int N>
__device__ __forceinline__ void load_vec(const float *__restrict__ src, float (&v)[N])
{
    if constexpr (N == 4) {
        const float4 t = *reinterpret_cast<const float4 *>(src);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (N == 2) {
        const float2 t = *reinterpret_cast<const float2 *>(src);
        v[0] = t.x; v[1] = t.y;
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = src[i];
    }
}

template <int N>
__device__ __forceinline__ void store_vec(float *__restrict__ dst, const float (&v)[N])
{
    if constexpr (N == 4) {
        *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (N == 2) {
        *reinterpret_cast<float2 *>(dst) = make_float2(v[0], v[1]);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) dst[i] = v[i];
    }
}

// Streaming accesses for data each launch touches exactly once (memory
// variables, own velocity/pressure values): the non-temporal hint lets the
// caches keep the halo planes that neighbouring tiles read again.
#ifndef FW_STREAMING
#define FW_STREAMING 1
#endif
typedef float fw_v4f __attribute__((ext_vector_type(4)));
typedef float fw_v2f __attribute__((ext_vector_type(2)));

template <int N>
__device__ __forceinline__ void load_stream(const float *__restrict__ src, float (&v)[N])
{
#if FW_STREAMING
    if constexpr (N == 4) {
        const fw_v4f t = __builtin_nontemporal_load(reinterpret_cast<const fw_v4f *>(src));
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (N == 2) {
        const fw_v2f t = __builtin_nontemporal_load(reinterpret_cast<const fw_v2f *>(src));
        v[0] = t.x; v[1] = t.y;
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = __builtin_nontemporal_load(src + i);
    }
#else
    load_vec<N>(src, v);
#endif
}

template <int N>
__device__ __forceinline__ void store_stream(float *__restrict__ dst, const float (&v)[N])
{
#if FW_STREAMING
    if constexpr (N == 4) {
        fw_v4f t = {v[0], v[1], v[2], v[3]};
        __builtin_nontemporal_store(t, reinterpret_cast<fw_v4f *>(dst));
    } else if constexpr (N == 2) {
        fw_v2f t = {v[0], v[1]};
        __builtin_nontemporal_store(t, reinterpret_cast<fw_v2f *>(dst));
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) __builtin_nontemporal_store(v[i], dst + i);
    }
#else
    store_vec<N>(dst, v);
#endif
}

__device__ __forceinline__ float load1_stream(const float *__restrict__ src)
{
#if FW_STREAMING
    return __builtin_nontemporal_load(src);
#else
    return *src;
#endif
}

__device__ __forceinline__ void store1_stream(float *__restrict__ dst, float v)
{
#if FW_STREAMING
    __builtin_nontemporal_store(v, dst);
#else
    *dst = v;
#endif
}

}  // namespace fw

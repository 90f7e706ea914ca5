// Device helpers shared by the step and adjoint kernels: vector loads and
// stores of a cell's N memory variables (stored contiguously, N * 4 bytes,
// aligned to N * 4 bytes for N = 2, 4), and their non-temporal forms.
#pragma once

#include <hip/hip_runtime.h>

namespace fw {

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

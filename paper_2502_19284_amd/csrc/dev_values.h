// dev_values.h -- streaming loads/stores and stored-value decoding shared by the product kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

template <typename T>
__device__ __forceinline__ T ntload(const T* p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void ntstore(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

// stored value -> arithmetic type
__device__ __forceinline__ double vget(const double* p) { return ntload(p); }
__device__ __forceinline__ float vget(const float* p) { return ntload(p); }
__device__ __forceinline__ float vget(const uint16_t* p) {  // bfloat16: the upper half of a float
    return __uint_as_float((uint32_t)ntload(p) << 16);
}
// a stored value already loaded -> arithmetic type (lets a kernel issue all its loads first)
__device__ __forceinline__ double vdec(double v) { return v; }
__device__ __forceinline__ float vdec(float v) { return v; }
__device__ __forceinline__ float vdec(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ double vget_plain(const double* p) { return *p; }
__device__ __forceinline__ float vget_plain(const float* p) { return *p; }
__device__ __forceinline__ float vget_plain(const uint16_t* p) {
    return __uint_as_float((uint32_t)(*p) << 16);
}

// Host stand-in for the few HIP runtime calls of the tile builder, so that it
// can be compiled with g++ and run under AddressSanitizer and UBSan on a
// machine without a GPU: "device" memory is host memory.
#pragma once
#include <cstddef>
#include <cstdlib>
#include <cstring>

#define __host__
#define __device__

typedef int hipError_t;
typedef void *hipStream_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorMemoryAllocation = 2 };
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3 };

template <class T>
inline hipError_t hipMalloc(T **p, size_t bytes) {
    *p = (T *)std::malloc(bytes ? bytes : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t b, hipMemcpyKind) {
    if (b) std::memmove(d, s, b);
    return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t) { return "host stand-in error"; }

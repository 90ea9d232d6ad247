// Host-only stand-in for the few HIP runtime calls the task-graph executor makes,
// so that the executor (CPU and GPU-domain workers, the inference pipeline) can be
// built with the thread and address sanitizers and run without a GPU: streams are
// plain heap objects, copies are memcpy, pinned allocations are malloc.
#pragma once
#include <cstdlib>
#include <cstring>
#include <cstddef>
typedef int hipError_t;
typedef struct fake_stream { int id; } *hipStream_t;
enum { hipSuccess = 0, hipStreamNonBlocking = 1 };
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new fake_stream{7}; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = std::malloc(n); return *p ? hipSuccess : 2; }
inline hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "fake"; }

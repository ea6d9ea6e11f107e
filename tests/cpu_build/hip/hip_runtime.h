// CPU shim for running the gfx950 kernel bodies as host threads (one OS
// thread per GPU thread of a block, std::barrier for __syncthreads).
#pragma once
#include <barrier>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
struct dim3 { unsigned x, y, z; dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {} };
extern thread_local dim3 blockIdx, threadIdx;
extern dim3 gridDim, blockDim;
extern thread_local std::barrier<> *emu_bar;
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define __shared__ static
#define __syncthreads() emu_bar->arrive_and_wait()
typedef int hipError_t;
typedef void *hipStream_t;
typedef void *hipEvent_t;
#define hipSuccess 0
#define hipErrorNotSupported 801
#define hipErrorInvalidValue 1
enum { hipMemcpyDeviceToHost = 2 };
extern "C" float __expf(float) throw();
extern "C" float __logf(float) throw();
static inline float rsqrtf(float x) { return 1.0f / std::sqrt(x); }
static inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
static inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
static inline int atomicOr(int32_t *p, int v) { int o = *p; *p |= v; return o; }
static inline int min(int a, int b) { return a < b ? a : b; }
static inline int max(int a, int b) { return a > b ? a : b; }
extern "C" hipError_t hipMemcpyAsync(void *, const void *, size_t, int, hipStream_t);
extern "C" hipError_t hipStreamSynchronize(hipStream_t);
extern "C" const char *hipGetErrorString(hipError_t);
typedef int hipDevice_t;
static inline hipError_t hipGetDevice(int *d) { *d = 0; return 0; }
static inline hipError_t hipStreamGetDevice(hipStream_t, hipDevice_t *d) { *d = 0; return 0; }
// one device: the host array itself stands for its device copy
#define HIP_SYMBOL(x) (&(x))
template <typename T> static inline hipError_t hipGetSymbolAddress(void **p, T *sym) { *p = (void *)sym; return 0; }
static inline hipError_t hipEventCreate(hipEvent_t *) { return 1; }
static inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return 0; }
static inline hipError_t hipEventDestroy(hipEvent_t) { return 0; }
static inline hipError_t hipEventElapsedTime(float *, hipEvent_t, hipEvent_t) { return 0; }

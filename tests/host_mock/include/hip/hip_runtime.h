// CPU mock of the HIP runtime surface used by libga's host files (server,
// batched launches, API), for running their host logic under sanitizers.
#pragma once
#include <cstddef>
#include <cstdint>
#include <cstring>

#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __shared__ static
#define __launch_bounds__(...)
#define __align__(x) alignas(x)
#define HIP_SYMBOL(x) (&x)

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 };
typedef struct MockStream* hipStream_t;
typedef struct MockEvent* hipEvent_t;
typedef struct MockGraph* hipGraph_t;
typedef struct MockGraph* hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice,
                     hipMemcpyHostToHost, hipMemcpyDefault };
enum { hipStreamNonBlocking = 1, hipHostMallocDefault = 0, hipEventDisableTiming = 2,
       hipStreamCaptureModeThreadLocal = 1, hipDeviceAttributeMultiprocessorCount = 5 };
typedef int hipStreamCaptureMode;
typedef int hipDeviceAttribute_t;

struct dim3 { uint32_t x = 1, y = 1, z = 1; dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {} };
extern dim3 threadIdx, blockIdx, blockDim, gridDim;
struct uint2 { uint32_t x, y; };
struct uint4 { uint32_t x, y, z, w; };
inline uint2 make_uint2(uint32_t a, uint32_t b) { return uint2{a, b}; }
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return uint4{a, b, c, d}; }
template <typename T> T __shfl_xor(T v, int, int = 64) { return v; }
template <typename T> T __shfl_up(T v, unsigned, int = 64) { return v; }
inline unsigned long long __ballot(int p) { return p ? 1ull : 0ull; }
template <typename T> T atomicMin(T* p, T v) { T o = *p; if (v < o) *p = v; return o; }
template <typename T> T atomicAdd(T* p, T v) { T o = *p; *p = o + v; return o; }
inline void __syncthreads() {}

hipError_t hipSetDevice(int);
hipError_t hipGetDevice(int*);
hipError_t hipDeviceGetAttribute(int*, int, int);
hipError_t hipDeviceSynchronize();
const char* hipGetErrorString(hipError_t);
hipError_t hipGetLastError();
hipError_t hipMalloc(void** p, size_t n);
template <typename T> hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags);
template <typename T> hipError_t hipHostMalloc(T** p, size_t n, unsigned flags) { return hipHostMalloc((void**)p, n, flags); }
hipError_t hipFree(void* p);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t);
hipError_t hipMemset(void* d, int v, size_t n);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t);
hipError_t hipStreamCreate(hipStream_t*);
hipError_t hipStreamCreateWithFlags(hipStream_t*, unsigned);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned);
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode);
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*);
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, void*, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t);
hipError_t hipGraphDestroy(hipGraph_t);
hipError_t hipGraphExecDestroy(hipGraphExec_t);
hipError_t hipEventCreate(hipEvent_t*);
hipError_t hipEventCreateWithFlags(hipEvent_t*, unsigned);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr);
hipError_t hipEventSynchronize(hipEvent_t);
hipError_t hipEventElapsedTime(float*, hipEvent_t, hipEvent_t);

// an operation on a stream: run now, or recorded when this thread captures
#include <functional>
void mock_enqueue(hipStream_t s, std::function<void()> op);

// Host-only stand-in for the HIP runtime: lets the request server's host logic (serve.hip) be
// compiled with g++ and run on the CPU against the mocks of server_mock.cpp.
#pragma once
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __shared__
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorUnknown = 999 };
struct ihipStream_t { int id; };
struct ihipEvent_t { int id; };
typedef ihipStream_t *hipStream_t;
typedef ihipEvent_t *hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
#define hipStreamNonBlocking 1u
#define hipHostMallocDefault 0u
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t);
hipError_t hipHostMalloc(void **p, size_t n, unsigned);
hipError_t hipHostFree(void *p);
hipError_t hipSetDevice(int);
hipError_t hipGetDevice(int *);
hipError_t hipMalloc(void **p, size_t n);
hipError_t hipFree(void *p);
const char *hipGetErrorString(hipError_t);

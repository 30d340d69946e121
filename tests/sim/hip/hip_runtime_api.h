// Test stand-in for the subset of the HIP runtime API the host engine uses.
// Only the CPU simulation tests compile against it; the product library
// links the real HIP runtime.
#pragma once
#include <stddef.h>
#include <stdint.h>
typedef int hipError_t;
#define hipSuccess 0
#define hipErrorInvalidValue 1
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
#define hipStreamNonBlocking 1
#define hipHostMallocDefault 0
#define hipHostMallocCoherent 1
#define hipHostMallocMapped 2
enum hipDeviceAttribute_t { hipDeviceAttributeWallClockRate = 1 };
struct hipDeviceProp_t { char gcnArchName[256]; int multiProcessorCount; };
hipError_t hipGetDeviceCount(int*);
hipError_t hipGetDevice(int*);
hipError_t hipGetDeviceProperties(hipDeviceProp_t*, int);
hipError_t hipDeviceGetAttribute(int*, hipDeviceAttribute_t, int);
hipError_t hipStreamCreateWithFlags(hipStream_t*, unsigned);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipDeviceSynchronize();
hipError_t hipMalloc(void**, size_t);
hipError_t hipFree(void*);
hipError_t hipHostMalloc(void**, size_t, unsigned);
hipError_t hipHostFree(void*);
hipError_t hipHostGetDevicePointer(void**, void*, unsigned);
hipError_t hipMemset(void*, int, size_t);
hipError_t hipMemcpy(void*, const void*, size_t, hipMemcpyKind);
hipError_t hipMemcpyAsync(void*, const void*, size_t, hipMemcpyKind, hipStream_t);
hipError_t hipEventRecord(hipEvent_t, hipStream_t);
#define hipEventDisableTiming 2
hipError_t hipEventCreateWithFlags(hipEvent_t*, unsigned);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipEventQuery(hipEvent_t);
hipError_t hipEventSynchronize(hipEvent_t);
const char* hipGetErrorString(hipError_t);
hipError_t hipGetLastError();
enum hipMemoryType { hipMemoryTypeUnregistered = 0, hipMemoryTypeHost = 1, hipMemoryTypeDevice = 2 };
typedef struct hipPointerAttribute_t {
  enum hipMemoryType type;
  int device;
  void* devicePointer;
  void* hostPointer;
  int isManaged;
  unsigned allocationFlags;
} hipPointerAttribute_t;
hipError_t hipPointerGetAttributes(hipPointerAttribute_t*, const void*);

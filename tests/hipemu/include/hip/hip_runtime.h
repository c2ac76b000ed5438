// hip/hip_runtime.h for the CPU emulation of the host runtime (test
// infrastructure only).  Declares the subset of the HIP runtime API that the
// library's host code uses; tests/hipemu/hipemu.cpp implements it on the host,
// with every "device" allocation in ordinary memory and every kernel replaced
// by a host routine that has the kernel's effect on the buffers the host reads
// back.  Device-side keywords compile away.
#pragma once

#include <stddef.h>
#include <stdint.h>

#define __host__
#define __device__
#define __global__
#define __align__(n) __attribute__((aligned(n)))
#define __launch_bounds__(...)
#define HIP_SYMBOL(x) ((const void*)&(x))

enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorInvalidDevice = 101,
    hipErrorInvalidSymbol = 701,
    hipErrorNotReady = 600,
    hipErrorNotSupported = 801,
    hipErrorUnknown = 999,
};

enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1,
                            hipStreamCaptureModeRelaxed = 2 };

#define hipHostMallocDefault 0x0u
#define hipHostMallocMapped 0x2u
#define hipHostMallocCoherent 0x40000000u
#define hipStreamNonBlocking 0x1u
#define hipEventDisableTiming 0x2u

typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph* hipGraph_t;
typedef struct hipGraphExec* hipGraphExec_t;
typedef struct hipGraphNode* hipGraphNode_t;
typedef struct ihipModule_t* hipModule_t;
typedef struct ihipModuleSymbol_t* hipFunction_t;

struct dim3 {
    uint32_t x, y, z;
    dim3(uint32_t x_ = 1, uint32_t y_ = 1, uint32_t z_ = 1) : x(x_), y(y_), z(z_) {}
};

struct hipDeviceProp_t {
    char name[256];
    char gcnArchName[256];
    int multiProcessorCount;
};

hipError_t hipGetDeviceCount(int* count);
hipError_t hipSetDevice(int device);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int device);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);

hipError_t hipMalloc(void** ptr, size_t bytes);
template <class T>
inline hipError_t hipMalloc(T** ptr, size_t bytes)
{
    return hipMalloc(reinterpret_cast<void**>(ptr), bytes);
}
hipError_t hipFree(void* ptr);
hipError_t hipHostMalloc(void** ptr, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* ptr);
hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned flags);
hipError_t hipGetSymbolAddress(void** dev, const void* symbol);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t stream);
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t stream);

hipError_t hipStreamCreateWithFlags(hipStream_t* stream, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t stream);
hipError_t hipStreamSynchronize(hipStream_t stream);
hipError_t hipStreamQuery(hipStream_t stream);
hipError_t hipStreamWaitEvent(hipStream_t stream, hipEvent_t event, unsigned flags);

hipError_t hipEventCreate(hipEvent_t* event);
hipError_t hipEventCreateWithFlags(hipEvent_t* event, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t event);
hipError_t hipEventRecord(hipEvent_t event, hipStream_t stream);
hipError_t hipEventQuery(hipEvent_t event);
hipError_t hipEventSynchronize(hipEvent_t event);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t start, hipEvent_t stop);

hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* blocks, const void* kernel, int block_size,
                                                        size_t dyn_shared);
hipError_t hipLaunchKernel(const void* kernel, dim3 grid, dim3 block, void** args, size_t shared,
                           hipStream_t stream);

hipError_t hipStreamBeginCapture(hipStream_t stream, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t stream, hipGraph_t* graph);
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, hipGraphNode_t* error_node, char* log,
                               size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t stream);
hipError_t hipGraphDestroy(hipGraph_t graph);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);

hipError_t hipModuleLoadData(hipModule_t* module, const void* image);
hipError_t hipModuleGetFunction(hipFunction_t* function, hipModule_t module, const char* name);
hipError_t hipModuleUnload(hipModule_t module);
hipError_t hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(int* blocks, hipFunction_t f, int block_size,
                                                              size_t dyn_shared);
hipError_t hipModuleLaunchKernel(hipFunction_t f, unsigned gx, unsigned gy, unsigned gz, unsigned bx, unsigned by,
                                 unsigned bz, unsigned shared, hipStream_t stream, void** args, void** extra);

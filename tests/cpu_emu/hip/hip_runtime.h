// CPU emulation of the subset of HIP used by paper_2209_04634_amd/csrc (TEST INFRASTRUCTURE).
//
// Lets the unmodified kernel and runtime sources compile with a host C++ compiler so their exact
// logic can be executed and bounds-checked (optionally under AddressSanitizer) without a GPU.
// Each GPU thread runs as a fiber; wave64 intrinsics are lockstep rendezvous among the live lanes
// of a wave; __syncthreads() is a barrier among the live threads of the block; blocks run one after
// another.  Runtime API calls are synchronous host operations.  Every emulated API symbol is
// renamed (emu_*) so nothing here can bind to, or be bound by, a real HIP runtime in the process.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <cstdint>
#include <functional>
#include <tuple>
#include <type_traits>
#include <utility>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define __shared__ thread_local
#ifndef __restrict__
#define __restrict__ __restrict
#endif

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_uint3 {
    unsigned x, y, z;
};

typedef int hipError_t;
enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorLaunchFailure = 719,
};
typedef struct emu_stream_t* hipStream_t;
typedef struct emu_event_t* hipEvent_t;
enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
};
enum hipMemoryType {
    hipMemoryTypeUnregistered = 0,
    hipMemoryTypeHost = 1,
    hipMemoryTypeDevice = 2,
};
typedef struct hipPointerAttribute_t {
    enum hipMemoryType type;
    int device;
    void* devicePointer;
    void* hostPointer;
    int isManaged;
    unsigned allocationFlags;
} hipPointerAttribute_t;
#define hipStreamNonBlocking 0x01
#define hipEventDisableTiming 0x02

// ---- thread geometry of the fiber currently running
const emu_uint3& emu_thread_idx();
const emu_uint3& emu_block_idx();
const dim3& emu_block_dim();
const dim3& emu_grid_dim();
#define threadIdx (emu_thread_idx())
#define blockIdx (emu_block_idx())
#define blockDim (emu_block_dim())
#define gridDim (emu_grid_dim())

// ---- barriers and wave intrinsics (line numbers detect divergent use)
void emu_syncthreads(int line);
uint64_t emu_wave_exchange(int op, uint64_t value, int arg, int line);
enum { EMU_SHFL = 0, EMU_SHFL_UP = 1, EMU_BALLOT = 2, EMU_SHFL_DOWN = 3 };

#define __syncthreads() emu_syncthreads(__LINE__)

template <class T>
inline T emu_from_bits(uint64_t b) {
    T v;
    memcpy(&v, &b, sizeof(T));
    return v;
}
template <class T>
inline uint64_t emu_to_bits(T v) {
    static_assert(sizeof(T) <= 8, "64-bit max");
    uint64_t b = 0;
    memcpy(&b, &v, sizeof(T));
    return b;
}
template <class T>
inline T emu_shfl(T v, int src, int width, int line) {
    (void)width;
    return emu_from_bits<T>(emu_wave_exchange(EMU_SHFL, emu_to_bits(v), src, line));
}
template <class T>
inline T emu_shfl_up(T v, unsigned delta, int width, int line) {
    (void)width;
    return emu_from_bits<T>(emu_wave_exchange(EMU_SHFL_UP, emu_to_bits(v), (int)delta, line));
}
template <class T>
inline T emu_shfl_down(T v, unsigned delta, int width, int line) {
    (void)width;
    return emu_from_bits<T>(emu_wave_exchange(EMU_SHFL_DOWN, emu_to_bits(v), (int)delta, line));
}
#define __shfl(v, src, ...) emu_shfl((v), (src), 64, __LINE__)
#define __shfl_down(v, d, ...) emu_shfl_down((v), (d), 64, __LINE__)
#define __shfl_up(v, d, ...) emu_shfl_up((v), (d), 64, __LINE__)
#define __ballot(p) ((unsigned long long)emu_wave_exchange(EMU_BALLOT, (p) ? 1 : 0, 0, __LINE__))
#define __any(p) (__ballot(p) != 0ull ? 1 : 0)

inline int __popc(unsigned v) { return __builtin_popcount(v); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __ffs(unsigned v) { return __builtin_ffs((int)v); }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
inline unsigned __umul24(unsigned a, unsigned b) { return (a & 0xFFFFFFu) * (b & 0xFFFFFFu); }

// single OS thread runs every fiber: plain read-modify-write is atomic
template <class T, class U>
inline T atomicAdd(T* p, U v) {
    T old = *p;
    *p = (T)(old + (T)v);
    return old;
}

template <class A, class B>
inline typename std::common_type<A, B>::type min(A a, B b) {
    typedef typename std::common_type<A, B>::type C;
    return (C)a < (C)b ? (C)a : (C)b;
}
template <class A, class B>
inline typename std::common_type<A, B>::type max(A a, B b) {
    typedef typename std::common_type<A, B>::type C;
    return (C)a > (C)b ? (C)a : (C)b;
}

// ---- kernel launch: every block of the grid, one fiber per thread
void emu_run_grid(dim3 grid, dim3 block, size_t shmem, const std::function<void()>& body,
                  const char* name);

// Stream capture (HIP graphs): while a capture is open, launches and asynchronous copies are
// recorded, not run; a launched graph runs its records in order (a memcpy node reads its source
// when it runs, as on the device).
bool emu_capturing();
void emu_record(std::function<void()> op);
// Queues work on a stream: run at once, or (deferred execution) when a synchronisation reaches it.
void emu_submit(hipStream_t s, std::function<void()> op);

template <class... P, class... A>
inline void emu_launch(const char* name, void (*k)(P...), dim3 grid, dim3 block, size_t shmem,
                       hipStream_t stream, A... args) {
    std::tuple<typename std::decay<P>::type...> params(args...);
    auto op = [=]() {
        auto p = params;
        emu_run_grid(grid, block, shmem, [&]() { std::apply(k, p); }, name);
    };
    if (emu_capturing()) {
        emu_record(op);
        return;
    }
    emu_submit(stream, op);
}
#define hipLaunchKernelGGL(k, grid, block, shmem, stream, ...) \
    emu_launch(#k, k, grid, block, shmem, stream, __VA_ARGS__)

// ---- runtime API (synchronous by default; see emu_set_execution for deferred execution)
#define hipMalloc emu_hipMalloc
#define hipFree emu_hipFree
#define hipHostMalloc emu_hipHostMalloc
#define hipHostFree emu_hipHostFree
#define hipMemcpy emu_hipMemcpy
#define hipMemcpyAsync emu_hipMemcpyAsync
#define hipMemcpy2DAsync emu_hipMemcpy2DAsync
#define hipMemsetAsync emu_hipMemsetAsync
#define hipStreamCreateWithFlags emu_hipStreamCreateWithFlags
#define hipStreamSynchronize emu_hipStreamSynchronize
#define hipStreamDestroy emu_hipStreamDestroy
#define hipEventCreate emu_hipEventCreate
#define hipPointerGetAttributes emu_hipPointerGetAttributes
#define hipEventCreateWithFlags emu_hipEventCreateWithFlags
#define hipStreamWaitEvent emu_hipStreamWaitEvent
#define hipEventRecord emu_hipEventRecord
#define hipEventSynchronize emu_hipEventSynchronize
#define hipEventElapsedTime emu_hipEventElapsedTime
#define hipEventDestroy emu_hipEventDestroy
#define hipGetLastError emu_hipGetLastError
#define hipGetErrorString emu_hipGetErrorString
#define hipGetDevice emu_hipGetDevice
#define hipGetDeviceProperties emu_hipGetDeviceProperties
#define hipStreamBeginCapture emu_hipStreamBeginCapture
#define hipStreamEndCapture emu_hipStreamEndCapture
#define hipGraphInstantiate emu_hipGraphInstantiate
#define hipGraphLaunch emu_hipGraphLaunch
#define hipGraphDestroy emu_hipGraphDestroy
#define hipGraphExecDestroy emu_hipGraphExecDestroy
#define hipGetSymbolAddress emu_hipGetSymbolAddress
#define HIP_SYMBOL(x) ((const void*)&(x))

hipError_t emu_hipMalloc(void** p, size_t n);
hipError_t emu_hipFree(void* p);
hipError_t emu_hipHostMalloc(void** p, size_t n, unsigned flags);
hipError_t emu_hipHostFree(void* p);
hipError_t emu_hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k);
hipError_t emu_hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k,
                              hipStream_t s);
hipError_t emu_hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch,
                                size_t width, size_t height, hipMemcpyKind k, hipStream_t s);
hipError_t emu_hipMemsetAsync(void* p, int v, size_t n, hipStream_t s);
hipError_t emu_hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t emu_hipStreamSynchronize(hipStream_t s);
hipError_t emu_hipStreamDestroy(hipStream_t s);
hipError_t emu_hipEventCreate(hipEvent_t* e);
hipError_t emu_hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p);
hipError_t emu_hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t emu_hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t emu_hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t emu_hipEventSynchronize(hipEvent_t e);
hipError_t emu_hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t emu_hipEventDestroy(hipEvent_t e);
hipError_t emu_hipGetLastError();
const char* emu_hipGetErrorString(hipError_t e);
hipError_t emu_hipGetDevice(int* dev);
struct hipDeviceProp_t {
    char gcnArchName[256];
};
hipError_t emu_hipGetDeviceProperties(hipDeviceProp_t* p, int dev);
typedef struct emu_graph_t* hipGraph_t;
typedef struct emu_graph_t* hipGraphExec_t;
typedef struct emu_graph_node_t* hipGraphNode_t;
enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1,
       hipStreamCaptureModeRelaxed = 2 };
typedef int hipStreamCaptureMode;
hipError_t emu_hipStreamBeginCapture(hipStream_t s, int mode);
hipError_t emu_hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t emu_hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* err,
                                   char* log, size_t log_size);
hipError_t emu_hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t emu_hipGraphDestroy(hipGraph_t g);
hipError_t emu_hipGraphExecDestroy(hipGraphExec_t e);
// a __device__ variable is host memory here: its "device address" is its own address
hipError_t emu_hipGetSymbolAddress(void** p, const void* symbol);

// Host stand-in for <hip/hip_runtime.h> used by the kernel bounds check
// (tests/test_kernel_bounds_cpu.py): the library's kernels compile as plain
// C++ and run on the CPU, one fiber per GPU thread and one block after
// another, with block (__syncthreads) and wavefront barriers and shuffles.
// Device memory is host memory from exact-size allocations, so
// AddressSanitizer reports any kernel access outside a buffer. Matrix-core
// calls return their accumulator unchanged (their operands are still read):
// the check concerns addresses, not values.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <tuple>
#include <type_traits>
#include <utility>

#define __global__
#define __device__
#define __align__(n) __attribute__((aligned(n)))
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_u3 {
    unsigned x, y, z;
};
struct EmuCtx {
    emu_u3 tid, bid;
    dim3 bdim, gdim;
};
EmuCtx *emu_ctx();
#define threadIdx (emu_ctx()->tid)
#define blockIdx (emu_ctx()->bid)
#define blockDim (emu_ctx()->bdim)
#define gridDim (emu_ctx()->gdim)

void emu_syncthreads();
void emu_wave_barrier();
void *emu_wave_xchg();          // 64 x 8 bytes, shared by the wave
void *emu_dyn_shared();
#define __syncthreads() emu_syncthreads()
#define __builtin_amdgcn_wave_barrier() emu_wave_barrier()
#define __builtin_amdgcn_fence(a, b) ((void)0)
#define __builtin_amdgcn_readfirstlane(x) (x)
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
inline float cospif(float x) { return float(std::cos(3.14159265358979323846 * double(x))); }
template <class A, class B, class C>
inline C emu_mfma(const A &a, const B &b, const C &c)
{
    volatile float sink = float(a[0]) + float(b[0]);
    (void)sink;
    return c;
}
#define __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, x, y, z) emu_mfma(a, b, c)

template <class T>
inline T emu_shfl(T v, int src)
{
    const int lane = int(threadIdx.x & 63);
    T *slot = static_cast<T *>(emu_wave_xchg());
    slot[lane] = v;
    emu_wave_barrier();
    T r = slot[src];
    emu_wave_barrier();
    return r;
}
template <class T>
inline T __shfl_xor(T v, int mask, int width = 64)
{
    return emu_shfl(v, int(threadIdx.x & 63) ^ mask);
}
template <class T>
inline T __shfl_up(T v, unsigned d, int width = 64)
{
    const int lane = int(threadIdx.x & 63);
    const int s = lane - int(d);
    return emu_shfl(v, s >= 0 ? s : lane);
}
template <class T>
inline T __shfl_down(T v, unsigned d, int width = 64)
{
    const int lane = int(threadIdx.x & 63);
    const int s = lane + int(d);
    return emu_shfl(v, s < 64 ? s : lane);
}

template <class A, class B>
inline auto min(A a, B b) -> typename std::common_type<A, B>::type
{
    typedef typename std::common_type<A, B>::type T;
    return T(a) < T(b) ? T(a) : T(b);
}
template <class A, class B>
inline auto max(A a, B b) -> typename std::common_type<A, B>::type
{
    typedef typename std::common_type<A, B>::type T;
    return T(a) < T(b) ? T(b) : T(a);
}

struct uint2 {
    unsigned x, y;
};
struct uint4 {
    unsigned x, y, z, w;
};
struct float2 {
    float x, y;
};
struct float4 {
    float x, y, z, w;
};
inline uint2 make_uint2(unsigned a, unsigned b) { return uint2{a, b}; }
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return uint4{a, b, c, d}; }
inline float2 make_float2(float a, float b) { return float2{a, b}; }
inline float4 make_float4(float a, float b, float c, float d) { return float4{a, b, c, d}; }

typedef int hipError_t;
enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotSupported = 801,
};
typedef struct EmuStream *hipStream_t;
typedef struct EmuEvent *hipEvent_t;
typedef struct EmuGraph *hipGraph_t;
typedef struct EmuGraphExec *hipGraphExec_t;
typedef struct EmuGraphNode *hipGraphNode_t;
enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
};
enum hipStreamCaptureMode {
    hipStreamCaptureModeGlobal = 0,
    hipStreamCaptureModeThreadLocal = 1,
    hipStreamCaptureModeRelaxed = 2
};
#define hipStreamNonBlocking 1u
#define hipHostMallocDefault 0u

const char *hipGetErrorString(hipError_t e);
hipError_t hipGetLastError();
hipError_t hipGetDeviceCount(int *n);
hipError_t hipSetDevice(int d);
hipError_t hipDeviceSynchronize();
hipError_t hipMemGetInfo(size_t *fr, size_t *tot);
hipError_t hipMalloc(void **p, size_t n);
// a __device__ variable is host memory here: its address is the symbol
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void **p, const void *sym)
{
    *p = const_cast<void *>(sym);
    return hipSuccess;
}
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t n, unsigned flags);
hipError_t hipHostFree(void *p);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphGetNodes(hipGraph_t g, hipGraphNode_t *nodes, size_t *n);
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *err, char *log, size_t sz);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);

// kernel launch: every block runs to completion before the next one starts
void emu_run_grid(void (*entry)(void *), void *arg, dim3 g, dim3 b, size_t shmem, const char *name);

template <class Tup, class K>
struct EmuLaunch {
    K k;
    Tup args;
    static void entry(void *p)
    {
        auto *self = static_cast<EmuLaunch *>(p);
        std::apply(self->k, self->args);
    }
};

template <class... P, class... A>
void emu_launch(void (*k)(P...), dim3 g, dim3 b, size_t sh, const char *name, A &&...args)
{
    typedef std::tuple<typename std::decay<P>::type...> Tup;
    EmuLaunch<Tup, void (*)(P...)> L{k, Tup(std::forward<A>(args)...)};
    emu_run_grid(&EmuLaunch<Tup, void (*)(P...)>::entry, &L, g, b, sh, name);
}
#define hipLaunchKernelGGL(K, G, B, SH, S, ...) emu_launch(K, dim3(G), dim3(B), size_t(SH), #K, __VA_ARGS__)

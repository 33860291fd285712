// hip_runtime.h -- CPU stand-in for the HIP runtime and device builtins,
// used only to build the library's kernel sources as host code for tests
// (tests/hostemu).  It is never used by the GPU build.
//
// Execution model: a launch runs its blocks one after another; the threads
// of a block are cooperative fibers on one OS thread, switched only at
// barriers (__syncthreads and the wavefront operations), in thread order.
// Wavefront operations (__ballot, __shfl*) exchange values through a
// per-wavefront slot array between two wavefront barriers, so every lane that
// has not exited must reach the same call (as on the GPU, where the
// operation would otherwise read inactive lanes); a wavefront whose lanes
// wait at different barriers aborts the run.  __shared__ variables are
// function-scope statics: blocks run one at a time, so a static is exactly
// the block's shared copy.  "Device" memory is host memory.
#pragma once

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <tuple>
#include <type_traits>
#include <utility>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __shared__ static
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))

// ---------------------------------------------------------------- vector types
struct uint3 {
    unsigned x, y, z;
};
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct int2 {
    int x, y;
};
struct uint4 {
    unsigned x, y, z, w;
};
struct int4 {
    int x, y, z, w;
};
struct float4 {
    float x, y, z, w;
};
struct double2 {
    double x, y;
};
struct double4 {
    double x, y, z, w;
};
inline int2 make_int2(int a, int b) { return int2{a, b}; }
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return uint4{a, b, c, d}; }
inline int4 make_int4(int a, int b, int c, int d) { return int4{a, b, c, d}; }
inline double2 make_double2(double a, double b) { return double2{a, b}; }
inline double4 make_double4(double a, double b, double c, double d) { return double4{a, b, c, d}; }
inline float4 make_float4(float a, float b, float c, float d) { return float4{a, b, c, d}; }

inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }

// ---------------------------------------------------------------- fibers
namespace hipemu {

struct Fiber;
Fiber *current();
const uint3 &thread_idx();
const uint3 &block_idx();
const dim3 &block_dim();
const dim3 &grid_dim();
void block_barrier();
// exchange 8 bytes with the lanes of the wavefront: all lanes store theirs,
// then read slot `src`; returns the value of lane src (or of this lane when
// src is outside the wavefront)
uint64_t wave_exchange(uint64_t mine, int src);
uint64_t wave_ballot(bool pred);
int lane_id();
void run_launch(dim3 grid, dim3 block, void (*thread_fn)(void *), void *arg);

template <class T> inline uint64_t to_bits(T v)
{
    static_assert(sizeof(T) <= 8, "8-byte lanes");
    uint64_t u = 0;
    memcpy(&u, &v, sizeof(T));
    return u;
}
template <class T> inline T from_bits(uint64_t u)
{
    T v;
    memcpy(&v, &u, sizeof(T));
    return v;
}

struct Cfg {
    dim3 grid, block;
};
inline Cfg cfg(dim3 g, dim3 b, size_t = 0, void * = nullptr) { return Cfg{g, b}; }

template <class Tuple, class K> struct LaunchArg {
    K kernel;
    Tuple args;
};

template <class Tuple, class K> void thread_entry(void *p)
{
    auto *a = static_cast<LaunchArg<Tuple, K> *>(p);
    Tuple local = a->args;  // each thread gets its own copy of the arguments
    std::apply(a->kernel, local);
}

template <class... P, class... A> void launch(Cfg c, void (*k)(P...), A &&...a)
{
    using Tuple = std::tuple<std::decay_t<P>...>;
    LaunchArg<Tuple, void (*)(P...)> arg{k, Tuple(std::forward<A>(a)...)};
    run_launch(c.grid, c.block, &thread_entry<Tuple, void (*)(P...)>, &arg);
}

}  // namespace hipemu

#define threadIdx (hipemu::thread_idx())
#define blockIdx (hipemu::block_idx())
#define blockDim (hipemu::block_dim())
#define gridDim (hipemu::grid_dim())

inline void __syncthreads() { hipemu::block_barrier(); }
inline int __lane_id() { return hipemu::lane_id(); }
inline uint64_t __ballot(int pred) { return hipemu::wave_ballot(pred != 0); }
template <class T> inline T __shfl(T v, int src, int = 64)
{
    return hipemu::from_bits<T>(hipemu::wave_exchange(hipemu::to_bits(v), src & 63));
}
template <class T> inline T __shfl_xor(T v, int mask, int = 64)
{
    return hipemu::from_bits<T>(hipemu::wave_exchange(hipemu::to_bits(v), hipemu::lane_id() ^ mask));
}
template <class T> inline T __shfl_up(T v, unsigned delta, int = 64)
{
    const int l = hipemu::lane_id();
    const int s = l - (int)delta;
    return hipemu::from_bits<T>(hipemu::wave_exchange(hipemu::to_bits(v), s < 0 ? l : s));
}
// The library applies readfirstlane only to values that are the same on
// every lane (it moves them to scalar registers), and may do so inside
// divergent code, where a lane exchange cannot run: the lane's own value is
// the wavefront's.
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }
// Buffer descriptors: base and size in bytes.  Every access of the library
// lies inside its descriptor (the hardware would return 0 for a load beyond
// it and drop a store), so an access outside one stops the run here.
namespace hipemu {
struct BufRsrc {
    char *base;
    uint32_t bytes;
};
inline char *buf_at(BufRsrc r, uint32_t voff, uint32_t soff, uint32_t n)
{
    const uint64_t o = (uint64_t)voff + soff;
    if (o + n > r.bytes) {
        fprintf(stderr, "hostemu: buffer access at byte %llu (+%u) beyond a descriptor of %u bytes\n",
                (unsigned long long)o, n, r.bytes);
        abort();
    }
    return r.base + o;
}
}  // namespace hipemu
#define __amdgpu_buffer_rsrc_t hipemu::BufRsrc
inline hipemu::BufRsrc __builtin_amdgcn_make_buffer_rsrc(void *p, short, int bytes, int)
{
    return hipemu::BufRsrc{(char *)p, (uint32_t)bytes};
}
#define HIPEMU_BUF_IO(bits, T)                                                                        \
    inline T __builtin_amdgcn_raw_buffer_load_b##bits(hipemu::BufRsrc r, uint32_t vo, uint32_t so, int) \
    {                                                                                                 \
        T v;                                                                                          \
        memcpy(&v, hipemu::buf_at(r, vo, so, sizeof(T)), sizeof(T));                                  \
        return v;                                                                                     \
    }                                                                                                 \
    inline void __builtin_amdgcn_raw_buffer_store_b##bits(T v, hipemu::BufRsrc r, uint32_t vo, uint32_t so, int) \
    {                                                                                                 \
        memcpy(hipemu::buf_at(r, vo, so, sizeof(T)), &v, sizeof(T));                                  \
    }
typedef unsigned int hipemu_u32x2 __attribute__((ext_vector_type(2)));
HIPEMU_BUF_IO(16, unsigned short)
HIPEMU_BUF_IO(32, uint32_t)
HIPEMU_BUF_IO(64, hipemu_u32x2)
#undef HIPEMU_BUF_IO

inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __clz(int v) { return v == 0 ? 32 : __builtin_clz((unsigned)v); }
inline int __ffsll(unsigned long long v) { return __builtin_ffsll((long long)v); }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }

// ---------------------------------------------------------------- atomics
// one OS thread runs every fiber and fibers switch only at barriers, so a
// read-modify-write is atomic as written; the operand converts to the
// pointee type (as HIP's overloads do for enums and literals)
namespace hipemu {
template <class T> struct same {
    using type = T;
};
}  // namespace hipemu
template <class T> inline T atomicAdd(T *p, typename hipemu::same<T>::type v)
{
    T o = *p;
    *p = o + v;
    return o;
}
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v)
{
    unsigned long long o = *p;
    *p = o + v;
    return o;
}
template <class T> inline T atomicMax(T *p, typename hipemu::same<T>::type v)
{
    T o = *p;
    if (v > o) *p = v;
    return o;
}
template <class T> inline T atomicMin(T *p, typename hipemu::same<T>::type v)
{
    T o = *p;
    if (v < o) *p = v;
    return o;
}
template <class T> inline T atomicOr(T *p, typename hipemu::same<T>::type v)
{
    T o = *p;
    *p = o | v;
    return o;
}

template <class T>
inline T atomicCAS(T *p, typename hipemu::same<T>::type cmp, typename hipemu::same<T>::type v)
{
    T o = *p;
    if (o == cmp) *p = v;
    return o;
}

inline double __dadd_rn(double a, double b) { return a + b; }
inline double __dmul_rn(double a, double b) { return a * b; }
inline double __dsub_rn(double a, double b) { return a - b; }

#define __builtin_amdgcn_sched_barrier(x) ((void)0)
inline float __builtin_amdgcn_rcpf(float x) { return 1.0f / x; }
inline float __builtin_amdgcn_exp2f(float x) { return exp2f(x); }
typedef short hipemu_v4s __attribute__((ext_vector_type(4)));
typedef float hipemu_v4f __attribute__((ext_vector_type(4)));
hipemu_v4f hipemu_mfma_16x16x16_bf16(hipemu_v4s a, hipemu_v4s b, hipemu_v4f c);
#define __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, x, y, z) hipemu_mfma_16x16x16_bf16(a, b, c)

// ---------------------------------------------------------------- runtime
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorUnknown = 999, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 };
typedef enum {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
} hipMemcpyKind;
typedef struct hipemu_stream *hipStream_t;
typedef struct hipemu_event *hipEvent_t;

hipError_t hipMalloc(void **p, size_t n);
template <class T> inline hipError_t hipMalloc(T **p, size_t n) { return hipMalloc((void **)p, n); }
hipError_t hipFree(void *p);
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st = nullptr);
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t st = nullptr);
hipError_t hipStreamSynchronize(hipStream_t st);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t st = nullptr);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetSymbolAddress(void **p, const void *sym);
inline hipError_t hipGetDevice(int *dev)
{
    *dev = 0;
    return hipSuccess;
}

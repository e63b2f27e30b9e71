// Host emulation of the small part of the HIP runtime and device language that
// libsfft's sources use, for running the library's kernels on the CPU under
// AddressSanitizer or ThreadSanitizer (test infrastructure only; the product is
// built with hipcc for gfx950 and never sees this header).
//
// A launch runs its work-groups one after another; each work-group is
// blockDim.x host threads.  __syncthreads() is a checked barrier: every thread
// of the work-group must reach the same barrier (file and line), else the run
// stops with a report; a barrier that some threads never reach is reported
// after a time-out.  Wavefront-wide operations (the FP32 matrix instruction)
// exchange their operands through a per-wave buffer between two wave barriers.
// __shared__ variables become function statics (one work-group runs at a
// time); the dynamic LDS array is one heap block of exactly the launch's size,
// so ASan sees any access past it.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

// ------------------------------------------------------------ qualifiers ----
#define __global__
#define __device__
#define __host__
#define __shared__ static
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define amdgpu_waves_per_eu(n) unused

// ------------------------------------------------------------ vector types --
struct double2 { double x, y; };
struct float2 { float x, y; };
struct uint4 { unsigned x, y, z, w; };
inline double2 make_double2(double x, double y) { return double2{x, y}; }
inline float2 make_float2(float x, float y) { return float2{x, y}; }
inline uint4 make_uint4(unsigned x, unsigned y, unsigned z, unsigned w) { return uint4{x, y, z, w}; }

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace emu {
struct Idx { unsigned x, y, z; };
extern thread_local Idx t_thread, t_block;
extern Idx g_block_dim, g_grid_dim;
void syncthreads(const char* file, int line);
void mfma_f32_16x16x4(float a, float b, const float* c, float* d);
long long wall_clock();
char* dyn_lds();
}  // namespace emu

#define threadIdx (::emu::t_thread)
#define blockIdx (::emu::t_block)
#define blockDim (::emu::g_block_dim)
#define gridDim (::emu::g_grid_dim)
#define __syncthreads() ::emu::syncthreads(__FILE__, __LINE__)

// --------------------------------------------------------- device builtins --
#define EMU_MINMAX(T)                                   \
  inline T min(T a, T b) { return a < b ? a : b; }      \
  inline T max(T a, T b) { return a < b ? b : a; }
EMU_MINMAX(int)
EMU_MINMAX(unsigned)
EMU_MINMAX(long)
EMU_MINMAX(unsigned long)
EMU_MINMAX(long long)
EMU_MINMAX(unsigned long long)
EMU_MINMAX(float)
EMU_MINMAX(double)
#undef EMU_MINMAX
template <typename T>
inline T min(T a, T b) { return a < b ? a : b; }
template <typename T>
inline T max(T a, T b) { return a < b ? b : a; }

inline uint64_t __umul64hi(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
}
inline uint32_t __umul24(uint32_t a, uint32_t b) {
  return (uint32_t)((uint64_t)(a & 0xFFFFFFu) * (uint64_t)(b & 0xFFFFFFu));
}
inline unsigned __float_as_uint(float f) {
  unsigned u;
  memcpy(&u, &f, 4);
  return u;
}
inline float __uint_as_float(unsigned u) {
  float f;
  memcpy(&f, &u, 4);
  return f;
}
inline long long __double_as_longlong(double f) {
  long long u;
  memcpy(&u, &f, 8);
  return u;
}
inline void sincospi(double x, double* s, double* c) {
  *s = std::sin(M_PI * x);
  *c = std::cos(M_PI * x);
}
inline void sincospif(float x, float* s, float* c) {
  *s = (float)std::sin(M_PI * (double)x);
  *c = (float)std::cos(M_PI * (double)x);
}
inline long long wall_clock64() { return ::emu::wall_clock(); }

// atomics: sequentially consistent read-modify-writes (GCC builtins, which both
// sanitizers understand)
inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicAdd(unsigned* p, unsigned v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline float atomicAdd(float* p, float v) {
  float old, nw;
  __atomic_load(p, &old, __ATOMIC_SEQ_CST);
  do {
    nw = old + v;
  } while (!__atomic_compare_exchange(p, &old, &nw, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST));
  return old;
}

#if defined(__clang__)
typedef float emu_floatx4 __attribute__((ext_vector_type(4)));
#else
typedef float emu_floatx4 __attribute__((vector_size(16)));
#endif
inline emu_floatx4 emu_mfma(float a, float b, emu_floatx4 c) {
  float cin[4] = {c[0], c[1], c[2], c[3]}, d[4];
  ::emu::mfma_f32_16x16x4(a, b, cin, d);
  return emu_floatx4{d[0], d[1], d[2], d[3]};
}
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) emu_mfma((a), (b), (c))
#define __builtin_amdgcn_sched_group_barrier(a, b, c) ((void)0)
// The kernels apply it only to values that are the same on every lane of the wave
// (the wave index), where lane 0's value is the thread's own.
#define __builtin_amdgcn_readfirstlane(v) (v)

// ------------------------------------------------------------- runtime API --
typedef int hipError_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotInitialized = 3,
  hipErrorInvalidDevice = 101,
  hipErrorInvalidSymbol = 13,
  hipErrorLaunchFailure = 719,
};
typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef enum {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
struct hipDeviceProp_t {
  int multiProcessorCount;
  size_t sharedMemPerBlock;
  char name[256];
};

hipError_t hipGetDevice(int* d);
hipError_t hipSetDevice(int d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
hipError_t hipMalloc(void** p, size_t n);
hipError_t hipFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st = 0);
hipError_t hipMemset(void* p, int v, size_t n);
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t st = 0);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute a, int v);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = 0);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
#define HIP_SYMBOL(x) ((const void*)&(x))

namespace emu {
struct Launch {
  dim3 grid, block;
  size_t lds;
};
void run_blocks(const Launch& l, void (*body)(void*), void* ctx);
}  // namespace emu

// Kernel launch: every work-group of the grid in turn, blockDim.x threads each.
template <typename F, typename... Args>
void emu_launch(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t, Args... args) {
  auto call = [&]() { kernel(args...); };
  ::emu::run_blocks(::emu::Launch{grid, block, lds},
                    [](void* c) { (*static_cast<decltype(call)*>(c))(); }, &call);
}
#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...)                           \
  emu_launch([](auto... a) { kernel(a...); }, dim3(grid), dim3(block), (size_t)(lds),      \
             (hipStream_t)(stream), __VA_ARGS__)

// Host emulation runtime (see hip/hip_runtime.h): work-group threads, the
// checked barrier, the wavefront exchange of the matrix instruction, memory.
#include "hip/hip_runtime.h"

#include <linux/futex.h>
#include <sys/syscall.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#if defined(__SANITIZE_THREAD__)
#define EMU_TSAN 1
#elif defined(__has_feature)
#if __has_feature(thread_sanitizer)
#define EMU_TSAN 1
#endif
#endif
#ifdef EMU_TSAN
#include <sanitizer/tsan_interface.h>
#define EMU_RELEASE(a) __tsan_release(a)
#define EMU_ACQUIRE(a) __tsan_acquire(a)
#endif
#ifndef EMU_RELEASE
#define EMU_RELEASE(a) ((void)(a))
#define EMU_ACQUIRE(a) ((void)(a))
#endif

namespace emu {

thread_local Idx t_thread, t_block;
Idx g_block_dim, g_grid_dim;

namespace {

int g_timeout_s = [] {
  const char* e = getenv("EMU_BARRIER_TIMEOUT_S");
  return e ? atoi(e) : 120;
}();

[[noreturn]] void die(const char* fmt, const char* a, int b, int c, int d) {
  fprintf(stderr, fmt, a, b, c, d);
  fflush(stderr);
  abort();
}

// A barrier for n threads that checks that every thread waits at the same call
// site, and reports a barrier that not every thread reaches.
//
// Under ThreadSanitizer the barrier must order exactly what a work-group
// barrier orders and nothing more: everything a thread did before arriving at
// barrier k happens before everything any thread does after leaving barrier k,
// and nothing else.  A mutex would add edges (a thread that already left
// barrier k and arrives at k + 1 would release into the same mutex that a late
// thread acquires when it leaves k), which hides real races.  So the barrier
// itself uses relaxed atomics and raw futex calls, which ThreadSanitizer does
// not treat as synchronisation, plus fences for the real ordering, and states
// the barrier's edges explicitly: release into the sync object of generation
// k's parity on arrival, acquire from it on departure.
struct Barrier {
  std::atomic<int> arrived{0};
  std::atomic<uint32_t> gen{0};
  int n = 0;
  char sync[2] = {0, 0};
  std::atomic<const char*> site_file[1024];
  std::atomic<int> site_line[1024];

  void reset(int count) {
    n = count;
    arrived.store(0, std::memory_order_relaxed);
  }
  void wait(int tid, const char* f, int l) {
    const uint32_t g = gen.load(std::memory_order_relaxed);
    site_file[tid].store(f, std::memory_order_relaxed);
    site_line[tid].store(l, std::memory_order_relaxed);
    EMU_RELEASE(&sync[g & 1]);
    std::atomic_thread_fence(std::memory_order_seq_cst);
    const int a = arrived.fetch_add(1, std::memory_order_relaxed);
    if (a == n - 1) {
      std::atomic_thread_fence(std::memory_order_seq_cst);
      const char* f0 = site_file[0].load(std::memory_order_relaxed);
      const int l0 = site_line[0].load(std::memory_order_relaxed);
      for (int t = 1; t < n; ++t) {
        const char* ft = site_file[t].load(std::memory_order_relaxed);
        const int lt = site_line[t].load(std::memory_order_relaxed);
        if (lt != l0 || strcmp(ft, f0) != 0)
          die("[emu] barrier divergence: thread 0 waits at %s:%d, thread %d at line %d\n", f0,
              l0, t, lt);
      }
      arrived.store(0, std::memory_order_relaxed);
      std::atomic_thread_fence(std::memory_order_seq_cst);
      gen.store(g + 1, std::memory_order_relaxed);
      syscall(SYS_futex, reinterpret_cast<uint32_t*>(&gen), FUTEX_WAKE_PRIVATE, INT32_MAX,
              nullptr, nullptr, 0);
    } else {
      const auto t0 = std::chrono::steady_clock::now();
      while (gen.load(std::memory_order_relaxed) == g) {
        struct timespec ts = {1, 0};
        syscall(SYS_futex, reinterpret_cast<uint32_t*>(&gen), FUTEX_WAIT_PRIVATE, g, &ts,
                nullptr, 0);
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(g_timeout_s))
          die("[emu] barrier at %s:%d never completed: %d of %d threads arrived\n", f, l,
              arrived.load(std::memory_order_relaxed), n);
      }
      std::atomic_thread_fence(std::memory_order_seq_cst);
    }
    EMU_ACQUIRE(&sync[g & 1]);
  }
};

Barrier g_block_barrier;
Barrier g_wave_barrier[16];

// per-wave operand exchange of the matrix instruction
struct WaveX {
  float a[64], b[64];
};
WaveX g_wavex[16];

char* g_lds = nullptr;
size_t g_lds_bytes = 0;

}  // namespace

void syncthreads(const char* file, int line) {
  g_block_barrier.wait((int)t_thread.x, file, line);
}

// v_mfma_f32_16x16x4f32: A is 16 x 4 (lane l holds A[l % 16][l / 16]), B is
// 4 x 16 (lane l holds B[l / 16][l % 16]), D = A B + C is 16 x 16 (lane l holds
// D[4 (l / 16) + i][l % 16], i = 0..3).  All 64 lanes of the wave take part.
void mfma_f32_16x16x4(float a, float b, const float* c, float* d) {
  const int tid = (int)t_thread.x;
  const int wave = tid / 64, lane = tid % 64;
  WaveX& x = g_wavex[wave];
  Barrier& wb = g_wave_barrier[wave];
  x.a[lane] = a;
  x.b[lane] = b;
  wb.wait(lane, "mfma operands", 0);
  const int col = lane % 16, r0 = 4 * (lane / 16);
  for (int i = 0; i < 4; ++i) {
    const int row = r0 + i;
    float acc = c[i];
    for (int k = 0; k < 4; ++k) acc = std::fma(x.a[k * 16 + row], x.b[k * 16 + col], acc);
    d[i] = acc;
  }
  wb.wait(lane, "mfma results", 0);
}

long long wall_clock() {
  return (long long)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count() / 10;
}

char* dyn_lds() { return g_lds; }

void run_blocks(const Launch& l, void (*body)(void*), void* ctx) {
  const int nt = (int)l.block.x;
  if (nt < 1 || nt > 1024 || l.block.y != 1 || l.block.z != 1 || l.grid.y != 1 || l.grid.z != 1)
    die("[emu] unsupported launch shape %s%d x %d (grid %d)\n", "", nt, (int)l.block.y,
        (int)l.grid.x);
  g_block_dim = Idx{l.block.x, 1, 1};
  g_grid_dim = Idx{l.grid.x, 1, 1};
  // Work-groups run one at a time, the last first: in the persistent kernels the
  // first work-group to run takes every signal from the queue, and the last
  // work-group's workspace slot ends where the allocation (and ASan's red zone)
  // begins, so that an access past the end of a slot is reported.
  for (int b = (int)l.grid.x - 1; b >= 0; --b) {
    // exactly the launch's dynamic LDS, fresh per work-group, filled with a
    // pattern (not zero: the hardware does not clear LDS either)
    g_lds_bytes = l.lds;
    g_lds = l.lds ? static_cast<char*>(malloc(l.lds)) : nullptr;
    if (g_lds) memset(g_lds, 0xA5, l.lds);
    g_block_barrier.reset(nt);
    const int nw = (nt + 63) / 64;
    for (int w = 0; w < nw; ++w) g_wave_barrier[w].reset(std::min(64, nt - 64 * w));
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t)
      th.emplace_back([=] {
        t_thread = Idx{(unsigned)t, 0, 0};
        t_block = Idx{(unsigned)b, 0, 0};
        body(ctx);
      });
    for (auto& x : th) x.join();
    free(g_lds);
    g_lds = nullptr;
  }
}

}  // namespace emu

// ------------------------------------------------------------- runtime API --
namespace {
thread_local hipError_t g_last = hipSuccess;
}

hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  memset(p, 0, sizeof(*p));
  p->multiProcessorCount = 2;
  p->sharedMemPerBlock = 160 * 1024;
  strcpy(p->name, "host emulation");
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
  // exactly n bytes (256-byte aligned), so that ASan's red zone starts at byte n
  if (posix_memalign(p, 256, n ? n : 1) != 0) return hipErrorOutOfMemory;
  memset(*p, 0x5A, n);  // device memory is not cleared by allocation either
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (n) memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, n, k);
}
hipError_t hipMemset(void* p, int v, size_t n) {
  if (n) memset(p, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) { return hipMemset(p, v, n); }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() {
  const hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int v) {
  return v <= 160 * 1024 ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new long long(0);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete static_cast<long long*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  *static_cast<long long*>(e) = emu::wall_clock();
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)(*static_cast<long long*>(b) - *static_cast<long long*>(a)) * 1e-5f;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}

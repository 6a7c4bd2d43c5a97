// Test-only CPU build of the library's HIP kernels.
//
// This header stands in for <hip/hip_runtime.h> when tests/cpu_emu/build_emu.py
// compiles the kernel sources for the host: every GPU thread of a block runs as
// a cooperative fiber, __syncthreads is a block barrier, wavefront shuffles and
// the matrix-core builtins exchange operands through a per-wavefront buffer with
// the lane layouts measured on gfx950, and device memory is host memory.  Built
// with AddressSanitizer it finds out-of-bounds accesses in the kernels exactly.
// It is never part of the product: the product library is only ever built by
// hipcc for gfx950.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

// ------------------------------------------------------------------ attributes
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static thread_local
#define __align__(n) __attribute__((aligned(n)))
// a device variable's address on the host: the variable itself in this build
#define HIP_SYMBOL(x) (&(x))
#define __HIPCC__ 1

// ------------------------------------------------------------------ runtime types
typedef enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotSupported = 801,
  hipErrorInvalidDevice = 101,
  hipErrorIllegalAddress = 700,
} hipError_t;
typedef void* hipStream_t;
typedef struct lrdm_emu_event* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost,
                     hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint3 {
  unsigned x, y, z;
};

struct double2 { double x, y; };
struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
struct int2 { int x, y; };
inline double2 make_double2(double x, double y) { return double2{x, y}; }
inline int2 make_int2(int x, int y) { return int2{x, y}; }
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }

extern thread_local uint3 threadIdx;
extern thread_local uint3 blockIdx;
extern thread_local dim3 blockDim;
extern thread_local dim3 gridDim;

namespace lrdm_emu {

// Cooperative fibers: every GPU thread of a block is a user-level context on one
// host thread; barriers switch back to the block scheduler.  Blocks of a grid
// run in parallel on a few host threads.
struct Fiber {
  void* sp = nullptr;
  char* stack = nullptr;
  int tid = 0;
  uint3 idx{0, 0, 0};
  int wait = 0;  // 0 running, 1 block barrier, 2 wavefront barrier
  bool done = false;
};

struct Block {
  std::vector<Fiber> fibers;
  int nthreads = 0;
  void* sched_sp = nullptr;
  const void* sched_stack_bottom = nullptr;
  size_t sched_stack_size = 0;
  std::vector<std::vector<double>> xch;  // per wave exchange buffer
  std::vector<unsigned char> dyn;
  std::function<void()> body;
};

extern thread_local Block* cur;
extern thread_local Fiber* cur_fiber;
extern thread_local int tid_linear;

void run_block(Block& b, dim3 block, uint3 bidx, size_t smem);
void yield_wait(int kind);

inline int lane() { return tid_linear & 63; }
inline int wave() { return tid_linear >> 6; }
inline void wave_sync() { yield_wait(2); }
inline double* wave_buf() { return cur->xch[wave()].data(); }
inline unsigned char* dyn_smem() { return cur->dyn.data(); }

void parallel_blocks(dim3 grid, const std::function<void(uint3)>& fn);
Block& worker_block();

template <typename K, typename... Args>
void launch(K kernel, dim3 grid, dim3 block, size_t smem, hipStream_t, Args... args) {
  parallel_blocks(grid, [&](uint3 bidx) {
    Block& b = worker_block();
    b.body = [&]() { kernel(args...); };
    blockDim = block;
    gridDim = grid;
    blockIdx = bidx;
    run_block(b, block, bidx, smem);
  });
}

// ------------------------------------------------------------------ wavefront ops
template <typename T>
T shfl(T v, int src_lane) {
  double* buf = wave_buf();
  std::memcpy(&buf[lane()], &v, sizeof(T));
  wave_sync();
  T out;
  std::memcpy(&out, &buf[src_lane], sizeof(T));
  wave_sync();
  return out;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// v_mfma_f64_16x16x4f64: A lane l -> A[l%16][l/16]; B lane l -> B[l/16][l%16];
// D lane l, register v -> D[4v + l/16][l%16].
inline d4 mfma_f64_16x16x4(double a, double b, d4 c, int, int, int) {
  double* buf = wave_buf();
  buf[lane()] = a;
  buf[64 + lane()] = b;
  wave_sync();
  d4 out = c;
  const int l = lane();
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * v + l / 16, j = l % 16;
    double s = 0.0;
    for (int k = 0; k < 4; ++k) s += buf[i + 16 * k] * buf[64 + j + 16 * k];
    out[v] += s;
  }
  wave_sync();
  return out;
}

// v_mfma_f32_16x16x4f32: same operand layout; D lane l, v -> D[4(l/16) + v][l%16].
inline f4 mfma_f32_16x16x4(float a, float b, f4 c, int, int, int) {
  double* buf = wave_buf();
  buf[lane()] = a;
  buf[64 + lane()] = b;
  wave_sync();
  f4 out = c;
  const int l = lane();
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * (l / 16) + v, j = l % 16;
    float s = 0.f;
    for (int k = 0; k < 4; ++k) s += (float)buf[i + 16 * k] * (float)buf[64 + j + 16 * k];
    out[v] += s;
  }
  wave_sync();
  return out;
}

// v_mfma_f32_16x16x32_bf16: A lane l -> A[l%16][8(l/16) + e]; B lane l ->
// B[8(l/16) + e][l%16]; D as the f32 16x16 shape.
inline f4 mfma_f32_16x16x32_bf16(bf8 a, bf8 b, f4 c, int, int, int) {
  double* buf = wave_buf();
  for (int e = 0; e < 8; ++e) {
    buf[8 * lane() + e] = (double)(float)a[e];
    buf[512 + 8 * lane() + e] = (double)(float)b[e];
  }
  wave_sync();
  f4 out = c;
  const int l = lane();
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * (l / 16) + v, j = l % 16;
    float s = 0.f;
    for (int k = 0; k < 32; ++k) {
      const int la = i + 16 * (k / 8), lb = j + 16 * (k / 8);
      s += (float)buf[8 * la + k % 8] * (float)buf[512 + 8 * lb + k % 8];
    }
    out[v] += s;
  }
  wave_sync();
  return out;
}

// global_load_lds_dwordx4: lane l copies `size` bytes from its own address to
// base + size * l (base is the same for the whole wavefront).
inline void global_load_lds(const void* src, void* base, unsigned size) {
  std::memcpy(static_cast<unsigned char*>(base) + (size_t)size * lane(), src, size);
}

}  // namespace lrdm_emu

#define __builtin_amdgcn_global_load_lds(src, dst, size, off, aux) \
  lrdm_emu::global_load_lds((const void*)(src), (void*)(dst), (size))
#define __builtin_amdgcn_mfma_f64_16x16x4f64 lrdm_emu::mfma_f64_16x16x4
#define __builtin_amdgcn_mfma_f32_16x16x4f32 lrdm_emu::mfma_f32_16x16x4
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16 lrdm_emu::mfma_f32_16x16x32_bf16
// instruction-scheduling hints: nothing to do on the CPU
#define __builtin_amdgcn_sched_group_barrier(mask, count, id) ((void)0)
#define __builtin_amdgcn_sched_barrier(mask) ((void)0)

inline void __syncthreads() { lrdm_emu::yield_wait(1); }
template <typename T>
inline T __shfl_down(T v, unsigned off, int = 64) {
  const int src = lrdm_emu::lane() + (int)off;
  return lrdm_emu::shfl(v, src < 64 ? src : lrdm_emu::lane());
}
template <typename T>
inline T __shfl_xor(T v, int m, int = 64) {
  return lrdm_emu::shfl(v, lrdm_emu::lane() ^ m);
}
inline int atomicOr(int* p, int v) {
  return std::atomic_ref<int>(*p).fetch_or(v);
}
inline unsigned __float_as_uint(float x) { return __builtin_bit_cast(unsigned, x); }
// v_rcp_f32 stand-in (the hardware result is within 1 ulp of this)
inline float lrdm_emu_rcpf(float x) { return 1.0f / x; }
#define __builtin_amdgcn_rcpf lrdm_emu_rcpf
// v_rsq_f32 stand-in (the hardware result is within 1 ulp of this)
inline float lrdm_emu_rsqf(float x) { return 1.0f / std::sqrt(x); }
#define __builtin_amdgcn_rsqf lrdm_emu_rsqf
inline float __uint_as_float(unsigned x) { return __builtin_bit_cast(float, x); }

// ------------------------------------------------------------------ device math
using std::exp;
using std::expm1;
using std::fabs;
using std::fmax;
using std::fmin;
using std::isfinite;
using std::nextafter;
using std::sqrt;
inline void sincospi(double x, double* s, double* c) {
  *s = std::sin(M_PI * x);
  *c = std::cos(M_PI * x);
}
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline int64_t min(int64_t a, int64_t b) { return a < b ? a : b; }
inline int64_t max(int64_t a, int64_t b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }

// ------------------------------------------------------------------ host API
struct lrdm_emu_event {
  std::chrono::steady_clock::time_point t;
};
inline const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipMalloc(void** p, size_t n) {
  *p = std::malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
template <typename T>
inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc(reinterpret_cast<void**>(p), n); }
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { std::memmove(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memmove(d, s, n); return hipSuccess; }
inline hipError_t hipMemset(void* d, int v, size_t n) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
typedef enum { hipStreamCaptureStatusNone = 0, hipStreamCaptureStatusActive = 1 } hipStreamCaptureStatus;
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  static int dummy[64];
  static int next = 0;
  *s = &dummy[next++ % 64];
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus* c) {
  *c = hipStreamCaptureStatusNone;
  return hipSuccess;
}
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
inline hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = new lrdm_emu_event(); return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->t = std::chrono::steady_clock::now(); return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
  return hipSuccess;
}

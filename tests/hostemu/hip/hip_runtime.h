// Host emulation of the HIP device environment used by the RTU kernels: each
// workgroup runs as blockDim std::threads with real barriers; wave-level
// operations (DPP moves, readlane, ballot, shfl_up, MFMA 16x16x4 f32) exchange
// values through a per-wave buffer and a 64-thread barrier.  Built with ASan
// on the host only, to check every memory access of the kernels.
#pragma once
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

#include <algorithm>
#include <atomic>
#include <barrier>
#include <cmath>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>
#include <sanitizer/asan_interface.h>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __constant__
#define __restrict__
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) ((const void*)&(x))

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
struct double2 { double x, y; };
struct int2 { int x, y; };
struct int4 { int x, y, z, w; };
struct uint2 { unsigned x, y; };
struct uint4 { unsigned x, y, z, w; };
struct uchar4 { unsigned char x, y, z, w; };
inline float2 make_float2(float a, float b) { return {a, b}; }
inline float4 make_float4(float a, float b, float c, float d) { return {a, b, c, d}; }
inline int4 make_int4(int a, int b, int c, int d) { return {a, b, c, d}; }
inline uint2 make_uint2(unsigned a, unsigned b) { return {a, b}; }
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return {a, b, c, d}; }

inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline long max(long a, long b) { return a > b ? a : b; }
inline unsigned long long min(unsigned long long a, unsigned long long b) { return a < b ? a : b; }
inline unsigned long long max(unsigned long long a, unsigned long long b) { return a > b ? a : b; }
using std::isfinite;
using std::isinf;
using std::isnan;
using std::signbit;

// ---- per-thread launch state
struct EmuWave {
  std::barrier<>* bar;
  alignas(16) unsigned char buf[64][16];
};
struct EmuBlock {
  std::barrier<>* bar;
  EmuWave* waves;
  unsigned char* dyn;
};
extern thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
extern thread_local EmuBlock* emu_blk;
inline unsigned char* emu_dyn_lds() { return emu_blk->dyn; }
inline void __syncthreads() { emu_blk->bar->arrive_and_wait(); }
inline int emu_lane() { return (int)(threadIdx.x & 63); }
inline EmuWave& emu_wave() { return emu_blk->waves[threadIdx.x >> 6]; }

// publish this lane's value, read lane `src`'s, then wait until every lane has read
template <class T>
inline void emu_wave_publish(const T& v) {
  static_assert(sizeof(T) <= 16, "");
  EmuWave& w = emu_wave();
  memcpy(w.buf[emu_lane()], &v, sizeof(T));
  w.bar->arrive_and_wait();
}
template <class T>
inline T emu_wave_get(int lane) {
  T v;
  memcpy(&v, emu_wave().buf[lane], sizeof(T));
  return v;
}
inline void emu_wave_done() { emu_wave().bar->arrive_and_wait(); }

inline int __builtin_amdgcn_update_dpp_emu(int old, int src, int ctrl) {
  (void)old;
  emu_wave_publish(src);
  const int l = emu_lane();
  int s;
  if (ctrl < 0x100) s = (l & ~3) | ((ctrl >> (2 * (l & 3))) & 3);
  else if (ctrl == 0x140) s = (l & ~15) | (15 - (l & 15));
  else if (ctrl == 0x141) s = (l & ~7) | (7 - (l & 7));
  else { fprintf(stderr, "emu: dpp ctrl %x\n", ctrl); abort(); }
  const int v = emu_wave_get<int>(s);
  emu_wave_done();
  return v;
}
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) __builtin_amdgcn_update_dpp_emu(old, src, ctrl)
inline int __builtin_amdgcn_readlane(int v, int l) {
  emu_wave_publish(v);
  const int r = emu_wave_get<int>(l);
  emu_wave_done();
  return r;
}
inline unsigned long long __ballot(int p) {
  emu_wave_publish(p);
  unsigned long long m = 0;
  for (int l = 0; l < 64; ++l) m |= (unsigned long long)(emu_wave_get<int>(l) != 0) << l;
  emu_wave_done();
  return m;
}
// the kernels use __any only to take a branch whose per-lane result does not
// depend on other lanes: this lane's predicate gives the same per-lane result
inline int __any(int p) { return p != 0; }
template <class T>
inline T __shfl_up(T v, unsigned o, int width = 64) {
  (void)width;
  emu_wave_publish(v);
  const int l = emu_lane();
  const T r = l >= (int)o ? emu_wave_get<T>(l - (int)o) : v;
  emu_wave_done();
  return r;
}
typedef float emu_f4 __attribute__((ext_vector_type(4)));
inline emu_f4 emu_mfma_16x16x4(float a, float b, emu_f4 c) {
  struct AB { float a, b; };
  emu_wave_publish(AB{a, b});
  const int l = emu_lane(), j = l & 15, i0 = 4 * (l >> 4);
  emu_f4 d = c;
  for (int r = 0; r < 4; ++r)
    for (int k = 0; k < 4; ++k) d[r] += emu_wave_get<AB>(i0 + r + 16 * k).a * emu_wave_get<AB>(j + 16 * k).b;
  emu_wave_done();
  return d;
}
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) emu_mfma_16x16x4(a, b, c)

inline float __builtin_amdgcn_rcpf(float x) { return 1.f / x; }
inline float __builtin_amdgcn_sqrtf(float x) { return sqrtf(x); }
inline float __builtin_amdgcn_rsqf(float x) { return 1.f / sqrtf(x); }
inline float __builtin_amdgcn_logf(float x) { return log2f(x); }
inline float __builtin_amdgcn_exp2f(float x) { return exp2f(x); }
inline float __expf(float x) { return expf(x); }
inline float __logf(float x) { return logf(x); }
inline float __cosf(float x) { return cosf(x); }
inline float __sinf(float x) { return sinf(x); }
inline unsigned __umulhi(unsigned a, unsigned b) { return (unsigned)(((uint64_t)a * b) >> 32); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __popc(unsigned v) { return __builtin_popcount(v); }
inline int __ffs(unsigned v) { return __builtin_ffs((int)v); }
inline int __clz(int v) { return v ? __builtin_clz((unsigned)v) : 32; }
inline float __int_as_float(int v) { float f; memcpy(&f, &v, 4); return f; }
inline float __uint_as_float(unsigned v) { float f; memcpy(&f, &v, 4); return f; }
inline int __float_as_int(float f) { int v; memcpy(&v, &f, 4); return v; }
inline unsigned __float_as_uint(float f) { unsigned v; memcpy(&v, &f, 4); return v; }
inline double __hiloint2double(int hi, int lo) {
  const uint64_t u = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
  double d; memcpy(&d, &u, 8); return d;
}
inline int __double2hiint(double d) { uint64_t u; memcpy(&u, &d, 8); return (int)(u >> 32); }
inline int __double2loint(double d) { uint64_t u; memcpy(&u, &d, 8); return (int)(uint32_t)u; }

extern std::mutex emu_atomic_mu;
template <class T>
inline T atomicAdd(T* p, T v) { std::lock_guard<std::mutex> g(emu_atomic_mu); T o = *p; *p = o + v; return o; }
template <class T>
inline T atomicMin(T* p, T v) { std::lock_guard<std::mutex> g(emu_atomic_mu); T o = *p; *p = o < v ? o : v; return o; }
template <class T>
inline T atomicMax(T* p, T v) { std::lock_guard<std::mutex> g(emu_atomic_mu); T o = *p; *p = o > v ? o : v; return o; }
template <class T>
inline T atomicOr(T* p, T v) { std::lock_guard<std::mutex> g(emu_atomic_mu); T o = *p; *p = o | v; return o; }

// ---- runtime
typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum { hipSuccess = 0, hipErrorUnknown = 999 };
enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum { hipHostMallocDefault = 0, hipEventDisableTiming = 2, hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
hipError_t hipMalloc(void** p, size_t n);
template <class T> hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipHostMalloc(void** p, size_t n, int);
template <class T> hipError_t hipHostMalloc(T** p, size_t n, int f) { return hipHostMalloc((void**)p, n, f); }
hipError_t hipFree(void* p);
hipError_t hipHostFree(void* p);
void emu_copy(void* d, const void* s, size_t n);
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, int) { emu_copy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, int, hipStream_t) { emu_copy(d, s, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { memset(d, v, n); return hipSuccess; }
inline hipError_t hipMemcpyToSymbol(const void* sym, const void* s, size_t n) { memcpy(const_cast<void*>(sym), s, n); return hipSuccess; }
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, int, int) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = nullptr; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, int) { *e = nullptr; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }

// run every workgroup of a launch, one after another
void emu_run_grid(dim3 g, dim3 b, size_t lds, const char* name, const std::function<void()>& body);
template <class F, class... A>
inline void emu_launch(const char* name, F f, dim3 g, dim3 b, size_t lds, hipStream_t, A... args) {
  emu_run_grid(g, b, lds, name, [=]() { f(args...); });
}
#define hipLaunchKernelGGL(k, g, b, l, s, ...) emu_launch(#k, k, g, b, l, s, __VA_ARGS__)

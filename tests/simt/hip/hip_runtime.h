// CPU execution of the library's HIP kernel source, for tests only.
//
// Stands in for <hip/hip_runtime.h> when the kernel file is compiled with g++:
// every lane of a wave is one host thread; the cross-lane builtins (ballot,
// readlane, readfirstlane, shuffles) and the points where a wave reconverges
// are barrier exchanges among the 64 lane threads, so a wave executes in
// lockstep exactly where the kernel relies on it. A cross-lane builtin reached
// by only part of a wave deadlocks here, which exposes divergent use.
#pragma once

#include <atomic>
#include <barrier>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <execinfo.h>

#define __device__
#define __global__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum { hipSuccess = 0 };

namespace simt {
struct Wave {
  std::barrier<> bar{64};
  uint64_t slot[64];
  uint64_t seq[64];  // per-lane count of wave operations, must agree
  const char* site[64];
  uint64_t stack_hash[64];
  void* stack[64][12];
  int depth[64];
};
struct Group {
  std::barrier<>* bar;
  uint8_t* lds;
};
extern thread_local unsigned lane;
extern thread_local Wave* wave;
extern thread_local Group* group;
extern thread_local dim3 tidx, bidx, bdim, gdim;
extern thread_local uint64_t nops;

// Every lane of a wave must reach the same wave operation; a mismatch means
// the kernel let lanes diverge around a cross-lane builtin.
extern bool check_stacks;
inline void record_site() {
  if (!check_stacks) return;
  int d = backtrace(wave->stack[lane], 12);
  wave->depth[lane] = d;
  uint64_t h = 1469598103934665603ull;
  for (int i = 2; i < d; ++i) h = (h ^ (uint64_t)wave->stack[lane][i]) * 1099511628211ull;
  wave->stack_hash[lane] = h;
}
inline void check_lockstep(const char* what) {
  if (lane == 0) {
    for (int i = 1; i < 64 && check_stacks; ++i)
      if (wave->stack_hash[i] != wave->stack_hash[0]) {
        fprintf(stderr, "simt: lanes 0 and %d reached a wave op from different call stacks\n", i);
        fprintf(stderr, "lane 0:\n");
        backtrace_symbols_fd(wave->stack[0], wave->depth[0], 2);
        fprintf(stderr, "lane %d:\n", i);
        backtrace_symbols_fd(wave->stack[i], wave->depth[i], 2);
        abort();
      }
    for (int i = 1; i < 64; ++i)
      if (wave->seq[i] != wave->seq[0]) {
        fprintf(stderr, "simt: lanes diverged at wave op #%llu (%s): lane %d is at #%llu (%s)\n",
                (unsigned long long)wave->seq[0], wave->site[0], i, (unsigned long long)wave->seq[i],
                wave->site[i]);
        abort();
      }
  }
}
inline void wave_sync_at(const char* what) {
  record_site();
  wave->seq[lane] = ++nops;
  wave->site[lane] = what;
  wave->bar.arrive_and_wait();
  check_lockstep(what);
  wave->bar.arrive_and_wait();
}
inline void wave_sync() { wave_sync_at("sync"); }
// Publish one value per lane, then every lane may read all 64.
inline const uint64_t* exchange_at(uint64_t v, const char* what) {
  record_site();
  wave->slot[lane] = v;
  wave->seq[lane] = ++nops;
  wave->site[lane] = what;
  wave->bar.arrive_and_wait();
  check_lockstep(what);
  return wave->slot;
}
#define exchange(v) exchange_at((v), __func__)
inline void done_reading() { wave->bar.arrive_and_wait(); }
}  // namespace simt

#define threadIdx (simt::tidx)
#define blockIdx (simt::bidx)
#define blockDim (simt::bdim)
#define gridDim (simt::gdim)

inline unsigned __lane_id() { return simt::lane; }

inline unsigned long long __ballot(int p) {
  const uint64_t* s = simt::exchange(p ? 1 : 0);
  unsigned long long m = 0;
  for (int i = 0; i < 64; ++i) m |= (unsigned long long)(s[i] & 1) << i;
  simt::done_reading();
  return m;
}
inline uint32_t __builtin_amdgcn_readlane(uint32_t x, uint32_t l) {
  const uint64_t* s = simt::exchange(x);
  uint32_t r = (uint32_t)s[l & 63];
  simt::done_reading();
  return r;
}
inline uint32_t __builtin_amdgcn_readfirstlane(uint32_t x) { return __builtin_amdgcn_readlane(x, 0); }
template <class T>
inline T simt_shfl_src(T x, int src) {
  const uint64_t* s = simt::exchange((uint64_t)(uint32_t)x);
  T r = (T)(uint32_t)s[src & 63];
  simt::done_reading();
  return r;
}
inline int __shfl(int x, int src) { return simt_shfl_src(x, src); }
inline unsigned __shfl(unsigned x, int src) { return simt_shfl_src(x, src); }
inline int __shfl_xor(int x, int m) { return simt_shfl_src(x, (int)(simt::lane ^ (unsigned)m)); }
inline unsigned __shfl_xor(unsigned x, int m) { return simt_shfl_src(x, (int)(simt::lane ^ (unsigned)m)); }
inline unsigned __shfl_up(unsigned x, unsigned d) {
  unsigned v = simt_shfl_src(x, (int)(simt::lane >= d ? simt::lane - d : simt::lane));
  return v;
}
inline int __shfl_up(int x, unsigned d) { return (int)__shfl_up((unsigned)x, d); }
inline uint32_t __builtin_amdgcn_mbcnt_lo(uint32_t m, uint32_t acc) {
  uint32_t mask = simt::lane >= 32 ? 0xFFFFFFFFu : ((1u << simt::lane) - 1u);
  return acc + (uint32_t)__builtin_popcount(m & mask);
}
inline uint32_t __builtin_amdgcn_mbcnt_hi(uint32_t m, uint32_t acc) {
  uint32_t mask = simt::lane < 32 ? 0u : (simt::lane == 63 ? 0x7FFFFFFFu : ((1u << (simt::lane - 32)) - 1u));
  return acc + (uint32_t)__builtin_popcount(m & mask);
}
inline int __popcll(unsigned long long m) { return __builtin_popcountll(m); }
inline int __ffsll(long long m) { return __builtin_ffsll(m); }
inline int __clzll(long long m) { return m ? __builtin_clzll((unsigned long long)m) : 64; }
inline int __clz(int x) { return x ? __builtin_clz((unsigned)x) : 32; }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline void __syncthreads() { simt::group->bar->arrive_and_wait(); }
inline void __builtin_amdgcn_wave_barrier() { simt::wave_sync(); }
#define __builtin_amdgcn_s_sleep(n) std::this_thread::sleep_for(std::chrono::microseconds(4 * (n)))
// The GPU reads its clock with a scalar instruction, one value per wave; so
// does this: lane 0 reads, every lane gets its value.
inline long long wall_clock64() {
  using namespace std::chrono;
  const long long t = (long long)(duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() / 10);
  const uint64_t* s = simt::exchange((uint64_t)t);
  const long long r = (long long)s[0];
  simt::done_reading();
  return r;
}
template <class T>
inline T min(T a, T b) { return a < b ? a : b; }

// Index check used by the CPU build: reports the kernel line and aborts.
template <class T, class U>
inline T simt_chk(T i, U bound, const char* what, int line) {
  if ((uint64_t)i >= (uint64_t)bound) {
    fprintf(stderr, "simt: %s index %llu out of range %llu at kernel line %d (lane %u)\n", what,
            (unsigned long long)i, (unsigned long long)bound, line, simt::lane);
    abort();
  }
  return i;
}

#define __ATOMIC_RELAXED_ __ATOMIC_SEQ_CST
#define __HIP_MEMORY_SCOPE_WAVEFRONT 1
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_SYSTEM 4
template <class T>
inline T __hip_atomic_load(const T* p, int, int) { return __atomic_load_n(p, __ATOMIC_SEQ_CST); }
template <class T, class U>
inline void __hip_atomic_store(T* p, U v, int, int) { __atomic_store_n(p, (T)v, __ATOMIC_SEQ_CST); }
template <class T, class U>
inline T __hip_atomic_fetch_add(T* p, U v, int, int) { return __atomic_fetch_add(p, (T)v, __ATOMIC_SEQ_CST); }
template <class T, class U>
inline T __hip_atomic_fetch_or(T* p, U v, int, int) { return __atomic_fetch_or(p, (T)v, __ATOMIC_SEQ_CST); }
inline void __builtin_amdgcn_fence(int, const char*) { __atomic_thread_fence(__ATOMIC_SEQ_CST); }
template <class T, class U>
inline T __hip_atomic_fetch_min(T* p, U v, int, int) {
  T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (old > (T)v && !__atomic_compare_exchange_n(p, &old, (T)v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return old;
}
template <class T, class U>
inline bool __hip_atomic_compare_exchange_strong(T* p, T* expect, U v, int, int, int) {
  return __atomic_compare_exchange_n(p, expect, (T)v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
}
inline int atomicCAS(int* p, int cmp, int v) {
  __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return cmp;
}
inline int atomicExch(int* p, int v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }

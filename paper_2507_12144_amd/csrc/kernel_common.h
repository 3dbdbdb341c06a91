// Small device helpers shared by the contraction kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace sht {

// Work item of this workgroup.  The hardware deals workgroups to the 8 XCDs
// round-robin (workgroup b runs on XCD b % 8); work lists hold 8 slices of
// `per` items, one per XCD, so slice x is processed in order on XCD x.
__device__ __forceinline__ int2 take_work(const int2* __restrict__ work, int per) {
  const int slot = (blockIdx.x % 8) * per + blockIdx.x / 8;
  return work[slot];
}

}  // namespace sht

namespace sht {

// Global-memory (address space 1) views of generic pointers: accesses
// through them compile to global_* instead of flat_* instructions.  A flat
// store may address LDS, so while global->LDS copies are in flight the
// compiler makes it wait for all of them; a global store needs no such wait.
typedef __attribute__((address_space(1))) float gfloat;
typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) v2f_t gfloat2;
__device__ __forceinline__ gfloat* as_global(float* p) { return (gfloat*)p; }

// s_waitcnt immediate that waits until at most n vector-memory operations of
// this wave are outstanding (expcnt and lgkmcnt left at their maxima).
constexpr int vm_wait(int n) { return 0x0F70 | (n & 15) | (((n >> 4) & 3) << 14); }

// Wait for vector memory (at most n copies of this wave in flight) and for
// every LDS read of this wave, so that after the barrier that follows no
// wave still reads a buffer the next copies overwrite.
constexpr int vm_lds_wait(int n) { return vm_wait(n) & ~0x0F00; }

// Race-check build (SHT_DEBUG_BARRIERS defined, libsht_debug.so): every
// barrier below first drains all of the wave's memory counters, and every
// stage of the Legendre kernels ends with a drain and a workgroup barrier,
// so no copy, load or store of one stage overlaps another stage's work.  Its
// results must equal the release build's bit for bit; a difference points
// at a missing wait or barrier.
#ifdef SHT_DEBUG_BARRIERS
constexpr bool kDebugBarriers = true;
#else
constexpr bool kDebugBarriers = false;
#endif

__device__ __forceinline__ void debug_drain() {
  if constexpr (kDebugBarriers) {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0);  // vmcnt, expcnt and lgkmcnt all zero
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  }
}

// End of one stage of a Legendre kernel: nothing in the release build.
__device__ __forceinline__ void debug_stage_end() { debug_drain(); }

// Workgroup barrier for LDS filled by asynchronous global->LDS copies.  The
// caller first waits (vm_wait) for its own copies of the stage; the barrier
// then makes every wave's copies visible.  The empty asm statements keep the
// compiler from moving memory operations across the barrier; unlike
// __syncthreads() no fence is emitted, so copies of later stages stay in
// flight.
__device__ __forceinline__ void stage_barrier() {
  debug_drain();
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

}  // namespace sht

namespace sht {

// Workgroup barrier for data exchanged through LDS only: the wave waits for
// its own LDS operations (lgkmcnt(0)), then s_barrier.  Unlike
// __syncthreads(), whose release fence also waits for every outstanding
// global load and store (vmcnt(0)), it leaves prefetches in flight.
__device__ __forceinline__ void lds_barrier() {
  debug_drain();
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt unconstrained
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

}  // namespace sht

namespace sht {

// Calls f(integral_constant<U>) for U = 0, 1, ..., END-1 as straight-line
// code, stopping after the first call that returns false.
template <int U, int END, class F>
__device__ __forceinline__ bool unrolled(F&& f) {
  if constexpr (U < END) {
    if (!f(std::integral_constant<int, U>{})) return false;
    return unrolled<U + 1, END>(f);
  }
  return true;
}

// LDS buffer of stage u of a ring of three.
template <int U, class T>
__device__ __forceinline__ T* ring_buf(T* b0, T* b1, T* b2) {
  if constexpr (U % 3 == 0) return b0;
  else if constexpr (U % 3 == 1) return b1;
  else return b2;
}

}  // namespace sht

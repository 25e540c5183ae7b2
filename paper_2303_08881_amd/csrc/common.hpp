// common.hpp -- device helpers shared by the gfx950 kernels of libschurilu.
//
// Conventions
//  * one wavefront = 64 lanes; kernels that need a single wave use 64-thread
//    workgroups so __syncthreads() is a cheap wave-local fence for LDS;
//  * every dependency wait is bounded: after SPIN_LIMIT polls it records
//    ILU_ERR_TIMEOUT in the status word and gives up, so no launch can hang;
//  * cross-workgroup handoffs use agent-scope release stores and relaxed
//    polls, followed either by one agent-scope acquire fence or by
//    device-scope loads of exactly the data handed over;
//  * floating-point contraction is off for the whole library (-ffp-contract=off)
//    and every fused multiply-add is an explicit fma(), so the rounding order of
//    each row operation is fixed and matches the sequential definition.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "schurilu.h"

#define WAVE 64

namespace silu {

constexpr long SPIN_LIMIT = 1L << 24;

// status word layout (device, int32[8]):
//  [0] first error code (0 = none)   [1] error row (int32, -1)
//  [2] abort flag seen by spinners     [3..7] reserved / counters
struct Status {
  int32_t code;
  int32_t row;
  int32_t abort;
  int32_t pad[5];
};

__device__ inline void raise_error(Status *st, int32_t code, int64_t row) {
  if (atomicCAS(&st->code, 0, code) == 0) st->row = (int32_t)row;
  __hip_atomic_store(&st->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int ld_relaxed(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long ld_relaxed_u64(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_release(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// Device-scope (write-through) store: leaves no dirty line in this XCD's L2,
// which keeps the L2 write-back of the next device-scope release short.
template <typename T>
__device__ inline void st_dev(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Device-scope load: reads the coherent copy (what st_dev and the stores
// before a device-scope release wrote) without the cache invalidation of an
// acquire fence.  A wave that has seen another wave's release flag reads
// that wave's data this way.
template <typename T>
__device__ inline T ld_dev(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ inline void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// Wait (one lane) until *flag == want.  Returns false on timeout / abort.
__device__ inline bool wait_flag_eq(const int *flag, int want, Status *st, int64_t row) {
  long it = 0;
  while (ld_relaxed(flag) != want) {
    if (++it > SPIN_LIMIT) {
      raise_error(st, ILU_ERR_TIMEOUT, row);
      return false;
    }
    if ((it & 255) == 0 && ld_relaxed(&st->abort)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Wait (one lane) until *ctr >= want.
__device__ inline bool wait_ctr_ge(const unsigned long long *ctr, unsigned long long want, Status *st,
                                   int64_t row) {
  long it = 0;
  while (ld_relaxed_u64(ctr) < want) {
    if (++it > SPIN_LIMIT) {
      raise_error(st, ILU_ERR_TIMEOUT, row);
      return false;
    }
    if ((it & 255) == 0 && ld_relaxed(&st->abort)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

__device__ inline int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

// Orders the LDS accesses of one wave around this point (a workgroup
// barrier for a wave that shares its workgroup with others working
// independently): the wave's earlier LDS writes are seen by its later reads.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// value of v on lane l (l wave-uniform): two scalar reads, no LDS
__device__ inline double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Values that steer the control flow of a wave must be wave-uniform in the
// compiler's eyes (scalar registers).  With one wave per workgroup the
// compiler drops __syncthreads(), so a value written to LDS by lane 0 and
// re-read by the other lanes does NOT keep them in one control-flow path: a
// loop whose exit depends on it may be split per lane.  readfirstlane
// (executed with all lanes active) returns lane 0's value as a uniform.
__device__ inline int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline unsigned long long uniform_u64(unsigned long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ inline double uniform_f64(double v) {
  return __longlong_as_double((long long)uniform_u64((unsigned long long)__double_as_longlong(v)));
}

// One ticket per wave from a global counter: lane 0 takes it, all lanes get
// it as a uniform value.
__device__ inline unsigned long long wave_ticket(unsigned long long *ctr) {
  unsigned long long v = 0;
  if (threadIdx.x == 0) v = atomicAdd(ctr, 1ull);
  return uniform_u64(v);
}
__device__ inline unsigned int wave_ticket(unsigned int *ctr) {
  unsigned int v = 0;
  if (threadIdx.x == 0) v = atomicAdd(ctr, 1u);
  return (unsigned int)uniform_i32((int)v);
}

__device__ inline unsigned long long ballot(bool p) { return __ballot(p); }

__device__ inline int popc64(unsigned long long m) { return __popcll(m); }

// exclusive count of set bits below this lane
__device__ inline int mbcnt(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

template <typename T>
__device__ inline T wave_bcast(T v, int src) {
  return __shfl(v, src, WAVE);
}

__device__ inline int wave_sum_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ inline int wave_max_int(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
  return v;
}

}  // namespace silu

// host-side launch check
#define SILU_LAUNCH_CHECK()                                   \
  do {                                                        \
    hipError_t _e = hipGetLastError();                        \
    if (_e != hipSuccess) return silu_hip_fail(_e, __LINE__); \
  } while (0)

// Device-side helpers shared by the LD-Leiden HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldl {

typedef __int128 i128;
typedef unsigned long long u64a;   // type taken by the 64-bit atomics
typedef long long i64a;

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kWave = 64;

// ------------------------------------------------------------------ stamped sets
// A set over ids [0, n) is a stamp array plus an append list: x is in the set iff
// stamp[x] == epoch.  The first inserter of x appends it to the list.
__device__ __forceinline__ bool set_claim(uint32_t* stamp, uint32_t epoch, uint32_t x) {
  if (__hip_atomic_load(&stamp[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) return false;
  return atomicExch(&stamp[x], epoch) != epoch;
}
// Reserve slots in an append list for the active lanes with `pred`: one atomic per wave.
// Call from every active lane of the wave (any subset of lanes may be active).
__device__ __forceinline__ uint32_t wave_reserve(uint32_t* count, bool pred) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return 0;
  const int lane = (int)__lane_id();
  const int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
  return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}
__device__ __forceinline__ unsigned long long wave_reserve64(unsigned long long* count, bool pred,
                                                             unsigned long long per) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return 0;
  const int lane = (int)__lane_id();
  const int leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(m) * per);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)base, leader);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(base >> 32), leader);
  base = ((unsigned long long)hi << 32) | lo;
  return base + per * (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
}
// Insert x (when `valid`) into a stamped set; called from every active lane.
__device__ __forceinline__ void set_add(uint32_t* stamp, uint32_t epoch, uint32_t* list, uint32_t* count,
                                        uint32_t x, bool valid = true) {
  const bool claimed = valid && set_claim(stamp, epoch, x);
  const uint32_t at = wave_reserve(count, claimed);
  if (claimed) list[at] = x;
}
// ------------------------------------------------------------------ record keys
// A (row, col) record key is row << ks | col with ks >= the bits of a vertex id, so keys sort by
// row, then column, over their low 2 ks bits.
__device__ __forceinline__ uint64_t kpack(uint32_t r, uint32_t c, int ks) { return ((uint64_t)r << ks) | c; }
__device__ __forceinline__ uint32_t krow(uint64_t k, int ks) { return (uint32_t)(k >> ks); }
__device__ __forceinline__ uint32_t kcol(uint64_t k, int ks) { return (uint32_t)(k & ((1ull << ks) - 1ull)); }

// ------------------------------------------------------------------ exact accumulation
// Signed 128-bit accumulation into (lo, hi) words with two 64-bit atomics: the carry out of
// the low word is detected from the value returned by the low-word atomic.
__device__ __forceinline__ void atomic_add_i128(u64a* lo, i64a* hi, i128 v) {
  const u64a vlo = (u64a)v;
  const i64a vhi = (i64a)(v >> 64);
  const u64a old = atomicAdd(lo, vlo);
  const i64a carry = (old + vlo < old) ? 1 : 0;
  if (vhi + carry != 0) atomicAdd((u64a*)hi, (u64a)(vhi + carry));
}
__device__ __forceinline__ void atomic_add_i64(int64_t* p, int64_t v) { atomicAdd((u64a*)p, (u64a)v); }

// Orders the LDS accesses of one wavefront (all its lanes) with respect to each other.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ wave reductions
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ i128 wave_sum_i128(i128 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t lo = (uint64_t)__shfl_xor((long long)(uint64_t)v, o, 64);
    const int64_t hi = (int64_t)__shfl_xor((long long)(int64_t)(v >> 64), o, 64);
    v += ((i128)hi << 64) | (i128)lo;
  }
  return v;
}

// Best (gain, id): larger gain wins, equal gains go to the lower id.  valid == 0 is worse than
// anything.  A valid entry's `valid` is 1, or, for the randomised refinement, the target's draw
// priority (odd, compared as unsigned before the gain).
struct Best {
  int64_t hi;
  uint64_t lo;
  uint32_t id;
  int valid;
};
__device__ __forceinline__ i128 best_gain(const Best& b) { return ((i128)b.hi << 64) | (i128)b.lo; }
__device__ __forceinline__ bool better(const Best& x, const Best& y) {
  if (!x.valid) return false;
  if (!y.valid) return true;
  if (x.valid != y.valid) return (uint32_t)x.valid > (uint32_t)y.valid;
  if (x.hi != y.hi) return x.hi > y.hi;
  if (x.lo != y.lo) return x.lo > y.lo;
  return x.id < y.id;
}
__device__ __forceinline__ Best shfl_xor_best(const Best& b, int mask, int width) {
  Best r;
  r.hi = __shfl_xor(b.hi, mask, width);
  r.lo = (uint64_t)__shfl_xor((long long)b.lo, mask, width);
  r.id = (uint32_t)__shfl_xor((int)b.id, mask, width);
  r.valid = __shfl_xor(b.valid, mask, width);
  return r;
}
// reduce over aligned groups of `width` lanes (width a power of two <= 64)
__device__ __forceinline__ Best group_best(Best b, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) {
    Best t = shfl_xor_best(b, o, width);
    if (better(t, b)) b = t;
  }
  return b;
}
__device__ __forceinline__ Best make_best(i128 g, uint32_t id) {
  Best b;
  b.hi = (int64_t)(g >> 64);
  b.lo = (uint64_t)g;
  b.id = id;
  b.valid = 1;
  return b;
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// ------------------------------------------------------------------ launch shapes (host)
// Workgroups of `kernel` (launched with `threads` per workgroup) that are resident on the
// current device at once.  Kernels whose work count is read on the device loop over it
// grid-stride; a grid larger than this only adds workgroups that wait for a free slot and then
// find nothing to do, which costs more than the work itself when the count is small.
inline unsigned resident_blocks(const void* kernel, int threads) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 1;
  }
  return (unsigned)per_cu * (unsigned)cus;
}
// resident_blocks of one kernel, computed on its first launch (per template instantiation)
#define LDL_RESIDENT(kern, threads)                                                     \
  ([] {                                                                                 \
    static const unsigned resident_ = ::ldl::resident_blocks((const void*)(kern), (threads)); \
    return resident_;                                                                   \
  }())
inline unsigned cap_blocks(uint64_t want, unsigned resident) {
  if (want < 1) want = 1;
  return want < resident ? (unsigned)want : resident;
}

}  // namespace ldl

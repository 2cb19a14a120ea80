// Library primitives (radix sort, reduce-by-key, scan, max) from hipCUB and rocPRIM, with temporary
// storage grown on demand.
#include <hipcub/hipcub.hpp>
#include <rocprim/device/device_radix_sort.hpp>

#include "ldl_kernels.h"

namespace ldl {

namespace {

thread_local const PrimAlloc* t_alloc = nullptr;   // set by the handle that calls in

void tmp_free(void* p, size_t bytes) {
  if (!p) return;
  if (t_alloc && t_alloc->free) t_alloc->free(t_alloc->ctx, p, bytes);
  else (void)hipFree(p);
}

int ensure(void** tmp, size_t* bytes, size_t need) {
  if (need <= *bytes && *tmp) return 0;
  tmp_free(*tmp, *bytes);
  *tmp = nullptr;
  size_t n = need + (need >> 2) + 256;
  void* p = nullptr;
  if (t_alloc && t_alloc->alloc) p = t_alloc->alloc(t_alloc->ctx, n);
  else if (hipMalloc(&p, n) != hipSuccess) p = nullptr;
  if (!p) {
    (void)hipGetLastError();
    *tmp = nullptr;
    *bytes = 0;
    return -1;
  }
  *tmp = p;
  *bytes = n;
  return 0;
}

struct StampIs {
  const uint32_t* stamp;
  uint32_t ep;
  __host__ __device__ __forceinline__ bool operator()(const uint32_t& i) const { return stamp[i] == ep; }
};

struct RowHead {
  const uint64_t* keys;
  int ks;
  __host__ __device__ __forceinline__ bool operator()(const uint64_t& i) const {
    return i == 0 || (keys[i] >> ks) != (keys[i - 1] >> ks);
  }
};

struct SumU64x3 {
  __host__ __device__ __forceinline__ U64x3 operator()(const U64x3& a, const U64x3& b) const {
    return U64x3{a.x + b.x, a.y + b.y, a.z + b.z};
  }
};

struct SumI64 {
  __host__ __device__ __forceinline__ int64_t operator()(const int64_t& a, const int64_t& b) const { return a + b; }
};

}  // namespace

void prim_set_allocator(const PrimAlloc* a) { t_alloc = a; }
void prim_free_tmp(void* tmp, size_t bytes) { tmp_free(tmp, bytes); }

int prim_sort_pairs_u64_u32(void** tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout, const uint32_t* vin,
                            uint32_t* vout, uint64_t n, int begin_bit, int end_bit, hipStream_t s) {
  if (n == 0) return 0;
  if (n > (uint64_t)INT32_MAX) return -2;   // counts are int in the library
  size_t need = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, need, kin, kout, vin, vout, (int)n, begin_bit, end_bit, s) !=
      hipSuccess)
    return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  return hipcub::DeviceRadixSort::SortPairs(*tmp, have, kin, kout, vin, vout, (int)n, begin_bit, end_bit, s) ==
                 hipSuccess
             ? 0
             : -1;
}

// Ping-pong form with a 64-bit count (rocPRIM sorts in batches of 2^30 items): the sorted pairs
// end in buffers 0 or 1 (*sel), both of which are overwritten; the temporary storage does not hold
// a copy of the data.
int prim_sort_pairs_u64_u32_db(void** tmp, size_t* tmp_bytes, uint64_t* k0, uint64_t* k1, uint32_t* v0, uint32_t* v1,
                               uint64_t n, int begin_bit, int end_bit, int* sel, hipStream_t s) {
  *sel = 0;
  if (n == 0) return 0;
  rocprim::double_buffer<uint64_t> keys(k0, k1);
  rocprim::double_buffer<uint32_t> vals(v0, v1);
  const size_t count = (size_t)n;
  size_t need = 0;
  if (rocprim::radix_sort_pairs(nullptr, need, keys, vals, count, (unsigned)begin_bit, (unsigned)end_bit, s) !=
      hipSuccess)
    return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  if (rocprim::radix_sort_pairs(*tmp, have, keys, vals, count, (unsigned)begin_bit, (unsigned)end_bit, s) != hipSuccess)
    return -1;
  *sel = keys.current() == k0 ? 0 : 1;
  return 0;
}

int prim_sort_pairs_u64_i64(void** tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout, const int64_t* vin,
                            int64_t* vout, uint64_t n, int begin_bit, int end_bit, hipStream_t s) {
  if (n == 0) return 0;
  if (n > (uint64_t)INT32_MAX) return -2;   // counts are int in the library
  size_t need = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, need, kin, kout, vin, vout, (int)n, begin_bit, end_bit, s) !=
      hipSuccess)
    return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  return hipcub::DeviceRadixSort::SortPairs(*tmp, have, kin, kout, vin, vout, (int)n, begin_bit, end_bit, s) ==
                 hipSuccess
             ? 0
             : -1;
}

int prim_reduce_by_key(void** tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout, const int64_t* vin,
                       int64_t* vout, u64a* nruns, uint64_t n, hipStream_t s) {
  if (n == 0) return 0;
  if (n > (uint64_t)INT32_MAX) return -2;   // counts are int in the library
  size_t need = 0;
  if (hipcub::DeviceReduce::ReduceByKey(nullptr, need, kin, kout, vin, vout, nruns, SumI64(), (int)n, s) !=
      hipSuccess)
    return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  return hipcub::DeviceReduce::ReduceByKey(*tmp, have, kin, kout, vin, vout, nruns, SumI64(), (int)n, s) ==
                 hipSuccess
             ? 0
             : -1;
}

int prim_exclusive_sum_u64(void** tmp, size_t* tmp_bytes, const uint64_t* in, uint64_t* out, uint64_t n,
                           hipStream_t s) {
  if (n == 0) return 0;
  if (n > (uint64_t)INT32_MAX) return -2;   // counts are int in the library
  size_t need = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, need, in, out, (int)n, s) != hipSuccess) return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  return hipcub::DeviceScan::ExclusiveSum(*tmp, have, in, out, (int)n, s) == hipSuccess ? 0 : -1;
}

int prim_max_u64(void** tmp, size_t* tmp_bytes, const uint64_t* in, u64a* out, uint64_t n, hipStream_t s) {
  if (n == 0) return 0;
  if (n > (uint64_t)INT32_MAX) return -2;   // counts are int in the library
  size_t need = 0;
  if (hipcub::DeviceReduce::Max(nullptr, need, in, (uint64_t*)out, (int)n, s) != hipSuccess) return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  return hipcub::DeviceReduce::Max(*tmp, have, in, (uint64_t*)out, (int)n, s) == hipSuccess ? 0 : -1;
}

int prim_select_stamp(void** tmp, size_t* tmp_bytes, const uint32_t* stamp, uint32_t ep, uint32_t n, uint32_t* out,
                      uint32_t* d_count, hipStream_t s) {
  if (n == 0) return 0;
  if (n > (uint64_t)INT32_MAX) return -2;   // counts are int in the library
  hipcub::CountingInputIterator<uint32_t> ids(0);
  StampIs pred{stamp, ep};
  size_t need = 0;
  if (hipcub::DeviceSelect::If(nullptr, need, ids, out, d_count, (int)n, pred, s) != hipSuccess) return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  return hipcub::DeviceSelect::If(*tmp, have, ids, out, d_count, (int)n, pred, s) == hipSuccess ? 0 : -1;
}

int prim_select_heads(void** tmp, size_t* tmp_bytes, const uint64_t* keys, uint64_t k, int ks, uint64_t* out,
                      uint32_t* d_count, hipStream_t s) {
  if (k == 0) return 0;
  if (k > (uint64_t)INT32_MAX) return -2;   // counts are int in the library
  hipcub::CountingInputIterator<uint64_t> ids(0);
  RowHead pred{keys, ks};
  size_t need = 0;
  if (hipcub::DeviceSelect::If(nullptr, need, ids, out, d_count, (int)k, pred, s) != hipSuccess) return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  return hipcub::DeviceSelect::If(*tmp, have, ids, out, d_count, (int)k, pred, s) == hipSuccess ? 0 : -1;
}

int prim_exclusive_sum_u64x3(void** tmp, size_t* tmp_bytes, const U64x3* in, U64x3* out, uint64_t n, hipStream_t s) {
  if (n == 0) return 0;
  if (n > (uint64_t)INT32_MAX) return -2;   // counts are int in the library
  size_t need = 0;
  const U64x3 zero{0, 0, 0};
  if (hipcub::DeviceScan::ExclusiveScan(nullptr, need, in, out, SumU64x3(), zero, (int)n, s) != hipSuccess) return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  return hipcub::DeviceScan::ExclusiveScan(*tmp, have, in, out, SumU64x3(), zero, (int)n, s) == hipSuccess ? 0 : -1;
}

int prim_exclusive_sum_u32(void** tmp, size_t* tmp_bytes, const uint32_t* in, uint32_t* out, uint64_t n,
                           hipStream_t s) {
  if (n == 0) return 0;
  if (n > (uint64_t)INT32_MAX) return -2;   // counts are int in the library
  size_t need = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, need, in, out, (int)n, s) != hipSuccess) return -1;
  if (ensure(tmp, tmp_bytes, need)) return -2;
  size_t have = *tmp_bytes;
  return hipcub::DeviceScan::ExclusiveSum(*tmp, have, in, out, (int)n, s) == hipSuccess ? 0 : -1;
}

}  // namespace ldl

// Device helpers shared by the level-kernel translation units.
#pragma once

#include "lv_internal.h"

namespace lv {
namespace {

// 16-byte vector of T held as an array.
template <typename T> struct alignas(16) V16 { T v[16 / sizeof(T)]; };

template <typename T> __device__ __forceinline__ V16<T> ld16(const T* p) {
  return *reinterpret_cast<const V16<T>*>(p);
}
template <typename T> __device__ __forceinline__ void st16(T* p, const V16<T>& x) {
  *reinterpret_cast<V16<T>*>(p) = x;
}

// Streaming variants for data touched once per pass (the stored powers):
// non-temporal loads and stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T> __device__ __forceinline__ V16<T> ld16_nt(const T* p) {
  return __builtin_bit_cast(V16<T>, __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p)));
}
template <typename T> __device__ __forceinline__ void st16_nt(T* p, const V16<T>& x) {
  __builtin_nontemporal_store(__builtin_bit_cast(u32x4, x), reinterpret_cast<u32x4*>(p));
}

// Value of x in lane l (l uniform), broadcast to the whole wave.
template <typename T> __device__ __forceinline__ T lane_bcast(T x, int l) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
  } else {
    static_assert(sizeof(T) == 8, "32- or 64-bit values");
    const int2 h = __builtin_bit_cast(int2, x);
    return __builtin_bit_cast(T, make_int2(__builtin_amdgcn_readlane(h.x, l), __builtin_amdgcn_readlane(h.y, l)));
  }
}

// Staging of a work-group's operand tile: thread tid moves entries
// e = 0 .. COUNT-1 (entry e is the group-wide index tid + NT e; entries at
// or beyond N are skipped).  The loads of a batch of up to 16 entries are all
// issued before any of them is stored, so the staging costs a few memory
// latencies rather than one per entry.  ld(idx) returns the value of entry
// idx, st(idx, v) stores it.
template <int COUNT, int NT, typename V, typename Ld, typename St>
__device__ __forceinline__ void batched_stage(const int tid, const int N, Ld&& ld, St&& st) {
  constexpr int B = COUNT < 16 ? COUNT : 16;
#pragma unroll
  for (int e0 = 0; e0 < COUNT; e0 += B) {
    V v[B];
#pragma unroll
    for (int e = 0; e < B; ++e) {
      const int idx = tid + NT * (e0 + e);
      if (e0 + e < COUNT) v[e] = idx < N ? ld(idx) : V(0);
    }
#pragma unroll
    for (int e = 0; e < B; ++e) {
      const int idx = tid + NT * (e0 + e);
      if (e0 + e < COUNT && idx < N) st(idx, v[e]);
    }
  }
}

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Index of the descriptor whose block range holds block `b` (descriptors are
// sorted by block_begin, the first starts at 0): binary search, uniform.
template <typename D>
__device__ __forceinline__ int find_desc(const D* __restrict__ ds, int nd, int b) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace
}  // namespace lv

// switch over the level ranks 1..128 with RR a constant expression
#define LV_RANK_SWITCH(R, CALL)            \
  switch (R) {                              \
    case 1: { constexpr int RR = 1; CALL; }   \
    case 2: { constexpr int RR = 2; CALL; }   \
    case 4: { constexpr int RR = 4; CALL; }   \
    case 8: { constexpr int RR = 8; CALL; }   \
    case 16: { constexpr int RR = 16; CALL; } \
    case 32: { constexpr int RR = 32; CALL; } \
    case 64: { constexpr int RR = 64; CALL; } \
    case 128: { constexpr int RR = 128; CALL; } \
    default: return hipErrorInvalidValue;   \
  }

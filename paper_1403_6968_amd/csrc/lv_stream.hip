// Streaming kernels that measure the device's attainable HBM rate with the
// access pattern of the level passes: 16-byte non-temporal loads and stores,
// each wave touching whole 1 KiB row segments (64 lanes x 16 bytes).  They
// give the measured ceiling that the level passes are compared with; the
// kernels carry none of the method's arithmetic.
//
// Kinds:
//   LV_STREAM_RMW    x = a * x in place (one read and one write of every
//                    element at the same address: the level passes' pattern)
//   LV_STREAM_COPY   dst = a * src
//   LV_STREAM_READ   read every element; one float per thread (the sum of
//                    what it read) goes to dst so the loads stay live
//   LV_STREAM_WRITE  dst = a
// A work-group iteration covers `depth` x 4 KiB of contiguous bytes (thread t
// of the group loads vector t, t + 256, ...); groups stride over the buffer.
// `pipelined` issues the loads of the group's next iteration before storing
// the current one (twice the bytes in flight per wave).
#include "lv_view_impl.h"

namespace lv {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 ldnt(const f32x4* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void stnt(f32x4* p, f32x4 x) { __builtin_nontemporal_store(x, p); }

template <int KIND, int D, bool PIPE>
__global__ void __launch_bounds__(256)
k_stream(f32x4* __restrict__ dst, const f32x4* __restrict__ src, int64_t nchunks, float a,
         float* __restrict__ sink) {
  constexpr int64_t CH = 256 * D;   // vectors per chunk
  const int tid = threadIdx.x;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  int64_t c = blockIdx.x;
  if constexpr (KIND == LV_STREAM_WRITE) {
    const f32x4 w = {a, a, a, a};
    for (; c < nchunks; c += gridDim.x) {
#pragma unroll
      for (int d = 0; d < D; ++d) stnt(dst + c * CH + d * 256 + tid, w);
    }
    return;
  }
  const f32x4* in = KIND == LV_STREAM_RMW ? dst : src;
  f32x4 v[D];
  if (c < nchunks) {
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = ldnt(in + c * CH + d * 256 + tid);
  }
  for (; c < nchunks; c += gridDim.x) {
    const int64_t cn = c + gridDim.x;
    f32x4 w[PIPE ? D : 1];
    if constexpr (PIPE) {
      if (cn < nchunks) {
#pragma unroll
        for (int d = 0; d < D; ++d) w[d] = ldnt(in + cn * CH + d * 256 + tid);
      }
    }
    if constexpr (KIND == LV_STREAM_READ) {
#pragma unroll
      for (int d = 0; d < D; ++d) acc += v[d];
    } else {
#pragma unroll
      for (int d = 0; d < D; ++d) stnt(dst + c * CH + d * 256 + tid, v[d] * a);
    }
    if constexpr (PIPE) {
#pragma unroll
      for (int d = 0; d < D; ++d) v[d] = w[d];
    } else if (cn < nchunks) {
#pragma unroll
      for (int d = 0; d < D; ++d) v[d] = ldnt(in + cn * CH + d * 256 + tid);
    }
  }
  if constexpr (KIND == LV_STREAM_READ) sink[(int64_t)blockIdx.x * 256 + tid] = acc.x + acc.y + acc.z + acc.w;
}

template <int KIND, bool PIPE>
hipError_t stream_depth(int depth, unsigned blocks, f32x4* dst, const f32x4* src, int64_t nvec, float a,
                        float* sink, hipStream_t s) {
  switch (depth) {
#define LV_STREAM_CASE(D)                                                                                  \
    case D:                                                                                                \
      hipLaunchKernelGGL((k_stream<KIND, D, PIPE>), dim3(blocks), dim3(256), 0, s, dst, src, nvec / (256 * D), a, \
                         sink);                                                                            \
      return hipGetLastError();
    LV_STREAM_CASE(1)
    LV_STREAM_CASE(2)
    LV_STREAM_CASE(4)
    LV_STREAM_CASE(8)
    LV_STREAM_CASE(16)
    LV_STREAM_CASE(32)
#undef LV_STREAM_CASE
    default: return hipErrorInvalidValue;
  }
}

template <int KIND>
hipError_t stream_kind(int depth, bool pipe, unsigned blocks, f32x4* dst, const f32x4* src, int64_t nvec, float a,
                       float* sink, hipStream_t s) {
  return pipe ? stream_depth<KIND, true>(depth, blocks, dst, src, nvec, a, sink, s)
              : stream_depth<KIND, false>(depth, blocks, dst, src, nvec, a, sink, s);
}

}  // namespace
}  // namespace lv

using namespace lv;

extern "C" {

lv_status lv_stream_probe(int kind, void* dst, const void* src, size_t bytes, int blocks, int depth, int pipelined,
                          void* stream) {
  g_err[0] = 0;
  if (kind < LV_STREAM_RMW || kind > LV_STREAM_WRITE) return fail(LV_EINVAL, "unknown stream kind %d", kind);
  if (depth != 1 && depth != 2 && depth != 4 && depth != 8 && depth != 16 && depth != 32)
    return fail(LV_EINVAL, "depth %d is not one of 1, 2, 4, 8, 16, 32", depth);
  if (blocks < 1 || blocks > (1 << 20)) return fail(LV_EINVAL, "blocks %d out of range", blocks);
  const size_t chunk = (size_t)4096 * depth;
  if (bytes == 0 || bytes % chunk) return fail(LV_EINVAL, "bytes %zu is not a positive multiple of %zu", bytes, chunk);
  if (!dst || (kind == LV_STREAM_COPY && !src)) return fail(LV_EINVAL, "NULL pointer");
  if (reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
    return fail(LV_EINVAL, "buffers must be 16-byte aligned");
  auto* d = static_cast<f32x4*>(dst);
  const auto* sp = static_cast<const f32x4*>(src);
  const int64_t nvec = (int64_t)(bytes / 16);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // READ: the source is `src` when given, else `dst`; one float per thread
  // of the grid goes to dst (at its start), so dst needs blocks * 1 KiB.
  float* sink = reinterpret_cast<float*>(dst);
  hipError_t e;
  switch (kind) {
    case LV_STREAM_RMW: e = stream_kind<LV_STREAM_RMW>(depth, pipelined != 0, blocks, d, sp, nvec, 1.0f, nullptr, s); break;
    case LV_STREAM_COPY: e = stream_kind<LV_STREAM_COPY>(depth, pipelined != 0, blocks, d, sp, nvec, 1.0f, nullptr, s); break;
    case LV_STREAM_READ:
      if (!src) return fail(LV_EINVAL, "READ needs src (the buffer read) and dst (blocks * 1024 bytes)");
      e = stream_kind<LV_STREAM_READ>(depth, pipelined != 0, blocks, nullptr, sp, nvec, 1.0f, sink, s);
      break;
    default: e = stream_kind<LV_STREAM_WRITE>(depth, pipelined != 0, blocks, d, nullptr, nvec, 0.0f, nullptr, s); break;
  }
  return hip_check(e, "stream probe");
}

}  // extern "C"

// Streaming-read reference for the roofline of the HBM-bound kernels: read a
// device buffer once with 16-byte loads and nothing else, so that the
// achieved rate of a kernel that streams the same bytes (the skeleton
// product streams its operators) can be set beside what this chip delivers
// to a pure read stream, as well as beside the published peak.  Not a step
// of the method.
#include <climits>

#include "el_internal.h"

namespace el {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 16;                                    // 16-byte loads in flight per thread
constexpr int64_t kProbeChunk = (int64_t)kProbeThreads * kProbeUnroll * 16;   // 16-byte words per block (1 MiB)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Each workgroup reads one contiguous 1 MiB chunk, kProbeUnroll
// non-temporal 16-byte loads per thread in flight (the fastest of the
// grid-stride and chunked forms with plain or non-temporal loads measured on
// MI355X); the XOR of every 32-bit word read is folded per thread, then
// over the wave, and combined with one vector atomic per wave into *sink,
// which keeps the loads from being removed.
__global__ void __launch_bounds__(kProbeThreads) k_stream_read(const u32x4* __restrict__ p, int64_t n16,
                                                                 uint32_t* __restrict__ sink) {
  const int64_t b0 = (int64_t)blockIdx.x * kProbeChunk, b1 = min(n16, b0 + kProbeChunk);
  uint32_t acc = 0;
  int64_t i = b0 + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * kProbeThreads < b1; i += kProbeUnroll * kProbeThreads) {
    u32x4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(p + i + u * kProbeThreads);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < b1; i += kProbeThreads) {
    const u32x4 v = p[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) atomicXor(sink, acc);
}

}  // namespace
}  // namespace el

using namespace el;

extern "C" el_status el_stream_read(el_ctx* ctx, const void* buf, size_t bytes, uint32_t* sink) {
  if (!ctx) return EL_ERR_ARG;
  if (!buf || !sink || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(buf) % 16 != 0)
    return set_error(ctx, EL_ERR_ARG, "el_stream_read: null pointer, or size or address not a multiple of 16");
  if (bytes == 0) return EL_OK;
  hipSetDevice(ctx->device);
  const int64_t n16 = (int64_t)(bytes / 16);
  const int64_t grid = (n16 + kProbeChunk - 1) / kProbeChunk;
  if (grid > INT32_MAX) return set_error(ctx, EL_ERR_ARG, "el_stream_read: buffer too large");
  hipLaunchKernelGGL(k_stream_read, dim3((unsigned)grid), dim3(kProbeThreads), 0, ctx->stream,
                     reinterpret_cast<const u32x4*>(buf), n16, sink);
  return hip_check(ctx, hipGetLastError(), "launch k_stream_read");
}

// BF16 matrix-core GEMM for the element network (Sec. 2.4.1: fully connected
// layers x_i = f_i(A_i x_{i-1} + b_i)), gfx950 v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation.
//
//   C[M x N] = sum_k A(m, k) B(k, n)  over k in [k_begin, k_end)
//
// A(m,k) = A[m*lda + k] if A_KC (k contiguous) else A[k*lda + m];
// B(k,n) = B[n*ldb + k] if B_KC (k contiguous) else B[k*ldb + n].
// Block tile 128 x 128 x 32, 256 threads; each wave64 owns a 64 x 64 sub-tile
// (4 x 4 MFMA tiles).  Tiles are staged in LDS with k contiguous (the layout
// the MFMA operands want: 8 consecutive k per lane), double buffered, with
// a row pitch of 40 bf16 to spread LDS banks.  Operands not k-contiguous in
// HBM are transposed on the way into LDS.  Split-K runs over gridDim.z.
// The kernel itself (k_mm) lives with its epilogues in k_net.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace el {
namespace gemm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int PITCH = 40;            // bf16 per LDS row
constexpr int kThreads = 256;

__device__ inline uint16_t f2bf(float f) {
  // round to nearest even (NaN kept quiet)
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

template <bool KC>
__device__ inline void load_tile(const uint16_t* __restrict__ G, int64_t ld, int rows, int r0, int k0, int kend,
                                 uint16_t* __restrict__ S, int tid) {
  // S[r][k], r < 128, k < 32
  if (KC) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int idx = tid + it * kThreads;
      const int r = idx >> 2, seg = (idx & 3) * 8;
      const int gr = r0 + r, gk = k0 + seg;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gr < rows) {
        const uint16_t* p = G + (int64_t)gr * ld + gk;
        if (gk + 8 <= kend) {
          v = *reinterpret_cast<const uint4*>(p);
        } else if (gk < kend) {
          uint16_t tmp[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) tmp[u] = (gk + u < kend) ? p[u] : (uint16_t)0;
          v = *reinterpret_cast<uint4*>(tmp);
        }
      }
      *reinterpret_cast<uint4*>(S + r * PITCH + seg) = v;
    }
  } else {
    // G[k*ld + r]: 32 k-rows of 128 r-values; thread loads 8 r at one k
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int idx = tid + it * kThreads;
      const int kr = idx >> 4, seg = (idx & 15) * 8;
      const int gk = k0 + kr, gr = r0 + seg;
      uint16_t tmp[8];
      if (gk < kend && gr + 8 <= rows) {
        uint4 v = *reinterpret_cast<const uint4*>(G + (int64_t)gk * ld + gr);
        *reinterpret_cast<uint4*>(tmp) = v;
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) tmp[u] = (gk < kend && gr + u < rows) ? G[(int64_t)gk * ld + gr + u] : (uint16_t)0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) S[(seg + u) * PITCH + kr] = tmp[u];
    }
  }
}

}  // namespace gemm
}  // namespace el

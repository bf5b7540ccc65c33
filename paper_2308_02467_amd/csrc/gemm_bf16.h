// BF16 matrix-core GEMM for the element network (Sec. 2.4.1: fully connected
// layers x_i = f_i(A_i x_{i-1} + b_i)), gfx950 v_mfma_f32_32x32x16_bf16 with
// FP32 accumulation.
//
//   C[M x N] = sum_k A(m, k) B(k, n)  over k in [k_begin, k_end)
//
// A(m,k) = A[m*lda + k] if A_KC (k contiguous) else A[k*lda + m];
// B(k,n) = B[n*ldb + k] if B_KC (k contiguous) else B[k*ldb + n].
// 256 threads = 2 x 2 waves; each wave owns TM x TN MFMA tiles of 32 x 32,
// so the block tile is (64 TM) x (64 TN) x 64.  Tiles are staged in LDS with
// k contiguous (the operand layout of the MFMA: 8 consecutive k per lane),
// double buffered, row pitch 72 bf16 (conflict-free 16-byte fragment reads).
// The k tile two steps ahead is loaded from HBM into registers while the
// current one is multiplied, and the next one is written from registers to
// the other LDS buffer: one barrier per k tile.  Operands not k-contiguous in HBM are transposed on the way into
// LDS.  Split-K runs over gridDim.z.  The kernel itself (k_mm) lives with
// its epilogues in k_net.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace el {
namespace gemm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BK = 64;
constexpr int PITCH = 72;            // bf16 per LDS row
constexpr int kThreads = 256;

__device__ inline uint16_t f2bf(float f) {
  // round to nearest even (NaN kept quiet)
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// One operand tile of R rows (M or N) x BK k, HBM -> registers -> LDS
// S[r * PITCH + k].  The loads are unconditional (addresses clamped into the
// operand, out-of-range segments replaced by zeros), so every k tile issues
// the same loads and the waits for a tile do not cover the loads issued
// after it.  Requires the contiguous dimension and K to be multiples of 8
// (checked by the host).
//
// k contiguous in HBM: each thread moves NSEG segments of 8 k (16 bytes).
// r contiguous in HBM (transposed on the way): each work item reads 8 r at
// two consecutive k (two 16-byte loads) and writes 8 packed (k, k+1) pairs;
// the 32 items of a half-wave cover 64 consecutive k of one row, so the
// 4-byte LDS writes of a wave hit 64 different banks.
template <bool KC, int R>
struct TileLoader {
  static constexpr int NSEG = R * BK / 8 / kThreads;   // 16-byte loads per thread
  uint4 v[NSEG];

  __device__ inline void load(const uint16_t* __restrict__ G, int64_t ld, int rows, int r0, int k0, int kend,
                              int tid) {
#pragma unroll
    for (int it = 0; it < NSEG; ++it) {
      int gr, gk;
      if (KC) {
        const int idx = tid + it * kThreads;
        gr = r0 + (idx >> 3);
        gk = k0 + (idx & 7) * 8;
      } else {
        const int idx = tid + (it >> 1) * kThreads;   // work item
        gk = k0 + 2 * (idx & 31) + (it & 1);
        gr = r0 + (idx >> 5) * 8;
      }
      const bool ok = gr < rows && gk < kend;
      const int cr = min(gr, rows - (KC ? 1 : 8)), ck = min(gk, kend - (KC ? 8 : 1));
      const uint16_t* p = KC ? G + (int64_t)cr * ld + ck : G + (int64_t)ck * ld + cr;
      const uint4 x = *reinterpret_cast<const uint4*>(p);
      v[it] = ok ? x : make_uint4(0, 0, 0, 0);
    }
  }

  __device__ inline void store(uint16_t* __restrict__ S, int tid) const {
    if (KC) {
#pragma unroll
      for (int it = 0; it < NSEG; ++it) {
        const int idx = tid + it * kThreads;
        const int r = idx >> 3, seg = (idx & 7) * 8;
        *reinterpret_cast<uint4*>(S + r * PITCH + seg) = v[it];
      }
    } else {
#pragma unroll
      for (int it = 0; it < NSEG; it += 2) {
        const int idx = tid + (it >> 1) * kThreads;
        const int c = idx & 31, r = (idx >> 5) * 8;
        const uint32_t lo[4] = {v[it].x, v[it].y, v[it].z, v[it].w};           // k = 2c
        const uint32_t hi[4] = {v[it + 1].x, v[it + 1].y, v[it + 1].z, v[it + 1].w};   // k = 2c + 1
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          *reinterpret_cast<uint32_t*>(S + (r + 2 * u) * PITCH + 2 * c) = (lo[u] & 0xffffu) | (hi[u] << 16);
          *reinterpret_cast<uint32_t*>(S + (r + 2 * u + 1) * PITCH + 2 * c) = (lo[u] >> 16) | (hi[u] & 0xffff0000u);
        }
      }
    }
  }
};

}  // namespace gemm
}  // namespace el

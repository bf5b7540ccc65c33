// Element network (Sec. 2.4.1 architecture, Sec. 2.4.2 / 3.1 training):
// features, forward, MAE loss, backward, Adam, statistics, inference with
// range check and plain-solver fallback.  All GEMMs run on the BF16 matrix
// cores (gemm_bf16.h) with FP32 accumulation; master weights and optimizer
// state are FP32.
#include <atomic>
#include <climits>
#include <cmath>
#include <type_traits>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "el_internal.h"
#include "gemm_bf16.h"

struct el_net {
  el_net_desc desc{};
  int k0 = 0;                       // padded input width
  int64_t n_params = 0;
  std::vector<int64_t> w_off, b_off, in_dim, out_dim;   // per layer 0..depth
  float* theta = nullptr;
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t* wbf = nullptr;          // bfloat16 copy of theta
  float* feat_mean = nullptr;
  float* feat_std = nullptr;
  float* y_mean = nullptr;
  float* y_std = nullptr;
  double box[6] = {0, 0, 0, 0, 0, 0};
  int64_t step = 0;
  bool fitted = false;
  int device = 0;
  el::Workspace scratch;
  el::Workspace scratch32;         // FP32 network path (el_train_step_f32, el_net_forward_f32)
};

namespace el {
namespace {

using gemm::bf2f;
using gemm::f2bf;

constexpr float kTauFloor = 1e-12f;

__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void k_init_uniform(float* p, int64_t count, int64_t in_total, int64_t in_valid, float bound,
                               uint64_t seed, int64_t offset) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  if (in_total > 0 && (i % in_total) >= in_valid) { p[i] = 0.f; return; }
  uint64_t r = splitmix64(seed ^ splitmix64((uint64_t)(offset + i)));
  double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);
  p[i] = (float)((2.0 * u - 1.0) * bound);
}

__global__ void k_fill_f(float* p, int64_t n, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_to_bf16(const float* __restrict__ s, uint16_t* __restrict__ d, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = f2bf(s[i]);
}

__device__ inline float feature_value(int f, double h, double v) {
  // f == 0: log10 h; else log10 max(h v / 2, floor)
  if (f == 0) return (float)log10(h);
  return (float)log10(fmax(0.5 * h * v, (double)kTauFloor));
}

struct Box {
  double v[6];
};

// raw inputs (FP32 [B][n_in] or FP64 h/kappa/sigma) -> z-scored bfloat16 X0 [B][k0]
__global__ void k_features(const float* __restrict__ x32, const double* __restrict__ h64,
                           const double* __restrict__ kap64, const double* __restrict__ sig64, int64_t B,
                           int n_in, int k0, const float* __restrict__ mean, const float* __restrict__ stdv,
                           uint16_t* __restrict__ X0, Box box, uint8_t* __restrict__ in_range) {
  const int64_t b = blockIdx.x;
  if (b >= B) return;
  const int nn = (n_in - 1) / 2;
  __shared__ int ok;
  if (threadIdx.x == 0) ok = 1;
  __syncthreads();
  double h = x32 ? (double)x32[b * n_in] : h64[b];
  for (int f = threadIdx.x; f < k0; f += blockDim.x) {
    uint16_t out = 0;
    if (f < n_in) {
      double v = 0.0;
      bool inside;
      if (f == 0) {
        inside = h >= box.v[0] && h <= box.v[1];
      } else if (f <= nn) {
        v = x32 ? (double)x32[b * n_in + f] : kap64[b * nn + f - 1];
        inside = v >= box.v[2] && v <= box.v[3];
      } else {
        v = x32 ? (double)x32[b * n_in + f] : sig64[b * nn + f - 1 - nn];
        inside = v >= box.v[4] && v <= box.v[5];
      }
      if (!inside) ok = 0;
      float z = (feature_value(f, h, v) - mean[f]) / stdv[f];
      out = f2bf(z);
    }
    X0[b * k0 + f] = out;
  }
  __syncthreads();
  if (in_range && threadIdx.x == 0) in_range[b] = (uint8_t)ok;
}

__device__ inline float act_f(int act, float z) {
  if (act == EL_ACT_LINEAR) return z;
  if (act == EL_ACT_ELU) return z > 0.f ? z : expm1f(z);
  return 0.5f * z * (1.f + erff(z * 0.70710678118654752f));
}
__device__ inline float act_df(int act, float z) {
  if (act == EL_ACT_LINEAR) return 1.f;
  if (act == EL_ACT_ELU) return z > 0.f ? 1.f : expf(z);
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// GEMM epilogues.  The kernel calls col(n) once per output column a lane
// owns; per 32 x 32 MFMA block it then loads pre(m, n) for the block's rows
// of that column (all loads issued before any is used), calls
// block_begin(), (m, n, acc, z, c, pre) for each row and block_end(); so
// that per-column data (bias, output scaling) is loaded once and per-element
// inputs (the training targets) are fetched in one batch.
struct NoPre {};
#define EL_EPI_DEFAULT_HOOKS                                              \
  typedef NoPre Pre;                                                      \
  static constexpr bool kHasPre = false;                                  \
  static constexpr bool kStageLds = false;                                \
  __device__ Pre pre(int, int) const { return Pre{}; }                    \
  __device__ void block_begin() {}                                        \
  __device__ void block_end(int, int, int, int, int) {}

// hidden layer epilogue: z = acc + b; Z (optional) = z; H = bf16(act(z))
struct EpiHidden {
  static constexpr const char* kName = "hidden";
  static constexpr bool kRepeatable = true;   // running it twice gives the same outputs
  const float* bias;
  float* Z;
  uint16_t* H;
  int64_t ld;
  int act;
  struct Col { float b; };
  EL_EPI_DEFAULT_HOOKS
  __device__ Col col(int n) const { return Col{bias[n]}; }
  __device__ void operator()(int m, int n, float acc, int, const Col& c, Pre) {
    const float z = acc + c.b;
    if (Z) Z[(int64_t)m * ld + n] = z;
    H[(int64_t)m * ld + n] = f2bf(act_f(act, z));
  }
  __device__ void flush() {}
};

// output layer, normalized FP32 (testing the forward pass)
struct EpiOutNorm {
  static constexpr const char* kName = "out_norm";
  static constexpr bool kRepeatable = true;
  const float* bias;
  float* Y;
  int64_t ld;
  struct Col { float b; };
  EL_EPI_DEFAULT_HOOKS
  __device__ Col col(int n) const { return Col{bias[n]}; }
  __device__ void operator()(int m, int n, float acc, int, const Col& c, Pre) { Y[(int64_t)m * ld + n] = acc + c.b; }
  __device__ void flush() {}
};

// output layer, de-normalized operators (bfloat16 or float32): n < mm -> in2out, else in2sol
template <typename OutT>
struct EpiOutOps {
  static constexpr const char* kName = std::is_same<OutT, _Float16>::value ? "out_ops_f16"
                                       : sizeof(OutT) == 2 ? "out_ops_bf16" : "out_ops_f32";
  static constexpr bool kRepeatable = true;
  const float* bias;
  const float* ymean;
  const float* ystd;
  OutT* i2o;
  OutT* i2s;
  int64_t mm, nm;
  struct Col {
    float b, sd, mean;   // y = (acc + b) sd + mean
    OutT* base;          // column n of element 0, or null
    int64_t stride;      // per element
  };
  EL_EPI_DEFAULT_HOOKS
  __device__ static inline OutT cvt(float y) {
    if constexpr (std::is_same<OutT, _Float16>::value) return (_Float16)y;
    else if constexpr (sizeof(OutT) == 2) return f2bf(y);
    else return y;
  }
  __device__ Col col(int n) const {
    Col c;
    c.b = bias[n];
    c.sd = ystd[n];
    c.mean = ymean[n];
    if (n < mm) { c.base = i2o ? i2o + n : nullptr; c.stride = mm; }
    else { c.base = i2s ? i2s + (n - mm) : nullptr; c.stride = nm; }
    return c;
  }
  __device__ void operator()(int e, int, float acc, int, const Col& c, Pre) {
    if (c.base) c.base[(int64_t)e * c.stride] = cvt((acc + c.b) * c.sd + c.mean);
  }
  __device__ void flush() {}
};

// output layer in training: MAE against normalized targets; dY = sign(pred -
// target).  Repeatable (every run writes the same outputs): instead of
// accumulating, each 32 x 32 block writes the sum of its |d| to
// lossp[m / 32][n / 32] and, per column, the sum of its 32 signs to
// colp[m / 32][n] (the output-layer bias gradient in loss units: sums of
// +-1, exact in FP32 in any order); fixed-order reductions follow.
struct EpiMAE {
  static constexpr const char* kName = "mae";
  static constexpr bool kRepeatable = true;
  const float* bias;
  const uint16_t* y;
  const float* ymean;
  const float* ystd;
  uint16_t* dY;
  float* colp;    // [ceil(M/32)][ld]
  float* lossp;   // [ceil(M/32)][ceil(ld/32)]
  int64_t ld;
  float s_abs, s_sgn;
  struct Col { float b, mean, rsd; };
  typedef uint16_t Pre;
  static constexpr bool kHasPre = true;
  // the direct-to-LDS GEMM stages the block tile's targets in LDS first
  // (rows ym0.., columns yn0..; pitch ypitch; tile rows below ysplit from ys,
  // the others from ys2)
  static constexpr bool kStageLds = true;
  int ypitch, ysplit, ym0, yn0;
  // optionally the same codes transposed, dYT[n][m] (ldT = M, a multiple of
  // 4): a lane holds four consecutive rows of its column in consecutive
  // registers (block_begin starts each group of 32 rows), so it packs them
  // into one 8-byte store
  uint16_t* dYT;
  int64_t ldT;
  uint64_t pack;
  // LDS pointers are 4 bytes on the device and 8 on the host, so they come
  // last: every member the host sets has the same offset on both sides (the
  // host passes them null; the kernel sets them)
  const __attribute__((address_space(3))) uint16_t* ys;
  const __attribute__((address_space(3))) uint16_t* ys2;
  __device__ Col col(int n) const { return Col{bias[n], ymean[n], 1.f / ystd[n]}; }
  // from the LDS tile, or from HBM with 32-bit byte offsets from the
  // kernel-argument base (the host keeps B * n_out below 2^31): one address
  // register per load
  __device__ Pre pre(int m, int n) const {
    if (ys) {
      const int r = m - ym0;
      return r < ysplit ? ys[r * ypitch + (n - yn0)] : ys2[(r - ysplit) * ypitch + (n - yn0)];
    }
    const uint32_t off = ((uint32_t)m * (uint32_t)ld + (uint32_t)n) * 2u;
    return *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(y) + off);
  }
  __device__ void block_begin() { s_abs = 0.f; s_sgn = 0.f; pack = 0; }
  __device__ void operator()(int m, int n, float acc, int, const Col& c, Pre t) {
    const uint32_t i = (uint32_t)m * (uint32_t)ld + (uint32_t)n;   // below 2^31 (host check)
    const float pred = acc + c.b;
    const float tgt = (bf2f(t) - c.mean) * c.rsd;
    const float d = pred - tgt;
    s_abs += fabsf(d);
    const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
    s_sgn += sg;
    const uint16_t code = d > 0.f ? (uint16_t)0x3f80 : (d < 0.f ? (uint16_t)0xbf80 : (uint16_t)0);
    dY[i] = code;
    if (dYT) {
      pack |= (uint64_t)code << (16 * (m & 3));
      if ((m & 3) == 3) {
        *reinterpret_cast<uint64_t*>(dYT + (int64_t)n * ldT + (m - 3)) = pack;
        pack = 0;
      }
    }
  }
  // all 64 lanes call it: lanes l and l + 32 hold the two row halves of
  // column n0 + l % 32 of the block at rows m0.  Blocks past the output
  // (m0 >= M or n0 >= N: partial wave tiles) own no partial sums and write
  // nothing; for the others m0 / 32 < ceil(M / 32) and n0 / 32 < ceil(N / 32).
  __device__ void block_end(int m0, int n0, int lane, int M, int N) {
    const float a = s_abs + __shfl_xor(s_abs, 32);
    const float g = s_sgn + __shfl_xor(s_sgn, 32);
    float t = a;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (m0 >= M || n0 >= N) return;
    const int n = n0 + (lane & 31);
    if (lane < 32 && n < N) colp[(int64_t)(m0 >> 5) * ld + n] = g;
    if (lane == 0) lossp[(int64_t)(m0 >> 5) * ((ld + 31) >> 5) + (n0 >> 5)] = t;
  }
  __device__ void flush() {}
};

struct EpiF32 {
  static constexpr const char* kName = "f32";
  static constexpr bool kRepeatable = true;
  float* C;
  int64_t ldc, zstride;
  struct Col {};
  EL_EPI_DEFAULT_HOOKS
  __device__ Col col(int) const { return Col{}; }
  __device__ void operator()(int m, int n, float acc, int z, const Col&, Pre) {
    C[z * zstride + (int64_t)m * ldc + n] = acc;
  }
  __device__ void flush() {}
};

// Epilogue of a wave's TM x TN MFMA tiles of 32 x 32 (wave tile at rows mw,
// columns nw).  Output layout of the 32x32 MFMA (measured on gfx950):
// register r of lane l holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].  The
// per-column data of all TN columns is fetched first (columns past N read
// column N - 1 and are never stored) and waited for once, so that the
// guarded stores that follow wait for nothing (a wait inside the guarded
// blocks would also wait for the stores before it).
template <int TM, int TN, typename Epi, bool kBlockPre = false>
__device__ inline void store_tiles(Epi& epi, const gemm::f32x16 (&acc)[TM][TN], int mw, int nw, int M, int N,
                                   int lane, int z) {
  const int lr = lane & 31, hi = lane >> 5;
  decltype(epi.col(0)) cols[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) cols[j] = epi.col(min(nw + 32 * j + lr, N - 1));
  __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = nw + 32 * j + lr;
    typename Epi::Pre pre[TM][16];
    // the per-element inputs: all loads of a column before any is used
    // (addresses clamped into the operand; rows and columns past it are not
    // stored), or, kBlockPre (inputs staged in LDS), read where used
    auto fetch = [&](int i) {
#pragma unroll
      for (int r = 0; r < 16; ++r)
        pre[i][r] = epi.pre(min(mw + 32 * i + 8 * (r >> 2) + 4 * hi + (r & 3), M - 1), min(n, N - 1));
    };
    if constexpr (Epi::kHasPre && !kBlockPre) {
#pragma unroll
      for (int i = 0; i < TM; ++i) fetch(i);
      __builtin_amdgcn_s_waitcnt(0);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      epi.block_begin();
      if (n < N) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = mw + 32 * i + 8 * (r >> 2) + 4 * hi + (r & 3);
          if (m < M) {
            if constexpr (Epi::kHasPre && kBlockPre) epi(m, n, acc[i][j][r], z, cols[j], epi.pre(m, n));
            else epi(m, n, acc[i][j][r], z, cols[j], pre[i][r]);
          }
        }
      }
      epi.block_end(mw + 32 * i, nw + 32 * j, lane, M, N);
    }
  }
  epi.flush();
}

// at least two workgroups per CU (LDS), so the registers of a wave must fit
// 2 waves/SIMD
template <bool A_KC, bool B_KC, int TM, int TN, typename Epi>
__global__ void __launch_bounds__(gemm::kThreads) __attribute__((amdgpu_waves_per_eu(2))) k_mm(const uint16_t* __restrict__ A, int64_t lda,
                                                        const uint16_t* __restrict__ B, int64_t ldb, int M, int N,
                                                        int K, int k_split, int m_fast, Epi epi) {
  using namespace gemm;
  constexpr int BM = 64 * TM, BN = 64 * TN;
  extern __shared__ __align__(16) uint16_t lds_mm[];
  uint16_t* As = lds_mm;                    // [2][BM * PITCH]
  uint16_t* Bs = lds_mm + 2 * BM * PITCH;   // [2][BN * PITCH]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // Tile order, XCD-aware: workgroups are dealt round-robin to the 8 XCDs,
  // so workgroup b runs on XCD b % 8.  Each XCD gets a contiguous range of
  // the tile sequence, and the sequence walks groups of 8 M tiles, M fastest
  // within a group, so that the workgroups resident on one XCD share a few A
  // and B panels in that XCD's L2.
  int tile_m, tile_n;
  {
    const int tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
    const int T = tm * tn;
    const int b = blockIdx.x;
    // XCD x holds workgroups b = 8 i + x, i < T/8 (+1 for x < T%8); it gets
    // the contiguous range starting at x (T/8) + min(x, T%8): a bijection
    const int xcd = b & 7, loc = b >> 3;
    const int pid = xcd * (T >> 3) + min(xcd, T & 7) + loc;
    constexpr int G = 8;
    const int group = pid / (G * tn), first = group * G;
    const int gsz = min(tm - first, G);
    tile_m = first + (pid % (G * tn)) % gsz;
    tile_n = (pid % (G * tn)) / gsz;
    (void)m_fast;
  }
  const int m0 = tile_m * BM, n0 = tile_n * BN;
  const int kb = blockIdx.z * k_split;
  const int ke = min(K, kb + k_split);
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  // two register stages: tile s+2 is in flight while tile s is multiplied
  // and tile s+1 goes from registers to LDS
  TileLoader<A_KC, BM> la0, la1;
  TileLoader<B_KC, BN> lb0, lb1;
  const int nsteps = kb < ke ? (ke - kb + BK - 1) / BK : 0;
  auto kt = [&](int s) { return kb + min(s, max(nsteps - 1, 0)) * BK; };   // clamped: loads past the end repeat the last tile
  if (nsteps > 0) {
    la0.load(A, lda, M, m0, kt(0), ke, tid);
    lb0.load(B, ldb, N, n0, kt(0), ke, tid);
    la1.load(A, lda, M, m0, kt(1), ke, tid);
    lb1.load(B, ldb, N, n0, kt(1), ke, tid);
    la0.store(As, tid);
    lb0.store(Bs, tid);
  }
  __syncthreads();
  const int lr = lane & 31, lq = (lane >> 5) * 8;
  auto compute = [&](int buf) {
    const uint16_t* as = As + buf * BM * PITCH + (wm * 32 * TM + lr) * PITCH + lq;
    const uint16_t* bs = Bs + buf * BN * PITCH + (wn * 32 * TN + lr) * PITCH + lq;
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = *reinterpret_cast<const bf16x8*>(as + 32 * i * PITCH + ks);
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = *reinterpret_cast<const bf16x8*>(bs + 32 * j * PITCH + ks);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
  };
  for (int s = 0; s < nsteps; s += 2) {
    // even step: registers 0 are free (stored), registers 1 hold tile s+1
    la0.load(A, lda, M, m0, kt(s + 2), ke, tid);
    lb0.load(B, ldb, N, n0, kt(s + 2), ke, tid);
    compute(0);
    if (s + 1 < nsteps) {
      la1.store(As + BM * PITCH, tid);
      lb1.store(Bs + BN * PITCH, tid);
    }
    __syncthreads();
    if (s + 1 >= nsteps) break;
    // odd step: registers 1 are free, registers 0 hold tile s+2
    la1.load(A, lda, M, m0, kt(s + 3), ke, tid);
    lb1.load(B, ldb, N, n0, kt(s + 3), ke, tid);
    compute(1);
    if (s + 2 < nsteps) {
      la0.store(As, tid);
      lb0.store(Bs, tid);
    }
    __syncthreads();
  }
  store_tiles<TM, TN>(epi, acc, m0 + wm * 32 * TM, n0 + wn * 32 * TN, M, N, lane, blockIdx.z);
}

// Large-tile variant for k-contiguous operands with K a multiple of BK: a
// BM x BN block tile of WM x WN waves, each (BM / WM) x (BN / WN) in MFMA
// tiles of 32 x 32 (in use: 256 x 256 with 8 waves of 128 x 64), operand
// tiles moved from HBM straight into LDS by global_load_lds_dwordx4 (no
// register staging, so the accumulators of the larger wave tile fit), NS LDS
// stages of BK k (128 KB for 256 x 256 in two stages of 64), loads NS - 1
// tiles ahead, one barrier per k tile.  An epilogue with per-element inputs
// (the training targets) has them staged in LDS, the first three quarters of
// the rows fetched while the last k tile multiplies (into the stage it leaves
// free and the 32 KB beyond the stages).  A row of an operand tile is BK / 8 chunks of 16 bytes
// (8 k); chunk c of row r sits at position c ^ f(r) of the row (gemm_lds::swz),
// so the 16-byte fragment reads of consecutive rows at one chunk spread over
// all banks.  One load instruction
// of a wave fills 1 KB: lane l writes position l % (BK / 8) of row
// l / (BK / 8) of its group of rows, so it fetches the chunk that belongs
// there.  Per k16 step a wave reads 6 fragments for 8 MFMAs (the 64 x 64
// wave tile of k_mm reads 4 for 4).
namespace gemm_lds {
// LDS bytes of NS stages of BK k for a BM x BN block tile
template <int BK, int NS, int BM, int BN>
constexpr size_t smem() { return (size_t)NS * BK * (BM + BN) * 2; }
constexpr size_t kMaxLds = 160 * 1024;
// two stages and an epilogue that stages its inputs: the inputs' first rows
// are fetched into the stage the last k tile leaves free and the LDS beyond
// the stages while that tile multiplies
template <typename Epi, int NS>
constexpr bool prefetch_epi() { return Epi::kStageLds && NS == 2; }
template <typename Epi, int BK, int NS, int BM, int BN>
constexpr size_t lds_bytes() { return prefetch_epi<Epi, NS>() ? kMaxLds : smem<BK, NS, BM, BN>(); }
// chunk position of row r: conflict-free 16-byte fragment reads of 32
// consecutive rows whether a read is served 8 lanes at a time over 32 banks
// or 16 lanes at a time over 64 banks (rows r and r + 8 must differ too)
template <int BK>
__device__ inline int swz(int r) {
  return BK == 64 ? ((r & 7) ^ ((r >> 3) & 1)) : (((r >> 1) & 3) ^ ((r >> 3) & 1));
}
// s_waitcnt immediate that waits until at most n vector memory operations
// are outstanding (expcnt and lgkmcnt left alone)
constexpr int vmcnt_imm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14); }
}  // namespace gemm_lds

typedef __attribute__((address_space(3))) uint16_t lds_u16;

// one R x BK operand tile (rows r0.., k0..k0+BK-1) into LDS S; rows past the
// operand are clamped to its last row (their products are never stored)
template <int BK, int R, int NW>
__device__ inline void lds_tile_load(const uint16_t* __restrict__ G, int64_t ld, int rows, int r0, int k0,
                                     lds_u16* S, int wave, int lane) {
  constexpr int CPR = BK / 8;                        // 16-byte chunks per row
  constexpr int RPI = 64 / CPR;                      // rows per load instruction
  constexpr int NI = R / RPI / NW;                   // instructions per wave
  static_assert(NI * NW * RPI == R, "whole row groups per wave");
  const int sub = lane / CPR;
#pragma unroll
  for (int t = 0; t < NI; ++t) {
    const int q = wave * NI + t;                     // row group of the tile
    const int c = (lane % CPR) ^ gemm_lds::swz<BK>(q * RPI + sub);
    const int r = min(r0 + q * RPI + sub, rows - 1);
    const uint16_t* src = G + (int64_t)r * ld + k0 + c * 8;
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                     reinterpret_cast<__attribute__((address_space(3))) void*>(S + q * 512), 16, 0,
                                     0);
  }
}

template <int BK, int NS, int BM, int BN, int WM, int WN, typename Epi>
__global__ void __launch_bounds__(64 * WM * WN) k_mm_lds(const uint16_t* __restrict__ A, int64_t lda,
                                                          const uint16_t* __restrict__ B, int64_t ldb, int M, int N,
                                                          int K, int k_split, Epi epi) {
  using namespace gemm;
  constexpr int NW = WM * WN;                        // waves
  constexpr int TM = BM / (32 * WM), TN = BN / (32 * WN);   // MFMA tiles per wave
  static_assert(TM * 32 * WM == BM && TN * 32 * WN == BN, "wave tiles");
  static_assert(gemm_lds::lds_bytes<Epi, BK, NS, BM, BN>() <= gemm_lds::kMaxLds, "LDS stages");
  constexpr int kTileA = BM * BK, kTileB = BN * BK;   // bf16 per operand tile
  constexpr int LW = (BM + BN) * BK / 8 / 64 / NW;   // load instructions per wave per k tile
  static_assert(LW * 64 * NW * 8 == (BM + BN) * BK, "whole load instructions per wave");
  extern __shared__ __align__(16) uint16_t lds_mm_big[];
  lds_u16* L = (lds_u16*)lds_mm_big;   // the dynamic LDS array, as an LDS-space pointer
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  int tile_m, tile_n;
  {
    // the XCD-aware tile order of k_mm
    const int tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
    const int T = tm * tn;
    const int b = blockIdx.x;
    const int xcd = b & 7, loc = b >> 3;
    const int pid = xcd * (T >> 3) + min(xcd, T & 7) + loc;
    constexpr int G = 8;
    const int group = pid / (G * tn), first = group * G;
    const int gsz = min(tm - first, G);
    tile_m = first + (pid % (G * tn)) % gsz;
    tile_n = (pid % (G * tn)) / gsz;
  }
  const int m0 = tile_m * BM, n0 = tile_n * BN;
  const int kb = blockIdx.z * k_split;
  const int ke = min(K, kb + k_split);
  const int nsteps = kb < ke ? (ke - kb) / BK : 0;   // the host checks that 64 divides both
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  auto stage_a = [&](int st) { return L + st * (kTileA + kTileB); };
  auto stage_b = [&](int st) { return L + st * (kTileA + kTileB) + kTileA; };
  // k tile t goes to stage (t + sh) % NS; with the epilogue prefetch the last
  // tile lands in stage 0 and leaves stage 1 free, which is contiguous with
  // the LDS beyond the stages
  constexpr bool kPre = gemm_lds::prefetch_epi<Epi, NS>();
  const int sh = kPre ? nsteps + 1 : 0;
  auto load_tile = [&](int t) {
    const int k = kb + t * BK;
    lds_tile_load<BK, BM, NW>(A, lda, M, m0, k, stage_a((t + sh) % NS), wave, lane);
    lds_tile_load<BK, BN, NW>(B, ldb, N, n0, k, stage_b((t + sh) % NS), wave, lane);
  };
  // rows [r0, r1) of the block tile's epilogue inputs (ld = N) into LDS at D
  // (pitch BN): 16-byte chunks, chunk i of the range at i * 16 bytes, one
  // instruction per 64 chunks; rows past M and chunks past N are clamped into
  // the operand (never used)
  auto stage_inputs = [&](int r0, int r1, lds_u16* D) {
    if constexpr (Epi::kStageLds) {
      static_assert((BN / 8) % 64 == 0 || 64 % (BN / 8) == 0, "whole rows per instruction group");
      const uint16_t* Y = epi.y;
      const int nq = (r1 - r0) * (BN / 8) / 64;
      for (int q = wave; q < nq; q += NW) {
        const int ci = q * 64 + lane;
        const int r = min(m0 + r0 + ci / (BN / 8), M - 1);
        const int c = min(n0 + 8 * (ci % (BN / 8)), N - 8);
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(Y + (int64_t)r * N + c),
                                         reinterpret_cast<__attribute__((address_space(3))) void*>(D + q * 512), 16,
                                         0, 0);
      }
    }
  };
  constexpr int kStageElems = BK * (BM + BN);
  constexpr int kPreRows = kPre ? (int)((gemm_lds::kMaxLds / 2 - kStageElems) / BN) : 0;   // rows fetched early
  static_assert(!kPre || (kPreRows < BM && (BM - kPreRows) * BN <= kStageElems && kPreRows % 8 == 0),
                "epilogue prefetch layout");
#pragma unroll
  for (int t = 0; t < NS - 1; ++t)
    if (t < nsteps) load_tile(t);
  const int lr = lane & 31, hi = lane >> 5;
  const int sw = gemm_lds::swz<BK>(lr);
  for (int s = 0; s < nsteps; ++s) {
    // tile s has landed (the loads of the tiles after it may still be in
    // flight) for every wave, and every wave is done with tile s - 1
    const int pending = min(NS - 2, nsteps - 1 - s);
    if constexpr (NS > 2) {
      if (pending >= 2) __builtin_amdgcn_s_waitcnt(gemm_lds::vmcnt_imm(2 * LW));
      else if (pending == 1) __builtin_amdgcn_s_waitcnt(gemm_lds::vmcnt_imm(LW));
      else __builtin_amdgcn_s_waitcnt(gemm_lds::vmcnt_imm(0));
      static_assert(NS <= 4, "wait counts for more stages");
    } else {
      (void)pending;
      __builtin_amdgcn_s_waitcnt(gemm_lds::vmcnt_imm(0));
    }
    // a bare barrier: the wait above covers the LDS writes of this wave's
    // loads, and every LDS read of the previous tile has returned (the MFMAs
    // consumed it); __syncthreads would add a fence that waits for all loads
    // in flight, the later tiles' included
    asm volatile("s_barrier" ::: "memory");
    if (s + NS - 1 < nsteps) load_tile(s + NS - 1);
    else if (kPre && s == nsteps - 1) stage_inputs(0, kPreRows, L + kStageElems);
    const lds_u16* as = stage_a((s + sh) % NS) + (wm * 32 * TM + lr) * BK;
    const lds_u16* bs = stage_b((s + sh) % NS) + (wn * 32 * TN + lr) * BK;
    // fragments of the next k16 step are read while this one multiplies
    bf16x8 af[2][TM], bfr[2][TN];
    auto frags = [&](int ks, int b) {
      const int off = (((ks >> 3) + hi) ^ sw) << 3;
#pragma unroll
      for (int i = 0; i < TM; ++i)
        af[b][i] = *reinterpret_cast<const __attribute__((address_space(3))) bf16x8*>(as + 32 * i * BK + off);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bfr[b][j] = *reinterpret_cast<const __attribute__((address_space(3))) bf16x8*>(bs + 32 * j * BK + off);
    };
    frags(0, 0);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const int b = (ks >> 4) & 1;
      if (ks + 16 < BK) frags(ks + 16, b ^ 1);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[b][i], bfr[b][j], acc[i][j], 0, 0, 0);
    }
    // issue order of the k tile (left to itself the scheduler groups each
    // step's reads and waits for all of them before the MFMAs that need the
    // first): the first step's fragment reads, then each step's MFMAs with
    // the next step's reads placed between them, one wait per step
    static_assert(TM * TN >= TM + TN, "a read between MFMAs");
    __builtin_amdgcn_sched_group_barrier(0x100, TM + TN, 0);   // 0x100: LDS reads
#pragma unroll
    for (int ks = 0; ks < BK - 16; ks += 16) {
#pragma unroll
      for (int q = 0; q < TM + TN; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);     // 0x008: MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, TM * TN - TM - TN, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, TM * TN, 0);
  }
  if constexpr (Epi::kStageLds) {
    // the block tile's per-element epilogue inputs in LDS: with the prefetch,
    // rows below kPreRows are already on their way (into stage 1 and the LDS
    // beyond the stages) and the rest go to stage 0 once every wave is past
    // its last MFMA reads; without it (or without k tiles) all rows go to the
    // stages from 0
    static_assert(BM * BN * 2 <= gemm_lds::lds_bytes<Epi, BK, NS, BM, BN>(), "epilogue tile");
    static_assert((BM * BN / 8) % 64 == 0, "whole instructions");
    __syncthreads();
    if (kPre && nsteps > 0) {
      stage_inputs(kPreRows, BM, L);
      epi.ys = L + kStageElems;
      epi.ys2 = L;
      epi.ysplit = kPreRows;
    } else {
      stage_inputs(0, BM, L);
      epi.ys = L;
      epi.ys2 = L;
      epi.ysplit = BM;
    }
    __builtin_amdgcn_s_waitcnt(gemm_lds::vmcnt_imm(0));
    __syncthreads();
    epi.ypitch = BN;
    epi.ym0 = m0;
    epi.yn0 = n0;
    store_tiles<TM, TN, Epi, true>(epi, acc, m0 + wm * 32 * TM, n0 + wn * 32 * TN, M, N, lane, blockIdx.z);
  } else {
    store_tiles<TM, TN>(epi, acc, m0 + wm * 32 * TM, n0 + wn * 32 * TN, M, N, lane, blockIdx.z);
  }
}

// whether k_mm_lds can take a GEMM (k-contiguous operands, 16-byte aligned
// rows, K and the split-K chunk multiples of 64, the k tile of every
// direct-to-LDS variant)
inline bool mm_lds_ok(const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, int64_t K, int splits) {
  int64_t ks = (K + splits - 1) / splits;
  ks = (ks + gemm::BK - 1) / gemm::BK * gemm::BK;
  return K % 64 == 0 && ks % 64 == 0 && lda % 8 == 0 && ldb % 8 == 0 &&
         reinterpret_cast<uintptr_t>(A) % 16 == 0 && reinterpret_cast<uintptr_t>(B) % 16 == 0;
}

template <int BK, int NS, int BM, int BN, int WM, int WN, typename Epi>
el_status mm_lds(el_ctx* ctx, const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, int64_t M, int64_t N,
                 int64_t K, int splits, Epi epi) {
  static_assert(BK == 64, "mm_lds_ok checks k tiles of 64");
  if (!mm_lds_ok(A, lda, B, ldb, K, splits) || !epi_lds_ok(epi, N))
    return set_error(ctx, EL_ERR_ARG, "internal GEMM: the direct-to-LDS tile needs K % 64 == 0 and aligned rows");
  constexpr size_t smem = gemm_lds::lds_bytes<Epi, BK, NS, BM, BN>();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mm_lds<BK, NS, BM, BN, WM, WN, Epi>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return hip_check(ctx, e, "hipFuncSetAttribute(k_mm_lds)");
    attr_set = true;
  }
  int64_t ks = (K + splits - 1) / splits;
  ks = (ks + gemm::BK - 1) / gemm::BK * gemm::BK;
  const int nz = (int)((K + ks - 1) / ks);
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (tiles > INT_MAX / 2) return set_error(ctx, EL_ERR_ARG, "internal GEMM: too many tiles");
  hipLaunchKernelGGL((k_mm_lds<BK, NS, BM, BN, WM, WN, Epi>), dim3((unsigned)tiles, 1, (unsigned)nz),
                     dim3(64 * WM * WN), smem, ctx->stream, A, lda, B, ldb, (int)M, (int)N, (int)K, (int)ks, epi);
  return hip_check(ctx, hipGetLastError(), "launch k_mm_lds");
}

template <bool A_KC, bool B_KC, int TM, int TN, typename Epi>
el_status mm_t(el_ctx* ctx, const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, int64_t M, int64_t N,
               int64_t K, int splits, Epi epi, bool m_fast) {
  constexpr int BM = 64 * TM, BN = 64 * TN;
  constexpr size_t smem = 2 * (size_t)(BM + BN) * gemm::PITCH * sizeof(uint16_t);
  // the tile loaders move whole 16-byte segments along the contiguous
  // dimension of each operand
  const int64_t a_cont = A_KC ? K : M, b_cont = B_KC ? K : N;
  if (a_cont % 8 || b_cont % 8 || lda % 8 || ldb % 8)
    return set_error(ctx, EL_ERR_ARG, "internal GEMM: contiguous dimensions must be multiples of 8");
  static bool attr_set = false;   // per instantiation; the attribute is per function
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mm<A_KC, B_KC, TM, TN, Epi>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return hip_check(ctx, e, "hipFuncSetAttribute(k_mm)");
    attr_set = true;
  }
  int64_t ks = (K + splits - 1) / splits;
  ks = (ks + gemm::BK - 1) / gemm::BK * gemm::BK;
  const int nz = (int)((K + ks - 1) / ks);
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (tiles > INT_MAX / 2) return set_error(ctx, EL_ERR_ARG, "internal GEMM: too many tiles");
  dim3 grid((unsigned)tiles, 1, (unsigned)nz);
  hipLaunchKernelGGL((k_mm<A_KC, B_KC, TM, TN, Epi>), grid, dim3(gemm::kThreads), smem, ctx->stream, A, lda, B, ldb,
                     (int)M, (int)N, (int)K, (int)ks, (int)m_fast, epi);
  return hip_check(ctx, hipGetLastError(), "launch k_mm");
}

// ---- GEMM autotuner --------------------------------------------------------
// The block tile is chosen per GEMM shape and device architecture, on first
// use, by timing the candidates below on the call's own operands (outputs are
// overwritten by the chosen run); epilogues whose runs are not repeatable use
// the default.  Choices are kept per process and can be saved to and loaded
// from a text file (el_tuning_save / el_tuning_load), which then replaces the
// timing.
struct TileVariant {
  int tm, tn;
  bool lds;   // k_mm_lds (k-contiguous operands only)
};
// the tile's name in reports and cache files
inline std::string tile_name(const TileVariant& v) {
  std::ostringstream os;
  os << 64 * v.tm << "x" << 64 * v.tn << (v.lds ? " direct-to-LDS" : "");
  return os.str();
}
constexpr TileVariant kVariants[] = {{2, 2, false}, {1, 2, false}, {2, 1, false}, {4, 4, true}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

std::atomic<int> g_force_tile{-1};   // >= 0: this variant wherever it applies (el_gemm_tile)

// an epilogue that stages per-element inputs (ld = N) in LDS needs 16-byte
// aligned rows of them
template <typename Epi>
bool epi_lds_ok(const Epi& epi, int64_t N) {
  if constexpr (Epi::kStageLds) {
    return N % 8 == 0 && reinterpret_cast<uintptr_t>(epi.y) % 16 == 0;
  } else {
    (void)epi;
    (void)N;
    return true;
  }
}

template <bool A_KC, bool B_KC, typename Epi>
bool variant_applies(int v, const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, int64_t N, int64_t K,
                     int splits, const Epi& epi) {
  return !kVariants[v].lds || (A_KC && B_KC && mm_lds_ok(A, lda, B, ldb, K, splits) && epi_lds_ok(epi, N));
}

template <bool A_KC, bool B_KC, typename Epi>
el_status mm_variant(el_ctx* ctx, int v, const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, int64_t M,
                     int64_t N, int64_t K, int splits, const Epi& epi, bool m_fast) {
  switch (v) {
    case 1: return mm_t<A_KC, B_KC, 1, 2, Epi>(ctx, A, lda, B, ldb, M, N, K, splits, epi, m_fast);
    case 2: return mm_t<A_KC, B_KC, 2, 1, Epi>(ctx, A, lda, B, ldb, M, N, K, splits, epi, m_fast);
    case 3:
      // 256 x 256, 8 waves of 128 x 64, k tiles of 64 in two stages.  Slower
      // on every network GEMM of the 128^2, p = 6 workload: k tiles of 32 in
      // four or five stages, 4 waves of 128 x 128, 192 x 192 in three stages
      // (6 waves: two SIMDs carry two waves, two carry one), 256 x 128 and
      // 128 x 256 in three stages (4 waves, one per SIMD)
      if constexpr (A_KC && B_KC) {
        return mm_lds<64, 2, 256, 256, 2, 4, Epi>(ctx, A, lda, B, ldb, M, N, K, splits, epi);
      } else {
        return set_error(ctx, EL_ERR_ARG, "internal GEMM: the direct-to-LDS tile needs k-contiguous operands");
      }
    default: return mm_t<A_KC, B_KC, 2, 2, Epi>(ctx, A, lda, B, ldb, M, N, K, splits, epi, m_fast);
  }
}

template <bool A_KC, bool B_KC, typename Epi>
el_status mm(el_ctx* ctx, const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, int64_t M, int64_t N,
             int64_t K, int splits, Epi epi, bool m_fast = false) {
  if (M <= 0 || N <= 0) return EL_OK;
  const int forced = g_force_tile.load();
  if (forced >= 0 && variant_applies<A_KC, B_KC>(forced, A, lda, B, ldb, N, K, splits, epi))
    return mm_variant<A_KC, B_KC, Epi>(ctx, forced, A, lda, B, ldb, M, N, K, splits, epi, m_fast);
  if constexpr (!Epi::kRepeatable) {
    return mm_variant<A_KC, B_KC, Epi>(ctx, 0, A, lda, B, ldb, M, N, K, splits, epi, m_fast);
  } else {
    std::ostringstream ks;
    ks << ctx->arch << " gemm " << (A_KC ? "A" : "At") << (B_KC ? "B" : "Bt") << ' ' << Epi::kName << " M=" << M << " N=" << N
       << " K=" << K << " splits=" << splits;
    const std::string key = ks.str();
    int choice = -1;
    if (!tune_find(key, &choice) || choice < 0 || choice >= kNumVariants) {
      std::vector<float> ms(kNumVariants, 0.f);
      hipEvent_t e0, e1;
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return hip_check(ctx, hipGetLastError(), "autotune events");
      int best = 0;
      for (int v = 0; v < kNumVariants; ++v) {
        if (!variant_applies<A_KC, B_KC>(v, A, lda, B, ldb, N, K, splits, epi)) {
          ms[v] = INFINITY;   // not a candidate for this GEMM
          continue;
        }
        el_status st = mm_variant<A_KC, B_KC, Epi>(ctx, v, A, lda, B, ldb, M, N, K, splits, epi, m_fast);   // warm-up
        if (st) return st;
        hipEventRecord(e0, ctx->stream);
        st = mm_variant<A_KC, B_KC, Epi>(ctx, v, A, lda, B, ldb, M, N, K, splits, epi, m_fast);
        if (st) return st;
        hipEventRecord(e1, ctx->stream);
        hipError_t he = hipEventSynchronize(e1);
        if (he != hipSuccess) return hip_check(ctx, he, "autotune");
        hipEventElapsedTime(&ms[v], e0, e1);
        if (ms[v] < ms[best]) best = v;
      }
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      choice = best;
      tune_store(key, choice, ms);
    }
    return mm_variant<A_KC, B_KC, Epi>(ctx, choice, A, lda, B, ldb, M, N, K, splits, epi, m_fast);
  }
}

// Column sums of a float matrix X [B][N] over the row range of chunk
// blockIdx.y (rows rows each): out[blockIdx.y][n].  256 threads = 4 waves of
// 64 consecutive columns (each load instruction of a wave reads 256
// contiguous bytes of one row); wave w adds rows w, w + 4, ... of the chunk
// in order and the four wave sums are added in wave order (deterministic).
__global__ void __launch_bounds__(256) k_colsum(const float* __restrict__ X, int64_t B, int64_t N, int64_t rows,
                                                 float* __restrict__ out) {
  __shared__ float part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * 64 + lane;
  const int64_t r0 = (int64_t)blockIdx.y * rows, r1 = min(B, r0 + rows);
  float acc = 0.f;
  if (n < N) {
#pragma unroll 8
    for (int64_t b = r0 + w; b < r1; b += 4) acc += X[b * N + n];
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && n < N) out[(int64_t)blockIdx.y * N + n] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// out[n] = sum_b X[b][n] for X [B][N] float: row chunks of at most rows_max
// rows summed into tmp [ceil(B / rows_max)][N] and the chunk sums reduced in
// chunk order (one launch when B <= rows_max; tmp may be null then)
el_status colsum(el_ctx* ctx, const float* X, int64_t B, int64_t N, int64_t rows_max, float* tmp, float* out) {
  const unsigned cb = (unsigned)((N + 63) / 64);
  if (B <= rows_max) {
    hipLaunchKernelGGL(k_colsum, dim3(cb, 1), dim3(256), 0, ctx->stream, X, B, N, B, out);
  } else {
    const int64_t chunks = (B + rows_max - 1) / rows_max;
    if (!tmp || chunks > 65535) return set_error(ctx, EL_ERR_ARG, "internal column sum: bad chunking");
    hipLaunchKernelGGL(k_colsum, dim3(cb, (unsigned)chunks), dim3(256), 0, ctx->stream, X, B, N, rows_max, tmp);
    hipLaunchKernelGGL(k_colsum, dim3(cb, 1), dim3(256), 0, ctx->stream, tmp, chunks, N, chunks, out);
  }
  return hip_check(ctx, hipGetLastError(), "launch k_colsum");
}

// dZ = (sum_s P[s]) * act'(Z); writes FP32 and (dZ16 not null) bfloat16
__global__ void k_reduce_dact(const float* __restrict__ P, int S, int64_t count, const float* __restrict__ Z, int act,
                              float* __restrict__ dZ, uint16_t* __restrict__ dZ16) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float acc = 0.f;
  for (int s = 0; s < S; ++s) acc += P[s * count + i];
  float g = acc * act_df(act, Z[i]);
  dZ[i] = g;
  if (dZ16) dZ16[i] = f2bf(g);
}

__global__ void k_reduce_sum(const float* __restrict__ P, int S, int64_t count, float* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float acc = 0.f;
  for (int s = 0; s < S; ++s) acc += P[s * count + i];
  out[i] = acc;
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ wbf, int64_t n, float lr, float gscale,
                       float bc1, float bc2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float gi = g[i] * gscale;
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float t = th[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  th[i] = t;
  wbf[i] = f2bf(t);
}

// out[b] = sum of p[b * chunk .. min(n, (b + 1) * chunk)) in a fixed order
// (workgroups of 256 threads; one workgroup per output)
__global__ void k_sum_chunks(const float* __restrict__ p, int64_t n, int64_t chunk, float* __restrict__ out) {
  __shared__ double part[256];
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = min(n, b0 + chunk);
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) acc += p[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = (float)part[0];
}

// dst [cols][rows] = src [rows][cols]^T for 16-bit values, rows and cols
// multiples of 64: 64 x 64 tiles through LDS, 16-byte loads and stores
// (256 threads; each moves two 16-byte row chunks in and two column chunks
// out)
__global__ void __launch_bounds__(256) k_transpose16(const uint16_t* __restrict__ src, int64_t rows, int64_t cols,
                                                     uint16_t* __restrict__ dst) {
  __shared__ uint16_t t[64][64 + 2];
  const int64_t tiles_c = cols / 64;
  const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * 64, c0 = (int64_t)(blockIdx.x % tiles_c) * 64;
  const int tid = threadIdx.x;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q = tid + 256 * h, r = q >> 3, ch = (q & 7) * 8;
    const uint4 v = *reinterpret_cast<const uint4*>(src + (r0 + r) * cols + c0 + ch);
    const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
    for (int k = 0; k < 8; ++k) t[r][ch + k] = e[k];
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int q = tid + 256 * h, c = q >> 3, rh = (q & 7) * 8;
    uint4 v;
    uint16_t* e = reinterpret_cast<uint16_t*>(&v);
#pragma unroll
    for (int k = 0; k < 8; ++k) e[k] = t[rh + k][c];
    *reinterpret_cast<uint4*>(dst + (c0 + c) * rows + r0 + rh) = v;
  }
}

__global__ void k_loss_out(const float* acc, float scale, float* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = *acc * scale;
}

// feature statistics: one block per feature, FP64 accumulation over N samples
__global__ void k_feat_stats(const float* __restrict__ x, int64_t N, int n_in, float* mean, float* stdv) {
  const int f = blockIdx.x;
  double s = 0.0, s2 = 0.0;
  for (int64_t b = threadIdx.x; b < N; b += blockDim.x) {
    double h = x[b * n_in];
    double v = f == 0 ? 0.0 : x[b * n_in + f];
    double z = feature_value(f, h, v);
    s += z;
    s2 += z * z;
  }
  __shared__ double r1[256], r2[256];
  r1[threadIdx.x] = s;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) { r1[threadIdx.x] += r1[threadIdx.x + o]; r2[threadIdx.x] += r2[threadIdx.x + o]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double mu = r1[0] / N;
    double var = fmax(r2[0] / N - mu * mu, 0.0);
    mean[f] = (float)mu;
    stdv[f] = (float)fmax(sqrt(var), 1e-6);
  }
}

// min / max of raw h (f == 0), kappa (1..nn), sigma (nn+1..2nn): block 0..2
__global__ void k_box(const float* __restrict__ x, int64_t N, int n_in, double* box) {
  const int which = blockIdx.x;
  const int nn = (n_in - 1) / 2;
  const int f0 = which == 0 ? 0 : (which == 1 ? 1 : 1 + nn);
  const int f1 = which == 0 ? 1 : (which == 1 ? 1 + nn : n_in);
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t i = threadIdx.x; i < N * (f1 - f0); i += blockDim.x) {
    int64_t b = i / (f1 - f0);
    int f = f0 + (int)(i % (f1 - f0));
    double v = x[b * n_in + f];
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  __shared__ double rl[256], rh[256];
  rl[threadIdx.x] = lo;
  rh[threadIdx.x] = hi;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      rl[threadIdx.x] = fmin(rl[threadIdx.x], rl[threadIdx.x + o]);
      rh[threadIdx.x] = fmax(rh[threadIdx.x], rh[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { box[2 * which] = rl[0]; box[2 * which + 1] = rh[0]; }
}

// per-output mean / std of bfloat16 targets (FP64 accumulation)
__global__ void k_y_stats(const uint16_t* __restrict__ y, int64_t N, int64_t n_out, float* mean, float* stdv) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_out) return;
  double s = 0.0, s2 = 0.0;
  for (int64_t b = 0; b < N; ++b) {
    double v = bf2f(y[b * n_out + c]);
    s += v;
    s2 += v * v;
  }
  double mu = s / N;
  double var = fmax(s2 / N - mu * mu, 0.0);
  mean[c] = (float)mu;
  stdv[c] = (float)fmax(sqrt(var), 1e-6 * fmax(fabs(mu), 1e-30) + 1e-12);
}

__global__ void k_fill_int32(int* p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_count_out(const uint8_t* in_range, int64_t E, int32_t* idx, int* count) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  if (!in_range[e]) {
    int pos = atomicAdd(count, 1);
    idx[pos] = (int32_t)e;
  }
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

int64_t layer_count(const el_net* net) { return net->desc.depth + 1; }

void layout(el_net* net) {
  const el_net_desc& d = net->desc;
  net->k0 = (d.n_in + 31) / 32 * 32;
  const int L = d.depth + 1;
  net->w_off.resize(L); net->b_off.resize(L); net->in_dim.resize(L); net->out_dim.resize(L);
  int64_t off = 0;
  for (int l = 0; l < L; ++l) {
    net->in_dim[l] = l == 0 ? net->k0 : d.width;
    net->out_dim[l] = l == d.depth ? d.n_out : d.width;
    net->w_off[l] = off;
    off += net->in_dim[l] * net->out_dim[l];
    net->b_off[l] = off;
    off += net->out_dim[l];
    off = (off + 63) / 64 * 64;   // keep every W_l 128-byte aligned
  }
  net->n_params = off;
}

el_status alloc_net(el_ctx* ctx, el_net* net) {
  const int64_t P = net->n_params;
  const int64_t nin = net->desc.n_in, nout = net->desc.n_out;
  void* p;
  size_t bytes = (size_t)P * (4 * 4 + 2) + (size_t)(2 * nin + 2 * nout) * 4 + 1024;
  el_status st = hip_check(ctx, hipMalloc(&p, bytes), "hipMalloc(network)");
  if (st) return st;
  char* c = reinterpret_cast<char*>(p);
  auto take = [&](size_t b) { char* r = c; c += (b + 255) / 256 * 256; return r; };
  net->theta = reinterpret_cast<float*>(take(P * 4));
  net->grad = reinterpret_cast<float*>(take(P * 4));
  net->adam_m = reinterpret_cast<float*>(take(P * 4));
  net->adam_v = reinterpret_cast<float*>(take(P * 4));
  net->wbf = reinterpret_cast<uint16_t*>(take(P * 2));
  net->feat_mean = reinterpret_cast<float*>(take(nin * 4));
  net->feat_std = reinterpret_cast<float*>(take(nin * 4));
  net->y_mean = reinterpret_cast<float*>(take(nout * 4));
  net->y_std = reinterpret_cast<float*>(take(nout * 4));
  return EL_OK;
}

bool desc_ok(const el_net_desc& d) {
  return d.n_in >= 3 && d.n_in % 2 == 1 && d.width >= 16 && d.width % 8 == 0 && d.depth >= 1 && d.depth <= 16 &&
         d.n_out >= 1 && d.n_out % 8 == 0 && (d.act == EL_ACT_GELU || d.act == EL_ACT_ELU || d.act == EL_ACT_LINEAR);
}

// scratch layout for a batch of B rows
struct Scratch {
  uint16_t* X0;      // [B][k0]
  float* Z;          // [depth][B][width]
  uint16_t* H;       // [depth][B][width]
  uint16_t* dY;      // [B][n_out] (training only)
  float* part;       // split-K partials
  float* dZ;         // [B][width]
  uint16_t* dZ16;    // [B][width]
  float* loss;       // [1]
  float* colp;       // [ceil(B/32)][n_out] per-block sums of the output-layer signs (training only)
  uint16_t* dYT;     // [n_out][B] (training with 64 | B, n_out, width: the transposed output-layer GEMMs)
  uint16_t* HT;      // [width][B] last hidden layer, transposed
  uint16_t* WT;      // [width][n_out] output-layer weights, transposed
  float* lossp;      // [ceil(B/32)][ceil(n_out/32)] per-block sums of |d| (training only)
  float* cst;        // [ceil(B/128)][width] row-chunk sums of the hidden bias gradients (training only)
  int64_t part_elems;
};

constexpr int kSplitOut = 32;   // split-K of dY * W_out (K = n_out)
constexpr int64_t kColsumRows = 128;   // rows per chunk of the column sums
constexpr int kLossChunks = 256;   // first-level workgroups of the loss reduction

// The output layer's dW (dY^T H) and dX (dY W) products take the
// direct-to-LDS tile through transposed copies of dY, H and W when every
// dimension is a multiple of 64; otherwise the register-staged tile
// transposes on the way into LDS.
inline bool transposed_ok(int64_t B, int64_t nout, int64_t W) { return B % 64 == 0 && nout % 64 == 0 && W % 64 == 0; }
constexpr int kSplitW = 8;      // split-K of the hidden dW GEMMs (K = batch)

el_status get_scratch(el_ctx* ctx, el_net* net, int64_t B, bool train, Scratch& s) {
  const int64_t W = net->desc.width, D = net->desc.depth, nout = net->desc.n_out;
  int64_t part = std::max<int64_t>((int64_t)kSplitOut * B * W, (int64_t)kSplitW * W * std::max<int64_t>(W, net->k0));
  size_t need = 0;
  auto add = [&](size_t b) { size_t r = need; need += (b + 255) / 256 * 256; return r; };
  size_t oX0 = add((size_t)B * net->k0 * 2), oZ = add((size_t)D * B * W * 4), oH = add((size_t)D * B * W * 2);
  size_t odY = train ? add((size_t)B * nout * 2) : 0;
  size_t opart = train ? add((size_t)part * 4) : 0;
  size_t odZ = train ? add((size_t)B * W * 4) : 0, odZ16 = train ? add((size_t)B * W * 2) : 0;
  size_t oloss = add(256);
  const int64_t rb = (B + 31) / 32;
  size_t ocolp = train ? add((size_t)rb * nout * 4) : 0;
  size_t olossp = train ? add(((size_t)rb * ((nout + 31) / 32) + kLossChunks) * 4) : 0;
  size_t ocst = train ? add((size_t)((B + kColsumRows - 1) / kColsumRows) * W * 4) : 0;
  const bool tr = train && transposed_ok(B, nout, W);
  size_t odYT = tr ? add((size_t)nout * B * 2) : 0, oHT = tr ? add((size_t)W * B * 2) : 0;
  size_t oWT = tr ? add((size_t)W * nout * 2) : 0;
  if (net->scratch.bytes < need) {
    if (net->scratch.ptr) {
      hipStreamSynchronize(ctx->stream);
      hipFree(net->scratch.ptr);
      net->scratch.ptr = nullptr;
      net->scratch.bytes = 0;
    }
    el_status st = hip_check(ctx, hipMalloc(&net->scratch.ptr, need), "hipMalloc(network scratch)");
    if (st) return st;
    net->scratch.bytes = need;
  }
  char* b = reinterpret_cast<char*>(net->scratch.ptr);
  s.X0 = reinterpret_cast<uint16_t*>(b + oX0);
  s.Z = reinterpret_cast<float*>(b + oZ);
  s.H = reinterpret_cast<uint16_t*>(b + oH);
  s.dY = train ? reinterpret_cast<uint16_t*>(b + odY) : nullptr;
  s.part = train ? reinterpret_cast<float*>(b + opart) : nullptr;
  s.dZ = train ? reinterpret_cast<float*>(b + odZ) : nullptr;
  s.dZ16 = train ? reinterpret_cast<uint16_t*>(b + odZ16) : nullptr;
  s.loss = reinterpret_cast<float*>(b + oloss);
  s.colp = train ? reinterpret_cast<float*>(b + ocolp) : nullptr;
  s.lossp = train ? reinterpret_cast<float*>(b + olossp) : nullptr;
  s.cst = train ? reinterpret_cast<float*>(b + ocst) : nullptr;
  s.dYT = tr ? reinterpret_cast<uint16_t*>(b + odYT) : nullptr;
  s.HT = tr ? reinterpret_cast<uint16_t*>(b + oHT) : nullptr;
  s.WT = tr ? reinterpret_cast<uint16_t*>(b + oWT) : nullptr;
  s.part_elems = part;
  return EL_OK;
}

Box make_box(const el_net* net) {
  Box b;
  for (int i = 0; i < 6; ++i) b.v[i] = net->box[i];
  return b;
}

// Block tile of a k-contiguous GEMM without the autotuner (no timing, no
// host-side state): the 256 x 256 direct-to-LDS tile where it applies, else
// 128 x 128.
inline int fixed_variant(const uint16_t* A, int64_t lda, const uint16_t* B, int64_t ldb, int64_t K) {
  return mm_lds_ok(A, lda, B, ldb, K, 1) ? 3 : 0;
}

// hidden layers: X0 -> H[depth-1]; Z saved when save_z; tiles autotuned, or
// fixed by fixed_variant() when no_tune
el_status forward_hidden(el_ctx* ctx, el_net* net, int64_t B, const Scratch& s, bool save_z, bool no_tune = false) {
  const int64_t W = net->desc.width;
  for (int l = 0; l < net->desc.depth; ++l) {
    const uint16_t* X = l == 0 ? s.X0 : s.H + (size_t)(l - 1) * B * W;
    const int64_t in = net->in_dim[l];
    const uint16_t* Wl = net->wbf + net->w_off[l];
    EpiHidden epi{net->theta + net->b_off[l], save_z ? s.Z + (size_t)l * B * W : nullptr, s.H + (size_t)l * B * W, W,
                  net->desc.act};
    el_status st = no_tune ? mm_variant<true, true>(ctx, fixed_variant(X, in, Wl, in, in), X, in, Wl, in, B, W, in, 1,
                                                    epi, false)
                           : mm<true, true>(ctx, X, in, Wl, in, B, W, in, 1, epi);
    if (st) return st;
  }
  return EL_OK;
}

// ---- FP32 network path ----------------------------------------------------------
// The same network, loss and optimizer with FP32 operands everywhere: the
// FP32 master weights feed the products directly, the features, hidden
// activations, sign matrix and backpropagated gradients stay FP32, and the
// targets are FP32.  For measuring what the bfloat16 operands of the
// matrix-core path cost in accuracy (Sec. 3.1 training); not a hot path.

// C[z] = sum over k in chunk z of A(i, k) B(k, j), with A(i, k) = A[i a_i +
// k a_k] and B(k, j) = B[k b_k + j b_j] (any transposition through the
// strides), C[z][i][j] at C + z zstride + i ldc + j.  64 x 64 block tiles of
// 256 threads with 4 x 4 outputs each, k tiles of 16 through LDS, FMAs in k
// order within the chunk.
__global__ void __launch_bounds__(256) k_sgemm(const float* __restrict__ A, int64_t a_i, int64_t a_k,
                                               const float* __restrict__ Bm, int64_t b_k, int64_t b_j,
                                               float* __restrict__ C, int64_t ldc, int64_t zstride, int64_t M,
                                               int64_t N, int64_t K, int64_t kchunk) {
  __shared__ float As[16][68];
  __shared__ float Bs[16][68];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int ti = tid >> 4, tj = tid & 15;
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.f;
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = tid + 256 * u;   // 0 .. 1023: 64 rows x 16 k
      // consecutive threads along the operand's contiguous dimension
      int ii, kk;
      if (a_k == 1) { kk = idx & 15; ii = idx >> 4; } else { ii = idx & 63; kk = idx >> 6; }
      int64_t gi = i0 + ii, gk = k0 + kk;
      As[kk][ii] = (gi < M && gk < ke) ? A[gi * a_i + gk * a_k] : 0.f;
      int jj;
      if (b_j == 1) { jj = idx & 63; kk = idx >> 6; } else { kk = idx & 15; jj = idx >> 4; }
      const int64_t gj = j0 + jj;
      gk = k0 + kk;
      Bs[kk][jj] = (gj < N && gk < ke) ? Bm[gk * b_k + gj * b_j] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const float4 a = *reinterpret_cast<const float4*>(&As[kk][ti * 4]);
      const float4 b = *reinterpret_cast<const float4*>(&Bs[kk][tj * 4]);
      const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(av[r], bv[c], acc[r][c]);
    }
    __syncthreads();
  }
  float* Cz = C + (int64_t)blockIdx.z * zstride;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = i0 + ti * 4 + r;
    if (i >= M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t j = j0 + tj * 4 + c;
      if (j < N) Cz[i * ldc + j] = acc[r][c];
    }
  }
}

// raw inputs x [B][n_in] -> z-scored FP32 features X0 [B][k0] (zero padded)
__global__ void k_features_f32(const float* __restrict__ x, int64_t B, int n_in, int k0,
                               const float* __restrict__ mean, const float* __restrict__ stdv,
                               float* __restrict__ X0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * k0) return;
  const int64_t b = i / k0;
  const int f = (int)(i - b * k0);
  float out = 0.f;
  if (f < n_in) {
    const double h = (double)x[b * n_in];
    const double v = f == 0 ? 0.0 : (double)x[b * n_in + f];
    out = (feature_value(f, h, v) - mean[f]) / stdv[f];
  }
  X0[i] = out;
}

// hidden layer: Z = P + b (in place), H = act(Z)
__global__ void k_bias_act_f32(float* __restrict__ Z, const float* __restrict__ bias, int64_t count, int64_t N,
                               int act, float* __restrict__ H) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float z = Z[i] + bias[i % N];
  Z[i] = z;
  H[i] = act_f(act, z);
}

// output layer: y = P + b (normalized) or (P + b) sd + mean (operators)
__global__ void k_out_f32(const float* __restrict__ P, const float* __restrict__ bias, const float* __restrict__ ymean,
                          const float* __restrict__ ystd, int64_t count, int64_t N, int denorm, float* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t n = i % N;
  const float pred = P[i] + bias[n];
  Y[i] = denorm ? pred * ystd[n] + ymean[n] : pred;
}

// MAE against FP32 targets: d = (P + b) - (y - mean) / sd; P <- sign(d),
// absd = |d|
__global__ void k_mae_f32(float* __restrict__ P, const float* __restrict__ bias, const float* __restrict__ y,
                          const float* __restrict__ ymean, const float* __restrict__ ystd, int64_t count, int64_t N,
                          float* __restrict__ absd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t n = i % N;
  const float pred = P[i] + bias[n];
  const float tgt = (y[i] - ymean[n]) * (1.f / ystd[n]);
  const float d = pred - tgt;
  absd[i] = fabsf(d);
  P[i] = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
}

struct Scratch32 {
  float* X0;     // [B][k0]
  float* Z;      // [depth][B][width]
  float* H;      // [depth][B][width]
  float* P;      // [B][n_out]: output-layer product, then the sign matrix
  float* absd;   // [B][n_out] (training)
  float* dZ;     // [B][width] (training)
  float* part;   // split-K partials (training)
  float* cst;    // column-sum chunks (training)
  float* lossp;  // [kLossChunks] (training)
  float* loss;   // [1]
};

constexpr int64_t kSgemmChunk = 2048;   // k per split of a long FP32 product

inline int64_t sgemm_splits(int64_t K) { return std::max<int64_t>(1, (K + kSgemmChunk - 1) / kSgemmChunk); }

el_status get_scratch32(el_ctx* ctx, el_net* net, int64_t B, bool train, Scratch32& s) {
  const int64_t W = net->desc.width, D = net->desc.depth, nout = net->desc.n_out;
  const int64_t chunks = (B + kColsumRows - 1) / kColsumRows;
  size_t need = 0;
  auto add = [&](size_t b) { size_t r = need; need += (b + 255) / 256 * 256; return r; };
  const size_t oX0 = add((size_t)B * net->k0 * 4), oZ = add((size_t)D * B * W * 4), oH = add((size_t)D * B * W * 4);
  const size_t oP = add((size_t)B * nout * 4);
  const size_t oabs = train ? add((size_t)B * nout * 4) : 0, odZ = train ? add((size_t)B * W * 4) : 0;
  const size_t opart = train ? add((size_t)sgemm_splits(nout) * B * W * 4) : 0;
  const size_t ocst = train && chunks > 1 ? add((size_t)chunks * std::max<int64_t>(nout, W) * 4) : 0;
  const size_t olossp = train ? add((size_t)kLossChunks * 4) : 0;
  const size_t oloss = add(256);
  if (net->scratch32.bytes < need) {
    if (net->scratch32.ptr) {
      hipStreamSynchronize(ctx->stream);
      hipFree(net->scratch32.ptr);
      net->scratch32.ptr = nullptr;
      net->scratch32.bytes = 0;
    }
    el_status st = hip_check(ctx, hipMalloc(&net->scratch32.ptr, need), "hipMalloc(FP32 network scratch)");
    if (st) return st;
    net->scratch32.bytes = need;
  }
  char* b = reinterpret_cast<char*>(net->scratch32.ptr);
  auto f = [&](size_t o, bool on) { return on ? reinterpret_cast<float*>(b + o) : nullptr; };
  s.X0 = f(oX0, true); s.Z = f(oZ, true); s.H = f(oH, true); s.P = f(oP, true);
  s.absd = f(oabs, train); s.dZ = f(odZ, train); s.part = f(opart, train);
  s.cst = f(ocst, train && chunks > 1); s.lossp = f(olossp, train); s.loss = f(oloss, true);
  return EL_OK;
}

// C = A B with the strides of k_sgemm; splits > 1: partials C[z] at zstride
el_status sgemm(el_ctx* ctx, const float* A, int64_t a_i, int64_t a_k, const float* Bm, int64_t b_k, int64_t b_j,
                float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, int64_t splits, int64_t zstride) {
  const int64_t mt = (M + 63) / 64, nt = (N + 63) / 64;
  const int64_t kchunk = (K + splits - 1) / splits;
  if (mt > 65535 || splits > 65535 || nt > INT32_MAX)
    return set_error(ctx, EL_ERR_ARG, "FP32 network product: shape too large");
  hipLaunchKernelGGL(k_sgemm, dim3((unsigned)nt, (unsigned)mt, (unsigned)splits), dim3(256), 0, ctx->stream, A, a_i,
                     a_k, Bm, b_k, b_j, C, ldc, zstride, M, N, K, kchunk);
  return hip_check(ctx, hipGetLastError(), "launch k_sgemm");
}

// features and hidden layers (Z and H kept), then the output-layer product
// P = H[depth-1] W_out^T (bias not yet added)
el_status forward32(el_ctx* ctx, el_net* net, int64_t B, const float* x, const Scratch32& s) {
  hipStream_t str = ctx->stream;
  const int64_t W = net->desc.width, k0 = net->k0;
  const int D = net->desc.depth;
  hipLaunchKernelGGL(k_features_f32, dim3(nblk(B * k0)), dim3(256), 0, str, x, B, net->desc.n_in, (int)k0,
                     net->feat_mean, net->feat_std, s.X0);
  for (int l = 0; l < D; ++l) {
    const int64_t in = net->in_dim[l];
    const float* X = l == 0 ? s.X0 : s.H + (size_t)(l - 1) * B * W;
    float* Z = s.Z + (size_t)l * B * W;
    el_status st = sgemm(ctx, X, in, 1, net->theta + net->w_off[l], 1, in, Z, W, B, W, in, 1, 0);
    if (st) return st;
    hipLaunchKernelGGL(k_bias_act_f32, dim3(nblk(B * W)), dim3(256), 0, str, Z, net->theta + net->b_off[l], B * W, W,
                       net->desc.act, s.H + (size_t)l * B * W);
  }
  return sgemm(ctx, s.H + (size_t)(D - 1) * B * W, W, 1, net->theta + net->w_off[D], 1, W, s.P, net->desc.n_out, B,
               net->desc.n_out, W, 1, 0);
}

}  // namespace

// ---- allocation-free inference: the static scratch array ----------------------
// One array per GPU the library runs on, held until the process ends.  Host
// code never uses its name as an address: noalloc_init() resolves the
// device address once per device and the entry point passes that pointer
// to the kernels.
constexpr size_t kNoAllocBytes = size_t(64) << 20;

}  // namespace el

static __device__ __align__(256) unsigned char scratch[el::kNoAllocBytes];

namespace el {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

el_status noalloc_init(el_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return set_error(ctx, EL_ERR_ARG, "el_create: device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[ctx->device]) return EL_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_check(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
  g_noalloc_ptr[ctx->device] = p;
  return EL_OK;
}

el_status launch_local_solve_ex(el_ctx* ctx, el_ctx::DiscEntry* de, int precision, int64_t E, const double* h,
                                const double* kappa, const double* sigma, const int32_t* emap, void* o_i2o,
                                void* o_i2v, int form, int out_dtype, uint16_t* pairs);

std::vector<std::string> gemm_tile_names() {
  std::vector<std::string> v;
  for (int i = 0; i < kNumVariants; ++i) v.push_back(tile_name(kVariants[i]));
  return v;
}

}  // namespace el

using namespace el;

extern "C" {

el_status el_net_create(el_ctx* ctx, const el_net_desc* desc, el_net** out) {
  if (!ctx || !desc || !out) return EL_ERR_ARG;
  *out = nullptr;
  if (!desc_ok(*desc)) return set_error(ctx, EL_ERR_ARG, "el_net_create: bad network description");
  hipSetDevice(ctx->device);
  el_net* net = new el_net();
  net->desc = *desc;
  net->device = ctx->device;
  layout(net);
  el_status st = alloc_net(ctx, net);
  if (st) { delete net; return st; }
  for (int l = 0; l <= desc->depth; ++l) {
    const int64_t fan_in = l == 0 ? desc->n_in : desc->width;
    const float bound = (float)(1.0 / std::sqrt((double)fan_in));
    const int64_t nw = net->in_dim[l] * net->out_dim[l];
    hipLaunchKernelGGL(k_init_uniform, dim3(nblk(nw)), dim3(256), 0, ctx->stream, net->theta + net->w_off[l], nw,
                       net->in_dim[l], (int64_t)(l == 0 ? desc->n_in : desc->width), bound, desc->seed,
                       net->w_off[l]);
    hipLaunchKernelGGL(k_init_uniform, dim3(nblk(net->out_dim[l])), dim3(256), 0, ctx->stream,
                       net->theta + net->b_off[l], net->out_dim[l], (int64_t)0, (int64_t)0, bound, desc->seed,
                       net->b_off[l]);
  }
  const int64_t P = net->n_params;
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(P)), dim3(256), 0, ctx->stream, net->adam_m, P, 0.f);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(P)), dim3(256), 0, ctx->stream, net->adam_v, P, 0.f);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(P)), dim3(256), 0, ctx->stream, net->grad, P, 0.f);
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(P)), dim3(256), 0, ctx->stream, net->theta, net->wbf, P);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(desc->n_in)), dim3(256), 0, ctx->stream, net->feat_mean,
                     (int64_t)desc->n_in, 0.f);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(desc->n_in)), dim3(256), 0, ctx->stream, net->feat_std,
                     (int64_t)desc->n_in, 1.f);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(desc->n_out)), dim3(256), 0, ctx->stream, net->y_mean, desc->n_out, 0.f);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(desc->n_out)), dim3(256), 0, ctx->stream, net->y_std, desc->n_out, 1.f);
  net->box[0] = net->box[2] = net->box[4] = 0.0;
  net->box[1] = net->box[3] = net->box[5] = 0.0;
  st = hip_check(ctx, hipGetLastError(), "el_net_create init");
  if (st) { el_net_destroy(net); return st; }
  *out = net;
  return EL_OK;
}

el_status el_net_destroy(el_net* net) {
  if (!net) return EL_OK;
  hipSetDevice(net->device);
  hipDeviceSynchronize();
  hipFree(net->theta);
  hipFree(net->scratch.ptr);
  hipFree(net->scratch32.ptr);
  delete net;
  return EL_OK;
}

el_status el_net_num_params(const el_net* net, int64_t* n) {
  if (!net || !n) return EL_ERR_ARG;
  *n = net->n_params;
  return EL_OK;
}

static const size_t kHeader = 112;

el_status el_net_save(el_ctx* ctx, const el_net* net, void* host_buf, size_t* bytes) {
  if (!ctx || !net || !bytes) return EL_ERR_ARG;
  const int64_t P = net->n_params, nin = net->desc.n_in, nout = net->desc.n_out;
  const size_t need = kHeader + 4 * (size_t)(2 * nin + 2 * nout + 3 * P);
  if (!host_buf) { *bytes = need; return EL_OK; }
  if (*bytes < need) return set_error(ctx, EL_ERR_ARG, "el_net_save: buffer too small");
  char* b = reinterpret_cast<char*>(host_buf);
  std::memset(b, 0, kHeader);
  std::memcpy(b, "ELNET01", 8);
  int32_t hi[6] = {net->desc.n_in, net->desc.width, net->desc.depth, net->desc.act, net->k0, 0};
  std::memcpy(b + 8, hi, sizeof hi);
  int64_t hl[3] = {nout, net->step, P};
  std::memcpy(b + 32, hl, sizeof hl);
  std::memcpy(b + 56, net->box, sizeof net->box);
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  char* o = b + kHeader;
  auto get = [&](const float* src, int64_t cnt) {
    hipError_t e = hipMemcpy(o, src, cnt * 4, hipMemcpyDeviceToHost);
    o += cnt * 4;
    return e;
  };
  hipError_t e = get(net->feat_mean, nin);
  if (e == hipSuccess) e = get(net->feat_std, nin);
  if (e == hipSuccess) e = get(net->y_mean, nout);
  if (e == hipSuccess) e = get(net->y_std, nout);
  if (e == hipSuccess) e = get(net->theta, P);
  if (e == hipSuccess) e = get(net->adam_m, P);
  if (e == hipSuccess) e = get(net->adam_v, P);
  if (e != hipSuccess) return hip_check(ctx, e, "el_net_save");
  *bytes = need;
  return EL_OK;
}

el_status el_net_load(el_ctx* ctx, const void* host_buf, size_t bytes, el_net** out) {
  if (!ctx || !host_buf || !out) return EL_ERR_ARG;
  *out = nullptr;
  const char* b = reinterpret_cast<const char*>(host_buf);
  if (bytes < kHeader || std::memcmp(b, "ELNET01", 8) != 0) return set_error(ctx, EL_ERR_ARG, "el_net_load: bad magic");
  int32_t hi[6];
  int64_t hl[3];
  std::memcpy(hi, b + 8, sizeof hi);
  std::memcpy(hl, b + 32, sizeof hl);
  el_net_desc d{};
  d.n_in = hi[0]; d.width = hi[1]; d.depth = hi[2]; d.act = hi[3]; d.n_out = hl[0]; d.seed = 0;
  if (!desc_ok(d)) return set_error(ctx, EL_ERR_ARG, "el_net_load: bad header");
  hipSetDevice(ctx->device);
  el_net* net = new el_net();
  net->desc = d;
  net->device = ctx->device;
  layout(net);
  if (net->k0 != hi[4] || net->n_params != hl[2]) { delete net; return set_error(ctx, EL_ERR_ARG, "el_net_load: layout mismatch"); }
  const int64_t P = net->n_params, nin = d.n_in, nout = d.n_out;
  if (bytes < kHeader + 4 * (size_t)(2 * nin + 2 * nout + 3 * P)) {
    delete net;
    return set_error(ctx, EL_ERR_ARG, "el_net_load: truncated blob");
  }
  el_status st = alloc_net(ctx, net);
  if (st) { delete net; return st; }
  net->step = hl[1];
  std::memcpy(net->box, b + 56, sizeof net->box);
  net->fitted = true;
  const char* o = b + kHeader;
  auto put = [&](float* dst, int64_t cnt) {
    hipError_t e = hipMemcpy(dst, o, cnt * 4, hipMemcpyHostToDevice);
    o += cnt * 4;
    return e;
  };
  hipError_t e = put(net->feat_mean, nin);
  if (e == hipSuccess) e = put(net->feat_std, nin);
  if (e == hipSuccess) e = put(net->y_mean, nout);
  if (e == hipSuccess) e = put(net->y_std, nout);
  if (e == hipSuccess) e = put(net->theta, P);
  if (e == hipSuccess) e = put(net->adam_m, P);
  if (e == hipSuccess) e = put(net->adam_v, P);
  if (e != hipSuccess) { el_net_destroy(net); return hip_check(ctx, e, "el_net_load"); }
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(P)), dim3(256), 0, ctx->stream, net->theta, net->wbf, P);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(P)), dim3(256), 0, ctx->stream, net->grad, P, 0.f);
  *out = net;
  return hip_check(ctx, hipGetLastError(), "el_net_load");
}

el_status el_net_params(el_ctx* ctx, const el_net* net, int which, float* dst) {
  if (!ctx || !net || !dst || which < 0 || which > 3) return EL_ERR_ARG;
  const float* src = which == 0 ? net->theta : which == 1 ? net->grad : which == 2 ? net->adam_m : net->adam_v;
  return hip_check(ctx, hipMemcpyAsync(dst, src, net->n_params * 4, hipMemcpyDeviceToDevice, ctx->stream),
                   "el_net_params");
}

el_status el_net_fit_normalization(el_ctx* ctx, el_net* net, int64_t N, const float* x, const uint16_t* y) {
  if (!ctx || !net || N <= 0 || !x || !y) return set_error(ctx, EL_ERR_ARG, "el_net_fit_normalization: bad argument");
  hipSetDevice(ctx->device);
  const int nin = net->desc.n_in;
  hipLaunchKernelGGL(k_feat_stats, dim3(nin), dim3(256), 0, ctx->stream, x, N, nin, net->feat_mean, net->feat_std);
  hipLaunchKernelGGL(k_y_stats, dim3(nblk(net->desc.n_out)), dim3(256), 0, ctx->stream, y, N, net->desc.n_out,
                     net->y_mean, net->y_std);
  el_status st = ensure_ws(ctx, ctx->ws_small, 4096 + 1024);
  if (st) return st;
  double* dbox = reinterpret_cast<double*>(reinterpret_cast<char*>(ctx->ws_small.ptr) + 4096);
  hipLaunchKernelGGL(k_box, dim3(3), dim3(256), 0, ctx->stream, x, N, nin, dbox);
  hipError_t e = hipMemcpyAsync(net->box, dbox, sizeof net->box, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_check(ctx, e, "el_net_fit_normalization");
  net->fitted = true;
  return EL_OK;
}

el_status el_make_pairs(el_ctx* ctx, el_disc d, int64_t E, const double* h, const double* kappa,
                        const double* sigma, int form, uint16_t* y) {
  if (!ctx) return EL_ERR_ARG;
  if (form != EL_FORM_IN2SOL && form != EL_FORM_IN2MEAN) return set_error(ctx, EL_ERR_ARG, "el_make_pairs: form");
  if (E == 0) return EL_OK;
  if (E < 0 || !h || !kappa || !sigma || !y) return set_error(ctx, EL_ERR_ARG, "el_make_pairs: bad argument");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  const int precision = local_fp64_fits(ctx, de) ? EL_FP64 : EL_FP32_IR;
  return launch_local_solve_ex(ctx, de, precision, E, h, kappa, sigma, nullptr, nullptr, nullptr, form, EL_BF16, y);
}

el_status el_net_forward(el_ctx* ctx, const el_net* cnet, int64_t B, const float* x, float* y_norm) {
  if (!ctx || !cnet) return EL_ERR_ARG;
  if (B == 0) return EL_OK;
  if (B < 0 || !x || !y_norm) return set_error(ctx, EL_ERR_ARG, "el_net_forward: bad argument");
  el_net* net = const_cast<el_net*>(cnet);
  hipSetDevice(ctx->device);
  Scratch s;
  el_status st = get_scratch(ctx, net, B, false, s);
  if (st) return st;
  Box open{{-1e300, 1e300, -1e300, 1e300, -1e300, 1e300}};
  hipLaunchKernelGGL(k_features, dim3((unsigned)B), dim3(128), 0, ctx->stream, x, nullptr, nullptr, nullptr, B,
                     net->desc.n_in, net->k0, net->feat_mean, net->feat_std, s.X0, open, nullptr);
  st = forward_hidden(ctx, net, B, s, false);
  if (st) return st;
  const int D = net->desc.depth;
  const int64_t W = net->desc.width;
  EpiOutNorm epi{net->theta + net->b_off[D], y_norm, net->desc.n_out};
  return mm<true, true>(ctx, s.H + (size_t)(D - 1) * B * W, W, net->wbf + net->w_off[D], W, B, net->desc.n_out, W, 1,
                        epi, true);
}

el_status el_train_step(el_ctx* ctx, el_net* net, int64_t B, const float* x, const uint16_t* y, float lr,
                        float* loss) {
  if (!ctx || !net || B <= 0 || !x || !y) return set_error(ctx, EL_ERR_ARG, "el_train_step: bad argument");
  if (!(lr >= 0.f)) return set_error(ctx, EL_ERR_ARG, "el_train_step: lr must be >= 0");
  hipSetDevice(ctx->device);
  Scratch s;
  el_status st = get_scratch(ctx, net, B, true, s);
  if (st) return st;
  hipStream_t str = ctx->stream;
  const int D = net->desc.depth;
  const int64_t W = net->desc.width, nout = net->desc.n_out;
  Box open{{-1e300, 1e300, -1e300, 1e300, -1e300, 1e300}};
  hipLaunchKernelGGL(k_features, dim3((unsigned)B), dim3(128), 0, str, x, nullptr, nullptr, nullptr, B,
                     net->desc.n_in, net->k0, net->feat_mean, net->feat_std, s.X0, open, nullptr);
  st = forward_hidden(ctx, net, B, s, true);
  if (st) return st;
  const uint16_t* Hlast = s.H + (size_t)(D - 1) * B * W;
  if (B * nout >= ((int64_t)1 << 31))
    return set_error(ctx, EL_ERR_ARG, "el_train_step: batch x n_out must stay below 2^31");
  // with the transposed output-layer GEMMs (64 | B) the epilogue also
  // writes dY transposed for dW
  EpiMAE mae{net->theta + net->b_off[D], y, net->y_mean, net->y_std, s.dY, s.colp, s.lossp, nout, 0.f, 0.f,
             0, 0, 0, 0, s.dYT, B, 0, nullptr, nullptr};
  st = mm<true, true>(ctx, Hlast, W, net->wbf + net->w_off[D], W, B, nout, W, 1, mae, true);
  if (st) return st;
  // output layer gradients: the bias from the epilogue's per-block column
  // sums, the loss from its per-block sums (fixed-order reductions)
  const int64_t rb = (B + 31) / 32;
  st = colsum(ctx, s.colp, rb, nout, rb, nullptr, net->grad + net->b_off[D]);
  if (st) return st;
  {
    const int64_t nl = rb * ((nout + 31) / 32), chunk = (nl + kLossChunks - 1) / kLossChunks;
    float* lp2 = s.lossp + nl;
    hipLaunchKernelGGL(k_sum_chunks, dim3(kLossChunks), dim3(256), 0, str, s.lossp, nl, chunk, lp2);
    hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(256), 0, str, lp2, (int64_t)kLossChunks, (int64_t)kLossChunks,
                       s.loss);
  }
  if (s.dYT) {
    auto tp = [&](const uint16_t* src, int64_t rows, int64_t cols, uint16_t* dst) {
      hipLaunchKernelGGL(k_transpose16, dim3((unsigned)((rows / 64) * (cols / 64))), dim3(256), 0, str, src, rows,
                         cols, dst);
    };
    tp(Hlast, B, W, s.HT);
    tp(net->wbf + net->w_off[D], nout, W, s.WT);
    st = mm<true, true>(ctx, s.dYT, B, s.HT, B, nout, W, B, 1, EpiF32{net->grad + net->w_off[D], W, 0});
    if (st) return st;
    st = mm<true, true>(ctx, s.dY, nout, s.WT, nout, B, W, nout, kSplitOut, EpiF32{s.part, W, B * W});
    if (st) return st;
  } else {
    st = mm<false, false>(ctx, s.dY, nout, Hlast, W, nout, W, B, 1, EpiF32{net->grad + net->w_off[D], W, 0});
    if (st) return st;
    st = mm<true, false>(ctx, s.dY, nout, net->wbf + net->w_off[D], W, B, W, nout, kSplitOut,
                         EpiF32{s.part, W, B * W});
    if (st) return st;
  }
  {
    int64_t ks = (nout + kSplitOut - 1) / kSplitOut;
    ks = (ks + gemm::BK - 1) / gemm::BK * gemm::BK;
    const int S = (int)((nout + ks - 1) / ks);
    hipLaunchKernelGGL(k_reduce_dact, dim3(nblk(B * W)), dim3(256), 0, str, s.part, S, B * W,
                       s.Z + (size_t)(D - 1) * B * W, net->desc.act, s.dZ, s.dZ16);
  }
  for (int l = D - 1; l >= 0; --l) {
    const int64_t in = net->in_dim[l];
    const uint16_t* X = l == 0 ? s.X0 : s.H + (size_t)(l - 1) * B * W;
    st = colsum(ctx, s.dZ, B, W, kColsumRows, s.cst, net->grad + net->b_off[l]);
    if (st) return st;
    st = mm<false, false>(ctx, s.dZ16, W, X, in, W, in, B, kSplitW, EpiF32{s.part, in, W * in});
    if (st) return st;
    {
      int64_t ks = (B + kSplitW - 1) / kSplitW;
      ks = (ks + gemm::BK - 1) / gemm::BK * gemm::BK;
      const int S = (int)((B + ks - 1) / ks);
      hipLaunchKernelGGL(k_reduce_sum, dim3(nblk(W * in)), dim3(256), 0, str, s.part, S, W * in,
                         net->grad + net->w_off[l]);
    }
    if (l > 0) {
      st = mm<true, false>(ctx, s.dZ16, W, net->wbf + net->w_off[l], in, B, in, W, 1, EpiF32{s.part, in, 0});
      if (st) return st;
      hipLaunchKernelGGL(k_reduce_dact, dim3(nblk(B * W)), dim3(256), 0, str, s.part, 1, B * W,
                         s.Z + (size_t)(l - 1) * B * W, net->desc.act, s.dZ, s.dZ16);
    }
  }
  net->step += 1;
  const double t = (double)net->step;
  const float bc1 = (float)(1.0 - std::pow(0.9, t)), bc2 = (float)(1.0 - std::pow(0.999, t));
  const float gscale = (float)(1.0 / ((double)B * (double)nout));
  hipLaunchKernelGGL(k_adam, dim3(nblk(net->n_params)), dim3(256), 0, str, net->theta, net->grad, net->adam_m,
                     net->adam_v, net->wbf, net->n_params, lr, gscale, bc1, bc2);
  if (loss) hipLaunchKernelGGL(k_loss_out, dim3(1), dim3(64), 0, str, s.loss, gscale, loss);
  return hip_check(ctx, hipGetLastError(), "el_train_step");
}

el_status el_net_forward_f32(el_ctx* ctx, const el_net* cnet, int64_t B, const float* x, float* y, int denormalize) {
  if (!ctx || !cnet) return EL_ERR_ARG;
  if (B == 0) return EL_OK;
  if (B < 0 || !x || !y) return set_error(ctx, EL_ERR_ARG, "el_net_forward_f32: bad argument");
  el_net* net = const_cast<el_net*>(cnet);
  hipSetDevice(ctx->device);
  Scratch32 s;
  el_status st = get_scratch32(ctx, net, B, false, s);
  if (st) return st;
  st = forward32(ctx, net, B, x, s);
  if (st) return st;
  const int64_t nout = net->desc.n_out;
  const int D = net->desc.depth;
  hipLaunchKernelGGL(k_out_f32, dim3(nblk(B * nout)), dim3(256), 0, ctx->stream, s.P, net->theta + net->b_off[D],
                     net->y_mean, net->y_std, B * nout, nout, denormalize ? 1 : 0, y);
  return hip_check(ctx, hipGetLastError(), "el_net_forward_f32");
}

el_status el_train_step_f32(el_ctx* ctx, el_net* net, int64_t B, const float* x, const float* y, float lr,
                            float* loss) {
  if (!ctx || !net || B <= 0 || !x || !y) return set_error(ctx, EL_ERR_ARG, "el_train_step_f32: bad argument");
  if (!(lr >= 0.f)) return set_error(ctx, EL_ERR_ARG, "el_train_step_f32: lr must be >= 0");
  hipSetDevice(ctx->device);
  Scratch32 s;
  el_status st = get_scratch32(ctx, net, B, true, s);
  if (st) return st;
  hipStream_t str = ctx->stream;
  const int D = net->desc.depth;
  const int64_t W = net->desc.width, nout = net->desc.n_out;
  st = forward32(ctx, net, B, x, s);
  if (st) return st;
  // output layer: signs of the MAE residuals in P, |residual| in absd
  hipLaunchKernelGGL(k_mae_f32, dim3(nblk(B * nout)), dim3(256), 0, str, s.P, net->theta + net->b_off[D], y,
                     net->y_mean, net->y_std, B * nout, nout, s.absd);
  st = colsum(ctx, s.P, B, nout, kColsumRows, s.cst, net->grad + net->b_off[D]);
  if (st) return st;
  {
    const int64_t n = B * nout, chunk = (n + kLossChunks - 1) / kLossChunks;
    hipLaunchKernelGGL(k_sum_chunks, dim3(kLossChunks), dim3(256), 0, str, s.absd, n, chunk, s.lossp);
    hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(256), 0, str, s.lossp, (int64_t)kLossChunks,
                       (int64_t)kLossChunks, s.loss);
  }
  const float* Hlast = s.H + (size_t)(D - 1) * B * W;
  // dW_out = dY^T H [n_out][W]; dX = dY W_out [B][W] (split over n_out)
  st = sgemm(ctx, s.P, 1, nout, Hlast, W, 1, net->grad + net->w_off[D], W, nout, W, B, 1, 0);
  if (st) return st;
  const int64_t S = sgemm_splits(nout);
  st = sgemm(ctx, s.P, nout, 1, net->theta + net->w_off[D], W, 1, s.part, W, B, W, nout, S, B * W);
  if (st) return st;
  hipLaunchKernelGGL(k_reduce_dact, dim3(nblk(B * W)), dim3(256), 0, str, s.part, (int)S, B * W,
                     s.Z + (size_t)(D - 1) * B * W, net->desc.act, s.dZ, nullptr);
  for (int l = D - 1; l >= 0; --l) {
    const int64_t in = net->in_dim[l];
    const float* X = l == 0 ? s.X0 : s.H + (size_t)(l - 1) * B * W;
    st = colsum(ctx, s.dZ, B, W, kColsumRows, s.cst, net->grad + net->b_off[l]);
    if (st) return st;
    // dW_l = dZ^T X [W][in]
    st = sgemm(ctx, s.dZ, 1, W, X, in, 1, net->grad + net->w_off[l], in, W, in, B, 1, 0);
    if (st) return st;
    if (l > 0) {
      // dX = dZ W_l [B][in], then dZ of the layer below
      st = sgemm(ctx, s.dZ, W, 1, net->theta + net->w_off[l], in, 1, s.part, in, B, in, W, 1, 0);
      if (st) return st;
      hipLaunchKernelGGL(k_reduce_dact, dim3(nblk(B * W)), dim3(256), 0, str, s.part, 1, B * W,
                         s.Z + (size_t)(l - 1) * B * W, net->desc.act, s.dZ, nullptr);
    }
  }
  net->step += 1;
  const double t = (double)net->step;
  const float bc1 = (float)(1.0 - std::pow(0.9, t)), bc2 = (float)(1.0 - std::pow(0.999, t));
  const float gscale = (float)(1.0 / ((double)B * (double)nout));
  hipLaunchKernelGGL(k_adam, dim3(nblk(net->n_params)), dim3(256), 0, str, net->theta, net->grad, net->adam_m,
                     net->adam_v, net->wbf, net->n_params, lr, gscale, bc1, bc2);
  if (loss) hipLaunchKernelGGL(k_loss_out, dim3(1), dim3(64), 0, str, s.loss, gscale, loss);
  return hip_check(ctx, hipGetLastError(), "el_train_step_f32");
}

el_status el_infer(el_ctx* ctx, const el_net* cnet, el_disc d, int64_t E, const double* h, const double* kappa,
                   const double* sigma, void* in2out, void* in2vol, int out_dtype, uint8_t* in_range, int fallback,
                   int precision, int64_t* n_fallback_host) {
  if (!ctx || !cnet) return EL_ERR_ARG;
  if (out_dtype != EL_BF16 && out_dtype != EL_F32 && out_dtype != EL_F16)
    return set_error(ctx, EL_ERR_ARG, "el_infer: out_dtype");
  if (precision != EL_FP64 && precision != EL_FP32_IR)
    return set_error(ctx, EL_ERR_ARG, "el_infer: unknown fallback precision");
  if (E == 0) {
    if (n_fallback_host) *n_fallback_host = 0;
    return EL_OK;
  }
  if (E < 0 || !h || !kappa || !sigma) return set_error(ctx, EL_ERR_ARG, "el_infer: bad argument");
  const size_t osz = out_dtype == EL_F32 ? 4 : 2;
  el_net* net = const_cast<el_net*>(cnet);
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  const DiscHost& dh = de->host;
  const int64_t mm_ = (int64_t)dh.m * dh.m;
  // the network's output size tells its form: (in2out, in2sol) or (in2out, in2mean)
  int form;
  if (net->desc.n_out == mm_ + (int64_t)dh.n * dh.m) form = EL_FORM_IN2SOL;
  else if (net->desc.n_out == mm_ + (int64_t)dh.nn * dh.m) form = EL_FORM_IN2MEAN;
  else return set_error(ctx, EL_ERR_ARG, "el_infer: network output size does not match the discretization");
  const int64_t nm = net->desc.n_out - mm_;   // per-element size of in2sol or in2mean
  if (net->desc.n_in != 1 + 2 * dh.nn)
    return set_error(ctx, EL_ERR_ARG, "el_infer: network input size does not match the discretization");
  if (!net->fitted) return set_error(ctx, EL_ERR_STATE, "el_infer: network has no training statistics");
  const int D = net->desc.depth;
  const int64_t W = net->desc.width;
  // chunk the batch so that scratch stays bounded
  const int64_t chunk = 16384;
  el_status st2 = ensure_ws(ctx, ctx->ws_small, 4096 + 1024);
  if (st2) return st2;
  int* dcount = reinterpret_cast<int*>(reinterpret_cast<char*>(ctx->ws_small.ptr) + 4096 + 512);
  // context workspace: fallback index [E] int32, then the range mask [E]
  // when the caller passes none (grown on demand, kept across calls)
  const size_t idx_bytes = (sizeof(int32_t) * (size_t)E + 255) / 256 * 256;
  st = ensure_ws(ctx, ctx->ws_infer, idx_bytes + (in_range ? 0 : (size_t)E));
  if (st) return st;
  int32_t* idx = reinterpret_cast<int32_t*>(ctx->ws_infer.ptr);
  uint8_t* mask = in_range ? in_range : reinterpret_cast<uint8_t*>(ctx->ws_infer.ptr) + idx_bytes;
  for (int64_t e0 = 0; e0 < E; e0 += chunk) {
    const int64_t B = std::min(chunk, E - e0);
    Scratch s;
    st = get_scratch(ctx, net, B, false, s);
    if (st) break;
    hipLaunchKernelGGL(k_features, dim3((unsigned)B), dim3(128), 0, ctx->stream, nullptr, h + e0,
                       kappa + e0 * dh.nn, sigma + e0 * dh.nn, B, net->desc.n_in, net->k0, net->feat_mean,
                       net->feat_std, s.X0, make_box(net), mask + e0);
    st = forward_hidden(ctx, net, B, s, false);
    if (st) break;
    char* po = in2out ? reinterpret_cast<char*>(in2out) + (size_t)e0 * mm_ * osz : nullptr;
    char* ps = in2vol ? reinterpret_cast<char*>(in2vol) + (size_t)e0 * nm * osz : nullptr;
    const uint16_t* Hl = s.H + (size_t)(D - 1) * B * W;
    if (out_dtype == EL_F32) {
      EpiOutOps<float> epi{net->theta + net->b_off[D], net->y_mean, net->y_std, reinterpret_cast<float*>(po),
                           reinterpret_cast<float*>(ps), mm_, nm};
      st = mm<true, true>(ctx, Hl, W, net->wbf + net->w_off[D], W, B, net->desc.n_out, W, 1, epi, true);
    } else if (out_dtype == EL_F16) {
      EpiOutOps<_Float16> epi{net->theta + net->b_off[D], net->y_mean, net->y_std, reinterpret_cast<_Float16*>(po),
                              reinterpret_cast<_Float16*>(ps), mm_, nm};
      st = mm<true, true>(ctx, Hl, W, net->wbf + net->w_off[D], W, B, net->desc.n_out, W, 1, epi, true);
    } else {
      EpiOutOps<uint16_t> epi{net->theta + net->b_off[D], net->y_mean, net->y_std, reinterpret_cast<uint16_t*>(po),
                              reinterpret_cast<uint16_t*>(ps), mm_, nm};
      st = mm<true, true>(ctx, Hl, W, net->wbf + net->w_off[D], W, B, net->desc.n_out, W, 1, epi, true);
    }
    if (st) break;
  }
  int64_t nfb = 0;
  if (!st) {
    // count and compact the elements outside the training box
    hipLaunchKernelGGL(k_fill_int32, dim3(1), dim3(64), 0, ctx->stream, dcount, 1, 0);
    hipLaunchKernelGGL(k_count_out, dim3(nblk(E)), dim3(256), 0, ctx->stream, mask, E, idx, dcount);
    int hc = 0;
    hipError_t e = hipMemcpyAsync(&hc, dcount, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    st = hip_check(ctx, e, "el_infer count");
    nfb = hc;
    if (!st && fallback && hc > 0)
      st = launch_local_solve_ex(ctx, de, precision, hc, h, kappa, sigma, idx, in2out, in2vol, form, out_dtype,
                                 nullptr);
  }
  if (n_fallback_host) *n_fallback_host = nfb;
  return st;
}

el_status el_infer_noalloc(el_ctx* ctx, const el_net* cnet, el_disc d, int64_t E, const double* h,
                           const double* kappa, const double* sigma, void* in2out, void* in2vol, int out_dtype,
                           uint8_t* in_range) {
  if (!ctx || !cnet) return EL_ERR_ARG;
  if (out_dtype != EL_BF16 && out_dtype != EL_F32 && out_dtype != EL_F16)
    return set_error(ctx, EL_ERR_ARG, "el_infer_noalloc: out_dtype");
  if (E == 0) return EL_OK;
  if (E < 0 || !h || !kappa || !sigma) return set_error(ctx, EL_ERR_ARG, "el_infer_noalloc: bad argument");
  int64_t nn = 0, n = 0, m = 0;
  if (el_disc_sizes(d, &nn, &n, &m) != EL_OK) return set_error(ctx, EL_ERR_ARG, "el_infer_noalloc: bad el_disc");
  el_net* net = const_cast<el_net*>(cnet);
  const int64_t mm_ = m * m;
  if (net->desc.n_out != mm_ + n * m && net->desc.n_out != mm_ + nn * m)
    return set_error(ctx, EL_ERR_ARG, "el_infer_noalloc: network output size does not match the discretization");
  if (net->desc.n_in != 1 + 2 * nn)
    return set_error(ctx, EL_ERR_ARG, "el_infer_noalloc: network input size does not match the discretization");
  if (!net->fitted) return set_error(ctx, EL_ERR_STATE, "el_infer_noalloc: network has no training statistics");
  hipSetDevice(ctx->device);
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    base = reinterpret_cast<char*>(g_noalloc_ptr[ctx->device]);
  }
  if (!base) return set_error(ctx, EL_ERR_STATE, "el_infer_noalloc: static scratch not initialized on this device");
  const int D = net->desc.depth;
  const int64_t W = net->desc.width, k0 = net->k0, nm = net->desc.n_out - mm_;
  // rows per pass: features [rows][k0] and hidden activations [D][rows][W]
  // (bfloat16) in the static array, a multiple of 256 rows
  const int64_t row_bytes = 2 * (k0 + (int64_t)D * W);
  const int64_t fit = (int64_t)(kNoAllocBytes / (size_t)row_bytes) / 256 * 256;
  if (fit < 256) {
    std::ostringstream os;
    os << "el_infer_noalloc: the network needs " << row_bytes << " B of scratch per element; the "
       << (kNoAllocBytes >> 20) << " MiB static scratch holds fewer than 256 elements";
    return set_error(ctx, EL_ERR_ARG, os.str());
  }
  const int64_t rows = std::min<int64_t>(fit, 16384);
  const size_t osz = out_dtype == EL_F32 ? 4 : 2;
  for (int64_t e0 = 0; e0 < E; e0 += rows) {
    const int64_t B = std::min(rows, E - e0);
    Scratch s{};
    s.X0 = reinterpret_cast<uint16_t*>(base);
    s.H = reinterpret_cast<uint16_t*>(base + (size_t)rows * k0 * 2);
    hipLaunchKernelGGL(k_features, dim3((unsigned)B), dim3(128), 0, ctx->stream, nullptr, h + e0,
                       kappa + e0 * nn, sigma + e0 * nn, B, net->desc.n_in, net->k0, net->feat_mean,
                       net->feat_std, s.X0, make_box(net), in_range ? in_range + e0 : nullptr);
    el_status st = forward_hidden(ctx, net, B, s, false, true);
    if (st) return st;
    char* po = in2out ? reinterpret_cast<char*>(in2out) + (size_t)e0 * mm_ * osz : nullptr;
    char* ps = in2vol ? reinterpret_cast<char*>(in2vol) + (size_t)e0 * nm * osz : nullptr;
    const uint16_t* Hl = s.H + (size_t)(D - 1) * B * W;
    const uint16_t* WD = net->wbf + net->w_off[D];
    const int v = fixed_variant(Hl, W, WD, W, W);
    if (out_dtype == EL_F32) {
      EpiOutOps<float> epi{net->theta + net->b_off[D], net->y_mean, net->y_std, reinterpret_cast<float*>(po),
                           reinterpret_cast<float*>(ps), mm_, nm};
      st = mm_variant<true, true>(ctx, v, Hl, W, WD, W, B, net->desc.n_out, W, 1, epi, true);
    } else if (out_dtype == EL_F16) {
      EpiOutOps<_Float16> epi{net->theta + net->b_off[D], net->y_mean, net->y_std, reinterpret_cast<_Float16*>(po),
                              reinterpret_cast<_Float16*>(ps), mm_, nm};
      st = mm_variant<true, true>(ctx, v, Hl, W, WD, W, B, net->desc.n_out, W, 1, epi, true);
    } else {
      EpiOutOps<uint16_t> epi{net->theta + net->b_off[D], net->y_mean, net->y_std, reinterpret_cast<uint16_t*>(po),
                              reinterpret_cast<uint16_t*>(ps), mm_, nm};
      st = mm_variant<true, true>(ctx, v, Hl, W, WD, W, B, net->desc.n_out, W, 1, epi, true);
    }
    if (st) return st;
  }
  return hip_check(ctx, hipGetLastError(), "el_infer_noalloc");
}

el_status el_gemm_tile(int variant) {
  if (variant < -1 || variant >= kNumVariants) return EL_ERR_ARG;
  g_force_tile.store(variant);
  return EL_OK;
}

}  // extern "C"

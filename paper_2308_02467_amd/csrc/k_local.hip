// Batched element local solve (Alg. 1 step 1; eq. hdg_local_f2u_i2u and
// eq. hdg_local_f2o_i2o): for every element, factor
//     A = B - C + M - S          (eq. hdg_local_all_sub_mat)
// by dense LU with partial pivoting and solve A X = -B_hat for the m inflow
// columns, giving in2sol = X, in2out = rows of X at the outflow DOFs and
// in2mean = ordinate average of X.
//
// Kernel design (gfx950):
//  * one workgroup of 512 threads (8 wave64) per element, persistent over
//    elements; each workgroup owns one factor slot in HBM;
//  * left-looking LU in column panels of NB = 16: the current panel lives in
//    LDS in logical (pivoted) row order; the original matrix is never stored:
//    each panel of A is generated on the fly from the tau-independent
//    transport blocks B_k - C_k plus the node-diagonal M and S terms;
//  * row interchanges never move data in HBM: factor rows stay at their
//    physical (original) row and a permutation perm[logical] = physical is
//    kept in LDS;
//  * each factor panel is stored pre-multiplied by the inverse of its
//    diagonal block and negated (-L inv(L_II) below, -U inv(U_II) above the
//    block), so that a block sweep step is a single rank-16 update
//        rows += F_I pan[I]
//    with one barrier per step, and the 16x16 diagonal-block solves of a
//    whole sweep run afterwards, independently, on all waves;
//  * the sweep updates run on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
//    factor tiles are streamed from HBM two steps ahead of their use with
//    16-byte loads, the panel tiles are read-modified-written in LDS;
//  * the right-hand side -B_hat (one nonzero per column) is generated in
//    panels of 16 columns, forward-swept (skipping the leading zero blocks)
//    and back-swept, and the solution panel is written straight to in2sol /
//    in2out / in2mean (FP64, FP32 or bfloat16).
// With NB = 16 each factor byte feeds 4 flops, so the sweeps are bound by
// HBM bandwidth rather than by the matrix cores.
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <sstream>

#include "el_internal.h"
#include "gemm_bf16.h"

namespace el {
namespace {

constexpr int NB = 16;
constexpr int LDP = NB + 1;       // padded LDS row stride (bank spread)
constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Output layout of the 16x16x4 MFMAs (measured on gfx950): register r of lane
// l holds D[row][l % 16] with row = l/16 + 4r for f64 and 4(l/16) + r for f32.
// A[i][k] sits in lane i + 16k and B[k][j] in lane j + 16k for both.
template <typename T> struct Acc;
template <> struct Acc<double> {
  typedef d4 type;
  static __device__ inline int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Acc<float> {
  typedef f4 type;
  static __device__ inline int row(int lk, int r) { return 4 * lk + r; }
};

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
struct LuArgs {
  DiscDev dv;
  int64_t E;
  int npad, mpad;
  const double* h;
  const double* kappa;
  const double* sigma;
  double* in2out;
  double* in2sol;
  double* in2mean;
  uint16_t* b_i2o;        // bfloat16 in2out [E][m][m]
  uint16_t* b_i2s;        // bfloat16 in2sol [E][n][m]
  float* f_i2o;           // float32 in2out [E][m][m]
  float* f_i2s;           // float32 in2sol [E][n][m]
  uint16_t* b_i2m;        // bfloat16 in2mean [E][nn][m]
  float* f_i2m;           // float32 in2mean [E][nn][m]
  _Float16* h_i2o;        // float16 in2out [E][m][m]
  _Float16* h_i2s;        // float16 in2sol [E][n][m]
  _Float16* h_i2m;        // float16 in2mean [E][nn][m]
  uint16_t* pairs;        // bfloat16 (in2out, in2sol) [E][m*m + n*m] or (in2out, in2mean) [E][m*m + nn*m]
  const double* src;      // volume source f at the nodes [E][n_a][nn], or null: one more right-hand side
  double* s2out;          // its outflow response f_hat_u [E][m]
  double* s2sol;          // its volume response f_u [E][n]
  double* s2mean;         // ordinate average of f_u [E][nn]
  int pairs_form;         // EL_FORM_IN2SOL or EL_FORM_IN2MEAN
  const int32_t* emap;    // batch slot -> element index (inputs and outputs), or null
  T* fac;        // [slots][npan][npad][NB]
  T* inv;        // [slots][npan][2][NB][NB]
  int* flags;    // [0] first singular element, [1] first bad-input element
  // iterative refinement (T = float): FP64 solution panel per slot, report
  double* xbuf;       // [slots][npad][NB]: paired panel during the LU, FP64 solution during refinement
  int refine;         // FP32 factorization with FP64 refinement
  double* rel_resid;  // [E] or null
  int ir_steps;
  double ir_tol;
  int ir_cols;          // solution columns staged in LDS per residual pass (8, 4 or 2)
  const double* Tt;     // refinement: transport table transposed per ordinate [n_a][nn][nn]
};

// Entry (i, j) of the padded local matrix A (identity outside n x n), with
// i = k nn + ndi and j = kp nn + ndj already split into ordinate and node.
template <typename T>
__device__ inline T amat(const DiscDev& dv, const double* tau_e, const double* tau_s, int i, int k, int ndi, int j,
                         int kp, int ndj) {
  if (i >= dv.n || j >= dv.n) return i == j ? T(1) : T(0);
  const int nn = dv.nn;
  double v = 0.0;
  if (k == kp) {
    v = dv.T[((size_t)k * nn + ndi) * nn + ndj];
    if (ndi == ndj) v += dv.W[ndi] * tau_e[ndi];
  }
  if (ndi == ndj) v -= dv.W[ndi] * tau_s[ndi] * dv.Q[k * dv.n_a + kp];
  return (T)v;
}

// floor(i / nn) as (i inv) >> 32 with inv = floor(2^32 / nn) + 1, exact for
// 0 <= i < 2^32 / nn (i < npad)
__device__ inline int div_nn(int i, uint64_t inv) { return (int)(((uint64_t)(uint32_t)i * inv) >> 32); }

// pan[I..I+16) = Tinv * pan[I..I+16), Tinv a 16x16 block (row-major).
// Executed by one wave.
template <typename T>
__device__ inline void tri_apply(T* pan, const T* tinv, int I, int lane, int ld = LDP) {
  typedef typename Acc<T>::type A4;
  A4 c = {0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
  T a[4], b[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    a[kk] = tinv[li * NB + 4 * lk + kk];
    b[kk] = pan[(I + 4 * lk + kk) * ld + li];
  }
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) c = mfma16(a[kk], b[kk], c);
#pragma unroll
  for (int r = 0; r < 4; ++r) pan[(I + Acc<T>::row(lk, r)) * ld + li] = c[r];
}

// pan[I] = inv_I pan[I] for the 16-row blocks I in [tb, te), spread over the
// waves (the blocks are independent).  which = 0: unit-lower inverse,
// 1: upper inverse.
template <typename T>
__device__ inline void transform_blocks(T* pan, const T* inv, int which, int tb, int te, int wave, int lane,
                                        int ld = LDP) {
  for (int t = tb + wave; t < te; t += kWaves)
    tri_apply<T>(pan, inv + (size_t)t * 2 * NB * NB + which * NB * NB, 16 * t, lane, ld);
}

// Address-space-qualified pointers for the out-of-line sweep: without them
// its pointer arguments are generic and every access becomes a FLAT
// instruction, whose completion the LDS wait counter also tracks.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
using gmut = __attribute__((address_space(1))) T*;
template <typename T>
using lptr = __attribute__((address_space(3))) T*;

__device__ inline uintptr_t uniform_ptr(uintptr_t p) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
  return ((uintptr_t)hi << 32) | lo;
}

// ---- block sweeps ---------------------------------------------------------------
//
// Tile t (rows 16t..16t+16 of the LDS panel) belongs to wave w for the whole
// sweep, in slot u:
//     forward:  t = npan - 1 - (w + kWaves u)      backward:  t = w + kWaves u
// so that the tiles updated at any step are a prefix of every wave's slots
// (forward steps update the tiles below the current block, backward steps
// the tiles above it).  A step is straight-line code for a known number of
// slots (one uniform switch): read two tiles from LDS, run their MFMA chains
// interleaved, write them back.  The factor tiles (A operands, from HBM) are
// loaded two steps ahead into two register buffers, the same number of loads
// every step so that the compiler's waits are exact.

template <typename T, int MAXT>
struct FBuf {
  T f[MAXT][4];
};

// B-operand values of a 16x16 block stored row-major with row stride ld
template <typename T, typename P>
__device__ inline void load_b(T (&b)[4], P blk, int ld, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) b[kk] = blk[(4 * lk + kk) * ld + li];
}


struct SweepGeom {
  int npan, wave, nslots;
  bool down;
  __device__ int tile(int u) const { return down ? npan - 1 - (wave + kWaves * u) : wave + kWaves * u; }
  // slots updated by the step at block I
  __device__ int active(int I) const {
    if (down) {
      const int top = npan - 1 - (I / NB + 1) - wave;   // t >= I/16 + 1
      return top < 0 ? 0 : min(nslots, top / kWaves + 1);
    }
    const int te = I / NB;                             // t < I/16
    return te <= wave ? 0 : min(nslots, (te - 1 - wave) / kWaves + 1);
  }
};

// pan[tile(u)] += F.f[u] b for u < N, two tiles at a time
template <typename T, int MAXT, int N>
__device__ inline void apply_n(lptr<T> pan, const SweepGeom& g, const FBuf<T, MAXT>& F, const T (&b)[4], int lane) {
  typedef typename Acc<T>::type A4;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int u0 = 0; u0 < N; u0 += 2) {
    const int nu = (u0 + 1 < N) ? 2 : 1;
    A4 c[2];
    int base[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      if (v < nu) {
        base[v] = 16 * g.tile(u0 + v) * LDP + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) c[v][r] = pan[base[v] + Acc<T>::row(lk, r) * LDP];
      }
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int v = 0; v < 2; ++v)
        if (v < nu) c[v] = mfma16(F.f[u0 + v][kk], b[kk], c[v]);
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      if (v < nu) {
#pragma unroll
        for (int r = 0; r < 4; ++r) pan[base[v] + Acc<T>::row(lk, r) * LDP] = c[v][r];
      }
    }
  }
}

template <typename T, int MAXT>
__device__ inline void apply_active(lptr<T> pan, const SweepGeom& g, const FBuf<T, MAXT>& F, const T (&b)[4], int na,
                                    int lane) {
  switch (na) {
    case 1: apply_n<T, MAXT, 1>(pan, g, F, b, lane); break;
    case 2: if constexpr (MAXT >= 2) apply_n<T, MAXT, 2>(pan, g, F, b, lane); break;
    case 3: if constexpr (MAXT >= 3) apply_n<T, MAXT, 3>(pan, g, F, b, lane); break;
    case 4: if constexpr (MAXT >= 4) apply_n<T, MAXT, 4>(pan, g, F, b, lane); break;
    case 5: if constexpr (MAXT >= 5) apply_n<T, MAXT, 5>(pan, g, F, b, lane); break;
    case 6: if constexpr (MAXT >= 6) apply_n<T, MAXT, 6>(pan, g, F, b, lane); break;
    case 7: if constexpr (MAXT >= 7) apply_n<T, MAXT, 7>(pan, g, F, b, lane); break;
    case 8: if constexpr (MAXT >= 8) apply_n<T, MAXT, 8>(pan, g, F, b, lane); break;
    case 9: if constexpr (MAXT >= 9) apply_n<T, MAXT, 9>(pan, g, F, b, lane); break;
    case 10: if constexpr (MAXT >= 10) apply_n<T, MAXT, 10>(pan, g, F, b, lane); break;
    case 11: if constexpr (MAXT >= 11) apply_n<T, MAXT, 11>(pan, g, F, b, lane); break;
    case 12: if constexpr (MAXT >= 12) apply_n<T, MAXT, 12>(pan, g, F, b, lane); break;
    case 13: if constexpr (MAXT >= 13) apply_n<T, MAXT, 13>(pan, g, F, b, lane); break;
    default: break;
  }
}

// F.f[u] = factor rows of tile(u) for the first na slots (16-byte loads: lane
// (i, lk) holds columns 4 lk .. 4 lk + 3 of row i, the k order used by every
// MFMA in this file)
template <typename T, int MAXT, int LO, int HI>
__device__ inline void load_f_part(FBuf<T, MAXT>& F, gptr<T> fp, lptr<const int> perm, const SweepGeom& g, int na,
                                   int lane) {
  const int li = lane & 15, lk = lane >> 4;
  // Every slot is loaded (slots past na repeat slot 0's rows, which are then
  // in cache) so that each step issues the same number of loads and the
  // waits before a step's MFMAs cover only that step's tiles.  Row indices
  // first, then the loads from the uniform base with 32-bit offsets.
  uint32_t off[MAXT];
#pragma unroll
  for (int u = LO; u < HI; ++u) {
    const int t = min(max(g.tile(u < na ? u : 0), 0), g.npan - 1);
    off[u] = (uint32_t)((perm[16 * t + li] * NB + 4 * lk) * (int)sizeof(T));
  }
  gptr<char> base = reinterpret_cast<gptr<char>>(fp);
#pragma unroll
  for (int u = LO; u < HI; ++u) {
    if constexpr (sizeof(T) == 8) {
      typedef double dv2 __attribute__((ext_vector_type(2)));
      const dv2 v0 = *reinterpret_cast<gptr<dv2>>(base + off[u]);
      const dv2 v1 = *reinterpret_cast<gptr<dv2>>(base + off[u] + 16);
      F.f[u][0] = v0[0]; F.f[u][1] = v0[1]; F.f[u][2] = v1[0]; F.f[u][3] = v1[1];
    } else {
      typedef float fv4 __attribute__((ext_vector_type(4)));
      const fv4 v = *reinterpret_cast<gptr<fv4>>(base + off[u]);
      F.f[u][0] = v[0]; F.f[u][1] = v[1]; F.f[u][2] = v[2]; F.f[u][3] = v[3];
    }
  }
}

template <typename T, int MAXT>
__device__ inline void load_f(FBuf<T, MAXT>& F, gptr<T> fp, lptr<const int> perm, const SweepGeom& g, int na,
                              int lane) {
  load_f_part<T, MAXT, 0, MAXT>(F, fp, perm, g, na, lane);
}

// Block sweep over the factor panels, one barrier per step.
//   down:  steps I = I0, I0+16, ..., < Iend:  rows below I+16 += F_I pan[I]
//          (F_I = -L[:, I] inv(L_II): forward substitution with the
//          diagonal-block solves deferred to transform_blocks)
//   !down: steps I = npad-16, ..., 16:        rows above I   += F_I pan[I]
//          (F_I = -U[:, I] inv(U_II))
// All threads call it; it ends on a barrier.  Kept out of line so that its
// registers do not compete with the values live in the caller.
template <typename T, int MAXT>
__device__ __attribute__((noinline)) void sweep(T* pan_g, const T* fac_g, const int* perm_g, int npad, int I0,
                                                int Iend, bool down, int wave, int lane) {
  // the arguments are wave-uniform: say so, so that the branches below are
  // scalar (arguments of an out-of-line function arrive in vector registers)
  wave = __builtin_amdgcn_readfirstlane(wave);
  I0 = __builtin_amdgcn_readfirstlane(I0);
  Iend = __builtin_amdgcn_readfirstlane(Iend);
  npad = __builtin_amdgcn_readfirstlane(npad);
  down = __builtin_amdgcn_readfirstlane((int)down) != 0;
  gptr<T> fac = (gptr<T>)uniform_ptr(reinterpret_cast<uintptr_t>(fac_g));
  lptr<T> pan = (lptr<T>)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lptr<T>)pan_g);
  lptr<const int> perm =
      (lptr<const int>)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lptr<const int>)perm_g);
  const int npan = npad / NB;
  const int nsteps = down ? max(0, min(Iend, npad - NB) - I0 + NB - 1) / NB : npan - 1;
  if (nsteps <= 0) return;
  SweepGeom g;
  g.npan = npan;
  g.wave = wave;
  g.down = down;
  g.nslots = wave < npan ? (npan - 1 - wave) / kWaves + 1 : 0;
  auto I_of = [&](int s) { return down ? I0 + s * NB : npad - NB - s * NB; };
  auto F_of = [&](int I) { return fac + (size_t)(I / NB) * npad * NB; };
  // step index clamped to the last step: past the end the last step's tiles
  // are loaded again (cache hits), keeping the number of loads per step fixed
  auto I_cl = [&](int s) { return I_of(min(s, nsteps - 1)); };
  FBuf<T, MAXT> F0, F1;
  load_f<T, MAXT>(F0, F_of(I_cl(0)), perm, g, g.active(I_cl(0)), lane);
  load_f<T, MAXT>(F1, F_of(I_cl(1)), perm, g, g.active(I_cl(1)), lane);
  auto step = [&](int s, FBuf<T, MAXT>& Fb) {
    const int I = I_of(s);
    T b[4];
    load_b<T>(b, pan + I * LDP, LDP, lane);
    apply_active<T, MAXT>(pan, g, Fb, b, g.active(I), lane);
    load_f<T, MAXT>(Fb, F_of(I_cl(s + 2)), perm, g, g.active(I_cl(s + 2)), lane);
    __syncthreads();
  };
  for (int s = 0; s < nsteps; s += 2) {
    step(s, F0);
    if (s + 1 < nsteps) step(s + 1, F1);
  }
}

// The sweep of sweep() applied to two panels with one pass over the factor
// panels: the left panel in LDS as in sweep(), the right panel in MFMA
// accumulators, loaded from and stored back to the global scratch rs
// [npad][16] (logical row order).  Each factor tile read from HBM feeds both
// panels, halving the factor traffic (two consecutive panels of the
// left-looking factorization, or two right-hand-side panels).  The right
// panel's block row of each step (its B operand) is published through the
// LDS buffer bbuf [2][16][16] by the wave that owns it.  All threads call
// it; it ends on a barrier.
template <typename T, int MAXT, int LO, int N>
__device__ inline void apply2_n(lptr<T> pan, const SweepGeom& g, const FBuf<T, MAXT>& F, const T (&b)[4],
                                const T (&b2)[4], typename Acc<T>::type (&acc)[MAXT], int lane) {
  typedef typename Acc<T>::type A4;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int u0 = LO; u0 < LO + N; u0 += 2) {
    const int nu = (u0 + 1 < LO + N) ? 2 : 1;
    A4 c[2];
    int base[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      if (v < nu) {
        base[v] = 16 * g.tile(u0 + v) * LDP + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) c[v][r] = pan[base[v] + Acc<T>::row(lk, r) * LDP];
      }
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int v = 0; v < 2; ++v)
        if (v < nu) {
          c[v] = mfma16(F.f[u0 + v][kk], b[kk], c[v]);
          acc[u0 + v] = mfma16(F.f[u0 + v][kk], b2[kk], acc[u0 + v]);
        }
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      if (v < nu) {
#pragma unroll
        for (int r = 0; r < 4; ++r) pan[base[v] + Acc<T>::row(lk, r) * LDP] = c[v][r];
      }
    }
  }
}

// slots [LO, LO + cnt) with 0 <= cnt <= N, dispatched to straight-line code
template <typename T, int MAXT, int LO, int N>
__device__ inline void apply2_part(lptr<T> pan, const SweepGeom& g, const FBuf<T, MAXT>& F, const T (&b)[4],
                                   const T (&b2)[4], typename Acc<T>::type (&acc)[MAXT], int cnt, int lane) {
  if constexpr (N > 0) {
    if (cnt == N) apply2_n<T, MAXT, LO, N>(pan, g, F, b, b2, acc, lane);
    else apply2_part<T, MAXT, LO, N - 1>(pan, g, F, b, b2, acc, cnt, lane);
  }
}

template <typename T, int MAXT>
__device__ __attribute__((noinline)) void sweep2(T* pan_g, T* rs_g, T* bbuf_g, const T* fac_g, const int* perm_g,
                                                 int npad, int I0, int Iend, bool down, int wave, int lane) {
  typedef typename Acc<T>::type A4;
  // The right panel's accumulators take the registers of the second factor
  // buffer that sweep() uses, so the factor tiles of a step are split into
  // two halves, slots [0, H) and [H, MAXT): each half is reloaded for the
  // next step as soon as its MFMAs of this step are issued.
  constexpr int H = (MAXT + 1) / 2;
  wave = __builtin_amdgcn_readfirstlane(wave);
  I0 = __builtin_amdgcn_readfirstlane(I0);
  Iend = __builtin_amdgcn_readfirstlane(Iend);
  npad = __builtin_amdgcn_readfirstlane(npad);
  down = __builtin_amdgcn_readfirstlane((int)down) != 0;
  gptr<T> fac = (gptr<T>)uniform_ptr(reinterpret_cast<uintptr_t>(fac_g));
  gmut<T> rs = (gmut<T>)uniform_ptr(reinterpret_cast<uintptr_t>(rs_g));
  lptr<T> pan = (lptr<T>)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lptr<T>)pan_g);
  lptr<T> bbuf = (lptr<T>)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lptr<T>)bbuf_g);
  lptr<const int> perm =
      (lptr<const int>)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lptr<const int>)perm_g);
  const int npan = npad / NB;
  const int nsteps = down ? max(0, min(Iend, npad - NB) - I0 + NB - 1) / NB : npan - 1;
  const int li = lane & 15, lk = lane >> 4;
  SweepGeom g;
  g.npan = npan;
  g.wave = wave;
  g.down = down;
  g.nslots = wave < npan ? (npan - 1 - wave) / kWaves + 1 : 0;
  A4 acc[MAXT];
#pragma unroll
  for (int u = 0; u < MAXT; ++u) {
    if (u < g.nslots) {
      const int t = g.tile(u);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[u][r] = rs[(16 * t + Acc<T>::row(lk, r)) * NB + li];
    } else {
      acc[u] = A4{0, 0, 0, 0};
    }
  }
  auto I_of = [&](int s) { return down ? I0 + s * NB : npad - NB - s * NB; };
  // the wave owning the right panel's block row of step s publishes it to
  // bbuf[s & 1]
  auto publish = [&](int s) {
    const int t = I_of(s) / NB;
    const int d = down ? npan - 1 - t - wave : t - wave;
    if (d >= 0 && d % kWaves == 0) {
      const int un = d / kWaves;
      lptr<T> o = bbuf + (s & 1) * NB * NB;
#pragma unroll
      for (int u = 0; u < MAXT; ++u)
        if (u == un) {
#pragma unroll
          for (int r = 0; r < 4; ++r) o[Acc<T>::row(lk, r) * NB + li] = acc[u][r];
        }
    }
  };
  if (nsteps > 0) {
    auto F_of = [&](int s) { return fac + (size_t)(I_of(min(s, nsteps - 1)) / NB) * npad * NB; };
    auto na_of = [&](int s) { return g.active(I_of(min(s, nsteps - 1))); };
    FBuf<T, MAXT> F;
    load_f_part<T, MAXT, 0, H>(F, F_of(0), perm, g, na_of(0), lane);
    load_f_part<T, MAXT, H, MAXT>(F, F_of(0), perm, g, na_of(0), lane);
    publish(0);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
      const int I = I_of(s);
      const int na = g.active(I);
      T b[4], b2[4];
      load_b<T>(b, pan + I * LDP, LDP, lane);
      load_b<T>(b2, bbuf + (s & 1) * NB * NB, NB, lane);
      apply2_part<T, MAXT, 0, H>(pan, g, F, b, b2, acc, min(na, H), lane);
      load_f_part<T, MAXT, 0, H>(F, F_of(s + 1), perm, g, na_of(s + 1), lane);
      apply2_part<T, MAXT, H, MAXT - H>(pan, g, F, b, b2, acc, max(na - H, 0), lane);
      load_f_part<T, MAXT, H, MAXT>(F, F_of(s + 1), perm, g, na_of(s + 1), lane);
      // the next step's block row of the right panel is complete now
      if (s + 1 < nsteps) publish(s + 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int u = 0; u < MAXT; ++u) {
    if (u < g.nslots) {
      const int t = g.tile(u);
#pragma unroll
      for (int r = 0; r < 4; ++r) rs[(16 * t + Acc<T>::row(lk, r)) * NB + li] = acc[u][r];
    }
  }
  __threadfence_block();
  __syncthreads();
}

// pan = U^{-1} L^{-1} pan for a right-hand-side panel already in logical
// (pivoted) row order; the forward sweep starts at block Istart (rows above
// it are zero).  All threads of the workgroup call this; it ends on a barrier.
template <typename T, int MAXT>
__device__ inline void panel_solve(T* pan, const T* fac, const T* inv, const int* perm, int npad, int Istart,
                                   int wave, int lane) {
  const int npan = npad / NB;
  sweep<T, MAXT>(pan, fac, perm, npad, Istart, npad, true, wave, lane);
  transform_blocks<T>(pan, inv, 0, Istart / NB, npan, wave, lane);
  __syncthreads();
  sweep<T, MAXT>(pan, fac, perm, npad, 0, 0, false, wave, lane);
  transform_blocks<T>(pan, inv, 1, 0, npan, wave, lane);
  __syncthreads();
}

// panel_solve() for two right-hand-side panels at once: pan (LDS) and rs
// (global scratch [npad][NB], logical row order), both zero above block
// Istart.  All threads call it; it ends on a barrier.
template <typename T, int MAXT>
__device__ inline void panel_solve2(T* pan, T* rs, T* bbuf, const T* fac, const T* inv, const int* perm, int npad,
                                    int Istart, int wave, int lane) {
  const int npan = npad / NB;
  sweep2<T, MAXT>(pan, rs, bbuf, fac, perm, npad, Istart, npad, true, wave, lane);
  transform_blocks<T>(pan, inv, 0, Istart / NB, npan, wave, lane);
  transform_blocks<T>(rs, inv, 0, Istart / NB, npan, wave, lane, NB);
  __threadfence_block();
  __syncthreads();
  sweep2<T, MAXT>(pan, rs, bbuf, fac, perm, npad, 0, 0, false, wave, lane);
  transform_blocks<T>(pan, inv, 1, 0, npan, wave, lane);
  transform_blocks<T>(rs, inv, 1, 0, npan, wave, lane, NB);
  __threadfence_block();
  __syncthreads();
}

// Largest 64-bit value over the wave, on every lane: an inclusive max scan
// within each row of 16 lanes (DPP row shifts by 1, 2, 4, 8), then the row
// broadcasts of lanes 15 and 31, which leave the wave's maximum in lane 63.
// A lane whose shift source lies outside its row keeps its own value.
template <int CTRL, int ROWS>
__device__ inline unsigned long long dpp_u64(unsigned long long v) {
  const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xf, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xf, false);
  return ((unsigned long long)(uint32_t)h2 << 32) | (uint32_t)l2;
}
__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
  unsigned long long o;
  o = dpp_u64<0x111, 0xf>(v); v = o > v ? o : v;   // row_shr:1
  o = dpp_u64<0x112, 0xf>(v); v = o > v ? o : v;   // row_shr:2
  o = dpp_u64<0x114, 0xf>(v); v = o > v ? o : v;   // row_shr:4
  o = dpp_u64<0x118, 0xf>(v); v = o > v ? o : v;   // row_shr:8
  o = dpp_u64<0x142, 0xa>(v); v = o > v ? o : v;   // row_bcast:15 into rows 1 and 3
  o = dpp_u64<0x143, 0xc>(v); v = o > v ? o : v;   // row_bcast:31 into rows 2 and 3
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// rows per thread of factor_panel for at most kWaves * MAXT row tiles
template <int MAXT>
constexpr int kMaxRows = (kWaves * MAXT * NB + kThreads - 1) / kThreads;

// Partial-pivoting factorization of the 16 columns of the LDS panel, rows
// [J, npad) in logical order, with the rows held in registers: thread tid
// owns the rows that sit at logical positions J + tid + kThreads k when the
// panel starts (their "home"), R of them at most.  Rows never move while
// the columns are eliminated; each thread tracks the current logical
// position of its rows.  One barrier per column: every wave publishes its
// best candidate (key, position, 16 values) to its slot in cand (two sets
// of slots, alternating by column, so that a slot is rewritten only after
// every thread has passed the barrier that follows its last read); after
// the barrier all threads pick the same winner, which takes position J + c
// (the row there takes the winner's old position), and every other live row
// is eliminated by it.  The key orders candidates by |value| (the top 32
// bits of its FP64 pattern, monotonic for non-negative values), then by the
// lower home position; a NaN ranks below every number, so that a column
// without a nonzero candidate still picks a row (and is reported singular).
// On return the rows are back in pan at their final logical positions and
// perm is permuted to match.  All threads call it; it ends on a barrier.
template <typename T, int R>
__device__ __attribute__((noinline)) void factor_panel(T* pan_g, int* perm_g, T* cand_g, int* sflag_g, int J,
                                                       int npad, int tid) {
  J = __builtin_amdgcn_readfirstlane(J);
  npad = __builtin_amdgcn_readfirstlane(npad);
  lptr<T> pan = (lptr<T>)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lptr<T>)pan_g);
  lptr<int> perm = (lptr<int>)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lptr<int>)perm_g);
  lptr<T> cval = (lptr<T>)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lptr<T>)cand_g);
  lptr<unsigned long long> ckey = (lptr<unsigned long long>)(cval + 2 * kWaves * NB);
  lptr<int> cpos = (lptr<int>)(ckey + 2 * kWaves);
  const int wave = tid >> 6;
  auto key_of = [](T v, int home) -> unsigned long long {
    const double a = fabs((double)v);
    const uint32_t hi = a == a ? (uint32_t)((unsigned long long)__double_as_longlong(a) >> 32) + 2u : 1u;
    return ((unsigned long long)hi << 32) | (unsigned long long)(0xffffffffu - (uint32_t)home);
  };
  T row[R][NB];
  int pos[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int r = J + tid + kThreads * k;
    pos[k] = r < npad ? r : -1;   // -1: no row
#pragma unroll
    for (int j = 0; j < NB; ++j) row[k][j] = r < npad ? pan[r * LDP + j] : T(0);
  }
  unsigned long long best = 0ull;
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (pos[k] >= J) {
      const unsigned long long kk = key_of(row[k][0], J + tid + kThreads * k);
      best = kk > best ? kk : best;
    }
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int par = (c & 1) * kWaves;
    const unsigned long long wk = wave_max_u64(best);
    if (wk == 0ull) {
      if ((tid & 63) == 0) ckey[par + wave] = 0ull;
    } else if (best == wk) {
      // this lane holds the wave's best row
#pragma unroll
      for (int k = 0; k < R; ++k)
        if (pos[k] >= J + c && key_of(row[k][c], J + tid + kThreads * k) == wk) {
#pragma unroll
          for (int j = 0; j < NB; ++j) cval[(par + wave) * NB + j] = row[k][j];
          cpos[par + wave] = pos[k];
        }
      ckey[par + wave] = wk;
    }
    __syncthreads();
    unsigned long long gk = ckey[par];
    int gw = 0;
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
      const unsigned long long o = ckey[par + w];
      if (o > gk) { gk = o; gw = w; }
    }
    const int ghome = (int)(0xffffffffu - (uint32_t)gk);
    const int gpos = cpos[par + gw];
    // the pivot row (loops over all 16 columns with the column test inside,
    // so that their trip counts are constant before the column loop is
    // unrolled and the row arrays stay in registers)
    T pr[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) pr[j] = j >= c ? cval[(par + gw) * NB + j] : T(0);
    const T piv = pr[c];
    if (tid == 0 && !(fabs((double)piv) > 0.0)) sflag_g[0] = 1;
    const T rp = piv != T(0) ? T(1) / piv : T(0);
    best = 0ull;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int home = J + tid + kThreads * k;
      if (pos[k] >= J + c) {
        if (home == ghome) {
          pos[k] = J + c;
        } else {
          if (pos[k] == J + c) pos[k] = gpos;   // makes room for the pivot row
          const T l = row[k][c] * rp;
          row[k][c] = l;
#pragma unroll
          for (int j = 0; j < NB; ++j)
            if (j > c) row[k][j] -= l * pr[j];
          if (c + 1 < NB) {
            const unsigned long long kk = key_of(row[k][c + 1], home);
            best = kk > best ? kk : best;
          }
        }
      }
    }
  }
  // rows and perm to their final logical positions
  int pv[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int home = J + tid + kThreads * k;
    pv[k] = pos[k] >= 0 ? perm[home] : 0;
    if (pos[k] >= 0) {
#pragma unroll
      for (int j = 0; j < NB; ++j) pan[pos[k] * LDP + j] = row[k][j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (pos[k] >= 0) perm[pos[k]] = pv[k];
  __syncthreads();
}

__device__ inline void argmax_combine(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

// LDS bytes before the diagonal-block inverses (panel, permutations,
// coefficients, reduction scratch), rounded up to 16.
template <typename T>
__host__ __device__ inline size_t lds_base_bytes(int npad, int nn) {
  size_t b = sizeof(T) * (size_t)npad * LDP + 2 * sizeof(int) * (size_t)npad + 2 * sizeof(double) * nn +
             kWaves * (sizeof(double) + sizeof(int)) + 2 * sizeof(int);
  return (b + 15) / 16 * 16;
}

// FP64 residual of a solution panel for the refinement: for every equation
// q (natural order), pan[pinv[q]][c] = (-B_hat - A x)[q][c], x the FP64
// solution panel xg [npad][NB] in HBM, using the structure of A (per-ordinate
// transport blocks, node-diagonal M and S); colmax[c] = max |residual| of
// column c.  x is staged through LDS column by column (xs [XC][npad]
// doubles), XC columns at a time.  Consecutive threads take consecutive
// equations, so that the reads of x are conflict-free and those of the
// transposed transport table Tt (Tt[k][j][i] = T[k][i][j]) are coalesced.
// All threads call it; it ends on a barrier.
template <typename T, int XC>
__device__ inline void ir_residual(const LuArgs<T>& a, T* pan, const int* pinv, const int* corder, const double* tau_e,
                                   const double* tau_s, const double* xg, double* xs, unsigned long long* colmax,
                                   int npad, int P0, int tid, int64_t e, double he) {
  const DiscDev& dv = a.dv;
  const int n = dv.n, m = dv.m, nn = dv.nn, qd = dv.q, n_a = dv.n_a;
  for (int c0 = 0; c0 < NB; c0 += XC) {
    for (int idx = tid; idx < npad * XC; idx += kThreads) {
      const int r = idx / XC, c = idx % XC;
      xs[c * npad + r] = xg[r * NB + c0 + c];
    }
    // the right-hand side's nonzero of each column (one per inflow column)
    int irow[XC];
    double ival[XC];
#pragma unroll
    for (int c = 0; c < XC; ++c) {
      const int slot = P0 + c0 + c;
      irow[c] = slot < m ? dv.in_row[corder[slot]] : -1;
      ival[c] = slot < m ? dv.in_val[corder[slot]] : 0.0;
    }
    const bool src_col = a.src && P0 + c0 <= m && m < P0 + c0 + XC;
    __syncthreads();
    // running max of |residual| per column as bit patterns (a NaN beats
    // every number), reduced over the wave before one atomic per column
    unsigned long long mb[XC];
#pragma unroll
    for (int c = 0; c < XC; ++c) mb[c] = 0ull;
    for (int q = tid; q < npad; q += kThreads) {
      double acc[XC];
      if (q >= n) {
#pragma unroll
        for (int c = 0; c < XC; ++c) acc[c] = -xs[c * npad + q];
      } else {
        const int k = q / nn, nd = q - k * nn;
        const int na = nd % qd, nb = nd / qd;
        const double* Tk = a.Tt + (size_t)k * nn * nn;
        const double* xk = xs + k * nn;
#pragma unroll
        for (int c = 0; c < XC; ++c) acc[c] = 0.0;
        // the transport block row has nonzeros only at trial nodes in the
        // same node row (c', nb) or the same node column (na, d'): 2q - 1 of
        // the nn entries
#pragma unroll 4
        for (int u = 0; u < qd; ++u) {
          const int j1 = nb * qd + u;
          const double t1 = Tk[j1 * nn + nd];
#pragma unroll
          for (int c = 0; c < XC; ++c) acc[c] += t1 * xk[c * npad + j1];
          if (u != nb) {
            const int j2 = u * qd + na;
            const double t2 = Tk[j2 * nn + nd];
#pragma unroll
            for (int c = 0; c < XC; ++c) acc[c] += t2 * xk[c * npad + j2];
          }
        }
        const double wd = dv.W[nd] * tau_e[nd], ws = dv.W[nd] * tau_s[nd];
        const double* Qr = dv.Q + k * n_a;
        double sc[XC];
#pragma unroll
        for (int c = 0; c < XC; ++c) sc[c] = 0.0;
#pragma unroll 8
        for (int kp = 0; kp < n_a; ++kp) {
          const double qk = Qr[kp];
#pragma unroll
          for (int c = 0; c < XC; ++c) sc[c] += qk * xs[c * npad + kp * nn + nd];
        }
        const double sv = src_col ? 0.5 * he * dv.W[nd] * a.src[e * n + q] : 0.0;
#pragma unroll
        for (int c = 0; c < XC; ++c) {
          const double rv = q == irow[c] ? ival[c] : (src_col && P0 + c0 + c == m ? sv : 0.0);
          acc[c] = rv - (acc[c] + wd * xs[c * npad + q] - ws * sc[c]);
        }
      }
      const int i = pinv[q];
#pragma unroll
      for (int c = 0; c < XC; ++c) {
        pan[i * LDP + c0 + c] = (T)acc[c];
        const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(acc[c]));
        mb[c] = b > mb[c] ? b : mb[c];
      }
    }
#pragma unroll
    for (int c = 0; c < XC; ++c) {
      unsigned long long v = mb[c];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
      }
      if ((tid & 63) == 0) atomicMax(&colmax[c0 + c], v);
    }
    __syncthreads();
  }
}

// Tt[k][j][i] = T[k][i][j]: the transport table transposed per ordinate
__global__ void k_transpose_transport(const double* T, double* Tt, int n_a, int nn) {
  const int64_t total = (int64_t)n_a * nn * nn;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = idx / ((int64_t)nn * nn);
    const int rem = (int)(idx - k * nn * nn), i = rem / nn, j = rem - i * nn;
    Tt[(k * nn + j) * nn + i] = T[idx];
  }
}

// doubles of the per-slot global scratch: the second panel of a pair (one
// panel of doubles also holds it in FP32), plus two FP64 solution panels
// with refinement
__host__ __device__ inline size_t xbuf_doubles_per_slot(int npad, bool ir) {
  return (size_t)npad * NB * (ir ? 3 : 1);
}

template <typename T, int MAXT>
__global__ void __launch_bounds__(kThreads) k_local_lu(LuArgs<T> a) {
  typedef typename Acc<T>::type A4;
  __shared__ unsigned long long src_max;   // bits of max |source column|
  extern __shared__ __align__(16) unsigned char smem[];
  const DiscDev& dv = a.dv;
  const int npad = a.npad, mpad = a.mpad, n = dv.n, m = dv.m, nn = dv.nn;
  const int npan = npad / NB;
  const uint64_t nn_inv = (1ull << 32) / (uint64_t)nn + 1ull;
  T* pan = reinterpret_cast<T*>(smem);                                   // [npad][LDP]
  int* perm = reinterpret_cast<int*>(smem + sizeof(T) * npad * LDP);     // [npad]
  int* pinv = perm + npad;                                               // [npad]
  double* tau_e = reinterpret_cast<double*>(pinv + npad);                // [nn]
  double* tau_s = tau_e + nn;                                            // [nn]
  double* redv = tau_s + nn;                                             // [kWaves]
  int* redi = reinterpret_cast<int*>(redv + kWaves);                     // [kWaves]
  int* sflag = redi + kWaves;                                            // [2]
  T* sinv = reinterpret_cast<T*>(smem + lds_base_bytes<T>(npad, nn));    // [2][NB][NB]
  T* bbuf = sinv + 2 * NB * NB;                                          // [2][NB][NB]
  int* perm_old = reinterpret_cast<int*>(bbuf + 2 * NB * NB);             // [npad]
  // iterative refinement scratch (only allocated when a.xbuf != null)
  unsigned long long* colmax = reinterpret_cast<unsigned long long*>(
      reinterpret_cast<unsigned char*>(perm_old) + ((sizeof(int) * npad + 15) / 16) * 16);   // [2][NB]
  double* xs = reinterpret_cast<double*>(colmax + 2 * NB);                // [npad][ir_cols]
  const bool ir = sizeof(T) == 4 && a.refine;   // refinement only for the FP32 factorization
  // per slot: the second panel of a pair (T), then the FP64 solutions of the
  // refinement, one per panel of a pair
  double* slot = a.xbuf + (size_t)blockIdx.x * xbuf_doubles_per_slot(npad, ir);
  T* rs = reinterpret_cast<T*>(slot);
  double* xg = ir ? slot + npad * NB : nullptr;
  double* xg2 = ir ? slot + 2 * npad * NB : nullptr;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  T* fac = a.fac + (size_t)blockIdx.x * npan * npad * NB;
  T* inv = a.inv + (size_t)blockIdx.x * npan * 2 * NB * NB;

  for (int64_t eb = blockIdx.x; eb < a.E; eb += gridDim.x) {
    const int64_t e = a.emap ? (int64_t)a.emap[eb] : eb;
    // ---- coefficients and input check
    const double he = a.h[e];
    __syncthreads();   // every thread has read the previous element's flags
    if (tid == 0) { sflag[0] = 0; sflag[1] = 0; }
    __syncthreads();
    if (tid == 0) src_max = 0ull;
    for (int i = tid; i < nn; i += kThreads) {
      double kap = a.kappa[e * nn + i], sig = a.sigma[e * nn + i];
      bool ok = isfinite(kap) && isfinite(sig) && kap >= 0.0 && sig >= 0.0 && isfinite(he) && he > 0.0;
      if (!ok) sflag[1] = 1;
      tau_e[i] = 0.5 * he * (kap + sig);
      tau_s[i] = 0.5 * he * sig;
    }
    __syncthreads();
    if (a.src) {
      // largest entry of the source column (scale of its refinement residual)
      unsigned long long mx = 0ull;
      for (int i = tid; i < n; i += kThreads) {
        const double f = a.src[e * n + i];
        if (!isfinite(f)) sflag[1] = 1;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(0.5 * he * dv.W[i % nn] * f));
        mx = bits > mx ? bits : mx;
      }
      atomicMax(&src_max, mx);
    }
    for (int r = tid; r < npad; r += kThreads) perm[r] = r;
    __syncthreads();
    if (sflag[1]) {
      if (tid == 0) atomicMin(&a.flags[1], (int)e);
      continue;
    }

    // ---- LU panels, in pairs: the second panel of a pair rides along in
    // registers through the sweep of the first (sweep2), waits in the
    // scratch rs while the first is factored, and then only needs the update
    // by the first
    bool pending = false;   // panel J is the second of a pair, waiting in rs
    for (int J = 0; J < npad; J += NB) {
      if (!pending) {
        // generate the panel of A, rows in current logical order
        // (a thread's column c = tid % 16 is the same in all its iterations)
        const int c = tid & 15, j1 = J + c, j2 = J + NB + c;
        const int kp1 = div_nn(j1, nn_inv), kp2 = div_nn(j2, nn_inv);
        const int ndj1 = j1 - kp1 * nn, ndj2 = j2 - kp2 * nn;
        for (int idx = tid; idx < npad * NB; idx += kThreads) {
          const int r = idx >> 4, i = perm[r], k = div_nn(i, nn_inv), ndi = i - k * nn;
          pan[r * LDP + c] = amat<T>(dv, tau_e, tau_s, i, k, ndi, j1, kp1, ndj1);
        }
        const bool pair = J + NB < npad;
        if (pair) {
          for (int idx = tid; idx < npad * NB; idx += kThreads) {
            const int r = idx >> 4, i = perm[r], k = div_nn(i, nn_inv), ndi = i - k * nn;
            rs[r * NB + c] = amat<T>(dv, tau_e, tau_s, i, k, ndi, j2, kp2, ndj2);
          }
          for (int r = tid; r < npad; r += kThreads) perm_old[r] = perm[r];
          __threadfence_block();
        }
        __syncthreads();
        // left-looking update by the previous panels (their factors are stored
        // pre-multiplied: -L[:, I] inv(L_II)), then the U rows of this panel
        if (pair) sweep2<T, MAXT>(pan, rs, bbuf, fac, perm, npad, 0, J, true, wave, lane);
        else sweep<T, MAXT>(pan, fac, perm, npad, 0, J, true, wave, lane);
        pending = pair;
      } else {
        // second panel of the pair: rows of rs are in the logical order of
        // before the first panel's interchanges; physical row perm[r] sat at
        // logical row pinv_old[perm[r]] then
        for (int r = tid; r < npad; r += kThreads) pinv[perm_old[r]] = r;
        __syncthreads();
        for (int idx = tid; idx < npad * NB; idx += kThreads) {
          int r = idx >> 4, c = idx & 15;
          pan[r * LDP + c] = rs[pinv[perm[r]] * NB + c];
        }
        __syncthreads();
        // the remaining update: by the first panel of the pair
        sweep<T, MAXT>(pan, fac, perm, npad, J - NB, J, true, wave, lane);
        pending = false;
      }
      transform_blocks<T>(pan, inv, 0, 0, J / NB, wave, lane);
      // factor rows [J, npad) of the panel with partial pivoting (the rows
      // in registers; the candidate slots use bbuf, idle between sweeps)
      switch ((npad + kThreads - 1) / kThreads) {
        case 1: factor_panel<T, 1>(pan, perm, bbuf, sflag, J, npad, tid); break;
        case 2: factor_panel<T, 2>(pan, perm, bbuf, sflag, J, npad, tid); break;
        case 3: if constexpr (kMaxRows<MAXT> >= 3) factor_panel<T, 3>(pan, perm, bbuf, sflag, J, npad, tid); break;
        default: if constexpr (kMaxRows<MAXT> >= 4) factor_panel<T, 4>(pan, perm, bbuf, sflag, J, npad, tid); break;
      }
      // inverses of the unit-lower and upper diagonal blocks: lane j of wave
      // 0 computes column j of L^{-1}, lane j of wave 1 column j of U^{-1}.
      // The entries of a column above (L) or below (U) the diagonal are
      // exact zeros, so the substitutions run over full, uniform ranges
      // (no divergence) and each row of the block is read once from LDS
      // (the same address for all lanes).
      if (wave < 2 && lane < NB) {
        const T* D = pan + J * LDP;
        const int j = lane;
        T x[NB];
        if (wave == 0) {
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            T r[NB];
#pragma unroll
            for (int k = 0; k < i; ++k) r[k] = D[i * LDP + k];
            T s = (i == j) ? T(1) : T(0);
#pragma unroll
            for (int k = 0; k < i; ++k) s -= r[k] * x[k];
            x[i] = s;
          }
          T* o = inv + (size_t)(J / NB) * 2 * NB * NB;
#pragma unroll
          for (int i = 0; i < NB; ++i) { o[i * NB + j] = x[i]; sinv[i * NB + j] = x[i]; }
        } else {
#pragma unroll
          for (int ii = NB - 1; ii >= 0; --ii) {
            T r[NB];
#pragma unroll
            for (int k = ii; k < NB; ++k) r[k] = D[ii * LDP + k];
            T s = (ii == j) ? T(1) : T(0);
#pragma unroll
            for (int k = ii + 1; k < NB; ++k) s -= r[k] * x[k];
            x[ii] = (ii > j) ? T(0) : s / r[ii];
          }
          T* o = inv + (size_t)(J / NB) * 2 * NB * NB + NB * NB;
#pragma unroll
          for (int i = 0; i < NB; ++i) { o[i * NB + j] = x[i]; sinv[NB * NB + i * NB + j] = x[i]; }
        }
      }
      __syncthreads();
      // store the factor panel at the physical rows, pre-multiplied and
      // negated: rows above the diagonal block -U[r, J] inv(U_JJ), rows below
      // -L[r, J] inv(L_JJ) (the diagonal block itself is kept as inverses)
      {
        T* F = fac + (size_t)(J / NB) * npad * NB;
        const int li = lane & 15, lk = lane >> 4;
        for (int t = wave; t < npan; t += kWaves) {
          if (t == J / NB) continue;
          const T* Bi = sinv + (t < J / NB ? NB * NB : 0);
          T av[4], bv[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            av[kk] = pan[(16 * t + li) * LDP + 4 * lk + kk];
            bv[kk] = Bi[(4 * lk + kk) * NB + li];
          }
          A4 c = {0, 0, 0, 0};
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) c = mfma16(av[kk], bv[kk], c);
#pragma unroll
          for (int r = 0; r < 4; ++r) F[(size_t)perm[16 * t + Acc<T>::row(lk, r)] * NB + li] = -c[r];
        }
      }
      __threadfence_block();
      __syncthreads();
    }
    if (sflag[0]) {
      if (tid == 0) atomicMin(&a.flags[0], (int)e);
      continue;
    }
    for (int r = tid; r < npad; r += kThreads) pinv[perm[r]] = r;
    __syncthreads();
    // The inflow columns are solved in the order of the logical row of their
    // one nonzero (ties by column), so that the forward sweep of each panel
    // starts at its first column's block and later panels skip more of it:
    // slot s < m holds column corder[s] (perm_old is free after the
    // factorization; m <= npad <= kThreads * kMaxRows).
    int* corder = perm_old;
    for (int t = tid; t < m; t += kThreads) corder[t] = pinv[dv.in_row[t]];
    __syncthreads();
    {
      int rk[kMaxRows<MAXT>];
#pragma unroll
      for (int u = 0; u < kMaxRows<MAXT>; ++u) {
        const int t = tid + u * kThreads;
        rk[u] = -1;
        if (t < m) {
          const int key = corder[t];
          int rank = 0;
          for (int c2 = 0; c2 < m; ++c2) {
            const int k2 = corder[c2];
            rank += (k2 < key || (k2 == key && c2 < t)) ? 1 : 0;
          }
          rk[u] = rank;
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kMaxRows<MAXT>; ++u)
        if (rk[u] >= 0) corder[rk[u]] = tid + u * kThreads;
      __syncthreads();
    }
    // column of slot s (the source column m and the padding keep theirs)
    auto colof = [&](int slot) { return slot < m ? corder[slot] : slot; };

    // ---- right-hand side panels: X = U^{-1} L^{-1} P (-B_hat), two at a
    // time (the second in rs)
    double elem_res = 0.0;
    for (int P0 = 0; P0 < mpad;) {
      const bool two = P0 + NB < mpad;
      // column col < m: -B_hat (one nonzero); column m: the source (h/2) W f
      auto rhs = [&](int r, int slot) {
        const int col = colof(slot);
        const int q = perm[r];
        if (col < m) return q == dv.in_row[col] ? (T)dv.in_val[col] : T(0);
        if (col == m && a.src && q < n) {
          const int nd = q % nn;
          return (T)(0.5 * he * dv.W[nd] * a.src[e * n + q]);
        }
        return T(0);
      };
      for (int idx = tid; idx < npad * NB; idx += kThreads) {
        int r = idx >> 4, c = idx & 15;
        pan[r * LDP + c] = rhs(r, P0 + c);
        if (two) rs[r * NB + c] = rhs(r, P0 + NB + c);
      }
      // first nonzero logical row of the panel(s)
      if (tid == 0) {
        int mn = npad;
        for (int c = 0; c < (two ? 2 * NB : NB); ++c) {
          if (P0 + c < m) mn = min(mn, pinv[dv.in_row[colof(P0 + c)]]);
          else if (P0 + c == m && a.src) mn = 0;   // dense column
        }
        sflag[1] = (mn / NB) * NB;
      }
      __threadfence_block();
      __syncthreads();
      if (two) panel_solve2<T, MAXT>(pan, rs, bbuf, fac, inv, perm, npad, sflag[1], wave, lane);
      else panel_solve<T, MAXT>(pan, fac, inv, perm, npad, sflag[1], wave, lane);
      if (ir) {
        // FP64 solution panels in HBM, refined with FP64 residuals and FP32
        // corrections (both panels of a pair until both meet the tolerance)
        for (int idx = tid; idx < npad * NB; idx += kThreads) {
          int r = idx >> 4, c = idx & 15;
          xg[r * NB + c] = (double)pan[r * LDP + c];
          if (two) xg2[r * NB + c] = (double)rs[r * NB + c];
        }
        __threadfence_block();
        __syncthreads();
        auto residual = [&](const double* x, unsigned long long* cm, int p0) {
          if (a.ir_cols == 8) ir_residual<T, 8>(a, pan, pinv, corder, tau_e, tau_s, x, xs, cm, npad, p0, tid, e, he);
          else if (a.ir_cols == 4)
            ir_residual<T, 4>(a, pan, pinv, corder, tau_e, tau_s, x, xs, cm, npad, p0, tid, e, he);
          else ir_residual<T, 2>(a, pan, pinv, corder, tau_e, tau_s, x, xs, cm, npad, p0, tid, e, he);
        };
        auto worst_of = [&](const unsigned long long* cm, int p0) {
          double w = 0.0;
          for (int c = 0; c < NB; ++c) {
            const double r = __longlong_as_double((long long)cm[c]);
            if (p0 + c < m) w = fmax(w, r / dv.in_val[colof(p0 + c)]);
            else if (p0 + c == m && a.src) w = fmax(w, r / fmax(__longlong_as_double((long long)src_max), 1e-300));
          }
          return w;
        };
        for (int it = 0;; ++it) {
          if (tid < 2 * NB) colmax[tid] = 0ull;
          __syncthreads();
          if (two) {
            // the second panel's residual goes to rs, then the first's to pan
            residual(xg2, colmax + NB, P0 + NB);
            for (int idx = tid; idx < npad * NB; idx += kThreads) rs[idx] = pan[(idx >> 4) * LDP + (idx & 15)];
            __threadfence_block();
            __syncthreads();
          }
          residual(xg, colmax, P0);
          const double worst = two ? fmax(worst_of(colmax, P0), worst_of(colmax + NB, P0 + NB)) : worst_of(colmax, P0);
          if (worst <= a.ir_tol || it >= a.ir_steps) {
            elem_res = fmax(elem_res, worst);
            break;
          }
          if (two) panel_solve2<T, MAXT>(pan, rs, bbuf, fac, inv, perm, npad, 0, wave, lane);
          else panel_solve<T, MAXT>(pan, fac, inv, perm, npad, 0, wave, lane);
          for (int idx = tid; idx < npad * NB; idx += kThreads) {
            int r = idx >> 4, c = idx & 15;
            xg[r * NB + c] += (double)pan[r * LDP + c];
            if (two) xg2[r * NB + c] += (double)rs[r * NB + c];
          }
          __threadfence_block();
          __syncthreads();
        }
      }
      // outputs (pan rows are volume DOFs in natural order)
      for (int half = 0; half < (two ? 2 : 1); ++half) {
        const double* xsol = half == 0 ? xg : xg2;   // refined FP64 solution (with ir)
        if (half == 1) {
          // the second panel's solution: rs -> pan
          __syncthreads();
          if (!ir)
            for (int idx = tid; idx < npad * NB; idx += kThreads) pan[(idx >> 4) * LDP + (idx & 15)] = rs[idx];
          __syncthreads();
          P0 += NB;
        }
        const bool pairs_sol = a.pairs && a.pairs_form == EL_FORM_IN2SOL;
        const bool pairs_mean = a.pairs && a.pairs_form == EL_FORM_IN2MEAN;
        const int64_t n_out = (int64_t)m * m + (int64_t)(pairs_mean ? nn : n) * m;
        if (a.in2sol || a.b_i2s || a.f_i2s || a.h_i2s || pairs_sol) {
          for (int idx = tid; idx < n * NB; idx += kThreads) {
            int r = idx >> 4, c = idx & 15;
            if (P0 + c < m) {
              const double v = ir ? xsol[r * NB + c] : (double)pan[r * LDP + c];
              const int col = colof(P0 + c);
              const int64_t o = ((int64_t)e * n + r) * m + col;
              if (a.in2sol) a.in2sol[o] = v;
              if (a.b_i2s) a.b_i2s[o] = gemm::f2bf((float)v);
              if (a.f_i2s) a.f_i2s[o] = (float)v;
              if (a.h_i2s) a.h_i2s[o] = (_Float16)(float)v;
              if (pairs_sol) a.pairs[(int64_t)e * n_out + (int64_t)m * m + (int64_t)r * m + col] = gemm::f2bf((float)v);
            }
          }
        }
        if (a.in2out || a.b_i2o || a.f_i2o || a.h_i2o || a.pairs) {
          for (int idx = tid; idx < m * NB; idx += kThreads) {
            int r = idx >> 4, c = idx & 15;
            if (P0 + c < m) {
              const double v = ir ? xsol[dv.out_row[r] * NB + c] : (double)pan[dv.out_row[r] * LDP + c];
              const int col = colof(P0 + c);
              const int64_t o = ((int64_t)e * m + r) * m + col;
              if (a.in2out) a.in2out[o] = v;
              if (a.b_i2o) a.b_i2o[o] = gemm::f2bf((float)v);
              if (a.f_i2o) a.f_i2o[o] = (float)v;
              if (a.h_i2o) a.h_i2o[o] = (_Float16)(float)v;
              if (a.pairs) a.pairs[(int64_t)e * n_out + (int64_t)r * m + col] = gemm::f2bf((float)v);
            }
          }
        }
        if (a.src && P0 <= m && m < P0 + NB) {
          // the source column: f_u, its outflow rows, its ordinate average
          const int c = m - P0;
          auto val = [&](int r) { return ir ? xsol[r * NB + c] : (double)pan[r * LDP + c]; };
          if (a.s2sol)
            for (int r = tid; r < n; r += kThreads) a.s2sol[(int64_t)e * n + r] = val(r);
          if (a.s2out)
            for (int r = tid; r < m; r += kThreads) a.s2out[(int64_t)e * m + r] = val(dv.out_row[r]);
          if (a.s2mean)
            for (int r = tid; r < nn; r += kThreads) {
              double acc = 0.0;
              for (int k = 0; k < dv.n_a; ++k) acc += val(k * nn + r);
              a.s2mean[(int64_t)e * nn + r] = acc / dv.n_a;
            }
        }
        if (a.in2mean || a.b_i2m || a.f_i2m || a.h_i2m || pairs_mean) {
          const double s = 1.0 / dv.n_a;
          for (int idx = tid; idx < nn * NB; idx += kThreads) {
            int r = idx >> 4, c = idx & 15;
            if (P0 + c < m) {
              double acc = 0.0;
              for (int k = 0; k < dv.n_a; ++k)
                acc += ir ? xsol[(k * nn + r) * NB + c] : (double)pan[(k * nn + r) * LDP + c];
              const double v = acc * s;
              const int col = colof(P0 + c);
              const int64_t o = ((int64_t)e * nn + r) * m + col;
              if (a.in2mean) a.in2mean[o] = v;
              if (a.b_i2m) a.b_i2m[o] = gemm::f2bf((float)v);
              if (a.f_i2m) a.f_i2m[o] = (float)v;
              if (a.h_i2m) a.h_i2m[o] = (_Float16)(float)v;
              if (pairs_mean) a.pairs[(int64_t)e * n_out + (int64_t)m * m + (int64_t)r * m + col] = gemm::f2bf((float)v);
            }
          }
        }
      }
      __syncthreads();
      P0 += NB;
    }
    if (ir && tid == 0 && a.rel_resid) a.rel_resid[e] = elem_res;
  }
}

__global__ void k_fill_double(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_int(int* p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
size_t lu_smem_bytes(int npad, int nn, int ir_cols) {
  size_t b = lds_base_bytes<T>(npad, nn) + sizeof(T) * 4 * NB * NB + ((sizeof(int) * (size_t)npad + 15) / 16) * 16;
  if (ir_cols) b += 2 * NB * sizeof(unsigned long long) + sizeof(double) * (size_t)npad * ir_cols;
  return b + 16;
}

}  // namespace

namespace {

struct LocalOut {
  double* in2out = nullptr;
  double* in2sol = nullptr;
  double* in2mean = nullptr;
  uint16_t* b_i2o = nullptr;
  uint16_t* b_i2s = nullptr;
  float* f_i2o = nullptr;
  float* f_i2s = nullptr;
  uint16_t* b_i2m = nullptr;
  float* f_i2m = nullptr;
  _Float16* h_i2o = nullptr;
  _Float16* h_i2s = nullptr;
  _Float16* h_i2m = nullptr;
  uint16_t* pairs = nullptr;
  int pairs_form = EL_FORM_IN2SOL;
  const int32_t* emap = nullptr;
  const double* src = nullptr;
  double* s2out = nullptr;
  double* s2sol = nullptr;
  double* s2mean = nullptr;
};

template <typename T>
el_status run_local_t(el_ctx* ctx, el_ctx::DiscEntry* de, bool ir, int64_t E, const double* h,
                      const double* kappa, const double* sigma, const LocalOut& out, double* rel_resid) {
  const DiscHost& dh = de->host;
  const int npad = (dh.n + NB - 1) / NB * NB;
  // the source, if any, is right-hand side column m
  const int mpad = (dh.m + (out.src ? 1 : 0) + NB - 1) / NB * NB;
  if (rel_resid) {
    hipLaunchKernelGGL(k_fill_double, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, ctx->stream, rel_resid, E, 0.0);
  }
  int max_smem = 0;
  hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device);
  // refinement: stage as many solution columns per residual pass as fit
  int ir_cols = 0;
  if (ir) {
    for (int c : {8, 4, 2})
      if (lu_smem_bytes<T>(npad, dh.nn, c) <= (size_t)max_smem) { ir_cols = c; break; }
    if (!ir_cols) ir_cols = 2;
  }
  size_t smem = lu_smem_bytes<T>(npad, dh.nn, ir_cols);
  if ((int)smem > max_smem) {
    std::ostringstream os;
    os << "el_local_solve: n = " << dh.n << " needs " << smem << " B of LDS (limit " << max_smem << ")";
    return set_error(ctx, EL_ERR_ARG, os.str());
  }
  const int npan = npad / NB;
  const int64_t slots = std::min<int64_t>(E, (int64_t)ctx->num_cus * 2);
  size_t fac_bytes = sizeof(T) * (size_t)slots * npan * npad * NB;
  size_t inv_bytes = sizeof(T) * (size_t)slots * npan * 2 * NB * NB;
  size_t x_bytes = sizeof(double) * (size_t)slots * xbuf_doubles_per_slot(npad, ir);
  // refinement: the transport table transposed per ordinate, after xbuf
  const size_t x_off = (fac_bytes + inv_bytes + 255) / 256 * 256;
  const size_t tt_off = (x_off + x_bytes + 255) / 256 * 256;
  const size_t tt_bytes = ir ? sizeof(double) * (size_t)dh.n_a * dh.nn * dh.nn : 0;
  el_status st = ensure_ws(ctx, ctx->ws_local, tt_off + tt_bytes + 256);
  if (st) return st;
  st = ensure_ws(ctx, ctx->ws_small, 8192);
  if (st) return st;
  int* flags = reinterpret_cast<int*>(ctx->ws_small.ptr);
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, ctx->stream, flags, 2, INT_MAX);
  LuArgs<T> args;
  args.dv = de->view;
  args.E = E;
  args.npad = npad;
  args.mpad = mpad;
  args.h = h; args.kappa = kappa; args.sigma = sigma;
  args.in2out = out.in2out; args.in2sol = out.in2sol; args.in2mean = out.in2mean;
  args.b_i2o = out.b_i2o; args.b_i2s = out.b_i2s; args.pairs = out.pairs; args.emap = out.emap;
  args.f_i2o = out.f_i2o; args.f_i2s = out.f_i2s;
  args.b_i2m = out.b_i2m; args.f_i2m = out.f_i2m; args.pairs_form = out.pairs_form;
  args.h_i2o = out.h_i2o; args.h_i2s = out.h_i2s; args.h_i2m = out.h_i2m;
  args.src = out.src; args.s2out = out.s2out; args.s2sol = out.s2sol; args.s2mean = out.s2mean;
  char* base = reinterpret_cast<char*>(ctx->ws_local.ptr);
  args.fac = reinterpret_cast<T*>(base);
  args.inv = reinterpret_cast<T*>(base + fac_bytes);
  args.xbuf = reinterpret_cast<double*>(base + x_off);
  args.Tt = nullptr;
  if (ir) {
    double* tt = reinterpret_cast<double*>(base + tt_off);
    const int64_t total = (int64_t)dh.n_a * dh.nn * dh.nn;
    hipLaunchKernelGGL(k_transpose_transport, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 1024)), dim3(256),
                       0, ctx->stream, de->view.T, tt, dh.n_a, dh.nn);
    args.Tt = tt;
  }
  args.refine = ir ? 1 : 0;
  args.rel_resid = rel_resid;
  args.ir_steps = 3;
  args.ir_tol = 1e-13;
  args.ir_cols = ir_cols;
  args.flags = flags;
  // tiles per wave in a sweep step: ceil(npan / kWaves), rounded up to an
  // instantiated size
  const int need = (npan + kWaves - 1) / kWaves;
  auto pick = [&]() -> void (*)(LuArgs<T>) {
    if (need <= 1) return k_local_lu<T, 1>;
    if (need <= 2) return k_local_lu<T, 2>;
    if (need <= 4) return k_local_lu<T, 4>;
    if (need <= 7) return k_local_lu<T, 7>;
    if (need <= 10) return k_local_lu<T, 10>;
    if constexpr (sizeof(T) == 4) {
      if (need <= 13) return k_local_lu<T, 13>;
    }
    return nullptr;
  };
  void (*kern)(LuArgs<T>) = pick();
  if (!kern) {
    std::ostringstream os;
    os << "el_local_solve: n = " << dh.n << " is too large for this precision";
    return set_error(ctx, EL_ERR_ARG, os.str());
  }
  hipError_t he = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)smem);
  if (he != hipSuccess) return hip_check(ctx, he, "hipFuncSetAttribute(k_local_lu)");
  hipLaunchKernelGGL(kern, dim3((unsigned)slots), dim3(kThreads), smem, ctx->stream, args);
  he = hipGetLastError();
  if (he != hipSuccess) return hip_check(ctx, he, "launch k_local_lu");
  int hflags[2];
  he = hipMemcpyAsync(hflags, flags, sizeof hflags, hipMemcpyDeviceToHost, ctx->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return hip_check(ctx, he, "el_local_solve");
  if (hflags[1] != INT_MAX) {
    std::ostringstream os;
    os << "el_local_solve: non-finite or negative coefficient (or h <= 0) at element " << hflags[1];
    return set_error(ctx, EL_ERR_NONFINITE, os.str());
  }
  if (hflags[0] != INT_MAX) {
    std::ostringstream os;
    os << "el_local_solve: zero pivot (singular local matrix) at element " << hflags[0];
    return set_error(ctx, EL_ERR_SINGULAR, os.str());
  }
  return EL_OK;
}

el_status run_local(el_ctx* ctx, el_ctx::DiscEntry* de, int precision, int64_t E, const double* h,
                    const double* kappa, const double* sigma, const LocalOut& out, double* rel_resid) {
  if (precision == EL_FP32_IR) return run_local_t<float>(ctx, de, true, E, h, kappa, sigma, out, rel_resid);
  return run_local_t<double>(ctx, de, false, E, h, kappa, sigma, out, rel_resid);
}

}  // namespace

bool local_fp64_fits(el_ctx* ctx, el_ctx::DiscEntry* de) {
  int max_smem = 0;
  hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device);
  const int npad = (de->host.n + NB - 1) / NB * NB;
  return lu_smem_bytes<double>(npad, de->host.nn, 0) <= (size_t)max_smem &&
         (npad / NB + kWaves - 1) / kWaves <= 10;
}

el_status launch_local_solve(el_ctx* ctx, el_ctx::DiscEntry* de, int precision, int64_t E,
                             const double* h, const double* kappa, const double* sigma,
                             double* in2out, double* in2sol, double* in2mean, double* rel_resid,
                             const double* src, double* s2out, double* s2sol, double* s2mean) {
  LocalOut o;
  o.in2out = in2out; o.in2sol = in2sol; o.in2mean = in2mean;
  o.src = src; o.s2out = s2out; o.s2sol = s2sol; o.s2mean = s2mean;
  return run_local(ctx, de, precision, E, h, kappa, sigma, o, rel_resid);
}

el_status launch_local_solve_ex(el_ctx* ctx, el_ctx::DiscEntry* de, int precision, int64_t E, const double* h,
                                const double* kappa, const double* sigma, const int32_t* emap, void* o_i2o,
                                void* o_i2v, int form, int out_dtype, uint16_t* pairs) {
  LocalOut o;
  const bool mean = form == EL_FORM_IN2MEAN;
  if (out_dtype == EL_F32) {
    o.f_i2o = reinterpret_cast<float*>(o_i2o);
    (mean ? o.f_i2m : o.f_i2s) = reinterpret_cast<float*>(o_i2v);
  } else if (out_dtype == EL_F16) {
    o.h_i2o = reinterpret_cast<_Float16*>(o_i2o);
    (mean ? o.h_i2m : o.h_i2s) = reinterpret_cast<_Float16*>(o_i2v);
  } else {
    o.b_i2o = reinterpret_cast<uint16_t*>(o_i2o);
    (mean ? o.b_i2m : o.b_i2s) = reinterpret_cast<uint16_t*>(o_i2v);
  }
  o.pairs = pairs; o.pairs_form = form; o.emap = emap;
  return run_local(ctx, de, precision, E, h, kappa, sigma, o, nullptr);
}

}  // namespace el

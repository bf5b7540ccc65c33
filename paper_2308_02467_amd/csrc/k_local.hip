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
//    kept in LDS, so reading the factors through perm gives the
//    LAPACK-ordered L and U;
//  * the block updates pan[I+16:] -= L[I+16:, I] * U[I, panel] run on the
//    FP64 matrix cores (v_mfma_f64_16x16x4f64), L streamed from HBM, U and
//    the panel from LDS; triangular diagonal blocks are applied as products
//    with their precomputed inverses (also on the matrix cores);
//  * the right-hand side -B_hat (one nonzero per column) is generated in
//    panels of 16 columns, forward-substituted (skipping the leading zero
//    blocks) and back-substituted in LDS, and the solution panel is written
//    straight to in2sol / in2out / in2mean.
#include <climits>
#include <cstdio>
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
  uint16_t* pairs;        // bfloat16 (in2out, in2sol) [E][m*m + n*m]
  const int32_t* emap;    // batch slot -> element index (inputs and outputs), or null
  T* fac;        // [slots][npan][npad][NB]
  T* inv;        // [slots][npan][2][NB][NB]
  int* flags;    // [0] first singular element, [1] first bad-input element
  // iterative refinement (T = float): FP64 solution panel per slot, report
  double* xbuf;       // [slots][npad][NB] or null
  double* rel_resid;  // [E] or null
  int ir_steps;
  double ir_tol;
};

// Entry (i, j) of the padded local matrix A (identity outside n x n).
template <typename T>
__device__ inline T amat(const DiscDev& dv, const double* tau_e, const double* tau_s, int i, int j) {
  if (i >= dv.n || j >= dv.n) return i == j ? T(1) : T(0);
  const int nn = dv.nn;
  const int k = i / nn, ndi = i - k * nn;
  const int kp = j / nn, ndj = j - kp * nn;
  double v = 0.0;
  if (k == kp) {
    v = dv.T[((size_t)k * nn + ndi) * nn + ndj];
    if (ndi == ndj) v += dv.W[ndi] * tau_e[ndi];
  }
  if (ndi == ndj) v -= dv.W[ndi] * tau_s[ndi] * dv.Q[k * dv.n_a + kp];
  return (T)v;
}

// pan[I..I+16) = Tinv * pan[I..I+16), Tinv a 16x16 block in global memory
// (row-major).  Executed by one wave.
template <typename T>
__device__ inline void tri_apply(T* pan, const T* tinv, int I, int lane) {
  typedef typename Acc<T>::type A4;
  A4 c = {0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
  T a[4], b[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    a[kk] = tinv[li * NB + 4 * kk + lk];
    b[kk] = pan[(I + 4 * kk + lk) * LDP + li];
  }
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) c = mfma16(a[kk], b[kk], c);
#pragma unroll
  for (int r = 0; r < 4; ++r) pan[(I + Acc<T>::row(lk, r)) * LDP + li] = c[r];
}

// pan[rows of tiles t in [t_begin, t_end)] -= F[perm[row]][0..16) * pan[I..I+16)
// F = one factor panel (physical rows, 16 columns), read from HBM.
template <typename T>
__device__ inline void block_update(T* pan, const T* __restrict__ F, const int* perm, int I,
                                    int t_begin, int t_end, int wave, int lane) {
  typedef typename Acc<T>::type A4;
  const int li = lane & 15, lk = lane >> 4;
  T b[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) b[kk] = pan[(I + 4 * kk + lk) * LDP + li];
  int t = t_begin + wave;
  // two tiles per iteration to keep more loads in flight
  for (; t + kWaves < t_end; t += 2 * kWaves) {
    const int t2 = t + kWaves;
    const T* r0 = F + (size_t)perm[16 * t + li] * NB + lk;
    const T* r1 = F + (size_t)perm[16 * t2 + li] * NB + lk;
    T a0[4], a1[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) { a0[kk] = -r0[4 * kk]; a1[kk] = -r1[4 * kk]; }
    A4 c0, c1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      c0[r] = pan[(16 * t + Acc<T>::row(lk, r)) * LDP + li];
      c1[r] = pan[(16 * t2 + Acc<T>::row(lk, r)) * LDP + li];
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) { c0 = mfma16(a0[kk], b[kk], c0); c1 = mfma16(a1[kk], b[kk], c1); }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      pan[(16 * t + Acc<T>::row(lk, r)) * LDP + li] = c0[r];
      pan[(16 * t2 + Acc<T>::row(lk, r)) * LDP + li] = c1[r];
    }
  }
  if (t < t_end) {
    const T* r0 = F + (size_t)perm[16 * t + li] * NB + lk;
    T a0[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) a0[kk] = -r0[4 * kk];
    A4 c0;
#pragma unroll
    for (int r = 0; r < 4; ++r) c0[r] = pan[(16 * t + Acc<T>::row(lk, r)) * LDP + li];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) c0 = mfma16(a0[kk], b[kk], c0);
#pragma unroll
    for (int r = 0; r < 4; ++r) pan[(16 * t + Acc<T>::row(lk, r)) * LDP + li] = c0[r];
  }
}

// pan = U^{-1} L^{-1} pan for a right-hand-side panel already in logical
// (pivoted) row order; the forward sweep starts at block Istart (rows above
// it are zero).  All threads of the workgroup call this.
template <typename T>
__device__ inline void panel_solve(T* pan, const T* fac, const T* inv, const int* perm, int npad, int Istart,
                                   int wave, int lane) {
  for (int I = Istart; I < npad; I += NB) {
    if (wave == 0) tri_apply<T>(pan, inv + (size_t)(I / NB) * 2 * NB * NB, I, lane);
    __syncthreads();
    if (I + NB < npad) {
      block_update<T>(pan, fac + (size_t)(I / NB) * npad * NB, perm, I, (I + NB) / 16, npad / 16, wave, lane);
      __syncthreads();
    }
  }
  for (int I = npad - NB; I >= 0; I -= NB) {
    if (wave == 0) tri_apply<T>(pan, inv + (size_t)(I / NB) * 2 * NB * NB + NB * NB, I, lane);
    __syncthreads();
    if (I > 0) {
      block_update<T>(pan, fac + (size_t)(I / NB) * npad * NB, perm, I, 0, I / 16, wave, lane);
      __syncthreads();
    }
  }
}

__device__ inline void argmax_combine(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_local_lu(LuArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const DiscDev& dv = a.dv;
  const int npad = a.npad, mpad = a.mpad, n = dv.n, m = dv.m, nn = dv.nn;
  const int npan = npad / NB;
  T* pan = reinterpret_cast<T*>(smem);                                   // [npad][LDP]
  int* perm = reinterpret_cast<int*>(smem + sizeof(T) * npad * LDP);     // [npad]
  int* pinv = perm + npad;                                               // [npad]
  double* tau_e = reinterpret_cast<double*>(pinv + npad);                // [nn]
  double* tau_s = tau_e + nn;                                            // [nn]
  double* redv = tau_s + nn;                                             // [kWaves]
  int* redi = reinterpret_cast<int*>(redv + kWaves);                     // [kWaves]
  int* sflag = redi + kWaves;                                            // [2]
  // iterative refinement scratch (only allocated when a.xbuf != null)
  unsigned long long* colmax = reinterpret_cast<unsigned long long*>(
      smem + ((sizeof(T) * npad * LDP + 2 * sizeof(int) * npad + 2 * sizeof(double) * nn +
               kWaves * (sizeof(double) + sizeof(int)) + 2 * sizeof(int) + 15) / 16) * 16);   // [NB]
  double* xs = reinterpret_cast<double*>(colmax + NB);                    // [npad][8]
  const bool ir = a.xbuf != nullptr;
  double* xg = ir ? a.xbuf + (size_t)blockIdx.x * npad * NB : nullptr;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  T* fac = a.fac + (size_t)blockIdx.x * npan * npad * NB;
  T* inv = a.inv + (size_t)blockIdx.x * npan * 2 * NB * NB;

  for (int64_t eb = blockIdx.x; eb < a.E; eb += gridDim.x) {
    const int64_t e = a.emap ? (int64_t)a.emap[eb] : eb;
    // ---- coefficients and input check
    const double he = a.h[e];
    __syncthreads();   // every thread has read the previous element's flags
    if (tid == 0) { sflag[0] = 0; sflag[1] = 0; }
    __syncthreads();
    for (int i = tid; i < nn; i += kThreads) {
      double kap = a.kappa[e * nn + i], sig = a.sigma[e * nn + i];
      bool ok = isfinite(kap) && isfinite(sig) && kap >= 0.0 && sig >= 0.0 && isfinite(he) && he > 0.0;
      if (!ok) sflag[1] = 1;
      tau_e[i] = 0.5 * he * (kap + sig);
      tau_s[i] = 0.5 * he * sig;
    }
    for (int r = tid; r < npad; r += kThreads) perm[r] = r;
    __syncthreads();
    if (sflag[1]) {
      if (tid == 0) atomicMin(&a.flags[1], (int)e);
      continue;
    }

    // ---- LU panels
    for (int J = 0; J < npad; J += NB) {
      // generate the panel of A, rows in current logical order
      for (int idx = tid; idx < npad * NB; idx += kThreads) {
        int r = idx >> 4, c = idx & 15;
        pan[r * LDP + c] = amat<T>(dv, tau_e, tau_s, perm[r], J + c);
      }
      __syncthreads();
      for (int I = 0; I < J; I += NB) {
        if (wave == 0) tri_apply<T>(pan, inv + (size_t)(I / NB) * 2 * NB * NB, I, lane);
        __syncthreads();
        block_update<T>(pan, fac + (size_t)(I / NB) * npad * NB, perm, I, (I + NB) / 16, npad / 16, wave, lane);
        __syncthreads();
      }
      // factor rows [J, npad) of the panel with partial pivoting
      double best = -1.0;
      int bidx = INT_MAX;
      for (int r = J + tid; r < npad; r += kThreads) {
        double v = fabs((double)pan[r * LDP]);
        if (v > best) { best = v; bidx = r; }
      }
      for (int c = 0; c < NB; ++c) {
        const int col = J + c;
        for (int off = 32; off > 0; off >>= 1) {
          double v2 = __shfl_xor(best, off);
          int i2 = __shfl_xor(bidx, off);
          argmax_combine(best, bidx, v2, i2);
        }
        if (lane == 0) { redv[wave] = best; redi[wave] = bidx; }
        __syncthreads();
        double gv = redv[0];
        int gi = redi[0];
        for (int w = 1; w < kWaves; ++w) argmax_combine(gv, gi, redv[w], redi[w]);
        if (gi < col || gi >= npad) { gi = col; gv = 0.0; }   // NaN column: no candidate
        if (gi != col) {
          if (tid < NB) {
            T tmp = pan[col * LDP + tid];
            pan[col * LDP + tid] = pan[gi * LDP + tid];
            pan[gi * LDP + tid] = tmp;
          }
          if (tid == NB) { int tp = perm[col]; perm[col] = perm[gi]; perm[gi] = tp; }
        }
        if (tid == 0 && !(gv > 0.0)) sflag[0] = 1;
        __syncthreads();
        const T piv = pan[col * LDP + c];
        const T rp = piv != T(0) ? T(1) / piv : T(0);
        best = -1.0;
        bidx = INT_MAX;
        for (int r = col + 1 + tid; r < npad; r += kThreads) {
          T* row = pan + r * LDP;
          T l = row[c] * rp;
          row[c] = l;
#pragma unroll
          for (int j = 0; j < NB; ++j)
            if (j > c) row[j] -= l * pan[col * LDP + j];
          if (c + 1 < NB) {
            double v = fabs((double)row[c + 1]);
            if (v > best) { best = v; bidx = r; }
          }
        }
      }
      __syncthreads();
      // inverses of the unit-lower and upper diagonal blocks (wave 0:
      // lanes 0..15 columns of L^{-1}, lanes 16..31 columns of U^{-1})
      if (wave == 0 && lane < 32) {
        const T* D = pan + J * LDP;
        T x[NB];
        const int j = lane & 15;
        if (lane < 16) {
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            T s = (i == j) ? T(1) : T(0);
            if (i > j) {
#pragma unroll
              for (int k = 0; k < NB; ++k)
                if (k >= j && k < i) s -= D[i * LDP + k] * x[k];
            }
            x[i] = (i < j) ? T(0) : s;
          }
          T* o = inv + (size_t)(J / NB) * 2 * NB * NB;
#pragma unroll
          for (int i = 0; i < NB; ++i) o[i * NB + j] = x[i];
        } else {
#pragma unroll
          for (int ii = NB - 1; ii >= 0; --ii) {
            T s = (ii == j) ? T(1) : T(0);
#pragma unroll
            for (int k = 0; k < NB; ++k)
              if (k > ii && k <= j) s -= D[ii * LDP + k] * x[k];
            x[ii] = (ii > j) ? T(0) : s / D[ii * LDP + ii];
          }
          T* o = inv + (size_t)(J / NB) * 2 * NB * NB + NB * NB;
#pragma unroll
          for (int i = 0; i < NB; ++i) o[i * NB + j] = x[i];
        }
      }
      // store the factored panel at the physical rows
      {
        T* F = fac + (size_t)(J / NB) * npad * NB;
        for (int idx = tid; idx < npad * NB; idx += kThreads) {
          int r = idx >> 4, c = idx & 15;
          F[(size_t)perm[r] * NB + c] = pan[r * LDP + c];
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

    // ---- right-hand side panels: X = U^{-1} L^{-1} P (-B_hat)
    double elem_res = 0.0;
    for (int P0 = 0; P0 < mpad; P0 += NB) {
      for (int idx = tid; idx < npad * NB; idx += kThreads) {
        int r = idx >> 4, c = idx & 15;
        int col = P0 + c;
        T v = T(0);
        if (col < m && perm[r] == dv.in_row[col]) v = (T)dv.in_val[col];
        pan[r * LDP + c] = v;
      }
      // first nonzero logical row of the panel
      if (tid == 0) {
        int mn = npad;
        for (int c = 0; c < NB; ++c)
          if (P0 + c < m) mn = min(mn, pinv[dv.in_row[P0 + c]]);
        sflag[1] = (mn / NB) * NB;
      }
      __syncthreads();
      panel_solve<T>(pan, fac, inv, perm, npad, sflag[1], wave, lane);
      if (ir) {
        // FP64 solution panel in HBM, refined with FP64 residuals and FP32 corrections
        for (int idx = tid; idx < npad * NB; idx += kThreads) {
          int r = idx >> 4, c = idx & 15;
          xg[r * NB + c] = (double)pan[r * LDP + c];
        }
        __threadfence_block();
        __syncthreads();
        for (int it = 0;; ++it) {
          if (tid < NB) colmax[tid] = 0ull;
          __syncthreads();
          for (int half = 0; half < 2; ++half) {
            for (int idx = tid; idx < npad * 8; idx += kThreads) {
              int r = idx >> 3, c = idx & 7;
              xs[idx] = xg[r * NB + half * 8 + c];
            }
            __syncthreads();
            for (int i = tid; i < npad; i += kThreads) {
              const int q = perm[i];
              double acc[8];
              if (q >= n) {
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] = -xs[q * 8 + c];
              } else {
                const int k = q / nn, nd = q - k * nn;
                const double* Trow = dv.T + ((size_t)k * nn + nd) * nn;
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] = 0.0;
                for (int j = 0; j < nn; ++j) {
                  const double t = Trow[j];
                  if (t != 0.0) {
                    const double* xr = xs + (k * nn + j) * 8;
#pragma unroll
                    for (int c = 0; c < 8; ++c) acc[c] += t * xr[c];
                  }
                }
                const double wd = dv.W[nd] * tau_e[nd], ws = dv.W[nd] * tau_s[nd];
                const double* Qr = dv.Q + k * dv.n_a;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                  double sc = 0.0;
                  for (int kp = 0; kp < dv.n_a; ++kp) sc += Qr[kp] * xs[(kp * nn + nd) * 8 + c];
                  const int col = P0 + half * 8 + c;
                  const double rv = (col < m && q == dv.in_row[col]) ? dv.in_val[col] : 0.0;
                  acc[c] = rv - (acc[c] + wd * xs[q * 8 + c] - ws * sc);
                }
              }
#pragma unroll
              for (int c = 0; c < 8; ++c) {
                pan[i * LDP + half * 8 + c] = (T)acc[c];
                atomicMax(&colmax[half * 8 + c], (unsigned long long)__double_as_longlong(fabs(acc[c])));
              }
            }
            __syncthreads();
          }
          double worst = 0.0;
          for (int c = 0; c < NB; ++c)
            if (P0 + c < m) worst = fmax(worst, __longlong_as_double((long long)colmax[c]) / dv.in_val[P0 + c]);
          if (worst <= a.ir_tol || it >= a.ir_steps) {
            elem_res = fmax(elem_res, worst);
            break;
          }
          panel_solve<T>(pan, fac, inv, perm, npad, 0, wave, lane);
          for (int idx = tid; idx < npad * NB; idx += kThreads) {
            int r = idx >> 4, c = idx & 15;
            xg[r * NB + c] += (double)pan[r * LDP + c];
          }
          __threadfence_block();
          __syncthreads();
        }
      }
      // outputs (pan rows are volume DOFs in natural order)
      const int64_t n_out = (int64_t)m * m + (int64_t)n * m;
      if (a.in2sol || a.b_i2s || a.f_i2s || a.pairs) {
        for (int idx = tid; idx < n * NB; idx += kThreads) {
          int r = idx >> 4, c = idx & 15;
          if (P0 + c < m) {
            const double v = ir ? xg[r * NB + c] : (double)pan[r * LDP + c];
            const int64_t o = ((int64_t)e * n + r) * m + P0 + c;
            if (a.in2sol) a.in2sol[o] = v;
            if (a.b_i2s) a.b_i2s[o] = gemm::f2bf((float)v);
            if (a.f_i2s) a.f_i2s[o] = (float)v;
            if (a.pairs) a.pairs[(int64_t)e * n_out + (int64_t)m * m + (int64_t)r * m + P0 + c] = gemm::f2bf((float)v);
          }
        }
      }
      if (a.in2out || a.b_i2o || a.f_i2o || a.pairs) {
        for (int idx = tid; idx < m * NB; idx += kThreads) {
          int r = idx >> 4, c = idx & 15;
          if (P0 + c < m) {
            const double v = ir ? xg[dv.out_row[r] * NB + c] : (double)pan[dv.out_row[r] * LDP + c];
            const int64_t o = ((int64_t)e * m + r) * m + P0 + c;
            if (a.in2out) a.in2out[o] = v;
            if (a.b_i2o) a.b_i2o[o] = gemm::f2bf((float)v);
            if (a.f_i2o) a.f_i2o[o] = (float)v;
            if (a.pairs) a.pairs[(int64_t)e * n_out + (int64_t)r * m + P0 + c] = gemm::f2bf((float)v);
          }
        }
      }
      if (a.in2mean) {
        double* o = a.in2mean + (size_t)e * nn * m;
        const double s = 1.0 / dv.n_a;
        for (int idx = tid; idx < nn * NB; idx += kThreads) {
          int r = idx >> 4, c = idx & 15;
          if (P0 + c < m) {
            double acc = 0.0;
            for (int k = 0; k < dv.n_a; ++k)
              acc += ir ? xg[(k * nn + r) * NB + c] : (double)pan[(k * nn + r) * LDP + c];
            o[(size_t)r * m + P0 + c] = acc * s;
          }
        }
      }
      __syncthreads();
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
size_t lu_smem_bytes(int npad, int nn, bool ir) {
  size_t base = sizeof(T) * (size_t)npad * LDP + 2 * sizeof(int) * (size_t)npad + 2 * sizeof(double) * nn +
                kWaves * (sizeof(double) + sizeof(int)) + 2 * sizeof(int);
  base = (base + 15) / 16 * 16;
  if (ir) base += NB * sizeof(unsigned long long) + sizeof(double) * (size_t)npad * 8;
  return base + 16;
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
  uint16_t* pairs = nullptr;
  const int32_t* emap = nullptr;
};

template <typename T>
el_status run_local_t(el_ctx* ctx, el_ctx::DiscEntry* de, bool ir, int64_t E, const double* h,
                      const double* kappa, const double* sigma, const LocalOut& out, double* rel_resid) {
  const DiscHost& dh = de->host;
  const int npad = (dh.n + NB - 1) / NB * NB;
  const int mpad = (dh.m + NB - 1) / NB * NB;
  if (rel_resid) {
    hipLaunchKernelGGL(k_fill_double, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, ctx->stream, rel_resid, E, 0.0);
  }
  size_t smem = lu_smem_bytes<T>(npad, dh.nn, ir);
  int max_smem = 0;
  hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device);
  if ((int)smem > max_smem) {
    std::ostringstream os;
    os << "el_local_solve: n = " << dh.n << " needs " << smem << " B of LDS (limit " << max_smem << ")";
    return set_error(ctx, EL_ERR_ARG, os.str());
  }
  const int npan = npad / NB;
  const int64_t slots = std::min<int64_t>(E, (int64_t)ctx->num_cus * 2);
  size_t fac_bytes = sizeof(T) * (size_t)slots * npan * npad * NB;
  size_t inv_bytes = sizeof(T) * (size_t)slots * npan * 2 * NB * NB;
  size_t x_bytes = ir ? sizeof(double) * (size_t)slots * npad * NB : 0;
  el_status st = ensure_ws(ctx, ctx->ws_local, fac_bytes + inv_bytes + x_bytes + 256);
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
  char* base = reinterpret_cast<char*>(ctx->ws_local.ptr);
  args.fac = reinterpret_cast<T*>(base);
  args.inv = reinterpret_cast<T*>(base + fac_bytes);
  args.xbuf = ir ? reinterpret_cast<double*>(base + ((fac_bytes + inv_bytes + 255) / 256) * 256) : nullptr;
  args.rel_resid = rel_resid;
  args.ir_steps = 3;
  args.ir_tol = 1e-13;
  args.flags = flags;
  hipError_t he = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_local_lu<T>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (he != hipSuccess) return hip_check(ctx, he, "hipFuncSetAttribute(k_local_lu)");
  hipLaunchKernelGGL(k_local_lu<T>, dim3((unsigned)slots), dim3(kThreads), smem, ctx->stream, args);
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

el_status launch_local_solve(el_ctx* ctx, el_ctx::DiscEntry* de, int precision, int64_t E,
                             const double* h, const double* kappa, const double* sigma,
                             double* in2out, double* in2sol, double* in2mean, double* rel_resid) {
  LocalOut o;
  o.in2out = in2out; o.in2sol = in2sol; o.in2mean = in2mean;
  return run_local(ctx, de, precision, E, h, kappa, sigma, o, rel_resid);
}

el_status launch_local_solve_ex(el_ctx* ctx, el_ctx::DiscEntry* de, int precision, int64_t E, const double* h,
                                const double* kappa, const double* sigma, const int32_t* emap,
                                void* o_i2o, void* o_i2s, int out_dtype, uint16_t* pairs) {
  LocalOut o;
  if (out_dtype == EL_F32) {
    o.f_i2o = reinterpret_cast<float*>(o_i2o); o.f_i2s = reinterpret_cast<float*>(o_i2s);
  } else {
    o.b_i2o = reinterpret_cast<uint16_t*>(o_i2o); o.b_i2s = reinterpret_cast<uint16_t*>(o_i2s);
  }
  o.pairs = pairs; o.emap = emap;
  return run_local(ctx, de, precision, E, h, kappa, sigma, o, nullptr);
}

}  // namespace el

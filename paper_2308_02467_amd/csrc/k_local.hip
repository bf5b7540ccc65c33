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
      const int Istart = sflag[1];
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
      // outputs (pan rows are volume DOFs in natural order)
      const int64_t n_out = (int64_t)m * m + (int64_t)n * m;
      if (a.in2sol || a.b_i2s || a.f_i2s || a.pairs) {
        for (int idx = tid; idx < n * NB; idx += kThreads) {
          int r = idx >> 4, c = idx & 15;
          if (P0 + c < m) {
            const double v = (double)pan[r * LDP + c];
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
            const double v = (double)pan[dv.out_row[r] * LDP + c];
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
            for (int k = 0; k < dv.n_a; ++k) acc += (double)pan[(k * nn + r) * LDP + c];
            o[(size_t)r * m + P0 + c] = acc * s;
          }
        }
      }
      __syncthreads();
    }
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
size_t lu_smem_bytes(int npad, int nn) {
  return sizeof(T) * (size_t)npad * LDP + 2 * sizeof(int) * (size_t)npad + 2 * sizeof(double) * nn +
         kWaves * (sizeof(double) + sizeof(int)) + 2 * sizeof(int) + 16;
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

el_status run_local(el_ctx* ctx, el_ctx::DiscEntry* de, int precision, int64_t E, const double* h,
                    const double* kappa, const double* sigma, const LocalOut& out, double* rel_resid) {
  const DiscHost& dh = de->host;
  const int npad = (dh.n + NB - 1) / NB * NB;
  const int mpad = (dh.m + NB - 1) / NB * NB;
  if (precision != EL_FP64)
    return set_error(ctx, EL_ERR_ARG, "el_local_solve: EL_FP32_IR is not available in this build");
  if (rel_resid) {
    hipLaunchKernelGGL(k_fill_double, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, ctx->stream, rel_resid, E, 0.0);
  }
  size_t smem = lu_smem_bytes<double>(npad, dh.nn);
  int max_smem = 0;
  hipDeviceGetAttribute(&max_smem, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device);
  if ((int)smem > max_smem) {
    std::ostringstream os;
    os << "el_local_solve: n = " << dh.n << " needs " << smem << " B of LDS (limit " << max_smem << ")";
    return set_error(ctx, EL_ERR_ARG, os.str());
  }
  const int npan = npad / NB;
  const int64_t slots = std::min<int64_t>(E, (int64_t)ctx->num_cus * 2);
  size_t fac_bytes = sizeof(double) * (size_t)slots * npan * npad * NB;
  size_t inv_bytes = sizeof(double) * (size_t)slots * npan * 2 * NB * NB;
  el_status st = ensure_ws(ctx, ctx->ws_local, fac_bytes + inv_bytes);
  if (st) return st;
  st = ensure_ws(ctx, ctx->ws_small, 8192);
  if (st) return st;
  int* flags = reinterpret_cast<int*>(ctx->ws_small.ptr);
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, ctx->stream, flags, 2, INT_MAX);
  LuArgs<double> args;
  args.dv = de->view;
  args.E = E;
  args.npad = npad;
  args.mpad = mpad;
  args.h = h; args.kappa = kappa; args.sigma = sigma;
  args.in2out = out.in2out; args.in2sol = out.in2sol; args.in2mean = out.in2mean;
  args.b_i2o = out.b_i2o; args.b_i2s = out.b_i2s; args.pairs = out.pairs; args.emap = out.emap;
  args.f_i2o = out.f_i2o; args.f_i2s = out.f_i2s;
  args.fac = reinterpret_cast<double*>(ctx->ws_local.ptr);
  args.inv = reinterpret_cast<double*>(reinterpret_cast<char*>(ctx->ws_local.ptr) + fac_bytes);
  args.flags = flags;
  hipError_t he = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_local_lu<double>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (he != hipSuccess) return hip_check(ctx, he, "hipFuncSetAttribute(k_local_lu)");
  hipLaunchKernelGGL(k_local_lu<double>, dim3((unsigned)slots), dim3(kThreads), smem, ctx->stream, args);
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

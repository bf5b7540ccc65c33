// Batched restarted GMRES for the skeleton systems (I - P) t = b of several
// independent meshes (eq. hdg_global_mat, Sec. 2.3), entirely on the device.
//
// All meshes of a call share one set of launches: their trace vectors are
// concatenated (each mesh's segment padded to a whole number of vector
// blocks), the product runs one workgroup per element of every mesh, and
// every dot product is reduced per mesh in a fixed order (deterministic).
// Each mesh carries its own Arnoldi state (Hessenberg matrix, Givens
// rotations, residual estimate, flags) in device memory; a mesh that has
// converged or stopped simply makes the later launches skip its blocks.
//
// Per Arnoldi step (the same for every mesh):
//   w = P v_j;  h = V^T w and |w|^2 (one pass);  w -= V h and |w|^2;
//   when |w| < |w_before| / sqrt(2) (DGKS test, decided on the device) a
//   second classical Gram-Schmidt pass;  v_{j+1} = w / |w|.
// The Krylov spaces of P and I - P are the same, and (I - P) V_j =
// V_{j+1} (I~ - H_P), so the least-squares problem of I - P is updated with
// the column e_j - h (and -|w| below the diagonal) by Givens rotations on
// the device, with the stopping test.  Arnoldi on P instead of I - P avoids
// projecting out the large v_j component of (I - P) v_j, so the second
// Gram-Schmidt pass is needed less often.
// One restart cycle (restart steps) is captured once as a HIP graph and
// replayed; the host synchronizes once per cycle, after the true residual
// b - (I - P) x of every mesh has been formed and tested.  x0 = 0 or a
// given starting guess.  Dot products, scalars, the solution and the working
// vectors are FP64; the stored basis V is FP64, or FP32 to halve the bytes
// of the Gram-Schmidt sweeps (each v_j is rounded once, and the product of
// step j takes the rounded v_j, so the Arnoldi relation holds for the stored
// basis up to the rounding of its newest column; the true residual of every
// restart stays FP64).
#include <climits>
#include <cmath>
#include <cstdio>
#include <sstream>
#include <vector>

#include "el_internal.h"
#include "trace_dev.h"

namespace el {

namespace {

constexpr int kVThreads = 256;
constexpr int kVec = 8;                       // values per thread in vector kernels
constexpr int kChunk = kVThreads * kVec;      // DOFs per vector block
constexpr int kMaxCnt = 258;                  // restart + 2
constexpr int kGrp = 4;                       // basis vectors per pass of the sweep loops
                                              // (their loads are in flight together)

struct BMesh {
  int n_x, n_y, n_vf;
  int b0, nb;          // vector blocks [b0, b0 + nb) of this mesh
  int pad;
  int64_t e0;          // first element of the mesh in the batch
  int64_t d0;          // first DOF of the mesh in the concatenated vectors
  int64_t N;           // trace DOFs of the mesh
  const void* op;      // in2out [E][m][m]
};

struct BState {
  double bn;           // |b|
  double relres;       // true relative residual at the last cycle start
  double inv;          // scale of the newest basis vector
  int active;          // running Arnoldi steps in the current cycle
  int reorth;          // second Gram-Schmidt pass in the current step
  int kused;           // Arnoldi steps taken in the current cycle
  int iters, restarts;
  int done, conv, bad;
  int reorths;         // second Gram-Schmidt passes taken
};

// Per-mesh array of S doubles: Hessenberg matrix (column-major, R+1 rows),
// rotations, least-squares right-hand side, solution, the two sets of
// Gram-Schmidt coefficients and four scalars
// ([0] b.b, [1] r.r, [2] |w|^2 after pass 1, [3] |w|^2 after pass 2).
struct BLay {
  int R, S;
  int H, cs, sn, g, y, h1, h2, sc;
};

BLay make_layout(int R) {
  BLay l;
  l.R = R;
  int o = 0;
  l.H = o; o += (R + 1) * R;
  l.cs = o; o += R;
  l.sn = o; o += R;
  l.g = o; o += R + 1;
  l.y = o; o += R;
  l.h1 = o; o += R + 2;
  l.h2 = o; o += R + 2;
  l.sc = o; o += 4;
  l.S = (o + 7) / 8 * 8;
  return l;
}

enum Pred { P_ACTIVE = 0, P_REORTH = 1, P_NOT_DONE = 2, P_ALL = 3, P_USED = 4 };

__device__ inline bool skip(const BState& s, int pred) {
  switch (pred) {
    case P_ACTIVE: return !s.active;
    case P_REORTH: return !(s.active && s.reorth);
    case P_NOT_DONE: return s.done != 0;
    case P_USED: return s.kused == 0;
    default: return false;
  }
}

__device__ inline int mesh_of_block(const BMesh* ms, int n_mesh, int b) {
  int lo = 0, hi = n_mesh - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ms[mid].b0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline int mesh_of_elem(const BMesh* ms, int n_mesh, int64_t e) {
  int lo = 0, hi = n_mesh - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ms[mid].e0 <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ---- products -----------------------------------------------------------------
template <typename OpT, bool IMP, int R, typename XT>
__global__ void __launch_bounds__(kMVThreads) k_bmatvec(DiscDev dv, const BMesh* __restrict__ ms, int n_mesh,
                                                         const BState* __restrict__ st, int pred,
                                                         const XT* __restrict__ x, double* __restrict__ y) {
  extern __shared__ double sm[];
  const int mi = mesh_of_elem(ms, n_mesh, blockIdx.x);
  if (skip(st[mi], pred)) return;
  const BMesh M = ms[mi];
  const int e = (int)((int64_t)blockIdx.x - M.e0);
  const MeshDev md{M.n_x, M.n_y, M.n_vf};
  matvec_element<OpT, IMP, R, XT>(dv, md, e, reinterpret_cast<const OpT*>(M.op) + (size_t)e * dv.m * dv.m,
                                  x + M.d0, y + M.d0, sm);
}

// ---- vector kernels (one block = kChunk DOFs of one mesh) ---------------------
struct Span {
  int mi;
  int64_t base;   // first DOF handled by thread 0 of the block
  int64_t lim;    // end of the mesh segment
};

__device__ inline Span block_span(const BMesh* ms, int n_mesh) {
  Span s;
  s.mi = mesh_of_block(ms, n_mesh, blockIdx.x);
  const BMesh& M = ms[s.mi];
  s.base = M.d0 + (int64_t)(blockIdx.x - M.b0) * kChunk;
  s.lim = M.d0 + M.N;
  return s;
}

// v[ix] for ix < lim, else 0, without a branch: the index is clamped into
// the mesh segment (never empty) and the value selected, so the loads of a
// sweep stay in flight together
template <typename VT>
__device__ inline double ld_masked(const VT* __restrict__ v, int64_t ix, int64_t lim) {
  const double x = (double)v[ix < lim ? ix : lim - 1];
  return ix < lim ? x : 0.0;
}
// the same for the basis vectors, streamed with non-temporal loads
template <typename VT>
__device__ inline double ld_masked_nt(const VT* __restrict__ v, int64_t ix, int64_t lim) {
  const double x = (double)__builtin_nontemporal_load(v + (ix < lim ? ix : lim - 1));
  return ix < lim ? x : 0.0;
}

// partials[blk][i] = V[i] . w over the block chunk (i < cnt); with self also
// partials[blk][cnt] = w . w.
template <typename VT>
__global__ void __launch_bounds__(kVThreads) k_bdot(const VT* __restrict__ V, int64_t ldv, int cnt,
                                                     const double* __restrict__ w, int self,
                                                     const BMesh* __restrict__ ms, int n_mesh,
                                                     const BState* __restrict__ st, int pred,
                                                     double* __restrict__ partials) {
  __shared__ double s[kVThreads / 64][kMaxCnt];
  const Span sp = block_span(ms, n_mesh);
  if (skip(st[sp.mi], pred)) return;
  const int64_t base = sp.base + threadIdx.x;
  double wr[kVec];
#pragma unroll
  for (int v = 0; v < kVec; ++v) wr[v] = ld_masked(w, base + v * kVThreads, sp.lim);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int i = 0;
  for (; i + kGrp <= cnt; i += kGrp) {
    double x[kGrp][kVec];
#pragma unroll
    for (int u = 0; u < kGrp; ++u) {
      const VT* vu = V + (size_t)(i + u) * ldv;
#pragma unroll
      for (int v = 0; v < kVec; ++v) x[u][v] = ld_masked_nt(vu, base + v * kVThreads, sp.lim);
    }
    double a[kGrp];
#pragma unroll
    for (int u = 0; u < kGrp; ++u) {
      a[u] = 0.0;
#pragma unroll
      for (int v = 0; v < kVec; ++v) a[u] += x[u][v] * wr[v];
      a[u] = wave_sum(a[u]);
    }
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < kGrp; ++u) s[wave][i + u] = a[u];
    }
  }
  for (; i < cnt; ++i) {
    const VT* v0 = V + (size_t)i * ldv;
    double a0 = 0.0;
#pragma unroll
    for (int v = 0; v < kVec; ++v) a0 += ld_masked_nt(v0, base + v * kVThreads, sp.lim) * wr[v];
    a0 = wave_sum(a0);
    if (lane == 0) s[wave][i] = a0;
  }
  if (self) {
    double a = 0.0;
#pragma unroll
    for (int v = 0; v < kVec; ++v) a += wr[v] * wr[v];
    a = wave_sum(a);
    if (lane == 0) s[wave][cnt] = a;
  }
  __syncthreads();
  const int outc = cnt + (self ? 1 : 0);
  for (int k = threadIdx.x; k < outc; k += kVThreads) {
    double t = 0.0;
    for (int wv = 0; wv < kVThreads / 64; ++wv) t += s[wv][k];
    partials[(size_t)blockIdx.x * outc + k] = t;
  }
}

// w -= sign * sum_i c_i V[i] with c = the mesh's coefficients at offset coef
// (cnt >= 0: cnt of them; cnt < 0: the mesh's kused); with norm also
// partials[blk] = w . w of the updated chunk.
template <typename VT>
__global__ void __launch_bounds__(kVThreads) k_bupdate(const VT* __restrict__ V, int64_t ldv, int cnt,
                                                        const double* __restrict__ hs, BLay lay, int coef,
                                                        double* __restrict__ w, double sign, int norm,
                                                        const BMesh* __restrict__ ms, int n_mesh,
                                                        const BState* __restrict__ st, int pred,
                                                        double* __restrict__ partials) {
  __shared__ double cs[kMaxCnt];
  __shared__ double red[kVThreads / 64];
  const Span sp = block_span(ms, n_mesh);
  const BState& S = st[sp.mi];
  if (skip(S, pred)) return;
  const int c = cnt >= 0 ? cnt : S.kused;
  const double* co = hs + (size_t)sp.mi * lay.S + coef;
  for (int k = threadIdx.x; k < c; k += kVThreads) cs[k] = sign * co[k];
  __syncthreads();
  const int64_t base = sp.base + threadIdx.x;
  double wr[kVec];
#pragma unroll
  for (int v = 0; v < kVec; ++v) wr[v] = ld_masked(w, base + v * kVThreads, sp.lim);
  int i = 0;
  for (; i + kGrp <= c; i += kGrp) {
    double x[kGrp][kVec];
#pragma unroll
    for (int u = 0; u < kGrp; ++u) {
      const VT* vu = V + (size_t)(i + u) * ldv;
#pragma unroll
      for (int v = 0; v < kVec; ++v) x[u][v] = ld_masked_nt(vu, base + v * kVThreads, sp.lim);
    }
#pragma unroll
    for (int u = 0; u < kGrp; ++u) {
      const double hu = cs[i + u];
#pragma unroll
      for (int v = 0; v < kVec; ++v) wr[v] -= hu * x[u][v];
    }
  }
  for (; i < c; ++i) {
    const VT* v0 = V + (size_t)i * ldv;
    const double h0 = cs[i];
#pragma unroll
    for (int v = 0; v < kVec; ++v) wr[v] -= h0 * ld_masked_nt(v0, base + v * kVThreads, sp.lim);
  }
#pragma unroll
  for (int v = 0; v < kVec; ++v) {
    const int64_t ix = base + v * kVThreads;
    if (ix < sp.lim) w[ix] = wr[v];
  }
  if (!norm) return;
  double a = 0.0;
#pragma unroll
  for (int v = 0; v < kVec; ++v) a += wr[v] * wr[v];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int wv = 0; wv < kVThreads / 64; ++wv) t += red[wv];
    partials[blockIdx.x] = t;
  }
}

// w *= inv of the mesh
__global__ void __launch_bounds__(kVThreads) k_bscale(double* __restrict__ w, const BMesh* __restrict__ ms,
                                                       int n_mesh, const BState* __restrict__ st, int pred) {
  const Span sp = block_span(ms, n_mesh);
  const BState& S = st[sp.mi];
  if (skip(S, pred)) return;
  const double s = S.inv;
  const int64_t base = sp.base + threadIdx.x;
  double x[kVec];
#pragma unroll
  for (int v = 0; v < kVec; ++v) x[v] = ld_masked(w, base + v * kVThreads, sp.lim);
#pragma unroll
  for (int v = 0; v < kVec; ++v) {
    const int64_t ix = base + v * kVThreads;
    if (ix < sp.lim) w[ix] = x[v] * s;
  }
}

// FP32 basis: v = w * inv of the mesh rounded to FP32 once, stored as the
// basis column vb, which is also the next product's input (widened as it is
// gathered)
__global__ void __launch_bounds__(kVThreads) k_bscale_to(const double* __restrict__ w,
                                                          float* __restrict__ vb, const BMesh* __restrict__ ms,
                                                          int n_mesh, const BState* __restrict__ st, int pred) {
  const Span sp = block_span(ms, n_mesh);
  const BState& S = st[sp.mi];
  if (skip(S, pred)) return;
  const double s = S.inv;
  const int64_t base = sp.base + threadIdx.x;
  double x[kVec];
#pragma unroll
  for (int v = 0; v < kVec; ++v) x[v] = ld_masked(w, base + v * kVThreads, sp.lim);
#pragma unroll
  for (int v = 0; v < kVec; ++v) {
    const int64_t ix = base + v * kVThreads;
    if (ix < sp.lim) {
      vb[ix] = (float)(x[v] * s);
    }
  }
}

// out = a - b
__global__ void __launch_bounds__(kVThreads) k_bsub(const double* __restrict__ a, const double* __restrict__ b,
                                                     double* __restrict__ out, const BMesh* __restrict__ ms,
                                                     int n_mesh, const BState* __restrict__ st, int pred) {
  const Span sp = block_span(ms, n_mesh);
  if (skip(st[sp.mi], pred)) return;
#pragma unroll
  for (int v = 0; v < kVec; ++v) {
    const int64_t ix = sp.base + threadIdx.x + v * kVThreads;
    if (ix < sp.lim) out[ix] = a[ix] - b[ix];
  }
}

__global__ void k_bzero(double* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// hs[mesh][dst + i] = sum over the mesh's blocks of partials[blk][i], grid
// (outc, n_mesh), fixed order.  With decide >= 0 (the norm after the first
// pass), also sets the mesh's DGKS flag from h1[decide] = |w|^2 before the
// projection.
__global__ void k_breduce(const double* __restrict__ partials, int outc, const BMesh* __restrict__ ms,
                          BState* __restrict__ st, int pred, double* __restrict__ hs, BLay lay, int dst,
                          int decide) {
  __shared__ double s[256 / 64];
  const int i = blockIdx.x, mi = blockIdx.y;
  if (skip(st[mi], pred)) return;
  const int b0 = ms[mi].b0, nb = ms[mi].nb;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += partials[(size_t)(b0 + b) * outc + i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = s[0] + s[1] + s[2] + s[3];
    double* H = hs + (size_t)mi * lay.S;
    H[dst + i] = t;
    if (decide >= 0) {
      const double w0 = sqrt(fmax(H[lay.h1 + decide], 0.0));
      st[mi].reorth = sqrt(fmax(t, 0.0)) < 0.70710678118654752 * w0;
    }
  }
}

// ---- per-mesh scalar steps (one thread per mesh) -------------------------------
__global__ void k_binit(int n_mesh, const double* __restrict__ hs, BLay lay, BState* __restrict__ st) {
  const int mi = blockIdx.x * blockDim.x + threadIdx.x;
  if (mi >= n_mesh) return;
  BState s{};
  s.bn = sqrt(fmax(hs[(size_t)mi * lay.S + lay.sc + 0], 0.0));
  if (!isfinite(s.bn)) {
    s.bad = 1;
    s.done = 1;
  } else if (s.bn == 0.0) {
    s.done = 1;
    s.conv = 1;
  }
  st[mi] = s;
}

// after r = b - (I - P) x and r.r: test, and start a cycle with v0 = r / |r|
__global__ void k_bstart(int n_mesh, double* __restrict__ hs, BLay lay, BState* __restrict__ st, double tol,
                         int max_iter) {
  const int mi = blockIdx.x * blockDim.x + threadIdx.x;
  if (mi >= n_mesh) return;
  BState& s = st[mi];
  if (s.done) return;
  double* H = hs + (size_t)mi * lay.S;
  const double beta = sqrt(fmax(H[lay.sc + 1], 0.0));
  s.relres = beta / s.bn;
  s.kused = 0;
  s.reorth = 0;
  if (!isfinite(s.relres)) {
    s.bad = 1;
    s.done = 1;
    s.active = 0;
    return;
  }
  if (s.relres <= tol || s.iters >= max_iter) {
    s.done = 1;
    s.active = 0;
    s.conv = s.relres <= tol;
    return;
  }
  s.active = 1;
  H[lay.g] = beta;
  for (int i = 1; i <= lay.R; ++i) H[lay.g + i] = 0.0;
  s.inv = 1.0 / beta;
}

// Arnoldi column j: H[:, j] = h1 (+ h2), |w|, rotations, stopping test.  One
// 64-lane block per mesh: the column, the rotations and g are staged in LDS
// by all lanes, lane 0 applies the rotations (a serial recurrence), all lanes
// write back.
__global__ void __launch_bounds__(64) k_bgivens(int j, int n_mesh, double* __restrict__ hs, BLay lay,
                                                BState* __restrict__ st, double tol, int max_iter) {
  __shared__ double col[kMaxCnt], c_s[kMaxCnt], s_n[kMaxCnt];
  const int mi = blockIdx.x;
  BState& s = st[mi];
  if (!s.active) return;
  const int t = threadIdx.x;
  double* B = hs + (size_t)mi * lay.S;
  const int ld = lay.R + 1;
  double* colg = B + lay.H + (size_t)j * ld;
  const double* h1 = B + lay.h1;
  const double* h2 = B + lay.h2;
  double* cs = B + lay.cs;
  double* sn = B + lay.sn;
  double* g = B + lay.g;
  const bool re = s.reorth;
  // Arnoldi on P: P v_j = V h + |w| v_{j+1}, so column j of the Hessenberg
  // matrix of I - P is e_j - h with -|w| below the diagonal
  for (int i = t; i <= j; i += 64) {
    col[i] = (i == j ? 1.0 : 0.0) - (re ? h1[i] + h2[i] : h1[i]);
    if (i < j) { c_s[i] = cs[i]; s_n[i] = sn[i]; }
  }
  __syncthreads();
  if (t == 0) {
    const double hn = sqrt(fmax(re ? B[lay.sc + 3] : B[lay.sc + 2], 0.0));
    s.reorths += re;
    col[j + 1] = -hn;
    double a_prev = col[0];
    for (int i = 0; i < j; ++i) {
      const double a1 = col[i + 1];
      col[i] = c_s[i] * a_prev + s_n[i] * a1;
      a_prev = -s_n[i] * a_prev + c_s[i] * a1;
    }
    const double a0 = a_prev, a1 = col[j + 1];
    const double den = hypot(a0, a1);
    cs[j] = a0 / den;
    sn[j] = a1 / den;
    col[j] = den;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sn[j] * gj;
    g[j] = cs[j] * gj;
    s.iters += 1;
    s.kused = j + 1;
    s.inv = hn > 0.0 ? 1.0 / hn : 0.0;
    if (fabs(g[j + 1]) / s.bn <= tol || s.iters >= max_iter || hn == 0.0 || j + 1 == lay.R) s.active = 0;
  }
  __syncthreads();
  for (int i = t; i <= j + 1; i += 64) colg[i] = col[i];
}

// end of a cycle: y = H^{-1} g (upper triangular), one 64-lane block per
// mesh: y_k from the diagonal, then every lane updates its rows i < k
// (column-oriented back substitution)
__global__ void __launch_bounds__(64) k_bfinish(int n_mesh, double* __restrict__ hs, BLay lay,
                                                BState* __restrict__ st) {
  __shared__ double acc[kMaxCnt];
  const int mi = blockIdx.x;
  BState& s = st[mi];
  const int n = s.kused;
  __syncthreads();
  if (threadIdx.x == 0) s.active = 0;
  if (n == 0) return;
  const int t = threadIdx.x;
  double* B = hs + (size_t)mi * lay.S;
  const int ld = lay.R + 1;
  const double* H = B + lay.H;
  const double* g = B + lay.g;
  double* y = B + lay.y;
  for (int i = t; i < n; i += 64) acc[i] = g[i];
  __syncthreads();
  for (int k = n - 1; k >= 0; --k) {
    const double* hk = H + (size_t)k * ld;
    const double yk = acc[k] / hk[k];
    __syncthreads();
    for (int i = t; i < k; i += 64) acc[i] -= hk[i] * yk;
    if (t == 0) { acc[k] = yk; y[k] = yk; }
    __syncthreads();
  }
  if (t == 0) s.restarts += 1;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Launch context of one batched solve.
struct Batch {
  el_ctx* ctx;
  DiscDev dv;
  int m;
  int op_dtype;
  int mv_shape;      // row shape of the product (index into matvec_shape_names())
  int n_mesh;
  int64_t E, Np;
  int nblk;
  BLay lay;
  double tol;
  int max_iter;
  bool f32;          // FP32 basis
  double* V;         // FP64 basis [R + 1][Np] (null with the FP32 basis)
  float* Vf;         // FP32 basis [R + 1][Np] (null with the FP64 basis)
  double* W;         // FP32 basis: working vector w [Np]
  double* tmp;       // [Np]
  double* bcat;      // [Np]
  double* xcat;      // [Np]
  double* partials;  // [nblk][R + 2]
  double* hs;        // [n_mesh][S]
  BState* st;        // [n_mesh]
  BMesh* ms;         // [n_mesh]

  // imp: y = (I - P) x (true residuals); otherwise y = P x (Arnoldi)
  template <bool IMP, typename XT>
  void matvec_t(hipStream_t s, int pred, const XT* x, double* y) const {
    const size_t smem = matvec_smem_bytes(m);
    with_op_type(op_dtype, [&](auto tag) {
      using T = decltype(tag);
      switch (mv_shape) {
        case 1:
          hipLaunchKernelGGL((k_bmatvec<T, IMP, 2, XT>), dim3((unsigned)E), dim3(kMVThreads), smem, s, dv, ms, n_mesh,
                             st, pred, x, y);
          break;
        case 2:
          hipLaunchKernelGGL((k_bmatvec<T, IMP, 8, XT>), dim3((unsigned)E), dim3(kMVThreads), smem, s, dv, ms, n_mesh,
                             st, pred, x, y);
          break;
        default:
          hipLaunchKernelGGL((k_bmatvec<T, IMP, 4, XT>), dim3((unsigned)E), dim3(kMVThreads), smem, s, dv, ms, n_mesh,
                             st, pred, x, y);
      }
    });
  }
  void matvec(hipStream_t s, int pred, const double* x, double* y, bool imp) const {
    if (imp) matvec_t<true>(s, pred, x, y);
    else matvec_t<false>(s, pred, x, y);
  }
  void dot(hipStream_t s, int pred, int cnt, const double* w, int self, int dst, int decide = -1) const {
    const int outc = cnt + (self ? 1 : 0);
    if (f32)
      hipLaunchKernelGGL(k_bdot<float>, dim3(nblk), dim3(kVThreads), 0, s, Vf, Np, cnt, w, self, ms, n_mesh, st,
                         pred, partials);
    else
      hipLaunchKernelGGL(k_bdot<double>, dim3(nblk), dim3(kVThreads), 0, s, V, Np, cnt, w, self, ms, n_mesh, st,
                         pred, partials);
    hipLaunchKernelGGL(k_breduce, dim3(outc, n_mesh), dim3(256), 0, s, partials, outc, ms, st, pred, hs, lay, dst,
                       decide);
  }
  // w -= sign V c; with dst >= 0 also |w|^2 into hs[dst]
  void update(hipStream_t s, int pred, int cnt, int coef, double* w, double sign, int dst, int decide = -1) const {
    if (f32)
      hipLaunchKernelGGL(k_bupdate<float>, dim3(nblk), dim3(kVThreads), 0, s, Vf, Np, cnt, hs, lay, coef, w, sign,
                         dst >= 0 ? 1 : 0, ms, n_mesh, st, pred, partials);
    else
      hipLaunchKernelGGL(k_bupdate<double>, dim3(nblk), dim3(kVThreads), 0, s, V, Np, cnt, hs, lay, coef, w, sign,
                         dst >= 0 ? 1 : 0, ms, n_mesh, st, pred, partials);
    if (dst >= 0)
      hipLaunchKernelGGL(k_breduce, dim3(1, n_mesh), dim3(256), 0, s, partials, 1, ms, st, pred, hs, lay, dst,
                         decide);
  }
  // v_0 = r / |r| from r in the working vector (FP64 basis: V[0])
  void start_vector(hipStream_t s) const {
    if (f32)
      hipLaunchKernelGGL(k_bscale_to, dim3(nblk), dim3(kVThreads), 0, s, W, Vf, ms, n_mesh, st, P_ACTIVE);
    else
      hipLaunchKernelGGL(k_bscale, dim3(nblk), dim3(kVThreads), 0, s, V, ms, n_mesh, st, P_ACTIVE);
  }
  // one Arnoldi step j on every active mesh
  void step(hipStream_t s, int j) const {
    const int cnt = j + 1;
    double* w = f32 ? W : V + (size_t)(j + 1) * Np;
    // with the FP32 basis the product reads the stored (rounded) v_j
    if (f32) matvec_t<false>(s, P_ACTIVE, Vf + (size_t)j * Np, w);
    else matvec_t<false>(s, P_ACTIVE, V + (size_t)j * Np, w);
    dot(s, P_ACTIVE, cnt, w, 1, lay.h1);
    update(s, P_ACTIVE, cnt, lay.h1, w, 1.0, lay.sc + 2, cnt);
    dot(s, P_REORTH, cnt, w, 0, lay.h2);
    update(s, P_REORTH, cnt, lay.h2, w, 1.0, lay.sc + 3);
    hipLaunchKernelGGL(k_bgivens, dim3(n_mesh), dim3(64), 0, s, j, n_mesh, hs, lay, st, tol, max_iter);
    if (f32)
      hipLaunchKernelGGL(k_bscale_to, dim3(nblk), dim3(kVThreads), 0, s, W, Vf + (size_t)(j + 1) * Np, ms,
                         n_mesh, st, P_ACTIVE);
    else
      hipLaunchKernelGGL(k_bscale, dim3(nblk), dim3(kVThreads), 0, s, w, ms, n_mesh, st, P_ACTIVE);
  }
};

}  // namespace

el_status run_trace_solve(el_ctx* ctx, el_ctx::DiscEntry* de, int n_mesh, const el_mesh* meshes,
                          const void* const* in2out, int op_dtype, const double* const* b,
                          double* const* trace, const el_gmres_opts& opts, el_gmres_report* rep) {
  const int R = opts.restart;
  const int na = de->host.n_a, q = de->host.q;
  std::vector<BMesh> hm(n_mesh);
  int64_t E = 0, Np = 0;
  int64_t nblk = 0;
  for (int i = 0; i < n_mesh; ++i) {
    const el_mesh& M = meshes[i];
    BMesh& B = hm[i];
    B.n_x = M.n_x;
    B.n_y = M.n_y;
    B.n_vf = (M.n_x + 1) * M.n_y;
    B.N = mesh_faces(M) * na * q;
    B.nb = (int)((B.N + kChunk - 1) / kChunk);
    B.b0 = (int)nblk;
    B.pad = 0;
    B.e0 = E;
    B.d0 = Np;
    B.op = in2out[i];
    E += (int64_t)M.n_x * M.n_y;
    Np += (int64_t)B.nb * kChunk;
    nblk += B.nb;
  }
  if (E > INT_MAX || nblk > INT_MAX / 2) return set_error(ctx, EL_ERR_ARG, "el_trace_solve: batch too large");
  const BLay lay = make_layout(R);
  const bool f32 = opts.basis == EL_F32;
  // tmp, b, x (+ w and v_j with the FP32 basis) in FP64, then the basis
  const size_t v_bytes = sizeof(double) * (size_t)(f32 ? 4 : 3) * Np +
                         (f32 ? sizeof(float) : sizeof(double)) * (size_t)(R + 1) * Np;
  const size_t p_bytes = sizeof(double) * (size_t)nblk * (R + 2);
  const size_t h_bytes = sizeof(double) * (size_t)n_mesh * lay.S;
  const size_t s_bytes = (sizeof(BState) * n_mesh + 255) / 256 * 256;
  const size_t m_bytes = (sizeof(BMesh) * n_mesh + 255) / 256 * 256;
  el_status stt = ensure_ws(ctx, ctx->ws_gmres, v_bytes + p_bytes + h_bytes + s_bytes + m_bytes + 1024);
  if (stt) return stt;
  Batch bt;
  bt.ctx = ctx;
  bt.dv = de->view;
  bt.m = de->host.m;
  bt.op_dtype = op_dtype;
  bt.n_mesh = n_mesh;
  bt.E = E;
  bt.Np = Np;
  bt.nblk = (int)nblk;
  bt.lay = lay;
  bt.tol = opts.tol;
  bt.max_iter = opts.max_iter;
  bt.f32 = f32;
  char* base = reinterpret_cast<char*>(ctx->ws_gmres.ptr);
  bt.tmp = reinterpret_cast<double*>(base);
  bt.bcat = bt.tmp + Np;
  bt.xcat = bt.bcat + Np;
  if (f32) {
    bt.V = nullptr;
    bt.W = bt.xcat + Np;
    bt.Vf = reinterpret_cast<float*>(bt.W + Np);
    bt.partials = reinterpret_cast<double*>(bt.Vf + (size_t)(R + 1) * Np);   // Np is a multiple of kChunk
  } else {
    bt.V = bt.xcat + Np;
    bt.Vf = nullptr;
    bt.W = nullptr;
    bt.partials = bt.V + (size_t)(R + 1) * Np;
  }
  bt.hs = bt.partials + (size_t)nblk * (R + 2);
  bt.st = reinterpret_cast<BState*>(reinterpret_cast<char*>(bt.hs) + h_bytes);
  bt.ms = reinterpret_cast<BMesh*>(reinterpret_cast<char*>(bt.st) + s_bytes);
  hipStream_t s = ctx->stream;

  hipError_t he = hipMemcpyAsync(bt.ms, hm.data(), sizeof(BMesh) * n_mesh, hipMemcpyHostToDevice, s);
  for (int i = 0; i < n_mesh && he == hipSuccess; ++i)
    he = hipMemcpyAsync(bt.bcat + hm[i].d0, b[i], sizeof(double) * hm[i].N, hipMemcpyDeviceToDevice, s);
  if (he != hipSuccess) return hip_check(ctx, he, "el_trace_solve: staging");
  // the product's row shape (timed on the first mesh's product b -> tmp when
  // this operator type and size are new), fixed before the cycle is captured
  stt = matvec_shape(ctx, de, meshes[0], in2out[0], op_dtype, bt.bcat, bt.tmp, &bt.mv_shape);
  if (stt) return stt;
  hipLaunchKernelGGL(k_bzero, dim3(nblocks(Np, 256)), dim3(256), 0, s, bt.xcat, Np);
  if (opts.x0)   // starting guess (the padding between segments stays zero)
    for (int i = 0; i < n_mesh && he == hipSuccess; ++i)
      he = hipMemcpyAsync(bt.xcat + hm[i].d0, trace[i], sizeof(double) * hm[i].N, hipMemcpyDeviceToDevice, s);
  if (he != hipSuccess) return hip_check(ctx, he, "el_trace_solve: starting guess");
  // |b| per mesh (the state is not initialized yet: no skipping)
  hipLaunchKernelGGL(k_bdot<double>, dim3(bt.nblk), dim3(kVThreads), 0, s, bt.bcat, (int64_t)0, 0, bt.bcat, 1,
                     bt.ms, n_mesh, bt.st, P_ALL, bt.partials);
  hipLaunchKernelGGL(k_breduce, dim3(1, n_mesh), dim3(256), 0, s, bt.partials, 1, bt.ms, bt.st, P_ALL, bt.hs, lay,
                     lay.sc + 0, -1);
  hipLaunchKernelGGL(k_binit, dim3(nblocks(n_mesh, 64)), dim3(64), 0, s, n_mesh, bt.hs, lay, bt.st);
  stt = hip_check(ctx, hipGetLastError(), "el_trace_solve: init");
  if (stt) return stt;

  // graph of one restart cycle, cached on the context
  std::ostringstream key;
  key << base << ':' << R << ':' << n_mesh << ':' << E << ':' << Np << ':' << nblk << ':' << op_dtype << ':'
      << (const void*)de << ':' << opts.tol << ':' << opts.max_iter << ':' << f32 << ':' << bt.mv_shape;
  bool use_graph = opts.graph != 0;
  if (use_graph && (ctx->gm_key != key.str() || !ctx->gm_exec)) {
    if (ctx->gm_exec) {
      hipGraphExecDestroy(ctx->gm_exec);
      ctx->gm_exec = nullptr;
    }
    ctx->gm_key.clear();
    if (!ctx->cap_stream) {
      he = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
      if (he != hipSuccess) return hip_check(ctx, he, "el_trace_solve: capture stream");
    }
    he = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) return hip_check(ctx, he, "el_trace_solve: begin capture");
    for (int j = 0; j < R; ++j) bt.step(ctx->cap_stream, j);
    hipGraph_t graph = nullptr;
    he = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (he != hipSuccess) return hip_check(ctx, he, "el_trace_solve: end capture");
    he = hipGraphInstantiate(&ctx->gm_exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (he != hipSuccess) {
      ctx->gm_exec = nullptr;
      return hip_check(ctx, he, "el_trace_solve: graph instantiate");
    }
    ctx->gm_key = key.str();
  }

  std::vector<BState> hst(n_mesh);
  for (;;) {
    // true residual r = b - (I - P) x into V[0] (FP32 basis: into w), its
    // norm, test, v0 = r / |r|
    double* r = f32 ? bt.W : bt.V;
    bt.matvec(s, P_NOT_DONE, bt.xcat, bt.tmp, true);
    hipLaunchKernelGGL(k_bsub, dim3(bt.nblk), dim3(kVThreads), 0, s, bt.bcat, bt.tmp, r, bt.ms, n_mesh, bt.st,
                       P_NOT_DONE);
    hipLaunchKernelGGL(k_bdot<double>, dim3(bt.nblk), dim3(kVThreads), 0, s, r, (int64_t)0, 0, r, 1, bt.ms, n_mesh,
                       bt.st, P_NOT_DONE, bt.partials);
    hipLaunchKernelGGL(k_breduce, dim3(1, n_mesh), dim3(256), 0, s, bt.partials, 1, bt.ms, bt.st, P_NOT_DONE,
                       bt.hs, lay, lay.sc + 1, -1);
    hipLaunchKernelGGL(k_bstart, dim3(nblocks(n_mesh, 64)), dim3(64), 0, s, n_mesh, bt.hs, lay, bt.st, opts.tol,
                       opts.max_iter);
    bt.start_vector(s);
    he = hipMemcpyAsync(hst.data(), bt.st, sizeof(BState) * n_mesh, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return hip_check(ctx, he, "el_trace_solve: cycle");
    int active = 0;
    for (int i = 0; i < n_mesh; ++i) {
      if (hst[i].bad) {
        std::ostringstream os;
        os << "el_trace_solve: non-finite right-hand side or residual on mesh " << i;
        return set_error(ctx, EL_ERR_NONFINITE, os.str());
      }
      active += hst[i].active;
    }
    if (!active) break;
    if (use_graph) {
      he = hipGraphLaunch(ctx->gm_exec, s);
      if (he != hipSuccess) return hip_check(ctx, he, "el_trace_solve: graph launch");
    } else {
      for (int j = 0; j < R; ++j) bt.step(s, j);
    }
    hipLaunchKernelGGL(k_bfinish, dim3(n_mesh), dim3(64), 0, s, n_mesh, bt.hs, lay, bt.st);
    bt.update(s, P_USED, -1, lay.y, bt.xcat, -1.0, -1);
    stt = hip_check(ctx, hipGetLastError(), "el_trace_solve: step");
    if (stt) return stt;
  }
  bool all_conv = true;
  for (int i = 0; i < n_mesh; ++i) {
    // b = 0 has the solution 0 whatever the starting guess
    if (hst[i].bn == 0.0) he = hipMemsetAsync(trace[i], 0, sizeof(double) * hm[i].N, s);
    else he = hipMemcpyAsync(trace[i], bt.xcat + hm[i].d0, sizeof(double) * hm[i].N, hipMemcpyDeviceToDevice, s);
    if (he != hipSuccess) return hip_check(ctx, he, "el_trace_solve: copy out");
    rep[i].iters = hst[i].iters;
    rep[i].restarts = hst[i].restarts;
    rep[i].relres = hst[i].bn == 0.0 ? 0.0 : hst[i].relres;
    rep[i].converged = hst[i].conv;
    rep[i].reorth_passes = hst[i].reorths;
    if (!hst[i].conv) all_conv = false;
  }
  if (!all_conv) {
    set_error(ctx, EL_WARN_NOT_CONVERGED, "el_trace_solve: GMRES did not reach the tolerance within max_iter");
    return EL_WARN_NOT_CONVERGED;
  }
  return EL_OK;
}

}  // namespace el

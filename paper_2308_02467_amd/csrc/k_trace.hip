// Skeleton (trace) system of eq. hdg_global_mat and its GMRES solve (Sec. 2.3).
//
//   (I - P) t = b,  (P t)[out dofs of e] = in2out_e t[in dofs of e],
//   P = 0 on domain-inflow rows, b = boundary data on domain-inflow DOFs.
//
// k_matvec streams in2out (FP64 or bfloat16) from HBM once per product: one
// workgroup per element gathers the m inflow traces into LDS, groups of 8
// lanes reduce one operator row each with 16-byte loads, and each outflow
// DOF is written by its unique upwind element (no atomics).  Domain-inflow
// DOFs are copied through by the boundary element that sees them.
//
// GMRES(restart): x0 = 0, classical Gram-Schmidt with the DGKS
// reorthogonalization test (a second pass only when the norm of the new
// vector drops below 1/sqrt(2) of its value before the projection; the norms
// are fused into the dot-product and update passes), Givens rotations on the
// host from the scalars of each step, true residual checked at every
// restart.  Vectors and reductions are FP64.
#include <climits>
#include <cmath>
#include <cstdio>
#include <sstream>
#include <vector>

#include "el_internal.h"

namespace el {

namespace {

constexpr int kMVThreads = 256;
constexpr int kVec = 8;                       // values per thread in vector kernels
constexpr int kVThreads = 256;
constexpr int kChunk = kVThreads * kVec;      // elements per block
constexpr int kMaxCnt = 258;

struct MeshDev {
  int n_x, n_y, n_vf;
};

__device__ inline int face_of(const MeshDev& ms, int i, int j, int f) {
  switch (f) {
    case 0: return j * (ms.n_x + 1) + i;
    case 1: return j * (ms.n_x + 1) + i + 1;
    case 2: return ms.n_vf + j * ms.n_x + i;
    default: return ms.n_vf + (j + 1) * ms.n_x + i;
  }
}

__device__ inline bool on_domain_boundary(const MeshDev& ms, int i, int j, int f) {
  return (f == 0 && i == 0) || (f == 1 && i == ms.n_x - 1) || (f == 2 && j == 0) || (f == 3 && j == ms.n_y - 1);
}

__device__ inline double bf16_to_double(uint16_t b) {
  return (double)__uint_as_float(((uint32_t)b) << 16);
}

__global__ void k_element_dofs(DiscDev dv, MeshDev ms, int32_t* in_dofs, int32_t* out_dofs) {
  const int e = blockIdx.x;
  const int i = e % ms.n_x, j = e / ms.n_x;
  for (int t = threadIdx.x; t < dv.m; t += blockDim.x) {
    if (in_dofs) {
      int F = face_of(ms, i, j, dv.in_f[t]);
      in_dofs[(size_t)e * dv.m + t] = (F * dv.n_a + dv.in_k[t]) * dv.q + dv.in_j[t];
    }
    if (out_dofs) {
      int F = face_of(ms, i, j, dv.out_f[t]);
      out_dofs[(size_t)e * dv.m + t] = (F * dv.n_a + dv.out_k[t]) * dv.q + dv.out_j[t];
    }
  }
}

struct SideData {
  double g[4 * kMaxNa];
};

__global__ void k_trace_rhs(DiscDev dv, MeshDev ms, SideData sd, int64_t n_trace, double* b) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_trace) return;
  const int q = dv.q, na = dv.n_a;
  const int64_t fk = t / q;
  const int k = (int)(fk % na);
  const int64_t F = fk / na;
  int side = -1;
  if (F < ms.n_vf) {
    int i = (int)(F % (ms.n_x + 1));
    if (i == 0) side = 0;
    else if (i == ms.n_x) side = 1;
  } else {
    int jj = (int)((F - ms.n_vf) / ms.n_x);
    if (jj == 0) side = 2;
    else if (jj == ms.n_y) side = 3;
  }
  double v = 0.0;
  if (side >= 0) {
    const double sx = dv.sx[k], sy = dv.sy[k];
    bool inflow = (side == 0 && sx > 0) || (side == 1 && sx < 0) || (side == 2 && sy > 0) || (side == 3 && sy < 0);
    if (inflow) v = sd.g[side * na + k];
  }
  b[t] = v;
}

// Row dot products of one element operator with the gathered inflow traces.
// Groups of 8 lanes per row; each lane loads 16 bytes per step.
template <typename OpT>
__device__ inline double row_dot(const OpT* __restrict__ row, const double* tin, int m, int gl);

template <>
__device__ inline double row_dot<double>(const double* __restrict__ row, const double* tin, int m, int gl) {
  double acc = 0.0;
  for (int c = 2 * gl; c < m; c += 16) {
    double2 v = *reinterpret_cast<const double2*>(row + c);
    acc += v.x * tin[c] + v.y * tin[c + 1];
  }
  return acc;
}

template <>
__device__ inline double row_dot<float>(const float* __restrict__ row, const double* tin, int m, int gl) {
  double acc = 0.0;
  for (int c = 4 * gl; c < m; c += 32) {
    if (c + 4 <= m) {
      float4 v = *reinterpret_cast<const float4*>(row + c);
      acc += (double)v.x * tin[c] + (double)v.y * tin[c + 1] + (double)v.z * tin[c + 2] + (double)v.w * tin[c + 3];
    } else {
      for (int cc = c; cc < m; ++cc) acc += (double)row[cc] * tin[cc];
    }
  }
  return acc;
}

template <>
__device__ inline double row_dot<uint16_t>(const uint16_t* __restrict__ row, const double* tin, int m, int gl) {
  double acc = 0.0;
  for (int c = 8 * gl; c < m; c += 64) {
    if (c + 8 <= m) {
      uint4 v = *reinterpret_cast<const uint4*>(row + c);
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc += (double)__uint_as_float(w[u] << 16) * tin[c + 2 * u];
        acc += (double)__uint_as_float(w[u] & 0xffff0000u) * tin[c + 2 * u + 1];
      }
    } else {
      for (int cc = c; cc < m; ++cc) acc += bf16_to_double(row[cc]) * tin[cc];
    }
  }
  return acc;
}

template <typename OpT>
__global__ void __launch_bounds__(kMVThreads) k_matvec(DiscDev dv, MeshDev ms, const OpT* __restrict__ op,
                                                        const double* __restrict__ x, double* __restrict__ y) {
  extern __shared__ double tin[];
  const int e = blockIdx.x;
  const int i = e % ms.n_x, j = e / ms.n_x;
  const int m = dv.m;
  for (int t = threadIdx.x; t < m; t += kMVThreads) {
    const int f = dv.in_f[t];
    const int F = face_of(ms, i, j, f);
    const int dof = (F * dv.n_a + dv.in_k[t]) * dv.q + dv.in_j[t];
    const double v = x[dof];
    tin[t] = v;
    if (on_domain_boundary(ms, i, j, f)) y[dof] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 3, gl = lane & 7;
  const OpT* base = op + (size_t)e * m * m;
  for (int o = wave * 8 + g; o < m; o += (kMVThreads / 64) * 8) {
    double acc = row_dot<OpT>(base + (size_t)o * m, tin, m, gl);
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    if (gl == 0) {
      const int F = face_of(ms, i, j, dv.out_f[o]);
      const int dof = (F * dv.n_a + dv.out_k[o]) * dv.q + dv.out_j[o];
      y[dof] = x[dof] - acc;
    }
  }
}

// ---- vector kernels for GMRES -----------------------------------------------
__global__ void k_fill_d(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// out = a - b
__global__ void k_sub(const double* a, const double* b, double* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

__global__ void k_scale(double* p, int64_t n, double s) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] *= s;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// partials[blk][i] = sum over the block chunk of V[i] . w, i < cnt; with
// self_dot also partials[blk][cnt] = w . w
__global__ void __launch_bounds__(kVThreads) k_mdot(const double* __restrict__ V, int64_t ldv, int cnt,
                                                     const double* __restrict__ w, int64_t n, int self_dot,
                                                     double* __restrict__ partials) {
  __shared__ double s[kVThreads / 64][kMaxCnt];
  const int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x;
  double wr[kVec];
#pragma unroll
  for (int v = 0; v < kVec; ++v) {
    int64_t ix = base + v * kVThreads;
    wr[v] = ix < n ? w[ix] : 0.0;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = 0; i < cnt; ++i) {
    const double* vi = V + (size_t)i * ldv;
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      int64_t ix = base + v * kVThreads;
      if (ix < n) acc += vi[ix] * wr[v];
    }
    acc = wave_sum(acc);
    if (lane == 0) s[wave][i] = acc;
  }
  if (self_dot) {
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < kVec; ++v) acc += wr[v] * wr[v];
    acc = wave_sum(acc);
    if (lane == 0) s[wave][cnt] = acc;
  }
  __syncthreads();
  const int outc = cnt + (self_dot ? 1 : 0);
  for (int i = threadIdx.x; i < outc; i += kVThreads) {
    double t = 0.0;
    for (int wv = 0; wv < kVThreads / 64; ++wv) t += s[wv][i];
    partials[(size_t)blockIdx.x * outc + i] = t;
  }
}

// w -= sum_i h[i] V[i]; then partials of either V[i] . w (mode 0, cnt values)
// or w . w (mode 1, one value).
__global__ void __launch_bounds__(kVThreads) k_update(const double* __restrict__ V, int64_t ldv, int cnt,
                                                       const double* __restrict__ h, double* __restrict__ w,
                                                       int64_t n, double sign, int mode,
                                                       double* __restrict__ partials) {
  __shared__ double s[kVThreads / 64][kMaxCnt];
  __shared__ double hs[kMaxCnt];
  for (int i = threadIdx.x; i < cnt; i += kVThreads) hs[i] = sign * h[i];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x;
  double wr[kVec];
#pragma unroll
  for (int v = 0; v < kVec; ++v) {
    int64_t ix = base + v * kVThreads;
    wr[v] = ix < n ? w[ix] : 0.0;
  }
  for (int i = 0; i < cnt; ++i) {
    const double* vi = V + (size_t)i * ldv;
    const double hi = hs[i];
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      int64_t ix = base + v * kVThreads;
      if (ix < n) wr[v] -= hi * vi[ix];
    }
  }
#pragma unroll
  for (int v = 0; v < kVec; ++v) {
    int64_t ix = base + v * kVThreads;
    if (ix < n) w[ix] = wr[v];
  }
  if (mode < 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (mode == 0) {
    for (int i = 0; i < cnt; ++i) {
      const double* vi = V + (size_t)i * ldv;
      double acc = 0.0;
#pragma unroll
      for (int v = 0; v < kVec; ++v) {
        int64_t ix = base + v * kVThreads;
        if (ix < n) acc += vi[ix] * wr[v];
      }
      acc = wave_sum(acc);
      if (lane == 0) s[wave][i] = acc;
    }
  } else {
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < kVec; ++v) acc += wr[v] * wr[v];
    acc = wave_sum(acc);
    if (lane == 0) s[wave][0] = acc;
  }
  __syncthreads();
  const int outc = mode == 0 ? cnt : 1;
  for (int i = threadIdx.x; i < outc; i += kVThreads) {
    double t = 0.0;
    for (int wv = 0; wv < kVThreads / 64; ++wv) t += s[wv][i];
    partials[(size_t)blockIdx.x * outc + i] = t;
  }
}

// out[i] = sum_b partials[b][i], one block per i (fixed order: deterministic)
__global__ void k_reduce(const double* __restrict__ partials, int nblk, int cnt, double* __restrict__ out) {
  __shared__ double s[256 / 64];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) acc += partials[(size_t)b * cnt + i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[i] = s[0] + s[1] + s[2] + s[3];
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

el_status launch_element_dofs(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh,
                              int32_t* in_dofs, int32_t* out_dofs) {
  MeshDev ms{mesh.n_x, mesh.n_y, (mesh.n_x + 1) * mesh.n_y};
  int64_t E = (int64_t)mesh.n_x * mesh.n_y;
  hipLaunchKernelGGL(k_element_dofs, dim3((unsigned)E), dim3(256), 0, ctx->stream, de->view, ms, in_dofs, out_dofs);
  return hip_check(ctx, hipGetLastError(), "launch k_element_dofs");
}

el_status launch_trace_rhs(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh,
                           const double* g_side_host, double* b) {
  MeshDev ms{mesh.n_x, mesh.n_y, (mesh.n_x + 1) * mesh.n_y};
  SideData sd;
  const int na = de->host.n_a;
  for (int s = 0; s < 4; ++s)
    for (int k = 0; k < na; ++k) {
      double v = g_side_host[s * na + k];
      if (!std::isfinite(v)) return set_error(ctx, EL_ERR_NONFINITE, "el_trace_rhs: non-finite boundary value");
      sd.g[s * na + k] = v;
    }
  int64_t nt = mesh_faces(mesh) * na * de->host.q;
  hipLaunchKernelGGL(k_trace_rhs, dim3(blocks_for(nt, 256)), dim3(256), 0, ctx->stream, de->view, ms, sd, nt, b);
  return hip_check(ctx, hipGetLastError(), "launch k_trace_rhs");
}

el_status launch_trace_matvec(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh, const void* in2out,
                              int op_dtype, const double* x, double* y) {
  MeshDev ms{mesh.n_x, mesh.n_y, (mesh.n_x + 1) * mesh.n_y};
  const int64_t E = (int64_t)mesh.n_x * mesh.n_y;
  const size_t smem = sizeof(double) * de->host.m;
  if (op_dtype == EL_F64)
    hipLaunchKernelGGL(k_matvec<double>, dim3((unsigned)E), dim3(kMVThreads), smem, ctx->stream, de->view, ms,
                       reinterpret_cast<const double*>(in2out), x, y);
  else if (op_dtype == EL_F32)
    hipLaunchKernelGGL(k_matvec<float>, dim3((unsigned)E), dim3(kMVThreads), smem, ctx->stream, de->view, ms,
                       reinterpret_cast<const float*>(in2out), x, y);
  else
    hipLaunchKernelGGL(k_matvec<uint16_t>, dim3((unsigned)E), dim3(kMVThreads), smem, ctx->stream, de->view, ms,
                       reinterpret_cast<const uint16_t*>(in2out), x, y);
  return hip_check(ctx, hipGetLastError(), "launch k_matvec");
}

namespace {

struct Gm {
  el_ctx* ctx;
  int64_t n;
  int nblk;
  double* partials;
  double* hdev;   // [3 * kMaxCnt]
  hipStream_t s;

  el_status err(const char* what) { return hip_check(ctx, hipGetLastError(), what); }

  // out_dev[0..cnt) = V[0..cnt) . w; with self_dot also out_dev[cnt] = w . w
  el_status mdot(const double* V, int64_t ldv, int cnt, const double* w, double* out_dev, int self_dot = 0) {
    hipLaunchKernelGGL(k_mdot, dim3(nblk), dim3(kVThreads), 0, s, V, ldv, cnt, w, n, self_dot, partials);
    hipLaunchKernelGGL(k_reduce, dim3(cnt + self_dot), dim3(256), 0, s, partials, nblk, cnt + self_dot, out_dev);
    return err("gmres mdot");
  }
  // w -= sign * V h; then dots (mode 0) or norm^2 (mode 1) into out_dev
  el_status update(const double* V, int64_t ldv, int cnt, const double* h, double* w, double sign, int mode,
                   double* out_dev) {
    hipLaunchKernelGGL(k_update, dim3(nblk), dim3(kVThreads), 0, s, V, ldv, cnt, h, w, n, sign, mode, partials);
    if (mode >= 0)
      hipLaunchKernelGGL(k_reduce, dim3(mode == 0 ? cnt : 1), dim3(256), 0, s, partials, nblk, mode == 0 ? cnt : 1,
                         out_dev);
    return err("gmres update");
  }
};

}  // namespace

el_status run_trace_solve(el_ctx* ctx, el_ctx::DiscEntry* de, int n_mesh, const el_mesh* meshes,
                          const void* const* in2out, int op_dtype, const double* const* b,
                          double* const* trace, const el_gmres_opts& opts, el_gmres_report* rep) {
  const int R = opts.restart;
  bool all_conv = true;
  for (int mi = 0; mi < n_mesh; ++mi) {
    const el_mesh& mesh = meshes[mi];
    const int64_t N = mesh_faces(mesh) * de->host.n_a * de->host.q;
    const int nblk = (int)((N + kChunk - 1) / kChunk);
    size_t vbytes = sizeof(double) * (size_t)(R + 2) * N;
    size_t pbytes = sizeof(double) * (size_t)nblk * kMaxCnt;
    size_t hbytes = sizeof(double) * 4 * kMaxCnt;
    el_status st = ensure_ws(ctx, ctx->ws_gmres, vbytes + pbytes + hbytes);
    if (st) return st;
    double* V = reinterpret_cast<double*>(ctx->ws_gmres.ptr);     // [R+1][N]
    double* tmp = V + (size_t)(R + 1) * N;                          // [N]
    Gm g{ctx, N, nblk, tmp + N, nullptr, ctx->stream};
    g.hdev = g.partials + (size_t)nblk * kMaxCnt;
    double* x = trace[mi];
    hipStream_t s = ctx->stream;
    const unsigned nb256 = blocks_for(N, 256);
    hipLaunchKernelGGL(k_fill_d, dim3(nb256), dim3(256), 0, s, x, N, 0.0);
    // ||b||
    st = g.mdot(b[mi], 0, 1, b[mi], g.hdev, 0);
    if (st) return st;
    double bnorm2 = 0.0;
    hipMemcpyAsync(&bnorm2, g.hdev, sizeof(double), hipMemcpyDeviceToHost, s);
    st = hip_check(ctx, hipStreamSynchronize(s), "gmres ||b||");
    if (st) return st;
    const double bn = std::sqrt(bnorm2);
    el_gmres_report& r = rep[mi];
    r.iters = 0; r.restarts = 0; r.relres = 0.0; r.converged = 1;
    if (bn == 0.0) continue;
    if (!std::isfinite(bn)) {
      std::ostringstream os;
      os << "el_trace_solve: non-finite right-hand side on mesh " << mi;
      return set_error(ctx, EL_ERR_NONFINITE, os.str());
    }
    std::vector<double> H((size_t)(R + 1) * R), cs(R), sn(R), gv(R + 1), y(R), hh(2 * kMaxCnt + 1);
    int it = 0;
    double relres = 1.0;
    while (true) {
      // r = b - (I - P) x  into V[0]
      if (it == 0) {
        hipMemcpyAsync(V, b[mi], sizeof(double) * N, hipMemcpyDeviceToDevice, s);
      } else {
        st = launch_trace_matvec(ctx, de, mesh, in2out[mi], op_dtype, x, tmp);
        if (st) return st;
        hipLaunchKernelGGL(k_sub, dim3(nb256), dim3(256), 0, s, b[mi], tmp, V, N);
      }
      st = g.mdot(V, 0, 1, V, g.hdev, 0);
      if (st) return st;
      double beta2 = 0.0;
      hipMemcpyAsync(&beta2, g.hdev, sizeof(double), hipMemcpyDeviceToHost, s);
      st = hip_check(ctx, hipStreamSynchronize(s), "gmres residual");
      if (st) return st;
      const double beta = std::sqrt(beta2);
      relres = beta / bn;
      if (!std::isfinite(relres)) {
        std::ostringstream os;
        os << "el_trace_solve: GMRES produced a non-finite residual on mesh " << mi;
        return set_error(ctx, EL_ERR_NONFINITE, os.str());
      }
      if (relres <= opts.tol || it >= opts.max_iter) break;
      hipLaunchKernelGGL(k_scale, dim3(nb256), dim3(256), 0, s, V, N, 1.0 / beta);
      std::fill(H.begin(), H.end(), 0.0);
      std::fill(gv.begin(), gv.end(), 0.0);
      gv[0] = beta;
      int kused = 0;
      for (int j = 0; j < R; ++j) {
        double* vj1 = V + (size_t)(j + 1) * N;
        st = launch_trace_matvec(ctx, de, mesh, in2out[mi], op_dtype, V + (size_t)j * N, vj1);
        if (st) return st;
        const int cnt = j + 1;
        double* h1 = g.hdev;                    // [cnt] coefficients, [cnt] = ||w||^2 before
        double* h2 = g.hdev + kMaxCnt;
        double* nrm = g.hdev + 2 * kMaxCnt;
        // classical Gram-Schmidt, one pass; a second pass when the norm drops
        // below 1/sqrt(2) of its value before the projection (DGKS criterion)
        st = g.mdot(V, N, cnt, vj1, h1, 1);
        if (st) return st;
        st = g.update(V, N, cnt, h1, vj1, 1.0, 1, nrm);
        if (st) return st;
        hipMemcpyAsync(hh.data(), h1, sizeof(double) * (cnt + 1), hipMemcpyDeviceToHost, s);
        hipMemcpyAsync(hh.data() + kMaxCnt, nrm, sizeof(double), hipMemcpyDeviceToHost, s);
        st = hip_check(ctx, hipStreamSynchronize(s), "gmres step");
        if (st) return st;
        double* Hc = H.data();  // column-major: H[i + j*(R+1)]
        for (int i = 0; i <= j; ++i) Hc[i + (size_t)j * (R + 1)] = hh[i];
        const double w0 = std::sqrt(std::max(hh[cnt], 0.0));
        double hn = std::sqrt(std::max(hh[kMaxCnt], 0.0));
        if (hn < 0.70710678118654752 * w0) {
          st = g.mdot(V, N, cnt, vj1, h2, 0);
          if (st) return st;
          st = g.update(V, N, cnt, h2, vj1, 1.0, 1, nrm);
          if (st) return st;
          hipMemcpyAsync(hh.data(), h2, sizeof(double) * cnt, hipMemcpyDeviceToHost, s);
          hipMemcpyAsync(hh.data() + kMaxCnt, nrm, sizeof(double), hipMemcpyDeviceToHost, s);
          st = hip_check(ctx, hipStreamSynchronize(s), "gmres reorthogonalization");
          if (st) return st;
          for (int i = 0; i <= j; ++i) Hc[i + (size_t)j * (R + 1)] += hh[i];
          hn = std::sqrt(std::max(hh[kMaxCnt], 0.0));
        }
        Hc[j + 1 + (size_t)j * (R + 1)] = hn;
        if (hn > 0.0) hipLaunchKernelGGL(k_scale, dim3(nb256), dim3(256), 0, s, vj1, N, 1.0 / hn);
        for (int i = 0; i < j; ++i) {
          double a0 = Hc[i + (size_t)j * (R + 1)], a1 = Hc[i + 1 + (size_t)j * (R + 1)];
          Hc[i + (size_t)j * (R + 1)] = cs[i] * a0 + sn[i] * a1;
          Hc[i + 1 + (size_t)j * (R + 1)] = -sn[i] * a0 + cs[i] * a1;
        }
        const double a0 = Hc[j + (size_t)j * (R + 1)], a1 = Hc[j + 1 + (size_t)j * (R + 1)];
        const double den = std::hypot(a0, a1);
        cs[j] = a0 / den;
        sn[j] = a1 / den;
        Hc[j + (size_t)j * (R + 1)] = den;
        Hc[j + 1 + (size_t)j * (R + 1)] = 0.0;
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
        ++it;
        kused = j + 1;
        if (std::fabs(gv[j + 1]) / bn <= opts.tol || it >= opts.max_iter || hn == 0.0) break;
      }
      // y = H^{-1} g (upper triangular), x += V y
      for (int i = kused - 1; i >= 0; --i) {
        double acc = gv[i];
        for (int k = i + 1; k < kused; ++k) acc -= H[i + (size_t)k * (R + 1)] * y[k];
        y[i] = acc / H[i + (size_t)i * (R + 1)];
      }
      hipMemcpyAsync(g.hdev + 3 * kMaxCnt, y.data(), sizeof(double) * kused, hipMemcpyHostToDevice, s);
      st = g.update(V, N, kused, g.hdev + 3 * kMaxCnt, x, -1.0, -1, nullptr);
      if (st) return st;
      r.restarts++;
    }
    r.iters = it;
    r.relres = relres;
    r.converged = relres <= opts.tol;
    if (!r.converged) all_conv = false;
  }
  if (!all_conv) {
    set_error(ctx, EL_WARN_NOT_CONVERGED, "el_trace_solve: GMRES did not reach the tolerance within max_iter");
    return EL_WARN_NOT_CONVERGED;
  }
  return EL_OK;
}

}  // namespace el

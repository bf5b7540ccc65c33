// Element-wise recovery (Alg. 1 step 4, eq. hdg_local_mat_sol) and the mean
// intensity (eq. ang_ave), plus the element L2 norms used for the relative
// error of Sec. 3.2.1.
//
// k_recover streams in2sol [E][n][m] (FP64, FP32, FP16 or bfloat16) once: one workgroup
// per element gathers the m inflow traces into LDS, groups of 8 lanes reduce
// one operator row each, u is staged in LDS and the ordinate average is taken
// there.  HBM-bound: n*m operator entries per element.
#include <cmath>
#include <sstream>

#include "el_internal.h"
#include "trace_dev.h"

namespace el {
namespace {

constexpr int kThreads = 256;

// rows = number of operator rows (n for in2sol, nn for in2mean);
// mode 0: u (and optional mean over ordinates) from in2sol;
// mode 1: mean directly from in2mean.
// add: the element's source response [E][rows] added to the rows, or null.
template <typename OpT>
__global__ void __launch_bounds__(kThreads) k_recover(DiscDev dv, MeshDev ms, const OpT* __restrict__ op,
                                                       int rows, int mode, const double* __restrict__ t,
                                                       double* __restrict__ u, double* __restrict__ mean,
                                                       const double* __restrict__ add) {
  extern __shared__ double sm[];
  double* tin = sm;             // [m]
  double* ub = sm + dv.m;       // [rows]
  const int e = blockIdx.x;
  const int i = e % ms.n_x, j = e / ms.n_x;
  const int m = dv.m;
  for (int c = threadIdx.x; c < m; c += kThreads) {
    const int F = face_of(ms, i, j, dv.in_f[c]);
    tin[c] = t[(F * dv.n_a + dv.in_k[c]) * dv.q + dv.in_j[c]];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 3, gl = lane & 7;
  const OpT* base = op + (size_t)e * rows * m;
  for (int r = wave * 8 + g; r < rows; r += (kThreads / 64) * 8) {
    double acc = row_dot<OpT>(base + (size_t)r * m, tin, m, gl);
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    if (gl == 0) ub[r] = add ? acc + add[(size_t)e * rows + r] : acc;
  }
  __syncthreads();
  if (mode == 1) {
    for (int r = threadIdx.x; r < rows; r += kThreads) mean[(size_t)e * rows + r] = ub[r];
    return;
  }
  if (u)
    for (int r = threadIdx.x; r < rows; r += kThreads) u[(size_t)e * rows + r] = ub[r];
  if (mean) {
    const int nn = dv.nn;
    const double s = 1.0 / dv.n_a;
    for (int nd = threadIdx.x; nd < nn; nd += kThreads) {
      double acc = 0.0;
      for (int k = 0; k < dv.n_a; ++k) acc += ub[k * nn + nd];
      mean[(size_t)e * nn + nd] = acc * s;
    }
  }
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// partial[blk][0..1] over elements of the block chunk
__global__ void k_l2_partial(const double* __restrict__ W, int nn, int64_t E, const double* __restrict__ h,
                             const double* __restrict__ a, const double* __restrict__ ref, double* partial) {
  __shared__ double s0[4], s1[4];
  double d2 = 0.0, r2 = 0.0;
  const int64_t total = E * nn;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / nn;
    const int nd = (int)(idx - e * nn);
    const double hw = 0.25 * h[e] * h[e] * W[nd];
    const double d = a[idx] - ref[idx];
    d2 += hw * d * d;
    r2 += hw * ref[idx] * ref[idx];
  }
  d2 = wave_sum(d2);
  r2 = wave_sum(r2);
  if ((threadIdx.x & 63) == 0) { s0[threadIdx.x >> 6] = d2; s1[threadIdx.x >> 6] = r2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s0[0] + s0[1] + s0[2] + s0[3];
    partial[2 * blockIdx.x + 1] = s1[0] + s1[1] + s1[2] + s1[3];
  }
}

// Energy balance of one element, column by column: sum_o w_o in2out[o][i] +
// sum_(k,nd) W_nd (h kappa_nd / 2) in2sol[(k,nd)][i] = w_i.  Each column of
// in2out is rescaled so that the balance holds exactly; the scale is taken in
// FP64 from the stored values and the result is rounded once to the output
// type TW (out may be i2o itself when TW == T).  Elements with mask == 0 are
// copied unchanged (converted to TW); in place they are skipped.
template <typename T, typename TW>
__global__ void k_conserve(DiscDev dv, int64_t E, const double* __restrict__ h, const double* __restrict__ kappa,
                           const T* i2o, const T* __restrict__ i2s, TW* out, int rows, double mult,
                           const uint8_t* __restrict__ mask) {
  const int64_t e = blockIdx.x;
  if (e >= E) return;
  const bool keep = mask && !mask[e];
  const bool in_place = reinterpret_cast<const void*>(out) == reinterpret_cast<const void*>(i2o);
  if (keep && in_place) return;
  extern __shared__ double wa[];   // [nn] = W_nd h kappa_nd / 2
  const int nn = dv.nn, m = dv.m;
  for (int nd = threadIdx.x; nd < nn; nd += blockDim.x) wa[nd] = dv.W[nd] * 0.5 * h[e] * kappa[e * nn + nd];
  __syncthreads();
  const T* S = i2s + (size_t)e * rows * m;
  const T* O = i2o + (size_t)e * m * m;
  TW* W = out + (size_t)e * m * m;
  // (four partial sums per thread, so that four loads of a column are in
  // flight at a time; rows = k nn + nd, a multiple of nn)
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    double s = 1.0;
    if (!keep) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
      for (int r0 = 0; r0 < rows; r0 += nn) {
        const T* Sk = S + (int64_t)r0 * m + c;
        int nd = 0;
        for (; nd + 4 <= nn; nd += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) a[u] += wa[nd + u] * op_to_double(Sk[(int64_t)(nd + u) * m]);
        }
        for (; nd < nn; ++nd) a[0] += wa[nd] * op_to_double(Sk[(int64_t)nd * m]);
      }
      const double absorb = ((a[0] + a[1]) + (a[2] + a[3])) * mult;
      double b[4] = {0.0, 0.0, 0.0, 0.0};
      int o = 0;
      for (; o + 4 <= m; o += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) b[u] += dv.out_val[o + u] * op_to_double(O[(int64_t)(o + u) * m + c]);
      }
      for (; o < m; ++o) b[0] += dv.out_val[o] * op_to_double(O[(int64_t)o * m + c]);
      const double sum = (b[0] + b[1]) + (b[2] + b[3]);
      const double target = dv.in_val[c] - absorb;
      if (sum > 0.0 && target > 0.0) s = target / sum;
    }
#pragma unroll 4
    for (int o = 0; o < m; ++o) W[(int64_t)o * m + c] = op_from_double<TW>(s * op_to_double(O[(int64_t)o * m + c]));
  }
}

}  // namespace

el_status launch_conserve(el_ctx* ctx, el_ctx::DiscEntry* de, int64_t E, const double* h, const double* kappa,
                          const void* in2out, const void* in2vol, int form, int op_dtype, const uint8_t* mask,
                          void* out, int out_dtype) {
  const size_t smem = sizeof(double) * de->host.nn;
  // in2sol: absorption sums all (k, nd) rows; in2mean holds the ordinate
  // average, so its nn rows are summed and multiplied by N_a
  const bool mean = form == EL_FORM_IN2MEAN;
  const int rows = mean ? de->host.nn : de->host.n;
  const double mult = mean ? (double)de->host.n_a : 1.0;
  auto run = [&](auto in_tag, auto out_tag) {
    using T = decltype(in_tag);
    using TW = decltype(out_tag);
    hipLaunchKernelGGL((k_conserve<T, TW>), dim3((unsigned)E), dim3(256), smem, ctx->stream, de->view, E, h, kappa,
                       reinterpret_cast<const T*>(in2out), reinterpret_cast<const T*>(in2vol),
                       reinterpret_cast<TW*>(out), rows, mult, mask);
  };
  if (out_dtype == op_dtype) with_op_type(op_dtype, [&](auto tag) { run(tag, tag); });
  else if (op_dtype == EL_F32 && out_dtype == EL_F16) run(float{}, _Float16{});
  else if (op_dtype == EL_F32 && out_dtype == EL_BF16) run(float{}, uint16_t{});
  else return set_error(ctx, EL_ERR_ARG, "el_conserve: output type must be the input type, or FP16/BF16 from FP32");
  return hip_check(ctx, hipGetLastError(), "launch k_conserve");
}

el_status launch_recover(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh, const void* in2sol,
                         int op_dtype, const double* trace, double* u, double* mean, const double* src2sol) {
  MeshDev ms{mesh.n_x, mesh.n_y, (mesh.n_x + 1) * mesh.n_y};
  const int64_t E = (int64_t)mesh.n_x * mesh.n_y;
  const DiscHost& dh = de->host;
  const size_t smem = sizeof(double) * (dh.m + dh.n);
  with_op_type(op_dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL(k_recover<T>, dim3((unsigned)E), dim3(kThreads), smem, ctx->stream, de->view, ms,
                       reinterpret_cast<const T*>(in2sol), dh.n, 0, trace, u, mean, src2sol);
  });
  return hip_check(ctx, hipGetLastError(), "launch k_recover");
}

el_status launch_recover_mean(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh, const void* in2mean,
                              int op_dtype, const double* trace, double* mean, const double* src2mean) {
  MeshDev ms{mesh.n_x, mesh.n_y, (mesh.n_x + 1) * mesh.n_y};
  const int64_t E = (int64_t)mesh.n_x * mesh.n_y;
  const DiscHost& dh = de->host;
  const size_t smem = sizeof(double) * (dh.m + dh.nn);
  with_op_type(op_dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL(k_recover<T>, dim3((unsigned)E), dim3(kThreads), smem, ctx->stream, de->view, ms,
                       reinterpret_cast<const T*>(in2mean), dh.nn, 1, trace, nullptr, mean, src2mean);
  });
  return hip_check(ctx, hipGetLastError(), "launch k_recover(mean)");
}

// b[outflow DOF o of element e] += src2out[e][o] (each outflow DOF belongs to
// exactly one element)
__global__ void k_trace_add_source(DiscDev dv, MeshDev ms, int64_t E, const double* __restrict__ s2out,
                                   double* __restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * dv.m) return;
  const int64_t e = t / dv.m;
  const int o = (int)(t - e * dv.m);
  const int i = (int)(e % ms.n_x), j = (int)(e / ms.n_x);
  const int F = face_of(ms, i, j, dv.out_f[o]);
  b[(F * dv.n_a + dv.out_k[o]) * dv.q + dv.out_j[o]] += s2out[t];
}

el_status launch_trace_add_source(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh, const double* s2out,
                                  double* b) {
  MeshDev ms{mesh.n_x, mesh.n_y, (mesh.n_x + 1) * mesh.n_y};
  const int64_t E = (int64_t)mesh.n_x * mesh.n_y;
  hipLaunchKernelGGL(k_trace_add_source, dim3((unsigned)((E * de->host.m + 255) / 256)), dim3(256), 0, ctx->stream,
                     de->view, ms, E, s2out, b);
  return hip_check(ctx, hipGetLastError(), "launch k_trace_add_source");
}

el_status launch_mean_l2(el_ctx* ctx, el_ctx::DiscEntry* de, int64_t E, const double* h, const double* a,
                         const double* ref, double* out_host) {
  const int nblk = 512;
  el_status st = ensure_ws(ctx, ctx->ws_small, sizeof(double) * 2 * nblk + 4096);
  if (st) return st;
  double* partial = reinterpret_cast<double*>(reinterpret_cast<char*>(ctx->ws_small.ptr) + 4096);
  hipLaunchKernelGGL(k_l2_partial, dim3(nblk), dim3(256), 0, ctx->stream, de->view.W, de->host.nn, E, h, a, ref,
                     partial);
  st = hip_check(ctx, hipGetLastError(), "launch k_l2_partial");
  if (st) return st;
  std::vector<double> hp(2 * nblk);
  hipError_t he = hipMemcpyAsync(hp.data(), partial, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, ctx->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return hip_check(ctx, he, "el_mean_l2");
  double d2 = 0.0, r2 = 0.0;
  for (int b = 0; b < nblk; ++b) { d2 += hp[2 * b]; r2 += hp[2 * b + 1]; }
  out_host[0] = d2;
  out_host[1] = r2;
  return EL_OK;
}

}  // namespace el

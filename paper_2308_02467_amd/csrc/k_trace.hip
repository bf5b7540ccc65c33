// Skeleton (trace) system of eq. hdg_global_mat (Sec. 2.3): element DOF
// maps, the right-hand side and the single-mesh product
//
//   (I - P) t,  (P t)[out dofs of e] = in2out_e t[in dofs of e],
//   P = 0 on domain-inflow rows, b = boundary data on domain-inflow DOFs.
//
// k_matvec streams in2out (FP64, FP32 or bfloat16) from HBM once per
// product: one workgroup per element (body in trace_dev.h).  The batched
// GMRES solve lives in k_gmres.hip.
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <sstream>
#include <vector>

#include "el_internal.h"
#include "trace_dev.h"

namespace el {

namespace {

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

template <typename OpT, int R>
__global__ void __launch_bounds__(kMVThreads) k_matvec(DiscDev dv, MeshDev ms, const OpT* __restrict__ op,
                                                        const double* __restrict__ x, double* __restrict__ y) {
  extern __shared__ double sm[];
  const int e = blockIdx.x;
  matvec_element<OpT, true, R>(dv, ms, e, op + (size_t)e * dv.m * dv.m, x, y, sm);
}

// one product with row shape index `shape` (kMvShapes)
template <typename OpT>
void launch_matvec_shape(int shape, hipStream_t s, const DiscDev& dv, const MeshDev& ms, int64_t E, size_t smem,
                         const OpT* op, const double* x, double* y) {
  switch (shape) {
    case 1: hipLaunchKernelGGL((k_matvec<OpT, 2>), dim3((unsigned)E), dim3(kMVThreads), smem, s, dv, ms, op, x, y); break;
    case 2: hipLaunchKernelGGL((k_matvec<OpT, 8>), dim3((unsigned)E), dim3(kMVThreads), smem, s, dv, ms, op, x, y); break;
    default: hipLaunchKernelGGL((k_matvec<OpT, 4>), dim3((unsigned)E), dim3(kMVThreads), smem, s, dv, ms, op, x, y);
  }
}

const char* op_dtype_name(int t) {
  return t == EL_F64 ? "f64" : t == EL_F32 ? "f32" : t == EL_F16 ? "f16" : "bf16";
}

std::atomic<int> g_force_shape{-1};   // >= 0: this row shape everywhere (el_matvec_shape)

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

std::vector<std::string> matvec_shape_names() {
  return {"4 rows x 4 chunks", "2 rows x 8 chunks", "8 rows x 2 chunks"};
}

// The skeleton product's row shape for operators of op_dtype with m inflow
// DOFs per element: the pinned one, the tuned one, or, on first use, the
// fastest of the candidates timed (one warm-up and two timed launches each)
// on this call's own product, whose output y it overwrites.
el_status matvec_shape(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh, const void* in2out, int op_dtype,
                       const double* x, double* y, int* shape) {
  const int forced = g_force_shape.load();
  if (forced >= 0) {
    *shape = forced;
    return EL_OK;
  }
  std::ostringstream ks;
  ks << ctx->arch << " matvec " << op_dtype_name(op_dtype) << " m=" << de->host.m;
  const std::string key = ks.str();
  const int n_shapes = (int)matvec_shape_names().size();
  if (tune_find(key, shape) && *shape >= 0 && *shape < n_shapes) return EL_OK;
  MeshDev ms{mesh.n_x, mesh.n_y, (mesh.n_x + 1) * mesh.n_y};
  const int64_t E = (int64_t)mesh.n_x * mesh.n_y;
  const size_t smem = matvec_smem_bytes(de->host.m);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return hip_check(ctx, hipGetLastError(), "matvec tuner events");
  std::vector<float> ms_of(n_shapes, 0.f);
  int best = 0;
  el_status st = EL_OK;
  for (int v = 0; v < n_shapes && !st; ++v) {
    with_op_type(op_dtype, [&](auto tag) {
      using T = decltype(tag);
      const T* op = reinterpret_cast<const T*>(in2out);
      launch_matvec_shape<T>(v, ctx->stream, de->view, ms, E, smem, op, x, y);
      hipEventRecord(e0, ctx->stream);
      launch_matvec_shape<T>(v, ctx->stream, de->view, ms, E, smem, op, x, y);
      launch_matvec_shape<T>(v, ctx->stream, de->view, ms, E, smem, op, x, y);
      hipEventRecord(e1, ctx->stream);
    });
    st = hip_check(ctx, hipEventSynchronize(e1), "matvec tuner");
    if (!st) {
      hipEventElapsedTime(&ms_of[v], e0, e1);
      ms_of[v] *= 0.5f;
      if (ms_of[v] < ms_of[best]) best = v;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  tune_store(key, best, ms_of);
  *shape = best;
  return EL_OK;
}

el_status launch_trace_matvec(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh, const void* in2out,
                              int op_dtype, const double* x, double* y) {
  int shape = 0;
  el_status st = matvec_shape(ctx, de, mesh, in2out, op_dtype, x, y, &shape);
  if (st) return st;
  MeshDev ms{mesh.n_x, mesh.n_y, (mesh.n_x + 1) * mesh.n_y};
  const int64_t E = (int64_t)mesh.n_x * mesh.n_y;
  const size_t smem = matvec_smem_bytes(de->host.m);
  with_op_type(op_dtype, [&](auto tag) {
    using T = decltype(tag);
    launch_matvec_shape<T>(shape, ctx->stream, de->view, ms, E, smem, reinterpret_cast<const T*>(in2out), x, y);
  });
  return hip_check(ctx, hipGetLastError(), "launch k_matvec");
}

}  // namespace el

extern "C" el_status el_matvec_shape(int shape) {
  if (shape < -1 || shape >= (int)el::matvec_shape_names().size()) return EL_ERR_ARG;
  el::g_force_shape.store(shape);
  return EL_OK;
}

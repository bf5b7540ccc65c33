// Skeleton right-hand side from boundary radiance that varies along the
// boundary (Sec. 2.2.2: b = P_M g on the domain-inflow trace DOFs, which
// with collocated LGL face nodes is the nodal interpolation of g), the
// general form of el_trace_rhs (constant per side).
//
// g_bnd holds, for every boundary face, the values of g at the face's q LGL
// nodes for every ordinate: [side][face along the side][n_a][q], sides W, E
// (n_y faces each, bottom to top) then S, N (n_x faces each, left to
// right), nodes in increasing coordinate along the face.  Values at
// outflow (s . n >= 0) boundary DOFs are not read.
#include <climits>
#include <cmath>
#include <sstream>

#include "el_internal.h"
#include "trace_dev.h"

namespace el {
namespace {

__global__ void k_fill_flag(int* f, int v) {
  if (threadIdx.x == 0) f[0] = v;
}

// Offset of side s in g_bnd, in units of n_a * q values.
__device__ inline int64_t side_offset(const MeshDev& ms, int s) {
  return s == 0 ? 0 : s == 1 ? ms.n_y : s == 2 ? 2 * (int64_t)ms.n_y : 2 * (int64_t)ms.n_y + ms.n_x;
}

__global__ void k_trace_rhs_nodal(DiscDev dv, MeshDev ms, const double* __restrict__ g, int64_t n_trace,
                                  double* __restrict__ b, int* bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_trace) return;
  const int q = dv.q, na = dv.n_a;
  const int j = (int)(t % q);
  const int64_t fk = t / q;
  const int k = (int)(fk % na);
  const int64_t F = fk / na;
  int side = -1;
  int64_t pos = 0;   // face index along the side
  if (F < ms.n_vf) {
    const int i = (int)(F % (ms.n_x + 1));
    pos = F / (ms.n_x + 1);
    if (i == 0) side = 0;
    else if (i == ms.n_x) side = 1;
  } else {
    const int64_t G = F - ms.n_vf;
    const int jj = (int)(G / ms.n_x);
    pos = G % ms.n_x;
    if (jj == 0) side = 2;
    else if (jj == ms.n_y) side = 3;
  }
  double v = 0.0;
  if (side >= 0) {
    const double sx = dv.sx[k], sy = dv.sy[k];
    const bool inflow = (side == 0 && sx > 0) || (side == 1 && sx < 0) || (side == 2 && sy > 0) ||
                        (side == 3 && sy < 0);
    if (inflow) {
      v = g[((side_offset(ms, side) + pos) * na + k) * q + j];
      if (!isfinite(v)) atomicMin(bad, (int)min(t, (int64_t)INT_MAX - 1));
    }
  }
  b[t] = v;
}

bool mesh_valid(const el_mesh& m) {
  return m.n_x > 0 && m.n_y > 0 && std::isfinite(m.h) && m.h > 0 && std::isfinite(m.x0) && std::isfinite(m.y0);
}

}  // namespace
}  // namespace el

using namespace el;

extern "C" el_status el_trace_rhs_nodal(el_ctx* ctx, el_disc d, el_mesh mesh, const double* g_bnd, double* b) {
  if (!ctx) return EL_ERR_ARG;
  if (!mesh_valid(mesh) || !g_bnd || !b) return set_error(ctx, EL_ERR_ARG, "el_trace_rhs_nodal: bad argument");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  st = ensure_ws(ctx, ctx->ws_small, 8192);
  if (st) return st;
  int* bad = reinterpret_cast<int*>(ctx->ws_small.ptr);
  MeshDev ms{mesh.n_x, mesh.n_y, (mesh.n_x + 1) * mesh.n_y};
  const int64_t nt = mesh_faces(mesh) * de->host.n_a * de->host.q;
  hipLaunchKernelGGL(k_fill_flag, dim3(1), dim3(64), 0, ctx->stream, bad, INT_MAX);
  hipLaunchKernelGGL(k_trace_rhs_nodal, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, ctx->stream, de->view,
                     ms, g_bnd, nt, b, bad);
  hipError_t he = hipGetLastError();
  if (he != hipSuccess) return hip_check(ctx, he, "launch k_trace_rhs_nodal");
  int hbad = INT_MAX;
  he = hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, ctx->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return hip_check(ctx, he, "el_trace_rhs_nodal");
  if (hbad != INT_MAX) {
    std::ostringstream os;
    os << "el_trace_rhs_nodal: non-finite boundary value at trace DOF " << hbad;
    return set_error(ctx, EL_ERR_NONFINITE, os.str());
  }
  return EL_OK;
}

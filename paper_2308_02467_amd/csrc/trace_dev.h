// Device helpers shared by the skeleton kernels: face numbering of a mesh,
// and the per-element body of the skeleton product (I - P) x
// (eq. hdg_global_mat): gather the m inflow traces of the element into LDS,
// reduce each in2out row against them (groups of 8 lanes, 16-byte loads),
// and write each outflow DOF from its unique upwind element.
#pragma once

#include "el_internal.h"

namespace el {

constexpr int kMVThreads = 256;

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

// Storage types of the element operators (in2out, in2sol, in2mean): double
// (EL_F64), float (EL_F32), _Float16 (EL_F16) and bfloat16 bit patterns held
// in uint16_t (EL_BF16).  with_op_type calls f with a value of the type that
// op_dtype names.
template <typename F>
inline void with_op_type(int op_dtype, F&& f) {
  switch (op_dtype) {
    case EL_F64: f(double{}); break;
    case EL_F32: f(float{}); break;
    case EL_F16: f(_Float16{}); break;
    default: f(uint16_t{}); break;
  }
}

__device__ inline double op_to_double(double v) { return v; }
__device__ inline double op_to_double(float v) { return (double)v; }
__device__ inline double op_to_double(_Float16 v) { return (double)(float)v; }
__device__ inline double op_to_double(uint16_t v) { return bf16_to_double(v); }

// rounding to the storage type (round to nearest even; FP64 -> FP32 first)
template <typename T> __device__ inline T op_from_double(double v);
template <> __device__ inline double op_from_double<double>(double v) { return v; }
template <> __device__ inline float op_from_double<float>(double v) { return (float)v; }
template <> __device__ inline _Float16 op_from_double<_Float16>(double v) { return (_Float16)(float)v; }
template <> __device__ inline uint16_t op_from_double<uint16_t>(double v) {
  uint32_t u = __float_as_uint((float)v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
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

template <>
__device__ inline double row_dot<_Float16>(const _Float16* __restrict__ row, const double* tin, int m, int gl) {
  typedef _Float16 h8 __attribute__((ext_vector_type(8)));
  double acc = 0.0;
  for (int c = 8 * gl; c < m; c += 64) {
    if (c + 8 <= m) {
      const h8 v = *reinterpret_cast<const h8*>(row + c);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += (double)(float)v[u] * tin[c + u];
    } else {
      for (int cc = c; cc < m; ++cc) acc += (double)(float)row[cc] * tin[cc];
    }
  }
  return acc;
}

// R rows of one element operator against the gathered inflow traces at
// once: groups of 8 lanes, 16-byte loads.  The loads of a batch of KB chunks
// per lane and row are all issued before any product (R KB = 16 loads in
// flight per lane; m is a multiple of 8, so chunks never straddle the row
// end).  rows[r]: start of row r; a[r]: its partial sum of this lane.  The
// row shape R (2, 4 or 8 rows per group and pass) is chosen per operator
// type and m by the skeleton-product tuner.
template <typename OpT, int R_>
struct RowShape {
  static constexpr int V = 16 / sizeof(OpT);          // entries per 16-byte chunk
  static constexpr int R = R_;                        // rows per group and pass
  static constexpr int KB = 16 / R;                   // chunks per lane and row in a batch
  static_assert(R * KB == 16, "16 loads in flight per lane");
};

template <typename OpT, int R_>
__device__ inline void row_dots(const OpT* const (&rows)[R_], const double* tin, int m, int gl, double (&a)[R_]) {
  constexpr int V = RowShape<OpT, R_>::V, R = R_, KB = RowShape<OpT, R_>::KB;
  typedef OpT vec __attribute__((ext_vector_type(V)));
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = 0.0;
  for (int cb = V * gl; cb < m; cb += KB * 8 * V) {
    vec v[R][KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int c = cb + 8 * V * k;
      if (c < m) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // FP32 / FP64 operators stream with non-temporal loads (11-13 %
          // faster at 128^2); for 16-bit operators plain loads are faster
          const vec* src = reinterpret_cast<const vec*>(rows[r] + c);
          if constexpr (sizeof(OpT) >= 4) v[r][k] = __builtin_nontemporal_load(src);
          else v[r][k] = *src;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int c = cb + 8 * V * k;
      if (c < m) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const double t = tin[c + u];
#pragma unroll
          for (int r = 0; r < R; ++r) a[r] += op_to_double(v[r][k][u]) * t;
        }
      }
    }
  }
}

// LDS of one element's product: inflow traces, the x values at the outflow
// DOFs, and the outflow DOF indices
__host__ __device__ inline size_t matvec_smem_bytes(int m) { return (2 * sizeof(double) + sizeof(int)) * (size_t)m; }

// IMP: y = x - in2out_e x_in at the outflow DOFs of element e and y = x on
// the domain-inflow DOFs it sees, i.e. y = (I - P) x; !IMP: y = in2out_e x_in
// and 0 on the domain-inflow DOFs, i.e. y = P x.  x (FP64, or an FP32 vector
// widened as it is read), y: the mesh's trace vectors; sm:
// matvec_smem_bytes(m) of LDS.  Every index and x value the element needs is
// fetched up front, one per thread, so the row loop waits only on the
// operator stream.
template <typename OpT, bool IMP, int R, typename XT = double>
__device__ inline void matvec_element(const DiscDev& dv, const MeshDev& ms, int e, const OpT* __restrict__ op_e,
                                      const XT* __restrict__ x, double* __restrict__ y, double* sm) {
  const int i = e % ms.n_x, j = e / ms.n_x;
  const int m = dv.m;
  double* tin = sm;                                  // [m]
  double* xo = sm + m;                               // [m]
  int* odof = reinterpret_cast<int*>(sm + 2 * m);    // [m]
  for (int t = threadIdx.x; t < m; t += kMVThreads) {
    const int f = dv.in_f[t];
    const int F = face_of(ms, i, j, f);
    const int dof = (F * dv.n_a + dv.in_k[t]) * dv.q + dv.in_j[t];
    const int Fo = face_of(ms, i, j, dv.out_f[t]);
    const int od = (Fo * dv.n_a + dv.out_k[t]) * dv.q + dv.out_j[t];
    const double v = (double)x[dof];
    if (IMP) xo[t] = (double)x[od];
    odof[t] = od;
    tin[t] = v;
    if (on_domain_boundary(ms, i, j, f)) y[dof] = IMP ? v : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 3, gl = lane & 7;
  constexpr int kRowStep = (kMVThreads / 64) * 8;   // rows per pass of the block
  auto finish = [&](int o, double acc) {
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    if (gl == 0) y[odof[o]] = IMP ? xo[o] - acc : acc;
  };
  // R rows per group at a time (rows past the end repeat the group's first
  // row: loaded, not stored)
  for (int o = wave * 8 + g; o < m; o += R * kRowStep) {
    const OpT* rows[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rows[r] = op_e + (size_t)(o + r * kRowStep < m ? o + r * kRowStep : o) * m;
    double a[R];
    row_dots<OpT, R>(rows, tin, m, gl, a);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (o + r * kRowStep < m) finish(o + r * kRowStep, a[r]);
  }
}

}  // namespace el

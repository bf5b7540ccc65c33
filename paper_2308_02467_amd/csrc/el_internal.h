// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/el.h"

namespace el {

constexpr int kMaxQ = 13;      // p <= 12
constexpr int kMaxNa = 64;

// Host-side discretization data (built once per (p, n_a, scatter, g)).
struct DiscHost {
  int p = 0, q = 0, n_a = 0, nn = 0, n = 0, m = 0;
  int scatter = 0;
  double g = 0.0;
  std::vector<double> xi, omega;      // [q]
  std::vector<double> D;              // [q][q], D[i*q+j] = l_j'(x_i)
  std::vector<double> W;              // [nn]
  std::vector<double> sx, sy;         // [n_a]
  std::vector<double> Q;              // [n_a][n_a] = P[k][k'] * w_k'
  std::vector<double> T;              // [n_a][nn][nn] = B_k - C_k
  std::vector<int32_t> in_row, out_row;   // [m] volume rows
  std::vector<double> in_val;             // [m] entry of -B_hat (w_j |s.n_f|)
  std::vector<double> out_val;            // [m] outflow face weight w_j (s.n_f)
  std::vector<int32_t> in_f, in_k, in_j;  // [m]
  std::vector<int32_t> out_f, out_k, out_j;
};

// Device view of the same data (pointers into one device allocation).
struct DiscDev {
  int p, q, n_a, nn, n, m;
  const double* W;      // [nn]
  const double* Q;      // [n_a*n_a]
  const double* T;      // [n_a*nn*nn]
  const double* in_val; // [m]
  const double* out_val; // [m]
  const int32_t* in_row;
  const int32_t* out_row;
  const int32_t* in_f;
  const int32_t* in_k;
  const int32_t* in_j;
  const int32_t* out_f;
  const int32_t* out_k;
  const int32_t* out_j;
  const double* sx;     // [n_a]
  const double* sy;
};

bool build_disc(const el_disc& d, DiscHost& out, std::string& err);
bool lgl(int p, double* xi, double* w);

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace el

struct el_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  // cached discretizations: key -> (host, device buffer, view)
  struct DiscEntry {
    el::DiscHost host;
    void* dbuf = nullptr;
    el::DiscDev view{};
  };
  std::map<std::string, std::unique_ptr<DiscEntry>> discs;
  el::Workspace ws_local;    // LU factors
  el::Workspace ws_gmres;    // Krylov basis and scratch
  el::Workspace ws_small;    // flags, reductions
  el::Workspace ws_infer;    // el_infer: range mask (when the caller passes none) and fallback index
  int num_cus = 256;
  std::string arch = "unknown";   // the device's architecture name (e.g. gfx950), part of every autotuner key
  // captured GMRES restart cycle (rebuilt when the batch shape changes)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gm_exec = nullptr;
  std::string gm_key;
};

namespace el {
el_status set_error(el_ctx* ctx, el_status code, const std::string& msg);
el_status hip_check(el_ctx* ctx, hipError_t e, const char* what);
el_status get_disc(el_ctx* ctx, const el_disc& d, el_ctx::DiscEntry** out);
el_status ensure_ws(el_ctx* ctx, Workspace& ws, size_t bytes);
// resolves the device address of the allocation-free entry point's static
// scratch on ctx's device (once per device; the device must be current)
el_status noalloc_init(el_ctx* ctx);

// launchers implemented in the .hip files
el_status launch_local_solve(el_ctx* ctx, el_ctx::DiscEntry* de, int precision, int64_t E,
                             const double* h, const double* kappa, const double* sigma,
                             double* in2out, double* in2sol, double* in2mean, double* rel_resid,
                             const double* src, double* s2out, double* s2sol, double* s2mean);
// whether the FP64 factorization of this discretization fits one workgroup
bool local_fp64_fits(el_ctx* ctx, el_ctx::DiscEntry* de);
el_status launch_trace_add_source(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh, const double* s2out,
                                  double* b);
el_status launch_trace_rhs(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh,
                           const double* g_side_host, double* b);
el_status launch_trace_matvec(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh,
                              const void* in2out, int op_dtype, const double* x, double* y);
el_status launch_element_dofs(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh,
                              int32_t* in_dofs, int32_t* out_dofs);
el_status run_trace_solve(el_ctx* ctx, el_ctx::DiscEntry* de, int n_mesh, const el_mesh* meshes,
                          const void* const* in2out, int op_dtype, const double* const* b,
                          double* const* trace, const el_gmres_opts& opts, el_gmres_report* rep);
el_status launch_recover(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh,
                         const void* in2sol, int op_dtype, const double* trace,
                         double* u, double* mean, const double* src2sol);
el_status launch_recover_mean(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh,
                              const void* in2mean, int op_dtype, const double* trace, double* mean,
                              const double* src2mean);
el_status launch_conserve(el_ctx* ctx, el_ctx::DiscEntry* de, int64_t E, const double* h, const double* kappa,
                          const void* in2out, const void* in2vol, int form, int op_dtype, const uint8_t* mask,
                          void* out, int out_dtype);
el_status launch_mean_l2(el_ctx* ctx, el_ctx::DiscEntry* de, int64_t E, const double* h,
                         const double* a, const double* ref, double* out_host);

// ---- autotuner registry ----------------------------------------------------------
// Choices of the autotuners (GEMM block tile, skeleton-product row shape),
// kept per process: key "<arch> <kind> <shape>" (kind "gemm" or "matvec") ->
// the chosen candidate's index, the candidates' timings in ms (empty when the
// choice was loaded from a file) and the candidates' names.  Thread-safe.
bool tune_find(const std::string& key, int* choice);
void tune_store(const std::string& key, int choice, const std::vector<float>& ms);
// candidate names of each tuner, in index order (for reports and for checking
// loaded choices against this library's candidates)
std::vector<std::string> gemm_tile_names();
std::vector<std::string> matvec_shape_names();
// the skeleton product's row shape (index into matvec_shape_names()) for
// in2out of op_dtype on this discretization: pinned, tuned, or timed now on
// the product x -> y over mesh (y overwritten)
el_status matvec_shape(el_ctx* ctx, el_ctx::DiscEntry* de, const el_mesh& mesh, const void* in2out, int op_dtype,
                       const double* x, double* y, int* shape);

inline int64_t mesh_faces(const el_mesh& m) {
  return (int64_t)(m.n_x + 1) * m.n_y + (int64_t)m.n_x * (m.n_y + 1);
}

}  // namespace el

// Host runtime of the C ABI: context, error text, cached discretization
// tables on the device, workspace growth, argument checks and dispatch to
// the kernel launchers.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "el_internal.h"

namespace el {

el_status set_error(el_ctx* ctx, el_status code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

el_status hip_check(el_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return EL_OK;
  std::ostringstream os;
  os << what << ": " << hipGetErrorString(e);
  return set_error(ctx, e == hipErrorOutOfMemory ? EL_ERR_NOMEM : EL_ERR_HIP, os.str());
}

static std::string disc_key(const el_disc& d) {
  char buf[112];
  std::snprintf(buf, sizeof buf, "%d/%d/%d/%.17g/%d", d.p, d.n_a, d.scatter,
                d.scatter == EL_SCATTER_HG ? d.g_hg : 0.0, d.angular);
  return buf;
}

el_status get_disc(el_ctx* ctx, const el_disc& d, el_ctx::DiscEntry** out) {
  std::string key = disc_key(d);
  auto it = ctx->discs.find(key);
  if (it != ctx->discs.end()) { *out = it->second.get(); return EL_OK; }
  auto de = std::make_unique<el_ctx::DiscEntry>();
  std::string err;
  if (!build_disc(d, de->host, err)) return set_error(ctx, EL_ERR_ARG, "el_disc: " + err);
  const DiscHost& h = de->host;
  // one device allocation: doubles first, then int32 tables
  size_t nd = h.W.size() + h.Q.size() + h.T.size() + h.in_val.size() + h.out_val.size() + h.sx.size() + h.sy.size();
  size_t ni = 8 * (size_t)h.m;
  size_t bytes = nd * sizeof(double) + ni * sizeof(int32_t);
  el_status st = hip_check(ctx, hipMalloc(&de->dbuf, bytes), "hipMalloc(disc tables)");
  if (st) return st;
  std::vector<char> staging(bytes);
  double* dp = reinterpret_cast<double*>(staging.data());
  auto putd = [&](const std::vector<double>& v) { std::memcpy(dp, v.data(), v.size() * sizeof(double)); dp += v.size(); };
  double* base = reinterpret_cast<double*>(de->dbuf);
  size_t off = 0;
  auto devd = [&](size_t count) { const double* r = base + off; off += count; return r; };
  de->view.W = devd(h.W.size()); putd(h.W);
  de->view.Q = devd(h.Q.size()); putd(h.Q);
  de->view.T = devd(h.T.size()); putd(h.T);
  de->view.in_val = devd(h.in_val.size()); putd(h.in_val);
  de->view.out_val = devd(h.out_val.size()); putd(h.out_val);
  de->view.sx = devd(h.sx.size()); putd(h.sx);
  de->view.sy = devd(h.sy.size()); putd(h.sy);
  int32_t* ip = reinterpret_cast<int32_t*>(dp);
  int32_t* ibase = reinterpret_cast<int32_t*>(base + off);
  size_t ioff = 0;
  auto puti = [&](const std::vector<int32_t>& v) {
    std::memcpy(ip, v.data(), v.size() * sizeof(int32_t)); ip += v.size();
    const int32_t* r = ibase + ioff; ioff += v.size(); return r;
  };
  de->view.in_row = puti(h.in_row);
  de->view.out_row = puti(h.out_row);
  de->view.in_f = puti(h.in_f);
  de->view.in_k = puti(h.in_k);
  de->view.in_j = puti(h.in_j);
  de->view.out_f = puti(h.out_f);
  de->view.out_k = puti(h.out_k);
  de->view.out_j = puti(h.out_j);
  st = hip_check(ctx, hipMemcpy(de->dbuf, staging.data(), bytes, hipMemcpyHostToDevice), "upload disc tables");
  if (st) return st;
  de->view.p = h.p; de->view.q = h.q; de->view.n_a = h.n_a; de->view.nn = h.nn; de->view.n = h.n; de->view.m = h.m;
  *out = de.get();
  ctx->discs[key] = std::move(de);
  return EL_OK;
}

el_status ensure_ws(el_ctx* ctx, Workspace& ws, size_t bytes) {
  if (ws.bytes >= bytes) return EL_OK;
  if (ws.ptr) {
    el_status st = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync before workspace growth");
    if (st) return st;
    hipFree(ws.ptr);
    ws.ptr = nullptr;
    ws.bytes = 0;
  }
  el_status st = hip_check(ctx, hipMalloc(&ws.ptr, bytes), "hipMalloc(workspace)");
  if (st) return st;
  ws.bytes = bytes;
  return EL_OK;
}

static bool op_dtype_ok(int t) { return t == EL_F64 || t == EL_F32 || t == EL_F16 || t == EL_BF16; }

static bool mesh_ok(const el_mesh& m) {
  return m.n_x > 0 && m.n_y > 0 && std::isfinite(m.h) && m.h > 0 && std::isfinite(m.x0) && std::isfinite(m.y0);
}

}  // namespace el

namespace el {

namespace {
struct TuneEntry {
  int choice;
  std::vector<float> ms;   // per candidate; empty when loaded from a file
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;

// the tuner kind of a key "<arch> <kind> ..." and its candidates' names
std::vector<std::string> names_of(const std::string& key) {
  const size_t a = key.find(' ');
  if (a == std::string::npos) return {};
  const size_t b = key.find(' ', a + 1);
  const std::string kind = key.substr(a + 1, b == std::string::npos ? std::string::npos : b - a - 1);
  if (kind == "gemm") return gemm_tile_names();
  if (kind == "matvec") return matvec_shape_names();
  return {};
}
}  // namespace

bool tune_find(const std::string& key, int* choice) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *choice = it->second.choice;
  return true;
}

void tune_store(const std::string& key, int choice, const std::vector<float>& ms) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = TuneEntry{choice, ms};
}

}  // namespace el

using namespace el;

extern "C" {

el_status el_tuning_report(char* buf, size_t cap, size_t* len) {
  std::ostringstream os;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& kv : g_tune) {
      const std::vector<std::string> names = names_of(kv.first);
      const int c = kv.second.choice;
      os << kv.first << " -> " << (kv.first.find(" gemm ") != std::string::npos ? "tile " : "shape ")
         << (c >= 0 && c < (int)names.size() ? names[c] : std::string("?"));
      if (kv.second.ms.empty()) {
        os << " (from a cache file)\n";
        continue;
      }
      os << " (ms:";
      for (float t : kv.second.ms) os << ' ' << t;
      os << ")\n";
    }
  }
  const std::string s = os.str();
  if (len) *len = s.size() + 1;
  if (buf && cap > 0) {
    const size_t n = std::min(cap - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return EL_OK;
}

// Cache file: a first line naming the format, then one line per choice:
// "<key>\t<candidate index>\t<candidate name>".
static const char kTuneHeader[] = "# el autotuner choices v2";

el_status el_tuning_save(const char* path) {
  if (!path) return EL_ERR_ARG;
  std::ofstream f(path, std::ios::out | std::ios::trunc);
  if (!f) return EL_ERR_ARG;
  f << kTuneHeader << '\n';
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& kv : g_tune) {
      const std::vector<std::string> names = names_of(kv.first);
      const int c = kv.second.choice;
      if (c < 0 || c >= (int)names.size()) continue;
      f << kv.first << '\t' << c << '\t' << names[c] << '\n';
    }
  }
  f.flush();
  return f ? EL_OK : EL_ERR_ARG;
}

el_status el_tuning_load(const char* path, int64_t* loaded) {
  if (loaded) *loaded = 0;
  if (!path) return EL_ERR_ARG;
  std::ifstream f(path);
  if (!f) return EL_ERR_ARG;
  std::string line;
  if (!std::getline(f, line) || line != kTuneHeader) return EL_ERR_ARG;
  // parse everything first: a malformed line leaves the choices unchanged
  std::vector<std::pair<std::string, int>> take;
  while (std::getline(f, line)) {
    if (line.empty()) continue;
    const size_t t1 = line.find('\t');
    const size_t t2 = t1 == std::string::npos ? t1 : line.find('\t', t1 + 1);
    if (t1 == 0 || t2 == std::string::npos || line.find('\t', t2 + 1) != std::string::npos) return EL_ERR_ARG;
    const std::string key = line.substr(0, t1), idx = line.substr(t1 + 1, t2 - t1 - 1), name = line.substr(t2 + 1);
    if (idx.empty() || idx.size() > 3 || idx.find_first_not_of("0123456789") != std::string::npos)
      return EL_ERR_ARG;
    const int v = std::stoi(idx);
    // a kind or candidate this library numbers differently (or does not
    // have) is skipped
    const std::vector<std::string> names = names_of(key);
    if (v >= (int)names.size() || names[v] != name) continue;
    take.emplace_back(key, v);
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : take) g_tune[kv.first] = TuneEntry{kv.second, {}};
  if (loaded) *loaded = (int64_t)take.size();
  return EL_OK;
}

el_status el_tuning_reset(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return EL_OK;
}


el_status el_create(el_ctx** ctx, int device, void* hip_stream) {
  if (!ctx) return EL_ERR_ARG;
  *ctx = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EL_ERR_HIP;
  if (hipSetDevice(device) != hipSuccess) return EL_ERR_HIP;
  el_ctx* c = new el_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->num_cus = prop.multiProcessorCount;
    // "gfx950:sramecc+:xnack-" -> "gfx950"
    std::string a(prop.gcnArchName);
    a = a.substr(0, a.find(':'));
    if (!a.empty()) c->arch = a;
  }
  el_status st = noalloc_init(c);
  if (st) { delete c; return st; }
  *ctx = c;
  return EL_OK;
}

el_status el_destroy(el_ctx* ctx) {
  if (!ctx) return EL_OK;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  if (ctx->gm_exec) hipGraphExecDestroy(ctx->gm_exec);
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  for (auto& kv : ctx->discs) hipFree(kv.second->dbuf);
  hipFree(ctx->ws_local.ptr);
  hipFree(ctx->ws_gmres.ptr);
  hipFree(ctx->ws_small.ptr);
  hipFree(ctx->ws_infer.ptr);
  delete ctx;
  return EL_OK;
}

el_status el_set_stream(el_ctx* ctx, void* hip_stream) {
  if (!ctx) return EL_ERR_ARG;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return EL_OK;
}

const char* el_last_error(const el_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->last_error.c_str();
}

el_status el_workspace_bytes(const el_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return EL_ERR_ARG;
  *bytes = ctx->ws_local.bytes + ctx->ws_gmres.bytes + ctx->ws_small.bytes + ctx->ws_infer.bytes;
  return EL_OK;
}

el_status el_disc_sizes(el_disc d, int64_t* nn, int64_t* n, int64_t* m) {
  DiscHost h;
  std::string err;
  if (d.p < 1 || d.p > 12 || d.n_a < 4 || d.n_a > kMaxNa || d.n_a % 4) return EL_ERR_ARG;
  int64_t q = d.p + 1;
  if (nn) *nn = q * q;
  if (n) *n = q * q * d.n_a;
  if (m) *m = 2 * q * d.n_a;
  return EL_OK;
}

el_status el_lgl(int p, double* xi_host, double* w_host) {
  if (!xi_host || !w_host) return EL_ERR_ARG;
  return lgl(p, xi_host, w_host) ? EL_OK : EL_ERR_ARG;
}

el_status el_index_tables(el_disc d, int32_t* in_rows_host, int32_t* out_rows_host) {
  DiscHost h;
  std::string err;
  if (!build_disc(d, h, err)) return EL_ERR_ARG;
  if (in_rows_host) std::memcpy(in_rows_host, h.in_row.data(), h.m * sizeof(int32_t));
  if (out_rows_host) std::memcpy(out_rows_host, h.out_row.data(), h.m * sizeof(int32_t));
  return EL_OK;
}

el_status el_angular_tables(el_disc d, double* s_host, double* Q_host) {
  DiscHost h;
  std::string err;
  if (!build_disc(d, h, err)) return EL_ERR_ARG;
  if (s_host)
    for (int k = 0; k < h.n_a; ++k) { s_host[2 * k] = h.sx[k]; s_host[2 * k + 1] = h.sy[k]; }
  if (Q_host) std::memcpy(Q_host, h.Q.data(), sizeof(double) * h.n_a * h.n_a);
  return EL_OK;
}

el_status el_trace_size(el_disc d, el_mesh mesh, int64_t* n_trace) {
  if (!n_trace || !mesh_ok(mesh)) return EL_ERR_ARG;
  if (d.p < 1 || d.p > 12 || d.n_a < 4 || d.n_a % 4) return EL_ERR_ARG;
  *n_trace = mesh_faces(mesh) * d.n_a * (d.p + 1);
  return EL_OK;
}

el_status el_element_dofs(el_ctx* ctx, el_disc d, el_mesh mesh, int32_t* in_dofs, int32_t* out_dofs) {
  if (!ctx) return EL_ERR_ARG;
  if (!mesh_ok(mesh)) return set_error(ctx, EL_ERR_ARG, "el_element_dofs: bad mesh");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  return launch_element_dofs(ctx, de, mesh, in_dofs, out_dofs);
}

el_status el_local_solve(el_ctx* ctx, el_disc d, int precision, int64_t E, const double* h,
                         const double* kappa, const double* sigma, double* in2out, double* in2sol,
                         double* in2mean, double* rel_resid, const double* src, double* src2out,
                         double* src2sol, double* src2mean) {
  if (!ctx) return EL_ERR_ARG;
  if (E < 0) return set_error(ctx, EL_ERR_ARG, "el_local_solve: E < 0");
  if (precision != EL_FP64 && precision != EL_FP32_IR)
    return set_error(ctx, EL_ERR_ARG, "el_local_solve: unknown precision");
  if (E == 0) return EL_OK;
  if (!h || !kappa || !sigma) return set_error(ctx, EL_ERR_ARG, "el_local_solve: null input");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  if (!src && (src2out || src2sol || src2mean))
    return set_error(ctx, EL_ERR_ARG, "el_local_solve: source outputs without a source");
  return launch_local_solve(ctx, de, precision, E, h, kappa, sigma, in2out, in2sol, in2mean, rel_resid, src,
                            src2out, src2sol, src2mean);
}

el_status el_trace_rhs(el_ctx* ctx, el_disc d, el_mesh mesh, const double* g_side_host, double* b) {
  if (!ctx) return EL_ERR_ARG;
  if (!mesh_ok(mesh) || !g_side_host || !b) return set_error(ctx, EL_ERR_ARG, "el_trace_rhs: bad argument");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  return launch_trace_rhs(ctx, de, mesh, g_side_host, b);
}

el_status el_trace_add_source(el_ctx* ctx, el_disc d, el_mesh mesh, const double* src2out, double* b) {
  if (!ctx) return EL_ERR_ARG;
  if (!mesh_ok(mesh) || !src2out || !b) return set_error(ctx, EL_ERR_ARG, "el_trace_add_source: bad argument");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  return launch_trace_add_source(ctx, de, mesh, src2out, b);
}

el_status el_trace_matvec(el_ctx* ctx, el_disc d, el_mesh mesh, const void* in2out, int op_dtype,
                          const double* x, double* y) {
  if (!ctx) return EL_ERR_ARG;
  if (!mesh_ok(mesh) || !in2out || !x || !y || !op_dtype_ok(op_dtype))
    return set_error(ctx, EL_ERR_ARG, "el_trace_matvec: bad argument");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  return launch_trace_matvec(ctx, de, mesh, in2out, op_dtype, x, y);
}

el_status el_trace_solve(el_ctx* ctx, el_disc d, int n_mesh, const el_mesh* meshes_host,
                         const void* const* in2out, int op_dtype, const double* const* b,
                         double* const* trace, const el_gmres_opts* opts_host, el_gmres_report* rep_host) {
  if (!ctx) return EL_ERR_ARG;
  if (n_mesh <= 0 || !meshes_host || !in2out || !b || !trace || !opts_host || !rep_host)
    return set_error(ctx, EL_ERR_ARG, "el_trace_solve: bad argument");
  if (!op_dtype_ok(op_dtype))
    return set_error(ctx, EL_ERR_ARG, "el_trace_solve: op_dtype");
  const el_gmres_opts& o = *opts_host;
  if (!(o.tol > 0) || o.restart < 1 || o.restart > 256 || o.max_iter < 1 ||
      (o.basis != EL_F64 && o.basis != EL_F32))
    return set_error(ctx, EL_ERR_ARG, "el_trace_solve: bad GMRES options");
  for (int i = 0; i < n_mesh; ++i) {
    if (!mesh_ok(meshes_host[i]) || !in2out[i] || !b[i] || !trace[i]) {
      std::ostringstream os;
      os << "el_trace_solve: bad mesh or pointer for mesh " << i;
      return set_error(ctx, EL_ERR_ARG, os.str());
    }
  }
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  return run_trace_solve(ctx, de, n_mesh, meshes_host, in2out, op_dtype, b, trace, o, rep_host);
}

el_status el_recover(el_ctx* ctx, el_disc d, el_mesh mesh, const void* in2sol, int op_dtype,
                     const double* trace, double* u, double* mean, const double* src2sol) {
  if (!ctx) return EL_ERR_ARG;
  if (!mesh_ok(mesh) || !in2sol || !trace || !op_dtype_ok(op_dtype))
    return set_error(ctx, EL_ERR_ARG, "el_recover: bad argument");
  if (!u && !mean) return EL_OK;
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  return launch_recover(ctx, de, mesh, in2sol, op_dtype, trace, u, mean, src2sol);
}

el_status el_recover_mean(el_ctx* ctx, el_disc d, el_mesh mesh, const void* in2mean, int op_dtype,
                          const double* trace, double* mean, const double* src2mean) {
  if (!ctx) return EL_ERR_ARG;
  if (!mesh_ok(mesh) || !in2mean || !trace || !mean || !op_dtype_ok(op_dtype))
    return set_error(ctx, EL_ERR_ARG, "el_recover_mean: bad argument");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  return launch_recover_mean(ctx, de, mesh, in2mean, op_dtype, trace, mean, src2mean);
}

el_status el_conserve(el_ctx* ctx, el_disc d, int64_t E, const double* h, const double* kappa, void* in2out,
                      const void* in2vol, int form, int op_dtype, const uint8_t* mask, void* out, int out_dtype) {
  if (!ctx) return EL_ERR_ARG;
  if (!out) { out = in2out; out_dtype = op_dtype; }
  if (!op_dtype_ok(op_dtype) || !op_dtype_ok(out_dtype) || (form != EL_FORM_IN2SOL && form != EL_FORM_IN2MEAN))
    return set_error(ctx, EL_ERR_ARG, "el_conserve: bad dtype or form");
  if (E == 0) return EL_OK;
  if (E < 0 || !h || !kappa || !in2out || !in2vol) return set_error(ctx, EL_ERR_ARG, "el_conserve: bad argument");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  // out is in2out itself (same type) or a separate buffer that does not overlap it
  auto esz = [](int t) -> size_t { return t == EL_F64 ? 8 : t == EL_F32 ? 4 : 2; };
  const size_t per = (size_t)de->host.m * de->host.m;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(in2out), a1 = a0 + (size_t)E * per * esz(op_dtype);
  const uintptr_t b0 = reinterpret_cast<uintptr_t>(out), b1 = b0 + (size_t)E * per * esz(out_dtype);
  if (out == in2out ? out_dtype != op_dtype : (b0 < a1 && a0 < b1))
    return set_error(ctx, EL_ERR_ARG, "el_conserve: out must be in2out itself or not overlap it");
  return launch_conserve(ctx, de, E, h, kappa, in2out, in2vol, form, op_dtype, mask, out, out_dtype);
}

el_status el_mean_l2(el_ctx* ctx, el_disc d, int64_t E, const double* h, const double* a,
                     const double* ref, double* out_host) {
  if (!ctx) return EL_ERR_ARG;
  if (!out_host) return set_error(ctx, EL_ERR_ARG, "el_mean_l2: null out_host");
  if (E == 0) {
    out_host[0] = out_host[1] = 0.0;   // empty sums
    return EL_OK;
  }
  if (E < 0 || !h || !a || !ref) return set_error(ctx, EL_ERR_ARG, "el_mean_l2: bad argument");
  hipSetDevice(ctx->device);
  el_ctx::DiscEntry* de;
  el_status st = get_disc(ctx, d, &de);
  if (st) return st;
  return launch_mean_l2(ctx, de, E, h, a, ref, out_host);
}

}  // extern "C"

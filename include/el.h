/*
 * el.h -- C ABI of the element-learning hot path for the 2D steady radiative
 * transfer equation on one MI355X (gfx950).
 *
 * Method: upwind HDG with Q_p tensor LGL collocation in space and N_a discrete
 * ordinates in angle (paper: "Element learning ...", arXiv 2308.02467,
 * Sec. 2.2).  Per element the local problem (eq. hdg_local_mat) gives
 *     in2sol  = A_i2u = -(B - C + M - S)^{-1} B_hat      (eq. hdg_local_i2u)
 *     in2out  = A_i2o = R^o A_i2u                        (eq. hdg_local_i2o)
 *     in2mean = A_i2m = R_u2m A_i2u                      (Sec. 2.4, eq. ang_ave)
 * and the skeleton system (eq. hdg_global_mat) couples elements through in2out.
 * Algorithm 1 (HDG implementation): local solve -> assemble -> global solve
 * -> recover.  The learned form (Sec. 2.4, eq. param2sol) replaces the local
 * solve by a fully connected network.
 *
 * Conventions (all arrays row-major, all sizes in elements):
 *   q = p+1, nn = q*q, n = nn*N_a (volume DOFs), m = 2*q*N_a (inflow DOFs
 *   per element, equal to outflow DOFs per element).
 *   Node nd = b*q + a for the node (x_a, x_b); volume DOF v = k*nn + nd.
 *   Ordinate k at angle (k + 1/2) 2 pi / N_a, weight 2 pi / N_a.
 *   Faces f: 0 W (-1,0), 1 E (+1,0), 2 S (0,-1), 3 N (0,+1); face node j runs
 *   along increasing x or y.  I_f / O_f: ascending ordinates with s.n_f < 0 / > 0.
 *   Local inflow index iota = f*(N_a/2)*q + r*q + j (r = rank of k in I_f);
 *   outflow indices likewise with O_f.
 *   Mesh: element e = j*n_x + i; vertical face V(i,j) = j*(n_x+1) + i,
 *   horizontal face H(i,j) = (n_x+1)*n_y + j*n_x + i; trace DOF
 *   (F*N_a + k)*q + jn.
 *   Coefficients: kappa = absorption, sigma = scattering, both at the element
 *   LGL nodes; extinction = kappa + sigma (Sec. 2.1).  The square element of
 *   side h is the reference square with coefficients h*(kappa+sigma)/2 and
 *   h*sigma/2 (Sec. 2.4.1).
 *
 * Pointers are DEVICE pointers unless marked "host".  The caller allocates
 * and owns every input and output; the library owns only its workspace (kept
 * in the context, grown on demand) and network state.  No call keeps a
 * caller pointer after it returns.  Every call is ordered on the context's
 * stream; calls that report on the host (status flags, GMRES reports)
 * synchronize that stream before returning.
 *
 * Empty batches: a call with E = 0 elements (B = 0 rows for el_net_forward)
 * checks its enumerated arguments, launches nothing, leaves every output
 * untouched (el_mean_l2: both sums 0; el_infer: *n_fallback_host = 0) and
 * returns EL_OK; its pointers may then be NULL.  el_train_step and
 * el_net_fit_normalization need at least one pair, el_trace_solve at least
 * one mesh (EL_ERR_ARG); a mesh has n_x, n_y >= 1, and a 1 x 1 mesh is
 * valid: all of its faces are domain boundary.
 *
 * Errors: EL_OK = 0; negative values are errors (outputs undefined);
 * EL_WARN_NOT_CONVERGED = +1 means outputs are valid to the reported
 * residual.  el_last_error() returns text naming the failing element or mesh.
 */
#ifndef EL_H
#define EL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int el_status;
#define EL_OK 0
#define EL_WARN_NOT_CONVERGED 1
#define EL_ERR_ARG (-1)
#define EL_ERR_HIP (-2)
#define EL_ERR_SINGULAR (-3)
#define EL_ERR_NONFINITE (-4)
#define EL_ERR_NOMEM (-5)
#define EL_ERR_STATE (-6)

#define EL_SCATTER_ISO 0
#define EL_SCATTER_HG 1

/* angular discretization on the N_a uniform cells of the unit circle */
#define EL_ANG_ORDINATES 0  /* discrete ordinates at the cell centres */
#define EL_ANG_P0 1         /* piecewise-constant (P0) angular elements (Sec. 2.4.1) */

/* local-solve precision forms */
#define EL_FP64 0     /* FP64 LU with partial pivoting */
#define EL_FP32_IR 1  /* FP32 LU, FP64 residual, iterative refinement */

/* operator storage types for the trace sweep and recovery */
#define EL_F64 0
#define EL_BF16 1  /* bfloat16 bit patterns in uint16_t */
#define EL_F32 2
#define EL_F16 3   /* IEEE binary16 */

typedef struct el_ctx el_ctx;

/* Discretization: Q_p in space, n_a angular cells (n_a % 4 == 0, 1 <= p <=
 * 12), scattering kind and Henyey-Greenstein asymmetry g_hg in [0, 1)
 * (Sec. 2.1; exponent 3/2, normalized so that sum_k' w_k' P[k][k'] = 1).
 * angular = EL_ANG_ORDINATES: one direction per cell at its centre;
 * EL_ANG_P0: piecewise-constant angular basis on the cells (Sec. 2.4.1), i.e.
 * the cell averages of the direction, sin(pi/n_a)/(pi/n_a) times the centre
 * direction (no cell straddles an axis, so the face fluxes average the same
 * way), and the phase matrix averaged over pairs of cells. */
typedef struct {
  int p;
  int n_a;
  int scatter;
  double g_hg;
  int angular;
} el_disc;

/* Uniform mesh of n_x * n_y squares of side h, lower-left corner (x0, y0). */
typedef struct {
  int n_x, n_y;
  double x0, y0, h;
} el_mesh;

typedef struct {
  double tol;     /* relative residual ||b - (I-P)x|| / ||b|| */
  int restart;    /* Krylov dimension per cycle, 1..256 */
  int max_iter;   /* total Arnoldi steps */
  int graph;      /* 1: replay each restart cycle as a captured HIP graph;
                     0: launch its kernels one by one (same kernels, same results) */
  int x0;         /* 0: start from t = 0; 1: trace[] holds the starting guess
                     on entry (for instance the learned solution) */
  int basis;      /* storage of the Krylov basis: EL_F64, or EL_F32 (each
                     basis vector rounded once; dot products, the solution
                     and the restart residuals stay FP64; about half the
                     bytes of the Gram-Schmidt sweeps) */
} el_gmres_opts;

typedef struct {
  int iters;
  int restarts;
  double relres;  /* true relative residual at exit */
  int converged;
  int reorth_passes;  /* Arnoldi steps that needed the second Gram-Schmidt pass */
} el_gmres_report;

/* ---- context -------------------------------------------------------------- */
/* Create a context on HIP device `device`, ordered on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
el_status el_create(el_ctx** ctx, int device, void* hip_stream);
el_status el_destroy(el_ctx* ctx);
el_status el_set_stream(el_ctx* ctx, void* hip_stream);
/* Text of the last error on this context (never NULL). */
const char* el_last_error(const el_ctx* ctx);
/* Bytes of device workspace currently held by the context. */
el_status el_workspace_bytes(const el_ctx* ctx, size_t* bytes);

/* ---- discretization queries (host only, no device work) ------------------ */
/* nn, n, m of a discretization; EL_ERR_ARG if it is not supported. */
el_status el_disc_sizes(el_disc d, int64_t* nn, int64_t* n, int64_t* m);
/* LGL nodes and weights on [-1, 1] (Sec. 2.4.1, eq. sigma_se), host [p+1]. */
el_status el_lgl(int p, double* xi_host, double* w_host);
/* Volume row of each local inflow / outflow index (host int32 [m] each):
 * the bit-exact indexing contract above. */
el_status el_index_tables(el_disc d, int32_t* in_rows_host, int32_t* out_rows_host);

/* Angular tables of a discretization (host, no device needed): the
 * direction of each cell s_host [n_a][2] (centre direction or cell average)
 * and Q_host [n_a][n_a] = P[k][k'] w_k' (rows sum to 1).  Either may be NULL. */
el_status el_angular_tables(el_disc d, double* s_host, double* Q_host);
/* Number of trace DOFs of a mesh. */
el_status el_trace_size(el_disc d, el_mesh mesh, int64_t* n_trace);
/* Global trace DOF of every local inflow / outflow index, device int32 [E][m]. */
el_status el_element_dofs(el_ctx* ctx, el_disc d, el_mesh mesh, int32_t* in_dofs, int32_t* out_dofs);

/* ---- local solve (Alg. 1 step 1; eq. hdg_local_f2u_i2u, hdg_local_f2o_i2o) --
 * For E elements with side h[E] and nodal kappa, sigma [E][nn] (>= 0, finite,
 * h > 0): assemble A = B - C + M - S on the fly, factor it (dense LU with
 * partial pivoting, FP64 or FP32 + FP64 refinement), solve for the m inflow
 * columns of -B_hat and write any of
 *   in2out [E][m][m], in2sol [E][n][m], in2mean [E][nn][m]   (NULL = skip),
 * and for EL_FP32_IR the final relative residual per element rel_resid [E]
 * (max over columns of ||R||_inf / ||B_hat col||_inf; NULL = skip).
 * Volume source (Alg. 1 with f != 0): with src [E][n_a][nn] (nodal values
 * of f per ordinate; NULL = none) one more right-hand side (h/2) W f is
 * solved with the same factorization, giving f_u = A^{-1} (h/2) W f:
 *   src2sol [E][n] = f_u, src2out [E][m] = its outflow rows (f_hat_u),
 *   src2mean [E][nn] = its ordinate average            (NULL = skip).
 * Errors: EL_ERR_ARG (bad sizes / disc), EL_ERR_NONFINITE (non-finite or
 * negative coefficient; element named), EL_ERR_SINGULAR (zero pivot; element
 * named).  Synchronizes the stream to read the status flags. */
el_status el_local_solve(el_ctx* ctx, el_disc d, int precision, int64_t E,
                         const double* h, const double* kappa, const double* sigma,
                         double* in2out, double* in2sol, double* in2mean,
                         double* rel_resid, const double* src, double* src2out,
                         double* src2sol, double* src2mean);

/* ---- skeleton system (eq. hdg_global_mat) --------------------------------- */
/* Right-hand side b [n_trace]: per-side boundary radiance g_side (host
 * [4][n_a], sides W, E, S, N, constant along a side) on domain-inflow DOFs
 * (nodal interpolation = the L2 projection P_M g with collocated LGL,
 * Sec. 2.2.2), 0 elsewhere. */
el_status el_trace_rhs(el_ctx* ctx, el_disc d, el_mesh mesh, const double* g_side_host, double* b);

/* The same right-hand side for boundary radiance that varies along the
 * boundary (Sec. 2.2.2, b = P_M g, the nodal interpolation of g at the LGL
 * face nodes): g_bnd (device, FP64, read only) holds g at every boundary
 * face node for every ordinate, [side][face][n_a][p+1] with the sides in
 * the order W, E (n_y faces each, from bottom to top), S, N (n_x faces
 * each, from left to right), 2 (n_x + n_y) n_a (p+1) values in all, face
 * nodes in increasing coordinate.  b [n_trace] (device) gets g on the
 * domain-inflow DOFs (s . n < 0) and 0 elsewhere; values at the other
 * boundary DOFs are not read.  Synchronizes the stream; a non-finite value
 * on an inflow DOF returns EL_ERR_NONFINITE naming the trace DOF (b is then
 * written but not meaningful). */
el_status el_trace_rhs_nodal(el_ctx* ctx, el_disc d, el_mesh mesh, const double* g_bnd, double* b);

/* With a volume source: b[outflow DOFs of e] += src2out[e] (the f_hat_u of
 * el_local_solve, [E][m]; every outflow DOF belongs to one element). */
el_status el_trace_add_source(el_ctx* ctx, el_disc d, el_mesh mesh, const double* src2out, double* b);

/* y = (I - P) x on one mesh: (P x)[out dofs of e] = in2out_e x[in dofs of e],
 * P = 0 on domain-inflow rows.  in2out is [E][m][m] FP64 (op_dtype EL_F64),
 * FP32 (EL_F32), FP16 (EL_F16) or bfloat16 bit patterns (EL_BF16);
 * accumulation is FP64. */
el_status el_trace_matvec(el_ctx* ctx, el_disc d, el_mesh mesh, const void* in2out,
                          int op_dtype, const double* x, double* y);

/* Solve (I - P) t = b for n_mesh independent meshes of any sizes together
 * with restarted GMRES (Sec. 2.3) from t = 0 or from the guess in trace
 * (opts->x0), Arnoldi on P (the Krylov space
 * of I - P is the same; the Hessenberg matrix of I - P follows exactly),
 * classical Gram-Schmidt with DGKS reorthogonalization (second pass when the
 * norm drops below 1/sqrt(2)), Givens rotations, FP64 vectors and reductions.  All meshes share every
 * launch; the Arnoldi scalars stay on the device and the host synchronizes
 * once per restart cycle.  A mesh stops when its true relative residual
 * <= opts->tol (checked at each cycle start) or after max_iter steps.
 * in2out, b, trace: host arrays of n_mesh device pointers (all operators
 * of one op_dtype).  rep: host [n_mesh].  Returns EL_WARN_NOT_CONVERGED if
 * any mesh did not reach tol within max_iter, EL_ERR_NONFINITE (mesh named)
 * for a non-finite right-hand side or residual.  The workspace holds
 * (restart + 4) concatenated trace vectors.  Calls on one context must not
 * overlap (the captured cycle and the workspace are per context). */
el_status el_trace_solve(el_ctx* ctx, el_disc d, int n_mesh, const el_mesh* meshes_host,
                         const void* const* in2out, int op_dtype,
                         const double* const* b, double* const* trace,
                         const el_gmres_opts* opts_host, el_gmres_report* rep_host);

/* ---- recovery (Alg. 1 step 4, eq. hdg_local_mat_sol, eq. ang_ave) ----------
 * u [E][n] = in2sol_e t[in dofs of e] (+ src2sol [E][n], the f_u of a volume
 * source; NULL = none) (u NULL = skip) and the mean intensity
 * mean [E][nn] = (1/N_a) sum_k u (NULL = skip).  in2sol is [E][n][m] in
 * op_dtype (EL_F64, EL_F32, EL_F16, EL_BF16). */
el_status el_recover(el_ctx* ctx, el_disc d, el_mesh mesh, const void* in2sol, int op_dtype,
                     const double* trace, double* u, double* mean, const double* src2sol);
/* Mean intensity directly from in2mean [E][nn][m] in op_dtype (+ src2mean
 * [E][nn], the ordinate average of f_u; NULL = none). */
el_status el_recover_mean(el_ctx* ctx, el_disc d, el_mesh mesh, const void* in2mean,
                          int op_dtype, const double* trace, double* mean, const double* src2mean);

/* Forms of the volume operator that goes with in2out: the full in2sol
 * [n][m], or its ordinate average in2mean [nn][m] (the mean-intensity map,
 * Sec. 2.4.1: the network may learn it instead of in2sol). */
#define EL_FORM_IN2SOL 0
#define EL_FORM_IN2MEAN 1

/* Energy balance of learned operators.  For every element (with mask[e] != 0
 * when mask is given) and every inflow column i, the exact operators satisfy
 *   sum_o w_o in2out[o][i] + sum_(k,nd) W_nd (h kappa_nd / 2) in2sol[(k,nd)][i] = w_i
 * (outflow = inflow - absorption, obtained by testing the local equations
 * with v = 1 and summing over ordinates; w = face quadrature weight times
 * |s.n|); with in2mean the absorption is N_a sum_nd W_nd (h kappa_nd / 2)
 * in2mean[nd][i].  Each column i of in2out is multiplied by the one factor
 * s_i = (w_i - absorption_i) / sum_o w_o in2out[o][i] that makes this hold
 * (the column is left as it is when either is not positive).  Not part of the paper's method: a post-processing option for the
 * learned operators.  in2vol = in2sol or in2mean (form); in2out and in2vol
 * in op_dtype (EL_F64, EL_F32, EL_F16, EL_BF16).  The corrected in2out goes
 * to out in out_dtype: out = NULL or out = in2out corrects in place (out_dtype
 * = op_dtype); a separate out must not overlap in2out and may round FP32
 * operators to EL_F16 or EL_BF16 once, after the correction (correcting
 * values that are already rounded to 16 bits loses the correction whenever
 * it is below half a unit).  Elements with mask[e] == 0 are copied to out
 * unchanged. */
el_status el_conserve(el_ctx* ctx, el_disc d, int64_t E, const double* h, const double* kappa, void* in2out,
                      const void* in2vol, int form, int op_dtype, const uint8_t* mask, void* out, int out_dtype);

/* Squared element L2 norms of mean-intensity fields [E][nn] (relative error
 * measure of Sec. 3.2.1): out_host[0] = sum_e (h_e/2)^2 sum W (a - ref)^2,
 * out_host[1] = sum_e (h_e/2)^2 sum W ref^2.  Synchronizes. */
el_status el_mean_l2(el_ctx* ctx, el_disc d, int64_t E, const double* h,
                     const double* a, const double* ref, double* out_host);


/* ---- element network (Sec. 2.4, eq. param2sol; training Sec. 3.1) ---------
 * A fully connected network x_i = f_i(A_i x_{i-1} + b_i), f = GELU (exact
 * erf form) or ELU on the hidden layers and the identity on the output layer
 * (Sec. 2.4.1), maps the features of one element to its operators
 * (in2out [m][m] followed by in2sol [n][m], row-major; n_out = m*m + n*m;
 * or, in the in2mean form, in2out followed by in2mean [nn][m]; n_out =
 * m*m + nn*m).
 * Input of one element (raw): x = (h, kappa[nn], sigma[nn]).  Features:
 * log10 h, log10 max(h kappa/2, 1e-12), log10 max(h sigma/2, 1e-12)
 * (the reference-element coefficients of Sec. 2.4.1), z-scored with
 * training statistics.  Targets are z-scored per output entry.  Loss: mean
 * absolute error (Sec. 3.1; subgradient 0 at 0).  Optimizer: Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8), FP32 master weights, bfloat16 copies
 * for the matrix-core GEMMs, FP32 accumulation. */
#define EL_ACT_GELU 0
#define EL_ACT_ELU 1
#define EL_ACT_LINEAR 2  /* identity on the hidden layers: the linear network of the ablations of Sec. 3.1 */

typedef struct {
  int n_in;        /* raw inputs per element, 1 + 2*nn */
  int width;       /* hidden width */
  int depth;       /* hidden layers (>= 1) */
  int act;         /* EL_ACT_GELU, EL_ACT_ELU or EL_ACT_LINEAR */
  int64_t n_out;   /* m*m + n*m (in2sol form) or m*m + nn*m (in2mean form) */
  uint64_t seed;   /* initialization: W, b ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) */
} el_net_desc;

typedef struct el_net el_net;

/* Network state blob (el_net_save / el_net_load), little endian:
 *   bytes 0..7    magic "ELNET01\0"
 *   int32  n_in, width, depth, act, k0 (= n_in rounded up to 32), pad
 *   int64  n_out, step (Adam steps taken), n_params
 *   double box[6] = h_min, h_max, kappa_min, kappa_max, sigma_min, sigma_max
 *   (header = 112 bytes), then float32 arrays:
 *   feat_mean[n_in], feat_std[n_in], y_mean[n_out], y_std[n_out],
 *   theta[n_params], adam_m[n_params], adam_v[n_params]
 * theta = for l = 0..depth: W_l [out_l][in_l] row-major then b_l [out_l],
 * with in_0 = k0 (columns >= n_in are zero), in_l = width (l > 0),
 * out_l = width (l < depth), out_depth = n_out; every W_l starts at a
 * multiple of 64 floats (zero gap after the preceding b_l). */
el_status el_net_create(el_ctx* ctx, const el_net_desc* desc_host, el_net** net);
el_status el_net_destroy(el_net* net);
/* host_buf == NULL: *bytes receives the blob size. */
el_status el_net_save(el_ctx* ctx, const el_net* net, void* host_buf, size_t* bytes);
el_status el_net_load(el_ctx* ctx, const void* host_buf, size_t bytes, el_net** net);
/* Feature / target statistics and the training box from N training pairs:
 * x [N][n_in] float32 raw inputs, y [N][n_out] bfloat16 targets. */
el_status el_net_fit_normalization(el_ctx* ctx, el_net* net, int64_t N, const float* x, const uint16_t* y);
/* Copy an FP32 parameter-sized buffer (which: 0 theta, 1 gradient of the
 * last training step in units of the loss, 2 adam_m, 3 adam_v) to dst [n_params]. */
el_status el_net_params(el_ctx* ctx, const el_net* net, int which, float* dst);
el_status el_net_num_params(const el_net* net, int64_t* n_params);

/* Text report of the autotuners' choices so far in this process, one line
 * per key (key, chosen candidate, timing of each candidate in ms): the GEMM
 * block tile per GEMM shape, timed once on the first call of a shape on that
 * call's own operands, and the skeleton product's row shape per operator
 * type and m, timed on the first product (el_trace_matvec) or before the
 * first GMRES cycle (el_trace_solve) with such operators.  Writes at most cap
 * bytes (NUL-terminated) into host buf (may be NULL); *len (may be NULL)
 * receives the size needed including the NUL.  Never fails. */
el_status el_tuning_report(char* buf, size_t cap, size_t* len);

/* The autotuners' choices across processes.  el_tuning_save writes every
 * choice made or loaded so far in this process to the text file at host
 * string path (created or replaced): a header line, then one line per key,
 * "<key>\t<candidate index>\t<candidate name>", where the key begins with
 * the device architecture (e.g. gfx950) and names the tuner (gemm or
 * matvec).  el_tuning_load reads such a file; its choices are used from then
 * on instead of timing the candidates (a key is only ever looked up on a
 * device of its architecture); lines whose index and name do not match a
 * candidate of this library are skipped.  *loaded (may be NULL) receives the
 * number of choices taken.  Both: EL_ERR_ARG for a NULL path or a file that
 * cannot be written / opened; el_tuning_load also for a missing header or a
 * malformed line, and then takes nothing.  el_tuning_reset forgets every
 * choice of this process.  Host only; calls that overlap with tuned launches
 * on other threads are safe (one lock). */
el_status el_tuning_save(const char* path);
el_status el_tuning_load(const char* path, int64_t* loaded);
el_status el_tuning_reset(void);

/* Block tile of the network GEMMs in this process: -1 (default) = chosen
 * per shape by the autotuner; 0 = 128x128, 1 = 64x128, 2 = 128x64,
 * 3 = 256x256 with operand tiles loaded straight into LDS (only GEMMs
 * with k-contiguous operands and K a multiple of 64; the others keep the
 * autotuned tile).  For tests that pin one tile.  EL_ERR_ARG for another
 * value. */
el_status el_gemm_tile(int variant);

/* Row shape of the skeleton product in this process: -1 (default) = chosen
 * per operator type and m by the autotuner; 0 = 4 rows x 4 chunks, 1 = 2 rows
 * x 8 chunks, 2 = 8 rows x 2 chunks per 8-lane group (16 loads of 16 bytes in
 * flight per lane).  For tests that pin one shape.  EL_ERR_ARG for another
 * value. */
el_status el_matvec_shape(int shape);

/* Training pairs from the local solver (FP64 LU; FP32 LU with FP64
 * refinement when the FP64 factorization does not fit one workgroup, as at
 * n = 1568): y [E][n_out] bfloat16 (round to nearest even) = (in2out,
 * in2sol) of each element, or (in2out, in2mean) for form EL_FORM_IN2MEAN. */
el_status el_make_pairs(el_ctx* ctx, el_disc d, int64_t E, const double* h, const double* kappa,
                        const double* sigma, int form, uint16_t* y);

/* One training step on a batch of B pairs: forward, MAE loss, backward,
 * Adam with learning rate lr.  loss: device float, receives the batch loss
 * (mean absolute error in normalized units). */
el_status el_train_step(el_ctx* ctx, el_net* net, int64_t B, const float* x, const uint16_t* y, float lr,
                        float* loss);

/* Normalized network outputs y_norm [B][n_out] (float32) for raw inputs x
 * [B][n_in] (float32); for testing the forward pass. */
el_status el_net_forward(el_ctx* ctx, const el_net* net, int64_t B, const float* x, float* y_norm);

/* FP32 network path (Sec. 3.1 training, measured against the bfloat16
 * operands above): the same network, MAE loss and Adam step as
 * el_train_step / el_net_forward, with every product taking FP32 operands
 * (the FP32 master weights theta directly, FP32 features, hidden
 * activations, sign matrix and backpropagated gradients) and FP32
 * accumulation, and FP32 targets y [B][n_out] (same layout as the bfloat16
 * targets).  It shares the network state (theta, Adam moments, step count,
 * normalization) with the bfloat16 path and refreshes the bfloat16 weight
 * copy in its Adam step, so the two can be mixed.  A measuring path, not a
 * fast one: plain LDS-tiled FP32 products on the vector units.
 * el_net_forward_f32: y [B][n_out] float32 = the normalized outputs
 * (denormalize = 0) or the de-normalized operators (output sd + mean;
 * denormalize = 1).  Scratch: a per-network FP32 workspace grown on demand.
 * Errors: EL_ERR_ARG for null pointers, B < 0 (forward) or B <= 0 (step),
 * a negative or NaN lr, or a product beyond the launch limits. */
el_status el_train_step_f32(el_ctx* ctx, el_net* net, int64_t B, const float* x, const float* y, float lr,
                            float* loss);
el_status el_net_forward_f32(el_ctx* ctx, const el_net* net, int64_t B, const float* x, float* y, int denormalize);

/* Learned operators for E elements (inference): in2out [E][m][m] and
 * in2vol = in2sol [E][n][m] (network in the in2sol form) or in2mean
 * [E][nn][m] (in2mean form; the form follows from the network's n_out),
 * stored as out_dtype (EL_BF16: bfloat16 bits, EL_F16: binary16, both
 * rounded to nearest even from FP32; EL_F32: float32); either may be NULL.  in_range [E]
 * (1 = every input inside the training box; may be NULL).  fallback = 1:
 * elements outside the box are solved by the plain local solver
 * (precision) and written, rounded to out_dtype, into the same outputs;
 * *n_fallback_host receives their count.  Synchronizes. */
el_status el_infer(el_ctx* ctx, const el_net* net, el_disc d, int64_t E, const double* h,
                   const double* kappa, const double* sigma, void* in2out, void* in2vol, int out_dtype,
                   uint8_t* in_range, int fallback, int precision, int64_t* n_fallback_host);

/* ---- measurement aid (not a step of the method) ------------------------------
 * Reads bytes (a multiple of 16; buf 16-byte aligned, device) once with
 * 16-byte loads and XORs every 32-bit word read into *sink (device; the
 * caller sets its initial value), so that the reads cannot be removed: the
 * streaming-read rate of this chip, to set beside the achieved bandwidth of
 * the HBM-bound kernels (the skeleton product streams its operators).
 * Stream-ordered, does not synchronize.  EL_ERR_ARG for a null pointer or a
 * size or address not a multiple of 16; bytes = 0 does nothing. */
el_status el_stream_read(el_ctx* ctx, const void* buf, size_t bytes, uint32_t* sink);

/* ---- allocation-free inference ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  el_infer
 * without the plain-solver fallback that allocates nothing (no hipMalloc or
 * hipFree, no workspace growth, no autotuner timing) and does not
 * synchronize the stream.  Its scratch is one static 64 MiB device array
 * per GPU, resolved by el_create and held until the process ends.  The
 * elements are processed in passes of as many elements as the array holds
 * for this network (2 (k0 + depth width) bytes per element, rounded down to
 * a multiple of 256, at most 16,384 per pass); EL_ERR_ARG when fewer than
 * 256 fit (a network too wide or deep for the array).  The GEMM block tile
 * is fixed (256 x 256 direct-to-LDS where the operands allow it, else
 * 128 x 128), so outputs may differ from el_infer's in the last FP32 bits
 * where el_infer's autotuner chose another tile.  Every call on one GPU
 * shares that GPU's array and overwrites what the last call left there:
 * calls that overlap on one GPU (several streams or contexts) race, so
 * order them on one stream.  in2out, in2vol, out_dtype as in el_infer;
 * in_range [E] (may be NULL) receives the training-box mask, and elements
 * outside the box keep the network's output (no fallback). */
el_status el_infer_noalloc(el_ctx* ctx, const el_net* net, el_disc d, int64_t E, const double* h,
                           const double* kappa, const double* sigma, void* in2out, void* in2vol, int out_dtype,
                           uint8_t* in_range);

#ifdef __cplusplus
}
#endif
#endif /* EL_H */

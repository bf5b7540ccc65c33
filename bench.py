"""Benchmark of the element-learning hot path on one MI355X.

Workload (named in the output's config): 128 x 128 square elements on the
unit square, Q6 LGL (p = 6) x 16 discrete ordinates (n = 784 volume and
m = 224 inflow DOFs per element), isotropic scattering, the smooth Gaussian
cloud kappa = 0.01 + 0.5 G, sigma = 0.1 + 30 G (G a Gaussian bump of width
0.2 at the centre), radiance 1 entering through the left side.  GMRES
tolerance 3e-5, restart 40.  The plain step keeps every GMRES vector in FP64;
the learned step stores its Krylov basis in FP32 (dot products, the solution
and the restart residuals FP64) and is also timed with the FP64 basis.  Every
run measures the learned and the plain mean intensity against the plain FP64
solve converged to 1e-8 and reports them in the config, with a flag that says
whether both are inside the 1e-3 of the metric.

Steps (inputs resident in HBM before every timed region):
* plain:   el_local_solve (FP64 LU) -> el_trace_rhs -> el_trace_solve (FP64
           Krylov basis) -> el_recover
* learned: el_infer (BF16 MFMA network, FP32 outputs, plain fallback outside
           the training box) -> el_conserve (energy-balance correction,
           rounded once into FP16 operator storage) -> el_trace_rhs ->
           el_trace_solve -> el_recover
The network (99-1024x4-225792, GELU) is first trained on pairs from the GPU
local solver (not timed; reported).  value = elements per second of the whole
learned step; the plain step, the FP32 + refinement local solve, the error of
the learned mean intensity against the plain FP64 solve and the CPU oracle
timed on the host cores (process pool, one BLAS thread per worker) are reported
beside it.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 (vector and matrix)
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="elements per side")
    ap.add_argument("--tol", type=float, default=3e-5,
                    help="GMRES relative residual of the timed solves (3e-5 keeps both the learned and the plain "
                         "mean intensity within 1e-3 of the converged plain solution, measured in every run)")
    ap.add_argument("--restart", type=int, default=40)
    ap.add_argument("--gmres-basis", choices=("float64", "float32"), default="float32",
                    help="storage of the learned step's Krylov basis (dot products and restart residuals stay FP64)")
    ap.add_argument("--plain-gmres-basis", choices=("float64", "float32"), default="float64",
                    help="storage of the plain step's Krylov basis")
    ap.add_argument("--accuracy", action="store_true",
                    help="GMRES tolerance sweep and operator-storage errors against a 1e-12 FP64 solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1536, help="elements in the oracle's local-solve sample")
    ap.add_argument("--cpu-mesh", type=int, default=32, help="elements per side of the oracle's whole plain step")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle worker processes (0: min(16, os.cpu_count()))")
    ap.add_argument("--cpu-worker-json", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-samples", type=int, default=200000)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--train-time-limit", type=float, default=180.0, help="seconds")
    ap.add_argument("--lr-decay", type=float, default=0.7,
                    help="fraction of the training after which lr drops 10x (0 = constant)")
    ap.add_argument("--width", type=int, default=1024)
    ap.add_argument("--depth", type=int, default=4)
    ap.add_argument("--act", choices=("gelu", "elu", "linear"), default="gelu", help="hidden-layer activation")
    ap.add_argument("--no-conserve", action="store_true", help="skip the energy-balance correction")
    ap.add_argument("--op-dtype", choices=("float16", "float32"), default="float16",
                    help="storage of the learned operators (in2out and in2sol)")
    ap.add_argument("--storage-study", action="store_true",
                    help="learned-solve error for several operator storages")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for HBM byte counters)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-meshes leg (8 meshes of 16^2 .. 128^2 elements in one solve)")
    ap.add_argument("--cloud", action="store_true",
                    help="run only the realistic-cloud leg (256^2 elements, p=6, N_a=32, HG g=0.85, "
                         "log-normal sigma, learned in2mean form + FP32-refinement fallback)")
    ap.add_argument("--paper-generator", action="store_true",
                    help="run only the element-training study with the paper's coefficient generator "
                         "(P0 cells, N_a=28, g=0.8, albedo 1, 800 training / 200 test fields, batch 50, "
                         "networks of 1-4 layers)")
    ap.add_argument("--pg-time-limit", type=float, default=60.0, help="training seconds per network")
    ap.add_argument("--pg-schedule", choices=("time", "paper"), default="time",
                    help="time: --pg-time-limit seconds per network (lr / 10 after 70 %%); paper: 3000 epochs each "
                         "at lr 1e-3, 1e-4 and 1e-5 (Sec. 3.1)")
    ap.add_argument("--pg-layers", default="1,2,3,4", help="network depths (layers) of the generator study")
    ap.add_argument("--pg-precision", choices=("bf16", "fp32"), default="bf16",
                    help="network operands of the generator study: bf16 (matrix-core path, bfloat16 targets) or "
                         "fp32 (el_train_step_f32 / el_net_forward_f32, FP32 targets from the local solve)")
    ap.add_argument("--pg-train", type=int, default=800, help="training fields of the generator study")
    ap.add_argument("--pg-floor", type=float, default=0.0,
                    help="constant added to every generated field (0: the generator as printed)")
    ap.add_argument("--cloud-n", type=int, default=256)
    ap.add_argument("--cloud-na", type=int, default=32, help="angular cells of the cloud leg")
    ap.add_argument("--cloud-g", type=float, default=0.85, help="HG asymmetry of the cloud leg")
    ap.add_argument("--cloud-angular", choices=("ordinates", "p0"), default="ordinates",
                    help="angular discretization of the cloud leg (p0: the paper's piecewise-constant cells)")
    ap.add_argument("--cloud-train-samples", type=int, default=65536)
    ap.add_argument("--cloud-epochs", type=int, default=60)
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner choices: loaded from this file when it exists, saved to it at the end")
    ap.add_argument("--vendor-gemm-reference", action="store_true",
                    help="time torch.matmul (the vendor BLAS) in bfloat16 at the network's output-layer shapes "
                         "and print one JSON line (context for the network GEMMs; not part of the path)")
    ap.add_argument("--local-solve-only", action="store_true",
                    help="time only el_local_solve (FP64, then FP32 + refinement) on the --n mesh of the cloud "
                         "and print one JSON line (the command the local-solve counter profiles use)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


MATVEC_SOURCES = ("paper_2308_02467_amd/csrc/trace_dev.h", "paper_2308_02467_amd/csrc/k_trace.hip",
                  "paper_2308_02467_amd/csrc/el_internal.h")
TRAFFIC_SUMMARY = {"float16": "profiles/k_matvec_f16_128x128_p6_na16_hbm_traffic.md"}
MATVEC_ELEM = {"float32": ("f32", "float"), "float16": ("f16", "_Float16")}


def matvec_kernel(el, op_dtype, m):
    """Name of the skeleton product kernel that runs for operators stored as
    op_dtype with m trace unknowns per element: the row count in its name is
    the shape the autotuner chose for that pair (its tuning report line)."""
    short, elem = MATVEC_ELEM[op_dtype]
    hit = re.search(r" matvec " + short + r" m=" + str(m) + r" -> shape (\d+) rows", el.tuning_report())
    return f"k_matvec<{elem}, {hit.group(1)}>" if hit else f"k_matvec<{elem}, ?>"


def act_code(el, args):
    return {"gelu": el.EL_ACT_GELU, "elu": el.EL_ACT_ELU, "linear": el.EL_ACT_LINEAR}[args.act]


def gmres_basis(args, plain=False):
    import torch
    name = args.plain_gmres_basis if plain else args.gmres_basis
    return torch.float32 if name == "float32" else torch.float64


def matvec_source_hash():
    h = hashlib.sha256()
    for f in MATVEC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(op_dtype, kernel):
    """HBM bytes per launch of the skeleton product kernel `kernel` with
    operators stored as op_dtype, from the committed rocprofv3 counter
    summary, or None when the summary holds no line for that kernel or the
    kernel's source changed since."""
    try:
        text = open(os.path.join(ROOT, TRAFFIC_SUMMARY[op_dtype])).read()
    except (OSError, KeyError):
        return None
    kern = re.escape(kernel)
    m = re.search(r"traffic_bytes_per_launch " + kern + r" = ([0-9.eE+]+) source_sha256 = ([0-9a-f]+)", text)
    if not m or m.group(2) != matvec_source_hash():
        return None
    return float(m.group(1))


def vendor_gemm_reference():
    """torch.matmul (hipBLASLt) in bfloat16, bfloat16 output, no epilogue, at
    the output layer's shapes (inference of 16,384 elements, training batch
    4,096, the dW shape) and a square 8192^3: the vendor library's rate on
    the same box, as context for the network GEMMs' roofline fractions."""
    import torch
    dev = torch.device("cuda:0")
    out = {"what": "torch.matmul bf16 x bf16 -> bf16, operands resident, 5 timed calls after one warm-up",
           "peak_tflops": 2500.0, "shapes": []}
    for M, N, K in ((16384, 225792, 1024), (4096, 225792, 1024), (225792, 1024, 4096), (8192, 8192, 8192)):
        a = torch.randn(M, K, device=dev, dtype=torch.bfloat16)
        b = torch.randn(N, K, device=dev, dtype=torch.bfloat16)
        c = torch.matmul(a, b.t())
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            c = torch.matmul(a, b.t())
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        tf = 2.0 * M * N * K / (ms * 1e-3) / 1e12
        out["shapes"].append({"M": M, "N": N, "K": K, "ms": ms, "tflops": tf, "frac": tf / 2500.0})
        log(f"vendor GEMM M={M} N={N} K={K}: {ms:.3f} ms = {tf:.0f} TFLOP/s")
        del a, b, c
        torch.cuda.empty_cache()
    return out


def local_solve_main(args, ctx, d, hh, kap, sig, i2o, i2s, i2m):
    """The plain local solve alone (a1-a4 and a5): W untimed and K timed
    launches of el_local_solve per precision on the cloud mesh; median launch
    time by HIP events on the current stream."""
    import torch
    from paper_2308_02467_amd import el
    nn, n, m = el.disc_sizes(d)
    E = hh.shape[0]
    rr = torch.empty(E, dtype=torch.float64, device=hh.device)
    stream = torch.cuda.current_stream()
    flop_el = (2.0 / 3.0) * n ** 3 + 2.0 * n * n * m          # LU + solves for m columns
    out = {"workload": f"el_local_solve, {int(round(E ** 0.5))}^2 elements of the Gaussian cloud, p={d.p}, "
                       f"N_a={d.n_a} (n={n}, m={m})", "elements": E, "steps": args.steps, "warmup": args.warmup}
    for prec, name in ((el.EL_FP64, "fp64"), (el.EL_FP32_IR, "fp32_ir")):
        ts = []
        for it in range(args.warmup + args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.el_local_solve(d, hh, kap, sig, precision=prec, in2out=i2o, in2sol=i2s, in2mean=i2m,
                               rel_resid=rr if prec == el.EL_FP32_IR else None)
            e1.record(stream)
            torch.cuda.synchronize()
            if it >= args.warmup:
                ts.append(e0.elapsed_time(e1))
        t = float(np.median(ts))
        out[name] = {"ms": t, "el_per_s": E / (t * 1e-3), "tflops": flop_el * E / (t * 1e-3) / 1e12}
        if prec == el.EL_FP32_IR:
            out[name]["max_rel_resid"] = float(rr.max())
        log(f"local solve {name}: {t:.1f} ms")
    out["flop_per_element"] = flop_el
    return out


def main():
    args = parse()
    if args.cpu_worker_json:
        cpu_worker(args.cpu_worker_json)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2308_02467_amd import el, inputs

    if args.vendor_gemm_reference:
        print(json.dumps(vendor_gemm_reference()))
        return
    if args.cloud:
        print(json.dumps(cloud_main(args)))
        return
    if args.paper_generator:
        print(json.dumps(paper_generator_main(args)))
        return

    dev = torch.device("cuda:0")
    p, n_a, nx = 6, 16, args.n
    h = 1.0 / nx
    d = el.disc(p, n_a)
    ms = el.mesh(nx, nx, h)
    nn, n, m = el.disc_sizes(d)
    E = nx * nx
    xi, _ = el.lgl(p)
    X, Y = inputs.element_node_coords(nx, nx, h, xi)
    kap_np, sig_np = inputs.gaussian_cloud(X, Y)
    g_side = inputs.left_inflow(n_a)

    ctx = el.Context(0)
    stream = torch.cuda.current_stream()
    if args.tune_cache and os.path.exists(args.tune_cache):
        log(f"autotuner: {el.tuning_load(args.tune_cache)} choices from {args.tune_cache}")
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)      # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    hh, kap, sig = T(np.full(E, h)), T(kap_np), T(sig_np)
    i2o = torch.empty((E, m, m), dtype=torch.float64, device=dev)
    i2s = torch.empty((E, n, m), dtype=torch.float64, device=dev)
    i2m = torch.empty((E, nn, m), dtype=torch.float64, device=dev)
    if args.local_solve_only:
        print(json.dumps(local_solve_main(args, ctx, d, hh, kap, sig, i2o, i2s, i2m)))
        return
    nt = el.trace_size(d, ms)
    b = torch.empty(nt, dtype=torch.float64, device=dev)
    t = torch.empty(nt, dtype=torch.float64, device=dev)
    u = torch.empty((E, n), dtype=torch.float64, device=dev)
    mean = torch.empty((E, nn), dtype=torch.float64, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    # ---- plain FP64 path (FP64 LU, FP64 GMRES vectors) -------------------------
    rec = []

    def plain_step(record):
        e = [ev() for _ in range(5)]
        e[0].record(stream)
        ctx.el_local_solve(d, hh, kap, sig, in2out=i2o, in2sol=i2s, in2mean=i2m)
        e[1].record(stream)
        ctx.el_trace_rhs(d, ms, g_side, b)
        e[2].record(stream)
        st, rep = ctx.el_trace_solve(d, [ms], [i2o], [b], [t], tol=args.tol, restart=args.restart, max_iter=20000,
                                     basis=gmres_basis(args, plain=True))
        e[3].record(stream)
        ctx.el_recover(d, ms, i2s, t, u, mean)
        e[4].record(stream)
        if record:
            rec.append((e, rep[0]))

    log(f"plain: warmup {args.warmup}, timing {args.steps} step(s), E={E}")
    for _ in range(args.warmup):
        plain_step(False)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step(True)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - w0) * 1e3 / args.steps
    ph = np.array([[r[0][i].elapsed_time(r[0][i + 1]) for i in range(4)] for r in rec])
    local_ms = float(np.median(ph[:, 0]))
    flop_el = (2.0 / 3.0) * n ** 3 + 2.0 * n * n * m          # LU + solves for m columns
    lu_tf = flop_el * E / (local_ms * 1e-3) / 1e12
    plain = {
        "ms_per_step": plain_ms, "value": E / (plain_ms * 1e-3), "unit": "element solves/s (whole plain step)",
        "phases_ms": {"local_solve": local_ms, "trace_rhs": float(np.median(ph[:, 1])),
                      "gmres": float(np.median(ph[:, 2])), "recover": float(np.median(ph[:, 3]))},
        "local_solve_el_per_s": E / (local_ms * 1e-3), "gmres": rec[-1][1],
        "gmres_basis": args.plain_gmres_basis,
        "roofline_local_lu": {"bound": "mfma", "kernel": "k_local_lu<double>", "achieved": lu_tf,
                              "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": lu_tf / FP64_PEAK_TFLOPS,
                              "flop_per_element": flop_el},
    }

    # the same local solve with a volume source (one more right-hand side)
    src = torch.ones((E, n), dtype=torch.float64, device=dev)
    s2o = torch.empty((E, m), dtype=torch.float64, device=dev)
    s2s = torch.empty((E, n), dtype=torch.float64, device=dev)
    e0, e1 = ev(), ev()
    e0.record(stream)
    ctx.el_local_solve(d, hh, kap, sig, in2out=i2o, in2sol=i2s, in2mean=i2m, src=src, src2out=s2o, src2sol=s2s)
    e1.record(stream)
    torch.cuda.synchronize()
    plain["local_solve_with_source_ms"] = e0.elapsed_time(e1)
    del src, s2o, s2s

    # ---- FP32 LU + FP64 refinement (local solve only) -------------------------
    log("FP32 + refinement local solve")
    i2o_ir = torch.empty_like(i2o)
    rr = torch.empty(E, dtype=torch.float64, device=dev)
    ir_ms = []
    for _ in range(2):
        e0, e1 = ev(), ev()
        e0.record(stream)
        ctx.el_local_solve(d, hh, kap, sig, precision=el.EL_FP32_IR, in2out=i2o_ir, rel_resid=rr)
        e1.record(stream)
        torch.cuda.synchronize()
        ir_ms.append(e0.elapsed_time(e1))
    num = (i2o_ir - i2o).flatten(1).abs().amax(dim=1)
    den = i2o.flatten(1).abs().amax(dim=1)
    fp32_ir = {"local_solve_ms": ir_ms[-1], "local_solve_el_per_s": E / (ir_ms[-1] * 1e-3),
               "max_rel_residual": float(rr.max()), "in2out_max_rel_diff_vs_fp64": float((num / den).max())}
    del i2o_ir, rr

    acc = None
    if args.accuracy:
        log("accuracy diagnostics")
        acc = accuracy(ctx, d, ms, hh, i2o, i2s, b, mean, args.restart)

    batched = None
    if not args.no_batched:
        del i2s, u
        torch.cuda.empty_cache()
        batched = batched_leg(args, ctx, el, inputs, stream)
        i2s = u = None

    learned = None
    if not args.no_learned:
        i2s = u = None
        torch.cuda.empty_cache()
        learned = learned_leg(args, ctx, el, d, ms, hh, kap, sig, g_side, b, i2o, i2m, mean, stream, E, nn, n, m)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu oracle: {args.cpu_sample} local solves of the {nx}x{nx} mesh and the whole plain step on "
            f"{args.cpu_mesh}x{args.cpu_mesh}")
        cpu = cpu_baseline(args, p, n_a)

    if learned is not None:
        head_ms, head_value, unit = learned["ms_per_step"], learned["value"], "element solves/s (whole learned step)"
        roof = learned.pop("roofline_matvec")
        dtype = "bf16+" + {"float16": "f16", "float32": "f32"}[args.op_dtype] + "+f64"
        workload = (f"learned HDG (element network + GMRES), {nx}x{nx} elements, p=6, N_a=16, Gaussian cloud, "
                    f"left inflow; mean-intensity rel L2 vs plain FP64 {learned['mean_intensity_rel_l2_vs_plain']:.2e}")
    else:
        head_ms, head_value, unit = plain_ms, plain["value"], plain["unit"]
        roof = dict(plain["roofline_local_lu"])
        roof.pop("flop_per_element", None)
        dtype = "f64"
        workload = f"plain FP64 HDG, {nx}x{nx} elements, p=6, N_a=16, Gaussian cloud, left inflow"
    roof.setdefault("traffic", None)
    cfg = {"workload": workload, "elements": E, "p": p, "n_a": n_a, "gmres_tol": args.tol,
           "gmres_restart": args.restart, "plain_gmres_basis": args.plain_gmres_basis,
           "plain_ms_per_step": plain_ms, "plain_el_per_s": plain["value"],
           "plain_local_solve_ms": local_ms, "local_lu_mfma_frac": plain["roofline_local_lu"]["frac"]}
    if learned is not None:
        conv = learned["mean_rel_l2_vs_converged"]
        cfg.update({"learned_gmres_basis": args.gmres_basis,
                    "learned_fp64_basis_ms_per_step": learned["fp64_basis_ms_per_step"],
                    "speedup_learned_vs_plain": plain_ms / learned["ms_per_step"],
                    "mean_rel_l2_vs_converged": conv,
                    "reference": "plain FP64 step (FP64 LU, FP64 GMRES vectors) converged to a relative residual "
                                 "of 1e-8",
                    "within_1e-3": bool(max(conv.values()) <= 1e-3)})
        if max(conv.values()) > 1e-3:
            log(f"WARNING: mean intensity beyond 1e-3 of the converged solve: {conv}")
    out = {
        "metric": "element solves/s + full solve time at 1e-3 rel L2, learned vs plain (p=6)",
        "value": head_value, "unit": unit,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": head_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": cfg,
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain": plain,
        "learned": learned,
        "speedup_learned_vs_plain": (plain_ms / learned["ms_per_step"]) if learned else None,
        "fp32_ir": fp32_ir,
        "batched_meshes": batched,
        "gemm_tiles": el.tuning_report().strip().split("\n") if el.tuning_report().strip() else [],
        "accuracy": acc,
    }
    if args.tune_cache:
        el.tuning_save(args.tune_cache)
    print(json.dumps(out))
    ctx.close()


BATCH_SIDES = (16, 32, 48, 64, 64, 96, 128, 128)


def batched_leg(args, ctx, el, inputs, stream):
    """Eight independent solves of 16^2 .. 128^2 elements (p = 6, N_a = 16,
    sharp cloud edge with a seeded random centre per mesh) in one pass: one
    local solve over all 53,760 elements, one GMRES over all eight skeleton
    systems (captured restart cycle), recovery of the mean intensity."""
    import torch
    dev = torch.device("cuda:0")
    p, n_a = 6, 16
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    xi, _ = el.lgl(p)
    g_side = inputs.left_inflow(n_a)
    hs, ks, ss, meshes = [], [], [], []
    for i, s_ in enumerate(BATCH_SIDES):
        h = 1.0 / s_
        X, Y = inputs.element_node_coords(s_, s_, h, xi)
        kap, sig = inputs.sharp_cloud(X, Y, seed=100 + i)
        hs.append(np.full(s_ * s_, h)); ks.append(kap); ss.append(sig)
        meshes.append(el.mesh(s_, s_, h))
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    H, K, S = T(np.concatenate(hs)), T(np.concatenate(ks)), T(np.concatenate(ss))
    E = H.numel()
    i2o = torch.empty((E, m, m), dtype=torch.float64, device=dev)
    i2m = torch.empty((E, nn, m), dtype=torch.float64, device=dev)
    offs = np.cumsum([0] + [s_ * s_ for s_ in BATCH_SIDES])
    bs = [torch.empty(el.trace_size(d, ms), dtype=torch.float64, device=dev) for ms in meshes]
    ts = [torch.empty_like(b) for b in bs]
    means = [torch.empty((s_ * s_, nn), dtype=torch.float64, device=dev) for s_ in BATCH_SIDES]
    ops = [i2o[offs[i]:offs[i + 1]] for i in range(len(meshes))]
    ev = lambda: torch.cuda.Event(enable_timing=True)
    rec = []

    def step(record, graph=True):
        e = [ev() for _ in range(4)]
        e[0].record(stream)
        ctx.el_local_solve(d, H, K, S, in2out=i2o, in2mean=i2m)
        e[1].record(stream)
        for ms, b in zip(meshes, bs):
            ctx.el_trace_rhs(d, ms, g_side, b)
        st, rep = ctx.el_trace_solve(d, meshes, ops, bs, ts, tol=args.tol, restart=args.restart, max_iter=20000,
                                     graph=graph, basis=gmres_basis(args))
        e[2].record(stream)
        for i, ms in enumerate(meshes):
            ctx.el_recover_mean(d, ms, i2m[offs[i]:offs[i + 1]], ts[i], means[i])
        e[3].record(stream)
        if record:
            rec.append((e, rep))

    log(f"batched meshes {BATCH_SIDES}: {E} elements")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - w0) * 1e3 / args.steps
    ph = np.array([[r[0][i].elapsed_time(r[0][i + 1]) for i in range(3)] for r in rec])
    # the same eight skeleton solves one mesh at a time, for comparison
    t_seq = ev(), ev()
    t_seq[0].record(stream)
    seq_iters = []
    for i, ms in enumerate(meshes):
        st, rp = ctx.el_trace_solve(d, [ms], [ops[i]], [bs[i]], [ts[i]], tol=args.tol, restart=args.restart,
                                    max_iter=20000, basis=gmres_basis(args))
        seq_iters.append(rp[0]["iters"])
    t_seq[1].record(stream)
    torch.cuda.synchronize()
    reps = rec[-1][1]
    out = {
        "workload": f"{len(BATCH_SIDES)} meshes of {'/'.join(f'{s_}^2' for s_ in BATCH_SIDES)} elements, p=6, "
                    "N_a=16, sharp cloud edge (seeded random centres), plain FP64, one GMRES over all meshes",
        "elements": int(E), "ms_per_step": ms_step, "value": E / (ms_step * 1e-3),
        "unit": "element solves/s (whole batched step)",
        "phases_ms": {"local_solve": float(np.median(ph[:, 0])), "rhs_and_gmres": float(np.median(ph[:, 1])),
                      "recover_mean": float(np.median(ph[:, 2]))},
        "gmres_per_mesh": [{"side": s_, "iters": r["iters"], "relres": r["relres"], "converged": r["converged"]}
                           for s_, r in zip(BATCH_SIDES, reps)],
        "gmres_one_mesh_at_a_time_ms": t_seq[0].elapsed_time(t_seq[1]),
        "gmres_one_mesh_at_a_time_iters": seq_iters,
    }
    del i2o, i2m
    torch.cuda.empty_cache()
    return out


def paper_generator_main(args):
    """Element training as in the paper's numerical setting (Sec. 3.1): P0
    angular cells, N_a = 28, HG g = 0.8, albedo 1 (kappa = 0), reference-element
    scattering fields from the paper's generator (Alg. 2, A_sigma = 10,
    c_sm = 2; h = 2 so that the reference-element coefficient is sigma), 800
    training and 200 test fields, hidden width 2 N_in, ELU, MAE, batch 50, lr
    divided by 10 late.  Networks of 1 to 4 layers (1 layer: the linear map).
    Test error: relative L2 of the inferred in2out and in2mean of each test
    field against its local solve (FP32 + refinement to 1e-13)."""
    import torch
    from paper_2308_02467_amd import el, inputs, learned
    dev = torch.device("cuda:0")
    ctx = el.Context(0)
    p, n_a = 6, 28
    d = el.disc(p, n_a, 0.8, el.EL_ANG_P0)
    nn, n, m = el.disc_sizes(d)
    xi, _ = el.lgl(p)
    n_tr, n_te = args.pg_train, 200
    # the test fields are the same whatever the training size
    sig = np.concatenate([inputs.legendre_smooth_draws(n_tr, xi, seed=1234, a_sigma=10.0, c_sm=2.0),
                          inputs.legendre_smooth_draws(n_te, xi, seed=4321, a_sigma=10.0, c_sm=2.0)])
    sig += args.pg_floor
    h = np.full(n_tr + n_te, 2.0)
    kap = np.zeros_like(sig)
    x, y = learned.training_set(ctx, d, n_tr + n_te, form=el.EL_FORM_IN2MEAN, draws=(h, kap, sig), log=False)
    x_tr, y_tr = x[:n_tr].contiguous(), y[:n_tr].contiguous()
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    fp32 = args.pg_precision == "fp32"
    # operators of every field; FP32 + refinement (residual <= 1e-13): the
    # FP64 factorization of n = 1372 does not fit one workgroup
    n_all = n_tr + n_te if fp32 else n_te
    all_o = torch.empty((n_all, m, m), dtype=torch.float64, device=dev)
    all_m = torch.empty((n_all, nn, m), dtype=torch.float64, device=dev)
    ctx.el_local_solve(d, T(h[-n_all:]), T(kap[-n_all:]), T(sig[-n_all:]), precision=el.EL_FP32_IR,
                       in2out=all_o, in2mean=all_m)
    ref_o, ref_m = all_o[-n_te:], all_m[-n_te:]
    H, K, S = T(h[n_tr:]), T(kap[n_tr:]), T(sig[n_tr:])
    y32_tr = None
    if fp32:
        # FP32 targets (in2out, in2mean) of the training fields
        y32_tr = torch.cat([all_o[:n_tr].flatten(1), all_m[:n_tr].flatten(1)], dim=1).float().contiguous()
        del all_o, all_m
    n_in = 1 + 2 * nn
    width = (2 * n_in + 7) // 8 * 8
    n_out = m * m + nn * m
    # the floor set by the bfloat16 storage of the targets: the exact
    # operators of the test fields rounded to bfloat16
    fo = ((ref_o.to(torch.bfloat16).double() - ref_o).flatten(1).norm(dim=1) / ref_o.flatten(1).norm(dim=1))
    fm = ((ref_m.to(torch.bfloat16).double() - ref_m).flatten(1).norm(dim=1) / ref_m.flatten(1).norm(dim=1))
    floor = {"in2out_rel_l2_mean": float(fo.mean()), "in2mean_rel_l2_mean": float(fm.mean())}
    rows = []
    for layers in [int(v) for v in args.pg_layers.split(",")]:
        act = el.EL_ACT_LINEAR if layers == 1 else el.EL_ACT_ELU
        net = el.Net.create(ctx, n_in, width, max(1, layers - 1), n_out, act=act, seed=0)
        net.fit_normalization(x_tr, y_tr)
        yt = y32_tr if fp32 else y_tr
        step = net.train_step_f32 if fp32 else None
        t0 = time.perf_counter()
        if args.pg_schedule == "paper":
            hist = learned.train(net, x_tr, yt, 0, batch=50, schedule=[(3000, 1e-3), (3000, 1e-4), (3000, 1e-5)],
                                 log=True, log_every=500, step=step)
        else:
            hist = learned.train(net, x_tr, yt, 100000, batch=50, lr=1e-3, time_limit=args.pg_time_limit,
                                 decay_at=0.7, log=False, step=step)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        if fp32:
            yo = torch.empty((n_te, n_out), dtype=torch.float32, device=dev)
            net.forward_f32(x[n_tr:].contiguous(), yo, denormalize=True)
            po, pm = yo[:, :m * m].reshape(n_te, m, m), yo[:, m * m:].reshape(n_te, nn, m)
        else:
            po = torch.empty((n_te, m, m), dtype=torch.float32, device=dev)
            pm = torch.empty((n_te, nn, m), dtype=torch.float32, device=dev)
            net.infer(d, H, K, S, in2out=po, in2mean=pm, fallback=False)
        torch.cuda.synchronize()
        eo = ((po.double() - ref_o).flatten(1).norm(dim=1) / ref_o.flatten(1).norm(dim=1)).cpu().numpy()
        em = ((pm.double() - ref_m).flatten(1).norm(dim=1) / ref_m.flatten(1).norm(dim=1)).cpu().numpy()
        rows.append({"layers": layers, "network": f"{n_in}-{width}x{max(1, layers - 1)}-{n_out} "
                     + ("linear" if layers == 1 else "ELU"), "epochs": len(hist),
                     "final_train_loss": hist[-1] if hist else None, "training_s": t_train,
                     "train_loss_at_epochs": {str(e): hist[e - 1] for e in (1, 10, 100, 1000, 3000, 6000, 9000)
                                              if e <= len(hist)},
                     "test_in2out_rel_l2_mean": float(eo.mean()), "test_in2out_rel_l2_median": float(np.median(eo)),
                     "test_in2mean_rel_l2_mean": float(em.mean())})
        log(f"paper generator: {layers} layers, test in2out error {eo.mean():.3e}")
        net.close()
    ctx.close()
    return {"study": "element training with the paper's coefficient generator", "p": p, "n_a": n_a,
            "angular": "p0", "g": 0.8, "albedo": 1.0, "train": n_tr, "test": n_te, "batch": 50,
            "a_sigma": 10.0, "c_sm": 2.0, "floor": args.pg_floor, "schedule": args.pg_schedule,
            "precision": args.pg_precision,
            "bf16_target_rounding_floor": floor, "networks": rows}


def cloud_main(args):
    """Realistic synthetic cloud: 256^2 elements, p = 6, N_a = 32, Henyey-
    Greenstein g = 0.85, sigma a seeded log-normal field with a k^(-5/3)
    spectrum (mean 10, log-std 1) set to zero where the field is negative,
    kappa = 0.05 sigma + 0.01, radiance 1 entering through the left side.
    The network (in2mean form) is trained on elements drawn from
    independently seeded fields of the same statistics; elements outside its
    training box go to the FP32 + refinement local solver.  Reference: the
    FP32 + refinement local solve of every element (operators stored as
    float32) and GMRES to 1e-8."""
    import torch
    from paper_2308_02467_amd import el, inputs, learned
    dev = torch.device("cuda:0")
    ctx = el.Context(0)
    stream = torch.cuda.current_stream()
    p, n_a, g, nx = 6, args.cloud_na, args.cloud_g, args.cloud_n
    ang = el.EL_ANG_P0 if args.cloud_angular == "p0" else el.EL_ANG_ORDINATES
    h = 1.0 / nx
    d = el.disc(p, n_a, g, ang)
    ms = el.mesh(nx, nx, h)
    nn, n, m = el.disc_sizes(d)
    E = nx * nx
    xi, _ = el.lgl(p)
    X, Y = inputs.element_node_coords(nx, nx, h, xi)
    kap_np, sig_np = inputs.lognormal_cloud(X, Y, seed=2024)
    g_side = inputs.left_inflow(n_a)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    hh, kap, sig = T(np.full(E, h)), T(kap_np), T(sig_np)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    n_out = m * m + nn * m

    # training elements: random elements of independently seeded fields
    rng = np.random.default_rng(7)
    n_fields = max(4, -(-args.cloud_train_samples // E))   # enough fields to draw without repeats
    per = max(1, args.cloud_train_samples // n_fields)
    hs, ks, ss = [], [], []
    for f in range(n_fields):
        kf, sf = inputs.lognormal_cloud(X, Y, seed=3000 + f)
        sel = rng.choice(E, size=per, replace=False)
        hs.append(np.full(per, h)); ks.append(kf[sel]); ss.append(sf[sel])
    draws = (np.concatenate(hs), np.concatenate(ks), np.concatenate(ss))
    N = draws[0].size
    log(f"cloud: {N} training pairs (in2mean form, n = {n})")
    t0 = time.perf_counter()
    x, y = learned.training_set(ctx, d, N, form=el.EL_FORM_IN2MEAN, draws=draws)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    net = el.Net.create(ctx, 1 + 2 * nn, args.width, args.depth, n_out, act=act_code(el, args), seed=0)
    net.fit_normalization(x, y)
    t0 = time.perf_counter()
    hist = learned.train(net, x, y, args.cloud_epochs, batch=4096, lr=1e-3, time_limit=args.train_time_limit,
                         decay_at=args.lr_decay)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del x, y
    torch.cuda.empty_cache()

    nt = el.trace_size(d, ms)
    b = torch.empty(nt, dtype=torch.float64, device=dev)
    ctx.el_trace_rhs(d, ms, g_side, b)

    # reference: FP32 + refinement for every element, GMRES to 1e-8
    log("cloud: reference local solve (FP32 + refinement, all elements)")
    ro = torch.empty((E, m, m), dtype=torch.float32, device=dev)
    rmn = torch.empty((E, nn, m), dtype=torch.float64, device=dev)
    e0, e1 = ev(), ev()
    e0.record(stream)
    chunk = 16384
    for c0 in range(0, E, chunk):
        c1 = min(E, c0 + chunk)
        tmp_o = torch.empty((c1 - c0, m, m), dtype=torch.float64, device=dev)
        ctx.el_local_solve(d, hh[c0:c1], kap[c0:c1], sig[c0:c1], precision=el.EL_FP32_IR, in2out=tmp_o,
                           in2mean=rmn[c0:c1])
        ro[c0:c1] = tmp_o.to(torch.float32)
        del tmp_o
    e1.record(stream)
    torch.cuda.synchronize()
    ref_local_ms = e0.elapsed_time(e1)
    t_ref = torch.empty_like(b)
    log("cloud: reference GMRES")
    e0, e1 = ev(), ev()
    e0.record(stream)
    st, rep_ref = ctx.el_trace_solve(d, [ms], [ro], [b], [t_ref], tol=1e-8, restart=args.restart, max_iter=40000)
    e1.record(stream)
    torch.cuda.synchronize()
    ref_gmres_ms = e0.elapsed_time(e1)
    mean_ref = torch.empty((E, nn), dtype=torch.float64, device=dev)
    ctx.el_recover_mean(d, ms, rmn, t_ref, mean_ref)
    # the plain method's skeleton solve at the learned step's tolerance
    t_pl = torch.empty_like(b)
    e0, e1 = ev(), ev()
    e0.record(stream)
    st, rep_pl = ctx.el_trace_solve(d, [ms], [ro], [b], [t_pl], tol=args.tol, restart=args.restart, max_iter=40000,
                                    basis=gmres_basis(args))
    e1.record(stream)
    torch.cuda.synchronize()
    plain_gmres_ms = e0.elapsed_time(e1)
    mean_pl = torch.empty((E, nn), dtype=torch.float64, device=dev)
    ctx.el_recover_mean(d, ms, rmn, t_pl, mean_pl)
    d2p, r2p = ctx.el_mean_l2(d, hh, mean_pl, mean_ref)
    del rmn, t_pl, mean_pl

    lo32 = torch.empty((E, m, m), dtype=torch.float32, device=dev)
    lm = torch.empty((E, nn, m), dtype=torch.float32, device=dev)
    op_t = getattr(torch, args.op_dtype)
    lo = lo32 if op_t == torch.float32 else torch.empty((E, m, m), dtype=op_t, device=dev)
    mask = torch.empty(E, dtype=torch.uint8, device=dev)
    t = torch.empty_like(b)
    mean = torch.empty_like(mean_ref)
    rec = []

    def step(record):
        e = [ev() for _ in range(4)]
        e[0].record(stream)
        nfb = net.infer(d, hh, kap, sig, lo32, in2mean=lm, in_range=mask, fallback=True, precision=el.EL_FP32_IR)
        ctx.el_conserve(d, hh, kap, lo32, in2mean=lm, mask=mask, out=None if lo is lo32 else lo)
        e[1].record(stream)
        ctx.el_trace_rhs(d, ms, g_side, b)
        st, rep = ctx.el_trace_solve(d, [ms], [lo], [b], [t], tol=args.tol, restart=args.restart, max_iter=40000,
                                     basis=gmres_basis(args))
        e[2].record(stream)
        ctx.el_recover_mean(d, ms, lm, t, mean)
        e[3].record(stream)
        if record:
            rec.append((e, rep[0], nfb))

    log("cloud: learned solve")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - w0) * 1e3 / args.steps
    ph = np.array([[r[0][i].elapsed_time(r[0][i + 1]) for i in range(3)] for r in rec])
    d2, r2 = ctx.el_mean_l2(d, hh, mean, mean_ref)
    out = {
        "metric": "element solves/s + full solve time at 1e-3 rel L2, learned vs plain (p=6)",
        "value": E / (ms_step * 1e-3), "unit": "element solves/s (whole learned step)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+" + {"float16": "f16", "float32": "f32"}[args.op_dtype] + "+f64", "data": "synthetic",
        "config": {"workload": f"realistic cloud: {nx}x{nx} elements, p=6, N_a={n_a} "
                               f"({'P0 angular cells' if args.cloud_angular == 'p0' else 'ordinates'}), "
                               f"HG g={g}, log-normal sigma "
                               "(k^-5/3, mean 10, log-std 1, zero below threshold), kappa=0.05 sigma+0.01, "
                               "learned in2mean form + FP32-refinement fallback, FP64 GMRES",
                   "elements": E, "p": p, "n_a": n_a, "g": g, "angular": args.cloud_angular, "gmres_tol": args.tol,
                   "gmres_restart": args.restart, "gmres_basis": args.gmres_basis},
        "network": f"{1 + 2 * nn}-{args.width}x{args.depth}-{n_out} {args.act.upper()} (in2out + in2mean)",
        "train_samples": N, "epochs_run": len(hist), "final_train_loss": hist[-1] if hist else None,
        "pair_generation_s": t_gen, "training_s": t_train,
        "phases_ms": {"infer_fallback_and_correction": float(np.median(ph[:, 0])),
                      "rhs_and_gmres": float(np.median(ph[:, 1])), "recover_mean": float(np.median(ph[:, 2]))},
        "fallback_elements": rec[-1][2], "gmres": rec[-1][1],
        "mean_intensity_rel_l2_vs_reference": (d2 / r2) ** 0.5, "learned_in2out_storage": args.op_dtype,
        "reference": {"local_solve_ms": ref_local_ms, "local_solve_el_per_s": E / (ref_local_ms * 1e-3),
                      "gmres_ms": ref_gmres_ms, "gmres": rep_ref[0], "operator_storage": "float32"},
        "plain_step_ms": ref_local_ms + plain_gmres_ms,
        "plain": {"local_solve_ms": ref_local_ms, "gmres_ms": plain_gmres_ms, "gmres": rep_pl[0],
                  "mean_intensity_rel_l2_vs_reference": (d2p / r2p) ** 0.5,
                  "note": f"FP32 + refinement local solve (the FP64 factorization of n = {n} does not fit one "
                          "workgroup), float32 operators, GMRES at the learned step's tolerance"},
        "speedup_learned_vs_plain": (ref_local_ms + plain_gmres_ms) / ms_step,
    }
    net.close()
    ctx.close()
    return out


def learned_leg(args, ctx, el, d, ms, hh, kap, sig, g_side, b, i2o_plain, i2m_plain, mean_plain, stream, E, nn, n,
                m):
    """Train the element network on pairs from the GPU local solver, then time
    the learned solve on the same workload and compare its mean intensity
    with the plain FP64 solve."""
    import torch
    from paper_2308_02467_amd import learned
    dev = hh.device
    ev = lambda: torch.cuda.Event(enable_timing=True)
    net = el.Net.create(ctx, 1 + 2 * nn, args.width, args.depth, m * m + n * m, act=act_code(el, args), seed=0)
    log(f"learned: {args.train_samples} training pairs")
    t0 = time.perf_counter()
    x, y = learned.training_set(ctx, d, args.train_samples)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    net.fit_normalization(x, y)
    t0 = time.perf_counter()
    hist = learned.train(net, x, y, args.epochs, batch=4096, lr=1e-3, time_limit=args.train_time_limit,
                         decay_at=args.lr_decay)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del x, y
    torch.cuda.empty_cache()
    # the network writes FP32 operators; the energy-balance correction reads
    # them and writes the in2out that GMRES sweeps, rounded once to op_dtype
    op_t = getattr(torch, args.op_dtype)
    esz = torch.empty(0, dtype=op_t).element_size()
    lo32 = torch.empty((E, m, m), dtype=torch.float32, device=dev)
    ls = torch.empty((E, n, m), dtype=torch.float32, device=dev)
    lo = lo32 if op_t == torch.float32 else torch.empty((E, m, m), dtype=op_t, device=dev)
    mask = torch.empty(E, dtype=torch.uint8, device=dev)
    t = torch.empty_like(b)
    mean = torch.empty_like(mean_plain)
    rec = []

    def step(record, conserve=not args.no_conserve, basis=None, into=None):
        e = [ev() for _ in range(4)]
        e[0].record(stream)
        nfb = net.infer(d, hh, kap, sig, lo32, ls, mask, fallback=True)
        if conserve:
            ctx.el_conserve(d, hh, kap, lo32, ls, mask, out=None if lo is lo32 else lo)
        op = lo if conserve else lo32
        e[1].record(stream)
        ctx.el_trace_rhs(d, ms, g_side, b)
        st, rep = ctx.el_trace_solve(d, [ms], [op], [b], [t], tol=args.tol, restart=args.restart, max_iter=20000,
                                     basis=gmres_basis(args) if basis is None else basis)
        e[2].record(stream)
        ctx.el_recover(d, ms, ls, t, None, mean)
        e[3].record(stream)
        if record:
            (rec if into is None else into).append((e, rep[0], nfb))

    log("learned solve")
    step(False, conserve=False)
    d2, r2 = ctx.el_mean_l2(d, hh, mean, mean_plain)
    err_raw = (d2 / r2) ** 0.5
    op_raw = ((lo32.double() - i2o_plain).flatten(1).norm(dim=1) / i2o_plain.flatten(1).norm(dim=1)).cpu().numpy()
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - w0) * 1e3 / args.steps
    ph = np.array([[r[0][i].elapsed_time(r[0][i + 1]) for i in range(3)] for r in rec])
    d2, r2 = ctx.el_mean_l2(d, hh, mean, mean_plain)
    op_err = ((lo.double() - i2o_plain).flatten(1).norm(dim=1) / i2o_plain.flatten(1).norm(dim=1)).cpu().numpy()
    mean_head = mean.clone()

    # the same learned step with every GMRES vector in FP64
    rec64 = []
    log("learned solve, FP64 Krylov basis")
    step(False, basis=torch.float64)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        step(True, basis=torch.float64, into=rec64)
    torch.cuda.synchronize()
    ms_step64 = (time.perf_counter() - w0) * 1e3 / args.steps
    gm64 = float(np.median([r[0][1].elapsed_time(r[0][2]) for r in rec64]))
    mean_64 = mean.clone()

    # dominant kernel of the learned step: the in2out sweep (k_matvec<op type>), HBM-bound
    xv = torch.rand_like(b)
    yv = torch.empty_like(b)
    reps = 20
    e0, e1 = ev(), ev()
    ctx.el_trace_matvec(d, ms, lo, xv, yv)
    e0.record(stream)
    for _ in range(reps):
        ctx.el_trace_matvec(d, ms, lo, xv, yv)
    e1.record(stream)
    torch.cuda.synchronize()
    mv_ms = e0.elapsed_time(e1) / reps
    mv_bytes = E * m * (m * esz + 3 * 8)        # operator + gathered inflow + outflow read/write
    mv_gbs = mv_bytes / (mv_ms * 1e-3) / 1e9
    mv_kernel = matvec_kernel(el, args.op_dtype, m)
    # the chip's streaming-read rate over the same operator bytes (a read of
    # the in2out buffer and nothing else), beside the product's achieved rate
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    ctx.el_stream_read(lo, sink)
    e0.record(stream)
    for _ in range(reps):
        ctx.el_stream_read(lo, sink)
    e1.record(stream)
    torch.cuda.synchronize()
    sr_ms = e0.elapsed_time(e1) / reps
    sr_gbs = lo.numel() * lo.element_size() / (sr_ms * 1e-3) / 1e9

    study = storage_study(args, ctx, net, d, ms, hh, kap, sig, g_side, b, mean_plain, E, n, m) \
        if args.storage_study else None

    # the learned solution as the starting guess of the plain FP64 skeleton
    # solve (an accurate solve at a fraction of the plain iterations); the
    # cold solve is the converged reference of the error measures
    warm = {"tol": 1e-8}
    conv = {}
    for name, guess in (("cold", None), ("from_learned", t)):
        tw = torch.zeros_like(b) if guess is None else guess.clone()
        e0, e1 = ev(), ev()
        e0.record(stream)
        st, rw = ctx.el_trace_solve(d, [ms], [i2o_plain], [b], [tw], tol=1e-8, restart=args.restart,
                                    max_iter=40000, x0=guess is not None, basis=torch.float64)
        e1.record(stream)
        torch.cuda.synchronize()
        warm[name] = {"iters": rw[0]["iters"], "gmres_ms": e0.elapsed_time(e1), "converged": rw[0]["converged"]}
        if guess is None:
            # errors against the plain FP64 solution converged to 1e-8
            mean_conv = torch.empty_like(mean_plain)
            ctx.el_recover_mean(d, ms, i2m_plain, tw, mean_conv)
            for key, mv in (("learned", mean_head), ("learned_fp64_basis", mean_64), ("plain", mean_plain)):
                dl, rl = ctx.el_mean_l2(d, hh, mv, mean_conv)
                conv[key] = (dl / rl) ** 0.5
            del mean_conv
    del tw, mean_head, mean_64

    n_in = 1 + 2 * nn
    flop_el = 2.0 * (n_in * args.width + (args.depth - 1) * args.width ** 2 + args.width * (m * m + n * m))
    inf_ms = float(np.median(ph[:, 0]))
    out = {
        "network": f"{n_in}-{args.width}x{args.depth}-{m * m + n * m} {args.act.upper()}, BF16 MFMA, FP32 accumulate",
        "train_samples": args.train_samples, "epochs_run": len(hist),
        "final_train_loss": hist[-1] if hist else None,
        "pair_generation_s": t_gen, "training_s": t_train,
        "ms_per_step": ms_step, "value": E / (ms_step * 1e-3), "unit": "element solves/s (whole learned step)",
        "phases_ms": {"infer_and_correction": inf_ms, "gmres": float(np.median(ph[:, 1])),
                      "recover": float(np.median(ph[:, 2]))},
        "infer_el_per_s": E / (inf_ms * 1e-3),
        "infer_network_tflops": flop_el * E / (inf_ms * 1e-3) / 1e12,
        "fallback_elements": rec[-1][2], "gmres": rec[-1][1],
        "mean_intensity_rel_l2_vs_plain": (d2 / r2) ** 0.5,
        "energy_balance_correction": not args.no_conserve,
        "in2out_rel_err_median": float(np.median(op_err)), "in2out_rel_err_max": float(op_err.max()),
        "without_correction": {"mean_intensity_rel_l2_vs_plain": err_raw,
                               "in2out_rel_err_median": float(np.median(op_raw))},
        "operator_storage": args.op_dtype,
        "storage_study": study,
        "plain_gmres_warm_start": warm,
        "gmres_basis": args.gmres_basis,
        "fp64_basis_ms_per_step": ms_step64, "fp64_basis_gmres_ms": gm64,
        "fp64_basis_gmres": rec64[-1][1],
        "mean_rel_l2_vs_converged": conv,
        "roofline_matvec": {"bound": "hbm",
                            "kernel": f"{mv_kernel} (element body shared with the GMRES product)",
                            "achieved": mv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": mv_gbs / HBM_PEAK_GBS,
                            "traffic": recorded_traffic(args.op_dtype, mv_kernel),
                            "bytes_per_launch": mv_bytes, "avg_launch_ms": mv_ms,
                            "stream_read_GBps": sr_gbs, "frac_of_stream_read": mv_gbs / sr_gbs},
    }
    net.close()
    return out


def storage_study(args, ctx, net, d, ms, hh, kap, sig, g_side, b, mean_plain, E, n, m):
    """Mean-intensity error of the learned solve for three storages of the
    learned in2out: float32; float16 rounded once after the float32
    energy-balance correction (the timed path); float16 written by the
    network and corrected afterwards (corrections below half a float16 unit
    are lost)."""
    import torch
    dev = hh.device
    res = {}
    lo32 = torch.empty((E, m, m), dtype=torch.float32, device=dev)
    ls32 = torch.empty((E, n, m), dtype=torch.float32, device=dev)
    lo16 = torch.empty((E, m, m), dtype=torch.float16, device=dev)
    mask = torch.empty(E, dtype=torch.uint8, device=dev)
    t = torch.empty_like(b)
    mean = torch.empty_like(mean_plain)

    def err(op_o, op_s):
        ctx.el_trace_solve(d, [ms], [op_o], [b], [t], tol=args.tol, restart=args.restart, max_iter=20000,
                           basis=gmres_basis(args))
        ctx.el_recover(d, ms, op_s, t, None, mean)
        d2, r2 = ctx.el_mean_l2(d, hh, mean, mean_plain)
        return (d2 / r2) ** 0.5

    net.infer(d, hh, kap, sig, lo32, ls32, mask, fallback=True)
    ctx.el_conserve(d, hh, kap, lo32, ls32, mask, out=lo16)
    res["float16_in2out_rounded_after_float32_correction"] = err(lo16, ls32)
    ctx.el_conserve(d, hh, kap, lo32, ls32, mask)
    res["float32_in2out"] = err(lo32, ls32)
    del lo32, ls32
    ls16 = torch.empty((E, n, m), dtype=torch.float16, device=dev)
    net.infer(d, hh, kap, sig, lo16, ls16, mask, fallback=True)
    ctx.el_conserve(d, hh, kap, lo16, ls16, mask)
    res["float16_network_output_corrected_in_float16"] = err(lo16, ls16)
    return res


def accuracy(ctx, d, ms, hh, i2o, i2s, b, mean_timed, restart):
    """Relative L2 errors of the mean intensity against the FP64 solve at 1e-12."""
    import torch
    t_ref = torch.empty_like(b)
    st, rep = ctx.el_trace_solve(d, [ms], [i2o], [b], [t_ref], tol=1e-12, restart=restart, max_iter=40000)
    mean_ref = torch.empty_like(mean_timed)
    ctx.el_recover(d, ms, i2s, t_ref, None, mean_ref)
    d2, r2 = ctx.el_mean_l2(d, hh, mean_timed, mean_ref)
    out = {"reference_gmres": rep[0], "timed_solution_rel_l2": (d2 / r2) ** 0.5}

    def solve_with(op_o, op_s, tol=1e-12):
        tt = torch.empty_like(b)
        st, rp = ctx.el_trace_solve(d, [ms], [op_o], [b], [tt], tol=tol, restart=restart, max_iter=40000)
        mm_ = torch.empty_like(mean_timed)
        ctx.el_recover(d, ms, op_s, tt, None, mm_)
        d2, r2 = ctx.el_mean_l2(d, hh, mm_, mean_ref)
        return (d2 / r2) ** 0.5, rp[0]["iters"]

    out["gmres_tol_sweep"] = {f"{tol:g}": dict(zip(("rel_l2", "iters"), solve_with(i2o, i2s, tol)))
                              for tol in (1e-4, 1e-5, 1e-6)}
    o16 = i2o.to(torch.bfloat16)
    out["bf16_in2out_f64_in2sol_rel_l2"] = solve_with(o16, i2s)[0]
    s16 = i2s.to(torch.bfloat16)
    out["bf16_in2out_bf16_in2sol_rel_l2"] = solve_with(o16, s16)[0]
    del o16
    o32 = i2o.to(torch.float32)
    out["f32_in2out_bf16_in2sol_rel_l2"] = solve_with(o32, s16)[0]
    o16h = i2o.to(torch.float16).to(torch.float32)       # FP16 rounding of the operator
    out["f16_in2out_f64_in2sol_rel_l2"] = solve_with(o16h, i2s)[0]
    return out


def cpu_baseline(args, p, n_a):
    """The CPU oracle (NumPy / LAPACK, FP64) timed on the host cores, in a
    child process that never touches the GPU (one BLAS thread per pool
    worker): local solves of a bounded sample of the 128^2 workload, and the
    whole plain step (local solves, skeleton GMRES at the timed tolerance,
    recovery) on a coarser mesh of the same cloud."""
    import subprocess
    workers = args.cpu_workers or min(16, os.cpu_count() or 1)
    payload = json.dumps({"p": p, "n_a": n_a, "n": args.n, "sample": args.cpu_sample, "mesh": args.cpu_mesh,
                          "tol": args.tol, "restart": args.restart, "workers": workers})
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-worker-json", payload], env=env,
                       capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        log("cpu oracle failed: " + r.stderr[-2000:])
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


_ORACLE = {}


def _oracle_local_chunk(task):
    """Pool worker: oracle local solves of elements [e0, e1) of the problem
    set up before the fork; results go to the shared output arrays when given."""
    from threadpoolctl import threadpool_limits
    key, e0, e1 = task
    prob = _ORACLE[key]
    with threadpool_limits(1):
        for e in range(e0, e1):
            o, s_, _ = prob["disc"].local_solve(prob["h"], prob["kap"][e], prob["sig"][e])
            if "i2o" in prob:
                prob["i2o"][e] = o
                prob["i2s"][e] = s_
    return e1 - e0


def cpu_worker(payload):
    """Child-process body of cpu_baseline (no torch, no GPU)."""
    import multiprocessing as mp
    import platform
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.local import LocalDisc
    from oracle.mesh import Mesh
    from oracle import trace as otrace, recover as orecover
    from paper_2308_02467_amd import inputs
    P = json.loads(payload)
    p, n_a, workers = P["p"], P["n_a"], P["workers"]
    disc = LocalDisc(p, n_a)
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = sorted({f"{i.get('internal_api')} {i.get('version')}" for i in threadpool_info()
                   if i.get("user_api") == "blas"})

    def problem(nx):
        h = 1.0 / nx
        X, Y = inputs.element_node_coords(nx, nx, h, disc.xi)
        kap, sig = inputs.gaussian_cloud(X, Y)
        return h, kap, sig

    def run_pool(key, E):
        chunks = [(key, e0, min(E, e0 + max(1, E // (4 * workers)))) for e0 in range(0, E, max(1, E // (4 * workers)))]
        with mp.get_context("fork").Pool(workers) as pool:
            t0 = time.perf_counter()
            done = sum(pool.map(_oracle_local_chunk, chunks))
            dt = time.perf_counter() - t0
        assert done == E
        return dt

    # (1) local solves of a sample spread over the 128^2 mesh
    h, kap, sig = problem(P["n"])
    sel = np.linspace(0, kap.shape[0] - 1, P["sample"]).astype(np.int64)
    _ORACLE["sample"] = {"disc": disc, "h": h, "kap": kap[sel], "sig": sig[sel]}
    t_sample = run_pool("sample", sel.size)
    # (2) the whole plain step on a coarser mesh of the same cloud
    nx = P["mesh"]
    h, kap, sig = problem(nx)
    E = nx * nx
    shared = lambda *shape: np.frombuffer(mp.get_context("fork").RawArray("d", int(np.prod(shape))),
                                          dtype=np.float64).reshape(shape)
    i2o, i2s = shared(E, disc.m, disc.m), shared(E, disc.n, disc.m)
    _ORACLE["mesh"] = {"disc": disc, "h": h, "kap": kap, "sig": sig, "i2o": i2o, "i2s": i2s}
    t_local = run_pool("mesh", E)
    mesh = Mesh(nx, nx, h)
    ind, outd = mesh.element_dofs(disc)
    b = mesh.boundary_vector_sides(disc, inputs.left_inflow(n_a))
    with threadpool_limits(workers):
        t0 = time.perf_counter()
        t_sol, iters, relres = otrace.gmres(lambda x: otrace.matvec(i2o, ind, outd, x), b, tol=P["tol"],
                                            restart=P["restart"], max_iter=20000)
        t_gmres = time.perf_counter() - t0
        t0 = time.perf_counter()
        orecover.mean_intensity(disc, orecover.recover(i2s, ind, t_sol))
        t_rec = time.perf_counter() - t0
    step_s = t_local + t_gmres + t_rec
    out = {"value": E / step_s, "unit": f"element solves/s (whole plain step, {nx}x{nx} mesh of the same cloud)",
           "cores": workers, "kind": "oracle",
           "sample": f"whole plain FP64 step of the oracle on the {nx}x{nx} mesh of the same Gaussian cloud "
                     f"(p={p}, N_a={n_a}): {E} local solves over a pool of {workers} processes with one BLAS "
                     f"thread each {t_local:.1f} s, skeleton GMRES (tol {P['tol']:g}, restart {P['restart']}, "
                     f"{workers} BLAS threads) {t_gmres:.1f} s for {iters} iterations, recovery {t_rec:.2f} s; "
                     f"plus local solves of {sel.size} of the {P['n']}x{P['n']} elements {t_sample:.1f} s",
           "host_cores": os.cpu_count(), "cpu_model": model, "blas": blas,
           "whole_step_s": step_s, "phases_s": {"local_solve": t_local, "gmres": t_gmres, "recover": t_rec},
           "gmres_iters": iters, "gmres_relres": relres,
           "local_solve_el_per_s_128x128_sample": sel.size / t_sample, "local_solve_sample": int(sel.size)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()

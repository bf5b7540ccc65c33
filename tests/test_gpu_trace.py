"""GPU parity of the skeleton pieces and the whole plain path against the oracle.

* element DOF maps and the boundary right-hand side: bit-exact (integers /
  copies of the boundary data);
* (I - P) x with FP64 operators: <= 1e-13 relative; with FP32, FP16 and
  bfloat16 operators against the oracle product with the same rounded
  operator: <= 1e-13 (the products accumulate in FP64);
* recovery from FP32, FP16 and bfloat16 in2sol / in2mean against the oracle
  with the same rounded operators: <= 1e-13;
* trace solution (GMRES at 1e-12 vs the oracle's sparse direct solve) and the
  recovered intensity / mean intensity: <= 1e-10 relative;
* at 32 x 32 (p = 6, N_a = 16) where the oracle cannot run whole: sampled
  element operators against the oracle one by one, GMRES residual, and the
  global energy balance (incoming = outgoing + absorbed), a property that
  holds at any size.
"""
import numpy as np
import pytest
import torch

from oracle.local import LocalDisc, local_solve_batch
from oracle.mesh import Mesh
from oracle import trace as otrace, recover as orecover
from paper_2308_02467_amd import inputs

from _util import mesh_problem, oracle_pipeline, per_element_rel, rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def T(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02467_amd import el
    c = el.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("p,n_a,nx,ny", [(3, 8, 4, 4), (6, 16, 5, 3), (2, 4, 1, 1)])
def test_element_dofs_bit_exact(ctx, p, n_a, nx, ny):
    from paper_2308_02467_amd import el
    d, ms = el.disc(p, n_a), el.mesh(nx, ny, 1.0 / max(nx, ny))
    _, _, m = el.disc_sizes(d)
    ind = torch.empty((nx * ny, m), dtype=torch.int32, device=DEV)
    outd = torch.empty_like(ind)
    print(f"[el_element_dofs] p={p} n_a={n_a} {nx}x{ny}", flush=True)
    ctx.el_element_dofs(d, ms, ind, outd)
    oi, oo = Mesh(nx, ny, 1.0 / max(nx, ny)).element_dofs(LocalDisc(p, n_a))
    assert np.array_equal(ind.cpu().numpy(), oi)
    assert np.array_equal(outd.cpu().numpy(), oo)


def test_trace_rhs_bit_exact(ctx):
    from paper_2308_02467_amd import el
    p, n_a, nx, ny = 4, 8, 3, 5
    d, ms = el.disc(p, n_a), el.mesh(nx, ny, 0.2)
    g = np.random.default_rng(0).uniform(0, 2, (4, n_a))
    b = torch.full((el.trace_size(d, ms),), float("nan"), dtype=torch.float64, device=DEV)
    print("[el_trace_rhs]", flush=True)
    ctx.el_trace_rhs(d, ms, g, b)
    ref = Mesh(nx, ny, 0.2).boundary_vector_sides(LocalDisc(p, n_a), g)
    assert np.array_equal(b.cpu().numpy(), ref)


@pytest.fixture
def matvec_shape():
    """Pins the skeleton product's row shape for one test and restores the
    autotuner."""
    from paper_2308_02467_amd import el
    yield el.matvec_shape
    el.matvec_shape(-1)


# shape -1: the autotuner's choice; 0-2: the three row shapes pinned
MV_SHAPES = [-1, 0, 1, 2]


@pytest.mark.parametrize("shape", MV_SHAPES)
@pytest.mark.parametrize("p,n_a,nx,ny", [(3, 8, 4, 4), (6, 16, 3, 2)])
def test_matvec_f64_and_bf16(ctx, matvec_shape, shape, p, n_a, nx, ny):
    from paper_2308_02467_amd import el
    matvec_shape(shape)
    od, oms, hh, kap, sig = mesh_problem(p, n_a, nx, ny)
    i2o, _, _ = local_solve_batch(od, hh, kap, sig)
    ind, outd = oms.element_dofs(od)
    d, ms = el.disc(p, n_a), el.mesh(nx, ny, oms.h)
    nt = el.trace_size(d, ms)
    x = np.random.default_rng(1).standard_normal(nt)
    y = torch.full((nt,), float("nan"), dtype=torch.float64, device=DEV)
    print(f"[el_trace_matvec] p={p} n_a={n_a} {nx}x{ny} shape={shape} f64", flush=True)
    ctx.el_trace_matvec(d, ms, T(i2o), T(x), y)
    ref = otrace.matvec(i2o, ind, outd, x)
    assert rel_err(y.cpu().numpy(), ref) <= 1e-13
    # bfloat16 operator (round to nearest even), FP64 accumulation
    op16 = T(i2o).to(torch.bfloat16)
    print(f"[el_trace_matvec] p={p} n_a={n_a} {nx}x{ny} bf16", flush=True)
    ctx.el_trace_matvec(d, ms, op16, T(x), y)
    ref16 = otrace.matvec(op16.to(torch.float64).cpu().numpy(), ind, outd, x)
    assert rel_err(y.cpu().numpy(), ref16) <= 1e-13
    op32 = T(i2o).to(torch.float32)
    print(f"[el_trace_matvec] p={p} n_a={n_a} {nx}x{ny} f32", flush=True)
    ctx.el_trace_matvec(d, ms, op32, T(x), y)
    ref32 = otrace.matvec(op32.to(torch.float64).cpu().numpy(), ind, outd, x)
    assert rel_err(y.cpu().numpy(), ref32) <= 1e-13
    # IEEE binary16 operator
    oph = T(i2o).to(torch.float16)
    print(f"[el_trace_matvec] p={p} n_a={n_a} {nx}x{ny} f16", flush=True)
    ctx.el_trace_matvec(d, ms, oph, T(x), y)
    refh = otrace.matvec(oph.to(torch.float64).cpu().numpy(), ind, outd, x)
    assert rel_err(y.cpu().numpy(), refh) <= 1e-13
    if shape < 0:
        # the autotuner timed the row shapes for each operator type of this m
        m = el.disc_sizes(d)[2]
        rep = el.tuning_report()
        for name in ("f64", "bf16", "f32", "f16"):
            assert f" matvec {name} m={m} -> shape " in rep, rep


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16, torch.bfloat16])
def test_recover_operator_dtypes(ctx, dtype):
    """u = in2sol t_in and the mean intensity (from in2sol and from in2mean)
    with rounded operators, against the oracle with the same rounding."""
    from paper_2308_02467_amd import el
    p, n_a, nx, ny = 3, 8, 3, 4
    od, oms, hh, kap, sig = mesh_problem(p, n_a, nx, ny)
    _, i2s, i2m = local_solve_batch(od, hh, kap, sig)
    ind, _ = oms.element_dofs(od)
    d, ms = el.disc(p, n_a), el.mesh(nx, ny, oms.h)
    nn, n, m = el.disc_sizes(d)
    E = nx * ny
    t = np.random.default_rng(3).standard_normal(el.trace_size(d, ms))
    S = T(i2s).to(dtype)
    Mn = T(i2m).to(dtype)
    u = torch.full((E, n), float("nan"), dtype=torch.float64, device=DEV)
    mean = torch.full((E, nn), float("nan"), dtype=torch.float64, device=DEV)
    mean2 = torch.full_like(mean, float("nan"))
    print(f"[el_recover] {dtype}", flush=True)
    ctx.el_recover(d, ms, S, T(t), u, mean)
    ctx.el_recover_mean(d, ms, Mn, T(t), mean2)
    Sr = S.to(torch.float64).cpu().numpy()
    Mr = Mn.to(torch.float64).cpu().numpy()
    u_ref = orecover.recover(Sr, ind, t)
    assert rel_err(u.cpu().numpy(), u_ref) <= 1e-13
    assert rel_err(mean.cpu().numpy(), orecover.mean_intensity(od, u_ref)) <= 1e-13
    assert rel_err(mean2.cpu().numpy(), orecover.recover(Mr, ind, t)) <= 1e-13


def _gpu_pipeline(ctx, p, n_a, g, nx, ny, hh, kap, sig, g_side, tol=1e-12, outputs=True, angular=None):
    from paper_2308_02467_amd import el
    d, ms = el.disc(p, n_a, g, angular), el.mesh(nx, ny, 1.0 / max(nx, ny))
    nn, n, m = el.disc_sizes(d)
    E = nx * ny
    i2o = torch.empty((E, m, m), dtype=torch.float64, device=DEV)
    i2s = torch.empty((E, n, m), dtype=torch.float64, device=DEV)
    i2m = torch.empty((E, nn, m), dtype=torch.float64, device=DEV)
    print(f"[pipeline] p={p} n_a={n_a} {nx}x{ny} local", flush=True)
    ctx.el_local_solve(d, T(hh), T(kap), T(sig), in2out=i2o, in2sol=i2s, in2mean=i2m)
    nt = el.trace_size(d, ms)
    b = torch.empty(nt, dtype=torch.float64, device=DEV)
    ctx.el_trace_rhs(d, ms, g_side, b)
    t = torch.empty(nt, dtype=torch.float64, device=DEV)
    print(f"[pipeline] p={p} n_a={n_a} {nx}x{ny} gmres", flush=True)
    st, rep = ctx.el_trace_solve(d, [ms], [i2o], [b], [t], tol=tol, restart=50, max_iter=3000)
    u = torch.empty((E, n), dtype=torch.float64, device=DEV)
    mean = torch.empty((E, nn), dtype=torch.float64, device=DEV)
    print(f"[pipeline] p={p} n_a={n_a} {nx}x{ny} recover", flush=True)
    ctx.el_recover(d, ms, i2s, t, u, mean)
    mean2 = torch.empty_like(mean)
    ctx.el_recover_mean(d, ms, i2m, t, mean2)
    torch.cuda.synchronize()
    res = dict(in2out=i2o, in2sol=i2s, in2mean=i2m, b=b, t=t, u=u, mean=mean, mean2=mean2)
    return {k: v.cpu().numpy() for k, v in res.items()}, rep[0], st


@pytest.mark.parametrize("p,n_a,nx,field", [(3, 8, 4, "const"), (6, 16, 6, "gauss"), (4, 8, 5, "sharp")])
def test_plain_pipeline_parity(ctx, p, n_a, nx, field):
    od, oms, hh, kap, sig = mesh_problem(p, n_a, nx, field=field)
    gs = inputs.left_inflow(n_a)
    ref = oracle_pipeline(od, oms, hh, kap, sig, gs)
    gpu, rep, st = _gpu_pipeline(ctx, p, n_a, 0.0, nx, nx, hh, kap, sig, gs)
    assert rep["converged"] and rep["relres"] <= 1e-12, rep
    for k in ("in2out", "in2sol", "in2mean"):
        assert per_element_rel(gpu[k], ref[k]) <= 1e-10, k
    assert np.array_equal(gpu["b"], ref["b"])
    for k in ("t", "u", "mean"):
        assert rel_err(gpu[k], ref[k]) <= 1e-10, (k, rel_err(gpu[k], ref[k]))
    assert rel_err(gpu["mean2"], ref["mean"]) <= 1e-10
    from paper_2308_02467_amd import el
    a = gpu["mean"] + 1e-3
    d2, r2 = ctx.el_mean_l2(el.disc(p, n_a), T(hh), T(a), T(ref["mean"]))
    exp_d2 = orecover.l2_norm_sq(od, hh, a - ref["mean"])
    assert abs(d2 - exp_d2) <= 1e-12 * exp_d2 + 1e-300
    assert abs(r2 - orecover.l2_norm_sq(od, hh, ref["mean"])) <= 1e-12 * r2


def test_hg_pipeline_parity(ctx):
    p, n_a, g, nx = 3, 12, 0.85, 4
    od, oms, hh, kap, sig = mesh_problem(p, n_a, nx, g=g)
    gs = inputs.left_inflow(n_a)
    gs[3, :] = 0.3
    ref = oracle_pipeline(od, oms, hh, kap, sig, gs)
    gpu, rep, st = _gpu_pipeline(ctx, p, n_a, g, nx, nx, hh, kap, sig, gs)
    for k in ("t", "u", "mean"):
        assert rel_err(gpu[k], ref[k]) <= 1e-10, k


@pytest.mark.parametrize("g", [0.0, 0.85])
def test_p0_angular_pipeline_parity(ctx, g):
    """P0 angular elements (cell-averaged directions and phase kernel): local
    operators, skeleton solution and recovery against the oracle's P0 form."""
    from paper_2308_02467_amd import el
    p, n_a, nx = 3, 12, 4
    _, oms, hh, kap, sig = mesh_problem(p, n_a, nx, g=g)
    od = LocalDisc(p, n_a, g, "p0")
    gs = inputs.left_inflow(n_a)
    ref = oracle_pipeline(od, oms, hh, kap, sig, gs)
    gpu, rep, st = _gpu_pipeline(ctx, p, n_a, g, nx, nx, hh, kap, sig, gs, angular=el.EL_ANG_P0)
    for k in ("in2out", "in2sol", "in2mean", "t", "u", "mean"):
        assert rel_err(gpu[k], ref[k]) <= 1e-10, k
    # and the form matters: the ordinates differ from it
    assert rel_err(gpu["in2out"], local_solve_batch(LocalDisc(p, n_a, g), hh, kap, sig)[0]) > 1e-4


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_volume_source_pipeline_parity(ctx, precision):
    """Alg. 1 with a volume source f: the source responses f_u and f_hat_u of
    the local solve, the skeleton right-hand side with f_hat_u, the trace and
    the recovered intensity against the oracle's source path."""
    from paper_2308_02467_amd import el
    p, n_a, g, nx = 3, 8, 0.5, 4
    od, oms, hh, kap, sig = mesh_problem(p, n_a, nx, g=g)
    E = nx * nx
    X, Y = inputs.element_node_coords(nx, nx, oms.h, od.xi)
    th = od.theta
    f = (1.0 + 0.5 * np.sin(3 * X)[:, None, :] * np.cos(th)[None, :, None]
         + 0.3 * Y[:, None, :] * np.sin(2 * th)[None, :, None])                # [E, n_a, nn]
    gs = inputs.left_inflow(n_a)
    i2o, i2s, _ = local_solve_batch(od, hh, kap, sig)
    ind, outd = oms.element_dofs(od)
    rhs = oms.boundary_vector_sides(od, gs)
    fus, fhats = [], []
    for e in range(E):
        fu, fhat = od.source_solve(hh[e], kap[e], sig[e], f[e])
        fus.append(fu)
        fhats.append(fhat)
        rhs[outd[e]] += fhat
    fus, fhats = np.array(fus), np.array(fhats)
    t_ref = otrace.solve_direct(i2o, ind, outd, rhs)
    u_ref = np.einsum("enm,em->en", i2s, t_ref[ind]) + fus
    mean_ref = orecover.mean_intensity(od, u_ref)

    d, ms = el.disc(p, n_a, g), el.mesh(nx, nx, oms.h)
    nn, n, m = el.disc_sizes(d)
    prec = el.EL_FP64 if precision == "fp64" else el.EL_FP32_IR
    o = torch.empty((E, m, m), dtype=torch.float64, device=DEV)
    sv = torch.empty((E, n, m), dtype=torch.float64, device=DEV)
    mv = torch.empty((E, nn, m), dtype=torch.float64, device=DEV)
    s2out = torch.full((E, m), float("nan"), dtype=torch.float64, device=DEV)
    s2sol = torch.full((E, n), float("nan"), dtype=torch.float64, device=DEV)
    s2mean = torch.full((E, nn), float("nan"), dtype=torch.float64, device=DEV)
    print(f"[el_local_solve] with source, {precision}", flush=True)
    ctx.el_local_solve(d, T(hh), T(kap), T(sig), precision=prec, in2out=o, in2sol=sv, in2mean=mv, src=T(f),
                       src2out=s2out, src2sol=s2sol, src2mean=s2mean)
    tol = 1e-10 if precision == "fp64" else 1e-9
    assert rel_err(s2sol.cpu().numpy(), fus) <= tol
    assert rel_err(s2out.cpu().numpy(), fhats) <= tol
    assert rel_err(o.cpu().numpy(), i2o) <= tol
    nt = el.trace_size(d, ms)
    b = torch.empty(nt, dtype=torch.float64, device=DEV)
    ctx.el_trace_rhs(d, ms, gs, b)
    ctx.el_trace_add_source(d, ms, s2out, b)
    assert rel_err(b.cpu().numpy(), rhs) <= tol
    t = torch.empty(nt, dtype=torch.float64, device=DEV)
    st, rep = ctx.el_trace_solve(d, [ms], [o], [b], [t], tol=1e-12, restart=30, max_iter=3000)
    assert st == 0
    u = torch.empty((E, n), dtype=torch.float64, device=DEV)
    mean = torch.empty((E, nn), dtype=torch.float64, device=DEV)
    mean2 = torch.empty((E, nn), dtype=torch.float64, device=DEV)
    ctx.el_recover(d, ms, sv, t, u, mean, src2sol=s2sol)
    ctx.el_recover_mean(d, ms, mv, t, mean2, src2mean=s2mean)
    assert rel_err(t.cpu().numpy(), t_ref) <= tol
    assert rel_err(u.cpu().numpy(), u_ref) <= tol
    assert rel_err(mean.cpu().numpy(), mean_ref) <= tol
    assert rel_err(mean2.cpu().numpy(), mean_ref) <= tol


def test_full_size_32x32_sampled_and_energy(ctx):
    """The 32x32, p=6, N_a=16 Gaussian-cloud workload: sampled element
    operators vs the oracle, GMRES residual, global energy balance."""
    p, n_a, nx = 6, 16, 32
    od, oms, hh, kap, sig = mesh_problem(p, n_a, nx)
    gs = inputs.left_inflow(n_a)
    gpu, rep, st = _gpu_pipeline(ctx, p, n_a, 0.0, nx, nx, hh, kap, sig, gs)
    assert rep["converged"] and rep["relres"] <= 1e-12, rep
    sel = np.array([0, 17, 31, 32, 500, 527, 777, 1023])
    i2o, i2s, i2m = local_solve_batch(od, hh[sel], kap[sel], sig[sel])
    assert per_element_rel(gpu["in2out"][sel], i2o) <= 1e-10
    assert per_element_rel(gpu["in2sol"][sel], i2s) <= 1e-10
    assert per_element_rel(gpu["in2mean"][sel], i2m) <= 1e-10
    inc, outg = orecover.boundary_fluxes(od, oms, gpu["t"], oms.inflow_mask(od))
    ab = orecover.absorption(od, hh, kap, gpu["u"])
    assert abs(inc - outg - ab) <= 1e-10 * inc, (inc, outg, ab)
    # the recovered outflow equals the trace on every outflow DOF (R^o u = t)
    ind, outd = oms.element_dofs(od)
    u = gpu["u"]
    assert rel_err(u[:, od.out_rows].reshape(-1), gpu["t"][outd].reshape(-1)) <= 1e-10


# balance after the rescaling, relative to the largest inflow weight: the
# rescaled entries are rounded back to the storage type
CONSERVE_TOL = {torch.float64: 1e-12, torch.float32: 2e-6, torch.float16: 2e-3}
# change of exact operators (which already balance) beyond their rounding
CONSERVE_KEEP = {torch.float64: 1e-13, torch.float32: 1e-6, torch.float16: 1e-3}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16])
def test_conserve_energy_balance(ctx, dtype):
    """el_conserve leaves exact operators unchanged (they already satisfy the
    per-element energy balance) and restores the balance of perturbed ones."""
    from paper_2308_02467_amd import el
    p, n_a = 3, 8
    o = LocalDisc(p, n_a)
    h, kap, sig = inputs.training_draws(20, o.xi, seed=4)
    i2o, i2s, _ = local_solve_batch(o, h, kap, sig)
    d = el.disc(p, n_a)
    wout = np.array([o.omega[j] * o.sn[k, f] for (f, k, j, nd, r) in o.out_tab])
    win = np.array([-o.omega[j] * o.sn[k, f] for (f, k, j, nd, r) in o.in_tab])

    def balance(O, S):
        ab = np.einsum("n,enm->em", np.tile(o.W, n_a), (0.5 * h[:, None, None] * np.tile(kap, (1, n_a))[:, :, None]) * S)
        return np.einsum("o,eom->em", wout, O) + ab - win[None, :]

    tol = CONSERVE_TOL[dtype]
    O = T(i2o).to(dtype)
    S = T(i2s).to(dtype)
    print(f"[el_conserve] {dtype}", flush=True)
    ctx.el_conserve(d, T(h), T(kap), O, S)
    assert rel_err(O.to(torch.float64).cpu().numpy(), i2o) <= CONSERVE_KEEP[dtype]
    rng = np.random.default_rng(0)
    Op = T(i2o * (1 + 0.02 * rng.standard_normal(i2o.shape))).to(dtype)
    before = Op.clone()
    mask = torch.ones(20, dtype=torch.uint8, device=DEV)
    mask[5] = 0
    ctx.el_conserve(d, T(h), T(kap), Op, S, mask)
    got = Op.to(torch.float64).cpu().numpy()
    Sd = S.to(torch.float64).cpu().numpy()
    bal = balance(got, Sd)
    keep = np.arange(20) != 5
    assert np.abs(bal[keep]).max() <= tol * np.abs(win).max()
    assert torch.equal(Op[5], before[5])          # masked element left bit-identical
    # the documented rule: column c of in2out is scaled by one factor
    # s_c = (w_c - absorption_c) / sum_o w_o in2out[o][c], computed here on
    # the host from the operators the kernel received
    P = before.to(torch.float64).cpu().numpy()
    ab = balance(np.zeros_like(P), Sd) + win[None, :]
    s_host = _column_factors(win[None, :] - ab, np.einsum("o,eom->em", wout, P))
    _check_column_scaling(got[keep], P[keep], s_host[keep], dtype)


def _column_factors(target, colsum):
    """One factor per column: target / colsum, or 1 where either is not
    positive (the column is then left as it is)."""
    ok = (target > 0) & (colsum > 0)
    return np.where(ok, target / np.where(ok, colsum, 1.0), 1.0)


def _check_column_scaling(got, P, s_host, dtype):
    """got == P * s_host per column, up to one rounding to dtype."""
    exp = P * s_host[:, None, :]
    rel, tiny = {torch.float64: (1e-14, 0.0), torch.float32: (2.0 ** -23, 1e-38),
                 torch.float16: (2.0 ** -10, 2.0 ** -24)}[dtype]
    err = np.abs(got - exp) - rel * np.abs(exp) - tiny
    print(f"[el_conserve] column scaling: worst excess {err.max():.3e}, "
          f"factors in [{s_host.min():.4f}, {s_host.max():.4f}]", flush=True)
    assert np.all(err <= 0)


@pytest.mark.parametrize("odt", [torch.float16, torch.bfloat16])
def test_conserve_out_of_place_rounds_once(ctx, odt):
    """float32 operators corrected into a float16 / bfloat16 output: the
    float32 in-place correction rounded to the 16-bit type (bit-exact up to
    ties); masked elements are copied unchanged; overlapping or widening
    outputs are refused."""
    from paper_2308_02467_amd import el
    p, n_a = 3, 8
    o = LocalDisc(p, n_a)
    E = 16
    h, kap, sig = inputs.training_draws(E, o.xi, seed=8)
    i2o, i2s, _ = local_solve_batch(o, h, kap, sig)
    d = el.disc(p, n_a)
    rng = np.random.default_rng(5)
    O32 = T(i2o * (1 + 0.01 * rng.standard_normal(i2o.shape))).to(torch.float32)
    S32 = T(i2s).to(torch.float32)
    mask = torch.ones(E, dtype=torch.uint8, device=DEV)
    mask[3] = 0
    out = torch.full(O32.shape, float("nan"), dtype=odt, device=DEV)
    print(f"[el_conserve] float32 -> {odt}", flush=True)
    ctx.el_conserve(d, T(h), T(kap), O32, S32, mask, out=out)
    src = O32.clone()
    ctx.el_conserve(d, T(h), T(kap), O32, S32, mask)
    # the kernel rounds the FP64 product once; the reference rounds it to FP32
    # first: they may differ only where the FP32 value is a tie between two
    # neighbours of the 16-bit type
    ref = O32.to(odt)
    bad = out != ref
    assert torch.all(out[bad].double() + ref[bad].double() == 2 * O32[bad].double())
    assert int(bad.sum()) <= 1e-3 * bad.numel()
    assert torch.equal(out[3], src[3].to(odt))
    assert not torch.equal(out[0], src[0].to(odt))
    overlap = O32.view(-1).view(odt)[2:2 + O32.numel()]       # inside in2out's memory, not at its start
    with pytest.raises(el.ElError):
        ctx.el_conserve(d, T(h), T(kap), O32, S32, mask, out=overlap)
    wide = torch.empty(O32.shape, dtype=torch.float64, device=DEV)
    with pytest.raises(el.ElError):
        ctx.el_conserve(d, T(h), T(kap), O32, S32, mask, out=wide)


# Batched uneven meshes in one call (sizes in the spirit of the 16^2 ... 128^2
# batch, scaled so the oracle's direct solves finish in seconds); sharp cloud
# edge with a seeded random centre per mesh.
BATCH = [(2, 2), (3, 3), (4, 4), (4, 4), (6, 6), (5, 3), (1, 1), (3, 7)]


def _batched_problem(p, n_a):
    probs = []
    for i, (nx, ny) in enumerate(BATCH):
        od, oms, hh, kap, sig = mesh_problem(p, n_a, nx, ny, field="sharp", seed=10 + i)
        probs.append((od, oms, hh, kap, sig))
    return probs


def _batched_gpu(ctx, p, n_a, probs, graph, tol=1e-12, basis=torch.float64):
    from paper_2308_02467_amd import el
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    hh = np.concatenate([pr[2] for pr in probs])
    kap = np.concatenate([pr[3] for pr in probs])
    sig = np.concatenate([pr[4] for pr in probs])
    E = hh.size
    i2o = torch.empty((E, m, m), dtype=torch.float64, device=DEV)
    print(f"[batched] local solve of {E} elements from {len(probs)} meshes", flush=True)
    ctx.el_local_solve(d, T(hh), T(kap), T(sig), in2out=i2o)
    meshes, ops, bs, ts = [], [], [], []
    e0 = 0
    gs = inputs.left_inflow(n_a)
    for od, oms, h, _, _ in probs:
        ms = el.mesh(oms.n_x, oms.n_y, oms.h)
        nt = el.trace_size(d, ms)
        b = torch.empty(nt, dtype=torch.float64, device=DEV)
        ctx.el_trace_rhs(d, ms, gs, b)
        meshes.append(ms)
        ops.append(i2o[e0:e0 + h.size])
        bs.append(b)
        ts.append(torch.full((nt,), float("nan"), dtype=torch.float64, device=DEV))
        e0 += h.size
    print(f"[batched] el_trace_solve n_mesh={len(meshes)} graph={graph} basis={basis}", flush=True)
    st, rep = ctx.el_trace_solve(d, meshes, ops, bs, ts, tol=tol, restart=20, max_iter=3000, graph=graph,
                                 basis=basis)
    torch.cuda.synchronize()
    return st, rep, [t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("basis", [torch.float64, torch.float32])
def test_batched_uneven_meshes_parity(ctx, basis):
    """Several meshes in one GMRES against the oracle's direct solves; with
    the FP32 Krylov basis the restart residuals are still FP64, so the same
    tolerance is reached."""
    p, n_a = 3, 8
    probs = _batched_problem(p, n_a)
    st, rep, ts = _batched_gpu(ctx, p, n_a, probs, graph=True, basis=basis)
    assert st == 0
    for (od, oms, hh, kap, sig), r, t in zip(probs, rep, ts):
        ref = oracle_pipeline(od, oms, hh, kap, sig, inputs.left_inflow(n_a))
        assert r["converged"] and r["relres"] <= 1e-12, r
        assert rel_err(t, ref["t"]) <= 1e-10, (oms.n_x, oms.n_y, rel_err(t, ref["t"]))


@pytest.mark.parametrize("shape", MV_SHAPES)
@pytest.mark.parametrize("basis", [torch.float64, torch.float32])
@pytest.mark.parametrize("dtype", [torch.float16, torch.float32])
def test_batched_rounded_operators_parity(ctx, matvec_shape, shape, dtype, basis):
    """GMRES over several meshes with FP16 / FP32 operators (the storage of
    the learned step), with either Krylov basis: the solution of
    (I - P~) t = b with the rounded operators P~, against the oracle's direct
    solve with the same rounded operators."""
    from paper_2308_02467_amd import el
    matvec_shape(shape)
    p, n_a = 3, 8
    probs = _batched_problem(p, n_a)[:4]
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    gs = inputs.left_inflow(n_a)
    meshes, ops, bs, ts, refs = [], [], [], [], []
    for od, oms, hh, kap, sig in probs:
        i2o, _, _ = local_solve_batch(od, hh, kap, sig)
        op = T(i2o).to(dtype)
        ind, outd = oms.element_dofs(od)
        rounded = op.to(torch.float64).cpu().numpy()
        refs.append(otrace.solve_direct(rounded, ind, outd, oms.boundary_vector_sides(od, gs)))
        ms = el.mesh(oms.n_x, oms.n_y, oms.h)
        nt = el.trace_size(d, ms)
        b = torch.empty(nt, dtype=torch.float64, device=DEV)
        ctx.el_trace_rhs(d, ms, gs, b)
        meshes.append(ms)
        ops.append(op)
        bs.append(b)
        ts.append(torch.full((nt,), float("nan"), dtype=torch.float64, device=DEV))
    print(f"[batched] el_trace_solve {dtype} basis={basis} shape={shape} n_mesh={len(meshes)}", flush=True)
    st, rep = ctx.el_trace_solve(d, meshes, ops, bs, ts, tol=1e-12, restart=20, max_iter=3000, basis=basis)
    assert st == 0
    for r, t, ref in zip(rep, ts, refs):
        assert r["converged"] and r["relres"] <= 1e-12, r
        assert rel_err(t.cpu().numpy(), ref) <= 1e-10


def test_gmres_starting_guess(ctx):
    """x0 = 1: starting from the converged solution takes no Arnoldi step and
    returns it; starting from a perturbed one converges to the oracle's
    solution; b = 0 returns 0 whatever the guess."""
    from paper_2308_02467_amd import el
    p, n_a, nx, ny = 3, 8, 4, 3
    od, oms, hh, kap, sig = mesh_problem(p, n_a, nx, ny, field="sharp", seed=3)
    i2o, _, _ = local_solve_batch(od, hh, kap, sig)
    ind, outd = oms.element_dofs(od)
    gs = inputs.left_inflow(n_a)
    ref = otrace.solve_direct(i2o, ind, outd, oms.boundary_vector_sides(od, gs))
    d, ms = el.disc(p, n_a), el.mesh(nx, ny, oms.h)
    nt = el.trace_size(d, ms)
    b = torch.empty(nt, dtype=torch.float64, device=DEV)
    ctx.el_trace_rhs(d, ms, gs, b)
    op = T(i2o)
    t = torch.zeros(nt, dtype=torch.float64, device=DEV)
    print("[el_trace_solve] cold", flush=True)
    st, rep = ctx.el_trace_solve(d, [ms], [op], [b], [t], tol=1e-12, restart=20, max_iter=3000)
    assert st == 0 and rep[0]["iters"] > 0
    t_cold = t.clone()
    print("[el_trace_solve] from the solution", flush=True)
    st, rep = ctx.el_trace_solve(d, [ms], [op], [b], [t], tol=1e-12, restart=20, max_iter=3000, x0=True)
    assert st == 0 and rep[0]["iters"] == 0 and torch.equal(t, t_cold)
    rng = np.random.default_rng(9)
    t.copy_(t_cold + T(1e-3 * rng.standard_normal(nt)))
    print("[el_trace_solve] from a perturbed solution", flush=True)
    st, rep = ctx.el_trace_solve(d, [ms], [op], [b], [t], tol=1e-12, restart=20, max_iter=3000, x0=True)
    assert st == 0 and rep[0]["converged"] and rep[0]["iters"] > 0
    assert rel_err(t.cpu().numpy(), ref) <= 1e-10
    z = torch.zeros_like(b)
    t.copy_(t_cold)
    print("[el_trace_solve] zero rhs from a nonzero guess", flush=True)
    st, rep = ctx.el_trace_solve(d, [ms], [op], [z], [t], tol=1e-12, restart=20, max_iter=3000, x0=True)
    assert st == 0 and rep[0]["converged"] and torch.all(t == 0)


@pytest.mark.parametrize("basis", [torch.float64, torch.float32])
def test_batched_graph_replays_match_eager(ctx, basis):
    """The captured restart cycle gives bit-identical results to launching the
    same kernels one by one, on every replay, with other device work and
    synchronizations between the solves."""
    p, n_a = 3, 8
    probs = _batched_problem(p, n_a)
    _, rep0, ref = _batched_gpu(ctx, p, n_a, probs, graph=False, basis=basis)
    for it in range(3):
        junk = torch.randn(1 << 20, dtype=torch.float64, device=DEV)
        (junk * 2).sum().item()
        _, rep, ts = _batched_gpu(ctx, p, n_a, probs, graph=True, basis=basis)
        for a, b, r, r0 in zip(ts, ref, rep, rep0):
            assert np.array_equal(a, b), it
            assert r == r0, it


def test_batched_single_mesh_converged_and_empty_rhs(ctx):
    """A mesh with a zero right-hand side returns t = 0 at once while the
    other meshes of the batch iterate."""
    from paper_2308_02467_amd import el
    p, n_a = 2, 4
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    od, oms, hh, kap, sig = mesh_problem(p, n_a, 3, 2, field="gauss")
    i2o = torch.empty((hh.size, m, m), dtype=torch.float64, device=DEV)
    ctx.el_local_solve(d, T(hh), T(kap), T(sig), in2out=i2o)
    ms = el.mesh(3, 2, oms.h)
    nt = el.trace_size(d, ms)
    b1 = torch.empty(nt, dtype=torch.float64, device=DEV)
    ctx.el_trace_rhs(d, ms, inputs.left_inflow(n_a), b1)
    b0 = torch.zeros(nt, dtype=torch.float64, device=DEV)
    t0 = torch.full((nt,), float("nan"), dtype=torch.float64, device=DEV)
    t1 = torch.full((nt,), float("nan"), dtype=torch.float64, device=DEV)
    print("[batched] zero rhs mesh", flush=True)
    st, rep = ctx.el_trace_solve(d, [ms, ms], [i2o, i2o], [b0, b1], [t0, t1], tol=1e-12, restart=5)
    assert st == 0
    assert rep[0]["iters"] == 0 and rep[0]["converged"] and torch.all(t0 == 0)
    ref = oracle_pipeline(od, oms, hh, kap, sig, inputs.left_inflow(n_a))
    assert rel_err(t1.cpu().numpy(), ref["t"]) <= 1e-10
    assert rep[1]["restarts"] >= 1


def test_gmres_max_iter_reports_not_converged(ctx):
    """Failure handling: with max_iter = 1 the solve stops after one Arnoldi
    step and returns EL_WARN_NOT_CONVERGED; the report says so, and its
    relative residual is the true residual of the trace it returned
    (recomputed here with the oracle's product)."""
    from paper_2308_02467_amd import el
    p, n_a = 3, 8
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    od, oms, hh, kap, sig = mesh_problem(p, n_a, 4, 4, field="const")
    i2o_np, _, _ = local_solve_batch(od, hh, kap, sig)
    i2o = T(i2o_np)
    ms = el.mesh(4, 4, oms.h)
    nt = el.trace_size(d, ms)
    b = torch.empty(nt, dtype=torch.float64, device=DEV)
    ctx.el_trace_rhs(d, ms, inputs.left_inflow(n_a), b)
    for basis in (torch.float64, torch.float32):
        t = torch.full((nt,), float("nan"), dtype=torch.float64, device=DEV)
        print(f"[gmres max_iter=1] basis {basis}", flush=True)
        st, rep = ctx.el_trace_solve(d, [ms], [i2o], [b], [t], tol=1e-12, restart=10, max_iter=1, basis=basis)
        assert st == el.EL_WARN_NOT_CONVERGED
        assert rep[0]["iters"] == 1 and not rep[0]["converged"]
        ind, outd = oms.element_dofs(od)
        bn = b.cpu().numpy()
        res = np.linalg.norm(bn - otrace.matvec(i2o_np, ind, outd, t.cpu().numpy())) / np.linalg.norm(bn)
        print(f"[gmres max_iter=1] reported {rep[0]['relres']:.6e}, recomputed {res:.6e}", flush=True)
        assert 1e-12 < res < 1.0
        assert abs(rep[0]["relres"] - res) <= 1e-12 * res + 1e-15


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16])
def test_conserve_in2mean_form(ctx, dtype):
    """The balance with the ordinate-averaged operator: exact (in2out, in2mean)
    pairs are left unchanged and perturbed ones are restored."""
    from paper_2308_02467_amd import el
    p, n_a = 3, 8
    o = LocalDisc(p, n_a)
    h, kap, sig = inputs.training_draws(12, o.xi, seed=6)
    i2o, _, i2m = local_solve_batch(o, h, kap, sig)
    d = el.disc(p, n_a)
    wout = np.array([o.omega[j] * o.sn[k, f] for (f, k, j, nd, r) in o.out_tab])
    win = np.array([-o.omega[j] * o.sn[k, f] for (f, k, j, nd, r) in o.in_tab])
    tol = CONSERVE_TOL[dtype]
    O = T(i2o).to(dtype)
    Mn = T(i2m).to(dtype)
    print(f"[el_conserve] in2mean {dtype}", flush=True)
    ctx.el_conserve(d, T(h), T(kap), O, in2mean=Mn)
    assert rel_err(O.to(torch.float64).cpu().numpy(), i2o) <= CONSERVE_KEEP[dtype]
    rng = np.random.default_rng(2)
    Op = T(i2o * (1 + 0.02 * rng.standard_normal(i2o.shape))).to(dtype)
    P = Op.to(torch.float64).cpu().numpy()
    ctx.el_conserve(d, T(h), T(kap), Op, in2mean=Mn)
    got = Op.to(torch.float64).cpu().numpy()
    ab = n_a * np.einsum("n,enm->em", o.W, (0.5 * h[:, None, None] * kap[:, :, None]) * Mn.to(torch.float64).cpu().numpy())
    bal = np.einsum("o,eom->em", wout, got) + ab - win[None, :]
    assert np.abs(bal).max() <= tol * np.abs(win).max()
    _check_column_scaling(got, P, _column_factors(win[None, :] - ab, np.einsum("o,eom->em", wout, P)), dtype)


@pytest.mark.parametrize("basis", [torch.float64, torch.float32])
def test_batched_full_size_sampled_and_energy(ctx, basis):
    """The batched workload at its real sizes (meshes of 16^2 ... 128^2
    elements, p = 6, N_a = 16, sharp cloud edge): one local solve over all
    53,760 elements and one GMRES over the eight skeleton systems.  Checked
    by sampled element operators against the oracle, the true residual of
    every mesh, and every mesh's global energy balance (incoming = outgoing
    + absorbed, the absorption from the mean intensity)."""
    from paper_2308_02467_amd import el
    p, n_a = 6, 16
    sides = (16, 32, 48, 64, 64, 96, 128, 128)
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    o = LocalDisc(p, n_a)
    probs = []
    for i, s_ in enumerate(sides):
        od, oms, hh, kap, sig = mesh_problem(p, n_a, s_, s_, field="sharp", seed=100 + i)
        probs.append((oms, hh, kap, sig))
    H = T(np.concatenate([pr[1] for pr in probs]))
    K = T(np.concatenate([pr[2] for pr in probs]))
    S = T(np.concatenate([pr[3] for pr in probs]))
    E = H.numel()
    i2o = torch.empty((E, m, m), dtype=torch.float64, device=DEV)
    i2m = torch.empty((E, nn, m), dtype=torch.float64, device=DEV)
    print(f"[batched full] local solve of {E} elements", flush=True)
    ctx.el_local_solve(d, H, K, S, in2out=i2o, in2mean=i2m)
    offs = np.cumsum([0] + [s_ * s_ for s_ in sides])
    gs = inputs.left_inflow(n_a)
    meshes, bs, ts = [], [], []
    for (oms, hh, _, _) in probs:
        ms = el.mesh(oms.n_x, oms.n_y, oms.h)
        b = torch.empty(el.trace_size(d, ms), dtype=torch.float64, device=DEV)
        ctx.el_trace_rhs(d, ms, gs, b)
        meshes.append(ms); bs.append(b); ts.append(torch.empty_like(b))
    ops = [i2o[offs[i]:offs[i + 1]] for i in range(len(sides))]
    print(f"[batched full] one GMRES over 8 meshes, basis {basis}", flush=True)
    st, rep = ctx.el_trace_solve(d, meshes, ops, bs, ts, tol=1e-11, restart=50, max_iter=20000, basis=basis)
    print(f"[batched full] iterations {[r['iters'] for r in rep]}", flush=True)
    assert st == 0 and all(r["converged"] and r["relres"] <= 1e-11 for r in rep), rep
    rng = np.random.default_rng(5)
    sel = np.sort(rng.choice(E, 6, replace=False))
    ro, _, rm = local_solve_batch(o, H.cpu().numpy()[sel], K.cpu().numpy()[sel], S.cpu().numpy()[sel])
    assert per_element_rel(i2o[sel].cpu().numpy(), ro) <= 1e-10
    assert per_element_rel(i2m[sel].cpu().numpy(), rm) <= 1e-10
    for i, ((oms, hh, kap, _), ms) in enumerate(zip(probs, meshes)):
        mean = torch.empty((hh.size, nn), dtype=torch.float64, device=DEV)
        ctx.el_recover_mean(d, ms, i2m[offs[i]:offs[i + 1]], ts[i], mean)
        inc, outg = orecover.boundary_fluxes(o, oms, ts[i].cpu().numpy(), oms.inflow_mask(o))
        mn = mean.cpu().numpy()
        ab = float(np.sum((0.5 * hh)[:, None] ** 2 * o.w_ang.sum() * o.W[None, :] * kap * mn))
        assert abs(inc - outg - ab) <= 1e-9 * inc, (sides[i], inc, outg, ab)

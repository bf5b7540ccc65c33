"""GPU parity of el_local_solve (FP64 LU path) against the CPU oracle.

Bar: per-element max|gpu - oracle| / max|oracle| <= 1e-10 for in2out,
in2sol and in2mean (FP64 dense LU with partial pivoting on both sides; the
difference is rounding order, far below 1e-10 for these condition numbers).
"""
import numpy as np
import pytest
import torch

from oracle.local import LocalDisc, local_solve_batch
from paper_2308_02467_amd import inputs

from _util import per_element_rel, refinement_bounds

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02467_amd import el
    c = el.Context(0)
    yield c
    c.close()


def _gpu_local(ctx, p, n_a, g, h, kap, sig, outputs=("in2out", "in2sol", "in2mean"), precision=0, resid=None):
    from paper_2308_02467_amd import el
    d = el.disc(p, n_a, g)
    nn, n, m = el.disc_sizes(d)
    E = h.size
    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    out = {}
    if "in2out" in outputs:
        out["in2out"] = torch.full((E, m, m), float("nan"), dtype=torch.float64, device=dev)
    if "in2sol" in outputs:
        out["in2sol"] = torch.full((E, n, m), float("nan"), dtype=torch.float64, device=dev)
    if "in2mean" in outputs:
        out["in2mean"] = torch.full((E, nn, m), float("nan"), dtype=torch.float64, device=dev)
    print(f"[el_local_solve] p={p} n_a={n_a} g={g} E={E} precision={precision}", flush=True)
    rr = torch.full((E,), float("nan"), dtype=torch.float64, device=dev) if resid is not None else None
    ctx.el_local_solve(d, t(h), t(kap), t(sig), precision=precision, rel_resid=rr, **out)
    if resid is not None:
        resid.append(rr.cpu().numpy())
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check(p, n_a, g, h, kap, sig, gpu, tol=TOL):
    o = LocalDisc(p, n_a, g)
    i2o, i2s, i2m = local_solve_batch(o, h, kap, sig)
    ref = {"in2out": i2o, "in2sol": i2s, "in2mean": i2m}
    for k, v in gpu.items():
        assert np.all(np.isfinite(v)), k
        err = per_element_rel(v, ref[k])
        assert err <= tol, (k, err)


def test_c1_constant(ctx):
    """4x4 elements, p=3, N_a=8, kappa=1, sigma=2 (every element identical)."""
    o = LocalDisc(3, 8)
    X, Y = inputs.element_node_coords(4, 4, 0.25, o.xi)
    kap, sig = inputs.const_fields(X)
    h = np.full(16, 0.25)
    _check(3, 8, 0.0, h, kap, sig, _gpu_local(ctx, 3, 8, 0.0, h, kap, sig))


def test_p3_random_many(ctx):
    """p=3, N_a=8 with random coefficients over many elements (several per slot)."""
    o = LocalDisc(3, 8)
    h, kap, sig = inputs.training_draws(700, o.xi, seed=7)
    _check(3, 8, 0.0, h, kap, sig, _gpu_local(ctx, 3, 8, 0.0, h, kap, sig))


def test_p6_paper_degree(ctx):
    """p=6, N_a=16 (n=784, m=224): cloud elements and training-range draws,
    including optically very thin and thick elements."""
    o = LocalDisc(6, 16)
    X, Y = inputs.element_node_coords(32, 32, 1 / 32, o.xi)
    kap, sig = inputs.gaussian_cloud(X, Y)
    sel = np.array([0, 31, 200, 495, 528, 1023])
    h2, k2, s2 = inputs.training_draws(10, o.xi, seed=3)
    h = np.concatenate([np.full(sel.size, 1 / 32), h2, [1 / 256, 1 / 16]])
    kap = np.concatenate([kap[sel], k2, np.full((1, 49), 1e-3), np.full((1, 49), 3.0)])
    sig = np.concatenate([sig[sel], s2, np.full((1, 49), 1e-2), np.full((1, 49), 100.0)])
    _check(6, 16, 0.0, h, kap, sig, _gpu_local(ctx, 6, 16, 0.0, h, kap, sig))


@pytest.mark.parametrize("p,n_a,g", [(4, 4, 0.0), (2, 12, 0.85), (5, 8, 0.5)])
def test_ragged_and_hg(ctx, p, n_a, g):
    """n and m not multiples of 16 (padded tiles) and Henyey-Greenstein."""
    o = LocalDisc(p, n_a, g)
    h, kap, sig = inputs.training_draws(37, o.xi, seed=p * 100 + n_a)
    _check(p, n_a, g, h, kap, sig, _gpu_local(ctx, p, n_a, g, h, kap, sig))


def test_subset_outputs(ctx):
    """NULL outputs are skipped; the requested ones are unchanged."""
    o = LocalDisc(3, 8)
    h, kap, sig = inputs.training_draws(5, o.xi, seed=1)
    _check(3, 8, 0.0, h, kap, sig, _gpu_local(ctx, 3, 8, 0.0, h, kap, sig, outputs=("in2out",)))


def test_bad_inputs_name_the_element(ctx):
    from paper_2308_02467_amd import el
    o = LocalDisc(3, 8)
    h, kap, sig = inputs.training_draws(9, o.xi, seed=2)
    kap[4, 3] = np.nan
    with pytest.raises(el.ElError) as ei:
        _gpu_local(ctx, 3, 8, 0.0, h, kap, sig)
    assert ei.value.code == el.EL_ERR_NONFINITE and "element 4" in str(ei.value)
    kap[4, 3] = 0.1
    sig[6, 0] = -1.0
    with pytest.raises(el.ElError) as ei:
        _gpu_local(ctx, 3, 8, 0.0, h, kap, sig)
    assert ei.value.code == el.EL_ERR_NONFINITE and "element 6" in str(ei.value)
    sig[6, 0] = 1.0
    # finite coefficients whose reference-element values overflow FP32 (the
    # FP32 factorization meets an infinite entry and then NaN columns): the
    # pivot search finds no usable pivot and the element is reported singular
    sig[2, :] = 1e300
    with pytest.raises(el.ElError) as ei:
        _gpu_local(ctx, 3, 8, 0.0, h, kap, sig, precision=1)
    print(f"[local solve] {ei.value}", flush=True)
    assert ei.value.code == el.EL_ERR_SINGULAR and "element 2" in str(ei.value)
    with pytest.raises(ValueError):
        ctx.el_local_solve(el.disc(3, 8), torch.ones(2, dtype=torch.float64, device="cuda"),
                           torch.ones(5, dtype=torch.float64, device="cuda"),
                           torch.ones(32, dtype=torch.float64, device="cuda"))


# ---- FP32 LU + FP64 iterative refinement (precision form) ------------------------
# Bar: every element reaches a relative residual <= 1e-13 (max over columns of
# ||R||_inf / ||B_hat col||_inf, FP64), and its outputs agree with the FP64
# oracle within the bound that residual implies (||A^-1||_inf ||R||_inf plus
# the oracle's own rounding, per element, from tests/_util.refinement_bounds)
# and to 1e-9 per element.
def _check_ir(p, n_a, g, h, kap, sig, gpu, rr):
    o = LocalDisc(p, n_a, g)
    i2o, i2s, i2m = local_solve_batch(o, h, kap, sig)
    ref = {"in2out": i2o, "in2sol": i2s, "in2mean": i2m}
    bnd = refinement_bounds(o, h, kap, sig, rr, ref)
    for k, v in gpu.items():
        a = v.reshape(v.shape[0], -1)
        b = ref[k].reshape(v.shape[0], -1)
        err = np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)
        print(f"[fp32_ir] {k}: max err {err.max():.2e}, max err / bound {np.max(err / bnd[k]):.3f}, "
              f"largest bound {bnd[k].max():.2e}", flush=True)
        assert np.all(err <= bnd[k]), (k, err, bnd[k])
        assert err.max() <= 1e-9, k

@pytest.mark.parametrize("p,n_a,g,E", [(3, 8, 0.0, 300), (6, 16, 0.0, 24), (4, 4, 0.0, 37), (2, 12, 0.85, 37)])
def test_fp32_ir_parity(ctx, p, n_a, g, E):
    o = LocalDisc(p, n_a, g)
    h, kap, sig = inputs.training_draws(E, o.xi, seed=p * 7 + n_a)
    res = []
    gpu = _gpu_local(ctx, p, n_a, g, h, kap, sig, precision=1, resid=res)
    print(f"[fp32_ir] max rel residual {res[0].max():.2e}", flush=True)
    assert np.all(res[0] <= 1e-13), res[0].max()
    _check_ir(p, n_a, g, h, kap, sig, gpu, res[0])


def test_fp32_ir_na32_hg_paper_cloud_size(ctx):
    """The n = 1568 discretization of the realistic-cloud workload (p = 6,
    N_a = 32, Henyey-Greenstein g = 0.85): FP32 LU + FP64 refinement against
    the FP64 oracle element by element.  The FP64 factorization of this size
    does not fit one workgroup and is refused with a clear error."""
    from paper_2308_02467_amd import el
    p, n_a, g, E = 6, 32, 0.85, 5
    o = LocalDisc(p, n_a, g)
    h, kap, sig = inputs.training_draws(E, o.xi, seed=77)
    res = []
    gpu = _gpu_local(ctx, p, n_a, g, h, kap, sig, precision=1, resid=res)
    print(f"[fp32_ir n=1568] max rel residual {res[0].max():.2e}", flush=True)
    assert np.all(res[0] <= 1e-13), res[0].max()
    _check_ir(p, n_a, g, h, kap, sig, gpu, res[0])
    with pytest.raises(el.ElError) as exc:
        _gpu_local(ctx, p, n_a, g, h[:1], kap[:1], sig[:1], outputs=("in2out",), precision=0)
    assert "LDS" in str(exc.value) or "too large" in str(exc.value)

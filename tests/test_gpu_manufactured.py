"""Boundary data that varies along the boundary, and the whole HIP path on a
manufactured solution.

* el_trace_rhs_nodal: bit-exact against the oracle's boundary vector (b is a
  copy of g on the domain-inflow DOFs); equal to el_trace_rhs for data that
  is constant per side; a NaN on an inflow DOF is reported, one on an
  outflow DOF is not read.
* p-convergence (Sec. 2.2: the HDG discretization is spectrally accurate in
  p for a smooth solution): u*(x, y, theta) = (1 + 0.3 x y + 0.2 sin 2x)
  (1 + 0.2 cos theta) solves the discrete-ordinate equations with the
  source f = s . grad u* + sigma_e u* - sigma_s sum_k' Q[k][k'] u*_k' (Q the
  library's own angular table) and inflow data u*; local solve with the
  source, nodal right-hand side, source added, GMRES and recovery on the GPU
  must approach u* at the nodes by a factor of 20 per two degrees, to 1e-8
  at p = 8 (the same bar as the oracle's own manufactured-solution pin).
"""
import math

import numpy as np
import pytest
import torch

from oracle.local import LocalDisc
from oracle.mesh import Mesh
from paper_2308_02467_amd import inputs

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


def boundary_nodes(n_x, n_y, h, xi, x0=0.0, y0=0.0):
    """(x, y) [2 (n_x + n_y), q] of the boundary face nodes in the order of
    el_trace_rhs_nodal: W faces bottom to top, E, then S left to right, N."""
    t = 0.5 * (np.asarray(xi) + 1.0) * h
    xs, ys = [], []
    for x_side in (x0, x0 + n_x * h):
        for jr in range(n_y):
            xs.append(np.full_like(t, x_side))
            ys.append(y0 + jr * h + t)
    for y_side in (y0, y0 + n_y * h):
        for i in range(n_x):
            xs.append(x0 + i * h + t)
            ys.append(np.full_like(t, y_side))
    return np.array(xs), np.array(ys)


def g_of_index(x, y, k):
    return 1.0 + x - 0.5 * y * y + 0.1 * (k + 1)


@pytest.mark.parametrize("p,n_a,nx,ny", [(3, 8, 3, 2), (6, 16, 2, 4)])
def test_rhs_nodal_matches_oracle(ctx, p, n_a, nx, ny):
    from paper_2308_02467_amd import el
    d = el.disc(p, n_a)
    h = 1.0 / max(nx, ny)
    ms = el.mesh(nx, ny, h)
    xi, _ = el.lgl(p)
    bx, by = boundary_nodes(nx, ny, h, xi)
    g = np.stack([g_of_index(bx, by, k) for k in range(n_a)], axis=1)      # [faces, n_a, q]
    nt = el.trace_size(d, ms)
    b = torch.full((nt,), float("nan"), dtype=torch.float64, device=DEV)
    print(f"[el_trace_rhs_nodal] p={p} n_a={n_a} {nx}x{ny}", flush=True)
    ctx.el_trace_rhs_nodal(d, ms, T(g), b)
    od = LocalDisc(p, n_a)
    om = Mesh(nx, ny, h)
    # the ordinate index from its angle (k + 1/2) 2 pi / n_a
    ref = om.boundary_vector(od, lambda x, y, th: g_of_index(x, y, int(round(th * n_a / (2 * math.pi) - 0.5))))
    assert np.array_equal(b.cpu().numpy(), ref)
    # data constant per side: the same as the per-side entry point
    g_side = np.arange(4 * n_a, dtype=np.float64).reshape(4, n_a) * 0.25 + 1.0
    side_of_face = np.array([0] * ny + [1] * ny + [2] * nx + [3] * nx)
    gc = np.broadcast_to(g_side[side_of_face][:, :, None], g.shape).copy()
    b2 = torch.empty_like(b)
    ctx.el_trace_rhs_nodal(d, ms, T(gc), b)
    ctx.el_trace_rhs(d, ms, g_side, b2)
    assert torch.equal(b, b2)


def test_rhs_nodal_nonfinite_and_sizes(ctx):
    from paper_2308_02467_amd import el
    p, n_a, nx, ny = 2, 4, 2, 2
    d = el.disc(p, n_a)
    ms = el.mesh(nx, ny, 0.5)
    nt = el.trace_size(d, ms)
    s, _ = el.angular_tables(d)
    g = np.ones((2 * (nx + ny), n_a, p + 1))
    b = torch.empty(nt, dtype=torch.float64, device=DEV)
    # a W-side face (first block) is inflow for s_x > 0 and outflow otherwise
    k_out = int(np.argmax(s[:, 0] < 0))
    k_in = int(np.argmax(s[:, 0] > 0))
    g[0, k_out, 1] = np.nan
    ctx.el_trace_rhs_nodal(d, ms, T(g), b)
    assert torch.isfinite(b).all()
    g[0, k_in, 1] = np.nan
    with pytest.raises(el.ElError) as ei:
        ctx.el_trace_rhs_nodal(d, ms, T(g), b)
    print(f"[el_trace_rhs_nodal] {ei.value}", flush=True)
    assert ei.value.code == el.EL_ERR_NONFINITE
    with pytest.raises(ValueError):
        ctx.el_trace_rhs_nodal(d, ms, T(g[:-1]), b)


def manufactured_error(ctx, p, n_a=8, g_hg=0.5, n=2):
    from paper_2308_02467_amd import el
    d = el.disc(p, n_a, g_hg=g_hg)
    nn, nd, m = el.disc_sizes(d)
    h = 1.0 / n
    ms = el.mesh(n, n, h)
    E = n * n
    xi, _ = el.lgl(p)
    X, Y = inputs.element_node_coords(n, n, h, xi)                      # [E, nn]
    kap = 0.3 + 0.1 * np.cos(X + Y)
    sig = 2.0 + np.sin(2 * X) * np.cos(Y)
    s, Q = el.angular_tables(d)

    def amp(x, y):
        return 1 + 0.3 * x * y + 0.2 * np.sin(2 * x)

    ang = 1 + 0.2 * s[:, 0]                                              # 1 + 0.2 cos theta_k
    ustar = amp(X, Y)[:, None, :] * ang[None, :, None]                   # [E, n_a, nn]
    ax = 0.3 * Y + 0.4 * np.cos(2 * X)
    ay = 0.3 * X
    grad_s = (s[:, 0][None, :, None] * ax[:, None, :] + s[:, 1][None, :, None] * ay[:, None, :]) * \
        ang[None, :, None]
    scat = np.einsum("kj,ejn->ekn", Q, ustar)
    f = grad_s + (kap + sig)[:, None, :] * ustar - sig[:, None, :] * scat
    i2o = torch.empty((E, m, m), dtype=torch.float64, device=DEV)
    i2s = torch.empty((E, nd, m), dtype=torch.float64, device=DEV)
    fo = torch.empty((E, m), dtype=torch.float64, device=DEV)
    fs = torch.empty((E, nd), dtype=torch.float64, device=DEV)
    ctx.el_local_solve(d, T(np.full(E, h)), T(kap), T(sig), in2out=i2o, in2sol=i2s, src=T(f), src2out=fo,
                       src2sol=fs)
    bx, by = boundary_nodes(n, n, h, xi)
    gb = amp(bx, by)[:, None, :] * ang[None, :, None]                   # [faces, n_a, q]
    nt = el.trace_size(d, ms)
    b = torch.empty(nt, dtype=torch.float64, device=DEV)
    t = torch.zeros(nt, dtype=torch.float64, device=DEV)
    ctx.el_trace_rhs_nodal(d, ms, T(gb), b)
    ctx.el_trace_add_source(d, ms, fo, b)
    _, rep = ctx.el_trace_solve(d, [ms], [i2o], [b], [t], tol=1e-13, restart=60, max_iter=4000)
    assert rep[0]["converged"], rep
    u = torch.empty((E, nd), dtype=torch.float64, device=DEV)
    ctx.el_recover(d, ms, i2s, t, u=u, src2sol=fs)
    return float(np.abs(u.cpu().numpy() - ustar.reshape(E, nd)).max())


def test_manufactured_p_convergence(ctx):
    errs = []
    for p in (2, 4, 6, 8):
        print(f"[manufactured] p={p}", flush=True)
        errs.append(manufactured_error(ctx, p))
    print(f"[manufactured] max nodal errors {errs}", flush=True)
    assert all(errs[i + 1] < 0.05 * errs[i] for i in range(3)), errs
    assert errs[-1] < 1e-8, errs

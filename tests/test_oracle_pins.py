"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them re-types the oracle's formula:
they check closed forms, exact identities (discrete integration by parts,
conservation), invariances, brute force and sizes printed in the paper.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle.quadrature import lgl_nodes_weights, lagrange_diff_matrix, lagrange_eval
from oracle.angles import ordinates, phase_matrix
from oracle.local import LocalDisc, local_solve_batch
from oracle.mesh import Mesh
from oracle import trace, recover
from oracle.dg import solve_dg
from paper_2308_02467_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- P1: LGL quadrature and differentiation (closed forms) -------------------
def test_lgl_closed_forms():
    x, w = lgl_nodes_weights(1)
    assert np.allclose(x, [-1, 1]) and np.allclose(w, [1, 1])
    x, w = lgl_nodes_weights(2)
    assert np.allclose(x, [-1, 0, 1]) and np.allclose(w, [1 / 3, 4 / 3, 1 / 3])
    x, w = lgl_nodes_weights(3)
    r = 1 / math.sqrt(5)
    assert np.allclose(x, [-1, -r, r, 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    x, w = lgl_nodes_weights(4)
    r = math.sqrt(3 / 7)
    assert np.allclose(x, [-1, -r, 0, r, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 6, 8, 10])
def test_lgl_exactness(p):
    """LGL with p+1 points integrates monomials up to degree 2p-1 exactly."""
    x, w = lgl_nodes_weights(p)
    assert abs(w.sum() - 2.0) < 1e-14
    for deg in range(2 * p):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(w @ x ** deg - exact) < 1e-13, deg
    # degree 2p is NOT exact (guards against silently using Gauss points)
    exact = 2.0 / (2 * p + 1)
    assert abs(w @ x ** (2 * p) - exact) > 1e-6


@pytest.mark.parametrize("p", [2, 3, 6, 9])
def test_diff_matrix_closed_form(p):
    """Textbook LGL closed form D_ij = P_p(x_i) / (P_p(x_j)(x_i - x_j)),
    D_00 = -p(p+1)/4, D_pp = p(p+1)/4, else 0 on the diagonal."""
    x, _ = lgl_nodes_weights(p)
    D = lagrange_diff_matrix(x)
    Pp = np.polynomial.legendre.legval(x, [0] * p + [1])
    ref = np.zeros((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            if i != j:
                ref[i, j] = Pp[i] / (Pp[j] * (x[i] - x[j]))
    ref[0, 0] = -p * (p + 1) / 4
    ref[p, p] = p * (p + 1) / 4
    assert np.allclose(D, ref, atol=1e-11 * p * p)
    # exact on polynomials of degree <= p
    for deg in range(p + 1):
        d = deg * x ** (deg - 1) if deg else np.zeros_like(x)
        assert np.allclose(D @ x ** deg, d, atol=1e-11 * p * p)


def test_lagrange_eval_is_identity_at_nodes():
    x, _ = lgl_nodes_weights(5)
    assert np.allclose(lagrange_eval(x, x), np.eye(6), atol=1e-14)


# ---- angles / phase ----------------------------------------------------------
def test_ordinates_conformity():
    for n_a in (4, 8, 16, 28, 32):
        th, w, s = ordinates(n_a)
        assert abs(w.sum() - 2 * math.pi) < 1e-13
        assert np.all(np.abs(s) > 1e-3)          # none tangent to an axis face
    with pytest.raises(ValueError):
        ordinates(6)


@pytest.mark.parametrize("g", [0.0, 0.5, 0.85])
def test_phase_normalization_and_symmetry(g):
    n_a = 16
    P = phase_matrix(n_a, g)
    _, w, _ = ordinates(n_a)
    assert np.allclose(P @ w, 1.0, atol=1e-14)       # sum_k' w P = 1
    assert np.allclose(P, P.T, atol=1e-15)           # depends on the angle only
    if g > 0:                                        # forward peaked: max on the diagonal
        assert np.all(np.argmax(P, axis=1) == np.arange(n_a))
    else:
        assert np.allclose(P, 1 / (2 * math.pi))


@pytest.mark.parametrize("g", [0.5, 0.8, 0.85])
def test_hg_normalization_closed_form(g):
    """The HG constant of Sec. 2.1 on the circle, with the exponent 3/2:
    integral over [0, 2 pi) of (1 - g^2) / (1 + g^2 - 2 g cos t)^{3/2} dt
    = 4 E(k^2) / (1 - g) with k^2 = 4 g / (1 + g)^2 (complete elliptic
    integral of the second kind; the exponent 1 would give 2 pi instead).
    * ordinates: the periodic trapezoidal sum converges geometrically, at
      N_a = 256 to round-off;
    * P0 cells: summing the cell-pair averages over k' integrates the kernel
      over one full period for every x in the cell, so the discrete constant
      equals the integral at any N_a (here the paper's N_a = 28).
    Also the entries themselves at N_a = 256: P[k, k] -> (1 + g) / (4 (1 - g) E)
    and, opposite, P[k, k + N_a/2] -> (1 - g)^2 / ((1 + g)^2 4 E)."""
    from scipy.special import ellipe
    from oracle.angles import hg_normalization
    E2 = ellipe(4 * g / (1 + g) ** 2)
    c = 4 * E2 / (1 - g)
    assert abs(hg_normalization(256, g) - c) <= 1e-12 * c
    assert abs(hg_normalization(28, g, "p0") - c) <= 1e-11 * c
    P = phase_matrix(256, g)
    assert abs(P[0, 0] - (1 + g) / (4 * (1 - g) * E2)) <= 1e-12 * P[0, 0]
    assert abs(P[5, 5 + 128] - (1 - g) ** 2 / ((1 + g) ** 2 * 4 * E2)) <= 1e-12 * P[5, 5 + 128]


# ---- sizes printed in the paper ------------------------------------------------
def test_sizes_match_paper():
    """Sec. 2.4.1: A_i2o is 2(p_x+p_y+2)(N_a/2)(p_a+1) square, A_i2m is
    (p_x+1)(p_y+1) x that; the tables' DOF counts are n_elem (p+1)^2 N_a."""
    for p, n_a in [(3, 8), (6, 16), (6, 28), (4, 28)]:
        d = LocalDisc(p, n_a)
        assert d.m == 2 * (2 * p + 2) * (n_a // 2)
        assert d.nn == (p + 1) ** 2
        n_out = (2 * p + 2) * n_a * ((2 * p + 2) * n_a + (p + 1) ** 2)
        assert d.m * d.m + d.nn * d.m == n_out
    gold = json.load(open(os.path.join(GOLDEN, "paper_sizes.json")))
    for t in gold["tables"]:
        per = (t["p"] + 1) ** 2 * t["n_a"]
        if "rows" in t:
            for dofs, ne in t["rows"]:
                assert dofs == ne * per
        else:
            assert t["dofs_last_row"] == t["elements"] * per


# ---- P2: discrete integration by parts -----------------------------------------
@pytest.mark.parametrize("p,n_a", [(2, 4), (3, 8), (6, 16)])
def test_integration_by_parts(p, n_a):
    """(B + B_hat - C) 1 = 0 and C + C^T = (face mass with sign of s.n)."""
    d = LocalDisc(p, n_a)
    B, C, Bh = d.matrix_B(), d.matrix_C(), d.matrix_Bhat()
    r = B @ np.ones(d.n) + Bh @ np.ones(d.m) - C @ np.ones(d.n)
    assert np.abs(r).max() < 1e-13
    # summation by parts: C + C^T is diagonal = sum over faces of w_j (s.n_f)
    full = np.zeros(d.n)
    for k in range(n_a):
        for f in range(4):
            for j, nd in enumerate(d.face_nodes[f]):
                full[k * d.nn + nd] += d.omega[j] * d.sn[k, f]
    assert np.allclose(C + C.T, np.diag(full), atol=1e-13)


# ---- P3: conservation (kappa = 0 keeps constants) -------------------------------
@pytest.mark.parametrize("g", [0.0, 0.85])
def test_pure_scattering_preserves_constants(g):
    d = LocalDisc(4, 8, g)
    rng = np.random.default_rng(3)
    sigma = rng.uniform(0.1, 20.0, d.nn)
    i2o, i2s, i2m = d.local_solve(0.3, np.zeros(d.nn), sigma)
    assert np.abs(i2o.sum(axis=1) - 1).max() < 1e-12
    assert np.abs(i2s.sum(axis=1) - 1).max() < 1e-12
    assert np.abs(i2m.sum(axis=1) - 1).max() < 1e-12
    # absorption must lower the transmitted power (flux-weighted outflow)
    i2o_k, _, _ = d.local_solve(0.3, np.full(d.nn, 1.0), sigma)
    wout = np.array([d.w_ang[k] * d.omega[j] * d.sn[k, f] for (f, k, j, nd, r) in d.out_tab])
    win = np.array([-d.w_ang[k] * d.omega[j] * d.sn[k, f] for (f, k, j, nd, r) in d.in_tab])
    assert abs(wout @ i2o.sum(axis=1) - win.sum()) < 1e-12 * win.sum()
    assert wout @ i2o_k.sum(axis=1) < 0.99 * win.sum()


# ---- P4: Beer-Lambert closed form ----------------------------------------------
def test_beer_lambert_spectral():
    """sigma = 0: u_k(x) = exp(-kappa s_k . x) solves the transport equation;
    in2out applied to the exact inflow values must return the exact outflow
    values, with an error that decays spectrally in p.  With sigma = 0 in2out
    is block diagonal in the ordinate."""
    kappa, h = 3.0, 1.0          # reference element: tau = h kappa / 2
    errs = []
    for p in (2, 4, 6, 8, 10):
        d = LocalDisc(p, 8)
        i2o, i2s, _ = d.local_solve(h, np.full(d.nn, kappa), np.zeros(d.nn))
        xh = 0.5 * h * (d.xi + 1)                         # physical node coordinates
        X = np.tile(xh, d.q)
        Y = np.repeat(xh, d.q)

        def exact(k, nd):
            return math.exp(-kappa * (d.s[k, 0] * X[nd] + d.s[k, 1] * Y[nd]))
        tin = np.array([exact(k, nd) for (f, k, j, nd, r) in d.in_tab])
        tout = np.array([exact(k, nd) for (f, k, j, nd, r) in d.out_tab])
        errs.append(np.abs(i2o @ tin - tout).max())
        kin = np.array([t[1] for t in d.in_tab])
        kout = np.array([t[1] for t in d.out_tab])
        assert np.all(i2o[kout[:, None] != kin[None, :]] == 0.0)
    # measured decay: 2.6, 8e-2, 1.1e-3, 8e-6, 4e-8 (values up to e^3)
    assert errs[-1] < 1e-6
    assert all(errs[i + 1] < 0.05 * errs[i] for i in range(len(errs) - 1)), errs


# ---- P5: energy balance ---------------------------------------------------------
@pytest.mark.parametrize("g", [0.0, 0.85])
def test_element_energy_balance(g):
    d = LocalDisc(5, 12, g)
    rng = np.random.default_rng(11)
    kap = rng.uniform(0.0, 2.0, d.nn)
    sig = rng.uniform(0.0, 30.0, d.nn)
    h = 0.2
    _, i2s, _ = d.local_solve(h, kap, sig)
    for trial in range(3):
        tin = rng.uniform(0, 1, d.m)
        u = i2s @ tin
        res, scale = recover.element_energy_residual(d, h, kap, u, tin)
        assert abs(res) < 1e-12 * scale


def test_global_energy_balance_and_dg_2x2():
    """P5 globally and P8: HDG (sparse direct and GMRES 1e-12) == monolithic
    upwind DG on a 2x2 mesh."""
    d = LocalDisc(3, 8)
    mesh = Mesh(2, 2, 0.5)
    X, Y = inputs.element_node_coords(2, 2, 0.5, d.xi)
    kap, sig = inputs.gaussian_cloud(X, Y)
    hh = np.full(mesh.E, 0.5)
    i2o, i2s, _ = local_solve_batch(d, hh, kap, sig)
    ind, outd = mesh.element_dofs(d)
    gs = inputs.left_inflow(d.n_a)
    gs[3, :] = 0.5                                   # also some inflow from the top
    b = mesh.boundary_vector_sides(d, gs)
    t = trace.solve_direct(i2o, ind, outd, b)
    tg, it, rr = trace.gmres(lambda x: trace.matvec(i2o, ind, outd, x), b, 1e-12)
    assert rr <= 1e-12 and np.abs(tg - t).max() < 1e-11
    u = recover.recover(i2s, ind, t)
    udg = solve_dg(d, mesh, 0.5, kap, sig, b)
    assert np.abs(u - udg).max() < 1e-11 * np.abs(udg).max()
    inc, outg = recover.boundary_fluxes(d, mesh, t, mesh.inflow_mask(d))
    ab = recover.absorption(d, hh, kap, u)
    assert abs(inc - outg - ab) < 1e-12 * inc


@pytest.mark.slow
def test_dg_2x2_paper_degree():
    """P8 at p = 6, N_a = 16 (n_trace = 1344 on 2x2)."""
    d = LocalDisc(6, 16)
    mesh = Mesh(2, 2, 0.5)
    assert mesh.n_trace(d) == 1344
    X, Y = inputs.element_node_coords(2, 2, 0.5, d.xi)
    kap, sig = inputs.gaussian_cloud(X, Y)
    i2o, i2s, _ = local_solve_batch(d, np.full(4, 0.5), kap, sig)
    ind, outd = mesh.element_dofs(d)
    b = mesh.boundary_vector_sides(d, inputs.left_inflow(d.n_a))
    t = trace.solve_direct(i2o, ind, outd, b)
    u = recover.recover(i2s, ind, t)
    udg = solve_dg(d, mesh, 0.5, kap, sig, b)
    assert np.abs(u - udg).max() < 1e-10 * np.abs(udg).max()


# ---- P6: scaling invariance -----------------------------------------------------
def test_scaling_invariance():
    d = LocalDisc(3, 8)
    rng = np.random.default_rng(5)
    kap = rng.uniform(0.1, 2, d.nn)
    sig = rng.uniform(0.1, 5, d.nn)
    a = d.local_solve(0.1, kap, sig)
    b = d.local_solve(0.4, kap / 4, sig / 4)
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-14)


# ---- P7: mirror / rotation equivariance pins the indexing -------------------------
def _mirror_x(d):
    """Maps for x -> -x: ordinate k -> N_a/2 - 1 - k, node a -> p - a, W <-> E."""
    q, n_a = d.q, d.n_a
    kmap = np.array([(n_a // 2 - 1 - k) % n_a for k in range(n_a)])
    ndmap = np.array([(nd // q) * q + (d.p - nd % q) for nd in range(d.nn)])
    fmap = [1, 0, 2, 3]
    # face node j: W/E run along y (unchanged), S/N along x (reversed)
    jmap = [lambda j: j, lambda j: j, lambda j: d.p - j, lambda j: d.p - j]
    return kmap, ndmap, fmap, jmap


def _rot90(d):
    """Maps for rotation by +90 degrees: (x, y) -> (-y, x), k -> k + N_a/4."""
    q, n_a = d.q, d.n_a
    kmap = np.array([(k + n_a // 4) % n_a for k in range(n_a)])
    # node (a, b) at (x_a, x_b) -> (-x_b, x_a) = node (p - b, a)
    ndmap = np.array([(nd % q) * q + (d.p - nd // q) for nd in range(d.nn)])
    # W(-1,0)->S(0,-1), E->N, S(0,-1)->E(1,0), N->W
    fmap = [2, 3, 1, 0]
    # W face node j at (-1, x_j) -> (-x_j, -1) on S: index p - j
    # E (1, x_j) -> (-x_j, 1) on N: p - j; S (x_j, -1) -> (1, x_j) on E: j
    # N (x_j, 1) -> (-1, x_j) on W: j
    jmap = [lambda j: d.p - j, lambda j: d.p - j, lambda j: j, lambda j: j]
    return kmap, ndmap, fmap, jmap


@pytest.mark.parametrize("which", ["mirror", "rot90"])
def test_equivariance(which):
    d = LocalDisc(3, 8, 0.5)
    rng = np.random.default_rng(2)
    kap = rng.uniform(0.1, 2, d.nn)
    sig = rng.uniform(0.1, 5, d.nn)
    kmap, ndmap, fmap, jmap = (_mirror_x if which == "mirror" else _rot90)(d)
    # transformed coefficients: value at node nd moves to ndmap[nd]
    kap2 = np.empty_like(kap)
    sig2 = np.empty_like(sig)
    kap2[ndmap] = kap
    sig2[ndmap] = sig
    i2o, i2s, _ = d.local_solve(0.3, kap, sig)
    i2o2, i2s2, _ = d.local_solve(0.3, kap2, sig2)
    # index maps on the local inflow / outflow lists
    in_pos = {(f, k, j): i for i, (f, k, j, nd, r) in enumerate(d.in_tab)}
    out_pos = {(f, k, j): i for i, (f, k, j, nd, r) in enumerate(d.out_tab)}
    imap = np.array([in_pos[(fmap[f], kmap[k], jmap[f](j))] for (f, k, j, nd, r) in d.in_tab])
    omap = np.array([out_pos[(fmap[f], kmap[k], jmap[f](j))] for (f, k, j, nd, r) in d.out_tab])
    assert np.allclose(i2o2[np.ix_(omap, imap)], i2o, atol=1e-13)
    vmap = np.array([kmap[v // d.nn] * d.nn + ndmap[v % d.nn] for v in range(d.n)])
    assert np.allclose(i2s2[np.ix_(vmap, imap)], i2s, atol=1e-13)


# ---- P9: p-convergence with scattering (manufactured solution) -------------------
def _manufactured(p, n_a=8, g=0.5, n=2):
    """u*(x, y, theta) = (1 + 0.3 x y + 0.2 sin(2x)) (1 + 0.2 cos theta) solves the
    discrete-ordinate RTE with the source f = s.grad u* + sigma_e u* - sigma_s
    sum_k' w P u*; returns the max nodal error of the HDG solution with source."""
    d = LocalDisc(p, n_a, g)
    h = 1.0 / n
    mesh = Mesh(n, n, h)
    X, Y = inputs.element_node_coords(n, n, h, d.xi)
    kap = 0.3 + 0.1 * np.cos(X + Y)
    sig = 2.0 + np.sin(2 * X) * np.cos(Y)

    def ustar(x, y, th):
        return (1 + 0.3 * x * y + 0.2 * np.sin(2 * x)) * (1 + 0.2 * np.cos(th))

    def grad(x, y, th):
        a = (1 + 0.2 * np.cos(th))
        return (0.3 * y + 0.4 * np.cos(2 * x)) * a, 0.3 * x * a

    i2o, i2s, _ = local_solve_batch(d, np.full(mesh.E, h), kap, sig)
    ind, outd = mesh.element_dofs(d)
    b = mesh.boundary_vector(d, lambda x, y, th: ustar(x, y, th))
    rhs = b.copy()
    fus = []
    for e in range(mesh.E):
        us = np.array([ustar(X[e], Y[e], th) for th in d.theta])          # [n_a, nn]
        f = np.empty_like(us)
        for k in range(n_a):
            gx, gy = grad(X[e], Y[e], d.theta[k])
            scat = sum(d.w_ang[kp] * d.P[k, kp] * us[kp] for kp in range(n_a))
            f[k] = d.s[k, 0] * gx + d.s[k, 1] * gy + (kap[e] + sig[e]) * us[k] - sig[e] * scat
        fu, fhat = d.source_solve(h, kap[e], sig[e], f)
        fus.append(fu)
        rhs[outd[e]] += fhat
    t = trace.solve_direct(i2o, ind, outd, rhs)
    err = 0.0
    for e in range(mesh.E):
        u = i2s[e] @ t[ind[e]] + fus[e]
        us = np.array([ustar(X[e], Y[e], th) for th in d.theta]).reshape(-1)
        err = max(err, np.abs(u - us).max())
    return err


def test_p_convergence_manufactured():
    errs = [_manufactured(p) for p in (2, 4, 6, 8)]
    assert all(errs[i + 1] < 0.05 * errs[i] for i in range(3)), errs
    assert errs[-1] < 1e-8, errs


# ---- element L2 norm of the mean intensity (relative L2 error of Sec. 3.2.1) ----
@pytest.mark.parametrize("p,nx,ny", [(3, 4, 4), (6, 6, 3), (2, 5, 7)])
def test_l2_norm_closed_forms(p, nx, ny):
    """||1||^2 = area, ||x||^2 = int x^2 (exact with LGL for p >= 2), on
    meshes with E != nn so that a mis-broadcast of h fails."""
    d = LocalDisc(p, 4)
    h = 1.0 / max(nx, ny)
    X, Y = inputs.element_node_coords(nx, ny, h, d.xi)
    hh = np.full(nx * ny, h)
    area = nx * ny * h * h
    assert abs(recover.l2_norm_sq(d, hh, np.ones_like(X)) - area) < 1e-13
    Lx, Ly = nx * h, ny * h
    assert abs(recover.l2_norm_sq(d, hh, X) - Lx ** 3 / 3 * Ly) < 1e-13
    assert abs(recover.rel_l2(d, hh, 2 * X, X) - 1.0) < 1e-13

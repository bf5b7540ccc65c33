"""Shared helpers for the tests: build oracle references and device inputs."""
import numpy as np

from oracle.local import LocalDisc, local_solve_batch
from oracle.mesh import Mesh
from oracle import trace as otrace, recover as orecover
from paper_2308_02467_amd import inputs


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def per_element_rel(a, b):
    """max over elements of max|a_e - b_e| / max|b_e|."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return float(np.max(np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)))


def refinement_bounds(disc, h, kappa, sigma, rel_resid, refs):
    """Per-element bounds on max|x - x*| / max|out*| for a solution x of
    A X = -B_hat whose columns have FP64 residuals R_c with
    ||R_c||_inf <= rel_resid_e ||B_hat_c||_inf (the quantity el_local_solve
    reports for EL_FP32_IR): ||x_c - x*_c||_inf <= ||A^-1||_inf ||R_c||_inf,
    and in2out (rows of X) and in2mean (ordinate averages of X) change by no
    more than max|x - x*|.  Added: the oracle's own FP64 error, at most
    4 n u ||A||_inf ||A^-1||_inf max|x*| (u = 2^-53).  refs: {name: oracle
    output [E, ...]}; returns {name: bounds [E]}."""
    h = np.asarray(h, dtype=np.float64).reshape(-1)
    Bh = disc.matrix_Bhat()
    bmax = np.abs(Bh).max(axis=0).max()
    u = 2.0 ** -53
    out = {k: np.empty(h.size) for k in refs}
    for e in range(h.size):
        A = disc.local_matrix(*disc.scaled_coefficients(h[e], kappa[e], sigma[e]))
        Ainv = np.linalg.inv(A)
        ninv = np.abs(Ainv).sum(axis=1).max()
        kap_inf = np.abs(A).sum(axis=1).max() * ninv
        xmax = np.abs(Ainv @ Bh).max()
        dx = ninv * rel_resid[e] * bmax + 4 * disc.n * u * kap_inf * xmax
        for k, r in refs.items():
            out[k][e] = dx / np.abs(r[e]).max()
    return out


def mesh_problem(p, n_a, n_x, n_y=None, field="gauss", g=0.0, seed=0):
    """Coefficients of a workload on the unit square (uniform mesh)."""
    n_y = n_x if n_y is None else n_y
    h = 1.0 / max(n_x, n_y)
    d = LocalDisc(p, n_a, g)
    X, Y = inputs.element_node_coords(n_x, n_y, h, d.xi)
    if field == "gauss":
        kap, sig = inputs.gaussian_cloud(X, Y)
    elif field == "const":
        kap, sig = inputs.const_fields(X)
    elif field == "sharp":
        kap, sig = inputs.sharp_cloud(X, Y, seed)
    else:
        raise ValueError(field)
    return d, Mesh(n_x, n_y, h), np.full(n_x * n_y, h), kap, sig


def oracle_pipeline(d, mesh, hh, kap, sig, g_side):
    i2o, i2s, i2m = local_solve_batch(d, hh, kap, sig)
    ind, outd = mesh.element_dofs(d)
    b = mesh.boundary_vector_sides(d, g_side)
    t = otrace.solve_direct(i2o, ind, outd, b)
    u = orecover.recover(i2s, ind, t)
    mean = orecover.mean_intensity(d, u)
    return dict(in2out=i2o, in2sol=i2s, in2mean=i2m, b=b, t=t, u=u, mean=mean, in_dofs=ind, out_dofs=outd)

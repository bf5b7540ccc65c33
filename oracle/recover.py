"""Recovery and diagnostics.

* Alg. 1 step 4 / eq. hdg_local_mat_sol: u_K = A_i2u^K u_hat + f_u^K.
* eq. ang_ave: mean intensity u^m(x) = (1/|S|) int_S u ds, on the ordinates
  (1/N_a) sum_k u_k since all weights are 2 pi / N_a.
* Relative L2 error of the mean intensity (the error measure of Sec. 3.2.1),
  with the element L2 norm ||v||^2 = (h/2)^2 sum_nd W_nd v(nd)^2.
* Energy balance: testing the local equations with v = 1 and summing over
  ordinates with weights w_k removes the advection volume term (sum of the
  Lagrange basis is 1) and, by the discrete normalization of the phase
  matrix, leaves outflow flux - inflow flux + absorption = 0 per element.
"""
import numpy as np


def recover(in2sol, in_dofs, t):
    """u [E, n] = in2sol[e] @ t[in_dofs[e]]."""
    E = in2sol.shape[0]
    return np.einsum("enm,em->en", in2sol, t[in_dofs])


def mean_intensity(disc, u):
    """[E, nn] mean over ordinates of u [E, n]."""
    return u.reshape(u.shape[0], disc.n_a, disc.nn).mean(axis=1)


def l2_norm_sq(disc, h, v):
    """sum_e (h_e/2)^2 sum_nd W_nd v[e, nd]^2 for v [E, nn]."""
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), (v.shape[0],))
    return float(np.sum((0.5 * h) ** 2 * ((v * v) @ disc.W)))


def rel_l2(disc, h, v, ref):
    return np.sqrt(l2_norm_sq(disc, h, v - ref) / l2_norm_sq(disc, h, ref))


def element_energy_residual(disc, h, kappa, u, t_in):
    """Per element: outflow - inflow flux + absorption, in reference units.

    u [n] volume solution, t_in [m] inflow trace values (local inflow order).
    Returns (residual, scale) where scale is the sum of absolute terms.
    """
    w = disc.w_ang
    out = 0.0
    for (f, k, j, nd, row) in disc.out_tab:
        out += w[k] * disc.omega[j] * disc.sn[k, f] * u[row]
    inn = 0.0
    for iota, (f, k, j, nd, row) in enumerate(disc.in_tab):
        inn += w[k] * disc.omega[j] * (-disc.sn[k, f]) * t_in[iota]
    tau_a = 0.5 * h * np.asarray(kappa, dtype=np.float64)
    absorb = float(np.sum(w[:, None] * (disc.W * tau_a)[None, :] * u.reshape(disc.n_a, disc.nn)))
    return out - inn + absorb, abs(out) + abs(inn) + abs(absorb)


def boundary_fluxes(disc, mesh, t, inflow_mask):
    """(incoming, outgoing) radiative power through the domain boundary.

    Physical units: face integrals carry h/2, ordinate sums carry w_k.
    """
    inc = 0.0
    outg = 0.0
    for F in range(mesh.n_faces):
        _, _, nrm = mesh.face_geometry(disc, F)
        if nrm is None:
            continue
        for k in range(disc.n_a):
            sn = disc.s[k, 0] * nrm[0] + disc.s[k, 1] * nrm[1]
            base = mesh.trace_dof(disc, F, k, 0)
            val = disc.w_ang[k] * abs(sn) * 0.5 * mesh.h * float(disc.omega @ t[base:base + disc.q])
            if sn < 0:
                inc += val
            else:
                outg += val
    return inc, outg


def absorption(disc, h, kappa, u):
    """Total absorbed power sum_e (h/2)^2 sum_k w_k sum_nd W_nd kappa u."""
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), (u.shape[0],))
    uu = u.reshape(u.shape[0], disc.n_a, disc.nn)
    return float(np.sum((0.5 * h)[:, None, None] ** 2 * disc.w_ang[None, :, None]
                        * (disc.W[None, None, :] * kappa[:, None, :]) * uu))

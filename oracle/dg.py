"""Monolithic upwind DG (eq. dg, eq. dg_flux) on a small mesh, solved densely.

Used only as a brute-force cross-check of the hybridized path: the upwind
flux takes the neighbour's volume value on inflow faces (or g on the domain
boundary).  With conforming LGL face nodes the neighbour value at face node j
is the neighbour's volume DOF at the matching node, so the DG system is the
block system A_e u_e + B_hat_e u_hat_e = 0 with u_hat_e gathered from the
neighbours' u.  Its solution must equal the HDG solution recovered from the
skeleton solve (Sec. 2.2.2: HDG with the upwind choice reproduces DG).
"""
import numpy as np


def solve_dg(disc, mesh, h, kappa, sigma, b_trace):
    """Return u [E, n] of the monolithic upwind DG system.

    b_trace [n_trace]: boundary data on domain-inflow DOFs (as from
    Mesh.boundary_vector); other entries ignored.
    """
    E, n, m = mesh.E, disc.n, disc.m
    inflow = mesh.inflow_mask(disc)
    in_dofs, out_dofs = mesh.element_dofs(disc)
    owner = {}                          # trace DOF -> (element, volume row)
    for e in range(E):
        for o, (f, k, j, nd, row) in enumerate(disc.out_tab):
            owner[int(out_dofs[e, o])] = (e, row)
    Bh = disc.matrix_Bhat()
    big = np.zeros((E * n, E * n))
    rhs = np.zeros(E * n)
    for e in range(E):
        tau_e, tau_s = disc.scaled_coefficients(h, kappa[e], sigma[e])
        big[e * n:(e + 1) * n, e * n:(e + 1) * n] = disc.local_matrix(tau_e, tau_s)
        for iota in range(m):
            dof = int(in_dofs[e, iota])
            col = Bh[:, iota]
            if inflow[dof]:
                rhs[e * n:(e + 1) * n] -= col * b_trace[dof]
            else:
                e2, row2 = owner[dof]
                big[e * n:(e + 1) * n, e2 * n + row2] += col
    return np.linalg.solve(big, rhs).reshape(E, n)

"""Angular discretization on the unit circle and the scattering phase matrix.

Sec. 2.4.1 takes S to be the unit circle, directions s = (cos t, sin t) with a
uniform partition of [0, 2 pi) into N_a angular elements.  The discrete
ordinates used here sit at the centres of those uniform cells,
t_k = (k + 1/2) 2 pi / N_a, with equal weights w_k = 2 pi / N_a.  Requiring
N_a % 4 == 0 makes every ordinate strictly inflow or strictly outflow on each
face of a square element (the conformity rule of Sec. 2.2.1): no ordinate is
tangent to an axis-aligned face.

Phase function (Sec. 2.1): Henyey-Greenstein
    p(s, s') = (1 - g^2) / (c (1 + g^2 - 2 g cos ang(s, s'))^{3/2}),
with c fixed by the normalization "integral of p over S equals 1".  On the
discrete ordinates the normalization is imposed discretely,
sum_k' w_k' P[k, k'] = 1 for every k, so discrete scattering conserves energy
exactly.  g = 0 gives isotropic scattering, P = 1 / (2 pi).

P0 angular elements (Sec. 2.4.1: piecewise-constant functions on the same
uniform cells) give the same algebra with cell averages: the streaming
direction of cell k is the average of s over the cell (written out with the
antiderivatives of cos and sin), and the scattering kernel between cells k
and k' is the average of p over the pair of cells (an adaptive double
integral).
"""
import numpy as np


def ordinates(n_a, angular="ordinates"):
    """Return (theta, w, s): cell-centre angles, weights and directions
    [n_a, 2]; with angular == "p0" the directions are the cell averages of s."""
    if n_a < 4 or n_a % 4 != 0:
        raise ValueError("N_a must be a positive multiple of 4")
    dth = 2.0 * np.pi / n_a
    theta = (np.arange(n_a) + 0.5) * dth
    w = np.full(n_a, dth)
    if angular == "ordinates":
        s = np.stack([np.cos(theta), np.sin(theta)], axis=1)
    elif angular == "p0":
        a, b = np.arange(n_a) * dth, (np.arange(n_a) + 1) * dth
        s = np.stack([(np.sin(b) - np.sin(a)) / dth, (np.cos(a) - np.cos(b)) / dth], axis=1)
    else:
        raise ValueError("angular must be 'ordinates' or 'p0'")
    return theta, w, s


def _hg_kernel(n_a, g, angular):
    """Unnormalized Henyey-Greenstein kernel between ordinates (or the cell-pair
    averages for P0 cells), exponent 3/2 as in Sec. 2.1."""
    theta, _, _ = ordinates(n_a)
    hg = lambda ang: (1.0 - g * g) / (1.0 + g * g - 2.0 * g * np.cos(ang)) ** 1.5
    if angular == "ordinates":
        return hg(theta[:, None] - theta[None, :])
    if angular == "p0":
        # average over pairs of cells: the kernel depends on k - k' only
        from scipy.integrate import dblquad
        dth = 2.0 * np.pi / n_a
        q = np.array([dblquad(lambda y, x: hg(dd * dth + x - y), 0.0, dth, 0.0, dth,
                              epsabs=1e-15, epsrel=1e-13)[0] / dth ** 2 for dd in range(n_a)])
        k = np.arange(n_a)
        return q[(k[:, None] - k[None, :]) % n_a]
    raise ValueError("angular must be 'ordinates' or 'p0'")


def hg_normalization(n_a, g, angular="ordinates"):
    """The constant c of Sec. 2.1 as fixed discretely: the row sum
    sum_k' w_k' (unnormalized kernel)[k, k'] (equal for every row: the kernel
    is circulant)."""
    if not (0.0 < g < 1.0):
        raise ValueError("HG asymmetry must be in (0, 1)")
    _, w, _ = ordinates(n_a)
    return float((_hg_kernel(n_a, g, angular) @ w)[0])


def phase_matrix(n_a, g=0.0, angular="ordinates"):
    """P[k, k'] on the ordinates; rows satisfy sum_k' w_k' P[k, k'] = 1.

    g == 0 is the isotropic case 1/(2 pi) (which satisfies the discrete
    normalization exactly); otherwise the Henyey-Greenstein kernel with the
    paper's exponent 3/2, normalized discretely.
    """
    if g == 0.0:
        ordinates(n_a)
        return np.full((n_a, n_a), 1.0 / (2.0 * np.pi))
    if not (0.0 <= g < 1.0):
        raise ValueError("HG asymmetry must be in [0, 1)")
    if angular not in ("ordinates", "p0"):
        raise ValueError("angular must be 'ordinates' or 'p0'")
    _, w, _ = ordinates(n_a)
    raw = _hg_kernel(n_a, g, angular)
    c = raw @ w                      # row integrals; equal for all rows (circulant)
    return raw / c[:, None]

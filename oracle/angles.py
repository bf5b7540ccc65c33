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
"""
import numpy as np


def ordinates(n_a):
    """Return (theta, w, s): angles, weights and unit directions [n_a, 2]."""
    if n_a < 4 or n_a % 4 != 0:
        raise ValueError("N_a must be a positive multiple of 4")
    theta = (np.arange(n_a) + 0.5) * (2.0 * np.pi / n_a)
    w = np.full(n_a, 2.0 * np.pi / n_a)
    s = np.stack([np.cos(theta), np.sin(theta)], axis=1)
    return theta, w, s


def phase_matrix(n_a, g=0.0):
    """P[k, k'] on the ordinates; rows satisfy sum_k' w_k' P[k, k'] = 1.

    g == 0 is the isotropic case 1/(2 pi) (which satisfies the discrete
    normalization exactly); otherwise the Henyey-Greenstein kernel with the
    paper's exponent 3/2, normalized discretely.
    """
    theta, w, _ = ordinates(n_a)
    if g == 0.0:
        return np.full((n_a, n_a), 1.0 / (2.0 * np.pi))
    if not (0.0 <= g < 1.0):
        raise ValueError("HG asymmetry must be in [0, 1)")
    cosang = np.cos(theta[:, None] - theta[None, :])
    raw = (1.0 - g * g) / (1.0 + g * g - 2.0 * g * cosang) ** 1.5
    c = raw @ w                      # row integrals; equal for all rows (circulant)
    return raw / c[:, None]

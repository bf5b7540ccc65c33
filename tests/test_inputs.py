"""Properties of the seeded input generators (CPU)."""
import numpy as np

from oracle.quadrature import lgl_nodes_weights
from paper_2308_02467_amd import inputs


def test_legendre_smooth_draws_properties():
    """Fields of the paper's generator (Alg. 2): minimum exactly 0, maximum
    in [0, A_sigma], and every field a polynomial of degree <= p in each of
    x and y (a tensor Legendre least-squares fit reproduces it); a larger
    c_sm damps the highest mode's share."""
    p = 6
    xi, _ = lgl_nodes_weights(p)
    q = p + 1
    s = inputs.legendre_smooth_draws(200, xi, seed=3, a_sigma=10.0, c_sm=2.0)
    assert s.shape == (200, q * q)
    assert np.all(s.min(axis=1) == 0.0)
    assert np.all(s.max(axis=1) <= 10.0) and np.all(s.max(axis=1) >= 0.0)
    V1 = np.polynomial.legendre.legvander(xi, p)                 # [node, degree]
    V = np.kron(V1, V1)                                           # node b*q + a -> (L_n(xi_b) L_m(xi_a))
    coef, *_ = np.linalg.lstsq(V, s.T, rcond=None)
    assert np.abs(V @ coef - s.T).max() < 1e-10 * max(1.0, s.max())
    top = lambda c: np.abs(c.reshape(q, q, -1)[p, p]).mean() / np.abs(c).mean()
    s_smooth = inputs.legendre_smooth_draws(200, xi, seed=3, a_sigma=10.0, c_sm=6.0)
    c2, *_ = np.linalg.lstsq(V, s_smooth.T, rcond=None)
    assert top(c2) < top(coef)

"""Legendre-Gauss-Lobatto (LGL) nodes, weights and the nodal differentiation
matrix on [-1, 1].

The paper represents coefficients nodally on the tensor LGL points of a Q_p
spectral element (Sec. 2.4.1, eq. sigma_se) and uses the same points as
quadrature points of the element (Fig. 4 caption).  Here:

* nodes  x_0 = -1 < x_1 < ... < x_p = 1, the interior ones being the roots of
  P_p' (derivative of the Legendre polynomial of degree p);
* weights w_i = 2 / (p (p+1) P_p(x_i)^2);
* D[i, j] = l_j'(x_i), the derivative of the j-th Lagrange basis polynomial at
  node i, computed from the barycentric form of the Lagrange basis (the plain
  definition; the textbook closed form is the pin in the tests).
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def lgl_nodes_weights(p):
    """Return (x, w): the p+1 LGL nodes (ascending) and weights on [-1, 1]."""
    if p < 1:
        raise ValueError("LGL needs p >= 1")
    cp = np.zeros(p + 1)
    cp[p] = 1.0                      # P_p in the Legendre basis
    dcp = npleg.legder(cp)           # P_p'
    ddcp = npleg.legder(dcp)         # P_p''
    if p >= 2:
        r = np.sort(np.real(npleg.legroots(dcp)))
        for _ in range(3):           # Newton polish of the roots of P_p'
            r = r - npleg.legval(r, dcp) / npleg.legval(r, ddcp)
        x = np.concatenate(([-1.0], r, [1.0]))
    else:
        x = np.array([-1.0, 1.0])
    pv = npleg.legval(x, cp)
    w = 2.0 / (p * (p + 1) * pv * pv)
    return x, w


def lagrange_diff_matrix(x):
    """D[i, j] = l_j'(x_i) for the Lagrange basis on nodes x (barycentric form).

    l_j'(x_i) = (lam_j / lam_i) / (x_i - x_j) for i != j, with barycentric
    weights lam_j = 1 / prod_{k != j}(x_j - x_k); the diagonal follows from
    sum_j l_j = 1, so every row of D sums to zero.
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    lam = np.empty(n)
    for j in range(n):
        prod = 1.0
        for k in range(n):
            if k != j:
                prod *= x[j] - x[k]
        lam[j] = 1.0 / prod
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D


def lagrange_eval(x_nodes, t):
    """Matrix Lm[q, j] = l_j(t_q): Lagrange basis on x_nodes evaluated at t."""
    x_nodes = np.asarray(x_nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = x_nodes.size
    Lm = np.ones((t.size, n))
    for j in range(n):
        for k in range(n):
            if k != j:
                Lm[:, j] *= (t - x_nodes[k]) / (x_nodes[j] - x_nodes[k])
    return Lm

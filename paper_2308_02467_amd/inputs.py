"""Seeded synthetic inputs (coefficient fields, boundary data, training draws).

This module holds no arithmetic of the method: it only evaluates prescribed
fields at given node coordinates and draws seeded random numbers.  Both the
HIP path (tests, bench) and the CPU oracle consume what it produces.  Node
coordinates are passed in (the 1-D LGL points ``xi`` come from whichever side
is being fed), so the generators do not depend on either implementation.

Workloads (all on the unit square unless stated otherwise):

* ``const_fields``   kappa, sigma constant (kappa = 1, sigma = 2 for the 4x4,
                     p = 3, N_a = 8 case).
* ``gaussian_cloud`` smooth idealized cloud: G = exp(-|x - c|^2 / (2 w^2)),
                     c = (1/2, 1/2), w = 0.2; kappa = 0.01 + 0.5 G,
                     sigma = 0.1 + 30 G.  Stands in for the paper's test 1
                     case 1 (two smooth round scatterers in [0,3]x[0,2]).
* ``sharp_cloud``    sharp-edged cloud sigma = 0.1 + 50 (1 + tanh((0.3-r)/0.01))/2,
                     r = |x - c_i|, c_i ~ U[0.3, 0.7]^2 from default_rng(i);
                     kappa = 0.05 sigma + 0.01.  Stands in for test 1 case 2.
* ``lognormal_cloud``  log-normal field with a k^(-5/3) energy spectrum
                     (Fourier amplitudes ~ |k|^(-4/3), random phases,
                     default_rng(seed)) on a periodic grid, mean 10,
                     log-std 1, masked to 0 where the Gaussian field is
                     negative; kappa = 0.05 sigma + 0.01.  Stands in for the
                     I3RC cloud of test 2, which is not available here.
* ``training_draws`` element samples for the network: h log-uniform on
                     [1/256, 1/16]; log10 sigma = mu + delta, mu ~ U[-2, 2],
                     delta a Gaussian field with squared-exponential
                     covariance (length 0.5 h, std 0.25 dex), clipped to
                     [-2, 2]; log10 kappa likewise with mu ~ U[-3, 0.5].
* ``left_inflow``    boundary radiance 1 entering through the left side
                     (ordinates with s_x > 0), 0 elsewhere.
"""
import numpy as np


def element_node_coords(n_x, n_y, h, xi, x0=0.0, y0=0.0):
    """X, Y [E, q*q] at the tensor nodes; element e = j n_x + i, node b q + a."""
    xi = np.asarray(xi, dtype=np.float64)
    q = xi.size
    t = 0.5 * (xi + 1.0) * h
    i = np.arange(n_x)
    j = np.arange(n_y)
    ex = (x0 + i * h)[None, :].repeat(n_y, 0).reshape(-1)     # [E]
    ey = (y0 + j * h)[:, None].repeat(n_x, 1).reshape(-1)
    ta = np.tile(t, q)            # a fastest
    tb = np.repeat(t, q)
    return ex[:, None] + ta[None, :], ey[:, None] + tb[None, :]


def const_fields(X, kappa=1.0, sigma=2.0):
    return np.full(X.shape, float(kappa)), np.full(X.shape, float(sigma))


def gaussian_cloud(X, Y, cx=0.5, cy=0.5, width=0.2):
    G = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * width * width))
    return 0.01 + 0.5 * G, 0.1 + 30.0 * G


def sharp_cloud(X, Y, seed):
    c = np.random.default_rng(seed).uniform(0.3, 0.7, size=2)
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2)
    sigma = 0.1 + 50.0 * (1.0 + np.tanh((0.3 - r) / 0.01)) / 2.0
    return 0.05 * sigma + 0.01, sigma


def _periodic_field(n_grid, seed):
    """Unit-variance Gaussian field on a periodic n_grid^2 grid, E(k) ~ k^-5/3."""
    rng = np.random.default_rng(seed)
    k = np.fft.fftfreq(n_grid) * n_grid
    kx, ky = np.meshgrid(k, k, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros_like(kk)
    amp[kk > 0] = kk[kk > 0] ** (-4.0 / 3.0)
    phase = np.exp(2j * np.pi * rng.random(kk.shape))
    G = np.real(np.fft.ifft2(amp * phase))
    G -= G.mean()
    G /= G.std()
    return G


def lognormal_cloud(X, Y, seed=2024, n_grid=2048, mean=10.0, log_std=1.0):
    G = _periodic_field(n_grid, seed)
    # bilinear sampling on the periodic grid covering [0, 1)^2
    gx = (np.mod(X, 1.0) * n_grid)
    gy = (np.mod(Y, 1.0) * n_grid)
    i0 = np.floor(gx).astype(np.int64) % n_grid
    j0 = np.floor(gy).astype(np.int64) % n_grid
    fx = gx - np.floor(gx)
    fy = gy - np.floor(gy)
    i1 = (i0 + 1) % n_grid
    j1 = (j0 + 1) % n_grid
    g = (G[i0, j0] * (1 - fx) * (1 - fy) + G[i1, j0] * fx * (1 - fy)
         + G[i0, j1] * (1 - fx) * fy + G[i1, j1] * fx * fy)
    mu = np.log(mean) - 0.5 * log_std * log_std
    sigma = np.where(g < 0.0, 0.0, np.exp(mu + log_std * g))
    return 0.05 * sigma + 0.01, sigma


def training_draws(n, xi, seed=1234, log_sigma=(-2.0, 2.0), log_kappa=(-3.0, 0.5),
                   h_range=(1.0 / 256, 1.0 / 16), corr_len=0.5, dex_std=0.25):
    """n element samples: h [n], kappa [n, q*q], sigma [n, q*q]."""
    xi = np.asarray(xi, dtype=np.float64)
    q = xi.size
    rng = np.random.default_rng(seed)
    h = np.exp(rng.uniform(np.log(h_range[0]), np.log(h_range[1]), size=n))
    # node positions in units of h: (xi + 1)/2; correlation length corr_len * h
    ta = np.tile(0.5 * (xi + 1.0), q)
    tb = np.repeat(0.5 * (xi + 1.0), q)
    d2 = (ta[:, None] - ta[None, :]) ** 2 + (tb[:, None] - tb[None, :]) ** 2
    cov = dex_std ** 2 * np.exp(-d2 / (2.0 * corr_len ** 2)) + 1e-10 * np.eye(q * q)
    Lc = np.linalg.cholesky(cov)

    def field(lo, hi):
        mu = rng.uniform(lo, hi, size=(n, 1))
        delta = rng.standard_normal((n, q * q)) @ Lc.T
        return 10.0 ** np.clip(mu + delta, lo, hi)

    sigma = field(*log_sigma)
    kappa = field(*log_kappa)
    return h, kappa, sigma


def legendre_smooth_draws(n, xi, seed=1234, a_sigma=10.0, c_sm=2.0):
    """n reference-element scattering fields sigma [n, q*q] following the
    paper's optical-coefficient generator (Sec. 2.4.2, Alg. 2): modal
    Legendre coefficients exp(-c_sm ((m/p)^2 + (n/p)^2)) (X_mn - 1/2) with
    X_mn ~ U[0, 1] (the printed minus between the two squares is read as a
    plus, so that both directions are damped), mapped to the nodes xi x xi,
    shifted to a zero minimum, scaled to a unit maximum and multiplied by a
    U[0, a_sigma] amplitude.  Node nd = b q + a is (xi_a, xi_b)."""
    xi = np.asarray(xi, dtype=np.float64)
    q = xi.size
    p = q - 1
    rng = np.random.default_rng(seed)
    L = np.stack([np.polynomial.legendre.legval(xi, np.eye(q)[k]) for k in range(q)])   # L[k][i] = L_k(xi_i)
    kk = np.arange(q) / p
    damp = np.exp(-c_sm * (kk[:, None] ** 2 + kk[None, :] ** 2))                    # [m (x), n (y)]
    coef = damp[None] * (rng.uniform(0.0, 1.0, size=(n, q, q)) - 0.5)
    # sigma(xi_a, xi_b) = sum_mn coef_mn L_m(xi_a) L_n(xi_b)
    nodal = np.einsum("emn,ma,nb->eba", coef, L, L).reshape(n, q * q)
    nodal -= nodal.min(axis=1, keepdims=True)
    nodal /= np.maximum(nodal.max(axis=1, keepdims=True), 1e-300)
    return nodal * rng.uniform(0.0, a_sigma, size=(n, 1))


def left_inflow(n_a):
    """Per-side boundary radiance g_side [4, n_a] (sides W, E, S, N).

    Radiance 1 enters through the left (W) side for every ordinate; only
    ordinates entering the domain are read by the solvers, i.e. those with
    s_x > 0 on the left side.  The other sides carry 0.
    """
    g = np.zeros((4, n_a))
    g[0, :] = 1.0
    return g

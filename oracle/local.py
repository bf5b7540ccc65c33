"""Local HDG problem on one square element: matrices B, B_hat, C, M, S and the
in2out / in2sol / in2mean operators.

Follows Sec. 2.2.3 (eq. hdg_local_mat, eq. hdg_local_all_sub_mat,
eq. hdg_local_f2u_i2u, eq. hdg_local_f2o_i2o), App. A, and the reference
element scaling of Sec. 2.4.1 (a square of side h is the reference square
[-1, 1]^2 with coefficients h sigma_e / 2, h sigma_s / 2 and source h f / 2).

Discretization (Q_p tensor LGL collocation in space, discrete ordinates in
angle; every row of the angular Galerkin system is divided by the common
angular weight w_k):

  * rows are test functions (k, i), columns trial functions (k', j);
  * node index nd = b (p+1) + a for the node (x_a, x_b); volume DOF
    v = k (p+1)^2 + nd (direction-major);
  * faces f = 0 W (normal (-1,0)), 1 E (+1,0), 2 S (0,-1), 3 N (0,+1);
    face node j runs along increasing x or y: W (0, j), E (p, j),
    S (j, 0), N (j, p);
  * I_f (O_f) = ascending list of ordinates with s_k . n_f < 0 (> 0);
    local inflow index  iota = f (N_a/2)(p+1) + r (p+1) + j, r = rank of k
    in I_f; local outflow indices use the same formula with O_f.

Matrix entries (W_nd = w_a w_b is the tensor LGL weight):

  C[(k,(a,b)), (k,(c,d))] = w_c w_d (s_x D[c,a] delta_db + s_y D[d,b] delta_ca)
                             (integral of u s . grad v, collocated)
  M = diag(W_nd tau_e(nd))
  S[(k,nd), (k',nd)]      = W_nd tau_s(nd) P[k,k'] w_k'
  B[(k,nd), (k,nd)]       = sum over faces f containing nd with s_k.n_f > 0
                             of w_j (s_k . n_f)
  B_hat[(k,nd), iota]     = w_j (s_k . n_f)  for iota = (f, k, j), nd = node
                             j of face f (s_k . n_f < 0)

  A = B - C + M - S,  in2sol = A_i2u = -A^{-1} B_hat,
  in2out = A_i2o = R^o A_i2u (rows at the outflow DOFs, in outflow order),
  in2mean = A_i2m = R_u2m A_i2u, (R_u2m u)(nd) = (1/N_a) sum_k u(k, nd),
  f_u = A^{-1} [f], [f]_(k,nd) = W_nd (h/2) f(x_nd, theta_k).
"""
import numpy as np

from .quadrature import lgl_nodes_weights, lagrange_diff_matrix
from .angles import ordinates, phase_matrix

FACE_NORMALS = np.array([[-1.0, 0.0], [1.0, 0.0], [0.0, -1.0], [0.0, 1.0]])


class LocalDisc:
    """Discretization data of one element type: Q_p in space, N_a angular
    cells (discrete ordinates at the centres, or P0 elements: angular ==
    "p0")."""

    def __init__(self, p, n_a, g=0.0, angular="ordinates"):
        if p < 1:
            raise ValueError("p must be >= 1")
        self.p, self.n_a, self.g = int(p), int(n_a), float(g)
        self.angular = angular
        self.q = self.p + 1
        self.xi, self.omega = lgl_nodes_weights(self.p)
        self.D = lagrange_diff_matrix(self.xi)
        self.theta, self.w_ang, self.s = ordinates(self.n_a, angular)
        self.P = phase_matrix(self.n_a, self.g, angular)
        q = self.q
        self.nn = q * q
        self.n = self.nn * self.n_a
        self.m = 2 * q * self.n_a
        # tensor weights W[nd], nd = b q + a
        self.W = np.array([self.omega[a] * self.omega[b]
                           for b in range(q) for a in range(q)])
        # face node lists: face_nodes[f][j] = nd
        self.face_nodes = [
            [j * q + 0 for j in range(q)],          # W: a = 0, b = j
            [j * q + self.p for j in range(q)],     # E: a = p, b = j
            [0 * q + j for j in range(q)],          # S: b = 0, a = j
            [self.p * q + j for j in range(q)],     # N: b = p, a = j
        ]
        sn = self.s @ FACE_NORMALS.T                 # [n_a, 4] = s_k . n_f
        self.sn = sn
        if np.any(np.abs(sn) < 1e-12):
            raise ValueError("an ordinate is tangent to a face")
        self.I_f = [[k for k in range(self.n_a) if sn[k, f] < 0] for f in range(4)]
        self.O_f = [[k for k in range(self.n_a) if sn[k, f] > 0] for f in range(4)]
        half = self.n_a // 2
        for f in range(4):
            assert len(self.I_f[f]) == half and len(self.O_f[f]) == half
        # index tables: each entry (f, k, j, nd, volume row)
        self.in_tab = []
        self.out_tab = []
        for f in range(4):
            for r in range(half):
                for j in range(q):
                    nd = self.face_nodes[f][j]
                    k = self.I_f[f][r]
                    self.in_tab.append((f, k, j, nd, k * self.nn + nd))
            for r in range(half):
                for j in range(q):
                    nd = self.face_nodes[f][j]
                    k = self.O_f[f][r]
                    self.out_tab.append((f, k, j, nd, k * self.nn + nd))
        self.in_rows = np.array([t[4] for t in self.in_tab], dtype=np.int64)
        self.out_rows = np.array([t[4] for t in self.out_tab], dtype=np.int64)
        self._transport = [self._transport_block(k) for k in range(self.n_a)]

    # -- matrices (eq. hdg_local_all_sub_mat) ---------------------------------
    def _transport_block(self, k):
        """B_k - C_k for direction k (the tau-independent part)."""
        q, p, om, D = self.q, self.p, self.omega, self.D
        sx, sy = self.s[k]
        T = np.zeros((self.nn, self.nn))
        for b in range(q):
            for a in range(q):
                i = b * q + a
                for c in range(q):              # x-derivative term, trial (c, b)
                    T[i, b * q + c] -= om[c] * om[b] * sx * D[c, a]
                for d in range(q):              # y-derivative term, trial (a, d)
                    T[i, d * q + a] -= om[a] * om[d] * sy * D[d, b]
        for f in range(4):                       # outflow face mass B
            snf = self.sn[k, f]
            if snf > 0:
                for j, nd in enumerate(self.face_nodes[f]):
                    T[nd, nd] += om[j] * snf
        return T

    def matrix_C(self):
        """C alone (block diagonal over directions); for the pins."""
        q, om, D = self.q, self.omega, self.D
        C = np.zeros((self.n, self.n))
        for k in range(self.n_a):
            sx, sy = self.s[k]
            o = k * self.nn
            for b in range(q):
                for a in range(q):
                    i = b * q + a
                    for c in range(q):
                        C[o + i, o + b * q + c] += om[c] * om[b] * sx * D[c, a]
                    for d in range(q):
                        C[o + i, o + d * q + a] += om[a] * om[d] * sy * D[d, b]
        return C

    def matrix_B(self):
        B = np.zeros((self.n, self.n))
        for k in range(self.n_a):
            for f in range(4):
                if self.sn[k, f] > 0:
                    for j, nd in enumerate(self.face_nodes[f]):
                        B[k * self.nn + nd, k * self.nn + nd] += self.omega[j] * self.sn[k, f]
        return B

    def matrix_Bhat(self):
        """B_hat [n, m]: inflow-face coupling (entries w_j (s_k . n_f) < 0)."""
        Bh = np.zeros((self.n, self.m))
        for iota, (f, k, j, nd, row) in enumerate(self.in_tab):
            Bh[row, iota] = self.omega[j] * self.sn[k, f]
        return Bh

    def matrix_S(self, tau_s):
        tau_s = np.asarray(tau_s, dtype=np.float64)
        S = np.zeros((self.n, self.n))
        ws = self.W * tau_s
        for k in range(self.n_a):
            for kp in range(self.n_a):
                coef = self.P[k, kp] * self.w_ang[kp]
                S[k * self.nn:(k + 1) * self.nn, kp * self.nn:(kp + 1) * self.nn] += np.diag(ws * coef)
        return S

    def local_matrix(self, tau_e, tau_s):
        """A = B - C + M - S for nodal reference coefficients tau_e, tau_s [nn]."""
        tau_e = np.asarray(tau_e, dtype=np.float64)
        A = -self.matrix_S(tau_s)
        for k in range(self.n_a):
            sl = slice(k * self.nn, (k + 1) * self.nn)
            A[sl, sl] += self._transport[k] + np.diag(self.W * tau_e)
        return A

    # -- local solve (eq. hdg_local_f2u_i2u, eq. hdg_local_f2o_i2o) -----------
    def scaled_coefficients(self, h, kappa, sigma):
        """Reference-element coefficients tau_e = h (kappa + sigma)/2, tau_s = h sigma/2.

        kappa is absorption, sigma scattering: sigma_e = kappa + sigma,
        sigma_s = sigma (Sec. 2.1).
        """
        kappa = np.asarray(kappa, dtype=np.float64)
        sigma = np.asarray(sigma, dtype=np.float64)
        return 0.5 * h * (kappa + sigma), 0.5 * h * sigma

    def local_solve(self, h, kappa, sigma):
        """Return (in2out [m,m], in2sol [n,m], in2mean [nn,m]) for one element."""
        tau_e, tau_s = self.scaled_coefficients(h, kappa, sigma)
        A = self.local_matrix(tau_e, tau_s)
        X = np.linalg.solve(A, -self.matrix_Bhat())      # A_i2u = -A^{-1} B_hat
        return self.extract(X)

    def extract(self, X):
        in2out = X[self.out_rows, :]
        in2mean = X.reshape(self.n_a, self.nn, self.m).mean(axis=0)
        return in2out, X, in2mean

    def source_solve(self, h, kappa, sigma, f_nodal):
        """f_u = A^{-1}[f] and f_hat_u = R^o f_u for a nodal source f[n_a, nn]."""
        tau_e, tau_s = self.scaled_coefficients(h, kappa, sigma)
        A = self.local_matrix(tau_e, tau_s)
        rhs = (np.asarray(f_nodal, dtype=np.float64) * (0.5 * h) * self.W[None, :]).reshape(-1)
        fu = np.linalg.solve(A, rhs)
        return fu, fu[self.out_rows]


def local_solve_batch(disc, h, kappa, sigma):
    """Loop of LocalDisc.local_solve over elements: h [E], kappa/sigma [E, nn]."""
    h = np.asarray(h, dtype=np.float64).reshape(-1)
    E = h.size
    i2o = np.empty((E, disc.m, disc.m))
    i2s = np.empty((E, disc.n, disc.m))
    i2m = np.empty((E, disc.nn, disc.m))
    for e in range(E):
        i2o[e], i2s[e], i2m[e] = disc.local_solve(h[e], kappa[e], sigma[e])
    return i2o, i2s, i2m

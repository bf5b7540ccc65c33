"""Skeleton system of eq. hdg_global_mat and its solution.

Summing R_hat^o u_hat - A_i2o u_hat over elements gives, row by row, for every
trace DOF that is the outflow of its (unique, upwind) element e:
    t[dof] - (A_i2o^e t[in dofs of e])[local outflow index] = (f_hat_u)
and, on domain-inflow DOFs, t = P_M g.  Written as (I - P) t = b with
(P t)[out dofs of e] = A_i2o^e t[in dofs of e] and P = 0 on domain-inflow rows.

Solvers (Sec. 2.3): a sparse direct solve (the plain definition of the
solution) and a textbook restarted GMRES (Saad & Schultz): x0 = 0, classical
Gram-Schmidt applied twice, Givens rotations, stop when the true relative
residual ||b - (I - P) x|| / ||b|| <= tol.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def matvec(in2out, in_dofs, out_dofs, x):
    """y = (I - P) x."""
    y = np.array(x, dtype=np.float64, copy=True)
    for e in range(in2out.shape[0]):
        y[out_dofs[e]] -= in2out[e] @ x[in_dofs[e]]
    return y


def assemble(in2out, in_dofs, out_dofs, n_trace):
    """Sparse CSR matrix of (I - P)."""
    E, m, _ = in2out.shape
    rows = np.repeat(out_dofs, m, axis=1).reshape(-1)          # [E, m*m]
    cols = np.tile(in_dofs, (1, m)).reshape(-1)
    vals = -in2out.reshape(-1)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(n_trace, n_trace)).tocsr()
    return sp.identity(n_trace, format="csr") + P


def solve_direct(in2out, in_dofs, out_dofs, b):
    A = assemble(in2out, in_dofs, out_dofs, b.size)
    return spla.spsolve(A.tocsc(), b)


def gmres(apply_op, b, tol=1e-12, restart=50, max_iter=2000):
    """Restarted GMRES(restart); returns (x, iterations, true relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, 0.0
    it = 0
    relres = 1.0
    while it < max_iter:
        r = b - apply_op(x)
        beta = np.linalg.norm(r)
        relres = beta / nb
        if relres <= tol:
            break
        V = np.zeros((restart + 1, b.size))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        gvec = np.zeros(restart + 1)
        gvec[0] = beta
        V[0] = r / beta
        k_used = 0
        for j in range(restart):
            w = apply_op(V[j])
            h1 = V[:j + 1] @ w                 # classical Gram-Schmidt, twice
            w = w - h1 @ V[:j + 1]
            h2 = V[:j + 1] @ w
            w = w - h2 @ V[:j + 1]
            H[:j + 1, j] = h1 + h2
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                   # apply previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            it += 1
            k_used = j + 1
            if abs(gvec[j + 1]) / nb <= tol or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), gvec[:k_used])
        x = x + y @ V[:k_used]
    relres = np.linalg.norm(b - apply_op(x)) / nb
    return x, it, relres

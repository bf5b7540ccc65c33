"""First-order running error bounds of the network kernels against the plain
FP64 definition of the network (oracle.mlp with bf16=False).

The HIP path rounds the features, the weights, the hidden activations and the
backpropagated pre-activation gradients to bfloat16 (unit roundoff U = 2^-8)
and accumulates every product in FP32 (unit roundoff U32 = 2^-24, at most
gamma_K = K U32 / (1 - K U32) relative to the sum of absolute terms for a sum
of K terms, in any order).  The bounds below propagate these roundings
elementwise through the layers with absolute-value products, using the
activation's Lipschitz constants (sup |f'| and sup |f''|):

    |x_hat - x| <= e_x
    |z_hat - z| <= e_z = (e_x (1 + U) + U |x|) |W|^T + gamma_K (|x| + e_x)(1 + U) |W|^T + U32 (|z| + ...)
    e_x(next)   = L e_z + (evaluation error of f in FP32) + U (|f(z)| + L e_z)

and, for the gradients in loss units (the MAE subgradient sign(d) taken as
identical on both sides, which the tests guarantee with targets far from the
outputs), the same reasoning through dX = dY W, dZ = dX f'(z) and
dW = dZ^T X.  They are worst-case bounds: a kernel that follows the
definition stays inside them, a wrong index, a dropped term or a lost split
does not.

Every function takes the operand unit roundoff u (default U): u = 0 gives the
bounds of the FP32 network path, whose operands are never rounded below FP32
(features, weights, activations and gradients in FP32; the FP32 roundings of
the arithmetic keep their U32 terms).
"""
import numpy as np

from oracle.mlp import act, dact, TAU_FLOOR

U = 2.0 ** -8
U32 = 2.0 ** -24
LIP = {"gelu": 1.13, "elu": 1.0, "linear": 1.0}     # sup |f'| (GELU: 1.1289 at z = sqrt(2))
LIP2 = {"gelu": 0.8, "elu": 1.0, "linear": 0.0}     # sup |f''| (GELU: 2 phi(0) = 0.798)


def gam(k):
    return k * U32 / (1.0 - k * U32)


def feature_bound(x, fm, fs, k0, u=U):
    """|X0_kernel - X0_exact| for raw inputs x [B, n_in]: the feature is
    rounded to FP32, z-scored in FP32 and rounded to bfloat16."""
    x = np.asarray(x, dtype=np.float64)
    B, n_in = x.shape
    f = np.empty((B, n_in))
    f[:, 0] = np.log10(x[:, 0])
    f[:, 1:] = np.log10(np.maximum(0.5 * x[:, :1] * x[:, 1:], TAU_FLOOR))
    z = (f - fm[None, :]) / fs[None, :]
    e_f = U32 * np.abs(f)
    e_z = (e_f + 2 * U32 * np.abs(f - fm[None, :])) / fs[None, :] + 2 * U32 * np.abs(z)
    e = np.zeros((B, k0))
    e[:, :n_in] = e_z + u * (np.abs(z) + e_z)
    return e


def forward_bounds(mlp, X0, e0, u=U):
    """Exact forward quantities and bounds: returns (out, Xs, Zs, e_out,
    e_xs, e_zs) with e_xs[l] bounding the kernel's layer-l input and
    e_zs[l] its pre-activation."""
    out, (Xs, Zs) = mlp.forward(X0, bf16=False)
    L = LIP[mlp.act]
    e_x = e0
    e_xs, e_zs = [e0], []
    D = len(mlp.Ws) - 1
    for l in range(D + 1):
        A = np.abs(mlp.Ws[l]).T
        X = np.abs(Xs[l])
        K = mlp.Ws[l].shape[1]
        e_p = (e_x * (1 + u) + u * X) @ A + gam(K) * (((X + e_x) * (1 + u)) @ A)
        Z = Zs[l] if l < D else out
        e_z = e_p + U32 * (np.abs(Z) + e_p)
        e_zs.append(e_z)
        if l < D:
            fz = np.abs(act(mlp.act, Zs[l]))
            e_a = L * e_z + 4 * U32 * (fz + np.abs(Zs[l]) + L * e_z)
            e_x = e_a + u * (np.abs(Xs[l + 1]) + e_a)
            e_xs.append(e_x)
    return out, Xs, Zs, e_zs[-1], e_xs, e_zs


def denorm_bound(out, e_out, ys, ym):
    """Bound of the FP32 de-normalized output (acc + b) sd + mean."""
    y = out * ys[None, :] + ym[None, :]
    return ys[None, :] * e_out + 3 * U32 * (np.abs(out) * ys[None, :] + np.abs(y))


def grad_bounds(mlp, Xs, Zs, e_xs, e_zs, dY, dX_last=None, u=U):
    """Exact gradients in loss units (sum over the batch of dY-weighted
    products, dY = sign(d) in {-1, 0, 1}) and their bounds, per layer:
    returns (gW, gb, eW, eb).  dX_last: the exact dY W_D when the caller has
    it (large output layers), else computed here."""
    D = len(mlp.Ws) - 1
    B = dY.shape[0]
    L2 = LIP2[mlp.act]
    aY = np.abs(dY)
    gW, gb, eW, eb = [None] * (D + 1), [None] * (D + 1), [None] * (D + 1), [None] * (D + 1)
    XD = np.abs(Xs[D])
    gW[D] = dY.T @ Xs[D]
    eW[D] = aY.T @ e_xs[D] + gam(B) * (aY.T @ (XD + e_xs[D]))
    gb[D] = dY.sum(axis=0)
    eb[D] = np.zeros_like(gb[D])              # sums of +-1 in FP32: exact
    WD = np.abs(mlp.Ws[D])
    dX = dY @ mlp.Ws[D] if dX_last is None else dX_last
    n_out = mlp.Ws[D].shape[0]
    e_dX = aY @ (u * WD) + gam(n_out) * (aY @ ((1 + u) * WD))
    for l in range(D - 1, -1, -1):
        Z = Zs[l]
        df = dact(mlp.act, Z)
        dZ = dX * df
        adX = np.abs(dX) + e_dX
        e_dZ = e_dX * np.abs(df) + adX * L2 * e_zs[l] + 4 * U32 * adX * (1 + np.abs(Z)) + U32 * np.abs(dZ)
        gb[l] = dZ.sum(axis=0)
        eb[l] = e_dZ.sum(axis=0) + gam(B) * np.abs(dZ).sum(axis=0)
        e_dZr = e_dZ + u * (np.abs(dZ) + e_dZ)
        X = np.abs(Xs[l])
        ex = e_xs[l]
        gW[l] = dZ.T @ Xs[l]
        eW[l] = e_dZr.T @ (X + ex) + np.abs(dZ).T @ ex + gam(B) * ((np.abs(dZ) + e_dZr).T @ (X + ex))
        if l > 0:
            Wl = np.abs(mlp.Ws[l])
            K = mlp.Ws[l].shape[0]
            dX = dZ @ mlp.Ws[l]
            e_dX = e_dZr @ ((1 + u) * Wl) + np.abs(dZ) @ (u * Wl) + gam(K) * ((np.abs(dZ) + e_dZr) @ ((1 + u) * Wl))
    return gW, gb, eW, eb


def check(got, ref, bound, what):
    """Every entry inside its bound; prints the measured error and the worst
    fraction of the bound used."""
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    frac = float(np.max(err / np.maximum(bound, 1e-300)))
    scale = float(np.abs(ref).max()) or 1.0
    print(f"[{what}] max |err| {err.max():.3e} (rel to max {err.max() / scale:.3e}), "
          f"worst fraction of the FP64-definition bound {frac:.3f}", flush=True)
    assert np.all(err <= bound), (what, frac)
    return frac

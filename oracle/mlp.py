"""FP64 fully connected element network, MAE loss and Adam.

Sec. 2.4.1: x_i = f_i(A_i x_{i-1} + b_i), f_i a nonlinear activation on the
hidden layers and the identity on the output layer.  Sec. 3.1: mean
absolute error loss, Adam optimizer.  GELU is the exact erf form
GELU(z) = z Phi(z); ELU(z) = z (z > 0), exp(z) - 1 otherwise; "linear" is the
identity (the linear network of the Sec. 3.1 ablations).

Input of one element: x = (h, kappa[nn], sigma[nn]).  Features: log10 h and
log10 max(h v / 2, 1e-12) for every nodal kappa and sigma (the
reference-element coefficients of Sec. 2.4.1), z-scored with the given
statistics and zero-padded to k0 columns.  Targets are z-scored per output.

``bf16=True`` rounds to bfloat16 (nearest even) exactly where the HIP kernels
do: the features, the weights used by the products, the hidden activations
and the backpropagated pre-activation gradients used by the products (not the
ones summed for the bias gradients).  Everything else is FP64.
"""
import numpy as np
from scipy.special import erf

TAU_FLOOR = 1e-12


def bf16_round(a):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def act(kind, z):
    if kind == "linear":
        return np.asarray(z, dtype=np.float64)
    if kind == "elu":
        return np.where(z > 0, z, np.expm1(np.minimum(z, 0.0)))
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def dact(kind, z):
    if kind == "linear":
        return np.ones_like(np.asarray(z, dtype=np.float64))
    if kind == "elu":
        return np.where(z > 0, 1.0, np.exp(np.minimum(z, 0.0)))
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def features(x, feat_mean, feat_std, k0):
    """z-scored features [B, k0] of raw inputs x [B, n_in] = (h, kappa, sigma)."""
    x = np.asarray(x, dtype=np.float64)
    B, n_in = x.shape
    h = x[:, :1]
    f = np.empty((B, n_in))
    f[:, 0] = np.log10(h[:, 0])
    f[:, 1:] = np.log10(np.maximum(0.5 * h * x[:, 1:], TAU_FLOOR))
    z = (f - feat_mean[None, :]) / feat_std[None, :]
    out = np.zeros((B, k0))
    out[:, :n_in] = z
    return out


class MLP:
    """Weights Ws[l] [out_l, in_l] and biases bs[l] [out_l], l = 0..depth."""

    def __init__(self, Ws, bs, act_kind="gelu"):
        self.Ws = [np.asarray(W, dtype=np.float64) for W in Ws]
        self.bs = [np.asarray(b, dtype=np.float64) for b in bs]
        self.act = act_kind

    def forward(self, X0, bf16=False):
        """Normalized outputs and the cache (inputs X_l, pre-activations Z_l)."""
        rnd = bf16_round if bf16 else (lambda a: a)
        X = rnd(X0)
        Xs, Zs = [X], []
        D = len(self.Ws) - 1
        for l in range(D):
            Z = X @ rnd(self.Ws[l]).T + self.bs[l]
            Zs.append(Z)
            X = rnd(act(self.act, Z))
            Xs.append(X)
        out = X @ rnd(self.Ws[D]).T + self.bs[D]
        return out, (Xs, Zs)

    def mae_grad(self, X0, target_norm, bf16=False):
        """Mean absolute error over all outputs and its gradient (subgradient
        sign(d) with sign(0) = 0) with respect to every W and b."""
        rnd = bf16_round if bf16 else (lambda a: a)
        out, (Xs, Zs) = self.forward(X0, bf16)
        d = out - target_norm
        count = d.size
        loss = np.abs(d).sum() / count
        dY = np.sign(d) / count
        D = len(self.Ws) - 1
        gW = [None] * (D + 1)
        gb = [None] * (D + 1)
        gW[D] = dY.T @ Xs[D]
        gb[D] = dY.sum(axis=0)
        dX = dY @ rnd(self.Ws[D])
        for l in range(D - 1, -1, -1):
            dZ = dX * dact(self.act, Zs[l])
            gb[l] = dZ.sum(axis=0)
            gW[l] = rnd(dZ * count).T @ Xs[l] / count
            if l > 0:
                dX = rnd(dZ * count) @ rnd(self.Ws[l]) / count
        return loss, gW, gb


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v

"""Pins of the FP64 network oracle (Sec. 2.4.1 network, Sec. 3.1 MAE + Adam).

* gradients against central finite differences (FP64, small widths);
* one Adam step from a zero state moves every weight by exactly lr * g / (|g| + eps);
* the bfloat16 rounding used to mimic the kernels equals torch's
  float32 -> bfloat16 conversion (round to nearest even);
* the network blob packer round-trips.
"""
import numpy as np
import pytest
import torch

from oracle.mlp import MLP, act, dact, adam_step, bf16_round, features


def _rand_mlp(rng, n_in, width, depth, n_out, kind):
    dims = [n_in] + [width] * depth + [n_out]
    Ws = [rng.uniform(-1, 1, (dims[l + 1], dims[l])) / np.sqrt(dims[l]) for l in range(depth + 1)]
    bs = [rng.uniform(-0.1, 0.1, dims[l + 1]) for l in range(depth + 1)]
    return MLP(Ws, bs, kind)


@pytest.mark.parametrize("kind", ["gelu", "elu", "linear"])
def test_activation_derivative_fd(kind):
    z = np.linspace(-4, 4, 101)
    z = z[np.abs(z) > 1e-3]
    eps = 1e-6
    fd = (act(kind, z + eps) - act(kind, z - eps)) / (2 * eps)
    assert np.abs(fd - dact(kind, z)).max() < 1e-8
    if kind == "gelu":                     # closed values: GELU(0) = 0, GELU(z) -> z for large z
        assert act(kind, np.array([0.0]))[0] == 0.0
        assert abs(act(kind, np.array([10.0]))[0] - 10.0) < 1e-12


def test_activation_tabulated_values():
    """Values fixed by the definitions, not by the oracle's formula: the exact
    GELU is z Phi(z), so GELU(1) = Phi(1) and GELU(-1) = -(1 - Phi(1)) with
    the standard normal CDF value Phi(1) = 0.8413447460685429 (the tanh
    approximation of GELU is 1.5e-4 off at z = 1); ELU(-1) = 1/e - 1; the
    derivative of the exact GELU at 1 is Phi(1) + phi(1), phi(1) =
    0.24197072451914337."""
    phi1, dens1 = 0.8413447460685429, 0.24197072451914337
    g = act("gelu", np.array([1.0, -1.0]))
    assert abs(g[0] - phi1) <= 1e-15 and abs(g[1] + (1.0 - phi1)) <= 1e-15
    assert abs(dact("gelu", np.array([1.0]))[0] - (phi1 + dens1)) <= 1e-15
    assert abs(act("elu", np.array([-1.0]))[0] - (1.0 / np.e - 1.0)) <= 1e-16
    assert act("elu", np.array([2.5]))[0] == 2.5
    assert abs(dact("elu", np.array([-1.0]))[0] - 1.0 / np.e) <= 1e-16


@pytest.mark.parametrize("kind", ["gelu", "elu", "linear"])
def test_mae_gradients_match_finite_differences(kind):
    rng = np.random.default_rng(4)
    net = _rand_mlp(rng, 7, 12, 3, 5, kind)
    X = rng.standard_normal((6, 7))
    T = rng.standard_normal((6, 5))
    loss, gW, gb = net.mae_grad(X, T)
    eps = 1e-6
    for l in range(len(net.Ws)):
        for (i, j) in [(0, 0), (1, 2), (net.Ws[l].shape[0] - 1, net.Ws[l].shape[1] - 1)]:
            W0 = net.Ws[l][i, j]
            net.Ws[l][i, j] = W0 + eps
            lp = net.mae_grad(X, T)[0]
            net.Ws[l][i, j] = W0 - eps
            lm = net.mae_grad(X, T)[0]
            net.Ws[l][i, j] = W0
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - gW[l][i, j]) <= 1e-7 * max(1.0, abs(fd)), (l, i, j, fd, gW[l][i, j])
        b0 = net.bs[l][1]
        net.bs[l][1] = b0 + eps
        lp = net.mae_grad(X, T)[0]
        net.bs[l][1] = b0 - eps
        lm = net.mae_grad(X, T)[0]
        net.bs[l][1] = b0
        assert abs((lp - lm) / (2 * eps) - gb[l][1]) <= 1e-7


def test_mae_is_mean_absolute_error():
    rng = np.random.default_rng(1)
    net = _rand_mlp(rng, 4, 8, 1, 3, "gelu")
    X = rng.standard_normal((5, 4))
    out, _ = net.forward(X)
    T = out + np.array([1.0, -2.0, 0.5])
    loss, _, gb = net.mae_grad(X, T)
    assert abs(loss - 3.5 / 3) < 1e-12
    # d loss / d b_out = mean over the batch of sign(out - T) / n_out
    assert np.allclose(gb[-1], np.array([-1.0, 1.0, -1.0]) * 5 / 15)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    t1, m, v = adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    assert np.allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(3)
    a = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-30, 30, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.4e38]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(bf16_round(a), ref)


def test_features_are_reference_element_coefficients():
    """Scaling invariance of Sec. 2.4.1: (h, kappa, sigma) and (2h, kappa/2, sigma/2)
    give the same kappa/sigma features; only the log10 h feature moves."""
    rng = np.random.default_rng(5)
    nn = 4
    x = np.concatenate([[0.1], rng.uniform(0.1, 1, nn), rng.uniform(1, 10, nn)])[None, :]
    x2 = np.concatenate([[0.2], x[0, 1:] / 2])[None, :]
    mean, std = np.zeros(9), np.ones(9)
    f1, f2 = features(x, mean, std, 32), features(x2, mean, std, 32)
    assert np.allclose(f1[0, 1:9], f2[0, 1:9], atol=1e-14)
    assert abs(f2[0, 0] - f1[0, 0] - np.log10(2)) < 1e-14
    assert np.all(f1[0, 9:] == 0)


def test_blob_roundtrip():
    from paper_2308_02467_amd import el
    k0, layers, P = el.net_layout(9, 16, 2, 24)
    assert k0 == 32 and all(w % 64 == 0 for (w, b, o, i) in layers)
    rng = np.random.default_rng(0)
    th = rng.standard_normal(P).astype(np.float32)
    blob = el.pack_net_blob(9, 16, 2, 0, 24, th, np.zeros(9), np.ones(9), np.zeros(24), np.ones(24),
                            [1, 2, 3, 4, 5, 6], step=7)
    u = el.unpack_net_blob(blob)
    assert u["step"] == 7 and u["box"] == [1, 2, 3, 4, 5, 6] and np.array_equal(u["theta"], th)
    assert len(blob) == el.HEADER_BYTES + 4 * (2 * 9 + 2 * 24 + 3 * P)


def test_linear_network_is_one_affine_map():
    """With the identity activation the network collapses to a single affine
    map x -> x A^T + c, A = W_D ... W_0, c = W_D(...(W_1 b_0 + b_1)...) + b_D,
    built here by folding the layers one at a time from the input side."""
    rng = np.random.default_rng(8)
    net = _rand_mlp(rng, 9, 16, 3, 5, "linear")
    X = rng.standard_normal((7, 9))
    A = np.eye(9)
    c = np.zeros(9)
    for W, b in zip(net.Ws, net.bs):
        A = W @ A
        c = W @ c + b
    out, _ = net.forward(X)
    assert np.abs(out - (X @ A.T + c)).max() < 1e-12


@pytest.mark.parametrize("kind", ["gelu", "elu", "linear"])
def test_bf16_emulation_inside_fp64_definition_bounds(kind):
    """The running error bounds used by the GPU tests (tests/_netbound.py)
    hold for the oracle's own emulation of the kernels' bfloat16 rounding
    points: forward outputs and (with targets far from the outputs, so the
    MAE signs agree) every gradient in loss units."""
    import _netbound as nb
    rng = np.random.default_rng(7)
    n_in, width, depth, n_out, B = 11, 48, 3, 40, 30
    net = _rand_mlp(rng, 16, width, depth, n_out, kind)
    net.Ws[0][:, n_in:] = 0.0
    h = rng.uniform(0.005, 0.1, (B, 1))
    x = np.concatenate([h, rng.uniform(0.01, 3, (B, 5)), rng.uniform(0.05, 30, (B, 5))], axis=1)
    fm, fs = rng.uniform(-2, 0, n_in), rng.uniform(0.5, 2, n_in)
    X0 = features(x, fm, fs, 16)
    e0 = nb.feature_bound(x, fm, fs, 16)
    assert np.all(np.abs(bf16_round(X0) - X0) <= e0)
    out, Xs, Zs, e_out, e_xs, e_zs = nb.forward_bounds(net, X0, e0)
    ob, _ = net.forward(X0, bf16=True)
    assert np.all(np.abs(ob - out) <= e_out)
    sgn = rng.choice([-1.0, 1.0], (B, n_out))
    tgt = out + sgn * 50.0
    _, gWb, gbb = net.mae_grad(X0, tgt, bf16=True)
    count = B * n_out
    gW, gb, eW, eb = nb.grad_bounds(net, Xs, Zs, e_xs, e_zs, -sgn)
    for l in range(depth + 1):
        assert np.all(np.abs(gWb[l] * count - gW[l]) <= eW[l]), l
        assert np.all(np.abs(gbb[l] * count - gb[l]) <= eb[l] + 1e-12 * (np.abs(gb[l]) + B)), l


@pytest.mark.parametrize("kind", ["gelu", "elu"])
def test_fp32_emulation_inside_fp32_path_bounds(kind):
    """The bounds with operand unit roundoff u = 0 (the FP32 network path)
    hold for a float32 emulation of the network, and are tight enough that
    the bfloat16 emulation falls outside them: a path that still rounded its
    operands to bfloat16 would fail the FP32 GPU tests."""
    import _netbound as nb
    rng = np.random.default_rng(11)
    n_in, width, depth, n_out, B = 11, 48, 3, 40, 30
    net = _rand_mlp(rng, 16, width, depth, n_out, kind)
    net.Ws[0][:, n_in:] = 0.0
    h = rng.uniform(0.005, 0.1, (B, 1))
    x = np.concatenate([h, rng.uniform(0.01, 3, (B, 5)), rng.uniform(0.05, 30, (B, 5))], axis=1)
    fm, fs = rng.uniform(-2, 0, n_in), rng.uniform(0.5, 2, n_in)
    X0 = features(x, fm, fs, 16)
    e0 = nb.feature_bound(x, fm, fs, 16, u=0.0)
    out, Xs, Zs, e_out, e_xs, e_zs = nb.forward_bounds(net, X0, e0, u=0.0)
    X = X0.astype(np.float32)
    D = len(net.Ws) - 1
    for l in range(D):
        Z = X @ net.Ws[l].astype(np.float32).T + net.bs[l].astype(np.float32)
        X = act(kind, Z.astype(np.float64)).astype(np.float32)
    o32 = X @ net.Ws[D].astype(np.float32).T + net.bs[D].astype(np.float32)
    assert np.all(np.abs(o32 - out) <= e_out)
    ob, _ = net.forward(X0, bf16=True)
    assert np.any(np.abs(ob - out) > e_out)

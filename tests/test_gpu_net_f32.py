"""GPU parity of the FP32 network path (el_train_step_f32, el_net_forward_f32)
against the plain FP64 definition of the network (oracle.mlp, no rounding),
entry by entry within the running error bounds of tests/_netbound.py taken
with operand unit roundoff 0: the path rounds nothing below FP32, so only the
FP32 roundings of its arithmetic remain (a path that rounded an operand to
bfloat16 falls outside these bounds; tests/test_oracle_mlp.py checks that on
the CPU).  Weights, statistics and inputs come from the host (numpy, seeded)
through the documented blob.

Shapes cover ragged block tiles (batch, width and outputs not multiples of
64), batches above the 128-row chunks of the column sums, and output counts
above the 2,048-long k chunks of the split dX product (several and ragged
splits)."""
import numpy as np
import pytest
import torch

from oracle.mlp import adam_step, features
import _netbound as nb
from test_gpu_net import _host_net, _load, _raw_inputs

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02467_amd import el
    c = el.Context(0)
    yield c
    c.close()


SHAPES = [(9, 64, 2, 96, 0, 6), (19, 200, 3, 520, 1, 50), (99, 256, 2, 5000, 0, 200), (19, 72, 1, 4104, 2, 130)]


@pytest.mark.parametrize("n_in,width,depth,n_out,act,B", SHAPES)
def test_forward_f32_fp64_definition(ctx, n_in, width, depth, n_out, act, B):
    rng = np.random.default_rng(n_in + width + 1)
    hn = _host_net(rng, n_in, width, depth, n_out, act)
    net = _load(ctx, hn, n_in, width, depth, n_out, act)
    x = _raw_inputs(rng, B, (n_in - 1) // 2).astype(np.float32)
    xd = torch.from_numpy(x).to(DEV)
    y = torch.empty((B, n_out), dtype=torch.float32, device=DEV)
    yd = torch.empty((B, n_out), dtype=torch.float32, device=DEV)
    print(f"[el_net_forward_f32] {n_in}-{width}x{depth}-{n_out} B={B}", flush=True)
    net.forward_f32(xd, y)
    net.forward_f32(xd, yd, denormalize=True)
    fm, fs = hn["fm"].astype(np.float64), hn["fs"].astype(np.float64)
    X0 = features(x.astype(np.float64), fm, fs, hn["k0"])
    e0 = nb.feature_bound(x, fm, fs, hn["k0"], u=0.0)
    out, _, _, e_out, _, _ = nb.forward_bounds(hn["oracle"], X0, e0, u=0.0)
    nb.check(y.cpu().numpy(), out, e_out, "el_net_forward_f32 vs FP64")
    ys, ym = hn["ys"].astype(np.float64), hn["ym"].astype(np.float64)
    nb.check(yd.cpu().numpy(), out * ys[None, :] + ym[None, :], nb.denorm_bound(out, e_out, ys, ym),
             "el_net_forward_f32 de-normalized vs FP64")
    net.close()


@pytest.mark.parametrize("n_in,width,depth,n_out,act,B", SHAPES)
def test_gradients_loss_and_adam_f32_fp64_definition(ctx, n_in, width, depth, n_out, act, B):
    """One FP32 training step: every gradient (loss units) against the FP64
    definition within the u = 0 bounds, the loss against the exact mean
    absolute error, and, with lr > 0, the Adam update against its closed
    form applied to the returned gradient.  The targets lie 50 to 100
    normalized units from every output, so the MAE subgradient signs are
    the same on both sides."""
    from paper_2308_02467_amd import el
    rng = np.random.default_rng(200 + n_out)
    hn = _host_net(rng, n_in, width, depth, n_out, act)
    net = _load(ctx, hn, n_in, width, depth, n_out, act)
    x = _raw_inputs(rng, B, (n_in - 1) // 2).astype(np.float32)
    sgn = rng.choice([-1.0, 1.0], (B, n_out))
    tn = sgn * rng.uniform(50.0, 100.0, (B, n_out))
    y32 = (tn * hn["ys"][None, :] + hn["ym"][None, :]).astype(np.float32)
    # the normalized target the kernel sees, (y - mean) / sd in FP32
    tn32 = ((y32.astype(np.float64) - hn["ym"][None, :]) / hn["ys"][None, :])
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    lr = 1e-3
    print(f"[el_train_step_f32] {n_in}-{width}x{depth}-{n_out} B={B}", flush=True)
    net.train_step_f32(torch.from_numpy(x).to(DEV), torch.from_numpy(y32).to(DEV), lr, loss)
    g = net.params(1).cpu().numpy().astype(np.float64)
    th = net.params(0).cpu().numpy().astype(np.float64)
    mom = net.params(2).cpu().numpy().astype(np.float64)
    fm, fs = hn["fm"].astype(np.float64), hn["fs"].astype(np.float64)
    X0 = features(x.astype(np.float64), fm, fs, hn["k0"])
    e0 = nb.feature_bound(x, fm, fs, hn["k0"], u=0.0)
    out, Xs, Zs, _, e_xs, e_zs = nb.forward_bounds(hn["oracle"], X0, e0, u=0.0)
    assert np.abs(out).max() < 40.0
    dY = -sgn
    gW, gb, eW, eb = nb.grad_bounds(hn["oracle"], Xs, Zs, e_xs, e_zs, dY, u=0.0)
    _, layers, P = el.net_layout(n_in, width, depth, n_out)
    for l, (w_off, b_off, fout, fin) in enumerate(layers):
        nb.check(g[w_off:w_off + fout * fin].reshape(fout, fin), gW[l], eW[l], f"dW layer {l}")
        nb.check(g[b_off:b_off + fout], gb[l], eb[l], f"db layer {l}")
    ref_loss = float(np.abs(out - tn32).mean())
    got_loss = float(loss.item())
    print(f"[el_train_step_f32] loss {got_loss:.7e} vs {ref_loss:.7e}", flush=True)
    assert abs(got_loss - ref_loss) <= 1e-5 * ref_loss
    # Adam, first step, from zero moments: closed form on the kernel's own gradient
    gs = g / (B * n_out)
    t_ref, m_ref, _ = adam_step(hn["theta"].astype(np.float64), gs, 0.0, 0.0, 1, lr)
    assert np.abs(mom - m_ref).max() <= 1e-6 * np.abs(m_ref).max() + 1e-30
    assert np.abs(th - t_ref).max() <= 1e-6 * (np.abs(t_ref).max() + lr)
    net.close()


def test_f32_training_reduces_loss_and_mixes_with_bf16_state(ctx):
    """A few FP32 steps on fixed targets lower the loss, and the network they
    leave is a valid state for the bfloat16 path (the same parameters; its
    forward agrees with the FP32 forward to the bfloat16 bound)."""
    rng = np.random.default_rng(5)
    n_in, width, depth, n_out, B = 19, 64, 2, 304, 64
    hn = _host_net(rng, n_in, width, depth, n_out, 0)
    net = _load(ctx, hn, n_in, width, depth, n_out, 0)
    x = torch.from_numpy(_raw_inputs(rng, B, (n_in - 1) // 2).astype(np.float32)).to(DEV)
    tn = 2.0 + 0.1 * rng.standard_normal((B, n_out))                # normalized targets
    y = torch.from_numpy((tn * hn["ys"][None, :] + hn["ym"][None, :]).astype(np.float32)).to(DEV)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    hist = []
    for _ in range(60):
        net.train_step_f32(x, y, 3e-3, loss)
        hist.append(loss.item())
    print(f"[el_train_step_f32] loss {hist[0]:.4f} -> {hist[-1]:.4f}", flush=True)
    assert hist[-1] < 0.8 * hist[0]
    a = torch.empty((B, n_out), dtype=torch.float32, device=DEV)
    b = torch.empty((B, n_out), dtype=torch.float32, device=DEV)
    net.forward_f32(x, a)
    net.forward(x, b)
    d = (a - b).abs().max().item()
    print(f"[el_net_forward vs el_net_forward_f32] max |diff| {d:.3e}", flush=True)
    assert d <= 0.05 * a.abs().max().item()
    net.close()


def test_f32_argument_errors(ctx):
    from paper_2308_02467_amd import el
    rng = np.random.default_rng(1)
    hn = _host_net(rng, 9, 64, 1, 96, 0)
    net = _load(ctx, hn, 9, 64, 1, 96, 0)
    x = torch.zeros((4, 9), dtype=torch.float32, device=DEV)
    y = torch.zeros((4, 96), dtype=torch.float32, device=DEV)
    with pytest.raises(el.ElError):
        net.train_step_f32(x, y, float("nan"))
    assert el.lib().el_train_step_f32(ctx.h, net.h, 0, None, None, 1e-3, None) != 0
    assert el.lib().el_net_forward_f32(ctx.h, net.h, 0, None, None, 0) == 0   # empty batch: nothing to do
    net.close()

"""The network kernels at the shapes of the timed learned step (p = 6,
N_a = 16: network 99-1024x4-225,792, GELU), against the oracle on sampled
rows (the oracle cannot run the whole batch in seconds) and by properties
that hold at any size.

* inference of 16,384 elements of the 128 x 128 Gaussian-cloud workload (the
  GEMM launch the benchmark times: 64 row tiles of 256 with the direct-to-LDS
  tile) and of a ragged 5,000-element batch, 64 sampled elements each, entry
  by entry: against the bfloat16-rounded oracle (one storage rounding plus
  FP32 accumulation, but for rare rounding-boundary flips of hidden
  activations) and against the plain FP64 definition within the running
  error bound of tests/_netbound.py;
* one training step at batch 4,096 (the output-layer dX product split 32
  ways over K = 225,792): the output-layer bias gradient of all 225,792
  outputs bit-exactly (sums of +-1), the weight gradient of 64 sampled
  output rows and every hidden-layer gradient entry within the bound.
"""
import numpy as np
import pytest
import torch

from oracle.mlp import dact, features
from paper_2308_02467_amd import inputs

import _netbound as nb
from test_gpu_net import _host_net, _load, bf16_mode_check

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
P_DEG, N_A, WIDTH, DEPTH = 6, 16, 1024, 4


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02467_amd import el
    c = el.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def headline_net():
    from paper_2308_02467_amd import el
    d = el.disc(P_DEG, N_A)
    nn, n, m = el.disc_sizes(d)
    n_in, n_out = 1 + 2 * nn, m * m + n * m
    print(f"[headline net] building {n_in}-{WIDTH}x{DEPTH}-{n_out} on the host", flush=True)
    hn = _host_net(np.random.default_rng(2468), n_in, WIDTH, DEPTH, n_out, 0)
    return d, hn, n_in, n_out


@pytest.fixture
def gemm_tile():
    from paper_2308_02467_amd import el
    yield el.gemm_tile
    el.gemm_tile(-1)


@pytest.mark.parametrize("E,tile", [(16384, 3), (16384, -1), (5000, -1)])
def test_infer_headline_shape(ctx, headline_net, gemm_tile, E, tile):
    from paper_2308_02467_amd import el
    d, hn, n_in, n_out = headline_net
    nn, n, m = el.disc_sizes(d)
    net = _load(ctx, hn, n_in, WIDTH, DEPTH, n_out)
    nx = 128
    xi, _ = el.lgl(P_DEG)
    X, Y = inputs.element_node_coords(nx, nx, 1.0 / nx, xi)
    kap, sig = inputs.gaussian_cloud(X, Y)
    kap, sig = kap[:E], sig[:E]
    hh = np.full(E, 1.0 / nx)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)
    i2o = torch.empty((E, m, m), dtype=torch.float32, device=DEV)
    i2s = torch.empty((E, n, m), dtype=torch.float32, device=DEV)
    gemm_tile(tile)
    print(f"[el_infer headline] E={E} tile={tile}", flush=True)
    net.infer(d, T(hh), T(kap), T(sig), i2o, i2s, None, fallback=False)
    torch.cuda.synchronize()
    rng = np.random.default_rng(E + tile)
    sel = np.unique(np.concatenate([[0, E - 1], rng.choice(E, 62, replace=False)]))
    st = torch.as_tensor(sel, device=DEV)
    got = torch.cat([i2o[st].reshape(sel.size, -1), i2s[st].reshape(sel.size, -1)], dim=1).double().cpu().numpy()
    del i2o, i2s
    torch.cuda.empty_cache()
    x = np.concatenate([hh[sel, None], kap[sel], sig[sel]], axis=1)
    fm, fs = hn["fm"].astype(np.float64), hn["fs"].astype(np.float64)
    ys, ym = hn["ys"].astype(np.float64), hn["ym"].astype(np.float64)
    X0 = features(x, fm, fs, hn["k0"])
    print("[el_infer headline] oracle on the sampled rows", flush=True)
    yb, _ = hn["oracle"].forward(X0, bf16=True)
    yb = yb * ys[None, :] + ym[None, :]
    bf16_mode_check(got, yb, nb.U32, 0.0, "el_infer headline")
    e0 = nb.feature_bound(x, fm, fs, hn["k0"])
    out, _, _, e_out, _, _ = nb.forward_bounds(hn["oracle"], X0, e0)
    y64 = out * ys[None, :] + ym[None, :]
    e_y = nb.denorm_bound(out, e_out, ys, ym)
    nb.check(got, y64, e_y * (1 + nb.U32) + nb.U32 * np.abs(y64), "el_infer headline vs FP64")
    net.close()


def test_train_step_headline_shape(ctx, headline_net):
    from paper_2308_02467_amd import el
    d, hn, n_in, n_out = headline_net
    B = 4096
    mlp = hn["oracle"]
    net = _load(ctx, hn, n_in, WIDTH, DEPTH, n_out)
    xi, _ = el.lgl(P_DEG)
    h, kap, sig = inputs.training_draws(B, xi, seed=97)
    x = np.concatenate([h[:, None], kap, sig], axis=1).astype(np.float32)
    # targets 64 normalized units above or below the outputs' range: the MAE
    # subgradient is -sign(target) on both sides
    rng = np.random.default_rng(98)
    sgn = (2 * rng.integers(0, 2, (B, n_out), dtype=np.int8) - 1)
    y16 = torch.empty((B, n_out), dtype=torch.bfloat16)
    ys32, ym32 = hn["ys"], hn["ym"]
    for r0 in range(0, B, 512):
        y16[r0:r0 + 512] = torch.from_numpy((sgn[r0:r0 + 512] * (64.0 * ys32)[None, :] + ym32[None, :])
                                            .astype(np.float32)).to(torch.bfloat16)
    print(f"[el_train_step headline] B={B} n_out={n_out}", flush=True)
    net.train_step(torch.from_numpy(x).to(DEV), y16.to(DEV), 0.0)
    g = net.params(1).cpu().numpy().astype(np.float64)
    del y16
    fm, fs = hn["fm"].astype(np.float64), hn["fs"].astype(np.float64)
    X0 = features(x.astype(np.float64), fm, fs, hn["k0"])
    e0 = nb.feature_bound(x, fm, fs, hn["k0"])
    print("[el_train_step headline] oracle: hidden layers", flush=True)
    # hidden layers only (the output layer's forward is not needed: the
    # signs are fixed by the targets)
    hid = type(mlp)(mlp.Ws[:DEPTH] + [np.zeros((1, WIDTH))], mlp.bs[:DEPTH] + [np.zeros(1)], mlp.act)
    _, Xs, Zs, _, e_xs, e_zs = nb.forward_bounds(hid, X0, e0)
    assert np.abs(Xs[DEPTH]).max() < 1e3
    WD = mlp.Ws[DEPTH]
    print("[el_train_step headline] oracle: dY W_out (FP64, 1.9 TFLOP)", flush=True)
    dX = np.empty((B, WIDTH))
    for r0 in range(0, B, 512):
        dX[r0:r0 + 512] = (-sgn[r0:r0 + 512]).astype(np.float64) @ WD
    colabs = np.abs(WD).sum(axis=0)
    e_dX = np.broadcast_to((nb.U + nb.gam(n_out) * (1 + nb.U)) * colabs, (B, WIDTH))
    _, layers, _ = el.net_layout(n_in, WIDTH, DEPTH, n_out)
    # output layer: bias gradient of every output (exact), weights of 64 rows
    w_off, b_off, fout, fin = layers[DEPTH]
    gb_exact = -sgn.sum(axis=0, dtype=np.int64).astype(np.float64)
    print(f"[el_train_step headline] output bias gradient: {int(np.sum(g[b_off:b_off + fout] != gb_exact))} "
          f"of {fout} entries differ", flush=True)
    assert np.array_equal(g[b_off:b_off + fout], gb_exact)
    rows = np.sort(rng.choice(n_out, 64, replace=False))
    dYs = (-sgn[:, rows]).astype(np.float64)
    gW_rows = dYs.T @ Xs[DEPTH]
    eW_rows = np.broadcast_to(e_xs[DEPTH].sum(axis=0) + nb.gam(B) * (np.abs(Xs[DEPTH]) + e_xs[DEPTH]).sum(axis=0),
                              gW_rows.shape)
    GWD = g[w_off:w_off + fout * fin].reshape(fout, fin)
    nb.check(GWD[rows], gW_rows, eW_rows, "dW output layer (64 rows)")
    # hidden layers, through the exact dX of the output layer
    L2 = nb.LIP2[mlp.act]
    for l in range(DEPTH - 1, -1, -1):
        Z = Zs[l]
        df = dact(mlp.act, Z)
        dZ = dX * df
        adX = np.abs(dX) + e_dX
        e_dZ = e_dX * np.abs(df) + adX * L2 * e_zs[l] + 4 * nb.U32 * adX * (1 + np.abs(Z)) + nb.U32 * np.abs(dZ)
        e_dZr = e_dZ + nb.U * (np.abs(dZ) + e_dZ)
        Xl, ex = np.abs(Xs[l]), e_xs[l]
        w_off, b_off, fout, fin = layers[l]
        nb.check(g[b_off:b_off + fout], dZ.sum(axis=0), e_dZ.sum(axis=0) + nb.gam(B) * np.abs(dZ).sum(axis=0),
                 f"db layer {l}")
        eW = e_dZr.T @ (Xl + ex) + np.abs(dZ).T @ ex + nb.gam(B) * ((np.abs(dZ) + e_dZr).T @ (Xl + ex))
        nb.check(g[w_off:w_off + fout * fin].reshape(fout, fin), dZ.T @ Xs[l], eW, f"dW layer {l}")
        if l > 0:
            Wl = mlp.Ws[l]
            aW = np.abs(Wl)
            dX = dZ @ Wl
            e_dX = e_dZr @ ((1 + nb.U) * aW) + np.abs(dZ) @ (nb.U * aW) + \
                nb.gam(WIDTH) * ((np.abs(dZ) + e_dZr) @ ((1 + nb.U) * aW))
    net.close()

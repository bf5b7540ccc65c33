"""GPU parity of the element network kernels against the FP64 oracle.

Weights, statistics and inputs are generated on the host (numpy, seeded) and
loaded into the library through the documented blob, so the oracle never
consumes anything the HIP path produced.  The oracle runs with bfloat16
rounding at the points where the kernels round (features, weights, hidden
activations, backpropagated products); the remaining difference is FP32
accumulation order, hence the tolerances below (written per test).

Each test also compares the kernels with the plain FP64 definition of the
network (no bfloat16 rounding anywhere) entry by entry, against the running
error bound of tests/_netbound.py built from the bfloat16 and FP32 unit
roundoffs.
"""
import numpy as np
import pytest
import torch

from oracle.local import LocalDisc, local_solve_batch
from oracle.mlp import MLP, bf16_round, features
from paper_2308_02467_amd import inputs

from _util import rel_err
import _netbound as nb

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02467_amd import el
    c = el.Context(0)
    yield c
    c.close()


def _host_net(rng, n_in, width, depth, n_out, act=0):
    """theta, statistics and the oracle MLP built on the host."""
    from paper_2308_02467_amd import el
    k0, layers, P = el.net_layout(n_in, width, depth, n_out)
    theta = np.zeros(P, np.float32)
    Ws, bs = [], []
    for l, (w_off, b_off, fout, fin) in enumerate(layers):
        fan = n_in if l == 0 else width
        W = np.zeros((fout, fin), np.float32)
        W[:, :fan] = rng.uniform(-1, 1, (fout, fan)) / np.sqrt(fan)
        b = (rng.uniform(-1, 1, fout) / np.sqrt(fan)).astype(np.float32)
        theta[w_off:w_off + fout * fin] = W.reshape(-1)
        theta[b_off:b_off + fout] = b
        Ws.append(W.astype(np.float64))
        bs.append(b.astype(np.float64))
    fm = rng.uniform(-2, 0, n_in).astype(np.float32)
    fs = rng.uniform(0.5, 2, n_in).astype(np.float32)
    ym = rng.uniform(-0.1, 0.1, n_out).astype(np.float32)
    ys = rng.uniform(0.01, 0.2, n_out).astype(np.float32)
    return dict(k0=k0, P=P, theta=theta, fm=fm, fs=fs, ym=ym, ys=ys,
                oracle=MLP(Ws, bs, {0: "gelu", 1: "elu", 2: "linear"}[act]))


def _load(ctx, hn, n_in, width, depth, n_out, act=0, box=(0, 1e9, 0, 1e9, 0, 1e9)):
    from paper_2308_02467_amd import el
    blob = el.pack_net_blob(n_in, width, depth, act, n_out, hn["theta"], hn["fm"], hn["fs"], hn["ym"], hn["ys"], box)
    return el.Net.load(ctx, blob)


def _raw_inputs(rng, B, nn):
    h = rng.uniform(0.005, 0.1, (B, 1))
    return np.concatenate([h, rng.uniform(0.01, 3, (B, nn)), rng.uniform(0.05, 30, (B, nn))], axis=1)


@pytest.fixture
def gemm_tile():
    """Pins the GEMM block tile for one test and restores the autotuner."""
    from paper_2308_02467_amd import el
    yield el.gemm_tile
    el.gemm_tile(-1)


# tile -1: the autotuner's choice; 3: the 256 x 256 direct-to-LDS tile for
# every GEMM that can take it (k-contiguous operands, K % 64 == 0)
LDS_TILES = [3]


@pytest.mark.parametrize("tile", [-1] + LDS_TILES)
@pytest.mark.parametrize("n_in,width,depth,n_out,act,B", [(9, 64, 2, 96, 0, 6), (19, 128, 3, 200, 1, 6),
                                                           (99, 1024, 4, 1024, 0, 6), (99, 256, 1, 225792, 0, 6),
                                                           (99, 256, 2, 1000, 0, 700), (19, 128, 3, 200, 2, 6)])
def test_forward_parity(ctx, gemm_tile, tile, n_in, width, depth, n_out, act, B):
    rng = np.random.default_rng(n_in + width)
    hn = _host_net(rng, n_in, width, depth, n_out, act)
    net = _load(ctx, hn, n_in, width, depth, n_out, act)
    x = _raw_inputs(rng, B, (n_in - 1) // 2).astype(np.float32)
    y = torch.empty((B, n_out), dtype=torch.float32, device=DEV)
    gemm_tile(tile)
    print(f"[el_net_forward] {n_in}-{width}x{depth}-{n_out} B={B} tile={tile}", flush=True)
    net.forward(torch.from_numpy(x).to(DEV), y)
    X0 = features(x.astype(np.float64), hn["fm"].astype(np.float64), hn["fs"].astype(np.float64), hn["k0"])
    ref, _ = hn["oracle"].forward(X0, bf16=True)
    got = y.cpu().numpy()
    print(f"[el_net_forward] vs the bfloat16-rounded oracle: {rel_err(got, ref):.3e}", flush=True)
    assert rel_err(got, ref) <= 2e-3
    # the plain FP64 definition, per entry
    e0 = nb.feature_bound(x, hn["fm"].astype(np.float64), hn["fs"].astype(np.float64), hn["k0"])
    out, _, _, e_out, _, _ = nb.forward_bounds(hn["oracle"], X0, e0)
    nb.check(got, out, e_out + nb.U32 * (np.abs(out) + e_out), "el_net_forward vs FP64")
    net.close()


@pytest.mark.parametrize("tile", [-1] + LDS_TILES)
def test_gradients_and_adam(ctx, gemm_tile, tile):
    from paper_2308_02467_amd import el
    n_in, width, depth, n_out, B = 9, 64, 3, 128, 48
    rng = np.random.default_rng(11)
    hn = _host_net(rng, n_in, width, depth, n_out)
    net = _load(ctx, hn, n_in, width, depth, n_out)
    gemm_tile(tile)
    x = _raw_inputs(rng, B, 4).astype(np.float32)
    y_raw = rng.uniform(-0.5, 0.5, (B, n_out))
    y16 = torch.from_numpy(y_raw.astype(np.float32)).to(torch.bfloat16)
    yb = y16.to(torch.float64).numpy()
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    print("[el_train_step] lr=0", flush=True)
    net.train_step(torch.from_numpy(x).to(DEV), y16.to(DEV), 0.0, loss)
    g = net.params(1).cpu().numpy().astype(np.float64) / (B * n_out)
    X0 = features(x.astype(np.float64), hn["fm"].astype(np.float64), hn["fs"].astype(np.float64), hn["k0"])
    tgt = (yb - hn["ym"].astype(np.float64)) / hn["ys"].astype(np.float64)
    lo, gW, gb = hn["oracle"].mae_grad(X0, tgt, bf16=True)
    assert abs(loss.item() - lo) <= 1e-4 * lo
    _, layers, _ = el.net_layout(n_in, width, depth, n_out)
    for l, (w_off, b_off, fout, fin) in enumerate(layers):
        assert rel_err(g[w_off:w_off + fout * fin], gW[l].reshape(-1)) <= 2e-3, l
        assert rel_err(g[b_off:b_off + fout], gb[l]) <= 2e-3, l
    th0 = net.params(0).cpu().numpy()
    assert np.array_equal(th0, hn["theta"])            # lr = 0 keeps the weights
    # one Adam step from the zero state: theta1 = theta0 - lr g / (|g| + eps)
    net2 = _load(ctx, hn, n_in, width, depth, n_out)
    net2.train_step(torch.from_numpy(x).to(DEV), y16.to(DEV), 1e-3)
    th1 = net2.params(0).cpu().numpy().astype(np.float64)
    gor = np.zeros_like(g)
    for l, (w_off, b_off, fout, fin) in enumerate(layers):
        gor[w_off:w_off + fout * fin] = gW[l].reshape(-1)
        gor[b_off:b_off + fout] = gb[l]
    big = np.abs(gor) > 1e-3 * np.abs(gor).max()
    step = th1 - th0
    expected = -1e-3 * gor / (np.abs(gor) + 1e-8)          # first Adam step, bias-corrected
    assert np.allclose(step[big], expected[big], rtol=0, atol=2e-7)
    net.close()
    net2.close()


@pytest.mark.parametrize("tile", [-1] + LDS_TILES)
@pytest.mark.parametrize("n_in,width,depth,n_out,act,B", [(9, 64, 3, 128, 0, 48), (19, 128, 2, 520, 1, 200),
                                                           (99, 256, 2, 1000, 0, 300), (99, 192, 2, 1000, 0, 300),
                                                           (99, 128, 2, 640, 0, 128)])
def test_gradients_fp64_definition(ctx, gemm_tile, tile, n_in, width, depth, n_out, act, B):
    """Gradients of one training step against the plain FP64 definition
    (oracle.mlp without rounding), entry by entry within the running error
    bound.  The targets lie at least 50 normalized units away from any
    output, so the MAE subgradient sign(pred - target) is the same on both
    sides (the outputs are O(1)).  Tile 3 runs the output layer's MAE
    epilogue with its targets staged in LDS: one k tile (width 64), an odd
    number of k tiles (width 192) and ragged row and column tiles.  With
    batch, outputs and width multiples of 64 (the last case) the output
    layer's dW reads the sign matrix that the MAE epilogue writes
    transposed."""
    from paper_2308_02467_amd import el
    gemm_tile(tile)
    rng = np.random.default_rng(100 + n_out)
    hn = _host_net(rng, n_in, width, depth, n_out, act)
    net = _load(ctx, hn, n_in, width, depth, n_out, act)
    x = _raw_inputs(rng, B, (n_in - 1) // 2).astype(np.float32)
    sgn = rng.choice([-1.0, 1.0], (B, n_out))
    tn = sgn * rng.uniform(50.0, 100.0, (B, n_out))                   # normalized targets
    y16 = torch.from_numpy((tn * hn["ys"][None, :] + hn["ym"][None, :]).astype(np.float32)).to(torch.bfloat16)
    print(f"[el_train_step] FP64 definition {n_in}-{width}x{depth}-{n_out} B={B}", flush=True)
    net.train_step(torch.from_numpy(x).to(DEV), y16.to(DEV), 0.0)
    g = net.params(1).cpu().numpy().astype(np.float64)              # loss units
    X0 = features(x.astype(np.float64), hn["fm"].astype(np.float64), hn["fs"].astype(np.float64), hn["k0"])
    e0 = nb.feature_bound(x, hn["fm"].astype(np.float64), hn["fs"].astype(np.float64), hn["k0"])
    out, Xs, Zs, _, e_xs, e_zs = nb.forward_bounds(hn["oracle"], X0, e0)
    assert np.abs(out).max() < 40.0
    dY = -sgn                                                          # sign(pred - target)
    gW, gb, eW, eb = nb.grad_bounds(hn["oracle"], Xs, Zs, e_xs, e_zs, dY)
    _, layers, _ = el.net_layout(n_in, width, depth, n_out)
    for l, (w_off, b_off, fout, fin) in enumerate(layers):
        nb.check(g[w_off:w_off + fout * fin].reshape(fout, fin), gW[l], eW[l], f"dW layer {l}")
        nb.check(g[b_off:b_off + fout], gb[l], eb[l], f"db layer {l}")
    net.close()


def test_tuning_cache_replaces_timing(ctx, tmp_path):
    """Choices saved by one process and loaded into a fresh autotuner give
    the same tiles without timing: bit-identical forward outputs, and the
    report marks every choice as taken from the file."""
    from paper_2308_02467_amd import el
    n_in, width, depth, n_out, B = 99, 256, 2, 1000, 700
    rng = np.random.default_rng(31)
    hn = _host_net(rng, n_in, width, depth, n_out)
    net = _load(ctx, hn, n_in, width, depth, n_out)
    x = torch.from_numpy(_raw_inputs(rng, B, (n_in - 1) // 2).astype(np.float32)).to(DEV)
    y1 = torch.empty((B, n_out), dtype=torch.float32, device=DEV)
    y2 = torch.empty_like(y1)
    el.tuning_reset()
    net.forward(x, y1)
    timed = el.tuning_report()
    print("[tuning] timed:\n" + timed, flush=True)
    keys = [l.split(" -> ")[0] for l in timed.splitlines()]
    arch = torch.cuda.get_device_properties(DEV).gcnArchName.split(":")[0]
    assert keys and all(k.split()[0] == arch for k in keys)
    f = tmp_path / "tune.txt"
    el.tuning_save(f)
    el.tuning_reset()
    assert el.tuning_load(f) == len(keys)
    net.forward(x, y2)
    loaded = el.tuning_report()
    assert [l.split(" (")[0] for l in loaded.splitlines()] == [l.split(" (")[0] for l in timed.splitlines()]
    assert all(l.endswith("(from a cache file)") for l in loaded.splitlines())
    assert torch.equal(y1, y2)
    el.tuning_reset()
    net.close()


def test_save_load_and_bitwise_resume(ctx):
    from paper_2308_02467_amd import el
    n_in, width, depth, n_out, B = 9, 64, 2, 64, 32
    rng = np.random.default_rng(5)
    hn = _host_net(rng, n_in, width, depth, n_out)
    xs = [torch.from_numpy(_raw_inputs(rng, B, 4).astype(np.float32)).to(DEV) for _ in range(4)]
    ys = [torch.from_numpy(rng.uniform(-0.3, 0.3, (B, n_out)).astype(np.float32)).to(torch.bfloat16).to(DEV)
          for _ in range(4)]
    a = _load(ctx, hn, n_in, width, depth, n_out)
    for i in range(4):
        a.train_step(xs[i], ys[i], 1e-3)
    b = _load(ctx, hn, n_in, width, depth, n_out)
    for i in range(2):
        b.train_step(xs[i], ys[i], 1e-3)
    blob = b.save()
    b.close()
    c = el.Net.load(ctx, blob)
    assert el.unpack_net_blob(blob)["step"] == 2
    for i in range(2, 4):
        c.train_step(xs[i], ys[i], 1e-3)
    for which in (0, 2, 3):
        assert torch.equal(a.params(which), c.params(which)), which
    a.close()
    c.close()


def test_make_pairs_match_oracle(ctx):
    from paper_2308_02467_amd import el
    p, n_a = 3, 8
    o = LocalDisc(p, n_a)
    h, kap, sig = inputs.training_draws(40, o.xi, seed=9)
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    y = torch.empty((40, m * m + n * m), dtype=torch.bfloat16, device=DEV)
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=DEV)
    print("[el_make_pairs]", flush=True)
    el.el_make_pairs(ctx, d, T(h), T(kap), T(sig), y)
    i2o, i2s, _ = local_solve_batch(o, h, kap, sig)
    ref = np.concatenate([i2o.reshape(40, -1), i2s.reshape(40, -1)], axis=1)
    got = y.to(torch.float64).cpu().numpy()
    # both sides round their FP64 value to bfloat16: at most one bfloat16 ulp apart
    assert np.all(np.abs(got - bf16_round(ref)) <= 2.0 ** -7 * np.abs(ref) + 1e-30)
    assert np.mean(got == bf16_round(ref)) > 0.99


# rounding of the stored operators: relative bound and the smallest spacing
# (binary16 subnormals)
ROUND = {torch.bfloat16: (2.0 ** -7, 1e-30), torch.float16: (2.0 ** -10, 2.0 ** -24), torch.float32: (1e-6, 1e-30)}
NP_ROUND = {torch.bfloat16: bf16_round,
            torch.float16: lambda a: a.astype(np.float16).astype(np.float64),
            torch.float32: lambda a: a.astype(np.float32).astype(np.float64)}


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32, torch.float16])
def test_infer_range_mask_and_fallback(ctx, dtype):
    from paper_2308_02467_amd import el
    p, n_a = 2, 4
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    n_in, n_out = 1 + 2 * nn, m * m + n * m
    rng = np.random.default_rng(21)
    hn = _host_net(rng, n_in, 64, 2, n_out)
    box = (0.01, 0.05, 0.02, 2.0, 0.1, 20.0)
    net = _load(ctx, hn, n_in, 64, 2, n_out, box=box)
    E = 50
    o = LocalDisc(p, n_a)
    hh = rng.uniform(0.012, 0.048, E)
    kap = rng.uniform(0.03, 1.9, (E, nn))
    sig = rng.uniform(0.2, 19, (E, nn))
    out_idx = [3, 17, 40]
    sig[3, 2] = 30.0                 # sigma above the box
    kap[17, 0] = 0.0                 # kappa below the box
    hh[40] = 0.2                     # h above the box
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=DEV)
    i2o = torch.empty((E, m, m), dtype=dtype, device=DEV)
    i2s = torch.empty((E, n, m), dtype=dtype, device=DEV)
    mask = torch.empty(E, dtype=torch.uint8, device=DEV)
    rnd = NP_ROUND[dtype]
    print(f"[el_infer] with fallback {dtype}", flush=True)
    nfb = net.infer(d, T(hh), T(kap), T(sig), i2o, i2s, mask, fallback=True)
    assert nfb == 3
    exp_mask = np.ones(E, np.uint8)
    exp_mask[out_idx] = 0
    assert np.array_equal(mask.cpu().numpy(), exp_mask)
    # fallback elements: plain FP64 local solve rounded to the storage type
    # (the kernel rounds through FP32: at most one unit apart)
    r_o, r_s, _ = local_solve_batch(o, hh[out_idx], kap[out_idx], sig[out_idx])
    got_o = i2o.to(torch.float64).cpu().numpy()[out_idx]
    rel, tiny = ROUND[dtype]
    assert np.all(np.abs(got_o - rnd(r_o)) <= rel * np.abs(r_o) + tiny)
    if dtype == torch.float32:
        assert rel_err(got_o, r_o) <= 1e-6
    # in-range elements: de-normalized network output rounded to bfloat16
    x = np.concatenate([hh[:, None], kap, sig], axis=1)
    X0 = features(x, hn["fm"].astype(np.float64), hn["fs"].astype(np.float64), hn["k0"])
    yn, _ = hn["oracle"].forward(X0, bf16=True)
    yv = yn * hn["ys"].astype(np.float64) + hn["ym"].astype(np.float64)
    keep = exp_mask.astype(bool)
    got = np.concatenate([i2o.to(torch.float64).cpu().numpy().reshape(E, -1),
                          i2s.to(torch.float64).cpu().numpy().reshape(E, -1)], axis=1)
    _infer_checks(hn, x, X0, got, yv, keep, dtype)
    net.close()


def bf16_mode_check(got, ref, u_st, tiny, what):
    """Entries within one storage rounding + 2e-4 of the largest entry of the
    bfloat16-rounded oracle, but for at most 5 in 1000 (rounding-boundary
    flips of hidden activations; up to 8.4e-4 measured)."""
    d = np.abs(got - ref)
    lim = u_st * np.abs(ref) + 2e-4 * np.abs(ref).max() + tiny
    over = float(np.mean(d > lim))
    print(f"[{what}] vs the bfloat16-rounded oracle: max |err| {d.max():.3e} (largest entry "
          f"{np.abs(ref).max():.3e}); median |err| {np.median(d):.3e}; entries beyond one storage unit + 2e-4 of "
          f"the largest: {over:.2e}", flush=True)
    assert over <= 5e-3


def _infer_checks(hn, x, X0, got, yv_bf, keep, dtype):
    """In-range elements.  Against the bfloat16-rounded oracle: entries agree
    to one rounding to the storage type plus FP32 accumulation (2e-4 of the
    largest entry), except where a hidden activation fell on the other side
    of a bfloat16 rounding boundary in the two computations (then the
    difference is one bfloat16 unit of that activation times its weights):
    at most 5 in 1000 entries.  Against the plain FP64 definition: every
    entry within the running error bound."""
    ys, ym = hn["ys"].astype(np.float64), hn["ym"].astype(np.float64)
    u_st = {torch.float32: nb.U32, torch.float16: 2.0 ** -11, torch.bfloat16: nb.U}[dtype]
    tiny = 2.0 ** -25 if dtype == torch.float16 else 0.0
    bf16_mode_check(got[keep], yv_bf[keep], u_st, tiny, "el_infer")
    e0 = nb.feature_bound(x[keep], hn["fm"].astype(np.float64), hn["fs"].astype(np.float64), hn["k0"])
    out, _, _, e_out, _, _ = nb.forward_bounds(hn["oracle"], X0[keep], e0)
    y64 = out * ys[None, :] + ym[None, :]
    e_y = nb.denorm_bound(out, e_out, ys, ym)
    nb.check(got[keep], y64, e_y * (1 + u_st) + u_st * np.abs(y64) + tiny, f"el_infer {dtype} vs FP64")


def test_training_learns_the_operator(ctx):
    """Small discretization (p = 1, N_a = 4): after training on pairs from the
    local solver, held-out operators are far closer to the plain solver's than
    those of the untrained network or of the mean operator."""
    from paper_2308_02467_amd import el
    p, n_a = 1, 4
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    n_in, n_out = 1 + 2 * nn, m * m + n * m
    o = LocalDisc(p, n_a)
    N, Nt = 16384, 512
    h, kap, sig = inputs.training_draws(N + Nt, o.xi, seed=1234)
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=DEV)
    y = torch.empty((N + Nt, n_out), dtype=torch.bfloat16, device=DEV)
    print("[train] pairs", flush=True)
    el.el_make_pairs(ctx, d, T(h), T(kap), T(sig), y)
    x = torch.as_tensor(np.concatenate([h[:, None], kap, sig], axis=1), dtype=torch.float32, device=DEV)
    net = el.Net.create(ctx, n_in, 128, 3, n_out, seed=0)
    net.fit_normalization(x[:N].contiguous(), y[:N].contiguous())

    def test_err():
        yy = torch.empty((Nt, n_out), dtype=torch.float32, device=DEV)
        net.forward(x[N:].contiguous(), yy)
        u = el.unpack_net_blob(net.save())
        pred = yy.cpu().numpy() * u["y_std"] + u["y_mean"]
        true = y[N:].to(torch.float32).cpu().numpy()
        mean_err = np.linalg.norm(u["y_mean"][None, :] - true) / np.linalg.norm(true)
        return np.linalg.norm(pred - true) / np.linalg.norm(true), mean_err

    e0, emean = test_err()
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    B = 512
    print("[train] steps", flush=True)
    for epoch in range(12):
        for b0 in range(0, N, B):
            net.train_step(x[b0:b0 + B], y[b0:b0 + B], 1e-3, loss)
    e1, _ = test_err()
    print(f"[train] untrained {e0:.3e}, mean operator {emean:.3e}, trained {e1:.3e}", flush=True)
    assert e1 < 0.2 * emean and e1 < 0.1 * e0
    net.close()


def test_make_pairs_in2mean_form(ctx):
    """Targets (in2out, in2mean): the oracle's in2mean rounded to bfloat16."""
    from paper_2308_02467_amd import el
    p, n_a = 3, 8
    o = LocalDisc(p, n_a)
    h, kap, sig = inputs.training_draws(24, o.xi, seed=19)
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    y = torch.empty((24, m * m + nn * m), dtype=torch.bfloat16, device=DEV)
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=DEV)
    print("[el_make_pairs] in2mean form", flush=True)
    el.el_make_pairs(ctx, d, T(h), T(kap), T(sig), y, form=el.EL_FORM_IN2MEAN)
    i2o, _, i2m = local_solve_batch(o, h, kap, sig)
    ref = np.concatenate([i2o.reshape(24, -1), i2m.reshape(24, -1)], axis=1)
    got = y.to(torch.float64).cpu().numpy()
    assert np.all(np.abs(got - bf16_round(ref)) <= 2.0 ** -7 * np.abs(ref) + 1e-30)
    assert np.mean(got == bf16_round(ref)) > 0.99


def test_infer_storage_types_are_the_rounded_float32_outputs(ctx):
    """The float16 and bfloat16 outputs of el_infer are its float32 outputs
    rounded to nearest: one GEMM, rounded in the epilogue."""
    from paper_2308_02467_amd import el
    p, n_a = 2, 4
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    n_in, n_out = 1 + 2 * nn, m * m + n * m
    rng = np.random.default_rng(29)
    hn = _host_net(rng, n_in, 64, 2, n_out)
    net = _load(ctx, hn, n_in, 64, 2, n_out)
    E = 37
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=DEV)
    hh = T(rng.uniform(0.012, 0.048, E))
    kap = T(rng.uniform(0.03, 1.9, (E, nn)))
    sig = T(rng.uniform(0.2, 19, (E, nn)))
    outs = {}
    for dt in (torch.float32, torch.float16, torch.bfloat16):
        i2o = torch.empty((E, m, m), dtype=dt, device=DEV)
        i2s = torch.empty((E, n, m), dtype=dt, device=DEV)
        print(f"[el_infer] {dt}", flush=True)
        net.infer(d, hh, kap, sig, i2o, i2s, None, fallback=False)
        outs[dt] = (i2o, i2s)
    for dt in (torch.float16, torch.bfloat16):
        for got, f32 in zip(outs[dt], outs[torch.float32]):
            # equal, except where the float32 output is a tie between two
            # 16-bit neighbours (the epilogue's value may differ from it in
            # the last float32 bit: its multiply-add is fused differently)
            ref = f32.to(dt)
            bad = got != ref
            assert torch.all(got[bad].double() + ref[bad].double() == 2 * f32[bad].double())
            assert int(bad.sum()) <= 1e-3 * bad.numel()
    net.close()


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32, torch.float16])
def test_infer_in2mean_form_with_fallback(ctx, dtype):
    """A network in the in2mean form writes (in2out, in2mean); elements
    outside the training box get the plain solver's in2out and in2mean."""
    from paper_2308_02467_amd import el
    p, n_a = 2, 4
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    n_in, n_out = 1 + 2 * nn, m * m + nn * m
    rng = np.random.default_rng(23)
    hn = _host_net(rng, n_in, 64, 2, n_out)
    box = (0.01, 0.05, 0.02, 2.0, 0.1, 20.0)
    net = _load(ctx, hn, n_in, 64, 2, n_out, box=box)
    E = 30
    o = LocalDisc(p, n_a)
    hh = rng.uniform(0.012, 0.048, E)
    kap = rng.uniform(0.03, 1.9, (E, nn))
    sig = rng.uniform(0.2, 19, (E, nn))
    out_idx = [4, 22]
    sig[4, 1] = 40.0
    hh[22] = 0.3
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=DEV)
    i2o = torch.empty((E, m, m), dtype=dtype, device=DEV)
    i2m = torch.empty((E, nn, m), dtype=dtype, device=DEV)
    print(f"[el_infer] in2mean form {dtype}", flush=True)
    nfb = net.infer(d, T(hh), T(kap), T(sig), i2o, in2mean=i2m, fallback=True)
    assert nfb == 2
    r_o, _, r_m = local_solve_batch(o, hh[out_idx], kap[out_idx], sig[out_idx])
    tol, tiny = ROUND[dtype]
    got_m = i2m.to(torch.float64).cpu().numpy()[out_idx]
    got_o = i2o.to(torch.float64).cpu().numpy()[out_idx]
    assert np.all(np.abs(got_m - r_m) <= tol * np.abs(r_m) + tiny)
    assert np.all(np.abs(got_o - r_o) <= tol * np.abs(r_o) + tiny)
    x = np.concatenate([hh[:, None], kap, sig], axis=1)
    X0 = features(x, hn["fm"].astype(np.float64), hn["fs"].astype(np.float64), hn["k0"])
    yn, _ = hn["oracle"].forward(X0, bf16=True)
    yv = yn * hn["ys"].astype(np.float64) + hn["ym"].astype(np.float64)
    keep = np.ones(E, bool)
    keep[out_idx] = False
    got = np.concatenate([i2o.to(torch.float64).cpu().numpy().reshape(E, -1),
                          i2m.to(torch.float64).cpu().numpy().reshape(E, -1)], axis=1)
    _infer_checks(hn, x, X0, got, yv, keep, dtype)
    net.close()

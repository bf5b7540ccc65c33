"""The allocation-free inference entry point (el_infer_noalloc) against
el_infer without fallback: same inputs, two calls in a row, the second with a
smaller batch, in both operator forms.  The two paths share their kernels;
with el_infer's GEMM tile pinned to the one the allocation-free path uses
(the 256 x 256 direct-to-LDS tile, which every GEMM of this network can
take) the outputs are bit-identical.  The context's workspace does not grow."""
import numpy as np
import pytest
import torch

from paper_2308_02467_amd import inputs

from test_gpu_net import _host_net, _load

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_02467_amd import el
    c = el.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("form", ["in2sol", "in2mean"])
def test_infer_noalloc_matches_infer(ctx, form):
    from paper_2308_02467_amd import el
    p, n_a, width, depth = 3, 8, 1024, 4
    d = el.disc(p, n_a)
    nn, n, m = el.disc_sizes(d)
    rows = n if form == "in2sol" else nn
    n_in, n_out = 1 + 2 * nn, m * m + rows * m
    hn = _host_net(np.random.default_rng(31), n_in, width, depth, n_out, 0)
    net = _load(ctx, hn, n_in, width, depth, n_out)
    xi, _ = el.lgl(p)
    el.gemm_tile(3)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)
    # 9,000 elements: two passes of the static scratch (7,936 elements per
    # pass for this network); then 1,300 elements: one pass
    for call, E in enumerate((9000, 1300)):
        h, kap, sig = inputs.training_draws(E, xi, seed=40 + call)
        H, K, S = T(h), T(kap), T(sig)
        ref_o = torch.empty((E, m, m), dtype=torch.float32, device=DEV)
        ref_v = torch.empty((E, rows, m), dtype=torch.float32, device=DEV)
        vol = {"in2sol": None, "in2mean": None}
        vol[form] = ref_v
        net.infer(d, H, K, S, ref_o, fallback=False, **vol)
        mask_ref = torch.empty(E, dtype=torch.uint8, device=DEV)
        net.infer(d, H, K, S, None, in_range=mask_ref, fallback=False, **vol)
        ws0 = ctx.workspace_bytes()
        got_o = torch.full((E, m, m), float("nan"), dtype=torch.float32, device=DEV)
        got_v = torch.full((E, rows, m), float("nan"), dtype=torch.float32, device=DEV)
        mask = torch.full((E,), 7, dtype=torch.uint8, device=DEV)
        vol[form] = got_v
        print(f"[el_infer_noalloc] call {call}: E={E} form={form}", flush=True)
        net.infer_noalloc(d, H, K, S, got_o, in_range=mask, **vol)
        torch.cuda.synchronize()
        assert ctx.workspace_bytes() == ws0
        assert torch.equal(mask, mask_ref)
        for got, ref in ((got_o, ref_o), (got_v, ref_v)):
            assert bool(torch.isfinite(got).all())
            diff = (got.double() - ref.double()).abs()
            print(f"[el_infer_noalloc] max |diff| / max |ref| = {float(diff.max() / ref.double().abs().max()):.3e}, "
                  f"bit-identical entries {float((got == ref).double().mean()):.6f}", flush=True)
            assert torch.equal(got, ref)
    el.gemm_tile(-1)
    net.close()

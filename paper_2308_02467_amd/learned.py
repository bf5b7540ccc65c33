"""Learned local solve ("element learning", Sec. 2.4 and 3.1) on the GPU.

* ``training_set``: seeded element draws (inputs.training_draws) and their
  operators from the FP64 GPU local solver (el_make_pairs), stored as
  bfloat16 targets (in2out followed by in2sol) on the device;
* ``train``: epochs of el_train_step over contiguous batches in a seeded
  random batch order;
* ``learned_solve``: el_infer (with plain fallback outside the training box)
  -> el_trace_solve -> el_recover.

Every numerical step runs in the library's HIP kernels; this module only
sequences calls and holds device buffers.
"""
import sys
import time

import numpy as np
import torch

from . import el, inputs


def training_set(ctx, d, N, seed=1234, chunk=8192, log=True, form=el.EL_FORM_IN2SOL, draws=None):
    """(x [N, 1+2nn] float32 raw inputs, y [N, n_out] bfloat16 targets), on the device.
    form: targets (in2out, in2sol) or (in2out, in2mean).  draws: optional
    (h, kappa, sigma) arrays replacing the default training distribution."""
    nn, n, m = el.disc_sizes(d)
    n_out = m * m + (n if form == el.EL_FORM_IN2SOL else nn) * m
    xi, _ = el.lgl(d.p)
    h, kap, sig = inputs.training_draws(N, xi, seed=seed) if draws is None else draws
    dev = torch.device(f"cuda:{ctx.device}")
    x = torch.as_tensor(np.concatenate([h[:, None], kap, sig], axis=1), dtype=torch.float32, device=dev)
    y = torch.empty((N, n_out), dtype=torch.bfloat16, device=dev)
    H = torch.as_tensor(h, dtype=torch.float64, device=dev)
    K = torch.as_tensor(kap, dtype=torch.float64, device=dev)
    S = torch.as_tensor(sig, dtype=torch.float64, device=dev)
    for c0 in range(0, N, chunk):
        c1 = min(N, c0 + chunk)
        el.el_make_pairs(ctx, d, H[c0:c1], K[c0:c1], S[c0:c1], y[c0:c1], form=form)
        if log:
            print(f"[learned] training pairs {c1}/{N}", file=sys.stderr, flush=True)
    return x, y


def train(net, x, y, epochs, batch=4096, lr=1e-3, seed=0, log=True, time_limit=None, decay_at=0.0,
          schedule=None, log_every=1, step=None):
    """Adam on the MAE loss; returns the per-epoch mean loss (normalized units).
    decay_at in (0, 1): lr is divided by 10 after that fraction of the epochs
    (or of the time limit), as in the paper's stepwise schedule (Sec. 3.1).
    schedule: a list of (epochs, lr) segments run one after the other (it
    replaces epochs, lr and decay_at), e.g. the paper's 3000 epochs each at
    1e-3, 1e-4 and 1e-5.  step: the training step to call (default
    net.train_step, bfloat16 targets; net.train_step_f32 takes float32
    targets)."""
    N = x.shape[0]
    nb = N // batch
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=x.device)
    acc = torch.zeros(1, dtype=torch.float32, device=x.device)
    hist = []
    t0 = time.perf_counter()
    lrs = None
    if schedule is not None:
        lrs = [l for (n_ep, l) in schedule for _ in range(n_ep)]
        epochs = len(lrs)
    for ep in range(epochs):
        acc.zero_()
        elapsed = time.perf_counter() - t0
        late = decay_at > 0 and (ep >= decay_at * epochs or (time_limit and elapsed >= decay_at * time_limit))
        lr_ep = lrs[ep] if lrs is not None else (lr * 0.1 if late else lr)
        for b in rng.permutation(nb):
            b0 = int(b) * batch
            (step or net.train_step)(x[b0:b0 + batch], y[b0:b0 + batch], lr_ep, loss)
            acc += loss
        hist.append(acc.item() / nb)
        if log and ((ep + 1) % log_every == 0 or ep + 1 == epochs):
            print(f"[learned] epoch {ep + 1}/{epochs} loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)",
                  file=sys.stderr, flush=True)
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
    return hist

"""The residual-implied error bound the FP32 + refinement parity tests use
(tests/_util.refinement_bounds), checked on the CPU against solutions with
known perturbations: it must hold, and it must not be vacuous."""
import numpy as np
import pytest

from oracle.local import LocalDisc
from paper_2308_02467_amd import inputs

from _util import refinement_bounds


@pytest.mark.parametrize("p,n_a,g", [(3, 8, 0.0), (2, 12, 0.85)])
def test_bound_holds_and_is_informative(p, n_a, g):
    o = LocalDisc(p, n_a, g)
    E = 4
    h, kap, sig = inputs.training_draws(E, o.xi, seed=5)
    rng = np.random.default_rng(1)
    Bh = o.matrix_Bhat()
    for scale in (1e-12, 1e-9, 1e-6):
        xs, outs, rr = [], [], np.empty(E)
        for e in range(E):
            A = o.local_matrix(*o.scaled_coefficients(h[e], kap[e], sig[e]))
            X = np.linalg.solve(A, -Bh)
            Xp = X + scale * np.abs(X).max() * rng.standard_normal(X.shape)
            R = -Bh - A @ Xp
            rr[e] = np.max(np.abs(R).max(axis=0) / np.abs(Bh).max(axis=0))
            xs.append(X)
            outs.append(Xp)
        ref = {"in2sol": np.stack(xs)}
        bnd = refinement_bounds(o, h, kap, sig, rr, ref)["in2sol"]
        err = np.array([np.abs(outs[e] - xs[e]).max() / np.abs(xs[e]).max() for e in range(E)])
        assert np.all(err <= bnd), (scale, err, bnd)
        # not vacuous: within a factor of the conditioning of these small systems
        assert np.all(bnd <= 1e4 * err), (scale, err, bnd)

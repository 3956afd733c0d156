"""GPU battery outputs (U_cell, volume means, conservation sums) vs the oracle."""
import numpy as np
import pytest

import synth
from oracle import model as om
from oracle import outputs as oout
from tests.helpers import problem_and_context

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("shape,seed,t", [((6, 5, 4), 1, 0.0), ((16, 16, 16), 2, 2.5), ((9, 7, 3), 3, 30.0)])
def test_outputs_match_oracle(shape, seed, t):
    nx, ny, nz = shape
    P, ctx, mask = problem_and_context(nx, ny, nz, mask_seed=seed, param_seed=seed, f_C=1.0)
    u = synth.random_state(P.n_elem, P.n_nodes, seed, phase=mask, phi_spread=5e-3)
    print(f"[outputs] {shape} seed {seed} t {t}", flush=True)
    got = ctx.outputs(torch.tensor(u, device="cuda:0"), t)
    U = oout.cell_voltage(P, u)
    means, cS = oout.volume_means(P, u)
    sums = np.array(oout.invariants(P, u, t))
    assert abs(got["U_cell"] - U) <= 1e-13 * abs(U)
    np.testing.assert_allclose(got["means"][:9], means, rtol=1e-13, atol=0)
    assert abs(got["means"][9] - cS) <= 1e-13 * cS
    np.testing.assert_allclose(got["sums"][:3], sums[:3], rtol=1e-13, atol=0)
    # the reaction current is a sum of signed terms: relative to its largest part
    assert abs(got["sums"][3] - sums[3]) <= 1e-12 * max(abs(sums[3]), 1e-30)

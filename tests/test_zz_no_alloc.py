"""dg_outputs_noalloc, the outputs entry point for callers that cannot
allocate, against dg_outputs (GPU).

Two calls in a row on one GPU, the second on a smaller mesh (so the shared
device scratch holds the first call's partial sums when the second starts):
each result equals dg_outputs on the same state bit for bit (the same
kernel, and the block partials summed in the same order), and the first
call in the process changes the device's free memory by nothing.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(nx, ny, nz, seed):
    from paper_2511_05233_amd import lsbdg
    mask = synth.porosity_mask((nz, ny, nx), 0.6, seed)
    D0, i0 = synth.sample_transport_kinetics(seed)
    ctx = lsbdg.Context(nx, ny, nz, 1e-6, 1, mask, D0=D0, kE=i0 / 96485.332, f_C=0.5)
    u = torch.tensor(synth.random_state(ctx.n_elem, 8, 40 + seed, phase=mask, phi_spread=5e-3),
                     device="cuda:0")
    return ctx, u


def test_noalloc_outputs_equal_dg_outputs_on_two_calls():
    big, ub = _case(20, 18, 17, 1)
    small, us = _case(5, 4, 3, 2)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    first = big.outputs(ub, 1.5, noalloc=True)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    second = small.outputs(us, 0.25, noalloc=True)
    print(f"[noalloc] free device memory before {free0}, after {free1}", flush=True)
    assert free1 == free0
    for got, (ctx, u, t) in ((first, (big, ub, 1.5)), (second, (small, us, 0.25))):
        ref = ctx.outputs(u, t)
        print(f"[noalloc] {ctx.nx}x{ctx.ny}x{ctx.nz}: U_cell {got['U_cell']!r} vs {ref['U_cell']!r}", flush=True)
        assert got["U_cell"] == ref["U_cell"]
        assert np.array_equal(got["means"], ref["means"])
        assert np.array_equal(got["sums"], ref["sums"])
    # the second, smaller call left no trace of the first: repeat the first
    again = big.outputs(ub, 1.5, noalloc=True)
    assert again["U_cell"] == first["U_cell"] and np.array_equal(again["sums"], first["sums"])
    big.close()
    small.close()

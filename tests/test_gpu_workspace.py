"""Contexts on a caller-owned device workspace (dg_workspace_bytes,
dg_setup_ws) (GPU).

A context set up on a workspace sized by dg_workspace_bytes takes every
device buffer from it: its initial state, implicit steps and controller
steps equal those of a library-allocating context bit for bit, the
device's free memory does not change across those calls, and uses the
workspace was not sized for fail with DG_ENOMEM naming the shortfall.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _make(ws=None, features=0, inner="f32", **opts):
    from paper_2511_05233_amd import lsbdg
    mask = synth.porosity_mask((3, 4, 5), 0.6, 1)
    D0, i0 = synth.sample_transport_kinetics(1)
    return lsbdg.Context(5, 4, 3, 1e-6, 1, mask, D0=D0, kE=i0 / 96485.332, f_C=0.1, workspace=ws,
                         features=features, ws_inner=inner, ws_opts=opts or None)


@pytest.mark.parametrize("inner", ["f32", "f64"])
def test_workspace_context_equals_allocating_context(inner):
    from paper_2511_05233_amd import lsbdg
    feats = lsbdg.DG_WS_STEP | lsbdg.DG_WS_NAIVE | lsbdg.DG_WS_OPERATORS
    n = lsbdg.workspace_bytes(5, 4, 3, 1e-6, 1, feats, inner=inner)
    print(f"[workspace] {inner}: {n} bytes", flush=True)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    ref = _make()
    ctx = _make(ws, feats, inner)
    # the library-allocating context first (its first calls allocate) ...
    u_ref, _ = ref.initial_state(inner=inner)
    u0 = u_ref.clone()
    r1 = ref.step(u_ref, 0.0, 0.1, inner=inner)
    u1 = u_ref.clone()
    c1 = lsbdg.controller("naive", dt0=0.05)
    t1, _ = ref.advance(c1, 0.1, u_ref, inner=inner)
    o1 = ref.outputs(u_ref, t1)
    # ... then the workspace context, which allocates nothing.  torch's first
    # comparison in a process loads its kernels, which takes device memory:
    # compare once beforehand so that only the library's calls are measured.
    u = torch.empty_like(u_ref)
    assert not torch.equal(u0, u1)

    def free():
        torch.cuda.synchronize()
        return torch.cuda.mem_get_info()[0]

    free0 = free()
    seen = {}
    ctx.initial_state(u=u, inner=inner)
    seen["initial_state"] = free()
    assert torch.equal(u, u0)
    r2 = ctx.step(u, 0.0, 0.1, inner=inner)
    seen["step"] = free()
    assert torch.equal(u, u1) and r1 == r2
    c2 = lsbdg.controller("naive", dt0=0.05)
    t2, _ = ctx.advance(c2, 0.1, u, inner=inner)
    seen["advance"] = free()
    assert t1 == t2 and torch.equal(u, u_ref)
    o2 = ctx.outputs(u, t2)
    seen["outputs"] = free()
    assert o1["U_cell"] == o2["U_cell"] and np.array_equal(o1["sums"], o2["sums"])
    print(f"[workspace] free device memory {free0} -> {seen}", flush=True)
    assert all(v == free0 for v in seen.values()), (free0, seen)
    # uses the workspace was not sized for
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.advance(lsbdg.controller("h211b", dt0=0.05, tol=1e-5), t2, u, inner=inner)
    assert ei.value.code == -2 and "workspace lacks" in str(ei.value)
    if inner == "f32":
        with pytest.raises(lsbdg.DgError) as ei:
            ctx.blockjacobi_setup(u, 0.3, 0.1)            # FP64 blocks on an FP32-sized workspace
        assert ei.value.code == -2
    ctx.close()
    ref.close()


def test_too_small_a_workspace_is_refused():
    from paper_2511_05233_amd import lsbdg
    feats = lsbdg.DG_WS_STEP
    n = lsbdg.workspace_bytes(5, 4, 3, 1e-6, 1, feats)
    ws = torch.empty(n - 4096, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(lsbdg.DgError) as ei:
        _make(ws, feats)
    assert ei.value.code == -2 and "workspace lacks" in str(ei.value)


def test_multigrid_on_a_workspace_context():
    """dg_mg_setup / dg_mg_apply on a workspace sized with DG_WS_MG equal the
    allocating context's bit for bit and allocate nothing."""
    from paper_2511_05233_amd import lsbdg
    feats = lsbdg.DG_WS_OPERATORS | lsbdg.DG_WS_MG
    opts = {"mg_levels": 2, "coarse_agg": 2}
    n = lsbdg.workspace_bytes(5, 4, 3, 1e-6, 1, feats, inner="f64", **opts)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    ref = _make()
    ctx = _make(ws, feats, "f64", **opts)
    u = torch.tensor(synth.random_state(60, 8, 5, phase=synth.porosity_mask((3, 4, 5), 0.6, 1)), device="cuda:0")
    r = torch.tensor(synth.random_vector(7, 60, 8, 6), device="cuda:0")
    ref.mg_setup(u, 0.3, 0.1, levels=2, agg=2)
    y_ref = ref.mg_apply(r)
    y = torch.empty_like(y_ref)
    assert torch.equal(y_ref, y_ref)                 # loads torch's comparison kernels before measuring
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.mg_setup(u, 0.3, 0.1, levels=2, agg=2)
    ctx.mg_apply(r, out=y)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert torch.equal(y, y_ref)
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.mg_setup(u, 0.3, 0.1, levels=3, agg=2)   # more levels than the workspace was sized for
    assert ei.value.code == -2
    ctx.close()
    ref.close()

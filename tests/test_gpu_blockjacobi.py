"""HIP element block-Jacobi vs the oracle's probed element blocks (GPU)."""
import numpy as np
import pytest

import synth
from oracle import dg as odg
from oracle import solve as osolve
from tests.helpers import problem_and_context

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _backward_error(Bor, y, x):
    """max_e ||B_e y_e - x_e|| / (||B_e|| ||y_e|| + ||x_e||) per element."""
    Ne = Bor.shape[0]
    ye = y.transpose(1, 0, 2).reshape(Ne, -1)
    xe = x.transpose(1, 0, 2).reshape(Ne, -1)
    r = np.einsum("eij,ej->ei", Bor, ye) - xe
    num = np.linalg.norm(r, axis=1)
    den = np.linalg.norm(Bor, axis=(1, 2)) * np.linalg.norm(ye, axis=1) + np.linalg.norm(xe, axis=1)
    return float(np.max(num / den))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
@pytest.mark.parametrize("shape,seed", [((5, 4, 3), 0), ((3, 3, 7), 1)])
def test_blockjacobi_apply_inverts_oracle_blocks(shape, seed, dtype, tol):
    nx, ny, nz = shape
    print(f"[bj] mesh {shape} seed {seed} {dtype}", flush=True)
    P, ctx, mask = problem_and_context(nx, ny, nz, mask_seed=seed, param_seed=seed)
    u = synth.random_state(P.n_elem, P.n_nodes, 500 + seed, phase=mask, phi_spread=5e-3)
    m = odg.old_mass(P, u)
    dev = torch.device("cuda:0")
    ut = torch.tensor(u, device=dev, dtype=dtype)
    ctx.blockjacobi_setup(ut, 0.9, 0.05)
    x = synth.random_vector(7, P.n_elem, P.n_nodes, 600 + seed)
    y = ctx.blockjacobi_apply(torch.tensor(x, device=dev, dtype=dtype)).cpu().numpy().astype(np.float64)
    uu = ut.cpu().numpy().astype(np.float64)
    Bor = osolve.element_blocks(P, uu, m, 0.9, 0.05, fields=range(7), condensed=True)
    err = _backward_error(Bor, y, x)
    print("  backward error", err, flush=True)
    assert err < tol
    # exported inverse blocks agree with the apply
    Binv = ctx.blockjacobi_export().cpu().numpy().astype(np.float64)       # [e][col][row]
    xe = x.transpose(1, 0, 2).reshape(P.n_elem, -1)
    y2 = np.einsum("ecr,ec->er", Binv, xe)
    ye = y.transpose(1, 0, 2).reshape(P.n_elem, -1)
    rel = np.linalg.norm(y2 - ye, axis=1) / np.linalg.norm(ye, axis=1)
    assert np.max(rel) < (1e-12 if dtype == torch.float64 else 1e-5)


def test_blockjacobi_errors():
    from paper_2511_05233_amd import lsbdg
    P, ctx, mask = problem_and_context(3, 2, 2, mask_seed=1, param_seed=1)
    dev = torch.device("cuda:0")
    x = torch.zeros((7, P.n_elem, 8), dtype=torch.float64, device=dev)
    with pytest.raises(lsbdg.DgError, match="DG_ESTATE"):
        ctx.blockjacobi_apply(x)
    u = torch.tensor(synth.random_state(P.n_elem, 8, 1, phase=mask), device=dev, dtype=torch.float32)
    ctx.blockjacobi_setup(u, 1.0, 0.1)
    with pytest.raises(lsbdg.DgError, match="DG_EINVAL"):
        ctx.blockjacobi_apply(x)


def test_bf16_apply_rounds_the_fp32_inverses():
    """dg_blockjacobi_apply_bf16 applies the FP32 inverses rounded to
    bfloat16 (nearest even), accumulating in FP32; a new setup replaces the
    bfloat16 copy."""
    P, ctx, mask = problem_and_context(5, 4, 3, mask_seed=2, param_seed=1)
    dev = torch.device("cuda:0")
    x = synth.random_vector(7, P.n_elem, P.n_nodes, 700)
    xt = torch.tensor(x, device=dev, dtype=torch.float32)
    xe = torch.tensor(x, dtype=torch.float64).permute(1, 0, 2).reshape(P.n_elem, 56)
    for seed in (0, 1):
        u = synth.random_state(P.n_elem, P.n_nodes, 710 + seed, phase=mask, phi_spread=5e-3)
        ut = torch.tensor(u, device=dev, dtype=torch.float32)
        ctx.blockjacobi_setup(ut, 0.9, 0.05)
        inv = ctx.blockjacobi_export().cpu()                        # [e][col][row]
        Bh = inv.to(torch.bfloat16).to(torch.float64)
        ref = (Bh * xe[:, :, None]).sum(dim=1)                      # [e][row]
        y = ctx.blockjacobi_apply(xt, bf16=True).cpu().to(torch.float64)
        ye = y.permute(1, 0, 2).reshape(P.n_elem, 56)
        scale = (Bh.abs() * xe.abs()[:, :, None]).sum(dim=1)
        err = float(((ye - ref).abs() / scale.clamp_min(1e-300)).max())
        print(f"[bj] bf16 apply, state {seed}: max error {err:.2e} of sum |B||x|", flush=True)
        assert err < 1e-6
        y32 = ctx.blockjacobi_apply(xt).cpu().to(torch.float64).permute(1, 0, 2).reshape(P.n_elem, 56)
        assert not torch.equal(ye, y32)          # the rounding is visible: a different apply


def test_bf16_apply_needs_an_fp32_setup():
    from paper_2511_05233_amd import lsbdg
    P, ctx, mask = problem_and_context(3, 3, 3, mask_seed=0, param_seed=0)
    dev = torch.device("cuda:0")
    x = torch.zeros((7, P.n_elem, 8), dtype=torch.float32, device=dev)
    with pytest.raises(lsbdg.DgError, match="DG_ESTATE"):
        ctx.blockjacobi_apply(x, bf16=True)
    u = synth.random_state(P.n_elem, P.n_nodes, 3, phase=mask)
    ctx.blockjacobi_setup(torch.tensor(u, device=dev), 0.9, 0.05)       # FP64 setup
    with pytest.raises(lsbdg.DgError, match="DG_ESTATE"):
        ctx.blockjacobi_apply(x, bf16=True)


def test_blocks_full_slab_sampled():
    """FP32 element blocks of the 96 x 96 x 192 slab as the solver builds
    them; the apply at sampled voxels, boundaries included, inverts the
    oracle's blocks of the same FP32-rounded state."""
    from synth import WORKLOADS
    from tests.helpers import oracle_blocks_at, sampled_voxels, slab_state
    w = WORKLOADS["slab96_q1"]
    print(f"[bj] full slab {w.nx}x{w.ny}x{w.nz}, FP32 blocks", flush=True)
    P, ctx, mask = problem_and_context(w.nx, w.ny, w.nz, porosity=w.porosity,
                                       mask_seed=w.mask_seed, param_seed=w.param_seed, f_C=w.f_C)
    u = slab_state(P, mask, 21).to(torch.float32)
    dev = torch.device("cuda:0")
    ud = u.to(dev)
    ctx.blockjacobi_setup(ud, 0.7, 0.05)
    g = torch.Generator(device="cpu").manual_seed(22)
    x = torch.randn((7, P.n_elem, P.n_nodes), generator=g, dtype=torch.float32)
    y = ctx.blockjacobi_apply(x.to(dev)).cpu().numpy().astype(np.float64)
    elems = sampled_voxels(w, 14, 2)
    u64 = u.numpy().astype(np.float64)
    Bor = oracle_blocks_at(P, u64, odg.old_mass(P, u64), 0.7, 0.05, elems)
    err = _backward_error(Bor, y[:, elems], x.numpy().astype(np.float64)[:, elems])
    print(f"  sampled backward error {err:.2e}", flush=True)
    assert err < 2e-5


def test_solver_leaves_bf16_inverses_only():
    """An FP32 inner solve with block_bf16 (the default) inverts its blocks
    straight into the bfloat16 copy: after dg_step the bfloat16 apply works
    and gives finite values, the FP32 apply needs a new setup, and a setup
    restores both."""
    from paper_2511_05233_amd import lsbdg
    P, ctx, mask = problem_and_context(5, 4, 3, mask_seed=1, param_seed=1, f_C=0.1)
    dev = torch.device("cuda:0")
    u, _ = ctx.initial_state(inner="f32")
    ctx.step(u, 0.0, 0.1, inner="f32")
    x = torch.tensor(synth.random_vector(7, P.n_elem, P.n_nodes, 720), device=dev, dtype=torch.float32)
    y = ctx.blockjacobi_apply(x, bf16=True)
    assert bool(torch.isfinite(y).all()) and float(y.abs().max()) > 0
    with pytest.raises(lsbdg.DgError, match="DG_ESTATE"):
        ctx.blockjacobi_apply(x)
    ctx.blockjacobi_setup(u.to(torch.float32), 0.1, 0.1)
    y32 = ctx.blockjacobi_apply(x)
    yh = ctx.blockjacobi_apply(x, bf16=True)
    assert float((yh - y32).abs().max() / y32.abs().max()) < 1e-2

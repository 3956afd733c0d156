"""HIP Jacobian-vector products vs the oracle's complex-step derivative (GPU)."""
import numpy as np
import pytest

import synth
from oracle import dg as odg
from tests.helpers import field_errors, problem_and_context

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# FP64: both sides are exact derivatives of the same arithmetic up to
# rounding; cancellation between flux terms inside a row is the limit.
TOL64 = 1e-10
# FP32 tangent against the FP64 derivative of the same FP32-rounded inputs:
# unit roundoff 6e-8 amplified by the cancellation inside a row (the full
# slab shows 2e-7).
TOL32 = 1e-5
# The full 9-field tangent at random states also carries the rows of S^2-
# and Li2S(S), whose sources are differences of Butler-Volmer and
# solubility exponentials near equilibrium (E4, E6, C2 with K_sp,2 = 8e-15):
# an exponential of an argument |A| ~ 20 rounds to about |A| u32 = 1.2e-6
# relative in FP32, and the difference of two such terms loses another
# order (observed 1.6e-5 and 1.0e-5 on those two rows, 1e-7 elsewhere).
TOL32_FULL = 5e-5


def _case(shape, seed, dtype, condensed, **kw):
    nx, ny, nz = shape
    print(f"[jvp] mesh {shape} seed {seed} {dtype} condensed={condensed}", flush=True)
    P, ctx, mask = problem_and_context(nx, ny, nz, mask_seed=seed, param_seed=seed, **kw)
    u = synth.random_state(P.n_elem, P.n_nodes, 300 + seed, phase=mask, phi_spread=5e-3)
    nf = 7 if condensed else 9
    rng = np.random.default_rng(400 + seed)
    scale = np.array([1500, 6, 6e-3, 4e-3, 2e-3, 4e-12, 3e-3, 0.2, 7e-6])[:nf]
    v = scale[:, None, None] * rng.standard_normal((nf, P.n_elem, P.n_nodes))
    v[:, mask.reshape(-1) == 0, :] *= np.array([1] * 7 + [0, 0])[:nf, None, None]
    dev = torch.device("cuda:0")
    jv = ctx.jvp(torch.tensor(u, device=dev, dtype=dtype), torch.tensor(v, device=dev, dtype=dtype),
                 0.9, 0.05, condensed=condensed).cpu().numpy().astype(np.float64)
    m = odg.old_mass(P, u)
    if dtype == torch.float32:
        u = u.astype(np.float32).astype(np.float64)
        v = v.astype(np.float32).astype(np.float64)
    if condensed:
        ref = odg.jvp_condensed(P, u, v, m, 0.9, 0.05)
    else:
        ref = odg.jvp(P, u, v, m, 0.9, 0.05)
    return field_errors(jv, ref)


@pytest.mark.parametrize("condensed", [False, True])
@pytest.mark.parametrize("shape,seed", [((5, 4, 3), 0), ((9, 3, 7), 1), ((16, 16, 16), 2)])
def test_jvp_fp64(shape, seed, condensed):
    err = _case(shape, seed, torch.float64, condensed)
    print("  errors", err, flush=True)
    assert np.all(err < TOL64), err


@pytest.mark.parametrize("condensed", [False, True])
def test_jvp_fp32(condensed):
    err = _case((12, 8, 6), 3, torch.float32, condensed)
    print("  errors", err, flush=True)
    assert np.all(err < (TOL32 if condensed else TOL32_FULL)), err


def test_jvp_paper_parameters_condensed():
    err = _case((6, 5, 4), 4, torch.float64, True, paper_params=True)
    assert np.all(err < TOL64), err


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_linearized_jvp_equals_condensed(dtype):
    """The Krylov operator with a stored linearisation gives the condensed
    product bit for bit; without a linearisation of its precision it is an
    error."""
    from paper_2511_05233_amd import lsbdg
    dt = torch.float64 if dtype == "f64" else torch.float32
    P, ctx, mask = problem_and_context(7, 6, 5, mask_seed=5, param_seed=5)
    u = torch.tensor(synth.random_state(P.n_elem, P.n_nodes, 5, phase=mask), device="cuda:0", dtype=dt)
    v = torch.tensor(synth.random_vector(7, P.n_elem, P.n_nodes, 6), device="cuda:0", dtype=dt)
    other = torch.float32 if dt == torch.float64 else torch.float64
    ctx.linearize(u.to(other), 0.7, 0.02)
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.jvp(u, v, 0.7, 0.02, linearized=True)
    assert ei.value.code == -6
    a = ctx.jvp(u, v, 0.7, 0.02, condensed=True)
    ctx.linearize(u, 0.7, 0.02)
    b = ctx.jvp(u, v, 0.7, 0.02, linearized=True)
    assert torch.equal(a, b)


def test_krylov_jvp_full_slab_sampled():
    """The Krylov operator as the solver and the benchmark launch it: FP32
    condensed tangent at a stored linearisation on the 96 x 96 x 192 slab
    (99 M DoF); sampled voxels, boundaries included, against the oracle's
    condensed tangent of the same FP32-rounded inputs."""
    from synth import WORKLOADS
    from tests.helpers import oracle_jvp_condensed_at, sampled_voxels, slab_state
    w = WORKLOADS["slab96_q1"]
    print(f"[jvp] full slab {w.nx}x{w.ny}x{w.nz}, FP32 linearised", flush=True)
    P, ctx, mask = problem_and_context(w.nx, w.ny, w.nz, porosity=w.porosity,
                                       mask_seed=w.mask_seed, param_seed=w.param_seed, f_C=w.f_C)
    u = slab_state(P, mask, 11).to(torch.float32)
    g = torch.Generator(device="cpu").manual_seed(12)
    scale = torch.tensor([1500, 6, 6e-3, 4e-3, 2e-3, 4e-12, 3e-3], dtype=torch.float32)
    v = scale[:, None, None] * torch.randn((7, P.n_elem, P.n_nodes), generator=g, dtype=torch.float32)
    dev = torch.device("cuda:0")
    ud, vd = u.to(dev), v.to(dev)
    ctx.linearize(ud, 0.7, 0.05)
    jv = ctx.jvp(ud, vd, 0.7, 0.05, linearized=True).cpu().numpy().astype(np.float64)
    elems = sampled_voxels(w, 40, 1)
    u64, v64 = u.numpy().astype(np.float64), v.numpy().astype(np.float64)
    m = odg.old_mass(P, u64)        # does not enter the tangent
    ref = oracle_jvp_condensed_at(P, u64, v64, m, 0.7, 0.05, elems)
    err = field_errors(jv[:, elems], ref)
    print("  sampled field errors", err, flush=True)
    assert np.all(err < TOL32), err


@pytest.mark.parametrize("condensed", [False, True])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_jvp_at_and_below_the_concentration_floor(dtype, condensed):
    """Tangents where S4^2- and S^2- sit at, below and across the activity
    clamp c_min and Li+ is negative at a node: the clamped activities have
    zero derivative on both sides, and the harmonic-mean guard switches."""
    from tests.test_gpu_residual import _floor_state
    P, ctx, mask = problem_and_context(6, 5, 4, mask_seed=11, param_seed=11)
    u = _floor_state(P, mask, 33)
    nf = 7 if condensed else 9
    rng = np.random.default_rng(34)
    scale = np.array([1500, 6, 6e-3, 4e-3, 2e-3, 4e-12, 3e-3, 0.2, 7e-6])[:nf]
    v = scale[:, None, None] * rng.standard_normal((nf, P.n_elem, P.n_nodes))
    v[:, mask.reshape(-1) == 0, :] *= np.array([1] * 7 + [0, 0])[:nf, None, None]
    dev = torch.device("cuda:0")
    jv = ctx.jvp(torch.tensor(u, device=dev, dtype=dtype), torch.tensor(v, device=dev, dtype=dtype),
                 0.9, 0.05, condensed=condensed).cpu().numpy().astype(np.float64)
    if dtype == torch.float32:
        u = u.astype(np.float32).astype(np.float64)
        v = v.astype(np.float32).astype(np.float64)
    m = odg.old_mass(P, u)
    ref = odg.jvp_condensed(P, u, v, m, 0.9, 0.05) if condensed else odg.jvp(P, u, v, m, 0.9, 0.05)
    err = field_errors(jv, ref)
    print(f"  {dtype} condensed={condensed} floor-state errors", err, flush=True)
    assert np.all(err < (TOL64 if dtype == torch.float64 else (TOL32 if condensed else TOL32_FULL))), err

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
# FP32 dual numbers against the FP64 derivative.
TOL32 = 5e-4


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
    assert np.all(err < TOL32), err


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

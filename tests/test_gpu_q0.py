"""The k = 0 scheme on the GPU (the finite-volume form of Eq. 48) against
the oracle: residual, old mass and the three tangent modes, element by
element (GPU).  The oracle's own k = 0 operator is pinned on the CPU to the
textbook seven-point finite-volume scheme with harmonic means."""
import numpy as np
import pytest

import synth
from oracle import dg as odg
from tests.helpers import field_errors, problem_and_context

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL64, TOL32, TOLJ64 = 1e-12, 2e-5, 1e-10


def _case(shape, seed, **kw):
    nx, ny, nz = shape
    print(f"[q0] mesh {shape} seed {seed}", flush=True)
    P, ctx, mask = problem_and_context(nx, ny, nz, k=0, mask_seed=seed, param_seed=seed, **kw)
    u = synth.random_state(P.n_elem, 1, 700 + seed, phase=mask, phi_spread=5e-3)
    uo = synth.random_state(P.n_elem, 1, 800 + seed, phase=mask)
    return P, ctx, mask, u, uo


@pytest.mark.parametrize("shape,seed", [((5, 4, 3), 0), ((9, 1, 7), 1), ((16, 16, 16), 2)])
def test_q0_residual_and_mass(shape, seed):
    P, ctx, mask, u, uo = _case(shape, seed)
    dev = torch.device("cuda:0")
    m = ctx.mass(torch.tensor(uo, device=dev))
    r = ctx.residual(torch.tensor(u, device=dev), m, 0.7, 0.05).cpu().numpy()
    m_ref = odg.old_mass(P, uo)
    assert np.all(field_errors(m.cpu().numpy(), m_ref) < 1e-15)
    ref = odg.residual(P, u, m_ref, 0.7, 0.05)
    err = field_errors(r, ref)
    print("  residual errors", err, flush=True)
    assert np.all(err < TOL64), err
    r32 = ctx.residual(torch.tensor(u, device=dev, dtype=torch.float32), m.float(), 0.7, 0.05)
    ref32 = odg.residual(P, u.astype(np.float32).astype(np.float64),
                         m.float().double().cpu().numpy(), 0.7, 0.05)
    assert np.all(field_errors(r32.double().cpu().numpy(), ref32) < TOL32)


@pytest.mark.parametrize("mode", ["full", "condensed", "linearized"])
def test_q0_tangents(mode):
    P, ctx, mask, u, _ = _case((7, 5, 4), 3)
    nf = 9 if mode == "full" else 7
    rng = np.random.default_rng(901)
    scale = np.array([1500, 6, 6e-3, 4e-3, 2e-3, 4e-12, 3e-3, 0.2, 7e-6])[:nf]
    v = scale[:, None, None] * rng.standard_normal((nf, P.n_elem, 1))
    v[:, mask.reshape(-1) == 0, :] *= np.array([1] * 7 + [0, 0])[:nf, None, None]
    dev = torch.device("cuda:0")
    ut, vt = torch.tensor(u, device=dev), torch.tensor(v, device=dev)
    if mode == "linearized":
        ctx.linearize(ut, 0.9, 0.05)
    jv = ctx.jvp(ut, vt, 0.9, 0.05, condensed=mode == "condensed", linearized=mode == "linearized")
    m = odg.old_mass(P, u)
    ref = odg.jvp(P, u, v, m, 0.9, 0.05) if mode == "full" else odg.jvp_condensed(P, u, v, m, 0.9, 0.05)
    err = field_errors(jv.cpu().numpy(), ref)
    print(f"  {mode} tangent errors", err, flush=True)
    assert np.all(err < TOLJ64), err


def test_q0_entry_points_beyond_the_operators_say_so():
    from paper_2511_05233_amd import lsbdg
    P, ctx, mask, u, _ = _case((4, 3, 2), 4)
    ut = torch.tensor(u, device="cuda:0")
    for call in (lambda: ctx.step(ut, 0.0, 0.1), lambda: ctx.outputs(ut, 0.0),
                 lambda: ctx.blockjacobi_setup(ut, 0.1, 0.1)):
        with pytest.raises(lsbdg.DgError) as ei:
            call()
        assert ei.value.code == -7

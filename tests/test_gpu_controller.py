"""GPU time controllers (dg_advance) vs the oracle's controllers driving the
oracle's backward-Euler step, and the failure path forced from the host."""
import numpy as np
import pytest

from oracle import controllers as octl
from oracle import solve as osolve
from tests.helpers import problem_and_context

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def case():
    P, ctx, mask = problem_and_context(5, 4, 3, mask_seed=1, param_seed=1, f_C=0.1)
    print("[ctl] oracle initial state 5x4x3", flush=True)
    u0, _ = osolve.initial_state(P)
    return P, ctx, u0


def _oracle_step(P):
    def step(z, t, dt):
        try:
            u, _ = osolve.be_step(P, z, t, dt)
        except osolve.NewtonFailure as e:
            raise octl.SolverFailure(str(e))
        return u
    return step


def rel_l2(a, b):
    return max(np.linalg.norm(a[f] - b[f]) / max(np.linalg.norm(b[f]), 1e-300) for f in range(9))


def test_naive_controller_matches_oracle(case):
    P, ctx, u0 = case
    from paper_2511_05233_amd import lsbdg
    c = lsbdg.controller("naive", dt0=0.1)
    ref = octl.Naive(0.1)
    ut = torch.tensor(u0, device="cuda:0")
    z, t, tg = u0.copy(), 0.0, 0.0
    step = _oracle_step(P)
    for k in range(5):
        z, t, dt_ref = ref.advance(step, z, t)
        tg, rep = ctx.advance(c, tg, ut, inner="f64")
        err = rel_l2(ut.cpu().numpy(), z)
        print(f"[ctl] naive step {k}: dt {rep['dt']} (oracle {dt_ref}), rel L2 {err:.2e}", flush=True)
        assert rep["dt"] == dt_ref and tg == t
        assert err < 1e-9
    assert c.dt == ref.dt and c.sct == ref.sct


def test_h211b_controller_matches_oracle(case):
    P, ctx, u0 = case
    from paper_2511_05233_amd import lsbdg
    tol = 1e-5
    c = lsbdg.controller("h211b", dt0=0.1, tol=tol)
    ref = octl.H211b(0.1, tol)
    ut = torch.tensor(u0, device="cuda:0")
    z, t, tg = u0.copy(), 0.0, 0.0
    step = _oracle_step(P)
    for k in range(2):
        z, t, dt_ref, err_ref = ref.advance(step, z, t)
        tg, rep = ctx.advance(c, tg, ut, inner="f64")
        err = rel_l2(ut.cpu().numpy(), z)
        print(f"[ctl] h211b step {k}: dt {rep['dt']:.6g} (oracle {dt_ref:.6g}), err {rep['err']:.6e} "
              f"(oracle {err_ref:.6e}), trials {rep['trials']}, rel L2 {err:.2e}", flush=True)
        assert rep["dt"] == pytest.approx(dt_ref, rel=1e-6)
        assert rep["err"] == pytest.approx(err_ref, rel=1e-3)
        assert err < 1e-8
    assert c.dt == pytest.approx(ref.dt, rel=1e-5)


def test_failed_solves_halve_then_abort_leaving_state(case):
    """Every solve is made to fail from the host (one Newton iteration
    allowed): dt is halved max_halvings times, then DG_ENOCONV with the
    state and time unchanged."""
    P, ctx, u0 = case
    from paper_2511_05233_amd import lsbdg
    c = lsbdg.controller("naive", dt0=0.1)
    c.max_halvings = 3
    ut = torch.tensor(u0, device="cuda:0")
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.advance(c, 0.0, ut, inner="f64", newton_maxit=1)
    assert ei.value.code == -4
    assert ei.value.report["halvings"] == 4
    assert c.dt == pytest.approx(0.1 / 8)
    assert np.array_equal(ut.cpu().numpy(), u0)

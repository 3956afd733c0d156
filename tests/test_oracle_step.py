"""Pins of the oracle's backward-Euler step and time controllers (CPU only)."""
import math

import numpy as np
import pytest

import synth
from oracle import controllers as C
from oracle import dg, outputs, solve
from oracle import model as M


@pytest.fixture(scope="module")
def stepped():
    mask = synth.porosity_mask((2, 2, 3), 0.5, 3)
    D0, i0 = synth.sample_transport_kinetics(3)
    P = M.Problem(3, 2, 2, 1e-6, 1, mask, D0=D0, kE=i0 / M.F, f_C=1.0)
    u0, info0 = solve.initial_state(P)
    u1, info1 = solve.be_step(P, u0, 0.0, 0.05)
    return P, u0, u1, info0, info1


def test_initial_potential_carries_the_applied_current(stepped):
    """The steady potential makes the reaction current equal j_el * A_sep
    (charge balance of the Phi_L equation with the separator inflow)."""
    P, u0, _, info0, _ = stepped
    *_, I = outputs.invariants(P, u0, 0.0)
    assert abs(I / (P.j_el * outputs.separator_area(P)) - 1.0) < 1e-10


def test_step_root_and_invariants(stepped):
    """At the Newton root: sulfur atoms unchanged; lithium atoms and stored
    electrons both rise by dt j_el A / F (one electron per E reaction, Tab. 3);
    reaction current = j_el A (Sec. 3.2's conservation, to solver tolerance)."""
    P, u0, u1, _, info = stepped
    dt = 0.05
    S0, Li0, Ne0, _ = outputs.invariants(P, u0, 0.0)
    S1, Li1, Ne1, I1 = outputs.invariants(P, u1, dt)
    q = dt * P.j_el * outputs.separator_area(P) / M.F
    assert abs(S1 - S0) < 1e-12 * S0
    assert abs((Li1 - Li0) - q) < 1e-12 * Li0
    assert abs((Ne1 - Ne0) - q) < 1e-9 * q
    assert abs(I1 / (P.j_el * outputs.separator_area(P)) - 1.0) < 1e-9
    R = dg.residual(P, u1, dg.old_mass(P, u0), dt, dt)
    # scale of the balanced terms: time term per mass row, face current for charge
    W = dg.basis(1).W3[None, :] * (P.h / 2) ** 3
    rhoM = M.RHO / M.MOLAR
    for f in range(9):
        if f == 6:
            # forward and backward Butler-Volmer terms in this row are ~1e4 x
            # the face current, and cancel at the root
            scale = 1e3 * P.h ** 2 * P.j_el
        elif f < 6:
            scale = np.max(np.abs(W * u1[f] / dt))
        else:
            scale = np.max(np.abs(W * rhoM[f - 7] * u1[f] / dt))
        assert np.max(np.abs(R[f])) <= 1e-10 * scale, f


def test_cell_voltage_inverts_the_anode_law():
    """U_cell: the anode rate a e^{-A} - e^{A} with e^{A} = y equals -q."""
    mask = np.ones((1, 1, 2), np.uint8)
    P = M.Problem(2, 1, 1, 1e-6, 1, mask, j_el=10.0)
    u = solve.uniform_state(P)
    u[6] = 0.01
    U = outputs.cell_voltage(P, u)
    q = P.j_el / (M.F * M.K_E_ANODE)
    a = u[0, 0, 0] / M.C_REF
    rtf = M.rt_over_f()
    A = (P.V - 0.01 - U) / (2 * rtf)         # = ln y
    y = math.exp(A)
    assert abs(a / y - y + q) < 1e-12 * q


# --------------------------------------------------------------------------
def test_naive_controller_growth_and_halving():
    """3 successes -> dt x 1.2; a failure halves dt and resets the counter."""
    calls = []
    script = iter([True, True, True, False, True, True, True])

    def step(z, t, dt):
        calls.append(dt)
        if not next(script):
            raise C.SolverFailure()
        return z + dt

    ctl = C.Naive(1.0, dt_max=100.0)
    z, t = 0.0, 0.0
    for _ in range(6):
        z, t, _ = ctl.advance(step, z, t)
    assert calls == [1.0, 1.0, 1.0, 1.2, 0.6, 0.6, 0.6]
    assert ctl.dt == pytest.approx(0.72)
    assert t == pytest.approx(1.0 + 1.0 + 1.0 + 0.6 + 0.6 + 0.6)


def test_naive_controller_aborts_after_30_halvings():
    def step(z, t, dt):
        raise C.SolverFailure()

    ctl = C.Naive(1.0)
    with pytest.raises(C.ControllerAbort):
        ctl.advance(step, 0.0, 0.0)
    assert ctl.dt == pytest.approx(2.0 ** -30)


def test_h211b_meets_tolerance_and_richardson_is_second_order():
    """On z' = lam z with backward Euler, the accepted local error estimate
    stays below 1.02 tol, and the extrapolated solution z = 2 z_F - z_C is
    second-order accurate (Eq. 53-54)."""
    lam = -2.0

    def step(z, t, dt):
        return z / (1.0 - lam * dt)

    for tol in (1e-4, 1e-6):
        ctl = C.H211b(0.01, tol, dt_max=1.0)
        z, t = 1.0, 0.0
        while t < 1.0:
            z, t, dt, err = ctl.advance(step, z, t)
            assert err <= 1.02 * tol
        assert abs(z - math.exp(lam * t)) < 50 * tol
    # fixed steps: Richardson error ~ dt^2, BE ~ dt
    errs = []
    for n in (20, 40, 80):
        dt = 1.0 / n
        z = 1.0
        for _ in range(n):
            zC = step(z, 0, dt)
            zF = step(step(z, 0, dt / 2), 0, dt / 2)
            z = 2 * zF - zC
        errs.append(abs(z - math.exp(lam)))
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_h211b_gives_up_on_an_error_floor_above_tol():
    """A solver whose steps carry an error floor (here 1e-7 relative, as an
    inner solve stalled at its attainable accuracy) cannot meet tol = 1e-9
    at any dt: the controller stops after 100 error rejections instead of
    shrinking dt forever."""
    lam = -2.0
    calls = [0]

    def step(z, t, dt):
        calls[0] += 1
        # backward Euler plus a deterministic 1e-7 perturbation that differs
        # between the coarse and the fine solves (an error floor)
        return z / (1.0 - lam * dt) * (1.0 + 1e-7 * (-1) ** calls[0])

    ctl = C.H211b(0.01, 1e-9, dt_max=1.0)
    with pytest.raises(C.ControllerAbort):
        ctl.advance(step, 1.0, 0.0)
    assert ctl.trials == 101
    assert ctl.dt < 0.01 * 0.9 ** 100 * 1.0001


def test_h211b_limiter_formula():
    """Eq. 51-52 with equal history: rho = (tol/err)^(1/2) and lim = 1 + atan(rho - 1)."""
    lim = C.h211b_limiter(1e-6, 1e-6, 1.0, 1.0, 4e-6)
    assert lim == pytest.approx(1.0 + math.atan(2.0 - 1.0))


def test_sparse_chord_solve_reaches_the_direct_root():
    """The oracle's GMRES on the probed sparse Jacobian (chord Newton, used
    for meshes too large for its direct solve) finds the root the direct
    sparse LU finds: the root is fixed by the residual, not by the solver."""
    D0, i0 = synth.sample_transport_kinetics(1)
    mask = synth.porosity_mask((3, 4, 5), 0.6, 1)
    P = M.Problem(5, 4, 3, 1e-6, 1, mask, D0=D0, kE=i0 / M.F, f_C=0.1)
    u0, _ = solve.initial_state(P)
    u1, _ = solve.be_step(P, u0, 0.0, 0.1)
    u2, info = solve.be_step(P, u0, 0.0, 0.1, linear="sparse", gmres_rtol=1e-8, restart=60)
    err = [np.linalg.norm(u1[f] - u2[f]) / np.linalg.norm(u1[f]) for f in range(9)]
    print("sparse vs direct root, relative L2 per field", err, info)
    assert max(err) < 1e-12

"""Direction of the chemical reactions' sources in a whole oracle step (CPU).

The rate tests pin the sign of each rate (Le Chatelier, Sec. 2.5); this pins
what the step does with it, i.e. the columns C1 and C2 of the stoichiometry
(Tab. 3) as they enter the sources of Eq. 05 and the solid mass balances of
Tab. 4.  A negated column passes every atom, charge and Faraday balance and
the rate tests, but fails here.

One structure voxel, electrochemistry switched off (k_E = 0), no applied
current and no T_H ramp, so only the two chemical reactions act and the
voxel is a closed box.  One backward-Euler step (Eq. 50) from a state that
is out of solubility equilibrium must move it back toward equilibrium, as
Le Chatelier's principle demands (Sec. 2.5):

  * S8(L) below K_sp,1 c_ref (undersaturated): S8(S) dissolves, so c_S8(L)
    rises and eps_S8 falls; above it, S8 precipitates.
  * c_Li^2 c_S2- below K_sp,2 c_ref^3: Li2S(S) dissolves, so eps_Li2S falls
    and c_S2-, c_Li rise; above it, Li2S precipitates.

The amounts are tied to each other by the reaction equations: one mol of
S8(S) dissolved gives one mol of S8(L) (C1); one mol of Li2S(S) gives two
mol of Li+ and one of S^2- (C2).
"""
import numpy as np
import pytest

from oracle import dg, solve
from oracle import model as M

DT = 0.5


def _voxel():
    P = M.Problem(1, 1, 1, 1e-6, 1, np.ones((1, 1, 1), np.uint8), kE=np.zeros(6), j_el=0.0, use_TH=False)
    return P


def _step(P, u0, dt=DT):
    m_old = dg.old_mass(P, u0)
    u1, _ = solve.newton(P, u0, m_old, dt, dt, fields=(0, 1, 2, 3, 4, 5, 7, 8))
    return u1


def _amounts(P, u):
    """Moles per node volume: eps_L c_i for the liquid, (rho/M) eps for the solids."""
    eL = 1.0 - P.epsCBD_e[0] - u[7] - u[8]
    rhoM = M.RHO / M.MOLAR
    return np.concatenate([eL[None] * u[0:6], (rhoM[:, None, None] * u[7:9])])


@pytest.mark.parametrize("factor", [0.5, 2.0])
def test_sulfur_dissolution_and_precipitation(factor):
    P = _voxel()
    u0 = solve.uniform_state(P)
    u0[1] = factor * M.K_SP[0] * M.C_REF
    u0[8] = 0.0        # no Li2S(S): C2 cannot answer the change of eps_L
    u1 = _step(P, u0)
    d = _amounts(P, u1) - _amounts(P, u0)
    s = 1.0 if factor < 1 else -1.0           # +1: dissolution expected
    print(f"S8(L) x{factor}: d n_S8(L) {d[1].mean():.3e}, d n_S8(S) {d[6].mean():.3e}")
    assert np.all(s * d[1] > 0) and np.all(s * d[6] < 0)
    # C1: S8(S) -> S8(L) one to one; nothing else moves
    assert np.allclose(d[1], -d[6], rtol=1e-9, atol=0)
    n0 = _amounts(P, u0)
    for i in (0, 2, 3, 4, 5, 7):
        assert np.all(np.abs(d[i]) <= 1e-11 * np.abs(n0[i])), i


@pytest.mark.parametrize("factor", [0.25, 4.0])
def test_lithium_sulfide_dissolution_and_precipitation(factor):
    P = _voxel()
    u0 = solve.uniform_state(P)
    # C2 is slow (k_C,2 sqrt(K_sp,2) ~ 3e-10 mol/(s m^3) per unit eps): a
    # small solid reservoir and a long step, so that the amounts of Li2S(S)
    # and S^2- moved are resolved in FP64 (the Li+ moved, ~1e-12 of its
    # amount, is not; the lithium balance is pinned by the invariants)
    u0[8] = 1e-8
    u0[5] = factor * M.K_SP[1] * M.C_REF ** 3 / u0[0] ** 2
    u1 = _step(P, u0, dt=1e6)
    n0 = _amounts(P, u0)
    d = _amounts(P, u1) - n0
    s = 1.0 if factor < 1 else -1.0
    print(f"S2- x{factor}: d n_Li2S {d[7].mean():.3e}, d n_S2- {d[5].mean():.3e}")
    assert np.all(s * d[7] < 0) and np.all(s * d[5] > 0)
    # C2: Li2S(S) -> 2 Li+ + S^2-
    assert np.allclose(d[5], -d[7], rtol=1e-6, atol=0)
    for i in (1, 2, 3, 4, 6):
        assert np.all(np.abs(d[i]) <= 1e-11 * np.abs(n0[i])), i


@pytest.mark.parametrize("column", [0, 1])
def test_a_negated_column_is_caught(column, monkeypatch):
    """Planted mistake (on the CPU): the C1 or C2 column of the
    stoichiometry negated.  Every balance of Tab. 3 still holds, but the
    undersaturated voxel now loses dissolved S8(L) (C1) or S^2- (C2), which
    the tests above reject."""
    nu = M.NU.copy()
    nu[:, column] *= -1.0
    monkeypatch.setattr(M, "NU", nu)
    P = _voxel()
    u0 = solve.uniform_state(P)
    if column == 0:
        u0[1] = 0.5 * M.K_SP[0] * M.C_REF
        d = _amounts(P, _step(P, u0)) - _amounts(P, u0)
        assert np.all(d[1] < 0) and np.all(d[6] > 0)
    else:
        u0[8] = 1e-8
        u0[5] = 0.25 * M.K_SP[1] * M.C_REF ** 3 / u0[0] ** 2
        d = _amounts(P, _step(P, u0, dt=1e6)) - _amounts(P, u0)
        assert np.all(d[5] < 0) and np.all(d[7] > 0)

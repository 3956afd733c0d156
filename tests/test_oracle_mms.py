"""Manufactured-solution convergence of the oracle's DG discretisation (CPU).

A column of pore voxels (no structure, so no reactions and no applied
current) along one axis, every field frozen at the uniform equilibrium
state except the uncharged polysulfide S8(L).  Its flux is D(c_S) grad c
with the viscosity law of Eq. 02-03, so the diffusion is nonlinear in c
through c_S.  The exact solution of one backward-Euler step (Eq. 50) is
taken to be

    c*(x) = c0 + A cos(pi x / L),

which has no flux through both ends; the old mass that makes it exact is

    m_old = c* - dt d/dx (D(c*) dc*/dx),
    d/dx (D dc/dx) = D (c'' - 8 eta c'^2),   D = D0 exp(-eta c_S),

evaluated at the nodes (the time term is collocated, Sec. 2.7).  A second
family pins the migration part of the Nernst-Planck flux (Tab. 4): Li+
(z = 1) drifts and diffuses in a frozen potential Phi(x) = B cos(pi x / L),
flux D (grad c + (F/RT) c grad Phi) with no flux through both ends, and

    m_old = c* - dt D (c*'' + (F/RT) (c*' Phi' + c* Phi'')).

The error of the oracle's Newton root at the Gauss-Legendre nodes must then
fall at the textbook rates of the interior-penalty schemes on uniform meshes:
second order for k = 0 (the two-point flux of Eq. 48 at the cell centres)
and k = 1, and -- the mark of the incomplete form, Eq. 46 without the
symmetrising term -- only second order again for k = 2, where the
symmetric scheme reaches third order; k = 3, odd again, reaches fourth.  A wrong sign, a dropped term or a
wrong length scale in any volume or face term, on any axis, makes the
scheme inconsistent and the error stall.
"""
import numpy as np
import pytest

from oracle import chem, dg, solve
from oracle import model as M

L = 32e-6           # column length [m]
AMP = 2.0           # amplitude of the cosine [mol/m^3]; c0 = 6 mol/m^3
DT = 1.0            # step [s]; about ten diffusion times (L/pi)^2/D


def _column(N, k, axis):
    shape = [1, 1, 1]
    shape[axis] = N
    nx, ny, nz = shape
    P = M.Problem(nx, ny, nz, L / N, k, np.zeros((nz, ny, nx), np.uint8))
    assert P.j_el == 0.0 and not P.react_e.any()
    return P


def _node_coordinate(P, axis):
    """Coordinate along ``axis`` of every node, shape (E, (k+1)^3)."""
    K = P.k + 1
    xi, _ = dg.gl_nodes_weights(P.k)
    e = np.arange(P.n_elem)
    elem = (e % P.nx, (e // P.nx) % P.ny, e // (P.nx * P.ny))[axis]
    n = np.arange(K ** 3)
    a = (n % K, (n // K) % K, n // (K * K))[axis]
    return (elem[:, None] + 0.5 * (1.0 + xi[a][None, :])) * P.h


def _mms_error(N, k, axis, transport=None, monkeypatch=None):
    """Relative discrete L2 error of the S8(L) root (quadrature weights)."""
    P = _column(N, k, axis)
    u = solve.uniform_state(P)
    c = u[0:6, 0, 0]
    c0 = c[1]
    rest = c[5] + 4.0 * c[4] + 6.0 * c[3] + 8.0 * c[2]     # c_S without S8(L)
    x = _node_coordinate(P, axis)
    q = np.pi / L
    cs = c0 + AMP * np.cos(q * x)
    d1 = -AMP * q * np.sin(q * x)
    d2 = -AMP * q * q * np.cos(q * x)
    D = P.D0[1] * np.exp(-M.ETA_K * (8.0 * cs + rest))
    m_old = dg.old_mass(P, u)
    m_old[1] = cs - DT * D * (d2 - 8.0 * M.ETA_K * d1 * d1)
    if transport is not None:
        monkeypatch.setattr(chem, "transport_coefficients", transport)
    sol, _ = solve.newton(P, u, m_old, 1.0, DT, fields=(1,))
    _, w = dg.gl_nodes_weights(k)
    K = k + 1
    n = np.arange(K ** 3)
    W = np.broadcast_to(w[n % K] * w[(n // K) % K] * w[n // (K * K)], cs.shape)
    err = sol[1] - cs
    return float(np.sqrt(np.sum(W * err ** 2) / np.sum(W * (cs - c0) ** 2)))


def _rates(k, axis, sizes):
    errs = [_mms_error(N, k, axis) for N in sizes]
    return errs, [float(np.log2(a / b)) for a, b in zip(errs, errs[1:])]


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("k", [0, 1])
def test_second_order_on_every_axis(k, axis):
    errs, rates = _rates(k, axis, (4, 8, 16, 32))
    print(f"k={k} axis={axis}: errors {errs}, rates {rates}")
    assert all(1.9 < r < 2.15 for r in rates), rates
    assert errs[-1] < 2e-3


def test_incomplete_penalty_loses_an_order_at_even_degree():
    """k = 2: second order, not the third order of the symmetric scheme."""
    errs, rates = _rates(2, 0, (4, 8, 16))
    print(f"k=2: errors {errs}, rates {rates}")
    assert all(1.9 < r < 2.15 for r in rates), rates


def test_a_wrong_transport_law_stalls(monkeypatch):
    """The pin is sharp: with the viscosity factor of Eq. 02 dropped from
    the oracle's transport law (a planted mistake, on the CPU) the error at
    32 cells is more than ten times the correct one and no longer falls."""
    good = chem.transport_coefficients

    def no_viscosity(P, c, eps, epsCBD):
        D, Mi, K, kap = good(P, c, eps, epsCBD)
        f = np.exp(M.ETA_K * chem.dissolved_sulfur(c))
        return D * f, Mi * f, K * f, kap * f

    ok = _mms_error(32, 1, 0)
    e16 = _mms_error(16, 1, 0, no_viscosity, monkeypatch)
    e32 = _mms_error(32, 1, 0, no_viscosity, monkeypatch)
    print(f"correct {ok:.3e}; planted mistake: 16 cells {e16:.3e}, 32 cells {e32:.3e}")
    assert e32 > 10.0 * ok and e32 > 0.8 * e16


# Li+ in a frozen potential: amplitudes [mol/m^3] and [V]; c0 = 1500 mol/m^3
AMP_LI, AMP_PHI = 100.0, 0.01


def _mms_error_li(N, k, axis, transport=None, monkeypatch=None):
    """Relative discrete L2 error of the Li+ root in the frozen potential."""
    P = _column(N, k, axis)
    u = solve.uniform_state(P)
    c = u[0:6, 0, 0]
    c0 = c[0]
    cS = c[5] + 4.0 * c[4] + 6.0 * c[3] + 8.0 * c[2] + 8.0 * c[1]
    x = _node_coordinate(P, axis)
    q = np.pi / L
    cs = c0 + AMP_LI * np.cos(q * x)
    c1, c2 = -AMP_LI * q * np.sin(q * x), -AMP_LI * q * q * np.cos(q * x)
    p1, p2 = -AMP_PHI * q * np.sin(q * x), -AMP_PHI * q * q * np.cos(q * x)
    D = P.D0[0] * np.exp(-M.ETA_K * cS)
    frt = 1.0 / M.rt_over_f(P.T)
    u[6] = AMP_PHI * np.cos(q * x)
    m_old = dg.old_mass(P, u)
    m_old[0] = cs - DT * D * (c2 + frt * (c1 * p1 + cs * p2))
    if transport is not None:
        monkeypatch.setattr(chem, "transport_coefficients", transport)
    sol, _ = solve.newton(P, u, m_old, 1.0, DT, fields=(0,))
    _, w = dg.gl_nodes_weights(k)
    K = k + 1
    n = np.arange(K ** 3)
    W = np.broadcast_to(w[n % K] * w[(n // K) % K] * w[n // (K * K)], cs.shape)
    err = sol[0] - cs
    return float(np.sqrt(np.sum(W * err ** 2) / np.sum(W * (cs - c0) ** 2)))


@pytest.mark.parametrize("axis", [0, 2])
@pytest.mark.parametrize("k", [0, 1])
def test_drift_diffusion_second_order(k, axis):
    errs = [_mms_error_li(N, k, axis) for N in (4, 8, 16, 32)]
    rates = [float(np.log2(a / b)) for a, b in zip(errs, errs[1:])]
    print(f"Li+ k={k} axis={axis}: errors {errs}, rates {rates}")
    assert all(1.9 < r < 2.15 for r in rates), rates


def test_dropped_migration_stalls(monkeypatch):
    """Planted mistake (on the CPU): the oracle's migration coefficients
    zeroed.  The error at 32 cells is then far above the correct one and no
    longer falls."""
    good = chem.transport_coefficients

    def no_migration(P, c, eps, epsCBD):
        D, Mi, K, kap = good(P, c, eps, epsCBD)
        return D, 0.0 * Mi, K, kap

    ok = _mms_error_li(32, 1, 0)
    e16 = _mms_error_li(16, 1, 0, no_migration, monkeypatch)
    e32 = _mms_error_li(32, 1, 0, no_migration, monkeypatch)
    print(f"correct {ok:.3e}; migration dropped: 16 cells {e16:.3e}, 32 cells {e32:.3e}")
    assert e32 > 10.0 * ok and e32 > 0.8 * e16


def test_degree_three_reaches_fourth_order():
    """k = 3 (the order of the high-order workload): odd degree, so the
    incomplete scheme keeps the optimal order k + 1 = 4, for the nonlinear
    diffusion and for drift-diffusion alike."""
    for fn in (_mms_error, _mms_error_li):
        errs = [fn(N, 3, 0) for N in (2, 4, 8)]
        rates = [float(np.log2(a / b)) for a, b in zip(errs, errs[1:])]
        print(f"{fn.__name__} k=3: errors {errs}, rates {rates}")
        assert all(3.8 < r < 4.2 for r in rates), rates

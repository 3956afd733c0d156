"""Manufactured solution for the charge balance of the oracle (CPU).

Pins the charge row of the DG operator -- the volume term and the
consistency term of the flux  sum_j K_j grad c_j + kappa grad Phi_L
(Tab. 4, discretised by Eq. 43-47 of Sec. 2.7) -- which neither the finite-
volume equivalence at k = 0 (gradients vanish inside a cell) nor the
species manufactured solutions (frozen potential) can see.

A column of pore voxels along one axis (no reactions, no applied current)
with every concentration frozen at a smooth profile: the uniform
equilibrium values plus cosine modes of Li+, S6^2- and S8(L)
(amplitudes chosen so the transport factor exp(-eta c_S) and the
conductivity kappa vary along the column).  The potential of the exact
solution is Phi*(x) = B cos(pi x / L).  Both the concentration modes and
Phi* have zero slope at the two ends, so the flux vanishes through both
ends, as the no-flux condition of the lateral and collector faces demands.

The charge equation alone fixes Phi_L only up to a constant (no exchange
current acts in a pore column), so the manufactured problem adds a linear
zero-order term that vanishes at Phi*:

    -d/dx F(x)  = s(x) - gamma (Phi_L - Phi*(x)),
    F = sum_j K_j dc_j/dx + kappa dPhi*/dx,     s = -dF/dx,

with the source collocated at the nodes like every pointwise source of the
operator.  The flux F(x) is written out here from Tab. 4 and the transport
laws of Eq. 02-03 (Sec. 2.2-2.3), and its derivative is taken by complex
step, exactly to rounding.  gamma is a quarter of kappa (pi/L)^2, so
transport dominates the balance.

The error of the oracle's root must fall at the interior-penalty rates:
second order for k = 0 and 1, fourth for k = 3.  Planted mistakes (on the
CPU): the kappa grad Phi_L term dropped from the volume integral only, and
the sign of the diffusion-potential term sum_j K_j grad c_j flipped; both
make the scheme inconsistent and the error stall.
"""
import numpy as np
import pytest

import synth
from oracle import chem, dg, solve
from oracle import model as M

L = 32e-6            # column length [m]
B_PHI = 5e-3         # amplitude of Phi* [V]
# cosine amplitudes of the frozen concentration modes [mol/m^3]
AMP = {0: 200.0, 3: 2e-3, 1: 2.0}


def _column(N, k, axis):
    shape = [1, 1, 1]
    shape[axis] = N
    nx, ny, nz = shape
    D0, _ = synth.sample_transport_kinetics(0)
    P = M.Problem(nx, ny, nz, L / N, k, np.zeros((nz, ny, nx), np.uint8), D0=D0)
    assert P.j_el == 0.0 and not P.react_e.any()
    return P


def _node_coordinate(P, axis):
    K = P.k + 1
    xi, _ = dg.gl_nodes_weights(P.k)
    e = np.arange(P.n_elem)
    elem = (e % P.nx, (e // P.nx) % P.ny, e // (P.nx * P.ny))[axis]
    n = np.arange(K ** 3)
    a = (n % K, (n // K) % K, n // (K * K))[axis]
    return (elem[:, None] + 0.5 * (1.0 + xi[a][None, :])) * P.h


def _profiles(P, x):
    """Frozen concentrations (6, ...) and the exact potential at points x
    (real or complex)."""
    c0 = P.initial_concentrations()
    q = np.pi / L
    c = [c0[i] + AMP.get(i, 0.0) * np.cos(q * x) for i in range(6)]
    return c, B_PHI * np.cos(q * x)


def _flux(P, x):
    """F(x) = sum_j K_j c_j' + kappa Phi*' in a pore voxel (eps_L = 1),
    from Tab. 4: K_j = z_j F (D_j - D_A), kappa = F^2/(RT) sum_j z_j (z_j D_j
    - z_A D_A) c_j, with D_i = D0_i exp(-eta c_S) (Eq. 02-03, Bruggeman
    factor 1 in the pore)."""
    q = np.pi / L
    c, _ = _profiles(P, x)
    dc = [-AMP.get(i, 0.0) * q * np.sin(q * x) for i in range(6)]
    dphi = -B_PHI * q * np.sin(q * x)
    cS = c[5] + 4 * c[4] + 6 * c[3] + 8 * c[2] + 8 * c[1]
    f = np.exp(-M.ETA_K * cS)
    frt = M.F / (M.R_GAS * P.T)
    D = [P.D0[i] * f for i in range(7)]
    Kdc = sum(M.Z[j] * M.F * (D[j] - D[6]) * dc[j] for j in range(6))
    kappa = M.F * frt * sum(M.Z[j] * (M.Z[j] * D[j] - M.Z_ANION * D[6]) * c[j] for j in range(6))
    return Kdc + kappa * dphi, kappa


def _manufactured(P, axis):
    x = _node_coordinate(P, axis)
    hcs = 1e-30
    s = -np.imag(_flux(P, x + 1j * hcs)[0]) / hcs          # s = -dF/dx
    _, kap0 = _flux(P, np.zeros(1))
    gamma = 0.25 * float(np.real(kap0[0])) * (np.pi / L) ** 2
    c, phi_star = _profiles(P, x)
    return x, np.array(c), phi_star, s, gamma


def _charge_error(N, k, axis, monkeypatch, plant=None):
    P = _column(N, k, axis)
    x, c, phi_star, s, gamma = _manufactured(P, axis)
    u = solve.uniform_state(P)
    u[0:6] = c
    m_old = dg.old_mass(P, u)
    W = dg.basis(k).W3[None, :] * (P.h / 2.0) ** 3
    base = dg.residual

    def residual_mms(P_, uu, mm, t_new, dt):
        R = base(P_, uu, mm, t_new, dt)
        R[6] -= W * (s - gamma * (uu[6] - phi_star))
        return R

    monkeypatch.setattr(dg, "residual", residual_mms)
    if plant is not None:
        plant(monkeypatch, P)
    sol, _ = solve.newton(P, u, m_old, 1.0, 1.0, fields=(6,))
    monkeypatch.undo()
    Wn = np.broadcast_to(dg.basis(k).W3[None, :], phi_star.shape)
    err = sol[6] - phi_star
    return float(np.sqrt(np.sum(Wn * err ** 2) / np.sum(Wn * phi_star ** 2)))


def _rates(k, axis, sizes, monkeypatch):
    errs = [_charge_error(N, k, axis, monkeypatch) for N in sizes]
    return errs, [float(np.log2(a / b)) for a, b in zip(errs, errs[1:])]


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("k", [0, 1])
def test_charge_balance_second_order(k, axis, monkeypatch):
    errs, rates = _rates(k, axis, (4, 8, 16, 32), monkeypatch)
    print(f"charge k={k} axis={axis}: errors {errs}, rates {rates}")
    assert all(1.9 < r < 2.2 for r in rates), rates
    assert errs[-1] < 5e-3


def test_charge_balance_fourth_order_at_degree_three(monkeypatch):
    errs, rates = _rates(3, 0, (2, 4, 8), monkeypatch)
    print(f"charge k=3: errors {errs}, rates {rates}")
    assert all(3.8 < r < 4.3 for r in rates), rates


def _drop_kappa_volume(monkeypatch, P):
    """The volume integral's kappa grad Phi_L term dropped; faces intact.
    (The residual evaluates the volume fluxes on arrays of every element,
    the face fluxes on arrays of the interior faces only.)"""
    good = dg._fluxes_along

    def fluxes(P_, c, phi, eps, eCBD, dc, dphi):
        coeffs, Fs, Fphi = good(P_, c, phi, eps, eCBD, dc, dphi)
        if eCBD.shape[0] == P_.n_elem:
            Fphi = Fphi - coeffs[3] * dphi
        return coeffs, Fs, Fphi

    monkeypatch.setattr(dg, "_fluxes_along", fluxes)


def _flip_diffusion_potential(monkeypatch, P):
    """The sign of sum_j K_j grad c_j flipped in every charge flux."""
    good = dg._fluxes_along

    def fluxes(P_, c, phi, eps, eCBD, dc, dphi):
        coeffs, Fs, Fphi = good(P_, c, phi, eps, eCBD, dc, dphi)
        Kdc = np.sum(coeffs[2] * dc, axis=0)
        return coeffs, Fs, Fphi - 2.0 * Kdc

    monkeypatch.setattr(dg, "_fluxes_along", fluxes)


@pytest.mark.parametrize("plant", [_drop_kappa_volume, _flip_diffusion_potential])
def test_planted_charge_mistakes_stall(plant, monkeypatch):
    ok = _charge_error(32, 1, 0, monkeypatch)
    e16 = _charge_error(16, 1, 0, monkeypatch, plant)
    e32 = _charge_error(32, 1, 0, monkeypatch, plant)
    print(f"{plant.__name__}: correct {ok:.3e}; planted 16 cells {e16:.3e}, 32 cells {e32:.3e}")
    assert e32 > 10.0 * ok and e32 > 0.8 * e16

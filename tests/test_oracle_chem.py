"""Pins of the oracle's pointwise constitutive laws and rates (CPU only)."""
import math

import numpy as np

import synth
from oracle import chem
from oracle import model as M


def _problem(k=1, **kw):
    ph = np.ones((1, 1, 1), dtype=np.uint8)
    return M.Problem(1, 1, 1, 1e-6, k, ph, **kw)


def _random_points(n, seed):
    rng = np.random.default_rng(seed)
    eq = M.equilibrium_state()["c"]
    c = eq[:, None] * np.exp(0.5 * rng.standard_normal((6, n)))
    phi = 0.05 * rng.standard_normal(n)
    eps = np.stack([0.2 * rng.random(n), 1e-4 * rng.random(n)])
    return c, phi, eps


def test_chemical_rate_closed_form_with_pure_solid_reactant():
    """Eq. 19-21 with a pure solid reactant reduce to -sqrt(K)(Q/K - 1) (Sec. 2.5)."""
    P = _problem(use_TH=False)
    c, phi, _ = _random_points(50, 1)
    r = chem.reaction_rates(P, c, phi, 5.0)
    for k, Q in ((0, c[1] / M.C_REF), (1, (c[0] / M.C_REF) ** 2 * (c[5] / M.C_REF))):
        K = M.K_SP[k]
        ref = -math.sqrt(K) * (Q / K - 1.0)
        # the rate is a difference of two terms of size ~sqrt(K)(1 + Q/K)
        scale = math.sqrt(K) * (1.0 + Q / K)
        assert np.all(np.abs(r[k] - ref) <= 1e-13 * scale)


def test_electrochemical_rate_equals_sinh_nernst_form():
    """r_A = -2 sqrt(a_r a_p) sinh(dG_E/2RT), dG_E = F(V - Phi - U_eq),
    U_eq = U0 - RT/F ln Q (Eq. 22-24), with activities formed as products."""
    P = _problem(use_TH=False)
    c, phi, _ = _random_points(80, 2)
    a = c / M.C_REF
    reac = [a[1] ** 0.5, a[2] ** 1.5, a[3], a[4] ** (1 / 6), a[2] ** 0.5, a[4] ** (1 / 6) * a[0] ** (4 / 3)]
    prod = [a[2] ** 0.5, a[3] ** 2, a[4] ** 1.5, a[5] ** (2 / 3), a[4], np.ones_like(a[0])]
    rt = M.R_GAS * P.T
    r = chem.reaction_rates(P, c, phi, 5.0)
    for k in range(6):
        Q = prod[k] / reac[k]
        Ueq = P.U0[k] - rt / M.F * np.log(Q)
        dG = M.F * (P.V - phi - Ueq)
        ref = -2.0 * np.sqrt(reac[k] * prod[k]) * np.sinh(dG / (2 * rt))
        x = M.F * (P.V - phi - P.U0[k]) / (2 * rt)
        scale = reac[k] * np.exp(-x) + prod[k] * np.exp(x)
        assert np.all(np.abs(r[2 + k] - ref) <= 1e-12 * scale), k


def test_all_rates_vanish_at_the_initial_equilibrium():
    P = _problem()
    c = P.initial_concentrations()[:, None]
    r = chem.reaction_rates(P, c, np.zeros(1), 0.0)
    scale = [math.sqrt(K) for K in M.K_SP] + [1.0] * 6
    for k in range(8):
        assert abs(r[k, 0]) < 1e-12 * scale[k] + 1e-15, (k, r[k, 0])


def test_le_chatelier_direction():
    """More product drives every reaction backwards (Sec. 2.5)."""
    P = _problem(use_TH=False)
    c = P.initial_concentrations()[:, None].repeat(2, 1)
    r0 = chem.reaction_rates(P, c, np.zeros(2), 5.0)
    prod_of = {0: 1, 1: 5, 2: 2, 3: 3, 4: 4, 5: 5, 6: 4}
    for k, sp in prod_of.items():
        c2 = c.copy()
        c2[sp] *= 2.0
        r = chem.reaction_rates(P, c2, np.zeros(2), 5.0)
        assert r[k, 0] < r0[k, 0] - 1e-30, k


def test_regularised_reactions_are_those_with_sulfide():
    """T_H multiplies exactly the reactions involving S^2- (C2 and E4)."""
    P = _problem()
    c, phi, _ = _random_points(5, 3)
    r_early = chem.reaction_rates(P, c, phi, 0.0)
    r_late = chem.reaction_rates(P, c, phi, 50.0)
    th = M.smooth_step(0.0)
    for k in range(8):
        expect = th if M.NU[5, k] != 0 else 1.0
        assert np.allclose(r_early[k], expect * r_late[k], rtol=1e-14, atol=0), k


def test_anion_eliminated_coefficients_match_full_electrolyte():
    """Tab. 4's charge coefficients with c_A = -sum z_j c_j / z_A equal the
    un-eliminated sums over all seven species: conductivity of Eq. 05 and the
    diffusion current sum_j z_j F D_j grad c_j (Eq. 04)."""
    D0, _ = synth.sample_transport_kinetics(7)
    P = _problem(D0=D0)
    c, _, eps = _random_points(40, 4)
    epsCBD = 0.1
    D, Mi, K, kap = chem.transport_coefficients(P, c, eps, epsCBD)
    cA = -np.sum(M.Z[:, None] * c, axis=0) / M.Z_ANION
    zall = np.concatenate([M.Z, [M.Z_ANION]])
    call = np.concatenate([c, cA[None]])
    frt = M.F / (M.R_GAS * P.T)
    kap_full = M.F * frt * np.sum(zall[:, None] ** 2 * D * call, axis=0)
    assert np.allclose(kap, kap_full, rtol=1e-12)
    rng = np.random.default_rng(9)
    g = rng.standard_normal((6, 40))
    gA = -np.sum(M.Z[:, None] * g, axis=0) / M.Z_ANION
    full = M.F * (np.sum(M.Z[:, None] * D[:6] * g, axis=0) + M.Z_ANION * D[6] * gA)
    assert np.allclose(np.sum(K * g, axis=0), full, rtol=1e-10, atol=1e-12 * np.abs(full).max())


def test_viscosity_and_bruggeman_factor():
    """D_i^eff = eps_L^(3/2) D0_i eta(0)/eta(c_S) with eta of Eq. 02."""
    P = _problem()
    c = np.zeros((6, 1))
    c[1] = 100.0                       # c_S = 8 * 100
    eps = np.array([[0.1], [0.05]])
    D, _, _, _ = chem.transport_coefficients(P, c, eps, 0.25)
    eta = lambda cs: 1.7e-3 * math.exp(7.76e-4 * cs)
    ref = 0.6 ** 1.5 * P.D0 * eta(0.0) / eta(800.0)
    assert np.allclose(D[:, 0], ref, rtol=1e-14)


def test_specific_surface_passivation_limits():
    """Eq. 18: a_V = a_V0 at zero solids, zero once eps_S8 reaches 1.2 eps_S8,0."""
    P = _problem()
    aV0, e0, pas = 2.0e8, 0.2, 0.05
    eps = np.array([[0.0, 1.2 * e0, 0.5 * e0], [0.0, 0.0, 0.3 * pas]])
    aV = chem.specific_surface(P, eps, aV0, e0, pas)
    assert aV[0] == aV0
    assert aV[1] == 0.0
    assert abs(aV[2] / aV0 - (1 - (0.5 / 1.2) ** 1.5 - 0.3 ** 1.5)) < 1e-14


def test_charge_source_equals_weighted_species_sources():
    """S_Phi = F sum_j z_j S_j (the chemical parts cancel, Sec. 2.2)."""
    P = _problem(use_TH=False)
    c, phi, eps = _random_points(30, 5)
    S_liq, S_phi, _, _, _ = chem.sources(P, c, phi, eps, 3.0, 1e8, 0.2, 0.1, 1.0)
    ref = M.F * np.sum(M.Z[:, None] * S_liq, axis=0)
    assert np.allclose(S_phi, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())

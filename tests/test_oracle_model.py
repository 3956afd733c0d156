"""Pins of the oracle's constants, initial state and stoichiometry (CPU only).

Each test checks the oracle against something the paper prints or a closed
form derived from it, never against the oracle's own formula retyped.
"""
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import model as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    out = {}
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                k, v, tol = line.split()[:3]
                out[k] = (float(v), float(tol))
    return out


def test_equilibrium_reproduces_printed_values():
    """Tab. InitialState at T = 298.15 K reproduces every printed "Equi." value
    of Tab. 5 to within one unit of its last printed digit."""
    eq = M.equilibrium_state()
    got = {
        "c_anion": eq["c_anion"], "c_S2m": eq["c"][5], "c_S4m": eq["c"][4],
        "c_S6m": eq["c"][3], "c_S8m": eq["c"][2], "c_S8": eq["c"][1],
        "U0_5": eq["U5"], "U0_6": eq["U6"],
    }
    for k, (v, unit) in _read_table("equilibrium_values.txt").items():
        assert abs(got[k] - v) <= unit, (k, got[k], v)


def test_equilibrium_at_298K_misses_printed_values():
    """The reading T = 298.15 K is what makes the printed values reproducible:
    with the text's 298 K the polysulfides come out >1 % high."""
    eq = M.equilibrium_state(T=298.0)
    assert eq["c"][2] / 6.184e-3 - 1.0 > 0.01


def test_standard_potentials_match_hess_law():
    """Closed forms: E5 = (E2 + 2 E3)/3 gives U5 = (U2 + 2 U3)/3 at any T; E6 =
    E4 plus 2/3 of the reverse of C2 gives U6 = U4 - (2/3)(RT/F) ln K_sp,2."""
    for T in (290.0, 298.15, 310.0):
        eq = M.equilibrium_state(T=T)
        U1, U2, U3, U4 = M.U0_PRINTED
        assert abs(eq["U5"] - (U2 + 2 * U3) / 3) < 1e-12
        rtf = M.R_GAS * T / M.F
        assert abs(eq["U6"] - (U4 - 2.0 / 3.0 * rtf * math.log(M.K_SP[1]))) < 1e-12


def test_equilibrium_has_zero_gibbs_energy_for_every_reaction():
    """Every reaction of Tab. 3 is at equilibrium (Delta_R G = 0) in the
    Tab. InitialState state with Phi_S - Phi_L = dPhi0 (Eq. 21, 23, 24)."""
    eq = M.equilibrium_state()
    c = eq["c"] / M.C_REF
    rtf = M.rt_over_f()
    # chemical: Q = K_sp
    assert abs(math.log(c[1] / M.K_SP[0])) < 1e-12
    assert abs(math.log(c[0] ** 2 * c[5] / M.K_SP[1])) < 1e-12
    # electrochemical: dPhi0 = U_eq = U0 - RT/F ln Q, Q = prod(products)/prod(reactants)
    act = dict(Li=c[0], S8L=c[1], S8m=c[2], S6m=c[3], S4m=c[4], S2m=c[5])
    Q = [act["S8m"] ** 0.5 / act["S8L"] ** 0.5,
         act["S6m"] ** 2 / act["S8m"] ** 1.5,
         act["S4m"] ** 1.5 / act["S6m"],
         act["S2m"] ** (2 / 3) / act["S4m"] ** (1 / 6),
         act["S4m"] / act["S8m"] ** 0.5,
         1.0 / (act["S4m"] ** (1 / 6) * act["Li"] ** (4 / 3))]
    for k in range(6):
        Ueq = eq["U0"][k] - rtf * math.log(Q[k])
        assert abs(Ueq - eq["dphi0"]) < 1e-12, k


# atoms and charge per species, independent of the stoichiometry table
_SULFUR = {"Li+": 0, "S8(L)": 8, "S8^2-": 8, "S6^2-": 6, "S4^2-": 4, "S^2-": 1,
           "S8(S)": 8, "Li2S(S)": 1, "e-": 0}
_LITHIUM = {"Li+": 1, "S8(L)": 0, "S8^2-": 0, "S6^2-": 0, "S4^2-": 0, "S^2-": 0,
            "S8(S)": 0, "Li2S(S)": 2, "e-": 0}
_CHARGE = {"Li+": 1, "S8(L)": 0, "S8^2-": -2, "S6^2-": -2, "S4^2-": -2, "S^2-": -2,
           "S8(S)": 0, "Li2S(S)": 0, "e-": -1}


def test_stoichiometry_conserves_atoms_and_charge_exactly():
    """Tab. 3: every reaction balances S, Li and charge (exact rationals); each
    E reaction transfers exactly one electron and the C reactions none."""
    for k, name in enumerate(M.REACTIONS):
        col = {sp: M.NU_EXACT[i][k] for i, sp in enumerate(M.SPECIES_ALL)}
        for table in (_SULFUR, _LITHIUM, _CHARGE):
            assert sum(col[sp] * table[sp] for sp in col) == 0, (name, table is _SULFUR)
        assert col["e-"] == (Fr(-1) if name.startswith("E") else Fr(0))


def test_liquid_charge_source_per_electron():
    """Sum_j z_j nu_jk over the dissolved species is -1 for every E reaction and
    0 for C1, C2: the basis of the charge source S_Phi = -F a_V sum k_E r_A."""
    for k, name in enumerate(M.REACTIONS):
        s = sum(M.NU_EXACT[i][k] * Fr(int(M.Z[i])) for i in range(6))
        assert s == (Fr(-1) if name.startswith("E") else Fr(0)), name


def test_printed_arithmetic_of_the_parameter_tables():
    """Sec. 3.1/3.4 dimensionless numbers and App. C capacities recomputed from
    the oracle's parameter tables reproduce the printed values."""
    tab = _read_table("printed_arithmetic.txt")
    F, R = M.F, M.R_GAS
    T_text = 298.0
    l1, l3 = 20e-6, 2e-6
    D0 = dict(zip(["Li", "S8L", "S8m", "S6m", "S4m", "S2m", "A"], M.D0_PAPER))
    ratio_printed = 0.013
    got = {}
    c_theo = 16 * F / M.MOLAR[0]
    got["c_theo_Ah_kg"] = c_theo / 3600.0
    m_A = M.RHO[0] * M.EPS_S8_0 * 105e-6
    got["m_A_S8"] = m_A
    j01 = 0.1 / 3600.0 * c_theo * m_A
    got["j_el_0p1C"] = j01
    got["A_1d"] = F / (R * T_text) * 3.45 * l1 / 0.19
    got["B_1d"] = M.K_C[0] * l1 ** 2 / (D0["S2m"] * ratio_printed * M.C_REF)
    got["C_1d"] = M.K_E_PAPER[0] * l1 / (D0["S2m"] * ratio_printed * M.C_REF)
    got["B_reevaluated"] = M.K_C[0] * l1 ** 2 / (D0["S8m"] * M.C_REF)
    got["eta_ratio"] = math.exp(-M.ETA_K * 5581.8)
    got["B_3d"] = M.K_C[0] * l3 ** 2 / (D0["S2m"] * ratio_printed * M.C_REF)
    got["C_3d"] = M.K_E_PAPER[0] * l3 / (D0["S2m"] * ratio_printed * M.C_REF)
    for k, (v, rtol) in tab.items():
        assert abs(got[k] / v - 1.0) <= rtol, (k, got[k], v)


def test_problem_current_matches_app_c_on_a_1d_column():
    """A laterally trivial Problem of 105 one-micron structure voxels gets the
    App. C current density of the 1D cell (3.45 A/m2 at 0.1C)."""
    ph = np.ones((1, 1, 105), dtype=np.uint8)
    P = M.Problem(105, 1, 1, 1e-6, 0, ph, f_C=0.1)
    assert abs(P.j_el - 3.4527) < 1e-3
    assert abs(P.eps_struct_used - 1.0) < 1e-15


def test_localisation_preserves_cathode_averages():
    """Eq. 57 with eps_struct = 1 - pore fraction keeps the voxel averages of
    eps_S8,0, eps_CBD and a_V0 equal to the homogenised values."""
    rng = np.random.default_rng(3)
    ph = (rng.random((6, 5, 7)) < 0.37).astype(np.uint8)
    P = M.Problem(7, 5, 6, 1e-6, 1, ph)
    assert abs(P.epsS8_0_e.mean() - M.EPS_S8_0) < 1e-14
    assert abs(P.epsCBD_e.mean() - (M.X_CATHODE - M.X_SULFUR)) < 1e-14
    assert abs(P.aV0_e.mean() / M.A_V0 - 1.0) < 1e-14


def test_smooth_step_values():
    """Eq. 56: T_H(1 s) = 1/2, T_H(0) = (1 - tanh 6)/2, T_H -> 1."""
    assert M.smooth_step(1.0) == 0.5
    assert abs(M.smooth_step(0.0) - 0.5 * (1 - math.tanh(6.0))) < 1e-18
    assert M.smooth_step(10.0) == 1.0

"""Battery outputs and discrete conservation invariants (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.
"""
from __future__ import annotations

import numpy as np

from . import chem, dg
from . import model as M


def cell_voltage(P, u):
    """U_cell from the separator-face traces (Eq. A1 with Eq. 26-27).

    The lithium anode (Phi_S,Ano = 0, U0_Ano = 0) carries the current j_el
    by the Butler-Volmer law of Eq. 27; its rate a_Li e^{-A} - e^{A} = -q
    with q = j_el/(F k_E,Ano) inverts in closed form to e^{A} = y,
    y = (q + sqrt(q^2 + 4 a_Li))/2, so the liquid potential next to the
    anode is -(2RT/F) ln y in the anode gauge.  Without a separator drop
    this is the separator-face liquid potential, and with the cathode solid
    at V the pointwise cell voltage is V - Phi_L - (2RT/F) ln y, averaged
    over the separator face with its quadrature weights.
    """
    B = dg.basis(P.k)
    es = dg.separator_elements(P)
    Tr = B.Tr[(0, 1)]
    phi = u[6, es] @ Tr.T
    cli = u[0, es] @ Tr.T
    q = P.j_el / (M.F * M.K_E_ANODE)
    a = np.maximum(cli, P.c_min) / M.C_REF
    y = 0.5 * (q + np.sqrt(q * q + 4.0 * a))
    rtf = M.rt_over_f(P.T)
    Uloc = P.V - phi - 2.0 * rtf * np.log(y)
    w = B.W2[None, :] * np.ones_like(Uloc)
    return float(np.sum(w * Uloc) / np.sum(w))


def volume_means(P, u):
    """Volume averages of the 9 fields and of c_S (Eq. A3)."""
    B = dg.basis(P.k)
    W = B.W3[None, :] / B.W3.sum()
    means = np.array([np.sum(W * u[f]) / P.n_elem for f in range(9)])
    cS = chem.dissolved_sulfur(u[0:6])
    return means, float(np.sum(W * cS) / P.n_elem)


def invariants(P, u, t=0.0):
    """(sulfur atoms, lithium atoms, stored electrons, reaction current) [mol, mol, mol, A].

    All per the nodal quadrature used by the time terms:
      S  = sum W (eps_L (8 c_S8 + 8 c_S8^2- + 6 c_S6^2- + 4 c_S4^2- + c_S^2-)
                  + 8 (rho/M)_S8 eps_S8 + (rho/M)_Li2S eps_Li2S)
      Li = sum W (eps_L c_Li + 2 (rho/M)_Li2S eps_Li2S)
      Ne = sum W (2 eps_L (c_S8^2- + c_S6^2- + c_S4^2- + c_S^2-) + 2 (rho/M)_Li2S eps_Li2S)
      I  = F sum W a_V sum_k k_E,k r_A,k    (equals j_el * A_sep at a root)
    """
    B = dg.basis(P.k)
    W = B.W3[None, :] * (P.h / 2.0) ** 3
    eL = chem.liquid_fraction(P, u[7:9], P.epsCBD_e[:, None])
    rhoM = M.RHO / M.MOLAR
    c = u[0:6]
    S = np.sum(W * (eL * (8 * c[1] + 8 * c[2] + 6 * c[3] + 4 * c[4] + c[5])
                    + 8 * rhoM[0] * u[7] + rhoM[1] * u[8]))
    Li = np.sum(W * (eL * c[0] + 2 * rhoM[1] * u[8]))
    Ne = np.sum(W * (2 * eL * (c[2] + c[3] + c[4] + c[5]) + 2 * rhoM[1] * u[8]))
    _, S_phi, _, _, _ = chem.sources(P, c, u[6], u[7:9], t, P.aV0_e[:, None],
                                     P.epsS8_0_e[:, None], P.pass_e[:, None], P.react_e[:, None])
    I = -np.sum(W * S_phi)
    return float(S), float(Li), float(Ne), float(I)


def separator_area(P):
    return P.ny * P.nz * P.h ** 2

"""Pointwise constitutive laws and reaction rates (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

All functions accept real or complex arrays (complex-step derivatives):
branch decisions look at real parts, and the derivative of a clamped value
is zero.
"""
from __future__ import annotations

import numpy as np

from . import model as M


def _re(x):
    return np.real(x)


def clamp_below(x, lo):
    """max(x, lo) with a zero derivative where the clamp is active."""
    return np.where(_re(x) > lo, x, lo)


def liquid_fraction(P, eps, epsCBD):
    """eps_L = 1 - eps_CBD - eps_S8 - eps_Li2S (Sec. 2.7, item (ii)), floored."""
    return clamp_below(1.0 - epsCBD - eps[0] - eps[1], P.epsL_min)


def dissolved_sulfur(c):
    """c_S = c_S^2- + 4 c_S4 + 6 c_S6 + 8 c_S8^2- + 8 c_S8 (Sec. 2.2)."""
    return c[5] + 4.0 * c[4] + 6.0 * c[3] + 8.0 * c[2] + 8.0 * c[1]


def transport_coefficients(P, c, eps, epsCBD):
    """Effective transport coefficients at points.

    c: (6, ...) concentrations; eps: (2, ...) solid fractions.
    Returns D (7, ...) [incl. anion], M (6, ...), K (6, ...), kappa (...).

    D_i^eff = eps_L^(3/2) D_i(c_S)            Bruggeman, tau = eps_L^(-1/2)
    D_i(c_S) = D0_i eta(0)/eta(c_S) = D0_i exp(-7.76e-4 c_S)   (Eq. 02-03)
    M_i = z_i F/(RT) D_i^eff c_i              (migration, Tab. 4 row 1)
    K_j = z_j F (D_j^eff - D_A^eff)           (Tab. 4 row 2, anion eliminated)
    kappa = F^2/(RT) sum_j z_j (z_j D_j^eff - z_A D_A^eff) c_j
    """
    eL = liquid_fraction(P, eps, epsCBD)
    cS = dissolved_sulfur(c)
    f = eL * np.sqrt(eL) * np.exp(-M.ETA_K * cS)
    shape = (7,) + (1,) * np.ndim(f)
    D = P.D0.reshape(shape) * f
    frt = 1.0 / M.rt_over_f(P.T)
    zz = M.Z.reshape((6,) + (1,) * np.ndim(f))
    Mi = zz * frt * D[:6] * c
    K = zz * M.F * (D[:6] - D[6])
    kappa = M.F * frt * np.sum(zz * (zz * D[:6] - M.Z_ANION * D[6]) * c, axis=0)
    return D, Mi, K, kappa


def ln_activity(P, c):
    """ln <a> = ln(max(c, c_min)/c_ref) for a dissolved species (Eq. 20)."""
    return np.log(clamp_below(c, P.c_min) / M.C_REF)


def specific_surface(P, eps, aV0, epsS8_0, pass_li2s):
    """Eq. 18 with the Eq. 57 localisation and a floor at zero.

    a_V = a_V0 max(0, 1 - (eps_S8+/(1.2 eps_S8,0))^(3/2) - (eps_Li2S+/(a e^{-b f_C}))^(3/2))
    where aV0, epsS8_0 and pass_li2s are already localised per voxel
    (all zero in pore voxels, where a_V = 0).
    """
    active = aV0 > 0
    d1 = np.where(active, 1.2 * epsS8_0, 1.0)
    d2 = np.where(active, pass_li2s, 1.0)
    x1 = clamp_below(eps[0], 0.0) / d1
    x2 = clamp_below(eps[1], 0.0) / d2
    inner = 1.0 - x1 * np.sqrt(x1) - x2 * np.sqrt(x2)
    return aV0 * clamp_below(inner, 0.0)


def reaction_rates(P, c, phi, t):
    """Rates of the eight Tradeoff-Chemistry reactions at points.

    Chemical (Eq. 19-21 with alpha_s = 1/2):
        r_V = -2 sqrt(a_reac a_prod) sinh(dG/(2RT)),  dG = RT ln(Q/K_sp)
            = sqrt(K_sp) a_reac - a_prod / sqrt(K_sp).
    Electrochemical (Eq. 22-24, n_e = 1 for every reaction of Tab. 3):
        r_A = -2 sqrt(a_reac a_prod) sinh(dG_E/(2RT)),
        dG_E = F (V - Phi_L - U_eq), U_eq = U0 - RT/F ln Q
            = a_reac exp(-A) - a_prod exp(A),  A = F (V - Phi_L - U0)/(2RT).
    Activities of solids and electrons are 1.  Reactions involving S^2-
    (C2 and E4) are multiplied by T_H(t) (Eq. 56; Sec. 2.10).

    Returns r of shape (8, ...) in the column order C1, C2, E1..E6.
    """
    la = [ln_activity(P, c[m]) for m in range(6)]
    Li, S8L, S8m, S6m, S4m, S2m = la
    sK = np.sqrt(M.K_SP)
    th = M.smooth_step(t) if P.use_TH else 1.0
    r = [None] * 8
    r[0] = sK[0] - np.exp(S8L) / sK[0]
    r[1] = (sK[1] - np.exp(2.0 * Li + S2m) / sK[1]) * th
    lnr = [0.5 * S8L, 1.5 * S8m, S6m, S4m / 6.0, 0.5 * S8m, S4m / 6.0 + 4.0 / 3.0 * Li]
    lnp = [0.5 * S8m, 2.0 * S6m, 1.5 * S4m, 2.0 / 3.0 * S2m, S4m, 0.0 * Li]
    frt2 = 0.5 / M.rt_over_f(P.T)
    for k in range(6):
        A = frt2 * (P.V - phi - P.U0[k])
        r[2 + k] = np.exp(lnr[k] - A) - np.exp(lnp[k] + A)
    r[5] = r[5] * th
    return np.stack(r)


def sources(P, c, phi, eps, t, aV0, epsS8_0, pass_li2s, react):
    """Volumetric sources at points.

    S_i = sum_C nu_ik eps_k k_C,k r_V,k + a_V sum_E nu_ik k_E,k r_A,k
    (Eq. 16a/17a with the normalisations of Eq. 05-06 cancelled), where
    eps_k is eps_S8 for C1 and eps_Li2S for C2.
    Returns (S_liq (6,...), S_phi (...), S_solid (2,...), a_V, r).
    S_phi = sum_j z_j F S_j restricted to the electrochemical part
          = -F a_V sum_k k_E,k r_A,k, since sum_j z_j nu_jk = -1 for every
    E reaction of Tab. 3 and the C reactions are electroneutral.
    """
    r = reaction_rates(P, c, phi, t)
    aV = specific_surface(P, eps, aV0, epsS8_0, pass_li2s)
    volC = [eps[0] * M.K_C[0] * react * r[0], eps[1] * M.K_C[1] * react * r[1]]
    surE = [aV * P.kE[k] * react * r[2 + k] for k in range(6)]
    rates = volC + surE
    S = [sum(M.NU[i, k] * rates[k] for k in range(8) if M.NU[i, k] != 0.0) for i in range(8)]
    S_liq = np.stack([np.asarray(S[i]) + 0.0 * c[0] for i in range(6)])
    S_sol = np.stack([np.asarray(S[6]) + 0.0 * c[0], np.asarray(S[7]) + 0.0 * c[0]])
    S_phi = -M.F * sum(surE)
    return S_liq, S_phi, S_sol, aV, r

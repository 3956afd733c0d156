"""Interior-penalty DG residual on voxel hexahedra (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Discretisation (Sec. 2.7, Eq. 43-47), for every scalar field psi with flux
f = -(K grad psi + ...):
  * nodal Lagrange basis of degree k per axis on the (k+1) Gauss-Legendre
    points of each voxel; volume quadrature on the same points (weights
    w_a (h/2)^3), so the mass matrix is diagonal; face quadrature on the
    (k+1)^2 tangential Gauss-Legendre points of each face (weights
    w_p (h/2)^2);
  * volume term  + sum_q w_q |J| (K grad psi)(x_q) . grad phi_a(x_q)
    (the -int f . grad v term of Eq. 43);
  * interior faces, Eq. 46, tested with phi_a on the element E (the "-"
    side) with outward normal n:
        - {K grad psi} . n phi_a  +  (sigma/h) {K}_H (psi^- - psi^+) phi_a,
    {K}_H the harmonic mean of Eq. 45, set to 0 unless K^- K^+ > 0;
    the symmetrising term of SIPG is absent (incomplete IP, as written).
    Every gradient term of a flux is penalised with the harmonic mean of its
    own coefficient ("component-wise", Sec. 2.7), which at k = 0 is the
    only place migration enters;
  * Neumann faces (Eq. 47): + int f^N phi_a, f^N the outward normal flux;
  * sigma = 1 at k = 0 (the paper's scheme, Eq. 48) and (k+1)^2 for k >= 1.
Coefficients at face points are evaluated from the traced state.

Traces at a face come from 1D Lagrange interpolation of the nodal values to
xi = +-1 along the normal line of nodes; normal derivatives from the 1D
derivative of that interpolant.

Residual rows per node a (W_a = w_a |J|):
  species i:  W_a (eps_L c_i - m_i^n)/dt + transport_i - W_a S_i
              - [separator] int g_i phi_a,  g_Li = j_el/F, others 0
  charge:     transport_phi - W_a S_phi - [separator] int j_el phi_a
  solids s:   W_a ((rho/M)_s (eps_s - eps_s^n)/dt - S_s)
with m^n = (eps_L c)^n the old mass (Eq. 50 applied to Eq. 16a/17a).
Fluxes: species  D_i grad c_i + M_i grad Phi_L;
        charge   sum_j K_j grad c_j + kappa grad Phi_L.
Face x = L_x is the separator; every other boundary face is no-flux.

Array layout: u[f, e, n] with e = ix + nx (iy + ny iz) and n = a0 + K (a1 +
K a2), K = k + 1, x fastest.
"""
from __future__ import annotations

import numpy as np

from . import chem
from . import model as M


# --------------------------------------------------------------------------
# 1D and tensor-product basis
# --------------------------------------------------------------------------
def gl_nodes_weights(k):
    xi, w = np.polynomial.legendre.leggauss(k + 1)
    return xi, w


def lagrange_values(nodes, x):
    """L[j, i] = l_i(x_j) for the Lagrange basis on ``nodes``."""
    K = len(nodes)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    L = np.ones((len(x), K))
    for i in range(K):
        for m in range(K):
            if m != i:
                L[:, i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
    return L


def lagrange_derivatives(nodes, x):
    """D[j, i] = l_i'(x_j): sum over m != i of the product rule terms."""
    K = len(nodes)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    D = np.zeros((len(x), K))
    for i in range(K):
        for m in range(K):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for l in range(K):
                if l != i and l != m:
                    term = term * (x - nodes[l]) / (nodes[i] - nodes[l])
            D[:, i] += term
    return D


class Basis:
    """Nodal Q_k element on Gauss-Legendre points, x-fastest node order."""

    def __init__(self, k):
        self.k = k
        K = k + 1
        self.K = K
        self.np = K ** 3
        xi, w = gl_nodes_weights(k)
        self.xi, self.w = xi, w
        D1 = lagrange_derivatives(xi, xi)              # (K, K)
        L_end = {s: lagrange_values(xi, [float(s)])[0] for s in (-1, 1)}
        D_end = {s: lagrange_derivatives(xi, [float(s)])[0] for s in (-1, 1)}
        idx = [(a0, a1, a2) for a2 in range(K) for a1 in range(K) for a0 in range(K)]
        self.idx = idx
        self.W3 = np.array([w[a[0]] * w[a[1]] * w[a[2]] for a in idx])
        # reference gradient matrices G[d][q, a] = d phi_a / d xi_d at node q
        self.G = np.zeros((3, self.np, self.np))
        for qi, q in enumerate(idx):
            for ai, a in enumerate(idx):
                for d in range(3):
                    others = [t for t in range(3) if t != d]
                    if all(q[t] == a[t] for t in others):
                        self.G[d, qi, ai] = D1[q[d], a[d]]
        # face trace / normal-derivative matrices Tr[(d,s)][p, a]
        self.Tr, self.Dn = {}, {}
        nf = K * K
        self.W2 = np.zeros(nf)
        for d in range(3):
            t1, t2 = [t for t in range(3) if t != d]
            for s in (-1, 1):
                Tr = np.zeros((nf, self.np))
                Dn = np.zeros((nf, self.np))
                for ai, a in enumerate(idx):
                    p = a[t1] + K * a[t2]
                    Tr[p, ai] = L_end[s][a[d]]
                    Dn[p, ai] = D_end[s][a[d]]
                self.Tr[(d, s)] = Tr
                self.Dn[(d, s)] = Dn
        for p2 in range(K):
            for p1 in range(K):
                self.W2[p1 + K * p2] = w[p1] * w[p2]


_BASES = {}


def basis(k):
    if k not in _BASES:
        _BASES[k] = Basis(k)
    return _BASES[k]


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------
def harmonic(a, b):
    """{K}_H = 2 a b/(a + b) if a b > 0, else 0 (Eq. 45 with a guard)."""
    ok = _re_prod_pos(a, b)
    den = np.where(ok, a + b, 1.0)
    return np.where(ok, 2.0 * a * b / den, 0.0)


def _re_prod_pos(a, b):
    return np.real(a) * np.real(b) > 0.0


def element_grid(P):
    return np.arange(P.n_elem).reshape(P.nz, P.ny, P.nx)


def face_pairs(P, d):
    """(minus, plus) element indices of all interior faces normal to axis d."""
    g = element_grid(P)
    if d == 0:
        return g[:, :, :-1].ravel(), g[:, :, 1:].ravel()
    if d == 1:
        return g[:, :-1, :].ravel(), g[:, 1:, :].ravel()
    return g[:-1, :, :].ravel(), g[1:, :, :].ravel()


def separator_elements(P):
    return element_grid(P)[:, :, -1].ravel()


def old_mass(P, u):
    """m[0:6] = eps_L c_i and m[6:8] = eps_s at the nodes of state u."""
    eCBD = P.epsCBD_e[:, None]
    eL = chem.liquid_fraction(P, u[7:9], eCBD)
    m = np.empty((8,) + u.shape[1:], dtype=u.dtype)
    m[0:6] = eL * u[0:6]
    m[6:8] = u[7:9]
    return m


# --------------------------------------------------------------------------
# residual
# --------------------------------------------------------------------------
def _fluxes_along(P, c, phi, eps, eCBD, dc, dphi):
    """Normal/axis flux components at points for all 7 transported rows."""
    D, Mi, K, kap = chem.transport_coefficients(P, c, eps, eCBD)
    Fs = D[:6] * dc + Mi * dphi
    Fphi = np.sum(K * dc, axis=0) + kap * dphi
    return (D, Mi, K, kap), Fs, Fphi


def residual(P, u, m_old, t_new, dt):
    """DG residual R(u) of the backward-Euler step to t_new (shape of u)."""
    B = basis(P.k)
    h = P.h
    J3 = (h / 2.0) ** 3
    J2 = (h / 2.0) ** 2
    g2h = 2.0 / h
    R = np.zeros_like(u)
    c, phi, eps = u[0:6], u[6], u[7:9]
    eCBD = P.epsCBD_e[:, None]
    W = B.W3[None, :] * J3

    # time terms (Eq. 50)
    eL = chem.liquid_fraction(P, eps, eCBD)
    R[0:6] += W * (eL * c - m_old[0:6]) / dt
    rhoM = M.RHO / M.MOLAR
    for s in range(2):
        R[7 + s] += W * rhoM[s] * (eps[s] - m_old[6 + s]) / dt

    # volume terms: + sum_q W_q flux(x_q) . grad phi_a(x_q)
    for d in range(3):
        Gd = B.G[d]
        dc = g2h * (c @ Gd.T)
        dphi = g2h * (phi @ Gd.T)
        _, Fs, Fphi = _fluxes_along(P, c, phi, eps, eCBD, dc, dphi)
        R[0:6] += g2h * ((W * Fs) @ Gd)
        R[6] += g2h * ((W * Fphi) @ Gd)

    # interior faces (Eq. 46), each face once, contributing to both sides
    sig_h = P.sigma / h
    for d in range(3):
        em, ep = face_pairs(P, d)
        if len(em) == 0:
            continue
        Trm, Dnm = B.Tr[(d, 1)], B.Dn[(d, 1)]      # "-" element, face at xi_d = +1
        Trp, Dnp = B.Tr[(d, -1)], B.Dn[(d, -1)]    # "+" element, face at xi_d = -1
        um = u[:, em] @ Trm.T
        up = u[:, ep] @ Trp.T
        gm = g2h * (u[:, em] @ Dnm.T)
        gp = g2h * (u[:, ep] @ Dnp.T)
        cm_, pm_, em_ = um[0:6], um[6], um[7:9]
        cp_, pp_, ep_ = up[0:6], up[6], up[7:9]
        (Dm, Mm, Km, km), Fsm, Fpm = _fluxes_along(P, cm_, pm_, em_, P.epsCBD_e[em][:, None], gm[0:6], gm[6])
        (Dp, Mp, Kp, kp), Fsp, Fpp = _fluxes_along(P, cp_, pp_, ep_, P.epsCBD_e[ep][:, None], gp[0:6], gp[6])
        # face quantity seen from the "-" element, outward normal n = +e_d
        qs = (-0.5 * (Fsm + Fsp)
              + sig_h * (harmonic(Dm[:6], Dp[:6]) * (cm_ - cp_)
                         + harmonic(Mm, Mp) * (pm_ - pp_)))
        qphi = (-0.5 * (Fpm + Fpp)
                + sig_h * (np.sum(harmonic(Km, Kp) * (cm_ - cp_), axis=0)
                           + harmonic(km, kp) * (pm_ - pp_)))
        WF = B.W2[None, :] * J2
        R[0:6, em] += (WF * qs) @ Trm
        R[0:6, ep] -= (WF * qs) @ Trp
        R[6, em] += (WF * qphi) @ Trm
        R[6, ep] -= (WF * qphi) @ Trp

    # separator face x = L_x (Eq. 47): inward Li+ flux j_el/F, inward current j_el
    es = separator_elements(P)
    Tr = B.Tr[(0, 1)]
    WF = (B.W2 * J2)[None, :]
    R[0, es] -= (WF * (P.j_el / M.F)) @ Tr
    R[6, es] -= (WF * P.j_el) @ Tr

    # pointwise sources at nodes
    S_liq, S_phi, S_sol, _, _ = chem.sources(
        P, c, phi, eps, t_new, P.aV0_e[:, None], P.epsS8_0_e[:, None],
        P.pass_e[:, None], P.react_e[:, None])
    R[0:6] -= W * S_liq
    R[6] -= W * S_phi
    R[7:9] -= W * S_sol
    return R


def jvp(P, u, v, m_old, t_new, dt, hstep=1e-30):
    """J(u) v by complex-step differentiation: Im R(u + i h v) / h.

    Exact to rounding for the analytic parts of R (Squire & Trapp 1998); the
    derivative of a clamped quantity is zero.
    """
    uc = u.astype(np.complex128) + 1j * hstep * v
    return np.imag(residual(P, uc, m_old, t_new, dt)) / hstep


def jvp_condensed(P, u, v7, m_old, t_new, dt):
    """Krylov-field operator with the node-local solid fractions condensed.

    J_red v = J_uu v + J_ue w,  w = -J_ee^{-1} J_eu v   (per node, 2x2),
    returned for the 7 transported rows.
    """
    z = np.zeros((2,) + v7.shape[1:])
    v9 = np.concatenate([v7, z])
    Jv = jvp(P, u, v9, m_old, t_new, dt)
    Jeu_v = Jv[7:9]
    Jee = solid_block(P, u, m_old, t_new, dt)          # (2, 2, Ne, np)
    w = -_solve2(Jee, Jeu_v)
    v9b = np.concatenate([v7, w])
    return jvp(P, u, v9b, m_old, t_new, dt)[0:7]


def solid_block(P, u, m_old, t_new, dt):
    """J_ee[r, s] per node: derivative of solid row r w.r.t. solid field s.

    The solid rows are node-local, so one probe per column gives the 2x2
    block at every node at once.
    """
    out = np.zeros((2, 2) + u.shape[1:])
    for s in range(2):
        e = np.zeros_like(u)
        e[7 + s] = 1.0
        out[:, s] = jvp(P, u, e, m_old, t_new, dt)[7:9]
    return out


def _solve2(A, b):
    det = A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0]
    x0 = (A[1, 1] * b[0] - A[0, 1] * b[1]) / det
    x1 = (-A[1, 0] * b[0] + A[0, 0] * b[1]) / det
    return np.stack([x0, x1])

"""One-dimensional DG engine for the canonical problems of App. B (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Linear diffusion d_t c = d_x (D(x) d_x c) on [-L/2, L/2] with no-flux ends,
discretised as the 3D scheme is (Sec. 2.7, Eq. 43-47, App. B Eq. B1): nodal
Lagrange basis of degree k on the k + 1 Gauss-Legendre points of each cell,
quadrature on the same points (diagonal mass matrix), incomplete interior
penalty with the harmonic mean of D on the penalty,

    a(c, v) = sum_cells int D c' v'
              - sum_faces {D c'} [v] + sum_faces sigma/h {D}_H [c] [v],

sigma = 1 for k = 0 and (k + 1)^2 otherwise, and implicit Euler (Eq. 50).
D is constant on each cell (a discontinuity sits on a face).  The problem
is linear, so the matrix M/dt + A is factorised once.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class Diffusion1D:
    def __init__(self, n, k, L, D_cell, sigma=None):
        self.n, self.k, self.L = n, k, L
        self.h = h = L / n
        self.x0 = -L / 2
        K = k + 1
        xi, w = np.polynomial.legendre.leggauss(K)
        self.xi, self.w = xi, w
        # 1D Lagrange basis on the Gauss nodes: values and derivatives at the
        # nodes and at the cell ends xi = -1, +1
        V = np.vander(xi, K, increasing=True)
        C = np.linalg.inv(V)                      # column j: coefficients of l_j
        dC = np.array([[p * C[p, j] for j in range(K)] for p in range(1, K)]) if K > 1 else np.zeros((0, K))

        def val(x):
            return np.array([[sum(C[p, j] * xx ** p for p in range(K)) for j in range(K)] for xx in np.atleast_1d(x)])

        def der(x):
            return np.array([[sum(dC[p - 1, j] * xx ** (p - 1) for p in range(1, K)) for j in range(K)]
                             for xx in np.atleast_1d(x)])

        Dn = der(xi)                              # Dn[q, j] = l_j'(xi_q)
        ends = val(np.array([-1.0, 1.0]))          # ends[s, j]
        dends = der(np.array([-1.0, 1.0]))
        g = 2.0 / h                               # d xi / dx
        J = h / 2.0
        self.D = np.asarray(D_cell, dtype=float)
        if sigma is None:
            sigma = 1.0 if k == 0 else float(K * K)
        N = n * K
        rows, cols, vals = [], [], []

        def add(i, j, v):
            rows.append(i)
            cols.append(j)
            vals.append(v)

        # volume: int D c' v' = sum_q w_q J D (g l_j'(q)) (g l_a'(q))
        for e in range(n):
            for a in range(K):
                for j in range(K):
                    s = sum(w[q] * J * self.D[e] * g * Dn[q, j] * g * Dn[q, a] for q in range(K))
                    if s != 0.0:
                        add(e * K + a, e * K + j, s)
        # interior faces between cells e (left, "-") and e + 1 (right, "+")
        for e in range(n - 1):
            Dm, Dp = self.D[e], self.D[e + 1]
            DH = 2.0 * Dm * Dp / (Dm + Dp) if Dm * Dp > 0 else 0.0
            # traces and derivatives at the face: left cell at xi = +1, right at -1
            tl, tr = ends[1], ends[0]
            dl, dr = g * dends[1], g * dends[0]
            jump_v = [(e, a, tl[a]) for a in range(K)] + [(e + 1, a, -tr[a]) for a in range(K)]
            for (ev, a, jv) in jump_v:
                # - {D c'} [v]
                for j in range(K):
                    add(ev * K + a, e * K + j, -0.5 * Dm * dl[j] * jv)
                    add(ev * K + a, (e + 1) * K + j, -0.5 * Dp * dr[j] * jv)
                # + sigma/h {D}_H [c] [v]
                for j in range(K):
                    add(ev * K + a, e * K + j, sigma / h * DH * tl[j] * jv)
                    add(ev * K + a, (e + 1) * K + j, -sigma / h * DH * tr[j] * jv)
        self.A = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
        self.Mdiag = np.tile(w * J, n)
        self.ends = ends

    def nodes_x(self):
        xc = self.x0 + self.h * (np.arange(self.n) + 0.5)
        return (xc[:, None] + 0.5 * self.h * self.xi[None, :]).ravel()

    def factor(self, dt):
        self.dt = dt
        self.lu = spla.splu((sp.diags(self.Mdiag / dt) + self.A).tocsc())

    def step(self, c):
        return self.lu.solve(self.Mdiag / self.dt * c)

    def means(self, c):
        K = self.k + 1
        return (c.reshape(self.n, K) * self.w[None, :]).sum(axis=1) / 2.0

    def evaluate(self, c, x):
        """The DG polynomial of state c at points x (inside the domain)."""
        K = self.k + 1
        e = np.clip(((x - self.x0) / self.h).astype(int), 0, self.n - 1)
        xi = 2.0 * (x - (self.x0 + self.h * (e + 0.5))) / self.h
        V = np.vander(self.xi, K, increasing=True)
        C = np.linalg.inv(V)
        P = np.vander(xi, K, increasing=True) @ C          # P[p, j] = l_j(xi_p)
        return np.sum(P * c.reshape(self.n, K)[e], axis=1)


def contact_solution(x, t, DL, DR, cL, cR):
    """Two semi-infinite media in contact (App. B.1): concentration and flux
    continuous at x = 0, so the contact value is
    c_m = (sqrt(DL) cL + sqrt(DR) cR) / (sqrt(DL) + sqrt(DR)) and each side
    relaxes from its initial value towards c_m as the error function of
    x / (2 sqrt(D t))."""
    from scipy.special import erfc
    cm = (math.sqrt(DL) * cL + math.sqrt(DR) * cR) / (math.sqrt(DL) + math.sqrt(DR))
    left = cL + (cm - cL) * erfc(-x / (2.0 * np.sqrt(DL * t)))
    right = cR + (cm - cR) * erfc(x / (2.0 * np.sqrt(DR * t)))
    return np.where(x < 0, left, right)


def rms_error(model, c, t, ref, window=None, pts=6):
    """e_rms of Eq. B4 by Gauss quadrature of (c - ref)^2 on every cell,
    over [-L/2, L/2] or the sub-interval `window`."""
    xi, w = np.polynomial.legendre.leggauss(pts)
    xc = model.x0 + model.h * (np.arange(model.n) + 0.5)
    x = (xc[:, None] + 0.5 * model.h * xi[None, :]).ravel()
    ww = np.tile(w * 0.5 * model.h, model.n)
    err2 = (model.evaluate(c, x) - ref(x, t)) ** 2
    if window is not None:
        keep = (x >= window[0]) & (x <= window[1])
        return math.sqrt(np.sum(ww[keep] * err2[keep]) / (window[1] - window[0]))
    return math.sqrt(np.sum(ww * err2) / model.L)

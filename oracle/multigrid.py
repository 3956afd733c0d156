"""Multilevel aggregation preconditioner of the Krylov system (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

The paper solves its linear systems with GMRES preconditioned by algebraic
multigrid (BoomerAMG, with options chosen for the elliptic potential
coupling; Sec. 2.9).  The GPU solver's counterpart is a geometric hierarchy
of voxel aggregates.  This module is its plain definition, written with
dense and sparse matrices so that every step can be read off:

* Level-1 aggregates are cubes of A x A x A voxels (x fastest; the last
  ones along an axis are thinner when A does not divide the mesh).  The
  aggregates of level l + 1 are the 2 x 2 x 2 groups of level-l aggregates
  by their integer coordinates (a // 2 per axis), so a level-l aggregate is
  a cube of A 2^(l-1) voxels per edge.
* Fine-to-level-1 basis: Z[(f, e, n), (f, a)] = s[f, e, n] when voxel e
  lies in aggregate a (s: positive weights per unknown, the unknown scales
  of the solver; all ones at the library's entry point), zero otherwise.
  Coarse vectors are ordered (f, a): field f, aggregate a.
* Level-to-level prolongation P_l: P[(f, a), (f, parent(a))] = 1.
* Galerkin operators: E_1 = Z^T J Z (J: the condensed 7-field tangent),
  E_{l+1} = P_l^T E_l P_l.
* Smoother: damped block Jacobi, x <- x + omega D_l^-1 (b - E_l x), with
  D_l the 7 x 7 diagonal blocks of E_l (the seven fields of one aggregate).
* V-cycle on level l with right side b: nu smoothing sweeps from x = 0, the
  level-(l+1) cycle on the restricted residual P_l^T (b - E_l x), its
  prolongation added to x, nu more sweeps; on the last level, x = E_L^-1 b
  exactly.
* Coarse correction of a fine vector r: Z V_1(Z^T r).  The solver adds it to
  the element block-Jacobi result (additive), or applies the blocks to the
  residual it leaves (multiplicative); the coarse correction alone is what
  the library's dg_mg_apply computes.
"""
from __future__ import annotations

import numpy as np

from . import dg


def aggregate_grid(nx, ny, nz, edge):
    """Aggregate counts per axis for cubes of edge^3 voxels."""
    return (-(-nx // edge), -(-ny // edge), -(-nz // edge))


def voxel_aggregates(nx, ny, nz, edge):
    """Aggregate index (x fastest) of every voxel, and the aggregate count."""
    e = np.arange(nx * ny * nz)
    ix, iy, iz = e % nx, (e // nx) % ny, e // (nx * ny)
    ax, ay, az = aggregate_grid(nx, ny, nz, edge)
    return (ix // edge) + ax * ((iy // edge) + ay * (iz // edge)), ax * ay * az


def level_grids(nx, ny, nz, edge, levels):
    """Aggregate grid (ax, ay, az) of levels 1..levels."""
    g = [aggregate_grid(nx, ny, nz, edge)]
    for _ in range(levels - 1):
        ax, ay, az = g[-1]
        g.append((-(-ax // 2), -(-ay // 2), -(-az // 2)))
    return g


def parent_map(grid):
    """Parent (next-level aggregate) of every aggregate of a level grid."""
    ax, ay, az = grid
    a = np.arange(ax * ay * az)
    x, y, z = a % ax, (a // ax) % ay, a // (ax * ay)
    px, py = -(-ax // 2), -(-ay // 2)
    return (x // 2) + px * ((y // 2) + py * (z // 2))


def prolongation(grid, nf=7):
    """P_l as a dense (nf na_l) x (nf na_{l+1}) 0/1 matrix, (field, aggregate) order."""
    par = parent_map(grid)
    na = len(par)
    nac = int(par.max()) + 1
    Pm = np.zeros((nf * na, nf * nac))
    for f in range(nf):
        Pm[f * na + np.arange(na), f * nac + par] = 1.0
    return Pm


def restrict_fine(r, agg, na, s=None):
    """Z^T r for a fine vector r of shape (nf, Ne, np): per field and
    aggregate, the sum of s r over the aggregate's nodes."""
    nf = r.shape[0]
    w = r if s is None else s * r
    out = np.zeros(nf * na)
    for f in range(nf):
        out[f * na:(f + 1) * na] = np.bincount(agg, weights=w[f].sum(axis=1), minlength=na)
    return out


def prolong_fine(y, agg, na, shape, s=None):
    """Z y as a fine vector of shape (nf, Ne, np)."""
    nf, Ne, npn = shape
    out = np.empty(shape)
    for f in range(nf):
        out[f] = np.repeat(y[f * na + agg][:, None], npn, axis=1)
    return out if s is None else s * out


def level1_operator(P, u, m_old, t_new, dt, edge, s=None):
    """E_1 = Z^T J Z, column by column: J (the condensed tangent at u, Krylov
    rows) applied to each basis vector Z_{f,a}, then restricted."""
    agg, na = voxel_aggregates(P.nx, P.ny, P.nz, edge)
    shape = (7, P.n_elem, P.n_nodes)
    E = np.zeros((7 * na, 7 * na))
    for f in range(7):
        for a in range(na):
            v = np.zeros(shape)
            v[f, agg == a, :] = 1.0
            if s is not None:
                v = s * v
            Jv = dg.jvp_condensed(P, u, v, m_old, t_new, dt)
            E[:, f * na + a] = restrict_fine(Jv, agg, na, s)
    return E


def hierarchy(E1, grid1, levels, nf=7):
    """Galerkin operators E_1..E_L and prolongations P_1..P_{L-1}."""
    Es, Ps, g = [E1], [], grid1
    for _ in range(levels - 1):
        Pm = prolongation(g, nf)
        Ps.append(Pm)
        Es.append(Pm.T @ Es[-1] @ Pm)
        ax, ay, az = g
        g = (-(-ax // 2), -(-ay // 2), -(-az // 2))
    return Es, Ps


def block_diagonal_inverse(E, nf=7):
    """Inverses of the nf x nf diagonal blocks (one per aggregate), shape (na, nf, nf)."""
    na = E.shape[0] // nf
    out = np.empty((na, nf, nf))
    for a in range(na):
        idx = np.arange(nf) * na + a
        out[a] = np.linalg.inv(E[np.ix_(idx, idx)])
    return out


def _jacobi(E, Dinv, x, b, omega, nf=7):
    na = E.shape[0] // nf
    r = (b - E @ x).reshape(nf, na)
    return x + omega * np.einsum("agf,fa->ga", Dinv, r).reshape(-1)


def vcycle(Es, Ps, b, nu=2, omega=0.7, level=0, Dinvs=None, nf=7):
    """V-cycle on level `level` (0-based) of the hierarchy with right side b."""
    E = Es[level]
    if level == len(Es) - 1:
        return np.linalg.solve(E, b)
    Dinv = Dinvs[level] if Dinvs is not None else block_diagonal_inverse(E, nf)
    x = np.zeros_like(b)
    for _ in range(nu):
        x = _jacobi(E, Dinv, x, b, omega, nf)
    Pm = Ps[level]
    xc = vcycle(Es, Ps, Pm.T @ (b - E @ x), nu, omega, level + 1, Dinvs, nf)
    x = x + Pm @ xc
    for _ in range(nu):
        x = _jacobi(E, Dinv, x, b, omega, nf)
    return x


def coarse_correction(P, r, Es, Ps, edge, nu=2, omega=0.7, s=None):
    """Z V_1(Z^T r) for a 7-field fine vector r of shape (7, Ne, np)."""
    agg, na = voxel_aggregates(P.nx, P.ny, P.nz, edge)
    y = vcycle(Es, Ps, restrict_fine(r, agg, na, s), nu, omega)
    return prolong_fine(y, agg, na, r.shape, s)

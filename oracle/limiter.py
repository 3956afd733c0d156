"""Vertex-based slope limiter for the Q1 scheme (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

The paper's DG1 computations use Kuzmin's vertex-based slope limiter
(App. B.1 and B.2), and its outlook (Sec. 4, with Sec. 2.7) asks for a
positivity-preserving p = 1 scheme.  This is that limiter, written from
Kuzmin's definition (D. Kuzmin, J. Comput. Appl. Math. 233 (2010)
3077-3085) for the trilinear polynomial of a voxel, applied after a step:

  * The limited quantities are the conserved densities m_i = eps_L c_i of
    the six dissolved species (the time term of Eq. 16a / Eq. 50), so the
    amount of every species in every voxel is unchanged; Phi_L and the
    solid fractions are not touched.
  * mbar_e, the mean of m over voxel e, is the quadrature mean of its
    nodal values (collocated Gauss nodes, equal weights).
  * Every mesh vertex v takes the largest and smallest mean over the voxels
    that share it, M_v and N_v.
  * For voxel e, the trilinear polynomial through its nodal values is
    evaluated at its eight corners, w_v.  The corner's ratio is
    (M_v - mbar_e)/(w_v - mbar_e) when w_v > mbar_e,
    (N_v - mbar_e)/(w_v - mbar_e) when w_v < mbar_e, and 1 when they are
    equal; alpha_e is the smallest ratio, at most 1.
  * The limited nodal values are mbar_e + alpha_e (m_a - mbar_e), and
    c_i = m_i / eps_L.

The limited polynomial keeps the voxel's mean, and its corner values lie in
[N_v, M_v]; a trilinear function takes values between its corner values, so
every nodal value lies between the smallest and largest voxel mean around
it.  When every mean is non-negative the limited state is non-negative:
this is the positivity property.  Degree 1 only (k = 0 has nothing to limit;
Kuzmin's hierarchical form for k > 1 is not used here).
"""
from __future__ import annotations

import numpy as np

from . import chem
from . import dg


def corner_matrix(k=1):
    """L[c, a]: value at corner c of the nodal basis function of node a.

    Corners c = cx + 2 cy + 4 cz (bit 0 = low, 1 = high side along each
    axis), nodes a = a0 + 2 a1 + 4 a2 as in the state layout."""
    if k != 1:
        raise ValueError("the vertex-based limiter is implemented for k = 1")
    xi, _ = dg.gl_nodes_weights(1)
    L1 = dg.lagrange_values(xi, np.array([-1.0, 1.0]))       # L1[side, node]
    L = np.empty((8, 8))
    for c in range(8):
        cb = [(c >> d) & 1 for d in range(3)]
        for a in range(8):
            ab = [(a >> d) & 1 for d in range(3)]
            L[c, a] = L1[cb[0], ab[0]] * L1[cb[1], ab[1]] * L1[cb[2], ab[2]]
    return L


def densities(P, u):
    """m[i] = eps_L c_i at every node (the conserved densities)."""
    eL = chem.liquid_fraction(P, u[7:9], P.epsCBD_e[:, None])
    return eL * u[0:6], eL


def vertex_bounds(P, mbar):
    """Largest and smallest voxel mean at every mesh vertex: arrays of shape
    (6, nz + 1, ny + 1, nx + 1)."""
    nx, ny, nz = P.nx, P.ny, P.nz
    g = mbar.reshape(6, nz, ny, nx)
    hi = np.full((6, nz + 1, ny + 1, nx + 1), -np.inf)
    lo = np.full((6, nz + 1, ny + 1, nx + 1), np.inf)
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                sl = (slice(None), slice(cz, cz + nz), slice(cy, cy + ny), slice(cx, cx + nx))
                hi[sl] = np.maximum(hi[sl], g)
                lo[sl] = np.minimum(lo[sl], g)
    return hi, lo


def limiter_factors(P, m):
    """alpha[i, e] of every species and voxel, with the voxel means."""
    nx, ny, nz = P.nx, P.ny, P.nz
    mbar = m.mean(axis=2)                                    # (6, Ne)
    hi, lo = vertex_bounds(P, mbar)
    w = np.einsum("ca,iea->iec", corner_matrix(1), m)        # corner values (6, Ne, 8)
    e = np.arange(P.n_elem)
    ix, iy, iz = e % nx, (e // nx) % ny, e // (nx * ny)
    alpha = np.ones((6, P.n_elem))
    for c in range(8):
        cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        Mv = hi[:, iz + cz, iy + cy, ix + cx]
        Nv = lo[:, iz + cz, iy + cy, ix + cx]
        d = w[:, :, c] - mbar
        r = np.ones_like(d)
        up, dn = d > 0, d < 0
        r[up] = (Mv[up] - mbar[up]) / d[up]
        r[dn] = (Nv[dn] - mbar[dn]) / d[dn]
        alpha = np.minimum(alpha, r)
    return alpha, mbar


def limit(P, u):
    """Limited copy of state u (9 fields, degree 1) and the factors alpha."""
    if P.k != 1:
        raise ValueError("the vertex-based limiter is implemented for k = 1")
    m, eL = densities(P, u)
    alpha, mbar = limiter_factors(P, m)
    ml = mbar[:, :, None] + alpha[:, :, None] * (m - mbar[:, :, None])
    out = u.copy()
    out[0:6] = ml / eL
    return out, alpha

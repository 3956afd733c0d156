"""Pins of the oracle's multilevel aggregation preconditioner (CPU).

oracle/multigrid.py is checked against what its definition fixes, by
routes other than its own formulas:
  * Galerkin nesting: the level-2 operator P^T E_1 P equals Z_2^T J Z_2
    formed directly from the fine matrix with aggregates of twice the edge
    (a wrong parent map, stride or ragged-edge rule fails it);
  * the two-level cycle without smoothing, I - P E_2^-1 P^T E_1, is a
    projection, and zero on the coarse space;
  * on a symmetric positive definite operator the V-cycle is a symmetric
    operator (pre- and post-smoothing must mirror each other and the
    restriction must be P^T);
  * as a stationary iteration on the seven-point Laplacian (a closed-form
    operator) the V-cycle contracts the error by 0.49 per cycle on 8^3
    aggregates and 0.68 on 16^3 (unsmoothed aggregation: the factor grows
    slowly with the number of levels), far below the same cycle with its
    coarse correction zeroed (four Jacobi sweeps: 0.70 and 0.86); a dropped
    or sign-flipped correction fails it;
  * the DG level-1 operator Z^T J Z, formed by the oracle's condensed
    Jacobian-vector products, equals the Schur complement of the oracle's
    complex-step probed sparse Jacobian (another route to the same
    condensed tangent) projected on the aggregates.
"""
import numpy as np
import pytest

import synth
from oracle import dg as odg
from oracle import model as om
from oracle import multigrid as mg
from oracle import solve as osolve


def _fine_basis(nx, ny, nz, npn, edge, nf=7, s=None):
    """Dense Z (fine (f, e, n) x coarse (f, a)) from the oracle's prolongation."""
    agg, na = mg.voxel_aggregates(nx, ny, nz, edge)
    shape = (nf, nx * ny * nz, npn)
    Z = np.empty((np.prod(shape), nf * na))
    for j in range(nf * na):
        y = np.zeros(nf * na)
        y[j] = 1.0
        Z[:, j] = mg.prolong_fine(y, agg, na, shape, s).reshape(-1)
    return Z


@pytest.mark.parametrize("dims", [(5, 4, 3), (4, 4, 4), (7, 3, 2)])
def test_galerkin_nesting_matches_direct_projection(dims):
    nx, ny, nz = dims
    npn, edge, nf = 2, 2, 3
    rng = np.random.default_rng(sum(dims))
    n = nf * nx * ny * nz * npn
    J = rng.standard_normal((n, n))
    s = np.exp(rng.standard_normal((nf, nx * ny * nz, npn)))
    Z1 = _fine_basis(nx, ny, nz, npn, edge, nf, s)
    Z2 = _fine_basis(nx, ny, nz, npn, 2 * edge, nf, s)
    E1 = Z1.T @ J @ Z1
    Es, Ps = mg.hierarchy(E1, mg.aggregate_grid(nx, ny, nz, edge), 2, nf)
    np.testing.assert_allclose(Es[1], Z2.T @ J @ Z2, rtol=1e-12, atol=1e-12 * np.abs(Es[1]).max())
    # restriction of a fine vector agrees with Z^T
    r = rng.standard_normal((nf, nx * ny * nz, npn))
    agg, na = mg.voxel_aggregates(nx, ny, nz, edge)
    np.testing.assert_allclose(mg.restrict_fine(r, agg, na, s), Z1.T @ r.reshape(-1), rtol=1e-13)


def test_two_level_correction_is_a_projection():
    rng = np.random.default_rng(3)
    grid = (4, 3, 3)
    n = 7 * np.prod(grid)
    E1 = rng.standard_normal((n, n)) + n * np.eye(n)
    Es, Ps = mg.hierarchy(E1, grid, 2)
    V = np.column_stack([mg.vcycle(Es, Ps, e, nu=0) for e in np.eye(n)])
    T = np.eye(n) - V @ E1
    np.testing.assert_allclose(T @ T, T, atol=1e-10)
    np.testing.assert_allclose(T @ Ps[0], 0.0, atol=1e-10)


def _laplacian(grid, nf=7, shift=0.0):
    """nf uncoupled copies of the seven-point Laplacian (Dirichlet outside)."""
    ax, ay, az = grid
    na = ax * ay * az
    L = np.zeros((na, na))
    for a in range(na):
        x, y, z = a % ax, (a // ax) % ay, a // (ax * ay)
        L[a, a] = 6.0 + shift
        for d, (dx, dy, dz) in enumerate([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]):
            xx, yy, zz = x + dx, y + dy, z + dz
            if 0 <= xx < ax and 0 <= yy < ay and 0 <= zz < az:
                L[a, xx + ax * (yy + ay * zz)] = -1.0
    return np.kron(np.eye(nf), L)


def test_vcycle_is_symmetric_on_a_symmetric_operator():
    rng = np.random.default_rng(5)
    grid = (6, 5, 4)
    E1 = _laplacian(grid)
    na = np.prod(grid)
    # couple the fields of each aggregate symmetrically (stays SPD)
    C = rng.standard_normal((7, 7))
    C = 0.1 * (C + C.T)
    E1 = E1 + np.kron(C, np.eye(na))
    Es, Ps = mg.hierarchy(E1, grid, 3)
    x, y = rng.standard_normal(7 * na), rng.standard_normal(7 * na)
    a = x @ mg.vcycle(Es, Ps, y)
    b = y @ mg.vcycle(Es, Ps, x)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def _contraction(E, step, iters=12, seed=0):
    rng = np.random.default_rng(seed)
    n = E.shape[0]
    b = rng.standard_normal(n)
    xs = np.linalg.solve(E, b)
    x = np.zeros(n)
    e0 = np.linalg.norm(xs)
    for _ in range(iters):
        x = x + step(b - E @ x)
    return (np.linalg.norm(xs - x) / e0) ** (1.0 / iters)


@pytest.mark.parametrize("edge,bound", [(8, 0.55), (16, 0.72)])
def test_vcycle_contracts_on_the_laplacian(edge, bound):
    grid = (edge, edge, edge)
    nf = 1
    E = _laplacian(grid, nf)
    levels = int(np.log2(edge))             # down to 2^3 on the last level
    Es, Ps = mg.hierarchy(E, grid, levels, nf)
    Dinvs = [mg.block_diagonal_inverse(Ek, nf) for Ek in Es[:-1]]
    rho_v = _contraction(E, lambda r: mg.vcycle(Es, Ps, r, nu=2, omega=0.7, Dinvs=Dinvs, nf=nf))
    # the same cycle with the coarse correction zeroed: smoothing only
    Pz = [np.zeros_like(Ps[0])] + Ps[1:]
    rho_s = _contraction(E, lambda r: mg.vcycle(Es, Pz, r, nu=2, omega=0.7, Dinvs=Dinvs, nf=nf))
    assert rho_v < bound, rho_v
    assert rho_s > 0.65 and rho_v < 0.8 * rho_s, (rho_v, rho_s)


def test_dg_level1_operator_equals_projected_schur_complement():
    nx, ny, nz, edge = 3, 2, 2, 2
    mask = synth.porosity_mask((nz, ny, nx), 0.5, 4)
    D0, i0 = synth.sample_transport_kinetics(4)
    P = om.Problem(nx, ny, nz, 1e-6, 1, mask, D0=D0, kE=i0 / om.F, f_C=0.1)
    u = synth.random_state(P.n_elem, P.n_nodes, 7, phase=mask, phi_spread=5e-3)
    m_old = odg.old_mass(P, synth.random_state(P.n_elem, P.n_nodes, 8, phase=mask))
    t_new, dt = 0.3, 0.1
    s = np.exp(0.3 * np.random.default_rng(9).standard_normal((7, P.n_elem, P.n_nodes)))
    E1 = mg.level1_operator(P, u, m_old, t_new, dt, edge, s)
    # condensed tangent from the full probed Jacobian: J_uu - J_ue J_ee^-1 J_eu
    Jf = osolve.sparse_jacobian(P, u, m_old, t_new, dt).toarray()
    n7 = 7 * P.n_elem * P.n_nodes
    Juu, Jue, Jeu, Jee = Jf[:n7, :n7], Jf[:n7, n7:], Jf[n7:, :n7], Jf[n7:, n7:]
    Jred = Juu - Jue @ np.linalg.solve(Jee, Jeu)
    Z = _fine_basis(nx, ny, nz, P.n_nodes, edge, 7, s)
    ref = Z.T @ Jred @ Z
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.max(np.abs(E1 - ref) / scale) < 1e-9

"""Pins of the oracle's DG residual and Jacobian products (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import chem, dg, solve
from oracle import model as M


def _prob(nx, ny, nz, k, mask=None, seed=0, **kw):
    if mask is None:
        mask = synth.porosity_mask((nz, ny, nx), 0.6, seed)
    D0, i0 = synth.sample_transport_kinetics(seed)
    kw.setdefault("D0", D0)
    kw.setdefault("kE", i0 / M.F)
    return M.Problem(nx, ny, nz, 1e-6, k, mask, **kw)


def _eq_state(P):
    return solve.uniform_state(P)


# --------------------------------------------------------------------------
def test_basis_partition_of_unity_and_exact_derivatives():
    for k in range(4):
        B = dg.basis(k)
        assert abs(B.w.sum() - 2.0) < 1e-14
        x = np.linspace(-1, 1, 7)
        L = dg.lagrange_values(B.xi, x)
        assert np.allclose(L.sum(axis=1), 1.0, atol=1e-14)
        # derivative of x^k interpolated on the nodes is k x^(k-1)
        if k >= 1:
            D = dg.lagrange_derivatives(B.xi, x)
            assert np.allclose(D @ B.xi ** k, k * x ** (k - 1), atol=1e-12)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_residual_vanishes_at_equilibrium(k):
    """Uniform equilibrium state, no current: every flux and source is zero
    for any mask (the pin of Sec. 2.10's consistent initial state)."""
    P = _prob(3, 4, 2, k, seed=k, j_el=0.0)
    u = _eq_state(P)
    R = dg.residual(P, u, dg.old_mass(P, u), 7.0, 0.1)
    # scale: the largest single flux-type contribution with O(1) gradients
    assert np.max(np.abs(R[0:6])) < 1e-24
    assert np.max(np.abs(R[6])) < 1e-22
    assert np.max(np.abs(R[7:9])) < 1e-30


def _fv7_residual(P, u, m_old, t, dt):
    """Eq. 48 written cell by cell and face by face (k = 0 only)."""
    h = P.h
    R = np.zeros_like(u)
    Ne = P.n_elem
    eCBD = P.epsCBD_e
    for e in range(Ne):
        c, phi, eps = u[0:6, e, 0], u[6, e, 0], u[7:9, e, 0]
        eL = max(1.0 - eCBD[e] - eps[0] - eps[1], P.epsL_min)
        for i in range(6):
            R[i, e, 0] += h ** 3 * (eL * c[i] - m_old[i, e, 0]) / dt
        rhoM = M.RHO / M.MOLAR
        for s in range(2):
            R[7 + s, e, 0] += h ** 3 * rhoM[s] * (eps[s] - m_old[6 + s, e, 0]) / dt
        Sl, Sp, Ss, _, _ = chem.sources(P, c[:, None], np.array([phi]), eps[:, None], t,
                                        P.aV0_e[e], P.epsS8_0_e[e], P.pass_e[e], P.react_e[e])
        R[0:6, e, 0] -= h ** 3 * Sl[:, 0]
        R[6, e, 0] -= h ** 3 * Sp[0]
        R[7:9, e, 0] -= h ** 3 * Ss[:, 0]

    def coef(e):
        D, Mi, K, kap = chem.transport_coefficients(P, u[0:6, e, :1], u[7:9, e, :1], eCBD[e])
        return D[:, 0], Mi[:, 0], K[:, 0], kap[0]

    def H(a, b):
        return 2 * a * b / (a + b) if a * b > 0 else 0.0

    def face(eL_, eR_):
        DL, ML, KL, kL = coef(eL_)
        DR, MR, KR, kR = coef(eR_)
        cL, cR = u[0:6, eL_, 0], u[0:6, eR_, 0]
        pL, pR = u[6, eL_, 0], u[6, eR_, 0]
        for i in range(6):
            q = (H(DL[i], DR[i]) * (cL[i] - cR[i]) + H(ML[i], MR[i]) * (pL - pR)) / h * h ** 2
            R[i, eL_, 0] += q
            R[i, eR_, 0] -= q
        q = (sum(H(KL[j], KR[j]) * (cL[j] - cR[j]) for j in range(6)) + H(kL, kR) * (pL - pR)) / h * h ** 2
        R[6, eL_, 0] += q
        R[6, eR_, 0] -= q

    idx = lambda ix, iy, iz: ix + P.nx * (iy + P.ny * iz)
    for iz in range(P.nz):
        for iy in range(P.ny):
            for ix in range(P.nx):
                if ix + 1 < P.nx:
                    face(idx(ix, iy, iz), idx(ix + 1, iy, iz))
                if iy + 1 < P.ny:
                    face(idx(ix, iy, iz), idx(ix, iy + 1, iz))
                if iz + 1 < P.nz:
                    face(idx(ix, iy, iz), idx(ix, iy, iz + 1))
            e = idx(P.nx - 1, iy, iz)
            R[0, e, 0] -= h ** 2 * P.j_el / M.F
            R[6, e, 0] -= h ** 2 * P.j_el
    return R


def test_k0_is_the_seven_point_finite_volume_scheme():
    """At p = 0 the DG form is the FV scheme with harmonic-mean two-point
    fluxes of Eq. 48 (migration through the penalty of its own coefficient)."""
    P = _prob(3, 3, 2, 0, seed=2)
    u = synth.random_state(P.n_elem, 1, 5, phase=P.phase, phi_spread=5e-3)
    m = dg.old_mass(P, synth.random_state(P.n_elem, 1, 6, phase=P.phase))
    R = dg.residual(P, u, m, 2.0, 0.1)
    Rf = _fv7_residual(P, u, m, 2.0, 0.1)
    for f in range(9):
        scale = np.max(np.abs(Rf[f])) + 1e-300
        assert np.max(np.abs(R[f] - Rf[f])) <= 1e-13 * scale, f


def _pore_problem(nx, ny, nz, k):
    D0, _ = synth.sample_transport_kinetics(0)       # D_Li != D_anion, so K_Li != 0
    return M.Problem(nx, ny, nz, 1e-6, k, np.zeros((nz, ny, nx), np.uint8), j_el=0.0,
                     eps_struct=1.0, D0=D0)


def _node_coords(P):
    """Physical coordinates (x, y, z) of every node, shape (3, Ne, np)."""
    B = dg.basis(P.k)
    g = dg.element_grid(P)
    iz, iy, ix = np.meshgrid(np.arange(P.nz), np.arange(P.ny), np.arange(P.nx), indexing="ij")
    base = [ix.reshape(-1), iy.reshape(-1), iz.reshape(-1)]
    X = np.zeros((3, P.n_elem, P.n_nodes))
    for n, a in enumerate(B.idx):
        for d in range(3):
            X[d, :, n] = (base[d] + 0.5 * (B.xi[a[d]] + 1.0)) * P.h
    return X


@pytest.mark.parametrize("k,deg", [(1, 1), (2, 2), (3, 2), (3, 3)])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_polynomial_consistency(k, deg, axis):
    """For c_Li a polynomial of degree <= k along one axis (all-pore mask,
    uniform everything else), interior elements give exactly the weak form of
    -div(D grad c): R_a = -W_a D c''(x_a) (Eq. 43 + 46 with exact quadrature)."""
    P = _pore_problem(4, 4, 4, k)
    u = _eq_state(P)
    X = _node_coords(P)[axis] / P.h           # in voxel units
    coefs = {1: [0.0, 30.0], 2: [0.0, 20.0, -7.0], 3: [0.0, 10.0, -6.0, 1.5]}[deg]
    cpoly = sum(a * X ** p for p, a in enumerate(coefs))
    d2 = np.zeros_like(X) + sum(p * (p - 1) * a * X ** (p - 2) for p, a in enumerate(coefs) if p >= 2) / P.h ** 2
    u[0] = 1500.0 + cpoly
    m = dg.old_mass(P, u)
    R = dg.residual(P, u, m, 5.0, 0.1)
    D, _, K, _ = chem.transport_coefficients(P, u[0:6, :1, :1], u[7:9, :1, :1], 0.0)
    B = dg.basis(k)
    W = B.W3[None, :] * (P.h / 2) ** 3
    g = dg.element_grid(P)
    inner = [slice(None)] * 3
    inner[2 - axis] = slice(1, -1)
    sel = g[tuple(inner)].reshape(-1)
    ref_li = -W * D[0, 0, 0] * d2
    ref_phi = -W * K[0, 0, 0] * d2
    scale = np.max(np.abs(W * D[0, 0, 0] * 30.0 / P.h ** 2))
    assert np.max(np.abs(R[0, sel] - ref_li[sel])) < 1e-10 * scale
    scale_p = np.max(np.abs(W * K[0, 0, 0] * 30.0 / P.h ** 2))
    assert np.max(np.abs(R[6, sel] - ref_phi[sel])) < 1e-10 * scale_p
    assert np.max(np.abs(R[1:6])) < 1e-12 * scale


@pytest.mark.parametrize("k", [1, 3])
def test_penalty_of_a_discontinuity(k):
    """Piecewise-constant c_Li on two voxels: only the penalty acts, and the
    element total is (sigma/h) {D}_H (c^- - c^+) |face| (Eq. 45-46)."""
    P = _pore_problem(2, 1, 1, k)
    u = _eq_state(P)
    u[0, 0] = 1600.0
    u[0, 1] = 1400.0
    m = dg.old_mass(P, u)
    R = dg.residual(P, u, m, 5.0, 0.1)
    D, _, K, _ = chem.transport_coefficients(P, u[0:6, :, :1], u[7:9, :, :1], 0.0)
    sigma = (k + 1) ** 2
    tot = sigma / P.h * D[0, 0, 0] * 200.0 * P.h ** 2
    assert abs(R[0, 0].sum() / tot - 1.0) < 1e-12
    assert abs(R[0, 1].sum() / tot + 1.0) < 1e-12
    totp = sigma / P.h * K[0, 0, 0] * 200.0 * P.h ** 2
    assert abs(R[6, 0].sum() / totp - 1.0) < 1e-12


def test_discrete_conservation_sums():
    """Testing with phi = 1 on every element: transport cancels face by face, so
    each row sums to its time term minus its source minus the separator inflow
    (local conservation of DG, Sec. 2.7)."""
    P = _prob(4, 3, 3, 1, seed=4)
    u = synth.random_state(P.n_elem, P.n_nodes, 11, phase=P.phase, phi_spread=5e-3)
    m = dg.old_mass(P, synth.random_state(P.n_elem, P.n_nodes, 12, phase=P.phase))
    dt, t = 0.2, 3.0
    R = dg.residual(P, u, m, t, dt)
    B = dg.basis(1)
    W = B.W3[None, :] * (P.h / 2) ** 3
    eL = chem.liquid_fraction(P, u[7:9], P.epsCBD_e[:, None])
    Sl, Sp, Ss, _, _ = chem.sources(P, u[0:6], u[6], u[7:9], t, P.aV0_e[:, None],
                                    P.epsS8_0_e[:, None], P.pass_e[:, None], P.react_e[:, None])
    A = P.ny * P.nz * P.h ** 2
    for i in range(6):
        expect = np.sum(W * (eL * u[i] - m[i]) / dt) - np.sum(W * Sl[i]) - (P.j_el * A / M.F if i == 0 else 0.0)
        scale = np.sum(np.abs(W * eL * u[i] / dt)) + np.sum(np.abs(R[i]))
        assert abs(R[i].sum() - expect) < 1e-12 * scale, i
    expect = -np.sum(W * Sp) - P.j_el * A
    assert abs(R[6].sum() - expect) < 1e-12 * (np.sum(np.abs(R[6])) + abs(expect))


def test_laterally_uniform_equals_one_dimensional():
    """A mask and state that depend on x only give the same residual per voxel
    as the nx x 1 x 1 column: lateral faces carry nothing."""
    k = 1
    rng = np.random.default_rng(5)
    line = (rng.random(5) < 0.5).astype(np.uint8)
    line[0] = 1
    m3 = np.broadcast_to(line[None, None, :], (3, 2, 5)).copy()
    m1 = line[None, None, :].copy()
    P3 = _prob(5, 2, 3, k, mask=m3)
    P1 = _prob(5, 1, 1, k, mask=m1)
    assert abs(P3.j_el - P1.j_el) < 1e-15 * P1.j_el
    u1 = synth.random_state(5, 8, 21, phase=m1, phi_spread=4e-3)
    # make the 1D state laterally uniform within each voxel: nodes depend on a0 only
    B = dg.basis(k)
    a0 = np.array([a[0] for a in B.idx])
    u1 = u1[:, :, a0]
    m_1 = dg.old_mass(P1, synth.random_state(5, 8, 22, phase=m1)[:, :, a0])
    R1 = dg.residual(P1, u1, m_1, 4.0, 0.1)
    u3 = np.tile(u1, (1, 6, 1))
    m_3 = np.tile(m_1, (1, 6, 1))
    R3 = dg.residual(P3, u3, m_3, 4.0, 0.1)
    for f in range(9):
        scale = np.max(np.abs(R1[f])) + 1e-300
        assert np.max(np.abs(R3[f] - np.tile(R1[f], (6, 1)))) < 1e-12 * scale, f


def test_mirror_symmetry_in_y():
    k = 1
    P = _prob(3, 4, 2, k, seed=6)
    u = synth.random_state(P.n_elem, 8, 31, phase=P.phase, phi_spread=4e-3)
    m = dg.old_mass(P, synth.random_state(P.n_elem, 8, 32, phase=P.phase))
    B = dg.basis(k)
    perm = np.array([B.idx.index((a[0], k - a[1], a[2])) for a in B.idx])

    def mirror(x):
        x = x.reshape(x.shape[0], P.nz, P.ny, P.nx, -1)[:, :, ::-1]
        return x.reshape(x.shape[0], P.n_elem, -1)[:, :, perm]

    Pm = _prob(3, 4, 2, k, mask=P.phase[:, ::-1, :].copy(), seed=6)
    R = dg.residual(P, u, m, 3.0, 0.1)
    Rm = dg.residual(Pm, mirror(u), mirror(m), 3.0, 0.1)
    for f in range(9):
        scale = np.max(np.abs(R[f])) + 1e-300
        assert np.max(np.abs(Rm[f] - mirror(R)[f])) < 1e-12 * scale, f


# --------------------------------------------------------------------------
def _dense_jacobian(P, u, m, t, dt):
    n = u.size
    J = np.zeros((n, n))
    for j in range(n):
        v = np.zeros(n)
        v[j] = 1.0
        J[:, j] = dg.jvp(P, u, v.reshape(u.shape), m, t, dt).reshape(-1)
    return J


@pytest.fixture(scope="module")
def tiny():
    P = _prob(2, 2, 2, 1, seed=1)
    u = synth.random_state(P.n_elem, 8, 41, phase=P.phase, phi_spread=4e-3)
    m = dg.old_mass(P, synth.random_state(P.n_elem, 8, 42, phase=P.phase))
    J = _dense_jacobian(P, u, m, 2.0, 0.1)
    return P, u, m, J


def test_jvp_matches_central_differences(tiny):
    P, u, m, _ = tiny
    rng = np.random.default_rng(3)
    S = np.maximum(np.abs(u), 1e-3 * np.abs(u).max(axis=(1, 2), keepdims=True) + 1e-12)
    v = S * rng.standard_normal(u.shape)
    d = 1e-6
    fd = (dg.residual(P, u + d * v, m, 2.0, 0.1) - dg.residual(P, u - d * v, m, 2.0, 0.1)) / (2 * d)
    Jv = dg.jvp(P, u, v, m, 2.0, 0.1)
    for f in range(9):
        scale = np.max(np.abs(Jv[f])) + 1e-300
        assert np.max(np.abs(Jv[f] - fd[f])) < 1e-6 * scale, f


def test_element_blocks_are_diagonal_blocks_of_the_jacobian(tiny):
    P, u, m, J = tiny
    blocks = solve.element_blocks(P, u, m, 2.0, 0.1)
    Ne, npn = P.n_elem, P.n_nodes
    idx = lambda f, e, a: (f * Ne + e) * npn + a
    for e in range(Ne):
        rows = [idx(f, e, a) for f in range(9) for a in range(npn)]
        ref = J[np.ix_(rows, rows)]
        assert np.allclose(blocks[e], ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_sparse_jacobian_equals_dense(tiny):
    P, u, m, J = tiny
    Js = solve.sparse_jacobian(P, u, m, 2.0, 0.1).toarray()
    assert np.allclose(Js, J, rtol=0, atol=1e-14 * np.abs(J).max())


def test_condensed_jvp_is_the_schur_complement(tiny):
    """J_red = J_uu - J_ue J_ee^-1 J_eu with the solid fractions eliminated."""
    P, u, m, J = tiny
    Ne, npn = P.n_elem, P.n_nodes
    nu = 7 * Ne * npn
    Juu, Jue, Jeu, Jee = J[:nu, :nu], J[:nu, nu:], J[nu:, :nu], J[nu:, nu:]
    Jred = Juu - Jue @ np.linalg.solve(Jee, Jeu)
    v = synth.random_vector(7, Ne, npn, 5)
    got = dg.jvp_condensed(P, u, v, m, 2.0, 0.1).reshape(-1)
    ref = Jred @ v.reshape(-1)
    for f in range(7):
        sl = slice(f * Ne * npn, (f + 1) * Ne * npn)
        scale = np.max(np.abs(ref[sl])) + 1e-300
        assert np.max(np.abs(got[sl] - ref[sl])) < 1e-10 * scale, f


@pytest.fixture(scope="module")
def tiny3():
    """k = 3 (64 nodes per voxel) on 2 x 2 x 1 voxels."""
    P = _prob(2, 2, 1, 3, seed=2)
    u = synth.random_state(P.n_elem, P.n_nodes, 43, phase=P.phase, phi_spread=4e-3)
    m = dg.old_mass(P, synth.random_state(P.n_elem, P.n_nodes, 44, phase=P.phase))
    return P, u, m


def test_jvp_matches_central_differences_at_degree_three(tiny3):
    P, u, m = tiny3
    rng = np.random.default_rng(4)
    S = np.maximum(np.abs(u), 1e-3 * np.abs(u).max(axis=(1, 2), keepdims=True) + 1e-12)
    v = S * rng.standard_normal(u.shape)
    d = 1e-6
    fd = (dg.residual(P, u + d * v, m, 2.0, 0.1) - dg.residual(P, u - d * v, m, 2.0, 0.1)) / (2 * d)
    Jv = dg.jvp(P, u, v, m, 2.0, 0.1)
    for f in range(9):
        scale = np.max(np.abs(Jv[f])) + 1e-300
        assert np.max(np.abs(Jv[f] - fd[f])) < 1e-6 * scale, f


def test_element_blocks_at_degree_three_are_jacobian_columns(tiny3):
    """Sampled columns of each 576 x 576 element block equal the element's
    rows of J e_j (J e_j by the complex-step product)."""
    P, u, m = tiny3
    blocks = solve.element_blocks(P, u, m, 2.0, 0.1)
    Ne, npn = P.n_elem, P.n_nodes
    rng = np.random.default_rng(6)
    for e in range(Ne):
        for col in rng.choice(9 * npn, size=6, replace=False):
            f, a = divmod(int(col), npn)
            v = np.zeros_like(u)
            v[f, e, a] = 1.0
            Jv = dg.jvp(P, u, v, m, 2.0, 0.1)
            ref = Jv[:, e, :].reshape(-1)
            scale = np.abs(blocks[e]).max()
            assert np.max(np.abs(blocks[e][:, col] - ref)) < 1e-14 * scale, (e, f, a)

"""Pins of the oracle's vertex-based Q1 limiter and of its 1D App. B engine (CPU).

The limiter (oracle/limiter.py) is checked against what its definition
fixes, not against a retyping of its formulas:
  * every voxel keeps the mean of each conserved density eps_L c_i;
  * every limited corner value lies within the largest and smallest voxel
    mean at that vertex, and every nodal value within those of its voxel;
  * alpha is the largest factor in [0, 1] that satisfies the corner
    bounds (found here by bisection on the bounds themselves);
  * a globally trilinear field is left alone in voxels away from the
    boundary, and a state with non-negative means comes out non-negative;
  * App. B.1 (diffusion across a discontinuity, Eq. B2-B4): the 1D engine
    converges at first order for DG0, and at least at first order for DG1
    with the limiter applied after every step, against the contact
    solution; unlimited DG1 undershoots below c_L at the discontinuity, as
    the paper reports, and the limited DG1 states stay within the means of
    their neighbourhood at every step.  (The paper also finds DG1 at first
    order with the larger error; this engine's DG1 converges at second
    order inside the window, so that is not asserted.)
"""
import numpy as np
import pytest

from oracle import appb, limiter
from oracle import model as M


def _problem(nx, ny, nz, seed=0, struct=0.4):
    rng = np.random.default_rng(seed)
    phase = (rng.random((nz, ny, nx)) < struct).astype(np.uint8)
    return M.Problem(nx, ny, nz, 1e-6, 1, phase)


def _state(P, seed, spread=0.5):
    """A smooth variation over the voxels (one period per mesh) plus nodal
    noise of relative size `spread`."""
    rng = np.random.default_rng(seed)
    u = np.empty((9, P.n_elem, 8))
    base = np.array([1000.0, 5.0, 6e-3, 4e-3, 2e-3, 4e-12])
    e = np.arange(P.n_elem)
    ix, iy, iz = e % P.nx, (e // P.nx) % P.ny, e // (P.nx * P.ny)
    x = (ix[:, None] + 0.5 + 0.29 * (2 * (np.arange(8)[None, :] & 1) - 1)) / P.nx
    y = (iy[:, None] + 0.5 + 0.29 * (2 * (np.arange(8)[None, :] >> 1 & 1) - 1)) / P.ny
    z = (iz[:, None] + 0.5 + 0.29 * (2 * (np.arange(8)[None, :] >> 2 & 1) - 1)) / P.nz
    smooth = 0.5 * np.sin(2 * np.pi * x + 1.0) * np.cos(2 * np.pi * y) + 0.3 * np.sin(2 * np.pi * z)
    u[0:6] = base[:, None, None] * np.exp(smooth[None] + spread * rng.standard_normal((6, P.n_elem, 8)))
    u[6] = 1e-3 * rng.standard_normal((P.n_elem, 8))
    struct = P.epsCBD_e > 0
    u[7] = np.where(struct[:, None], 0.2 + 0.05 * rng.random((P.n_elem, 8)), 0.0)
    u[8] = np.where(struct[:, None], 1e-5 * rng.random((P.n_elem, 8)), 0.0)
    return u


def test_means_are_kept_and_other_fields_untouched():
    P = _problem(5, 4, 3, seed=1)
    u = _state(P, 2, spread=0.01)
    ul, alpha = limiter.limit(P, u)
    m0, _ = limiter.densities(P, u)
    m1, _ = limiter.densities(P, ul)
    np.testing.assert_allclose(m1.mean(axis=2), m0.mean(axis=2), rtol=1e-14, atol=0)
    assert np.array_equal(ul[6:], u[6:])
    assert np.all((alpha >= 0) & (alpha <= 1)) and np.any(alpha < 1) and np.any(alpha == 1)


def test_corner_and_nodal_values_respect_the_vertex_bounds():
    P = _problem(6, 5, 4, seed=3)
    u = _state(P, 4)
    ul, _ = limiter.limit(P, u)
    m, _ = limiter.densities(P, ul)
    mbar = m.mean(axis=2)
    hi, lo = limiter.vertex_bounds(P, limiter.densities(P, u)[0].mean(axis=2))
    w = np.einsum("ca,iea->iec", limiter.corner_matrix(), m)
    e = np.arange(P.n_elem)
    ix, iy, iz = e % P.nx, (e // P.nx) % P.ny, e // (P.nx * P.ny)
    for c in range(8):
        cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        Mv, Nv = hi[:, iz + cz, iy + cy, ix + cx], lo[:, iz + cz, iy + cy, ix + cx]
        tol = 1e-12 * np.abs(mbar)
        assert np.all(w[:, :, c] <= Mv + tol) and np.all(w[:, :, c] >= Nv - tol)
    # nodal values lie between the voxel's smallest and largest corner bound
    cmax = np.max([hi[:, iz + (c >> 2 & 1), iy + (c >> 1 & 1), ix + (c & 1)] for c in range(8)], axis=0)
    cmin = np.min([lo[:, iz + (c >> 2 & 1), iy + (c >> 1 & 1), ix + (c & 1)] for c in range(8)], axis=0)
    assert np.all(m <= cmax[:, :, None] * (1 + 1e-12)) and np.all(m >= cmin[:, :, None] * (1 - 1e-12))


def test_alpha_is_the_largest_admissible_factor():
    """Bisection on the bounds alone: the largest a in [0, 1] for which
    mbar + a (w - mbar) lies in [N_v, M_v] at every corner."""
    P = _problem(4, 3, 3, seed=5)
    u = _state(P, 6)
    m, _ = limiter.densities(P, u)
    alpha, mbar = limiter.limiter_factors(P, m)
    hi, lo = limiter.vertex_bounds(P, mbar)
    w = np.einsum("ca,iea->iec", limiter.corner_matrix(), m)
    rng = np.random.default_rng(0)
    for _ in range(60):
        i, e = rng.integers(0, 6), rng.integers(0, P.n_elem)
        ix, iy, iz = e % P.nx, (e // P.nx) % P.ny, e // (P.nx * P.ny)
        Mv = np.array([hi[i, iz + (c >> 2 & 1), iy + (c >> 1 & 1), ix + (c & 1)] for c in range(8)])
        Nv = np.array([lo[i, iz + (c >> 2 & 1), iy + (c >> 1 & 1), ix + (c & 1)] for c in range(8)])

        def ok(a):
            v = mbar[i, e] + a * (w[i, e] - mbar[i, e])
            return np.all(v <= Mv) and np.all(v >= Nv)

        a0, a1 = 0.0, 1.0
        if ok(1.0):
            best = 1.0
        else:
            for _ in range(60):
                mid = 0.5 * (a0 + a1)
                a0, a1 = (mid, a1) if ok(mid) else (a0, mid)
            best = a0
        assert abs(alpha[i, e] - best) <= 1e-9, (i, e, alpha[i, e], best)


def test_a_trilinear_field_is_kept_away_from_the_boundary():
    P = _problem(6, 6, 6, seed=0, struct=0.0)          # all pore: eps_L = 1
    u = _state(P, 1)
    g = 1.0 / np.sqrt(3.0)
    e = np.arange(P.n_elem)
    ix, iy, iz = e % P.nx, (e // P.nx) % P.ny, e // (P.nx * P.ny)
    for a in range(8):
        x = ix + 0.5 + 0.5 * g * (2 * (a & 1) - 1)
        y = iy + 0.5 + 0.5 * g * (2 * (a >> 1 & 1) - 1)
        z = iz + 0.5 + 0.5 * g * (2 * (a >> 2 & 1) - 1)
        u[0, :, a] = 100.0 + 3.0 * x - 2.0 * y + 1.5 * z + 0.25 * x * y * z
    ul, alpha = limiter.limit(P, u)
    inner = (ix > 0) & (ix < P.nx - 1) & (iy > 0) & (iy < P.ny - 1) & (iz > 0) & (iz < P.nz - 1)
    assert np.all(alpha[0, inner] == 1.0)
    np.testing.assert_array_equal(ul[0, inner], u[0, inner])


def test_non_negative_means_give_a_non_negative_state():
    P = _problem(5, 5, 4, seed=7)
    u = _state(P, 8, spread=0.2)
    rng = np.random.default_rng(9)
    # push some nodes below zero while keeping every voxel mean positive
    m, eL = limiter.densities(P, u)
    dev = rng.standard_normal(m.shape)
    dev -= dev.mean(axis=2, keepdims=True)
    m = m + 1.5 * m.mean(axis=2, keepdims=True) * dev
    u[0:6] = m / eL
    assert np.any(u[0:6] < 0)
    ul, _ = limiter.limit(P, u)
    assert np.all(ul[0:6] >= -1e-12 * np.abs(u[0:6]).max())


# --------------------------------------------------------------------------
# App. B.1: diffusion across a discontinuity
# --------------------------------------------------------------------------
L, DL, DR, CL, CR = 0.2, 1e-4, 1e-3, 0.0, 1.0
DT, T_EVAL = 1e-4, 0.8
# |x| <= L/4: the contact solution is that of two unbounded media; inside
# this window the no-flux ends change it by less than 1e-4 at t = 0.8 s
WINDOW = (-L / 4, L / 4)


def _limit_1d(P, model, c):
    """The 3D limiter on an n x 1 x 1 pore mesh, the 1D state copied to
    the four nodes of each x-line position."""
    u = np.zeros((9, model.n, 8))
    cc = c.reshape(model.n, 2)
    for a in range(8):
        u[0, :, a] = cc[:, a & 1]
    ul, _ = limiter.limit(P, u)
    return ul[0][:, [0, 1]].reshape(-1)


def _run(n, k, limit):
    D = np.where((np.arange(n) + 0.5) * (L / n) - L / 2 < 0, DL, DR)
    model = appb.Diffusion1D(n, k, L, D)
    x = model.nodes_x()
    c = np.where(x < 0, CL, CR).astype(float)
    model.factor(DT)
    P = M.Problem(n, 1, 1, L / n, 1, np.zeros((1, 1, n), np.uint8)) if limit else None
    lo_seen = np.inf
    for _ in range(int(round(T_EVAL / DT))):
        c = model.step(c)
        if limit:
            mb = model.means(c)
            c = _limit_1d(P, model, c)
            # every limited nodal value between the means of its neighbourhood
            cc = c.reshape(n, 2)
            pad = np.concatenate([[mb[0]], mb, [mb[-1]]])
            nb_lo = np.minimum(np.minimum(pad[:-2], pad[1:-1]), pad[2:])
            nb_hi = np.maximum(np.maximum(pad[:-2], pad[1:-1]), pad[2:])
            assert np.all(cc >= nb_lo[:, None] - 1e-13) and np.all(cc <= nb_hi[:, None] + 1e-13)
        lo_seen = min(lo_seen, c.min())

    def ref(xx, t):
        return appb.contact_solution(xx, t, DL, DR, CL, CR)

    return appb.rms_error(model, c, T_EVAL, ref, WINDOW), lo_seen


@pytest.fixture(scope="module")
def contact_errors():
    out = {}
    for ndof in (100, 200, 400):
        out[("dg0", ndof)] = _run(ndof, 0, False)
        out[("dg1", ndof)] = _run(ndof // 2, 1, False)
        out[("dg1lim", ndof)] = _run(ndof // 2, 1, True)
    return out


def test_contact_problem_converges_at_first_order(contact_errors):
    for scheme, lo, hi in (("dg0", 0.8, 1.3), ("dg1lim", 0.8, 3.0)):
        e = [contact_errors[(scheme, n)][0] for n in (100, 200, 400)]
        orders = [np.log2(e[i] / e[i + 1]) for i in range(2)]
        print(scheme, e, orders)
        assert all(lo < p < hi for p in orders), (scheme, e, orders)


def test_unlimited_dg1_undershoots_and_the_limiter_bounds_it(contact_errors):
    for n in (100, 200, 400):
        e1, lo1 = contact_errors[("dg1", n)]
        el, lol = contact_errors[("dg1lim", n)]
        e0, lo0 = contact_errors[("dg0", n)]
        print(n, e0, e1, el, lo0, lo1, lol)
        assert lo0 >= -1e-12                   # DG0 (a monotone M-matrix scheme) stays in [c_L, c_R]
        assert lo1 < -1e-6                     # DG1 undershoots at the discontinuity
        assert lol > lo1                       # the limiter reduces the undershoot

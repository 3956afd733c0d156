"""Volume means of the oracle (Eq. A3) against exact integrals (CPU).

The Gauss-Legendre rule on k + 1 points per axis integrates polynomials of
degree 2k + 1 per axis exactly, and the nodal values of such a polynomial
are exactly its values at the quadrature points.  So for a field that is a
polynomial of degree <= 2k + 1 in each coordinate, the quadrature mean the
oracle reports must equal the exact volume average over the box, written
out here by integrating the polynomial term by term.  The test runs at
k = 1 (equal weights) and k = 3 (unequal weights, which also pins the node
order x fastest within a voxel against the weights).
"""
import numpy as np
import pytest

from oracle import dg, outputs
from oracle import model as M


def _coords(P):
    """Node coordinates (x, y, z), each of shape (E, (k+1)^3)."""
    K = P.k + 1
    xi, _ = dg.gl_nodes_weights(P.k)
    e = np.arange(P.n_elem)
    ex, ey, ez = e % P.nx, (e // P.nx) % P.ny, e // (P.nx * P.ny)
    n = np.arange(K ** 3)
    a0, a1, a2 = n % K, (n // K) % K, n // (K * K)
    x = (ex[:, None] + 0.5 * (1.0 + xi[a0][None, :])) * P.h
    y = (ey[:, None] + 0.5 * (1.0 + xi[a1][None, :])) * P.h
    z = (ez[:, None] + 0.5 * (1.0 + xi[a2][None, :])) * P.h
    return x, y, z


def _mono_mean(p, Lx):
    """Mean of x^p over [0, Lx]."""
    return Lx ** p / (p + 1)


# each field: a sum of terms c * x^a y^b z^d with a, b, d <= 2k + 1
def _terms(f, deg):
    rng = np.random.default_rng(100 + f)
    out = [(1.0 + f, 0, 0, 0)]
    for _ in range(4):
        a, b, d = rng.integers(0, deg + 1, 3)
        out.append((float(rng.uniform(-2, 2)), int(a), int(b), int(d)))
    return out


@pytest.mark.parametrize("k", [1, 3])
def test_volume_means_are_exact_for_polynomials(k):
    nx, ny, nz, h = 3, 2, 4, 0.5
    P = M.Problem(nx, ny, nz, h, k, np.zeros((nz, ny, nx), np.uint8))
    x, y, z = _coords(P)
    Lx, Ly, Lz = nx * h, ny * h, nz * h
    deg = 2 * k + 1
    u = np.zeros((9,) + x.shape)
    exact = np.zeros(9)
    for f in range(9):
        for c, a, b, d in _terms(f, deg):
            u[f] += c * (x / Lx) ** a * (y / Ly) ** b * (z / Lz) ** d
            exact[f] += c * _mono_mean(a, 1.0) * _mono_mean(b, 1.0) * _mono_mean(d, 1.0)
    means, cS = outputs.volume_means(P, u)
    print("means", means, "exact", exact)
    assert np.allclose(means, exact, rtol=1e-13, atol=1e-13)
    # dissolved sulfur c_S = c_S2- + 4 c_S4 + 6 c_S6 + 8 c_S8^2- + 8 c_S8 (Sec. 2.2)
    cS_exact = exact[5] + 4 * exact[4] + 6 * exact[3] + 8 * exact[2] + 8 * exact[1]
    assert abs(cS - cS_exact) <= 1e-13 * abs(cS_exact)


def test_volume_means_see_a_degree_beyond_the_rule():
    """Sharpness: x^(2k+2) is not integrated exactly by the k = 1 rule, so
    the reported mean of x^4 over one voxel misses 1/5 by exactly the
    two-point rule's error term (b - a)^5 f^(4) / 4320 = 24/4320 = 1/180."""
    nx, h = 1, 1.0
    P = M.Problem(nx, 1, 1, h, 1, np.zeros((1, 1, nx), np.uint8))
    x, _, _ = _coords(P)
    u = np.zeros((9,) + x.shape)
    u[0] = (x / (nx * h)) ** 4
    means, _ = outputs.volume_means(P, u)
    assert abs((0.2 - means[0]) - 1.0 / 180.0) < 1e-14

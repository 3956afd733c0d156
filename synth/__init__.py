"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and nothing else: porosity masks, kinetic
and transport parameter samples, and random states of realistic magnitude.
It contains none of the discretisation or chemistry arithmetic, so both the
CPU oracle and the HIP path can consume its output without sharing code.

The paper measures on a Blender-generated cathode (Voronoi particles of
10 um, macroscopic porosity 0.587) that is not available; these generators
stand in for it.  Every array that describes voxels uses numpy shape
(nz, ny, nx) in C order, so the flat index is ix + nx*(iy + ny*iz): x, the
transport axis, runs fastest.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "porosity_mask",
    "sample_transport_kinetics",
    "random_state",
    "Workload",
    "WORKLOADS",
    "batch_structures",
]

# Field order of a state vector (per node): six dissolved species, liquid
# potential, two solid volume fractions.
FIELDS = ("Li+", "S8(L)", "S8^2-", "S6^2-", "S4^2-", "S^2-", "Phi_L", "eps_S8", "eps_Li2S")


def _gauss_taps(sigma: float, radius: int) -> np.ndarray:
    s = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-0.5 * (s / sigma) ** 2)
    return w / w.sum()


def porosity_mask(shape, porosity: float, seed: int, sigma: float = 2.0) -> np.ndarray:
    """Binary voxel structure: 1 = cathode structure voxel, 0 = pore voxel.

    Standard-normal noise of the given (nz, ny, nx) shape is smoothed by a
    separable Gaussian (sigma in voxels, truncated at 4 sigma, periodic wrap)
    and thresholded at its ``porosity`` quantile, so the pore fraction is
    ``porosity`` up to ties.
    """
    nz, ny, nx = (int(v) for v in shape)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nz, ny, nx))
    taps = _gauss_taps(sigma, int(round(4 * sigma)))
    r = (len(taps) - 1) // 2
    for axis in range(3):
        acc = np.zeros_like(g)
        for j, w in enumerate(taps):
            acc += w * np.roll(g, j - r, axis=axis)
        g = acc
    q = np.quantile(g, porosity)
    pore = g <= q
    return (~pore).astype(np.uint8)


def sample_transport_kinetics(seed: int):
    """Per-seed synthetic diffusivities and exchange current densities.

    Returns (D0, i0): D0 holds infinite-dilution diffusivities [m^2/s] of
    (Li+, S8(L), S8^2-, S6^2-, S4^2-, S^2-, anion), log-uniform in
    [1e-11, 1e-9]; i0 holds exchange current densities [A/m^2] of the six
    electrochemical reactions, log-uniform in [1e-3, 1e-1].
    """
    rng = np.random.default_rng(10_000 + seed)
    D0 = 10.0 ** rng.uniform(-11.0, -9.0, 7)
    i0 = 10.0 ** rng.uniform(-3.0, -1.0, 6)
    return D0, i0


# Typical magnitudes of the nine fields in a structure voxel at the start of
# a discharge (concentrations in mol/m^3 as printed in the paper's liquid
# parameter table, potential in V, volume fractions as after localisation).
_TYPICAL = np.array([1500.0, 6.0, 6.2e-3, 3.9e-3, 1.9e-3, 3.6e-12, 0.0, 0.2375, 6.9e-6])


def random_state(n_elem: int, n_nodes: int, seed: int, spread: float = 0.1,
                 phi_spread: float = 2e-3, phase=None) -> np.ndarray:
    """Random positive state of shape (9, n_elem, n_nodes), float64.

    Concentrations and volume fractions are the typical magnitudes times
    exp(spread * N(0,1)); the potential is phi_spread * N(0,1) volts.  Where
    ``phase`` (flat, per element) is 0 the solid fractions are set to 0.
    """
    rng = np.random.default_rng(seed)
    u = np.empty((9, n_elem, n_nodes))
    for f in range(9):
        if f == 6:
            u[f] = phi_spread * rng.standard_normal((n_elem, n_nodes))
        else:
            u[f] = _TYPICAL[f] * np.exp(spread * rng.standard_normal((n_elem, n_nodes)))
    if phase is not None:
        ph = np.asarray(phase).reshape(-1)
        u[7:9, ph == 0, :] = 0.0
    return u


def random_vector(n_fields: int, n_elem: int, n_nodes: int, seed: int) -> np.ndarray:
    """Standard-normal direction vector of shape (n_fields, n_elem, n_nodes)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_fields, n_elem, n_nodes))


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named benchmark/test workload: mesh, order, mask recipe, C-rate."""
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    order: int
    porosity: float
    mask_seed: int
    param_seed: int
    f_C: float  # discharge rate [1/h]

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_elem(self):
        return self.nx * self.ny * self.nz

    def mask(self):
        return porosity_mask(self.shape, self.porosity, self.mask_seed)


WORKLOADS = {
    # 16^3 voxel cube, 1 um voxels, Q1, porosity 0.6, 0.1C, 5 BE steps.
    "cube16_q1": Workload("cube16_q1", 16, 16, 16, 1e-6, 1, 0.6, 0, 0, 0.1),
    # 96x96x192 cathode slab (x = transport axis), Q1, porosity 0.6, 1C; the
    # transport/kinetic draw of the 16^3 cube (parameter seed 0).  Under the
    # draw of seed 2 a 1C current drives S4^2- to the concentration floor
    # within a millisecond, where backward Euler has no positive root.
    "slab96_q1": Workload("slab96_q1", 96, 96, 192, 1e-6, 1, 0.6, 2, 0, 1.0),
    # 48^3 elements, Q3, porosity 0.6, 0.5C.
    "cube48_q3": Workload("cube48_q3", 48, 48, 48, 1e-6, 3, 0.6, 5, 5, 0.5),
}


def batch_structures(n: int = 64, seed: int = 4000, lo: int = 24, hi: int = 64):
    """Sizes and porosities of a batch of uneven cubic microstructures.

    Returns a list of (edge, porosity, mask_seed) with edge ~ U{lo..hi} and
    porosity ~ U(0.4, 0.75); mask seeds are 1000 + b.
    """
    rng = np.random.default_rng(seed)
    edges = rng.integers(lo, hi + 1, n)
    por = rng.uniform(0.4, 0.75, n)
    return [(int(edges[b]), float(por[b]), 1000 + b) for b in range(n)]

"""HIP residual vs the CPU oracle, element by element (GPU)."""
import numpy as np
import pytest

import synth
from oracle import dg as odg
from tests.helpers import field_errors, oracle_residual_at, problem_and_context

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# FP64: both sides evaluate the same sums in double; differences come from
# summation order and the libm/ocml exp/log/sqrt (each < 1 ulp).  Relative
# to the largest term of a field the error stays near 1e-15; 1e-12 leaves
# room for cancellation inside the field.
TOL64 = 1e-12
# FP32 kernel against the FP64 oracle: unit roundoff 6e-8 amplified by the
# same cancellation.
TOL32 = 2e-5


def _run(nx, ny, nz, seed, dtype=torch.float64, **kw):
    print(f"[residual] mesh {nx}x{ny}x{nz} seed {seed} dtype {dtype} {kw}", flush=True)
    P, ctx, mask = problem_and_context(nx, ny, nz, mask_seed=seed, param_seed=seed, **kw)
    u = synth.random_state(P.n_elem, P.n_nodes, 100 + seed, phase=mask, phi_spread=5e-3)
    uo = synth.random_state(P.n_elem, P.n_nodes, 200 + seed, phase=mask)
    dev = torch.device("cuda:0")
    m = ctx.mass(torch.tensor(uo, device=dev, dtype=dtype))
    r = ctx.residual(torch.tensor(u, device=dev, dtype=dtype), m, 0.7, 0.05)
    torch.cuda.synchronize()
    return P, ctx, u, uo, m.cpu().numpy(), r.cpu().numpy()


@pytest.mark.parametrize("shape,seed", [((5, 4, 3), 0), ((16, 16, 16), 1), ((7, 1, 2), 2),
                                        ((1, 3, 5), 3), ((33, 2, 9), 4)])
def test_residual_fp64_matches_oracle(shape, seed):
    P, ctx, u, uo, m, r = _run(*shape, seed)
    m_ref = odg.old_mass(P, uo)
    assert np.all(field_errors(m, m_ref) < 1e-15)
    ref = odg.residual(P, u, m_ref, 0.7, 0.05)
    err = field_errors(r, ref)
    print("  field errors", err, flush=True)
    assert np.all(err < TOL64), err


@pytest.mark.parametrize("porosity", [0.0, 1.0])
def test_residual_fp64_uniform_masks(porosity):
    """All-structure and all-pore voxel maps (no interfaces, or no reactions)."""
    P, ctx, u, uo, m, r = _run(6, 5, 4, 7, porosity=porosity)
    ref = odg.residual(P, u, odg.old_mass(P, uo), 0.7, 0.05)
    assert np.all(field_errors(r, ref) < TOL64)


def test_residual_fp64_paper_parameters():
    P, ctx, u, uo, m, r = _run(9, 6, 5, 8, paper_params=True)
    ref = odg.residual(P, u, odg.old_mass(P, uo), 0.7, 0.05)
    assert np.all(field_errors(r, ref) < TOL64)


def test_residual_vanishes_at_equilibrium():
    from oracle import solve as osolve
    P, ctx, mask = problem_and_context(8, 7, 6, mask_seed=3, param_seed=3, j_el=0.0)
    u = osolve.uniform_state(P)
    dev = torch.device("cuda:0")
    ut = torch.tensor(u, device=dev)
    r = ctx.residual(ut, ctx.mass(ut), 3.0, 0.1).cpu().numpy()
    assert np.max(np.abs(r[0:6])) < 1e-24
    assert np.max(np.abs(r[6])) < 1e-22
    assert np.max(np.abs(r[7:9])) < 1e-30


def test_residual_fp32_matches_oracle():
    P, ctx, u, uo, m, r = _run(12, 10, 9, 9, dtype=torch.float32)
    u32 = u.astype(np.float32).astype(np.float64)
    ref = odg.residual(P, u32, m.astype(np.float64), 0.7, 0.05)
    err = field_errors(r.astype(np.float64), ref)
    print("  fp32 field errors", err, flush=True)
    assert np.all(err < TOL32), err


def test_residual_full_slab_sampled():
    """96 x 96 x 192 Q1 slab (99 M DoF), launch as benchmarked, sampled voxels
    (all boundary types included) against the oracle."""
    from synth import WORKLOADS
    w = WORKLOADS["slab96_q1"]
    print(f"[residual] full slab {w.nx}x{w.ny}x{w.nz}", flush=True)
    P, ctx, mask = problem_and_context(w.nx, w.ny, w.nz, porosity=w.porosity,
                                       mask_seed=w.mask_seed, param_seed=w.param_seed, f_C=w.f_C)
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(5)
    Ne, npn = P.n_elem, P.n_nodes
    typical = torch.tensor([1500.0, 6.0, 6.2e-3, 3.9e-3, 1.9e-3, 3.6e-12, 0.0, 0.2375, 6.9e-6],
                           dtype=torch.float64)
    u = torch.empty((9, Ne, npn), dtype=torch.float64)
    for f in range(9):
        z = torch.randn((Ne, npn), generator=g, dtype=torch.float64)
        u[f] = 5e-3 * z if f == 6 else typical[f] * torch.exp(0.1 * z)
    pore = torch.tensor(mask.reshape(-1) == 0)
    u[7:9, pore, :] = 0.0
    uo = u * (1.0 + 0.01 * torch.randn(u.shape, generator=g, dtype=torch.float64))
    uo[6] = u[6]
    ud, uod = u.to(dev), uo.to(dev)
    m = ctx.mass(uod)
    r = ctx.residual(ud, m, 0.7, 0.05)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    corners = [0, w.nx - 1, (w.ny - 1) * w.nx, Ne - 1, Ne - w.nx, w.nx * w.ny * (w.nz // 2) + w.nx - 1]
    elems = np.concatenate([corners, rng.integers(0, Ne, 60)])
    un, mn, rn = u.numpy(), m.cpu().numpy(), r.cpu().numpy()
    ref = oracle_residual_at(P, un, mn, 0.7, 0.05, elems)
    err = field_errors(rn[:, elems], ref)
    print("  sampled field errors", err, flush=True)
    assert np.all(err < TOL64), err


def _floor_state(P, mask, seed):
    """A random state whose trace species sit at and below the activity
    clamp c_min: S4^2- and S^2- at exactly c_min, half of it, zero, slightly
    negative and clearly negative at scattered nodes; Li+ negative at one
    node (every clamp and the harmonic-mean guard take their other branch)."""
    u = synth.random_state(P.n_elem, P.n_nodes, seed, phase=mask, phi_spread=5e-3)
    rng = np.random.default_rng(seed)
    cmin = P.c_min
    vals = [cmin, 0.5 * cmin, 0.0, -1e-10, -1e-4]
    for f in (4, 5):
        idx = rng.choice(P.n_elem * P.n_nodes, size=40, replace=False)
        flat = u[f].reshape(-1)
        for j, k in enumerate(idx):
            flat[k] = vals[j % len(vals)]
    u[0].reshape(-1)[rng.integers(0, P.n_elem * P.n_nodes)] = -1e-6
    return u


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_residual_at_and_below_the_concentration_floor(dtype):
    P, ctx, mask = problem_and_context(6, 5, 4, mask_seed=11, param_seed=11)
    u = _floor_state(P, mask, 31)
    uo = synth.random_state(P.n_elem, P.n_nodes, 32, phase=mask)
    dev = torch.device("cuda:0")
    m = ctx.mass(torch.tensor(uo, device=dev, dtype=dtype))
    r = ctx.residual(torch.tensor(u, device=dev, dtype=dtype), m, 0.7, 0.05).cpu().numpy().astype(np.float64)
    uu = u.astype(np.float32).astype(np.float64) if dtype == torch.float32 else u
    ref = odg.residual(P, uu, m.cpu().numpy().astype(np.float64), 0.7, 0.05)
    err = field_errors(r, ref)
    print(f"  {dtype} floor-state field errors", err, flush=True)
    assert np.all(err < (TOL64 if dtype == torch.float64 else TOL32)), err

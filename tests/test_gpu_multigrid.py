"""Multilevel aggregation coarse correction (dg_mg_setup / dg_mg_apply /
dg_mg_export) against the oracle's definition (GPU).

Mesh 7 x 6 x 5 voxels with level-1 aggregates of 2^3 voxels: 4 x 3 x 3
aggregates, ragged along every axis (the last ones are one voxel thick);
level 2 has 2 x 2 x 2, level 3 one aggregate.

  * Level operators: every stencil entry of E_1 = Z^T J Z (49 coloured
    probes of the GPU's Krylov operator) and of the Galerkin products E_2,
    E_3, against the oracle's E_1 formed column by column from its condensed
    complex-step tangent: FP64 to 1e-12 and FP32 to 2e-5 of the block row's
    largest sum of contribution magnitudes (the Galerkin product of |E_1|:
    the sums cancel, on the last level down to the reaction terms alone).
  * The V-cycle, FP64, for 2 and 3 levels and 0, 1, 2 sweeps.  The coarse
    systems are badly conditioned (the level of Phi_L is held only by the
    exchange currents; the last level's condition number is about 1e7, and
    the fields' magnitudes differ by up to 1e15), so a rounding-level change
    of E_1 moves the cycle's result by up to about 1e-9 of its size.  The bar
    is 100 times what the oracle itself moves when its E_1 is perturbed at
    relative 2^-50 (a seeded perturbation), and at least 1e-12: rounding
    differences pass it, a wrong slot, sign, damping or transfer moves the
    result by O(1).
  * Error paths before and after a setup.
"""
import numpy as np
import pytest

import synth
from oracle import dg as odg
from oracle import model as om
from oracle import multigrid as mg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NX, NY, NZ, EDGE = 7, 6, 5, 2
T_NEW, DT = 0.3, 0.1


@pytest.fixture(scope="module")
def case():
    from paper_2511_05233_amd import lsbdg
    mask = synth.porosity_mask((NZ, NY, NX), 0.6, 3)
    D0, i0 = synth.sample_transport_kinetics(3)
    P = om.Problem(NX, NY, NZ, 1e-6, 1, mask, D0=D0, kE=i0 / om.F, f_C=0.1)
    ctx = lsbdg.Context(NX, NY, NZ, 1e-6, 1, mask, D0=D0, kE=i0 / om.F, f_C=0.1)
    u = synth.random_state(P.n_elem, P.n_nodes, 11, phase=mask, phi_spread=5e-3)
    print("[mg] oracle level-1 operator (252 condensed tangents)", flush=True)
    E1 = mg.level1_operator(P, u, odg.old_mass(P, u), T_NEW, DT, EDGE)
    return P, ctx, u, E1


def _stencil(E, grid):
    """Dense level operator (field, aggregate order) -> E[s][g][f][a]."""
    ax, ay, az = grid
    na = ax * ay * az
    out = np.zeros((7, 7, 7, na))
    for a in range(na):
        x, y, z = a % ax, (a // ax) % ay, a // (ax * ay)
        for s, (dx, dy, dz) in enumerate([(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0),
                                          (0, 0, -1), (0, 0, 1)]):
            xx, yy, zz = x + dx, y + dy, z + dz
            if not (0 <= xx < ax and 0 <= yy < ay and 0 <= zz < az):
                continue
            nb = xx + ax * (yy + ay * zz)
            out[s, :, :, a] = E[np.ix_(np.arange(7) * na + a, np.arange(7) * na + nb)]
    return out


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
def test_level_operators_match_the_oracle(case, dtype, tol):
    P, ctx, u, E1 = case
    L = 3
    ut = torch.tensor(u, device="cuda:0").to(dtype)
    ctx.mg_setup(ut, T_NEW, DT, levels=L, agg=EDGE)
    grids = mg.level_grids(NX, NY, NZ, EDGE, L)
    Es, _ = mg.hierarchy(E1, grids[0], L)
    # the Galerkin sums cancel (transport conserves: on the last level the
    # face terms of the whole mesh sum to zero), so the rounding of an entry
    # is bounded by the same sum over the contributions' magnitudes
    Ea, _ = mg.hierarchy(np.abs(E1), grids[0], L)
    for lev in range(L):
        na = int(np.prod(grids[lev]))
        got = ctx.mg_export(lev + 1, na).cpu().numpy()
        ref = _stencil(Es[lev], grids[lev])
        # scale: the largest such magnitude sum in each block row (g, a)
        scale = _stencil(Ea[lev], grids[lev]).max(axis=(0, 2), keepdims=True)
        err = np.max(np.abs(got - ref) / np.where(scale > 0, scale, 1.0))
        print(f"[mg] {dtype} level {lev + 1} ({na} aggregates): max relative entry error {err:.2e}", flush=True)
        assert err <= tol, (lev, err)


@pytest.mark.parametrize("levels", [2, 3])
@pytest.mark.parametrize("sweeps", [0, 1, 2])
def test_vcycle_matches_the_oracle(case, levels, sweeps):
    P, ctx, u, E1 = case
    omega = 0.7
    ut = torch.tensor(u, device="cuda:0")
    ctx.mg_setup(ut, T_NEW, DT, levels=levels, agg=EDGE, sweeps=sweeps, omega=omega)
    r = synth.random_vector(7, P.n_elem, P.n_nodes, 12)
    got = ctx.mg_apply(torch.tensor(r, device="cuda:0")).cpu().numpy()
    grid1 = mg.aggregate_grid(NX, NY, NZ, EDGE)
    Es, Ps = mg.hierarchy(E1, grid1, levels)
    ref = mg.coarse_correction(P, r, Es, Ps, EDGE, nu=sweeps, omega=omega)
    rng = np.random.default_rng(0)
    Esp, Psp = mg.hierarchy(E1 * (1.0 + 2.0 ** -50 * rng.standard_normal(E1.shape)), grid1, levels)
    moved = mg.coarse_correction(P, r, Esp, Psp, EDGE, nu=sweeps, omega=omega)
    for f in range(7):
        scale = np.abs(ref[f]).max()
        sens = np.abs(moved[f] - ref[f]).max() / scale
        err = np.abs(got[f] - ref[f]).max() / scale
        bar = max(1e-12, 100.0 * sens)
        print(f"[mg] levels {levels} sweeps {sweeps} field {f}: error {err:.2e}, oracle's own "
              f"sensitivity {sens:.2e}", flush=True)
        assert err <= bar, (f, err, bar)


def test_mg_entry_points_refuse_bad_calls(case):
    from paper_2511_05233_amd import lsbdg
    P, ctx0, u, _ = case
    mask = np.asarray(P.phase)
    ctx = lsbdg.Context(NX, NY, NZ, 1e-6, 1, mask)
    r = torch.zeros((7, P.n_elem, P.n_nodes), dtype=torch.float64, device="cuda:0")
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.mg_apply(r)
    assert ei.value.code == -6                       # no setup yet
    ut = torch.tensor(u, device="cuda:0")
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.mg_setup(ut, T_NEW, DT, levels=1, agg=EDGE)
    assert ei.value.code == -1
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.mg_setup(ut, T_NEW, DT, levels=2, agg=EDGE, omega=1.5)
    assert ei.value.code == -1
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.mg_setup(ut, T_NEW, DT, levels=9, agg=EDGE)
    assert ei.value.code == -1
    ctx.mg_setup(ut, T_NEW, DT, levels=2, agg=EDGE)
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.mg_apply(r.float())                      # precision of the setup only
    assert ei.value.code == -1
    with pytest.raises(lsbdg.DgError) as ei:
        ctx.mg_export(3, 1)                          # no third level
    assert ei.value.code == -1
    ctx.close()

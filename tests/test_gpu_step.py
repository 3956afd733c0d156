"""HIP backward-Euler step (Newton-GMRES) vs the oracle's Newton root (GPU)."""
import numpy as np
import pytest

import synth
from oracle import dg as odg
from oracle import model as om
from oracle import outputs as oout
from oracle import solve as osolve
from tests.helpers import problem_and_context

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel_l2(a, b):
    return np.array([np.linalg.norm(a[f] - b[f]) / max(np.linalg.norm(b[f]), 1e-300) for f in range(9)])


@pytest.fixture(scope="module")
def small_case():
    # a step whose root keeps every concentration positive (checked below):
    # with the synthetic kinetics larger steps drive S4^2- through zero, a
    # step the controller rejects by halving dt
    P, ctx, mask = problem_and_context(5, 4, 3, mask_seed=1, param_seed=1, f_C=0.1)
    print("[step] oracle initial state 5x4x3", flush=True)
    u0, _ = osolve.initial_state(P)
    print("[step] oracle BE step", flush=True)
    u1, info = osolve.be_step(P, u0, 0.0, 0.1)
    assert u1[0:6].min() > 0
    print("[step] oracle", info, flush=True)
    return P, ctx, u0, u1


def oracle_charge_noise(P, u0, m_old):
    """Rounding level of the oracle's charge residual: at uniform
    concentrations and uniform Phi_L its exact value is zero in every pore
    voxel off the separator column, so whatever it returns there is the
    rounding of its evaluation."""
    uz = osolve.uniform_state(P)
    uz[6] = u0[6].mean()
    Rz = odg.residual(P, uz, m_old, 0.0, 1.0)[6]
    ix = np.arange(P.n_elem) % P.nx
    sel = (np.asarray(P.phase).reshape(-1) == 0) & (ix < P.nx - 1)
    R0 = odg.residual(P, u0, m_old, 0.0, 1.0)[6]
    return max(np.abs(Rz[sel]).max(), np.abs(R0).max())


@pytest.fixture(scope="module")
def phi_bound(small_case):
    """Rounding-limited accuracy of the steady potential.

    With frozen concentrations the level of Phi_L is fixed only by the
    exchange currents (1e-3..1e-1 A/m^2 here), so the charge block is badly
    conditioned (about 1e7): a rounding-level change of the residual moves
    the root by up to sqrt(n) |dR|_max / sigma_min(J)."""
    P, ctx, u0, _ = small_case
    m_old = odg.old_mass(P, osolve.uniform_state(P))
    J = osolve.sparse_jacobian(P, u0, m_old, 0.0, 1.0, fields=(6,)).toarray()
    smin = np.linalg.svd(J, compute_uv=False)[-1]
    noise = oracle_charge_noise(P, u0, m_old)
    return m_old, noise, np.sqrt(J.shape[0]) * noise / smin


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_initial_state_matches_oracle(small_case, phi_bound, inner):
    """Equilibrium concentrations and solid fractions exactly; Phi_L solves
    the charge balance to the rounding level (GPU residual at the GPU root)
    and lies within the conditioning bound of the oracle's root."""
    P, ctx, u0, _ = small_case
    m_old, noise, bound = phi_bound
    ut, rep = ctx.initial_state(inner=inner, verbose=1)
    print(f"[init] {inner} report {rep}", flush=True)
    got = ut.cpu().numpy()
    assert np.array_equal(got[[0, 1, 2, 3, 4, 5, 7, 8]], u0[[0, 1, 2, 3, 4, 5, 7, 8]])
    diff = np.linalg.norm(got[6] - u0[6])
    rel = diff / np.linalg.norm(u0[6])
    r6 = np.abs(ctx.residual(ut, torch.tensor(m_old, device="cuda:0"), 0.0, 1.0)[6].cpu().numpy()).max()
    print(f"  Phi_L |diff| {diff:.3e} V (relative {rel:.3e}), bound {bound:.3e}; "
          f"GPU charge residual at its root {r6:.3e}, oracle rounding level {noise:.3e}", flush=True)
    assert r6 <= 2 * noise
    assert diff <= bound


@pytest.mark.parametrize("inner,tol", [("f64", 1e-10), ("f32", 1e-8)])
def test_step_matches_oracle_root(small_case, inner, tol):
    P, ctx, u0, u1 = small_case
    ut = torch.tensor(u0, device="cuda:0")
    rep = ctx.step(ut, 0.0, 0.1, inner=inner, verbose=1)
    assert rep["status"] == 0
    print(f"[step] {inner} report {rep}", flush=True)
    got = ut.cpu().numpy()
    err = rel_l2(got, u1)
    print("  relative L2 per field", err, flush=True)
    assert np.all(err[:7] < tol), err
    # solid fractions in pore voxels are identically zero on both sides
    assert np.all(err[7:] < tol), err


def test_step_invariants_on_cube16():
    """16^3 voxels, Q1, 0.1C, dt = 0.1 s from the steady initial potential:
    the GPU root satisfies the oracle's residual and the conservation laws."""
    w = synth.WORKLOADS["cube16_q1"]
    P, ctx, mask = problem_and_context(w.nx, w.ny, w.nz, porosity=w.porosity, mask_seed=w.mask_seed,
                                       param_seed=w.param_seed, f_C=w.f_C)
    print("[step] oracle initial state 16^3", flush=True)
    u0, _ = osolve.initial_state(P)
    ug, rep0 = ctx.initial_state(inner="f32")
    ug = ug.cpu().numpy()
    err0 = np.linalg.norm(ug[6] - u0[6]) / np.linalg.norm(u0[6])
    m_init = odg.old_mass(P, osolve.uniform_state(P))
    r6_gpu = np.abs(ctx.residual(torch.tensor(ug, device="cuda:0"), torch.tensor(m_init, device="cuda:0"),
                                 0.0, 1.0)[6].cpu().numpy()).max()
    noise = oracle_charge_noise(P, u0, m_init)
    print(f"[step] GPU initial state {rep0}, Phi_L relative L2 {err0:.3e}, "
          f"GPU charge residual {r6_gpu:.3e} (oracle rounding level {noise:.3e})", flush=True)
    assert r6_gpu <= 2 * noise
    assert err0 < 1e-7
    ut = torch.tensor(u0, device="cuda:0")
    rep = ctx.step(ut, 0.0, 0.1, inner="f32", verbose=1)
    print(f"[step] cube16 report {rep}", flush=True)
    u1 = ut.cpu().numpy()
    S0, Li0, Ne0, _ = oout.invariants(P, u0, 0.0)
    S1, Li1, Ne1, I1 = oout.invariants(P, u1, 0.1)
    q = 0.1 * P.j_el * oout.separator_area(P) / om.F
    assert abs(S1 - S0) < 1e-12 * S0
    assert abs((Li1 - Li0) - q) < 1e-12 * Li0
    assert abs((Ne1 - Ne0) / q - 1.0) < 1e-7
    assert abs(I1 / (P.j_el * oout.separator_area(P)) - 1.0) < 1e-7
    # oracle residual at the GPU root, per field against the larger of the
    # accumulation term and the field's residual at the start of the step
    # (trace species such as S^2- are governed by their reaction terms)
    m_old = odg.old_mass(P, u0)
    R = odg.residual(P, u1, m_old, 0.1, 0.1)
    R0 = odg.residual(P, u0, m_old, 0.1, 0.1)
    W = odg.basis(1).W3[None, :] * (P.h / 2) ** 3
    assert rep["last_update"] < 1e-7
    for f in range(6):
        scale = max(np.max(np.abs(W * u1[f] / 0.1)), np.max(np.abs(R0[f])))
        ratio = np.max(np.abs(R[f])) / scale
        print(f"[step] field {f} residual / scale {ratio:.3e}", flush=True)
        assert ratio <= 1e-6, f


@pytest.mark.parametrize("coarse", [3, 4])
@pytest.mark.parametrize("inner,tol", [("f64", 1e-10), ("f32", 1e-8)])
def test_step_with_aggregation_coarse_space(small_case, inner, tol, coarse):
    """The two-level preconditioner (per-field constants on 2x2x2-voxel
    aggregates, coarse operator by coloured probes, LU) reaches the same
    root."""
    P, ctx, u0, u1 = small_case
    ut = torch.tensor(u0, device="cuda:0")
    rep = ctx.step(ut, 0.0, 0.1, inner=inner, coarse=coarse, coarse_agg=2, verbose=1)
    print(f"[step] coarse={coarse} {inner} report {rep}", flush=True)
    err = rel_l2(ut.cpu().numpy(), u1)
    print("  relative L2 per field", err, flush=True)
    assert np.all(err < tol), err


@pytest.mark.parametrize("coarse", [3, 4])
@pytest.mark.parametrize("inner,tol", [("f64", 1e-10), ("f32", 1e-8)])
def test_step_with_multigrid_coarse_correction(small_case, inner, tol, coarse):
    """The coarse solve replaced by a three-level V-cycle (aggregates of 1,
    2 and 4 voxels per edge: 5x4x3, 3x2x2 and 2x1x1 of them) reaches the
    same root."""
    P, ctx, u0, u1 = small_case
    ut = torch.tensor(u0, device="cuda:0")
    rep = ctx.step(ut, 0.0, 0.1, inner=inner, coarse=coarse, coarse_agg=1, mg_levels=3, verbose=1)
    print(f"[step] multigrid coarse={coarse} {inner} report {rep}", flush=True)
    err = rel_l2(ut.cpu().numpy(), u1)
    print("  relative L2 per field", err, flush=True)
    assert np.all(err < tol), err


def test_automatic_multigrid_choice():
    """mg_levels = -1 (the default) runs the multilevel cycle only where the
    exact two-level space would need coarse aggregates: on 24^3 voxels with
    2^3-voxel aggregates (1,728 aggregates, 12,096 coarse unknowns) a
    two-level cycle down to 6^3 aggregates, with 4^3-voxel aggregates (1,512
    unknowns) and by default (edge up to 8) the exact solve.  The report
    names the levels used; every choice reaches the same root."""
    P, ctx, mask = problem_and_context(24, 24, 24, porosity=0.6, mask_seed=5, param_seed=5, f_C=0.1)
    u0, _ = ctx.initial_state(inner="f32")
    roots, levels = {}, {}
    for name, opts in (("agg2", {"coarse_agg": 2}), ("agg4", {"coarse_agg": 4}), ("default", {})):
        ut = u0.clone()
        rep = ctx.step(ut, 0.0, 0.1, inner="f32", **opts)
        roots[name], levels[name] = ut.cpu().numpy(), rep["mg_levels"]
        print(f"[step] 24^3 {name}: {rep}", flush=True)
    assert levels == {"agg2": 2, "agg4": 0, "default": 0}, levels
    for name in ("agg2", "agg4"):
        assert np.all(rel_l2(roots[name], roots["default"])[:7] < 1e-8)


def test_aggregation_coarse_space_cuts_gmres_on_cube16():
    """16^3 cube, first implicit step from the GPU initial state: the
    aggregation coarse space needs fewer GMRES iterations than the global
    per-field constants, for the same root."""
    w = synth.WORKLOADS["cube16_q1"]
    P, ctx, mask = problem_and_context(w.nx, w.ny, w.nz, porosity=w.porosity, mask_seed=w.mask_seed,
                                       param_seed=w.param_seed, f_C=w.f_C)
    u0, _ = ctx.initial_state(inner="f32")
    reps, roots = {}, {}
    for coarse in (1, 3, 4):
        ut = u0.clone()
        reps[coarse] = ctx.step(ut, 0.0, 0.1, inner="f32", coarse=coarse)
        roots[coarse] = ut.cpu().numpy()
        print(f"[step] cube16 coarse={coarse}: {reps[coarse]}", flush=True)
    # the multilevel V-cycle on 8^3, 4^3 and 2^3 aggregates of 2, 4, 8 voxels
    ut = u0.clone()
    reps["mg"] = ctx.step(ut, 0.0, 0.1, inner="f32", coarse=3, coarse_agg=2, mg_levels=3)
    roots["mg"] = ut.cpu().numpy()
    print(f"[step] cube16 multigrid: {reps['mg']}", flush=True)
    assert reps["mg"]["gmres_its"] < reps[1]["gmres_its"]
    for c in (3, 4, "mg"):
        err = rel_l2(roots[c], roots[1])
        print(f"  relative L2 between the roots (coarse {c} vs 1)", err, flush=True)
        assert np.all(err[:7] < 1e-8), err
    assert reps[3]["gmres_its"] < reps[1]["gmres_its"]


def test_step_with_bf16_block_inverses(small_case):
    """Streaming the FP32 block inverses as bfloat16 changes only the
    preconditioner: the mixed-precision step reaches the same root."""
    P, ctx, u0, u1 = small_case
    ut = torch.tensor(u0, device="cuda:0")
    rep = ctx.step(ut, 0.0, 0.1, inner="f32", block_bf16=1, verbose=1)
    print(f"[step] bf16 blocks report {rep}", flush=True)
    err = rel_l2(ut.cpu().numpy(), u1)
    print("  relative L2 per field", err, flush=True)
    assert np.all(err < 1e-8), err

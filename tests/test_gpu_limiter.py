"""dg_limit, the vertex-based Q1 limiter, against the oracle (GPU).

  * a 13 x 11 x 9 mesh (1,287 voxels: six workgroups of 256 and a ragged
    last one), structure and pore voxels, a smooth state with nodal noise
    and negative nodes: every limited value and every factor alpha against
    oracle/limiter.py;
  * the 96 x 96 x 192 slab: sampled voxels (corners, boundary and random
    ones) against the oracle on the 3 x 3 x 3 patch around each (a voxel's
    result depends on the means of those voxels only), and over the whole
    slab the properties that hold at any size -- each voxel's amounts kept,
    non-negative output where every mean is non-negative;
  * order 0: a no-op;
  * a limited backward-Euler step (opts.limiter = 1, FP64 inner solves)
    on 5 x 4 x 3 voxels against the oracle's limited step.
"""
import numpy as np
import pytest

import synth
from oracle import limiter as olim
from oracle import solve as osolve
from tests.helpers import _patch, problem_and_context

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-12          # FP64: means and corner values differ by summation order only


def _noisy_state(P, mask, seed, spread=0.02, negative=True):
    """Equilibrium-like state with a smooth variation over the mesh (one
    period), nodal noise of relative size `spread` and, optionally, a few
    negative nodes per species."""
    u = synth.random_state(P.n_elem, P.n_nodes, seed, phase=mask, phi_spread=5e-3)
    rng = np.random.default_rng(seed)
    e = np.arange(P.n_elem)[:, None]
    a = np.arange(8)[None, :]
    x = (e % P.nx + 0.5 + 0.29 * (2 * (a & 1) - 1)) / P.nx
    y = ((e // P.nx) % P.ny + 0.5 + 0.29 * (2 * (a >> 1 & 1) - 1)) / P.ny
    z = (e // (P.nx * P.ny) + 0.5 + 0.29 * (2 * (a >> 2 & 1) - 1)) / P.nz
    smooth = 0.8 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.5 * np.sin(2 * np.pi * z + 0.3)
    base = np.median(np.abs(u[0:6]), axis=(1, 2))
    u[0:6] = base[:, None, None] * np.exp(smooth[None] + spread * rng.standard_normal(u[0:6].shape))
    if negative:                                       # a few nodes below zero in every species
        for f in range(6):
            idx = rng.choice(P.n_elem * P.n_nodes, size=max(4, P.n_elem // 50), replace=False)
            u[f].reshape(-1)[idx] *= -0.5
    return u


def _rel(got, ref):
    scale = np.max(np.abs(ref), axis=(1, 2), keepdims=True)
    return np.max(np.abs(got - ref) / scale, axis=(1, 2))


def test_limiter_matches_oracle_on_a_ragged_mesh():
    P, ctx, mask = problem_and_context(13, 11, 9, porosity=0.6, mask_seed=3, param_seed=1)
    u = _noisy_state(P, mask, 11)
    ref, aref = olim.limit(P, u)
    ud = torch.tensor(u, device="cuda:0")
    alpha = ctx.limit(ud, alpha=True)
    got, ag = ud.cpu().numpy(), alpha.cpu().numpy()
    err = _rel(got[0:6], ref[0:6])
    print(f"[limiter] ragged mesh: field errors {err}, alpha error {np.max(np.abs(ag - aref)):.2e}, "
          f"limited voxels {np.mean(aref < 1):.2f}", flush=True)
    assert np.all(err < TOL), err
    assert np.max(np.abs(ag - aref)) < 1e-9
    assert np.array_equal(got[6:], u[6:])
    assert 0.05 < np.mean(aref < 1) < 0.95             # both branches exercised


def test_limiter_sampled_on_the_slab():
    from synth import WORKLOADS
    w = WORKLOADS["slab96_q1"]
    print(f"[limiter] slab {w.nx}x{w.ny}x{w.nz}", flush=True)
    P, ctx, mask = problem_and_context(w.nx, w.ny, w.nz, porosity=w.porosity, mask_seed=w.mask_seed,
                                       param_seed=w.param_seed, f_C=w.f_C)
    g = torch.Generator(device="cpu").manual_seed(21)
    u = torch.empty((9, P.n_elem, 8), dtype=torch.float64)
    typical = [1500.0, 6.0, 6.2e-3, 3.9e-3, 1.9e-3, 3.6e-12, 0.0, 0.2375, 6.9e-6]
    for f in range(9):
        z = torch.randn((P.n_elem, 8), generator=g, dtype=torch.float64)
        u[f] = 5e-3 * z if f == 6 else typical[f] * (1.0 + 0.4 * z)   # some nodes negative
    u[7:9, torch.tensor(mask.reshape(-1) == 0), :] = 0.0
    ud = u.to("cuda:0")
    m0 = ctx.mass(ud)                                      # eps_L c_i before
    ctx.limit(ud)
    m1 = ctx.mass(ud)
    # every voxel keeps its amounts
    a0 = m0[0:6].sum(dim=2)
    a1 = m1[0:6].sum(dim=2)
    drift = ((a1 - a0).abs() / a0.abs().amax(dim=1, keepdim=True)).max().item()
    print(f"[limiter] slab amounts drift {drift:.2e}", flush=True)
    assert drift < 1e-13
    # non-negative output wherever the means around a voxel are non-negative
    # (checked for the voxels whose own and neighbours' means are positive:
    # here every voxel's mean is positive)
    assert (a0 > 0).all()
    assert (ud[0:6] >= 0).all()
    un, got = u.numpy(), ud.cpu().numpy()
    rng = np.random.default_rng(2)
    Ne = P.n_elem
    corners = [0, w.nx - 1, (w.ny - 1) * w.nx, Ne - 1, Ne - w.nx, w.nx * w.ny * (w.nz // 2) + w.nx - 1]
    worst = 0.0
    for e in np.concatenate([corners, rng.integers(0, Ne, 40)]):
        Q, gidx, loc = _patch(P, int(e))
        ref, _ = olim.limit(Q, un[:, gidx])
        err = np.max(np.abs(got[0:6, e] - ref[0:6, loc]) / np.abs(ref[0:6, loc]).max(axis=1, keepdims=True))
        worst = max(worst, err)
    print(f"[limiter] slab sampled voxels: worst relative error {worst:.2e}", flush=True)
    assert worst < TOL


def test_order_zero_is_a_no_op():
    P, ctx, mask = problem_and_context(6, 5, 4, k=0, porosity=0.6, mask_seed=1)
    u = synth.random_state(P.n_elem, P.n_nodes, 3, phase=mask, phi_spread=5e-3)
    ud = torch.tensor(u, device="cuda:0")
    ctx.limit(ud)
    assert np.array_equal(ud.cpu().numpy(), u)


def test_limited_step_matches_the_oracle():
    P, ctx, mask = problem_and_context(5, 4, 3, porosity=0.6, mask_seed=1, param_seed=1, f_C=1.0)
    u0, _ = osolve.initial_state(P)
    dt = 0.05
    ref, info = osolve.be_step(P, u0, 0.0, dt, limiter=True)
    ud = torch.tensor(u0, device="cuda:0")
    rep = ctx.step(ud, 0.0, dt, inner="f64", limiter=1)
    got = ud.cpu().numpy()
    err = _rel(got, ref)
    print(f"[limiter] limited step: oracle {info}, GPU {rep['newton_its']} Newton; errors {err}", flush=True)
    assert np.all(err < 1e-10), err

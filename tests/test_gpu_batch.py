"""Batched operators (dg_batch_*): structures of uneven size, each on its
own clock, in one launch per operator.  Every structure's slice of a batch
result equals the single-structure call on that structure (the same node
code, with the array bases offset), and one batched residual is checked
against the oracle directly."""
import numpy as np
import pytest

import synth
from oracle import dg as odg
from oracle import model as om
from tests.helpers import field_errors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (nx, ny, nz, porosity, mask seed, parameter seed, C-rate): 60, 42, 64 and
# 54 voxels, so every structure ends in a partly filled 32-voxel tile
SHAPES = [(5, 4, 3, 0.6, 1, 1, 0.1), (7, 3, 2, 0.5, 2, 0, 1.0), (4, 4, 4, 0.7, 3, 0, 0.5),
          (9, 2, 3, 0.6, 4, 1, 0.1)]
T_NEW = [0.5, 1.2, 0.05, 3.0]
DT = [0.1, 0.2, 0.05, 1.0]


@pytest.fixture(scope="module")
def batch_case():
    from paper_2511_05233_amd import lsbdg
    structs, ctxs, masks, kin = [], [], [], []
    for nx, ny, nz, por, ms, ps, fc in SHAPES:
        mask = synth.porosity_mask((nz, ny, nx), por, ms)
        D0, i0 = synth.sample_transport_kinetics(ps)
        kw = dict(D0=D0, kE=i0 / om.F, f_C=fc)
        structs.append(dict(nx=nx, ny=ny, nz=nz, h=1e-6, phase=mask, **kw))
        ctxs.append(lsbdg.Context(nx, ny, nz, 1e-6, 1, mask, **kw))
        masks.append(mask)
        kin.append(kw)
    b = lsbdg.Batch(structs)
    print(f"[batch] {b.n} structures, {b.n_elem} voxels, {b.n_tiles} tiles, offsets {b.offsets}", flush=True)
    us = [synth.random_state(ctx.n_elem, 8, 10 + s, phase=masks[s], phi_spread=5e-3) for s, ctx in enumerate(ctxs)]
    uos = [synth.random_state(ctx.n_elem, 8, 20 + s, phase=masks[s]) for s, ctx in enumerate(ctxs)]
    return b, ctxs, masks, kin, us, uos


def _cat(parts, dtype):
    return torch.tensor(np.concatenate(parts, axis=1), dtype=dtype, device="cuda:0")


def test_layout(batch_case):
    b, ctxs, *_ = batch_case
    sizes = [c.n_elem for c in ctxs]
    assert b.offsets == list(np.concatenate([[0], np.cumsum(sizes)]))
    assert b.n_tiles == sum((n + 31) // 32 for n in sizes)


def _rel(a, b):
    """max |a - b| / max |b| over the whole array."""
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


# Largest relative deviation from the single-structure call allowed for the
# outputs that pass through the batched linearisation or block kernels: the
# same node code compiled into another kernel may contract multiply-adds
# differently (observed: FP64 blocks 1e-15); FP32 inverses amplify a
# rounding difference of the assembled block by its condition number.
LOOSE = {torch.float64: 1e-13, torch.float32: 1e-5}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batched_operators_equal_single_structure_calls(batch_case, dtype):
    """Mass, residual and full JVP: bit for bit.  Condensed and linearised
    JVP and the block apply: within LOOSE (bit for bit where the kernels
    compile alike)."""
    b, ctxs, masks, kin, us, uos = batch_case
    u = _cat(us, dtype)
    uo = _cat(uos, dtype)
    m = b.mass(uo)
    r = b.residual(u, m, T_NEW, DT)
    v9 = _cat([synth.random_vector(9, c.n_elem, 8, 30 + s) for s, c in enumerate(ctxs)], dtype)
    v7 = v9[:7].contiguous()
    jf = b.jvp(u, v9, T_NEW, DT)
    jc = b.jvp(u, v7, T_NEW, DT, condensed=True)
    b.linearize(u, T_NEW, DT)
    jl = b.jvp(u, v7, T_NEW, DT, linearized=True)
    b.blockjacobi_setup(u, T_NEW, DT)
    y = b.blockjacobi_apply(v7)
    torch.cuda.synchronize()
    for s, ctx in enumerate(ctxs):
        us_ = b.part(u, s).contiguous()
        ms_ = ctx.mass(b.part(uo, s).contiguous())
        vs = b.part(v7, s).contiguous()
        ref_c = ctx.jvp(us_, vs, T_NEW[s], DT[s], condensed=True)
        ctx.linearize(us_, T_NEW[s], DT[s])
        ref_l = ctx.jvp(us_, vs, T_NEW[s], DT[s], linearized=True)
        ctx.blockjacobi_setup(us_, T_NEW[s], DT[s])
        ref_y = ctx.blockjacobi_apply(vs)
        dc, dl, dy = _rel(b.part(jc, s), ref_c), _rel(b.part(jl, s), ref_l), _rel(b.part(y, s), ref_y)
        print(f"[batch] {dtype} structure {s} ({ctx.n_elem} voxels): condensed JVP {dc:.2e}, "
              f"linearised JVP {dl:.2e}, block apply {dy:.2e}", flush=True)
        assert torch.equal(b.part(m, s), ms_)
        assert torch.equal(b.part(r, s), ctx.residual(us_, ms_, T_NEW[s], DT[s]))
        assert torch.equal(b.part(jf, s), ctx.jvp(us_, b.part(v9, s).contiguous(), T_NEW[s], DT[s]))
        assert max(dc, dl, dy) <= LOOSE[dtype]


def test_batched_residual_matches_oracle(batch_case):
    """Structure 1 of the batch (7 x 3 x 2 voxels, 1C, its own clock)
    against the oracle's residual in FP64."""
    b, ctxs, masks, kin, us, uos = batch_case
    u = _cat(us, torch.float64)
    m = b.mass(_cat(uos, torch.float64))
    r = b.residual(u, m, T_NEW, DT).cpu().numpy()
    s = 1
    nx, ny, nz = SHAPES[s][:3]
    P = om.Problem(nx, ny, nz, 1e-6, 1, masks[s], **kin[s])
    ref = odg.residual(P, us[s], odg.old_mass(P, uos[s]), T_NEW[s], DT[s])
    err = field_errors(b.part(torch.tensor(r), s).numpy(), ref)
    print(f"[batch] oracle residual errors {err}", flush=True)
    assert np.all(err < 1e-11)


def test_batched_calls_check_their_arguments(batch_case):
    from paper_2511_05233_amd import lsbdg
    b, *_ = batch_case
    u = torch.zeros((9, b.n_elem, 8), dtype=torch.float64, device="cuda:0")
    m = torch.zeros((8, b.n_elem, 8), dtype=torch.float64, device="cuda:0")
    with pytest.raises(lsbdg.DgError, match="DG_EINVAL"):
        b.residual(u, m, T_NEW, [0.1, 0.0, 0.1, 0.1])
    fresh = lsbdg.Batch([dict(nx=2, ny=2, nz=2, h=1e-6, phase=np.ones(8, np.uint8))])
    with pytest.raises(lsbdg.DgError, match="DG_ESTATE"):
        fresh.blockjacobi_apply(torch.zeros((7, 8, 8), dtype=torch.float64, device="cuda:0"))


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_batched_solves_equal_single_structure_solves(batch_case, inner):
    """dg_batch_initial_state and dg_batch_step (three workers, four
    structures on their own clocks) leave every structure exactly where the
    single-structure solves do, with the same iteration counts."""
    b, ctxs, *_ = batch_case
    print(f"[batch] initial states, inner {inner}", flush=True)
    u, reps0 = b.initial_state(inner=inner, workers=3)
    for s, ctx in enumerate(ctxs):
        ref, rep = ctx.initial_state(inner=inner)
        assert torch.equal(b.part(u, s), ref), s
        assert (reps0[s]["newton_its"], reps0[s]["gmres_its"]) == (rep["newton_its"], rep["gmres_its"])
    from paper_2511_05233_amd import lsbdg
    t_n, dt = [0.0, 0.0, 0.0, 0.0], [0.1, 0.02, 0.05, 0.2]
    u0 = u.clone()
    print(f"[batch] steps, inner {inner}", flush=True)
    try:
        reps = b.step(u, t_n, dt, inner=inner, workers=3)
    except lsbdg.DgError as e:        # a structure that does not converge: compared below all the same
        print(f"[batch] {e}", flush=True)
        reps = e.reports
    converged = 0
    for s, ctx in enumerate(ctxs):
        ref = b.part(u0, s).contiguous()
        try:
            rep = ctx.step(ref, t_n[s], dt[s], inner=inner)
        except lsbdg.DgError as e:
            rep = e.report
        print(f"[batch] structure {s}: status {reps[s]['status']}, {reps[s]['newton_its']} Newton, "
              f"{reps[s]['gmres_its']} GMRES", flush=True)
        assert torch.equal(b.part(u, s), ref), s
        assert reps[s] == rep
        converged += reps[s]["status"] == 0
    assert converged >= 3


def test_batched_step_rejects_bad_steps(batch_case):
    from paper_2511_05233_amd import lsbdg
    b, *_ = batch_case
    u = torch.zeros((9, b.n_elem, 8), dtype=torch.float64, device="cuda:0")
    with pytest.raises(lsbdg.DgError, match="DG_EINVAL"):
        b.step(u, 0.0, [0.1, 0.1, -1.0, 0.1])


# Launch shapes tried beside the default (32 voxels, one workgroup per work
# item): every tile size, one workgroup per item and persistent grids.
LAUNCH_SHAPES = [(8, 0), (16, 0), (8, 1), (16, 2), (32, 1), (32, 3)]


@pytest.fixture(scope="module")
def shape_case():
    """Two structures, 4,096 and 1,287 voxels: with 8-voxel tiles 680 grid
    positions, so a persistent grid of one workgroup per compute unit makes
    several passes, and both structures end in a partly filled tile."""
    from paper_2511_05233_amd import lsbdg
    structs, us, uos = [], [], []
    for s, (nx, ny, nz, por, seed) in enumerate([(16, 16, 16, 0.6, 5), (13, 11, 9, 0.5, 6)]):
        mask = synth.porosity_mask((nz, ny, nx), por, seed)
        D0, i0 = synth.sample_transport_kinetics(s)
        structs.append(dict(nx=nx, ny=ny, nz=nz, h=1e-6, phase=mask, D0=D0, kE=i0 / om.F, f_C=0.5))
        us.append(synth.random_state(nx * ny * nz, 8, 40 + s, phase=mask, phi_spread=5e-3))
        uos.append(synth.random_state(nx * ny * nz, 8, 50 + s, phase=mask))
    b = lsbdg.Batch(structs)
    v9 = np.concatenate([synth.random_vector(9, nx * ny * nz, 8, 60 + s)
                         for s, (nx, ny, nz) in enumerate([(16, 16, 16), (13, 11, 9)])], axis=1)
    print(f"[batch] shape case: {b.n_elem} voxels", flush=True)
    return structs, b, us, uos, v9


def _operators(b, u, m, v9, t, dt):
    v7 = v9[:7].contiguous()
    return (b.residual(u, m, t, dt), b.jvp(u, v9, t, dt), b.jvp(u, v7, t, dt, condensed=True))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_every_launch_shape_gives_the_same_results(shape_case, dtype):
    """Residual, full and condensed tangent: bit for bit the default
    shape's values in every tile size, with and without a persistent grid
    (only the workgroup that computes a node changes)."""
    from paper_2511_05233_amd import lsbdg
    structs, b, us, uos, v9 = shape_case
    u = _cat(us, dtype)
    m = b.mass(_cat(uos, dtype))
    v = torch.tensor(v9, dtype=dtype, device="cuda:0")
    t, dt = [0.7, 2.0], [0.1, 0.5]
    for op in lsbdg.BATCH_OPS:
        b.set_shape(dtype, op, 32, 0)
    ref = _operators(b, u, m, v, t, dt)
    for tv, pers in LAUNCH_SHAPES:
        print(f"[batch] {dtype} shape ({tv}, {pers})", flush=True)
        for op in lsbdg.BATCH_OPS:
            b.set_shape(dtype, op, tv, pers)
            assert b.get_shape(dtype, op) == (tv, pers)
        got = _operators(b, u, m, v, t, dt)
        for name, g, r in zip(lsbdg.BATCH_OPS, got, ref):
            assert torch.equal(g, r), (tv, pers, name)
    # the brick shape of the condensed tangent sums in another order
    b.set_shape(dtype, "jvp_condensed", 64, 0)
    jb = b.jvp(u, v[:7].contiguous(), t, dt, condensed=True)
    print(f"[batch] {dtype} bricks vs tiles: condensed JVP {_rel(jb, ref[2]):.2e}", flush=True)
    assert _rel(jb, ref[2]) <= LOOSE[dtype]
    for op in lsbdg.BATCH_OPS:
        b.set_shape(dtype, op, 32, 0)


def test_set_shape_checks_its_arguments(shape_case):
    from paper_2511_05233_amd import lsbdg
    _, b, *_ = shape_case
    for tv, pers in [(4, 0), (64, 0), (32, -1), (32, 65)]:
        with pytest.raises(lsbdg.DgError, match="DG_EINVAL"):
            b.set_shape(torch.float32, "residual", tv, pers)
    with pytest.raises(lsbdg.DgError, match="DG_EINVAL"):
        b.set_shape(torch.float32, "jvp_condensed", 64, 1)
    assert b.get_shape(torch.float32, "residual") == (32, 0)


def test_autotune_keeps_the_fastest_timed_shape(shape_case):
    """FP32: every operator gets the shape with the smallest timed launch
    (never slower than the default, which is among the candidates), and a
    later batch of the same size class starts from it."""
    from paper_2511_05233_amd import lsbdg
    structs, b, us, uos, v9 = shape_case
    u = _cat(us, torch.float32)
    m = b.mass(_cat(uos, torch.float32))
    v = torch.tensor(v9, dtype=torch.float32, device="cuda:0")
    tune, ncand = b.autotune(u, v, m, [0.7, 2.0], [0.1, 0.5], reps=3)
    print(f"[batch] autotune: {tune}, {ncand} shapes per operator", flush=True)
    assert ncand in (3, 6)
    for op, (shape, ms, ms_def) in tune.items():
        assert shape[0] in (8, 16, 32) and shape[1] >= 0 or op == "jvp_condensed" and shape == (64, 0)
        assert 0.0 < ms <= ms_def
        assert b.get_shape(torch.float32, op) == shape
    b2 = lsbdg.Batch(structs)
    for op, (shape, _, _) in tune.items():
        assert b2.get_shape(torch.float32, op) == shape
    b2.close()
    for op in lsbdg.BATCH_OPS:
        b.set_shape(torch.float32, op, 32, 0)

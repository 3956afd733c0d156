"""The 64-structure batch workload against the oracle (GPU).

The batch workload: 64 cubic structures with edges U{24..64} voxels and
porosity U(0.4, 0.75) (seeded), each with its own transport and kinetics
draw, concatenated voxel by voxel.  The batched FP64 residual and the
batched condensed tangent at a stored linearisation (FP64 and FP32, the
Krylov operator) run as one launch over all 64 structures; on the four
smallest structures the result is compared with the oracle at sampled
voxels -- the eight corners, separator-face voxels and random ones -- each
evaluated on the 3 x 3 x 3 patch of voxels around it (a voxel's rows depend
on itself and its face neighbours only).
"""
import numpy as np
import pytest

import synth
from oracle import dg as odg
from oracle import model as om
from tests.helpers import field_errors, oracle_jvp_condensed_at, oracle_residual_at

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

T_NEW, DT = 0.4, 0.05


@pytest.fixture(scope="module")
def batch64():
    from paper_2511_05233_amd import lsbdg
    specs = synth.batch_structures(64)
    structs, problems = [], []
    for b, (edge, por, mseed) in enumerate(specs):
        mask = synth.porosity_mask((edge, edge, edge), por, mseed)
        D0, i0 = synth.sample_transport_kinetics(b)
        kw = dict(D0=D0, kE=i0 / om.F, f_C=0.1)
        structs.append(dict(nx=edge, ny=edge, nz=edge, h=1e-6, phase=mask, **kw))
        problems.append((edge, mask, kw))
    print(f"[batch64] setting up {len(structs)} structures", flush=True)
    B = lsbdg.Batch(structs)
    print(f"[batch64] {B.n_elem} voxels", flush=True)
    smallest = sorted(range(64), key=lambda s: (specs[s][0], s))[:4]
    return B, problems, smallest


def _sample(edge, n, seed):
    Ne = edge ** 3
    c = [0, edge - 1, edge * (edge - 1), edge * edge - 1, Ne - edge * edge, Ne - edge, Ne - 1,
         Ne - edge * edge + edge - 1]
    sep = [edge - 1 + edge * (edge // 2) + edge * edge * (edge // 3)]
    rng = np.random.default_rng(seed)
    return np.concatenate([c, sep, rng.integers(0, Ne, n)])


def _states(B, problems, dtype):
    parts, vparts = [], []
    for s, (edge, mask, _) in enumerate(problems):
        Ne = edge ** 3
        parts.append(synth.random_state(Ne, 8, 500 + s, phase=mask, phi_spread=5e-3))
        rng = np.random.default_rng(600 + s)
        scale = np.array([1500, 6, 6e-3, 4e-3, 2e-3, 4e-12, 3e-3])
        vparts.append(scale[:, None, None] * rng.standard_normal((7, Ne, 8)))
    u = np.concatenate(parts, axis=1)
    v = np.concatenate(vparts, axis=1)
    if dtype == torch.float32:
        u = u.astype(np.float32).astype(np.float64)
        v = v.astype(np.float32).astype(np.float64)
    return u, v


def test_batched_residual_of_the_smallest_structures(batch64):
    B, problems, smallest = batch64
    u, _ = _states(B, problems, torch.float64)
    ud = torch.tensor(u, device="cuda:0")
    m = B.mass(ud)
    r = B.residual(ud, m, T_NEW, DT).cpu().numpy()
    mh = m.cpu().numpy()
    for s in smallest:
        edge, mask, kw = problems[s]
        P = om.Problem(edge, edge, edge, 1e-6, 1, mask, **kw)
        lo, hi = B.offsets[s], B.offsets[s + 1]
        elems = _sample(edge, 24, s)
        ref = oracle_residual_at(P, u[:, lo:hi], mh[:, lo:hi], T_NEW, DT, elems)
        err = field_errors(r[:, lo:hi][:, elems], ref)
        print(f"[batch64] structure {s} ({edge}^3) residual errors {err}", flush=True)
        assert np.all(err < 1e-12), (s, err)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)], ids=["f64", "f32"])
def test_batched_krylov_operator_of_the_smallest_structures(batch64, dtype, tol):
    B, problems, smallest = batch64
    u, v = _states(B, problems, dtype)
    ud = torch.tensor(u, device="cuda:0", dtype=dtype)
    vd = torch.tensor(v, device="cuda:0", dtype=dtype)
    B.linearize(ud, T_NEW, DT)
    jv = B.jvp(ud, vd, T_NEW, DT, linearized=True).cpu().numpy().astype(np.float64)
    for s in smallest:
        edge, mask, kw = problems[s]
        P = om.Problem(edge, edge, edge, 1e-6, 1, mask, **kw)
        lo, hi = B.offsets[s], B.offsets[s + 1]
        elems = _sample(edge, 12, 100 + s)
        us, vs = u[:, lo:hi], v[:, lo:hi]
        ref = oracle_jvp_condensed_at(P, us, vs, odg.old_mass(P, us), T_NEW, DT, elems)
        err = field_errors(jv[:, lo:hi][:, elems], ref)
        print(f"[batch64] structure {s} ({edge}^3) {dtype} Krylov operator errors {err}", flush=True)
        assert np.all(err < tol), (s, err)

"""Shared test helpers: problem construction and oracle sampling."""
import numpy as np

import synth
from oracle import dg as odg
from oracle import model as om


def problem_and_context(nx, ny, nz, k=1, porosity=0.6, mask_seed=0, param_seed=0, mask=None,
                        paper_params=False, **kw):
    """Matching oracle Problem and HIP Context for a synthetic voxel structure."""
    from paper_2511_05233_amd import lsbdg
    if mask is None:
        mask = synth.porosity_mask((nz, ny, nx), porosity, mask_seed)
    if paper_params:
        D0, kE = om.D0_PAPER.copy(), om.K_E_PAPER.copy()
    else:
        D0, i0 = synth.sample_transport_kinetics(param_seed)
        kE = i0 / om.F
    P = om.Problem(nx, ny, nz, 1e-6, k, mask, D0=D0, kE=kE, **kw)
    ctx = lsbdg.Context(nx, ny, nz, 1e-6, k, mask, D0=D0, kE=kE,
                        f_C=kw.get("f_C"), j_el=kw.get("j_el"), eps_struct=kw.get("eps_struct"),
                        use_TH=kw.get("use_TH"))
    return P, ctx, mask


def field_errors(got, ref):
    """Per-field max |got - ref| / max |ref|."""
    out = []
    for f in range(ref.shape[0]):
        scale = np.max(np.abs(ref[f]))
        out.append(np.max(np.abs(got[f] - ref[f])) / (scale if scale > 0 else 1.0))
    return np.array(out)


def oracle_residual_at(P, u, m_old, t_new, dt, elems):
    """Oracle residual of the listed elements of a large mesh.

    The residual of a voxel depends on itself and its face neighbours only,
    so it is evaluated on the 3x3x3 patch around the voxel (clipped at the
    mesh boundary, which keeps the true boundary faces) with the full mesh's
    current density and structure fraction.
    """
    out = np.zeros((u.shape[0], len(elems), u.shape[2]))
    mask = P.phase
    for j, e in enumerate(elems):
        e = int(e)
        ix, iy, iz = e % P.nx, (e // P.nx) % P.ny, e // (P.nx * P.ny)
        xs = slice(max(ix - 1, 0), min(ix + 2, P.nx))
        ys = slice(max(iy - 1, 0), min(iy + 2, P.ny))
        zs = slice(max(iz - 1, 0), min(iz + 2, P.nz))
        sub = mask[zs, ys, xs]
        pz, py, px = sub.shape
        Q = om.Problem(px, py, pz, P.h, P.k, sub, D0=P.D0, kE=P.kE, f_C=P.f_C, T=P.T,
                       sigma=P.sigma, c_min=P.c_min, epsL_min=P.epsL_min, use_TH=P.use_TH,
                       j_el=P.j_el, eps_struct=P.eps_struct_used)
        g = np.arange(P.n_elem).reshape(P.nz, P.ny, P.nx)[zs, ys, xs].reshape(-1)
        R = odg.residual(Q, u[:, g], m_old[:, g], t_new, dt)
        loc = int(np.nonzero(g == e)[0][0])
        out[:, j] = R[:, loc]
    return out

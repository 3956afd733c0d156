"""Element blocks, Newton, backward-Euler step, potential initialisation.

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

The result of a step is the root u^{n+1} of the discrete backward-Euler
system R(u^{n+1}; u^n, dt) = 0 (Eq. 50 applied to the DG residual).  How
the root is found does not change it; this module uses plain Newton
iterations whose linear systems are solved by GMRES (Saad & Schultz 1986)
on the complex-step Jacobian-vector product, preconditioned by the exact
element-diagonal Jacobian blocks and diagonally scaled by the magnitude of
each unknown, plus an additive coarse correction on the space of one
global constant per field (Galerkin projection of J).  The coarse space
removes the near-null mode of the element-preconditioned operator: a
uniform shift of Phi_L, which only the reaction current (not transport)
resists.  The convergence test is deliberately tight (relative update
1e-12 per unknown) so that field comparisons at 1e-10 are meaningful.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import dg
from . import model as M

# per-field floors of the unknown scaling (concentrations, potential, solids)
_FLOOR = np.array([1e-20] * 6 + [M.R_GAS * M.T_K / M.F, 1e-12, 1e-12])


def colouring(P):
    """Checkerboard colour (ix + iy + iz) mod 2 per element (flat)."""
    iz, iy, ix = np.meshgrid(np.arange(P.nz), np.arange(P.ny), np.arange(P.nx), indexing="ij")
    return ((ix + iy + iz) % 2).reshape(-1)


def element_blocks(P, u, m_old, t_new, dt, fields=tuple(range(9)), condensed=False):
    """Element-diagonal Jacobian blocks, shape (Ne, nb, nb), nb = len(fields) n_p.

    Block index = field position * n_p + node.  Two probes per local unknown
    (one per checkerboard colour): perturbing one local unknown in every
    element of a colour reaches an element's own rows only from itself,
    because face neighbours have the other colour.  ``condensed`` applies
    the node-local elimination of the solid fractions (7 fields).
    """
    npn = P.n_nodes
    fields = tuple(fields)
    nf = len(fields)
    nb = nf * npn
    Ne = P.n_elem
    col = colouring(P)
    blocks = np.zeros((Ne, nb, nb))
    for colour in (0, 1):
        sel = col == colour
        for fi, f in enumerate(fields):
            for a in range(npn):
                if condensed:
                    v = np.zeros((7, Ne, npn))
                    v[f, sel, a] = 1.0
                    Jv = dg.jvp_condensed(P, u, v, m_old, t_new, dt)
                else:
                    v = np.zeros((9, Ne, npn))
                    v[f, sel, a] = 1.0
                    Jv = dg.jvp(P, u, v, m_old, t_new, dt)
                rows = Jv[list(fields)][:, sel, :]            # (nf, nsel, np)
                blocks[sel, :, fi * npn + a] = rows.transpose(1, 0, 2).reshape(-1, nb)
    return blocks


def block_apply_inverse(blocks, x_fields):
    """y_e = B_e^{-1} x_e for x of shape (nf, Ne, np)."""
    nf, Ne, npn = x_fields.shape
    xe = x_fields.transpose(1, 0, 2).reshape(Ne, nf * npn)
    ye = np.linalg.solve(blocks, xe[:, :, None])[:, :, 0]
    return ye.reshape(Ne, nf, npn).transpose(1, 0, 2)


def _neighbour_table(P):
    """Element index of the 7-point stencil members (self, -x, +x, -y, +y, -z, +z); -1 outside."""
    g = dg.element_grid(P)
    out = [g.reshape(-1)]
    for axis in (2, 1, 0):
        for step in (-1, 1):
            nb = np.full(g.shape, -1)
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if step == 1:
                dst[axis], src[axis] = slice(0, -1), slice(1, None)
            else:
                dst[axis], src[axis] = slice(1, None), slice(0, -1)
            nb[tuple(dst)] = g[tuple(src)]
            out.append(nb.reshape(-1))
    return np.stack(out)


def sparse_jacobian(P, u, m_old, t_new, dt, fields=tuple(range(9))):
    """Full Jacobian (CSR) restricted to ``fields`` by complex-step probing.

    Colour (ix + 2 iy + 3 iz) mod 7 gives the 7 members of every element's
    stencil distinct colours, so probing one local unknown in all elements of
    a colour lets each element attribute its response to exactly one source.
    Unknown order: (field position, element, node).
    """
    import scipy.sparse as sp
    fields = list(fields)
    nf, Ne, npn = len(fields), P.n_elem, P.n_nodes
    iz, iy, ix = np.meshgrid(np.arange(P.nz), np.arange(P.ny), np.arange(P.nx), indexing="ij")
    colour = ((ix + 2 * iy + 3 * iz) % 7).reshape(-1)
    nbt = _neighbour_table(P)
    rows, cols, vals = [], [], []
    b_idx = np.arange(npn)
    for c in range(7):
        src = np.full(Ne, -1)
        for nb in nbt:
            hit = (nb >= 0) & (colour[np.maximum(nb, 0)] == c)
            src = np.where(hit, nb, src)
        have = np.nonzero(src >= 0)[0]
        if len(have) == 0:
            continue
        sel = colour == c
        for fi, f in enumerate(fields):
            for a in range(npn):
                v = np.zeros_like(u)
                v[f, sel, a] = 1.0
                Jv = dg.jvp(P, u, v, m_old, t_new, dt)[fields]
                for gi in range(nf):
                    blk = Jv[gi][have]                       # (nh, np)
                    r = ((gi * Ne + have)[:, None] * npn + b_idx[None, :]).ravel()
                    cc = np.repeat((fi * Ne + src[have]) * npn + a, npn)
                    val = blk.ravel()
                    nz = val != 0.0
                    rows.append(r[nz]); cols.append(cc[nz]); vals.append(val[nz])
    n = nf * Ne * npn
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


class NewtonFailure(RuntimeError):
    pass


# Newton globalisation.  The Newton direction du solves J du = -R as usual;
# positive unknowns (concentrations, solid fractions) are then updated
# multiplicatively, x <- x exp(lam du/x), which is Newton's method in the
# logarithms of those unknowns (same linear system, column-scaled), keeps
# them positive and makes mass-action / Butler-Volmer terms near-linear.
# The exponent is capped at ln(10) per iteration.  The step length lam is
# halved while the merit ||W R|| does not decrease; W (element-block inverse
# and unknown scales at the start of the step) is fixed during a step.
_MAXLOG = np.log(10.0)


def _apply_update(u, du, lam, fields, two_sided=False):
    """two_sided: the exponent is also capped from below at -ln 10 (no
    unknown falls by more than a factor 10 in one iteration)."""
    out = u.copy()
    for fi, f in enumerate(fields):
        x = u[f]
        d = lam * du[fi]
        if f == 6:
            out[f] = x + d
            continue
        pos = x > 0
        ex = np.clip(np.where(pos, d / np.where(pos, x, 1.0), 0.0), -_MAXLOG if two_sided else -np.inf, _MAXLOG)
        out[f] = np.where(pos, x * np.exp(ex), x + d)
    return out


def _gmres_direction(P, u, R, m_old, t_new, dt, fields, S, blocks, rtol, restart):
    """Newton direction by preconditioned GMRES (element blocks + coarse)."""
    nf = len(fields)
    shape = (nf,) + u.shape[1:]
    n = int(np.prod(shape))
    if blocks is None:
        blocks = element_blocks(P, u, m_old, t_new, dt, fields)
    # coarse space: one global constant per field, weighted by S
    JZ = np.empty((nf,) + shape)
    for fi in range(nf):
        v = np.zeros_like(u)
        v[fields[fi]] = S[fi]
        JZ[fi] = dg.jvp(P, u, v, m_old, t_new, dt)[fields]
    Ac = np.array([[np.sum(S[gi] * JZ[fi][gi]) for fi in range(nf)] for gi in range(nf)])

    def precond(r):
        zr = np.array([np.sum(S[gi] * r[gi]) for gi in range(nf)])
        yc = np.linalg.solve(Ac, zr)
        out = block_apply_inverse(blocks, r)
        for fi in range(nf):
            out[fi] += S[fi] * yc[fi]
        return out

    b = -precond(R[fields]) / S

    def matvec(y):
        v = np.zeros_like(u)
        v[fields] = S * y.reshape(shape)
        Jv = dg.jvp(P, u, v, m_old, t_new, dt)[fields]
        return (precond(Jv) / S).reshape(-1)

    A = spla.LinearOperator((n, n), matvec=matvec, dtype=np.float64)
    count = [0]

    def cb(_x):
        count[0] += 1

    y, info = spla.gmres(A, b.reshape(-1), rtol=rtol, atol=0.0, restart=restart,
                         maxiter=40, callback=cb, callback_type="pr_norm")
    return S * y.reshape(shape), count, info


def _aggregate_index(P, edge):
    """Aggregate of every element: cubes of edge^3 voxels, x fastest."""
    e = np.arange(P.n_elem)
    ix, iy, iz = e % P.nx, (e // P.nx) % P.ny, e // (P.nx * P.ny)
    ax, ay = -(-P.nx // edge), -(-P.ny // edge)
    return (ix // edge) + ax * ((iy // edge) + ay * (iz // edge)), ax * ay * (-(-P.nz // edge))


class _SparseSolver:
    """Newton directions from the probed sparse Jacobian J (kept for several
    Newton iterations: the chord method, whose limit is the same root).

    GMRES on the equilibrated system A = D_r J diag(S) (columns scaled by
    the unknown magnitudes, rows by their largest entry), right-
    preconditioned by the exact element-diagonal blocks of A plus an
    additive coarse correction Z E^-1 Z^T on per-field constants over
    aggregates of edge^3 voxels (E = Z^T A Z, dense LU).  Right
    preconditioning makes GMRES minimise the residual of the equilibrated
    system itself, so its tolerance bounds the error of the direction.
    Only the speed of the linear solves depends on these choices, not the
    root."""

    def __init__(self, P, Jm, S, fields, edge=4):
        import scipy.sparse as sp
        import scipy.linalg as sla
        nf, Ne, npn = len(fields), P.n_elem, P.n_nodes
        nb = nf * npn
        self.shape = (nf, Ne, npn)
        A = (Jm @ sp.diags(S.reshape(-1))).tocsr()
        self.rs = 1.0 / np.maximum(abs(A).max(axis=1).toarray().ravel(), 1e-300)
        A = (sp.diags(self.rs) @ A).tocsr()
        self.A = A
        # element blocks: unknown (f, e, a) -> element e, block index f npn + a
        k = np.arange(nf * Ne * npn)
        f_, rem = k // (Ne * npn), k % (Ne * npn)
        e_, a_ = rem // npn, rem % npn
        bi = f_ * npn + a_
        C = A.tocoo()
        same = e_[C.row] == e_[C.col]
        blocks = np.zeros((Ne, nb, nb))
        blocks[e_[C.row[same]], bi[C.row[same]], bi[C.col[same]]] = C.data[same]
        self.binv = np.linalg.inv(blocks)
        self.e_, self.bi = e_, bi
        agg, na = _aggregate_index(P, edge)
        cols = f_ * na + agg[e_]
        self.Z = sp.csr_matrix((np.ones(len(k)), (k, cols)), shape=(len(k), nf * na))
        E = (self.Z.T @ (A @ self.Z)).toarray()
        self.lu = sla.lu_factor(E)
        self._sla = sla

    def precond(self, r):
        Ne = self.shape[1]
        rb = np.zeros((Ne, self.binv.shape[1]))
        rb[self.e_, self.bi] = r
        yb = np.einsum("eij,ej->ei", self.binv, rb)
        y = yb[self.e_, self.bi]
        return y + self.Z @ self._sla.lu_solve(self.lu, self.Z.T @ r)

    def direction(self, R, rtol, restart):
        """y with A y = -D_r R to relative residual rtol (du = S y)."""
        n = self.A.shape[0]
        b = -self.rs * R.reshape(-1)
        op = spla.LinearOperator((n, n), matvec=lambda z: self.A @ self.precond(z), dtype=np.float64)
        count = [0]
        z, info = spla.gmres(op, b, rtol=rtol, atol=0.0, restart=restart, maxiter=10,
                             callback=lambda _x: count.__setitem__(0, count[0] + 1), callback_type="pr_norm")
        return self.precond(z), count, info


def newton(P, u0, m_old, t_new, dt, fields=tuple(range(9)), tol=1e-12, maxit=80,
           gmres_rtol=1e-13, restart=120, log=None, linear=None, two_sided=False):
    """Damped Newton on the rows/columns ``fields``; other fields frozen.

    Each iteration solves J du = -R, either directly (sparse LU of the
    probed Jacobian; the default for small systems) or by GMRES
    (operator and right side preconditioned by the element-block inverse
    plus the global coarse correction, and scaled by the unknown
    magnitudes), applies the update above and backtracks on the merit.
    Converged when a full step's largest relative update is below ``tol``.
    linear="sparse": GMRES on the probed sparse Jacobian (see _SparseSolver),
    re-probed when a full step fails to halve the update.  two_sided: the
    multiplicative update is capped at a factor 10 both ways (the default
    caps growth only); the path differs, the root does not.
    Returns (u, info) with info = dict(iterations, gmres, update).
    """
    fields = list(fields)
    u = u0.copy()
    shape = (len(fields),) + u.shape[1:]
    n = int(np.prod(shape))
    nf = len(fields)
    if linear is None:
        linear = "direct" if n <= 40000 else "gmres"
    total_gm = 0
    upd = np.inf
    R = dg.residual(P, u, m_old, t_new, dt)
    blocks0 = element_blocks(P, u, m_old, t_new, dt, fields)
    S0 = np.maximum(np.abs(u[fields]), _FLOOR[fields][:, None, None])

    def merit_of(Rv):
        return float(np.linalg.norm(block_apply_inverse(blocks0, Rv[fields]) / S0))

    merit = merit_of(R)
    solver, prev_upd = None, np.inf
    for it in range(1, maxit + 1):
        if not np.all(np.isfinite(R)):
            raise NewtonFailure("non-finite residual")
        S = np.maximum(np.abs(u[fields]), _FLOOR[fields][:, None, None])
        if linear == "sparse":
            if solver is None:
                Jm = sparse_jacobian(P, u, m_old, t_new, dt, fields)
                solver = _SparseSolver(P, Jm, S, fields)
                S_solve = S
            y, count, info = solver.direction(R[fields], gmres_rtol, restart)
            du = (S_solve.reshape(-1) * y).reshape(shape)
            total_gm += count[0]
        elif linear == "direct":
            import scipy.sparse.linalg as _sl
            import scipy.sparse as _sp
            Jm = sparse_jacobian(P, u, m_old, t_new, dt, fields)
            # equilibrate: columns by the unknown scales, rows by their max
            Dc = _sp.diags(S.reshape(-1))
            Js = (Jm @ Dc).tocsr()
            rmax = np.maximum(abs(Js).max(axis=1).toarray().ravel(), 1e-300)
            Dr = _sp.diags(1.0 / rmax)
            Js = (Dr @ Js).tocsc()
            y = _sl.spsolve(Js, -(R[fields].reshape(-1) / rmax))
            du = (S.reshape(-1) * y).reshape(shape)
            count, info = [0], 0
        else:
            du, count, info = _gmres_direction(P, u, R, m_old, t_new, dt, fields, S,
                                               None if it > 1 else blocks0, gmres_rtol, restart)
            total_gm += count[0]
        upd = float(np.max(np.abs(du) / S))
        lam = 1.0
        for _ in range(40):
            ut = _apply_update(u, du, lam, fields, two_sided)
            Rt = dg.residual(P, ut, m_old, t_new, dt)
            mt = merit_of(Rt) if np.all(np.isfinite(Rt)) else np.inf
            if mt < merit or (lam == 1.0 and upd < 1e-8):
                break
            lam *= 0.5
        if log is not None:
            log(f"newton it {it}: gmres {count[0]} (info {info}) update {upd:.3e} "
                f"lambda {lam:.3g} merit {merit:.3e} -> {mt:.3e}")
        u, R, merit = ut, Rt, mt
        if lam == 1.0 and upd < tol:
            return u, {"iterations": it, "gmres": total_gm, "update": upd}
        if linear == "sparse" and (lam < 1.0 or upd > 0.5 * prev_upd):
            solver = None                  # chord slowed down: probe J again
        prev_upd = upd
    raise NewtonFailure(f"no convergence after {maxit} iterations (update {upd:.3e})")


def uniform_state(P):
    """Tab. InitialState concentrations everywhere, eps per phase, Phi_L = 0."""
    u = np.zeros((9, P.n_elem, P.n_nodes))
    c = P.initial_concentrations()
    for i in range(6):
        u[i] = c[i]
    u[7] = P.epsS8_0_e[:, None]
    u[8] = P.epsLi2S_0_e[:, None]
    return u


def initial_state(P, t0=0.0, **kw):
    """Equilibrium state of Tab. InitialState plus the steady potential.

    The paper relaxes the potentials with an added time derivative and a
    ramped current until steady (Sec. 2.10); this solves for the same fixed
    point directly: the charge equation for Phi_L at frozen concentrations
    and solid fractions with the full current and T_H at t0.
    """
    u = uniform_state(P)
    m_old = dg.old_mass(P, u)
    u, info = newton(P, u, m_old, t0, 1.0, fields=(6,), **kw)
    return u, info


def be_step(P, u_n, t_n, dt, limiter=False, **kw):
    """One backward-Euler step from (t_n, u_n) to t_n + dt (Eq. 50).
    limiter=True: the Newton root is then limited by the vertex-based
    limiter of oracle/limiter.py."""
    m_old = dg.old_mass(P, u_n)
    u, info = newton(P, u_n, m_old, t_n + dt, dt, **kw)
    if limiter:
        from . import limiter as lim
        u = lim.limit(P, u)[0]
    return u, info

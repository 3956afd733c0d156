"""ctypes binding of liblsbdg (include/lsbdg.h), argument marshalling only.

Every computation happens in the HIP library.  Arrays are torch device
tensors in the field-major layout a[f][e][n]; the current torch stream is
passed to each call.  A missing library raises instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsbdg.so")

DG_F64, DG_F32 = 0, 1
DG_JVP_FULL9, DG_JVP_CONDENSED7, DG_JVP_LINEARIZED7 = 0, 1, 2

_STATUS = {0: "DG_OK", -1: "DG_EINVAL", -2: "DG_ENOMEM", -3: "DG_EHIP", -4: "DG_ENOCONV",
           -5: "DG_ENAN", -6: "DG_ESTATE", -7: "DG_EUNSUPPORTED"}

# exported entry points and their ctypes signatures
_SIGNATURES = {
    "dg_params_default": (None, [C.c_void_p]),
    "dg_setup": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "dg_destroy": (C.c_int, [C.c_void_p]),
    "dg_workspace_bytes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_size_t)]),
    "dg_setup_ws": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t,
                              C.c_void_p, C.POINTER(C.c_void_p)]),
    "dg_info": (C.c_int, [C.c_void_p] + [C.c_void_p] * 5),
    "dg_mass": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_residual": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double,
                              C.c_double, C.c_void_p, C.c_void_p]),
    "dg_jvp": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_double,
                         C.c_double, C.c_void_p, C.c_void_p]),
    "dg_linearize": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_double, C.c_void_p]),
    "dg_blockjacobi_setup": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_double,
                                       C.c_void_p]),
    "dg_blockjacobi_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_blockjacobi_apply_bf16": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_blockjacobi_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_blockjacobi_info": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_solver_opts_default": (None, [C.c_void_p]),
    "dg_mg_setup": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p]),
    "dg_mg_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_mg_export": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p]),
    "dg_step": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                          C.c_void_p]),
    "dg_initial_state": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "dg_outputs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p]),
    "dg_outputs_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "dg_controller_init": (None, [C.c_void_p, C.c_int32, C.c_double, C.c_double]),
    "dg_advance": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p]),
    "dg_batch_setup": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "dg_batch_destroy": (C.c_int, [C.c_void_p]),
    "dg_batch_layout": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_batch_mass": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_batch_residual": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "dg_batch_linearize": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_batch_jvp": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p]),
    "dg_batch_blockjacobi_setup": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_void_p]),
    "dg_batch_blockjacobi_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_batch_initial_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                         C.c_void_p]),
    "dg_batch_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_int32, C.c_void_p]),
    "dg_batch_set_shape": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.c_void_p]),
    "dg_batch_get_shape": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.c_void_p]),
    "dg_batch_autotune": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dg_limit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dg_triad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int64, C.c_void_p]),
    "dg_last_error": (C.c_char_p, []),
}


class DgMesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("order", C.c_int32), ("h", C.c_double)]


class DgParams(C.Structure):
    _fields_ = [("T", C.c_double), ("D0", C.c_double * 7), ("kE", C.c_double * 6),
                ("f_C", C.c_double), ("j_el", C.c_double), ("eps_struct", C.c_double),
                ("sigma", C.c_double), ("c_min", C.c_double), ("epsL_min", C.c_double),
                ("use_TH", C.c_int32), ("reserved", C.c_int32)]


class DgSolverOpts(C.Structure):
    _fields_ = [("inner_prec", C.c_int32), ("gmres_restart", C.c_int32), ("gmres_maxit", C.c_int32),
                ("newton_maxit", C.c_int32), ("gmres_rtol", C.c_double), ("gmres_rtol_final", C.c_double),
                ("newton_tol", C.c_double),
                ("coarse", C.c_int32), ("coarse_agg", C.c_int32), ("block_bf16", C.c_int32),
                ("verbose", C.c_int32), ("coarse_every", C.c_int32), ("limiter", C.c_int32),
                ("mg_levels", C.c_int32), ("mg_sweeps", C.c_int32), ("mg_omega", C.c_double),
                ("block_reuse", C.c_double)]


class DgStepReport(C.Structure):
    _fields_ = [("newton_its", C.c_int32), ("gmres_its", C.c_int32), ("line_search_cuts", C.c_int32),
                ("status", C.c_int32), ("stalled", C.c_int32), ("mg_levels", C.c_int32), ("merit0", C.c_double), ("merit_final", C.c_double),
                ("last_update", C.c_double), ("gmres_last_rel", C.c_double), ("block_builds", C.c_int32),
                ("pad2", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad2"}


DG_BOP_RESIDUAL, DG_BOP_JVP_FULL9, DG_BOP_JVP_CONDENSED7 = 0, 1, 2
BATCH_OPS = {"residual": DG_BOP_RESIDUAL, "jvp": DG_BOP_JVP_FULL9, "jvp_condensed": DG_BOP_JVP_CONDENSED7}


class DgBatchShape(C.Structure):
    _fields_ = [("tile_voxels", C.c_int32), ("persistent", C.c_int32)]

    def as_tuple(self):
        return (self.tile_voxels, self.persistent)


class DgBatchTuning(C.Structure):
    _fields_ = [("shape", DgBatchShape * 3), ("ms", C.c_double * 3), ("ms_default", C.c_double * 3),
                ("candidates", C.c_int32), ("pad", C.c_int32)]


DG_CTRL_NAIVE, DG_CTRL_H211B = 0, 1
DG_WS_OPERATORS, DG_WS_BLOCKS, DG_WS_STEP, DG_WS_NAIVE, DG_WS_H211B, DG_WS_LIMITER = 1, 2, 4, 8, 16, 32
DG_WS_MG = 64
DG_WS_ALL = 127


class DgController(C.Structure):
    _fields_ = [("kind", C.c_int32), ("max_halvings", C.c_int32), ("successes", C.c_int32),
                ("sct", C.c_int32), ("dt", C.c_double), ("dt_max", C.c_double), ("grow", C.c_double),
                ("tol", C.c_double), ("err_prev", C.c_double), ("dt_prev", C.c_double)]


class DgAdvanceReport(C.Structure):
    _fields_ = [("dt", C.c_double), ("err", C.c_double), ("trials", C.c_int32), ("halvings", C.c_int32),
                ("newton_its", C.c_int32), ("gmres_its", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def controller(kind="naive", dt0=0.1, tol=1e-5, dt_max=None):
    """Time controller state (naive or H211b) with the paper's settings."""
    lib = load()
    c = DgController()
    lib.dg_controller_init(C.byref(c), DG_CTRL_H211B if kind == "h211b" else DG_CTRL_NAIVE,
                           float(dt0), float(tol))
    if dt_max is not None:
        c.dt_max = float(dt_max)
    return c


class DgError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed: {_STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load liblsbdg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run python -m paper_2511_05233_amd.build)")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(fn, code):
    if code != 0:
        raise DgError(fn, code, _lib.dg_last_error().decode())


def _ptr(t):
    import torch
    if not t.is_cuda:
        raise ValueError("arrays must be HIP device tensors")
    if not t.is_contiguous():
        raise ValueError("arrays must be contiguous")
    return C.c_void_p(t.data_ptr())


def _check_layout(t, shape, like=None):
    """Shape of an array argument, and dtype and device equal to those of
    `like` (the library reads and writes every array of a call in one
    precision: a mismatched buffer would be over- or under-run)."""
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if like is not None:
        if t.dtype != like.dtype:
            raise ValueError(f"expected dtype {like.dtype}, got {t.dtype}")
        if t.device != like.device:
            raise ValueError(f"expected device {like.device}, got {t.device}")


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _prec(t):
    return _prec_of(t.dtype)


def _prec_of(dtype):
    import torch
    if dtype == torch.float64:
        return DG_F64
    if dtype == torch.float32:
        return DG_F32
    raise ValueError(f"unsupported dtype {dtype}")


def default_params():
    lib = load()
    p = DgParams()
    lib.dg_params_default(C.byref(p))
    return p


def _solver_opts(inner, opts):
    """dg_solver_opts: library defaults, the inner precision, then opts."""
    o = DgSolverOpts()
    load().dg_solver_opts_default(C.byref(o))
    o.inner_prec = DG_F32 if inner == "f32" else DG_F64
    for k, v in opts.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solver option {k!r}")
        setattr(o, k, v)
    return o


def make_params(D0=None, kE=None, f_C=None, j_el=None, eps_struct=None, sigma=None, use_TH=None, T=None):
    """dg_params: the paper's defaults with the given entries replaced."""
    p = default_params()
    if D0 is not None:
        p.D0[:] = [float(x) for x in D0]
    if kE is not None:
        p.kE[:] = [float(x) for x in kE]
    if f_C is not None:
        p.f_C = float(f_C)
    if j_el is not None:
        p.j_el = float(j_el)
    if eps_struct is not None:
        p.eps_struct = float(eps_struct)
    if sigma is not None:
        p.sigma = float(sigma)
    if use_TH is not None:
        p.use_TH = int(bool(use_TH))
    if T is not None:
        p.T = float(T)
    return p


def workspace_bytes(nx, ny, nz, h, order, features, inner="f32", params=None, **opts):
    """dg_workspace_bytes: device bytes a workspace context needs for the
    uses in `features` (DG_WS_* mask) with these solver options."""
    lib = load()
    mesh = DgMesh(int(nx), int(ny), int(nz), int(order), float(h))
    p = params if params is not None else default_params()
    o = _solver_opts(inner, opts)
    n = C.c_size_t()
    _check("dg_workspace_bytes", lib.dg_workspace_bytes(C.byref(mesh), C.byref(p), C.byref(o), int(features),
                                                        C.byref(n)))
    return int(n.value)


def triad(out, a, b, s):
    """dg_triad: out = a + s b on FP64 device arrays of one length (STREAM
    triad, 24 bytes per element), on the current stream."""
    import torch
    lib = load()
    for t in (out, a, b):
        if t.dtype != torch.float64 or t.numel() != out.numel():
            raise ValueError("triad: FP64 arrays of one length")
    _check("dg_triad", lib.dg_triad(_ptr(out), _ptr(a), _ptr(b), float(s), int(out.numel()), _stream()))


class Context:
    """One voxel structure: mesh, phase map and parameters on the device.

    workspace: a device tensor (uint8, contiguous) the context takes all its
    device memory from (dg_setup_ws), sized for `features` and the solver
    options `ws_opts` (inner precision "ws_inner"); kept alive by the
    context."""

    def __init__(self, nx, ny, nz, h, order, phase, D0=None, kE=None, f_C=None, j_el=None,
                 eps_struct=None, sigma=None, use_TH=None, T=None, workspace=None, features=0, ws_inner="f32",
                 ws_opts=None):
        lib = load()
        self.nx, self.ny, self.nz, self.h, self.order = int(nx), int(ny), int(nz), float(h), int(order)
        self.n_elem = self.nx * self.ny * self.nz
        self.n_nodes = (self.order + 1) ** 3
        ph = np.ascontiguousarray(np.asarray(phase, dtype=np.uint8).reshape(-1))
        if ph.size != self.n_elem:
            raise ValueError("phase map size does not match the mesh")
        p = make_params(D0=D0, kE=kE, f_C=f_C, j_el=j_el, eps_struct=eps_struct, sigma=sigma,
                        use_TH=use_TH, T=T)
        self.params = p
        mesh = DgMesh(self.nx, self.ny, self.nz, self.order, self.h)
        handle = C.c_void_p()
        self._ws = workspace
        if workspace is None:
            _check("dg_setup", lib.dg_setup(C.byref(mesh), ph.ctypes.data_as(C.c_void_p),
                                            C.byref(p), C.byref(handle)))
        else:
            import torch
            if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("the workspace is a contiguous uint8 device tensor")
            o = _solver_opts(ws_inner, ws_opts or {})
            _check("dg_setup_ws", lib.dg_setup_ws(C.byref(mesh), ph.ctypes.data_as(C.c_void_p), C.byref(p),
                                                  C.byref(o), int(features), C.c_void_p(workspace.data_ptr()),
                                                  workspace.numel(), _stream(), C.byref(handle)))
        self._h = handle
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        V = C.c_double()
        c0 = (C.c_double * 6)()
        U0 = (C.c_double * 6)()
        j = C.c_double()
        es = C.c_double()
        _check("dg_info", self._lib.dg_info(self._h, C.byref(V), c0, U0, C.byref(j), C.byref(es)))
        return {"V": V.value, "c0": np.array(c0[:]), "U0": np.array(U0[:]),
                "j_el": j.value, "eps_struct": es.value}

    def _shape(self, nf):
        return (nf, self.n_elem, self.n_nodes)

    def _check_arr(self, t, nf, like=None):
        _check_layout(t, self._shape(nf), like)

    def mass(self, u, out=None):
        import torch
        self._check_arr(u, 9)
        if out is None:
            out = torch.empty(self._shape(8), dtype=u.dtype, device=u.device)
        self._check_arr(out, 8, like=u)
        _check("dg_mass", self._lib.dg_mass(self._h, _prec(u), _ptr(u), _ptr(out), _stream()))
        return out

    def residual(self, u, m_old, t_new, dt, out=None):
        import torch
        self._check_arr(u, 9)
        self._check_arr(m_old, 8, like=u)
        if out is None:
            out = torch.empty(self._shape(9), dtype=u.dtype, device=u.device)
        self._check_arr(out, 9, like=u)
        _check("dg_residual", self._lib.dg_residual(self._h, _prec(u), _ptr(u), _ptr(m_old),
                                                    float(t_new), float(dt), _ptr(out), _stream()))
        return out

    def linearize(self, u, t_new, dt):
        """Store the condensation coefficients at u (precision of u)."""
        self._check_arr(u, 9)
        _check("dg_linearize", self._lib.dg_linearize(self._h, _prec(u), _ptr(u), float(t_new), float(dt),
                                                      _stream()))

    def jvp(self, u, v, t_new, dt, out=None, condensed=False, linearized=False):
        """J(u) v: 9 fields, or 7 with the solid fractions condensed out
        (linearized: with the coefficients of the last linearize call)."""
        import torch
        condensed = condensed or linearized
        nf = 7 if condensed else 9
        self._check_arr(u, 9)
        self._check_arr(v, nf, like=u)
        if out is None:
            out = torch.empty(self._shape(nf), dtype=u.dtype, device=u.device)
        self._check_arr(out, nf, like=u)
        mode = DG_JVP_LINEARIZED7 if linearized else (DG_JVP_CONDENSED7 if condensed else DG_JVP_FULL9)
        _check("dg_jvp", self._lib.dg_jvp(self._h, _prec(u), mode, _ptr(u), _ptr(v), float(t_new),
                                          float(dt), _ptr(out), _stream()))
        return out

    def blockjacobi_setup(self, u, t_new, dt, dtype=None):
        """Build and invert the condensed element blocks at u (precision dtype)."""
        self._check_arr(u, 9)
        uu = u if dtype is None or u.dtype == dtype else u.to(dtype)
        _check("dg_blockjacobi_setup", self._lib.dg_blockjacobi_setup(
            self._h, _prec(uu), _ptr(uu), float(t_new), float(dt), _stream()))

    def blockjacobi_apply(self, x, out=None, bf16=False):
        """y = B^-1 x; bf16: from the bfloat16 copy of FP32 inverses."""
        import torch
        self._check_arr(x, 7)
        if out is None:
            out = torch.empty_like(x)
        self._check_arr(out, 7, like=x)
        if bf16:
            if x.dtype != torch.float32:
                raise ValueError("the bfloat16 apply takes FP32 vectors")
            _check("dg_blockjacobi_apply_bf16", self._lib.dg_blockjacobi_apply_bf16(
                self._h, _ptr(x), _ptr(out), _stream()))
            return out
        _check("dg_blockjacobi_apply", self._lib.dg_blockjacobi_apply(
            self._h, _prec(x), _ptr(x), _ptr(out), _stream()))
        return out

    def mg_setup(self, u, t_new, dt, levels, agg=0, sweeps=3, omega=0.7, dtype=None):
        """dg_mg_setup: linearise at u (precision dtype) and build the
        multilevel hierarchy (levels 2..8, level-1 aggregate edge agg)."""
        self._check_arr(u, 9)
        uu = u if dtype is None or u.dtype == dtype else u.to(dtype)
        o = _solver_opts("f32", {"mg_levels": int(levels), "coarse_agg": int(agg), "mg_sweeps": int(sweeps),
                                 "mg_omega": float(omega)})
        _check("dg_mg_setup", self._lib.dg_mg_setup(self._h, _prec(uu), _ptr(uu), float(t_new), float(dt),
                                                    C.byref(o), _stream()))

    def mg_apply(self, r, out=None):
        """dg_mg_apply: out = Z V(Z^T r) for a 7-field vector r."""
        import torch
        self._check_arr(r, 7)
        if out is None:
            out = torch.empty_like(r)
        self._check_arr(out, 7, like=r)
        _check("dg_mg_apply", self._lib.dg_mg_apply(self._h, _prec(r), _ptr(r), _ptr(out), _stream()))
        return out

    def mg_export(self, level, n_aggregates):
        """dg_mg_export: level operator as (7 slots, 7, 7, aggregates) FP64."""
        import torch
        out = torch.empty((7, 7, 7, int(n_aggregates)), dtype=torch.float64, device="cuda")
        _check("dg_mg_export", self._lib.dg_mg_export(self._h, int(level), _ptr(out), out.numel(), _stream()))
        return out

    def blockjacobi_export(self):
        import torch
        prec, nb = C.c_int32(), C.c_int32()
        _check("dg_blockjacobi_info", self._lib.dg_blockjacobi_info(self._h, C.byref(prec), C.byref(nb)))
        dtype = torch.float64 if prec.value == DG_F64 else torch.float32
        out = torch.empty((self.n_elem, nb.value, nb.value), dtype=dtype, device="cuda")
        _check("dg_blockjacobi_export", self._lib.dg_blockjacobi_export(self._h, _ptr(out), _stream()))
        return out

    def _opts(self, inner, opts):
        return _solver_opts(inner, opts)

    def initial_state(self, u=None, t0=0.0, inner="f64", **opts):
        """Equilibrium concentrations plus the steady potential (FP64, 9 fields)."""
        import torch
        if u is None:
            u = torch.empty(self._shape(9), dtype=torch.float64, device="cuda")
        self._check_arr(u, 9)
        if u.dtype != torch.float64:
            raise ValueError("the state is FP64")
        o = self._opts(inner, opts)
        rep = DgStepReport()
        code = self._lib.dg_initial_state(self._h, float(t0), _ptr(u), C.byref(o), C.byref(rep), _stream())
        if code != 0:
            err = DgError("dg_initial_state", code, self._lib.dg_last_error().decode())
            err.report = rep.as_dict()
            raise err
        return u, rep.as_dict()

    def step(self, u, t_n, dt, inner="f32", **opts):
        """One backward-Euler step in place on u (FP64, 9 fields); returns the report."""
        import torch
        self._check_arr(u, 9)
        if u.dtype != torch.float64:
            raise ValueError("the step state is FP64")
        o = self._opts(inner, opts)
        rep = DgStepReport()
        code = self._lib.dg_step(self._h, float(t_n), float(dt), _ptr(u), C.byref(o), C.byref(rep), _stream())
        if code != 0:
            err = DgError("dg_step", code, self._lib.dg_last_error().decode())
            err.report = rep.as_dict()
            raise err
        return rep.as_dict()

    def outputs(self, u, t, noalloc=False):
        """U_cell [V], means (9 unknowns + c_S), sums (S, Li, electrons [mol], current [A]);
        noalloc: through dg_outputs_noalloc (no device allocation)."""
        import torch
        self._check_arr(u, 9)
        if u.dtype != torch.float64:
            raise ValueError("the state is FP64")
        U = C.c_double()
        means = (C.c_double * 10)()
        sums = (C.c_double * 4)()
        fn = "dg_outputs_noalloc" if noalloc else "dg_outputs"
        _check(fn, getattr(self._lib, fn)(self._h, _ptr(u), float(t), C.byref(U), means, sums, _stream()))
        return {"U_cell": U.value, "means": np.array(means[:]), "sums": np.array(sums[:])}

    def limit(self, u, alpha=False):
        """dg_limit: the vertex-based limiter on state u (FP64, 9 fields) in
        place; alpha=True also returns the factors (6, n_elem)."""
        import torch
        self._check_arr(u, 9)
        if u.dtype != torch.float64:
            raise ValueError("the state is FP64")
        a = torch.empty((6, self.n_elem), dtype=torch.float64, device=u.device) if alpha else None
        _check("dg_limit", self._lib.dg_limit(self._h, _ptr(u), _ptr(a) if alpha else None, _stream()))
        return a

    def advance(self, ctrl, t, u, inner="f32", **opts):
        """One accepted controller step from t (u in place); returns (t_new, report)."""
        import torch
        self._check_arr(u, 9)
        if u.dtype != torch.float64:
            raise ValueError("the state is FP64")
        o = self._opts(inner, opts)
        rep = DgAdvanceReport()
        tt = C.c_double(float(t))
        code = self._lib.dg_advance(self._h, C.byref(ctrl), C.byref(tt), _ptr(u), C.byref(o), C.byref(rep),
                                    _stream())
        if code != 0:
            err = DgError("dg_advance", code, self._lib.dg_last_error().decode())
            err.report = rep.as_dict()
            raise err
        return tt.value, rep.as_dict()


_PARAM_KEYS = ("D0", "kE", "f_C", "j_el", "eps_struct", "sigma", "use_TH", "T")


class Batch:
    """Many voxel structures of uneven size behind one set of launches.

    Arrays concatenate the structures voxel by voxel: shape (nf, E, 8) with
    structure s in [offsets[s], offsets[s+1]) of the voxel axis.  Times and
    steps are one value per structure (a scalar is broadcast)."""

    def __init__(self, structures):
        """structures: sequence of dicts with nx, ny, nz, h, phase and
        optionally the parameter keys of Context (order 1)."""
        lib = load()
        n = len(structures)
        if n < 1:
            raise ValueError("a batch needs at least one structure")
        meshes = (DgMesh * n)()
        params = (DgParams * n)()
        ptrs = (C.c_void_p * n)()
        self._phases = []
        for i, st in enumerate(structures):
            nx, ny, nz = int(st["nx"]), int(st["ny"]), int(st["nz"])
            ph = np.ascontiguousarray(np.asarray(st["phase"], dtype=np.uint8).reshape(-1))
            if ph.size != nx * ny * nz:
                raise ValueError(f"structure {i}: phase map size does not match the mesh")
            self._phases.append(ph)
            ptrs[i] = ph.ctypes.data
            meshes[i] = DgMesh(nx, ny, nz, 1, float(st["h"]))
            params[i] = make_params(**{k: st[k] for k in _PARAM_KEYS if k in st})
        handle = C.c_void_p()
        _check("dg_batch_setup", lib.dg_batch_setup(n, meshes, ptrs, params, C.byref(handle)))
        self._h = handle
        self._lib = lib
        self.n = n
        offs = (C.c_int64 * (n + 1))()
        nt = C.c_int64()
        _check("dg_batch_layout", lib.dg_batch_layout(handle, offs, C.byref(nt)))
        self.offsets = [int(x) for x in offs]
        self.n_tiles = int(nt.value)
        self.n_elem = self.offsets[-1]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def part(self, a, s):
        """Structure s's slice of a batch array (a view)."""
        return a[:, self.offsets[s]:self.offsets[s + 1]]

    def _shape(self, nf):
        return (nf, self.n_elem, 8)

    def _check_arr(self, t, nf, like=None):
        _check_layout(t, self._shape(nf), like)

    def _times(self, x):
        a = np.broadcast_to(np.asarray(x, dtype=np.float64), (self.n,))
        return np.ascontiguousarray(a)

    def mass(self, u, out=None):
        import torch
        self._check_arr(u, 9)
        if out is None:
            out = torch.empty(self._shape(8), dtype=u.dtype, device=u.device)
        self._check_arr(out, 8, like=u)
        _check("dg_batch_mass", self._lib.dg_batch_mass(self._h, _prec(u), _ptr(u), _ptr(out), _stream()))
        return out

    def residual(self, u, m_old, t_new, dt, out=None):
        import torch
        self._check_arr(u, 9)
        self._check_arr(m_old, 8, like=u)
        if out is None:
            out = torch.empty(self._shape(9), dtype=u.dtype, device=u.device)
        self._check_arr(out, 9, like=u)
        t, d = self._times(t_new), self._times(dt)
        _check("dg_batch_residual", self._lib.dg_batch_residual(
            self._h, _prec(u), _ptr(u), _ptr(m_old), t.ctypes.data, d.ctypes.data, _ptr(out), _stream()))
        return out

    def linearize(self, u, t_new, dt):
        self._check_arr(u, 9)
        t, d = self._times(t_new), self._times(dt)
        _check("dg_batch_linearize", self._lib.dg_batch_linearize(
            self._h, _prec(u), _ptr(u), t.ctypes.data, d.ctypes.data, _stream()))

    def jvp(self, u, v, t_new, dt, out=None, condensed=False, linearized=False):
        import torch
        condensed = condensed or linearized
        nf = 7 if condensed else 9
        self._check_arr(u, 9)
        self._check_arr(v, nf, like=u)
        if out is None:
            out = torch.empty(self._shape(nf), dtype=u.dtype, device=u.device)
        self._check_arr(out, nf, like=u)
        mode = DG_JVP_LINEARIZED7 if linearized else (DG_JVP_CONDENSED7 if condensed else DG_JVP_FULL9)
        t, d = self._times(t_new), self._times(dt)
        _check("dg_batch_jvp", self._lib.dg_batch_jvp(self._h, _prec(u), mode, _ptr(u), _ptr(v), t.ctypes.data,
                                                      d.ctypes.data, _ptr(out), _stream()))
        return out

    def blockjacobi_setup(self, u, t_new, dt):
        self._check_arr(u, 9)
        t, d = self._times(t_new), self._times(dt)
        _check("dg_batch_blockjacobi_setup", self._lib.dg_batch_blockjacobi_setup(
            self._h, _prec(u), _ptr(u), t.ctypes.data, d.ctypes.data, _stream()))

    def blockjacobi_apply(self, x, out=None):
        import torch
        self._check_arr(x, 7)
        if out is None:
            out = torch.empty_like(x)
        self._check_arr(out, 7, like=x)
        _check("dg_batch_blockjacobi_apply", self._lib.dg_batch_blockjacobi_apply(
            self._h, _prec(x), _ptr(x), _ptr(out), _stream()))
        return out

    def set_shape(self, dtype, op, tile_voxels, persistent=0):
        """Launch shape of one batched operator ("residual", "jvp" or
        "jvp_condensed") in one precision."""
        sh = DgBatchShape(int(tile_voxels), int(persistent))
        _check("dg_batch_set_shape", self._lib.dg_batch_set_shape(self._h, _prec_of(dtype), BATCH_OPS[op],
                                                                  C.byref(sh)))

    def get_shape(self, dtype, op):
        sh = DgBatchShape()
        _check("dg_batch_get_shape", self._lib.dg_batch_get_shape(self._h, _prec_of(dtype), BATCH_OPS[op],
                                                                  C.byref(sh)))
        return sh.as_tuple()

    def autotune(self, u, v, m_old, t_new, dt, reps=5, work=None):
        """Time every launch shape of the residual and both tangents on
        these arrays (v: 9 fields), keep the fastest; returns, per operator,
        (shape, ms, ms of the default shape), and the number of shapes tried."""
        import torch
        self._check_arr(u, 9)
        self._check_arr(v, 9, like=u)
        self._check_arr(m_old, 8, like=u)
        if work is None:
            work = torch.empty(self._shape(9), dtype=u.dtype, device=u.device)
        self._check_arr(work, 9, like=u)
        rep = DgBatchTuning()
        t, d = self._times(t_new), self._times(dt)
        _check("dg_batch_autotune", self._lib.dg_batch_autotune(
            self._h, _prec(u), _ptr(u), _ptr(v), _ptr(m_old), t.ctypes.data, d.ctypes.data, _ptr(work),
            int(reps), C.byref(rep), _stream()))
        out = {op: (rep.shape[i].as_tuple(), rep.ms[i], rep.ms_default[i]) for op, i in BATCH_OPS.items()}
        return out, int(rep.candidates)

    def initial_state(self, t0=0.0, inner="f64", workers=4, **opts):
        """Initial states of every structure (FP64 batch array) and their reports."""
        import torch
        u = torch.empty(self._shape(9), dtype=torch.float64, device="cuda:0")
        o = _solver_opts(inner, opts)
        reps = (DgStepReport * self.n)()
        t = self._times(t0)
        code = self._lib.dg_batch_initial_state(self._h, t.ctypes.data, _ptr(u), C.byref(o), reps, int(workers),
                                                _stream())
        out = [r.as_dict() for r in reps]
        if code != 0:
            err = DgError("dg_batch_initial_state", code, self._lib.dg_last_error().decode())
            err.reports = out
            raise err
        return u, out

    def step(self, u, t_n, dt, inner="f32", workers=4, **opts):
        """One backward-Euler step of every structure in place on u; the reports."""
        import torch
        self._check_arr(u, 9)
        if u.dtype != torch.float64:
            raise ValueError("the step state is FP64")
        o = _solver_opts(inner, opts)
        reps = (DgStepReport * self.n)()
        t, d = self._times(t_n), self._times(dt)
        code = self._lib.dg_batch_step(self._h, t.ctypes.data, d.ctypes.data, _ptr(u), C.byref(o), reps,
                                       int(workers), _stream())
        out = [r.as_dict() for r in reps]
        if code != 0:
            err = DgError("dg_batch_step", code, self._lib.dg_last_error().decode())
            err.reports = out
            raise err
        return out

"""Thin ctypes binding of the C ABI in include/bsw.h.

Every function here marshals arguments and calls the same-named entry point of
libbsw.so; all arithmetic of the method runs in the library's HIP kernels.
Device arrays are torch tensors (memory and streams only).  The library must
be built (paper_2301_11238_amd/build.py); importing fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbsw.so")

BSW_OK, BSW_W_NOT_CONVERGED = 0, 1
BSW_FP64, BSW_FP32 = 0, 1
BSW_IC_SURFACE = 8
BSW_BED_FLAT, BSW_BED_COS, BSW_BED_GAUSS = 0, 1, 2


class BswError(RuntimeError):
    pass


class Params(C.Structure):
    _fields_ = [("g", C.c_double), ("rho", C.c_double), ("alpha", C.c_double), ("eta", C.c_double),
                ("sigma0", C.c_double), ("gamma", C.c_double), ("beta", C.c_double),
                ("reg", C.c_int32), ("bc", C.c_int32), ("dirichlet", C.c_double * 7),
                ("jac_frozen", C.c_int32), ("dirichlet_tag", (C.c_double * 7) * 3)]


class IC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("d", C.c_double), ("x0", C.c_double), ("y0", C.c_double), ("r", C.c_double),
                ("L", C.c_double)]


class Bed(C.Structure):
    _fields_ = [("kind", C.c_int32), ("order", C.c_int32), ("a", C.c_double), ("kx", C.c_double),
                ("ky", C.c_double), ("x0", C.c_double), ("y0", C.c_double), ("d", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("max_newton", C.c_int32), ("gmres_m", C.c_int32), ("gmres_max_iters", C.c_int32),
                ("newton_tol", C.c_double), ("gmres_rtol", C.c_double), ("cfl", C.c_double),
                ("t_end", C.c_double), ("dt", C.c_double), ("max_steps", C.c_int32), ("timing", C.c_int32),
                ("forcing_max", C.c_double), ("cont_steps", C.c_int32), ("cont_gamma0", C.c_double),
                ("precond_lag", C.c_int32), ("res_tol", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("newton_total", C.c_int32), ("gmres_total", C.c_int32),
                ("newton_max", C.c_int32), ("capped", C.c_int32), ("status", C.c_int32),
                ("dt", C.c_double), ("mass0", C.c_double), ("mass_end", C.c_double),
                ("max_mass_drift", C.c_double), ("active_pct", C.c_double), ("t_end", C.c_double),
                ("seconds", C.c_double), ("operator_applies", C.c_double),
                ("jacobian_applies", C.c_double), ("jac_apply_seconds", C.c_double),
                ("jac_apply_launches", C.c_double), ("queue_seconds", C.c_double),
                ("host_issue_seconds", C.c_double), ("host_wait_seconds", C.c_double),
                ("arnoldi_steps", C.c_double)]


class SolveRequest(C.Structure):
    _fields_ = [("n_vert", C.c_int64), ("xy", C.POINTER(C.c_double)), ("n_el", C.c_int64),
                ("el2vert", C.POINTER(C.c_int32)), ("P", C.c_int32), ("precision", C.c_int32),
                ("params", Params), ("ic", IC), ("W0", C.c_void_p), ("opts", SolveOpts), ("bed", Bed),
                ("mixed_orders", C.c_int32), ("m1", C.c_int32), ("m2", C.c_int32), ("m3", C.c_int32),
                ("face_bc", C.POINTER(C.c_int8))]


BSW_REQ_QUEUED, BSW_REQ_RUNNING, BSW_REQ_DONE, BSW_REQ_FAILED, BSW_REQ_CANCELLED = range(5)


# name -> (restype, argtypes); the exported symbols declared in include/bsw.h
_VP, _DP, _I64P = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
SIGNATURES = {
    "bsw_ctx_create": (C.c_int, [C.c_int, _VP, C.POINTER(_VP)]),
    "bsw_ctx_destroy": (C.c_int, [_VP]),
    "bsw_last_error": (C.c_char_p, [_VP]),
    "bsw_mesh_upload": (C.c_int, [_VP, C.c_int, C.c_int64, _DP, C.c_int64, C.POINTER(C.c_int32), C.POINTER(_VP)]),
    "bsw_mesh_destroy": (C.c_int, [_VP]),
    "bsw_mesh_set_boundary": (C.c_int, [_VP, C.POINTER(C.c_int8)]),
    "bsw_disc_create": (C.c_int, [_VP, C.c_int, C.c_int, C.POINTER(_VP)]),
    "bsw_disc_destroy": (C.c_int, [_VP]),
    "bsw_disc_info": (C.c_int, [_VP, _I64P]),
    "bsw_state_len": (C.c_int64, [_VP]),
    "bsw_project_ic": (C.c_int, [_VP, C.POINTER(IC), _VP]),
    "bsw_bed_interpolate": (C.c_int, [_VP, C.POINTER(Bed), _VP]),
    "bsw_disc_set_bed": (C.c_int, [_VP, _VP]),
    "bsw_disc_set_orders": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int]),
    "bsw_step_begin": (C.c_int, [_VP, C.POINTER(Params), C.c_double, _VP, _VP]),
    "bsw_operator_apply": (C.c_int, [_VP, C.POINTER(Params), C.c_double, _VP, _VP, _VP]),
    "bsw_jacobian_linearize": (C.c_int, [_VP, C.POINTER(Params), C.c_double, _VP]),
    "bsw_jacobian_apply": (C.c_int, [_VP, _VP, _VP]),
    "bsw_precond_apply": (C.c_int, [_VP, _VP, _VP]),
    "bsw_jacobian_blocks": (C.c_int, [_VP, _VP]),
    "bsw_stage_update": (C.c_int, [_VP, C.POINTER(Params), _VP, _VP, C.c_double, _DP]),
    "bsw_stage_update_noalloc": (C.c_int, [_VP, C.POINTER(Params), _VP, _VP, C.c_double, _DP]),
    "bsw_diagnostics": (C.c_int, [_VP, C.POINTER(Params), _VP, _DP]),
    "bsw_norm2": (C.c_int, [_VP, _VP, _DP]),
    "bsw_cfl_dt": (C.c_int, [_VP, C.POINTER(Params), _VP, C.c_double, _DP]),
    "bsw_solve": (C.c_int, [_VP, C.POINTER(Params), C.POINTER(SolveOpts), _VP, C.POINTER(SolveStats)]),
    "bsw_request_footprint": (C.c_int64, [C.POINTER(SolveRequest)]),
    "bsw_server_create": (C.c_int, [_VP, C.c_size_t, C.c_int, C.POINTER(_VP)]),
    "bsw_server_destroy": (C.c_int, [_VP]),
    "bsw_solve_submit": (C.c_int, [_VP, C.POINTER(SolveRequest), C.POINTER(C.c_uint64)]),
    "bsw_solve_poll": (C.c_int, [_VP, C.c_uint64, C.POINTER(C.c_int)]),
    "bsw_solve_wait": (C.c_int, [_VP, C.c_uint64, C.c_double, C.POINTER(C.c_int)]),
    "bsw_solve_fetch": (C.c_int, [_VP, C.c_uint64, _VP, C.POINTER(SolveStats)]),
    "bsw_solve_cancel": (C.c_int, [_VP, C.c_uint64]),
    "bsw_server_info": (C.c_int, [_VP, _DP]),
    "bsw_tile_policy": (C.c_int, [C.c_int, C.POINTER(C.c_int)]),
    "bsw_tile_table": (C.c_int, [_DP, C.c_int, C.POINTER(C.c_int)]),
}

_lib = None


def lib():
    """Load libbsw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise BswError(f"{LIB_PATH} is missing: build it with paper_2301_11238_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def check_tensor(t, device: int, dtype, min_numel: int, name: str = "tensor"):
    """Refuses, before any library call, a device argument the kernels would
    read or write out of bounds: it must be a contiguous CUDA tensor on the
    context's device, of the discretisation's dtype, with at least min_numel
    elements.  Returns its pointer."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name}: must be on cuda:{device}, is on {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, the discretisation needs {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() < min_numel:
        raise ValueError(f"{name}: {t.numel()} elements, at least {min_numel} needed")
    return _ptr(t)


def make_params(p, bc: int = 1, dirichlet=None, dirichlet_tags=None) -> Params:
    q = Params()
    for k in ("g", "rho", "alpha", "eta", "sigma0", "gamma", "beta"):
        setattr(q, k, float(getattr(p, k)))
    q.reg = int(p.reg)
    q.bc = int(bc)
    q.jac_frozen = int(getattr(p, "jac_frozen", 0))
    if dirichlet is not None:
        for i, v in enumerate(dirichlet):
            q.dirichlet[i] = float(v)
    for t, st in enumerate(dirichlet_tags or []):
        for i, v in enumerate(st):
            q.dirichlet_tag[t][i] = float(v)
    return q


def make_ic(ic) -> IC:
    c = IC()
    c.kind = int(ic.kind)
    for k in ("a", "b", "c", "d", "x0", "y0", "r", "L"):
        setattr(c, k, float(getattr(ic, k)))
    return c


def make_bed(bed) -> Bed:
    """bed: workloads.Bed (or anything with the same attributes)."""
    b = Bed()
    if bed is None:
        return b
    b.kind = int(bed.kind)
    b.order = int(bed.order)
    for k in ("a", "kx", "ky", "x0", "y0", "d"):
        setattr(b, k, float(getattr(bed, k)))
    return b


@dataclass
class Options:
    max_newton: int = 10
    gmres_m: int = 30
    gmres_max_iters: int = 1200
    newton_tol: float = 1e-10
    gmres_rtol: float = 1e-10
    cfl: float = 0.2
    t_end: float = 1.0
    dt: float = 0.0
    max_steps: int = -1
    timing: int = 0
    forcing_max: float = 0.0
    cont_steps: int = 0
    cont_gamma0: float = 0.0
    precond_lag: int = 0
    res_tol: float = 0.0

    def c(self) -> SolveOpts:
        o = SolveOpts()
        for k, _ in SolveOpts._fields_:
            setattr(o, k, getattr(self, k))
        return o


class Context:
    """bsw_ctx on one device, bound to a HIP stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = C.c_void_p()
        self._check(lib().bsw_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)), None)
        self.h = h

    def _check(self, rc, h=None):
        if rc < 0:
            msg = lib().bsw_last_error(h if h is not None else getattr(self, "h", None))
            raise BswError(f"bsw error {rc}: {msg.decode() if msg else ''}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().bsw_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    def __init__(self, ctx: Context, dim: int, xy, el2vert):
        import numpy as np
        self.ctx = ctx
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        e2v = np.ascontiguousarray(el2vert, dtype=np.int32)
        h = C.c_void_p()
        ctx._check(lib().bsw_mesh_upload(ctx.h, dim, xy.shape[0], xy.ctypes.data_as(_DP), e2v.shape[0],
                                         e2v.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(h)), ctx.h)
        self.h = h
        self.dim = dim
        self.n_el = e2v.shape[0]

    def set_boundary(self, face_bc=None):
        """Per-face boundary codes [n_el, faces] (kind | tag << 2), or None."""
        import numpy as np
        if face_bc is None:
            rc = lib().bsw_mesh_set_boundary(self.h, None)
        else:
            c = np.ascontiguousarray(face_bc, dtype=np.int8).reshape(-1)
            assert c.size == self.n_el * (self.dim + 1)
            rc = lib().bsw_mesh_set_boundary(self.h, c.ctypes.data_as(C.POINTER(C.c_int8)))
        self.ctx._check(rc, self.ctx.h)

    def close(self):
        if getattr(self, "h", None):
            lib().bsw_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Disc:
    """bsw_disc: one (mesh, order, precision); methods mirror the C ABI."""

    def __init__(self, mesh: Mesh, P: int, precision: int = BSW_FP64):
        import torch
        self.mesh, self.ctx = mesh, mesh.ctx
        h = C.c_void_p()
        self.ctx._check(lib().bsw_disc_create(mesh.h, P, precision, C.byref(h)), self.ctx.h)
        self.h = h
        info = (C.c_int64 * 8)()
        lib().bsw_disc_info(h, info)
        self.dim, self.P, self.np, self.nq, self.nfq, self.nfc, self.nf, self.n_el = [int(v) for v in info]
        self.precision = precision
        self.dtype = torch.float64 if precision == BSW_FP64 else torch.float32
        self.shape = (self.nf, self.np, self.n_el)

    def close(self):
        if getattr(self, "h", None):
            lib().bsw_disc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ck(self, rc):
        return self.ctx._check(rc, self.ctx.h)

    def _state(self, t, name="W"):
        """Pointer of a full state-sized device argument (n_f N_p n_el reals)."""
        return check_tensor(t, self.ctx.device, self.dtype, self.nf * self.np * self.n_el, name)

    def _rows(self, t, nfields, name):
        """Pointer of a device argument of nfields fields ([nfields][N_p][n_el])."""
        return check_tensor(t, self.ctx.device, self.dtype, nfields * self.np * self.n_el, name)

    def empty(self, nfields=None):
        import torch
        nf = self.nf if nfields is None else nfields
        return torch.empty((nf, self.np, self.n_el), dtype=self.dtype, device=self.ctx.torch_device)

    def zeros(self):
        import torch
        return torch.zeros(self.shape, dtype=self.dtype, device=self.ctx.torch_device)

    def state_len(self) -> int:
        return int(lib().bsw_state_len(self.h))

    def project_ic(self, ic, W=None):
        W = self.empty() if W is None else W
        self._ck(lib().bsw_project_ic(self.h, C.byref(make_ic(ic)), self._state(W)))
        return W

    def bed_interpolate(self, bed, H=None):
        """Order-m0 interpolant of an analytic bed, [N_p, n_el] on the device."""
        H = self.empty(1) if H is None else H
        self._ck(lib().bsw_bed_interpolate(self.h, C.byref(make_bed(bed)), self._rows(H, 1, "H")))
        return H[0] if H.dim() == 3 else H

    def set_orders(self, m1: int, m2: int, m3: int):
        """Orders of h, u and E (each 0..P; P is the storage order)."""
        self._ck(lib().bsw_disc_set_orders(self.h, int(m1), int(m2), int(m3)))

    def set_bed(self, H):
        """Bed coefficients [N_p, n_el] (device tensor kept by reference), or None."""
        self._bed = H
        self._ck(lib().bsw_disc_set_bed(self.h, self._rows(H, 1, "H") if H is not None else None))

    def step_begin(self, params: Params, dt: float, W_old, b_old=None):
        b_old = self.empty(1 + self.dim) if b_old is None else b_old
        self._ck(lib().bsw_step_begin(self.h, C.byref(params), float(dt), self._state(W_old, "W_old"),
                                    self._rows(b_old, 1 + self.dim, "b_old")))
        return b_old

    def operator_apply(self, params: Params, dt: float, W, b_old, R=None):
        R = self.empty() if R is None else R
        self._ck(lib().bsw_operator_apply(self.h, C.byref(params), float(dt), self._state(W),
                                         self._rows(b_old, 1 + self.dim, "b_old"), self._state(R, "R")))
        return R

    def jacobian_linearize(self, params: Params, dt: float, W):
        self._lin_W = W  # the library keeps a reference to W's memory
        self._ck(lib().bsw_jacobian_linearize(self.h, C.byref(params), float(dt), self._state(W)))

    def jacobian_apply(self, x, y=None):
        y = self.empty() if y is None else y
        self._ck(lib().bsw_jacobian_apply(self.h, self._state(x, "x"), self._state(y, "y")))
        return y

    def precond_apply(self, x, y=None):
        y = self.empty() if y is None else y
        self._ck(lib().bsw_precond_apply(self.h, self._state(x, "x"), self._state(y, "y")))
        return y

    def jacobian_blocks(self):
        import torch
        bs = self.nf * self.np
        out = torch.empty((self.n_el, bs, bs), dtype=self.dtype, device=self.ctx.torch_device)
        self._ck(lib().bsw_jacobian_blocks(self.h, check_tensor(out, self.ctx.device, self.dtype, self.n_el * bs * bs, "blocks")))
        return out

    def stage_update(self, params, W, dW, alpha: float = 1.0):
        out = (C.c_double * 4)()
        self._ck(lib().bsw_stage_update(self.h, C.byref(params) if params is not None else None, self._state(W),
                                        self._state(dW, "dW"), float(alpha), out))
        return list(out)

    def stage_update_noalloc(self, params, W, dW, alpha: float = 1.0):
        """bsw_stage_update_noalloc: the same update and norms, with the
        library's fixed scratch array instead of allocated partials."""
        out = (C.c_double * 4)()
        self._ck(lib().bsw_stage_update_noalloc(self.h, C.byref(params) if params is not None else None,
                                                self._state(W), self._state(dW, "dW"), float(alpha), out))
        return list(out)

    def diagnostics(self, params, W):
        out = (C.c_double * 4)()
        self._ck(lib().bsw_diagnostics(self.h, C.byref(params), self._state(W), out))
        return dict(mass=out[0], active_pct=out[1], lambda_max=out[2], h_min=out[3])

    def norm2(self, x) -> float:
        out = C.c_double(0.0)
        self._ck(lib().bsw_norm2(self.h, self._state(x, "x"), C.byref(out)))
        return out.value

    def cfl_dt(self, params: Params, W, cfl: float) -> float:
        out = C.c_double(0.0)
        self._ck(lib().bsw_cfl_dt(self.h, C.byref(params), self._state(W), float(cfl), C.byref(out)))
        return out.value

    def solve(self, params: Params, opts: Options, W):
        st = SolveStats()
        rc = lib().bsw_solve(self.h, C.byref(params), C.byref(opts.c()), self._state(W), C.byref(st))
        self._ck(rc)
        return {k: getattr(st, k) for k, _ in SolveStats._fields_}


class _ReqArrays:
    """Keeps the host arrays of a request alive until it is submitted."""

    def __init__(self, xy, el2vert, P, precision, params, ic, opts, W0=None, bed=None, orders=None, face_bc=None):
        import numpy as np
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        self.e2v = np.ascontiguousarray(el2vert, dtype=np.int32)
        self.W0 = None
        if W0 is not None:
            self.W0 = np.ascontiguousarray(W0, dtype=np.float64 if precision == BSW_FP64 else np.float32)
        r = SolveRequest()
        r.n_vert = self.xy.shape[0]
        r.xy = self.xy.ctypes.data_as(_DP)
        r.n_el = self.e2v.shape[0]
        r.el2vert = self.e2v.ctypes.data_as(C.POINTER(C.c_int32))
        r.P = int(P)
        r.precision = int(precision)
        r.params = params
        r.ic = make_ic(ic) if ic is not None else IC()
        r.W0 = C.c_void_p(self.W0.ctypes.data) if self.W0 is not None else None
        r.opts = opts.c()
        r.bed = make_bed(bed)
        self.fbc = None
        if face_bc is not None:
            self.fbc = np.ascontiguousarray(face_bc, dtype=np.int8).reshape(-1)
            r.face_bc = self.fbc.ctypes.data_as(C.POINTER(C.c_int8))
        if orders is not None:
            r.mixed_orders = 1
            r.m1, r.m2, r.m3 = (int(m) for m in orders)
        self.req = r


def tile_policy(policy: int) -> int:
    """-1: autotune the element-pass variant; 0/1/2: force one (triangles:
    occupancy target 1/2/3 waves per SIMD; 1-D: 128/256/512 lanes).
    Returns the previous policy."""
    prev = C.c_int(0)
    if lib().bsw_tile_policy(int(policy), C.byref(prev)) != BSW_OK:
        raise BswError("tile policy must be -1, 0, 1 or 2")
    return prev.value


def tile_table() -> list:
    """The autotuner's entries: one dict per (dim, P, precision, pass, size class)."""
    import numpy as np
    n = C.c_int(0)
    lib().bsw_tile_table(None, 0, C.byref(n))
    rows = np.zeros((max(n.value, 1), 10))
    lib().bsw_tile_table(rows.ctypes.data_as(_DP), n.value, C.byref(n))
    out = []
    for r in rows[: n.value]:
        out.append(dict(dim=int(r[0]), P=int(r[1]), bytes=int(r[2]), mode=int(r[3]), size_class=int(r[4]),
                        variant=int(r[5]), best_us={0: r[6], 1: r[7], 2: r[8]}, timed=int(r[9])))
    return out


def request_footprint(n_el: int, P: int, precision: int, gmres_m: int = 30) -> int:
    """Device bytes a served solve of this size occupies while resident."""
    r = SolveRequest()
    r.n_el, r.P, r.precision = int(n_el), int(P), int(precision)
    r.opts.gmres_m = int(gmres_m)
    return int(lib().bsw_request_footprint(C.byref(r)))


class Server:
    """bsw_server: a worker thread that batches resident solves (continuous
    batching at time-step granularity) under a device-memory budget."""

    def __init__(self, ctx: Context, budget_bytes: int, max_slots: int = 64):
        self.ctx = ctx
        h = C.c_void_p()
        ctx._check(lib().bsw_server_create(ctx.h, int(budget_bytes), int(max_slots), C.byref(h)), ctx.h)
        self.h = h
        self._shape = {}

    def close(self):
        if getattr(self, "h", None):
            lib().bsw_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, xy, el2vert, P: int, precision: int, params: Params, ic=None, opts: Options = None,
               W0=None, bed=None, orders=None, face_bc=None) -> int:
        opts = opts or Options()
        a = _ReqArrays(xy, el2vert, P, precision, params, ic, opts, W0, bed, orders, face_bc)
        t = C.c_uint64(0)
        self.ctx._check(lib().bsw_solve_submit(self.h, C.byref(a.req), C.byref(t)), self.ctx.h)
        n_p = (P + 1) * (P + 2) // 2
        self._shape[t.value] = ((7, n_p, a.req.n_el), precision)
        return t.value

    def poll(self, ticket: int) -> int:
        st = C.c_int(0)
        self.ctx._check(lib().bsw_solve_poll(self.h, C.c_uint64(ticket), C.byref(st)), self.ctx.h)
        return st.value

    def wait(self, ticket: int, timeout: float = 600.0) -> int:
        st = C.c_int(0)
        self.ctx._check(lib().bsw_solve_wait(self.h, C.c_uint64(ticket), float(timeout), C.byref(st)),
                        self.ctx.h)
        return st.value

    def fetch(self, ticket: int):
        """(final state as a numpy array [n_f, n_p, n_el], statistics dict)."""
        import numpy as np
        shape, prec = self._shape.pop(ticket)
        W = np.empty(shape, dtype=np.float64 if prec == BSW_FP64 else np.float32)
        st = SolveStats()
        rc = lib().bsw_solve_fetch(self.h, C.c_uint64(ticket), C.c_void_p(W.ctypes.data), C.byref(st))
        self.ctx._check(rc, self.ctx.h)
        return W, {k: getattr(st, k) for k, _ in SolveStats._fields_}

    def cancel(self, ticket: int):
        self.ctx._check(lib().bsw_solve_cancel(self.h, C.c_uint64(ticket)), self.ctx.h)

    def info(self) -> dict:
        out = (C.c_double * 8)()
        lib().bsw_server_info(self.h, out)
        keys = ("queued", "resident", "bytes_in_use", "budget", "steps", "launches", "completed", "peak_resident")
        return dict(zip(keys, [float(v) for v in out]))


"""Python front end of the plain FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never does.

The C source (bsw_oracle.c) is compiled with gcc into liboracle.so next to it.
Arrays cross this boundary in the shared state layout [n_f, N_p, n_el]; the C
side works per element ([n_el, n_f, N_p]) and this wrapper transposes.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAXNF = 7


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, -O2, OpenMP over elements)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrParams(C.Structure):
    _fields_ = [("g", C.c_double), ("rho", C.c_double), ("alpha", C.c_double),
                ("eta", C.c_double), ("sigma0", C.c_double), ("gamma", C.c_double),
                ("beta", C.c_double), ("reg", C.c_int32), ("bc", C.c_int32),
                ("dir", C.c_double * MAXNF), ("jac_frozen", C.c_int32),
                ("dir_tag", (C.c_double * MAXNF) * 3)]


class OrIC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("d", C.c_double), ("x0", C.c_double), ("y0", C.c_double), ("r", C.c_double),
                ("L", C.c_double)]


class OrBed(C.Structure):
    _fields_ = [("kind", C.c_int32), ("order", C.c_int32), ("a", C.c_double), ("kx", C.c_double),
                ("ky", C.c_double), ("x0", C.c_double), ("y0", C.c_double), ("d", C.c_double)]


class OrSolveOpts(C.Structure):
    _fields_ = [("max_newton", C.c_int32), ("gmres_m", C.c_int32),
                ("gmres_max_restarts", C.c_int32), ("newton_tol", C.c_double),
                ("gmres_rtol", C.c_double), ("cfl", C.c_double), ("t_end", C.c_double),
                ("dt_override", C.c_double), ("max_steps", C.c_int32), ("res_tol", C.c_double)]


class OrSolveStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("newton_total", C.c_int32), ("gmres_total", C.c_int32),
                ("newton_max", C.c_int32), ("capped", C.c_int32), ("dt", C.c_double),
                ("mass0", C.c_double), ("mass_end", C.c_double), ("max_mass_drift", C.c_double),
                ("active_pct", C.c_double), ("t_end", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_int, ip, C.POINTER(C.c_int)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
        L.or_ref_tables.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp]
        L.or_basis.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp]
        L.or_mesh_data.argtypes = [C.c_void_p, ip, ip, dp, dp, dp, dp, dp, dp]
        for name in ("or_step_begin",):
            getattr(L, name).argtypes = [C.c_void_p, C.POINTER(OrParams), C.c_double, dp, dp]
        L.or_residual.argtypes = [C.c_void_p, C.POINTER(OrParams), C.c_double, dp, dp, dp]
        L.or_jac_apply.argtypes = [C.c_void_p, C.POINTER(OrParams), C.c_double, dp, dp, dp]
        L.or_jac_blocks.argtypes = [C.c_void_p, C.POINTER(OrParams), C.c_double, dp, dp]
        L.or_jac_offdiag.argtypes = [C.c_void_p, C.POINTER(OrParams), C.c_double, dp, dp]
        L.or_newton_step.argtypes = [C.c_void_p, C.POINTER(OrParams), C.c_double, dp, dp,
                                     C.POINTER(OrSolveOpts), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.or_project_ic.argtypes = [C.c_void_p, C.POINTER(OrIC), dp]
        L.or_diagnostics.argtypes = [C.c_void_p, C.POINTER(OrParams), dp, dp]
        L.or_bed_interpolate.argtypes = [C.c_void_p, C.POINTER(OrBed), dp]
        L.or_set_bed.argtypes = [C.c_void_p, dp]
        L.or_set_orders.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.or_set_boundary.argtypes = [C.c_void_p, C.POINTER(C.c_int8)]
        L.or_eval_points.argtypes = [C.c_void_p, dp, dp]
        L.or_cfl_dt.restype = C.c_double
        L.or_cfl_dt.argtypes = [C.c_void_p, C.POINTER(OrParams), dp, C.c_double]
        L.or_solve.argtypes = [C.c_void_p, C.POINTER(OrParams), C.POINTER(OrSolveOpts), dp,
                               C.POINTER(OrSolveStats)]
        L.or_sigmaB_1d.restype = C.c_double
        L.or_sigmaB_1d.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.or_point_sigma.argtypes = [C.POINTER(OrParams), C.c_int, dp, dp, dp]
        L.or_point_hll.argtypes = [C.POINTER(OrParams), C.c_int, dp, dp, dp, dp, dp, dp, dp]
        L.or_point_psi.argtypes = [C.POINTER(OrParams), C.c_double, dp]
        L.or_point_wall.argtypes = [C.POINTER(OrParams), C.c_int, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def make_params(params, bc: int = 1, dirichlet=None, dirichlet_tags=None) -> OrParams:
    """params: workloads.Params (or anything with the same attributes);
    dirichlet_tags: up to three exterior states of Dirichlet tags 1..3."""
    p = OrParams()
    for k in ("g", "rho", "alpha", "eta", "sigma0", "gamma", "beta"):
        setattr(p, k, float(getattr(params, k)))
    p.reg = int(params.reg)
    p.bc = int(bc)
    p.jac_frozen = int(getattr(params, "jac_frozen", 0))
    if dirichlet is not None:
        for i, v in enumerate(dirichlet):
            p.dir[i] = float(v)
    for t, st in enumerate(dirichlet_tags or []):
        for i, v in enumerate(st):
            p.dir_tag[t][i] = float(v)
    return p


def make_ic(ic) -> OrIC:
    c = OrIC()
    c.kind = int(ic.kind)
    for k in ("a", "b", "c", "d", "x0", "y0", "r", "L"):
        setattr(c, k, float(getattr(ic, k)))
    return c


def basis(dim: int, P: int, pts) -> tuple:
    """Basis values [n_pts, N_p] and reference gradients [n_pts, N_p, 2] at
    reference points (1-D: a vector of xi; 2-D: [n_pts, 2])."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n = pts.shape[0]
    np_ = P + 1 if dim == 1 else (P + 1) * (P + 2) // 2
    phi = np.zeros((n, np_)); dphi = np.zeros((n, np_, 2))
    lib().or_basis(dim, P, n, _dp(pts), _dp(phi), _dp(dphi))
    return phi, dphi


def make_bed(bed) -> OrBed:
    b = OrBed()
    b.kind = int(bed.kind)
    b.order = int(bed.order)
    for k in ("a", "kx", "ky", "x0", "y0", "d"):
        setattr(b, k, float(getattr(bed, k)))
    return b


def to_elem(W: np.ndarray) -> np.ndarray:
    """[n_f, N_p, n_el] -> contiguous [n_el, n_f, N_p]."""
    return np.ascontiguousarray(np.transpose(W, (2, 0, 1)), dtype=np.float64)


def from_elem(We: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.transpose(We, (1, 2, 0)))


@dataclass
class SolveOptions:
    max_newton: int = 10
    gmres_m: int = 30
    gmres_max_restarts: int = 40
    newton_tol: float = 1e-10
    gmres_rtol: float = 1e-12
    cfl: float = 0.2
    t_end: float = 1.0
    dt_override: float = 0.0
    max_steps: int = -1
    # > 0: Newton also stops when ||R||_2 <= res_tol ||b_old||_2 (initial or
    # accepted residual); the scope table's second stopping rule
    res_tol: float = 1e-13
    # continuation on gamma (Sec. 6.3): n >= 2 Newton solves per time step at
    # gamma_i = gamma0 + (i - 1) (gamma - gamma0) / (n - 1), each from the last
    cont_steps: int = 0
    cont_gamma0: float = 0.0


class Oracle:
    """One discretisation (reference element + mesh) on the CPU."""

    def __init__(self, dim: int, P: int, xy: np.ndarray, el2vert: np.ndarray):
        L = lib()
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        self.e2v = np.ascontiguousarray(el2vert, dtype=np.int32)
        err = C.c_int(0)
        h = L.or_create(dim, P, self.xy.shape[0], _dp(self.xy), self.e2v.shape[0],
                        _ip(self.e2v), C.byref(err))
        if not h:
            raise ValueError(f"oracle setup failed ({err.value})")
        self.h = C.c_void_p(h)
        sz = (C.c_int * 8)()
        L.or_sizes(self.h, sz)
        self.dim, self.P, self.np, self.nq, self.nfq, self.nfc, self.nf, self.n_el = list(sz)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().or_destroy(self.h)
        except Exception:
            pass

    @property
    def shape(self):
        return (self.nf, self.np, self.n_el)

    # --------------------------------------------------------------- tables
    def ref_tables(self):
        nq, np_, nfc, nfq = self.nq, self.np, self.nfc, self.nfq
        qx = np.zeros((nq, 2)); qw = np.zeros(nq); phi = np.zeros((nq, np_))
        dphi = np.zeros((nq, np_, 2)); fphi = np.zeros((nfc, nfq, np_)); fw = np.zeros(nfq)
        lib().or_ref_tables(self.h, _dp(qx), _dp(qw), _dp(phi), _dp(dphi), _dp(fphi), _dp(fw))
        return dict(qx=qx, qw=qw, phi=phi, dphi=dphi, fphi=fphi, fw=fw)

    def mesh_data(self):
        n, nfc = self.n_el, self.nfc
        nbr = np.zeros((n, nfc), np.int32); nbrf = np.zeros((n, nfc), np.int32)
        detJ = np.zeros(n); dxi = np.zeros((n, 2, 2)); normal = np.zeros((n, nfc, 2))
        flen = np.zeros((n, nfc)); xq = np.zeros((n, self.nq, 2)); mh = np.zeros(2)
        lib().or_mesh_data(self.h, _ip(nbr), _ip(nbrf), _dp(detJ), _dp(dxi), _dp(normal),
                           _dp(flen), _dp(xq), _dp(mh))
        return dict(nbr=nbr, nbr_face=nbrf, detJ=detJ, dxi=dxi, normal=normal, flen=flen,
                    xq=xq, measure=mh[0], hmin=mh[1])

    # ------------------------------------------------------------------ bed
    def bed_interpolate(self, bed) -> np.ndarray:
        """Continuous order-m0 interpolant of an analytic bed (workloads.Bed),
        as modal coefficients [N_p, n_el] (the layout of one state field)."""
        H = np.zeros((self.n_el, self.np))
        if lib().or_bed_interpolate(self.h, C.byref(make_bed(bed)), _dp(H)) != 0:
            raise ValueError("bed order must be 1 <= m0 <= P")
        return np.ascontiguousarray(H.T)

    def set_bed(self, H) -> None:
        """Bed coefficients [N_p, n_el] used by the source term; None = flat."""
        if H is None:
            lib().or_set_bed(self.h, None)
            return
        He = np.ascontiguousarray(np.asarray(H, dtype=np.float64).T)
        assert He.shape == (self.n_el, self.np)
        lib().or_set_bed(self.h, _dp(He))

    def set_boundary(self, codes=None, dirichlet_tags=None) -> None:
        """Boundary codes per local face ([n_el, n_faces] int8, kind | tag << 2:
        kind 1 wall, 2 Neumann, 3 Dirichlet, 0 the bc argument of each call;
        tag 1..3 selects dirichlet_tags[tag - 1], tag 0 the dirichlet argument).
        None resets every face to the bc argument."""
        if codes is None:
            rc = lib().or_set_boundary(self.h, None)
        else:
            c = np.ascontiguousarray(codes, dtype=np.int8).reshape(self.n_el * self.nfc)
            rc = lib().or_set_boundary(self.h, c.ctypes.data_as(C.POINTER(C.c_int8)))
        if rc != 0:
            raise ValueError("boundary codes must be in 0..15")
        self._dir_tags = [list(t) for t in (dirichlet_tags or [])]

    def _mp(self, params, bc=1, dirichlet=None):
        return make_params(params, bc, dirichlet, getattr(self, "_dir_tags", None))

    def set_orders(self, m1: int, m2: int, m3: int) -> None:
        """Orders of h, u and E (each 0..P; P is the storage order)."""
        if lib().or_set_orders(self.h, int(m1), int(m2), int(m3)) != 0:
            raise ValueError("orders must be in 0..P")

    # ------------------------------------------------------------- operator
    def step_begin(self, params, Wold, dt, bc=1):
        p = self._mp(params, bc)
        We = to_elem(Wold); b = np.zeros_like(We)
        lib().or_step_begin(self.h, C.byref(p), float(dt), _dp(We), _dp(b))
        return from_elem(b)

    def residual(self, params, W, bold, dt, bc=1, dirichlet=None):
        p = self._mp(params, bc, dirichlet)
        We = to_elem(W); be = to_elem(bold); R = np.zeros_like(We)
        lib().or_residual(self.h, C.byref(p), float(dt), _dp(We), _dp(be), _dp(R))
        return from_elem(R)

    def jac_apply(self, params, W, x, dt, bc=1, dirichlet=None):
        p = self._mp(params, bc, dirichlet)
        We = to_elem(W); xe = to_elem(x); y = np.zeros_like(We)
        lib().or_jac_apply(self.h, C.byref(p), float(dt), _dp(We), _dp(xe), _dp(y))
        return from_elem(y)

    def jac_blocks(self, params, W, dt, bc=1, dirichlet=None):
        """Diagonal blocks, [n_el, bs, bs] with row/col index f*N_p + i."""
        p = self._mp(params, bc, dirichlet)
        We = to_elem(W); bs = self.nf * self.np
        B = np.zeros((self.n_el, bs, bs))
        lib().or_jac_blocks(self.h, C.byref(p), float(dt), _dp(We), _dp(B))
        return B

    def jac_offdiag(self, params, W, dt, bc=1, dirichlet=None):
        """Face-coupling blocks dR_e/dW_nbr, [n_el, n_faces, bs, bs]."""
        p = self._mp(params, bc, dirichlet)
        We = to_elem(W); bs = self.nf * self.np
        B = np.zeros((self.n_el, self.nfc, bs, bs))
        lib().or_jac_offdiag(self.h, C.byref(p), float(dt), _dp(We), _dp(B))
        return B

    # ----------------------------------------------- exact (sparse direct) solver
    def _jacobian_sparse(self, p, We, dt):
        import scipy.sparse as sp
        L = lib(); bs = self.nf * self.np; n = self.n_el
        Bd = np.zeros((n, bs, bs)); Bo = np.zeros((n, self.nfc, bs, bs))
        L.or_jac_blocks(self.h, C.byref(p), float(dt), _dp(We), _dp(Bd))
        L.or_jac_offdiag(self.h, C.byref(p), float(dt), _dp(We), _dp(Bo))
        if not hasattr(self, "_nbr"):
            self._nbr = self.mesh_data()["nbr"]
        nbr = self._nbr
        rows, cols, blocks = [np.arange(n)], [np.arange(n)], [Bd]
        for f in range(self.nfc):
            m = nbr[:, f] >= 0
            rows.append(np.nonzero(m)[0]); cols.append(nbr[m, f]); blocks.append(Bo[m, f])
        r = np.concatenate(rows); c = np.concatenate(cols); b = np.concatenate(blocks)
        ii = (r[:, None, None] * bs + np.arange(bs)[None, :, None]) + 0 * np.arange(bs)[None, None, :]
        jj = (c[:, None, None] * bs + np.arange(bs)[None, None, :]) + 0 * np.arange(bs)[None, :, None]
        return sp.csc_matrix((b.ravel(), (ii.ravel(), jj.ravel())), shape=(n * bs, n * bs))

    def _newton_direct(self, p, We, be, dt, o):
        """Newton for one backward-Euler step with exact linear solves (sparse
        LU); same iteration, line search and stopping rules as the C solver
        (the update test, and the residual test when res_tol > 0)."""
        import scipy.sparse.linalg as spla
        L = lib()
        R = np.zeros_like(We)
        L.or_residual(self.h, C.byref(p), float(dt), _dp(We), _dp(be), _dp(R))
        rn = float(np.linalg.norm(R))
        rstop = o.res_tol * float(np.linalg.norm(be)) if o.res_tol > 0 else -1.0
        if np.isfinite(rn) and rn <= rstop:
            return 0, 1
        conv, it = 0, 0
        for it in range(1, o.max_newton + 1):
            J = self._jacobian_sparse(p, We, dt)
            dW = spla.splu(J).solve(-R.ravel()).reshape(We.shape)
            dmax = float(np.abs(dW).max())
            if np.isfinite(dmax) and dmax <= o.newton_tol * (1.0 + float(np.abs(We).max())):
                We += dW
                conv = 1
                break
            a = 1.0
            while True:
                Wt = We + a * dW
                Rt = np.zeros_like(We)
                L.or_residual(self.h, C.byref(p), float(dt), _dp(Wt), _dp(be), _dp(Rt))
                rnt = float(np.linalg.norm(Rt))
                if (np.isfinite(rnt) and rnt <= (1.0 - 1e-4 * a) * rn) or a <= 1.0 / 64.0:
                    break
                a *= 0.5
            We[...] = Wt
            R, rn = Rt, rnt
            if not np.isfinite(rnt) or not np.isfinite(We).all():
                conv = -1
                break
            if rn <= rstop:
                conv = 1
                break
        return it, conv

    def project_ic(self, ic):
        c = make_ic(ic)
        We = np.zeros((self.n_el, self.nf, self.np))
        lib().or_project_ic(self.h, C.byref(c), _dp(We))
        return from_elem(We)

    def diagnostics(self, params, W):
        p = make_params(params)
        out = np.zeros(4)
        lib().or_diagnostics(self.h, C.byref(p), _dp(to_elem(W)), _dp(out))
        return dict(mass=out[0], active_pct=out[1], lambda_max=out[2], h_min=out[3])

    def eval_points(self, W):
        vals = np.zeros((self.n_el, self.nq, self.nf))
        lib().or_eval_points(self.h, _dp(to_elem(W)), _dp(vals))
        return vals

    def cfl_dt(self, params, W, cfl):
        p = make_params(params)
        return lib().or_cfl_dt(self.h, C.byref(p), _dp(to_elem(W)), float(cfl))

    def newton_step(self, params, W, bold, dt, opts: SolveOptions | None = None, bc=1,
                    dirichlet=None, linear: str = "direct"):
        """One backward-Euler step by Newton.  linear='direct' solves every
        Newton system exactly (sparse LU); 'gmres' uses the C block-Jacobi
        GMRES(m) path (for meshes too large to factor)."""
        o = _opts(opts or SolveOptions())
        p = self._mp(params, bc, dirichlet)
        We = to_elem(W); be = to_elem(bold)
        if linear == "direct":
            its, conv = self._newton_direct(p, We, be, dt, o)
            return from_elem(We), dict(newton=its, converged=conv == 1, status=conv, gmres=0)
        conv = C.c_int(0); gits = C.c_int(0)
        its = lib().or_newton_step(self.h, C.byref(p), float(dt), _dp(We), _dp(be), C.byref(o),
                                   C.byref(conv), C.byref(gits))
        return from_elem(We), dict(newton=its, converged=conv.value == 1, status=conv.value,
                                   gmres=gits.value)

    def solve(self, params, W0, opts: SolveOptions, bc=1, dirichlet=None, linear: str = "direct",
              record=None):
        """Backward-Euler time loop from W0 to t_end (fixed dt from the CFL rule
        on the initial state unless overridden, last step clipped to t_end).
        record: optional list receiving (step, newton_its, status) per step."""
        o = _opts(opts)
        p = self._mp(params, bc, dirichlet)
        if linear != "direct":
            We = to_elem(W0); st = OrSolveStats()
            lib().or_solve(self.h, C.byref(p), C.byref(o), _dp(We), C.byref(st))
            stats = {k: getattr(st, k) for k, _ in OrSolveStats._fields_}
            return from_elem(We), stats
        L = lib()
        We = to_elem(W0)
        dt = o.dt_override if o.dt_override > 0 else L.or_cfl_dt(self.h, C.byref(p), _dp(We), o.cfl)
        n_total = max(1, int(math.ceil(o.t_end / dt - 1e-12)))
        nsteps = n_total if o.max_steps < 0 else min(n_total, o.max_steps)
        diag = np.zeros(4)
        L.or_diagnostics(self.h, C.byref(p), _dp(We), _dp(diag))
        st = dict(steps=0, newton_total=0, gmres_total=0, newton_max=0, capped=0, dt=dt,
                  mass0=float(diag[0]), mass_end=0.0, max_mass_drift=0.0, active_pct=0.0, t_end=0.0)
        t = 0.0
        be = np.zeros_like(We)
        # continuation on gamma (Sec. 6.3): the regularisation parameter of the
        # i-th Newton solve of a step; beta and every other parameter stay
        if opts.cont_steps >= 2:
            n = opts.cont_steps
            g0, g1 = float(opts.cont_gamma0), float(params.gamma)
            stages = [self._mp(dataclasses.replace(params, gamma=g0 + (i - 1) * (g1 - g0) / (n - 1)), bc,
                                  dirichlet) for i in range(1, n + 1)]
        else:
            stages = [p]
        for k in range(1, nsteps + 1):
            dtk = dt if k < n_total else o.t_end - (k - 1) * dt
            L.or_step_begin(self.h, C.byref(p), float(dtk), _dp(We), _dp(be))
            its = 0
            for ps in stages:
                i_s, conv = self._newton_direct(ps, We, be, dtk, o)
                its += i_s
                if conv < 0:
                    break
            st["newton_total"] += its
            st["newton_max"] = max(st["newton_max"], its)
            st["capped"] += int(conv != 1)
            if record is not None:
                record.append((k, its, conv))
            L.or_diagnostics(self.h, C.byref(p), _dp(We), _dp(diag))
            st["max_mass_drift"] = max(st["max_mass_drift"], abs(diag[0] - st["mass0"]) / st["mass0"])
            t += dtk
            st["steps"] = k
            if conv < 0:
                break
        st["mass_end"] = float(diag[0]); st["active_pct"] = float(diag[1]); st["t_end"] = t
        return from_elem(We), st


def _opts(o: SolveOptions) -> OrSolveOpts:
    c = OrSolveOpts()
    for k, _ in OrSolveOpts._fields_:
        setattr(c, k, getattr(o, k))
    return c


# ------------------------------------------------------------- pointwise pins
def sigmaB_1d(reg, sigma0, gamma, beta, E):
    d = C.c_double(0.0)
    v = lib().or_sigmaB_1d(int(reg), float(sigma0), float(gamma), float(beta), float(E), C.byref(d))
    return v, d.value


def point_sigma(params, dim, Evec):
    p = make_params(params)
    E = np.ascontiguousarray(Evec, dtype=np.float64)
    sig = np.zeros(dim * dim); dsig = np.zeros(dim ** 4)
    lib().or_point_sigma(C.byref(p), dim, _dp(E), _dp(sig), _dp(dsig))
    return sig.reshape(dim, dim), dsig.reshape(dim, dim, dim, dim)


def point_psi(params, s):
    p = make_params(params)
    out = np.zeros(2)
    lib().or_point_psi(C.byref(p), float(s), _dp(out))
    return out[0], out[1]


def point_hll(params, dim, Xm, Xp, n, dXm=None, dXp=None):
    p = make_params(params)
    Xm = np.ascontiguousarray(Xm, dtype=np.float64); Xp = np.ascontiguousarray(Xp, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    F = np.zeros(1 + dim); dF = np.zeros(1 + dim)
    if dXm is None:
        lib().or_point_hll(C.byref(p), dim, _dp(Xm), _dp(Xp), _dp(n), None, None, _dp(F), None)
        return F
    dXm = np.ascontiguousarray(dXm, dtype=np.float64); dXp = np.ascontiguousarray(dXp, dtype=np.float64)
    lib().or_point_hll(C.byref(p), dim, _dp(Xm), _dp(Xp), _dp(n), _dp(dXm), _dp(dXp), _dp(F), _dp(dF))
    return F, dF


def point_wall(params, dim, n, Xin):
    p = make_params(params)
    Xin = np.ascontiguousarray(Xin, dtype=np.float64)
    out = np.zeros_like(Xin)
    lib().or_point_wall(C.byref(p), dim, _dp(np.ascontiguousarray(n, dtype=np.float64)), _dp(Xin), _dp(out))
    return out

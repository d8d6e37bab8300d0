"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds no arithmetic of the method: it only draws meshes (vertex
coordinates and element->vertex lists), random coefficient states, physical
parameters and initial-condition descriptors.  Everything that depends on the
discretisation (connectivity, metrics, basis functions, projections, fluxes)
is computed independently by each consumer.

Layout conventions (also the library's state layout):
  * state W is float64 array of shape [n_f, N_p, n_el] ("SoA", elements fastest)
  * 1-D fields  : (h, u, E11)                            n_f = 3
  * 2-D fields  : (h, u1, u2, E11, E21, E12, E22)        n_f = 7
    where E_ab = d u_b / d x_a (velocity gradient, paper Sec. 3, Eq. gradientVel)
  * N_p = P+1 (1-D) or (P+1)(P+2)/2 (triangles)

Every workload follows the shapes of the five benchmark configurations that
mirror the paper's test cases (dam break, flow on an incline, circular dam break,
ensembles of those); the numbers are stated in the functions below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import Optional

import numpy as np

# Boundary codes (library and oracle both understand these integers).
BC_WALL = 1
BC_NEUMANN = 2
BC_DIRICHLET = 3

# Initial-condition kinds (descriptors only; projection is done by the consumer).
IC_CONST = 0      # h = a, u = (b, c)
IC_STEP_X = 1     # h = a if x < x0 else b ; u = 0          (1-D / 2-D dam break)
IC_MOUND = 2      # h = a + b*exp(-|x-c|^2 / d) ; u = 0      (mound on an incline)
IC_DISK = 3       # h = a if |x-c| < r else b ; u = 0         (circular dam break)
IC_SINE_U = 4     # h = a ; u1 = b*sin(pi*x/L)                (decaying shear flow)
IC_LINEAR_X = 5   # h = a + b*x ; u = 0                      (tilted lake at rest)
IC_SHEAR_Y = 6    # h = a ; u1 = b*cos(pi*y/L)                (decaying shear mode)
IC_VORTEX = 7     # h = a ; u = b*(sin(pi x/L)cos(pi y/L), -cos(pi x/L)sin(pi y/L))
IC_SURFACE = 8    # h = a + b*x - H(x) ; u = 0 (free surface over the bed H)

BED_FLAT = 0      # H = 0
BED_COS = 1       # H = a cos(kx x) cos(ky y)   (1-D: a cos(kx x))
BED_GAUSS = 2     # H = a exp(-|x - (x0, y0)|^2 / d)

REG1, REG2, REG3 = 1, 2, 3


def n_modes(dim: int, P: int) -> int:
    return P + 1 if dim == 1 else (P + 1) * (P + 2) // 2


def n_fields(dim: int) -> int:
    return 1 + dim + dim * dim


def rng_for(seed: int, *spawn_key: int) -> np.random.Generator:
    ss = np.random.SeedSequence(seed, spawn_key=tuple(spawn_key))
    return np.random.Generator(np.random.PCG64(ss))


# ----------------------------------------------------------------------------- meshes

def mesh_1d(n_el: int, x0: float = 0.0, x1: float = 10.0):
    """Uniform 1-D mesh: vertices [n_el+1, 1] float64, el2vert [n_el, 2] int32."""
    xy = np.linspace(x0, x1, n_el + 1, dtype=np.float64).reshape(-1, 1)
    el2vert = np.stack([np.arange(n_el), np.arange(1, n_el + 1)], axis=1).astype(np.int32)
    return xy, el2vert


def mesh_tri(N: int, Lx: float = 20.0, Ly: float = 20.0, jitter: float = 0.1,
             seed: int = 0, Ny: Optional[int] = None):
    """Structured N x Ny squares on [0,Lx]x[0,Ly], each cut along its SW->NE
    diagonal into two counter-clockwise triangles; interior vertices moved by
    U[-jitter, jitter] * spacing in x and y (boundary vertices stay fixed).

    Element numbering: square (i, j) -> triangles 2*(j*N+i) (SW,SE,NE) and
    2*(j*N+i)+1 (SW,NE,NW).
    """
    Ny = N if Ny is None else Ny
    dx, dy = Lx / N, Ly / Ny
    I, J = np.meshgrid(np.arange(N + 1), np.arange(Ny + 1), indexing="xy")
    x = (I * dx).astype(np.float64).ravel()
    y = (J * dy).astype(np.float64).ravel()
    if jitter > 0:
        rng = rng_for(seed, 1)
        jx = rng.uniform(-jitter, jitter, size=x.shape) * dx
        jy = rng.uniform(-jitter, jitter, size=y.shape) * dy
        interior = ((I > 0) & (I < N) & (J > 0) & (J < Ny)).ravel()
        x = np.where(interior, x + jx, x)
        y = np.where(interior, y + jy, y)
    xy = np.stack([x, y], axis=1)
    vid = lambda i, j: j * (N + 1) + i
    ii, jj = np.meshgrid(np.arange(N), np.arange(Ny), indexing="xy")
    ii, jj = ii.ravel(), jj.ravel()
    sw, se, ne, nw = vid(ii, jj), vid(ii + 1, jj), vid(ii + 1, jj + 1), vid(ii, jj + 1)
    t0 = np.stack([sw, se, ne], axis=1)
    t1 = np.stack([sw, ne, nw], axis=1)
    el2vert = np.empty((2 * N * Ny, 3), dtype=np.int32)
    el2vert[0::2] = t0
    el2vert[1::2] = t1
    return xy, el2vert


def mesh_side_for_count(n_tri: float) -> int:
    """Square side N such that 2*N*N is nearest the requested triangle count."""
    return max(1, int(round(math.sqrt(n_tri / 2.0))))


# ----------------------------------------------------------------------------- states

def random_state(dim: int, P: int, n_el: int, seed: int, *, h_mean=(0.5, 2.0),
                 rel_hi_modes: float = 0.004, u_scale: float = 1.0,
                 frac_fast: float = 0.15, e_logrange=(-6.0, 0.5)) -> np.ndarray:
    """Random coefficient state W [n_f, N_p, n_el] spanning the regimes the
    operator has branches for:
      * mode-0 of h in h_mean, higher h modes relative amplitude rel_hi_modes
        (keeps h > 0 everywhere for orthonormal bases with P <= 4);
      * velocities O(u_scale), a fraction frac_fast of elements 4x faster
        (supercritical HLL branches);
      * strain-rate coefficients with a per-element log-uniform scale, so the
        shear rate falls on both sides of every regularisation breakpoint.
    """
    rng = rng_for(seed, 2)
    nf, Np = n_fields(dim), n_modes(dim, P)
    W = np.zeros((nf, Np, n_el), dtype=np.float64)
    c0 = rng.uniform(*h_mean, size=n_el)
    W[0, 0] = c0
    if Np > 1:
        W[0, 1:] = rng.uniform(-1, 1, size=(Np - 1, n_el)) * rel_hi_modes * c0
    fast = np.where(rng.uniform(size=n_el) < frac_fast, 4.0, 1.0)
    for b in range(dim):
        W[1 + b] = rng.uniform(-1, 1, size=(Np, n_el)) * u_scale * fast
        if Np > 1:
            W[1 + b, 1:] *= 0.3
    escale = 10.0 ** rng.uniform(*e_logrange, size=n_el)
    W[1 + dim:] = rng.uniform(-1, 1, size=(dim * dim, Np, n_el)) * escale
    return W


def random_vector(dim: int, P: int, n_el: int, seed: int) -> np.ndarray:
    rng = rng_for(seed, 3)
    return rng.standard_normal((n_fields(dim), n_modes(dim, P), n_el))


# ----------------------------------------------------------------------------- params

@dataclass
class Params:
    g: float = 9.81
    rho: float = 1000.0
    alpha: float = 0.0          # incline angle (rad)
    eta: float = 1.0            # plastic viscosity
    sigma0: float = 50.0        # yield stress
    gamma: float = 1e3          # regularisation parameter
    beta: float = 1e3           # smoothing parameter of regularisations 1, 2
    reg: int = REG1
    jac_frozen: int = 0         # 1: Jacobian with the HLL wave speeds held fixed

    @staticmethod
    def from_eps(eps: float, **kw) -> "Params":
        """Configurations quote a regularisation parameter eps; it maps to the
        paper's (gamma, beta) as gamma = beta = 1/eps."""
        return Params(gamma=1.0 / eps, beta=1.0 / eps, **kw)


@dataclass
class IC:
    kind: int = IC_CONST
    a: float = 1.0
    b: float = 0.0
    c: float = 0.0
    d: float = 0.0
    x0: float = 0.0
    y0: float = 0.0
    r: float = 0.0
    L: float = 1.0


@dataclass
class Bed:
    """Analytic bed H; order = m0, the interpolation order (0: the disc's P)."""
    kind: int = BED_FLAT
    order: int = 0
    a: float = 0.0
    kx: float = 0.0
    ky: float = 0.0
    x0: float = 0.0
    y0: float = 0.0
    d: float = 1.0


@dataclass
class Problem:
    name: str
    dim: int
    P: int
    xy: np.ndarray
    el2vert: np.ndarray
    params: Params
    ic: IC
    t_end: float
    cfl: float = 0.2
    bc: int = BC_WALL
    meta: dict = field(default_factory=dict)

    @property
    def n_el(self) -> int:
        return int(self.el2vert.shape[0])

    @property
    def n_dof(self) -> int:
        return n_fields(self.dim) * n_modes(self.dim, self.P) * self.n_el


# Configuration 1: 1-D Bingham dam break (plain FP64).
def config1(reg: int = REG1, n_el: int = 200, sigma0: float = 50.0, eta: float = 1.0,
            t_end: float = 1.0) -> Problem:
    xy, e2v = mesh_1d(n_el, 0.0, 10.0)
    prm = Params.from_eps(1e-3, g=9.81, rho=1000.0, alpha=0.0, eta=eta, sigma0=sigma0, reg=reg)
    ic = IC(kind=IC_STEP_X, a=1.0, b=0.1, x0=5.0)
    return Problem("c1_dambreak_1d", 1, 1, xy, e2v, prm, ic, t_end, 0.2, BC_WALL,
                   {"reg": reg, "eps": 1e-3})


# Configuration 2: 2-D Bingham flow on a 10% incline, 64x64 jittered -> 8192 triangles, P2.
C2_EPS = (1e-2, 1e-3, 1e-4)


def config2(reg: int = REG1, eps: float = 1e-3, N: int = 64, seed: int = 2,
            t_end: float = 2.0, P: int = 2) -> Problem:
    xy, e2v = mesh_tri(N, 20.0, 20.0, 0.1, seed)
    run = (reg - 1) * len(C2_EPS) + (C2_EPS.index(eps) if eps in C2_EPS else 0)
    sigma0 = float(rng_for(seed, 10, run).uniform(20.0, 200.0))
    alpha = math.atan(0.1)
    prm = Params.from_eps(eps, g=9.81, rho=1000.0, alpha=alpha, eta=1.0, sigma0=sigma0, reg=reg)
    ic = IC(kind=IC_MOUND, a=1.0, b=0.5, x0=10.0, y0=10.0, d=4.0)
    return Problem("c2_incline_2d", 2, P, xy, e2v, prm, ic, t_end, 0.2, BC_WALL,
                   {"reg": reg, "eps": eps, "N": N})


def config2_runs(N: int = 64, seed: int = 2, t_end: float = 2.0):
    return [config2(reg, eps, N, seed, t_end) for reg in (REG1, REG2, REG3) for eps in C2_EPS]


# Configuration 3: 2-D circular dam break, 256x256 jittered -> 131072 triangles, P3.
def config3(reg: int = REG1, N: int = 256, seed: int = 3, t_end: float = 1.0,
            P: int = 3) -> Problem:
    xy, e2v = mesh_tri(N, 20.0, 20.0, 0.1, seed)
    prm = Params.from_eps(1e-4, g=9.81, rho=1000.0, alpha=0.0, eta=0.5, sigma0=30.0, reg=reg)
    ic = IC(kind=IC_DISK, a=2.0, b=0.5, x0=10.0, y0=10.0, r=2.5)
    return Problem("c3_circular_dambreak", 2, P, xy, e2v, prm, ic, t_end, 0.2, BC_WALL,
                   {"reg": reg, "eps": 1e-4, "N": N})


# Configuration 4: ensemble of 512 circular dam breaks of mixed size/order/parameters.
def config4_instance(k: int, seed: int = 4, n_range=(500.0, 50000.0)) -> Problem:
    rng = rng_for(seed, 20, k)
    n = math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))
    N = mesh_side_for_count(n)
    P = int(rng.integers(1, 4))
    step = float(rng.uniform(0.5, 3.0))
    sigma0 = float(rng.uniform(10.0, 300.0))
    eta = float(rng.uniform(0.1, 5.0))
    eps = math.exp(rng.uniform(math.log(1e-5), math.log(1e-2)))
    reg = int(rng.integers(1, 4))
    mesh_seed = int(rng.integers(0, 2**31 - 1))
    xy, e2v = mesh_tri(N, 20.0, 20.0, 0.1, mesh_seed)
    prm = Params.from_eps(eps, g=9.81, rho=1000.0, alpha=0.0, eta=eta, sigma0=sigma0, reg=reg)
    ic = IC(kind=IC_DISK, a=0.5 + step, b=0.5, x0=10.0, y0=10.0, r=2.5)
    return Problem(f"c4_member_{k}", 2, P, xy, e2v, prm, ic, 1.0, 0.2, BC_WALL,
                   {"reg": reg, "eps": eps, "N": N, "k": k})


# Served requests: slope flows (the incline configuration's physics) of mixed
# mesh size, order and Bingham parameters, and dam breaks limited to
# eps >= 1e-3.  Ensemble draws with smaller eps cap the Newton iteration of the
# method itself (exact linear solves included), so their results carry no
# accuracy to compare.
def serving_request(k: int, seed: int = 6, n_range=(512.0, 8192.0)) -> Problem:
    rng = rng_for(seed, 40, k)
    n = math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))
    N = mesh_side_for_count(n)
    P = int(rng.integers(1, 4))
    reg = int(rng.integers(1, 4))
    eps = math.exp(rng.uniform(math.log(1e-3), math.log(1e-2)))
    eta = float(rng.uniform(0.5, 2.0))
    mesh_seed = int(rng.integers(0, 2**31 - 1))
    xy, e2v = mesh_tri(N, 20.0, 20.0, 0.1, mesh_seed)
    if rng.uniform() < 0.5:
        sigma0 = float(rng.uniform(20.0, 200.0))
        prm = Params.from_eps(eps, g=9.81, rho=1000.0, alpha=math.atan(0.1), eta=eta, sigma0=sigma0, reg=reg)
        ic = IC(kind=IC_MOUND, a=1.0, b=float(rng.uniform(0.2, 0.8)), x0=10.0, y0=10.0, d=4.0)
        kind = "slope"
    else:
        sigma0 = float(rng.uniform(10.0, 100.0))
        prm = Params.from_eps(eps, g=9.81, rho=1000.0, alpha=0.0, eta=eta, sigma0=sigma0, reg=reg)
        ic = IC(kind=IC_DISK, a=0.5 + float(rng.uniform(0.5, 1.5)), b=0.5, x0=10.0, y0=10.0, r=2.5)
        kind = "dambreak"
    return Problem(f"served_{kind}_{k}", 2, P, xy, e2v, prm, ic, 1.0, 0.2, BC_WALL,
                   {"reg": reg, "eps": eps, "N": N, "k": k, "kind": kind})


def config4(n_inst: int = 512, seed: int = 4):
    return [config4_instance(k, seed) for k in range(n_inst)]


# Configuration 5: Poisson request stream (98% config-4 draws, 2% large incline runs).
def config5_arrivals(rate: float = 200.0, duration: float = 60.0, seed: int = 5,
                     large_frac: float = 0.02):
    """Returns a list of (arrival_time_s, kind, index) with kind 'c4' or 'large'."""
    rng = rng_for(seed, 30)
    t, out, k = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        kind = "large" if rng.uniform() < large_frac else "c4"
        out.append((t, kind, k))
        k += 1
    return out


def config5_large(seed: int = 5, N: int = 707) -> Problem:
    p = config2(REG1, 1e-3, N=N, seed=seed, t_end=2.0)
    p.name = "c5_large_incline"
    return p


def params_dict(p: Params) -> dict:
    return asdict(p)

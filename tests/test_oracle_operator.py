"""Pins of the oracle's discrete operator (paper Sec. 5, Eq. WeakForm7) and of
its tangent (Appendix A): invariants that hold exactly for the discrete
scheme, a viscous decay rate fixed by the continuum equations, and finite
differences for the Jacobian.
"""
import math

import numpy as np
import pytest

import workloads as wl

CASES = [(1, 1), (1, 2), (1, 3), (2, 1), (2, 2), (2, 3)]


def make(oracle_mod, dim, P, n=3, L=20.0, jitter=0.1, seed=2):
    if dim == 1:
        xy, e2v = wl.mesh_1d(max(4, 3 * n), 0.0, L / 2)
    else:
        xy, e2v = wl.mesh_tri(n, L, L, jitter, seed)
    return oracle_mod.Oracle(dim, P, xy, e2v)


def scale_of(o, prm, W, dt):
    b = o.step_begin(prm, W, dt)
    return np.abs(b).max()


@pytest.mark.parametrize("dim,P", CASES)
@pytest.mark.parametrize("reg", [1, 2, 3])
def test_lake_at_rest_flat(oracle_mod, dim, P, reg):
    """h const, u = 0, E = 0, W_old = W: R = 0 to rounding, walls all round."""
    o = make(oracle_mod, dim, P)
    prm = wl.Params(alpha=0.0, eta=1.0, sigma0=30.0, gamma=1e3, beta=1e3, reg=reg)
    W = o.project_ic(wl.IC(kind=wl.IC_CONST, a=1.7))
    dt = 0.01
    R = o.residual(prm, W, o.step_begin(prm, W, dt), dt)
    assert np.abs(R).max() < 1e-14 * scale_of(o, prm, W, dt) * 10


@pytest.mark.parametrize("dim,P", CASES)
def test_tilted_lake_at_rest_on_incline(oracle_mod, dim, P):
    """Flat-bed form of the paper's constant-free-surface example (Sec. 6.1):
    on an incline, h = h0 - x tan(alpha) with u = 0 is an exact equilibrium of
    the source -g_s h and the pressure 1/2 g_c h^2; the discrete residual
    vanishes (the linear depth is represented exactly, walls all round)."""
    alpha = math.pi / 18
    o = make(oracle_mod, dim, P)
    L = 10.0 if dim == 1 else 20.0
    h0 = 3.0 if dim == 1 else 5.0
    prm = wl.Params(g=9.81, rho=1.0, alpha=alpha, eta=1.0, sigma0=1.0, gamma=1e3, beta=1e3, reg=1)
    W = o.project_ic(wl.IC(kind=wl.IC_LINEAR_X, a=h0, b=-math.tan(alpha)))
    dt = 0.01
    R = o.residual(prm, W, o.step_begin(prm, W, dt), dt)
    assert np.abs(R).max() < 1e-13 * scale_of(o, prm, W, dt)
    # the same depth with the wrong slope sign is not at rest
    W2 = o.project_ic(wl.IC(kind=wl.IC_LINEAR_X, a=h0 - L * math.tan(alpha), b=math.tan(alpha)))
    R2 = o.residual(prm, W2, o.step_begin(prm, W2, dt), dt)
    assert np.abs(R2[1]).max() > 1e-3


@pytest.mark.parametrize("dim,P", [(2, 1), (2, 2), (2, 3), (1, 1), (1, 2)])
def test_exact_gradient_gives_zero_RE(oracle_mod, dim, P):
    """Continuous linear velocity with E equal to its gradient
    (E_ab = d u_b / d x_a, Eq. gradientVel) makes R_E vanish (Neumann BC)."""
    o = make(oracle_mod, dim, P)
    m = o.mesh_data()
    t = o.ref_tables()
    rng = np.random.default_rng(1)
    A = rng.normal(size=(dim, dim))   # u_b = c_b + sum_a A[a, b] x_a
    c = rng.normal(size=dim)
    W = np.zeros(o.shape)
    W[0] = o.project_ic(wl.IC(kind=wl.IC_CONST, a=1.2))[0]
    xq = m["xq"][:, :, :dim]
    for b in range(dim):
        ub = c[b] + np.einsum("eqa,a->eq", xq, A[:, b])
        W[1 + b] = np.einsum("q,qi,eq->ie", t["qw"], t["phi"], ub)
        for a in range(dim):
            W[1 + dim + b * dim + a] = np.einsum("q,qi->i", t["qw"], t["phi"])[:, None] * A[a, b]
    prm = wl.Params(alpha=0.0, eta=1.0, sigma0=0.0, gamma=1e3, beta=1e3, reg=1)
    dt = 0.01
    R = o.residual(prm, W, o.step_begin(prm, W, dt), dt, bc=wl.BC_NEUMANN)
    assert np.abs(R[1 + dim:]).max() < 1e-12 * max(1.0, np.abs(W).max())
    # transposing the gradient breaks it (the ordering matters when A is not symmetric)
    if dim == 2:
        W2 = W.copy()
        W2[4], W2[5] = W[5].copy(), W[4].copy()
        R2 = o.residual(prm, W2, o.step_begin(prm, W2, dt), dt, bc=wl.BC_NEUMANN)
        assert np.abs(R2[3:]).max() > 1e-3


@pytest.mark.parametrize("dim,P", CASES)
def test_free_stream_preserved(oracle_mod, dim, P):
    """Constant h and u with E = 0, W_old = W and Dirichlet exterior equal to
    the same state: every element residual vanishes (flux consistency)."""
    o = make(oracle_mod, dim, P)
    u = (0.7, -0.4)[:dim]
    W = o.project_ic(wl.IC(kind=wl.IC_CONST, a=1.3, b=u[0], c=u[1] if dim == 2 else 0.0))
    prm = wl.Params(alpha=0.0, eta=1.0, sigma0=20.0, gamma=1e3, beta=1e3, reg=2)
    dirv = [1.3] + list(u) + [0.0] * (dim * dim)
    dt = 0.01
    R = o.residual(prm, W, o.step_begin(prm, W, dt), dt, bc=wl.BC_DIRICHLET, dirichlet=dirv)
    assert np.abs(R).max() < 1e-13 * scale_of(o, prm, W, dt)


@pytest.mark.parametrize("dim,P", CASES)
@pytest.mark.parametrize("reg", [1, 3])
def test_mass_telescoping(oracle_mod, dim, P, reg):
    """With walls, sum_e <1, R_h,e> = (M(W) - M(W_old)) / dt for ANY W: interior
    face fluxes cancel and the mirror wall carries no mass (Sec. 5, Eq. HLLSolver)."""
    o = make(oracle_mod, dim, P, n=4)
    prm = wl.Params(alpha=0.2, eta=1.0, sigma0=30.0, gamma=1e3, beta=1e3, reg=reg)
    W = wl.random_state(dim, P, o.n_el, 11)
    Wold = wl.random_state(dim, P, o.n_el, 12)
    dt = 0.013
    R = o.residual(prm, W, o.step_begin(prm, Wold, dt), dt)
    phi0 = math.sqrt(2.0) if dim == 2 else 1.0 / math.sqrt(2.0)
    meas = 0.5 if dim == 2 else 2.0
    detJ = o.mesh_data()["detJ"]
    lhs = (R[0, 0] * phi0 * meas).sum()   # <1, R_h> through the constant mode
    M1 = o.diagnostics(prm, W)["mass"]
    M0 = o.diagnostics(prm, Wold)["mass"]
    rhs = (M1 - M0) / dt
    assert abs(lhs - rhs) < 1e-12 * (M1 / dt)


@pytest.mark.parametrize("dim,P", CASES)
@pytest.mark.parametrize("reg", [1, 2, 3])
def test_jacobian_matches_finite_differences(oracle_mod, dim, P, reg):
    o = make(oracle_mod, dim, P)
    prm = wl.Params(alpha=0.15, eta=0.8, sigma0=5.0, gamma=1e2, beta=1e2, reg=reg, rho=50.0)
    W = wl.random_state(dim, P, o.n_el, 21 + reg)
    v = wl.random_vector(dim, P, o.n_el, 22)
    dt = 0.02
    b = o.step_begin(prm, wl.random_state(dim, P, o.n_el, 23), dt)
    Jv = o.jac_apply(prm, W, v, dt)
    # Richardson-extrapolated central differences
    def cd(eps):
        return (o.residual(prm, W + eps * v, b, dt) - o.residual(prm, W - eps * v, b, dt)) / (2 * eps)
    fd = (4 * cd(1e-6) - cd(2e-6)) / 3
    assert np.abs(Jv - fd).max() < 2e-6 * np.abs(fd).max()


@pytest.mark.parametrize("dim,P", [(1, 2), (2, 1), (2, 2), (2, 3)])
def test_diagonal_blocks_are_own_element_jacobian(oracle_mod, dim, P):
    o = make(oracle_mod, dim, P)
    prm = wl.Params(alpha=0.1, eta=1.0, sigma0=20.0, gamma=1e3, beta=1e3, reg=1)
    W = wl.random_state(dim, P, o.n_el, 31)
    dt = 0.02
    B = o.jac_blocks(prm, W, dt)
    rng = np.random.default_rng(0)
    for e in rng.choice(o.n_el, size=min(6, o.n_el), replace=False):
        v = np.zeros(o.shape)
        ve = rng.normal(size=(o.nf, o.np))
        v[:, :, e] = ve
        y = o.jac_apply(prm, W, v, dt)
        assert np.abs(y[:, :, e].ravel() - B[e] @ ve.ravel()).max() < 1e-10 * np.abs(B[e]).max()
    # the E-E part of every block is the mass matrix |J| I (Appendix A, dR_E/dE)
    detJ = o.mesh_data()["detJ"]
    nv = (1 + dim) * o.np
    for e in range(o.n_el):
        EE = B[e][nv:, nv:]
        assert np.abs(EE - detJ[e] * np.eye(EE.shape[0])).max() < 1e-11 * detJ[e]


def vortex_amplitude(o, W, L):
    t = o.ref_tables()
    m = o.mesh_data()
    vals = o.eval_points(W)
    x, y = m["xq"][:, :, 0], m["xq"][:, :, 1]
    w = t["qw"][None, :] * m["detJ"][:, None]
    m1 = np.sin(math.pi * x / L) * np.cos(math.pi * y / L)
    m2 = -np.cos(math.pi * x / L) * np.sin(math.pi * y / L)
    num = (w * (vals[:, :, 1] * m1 + vals[:, :, 2] * m2)).sum()
    return num / (w * (m1 * m1 + m2 * m2)).sum()


@pytest.mark.parametrize("reg,s0,gam", [(1, 0.0, 1e2), (1, 1.0, 1e2), (2, 1.0, 1e2), (3, 1.0, 1e2)])
def test_viscous_vortex_decay_rate(oracle_mod, reg, s0, gam):
    """A small divergence-free vortex u = U0 (sin(pi x/L) cos(pi y/L),
    -cos(pi x/L) sin(pi y/L)), h = 1, in a box with mirror walls is a
    free-slip eigenmode of the viscous term: div(h sigma)/rho = nu lap(u) with
    nu = (eta + psi(0)/2)/rho, since sigma = (2 eta + psi) (D + tr(D) I) and
    tr D = 0 (Eqs. binghamR, sigma1 and the 2-D regularisation).  In the
    unyielded band psi(0) = gamma (regs 1, 2) or sigma0 gamma (reg 3); 0 with
    no yield stress.  Backward Euler divides the mode by 1 + lambda dt per
    step, lambda = 2 nu (pi/L)^2."""
    L, eta, rho = 2.0, 0.2, 1.0
    xy, e2v = wl.mesh_tri(6, L, L, 0.0, 0)
    o = oracle_mod.Oracle(2, 3, xy, e2v)
    prm = wl.Params(g=9.81, rho=rho, alpha=0.0, eta=eta, sigma0=s0, gamma=gam, beta=gam, reg=reg)
    W = o.project_ic(wl.IC(kind=wl.IC_VORTEX, a=1.0, b=1e-5, L=L))
    psi0 = 0.0 if s0 == 0 else (gam if reg in (1, 2) else s0 * gam)
    lam = 2.0 * (eta + 0.5 * psi0) / rho * (math.pi / L) ** 2
    dt = 0.15 / lam
    a0 = vortex_amplitude(o, W, L)
    nsteps = 3
    for _ in range(nsteps):
        b = o.step_begin(prm, W, dt)
        W, info = o.newton_step(prm, W, b, dt, oracle_mod.SolveOptions(newton_tol=1e-12))
        assert info["converged"]
    ratio = vortex_amplitude(o, W, L) / a0
    expect = (1.0 + lam * dt) ** (-nsteps)
    assert abs(ratio - expect) < 1e-5 * expect, (ratio, expect)
    # a mis-scaled viscosity (factor 2 either way) is far outside that band
    assert abs(ratio - (1.0 + 2 * lam * dt) ** (-nsteps)) > 5e-2 * expect


def test_mass_conserved_through_newton(oracle_mod):
    pb = wl.config1(1, n_el=60, sigma0=50.0)
    o = oracle_mod.Oracle(pb.dim, pb.P, pb.xy, pb.el2vert)
    W0 = o.project_ic(pb.ic)
    W, st = o.solve(pb.params, W0, oracle_mod.SolveOptions(t_end=0.05, cfl=0.2))
    assert st["steps"] >= 5
    assert st["max_mass_drift"] < 1e-12
    xy, e2v = wl.mesh_tri(6, 20.0, 20.0, 0.1, 2)
    o2 = oracle_mod.Oracle(2, 2, xy, e2v)
    prm = wl.Params(alpha=math.atan(0.1), eta=1.0, sigma0=60.0, gamma=1e2, beta=1e2, reg=1)
    W0 = o2.project_ic(wl.IC(kind=wl.IC_MOUND, a=1.0, b=0.5, x0=10, y0=10, d=4.0))
    W, st = o2.solve(prm, W0, oracle_mod.SolveOptions(t_end=0.1, cfl=0.2))
    assert st["max_mass_drift"] < 1e-12 and st["capped"] == 0


def test_newton_converges_quadratically(oracle_mod):
    """Exact tangent => quadratic convergence on a smooth problem (paper Sec. 6
    reports 2-3 iterations per step)."""
    xy, e2v = wl.mesh_tri(5, 20.0, 20.0, 0.1, 2)
    o = oracle_mod.Oracle(2, 2, xy, e2v)
    prm = wl.Params(alpha=math.atan(0.1), eta=1.0, sigma0=60.0, gamma=1e2, beta=1e2, reg=3)
    W0 = o.project_ic(wl.IC(kind=wl.IC_MOUND, a=1.0, b=0.5, x0=10, y0=10, d=4.0))
    dt = 0.05
    b = o.step_begin(prm, W0, dt)
    norms = []
    for k in range(1, 5):
        Wk, _ = o.newton_step(prm, W0, b, dt, oracle_mod.SolveOptions(max_newton=k, newton_tol=0.0))
        norms.append(np.linalg.norm(o.residual(prm, Wk, b, dt)))
    r0 = np.linalg.norm(o.residual(prm, W0, b, dt))
    seq = [r0] + norms
    # find two consecutive reductions above the rounding floor and check the order
    orders = [math.log(seq[i + 2] / seq[i + 1]) / math.log(seq[i + 1] / seq[i])
              for i in range(len(seq) - 2) if seq[i + 2] > 1e-10 * r0]
    assert orders and max(orders) > 1.7, seq

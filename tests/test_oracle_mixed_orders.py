"""Pins of the oracle's mixed orders m1, m2, m3 for h, u and E (paper Sec. 5;
Sec. 6.1 Tables errorsEx1a/b; the dam break with m3 = 0 of Sec. 6.3).

With bases ordered by total degree, a field of order m lives in the span of
its first N(m) modes and is tested with them; the higher modes of the storage
order P carry the trivial equations W = 0.  The pins: the uniform setting
changes nothing; on a line with polynomial integrands (sigma0 = 0) the mixed
system on order-2 storage is exactly the order-1 scheme; the exact gradient
with piecewise-constant E; the lake at rest exact for m0 <= m1 whatever m2,
m3 (the tables' plain rows) and not for m0 > m1 (their shaded rows), with
errors falling under refinement; and the depth and velocity of an inviscid
dam break not depending on m3.
"""
import math

import numpy as np
import pytest

import workloads as wl

ALPHA = math.pi / 18


def line(oracle_mod, P, n, L=10.0):
    xy, e2v = wl.mesh_1d(n, 0.0, L)
    return oracle_mod.Oracle(1, P, xy, e2v)


def tri(oracle_mod, P, n):
    xy, e2v = wl.mesh_tri(n, 20.0, 20.0, 0.1, 2)
    return oracle_mod.Oracle(2, P, xy, e2v)


@pytest.mark.parametrize("dim,P", [(1, 2), (2, 3)])
def test_uniform_orders_change_nothing(oracle_mod, dim, P):
    o = line(oracle_mod, P, 30) if dim == 1 else tri(oracle_mod, P, 4)
    p = wl.Params(alpha=0.1, eta=0.8, sigma0=40.0, gamma=1e3, beta=1e3, reg=2)
    W = wl.random_state(dim, P, o.n_el, 11)
    b = o.step_begin(p, W, 0.01)
    R0 = o.residual(p, W, b, 0.01)
    o.set_orders(P, P, P)
    assert np.array_equal(o.residual(p, W, b, 0.01), R0)
    with pytest.raises(ValueError):
        o.set_orders(P + 1, P, P)


@pytest.mark.parametrize("reg", [1, 3])
def test_order_one_fields_on_order_two_storage_are_the_order_one_scheme(oracle_mod, reg):
    """1-D, sigma0 = 0: every volume integrand of order-1 fields is a cubic at
    most, which both the 2- and the 3-point Gauss rules integrate exactly, and
    faces are points.  So m1 = m2 = m3 = 1 on P = 2 storage must give the P = 1
    residual, Jacobian product and diagonal blocks on the used rows, the state
    itself on the trivial rows, and identity rows in the blocks."""
    n = 23
    o1, o2 = line(oracle_mod, 1, n), line(oracle_mod, 2, n)
    o2.set_orders(1, 1, 1)
    p = wl.Params(alpha=0.2, eta=0.7, sigma0=0.0, gamma=1e3, beta=1e3, reg=reg)
    W1 = wl.random_state(1, 1, n, 21)
    Wold1 = wl.random_state(1, 1, n, 22)
    x1 = wl.random_vector(1, 1, n, 23)

    def embed(A):
        B = np.zeros((A.shape[0], 3, n))
        B[:, :2] = A
        return B

    W2, Wold2, x2 = embed(W1), embed(Wold1), embed(x1)
    dt = 0.013
    R1 = o1.residual(p, W1, o1.step_begin(p, Wold1, dt), dt)
    R2 = o2.residual(p, W2, o2.step_begin(p, Wold2, dt), dt)
    scale = np.abs(R1).max()
    assert np.abs(R2[:, :2] - R1).max() <= 1e-13 * scale
    assert np.all(R2[:, 2] == 0.0)
    y1 = o1.jac_apply(p, W1, x1, dt)
    y2 = o2.jac_apply(p, W2, x2, dt)
    assert np.abs(y2[:, :2] - y1).max() <= 1e-13 * np.abs(y1).max()
    assert np.all(y2[:, 2] == 0.0)
    B1 = o1.jac_blocks(p, W1, dt)              # rows/cols f*2 + i
    B2 = o2.jac_blocks(p, W2, dt)              # rows/cols f*3 + i
    used = np.array([f * 3 + i for f in range(3) for i in range(2)])
    assert np.abs(B2[:, used][:, :, used] - B1).max() <= 1e-13 * np.abs(B1).max()
    for f in range(3):
        r = f * 3 + 2
        e_r = np.zeros(9)
        e_r[r] = 1.0
        assert np.all(B2[:, r, :] == e_r)
    # the mixed system is not the full order-2 one: the top modes matter there
    o2.set_orders(2, 2, 2)
    R2f = o2.residual(p, W2, o2.step_begin(p, Wold2, dt), dt)
    assert np.abs(R2f[:, 2]).max() > 1e-6 * scale


@pytest.mark.parametrize("dim,P", [(1, 1), (1, 2), (2, 1), (2, 2)])
def test_piecewise_constant_E_holds_an_exact_gradient(oracle_mod, dim, P):
    """m3 = 0 (the paper's dam break): for a continuous linear velocity the
    element mean of the lifted gradient is the gradient, so E = grad u
    (E_ab = d u_b / d x_a) zeroes R_E; its transpose does not (2-D)."""
    o = line(oracle_mod, P, 9) if dim == 1 else tri(oracle_mod, P, 3)
    o.set_orders(P, P, 0)
    m = o.mesh_data()
    t = o.ref_tables()
    rng = np.random.default_rng(4)
    A = rng.normal(size=(dim, dim))
    c = rng.normal(size=dim)
    W = np.zeros(o.shape)
    W[0] = o.project_ic(wl.IC(kind=wl.IC_CONST, a=1.3))[0]
    xq = m["xq"][:, :, :dim]
    mode0 = np.einsum("q,qi->i", t["qw"], t["phi"])           # projection of a constant
    for b in range(dim):
        ub = c[b] + np.einsum("eqa,a->eq", xq, A[:, b])
        W[1 + b] = np.einsum("q,qi,eq->ie", t["qw"], t["phi"], ub)
        for a in range(dim):
            W[1 + dim + b * dim + a] = mode0[:, None] * A[a, b]
    assert np.abs(W[1 + dim:, 1:]).max() < 1e-14                # E is constant per element
    prm = wl.Params(alpha=0.0, eta=1.0, sigma0=0.0, gamma=1e3, beta=1e3, reg=1)
    dt = 0.01
    R = o.residual(prm, W, o.step_begin(prm, W, dt), dt, bc=wl.BC_NEUMANN)
    assert np.abs(R[1 + dim:]).max() < 1e-12 * max(1.0, np.abs(W).max())
    if dim == 2:
        W2 = W.copy()
        W2[4], W2[5] = W[5].copy(), W[4].copy()
        R2 = o.residual(prm, W2, o.step_begin(prm, W2, dt), dt, bc=wl.BC_NEUMANN)
        assert np.abs(R2[3:]).max() > 1e-3


def lake(o, m0, surface=3.0 / math.cos(ALPHA)):
    o.set_bed(o.bed_interpolate(wl.Bed(kind=wl.BED_COS, order=m0, a=1.0, kx=math.pi)))
    return o.project_ic(wl.IC(kind=wl.IC_SURFACE, a=surface, b=-math.tan(ALPHA)))


def ex1_params(reg=1):
    return wl.Params(g=9.81, rho=1.0, alpha=ALPHA, eta=1.0, sigma0=1.0, gamma=1e3, beta=1e3, reg=reg)


# (m0, m1, m2, m3): the plain (balanced) rows of Tables errorsEx1a/b
@pytest.mark.parametrize("orders", [(2, 2, 1, 1), (1, 2, 1, 2), (1, 2, 2, 2), (2, 2, 1, 2), (3, 3, 2, 2), (1, 3, 1, 3)])
def test_lake_at_rest_exact_for_m0_not_above_m1(oracle_mod, orders):
    m0, m1, m2, m3 = orders
    P = max(orders)
    o = line(oracle_mod, P, 100)
    o.set_orders(m1, m2, m3)
    W = lake(o, m0)
    nm = m1 + 1
    assert np.all(W[0, nm:] == 0.0)
    prm = ex1_params()
    b = o.step_begin(prm, W, 0.01)
    R = o.residual(prm, W, b, 0.01)
    assert np.abs(R).max() <= 2e-14 * np.abs(b).max()


# the shaded rows: bed of higher order than the depth
@pytest.mark.parametrize("orders", [(2, 1, 1, 1), (2, 1, 2, 1), (2, 1, 1, 2), (3, 2, 2, 2), (3, 2, 3, 2)])
def test_lake_at_rest_not_kept_for_m0_above_m1(oracle_mod, orders):
    """Sec. 6.1 shaded rows: the depth cannot cancel the bed's source, the
    state moves (errors well above rounding at n_el = 100) and the errors at
    t = 1 fall under refinement (Table errorsEx1c's trend)."""
    import oracle
    m0, m1, m2, m3 = orders
    P = max(orders)
    errs = []
    for n in (100, 200):
        o = line(oracle_mod, P, n)
        o.set_orders(m1, m2, m3)
        W0 = lake(o, m0)
        W, st = o.solve(ex1_params(), W0, oracle.SolveOptions(t_end=1.0, dt_override=0.01))
        assert st["capped"] == 0
        X0, X = o.eval_points(W0), o.eval_points(W)
        errs.append(max(np.abs(X[:, :, 0] - X0[:, :, 0]).max(), np.abs(X[:, :, 1]).max()))
        # the unused modes stay exactly zero through the solve
        top = max(np.abs(W[0, m1 + 1:]).max(initial=0), np.abs(W[1, m2 + 1:]).max(initial=0),
                  np.abs(W[2, m3 + 1:]).max(initial=0))
        assert top == 0.0
    assert 1e-8 < errs[0] < 1e-1, errs
    assert errs[1] < errs[0] / 3.0, errs


def test_inviscid_dam_break_depth_does_not_depend_on_m3(oracle_mod):
    """Sec. 6.3 dam break set-up (m1 = m2 = 1, m3 = 0) in the sigma0 = eta = 0
    limit: the stress vanishes, E decouples, so h and u equal those of the
    uniform order-1 run (and the Stoker pin applies unchanged)."""
    import oracle
    pb = wl.config1(1, n_el=100, sigma0=0.0, eta=0.0, t_end=0.2)
    res = []
    for m3 in (1, 0):
        o = oracle_mod.Oracle(pb.dim, pb.P, pb.xy, pb.el2vert)
        o.set_orders(1, 1, m3)
        W, st = o.solve(pb.params, o.project_ic(pb.ic), oracle.SolveOptions(t_end=0.2, cfl=pb.cfl))
        assert st["capped"] == 0
        res.append(W)
    assert np.abs(res[0][:2] - res[1][:2]).max() <= 1e-10 * np.abs(res[0][:2]).max()
    assert np.all(res[1][2, 1:] == 0.0)
    assert np.abs(res[0][2, 1:]).max() > 1e-6

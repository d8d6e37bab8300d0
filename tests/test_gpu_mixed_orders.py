"""GPU parity of mixed orders m1, m2, m3 for h, u and E (paper Sec. 5; the
Sec. 6.1 rows with unequal orders; the Sec. 6.3 dam break with m3 = 0).
Same bars as the uniform-order entry points: 1e-13 for projections, 1e-12
for residuals, 1e-11 for Jacobian products, 1e-10 relative L2 after solves."""
import math

import numpy as np
import pytest

import workloads as wl
from _gpu_util import Pair, have_gpu, mesh_for, relerr
from test_gpu_parity import assert_preconditioner_matches, rel_l2_h_hu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

# dim, P, n, (m1, m2, m3)
CASES = [(1, 2, 257, (1, 2, 0)), (1, 3, 64, (3, 1, 2)), (1, 4, 40, (2, 2, 2)), (1, 1, 300, (1, 1, 0)),
         (2, 1, 13, (1, 1, 0)), (2, 2, 13, (1, 1, 0)), (2, 3, 11, (2, 3, 1)), (2, 3, 11, (3, 2, 2))]


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_11238_amd import bsw
    c = bsw.Context(0)
    yield c
    c.close()


def pair(ctx, dim, P, n, orders, precision=0):
    xy, e2v = mesh_for(dim, n)
    pr = Pair(ctx, dim, P, xy, e2v, precision)
    pr.disc.set_orders(*orders)
    pr.orc.set_orders(*orders)
    return pr


@pytest.mark.parametrize("dim,P,n,orders", CASES)
def test_projection_with_mixed_orders(ctx, dim, P, n, orders):
    pr = pair(ctx, dim, P, n, orders)
    for ic in (wl.IC(kind=wl.IC_MOUND, a=1.0, b=0.5, x0=4.0, y0=10.0, d=4.0),
               wl.IC(kind=wl.IC_DISK, a=2.0, b=0.5, x0=5.0, y0=10.0, r=2.5),
               wl.IC(kind=wl.IC_SINE_U, a=1.0, b=0.3, L=10.0)):
        Wg = pr.host(pr.disc.project_ic(ic))
        Wo = pr.orc.project_ic(ic)
        assert np.abs(Wg - Wo).max() <= 1e-13 * np.abs(Wo).max()
        m1, m2, _ = orders
        nm = (lambda m: m + 1) if dim == 1 else (lambda m: (m + 1) * (m + 2) // 2)
        assert np.all(Wg[0, nm(m1):] == 0.0) and np.all(Wg[1:1 + dim, nm(m2):] == 0.0)


@pytest.mark.parametrize("dim,P,n,orders", CASES)
@pytest.mark.parametrize("reg", [1, 3])
def test_operator_jacobian_and_blocks_with_mixed_orders(ctx, dim, P, n, orders, reg):
    from paper_2301_11238_amd import bsw
    pr = pair(ctx, dim, P, n, orders)
    p = wl.Params(g=9.81, rho=1000.0, alpha=0.12, eta=0.8, sigma0=40.0, gamma=1e3, beta=1e3, reg=reg)
    cp = bsw.make_params(p)
    W = wl.random_state(dim, P, pr.disc.n_el, 700 + reg)
    Wold = wl.random_state(dim, P, pr.disc.n_el, 800 + reg)
    dt = 0.0137
    bg = pr.disc.step_begin(cp, dt, pr.dev(Wold))
    bo = pr.orc.step_begin(p, Wold, dt)
    Rg = pr.host(pr.disc.operator_apply(cp, dt, pr.dev(W), bg))
    Ro = pr.orc.residual(p, W, bo, dt)
    assert relerr(Rg, Ro) <= 1e-12
    pr.disc.jacobian_linearize(cp, dt, pr.dev(W))
    x = wl.random_vector(dim, P, pr.disc.n_el, 901)
    yg = pr.host(pr.disc.jacobian_apply(pr.dev(x)))
    yo = pr.orc.jac_apply(p, W, x, dt)
    assert relerr(yg, yo) <= 1e-11
    Bg = pr.host(pr.disc.jacobian_blocks())
    Bo = pr.orc.jac_blocks(p, W, dt)
    assert np.abs(Bg - Bo).max() <= 1e-12 * np.abs(Bo).max()
    assert_preconditioner_matches(pr, dim, x, Bo)


def test_orders_are_checked_and_reset_the_linearisation(ctx):
    from paper_2301_11238_amd import bsw
    pr = pair(ctx, 2, 2, 5, (2, 2, 2))
    p = bsw.make_params(wl.Params(alpha=0.1, eta=1.0, sigma0=10.0, gamma=100.0, beta=100.0, reg=1))
    W = pr.dev(wl.random_state(2, 2, pr.disc.n_el, 3))
    pr.disc.jacobian_linearize(p, 0.01, W)
    pr.disc.set_orders(1, 1, 0)
    with pytest.raises(bsw.BswError):
        pr.disc.jacobian_apply(W)
    with pytest.raises(bsw.BswError):
        pr.disc.set_orders(3, 1, 1)
    with pytest.raises(bsw.BswError):
        pr.disc.set_orders(1, -1, 1)


def test_dam_break_with_piecewise_constant_E(ctx):
    """Sec. 6.3 set-up (Table damBreakFuns): L = 3, dam at 1.5 m, depths
    1.5 / 0.5, n_el = 100, m1 = m2 = 1, m3 = 0, sigma0 = 0.2, eta = 0.02,
    gamma = beta = 1e2, rho = 1, walls; 20 steps of 1e-5 s (the paper takes
    1e-6 s steps; at CFL-sized steps of ~1e-3 s Newton caps on this case,
    in the oracle's exact form too)."""
    import oracle
    from paper_2301_11238_amd import bsw
    xy, e2v = wl.mesh_1d(100, 0.0, 3.0)
    p = wl.Params(g=9.81, rho=1.0, alpha=0.0, eta=0.02, sigma0=0.2, gamma=1e2, beta=1e2, reg=1)
    ic = wl.IC(kind=wl.IC_STEP_X, a=1.5, b=0.5, x0=1.5)
    orc = oracle.Oracle(1, 1, xy, e2v)
    orc.set_orders(1, 1, 0)
    Wo, so = orc.solve(p, orc.project_ic(ic), oracle.SolveOptions(t_end=2e-4, dt_override=1e-5))
    for prec, bar in ((bsw.BSW_FP64, 1e-10), (bsw.BSW_FP32, 1e-5)):
        pr = Pair(ctx, 1, 1, xy, e2v, prec)
        pr.disc.set_orders(1, 1, 0)
        Wd = pr.disc.project_ic(ic)
        st = pr.disc.solve(bsw.make_params(p), bsw.Options(t_end=2e-4, dt=1e-5), Wd)
        W = pr.host(Wd)
        assert st["capped"] == 0 and so["capped"] == 0 and st["steps"] == so["steps"]
        eh, eq = rel_l2_h_hu(orc, W, Wo)
        assert eh <= bar and eq <= bar, (prec, eh, eq)
        assert np.all(W[2, 1:] == 0.0)


def test_unbalanced_lake_row_matches_oracle(ctx):
    """Sec. 6.1 shaded row (m0, m1, m2, m3) = (2, 1, 1, 1) on order-2 storage:
    the state moves and the GPU follows the oracle over ten steps."""
    import oracle
    from paper_2301_11238_amd import bsw
    alpha = math.pi / 18
    xy, e2v = wl.mesh_1d(100, 0.0, 10.0)
    # rho = 1000 (not the table's 1): with rho = 1 the viscous term is too stiff
    # for block-Jacobi GMRES (the oracle's own GMRES path caps there as well)
    p = wl.Params(g=9.81, rho=1000.0, alpha=alpha, eta=1.0, sigma0=1.0, gamma=1e3, beta=1e3, reg=1)
    bed = wl.Bed(kind=wl.BED_COS, order=2, a=1.0, kx=math.pi)
    ic = wl.IC(kind=wl.IC_SURFACE, a=3.0 / math.cos(alpha), b=-math.tan(alpha))
    pr = Pair(ctx, 1, 2, xy, e2v)
    pr.disc.set_orders(1, 1, 1)
    pr.orc.set_orders(1, 1, 1)
    pr.disc.set_bed(pr.disc.bed_interpolate(bed))
    pr.orc.set_bed(pr.orc.bed_interpolate(bed))
    W0 = pr.orc.project_ic(ic)
    Wd = pr.disc.project_ic(ic)
    assert np.abs(pr.host(Wd) - W0).max() <= 1e-13 * np.abs(W0).max()
    Wo, so = pr.orc.solve(p, W0, oracle.SolveOptions(t_end=0.1, dt_override=0.01))
    # near-exact Newton systems (tight forcing term), as the oracle solves them
    st = pr.disc.solve(bsw.make_params(p), bsw.Options(t_end=0.1, dt=0.01, forcing_max=1e-8, gmres_rtol=1e-12), Wd)
    W = pr.host(Wd)
    assert st["steps"] == so["steps"] == 10 and st["capped"] == 0 and so["capped"] == 0
    assert st["newton_total"] > 0
    eh, eq = rel_l2_h_hu(pr.orc, W, Wo)
    assert eh <= 1e-10 and eq <= 1e-9, (eh, eq)   # h u is the drift, ~30x below h
    assert np.abs(pr.orc.eval_points(Wo)[:, :, 1]).max() > 1e-3
    assert np.all(W[:, 2] == 0.0)


def test_served_mixed_orders_match_oracle_and_mix(ctx):
    """Served 2-D solves with m1 = m2 = 1, m3 = 0 on order-2 storage follow
    the oracle and are bitwise the same alone and batched with uniform ones."""
    import oracle
    from paper_2301_11238_amd import bsw
    slope = math.atan(0.1)
    p = wl.Params(g=9.81, rho=1000.0, alpha=slope, eta=1.0, sigma0=40.0, gamma=100.0, beta=100.0, reg=1)
    mound = wl.IC(kind=wl.IC_MOUND, a=1.0, b=0.5, x0=10.0, y0=10.0, d=4.0)
    xy, e2v = mesh_for(2, 8)
    orc = oracle.Oracle(2, 2, xy, e2v)
    orc.set_orders(1, 1, 0)
    Wo, so = orc.solve(p, orc.project_ic(mound), oracle.SolveOptions(t_end=0.1, cfl=0.2))
    xy7, e7 = mesh_for(2, 7)
    mixed = ((xy, e2v, 2, bsw.BSW_FP64, bsw.make_params(p)),
             dict(ic=mound, opts=bsw.Options(t_end=0.1, cfl=0.2), orders=(1, 1, 0)))
    other = ((xy7, e7, 2, bsw.BSW_FP64, bsw.make_params(p)), dict(ic=mound, opts=bsw.Options(t_end=0.1, cfl=0.2)))

    def serve(reqs):
        srv = bsw.Server(ctx, 1 << 31, 16)
        try:
            ts = [srv.submit(*a, **k) for a, k in reqs]
            out = []
            for t in ts:
                assert srv.wait(t, 300.0) == bsw.BSW_REQ_DONE
                out.append(srv.fetch(t))
            return out
        finally:
            srv.close()

    (Wa, sa), = serve([mixed])
    (Wm, sm), _ = serve([mixed, other])
    assert np.array_equal(Wa, Wm) and sa["newton_total"] == sm["newton_total"]
    assert sa["capped"] == 0 and so["capped"] == 0 and sa["steps"] == so["steps"]
    eh, eq = rel_l2_h_hu(orc, Wa, Wo)
    assert eh <= 1e-10 and eq <= 1e-10, (eh, eq)
    srv = bsw.Server(ctx, 1 << 30, 4)
    try:
        a, k = mixed
        k = dict(k, orders=(3, 1, 1))
        with pytest.raises(bsw.BswError):
            srv.submit(*a, **k)
    finally:
        srv.close()

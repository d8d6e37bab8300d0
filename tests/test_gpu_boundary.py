"""GPU parity of per-face boundary conditions (paper Sec. 5.2; the Dirichlet
ends of Sec. 6.1 and the Neumann / no-flow ends of Sec. 6.2): residual,
Jacobian product and blocks with random mixes of wall, Neumann and tagged
Dirichlet faces, whole solves with the paper's end conditions, and served
requests carrying face codes.  Bars as for the other entry points."""
import math

import numpy as np
import pytest

import workloads as wl
from _gpu_util import Pair, have_gpu, mesh_for, relerr
from test_gpu_parity import assert_preconditioner_matches, rel_l2_h_hu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

ALPHA = math.pi / 18
CASES = [(1, 1, 300), (1, 3, 64), (2, 1, 13), (2, 2, 13), (2, 3, 11)]


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_11238_amd import bsw
    c = bsw.Context(0)
    yield c
    c.close()


def states(dim):
    nf = 1 + dim + dim * dim
    base = [[1.1, 0.3, -0.2, 0.01, 0.02, -0.03, 0.04], [0.7, -0.5, 0.1, 0.0, 0.03, 0.0, -0.02],
            [1.6, 0.05, 0.4, -0.02, 0.0, 0.01, 0.0], [0.9, 0.2, 0.2, 0.0, 0.0, 0.0, 0.0]]
    return [s[:nf] for s in base]


@pytest.mark.parametrize("dim,P,n", CASES)
@pytest.mark.parametrize("default_bc", [1, 3])
def test_operator_and_jacobian_with_face_codes(ctx, dim, P, n, default_bc):
    from paper_2301_11238_amd import bsw
    xy, e2v = mesh_for(dim, n)
    pr = Pair(ctx, dim, P, xy, e2v)
    rng = np.random.default_rng(40 + dim * 10 + P)
    codes = (rng.integers(0, 4, size=(pr.disc.n_el, dim + 1)) |
             rng.integers(0, 4, size=(pr.disc.n_el, dim + 1)) << 2).astype(np.int8)
    st = states(dim)
    pr.mesh.set_boundary(codes)
    pr.orc.set_boundary(codes, dirichlet_tags=st[1:])
    p = wl.Params(g=9.81, rho=1000.0, alpha=0.12, eta=0.8, sigma0=40.0, gamma=1e3, beta=1e3, reg=1)
    cp = bsw.make_params(p, bc=default_bc, dirichlet=st[0], dirichlet_tags=st[1:])
    W = wl.random_state(dim, P, pr.disc.n_el, 51)
    dt = 0.017
    bo = pr.orc.step_begin(p, W * 0.9, dt)
    Rg = pr.host(pr.disc.operator_apply(cp, dt, pr.dev(W), pr.dev(bo[: 1 + dim])))
    Ro = pr.orc.residual(p, W, bo, dt, bc=default_bc, dirichlet=st[0])
    assert relerr(Rg, Ro) <= 1e-12
    pr.disc.jacobian_linearize(cp, dt, pr.dev(W))
    x = wl.random_vector(dim, P, pr.disc.n_el, 52)
    yg = pr.host(pr.disc.jacobian_apply(pr.dev(x)))
    yo = pr.orc.jac_apply(p, W, x, dt, bc=default_bc, dirichlet=st[0])
    assert relerr(yg, yo) <= 1e-11
    Bg = pr.host(pr.disc.jacobian_blocks())
    Bo = pr.orc.jac_blocks(p, W, dt, bc=default_bc, dirichlet=st[0])
    assert np.abs(Bg - Bo).max() <= 1e-12 * np.abs(Bo).max()
    # the block solve with these faces (on triangles the stress rows of the
    # block solve are formed from the faces' kinds)
    assert_preconditioner_matches(pr, dim, x, Bo)
    # the codes changed the result, and resetting them restores the default
    pr.mesh.set_boundary(None)
    R0 = pr.host(pr.disc.operator_apply(cp, dt, pr.dev(W), pr.dev(bo[: 1 + dim])))
    assert relerr(R0, Ro) > 1e-8
    pr.orc.set_boundary(None)
    assert relerr(R0, pr.orc.residual(p, W, bo, dt, bc=default_bc, dirichlet=st[0])) <= 1e-12
    with pytest.raises(bsw.BswError):
        pr.mesh.set_boundary(np.full(codes.shape, 17, np.int8))


def ends(n_el, left, right):
    c = np.zeros((n_el, 2), np.int8)
    c[0, 0] = left
    c[-1, 1] = right
    return c


@pytest.mark.parametrize("P", [1, 2])
def test_lake_kept_by_the_papers_dirichlet_ends(ctx, P):
    """Sec. 6.1 with its Dirichlet data at x = 0 and x = L: no Newton
    iteration is needed and the FP64 state does not change."""
    from paper_2301_11238_amd import bsw
    L, h0 = 10.0, 3.0
    xy, e2v = wl.mesh_1d(100, 0.0, L)
    pr = Pair(ctx, 1, P, xy, e2v)
    bed = wl.Bed(kind=wl.BED_COS, order=P, a=1.0, kx=math.pi)
    pr.disc.set_bed(pr.disc.bed_interpolate(bed))
    hL = h0 / math.cos(ALPHA) - 1.0
    hR = h0 / math.cos(ALPHA) - L * math.tan(ALPHA) - math.cos(math.pi * L)
    pr.mesh.set_boundary(ends(100, 3 | 1 << 2, 3 | 2 << 2))
    prm = wl.Params(g=9.81, rho=1.0, alpha=ALPHA, eta=1.0, sigma0=1.0, gamma=1e3, beta=1e3, reg=1)
    cp = bsw.make_params(prm, bc=1, dirichlet_tags=[[hL, 0.0, 0.0], [hR, 0.0, 0.0]])
    Wd = pr.disc.project_ic(wl.IC(kind=wl.IC_SURFACE, a=h0 / math.cos(ALPHA), b=-math.tan(ALPHA)))
    W0 = pr.host(Wd).copy()
    st = pr.disc.solve(cp, bsw.Options(t_end=0.05, dt=0.01), Wd)
    assert st["steps"] == 5 and st["newton_total"] == 0
    assert np.array_equal(pr.host(Wd), W0)


@pytest.mark.parametrize("precision,bar", [(0, 1e-10), (1, 1e-5)])
def test_open_and_closed_ends_solve_matches_oracle(ctx, precision, bar):
    """Sec. 6.2 end conditions (Neumann at x = 0, no-flow wall at x = L) on a
    case that moves: yield stress per density 2 m^2/s^2, below the threshold,
    20 steps.  rho = 1000 with sigma0 = 2000 Pa keeps sigma0 / rho of a
    rho = 1 run but divides the regularised slope 2 gamma / rho by 1000; at
    rho = 1 the Newton systems are too stiff for block-Jacobi GMRES."""
    import oracle
    from paper_2301_11238_amd import bsw
    xy, e2v = wl.mesh_1d(60, 0.0, 10.0)
    codes = ends(60, 2, 1)
    bed = wl.Bed(kind=wl.BED_COS, order=1, a=1.0, kx=math.pi)
    ic = wl.IC(kind=wl.IC_SURFACE, a=3.0, b=0.0)
    prm = wl.Params(g=9.81, rho=1000.0, alpha=ALPHA, eta=1.0, sigma0=2000.0, gamma=1e2, beta=1e2, reg=1)
    orc = oracle.Oracle(1, 1, xy, e2v)
    orc.set_bed(orc.bed_interpolate(bed))
    orc.set_boundary(codes)
    Wo, so = orc.solve(prm, orc.project_ic(ic), oracle.SolveOptions(t_end=0.2, dt_override=0.01))
    pr = Pair(ctx, 1, 1, xy, e2v, precision)
    pr.disc.set_bed(pr.disc.bed_interpolate(bed))
    pr.mesh.set_boundary(codes)
    Wd = pr.disc.project_ic(ic)
    st = pr.disc.solve(bsw.make_params(prm, bc=3), bsw.Options(t_end=0.2, dt=0.01), Wd)
    W = pr.host(Wd)
    assert so["capped"] == 0 and st["capped"] == 0 and st["steps"] == so["steps"] == 20
    assert np.abs(orc.eval_points(Wo)[:, :, 1]).max() > 0.1
    eh, eq = rel_l2_h_hu(orc, W, Wo)
    assert eh <= bar and eq <= bar, (eh, eq)


def test_served_request_with_face_codes(ctx):
    """A served 2-D request with Dirichlet inflow tags on part of the boundary
    and walls elsewhere follows the oracle; bad codes are refused."""
    import oracle
    from paper_2301_11238_amd import bsw
    xy, e2v = mesh_for(2, 8)
    n_el = e2v.shape[0]
    orc = oracle.Oracle(2, 2, xy, e2v)
    md = orc.mesh_data()
    codes = np.zeros((n_el, 3), np.int8)
    bnd = md["nbr"] < 0
    # x = 0 side: Dirichlet tag 1 (a slow inflow of the ambient depth); others walls
    left = bnd & (md["normal"][:, :, 0] < -0.9)
    codes[bnd] = 1
    codes[left] = 3 | 1 << 2
    inflow = [1.0, 0.2, 0.0, 0.0, 0.0, 0.0, 0.0]
    orc.set_boundary(codes, dirichlet_tags=[inflow])
    prm = wl.Params(g=9.81, rho=1000.0, alpha=0.0, eta=1.0, sigma0=20.0, gamma=100.0, beta=100.0, reg=2)
    ic = wl.IC(kind=wl.IC_CONST, a=1.0)
    Wo, so = orc.solve(prm, orc.project_ic(ic), oracle.SolveOptions(t_end=0.1, cfl=0.2))
    srv = bsw.Server(ctx, 1 << 30, 4)
    try:
        t = srv.submit(xy, e2v, 2, bsw.BSW_FP64, bsw.make_params(prm, bc=1, dirichlet_tags=[inflow]), ic=ic,
                       opts=bsw.Options(t_end=0.1, cfl=0.2), face_bc=codes)
        assert srv.wait(t, 300.0) == bsw.BSW_REQ_DONE
        W, st = srv.fetch(t)
        bad = codes.copy()
        bad[0, 0] = 33
        with pytest.raises(bsw.BswError):
            srv.submit(xy, e2v, 2, bsw.BSW_FP64, bsw.make_params(prm), ic=ic, face_bc=bad)
    finally:
        srv.close()
    assert so["capped"] == 0 and st["capped"] == 0 and st["steps"] == so["steps"]
    eh, eq = rel_l2_h_hu(orc, W, Wo)
    assert eh <= 1e-10 and eq <= 1e-10, (eh, eq)
    assert np.abs(Wo[1]).max() > 1e-3   # the inflow moved the fluid

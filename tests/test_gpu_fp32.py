"""FP32-mixed path: FP32 state and flux/source arithmetic with FP64 reductions
(mass, norms, Krylov dot products) and the regularisation's small-shear branch
in FP64.  Bar: 1e-5 relative against the FP64 oracle, per apply and after
whole solves (relative L2 on h and h u)."""
import math

import numpy as np
import pytest

import workloads as wl
from _gpu_util import Pair, have_gpu, mesh_for, relerr
from test_gpu_parity import SOLVES, rel_l2_h_hu

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

CASES = [(1, 1, 300), (1, 2, 257), (2, 1, 13), (2, 2, 13), (2, 3, 11)]


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_11238_amd import bsw
    c = bsw.Context(0)
    yield c
    c.close()


def pair32(ctx, dim, P, n):
    xy, e2v = mesh_for(dim, n)
    return Pair(ctx, dim, P, xy, e2v, precision=1)


@pytest.mark.parametrize("dim,P,n", CASES)
@pytest.mark.parametrize("reg", [1, 2, 3])
def test_fp32_operator_and_jacobian(ctx, dim, P, n, reg):
    from paper_2301_11238_amd import bsw
    pr = pair32(ctx, dim, P, n)
    p = wl.Params(g=9.81, rho=1000.0, alpha=0.12, eta=0.8, sigma0=40.0, gamma=1e3, beta=1e3, reg=reg)
    W = wl.random_state(dim, P, pr.disc.n_el, 100 + reg)
    # compare on the float-rounded state, so only the arithmetic differs
    W = W.astype(np.float32).astype(np.float64)
    dt = 0.0137
    cp = bsw.make_params(p)
    bo = pr.orc.step_begin(p, W, dt)
    bg = pr.disc.step_begin(cp, dt, pr.dev(W))
    assert relerr(pr.host(bg), bo[: 1 + dim]) <= 1e-6
    Rg = pr.host(pr.disc.operator_apply(cp, dt, pr.dev(W), pr.dev(bo[: 1 + dim])))
    Ro = pr.orc.residual(p, W, bo, dt)
    assert relerr(Rg, Ro) <= 1e-5
    x = wl.random_vector(dim, P, pr.disc.n_el, 7).astype(np.float32).astype(np.float64)
    pr.disc.jacobian_linearize(cp, dt, pr.dev(W))
    yg = pr.host(pr.disc.jacobian_apply(pr.dev(x)))
    yo = pr.orc.jac_apply(p, W, x, dt)
    assert relerr(yg, yo) <= 1e-5


@pytest.mark.parametrize("case", SOLVES, ids=[c[0] for c in SOLVES])
def test_fp32_whole_solve(ctx, case):
    import oracle
    from paper_2301_11238_amd import bsw
    name, dim, P, n, reg, s0, eta, eps, alpha, ic, t_end = case
    pr = pair32(ctx, dim, P, n)
    p = wl.Params(g=9.81, rho=1000.0, alpha=alpha, eta=eta, sigma0=s0, gamma=1 / eps, beta=1 / eps, reg=reg)
    W0 = pr.orc.project_ic(ic)
    Wo, so = pr.orc.solve(p, W0, oracle.SolveOptions(t_end=t_end, cfl=0.2))
    Wd = pr.dev(W0)
    sg = pr.disc.solve(bsw.make_params(p), bsw.Options(t_end=t_end, cfl=0.2), Wd)
    assert sg["steps"] == so["steps"]
    eh, eq = rel_l2_h_hu(pr.orc, pr.host(Wd), Wo)
    assert eh <= 1e-5 and eq <= 1e-5, (eh, eq, sg)
    assert sg["max_mass_drift"] <= 1e-6

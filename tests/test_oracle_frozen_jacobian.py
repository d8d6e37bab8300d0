"""The paper-literal Jacobian (Appendix A holds the HLL wave speeds S_L, S_R
fixed when differentiating the face flux).  Pins: with every face upwind
(S_L >= 0 or S_R <= 0) it equals the exact Jacobian; in general it differs;
Newton with either Jacobian reaches the same root of the same residual."""
import dataclasses

import numpy as np

import oracle
import workloads as wl


def supercritical_1d(n=40, seed=3):
    xy, e2v = wl.mesh_1d(n, 0.0, 10.0)
    orc = oracle.Oracle(1, 2, xy, e2v)
    rng = np.random.default_rng(seed)
    W = np.zeros((3, 3, n))
    W[0, 0] = 0.1 * (1 + 0.05 * rng.standard_normal(n)) * np.sqrt(2.0)  # h ~ 0.1 (phi_0 = 1/sqrt2)
    W[1, 0] = 3.0 * np.sqrt(2.0)                                          # u ~ 3 > sqrt(g h) ~ 1
    W[:, 1:] = 1e-3 * rng.standard_normal((3, 2, n))
    return orc, W


def test_frozen_equals_exact_when_every_face_is_upwind():
    orc, W = supercritical_1d()
    p = wl.Params(eta=1.0, sigma0=5.0, gamma=100.0, beta=100.0, reg=1)
    x = np.random.default_rng(4).standard_normal(W.shape)
    ye = orc.jac_apply(p, W, x, 0.01, bc=2)
    yf = orc.jac_apply(dataclasses.replace(p, jac_frozen=1), W, x, 0.01, bc=2)
    assert np.abs(yf - ye).max() <= 1e-13 * np.abs(ye).max()


def test_frozen_differs_in_general_and_newton_reaches_the_same_root():
    xy, e2v = wl.mesh_1d(60, 0.0, 10.0)
    orc = oracle.Oracle(1, 1, xy, e2v)
    p = wl.Params(eta=1.0, sigma0=50.0, gamma=100.0, beta=100.0, reg=1)
    pf = dataclasses.replace(p, jac_frozen=1)
    W0 = orc.project_ic(wl.IC(kind=wl.IC_STEP_X, a=1.0, b=0.1, x0=5.0))
    x = np.random.default_rng(5).standard_normal(W0.shape)
    W1 = W0 + 0.01 * np.random.default_rng(6).standard_normal(W0.shape)
    ye = orc.jac_apply(p, W1, x, 0.01)
    yf = orc.jac_apply(pf, W1, x, 0.01)
    assert np.abs(yf - ye).max() > 1e-6 * np.abs(ye).max()
    We, se = orc.solve(p, W0, oracle.SolveOptions(t_end=0.03, cfl=0.2))
    # frozen speeds make Newton converge only linearly where the HLL flux is
    # in its middle branch: it needs more iterations (here beyond the paper's
    # 10), but reaches the same root of the same residual
    _, sf10 = orc.solve(pf, W0, oracle.SolveOptions(t_end=0.03, cfl=0.2))
    Wf, sf = orc.solve(pf, W0, oracle.SolveOptions(t_end=0.03, cfl=0.2, max_newton=60))
    assert se["capped"] == 0 and sf["capped"] == 0
    assert sf["newton_total"] > se["newton_total"] and sf10["capped"] > 0
    assert np.abs(Wf - We).max() <= 1e-9 * np.abs(We).max()

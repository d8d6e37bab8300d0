"""Continuation on the regularisation parameter (Sec. 6.3): per time step,
Newton solves at gamma_i = gamma0 + (i - 1)(gamma - gamma0)/(n - 1), each from
the previous one.  Pins: the degenerate ramp gamma0 = gamma is plain Newton;
where plain Newton caps, the ramp converges, and the root it reaches at the
target gamma does not depend on the ramp (gamma0, n)."""
import numpy as np
import pytest

import oracle
import workloads as wl


def dam_break_1d(sigma0=20.0, eta=0.1, eps=1e-3, reg=1, n=100):
    xy, e2v = wl.mesh_1d(n, 0.0, 10.0)
    prm = wl.Params(g=9.81, rho=1000.0, alpha=0.0, eta=eta, sigma0=sigma0, gamma=1 / eps, beta=1 / eps, reg=reg)
    ic = wl.IC(kind=wl.IC_STEP_X, a=1.0, b=0.1, x0=5.0)
    orc = oracle.Oracle(1, 1, xy, e2v)
    return orc, prm, orc.project_ic(ic)


def test_degenerate_ramp_is_plain_newton():
    orc, prm, W0 = dam_break_1d(sigma0=50.0, eta=1.0, eps=1e-2)
    # Newton on the update test alone (res_tol off), so the count is exact
    W1, s1 = orc.solve(prm, W0, oracle.SolveOptions(t_end=0.03, cfl=0.2, res_tol=-1.0))
    rec = []
    W2, s2 = orc.solve(prm, W0, oracle.SolveOptions(t_end=0.03, cfl=0.2, cont_steps=3, cont_gamma0=prm.gamma,
                                                    res_tol=-1.0), record=rec)
    assert s1["capped"] == 0 and s2["capped"] == 0
    assert np.abs(W2 - W1).max() <= 1e-12 * np.abs(W1).max()
    # stages 2 and 3 start at the converged state: one Newton iteration each
    assert s2["newton_total"] == s1["newton_total"] + 2 * s1["steps"]


def test_ramp_converges_where_plain_newton_caps():
    orc, prm, W0 = dam_break_1d()
    _, plain = orc.solve(prm, W0, oracle.SolveOptions(t_end=0.05, cfl=0.2))
    assert plain["capped"] > 0
    Wa, a = orc.solve(prm, W0, oracle.SolveOptions(t_end=0.05, cfl=0.2, cont_steps=3, cont_gamma0=prm.gamma / 100))
    Wb, b = orc.solve(prm, W0, oracle.SolveOptions(t_end=0.05, cfl=0.2, cont_steps=5, cont_gamma0=prm.gamma / 100))
    Wc, c = orc.solve(prm, W0, oracle.SolveOptions(t_end=0.05, cfl=0.2, cont_steps=3, cont_gamma0=prm.gamma / 30))
    assert a["capped"] == 0 and b["capped"] == 0 and c["capped"] == 0
    # the same root at the target gamma, whatever the ramp
    for W in (Wb, Wc):
        assert np.abs(W - Wa).max() <= 1e-9 * np.abs(Wa).max()
    assert a["max_mass_drift"] <= 1e-12

"""Pins of the oracle's time-step rule, diagnostics and C Krylov solve path.

Each expected value below comes from a closed form or an independent
computation, not from the oracle:
  * the fixed step dt = CFL h_min / max(|u| + sqrt(g h)) (Sec. 6 examples,
    CFL rule of the scope table) on the 1-D dam break and on a hand-measured
    two-triangle mesh (h_min = the smallest altitude 2 |K| / side);
  * active% = 100 / |Omega| int H(|E| - sigma0 / gamma) (Sec. 6) on a
    piecewise-constant strain rate whose active set is known element by
    element, with groups on both sides of the threshold within a factor 1.2,
    so a threshold or shear-rate scale off by sqrt(2) or 2 fails;
  * the C path (restarted block-Jacobi GMRES inside Newton, and its time loop)
    against the exact sparse-LU Newton of the Python front end.
"""
import math

import numpy as np
import pytest

import workloads as wl

G = 9.81


def test_c1_time_step_and_step_count(oracle_mod):
    """Dam break C1: 200 elements of 0.05 m, h = 1 | 0.1 with the jump on a
    face, u = 0: lambda0 = sqrt(g 1), dt = 0.2 * 0.05 / sqrt(9.81) =
    3.192754e-3 s, 314 steps to t = 1 (the last one clipped)."""
    pb = wl.config1(wl.REG1)
    orc = oracle_mod.Oracle(1, 1, pb.xy, pb.el2vert)
    W0 = orc.project_ic(pb.ic)
    dt_closed = 0.2 * 0.05 / math.sqrt(G)
    assert abs(dt_closed - 3.192754e-3) < 1e-9
    dt = orc.cfl_dt(pb.params, W0, 0.2)
    assert abs(dt - dt_closed) <= 1e-13 * dt_closed
    assert math.ceil(1.0 / dt - 1e-12) == 314
    d = orc.diagnostics(pb.params, W0)
    assert abs(d["lambda_max"] - math.sqrt(G)) < 1e-13
    assert abs(d["mass"] - (5.0 * 1.0 + 5.0 * 0.1)) < 1e-12
    # the C time loop takes the same step and clips the last one onto t_end
    o = oracle_mod.SolveOptions(t_end=3.5 * dt_closed, max_newton=3)
    _, st = orc.solve(pb.params, W0, o, linear="gmres")
    assert st["steps"] == 4 and abs(st["dt"] - dt_closed) <= 1e-13 * dt_closed
    assert abs(st["t_end"] - 3.5 * dt_closed) < 1e-15
    _, st2 = orc.solve(pb.params, W0, o)
    assert st2["steps"] == 4 and abs(st2["t_end"] - 3.5 * dt_closed) < 1e-15


TWO_TRI_XY = np.array([[0.0, 0.0], [2.0, 0.0], [0.0, 1.0], [2.5, 1.5]])
TWO_TRI_E2V = np.array([[0, 1, 2], [1, 3, 2]], np.int32)


def _altitudes(xy, tri):
    p = xy[tri]
    area = 0.5 * abs((p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[1, 1] - p[0, 1]) * (p[2, 0] - p[0, 0]))
    sides = [np.linalg.norm(p[(k + 1) % 3] - p[k]) for k in range(3)]
    return area, [2.0 * area / s for s in sides]


def test_two_triangle_altitude_and_wave_speed(oracle_mod):
    # by hand: triangle 0 (legs 2 and 1, area 1) has altitudes 1, 2/sqrt5, 2;
    # triangle 1 (area 7/4) has altitudes 3.5/sqrt2.5, 3.5/sqrt6.5, 3.5/sqrt5
    a0, h0 = _altitudes(TWO_TRI_XY, TWO_TRI_E2V[0])
    a1, h1 = _altitudes(TWO_TRI_XY, TWO_TRI_E2V[1])
    assert abs(a0 - 1.0) < 1e-15 and abs(a1 - 1.75) < 1e-15
    assert abs(min(h0) - 2.0 / math.sqrt(5.0)) < 1e-15 and min(h1) > min(h0)
    hmin = 2.0 / math.sqrt(5.0)
    for P in (1, 2, 3):
        orc = oracle_mod.Oracle(2, P, TWO_TRI_XY, TWO_TRI_E2V)
        md = orc.mesh_data()
        assert abs(md["hmin"] - hmin) < 1e-15
        assert abs(md["measure"] - 2.75) < 1e-14
        prm = wl.Params(g=G, eta=1.0, sigma0=10.0, gamma=1e3, beta=1e3)
        W0 = orc.project_ic(wl.IC(kind=wl.IC_CONST, a=2.0, b=0.3, c=-0.4))
        lam = 0.5 + math.sqrt(G * 2.0)
        d = orc.diagnostics(prm, W0)
        assert abs(d["lambda_max"] - lam) < 1e-13
        assert abs(d["mass"] - 2.0 * 2.75) < 1e-13
        assert abs(d["h_min"] - 2.0) < 1e-13
        dt = orc.cfl_dt(prm, W0, 0.2)
        assert abs(dt - 0.2 * hmin / lam) <= 1e-14 * dt


def _piecewise_strain(n_el, nf, np_, values, comp, phi0):
    """State with h = 1, u = 0 and one strain component constant per element
    (value values[e]); phi0 is the constant mode of the orthonormal basis,
    1 / sqrt(|reference element|)."""
    W = np.zeros((nf, np_, n_el))
    W[0, 0] = 1.0 / phi0
    W[comp, 0] = np.asarray(values) / phi0
    return W


# strain rates as multiples of the threshold sigma0 / gamma: pairs straddle it
# within a factor 1.2, so any factor-sqrt(2) error in s or the threshold moves
# at least one group across
RATIOS = (0.25, 0.6, 0.85, -0.9, 1.1, -1.15, 1.3, 1.7, 2.6, 0.4)


def test_active_fraction_1d(oracle_mod):
    n = len(RATIOS)
    xy = np.concatenate([[0.0], np.cumsum(np.linspace(0.5, 1.5, n))]).reshape(-1, 1)
    e2v = np.stack([np.arange(n), np.arange(1, n + 1)], 1).astype(np.int32)
    orc = oracle_mod.Oracle(1, 2, xy, e2v)
    prm = wl.Params(sigma0=40.0, gamma=1e3, beta=1e3, reg=1)
    thr = prm.sigma0 / prm.gamma
    W = _piecewise_strain(n, 3, 3, [r * thr for r in RATIOS], 2, 1.0 / math.sqrt(2.0))
    lengths = np.diff(xy[:, 0])
    act = sum(L for L, r in zip(lengths, RATIOS) if abs(r) >= 1.0)
    d = orc.diagnostics(prm, W)
    assert abs(d["active_pct"] - 100.0 * act / lengths.sum()) < 1e-10
    assert 20.0 < d["active_pct"] < 80.0
    assert abs(d["mass"] - lengths.sum()) < 1e-12


@pytest.mark.parametrize("comp", [3, 6])
def test_active_fraction_2d(oracle_mod, comp):
    # E11 alone (comp 3) or E22 alone (comp 6): D = E, tr D = e, so
    # ||D||_c^2 = 2 e^2 and s = |e|, the 1-D shear rate (Sec. 4, 2-D reading)
    xy, e2v = wl.mesh_tri(4, 20.0, 20.0, 0.1, 7)
    n = e2v.shape[0]
    ratios = [RATIOS[k % len(RATIOS)] for k in range(n)]
    orc = oracle_mod.Oracle(2, 2, xy, e2v)
    prm = wl.Params(sigma0=25.0, gamma=1e4, beta=1e4, reg=3)
    thr = prm.sigma0 / prm.gamma
    W = _piecewise_strain(n, 7, 6, [r * thr for r in ratios], comp, math.sqrt(2.0))
    areas = np.array([_altitudes(xy, t)[0] for t in e2v])
    act = areas[np.abs(ratios) >= 1.0].sum()
    d = orc.diagnostics(prm, W)
    assert abs(d["active_pct"] - 100.0 * act / 400.0) < 1e-10
    assert abs(areas.sum() - 400.0) < 1e-10


def test_active_fraction_simple_shear(oracle_mod):
    # simple shear E12 = e (du2/dx1 = e): D has off-diagonal e/2, tr D = 0,
    # ||D||_c^2 = e^2 / 2 and s = |e| / 2, half the 1-D rate of the same entry
    xy, e2v = wl.mesh_tri(3, 20.0, 20.0, 0.1, 9)
    n = e2v.shape[0]
    ratios = [RATIOS[k % len(RATIOS)] * 2.0 for k in range(n)]
    orc = oracle_mod.Oracle(2, 1, xy, e2v)
    prm = wl.Params(sigma0=25.0, gamma=1e4, beta=1e4, reg=2)
    thr = prm.sigma0 / prm.gamma
    W = _piecewise_strain(n, 7, 3, [r * thr for r in ratios], 5, math.sqrt(2.0))
    areas = np.array([_altitudes(xy, t)[0] for t in e2v])
    act = areas[np.abs(ratios) >= 2.0].sum()
    d = orc.diagnostics(prm, W)
    assert abs(d["active_pct"] - 100.0 * act / 400.0) < 1e-10


def _incline_case(oracle_mod, N=5, P=2, reg=1, eps=1e-2):
    pb = wl.config2(reg, eps, N=N, seed=2)
    orc = oracle_mod.Oracle(2, P, pb.xy, pb.el2vert)
    return pb, orc, orc.project_ic(pb.ic)


@pytest.mark.parametrize("reg", [1, 3])
def test_c_gmres_newton_matches_direct(oracle_mod, reg):
    """The C Newton step with block-Jacobi GMRES(30) reaches the same root as
    Newton with exact sparse-LU solves (same iteration count, states within
    the Newton and Krylov tolerances)."""
    pb, orc, W0 = _incline_case(oracle_mod, reg=reg)
    dt = orc.cfl_dt(pb.params, W0, 0.2)
    b = orc.step_begin(pb.params, W0, dt)
    o = oracle_mod.SolveOptions(newton_tol=1e-11, gmres_rtol=1e-13, res_tol=-1.0)
    Wd, sd = orc.newton_step(pb.params, W0, b, dt, o, linear="direct")
    Wg, sg = orc.newton_step(pb.params, W0, b, dt, o, linear="gmres")
    assert sd["converged"] and sg["converged"]
    assert sg["gmres"] > 0
    assert abs(sd["newton"] - sg["newton"]) <= 1
    assert np.abs(Wg - Wd).max() <= 1e-9 * np.abs(Wd).max()
    R = orc.residual(pb.params, Wg, b, dt)
    assert np.linalg.norm(R) <= 1e-9 * np.linalg.norm(b)


def test_c_solve_loop_matches_direct(oracle_mod):
    """The C time loop (fixed CFL step, Newton per step, diagnostics) against
    the Python loop with exact solves: same step, step count, Newton counts
    within one, mass drift at the Krylov tolerance, same final state."""
    pb, orc, W0 = _incline_case(oracle_mod, N=4, P=2, reg=2, eps=1e-2)
    o = oracle_mod.SolveOptions(t_end=1.0, max_steps=3, newton_tol=1e-11, gmres_rtol=1e-13)
    Wg, sg = orc.solve(pb.params, W0, o, linear="gmres")
    Wd, sd = orc.solve(pb.params, W0, o)
    assert sg["steps"] == sd["steps"] == 3 and sg["dt"] == sd["dt"]
    assert sg["capped"] == sd["capped"] == 0
    assert abs(sg["newton_total"] - sd["newton_total"]) <= 3
    assert sg["max_mass_drift"] < 1e-11 and sd["max_mass_drift"] < 1e-12
    assert abs(sg["mass0"] - sd["mass0"]) < 1e-12 * sd["mass0"]
    assert np.abs(Wg - Wd).max() <= 1e-9 * np.abs(Wd).max()
    # a planted mistake the comparison catches: one step fewer differs
    o1 = oracle_mod.SolveOptions(t_end=1.0, max_steps=2, newton_tol=1e-11, gmres_rtol=1e-13)
    W2, _ = orc.solve(pb.params, W0, o1, linear="gmres")
    assert np.abs(W2 - Wd).max() > 1e-6 * np.abs(Wd).max()


def test_c1_newton_record(oracle_mod):
    """Newton on the first dam-break step (C1, regularisation 1, gamma = 1e3)
    from W_old with exact solves: capped at the paper's 10 iterations, it
    converges quadratically after about 20 (the paper reports the same
    difficulty for regularisations 1 and 2 at gamma = 1e3, Sec. 6.3).  The
    converged step keeps the mass to rounding."""
    pb = wl.config1(wl.REG1)
    orc = oracle_mod.Oracle(1, 1, pb.xy, pb.el2vert)
    W0 = orc.project_ic(pb.ic)
    dt = orc.cfl_dt(pb.params, W0, 0.2)
    b = orc.step_begin(pb.params, W0, dt)
    W10, s10 = orc.newton_step(pb.params, W0, b, dt, oracle_mod.SolveOptions(max_newton=10))
    assert not s10["converged"] and s10["newton"] == 10
    W40, s40 = orc.newton_step(pb.params, W0, b, dt, oracle_mod.SolveOptions(max_newton=40))
    assert s40["converged"] and 15 <= s40["newton"] <= 30
    m0 = orc.diagnostics(pb.params, W0)["mass"]
    assert abs(orc.diagnostics(pb.params, W40)["mass"] - m0) < 1e-13 * m0
    assert abs(orc.diagnostics(pb.params, W10)["mass"] - m0) < 1e-13 * m0


@pytest.mark.parametrize("dim,P", [(1, 2), (2, 1), (2, 3)])
@pytest.mark.parametrize("reg", [1, 3])
def test_jacobian_block_structure(oracle_mod, dim, P, reg):
    """The diagonal Jacobian blocks have the structure the block-Jacobi
    preconditioner's Schur form relies on (Sec. 3, the mixed form of the
    strain rate): the stress rows' own block is the element mass matrix
    |J| I of the orthonormal basis (|J| = length / 2 on an interval, twice
    the area on a triangle, measured here from the vertices), the depth rows
    do not involve E and the stress rows do not involve h.  The Schur
    complement solve then equals the direct block solve."""
    xy, e2v = wl.mesh_1d(7) if dim == 1 else wl.mesh_tri(3)
    orc = oracle_mod.Oracle(dim, P, xy, e2v)
    p = wl.Params(alpha=0.12, eta=0.8, sigma0=40.0, gamma=1e3, beta=1e3, reg=reg)
    W = wl.random_state(dim, P, orc.n_el, 11)
    B = orc.jac_blocks(p, W, 0.02)
    npm = wl.n_modes(dim, P)
    nv = (1 + dim) * npm
    if dim == 1:
        detJ = 0.5 * np.abs(xy[e2v[:, 1], 0] - xy[e2v[:, 0], 0])
    else:
        a, b, c = xy[e2v[:, 0]], xy[e2v[:, 1]], xy[e2v[:, 2]]
        detJ = np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    ne = B.shape[1] - nv
    AEE = B[:, nv:, nv:]
    assert np.abs(AEE - detJ[:, None, None] * np.eye(ne)).max() <= 1e-12 * detJ.max()
    assert np.all(B[:, :npm, nv:] == 0.0) and np.all(B[:, nv:, :npm] == 0.0)
    # and the velocity-stress couplings are there (the Schur correction is not empty)
    assert np.abs(B[:, npm:nv, nv:]).max() > 0.1 and np.abs(B[:, nv:, npm:nv]).max() > 0.1
    x = wl.rng_for(11, 1).standard_normal((orc.n_el, B.shape[1]))
    direct = np.linalg.solve(B, x[..., None])[..., 0]
    d = 1.0 / detJ
    G = B[:, npm:nv, nv:]
    H = d[:, None, None] * B[:, nv:, npm:nv]
    S = B[:, :nv, :nv].copy()
    S[:, npm:, npm:] -= G @ H
    t = d[:, None] * x[:, nv:]
    r = x[:, :nv].copy()
    r[:, npm:] -= np.einsum("eij,ej->ei", G, t)
    zv = np.linalg.solve(S, r[..., None])[..., 0]
    ze = t - np.einsum("eij,ej->ei", H, zv[:, npm:])
    assert np.abs(np.concatenate([zv, ze], 1) - direct).max() <= 1e-10 * np.abs(direct).max()

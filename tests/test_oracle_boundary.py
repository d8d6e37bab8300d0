"""Pins of per-face boundary conditions (paper Sec. 5.2: Dirichlet and
Neumann boundaries; the Sec. 6.1 example has Dirichlet data of different
depth at its two ends, the Sec. 6.2 example a Neumann end and a no-flow end).

A boundary face carries a code kind | tag << 2 (kind 1 wall, 2 Neumann,
3 Dirichlet, 0 the call's bc; a Dirichlet face takes the exterior state of
its tag).  The pins: uniform codes reproduce the global setting exactly; the
lake at rest over the cos bed is kept by the paper's own Dirichlet ends and
broken when the two ends' data are swapped; a free stream is kept by
Dirichlet faces that carry it, on any mix of tags, and not when one tag
carries another state; the Sec. 6.2 surface with a Neumann and a wall end is
held by a yield stress well above the printed threshold and flows well below.
"""
import math
import os

import numpy as np
import pytest

import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
ALPHA = math.pi / 18


def line(oracle_mod, P, n, L=10.0):
    xy, e2v = wl.mesh_1d(n, 0.0, L)
    return oracle_mod.Oracle(1, P, xy, e2v)


def tri(oracle_mod, P, n):
    xy, e2v = wl.mesh_tri(n, 20.0, 20.0, 0.1, 2)
    return oracle_mod.Oracle(2, P, xy, e2v)


def ends(o, left, right):
    """1-D codes: local face 0 of the first element, face 1 of the last."""
    c = np.zeros((o.n_el, 2), np.int8)
    c[0, 0] = left
    c[-1, 1] = right
    return c


@pytest.mark.parametrize("dim,P", [(1, 2), (2, 2)])
@pytest.mark.parametrize("kind", [1, 2, 3])
def test_uniform_codes_equal_the_global_boundary(oracle_mod, dim, P, kind):
    o = line(oracle_mod, P, 20) if dim == 1 else tri(oracle_mod, P, 4)
    p = wl.Params(alpha=0.1, eta=0.8, sigma0=30.0, gamma=1e3, beta=1e3, reg=1)
    W = wl.random_state(dim, P, o.n_el, 31)
    x = wl.random_vector(dim, P, o.n_el, 32)
    dirv = [1.1, 0.3, -0.2, 0.01, 0.02, -0.03, 0.04][: 1 + dim + dim * dim]
    b = o.step_begin(p, W * 0.9, 0.02)
    R0 = o.residual(p, W, b, 0.02, bc=kind, dirichlet=dirv)
    y0 = o.jac_apply(p, W, x, 0.02, bc=kind, dirichlet=dirv)
    o.set_boundary(np.full((o.n_el, o.nfc), kind, np.int8))
    other = 1 + kind % 3
    assert np.array_equal(o.residual(p, W, b, 0.02, bc=other, dirichlet=dirv), R0)
    assert np.array_equal(o.jac_apply(p, W, x, 0.02, bc=other, dirichlet=dirv), y0)
    # tag 2 carrying the same Dirichlet state gives the same bits as tag 0
    if kind == 3:
        o.set_boundary(np.full((o.n_el, o.nfc), 3 | 2 << 2, np.int8), dirichlet_tags=[[0] * 7, dirv])
        assert np.array_equal(o.residual(p, W, b, 0.02, bc=other, dirichlet=[5.0] * 7), R0)
    with pytest.raises(ValueError):
        o.set_boundary(np.full((o.n_el, o.nfc), 16, np.int8))


@pytest.mark.parametrize("P", [1, 2])
def test_lake_at_rest_with_the_papers_dirichlet_ends(oracle_mod, P):
    """Sec. 6.1 as printed: Dirichlet at both ends with h(0) = h0/cos(a) - 1,
    h(L) = h0/cos(a) - L tan(a) - cos(pi L), u = E = 0.  The interpolated depth
    equals these at the end vertices, so the residual vanishes; swapping the
    two ends' data does not."""
    L, h0 = 10.0, 3.0
    o = line(oracle_mod, P, 100, L)
    o.set_bed(o.bed_interpolate(wl.Bed(kind=wl.BED_COS, order=P, a=1.0, kx=math.pi)))
    W = o.project_ic(wl.IC(kind=wl.IC_SURFACE, a=h0 / math.cos(ALPHA), b=-math.tan(ALPHA)))
    hL = h0 / math.cos(ALPHA) - 1.0
    hR = h0 / math.cos(ALPHA) - L * math.tan(ALPHA) - math.cos(math.pi * L)
    prm = wl.Params(g=9.81, rho=1.0, alpha=ALPHA, eta=1.0, sigma0=1.0, gamma=1e3, beta=1e3, reg=1)
    dt = 0.01
    b = o.step_begin(prm, W, dt)
    tags = [[hL, 0.0, 0.0], [hR, 0.0, 0.0]]
    o.set_boundary(ends(o, 3 | 1 << 2, 3 | 2 << 2), dirichlet_tags=tags)
    R = o.residual(prm, W, b, dt)
    assert np.abs(R).max() <= 2e-14 * np.abs(b).max()
    o.set_boundary(ends(o, 3 | 2 << 2, 3 | 1 << 2), dirichlet_tags=tags)
    assert np.abs(o.residual(prm, W, b, dt)).max() > 1e-3 * np.abs(b).max()
    # and a solve keeps the state
    import oracle
    o.set_boundary(ends(o, 3 | 1 << 2, 3 | 2 << 2), dirichlet_tags=tags)
    W1, st = o.solve(prm, W, oracle.SolveOptions(t_end=0.05, dt_override=0.01))
    assert st["newton_total"] == 0 and np.array_equal(W1, W)


@pytest.mark.parametrize("P", [1, 3])
def test_free_stream_with_tagged_dirichlet_faces(oracle_mod, P):
    """2-D: a constant moving state with E = 0 is kept when every boundary
    face is Dirichlet with that state, whatever tag carries it; one tag with
    a different state breaks it."""
    o = tri(oracle_mod, P, 5)
    state = [1.3, 0.4, -0.25, 0.0, 0.0, 0.0, 0.0]
    W = o.project_ic(wl.IC(kind=wl.IC_CONST, a=state[0], b=state[1], c=state[2]))
    prm = wl.Params(alpha=0.0, eta=1.0, sigma0=20.0, gamma=1e3, beta=1e3, reg=2)
    dt = 0.01
    b = o.step_begin(prm, W, dt)
    rng = np.random.default_rng(5)
    codes = (3 | rng.integers(0, 4, size=(o.n_el, o.nfc)) << 2).astype(np.int8)
    o.set_boundary(codes, dirichlet_tags=[state, state, state])
    R = o.residual(prm, W, b, dt, bc=1, dirichlet=state)
    assert np.abs(R).max() <= 1e-13 * np.abs(b).max()
    bad = list(state)
    bad[1] = -0.4
    o.set_boundary(codes, dirichlet_tags=[state, bad, state])
    assert np.abs(o.residual(prm, W, b, dt, bc=1, dirichlet=state)).max() > 1e-3 * np.abs(b).max()


@pytest.mark.parametrize("reg", [1, 3])
def test_cos_bed_surface_with_the_papers_open_and_closed_ends(oracle_mod, reg):
    """Sec. 6.2 as printed: dh/dx = du/dx = dE/dx = 0 at x = 0 (Neumann) and
    u = 0 with dh/dx = dE/dx = 0 at x = L (the mirror wall in 1-D).  The
    surface h = h0 - cos(pi x) is held (no yielded region, creep O(1/gamma))
    at three times the printed threshold and flows at a third of it."""
    import oracle
    vals = {}
    with open(os.path.join(HERE, "golden", "yield_threshold.txt")) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                k, v = ln.split()
                vals[k] = float(v)
    thr = vals["threshold"]
    o = line(oracle_mod, 1, 40)
    o.set_bed(o.bed_interpolate(wl.Bed(kind=wl.BED_COS, order=1, a=1.0, kx=math.pi)))
    o.set_boundary(ends(o, 2, 1))
    W0 = o.project_ic(wl.IC(kind=wl.IC_SURFACE, a=3.0, b=0.0))
    opts = oracle.SolveOptions(t_end=0.3, dt_override=0.01, max_newton=25)
    umax = {}
    for gam in (1e2, 1e3):
        prm = wl.Params(g=9.81, rho=1.0, alpha=ALPHA, eta=1.0, sigma0=3 * thr, gamma=gam, beta=gam, reg=reg)
        W, st = o.solve(prm, W0, opts)
        assert st["capped"] == 0 and st["active_pct"] == 0.0
        umax[gam] = np.abs(o.eval_points(W)[:, :, 1]).max()
    assert 5.0 < umax[1e2] / umax[1e3] < 20.0, umax
    prm = wl.Params(g=9.81, rho=1.0, alpha=ALPHA, eta=1.0, sigma0=thr / 3, gamma=1e3, beta=1e3, reg=reg)
    W, st = o.solve(prm, W0, opts)
    assert st["active_pct"] > 5.0
    assert np.abs(o.eval_points(W)[:, :, 1]).max() > 20 * umax[1e3]

"""Pins of the oracle's reference elements and mesh handling.

Basis and quadrature are checked against an independent collapsed (Duffy)
Gauss product rule built here from numpy's Gauss-Legendre nodes, and against
exact monomial integrals; the mesh against geometric identities.
"""
import math

import numpy as np
import pytest

import workloads as wl


def duffy_rule(n=14):
    x, w = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (x + 1.0)
    wu = 0.5 * w
    U, V = np.meshgrid(u, u, indexing="ij")
    WU, WV = np.meshgrid(wu, wu, indexing="ij")
    xi = U.ravel()
    eta = (V * (1.0 - U)).ravel()
    ww = (WU * WV * (1.0 - U)).ravel()
    return np.stack([xi, eta], axis=1), ww


def exact_monomial(i, j):
    return math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_triangle_basis_orthonormal_and_complete(oracle_mod, P):
    pts, w = duffy_rule()
    phi = np.zeros((len(w), (P + 1) * (P + 2) // 2))
    dphi = np.zeros(phi.shape + (2,))
    import ctypes as C
    np_ = oracle_mod.lib().or_basis(2, P, len(w), oracle_mod._dp(np.ascontiguousarray(pts)),
                                   oracle_mod._dp(phi), oracle_mod._dp(dphi))
    assert np_ == phi.shape[1]
    M = (phi.T * w) @ phi
    assert np.abs(M - np.eye(np_)).max() < 1e-13
    # spans every monomial of total degree <= P (least-squares fit is exact)
    for i in range(P + 1):
        for j in range(P + 1 - i):
            f = pts[:, 0] ** i * pts[:, 1] ** j
            c, *_ = np.linalg.lstsq(phi, f, rcond=None)
            assert np.abs(phi @ c - f).max() < 1e-12
    # gradient matches central differences
    rng = np.random.default_rng(0)
    for _ in range(5):
        p = rng.uniform(0.05, 0.45, size=2)
        h = 1e-6
        def ev(q):
            out = np.zeros(np_)
            oracle_mod.lib().or_basis(2, P, 1, oracle_mod._dp(np.ascontiguousarray(q)), oracle_mod._dp(out), None)
            return out
        g = np.zeros(np_ * 2)
        v = np.zeros(np_)
        oracle_mod.lib().or_basis(2, P, 1, oracle_mod._dp(np.ascontiguousarray(p)), oracle_mod._dp(v), oracle_mod._dp(g))
        g = g.reshape(np_, 2)
        for a in range(2):
            e = np.zeros(2); e[a] = h
            fd = (ev(p + e) - ev(p - e)) / (2 * h)
            assert np.abs(fd - g[:, a]).max() < 1e-7 * max(1.0, np.abs(g).max())


@pytest.mark.parametrize("P,deg", [(1, 2), (2, 5), (3, 6)])
def test_triangle_rules_exact_to_degree(oracle_mod, P, deg):
    xy, e2v = wl.mesh_tri(1, 1.0, 1.0, 0.0, 0)
    o = oracle_mod.Oracle(2, P, xy, e2v)
    t = o.ref_tables()
    assert o.nq == {1: 3, 2: 7, 3: 12}[P]
    assert np.all(t["qw"] > 0)
    inside = (t["qx"][:, 0] > 0) & (t["qx"][:, 1] > 0) & (t["qx"].sum(1) < 1)
    assert inside.all()
    for i in range(deg + 1):
        for j in range(deg + 1 - i):
            q = (t["qw"] * t["qx"][:, 0] ** i * t["qx"][:, 1] ** j).sum()
            assert abs(q - exact_monomial(i, j)) < 2e-16 * 10
    # the rule is not exact one degree higher (it is the rule of that degree)
    errs = [abs((t["qw"] * t["qx"][:, 0] ** i * t["qx"][:, 1] ** (deg + 1 - i)).sum()
                - exact_monomial(i, deg + 1 - i)) for i in range(deg + 2)]
    assert max(errs) > 1e-8
    # reference mass matrix with the element rule is the identity
    M = (t["phi"].T * t["qw"]) @ t["phi"]
    assert np.abs(M - np.eye(o.np)).max() < 1e-12


@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
def test_line_basis_and_gauss(oracle_mod, P):
    xy, e2v = wl.mesh_1d(1, -1.0, 1.0)
    o = oracle_mod.Oracle(1, P, xy, e2v)
    t = o.ref_tables()
    xg, wg = np.polynomial.legendre.leggauss(P + 1)
    assert np.allclose(t["qx"][:, 0], xg, atol=1e-15, rtol=0)
    assert np.allclose(t["qw"], wg, atol=1e-15, rtol=0)
    xs, ws = np.polynomial.legendre.leggauss(20)
    phi = np.zeros((20, P + 1))
    oracle_mod.lib().or_basis(1, P, 20, oracle_mod._dp(np.ascontiguousarray(xs)), oracle_mod._dp(phi), None)
    assert np.abs((phi.T * ws) @ phi - np.eye(P + 1)).max() < 1e-14
    # normalised Legendre: phi_i = sqrt((2i+1)/2) P_i
    for i in range(P + 1):
        c = np.zeros(i + 1); c[i] = 1
        assert np.allclose(phi[:, i], math.sqrt((2 * i + 1) / 2) * np.polynomial.legendre.legval(xs, c), atol=1e-14)
    # face values at the end points
    assert np.allclose(t["fphi"][0, 0], [math.sqrt((2 * i + 1) / 2) * (-1) ** i for i in range(P + 1)])
    assert np.allclose(t["fphi"][1, 0], [math.sqrt((2 * i + 1) / 2) for i in range(P + 1)])


@pytest.mark.parametrize("N,jit", [(4, 0.1), (7, 0.1), (16, 0.0)])
def test_triangle_mesh_geometry(oracle_mod, N, jit):
    xy, e2v = wl.mesh_tri(N, 20.0, 20.0, jit, 3)
    o = oracle_mod.Oracle(2, 2, xy, e2v)
    m = o.mesh_data()
    assert abs(m["measure"] - 400.0) < 1e-10
    nbr, nbf = m["nbr"], m["nbr_face"]
    n_bnd = int((nbr < 0).sum())
    assert n_bnd == 4 * N
    t = o.ref_tables()
    tg = np.polynomial.legendre.leggauss(o.nfq)[0]
    for e in range(o.n_el):
        v = xy[e2v[e]]
        # sum of outward normals times lengths vanishes
        s = (m["normal"][e] * m["flen"][e][:, None]).sum(0)
        assert np.abs(s).max() < 1e-12
        for f in range(3):
            n = nbr[e, f]
            if n < 0:
                continue
            g = nbf[e, f]
            assert nbr[n, g] == e and nbf[n, g] == f
            assert np.allclose(m["normal"][e, f], -m["normal"][n, g], atol=1e-15)
            assert abs(m["flen"][e, f] - m["flen"][n, g]) < 1e-14
            # matched face points coincide physically (reversed order on the neighbour)
            A, B = v[f], v[(f + 1) % 3]
            w = xy[e2v[n]]
            C, D = w[g], w[(g + 1) % 3]
            for r in range(o.nfq):
                pe = A + 0.5 * (tg[r] + 1) * (B - A)
                pn = C + 0.5 * (tg[o.nfq - 1 - r] + 1) * (D - C)
                assert np.abs(pe - pn).max() < 1e-13


def test_line_mesh(oracle_mod):
    xy, e2v = wl.mesh_1d(10, 0.0, 10.0)
    o = oracle_mod.Oracle(1, 1, xy, e2v)
    m = o.mesh_data()
    assert abs(m["measure"] - 10.0) < 1e-14 and abs(m["hmin"] - 1.0) < 1e-14
    assert m["nbr"][0, 0] == -1 and m["nbr"][-1, 1] == -1
    assert all(m["nbr"][e, 1] == e + 1 and m["nbr_face"][e, 1] == 0 for e in range(9))


@pytest.mark.parametrize("P", [2, 3])
def test_disk_projection_positivity_reading(oracle_mod, P):
    """Discontinuous disk depth: element means equal the element rule's
    projection of the analytic depth; every volume and face point stays at or
    above a tenth of its element mean, with equality where modes were scaled."""
    xy, e2v = wl.mesh_tri(12, 20.0, 20.0, 0.1, 3)
    o = oracle_mod.Oracle(2, P, xy, e2v)
    ic = wl.IC(kind=wl.IC_DISK, a=2.0, b=0.5, x0=10.0, y0=10.0, r=2.5)
    W = o.project_ic(ic)
    t = o.ref_tables()
    m = o.mesh_data()
    x, y = m["xq"][:, :, 0], m["xq"][:, :, 1]
    hq = np.where((x - 10) ** 2 + (y - 10) ** 2 < 2.5 ** 2, 2.0, 0.5)
    c0 = np.einsum("q,q,eq->e", t["qw"], t["phi"][:, 0], hq)
    assert np.abs(W[0, 0] - c0).max() < 1e-14
    mean = W[0, 0] * t["phi"][0, 0]
    hv = np.einsum("qi,ie->eq", t["phi"], W[0])
    hf = np.einsum("fri,ie->efr", t["fphi"], W[0]).reshape(o.n_el, -1)
    mn = np.minimum(hv.min(1), hf.min(1))
    assert (mn >= 0.1 * mean - 1e-12).all()
    hit = mn < 0.1 * mean + 1e-12
    assert hit.any()   # the disk cuts elements whose projection had to be scaled
    # elements not cut by the disk keep the plain projection (constant depth)
    full = np.einsum("q,qi,eq->ie", t["qw"], t["phi"], hq)
    assert np.abs(W[0][:, ~hit] - full[:, ~hit]).max() < 1e-14

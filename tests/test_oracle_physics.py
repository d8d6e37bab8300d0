"""Pins of the oracle's pointwise physics: the regularised Bingham law
(paper Sec. 4 and Appendix A) and the HLL / wall fluxes (Sec. 5, Eq. HLLSolver,
Sec. 5.2).

The paper's printed 1-D regularisations are evaluated through their own
routine (or_sigmaB_1d, the literal formulas with the two readings noted in the
oracle) and the 2-D law through a separate one (psi(s) times D + tr(D) I);
the tests tie the two together and to the limits the paper states.
"""
import math

import numpy as np
import pytest

import workloads as wl


def prm(reg, s0=1.0, gam=1e3, bet=1e3, eta=0.0):
    return wl.Params(g=9.81, rho=1.0, alpha=0.0, eta=eta, sigma0=s0, gamma=gam, beta=bet, reg=reg)


FIG_SETS = [(1.0, 10.0, 1.0), (1.0, 1e3, 1e3), (50.0, 1e3, 1e3), (9.035, 1e4, 1e4)]


def breakpoints(reg, s0, gam, bet):
    h = 0.5 / bet
    if reg == 1:   # gamma|E| - s0 = +-h
        return [(s0 - h) / gam, (s0 + h) / gam]
    if reg == 2:
        return [(s0 - h) / gam, (s0 + h) / gam]
    return []


@pytest.mark.parametrize("reg", [1, 2, 3])
@pytest.mark.parametrize("s0,gam,bet", FIG_SETS)
def test_regularisation_shape(oracle_mod, reg, s0, gam, bet):
    f = lambda E: oracle_mod.sigmaB_1d(reg, s0, gam, bet, E)
    # odd symmetry
    for E in [1e-7, 3e-4, 0.02, 0.5, 3.0]:
        assert abs(f(E)[0] + f(-E)[0]) < 1e-14 * max(1, abs(f(E)[0]))
        assert abs(f(E)[1] - f(-E)[1]) < 1e-12 * max(1, abs(f(E)[1]))
    # saturation at 2 sigma0
    assert abs(f(1e6)[0] - 2 * s0) < 1e-5 * s0
    assert abs(f(-1e6)[0] + 2 * s0) < 1e-5 * s0
    # slope at 0: 2 gamma for regs 1-2, 2 sigma0 gamma for reg 3 (reading of Sec. 4)
    slope = 2 * gam if reg in (1, 2) else 2 * s0 * gam
    assert abs(f(0.0)[1] - slope) < 1e-12 * slope
    # continuity and C1 at every breakpoint
    for b in breakpoints(reg, s0, gam, bet):
        if b <= 0:
            continue
        d = 1e-12 * b
        lo, hi = f(b - d), f(b + d)
        assert abs(lo[0] - hi[0]) < 1e-9 * max(1, abs(hi[0]))
        assert abs(lo[1] - hi[1]) < 1e-6 * slope
    # printed derivative (with the reg-2 reading 2*gamma) matches central differences
    rng = np.random.default_rng(reg)
    bps = breakpoints(reg, s0, gam, bet)
    for E in np.concatenate([10 ** rng.uniform(-6, 0.5, 40), -(10 ** rng.uniform(-6, 0.5, 20))]):
        if any(abs(abs(E) - b) < 1e-6 * b + 1e-12 for b in bps):
            continue
        h = 1e-7 * max(abs(E), 1.0 / gam)
        fd = (f(E + h)[0] - f(E - h)[0]) / (2 * h)
        noise = 1e-13 * 2 * s0 / h   # rounding of the difference quotient
        assert abs(fd - f(E)[1]) <= 1e-5 * max(abs(fd), abs(f(E)[1])) + noise


@pytest.mark.parametrize("reg", [1, 2, 3])
@pytest.mark.parametrize("eta", [0.0, 1.3])
def test_2d_law_reduces_to_paper_1d(oracle_mod, reg, eta):
    """With E = [[e, 0], [0, 0]] the 2-D law gives sigma_11 = 4 eta e + sigma_B(e)
    (Eqs. sigma11D, sigmaTwoA/B/C), and the 1-D oracle path agrees too."""
    for s0, gam, bet in FIG_SETS:
        p = prm(reg, s0, gam, bet, eta)
        for e in [-2.0, -1e-3, -3e-7, 0.0, 2e-7, 4e-4, 0.01, 1.7]:
            sB, dB = oracle_mod.sigmaB_1d(reg, s0, gam, bet, e)
            sig2, dsig2 = oracle_mod.point_sigma(p, 2, [e, 0.0, 0.0, 0.0])
            sig1, dsig1 = oracle_mod.point_sigma(p, 1, [e])
            ref = 4 * eta * e + sB
            dref = 4 * eta + dB
            for s, ds in ((sig2[0, 0], dsig2[0, 0, 0, 0]), (sig1[0, 0], dsig1[0, 0, 0, 0])):
                assert abs(s - ref) <= 1e-12 * max(1.0, abs(ref))
                assert abs(ds - dref) <= 1e-9 * max(1.0, abs(dref))


def test_2d_law_limit_and_invariance(oracle_mod):
    """gamma -> infinity recovers Eq. bingham: sigma = 2 eta T + sqrt(2) sigma0 T / ||D||_c;
    sigma is symmetric and frame-indifferent; its derivative matches FD."""
    rng = np.random.default_rng(7)
    for reg in (1, 2, 3):
        for _ in range(20):
            Ev = rng.normal(size=4)
            p = prm(reg, s0=2.5, gam=1e12, bet=1e12, eta=0.7)
            sig, _ = oracle_mod.point_sigma(p, 2, Ev)
            Em = np.array([[Ev[0], Ev[2]], [Ev[1], Ev[3]]])   # Em[a][b] = E_ab
            D = 0.5 * (Em + Em.T)
            T = D + np.trace(D) * np.eye(2)
            nc = math.sqrt((D ** 2).sum() + np.trace(D) ** 2)
            ref = 2 * 0.7 * T + math.sqrt(2) * 2.5 * T / nc
            assert np.abs(sig - ref).max() < 1e-9 * np.abs(ref).max()
            # finite gamma: symmetry, rotation, derivative
            p = prm(reg, s0=2.5, gam=30.0, bet=30.0, eta=0.7)
            sig, dsig = oracle_mod.point_sigma(p, 2, Ev)
            assert np.abs(sig - sig.T).max() < 1e-13 * np.abs(sig).max()
            th = rng.uniform(0, 2 * math.pi)
            Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
            Er = Rm @ Em @ Rm.T
            sr, _ = oracle_mod.point_sigma(p, 2, [Er[0, 0], Er[1, 0], Er[0, 1], Er[1, 1]])
            assert np.abs(sr - Rm @ sig @ Rm.T).max() < 1e-12 * np.abs(sig).max()
            for c in range(2):
                for d in range(2):
                    h = 1e-6
                    Ep = Em.copy(); Ep[c, d] += h
                    Emn = Em.copy(); Emn[c, d] -= h
                    vp = lambda M: [M[0, 0], M[1, 0], M[0, 1], M[1, 1]]
                    fd = (oracle_mod.point_sigma(p, 2, vp(Ep))[0] - oracle_mod.point_sigma(p, 2, vp(Emn))[0]) / (2 * h)
                    assert np.abs(fd - dsig[:, :, c, d]).max() < 1e-6 * max(1.0, np.abs(dsig).max())


def test_reg3_small_shear_series(oracle_mod):
    """q = psi'/(2 s) stays finite and continuous through the series switch."""
    p = prm(3, s0=30.0, gam=1e4, bet=1e4)
    xs = np.concatenate([[0.0], np.logspace(-8, 1, 400)])
    q = np.array([oracle_mod.point_psi(p, x / 1e4)[1] for x in xs])
    assert np.isfinite(q).all()
    ref0 = 0.5 * 30.0 * 1e12 * (-2.0 / 3.0)
    assert abs(q[0] - ref0) < 1e-14 * abs(ref0)
    # both sides of the series switch at gamma s = 1e-2 agree
    qa = oracle_mod.point_psi(p, 1e-2 * (1 - 1e-12) / 1e4)[1]
    qb = oracle_mod.point_psi(p, 1e-2 * (1 + 1e-12) / 1e4)[1]
    assert abs(qa - qb) < 1e-9 * abs(qa)
    # against the Taylor series of (x sech^2 x - tanh x) / x^3 (Bernoulli-number
    # coefficients of tanh, summed to high order here)
    from fractions import Fraction
    B = [Fraction(1), Fraction(-1, 2), Fraction(1, 6), Fraction(0), Fraction(-1, 30), Fraction(0),
         Fraction(1, 42), Fraction(0), Fraction(-1, 30), Fraction(0), Fraction(5, 66), Fraction(0),
         Fraction(-691, 2730), Fraction(0), Fraction(7, 6)]
    # tanh x = sum_{n>=1} 2^{2n} (2^{2n} - 1) B_{2n} x^{2n-1} / (2n)!
    tc = {2 * n - 1: Fraction(2 ** (2 * n) * (2 ** (2 * n) - 1), math.factorial(2 * n)) * B[2 * n]
          for n in range(1, 8)}
    for x in (1e-4, 3e-3, 9e-3, 2e-2, 5e-2):
        # x sech^2 x - tanh x = x d/dx tanh x - tanh x = sum (k - 1) c_k x^k
        ser = sum(float((k - 1) * c) * x ** (k - 3) for k, c in tc.items())
        qv = oracle_mod.point_psi(p, x / 1e4)[1]
        assert abs(qv - 0.5 * 30.0 * 1e12 * ser) < 1e-9 * abs(qv)


def _X(h, u):
    X = np.zeros(3 if len(u) == 1 else 7)
    X[0] = h
    X[1:1 + len(u)] = u
    return X


def test_hll_properties(oracle_mod):
    rng = np.random.default_rng(3)
    p = wl.Params(g=9.81, rho=1000.0, alpha=0.3, eta=1.0, sigma0=10.0, gamma=100.0, beta=100.0, reg=1)
    gc = 9.81 * math.cos(0.3)
    for _ in range(200):
        hm, hp = rng.uniform(0.1, 3, 2)
        um, up = rng.normal(size=2) * 3, rng.normal(size=2) * 3
        th = rng.uniform(0, 2 * math.pi)
        n = np.array([math.cos(th), math.sin(th)])
        Xm, Xp = _X(hm, um), _X(hp, up)
        F = oracle_mod.point_hll(p, 2, Xm, Xp, n)
        # conservation: F(U-, U+; n) = -F(U+, U-; -n)
        G = oracle_mod.point_hll(p, 2, Xp, Xm, -n)
        assert np.abs(F + G).max() < 1e-12 * max(1, np.abs(F).max())
        # consistency: F(U, U; n) = F(U) . n (Eq. Fterm)
        Fc = oracle_mod.point_hll(p, 2, Xm, Xm, n)
        un = um @ n
        ref = np.array([hm * un, hm * um[0] * un + 0.5 * gc * hm ** 2 * n[0],
                        hm * um[1] * un + 0.5 * gc * hm ** 2 * n[1]])
        assert np.abs(Fc - ref).max() < 1e-12 * max(1, np.abs(ref).max())
        # rotational invariance
        a = rng.uniform(0, 2 * math.pi)
        Rm = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
        Fr = oracle_mod.point_hll(p, 2, _X(hm, Rm @ um), _X(hp, Rm @ up), Rm @ n)
        assert abs(Fr[0] - F[0]) < 1e-12 * max(1, abs(F[0]))
        assert np.abs(Fr[1:] - Rm @ F[1:]).max() < 1e-11 * max(1, np.abs(F).max())
        # both sides supercritical along n (S_L >= 0): the flux is the left
        # physical flux, independent of the right state
        Xfast = _X(hm, 10.0 * n * (1 + math.sqrt(9.81 * hm)))
        F1 = oracle_mod.point_hll(p, 2, Xfast, _X(hp, 10.0 * n * (1 + math.sqrt(9.81 * hp))), n)
        F2 = oracle_mod.point_hll(p, 2, Xfast, _X(0.5 * hp, 12.0 * n * (1 + math.sqrt(9.81 * hp))), n)
        F3 = oracle_mod.point_hll(p, 2, Xfast, Xfast, n)
        assert np.abs(F1 - F2).max() == 0.0 and np.abs(F1 - F3).max() == 0.0
        # mirror wall: exactly the reflected state, zero mass flux
        Xw = oracle_mod.point_wall(p, 2, n, Xm)
        assert abs(Xw[1:3] @ n + um @ n) < 1e-12 and abs(Xw[0] - hm) == 0
        Fw = oracle_mod.point_hll(p, 2, Xm, Xw, n)
        assert abs(Fw[0]) < 1e-12 * max(1.0, abs(hm * un))
        # exact derivative (including the wave-speed dependence) vs FD
        dXm, dXp = rng.normal(size=7), rng.normal(size=7)
        _, dF = oracle_mod.point_hll(p, 2, Xm, Xp, n, dXm, dXp)
        eps = 1e-7
        fd = (oracle_mod.point_hll(p, 2, Xm + eps * dXm, Xp + eps * dXp, n)
              - oracle_mod.point_hll(p, 2, Xm - eps * dXm, Xp - eps * dXp, n)) / (2 * eps)
        assert np.abs(fd - dF).max() < 1e-6 * max(1, np.abs(dF).max())


def test_hll_1d_matches_2d_embedding(oracle_mod):
    p = wl.Params(g=9.81, rho=1000.0, alpha=0.0, eta=1.0, sigma0=10.0, gamma=100.0, beta=100.0, reg=1)
    rng = np.random.default_rng(5)
    for _ in range(50):
        hm, hp = rng.uniform(0.1, 3, 2)
        um, up = rng.normal(size=2) * 3
        for s in (1.0, -1.0):
            F1 = oracle_mod.point_hll(p, 1, _X(hm, [um]), _X(hp, [up]), np.array([s, 0.0]))
            F2 = oracle_mod.point_hll(p, 2, _X(hm, [um, 0.0]), _X(hp, [up, 0.0]), np.array([s, 0.0]))
            assert np.abs(F1 - F2[:2]).max() < 1e-13 * max(1, np.abs(F2).max())

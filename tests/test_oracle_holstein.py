"""Pins of the oracle's Holstein DMFT pieces (oracle/holstein.py; Sec. "DMFT
for the Holstein model"):
  * the free phonon propagator D0 of X = a + a^dag, built from the free
    single-pole function by the contour relations, equals its closed forms
    D0^R(t) = -2 sin(w0 t), D0^<(t,t') = -i[(1+nB) e^{i w0 (t-t')} + nB e^{-i w0 (t-t')}],
    D0^M(tau) = -[(1+nB) e^{-w0 tau} + nB e^{w0 tau}] and the mixing component;
  * the displacement quadrature (Eq. X) against the exact solution of
    X'' + w0^2 X = -2 w0 g n(t) for a prescribed density, at the order of
    the quadrature;
  * at g = 0 the Bethe-lattice loop gives the semicircular density of states'
    G^R(t,0) = -i J_1(2t)/t (J = 1);
  * with g(t) and J(t) modulated away from half filling (mu = -1.3, n = 0.46;
    half filling is mu = g X = -2 g^2 / w0), the uMig + Bethe loop conserves
    the density n(t) up to a discretisation error that falls with h;
  * at constant g and J the propagation from the self-consistent Matsubara
    state is stationary (n, X and G^R(t+s, s) stay put).
Planted on the CPU, a lost conjugation in the transposed term of D0, a factor
1 for the 2 of Eq. X, or J(t) G J(t) for J(t) G J(t') fails one of these."""
import numpy as np
import pytest
from scipy.special import j1

from oracle import holstein as H


def grid(O, nt, h, ntau, beta, mu=0.0, k=5):
    return O.Grid(nt, ntau, 1, -1, k, beta, h, mu)


def test_phonon_d0_closed_forms(O):
    g = grid(O, 20, 0.1, 30, 3.0)
    w0 = 0.7
    D = H.phonon_d0(g, w0)
    nB = 1.0 / np.expm1(g.beta * w0)
    for n in range(g.nt + 1):
        for j in range(n + 1):
            t = (n - j) * g.h
            assert abs(D.R(n, j)[0, 0] - (-2 * np.sin(w0 * t))) < 1e-12
            assert abs(D.L(j, n)[0, 0] - (-1j) * ((1 + nB) * np.exp(-1j * w0 * t) + nB * np.exp(1j * w0 * t))) < 1e-12
        for m in range(g.ntau + 1):
            tau, tn = m * g.htau, n * g.h
            ref = -1j * ((1 + nB) * np.exp(1j * w0 * tn - w0 * tau) + nB * np.exp(-1j * w0 * tn + w0 * tau))
            assert abs(D.T(n, m)[0, 0] - ref) < 1e-12
    for m in range(g.ntau + 1):
        tau = m * g.htau
        assert abs(D.M(m)[0, 0] + (1 + nB) * np.exp(-w0 * tau) + nB * np.exp(w0 * tau)) < 1e-12


def fake_density(O, g, nfun):
    """A contour function whose densities are nfun(t) (both spins) on every
    slice and nfun(0) on the Matsubara branch."""
    G = O.HM(g)
    G.mat[g.ntau, 0, 0] = -nfun(0.0) / 2
    for n in range(g.nt + 1):
        G.L(n, n)[0, 0] = 0.5j * nfun(n * g.h)
    return G


def test_displacement_quadrature_order(O):
    w0, nu, gc, a = 0.7, 1.3, 0.4, 0.3
    nfun = lambda t: 1.0 + a * np.sin(nu * t)
    exact = lambda t: -2 * gc * 1.0 / w0 - 2 * gc * a * (w0 * np.sin(nu * t) - nu * np.sin(w0 * t)) / (w0 ** 2 - nu ** 2)
    errs = []
    for nt, h in ((40, 0.1), (80, 0.05)):
        g = grid(O, nt, h, 10, 2.0)
        G = fake_density(O, g, nfun)
        X = np.zeros(nt + 2)
        gel = np.full(nt + 2, gc)
        H.displacement(-1, G, gel, w0, X)
        assert abs(X[0] - exact(0.0)) < 1e-14
        for n in range(nt + 1):
            H.displacement(n, G, gel, w0, X)
        errs.append(max(abs(X[n + 1] - exact(n * h)) for n in range(nt + 1)))
    # (observed 1.7e-8 and 1.4e-10: order ~7)
    assert errs[0] < 1e-7, errs
    assert errs[1] < errs[0] / 2 ** 5, errs


def test_bethe_at_g0_is_the_semicircle(O):
    errs = []
    for nt, h in ((30, 0.1), (60, 0.05)):
        g = grid(O, nt, h, 60, 2.0)
        G = O.HM(g)
        J = np.ones(nt + 2)
        gel = np.zeros(nt + 2)
        H.solve_holstein(G, J, gel, 0.5, mats_iters=40, boot_iters=8, ncorr=6)
        ref = [-1j * (j1(2 * n * h) / (n * h) if n else 1.0) for n in range(nt + 1)]
        errs.append(max(abs(G.R(n, 0)[0, 0] - ref[n]) for n in range(nt + 1)))
    # (observed 6.3e-6 and 2.0e-7: order ~5)
    assert errs[0] < 1e-5, errs
    assert errs[1] < errs[0] / 16, errs


def drive(nt, h):
    t = np.arange(nt + 1) * h
    env = np.sin(np.pi * np.clip(t / 2.0, 0, 1)) ** 2
    J = np.concatenate([[1.0], 1.0 + 0.2 * env * np.sin(3.0 * t)])
    gel = np.concatenate([[0.5], 0.5 + 0.2 * env * np.sin(2.0 * t)])
    return J, gel


def test_umig_conserves_the_density(O):
    drift = []
    for nt, h in ((30, 0.1), (60, 0.05)):
        g = grid(O, nt, h, 40, 2.0, mu=-1.3)
        G = O.HM(g)
        J, gel = drive(nt, h)
        _, _, _, X, _ = H.solve_holstein(G, J, gel, 0.5, mats_iters=40, boot_iters=8, ncorr=6)
        n = np.array([H.density(m, G) for m in range(nt + 1)])
        assert 0.2 < n[0] < 0.9  # away from half filling
        assert np.ptp(X[1:]) > 1e-2  # the drive moves the phonon
        drift.append(np.abs(n - n[0]).max())
    # (observed 4.1e-4 and 1.4e-5: order ~5)
    assert drift[0] < 1e-3, drift
    assert drift[1] < drift[0] / 16, drift


def test_equilibrium_is_stationary(O):
    nt, h = 30, 0.05
    g = grid(O, nt, h, 40, 2.0, mu=-1.3)
    G = O.HM(g)
    J, gel = np.ones(nt + 2), np.full(nt + 2, 0.5)
    _, _, _, X, _ = H.solve_holstein(G, J, gel, 0.5, mats_iters=60, boot_iters=8, ncorr=6)
    n = np.array([H.density(m, G) for m in range(nt + 1)])
    # (observed 6.0e-7, 9.6e-8 and 3.2e-7; with the Matsubara sign of the
    # bubble flipped, G^R(t+s, s) drifts by 8.6e-5)
    assert np.abs(n - H.density(-1, G)).max() < 2e-6
    assert np.abs(X[1:] - X[0]).max() < 1e-6
    for m in (10, 20):
        for j in range(nt + 1 - m):
            assert abs(G.R(m + j, j)[0, 0] - G.R(m, 0)[0, 0]) < 2e-6

"""Pins of the free-propagator oracle (Sec. "Implementation: Free Green's
functions", Eqs. cf4 and G0_free) against closed forms, an independent ODE
integration, the order of the method and exact identities."""
import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

from oracle import free_green as F
from paper_1911_01211_amd import workloads as W


def ogrid(O, nt, ntau, d, k=5, h=0.05, beta=3.0, mu=0.2, sig=-1):
    return O.Grid(nt, ntau, d, sig, k, beta, h, mu)


def herm(r, d):
    a = r.normal(size=(d, d)) + 1j * r.normal(size=(d, d))
    return 0.5 * (a + a.conj().T)


def driven_eps(r, nt, d, h, amp=0.8, om=1.3):
    """eps(t) = H0 + cos(om t) H1, entry 0 = H0 (t = 0^-)."""
    H0, H1 = herm(r, d), amp * herm(r, d)
    eps = np.zeros((nt + 2, d, d), np.complex128)
    eps[0] = H0
    for n in range(nt + 1):
        eps[n + 1] = H0 + np.cos(om * n * h) * H1
    return eps, H0, H1


def test_constant_hamiltonian_is_exact(O):
    """For constant eps, Eq. cf4 is exact: U_{n,0} = exp(-i eps t_n)."""
    r = W.rng(301)
    d, nt, h = 3, 40, 0.07
    H = herm(r, d)
    eps = np.repeat(H[None], nt + 2, axis=0)
    U = F.propagators(eps, nt, 5, h)
    for n in (1, 7, nt):
        assert np.abs(U[n] - scipy.linalg.expm(-1j * H * n * h)).max() < 1e-13


def test_scalar_cubic_is_exact():
    """d = 1: the two exponents add up to the 2-point Gauss-Legendre rule of
    the step, exact for a cubic eps(t); the degree-5 interpolation is exact
    too, so U_{n,0} = exp(-i int_0^t eps)."""
    c = np.array([0.3, -1.1, 0.7, 0.25])  # eps(t) = c0 + c1 t + c2 t^2 + c3 t^3
    nt, h = 30, 0.1
    t = np.arange(nt + 1) * h
    eps = np.zeros((nt + 2, 1, 1), np.complex128)
    eps[1:, 0, 0] = c[0] + c[1] * t + c[2] * t ** 2 + c[3] * t ** 3
    eps[0] = eps[1]
    U = F.propagators(eps, nt, 5, h)
    phase = c[0] * t + c[1] * t ** 2 / 2 + c[2] * t ** 3 / 3 + c[3] * t ** 4 / 4
    assert np.abs(U[:, 0, 0] - np.exp(-1j * phase)).max() < 1e-13


def test_matches_ode_and_fourth_order():
    """Driven 2 x 2 Hamiltonian: U against a tight DOP853 integration of
    i dU/dt = eps(t) U, and the error falls as h^4 (ratio ~16 per halving)."""
    r = W.rng(302)
    d, T = 2, 2.0
    H0, H1 = herm(r, d), 0.8 * herm(r, d)

    def rhs(t, y):
        Um = y.reshape(d, d)
        return (-1j * (H0 + np.cos(1.3 * t) * H1) @ Um).ravel()

    sol = scipy.integrate.solve_ivp(rhs, (0, T), np.eye(d, dtype=np.complex128).ravel(), method="DOP853",
                                    rtol=1e-13, atol=1e-14)
    Uref = sol.y[:, -1].reshape(d, d)
    errs = []
    for nt in (20, 40, 80):
        h = T / nt
        eps = np.zeros((nt + 2, d, d), np.complex128)
        eps[0] = H0
        for n in range(nt + 1):
            eps[n + 1] = H0 + np.cos(1.3 * n * h) * H1
        errs.append(np.abs(F.propagators(eps, nt, 5, h)[nt] - Uref).max())
    assert errs[-1] < 1e-7
    for a, b in zip(errs, errs[1:]):
        assert 10.0 < a / b < 24.0, errs


def test_interpolation_points():
    assert list(F.interp_points(0, 5)) == [0, 1, 2, 3, 4, 5]
    assert list(F.interp_points(3, 5)) == [0, 1, 2, 3, 4, 5]
    assert list(F.interp_points(4, 5)) == [0, 1, 2, 3, 4, 5]
    assert list(F.interp_points(9, 5)) == [5, 6, 7, 8, 9, 10]
    # Lagrange weights reproduce a quintic exactly
    p = np.array([0.2, -0.4, 0.1, 0.05, -0.01, 0.003])
    pts = F.interp_points(9, 5)
    w = F.lagrange(pts, 9.3)
    assert abs(np.dot(w, np.polyval(p, pts)) - np.polyval(p, 9.3)) < 1e-11


@pytest.mark.parametrize("sig", [-1, 1])
def test_identities(O, sig):
    """Exact identities of the free function: G^R(t,t) = -i; G^<(t,t) is
    anti-hermitian; at t = 0 the lesser and mixed components follow from the
    Matsubara branch, G^<(0,0) = i xi G^M(beta^-) and G^rceil(0,tau) =
    i xi G^M(beta - tau); the particle number -xi Im tr G^<(t,t) is conserved;
    for constant eps, G^R(t,t') depends on t - t' only."""
    r = W.rng(303, sig + 2)
    d, nt, ntau = 2, 16, 12
    g = ogrid(O, nt, ntau, d, h=0.05, beta=2.0, mu=0.1 if sig < 0 else -3.0, sig=sig)
    eps, H0, _ = driven_eps(r, nt, d, g.h)
    G = F.green_from_H(g, eps)
    xi = sig
    for n in (0, 5, nt):
        assert np.abs(G.R(n, n) + 1j * np.eye(d)).max() < 1e-13
    for n in (0, 3, nt):
        assert np.abs(G.L(n, n) + G.L(n, n).conj().T).max() < 1e-13
    assert np.abs(G.L(0, 0) - 1j * xi * G.M(ntau)).max() < 1e-13
    for m in (1, ntau // 2, ntau - 1):
        assert np.abs(G.T(0, m) - 1j * xi * G.M(ntau - m)).max() < 1e-12
    # particle number conserved
    nums = [(-xi * np.trace(G.L(n, n))).imag for n in range(nt + 1)]
    assert np.ptp(nums) < 1e-12
    # time-translation invariance for constant eps
    epsc = np.repeat(H0[None], nt + 2, axis=0)
    Gc = F.green_from_H(g, epsc)
    assert np.abs(Gc.R(9, 4) - Gc.R(6, 1)).max() < 1e-13


def test_agrees_with_dyson_solver_at_zero_self_energy(O):
    """Two independent discretisations of the same free function: the
    commutator-free propagator and the Dyson time stepper (BDF + Gregory, k = 5)
    with Sigma = 0. They differ by the integrators' errors only, and the
    difference shrinks ~h^4 or faster when h is halved."""
    r = W.rng(304)
    d = 2
    H0, H1 = herm(r, d), 0.8 * herm(r, d)
    errs = []
    for nt, h in ((40, 0.05), (80, 0.025)):
        g = ogrid(O, nt, 20, d, k=5, h=h, beta=2.0, mu=0.1)
        eps = np.zeros((nt + 2, d, d), np.complex128)
        eps[0] = H0
        for n in range(nt + 1):
            eps[n + 1] = H0 + np.cos(1.3 * n * h) * H1
        Gf = F.green_from_H(g, eps)
        Gd = O.HM(g)
        rc, _ = O.solve_fixed(Gd, O.HM(g), eps)
        assert rc == 0
        e = max(np.abs(Gd.ret - Gf.ret).max(), np.abs(Gd.les - Gf.les).max(), np.abs(Gd.tv - Gf.tv).max())
        assert np.abs(Gd.mat - Gf.mat).max() < 1e-12
        errs.append(e)
    assert errs[0] < 1e-5, errs
    assert errs[0] / errs[1] > 12.0, errs

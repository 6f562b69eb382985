"""Pins of the oracle's contour convolution C = A * f * B for inputs that are
not hermitian, with a matrix-valued and a time-dependent f (Sec. "Numerical
details: convolution integrals on C", Eqs. cm1-cles3; Tab. convolution).

The inputs are free levels dressed by constant matrices that do not commute:
A = X g_a, B = g_b Y. Their hermitian conjugates (the partners used for the
values outside the stored triangles) are A^ddagger = X^dag g_a and
B^ddagger = Y^dag g_b, because a free level is itself hermitian. Then
C = X F Y (g_a * phi * g_b) for f(t) = phi(t) F. For phi = 1 the scalar
factor is the resolvent identity (g_a - g_b)/(e_a - e_b) on every component;
for a time-dependent phi it is computed here from the continuous Langreth
rules by Gauss-Legendre quadrature of the closed-form free propagators.
A partner swapped for the function itself, or the factors multiplied as
A B f, changes X F Y and fails these tests.
"""
import numpy as np
import pytest

from paper_1911_01211_amd import workloads as W
from tests.test_oracle_dyson import hm

KEYS = ("mat", "ret", "les", "tv")


def _mats(d, seed):
    r = W.rng(40, seed)
    X, F, Y = (r.normal(size=(d, d)) + 1j * r.normal(size=(d, d)) for _ in range(3))
    assert np.abs(X @ F @ Y - X @ Y @ F).max() > 0.1  # the order of the factors matters
    return X, F, Y


def _dress(c, L=None, R=None):
    """L c R for every block of the scalar contour function c (d = 1)."""
    out = {}
    for key in KEYS:
        s = c[key][:, 0, 0][:, None, None]
        m = np.eye(L.shape[0] if L is not None else R.shape[0])
        out[key] = s * ((L if L is not None else m) @ (R if R is not None else m))
    return out


def _grids(h, k, T=1.5, beta=2.0, d=2):
    g1 = W.GridSpec(nt=int(round(T / h)), ntau=int(round(beta / h)), d=1, beta=beta, h=h, k=k)
    gd = W.GridSpec(nt=g1.nt, ntau=g1.ntau, d=d, beta=beta, h=h, k=k)
    return g1, gd


def _setup(O, g1, gd, X, Y, ea, eb):
    ga = W.free_gf(np.array([[ea]], np.complex128), g1)
    gb = W.free_gf(np.array([[eb]], np.complex128), g1)
    A = hm(O, gd, _dress(ga, L=X))
    Acc = hm(O, gd, _dress(ga, L=X.conj().T))
    B = hm(O, gd, _dress(gb, R=Y))
    Bcc = hm(O, gd, _dress(gb, R=Y.conj().T))
    return A, Acc, B, Bcc


@pytest.mark.parametrize("k", [2, 5])
def test_convolution_noncommuting_matrix_factors(O, k):
    """C = X F Y (g_a - g_b)/(e_a - e_b) on every component, including the
    Matsubara one; the error falls like the quadrature order."""
    d = 3
    X, F, Y = _mats(d, k)
    ea, eb = 0.5, -0.7

    def run(h):
        g1, gd = _grids(h, k, d=d)
        A, Acc, B, Bcc = _setup(O, g1, gd, X, Y, ea, eb)
        f = np.broadcast_to(F, (gd.nt + 2, d, d)).astype(np.complex128).copy()
        C = hm(O, gd)
        for n in range(-1, gd.nt + 1):
            O.convolution_timestep(n, C, A, Acc, B, Bcc, f)
        ga = W.free_gf(np.array([[ea]], np.complex128), g1)
        gb = W.free_gf(np.array([[eb]], np.complex128), g1)
        res = {key: (ga[key] - gb[key]) / (ea - eb) for key in KEYS}
        XFY = X @ F @ Y
        return {key: float(np.abs(getattr(C, key) - res[key][:, 0, 0][:, None, None] * XFY).max()
                           / np.abs(XFY).max()) for key in KEYS}

    e1, e2 = run(0.05), run(0.025)
    for key in KEYS:
        assert e2[key] < 2e-3 and np.log2(e1[key] / e2[key]) > k - 0.6, (key, e1, e2)


# ------------------------------------------------ continuous reference
_XG, _WG = np.polynomial.legendre.leggauss(48)


def _quad(fun, a, b, pieces=4):
    """Composite Gauss-Legendre integral of a smooth complex function on [a, b]."""
    if b <= a:
        return 0.0
    edges = np.linspace(a, b, pieces + 1)
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        x = 0.5 * (hi - lo) * _XG + 0.5 * (hi + lo)
        tot = tot + 0.5 * (hi - lo) * np.dot(_WG, fun(x))
    return tot


class _Level:
    """Closed-form components of a free fermion level e (Eq. G0_free, the
    conventions of the library: xi = -1, mu = 0)."""

    def __init__(self, e, beta):
        self.e, self.beta = e, beta
        self.f = 1.0 / (np.exp(beta * e) + 1.0)

    def R(self, t, s):
        return -1j * np.exp(-1j * self.e * (t - s))

    def A(self, s, t):  # advanced g^A(s, t) = conj(g^R(t, s))
        return np.conj(self.R(t, s))

    def les(self, t, s):
        return 1j * self.f * np.exp(-1j * self.e * (t - s))

    def tv(self, t, tau):  # g^rceil(t, tau)
        return 1j * self.f * np.exp(-1j * self.e * t) * np.exp(self.e * tau)

    def vt(self, tau, t):  # g^lceil(tau, t) = -xi conj(g^rceil(t, beta - tau))
        return np.conj(self.tv(t, self.beta - tau))

    def M(self, tau):  # g^M(tau) on [-beta, beta] (antiperiodic continuation)
        tau = np.asarray(tau, float)
        base = -np.exp(-self.e * np.where(tau >= 0, tau, tau + self.beta)) / (1 + np.exp(-self.beta * self.e))
        return np.where(tau >= 0, base, -base)


def _continuous(a, b, phi, phiM, t, tp, kind, tau=None):
    """Scalar factor of C = g_a * phi * g_b from the Langreth rules of the
    contour convolution (Tab. convolution), with C^M(tau) = int A^M(tau -
    tau') B^M(tau'); the imaginary-branch integral of C^< carries -i, the one
    of C^rceil none."""
    beta = a.beta
    if kind == "ret":
        return _quad(lambda s: a.R(t, s) * phi(s) * b.R(s, tp), tp, t)
    if kind == "les":
        v = _quad(lambda s: a.R(t, s) * phi(s) * b.les(s, tp), 0.0, t)
        v += _quad(lambda s: a.les(t, s) * phi(s) * b.A(s, tp), 0.0, tp)
        v += -1j * phiM * _quad(lambda x: a.tv(t, x) * b.vt(x, tp), 0.0, beta)
        return v
    if kind == "tv":
        v = _quad(lambda s: a.R(t, s) * phi(s) * b.tv(s, tau), 0.0, t)
        v += phiM * (_quad(lambda x: a.tv(t, x) * b.M(x - tau), 0.0, tau)
                     + _quad(lambda x: a.tv(t, x) * b.M(x - tau), tau, beta))
        return v
    if kind == "mat":
        return phiM * (_quad(lambda x: a.M(tau - x) * b.M(x), 0.0, tau)
                       + _quad(lambda x: a.M(tau - x) * b.M(x), tau, beta))
    raise ValueError(kind)


def test_continuous_reference_reproduces_resolvent():
    """The quadrature reference itself, at phi = 1, against the resolvent
    identity (pins the Langreth rules and the signs written above)."""
    a, b = _Level(0.5, 2.0), _Level(-0.7, 2.0)
    one = lambda s: np.ones_like(s, dtype=np.complex128)
    g1 = W.GridSpec(nt=10, ntau=8, d=1, beta=2.0, h=0.1, k=5)
    ga = W.free_gf(np.array([[0.5]], np.complex128), g1)
    gb = W.free_gf(np.array([[-0.7]], np.complex128), g1)
    res = {key: (ga[key] - gb[key])[:, 0, 0] / 1.2 for key in KEYS}
    for n, j in ((10, 3), (7, 7), (4, 0)):
        t, tp = n * g1.h, j * g1.h
        assert abs(_continuous(a, b, one, 1.0, t, tp, "ret") - res["ret"][n * (n + 1) // 2 + j]) < 1e-13
        assert abs(_continuous(a, b, one, 1.0, tp, t, "les") - res["les"][n * (n + 1) // 2 + j]) < 1e-13
    for n, m in ((3, 2), (10, 8), (0, 5)):
        v = _continuous(a, b, one, 1.0, n * g1.h, None, "tv", tau=m * g1.htau)
        assert abs(v - res["tv"][n * (g1.ntau + 1) + m]) < 1e-13
    for m in (0, 3, 8):
        assert abs(_continuous(a, b, one, 1.0, None, None, "mat", tau=m * g1.htau) - res["mat"][m]) < 1e-13


@pytest.mark.parametrize("k", [3, 5])
def test_convolution_time_dependent_f_order(O, k):
    """f(t) = phi(t) F with a complex, time-dependent phi on the real branch
    and phi_M on the imaginary one: the discrete convolution converges to the
    quadrature of the continuous Langreth rules at the scheme's order."""
    d = 2
    X, F, Y = _mats(d, 10 + k)
    ea, eb, beta = 0.5, -0.7, 2.0
    phi = lambda s: 1.0 + 0.4 * np.sin(1.3 * s) + 0.3j * np.cos(0.7 * s)
    phiM = 0.8 - 0.1j
    a, b = _Level(ea, beta), _Level(eb, beta)
    XFY = X @ F @ Y

    def run(h):
        g1, gd = _grids(h, k, T=1.0, beta=beta, d=d)
        A, Acc, B, Bcc = _setup(O, g1, gd, X, Y, ea, eb)
        f = np.empty((gd.nt + 2, d, d), np.complex128)
        f[0] = phiM * F
        for n in range(gd.nt + 1):
            f[n + 1] = phi(n * h) * F
        C = hm(O, gd)
        for n in range(-1, gd.nt + 1):
            O.convolution_timestep(n, C, A, Acc, B, Bcc, f)
        err = {key: 0.0 for key in KEYS}
        nt, ntau = gd.nt, gd.ntau
        # sample points at fixed physical times (the same for both h)
        for tn in (0.0, 0.5, 1.0):
            n = int(round(tn / h))
            for tj in (0.0, 0.3, 0.5, 1.0):
                j = int(round(tj / h))
                if j > n:
                    continue
                ref = _continuous(a, b, phi, phiM, n * h, j * h, "ret")
                err["ret"] = max(err["ret"], np.abs(C.R(n, j) - ref * XFY).max())
                ref = _continuous(a, b, phi, phiM, j * h, n * h, "les")
                err["les"] = max(err["les"], np.abs(C.L(j, n) - ref * XFY).max())
            for tau in (0.0, 0.5, 1.5, beta):
                m = int(round(tau / gd.htau))
                ref = _continuous(a, b, phi, phiM, n * h, None, "tv", tau=m * gd.htau)
                err["tv"] = max(err["tv"], np.abs(C.T(n, m) - ref * XFY).max())
        for tau in (0.0, 0.5, 1.5, beta):
            m = int(round(tau / gd.htau))
            ref = _continuous(a, b, phi, phiM, None, None, "mat", tau=m * gd.htau)
            err["mat"] = max(err["mat"], np.abs(C.M(m) - ref * XFY).max())
        s = np.abs(XFY).max()
        assert nt == int(round(1.0 / h)) and ntau == int(round(beta / h))
        return {key: v / s for key, v in err.items()}

    e1, e2 = run(0.05), run(0.025)
    for key in KEYS:
        assert e2[key] < 1e-3 and np.log2(e1[key] / e2[key]) > k - 0.6, (key, e1, e2)

"""Pins of the oracle's Fourier-series Matsubara solver
(`oracle/matsubara_fourier.py`, Sec. "Implementation: dyson", Matsubara,
"Fourier series representation"), against things the oracle does not
compute itself:
  * the cubically corrected transform is exact on cubic polynomials (closed
    antiderivative of tau^3 e^{i w tau});
  * Sigma = 0: the free Matsubara function in closed form, for fermions and
    bosons, with the error of the truncated Fourier sum falling like 1/N_w
    (doubling the oversampling halves it); a wrong sign of the tail
    correction, of the jump function c(tau) or of the frequencies leaves an
    O(1) error;
  * the two-level embedding: Sigma^M = V^2 g_bath, whose exact G^M is the 2 x 2
    block of the free 4 x 4 function (downfolding); the mean error falls at
    second order in h_tau (the paper's statement for this method), the
    largest (at tau = 0, beta) like 1/N_w."""
import numpy as np
import pytest

from oracle import matsubara_fourier as MF
from paper_1911_01211_amd import workloads as W

H2 = np.array([[-1.0, 0.5], [0.5, 1.0]], np.complex128)


def test_transform_exact_on_cubics():
    b, n = 2.0, 12
    tau = np.arange(n + 1) * b / n
    w = np.array([0.7, 5.3, 31.0, -12.1])
    got = MF.fourier_samples(tau ** 3, b, w)

    def prim(t, ww):  # antiderivative of t^3 e^{i w t}
        z = 1j * ww
        return np.exp(z * t) * (t ** 3 / z - 3 * t ** 2 / z ** 2 + 6 * t / z ** 3 - 6 / z ** 4)

    ref = np.array([prim(b, ww) - prim(0.0, ww) for ww in w])
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("xi,mu", [(-1, 0.1), (1, -2.0)])
def test_free_function_and_tail(O, xi, mu):
    g = O.Grid(nt=4, ntau=100, d=2, sig=xi, beta=5.0, h=0.05, mu=mu)
    ref = O.free_mat(g, H2)
    zero = np.zeros((101, 2, 2), np.complex128)
    e = [np.abs(MF.solve(H2, zero, 5.0, mu, xi, p) - ref).max() for p in (10, 20)]
    assert e[0] < 2e-3 and 0.4 < e[1] / e[0] < 0.6, e


def test_embedding_orders():
    mean, mx = [], []
    for ntau in (50, 100, 200):
        g = W.GridSpec(nt=4, ntau=ntau, d=2, beta=5.0, h=0.05, k=5)
        eps, S, Ge = W.two_level_embedding(g)
        err = np.abs(MF.solve(eps[0], S["mat"], 5.0, 0.0, -1, 10) - Ge["mat"])
        mean.append(err.mean())
        mx.append(err.max())
    for a, b in zip(mean, mean[1:]):
        assert np.log2(a / b) > 1.8, mean
    for a, b in zip(mx, mx[1:]):
        assert 0.8 < np.log2(a / b) < 1.2, mx
    assert mx[-1] < 2e-4

"""Pins of the oracle's quadrature weights against the printed tables, an
independent exact-rational construction written here, polynomial
exactness and the Gregory convergence experiment (Fig. gregoryintegration)."""
import os
from fractions import Fraction as Fr
from math import factorial

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


def lagrange_coeffs(k):
    """Monomial coefficients c[l][a] of the Lagrange basis L_l on nodes 0..k,
    built by multiplying out prod_{i != l} (x - i)/(l - i)."""
    out = []
    for l in range(k + 1):
        poly = [Fr(1)]
        for i in range(k + 1):
            if i == l:
                continue
            new = [Fr(0)] * (len(poly) + 1)
            for a, c in enumerate(poly):
                new[a + 1] += c / (l - i)
                new[a] += c * Fr(-i, l - i)
            poly = new
        out.append(poly)
    return out


def poly_int(c, lo, hi):
    return sum(ca * (Fr(hi) ** (a + 1) - Fr(lo) ** (a + 1)) / (a + 1) for a, ca in enumerate(c))


def test_bdf_table(O):
    for row in _read("bdf_weights.txt"):
        k = int(row[0])
        printed = [float(Fr(x)) for x in row[1:]]
        got = O.weights(k)["a"]
        assert np.array_equal(got, np.array(printed)), (k, got, printed)


def test_gregory_table_exact(O):
    for k_, blk, l, *vals in _read("gregory_weights.txt"):
        k, l = int(k_), int(l)
        n = l if blk == "s" else k + 1 + l
        for j, v in enumerate(vals):
            assert Fr(*O.gregory_rational(k, n, j)) == Fr(v), (k, blk, l, j)
            assert O.gregory(k, n, j) == float(Fr(v))


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_weights_vs_independent_rationals(O, k):
    W = O.weights(k)
    c = lagrange_coeffs(k)
    # P_{a,l} = coefficient of x^a in L_l (Eq. integrator_P: P = M^{-1})
    P = np.array([[float(c[l][a]) for l in range(k + 1)] for a in range(k + 1)])
    assert np.allclose(W["P"], P, rtol=0, atol=1e-14 * np.abs(P).max())
    for m in range(k + 1):
        for l in range(k + 1):
            dl = sum(a * c[l][a] * Fr(m) ** (a - 1) for a in range(1, k + 1))
            assert abs(W["D"][m, l] - float(dl)) <= 1e-13 * max(1, abs(float(dl)))
            for n in range(k + 1):
                il = poly_int(c[l], m, n)
                assert abs(W["I"][m, n, l] - float(il)) <= 1e-13 * max(1, abs(float(il)))
    # R_{m;r,s} = int_0^m L_r(m - x) L_s(x) dx expanded term by term
    for m in range(k + 1):
        for r in range(k + 1):
            for s in range(k + 1):
                val = Fr(0)
                for a, ca in enumerate(c[r]):
                    for b, cb in enumerate(c[s]):
                        val += ca * cb * Fr(m) ** (a + b + 1) * Fr(
                            factorial(a) * factorial(b), factorial(a + b + 1))
                assert abs(W["R"][m, r, s] - float(val)) <= 1e-12 * max(1, abs(float(val)))


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5])
def test_gregory_exact_on_polynomials(O, k):
    # Gregory rules integrate polynomials of degree <= k exactly for every n,
    # and the weights of every row sum to n.
    for n in range(0, 3 * k + 5):
        jmax = max(n, k)
        w = [Fr(*O.gregory_rational(k, n, j)) for j in range(jmax + 1)]
        assert sum(w) == n
        for q in range(k + 1):
            assert sum(wj * Fr(j) ** q for j, wj in enumerate(w)) == Fr(n) ** (q + 1) / (q + 1)
        if n > 2 * k + 1:
            # interior weights exactly one, symmetric ends
            assert all(wj == 1 for wj in w[k + 1:n - k])
            assert w[:k + 1] == w[::-1][:k + 1]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_gregory_convergence_order(O, k):
    # Fig. gregoryintegration: mean |I_n - I_n^ex| over a grid on [0, 5 pi/2]
    # for int_0^x exp(i x') dx' = -i (exp(i x) - 1) scales as N^{-(k+2)}.
    def mean_err(N):
        xmax = 2.5 * np.pi
        h = xmax / N
        y = np.exp(1j * h * np.arange(N + k + 1))
        errs = []
        for n in range(N + 1):
            jmax = max(n, k)
            w = np.array([O.gregory(k, n, j) for j in range(jmax + 1)])
            val = h * np.dot(w, y[:jmax + 1])
            errs.append(abs(val - (-1j) * (np.exp(1j * n * h) - 1)))
        return np.mean(errs)

    e1, e2 = mean_err(40), mean_err(80)
    slope = np.log2(e1 / e2)
    assert slope > k + 1.5, (k, slope)


def test_boundary_convolution_exact(O):
    # Eq. integrator_R is exact when F and G are polynomials of degree <= k.
    k = 5
    W = O.weights(k)
    rr = np.random.default_rng(3)
    F = rr.normal(size=k + 1)
    G = rr.normal(size=k + 1)
    xs = np.arange(k + 1)
    for m in range(k + 1):
        approx = sum(W["R"][m, r, s] * np.polyval(F, r) * np.polyval(G, s)
                     for r in range(k + 1) for s in range(k + 1))
        # exact int_0^m F(m-x) G(x) dx with numpy polynomial algebra
        Fm = np.poly1d(F)(np.poly1d([-1, m]))
        prod = np.polyint(Fm * np.poly1d(G))
        exact = prod(m) - prod(0)
        assert abs(approx - exact) <= 1e-10 * max(1, abs(exact)), (m, approx, exact)
    assert xs.size == k + 1

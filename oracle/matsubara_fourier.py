"""Fourier-series solution of the Matsubara Dyson equation.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the GPU library never does.

Follows the "Fourier series representation" of Sec. "Implementation: dyson"
(the Matsubara part), the method the paper uses as a fast initial guess:
  * Sigma(i w_m) = int_0^beta Sigma^M(tau) e^{i w_m tau} dtau, integrating
    the piecewise-cubic interpolant of the samples on the tau grid exactly
    (the cubically corrected discrete Fourier transform): on interval
    [tau_J, tau_{J+1}] the cubic through the four grid points J-1 .. J+2
    (J .. J+3 on the first interval, J-2 .. J+1 on the last);
  * G(i w_m) = [i w_m - x - Sigma(i w_m)]^{-1} with x = eps(0^-) - mu: the
    algebraic form of the Matsubara Dyson equation (the printed form drops
    the 1 on the right); at Sigma = 0 it is the Fourier coefficient
    1 / (i w - x) of the free function -V e^{-x tau} / (1 - xi e^{-beta x}) V^dag;
  * the jump of G^M at tau = 0 and beta is removed before the sum: with the
    jump G^M(0+) - xi G^M(beta-) = -1 of this library's convention, the
    function G~ = G^M + c 1 with c = 1/2 (fermions) or c = 1/2 - tau/beta
    (bosons) is continuous in its (anti-)periodic extension; its
    coefficients are G~(i w) = G(i w) - 1/(i w) for both statistics (nothing
    at the bosonic w = 0), and G^M(tau) = (1/beta) sum_m e^{-i w_m tau}
    G~(i w_m) - c(tau) 1. (The printed bosonic c = tau/beta - 1/2 and tail
    -xi/(i w) have the opposite sign for bosons: with them the extension
    keeps a jump of 2; the fermionic case is the printed one.)
  * frequencies: fermions w_m = (2m+1) pi / beta, m = -Nw .. Nw-1; bosons
    w_m = 2 m pi / beta, m = -Nw .. Nw; Nw = p Ntau (oversampling p, 10 by
    default).
The interpolant times e^{i w tau} is integrated by 64-point Gauss-Legendre
quadrature on every interval (exact to rounding for the frequencies used:
w h_tau <= 2 pi p). Plain numpy, complex128.
"""
from __future__ import annotations

import numpy as np

NGL = 64


def frequencies(ntau: int, beta: float, xi: int, p: int = 10) -> np.ndarray:
    nw = p * ntau
    if xi == -1:
        m = np.arange(-nw, nw)
        return (2 * m + 1) * np.pi / beta
    m = np.arange(-nw, nw + 1)
    return 2 * m * np.pi / beta


def _stencil(J: int, ntau: int) -> int:
    """First of the four grid points whose cubic interpolates interval J."""
    return min(max(J - 1, 0), ntau - 3)


def fourier_samples(f: np.ndarray, beta: float, w: np.ndarray) -> np.ndarray:
    """int_0^beta f(tau) e^{i w tau} dtau for the piecewise-cubic interpolant
    of the samples f [ntau+1, ...] (ntau >= 3), at every frequency in w."""
    ntau = f.shape[0] - 1
    h = beta / ntau
    x, wt = np.polynomial.legendre.leggauss(NGL)
    u = 0.5 * (x + 1.0)  # nodes on [0, 1]
    wt = 0.5 * wt
    out = np.zeros((len(w),) + f.shape[1:], np.complex128)
    for J in range(ntau):
        s = _stencil(J, ntau)
        nodes = np.arange(s, s + 4) - J  # grid offsets of the stencil, in units of h
        # Lagrange basis of the stencil at the quadrature nodes
        L = np.ones((4, NGL))
        for i in range(4):
            for jj in range(4):
                if jj != i:
                    L[i] *= (u - nodes[jj]) / (nodes[i] - nodes[jj])
        vals = np.tensordot(L.T, f[s:s + 4], axes=(1, 0))  # interpolant at the nodes [NGL, ...]
        ph = np.exp(1j * np.outer(w, (J + u) * h)) * (wt * h)  # [nw, NGL]
        out += np.tensordot(ph, vals, axes=(1, 0))
    return out


def solve(eps_m1: np.ndarray, Smat: np.ndarray, beta: float, mu: float, xi: int, p: int = 10):
    """G^M on the tau grid of Smat [ntau+1, d, d] (Sigma^M; zeros for the free
    problem), eps_m1 = eps(0^-) [d, d]. Returns G^M [ntau+1, d, d]."""
    ntau, d = Smat.shape[0] - 1, Smat.shape[1]
    w = frequencies(ntau, beta, xi, p)
    Sw = fourier_samples(Smat, beta, w)
    x = np.asarray(eps_m1, np.complex128) - mu * np.eye(d)
    A = 1j * w[:, None, None] * np.eye(d)[None] - x[None] - Sw
    Gw = np.linalg.inv(A)
    nz = w != 0.0
    Gt = Gw.copy()
    Gt[nz] -= (1.0 / (1j * w[nz]))[:, None, None] * np.eye(d)[None]
    tau = np.arange(ntau + 1) * beta / ntau
    E = np.exp(-1j * np.outer(tau, w)) / beta  # [ntau+1, nw]
    G = np.tensordot(E, Gt, axes=(1, 0))
    c = 0.5 * np.ones_like(tau) if xi == -1 else 0.5 - tau / beta
    return G - c[:, None, None] * np.eye(d)[None]

"""Free Green's function of a time-dependent single-particle Hamiltonian.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the GPU library never does.

Follows Sec. "Implementation: Free Green's functions" of the paper:
  * G^M is the free Matsubara function of eps(0^-) - mu (the same formula the
    Matsubara solver starts from, `oracle.free_mat`);
  * the propagator U_{n+1,n} is the fourth-order commutator-free exponential
    of Eq. cf4, with eps at the two intermediate times taken from the
    polynomial through the k+1 points n-k+1 .. n+1 (0 .. k near the start);
  * U_{n,0} = U_{n,n-1} ... U_{1,0} (semigroup property);
  * the real-time and mixed components are those of Eq. G0_free:
      G^R(t_n, t_j)   = -i U_{n,0} U_{j,0}^dag,
      G^<(t_j, t_n)   = -i xi U_{j,0} rho U_{n,0}^dag,
      G^rceil(t_n, tau) = -i xi U_{n,0} R diag(f(x) e^{x tau}) R^dag,
    with eps(0^-) - mu = R diag(x) R^dag, f(x) = 1 / (e^{beta x} - xi) and
    rho = R diag(f(x)) R^dag.
The real-time branch evolves with eps(t) - mu, as the Dyson equations of this
library do on every branch (with mu = 0 this is the printed form; otherwise
the two differ by the gauge phase e^{i mu (t - t')}), so that G_0 solves the
library's own Dyson equation at Sigma = 0.
Readings of the printed text (also listed with the design notes): the
exponents of Eq. cf4 carry the step h (the printed form omits it; without it
a constant Hamiltonian would not give exp(-i h eps) per step); G^R carries
the factor -i that the printed right-hand side drops; G^< carries -i xi (the
printed i is its fermion case xi = -1, consistent with the printed G^rceil).
Plain numpy / scipy, complex128, loops over time steps.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import oracle as O

SQ3 = np.sqrt(3.0)
A1 = (3.0 - 2.0 * SQ3) / 12.0
A2 = (3.0 + 2.0 * SQ3) / 12.0
C1 = (1.0 - 1.0 / SQ3) / 2.0
C2 = (1.0 + 1.0 / SQ3) / 2.0


def interp_points(n: int, k: int) -> np.ndarray:
    """Grid indices of the k+1 interpolation points of the step n -> n+1."""
    j0 = max(0, n - k + 1)
    return np.arange(j0, j0 + k + 1)


def lagrange(pts: np.ndarray, t: float) -> np.ndarray:
    """Lagrange basis of the points pts (grid indices) at t (grid units)."""
    w = np.ones(len(pts))
    for i, pi in enumerate(pts):
        for m, pm in enumerate(pts):
            if m != i:
                w[i] *= (t - pm) / (pi - pm)
    return w


def eps_at(eps: np.ndarray, n: int, k: int, t: float) -> np.ndarray:
    """eps at time t (grid units) from the polynomial of the step n -> n+1.
    eps has entry m+1 for t_m (entry 0 is eps(0^-))."""
    pts = interp_points(n, k)
    w = lagrange(pts, t)
    return sum(w[i] * eps[p + 1] for i, p in enumerate(pts))


def step_propagator(eps: np.ndarray, n: int, k: int, h: float, mu: float = 0.0) -> np.ndarray:
    """U_{n+1,n} by Eq. cf4, for the one-body Hamiltonian eps(t) - mu."""
    d = eps.shape[-1]
    e1 = eps_at(eps, n, k, n + C1) - mu * np.eye(d)
    e2 = eps_at(eps, n, k, n + C2) - mu * np.eye(d)
    left = scipy.linalg.expm(-1j * h * (A1 * e1 + A2 * e2))
    right = scipy.linalg.expm(-1j * h * (A2 * e1 + A1 * e2))
    return left @ right


def propagators(eps: np.ndarray, nt: int, k: int, h: float, mu: float = 0.0) -> np.ndarray:
    """U_{n,0}, n = 0..nt, for eps(t) - mu."""
    d = eps.shape[-1]
    U = np.zeros((nt + 1, d, d), np.complex128)
    U[0] = np.eye(d)
    for n in range(nt):
        U[n + 1] = step_propagator(eps, n, k, h, mu) @ U[n]
    return U


def fermi(x: np.ndarray, beta: float, xi: int) -> np.ndarray:
    """f(x) = 1 / (e^{beta x} - xi), without overflow for large beta x."""
    out = np.empty_like(x)
    for i, xa in enumerate(x):
        if xa >= 0:
            out[i] = np.exp(-beta * xa) / (1.0 - xi * np.exp(-beta * xa))
        else:
            out[i] = 1.0 / (np.exp(beta * xa) - xi)
    return out


def mixed_factor(x: np.ndarray, beta: float, xi: int, tau: float) -> np.ndarray:
    """f(x) e^{x tau} for 0 <= tau <= beta, without overflow."""
    out = np.empty_like(x)
    for i, xa in enumerate(x):
        if xa >= 0:
            out[i] = np.exp(-xa * (beta - tau)) / (1.0 - xi * np.exp(-beta * xa))
        else:
            out[i] = np.exp(xa * tau) / (np.exp(beta * xa) - xi)
    return out


def green_slices(g: O.Grid, eps: np.ndarray, slices) -> dict:
    """Rows n of G^R and G^rceil and column n of G^< (same formulas as
    green_from_H) for the given slices only: {n: (ret[n+1], les[n+1], tv[ntau+1])}."""
    d, ntau, xi = g.d, g.ntau, g.sig
    x, R = np.linalg.eigh(eps[0] - g.mu * np.eye(d))
    rho = R @ np.diag(fermi(x, g.beta, xi)) @ R.conj().T
    F = [R @ np.diag(mixed_factor(x, g.beta, xi, m * g.htau)) @ R.conj().T for m in range(ntau + 1)]
    U = propagators(eps, max(slices), g.k, g.h, g.mu)
    out = {}
    for n in slices:
        ret = np.array([-1j * U[n] @ U[j].conj().T for j in range(n + 1)])
        les = np.array([-1j * xi * U[j] @ rho @ U[n].conj().T for j in range(n + 1)])
        tv = np.array([-1j * xi * U[n] @ F[m] for m in range(ntau + 1)])
        out[n] = (ret, les, tv)
    return out


def green_from_H(g: O.Grid, eps: np.ndarray) -> O.HM:
    """All components of G_0 on the grid g for eps[(nt+2), d, d]."""
    d, nt, ntau, xi = g.d, g.nt, g.ntau, g.sig
    G = O.HM(g)
    G.mat[...] = O.free_mat(g, eps)
    x, R = np.linalg.eigh(eps[0] - g.mu * np.eye(d))
    rho = R @ np.diag(fermi(x, g.beta, xi)) @ R.conj().T
    F = [R @ np.diag(mixed_factor(x, g.beta, xi, m * g.htau)) @ R.conj().T for m in range(ntau + 1)]
    U = propagators(eps, nt, g.k, g.h, g.mu)
    for n in range(nt + 1):
        for j in range(n + 1):
            G.R(n, j)[...] = -1j * U[n] @ U[j].conj().T
            G.L(j, n)[...] = -1j * xi * U[j] @ rho @ U[n].conj().T
        for m in range(ntau + 1):
            G.T(n, m)[...] = -1j * xi * U[n] @ F[m]
    return G

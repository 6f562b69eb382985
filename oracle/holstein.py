"""Holstein model in DMFT on the Bethe lattice with the unrenormalized Migdal
impurity solver (Sec. "DMFT for the Holstein model").

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the GPU library never does.

Single band, spin-symmetric, one phonon mode of frequency w0 per site:
  free phonon propagator   D0(z,z') = -i <T_C X(z) X(z')>_0,  X = a + a^dag,
  phonon displacement      X(t) = -2 g(0) n(0) / w0
                                  + int_0^t D0^R(t,s) [g(s) n(s) - g(0) n(0)] ds   (Eq. X),
  mean field               Sigma^MF(t) = g(t) X(t)                                (Eq. H_mf_Holstein),
  uMig self-energy         Sigma(t,t') = i g(t) g(t') D0(t,t') G(t,t')            (Eq. uMig_el),
  Bethe self-consistency   Delta(t,t') = J(t) G(t,t') J(t')                       (Eq. bethe_condition),
  impurity Dyson equation  [i d_t + mu - e0 - Sigma^MF(t)] G - (Delta + Sigma) * G = delta
                                                                                  (Eq. Dyson_imp),
with n(t) = 2 n_sigma(t) the density of both spins. Time-dependent scalars
(g, J) are arrays of nt + 2 entries, entry n + 1 at t_n and entry 0 on the
Matsubara branch (t = 0^-).
"""
from __future__ import annotations

import numpy as np

from . import free_green as FG
from . import kspace as KS
from . import oracle as O


def phonon_d0(g: O.Grid, w0: float) -> O.HM:
    """D0 of one mode on the bosonic grid of g (d = 1, mu = 0). The time
    ordering of X X gives D0(z,z') = G_a(z,z') + G_a(z',z), with G_a the free
    single-pole function of the level w0 (free_green, pinned on its own); the
    second term's components follow from the contour relations:
      M:     G_a(-tau) = xi G_a^M(beta - tau),
      R:     [G_a^A(t',t)] = conj(G_a^R(t,t'))                    (d = 1),
      <:     G_a^>(t_n,t_j) = G_a^R(t_n,t_j) + G_a^<(t_n,t_j),
      rceil: G_a^lceil(tau,t) = -xi conj(G_a^rceil(t, beta - tau)).
    """
    gb = O.Grid(g.nt, g.ntau, 1, +1, g.k, g.beta, g.h, 0.0)
    eps = np.full((g.nt + 2, 1, 1), w0, np.complex128)
    Ga = FG.green_from_H(gb, eps)
    D = O.HM(gb)
    xi = 1.0
    nt, ntau = g.nt, g.ntau
    for m in range(ntau + 1):
        D.mat[m] = Ga.mat[m] + xi * Ga.mat[ntau - m]
    for n in range(nt + 1):
        for j in range(n + 1):
            D.R(n, j)[...] = Ga.R(n, j) + np.conj(Ga.R(n, j))
            lo = Ga.L(j, n)                                     # G_a^<(t_j, t_n)
            back = lo if j == n else -np.conj(lo)               # G_a^<(t_n, t_j)
            D.L(j, n)[...] = lo + Ga.R(n, j) + back
        for m in range(ntau + 1):
            D.T(n, m)[...] = Ga.T(n, m) - xi * np.conj(Ga.T(n, ntau - m))
    return D


def scale(n: int, C: O.HM, A: O.HM, f, beta: float = 0.0):
    """C = beta C + f(t) A(t,t') f(t') on slice n (n = -1: Matsubara, both
    arguments on the vertical branch, f[0]); f real, entry m + 1 at t_m."""
    g = C.g
    f = np.asarray(f, float)
    if n == -1:
        C.mat[...] = beta * C.mat + f[0] * A.mat * f[0]
        return
    for j in range(n + 1):
        C.R(n, j)[...] = beta * C.R(n, j) + f[n + 1] * A.R(n, j) * f[j + 1]
        C.L(j, n)[...] = beta * C.L(j, n) + f[j + 1] * A.L(j, n) * f[n + 1]
    for m in range(g.ntau + 1):
        C.T(n, m)[...] = beta * C.T(n, m) + f[n + 1] * A.T(n, m) * f[0]


def add(n: int, C: O.HM, A: O.HM):
    """C += A on slice n."""
    scale(n, C, A, np.ones(C.g.nt + 2), 1.0)


def density(n: int, G: O.HM) -> float:
    """n(t_n) of both spins: 2 Im G^<(t_n,t_n); n = -1: -2 G^M(beta)."""
    if n == -1:
        return float(-2.0 * G.M(G.g.ntau)[0, 0].real)
    return float(2.0 * G.L(n, n)[0, 0].imag)


def displacement(n: int, G: O.HM, gel, w0: float, X):
    """X(t_n) by Eq. X into X[n + 1] (n = -1: the equilibrium value
    -2 g(0^-) n / w0 of the Matsubara density into X[0]). The integral is the
    library's quadrature of order k on [0, t_n]: the start weights over the
    points 0..k for n <= k, the Gregory weights beyond; D0^R(t,s) = -2 sin(w0 (t - s))."""
    g = G.g
    gel = np.asarray(gel, float)
    if n == -1:
        X[0] = -2.0 * gel[0] * density(-1, G) / w0
        return
    n0 = density(0, G)
    src0 = gel[1] * n0
    acc = 0.0
    for j in range(max(n, g.k) + 1):
        w = O.gregory(g.k, n, j)
        if w == 0.0:
            continue
        d0r = -2.0 * np.sin(w0 * (n - j) * g.h)
        acc += w * d0r * (gel[j + 1] * density(j, G) - src0)
    X[n + 1] = -2.0 * gel[1] * n0 / w0 + g.h * acc


def solve_holstein(G: O.HM, J, gel, w0: float, e0: float = 0.0, mats_iters=30, boot_iters=8, ncorr=4,
                   nt_stop=None):
    """Bethe-lattice DMFT with the uMig solver for the local G (zero on entry,
    d = 1, fermion grid with the chemical potential mu): the same sequence as
    the library's driver.
      Matsubara: mats_iters x {X, Delta^M, Sigma^M; G^M},
      start-up:  boot_iters x {X, Delta, Sigma on slices 0..k; start-up of G},
      steps:     extrapolation of G, then ncorr x {X, Delta, Sigma on slice n; step n}.
    The self-energy of the Dyson step is Delta + Sigma; the level is
    e0 + g(t) X(t). Returns (D0g, Delta, Sigma, X, eps)."""
    g = G.g
    k = g.k
    nt_stop = g.nt if nt_stop is None else nt_stop
    D0 = phonon_d0(g, w0)
    D0g = O.HM(D0.g)
    scale(-1, D0g, D0, gel)
    for n in range(g.nt + 1):
        scale(n, D0g, D0, gel)
    Delta, S, St = O.HM(g), O.HM(g), O.HM(g)
    X = np.zeros(g.nt + 2)
    eps = np.zeros((g.nt + 2, 1, 1), np.complex128)
    gel = np.asarray(gel, float)

    def selfenergies(n):
        scale(n, Delta, G, J)
        KS.sigma_gw(n, [G], [D0g], [S])
        scale(n, St, S, np.ones(g.nt + 2), 0.0)
        add(n, St, Delta)

    assert O.dyson_mat(G, St, np.full((1, 1), e0, np.complex128)) == 0
    for _ in range(mats_iters):
        displacement(-1, G, gel, w0, X)
        eps[0] = e0 + gel[0] * X[0]
        selfenergies(-1)
        assert O.dyson_mat(G, St, eps[0]) == 0
    for _ in range(boot_iters):
        for n in range(k + 1):
            displacement(n, G, gel, w0, X)
            eps[n + 1] = e0 + gel[n + 1] * X[n + 1]
            selfenergies(n)
        assert O.dyson_start(G, St, eps) == 0
    for n in range(k + 1, nt_stop + 1):
        O.extrapolate(n - 1, G)
        for _ in range(ncorr):
            displacement(n, G, gel, w0, X)
            eps[n + 1] = e0 + gel[n + 1] * X[n + 1]
            selfenergies(n)
            assert O.dyson_timestep(n, G, St, eps) == 0
    return D0g, Delta, S, X, eps

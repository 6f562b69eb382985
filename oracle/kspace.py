"""Momentum-convolution self-energies of the k-space GW example.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the GPU library never does.

For a translationally invariant lattice of Nk momenta (indices mod Nk) and
orbital-diagonal interaction (Sec. "Example: GW for the translationally
invariant Hubbard model"):
  polarization (Eq. Pol)     Pi_k(t,t')    = -(i/Nk) sum_q G_{k+q}(t,t') G_q(t',t),
  self-energy (Eq. Sigmak)   Sigma_k(t,t') =  (i/Nk) sum_q G_{k-q}(t,t') dW_q(t,t'),
element by element in the orbital indices (Pi_{k,ij} takes G_{q,ji}(t',t),
Sigma_{k,ij} takes dW_{q,ij}(t,t')). The two-time products are the bubble
diagrams of Sec. "Contour products" (Eqs. def_bubble1, def_bubble2), written
here on the stored components of one time slice n (tstp = -1: Matsubara).
Plain numpy; the momentum sums are explicit loops over q.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


# ------------------------------------------------ components at any times
# (hermitian contour functions in the canonical layout, Eq. storage_herm)
def R(X: O.HM, a, b):
    """X^R(t_a, t_b), a >= b (stored)."""
    return X.R(a, b)


def L(X: O.HM, a, b):
    """X^<(t_a, t_b) for any a, b: stored for a <= b, else -[X^<(t_b,t_a)]^dag."""
    if a <= b:
        return X.L(a, b)
    return -X.L(b, a).conj().T


def A(X: O.HM, a, b):
    """X^A(t_a, t_b) = [X^R(t_b, t_a)]^dag, a <= b."""
    return X.R(b, a).conj().T


def Gt(X: O.HM, a, b):
    """X^>(t_a, t_b), a >= b: X^R + X^< (G^R(t,t) = G^> - G^< at equal times)."""
    return X.R(a, b) + L(X, a, b)


def Tv(X: O.HM, n, m):
    """X^rceil(t_n, tau_m)."""
    return X.T(n, m)


def Vt(X: O.HM, m, n):
    """X^lceil(tau_m, t_n) = -xi [X^rceil(t_n, beta - tau_m)]^dag."""
    return -X.g.sig * X.T(n, X.g.ntau - m).conj().T


def Mneg(X: O.HM, m):
    """X^M(-tau_m) = xi X^M(beta - tau_m)."""
    return X.g.sig * X.M(X.g.ntau - m)


# ---------------------------------------------------------- the bubbles
def bubble1(n, Aa: O.HM, Bb: O.HM):
    """C(t,t') = i A(t,t') B(t',t) elementwise (C_ij = i A_ij B_ji), Eq. def_bubble1,
    on slice n: dict with the stored blocks ret[m], les[m] (C^<(t_m,t_n)),
    tv[m] (C^rceil(t_n,tau_m)); n = -1: mat[m]."""
    g = Aa.g
    out = {}
    if n == -1:
        # X^M(tau) = -i X(-i tau, 0) for every contour function (the form that
        # gives X^rceil(0, tau) = i xi X^M(beta - tau)), so
        # C^M(tau) = A(-i tau, 0) B(0, -i tau) = (i A^M(tau)) (i B^M(-tau))
        out["mat"] = np.array([-Aa.M(m) * Mneg(Bb, m).T for m in range(g.ntau + 1)])
        return out
    # C^R(t,t') = i A^R(t,t') B^<(t',t) + i A^<(t,t') B^A(t',t)
    out["ret"] = np.array([1j * R(Aa, n, m) * L(Bb, m, n).T + 1j * L(Aa, n, m) * A(Bb, m, n).T
                           for m in range(n + 1)])
    # C^<(t,t') = i A^<(t,t') B^>(t',t)
    out["les"] = np.array([1j * L(Aa, m, n) * Gt(Bb, n, m).T for m in range(n + 1)])
    # C^rceil(t,tau) = i A^rceil(t,tau) B^lceil(tau,t)
    out["tv"] = np.array([1j * Tv(Aa, n, m) * Vt(Bb, m, n).T for m in range(g.ntau + 1)])
    return out


def bubble2(n, Aa: O.HM, Bb: O.HM):
    """C(t,t') = i A(t,t') B(t,t') elementwise, Eq. def_bubble2, on slice n."""
    g = Aa.g
    out = {}
    if n == -1:
        # C^M(tau) = -i C(-i tau, 0) = A(-i tau, 0) B(-i tau, 0) = (i A^M) (i B^M)
        out["mat"] = np.array([-Aa.M(m) * Bb.M(m) for m in range(g.ntau + 1)])
        return out
    # C^R = i A^R B^R + i A^< B^R + i A^R B^<   (at (t_n, t_m), n >= m)
    out["ret"] = np.array([1j * R(Aa, n, m) * R(Bb, n, m) + 1j * L(Aa, n, m) * R(Bb, n, m)
                           + 1j * R(Aa, n, m) * L(Bb, n, m) for m in range(n + 1)])
    # C^< = i A^< B^<
    out["les"] = np.array([1j * L(Aa, m, n) * L(Bb, m, n) for m in range(n + 1)])
    # C^rceil = i A^rceil B^rceil
    out["tv"] = np.array([1j * Tv(Aa, n, m) * Tv(Bb, n, m) for m in range(g.ntau + 1)])
    return out


def _store(n, C: O.HM, blocks: dict, scale):
    g = C.g
    if n == -1:
        C.mat[...] = scale * blocks["mat"]
        return
    o = n * (n + 1) // 2
    C.ret[o:o + n + 1] = scale * blocks["ret"]
    C.les[o:o + n + 1] = scale * blocks["les"]
    C.tv[n * (g.ntau + 1):(n + 1) * (g.ntau + 1)] = scale * blocks["tv"]


def polarization(n, G: list, Pi: list, alpha=1.0):
    """alpha Pi_k, Pi_k = -(1/Nk) sum_q Bubble1(G_{k+q}, G_q), on slice n, for every k."""
    nk = len(G)
    for k in range(nk):
        acc = None
        for q in range(nk):
            b = bubble1(n, G[(k + q) % nk], G[q])
            acc = b if acc is None else {c: acc[c] + b[c] for c in acc}
        _store(n, Pi[k], acc, -alpha / nk)


def sigma_gw(n, G: list, dW: list, Sigma: list, alpha=1.0):
    """alpha Sigma_k, Sigma_k = (1/Nk) sum_q Bubble2(G_{k-q}, dW_q), on slice n, for every k."""
    nk = len(G)
    for k in range(nk):
        acc = None
        for q in range(nk):
            b = bubble2(n, G[(k - q) % nk], dW[q])
            acc = b if acc is None else {c: acc[c] + b[c] for c in acc}
        _store(n, Sigma[k], acc, alpha / nk)


def solve_gw(G: list, eps: list, U: float, mats_iters=10, boot_iters=6, ncorr=3, nt_stop=None):
    """Self-consistent k-space GW propagation (correlation part; Sec. "Example:
    GW for the translationally invariant Hubbard model"): with the bosonic
    kernel F_k = -U Pi_k, the screened interaction dW_k = U Pi_k U + U Pi_k * dW_k
    is dW_k = -U X_k with (1 + F_k) * X_k = F_k (the integral form, Eq. vie2),
    and Sigma_k = -U (i/Nk) sum_q G_{k-q} X_q.
      Matsubara: mats_iters x {Pi, X, Sigma on the Matsubara branch; G^M},
      start-up:  boot_iters x {Pi, X, Sigma on slices 0..k; start-up of G},
      steps:     extrapolation of G, then ncorr x {Pi, X, Sigma on slice n; step n}.
    G[k] are the momenta's functions (zero on entry), eps[k] their levels
    ((nt+2) x d x d, entry 0 = eps(0^-)). Returns (F, X, Sigma)."""
    g = G[0].g
    nk, k = len(G), g.k
    nt_stop = g.nt if nt_stop is None else nt_stop
    gb = O.Grid(g.nt, g.ntau, g.d, 1, g.k, g.beta, g.h, g.mu)
    F = [O.HM(gb) for _ in range(nk)]
    X = [O.HM(gb) for _ in range(nk)]
    S = [O.HM(g) for _ in range(nk)]
    for q in range(nk):
        assert O.dyson_mat(G[q], S[q], eps[q][0]) == 0
    for _ in range(mats_iters):
        polarization(-1, G, F, -U)
        for q in range(nk):
            assert O.vie2_mat(X[q], F[q], F[q]) == 0
        sigma_gw(-1, G, X, S, -U)
        for q in range(nk):
            assert O.dyson_mat(G[q], S[q], eps[q][0]) == 0
    for _ in range(boot_iters):
        for n in range(k + 1):
            polarization(n, G, F, -U)
        for q in range(nk):
            assert O.vie2_start(X[q], F[q], F[q], F[q]) == 0
        for n in range(k + 1):
            sigma_gw(n, G, X, S, -U)
        for q in range(nk):
            assert O.dyson_start(G[q], S[q], eps[q]) == 0
    for n in range(k + 1, nt_stop + 1):
        for q in range(nk):
            O.extrapolate(n - 1, G[q])
        for _ in range(ncorr):
            polarization(n, G, F, -U)
            for q in range(nk):
                assert O.vie2_timestep(n, X[q], F[q], F[q], F[q]) == 0
            sigma_gw(n, G, X, S, -U)
            for q in range(nk):
                assert O.dyson_timestep(n, G[q], S[q], eps[q]) == 0
    return F, X, S

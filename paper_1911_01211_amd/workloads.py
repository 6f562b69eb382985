"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module builds INPUTS only: Hamiltonians, interaction ramps, drive
samples, random contour-function histories, and the closed-form free
propagators of static Hamiltonians. Those propagators are the exact
solution of a quadratic problem, used as a given self-energy or as an exact
reference; none of the Dyson time stepper's own arithmetic is here.

Every generator draws from numpy's PCG64 seeded with
``SeedSequence([191101211, *key])``.

Canonical contour storage (Eq. storage_herm of the paper): ``mat``
[ntau+1, d, d]; ``ret``/``les`` [(nt+1)(nt+2)/2, d, d], where slice n starts
at n(n+1)/2, R_{n,j} = ret[n(n+1)/2 + j] and L_{j,n} = les[n(n+1)/2 + j];
``tv`` [(nt+1)(ntau+1), d, d].
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED = 191101211


def rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED, *key])))


@dataclasses.dataclass
class GridSpec:
    nt: int
    ntau: int
    d: int
    sig: int = -1
    k: int = 5
    beta: float = 1.0
    h: float = 0.01
    mu: float = 0.0

    @property
    def htau(self) -> float:
        return self.beta / self.ntau

    @property
    def ntri(self) -> int:
        return (self.nt + 1) * (self.nt + 2) // 2


def empty_contour(g: GridSpec) -> dict:
    d = g.d
    return dict(mat=np.zeros((g.ntau + 1, d, d), np.complex128),
                ret=np.zeros((g.ntri, d, d), np.complex128),
                les=np.zeros((g.ntri, d, d), np.complex128),
                tv=np.zeros(((g.nt + 1) * (g.ntau + 1), d, d), np.complex128))


def random_hermitian(r: np.random.Generator, d: int, scale: float = 1.0) -> np.ndarray:
    a = r.normal(size=(d, d)) + 1j * r.normal(size=(d, d))
    return scale * (a + a.conj().T) / 2


def haar_hermitian(r: np.random.Generator, d: int, lo: float = -2.0, hi: float = 2.0):
    """Random hermitian matrix with a uniform spectrum in [lo, hi] and a Haar
    distributed eigenbasis."""
    lam = r.uniform(lo, hi, d)
    z = (r.normal(size=(d, d)) + 1j * r.normal(size=(d, d))) / np.sqrt(2)
    q, rq = np.linalg.qr(z)
    q = q * (np.diag(rq) / np.abs(np.diag(rq)))
    return (q * lam) @ q.conj().T


def random_contour(r: np.random.Generator, g: GridSpec, scale: float = 1.0,
                   decay: float = 0.0) -> dict:
    """Random contour function in the canonical layout: complex gaussian
    blocks, hermitian Matsubara blocks, optionally damped like a Green's
    function (|C(t,t')| ~ exp(-decay |t - t'|))."""
    c = empty_contour(g)
    d = g.d
    for m in range(g.ntau + 1):
        c["mat"][m] = random_hermitian(r, d, scale)
    shape = (g.ntri, d, d)
    c["ret"][...] = scale * (r.normal(size=shape) + 1j * r.normal(size=shape))
    c["les"][...] = scale * (r.normal(size=shape) + 1j * r.normal(size=shape))
    shape = c["tv"].shape
    c["tv"][...] = scale * (r.normal(size=shape) + 1j * r.normal(size=shape))
    if decay > 0:
        for n in range(g.nt + 1):
            o = n * (n + 1) // 2
            damp = np.exp(-decay * g.h * (n - np.arange(n + 1)))[:, None, None]
            c["ret"][o:o + n + 1] *= damp
            c["les"][o:o + n + 1] *= damp
    return c


def free_gf(H: np.ndarray, g: GridSpec, H0: np.ndarray | None = None) -> dict:
    """Closed-form free propagator for H(t<0) = H0 (default H) and H(t>=0) = H,
    constant: Matsubara from H0, real-time parts from exp(-i H t) and the
    initial density matrix f(H0 - mu) (Sec. "Implementation: Free Green's
    functions", Eq. G0_free)."""
    if H0 is None:
        H0 = H
    d = H.shape[0]
    xi = g.sig
    x0, V0 = np.linalg.eigh(H0 - g.mu * np.eye(d))
    x1, V1 = np.linalg.eigh(H - g.mu * np.eye(d))
    with np.errstate(over="ignore"):
        f0 = 1.0 / (np.exp(g.beta * x0) - xi)
    c = empty_contour(g)

    def mk(V, diag):
        return (V * diag) @ V.conj().T

    def U(t):
        return mk(V1, np.exp(-1j * x1 * t))

    for m in range(g.ntau + 1):
        tau = m * g.htau
        with np.errstate(over="ignore"):
            val = np.where(x0 >= 0, -np.exp(-x0 * tau) / (1 - xi * np.exp(-g.beta * x0)),
                           -np.exp(x0 * (g.beta - tau)) / (np.exp(g.beta * x0) - xi))
        c["mat"][m] = mk(V0, val)
    rho = mk(V0, f0)
    Ut = [U(n * g.h) for n in range(g.nt + 1)]
    for n in range(g.nt + 1):
        o = n * (n + 1) // 2
        for j in range(n + 1):
            c["ret"][o + j] = -1j * U((n - j) * g.h)
            c["les"][o + j] = -1j * xi * Ut[j] @ rho @ Ut[n].conj().T
        for m in range(g.ntau + 1):
            tau = m * g.htau
            with np.errstate(over="ignore"):
                val = np.where(x0 >= 0,
                               np.exp(x0 * (tau - g.beta)) / (1 - xi * np.exp(-g.beta * x0)),
                               f0 * np.exp(x0 * tau))
            c["tv"][n * (g.ntau + 1) + m] = -1j * xi * Ut[n] @ mk(V0, val)
    return c


# --------------------------------------------------------------- workloads
def chain_hopping(nsites: int, J: float = 1.0, periodic: bool = False) -> np.ndarray:
    H = np.zeros((nsites, nsites), np.complex128)
    for i in range(nsites - 1):
        H[i, i + 1] = H[i + 1, i] = -J
    if periodic and nsites > 2:
        H[0, nsites - 1] = H[nsites - 1, 0] = -J
    return H


def two_level_embedding(g: GridSpec):
    """Plain Dyson solve of the 2x2 level H=[[-1,0.5],[0.5,1]] with a fixed
    diagonal self-energy 0.16 g_b of one free bath level eps_b = 0.3 per
    orbital. Returns (eps [nt+2,2,2], Sigma contour, exact 4x4 embedding G)."""
    H = np.array([[-1.0, 0.5], [0.5, 1.0]], np.complex128)
    V, eb = 0.4, 0.3
    g1 = dataclasses.replace(g, d=1)
    gb = free_gf(np.array([[eb]], np.complex128), g1)
    S = empty_contour(g)
    for key in S:
        S[key][:, 0, 0] = V * V * gb[key][:, 0, 0]
        S[key][:, 1, 1] = V * V * gb[key][:, 0, 0]
    Hf = np.zeros((4, 4), np.complex128)
    Hf[:2, :2] = H
    Hf[:2, 2:] = V * np.eye(2)
    Hf[2:, :2] = V * np.eye(2)
    Hf[2:, 2:] = eb * np.eye(2)
    Ge = free_gf(Hf, dataclasses.replace(g, d=4))
    Ge = {key: np.ascontiguousarray(v[:, :2, :2]) for key, v in Ge.items()}
    eps = np.broadcast_to(H, (g.nt + 2, 2, 2)).astype(np.complex128).copy()
    return eps, S, Ge


def hubbard_ramp(g: GridSpec, nsites: int = 4, J: float = 1.0, U0: float = 2.0,
                 U1: float = 1.0, t_ramp: float = 5.0):
    """Open Hubbard chain, second-Born workload: eps0 [nt+2,d,d] (index n+1),
    U [nt+2] with U_{-1} = U0 and a linear ramp U0 -> U1 on [0, t_ramp]."""
    H = chain_hopping(nsites, J)
    eps0 = np.broadcast_to(H, (g.nt + 2, nsites, nsites)).astype(np.complex128).copy()
    t = np.arange(-1, g.nt + 1) * g.h
    U = np.where(t < t_ramp, U0 + (U1 - U0) * t / t_ramp, U1)
    U[0] = U0
    return eps0, U.astype(np.float64)


def dimer_quench(g: GridSpec, U: float = 1.0, w0: float = 5.0):
    """Hubbard dimer with an on-site quench w0 of site 1 at t = 0."""
    H = chain_hopping(2, 1.0)
    eps0 = np.broadcast_to(H, (g.nt + 2, 2, 2)).astype(np.complex128).copy()
    eps0[1:, 0, 0] += w0
    return eps0, np.full(g.nt + 2, U)


def peierls_pulse(t: np.ndarray, E0: float = 1.0, omega: float = 2.0, t0: float = 5.0,
                  s: float = 1.5) -> np.ndarray:
    return E0 * np.sin(omega * t) * np.exp(-((t - t0) ** 2) / (2 * s * s))


def holstein_drive(g: GridSpec, g0: float = 0.5, dg: float = 0.05, J0: float = 1.0, dJ: float = 0.1,
                   omega: float = 1.2, t_end: float = 15.7):
    """Hopping J(t) and electron-phonon coupling g(t) of the Holstein example,
    both modulated as x0 + dx sin^2(pi t / t_end) sin(omega t) for t < t_end:
    returns (J, g), each nt + 2 real values (entry 0: the Matsubara branch)."""
    t = np.arange(g.nt + 1) * g.h
    env = np.where(t < t_end, np.sin(np.pi * t / t_end) ** 2, 0.0) * np.sin(omega * t)
    J = np.concatenate([[J0], J0 + dJ * env])
    gel = np.concatenate([[g0], g0 + dg * env])
    return J, gel


def kpoint_band(g: GridSpec, nk: int = 512):
    """Single-band lattice eps_k(t) = -2 cos(k - A(t)) for nk uniform k:
    returns eps [nk, nt+2, 1, 1] with eps_k(0^-) = -2 cos k."""
    k = 2 * np.pi * np.arange(nk) / nk
    t = np.arange(g.nt + 1) * g.h
    A = peierls_pulse(t)
    eps = np.zeros((nk, g.nt + 2, 1, 1), np.complex128)
    eps[:, 0, 0, 0] = -2 * np.cos(k)
    eps[:, 1:, 0, 0] = -2 * np.cos(k[:, None] - A[None, :])
    return eps


def ring_peierls(g: GridSpec, nsites: int = 8, J: float = 1.0):
    """Periodic ring with a Peierls phase on the hopping: eps_{i+1,i}(t) =
    -J e^{i A(t)} and its conjugate (Sec. "Example: GW for the translationally
    invariant Hubbard model"). Returns the bare hopping T [nt+2, d, d]
    (index n+1) and the phase pattern Phi [d, d] (+1 on i+1 <- i, -1 on
    i <- i+1), so that eps_n = T * exp(i A_n Phi) elementwise."""
    T = np.zeros((nsites, nsites), np.complex128)
    Phi = np.zeros((nsites, nsites))
    for i in range(nsites):
        j = (i + 1) % nsites
        T[j, i] = T[i, j] = -J
        Phi[j, i], Phi[i, j] = 1.0, -1.0
    return np.broadcast_to(T, (g.nt + 2, nsites, nsites)).copy(), Phi


def ring_drive(g: GridSpec, key: int = 5):
    """Seeded vector potential of the eight-site ring workload: four modes,
    c_q ~ N(0, 0.25^2), w_q ~ U[0.5, 3], phi_q ~ U[0, 2 pi), and
    A_n = sum_q c_q sin(w_q t_n + phi_q) (1 - exp(-t_n^2)) for n = 1..nt
    (smooth, A(0) = 0). Returns the nt samples A_1..A_nt."""
    r = rng(key)
    c = r.normal(0.0, 0.25, 4)
    w = r.uniform(0.5, 3.0, 4)
    ph = r.uniform(0.0, 2 * np.pi, 4)
    t = np.arange(1, g.nt + 1) * g.h
    return (c[None, :] * np.sin(w[None, :] * t[:, None] + ph[None, :])).sum(1) * (1 - np.exp(-t * t))


def peierls_levels(T: np.ndarray, Phi: np.ndarray, A_samples: np.ndarray) -> np.ndarray:
    """Input levels of the ring for the oracle: eps_n = T_n exp(i A_n Phi),
    with A = 0 at entries -1 and 0 and A_1..A_nt after them."""
    A = np.concatenate([[0.0, 0.0], A_samples])
    return T * np.exp(1j * A[:, None, None] * Phi[None, :, :])


def uneven_problem(p: int):
    """Problem p of the uneven batch: from PCG64(SeedSequence([191101211, p]))
    draw d from {1, 2, 4, 8}, nt uniform in [400, 3000], U uniform in
    [0.5, 2], then a hermitian H with spectrum uniform in [-2, 2] and a Haar
    distributed eigenbasis. Returns (d, nt, U, H)."""
    r = rng(p)
    d = int(r.choice([1, 2, 4, 8]))
    nt = int(r.integers(400, 3001))
    U = float(r.uniform(0.5, 2.0))
    H = haar_hermitian(r, d, -2.0, 2.0)
    return d, nt, U, H


def load_uneven(path: str):
    """The uneven batch as stored by data/make_uneven_batch.py: a list of
    (d, nt, U, H) per problem."""
    z = np.load(path)
    return [(int(d), int(nt), float(U), np.array(z["H"][i, :d, :d]))
            for i, (d, nt, U) in enumerate(zip(z["d"], z["nt"], z["U"]))]

"""ctypes binding of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the GPU library never does.

Contour functions use the canonical storage of the paper (Eq. storage_herm):
``mat`` [ntau+1, d, d], ``ret``/``les`` [(nt+1)(nt+2)/2, d, d] with slice n at
offset n(n+1)/2, ``tv`` [(nt+1)(ntau+1), d, d], all complex128.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["weights.cpp", "linalg.cpp", "convolution.cpp", "dyson.cpp", "vie2.cpp", "sigma.cpp", "capi.cpp"]


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with g++ (OpenMP over the independent loops)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", LIB + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Grid(C.Structure):
    _fields_ = [("nt", C.c_int32), ("ntau", C.c_int32), ("d", C.c_int32), ("sig", C.c_int32),
                ("k", C.c_int32), ("beta", C.c_double), ("h", C.c_double), ("mu", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _lib.oracle_gregory.restype = C.c_double
        _lib.oracle_distance.restype = C.c_double
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Grid:
    def __init__(self, nt, ntau, d, sig=-1, k=5, beta=1.0, h=0.01, mu=0.0):
        self.nt, self.ntau, self.d, self.sig, self.k = int(nt), int(ntau), int(d), int(sig), int(k)
        self.beta, self.h, self.mu = float(beta), float(h), float(mu)

    @property
    def htau(self):
        return self.beta / self.ntau

    def c(self):
        return _Grid(self.nt, self.ntau, self.d, self.sig, self.k, self.beta, self.h, self.mu)


class HM:
    """A hermitian contour function in the canonical layout (numpy owned)."""

    def __init__(self, g: Grid):
        self.g = g
        d, nt, ntau = g.d, g.nt, g.ntau
        self.mat = np.zeros((ntau + 1, d, d), np.complex128)
        self.ret = np.zeros(((nt + 1) * (nt + 2) // 2, d, d), np.complex128)
        self.les = np.zeros(((nt + 1) * (nt + 2) // 2, d, d), np.complex128)
        self.tv = np.zeros(((nt + 1) * (ntau + 1), d, d), np.complex128)

    def args(self):
        return [_p(self.mat), _p(self.ret), _p(self.les), _p(self.tv)]

    def copy(self):
        o = HM(self.g)
        for f in ("mat", "ret", "les", "tv"):
            getattr(o, f)[...] = getattr(self, f)
        return o

    # element access (views)
    def R(self, n, j):
        return self.ret[n * (n + 1) // 2 + j]

    def L(self, j, n):
        return self.les[n * (n + 1) // 2 + j]

    def T(self, n, m):
        return self.tv[n * (self.g.ntau + 1) + m]

    def M(self, m):
        return self.mat[m]

    def ret_row(self, n):
        return self.ret[n * (n + 1) // 2: n * (n + 1) // 2 + n + 1]

    def les_col(self, n):
        return self.les[n * (n + 1) // 2: n * (n + 1) // 2 + n + 1]

    def tv_row(self, n):
        return self.tv[n * (self.g.ntau + 1): (n + 1) * (self.g.ntau + 1)]


def weights(k):
    n = k + 1
    P, D = np.zeros(n * n), np.zeros(n * n)
    Iw = np.zeros(n ** 3)
    bdf, start, omega = np.zeros(n), np.zeros(n * n), np.zeros(n)
    R = np.zeros(n ** 3)
    if lib().oracle_weights(k, *(_p(x) for x in (P, D, Iw, bdf, start, omega, R))) != 0:
        raise ValueError(k)
    return dict(P=P.reshape(n, n), D=D.reshape(n, n), I=Iw.reshape(n, n, n), a=bdf,
                s=start.reshape(n, n), omega=omega, R=R.reshape(n, n, n))


def gregory(k, n, j):
    return lib().oracle_gregory(k, n, j)


def gregory_rational(k, n, j):
    num, den = C.c_int64(), C.c_int64()
    lib().oracle_gregory_rational(k, n, j, C.byref(num), C.byref(den))
    return num.value, den.value


def solve(A, B):
    A = np.ascontiguousarray(A, np.complex128).copy()
    B = np.ascontiguousarray(B, np.complex128).copy()
    n = A.shape[0]
    nrhs = 1 if B.ndim == 1 else B.shape[1]
    if lib().oracle_solve(n, nrhs, _p(A), _p(B)) != 0:
        raise np.linalg.LinAlgError("singular")
    return B


def eigh(A):
    A = np.ascontiguousarray(A, np.complex128)
    d = A.shape[0]
    w = np.zeros(d)
    V = np.zeros((d, d), np.complex128)
    lib().oracle_eigh(d, _p(A), _p(w), _p(V))
    return w, V


def free_mat(g: Grid, eps):
    out = np.zeros((g.ntau + 1, g.d, g.d), np.complex128)
    lib().oracle_free_mat(C.byref(g.c()), _p(np.ascontiguousarray(eps, np.complex128)), _p(out))
    return out


def convolution_timestep(n, C_: HM, A: HM, Acc: HM, B: HM, Bcc: HM, f=None):
    g = A.g
    lib().oracle_convolution_timestep(n, C.byref(g.c()), *C_.args(), *A.args(), *Acc.args(),
                                      *B.args(), *Bcc.args(), _p(f))


def conv_les_diag(n, A: HM, B: HM):
    out = np.zeros((A.g.d, A.g.d), np.complex128)
    lib().oracle_conv_les_diag(n, C.byref(A.g.c()), *A.args(), *B.args(), _p(out))
    return out


def dyson_mat(G: HM, S: HM, eps_m1):
    e = np.ascontiguousarray(eps_m1, np.complex128)
    return lib().oracle_dyson_mat(C.byref(G.g.c()), *G.args(), *S.args(), _p(e))


def dyson_start(G: HM, S: HM, eps):
    e = np.ascontiguousarray(eps, np.complex128)
    return lib().oracle_dyson_start(C.byref(G.g.c()), *G.args(), *S.args(), _p(e))


def dyson_timestep(n, G: HM, S: HM, eps, variant="B"):
    e = np.ascontiguousarray(eps, np.complex128)
    return lib().oracle_dyson_timestep(n, C.byref(G.g.c()), *G.args(), *S.args(), _p(e),
                                       ord(variant))


def vie2_mat(G: HM, F: HM, Q: HM):
    """Matsubara part of (1 + F) * G = Q (Eq. vie2_langreth_m)."""
    return lib().oracle_vie2_mat(C.byref(G.g.c()), *G.args(), *F.args(), *Q.args())


def vie2_start(G: HM, F: HM, Fcc: HM, Q: HM):
    """Slices 0..k of (1 + F) * G = Q (Sec. "Implementation: vie2", Start)."""
    return lib().oracle_vie2_start(C.byref(G.g.c()), *G.args(), *F.args(), *Fcc.args(), *Q.args())


def vie2_timestep(n, G: HM, F: HM, Fcc: HM, Q: HM):
    """Slice n > k of (1 + F) * G = Q (Sec. "Implementation: vie2", Time stepping)."""
    return lib().oracle_vie2_timestep(n, C.byref(G.g.c()), *G.args(), *F.args(), *Fcc.args(), *Q.args())


def solve_vie2(G: HM, F: HM, Fcc: HM, Q: HM, nt_stop=None):
    """Matsubara, start-up and every time step up to nt_stop; 0 or the first error."""
    nt_stop = G.g.nt if nt_stop is None else nt_stop
    rc = vie2_mat(G, F, Q) or vie2_start(G, F, Fcc, Q)
    for n in range(G.g.k + 1, nt_stop + 1):
        rc = rc or vie2_timestep(n, G, F, Fcc, Q)
    return rc


def sigma_2b(n, G: HM, U, S: HM):
    u = np.ascontiguousarray(U, np.float64)
    lib().oracle_sigma_2b(n, C.byref(G.g.c()), *G.args(), _p(u), *S.args())


def observables(n, G: HM, S: HM, eps0, eps_mf=None):
    """Per-spin observables of slice n (density matrix, Eq. Total_ener):
    [Re Tr rho, Re Tr rho eps0_n, Re Tr rho eps_mf_n, 1/2 Im Tr [S*G]^<(n,n),
    total energy], and rho."""
    em = eps0 if eps_mf is None else eps_mf
    rho = density_matrix(n, G)
    ec = conv_les_diag(n, S, G)
    e1 = np.trace(rho @ eps0[n + 1]).real
    emf = np.trace(rho @ em[n + 1]).real
    ecorr = 0.5 * np.trace(ec).imag
    return np.array([np.trace(rho).real, e1, emf, ecorr, 0.5 * (e1 + emf) + ecorr]), rho


def hartree(n, G: HM, U, eps0, eps_mf, nbar=0.5):
    lib().oracle_hartree(n, C.byref(G.g.c()), *G.args(), _p(np.ascontiguousarray(U, np.float64)),
                         _p(eps0), _p(eps_mf), C.c_double(nbar))


def density_matrix(n, G: HM):
    out = np.zeros((G.g.d, G.g.d), np.complex128)
    lib().oracle_density_matrix(n, C.byref(G.g.c()), *G.args(), _p(out))
    return out


def extrapolate(n, G: HM):
    lib().oracle_extrapolate(n, C.byref(G.g.c()), *G.args())


def distance(n, A: HM, B: HM):
    return lib().oracle_distance(n, C.byref(A.g.c()), *A.args(), *B.args())


def solve_fixed(G: HM, S: HM, eps, nt_stop=None, variant="B"):
    e = np.ascontiguousarray(eps, np.complex128)
    secs = np.zeros(3)
    nt_stop = G.g.nt if nt_stop is None else nt_stop
    rc = lib().oracle_solve_fixed(C.byref(G.g.c()), *G.args(), *S.args(), _p(e), nt_stop,
                                  ord(variant), _p(secs))
    return rc, secs


def solve_2b(G: HM, S: HM, eps0, U, nbar=0.5, mats_maxit=200, mats_tol=1e-14, mats_mix=0.5,
             boot_maxit=100, boot_tol=1e-14, ncorr=6, corr_tol=0.0, nt_stop=None, variant="B"):
    """Self-consistent 2B + Hartree run; returns (rc, eps_mf, stats)."""
    g = G.g
    e0 = np.ascontiguousarray(eps0, np.complex128)
    emf = np.zeros_like(e0)
    Gold = HM(g)
    stats = np.zeros(6)
    nt_stop = g.nt if nt_stop is None else nt_stop
    rc = lib().oracle_solve_2b(C.byref(g.c()), *G.args(), *S.args(), *Gold.args(), _p(e0),
                               _p(np.ascontiguousarray(U, np.float64)), _p(emf), C.c_double(nbar),
                               mats_maxit, C.c_double(mats_tol), C.c_double(mats_mix), boot_maxit,
                               C.c_double(boot_tol),
                               ncorr, C.c_double(corr_tol), nt_stop, ord(variant), _p(stats))
    return rc, emf, dict(mats_iter=int(stats[0]), boot_iter=int(stats[1]),
                         corr_total=int(stats[2]), mats_err=stats[3], boot_err=stats[4],
                         corr_err_max=stats[5])


def sigma_local(n, Gs, S: HM, lam):
    """Sigma = lam * (1/count) sum_i G_i on slice n (n = -1: Matsubara), every
    component; sequential sum over i."""
    w = lam / len(Gs)

    def acc(get):
        s = np.zeros_like(get(Gs[0]))
        for G in Gs:
            s = s + get(G)
        return w * s

    if n == -1:
        S.mat[...] = acc(lambda G: G.mat)
        return
    o, nt1 = n * (n + 1) // 2, S.g.ntau + 1
    S.ret[o:o + n + 1] = acc(lambda G: G.ret[o:o + n + 1])
    S.les[o:o + n + 1] = acc(lambda G: G.les[o:o + n + 1])
    S.tv[n * nt1:(n + 1) * nt1] = acc(lambda G: G.tv[n * nt1:(n + 1) * nt1])


def solve_local(Gs, S: HM, eps, lam, mats_iters=30, boot_iters=8, ncorr=5, nt_stop=None):
    """Batched lattice problems coupled by a local self-energy Sigma = lam *
    G_loc, G_loc = (1/count) sum_i G_i (per-k Dyson equations of the parallel
    k-point scheme). Fixed iteration counts:
      Matsubara: mats_iters x {Sigma^M from G^M; G_i^M = Dyson(Sigma^M)},
      bootstrap: boot_iters x {Sigma on slices 0..k; start-up of every G_i},
      steps    : extrapolation, then ncorr x {Sigma on slice n; time step},
                 and a last Sigma of slice n.
    Returns the L1 changes of Sigma^M and of the bootstrap slices in the last
    iteration (convergence diagnostics)."""
    g = Gs[0].g
    k = g.k
    nt_stop = g.nt if nt_stop is None else nt_stop
    dm = 0.0
    for it in range(mats_iters):
        prev = S.mat.copy()
        sigma_local(-1, Gs, S, lam)
        dm = float(np.abs(S.mat - prev).sum())
        for G, e in zip(Gs, eps):
            dyson_mat(G, S, e[0])
    sigma_local(-1, Gs, S, lam)
    db = 0.0
    for it in range(boot_iters):
        prev = S.copy()
        for n in range(k + 1):
            sigma_local(n, Gs, S, lam)
        db = float(np.abs(S.ret - prev.ret).sum() + np.abs(S.les - prev.les).sum() + np.abs(S.tv - prev.tv).sum())
        for G, e in zip(Gs, eps):
            dyson_start(G, S, e)
    for n in range(k + 1):
        sigma_local(n, Gs, S, lam)
    for n in range(k + 1, nt_stop + 1):
        for G in Gs:
            extrapolate(n - 1, G)
        for _ in range(ncorr):
            sigma_local(n, Gs, S, lam)
            for G, e in zip(Gs, eps):
                dyson_timestep(n, G, S, e, "B")
        sigma_local(n, Gs, S, lam)
    return dict(mats_change=dm, boot_change=db)


def num_threads():
    return lib().oracle_num_threads()


def set_threads(n: int):
    lib().oracle_set_threads(int(n))

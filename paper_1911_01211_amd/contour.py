"""Device-resident contour functions (torch complex128 tensors in the
canonical layout) and thin wrappers with the names of the C ABI.

torch provides device memory and the stream; the computation is done by the
HIP kernels of libcntr.so through ``_abi``.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import torch

from . import _abi
from .workloads import GridSpec

KEYS = ("mat", "ret", "les", "tv")


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def grid_c(g: GridSpec) -> _abi.Grid:
    return _abi.Grid(g.nt, g.ntau, g.d, g.sig, g.k, g.beta, g.h, g.mu)


class Contour:
    """Hermitian contour function on one grid, stored on a torch device."""

    def __init__(self, g: GridSpec, device="cuda", data: dict | None = None):
        self.g = g
        d = g.d
        shapes = dict(mat=(g.ntau + 1, d, d), ret=(g.ntri, d, d), les=(g.ntri, d, d),
                      tv=((g.nt + 1) * (g.ntau + 1), d, d))
        for key in KEYS:
            if data is not None:
                t = torch.as_tensor(np.ascontiguousarray(data[key]), dtype=torch.complex128)
                t = t.to(device).contiguous()
            else:
                t = torch.zeros(shapes[key], dtype=torch.complex128, device=device)
            assert tuple(t.shape) == shapes[key], (key, t.shape, shapes[key])
            setattr(self, key, t)

    def gf(self) -> _abi.GF:
        return _abi.GF(*(getattr(self, k).data_ptr() for k in KEYS))

    def numpy(self) -> dict:
        return {k: getattr(self, k).cpu().numpy() for k in KEYS}

    def zero_(self):
        for k in KEYS:
            getattr(self, k).zero_()
        return self


def _gfs(items):
    return _abi.arr(_abi.GF, [x.gf() for x in items])


def _ptrs(items):
    return _abi.arr(C.c_void_p, [None if x is None else x.data_ptr() for x in items])


def _grids(items):
    return _abi.arr(_abi.Grid, [grid_c(x.g) for x in items])


def init_matsubara(G: list, Sigma: list, eps: list, tol=1e-14, max_iter=200, stream=None):
    L = _abi.lib()
    _abi.check(L.cntr_init_matsubara(len(G), _grids(G), _gfs(G), _gfs(Sigma), _ptrs(eps), tol,
                                     max_iter, _stream(stream)))


def dyson_step(tstp: int, G: list, Sigma: list, eps: list, stream=None):
    L = _abi.lib()
    _abi.check(L.cntr_dyson_step(tstp, len(G), _grids(G), _gfs(G), _gfs(Sigma), _ptrs(eps),
                                 _stream(stream)))


def dyson_step_noalloc(tstp: int, G: list, Sigma: list, eps: list, stream=None):
    """cntr_dyson_step_noalloc: the same step with the library's static device
    scratch (no allocation; usable under graph capture)."""
    L = _abi.lib()
    _abi.check(L.cntr_dyson_step_noalloc(tstp, len(G), _grids(G), _gfs(G), _gfs(Sigma), _ptrs(eps),
                                         _stream(stream)))


def vie2_matsubara(G: list, F: list, Q: list, tol=1e-14, max_iter=200, stream=None):
    """G^M of (1 + F) * G = Q for each instance (cntr_vie2_matsubara)."""
    _abi.check(_abi.lib().cntr_vie2_matsubara(len(G), _grids(G), _gfs(G), _gfs(F), _gfs(Q), tol, max_iter,
                                               _stream(stream)))


def vie2_step(tstp: int, G: list, F: list, Fcc: list, Q: list, stream=None):
    """Start-up (tstp <= k: slices 0..k) or time step tstp of (1 + F) * G = Q
    (cntr_vie2_step); Fcc[i] is the hermitian conjugate of F[i]."""
    _abi.check(_abi.lib().cntr_vie2_step(tstp, len(G), _grids(G), _gfs(G), _gfs(F), _gfs(Fcc), _gfs(Q),
                                          _stream(stream)))


class Vie2Batch:
    """The C-ABI argument arrays of a fixed batch of (1 + F) * G = Q problems,
    built once (as Batch does for the Dyson step)."""

    def __init__(self, G: list, F: list, Fcc: list, Q: list):
        self.count = len(G)
        self.grids = _grids(G)
        self.gfs, self.f, self.fcc, self.q = _gfs(G), _gfs(F), _gfs(Fcc), _gfs(Q)

    def matsubara(self, tol=1e-14, max_iter=200, stream=None):
        _abi.check(_abi.lib().cntr_vie2_matsubara(self.count, self.grids, self.gfs, self.f, self.q, tol, max_iter,
                                                   _stream(stream)))

    def step(self, tstp: int, stream=None):
        _abi.check(_abi.lib().cntr_vie2_step(tstp, self.count, self.grids, self.gfs, self.f, self.fcc, self.q,
                                              _stream(stream)))


def solve_vie2(G: list, F: list, Fcc: list, Q: list, nt_stop=None, stream=None):
    """Matsubara, start-up and every time step up to nt_stop."""
    g = G[0].g
    nt_stop = g.nt if nt_stop is None else nt_stop
    B = Vie2Batch(G, F, Fcc, Q)
    B.matsubara(stream=stream)
    B.step(g.k, stream)
    for n in range(g.k + 1, nt_stop + 1):
        B.step(n, stream)


class KBatch:
    """The C-ABI argument arrays of the momentum-convolution calls over fixed
    lists of momenta (G_k, Pi_k, dW_k, Sigma_k), built once: marshalling
    hundreds of contours per call costs more host time than the kernel."""

    def __init__(self, G: list, Pi: list, dW: list, Sigma: list):
        self.nk = len(G)
        self.grids = _grids(G)
        self.g, self.pi, self.w, self.s = _gfs(G), _gfs(Pi), _gfs(dW), _gfs(Sigma)

    def polarization(self, tstp: int, alpha: float = 1.0, stream=None):
        _abi.check(_abi.lib().cntr_polarization_k(tstp, self.nk, self.grids, self.g, self.pi, float(alpha),
                                                   _stream(stream)))

    def sigma(self, tstp: int, alpha: float = 1.0, stream=None):
        _abi.check(_abi.lib().cntr_sigma_gw_k(tstp, self.nk, self.grids, self.g, self.w, self.s, float(alpha),
                                               _stream(stream)))


def polarization_k(tstp: int, G: list, Pi: list, alpha: float = 1.0, stream=None):
    """alpha Pi_k, Pi_k = -(i/Nk) sum_q G_{k+q}(t,t') G_q(t',t), on slice tstp (cntr_polarization_k)."""
    _abi.check(_abi.lib().cntr_polarization_k(tstp, len(G), _grids(G), _gfs(G), _gfs(Pi), float(alpha),
                                               _stream(stream)))


def sigma_gw_k(tstp: int, G: list, dW: list, Sigma: list, alpha: float = 1.0, stream=None):
    """alpha Sigma_k, Sigma_k = (i/Nk) sum_q G_{k-q}(t,t') dW_q(t,t'), on slice tstp (cntr_sigma_gw_k)."""
    _abi.check(_abi.lib().cntr_sigma_gw_k(tstp, len(G), _grids(G), _gfs(G), _gfs(dW), _gfs(Sigma), float(alpha),
                                           _stream(stream)))


def convolution(tstp: int, C_: list, A: list, Acc: list, B: list, Bcc: list, f=None, stream=None):
    L = _abi.lib()
    fp = None if f is None else _ptrs(f)
    _abi.check(L.cntr_convolution(tstp, len(C_), _grids(C_), _gfs(C_), _gfs(A), _gfs(Acc), _gfs(B),
                                  _gfs(Bcc), fp, _stream(stream)))


def sigma_2b(tstp: int, G: list, U: list, Sigma: list, eps0=None, eps_mf=None, nbar=0.5,
             stream=None):
    L = _abi.lib()
    e0 = None if eps0 is None else _ptrs(eps0)
    em = None if eps_mf is None else _ptrs(eps_mf)
    _abi.check(L.cntr_sigma_2b(tstp, len(G), _grids(G), _gfs(G), _ptrs(U), _gfs(Sigma), e0, em,
                               nbar, _stream(stream)))


def sigma_local(tstp: int, G: list, Sigma, lam: float, stream=None):
    """Sigma = lam * mean_i G_i on slice tstp (cntr_sigma_local)."""
    _abi.check(_abi.lib().cntr_sigma_local(tstp, len(G), _grids(G), _gfs(G), _gfs([Sigma]), float(lam),
                                           _stream(stream)))


class Batch:
    """The C-ABI argument arrays of a fixed batch (grids, contour descriptors,
    self-energies, levels), built once: the per-call marshalling of large
    batches would otherwise cost more host time than the launches."""

    def __init__(self, G: list, Sigma: list, eps: list):
        self.count = len(G)
        self.G = G
        self.grids = _grids(G)
        self.gfs = _gfs(G)
        self.sgfs = _gfs(Sigma)
        self.eps = _ptrs(eps)

    def step(self, tstp: int, stream=None):
        _abi.check(_abi.lib().cntr_dyson_step(tstp, self.count, self.grids, self.gfs, self.sgfs, self.eps,
                                              _stream(stream)))

    def extrapolate(self, tstp: int, stream=None):
        _abi.check(_abi.lib().cntr_extrapolate(tstp, self.count, self.grids, self.gfs, _stream(stream)))

    def sigma_local(self, tstp: int, lam: float, stream=None):
        """Sigma_0 = lam * mean_i G_i (the batch's first self-energy)."""
        _abi.check(_abi.lib().cntr_sigma_local(tstp, self.count, self.grids, self.gfs, self.sgfs, float(lam),
                                               _stream(stream)))

    def init_matsubara(self, tol=1e-14, max_iter=200, stream=None):
        _abi.check(_abi.lib().cntr_init_matsubara(self.count, self.grids, self.gfs, self.sgfs, self.eps, tol,
                                                  max_iter, _stream(stream)))


def solve_local(G: list, Sigma, eps: list, lam: float, mats_iters=30, boot_iters=8, ncorr=5, nt_stop=None,
                mats_tol=1e-14, stream=None):
    """Batched problems coupled by a local self-energy Sigma = lam * G_loc,
    G_loc = (1/count) sum_i G_i (the per-k Dyson equations of a lattice with a
    local self-energy), every step for all instances in one launch:
      Matsubara: mats_iters x {Sigma^M from G^M; G_i^M = Dyson(Sigma^M)},
      bootstrap: boot_iters x {Sigma on slices 0..k; start-up of every G_i},
      steps    : extrapolation, then ncorr x {Sigma on slice n; time step},
                 and a last Sigma of slice n.
    Fixed iteration counts (the same sequence as the reference driver)."""
    g = G[0].g
    k = g.k
    nt_stop = g.nt if nt_stop is None else nt_stop
    B = Batch(G, [Sigma] * len(G), eps)
    for _ in range(mats_iters):
        B.sigma_local(-1, lam, stream)
        B.init_matsubara(tol=mats_tol, stream=stream)
    B.sigma_local(-1, lam, stream)
    for _ in range(boot_iters):
        for n in range(k + 1):
            B.sigma_local(n, lam, stream)
        B.step(k, stream)
    for n in range(k + 1):
        B.sigma_local(n, lam, stream)
    for n in range(k + 1, nt_stop + 1):
        B.extrapolate(n - 1, stream)
        for _ in range(ncorr):
            B.sigma_local(n, lam, stream)
            B.step(n, stream)
        B.sigma_local(n, lam, stream)
    return B


def solve_gw_k(G: list, eps: list, U: float, mats_iters=10, boot_iters=6, ncorr=3, nt_stop=None, stream=None):
    """Self-consistent k-space GW propagation (correlation part) of the
    momenta's functions G[k] (zero on entry; levels eps[k], device tensors
    [(nt+2), d, d]): the bosonic kernel F_k = -U Pi_k (cntr_polarization_k
    with alpha = -U), X_k from (1 + F_k) * X_k = F_k (one batched
    cntr_vie2_step per slice; dW_k = -U X_k is the screened interaction's
    dynamic part), Sigma_k = -U (i/Nk) sum_q G_{k-q} X_q (cntr_sigma_gw_k), and
    the batched Dyson step of every G_k; the iteration counts as in
    solve_local. Returns (F, X, Sigma) as lists of contours."""
    g = G[0].g
    k, nk = g.k, len(G)
    nt_stop = g.nt if nt_stop is None else nt_stop
    gb = dataclasses.replace(g, sig=1)
    dev = G[0].ret.device
    F = [Contour(gb, dev) for _ in range(nk)]
    X = [Contour(gb, dev) for _ in range(nk)]
    S = [Contour(g, dev) for _ in range(nk)]
    B = Batch(G, S, eps)
    V = Vie2Batch(X, F, F, F)
    KB = KBatch(G, F, X, S)
    B.init_matsubara(stream=stream)
    for _ in range(mats_iters):
        KB.polarization(-1, -U, stream)
        V.matsubara(stream=stream)
        KB.sigma(-1, -U, stream)
        B.init_matsubara(stream=stream)
    for _ in range(boot_iters):
        for n in range(k + 1):
            KB.polarization(n, -U, stream)
        V.step(k, stream)
        for n in range(k + 1):
            KB.sigma(n, -U, stream)
        B.step(k, stream)
    for n in range(k + 1, nt_stop + 1):
        B.extrapolate(n - 1, stream)
        for _ in range(ncorr):
            KB.polarization(n, -U, stream)
            V.step(n, stream)
            KB.sigma(n, -U, stream)
            B.step(n, stream)
    return F, X, S


def bubble2_local(tstp: int, A: list, B: list, C_: list, alpha: float = 1.0, stream=None):
    """C_i = alpha i A_i B_i elementwise on slice tstp for each instance (cntr_bubble2_local)."""
    _abi.check(_abi.lib().cntr_bubble2_local(tstp, len(A), _grids(A), _gfs(A), _gfs(B), _gfs(C_), float(alpha),
                                              _stream(stream)))


def phonon_free(D: list, w0: list, stream=None):
    """D0 of X = a + a^dag for each mode frequency w0[i] into the bosonic D[i] (cntr_phonon_free)."""
    w = (C.c_double * len(D))(*[float(x) for x in w0])
    _abi.check(_abi.lib().cntr_phonon_free(len(D), _grids(D), _gfs(D), w, _stream(stream)))


def scale_slice(tstp: int, C_: list, A: list, f: list, beta: float = 0.0, stream=None):
    """C = beta C + f(t) A(t,t') f(t') on slice tstp (cntr_scale_slice); f[i] a device float64 tensor of nt+2."""
    _abi.check(_abi.lib().cntr_scale_slice(tstp, len(C_), _grids(C_), _gfs(C_), _gfs(A), _ptrs(f), float(beta),
                                            _stream(stream)))


def holstein_mf(tstp: int, G: list, g: list, w0: list, e0: float, X: list, eps: list, stream=None):
    """Phonon displacement X(t_tstp) of Eq. X and the level e0 + g X (cntr_holstein_mf)."""
    w = (C.c_double * len(G))(*[float(x) for x in w0])
    _abi.check(_abi.lib().cntr_holstein_mf(tstp, len(G), _grids(G), _gfs(G), _ptrs(g), w, float(e0), _ptrs(X),
                                            _ptrs(eps), _stream(stream)))


def solve_holstein(G, J, gel, w0, e0: float = 0.0, mats_iters=30, boot_iters=8, ncorr=4, nt_stop=None,
                   stream=None):
    """Bethe-lattice DMFT with the unrenormalized Migdal impurity solver for
    the local G (a zero Contour on entry, d = 1): Delta = J G J, Sigma =
    i g g D0 G (the bubble of G and g D0 g), the level
    e0 + g X with X of Eq. X, Dyson's self-energy Delta + Sigma (Sigma by
    cntr_bubble2_local, one launch for every impurity). J, gel:
    device float64 tensors of nt+2 (entry 0: Matsubara branch). G, J, gel and
    w0 may also be lists of equal length: independent impurities (one grid
    shape) advanced together, one launch per call for all of them. The
    sequence:
      Matsubara: mats_iters x {X, Delta^M, Sigma^M; G^M},
      start-up:  boot_iters x {X, Delta, Sigma on slices 0..k; start-up of G},
      steps:     extrapolation of G, then ncorr x {X, Delta, Sigma on slice n; step n}.
    Returns (D0g, Delta, Sigma, X, eps) on the device (lists for list input)."""
    many = isinstance(G, (list, tuple))
    Gs = list(G) if many else [G]
    Js = list(J) if many else [J]
    gels = list(gel) if many else [gel]
    w0s = [float(x) for x in w0] if many else [float(w0)]
    nb = len(Gs)
    g = Gs[0].g
    k = g.k
    nt_stop = g.nt if nt_stop is None else nt_stop
    dev = Gs[0].ret.device
    gb = dataclasses.replace(g, sig=1, mu=0.0)
    D0 = [Contour(gb, dev) for _ in range(nb)]
    D0g = [Contour(gb, dev) for _ in range(nb)]
    phonon_free(D0, w0s, stream)
    for n in range(-1, g.nt + 1):
        scale_slice(n, D0g, D0, gels, 0.0, stream)
    Delta = [Contour(x.g, dev) for x in Gs]
    S = [Contour(x.g, dev) for x in Gs]
    St = [Contour(x.g, dev) for x in Gs]
    X = [torch.zeros(g.nt + 2, dtype=torch.float64, device=dev) for _ in range(nb)]
    eps = [torch.zeros((g.nt + 2, 1, 1), dtype=torch.complex128, device=dev) for _ in range(nb)]
    for e in eps:
        e[0] = e0
    ones = [torch.ones(g.nt + 2, dtype=torch.float64, device=dev)] * nb
    B = Batch(Gs, St, eps)

    def selfenergies(n):
        scale_slice(n, Delta, Gs, Js, 0.0, stream)
        bubble2_local(n, Gs, D0g, S, 1.0, stream)
        scale_slice(n, St, S, ones, 0.0, stream)
        scale_slice(n, St, Delta, ones, 1.0, stream)

    def mf(n):
        holstein_mf(n, Gs, gels, w0s, e0, X, eps, stream)

    B.init_matsubara(stream=stream)
    for _ in range(mats_iters):
        mf(-1)
        selfenergies(-1)
        B.init_matsubara(stream=stream)
    for _ in range(boot_iters):
        for n in range(k + 1):
            mf(n)
            selfenergies(n)
        B.step(k, stream)
    for n in range(k + 1, nt_stop + 1):
        B.extrapolate(n - 1, stream)
        for _ in range(ncorr):
            mf(n)
            selfenergies(n)
            B.step(n, stream)
    if many:
        return D0g, Delta, S, X, eps
    return D0g[0], Delta[0], S[0], X[0], eps[0]


OBS_NAMES = ("N", "E1", "Emf", "Ecorr", "Etot")


def observables(tstp: int, G: list, Sigma: list, eps0: list, eps_mf=None, stream=None):
    """Per-spin observables of slice tstp (cntr_observables): a (count, 5)
    float64 device tensor [N, Tr rho eps0, Tr rho eps_mf, E_corr, E_total] and
    the (count, d, d) density matrices."""
    import torch
    dev = G[0].mat.device
    d = G[0].g.d
    obs = torch.empty((len(G), 5), dtype=torch.float64, device=dev)
    rho = torch.empty((len(G), d, d), dtype=torch.complex128, device=dev)
    em = None if eps_mf is None else _ptrs(eps_mf)
    _abi.check(_abi.lib().cntr_observables(tstp, len(G), _grids(G), _gfs(G), _gfs(Sigma), _ptrs(eps0), em,
                                           C.c_void_p(obs.data_ptr()), C.c_void_p(rho.data_ptr()),
                                           _stream(stream)))
    return obs, rho


def adjoint_sweep(G: list, Sigma: list, eps: list, Gbar: list, eps_bar: list, Sigmabar: list | None = None,
                  U: list | None = None, U_bar: list | None = None, nbar=0.5, niter=10, tol=0.0, stream=None):
    """Reverse-mode sweep of the Dyson solution (cntr_adjoint_sweep). Gbar
    holds dJ/dG on entry (consumed; Gbar.mat returns dJ/dM), eps_bar (+=)
    receives dJ/deps_n, Sigmabar (+=) dJ/dSigma. With U (second-Born mode:
    G, Sigma, eps the converged solution with eps = eps_mf) eps_bar receives
    dJ/deps0_n and U_bar (+=) dJ/dU_n. Returns the largest relative change of
    a slice adjoint in its last fixed-point iteration (0 for a given Sigma);
    with tol > 0 a change above tol raises CNTR_ENOCONV.
    Gradients are dJ/dRe + i dJ/dIm of every complex entry."""
    sb = None if Sigmabar is None else _gfs(Sigmabar)
    conv = C.c_double(0.0)
    up = None if U is None else _ptrs(U)
    ub = None if U_bar is None else _ptrs(U_bar)
    _abi.check(_abi.lib().cntr_adjoint_sweep(len(G), _grids(G), _gfs(G), _gfs(Sigma), _ptrs(eps), up, float(nbar),
                                             _gfs(Gbar), sb, _ptrs(eps_bar), ub, int(niter), float(tol), C.byref(conv),
                                             _stream(stream)))
    return conv.value


def green_from_H(G: list, eps: list, stream=None):
    """Free Green's function of eps(t) into every component of each G
    (cntr_green_from_H; eps[i]: device tensor [(nt+2), d, d], entry 0 = eps(0^-))."""
    _abi.check(_abi.lib().cntr_green_from_H(len(G), _grids(G), _gfs(G), _ptrs(eps), _stream(stream)))


def matsubara_fourier(G: list, Sigma, eps: list, oversample: int = 10, stream=None):
    """G^M of each G by the Fourier-series method (cntr_matsubara_fourier;
    Sigma: list of contours, or None for Sigma = 0; eps[i]: device tensor
    [(nt+2), d, d], entry 0 = eps(0^-))."""
    S = _gfs(Sigma) if Sigma is not None else None
    _abi.check(_abi.lib().cntr_matsubara_fourier(len(G), _grids(G), _gfs(G), S, _ptrs(eps), int(oversample),
                                                  _stream(stream)))


def extrapolate(tstp: int, G: list, stream=None):
    _abi.check(_abi.lib().cntr_extrapolate(tstp, len(G), _grids(G), _gfs(G), _stream(stream)))


def distance(tstp: int, A: list, B: list, stream=None):
    out = (C.c_double * (2 * len(A)))()
    _abi.check(_abi.lib().cntr_distance(tstp, len(A), _grids(A), _gfs(A), _gfs(B), out,
                                        _stream(stream)))
    return np.array(out[:]).reshape(len(A), 2)


def copy_slice(tstp: int, dst: list, src: list, stream=None):
    _abi.check(_abi.lib().cntr_copy_slice(tstp, len(dst), _grids(dst), _gfs(dst), _gfs(src),
                                          _stream(stream)))


class Graph:
    """A captured launch sequence (cntr_graph_begin / cntr_graph_end): the
    library calls made on `stream` inside the `with` block are recorded, then
    replayed by launch(). stream must be a non-default torch stream."""

    def __init__(self, stream):
        self.stream = stream
        self.h = C.c_void_p()

    def __enter__(self):
        _abi.check(_abi.lib().cntr_graph_begin(C.c_void_p(self.stream.cuda_stream)))
        return self

    def __exit__(self, exc_type, exc, tb):
        rc = _abi.lib().cntr_graph_end(C.c_void_p(self.stream.cuda_stream), C.byref(self.h))
        if exc_type is None:
            _abi.check(rc)
        return False

    def launch(self, stream=None):
        _abi.check(_abi.lib().cntr_graph_launch(self.h, _stream(stream)))

    def __del__(self):
        try:
            if self.h:
                _abi.lib().cntr_graph_destroy(self.h)
        except Exception:
            pass


def set_checks(order=False, finite=False, symmetry=False):
    """Optional precondition / value checks (cntr_set_checks)."""
    _abi.check(_abi.lib().cntr_set_checks((_abi.CHECK_ORDER if order else 0) | (_abi.CHECK_FINITE if finite else 0) |
                                          (_abi.CHECK_SYMMETRY if symmetry else 0)))


def mark_slices(G: list, last: int):
    """Declare slices -1..last of each G complete for the order checks (-2 forgets them)."""
    _abi.check(_abi.lib().cntr_mark_slices(len(G), _gfs(G), int(last)))


def sync(stream=None):
    _abi.check(_abi.lib().cntr_sync(_stream(stream)))


def profile_begin(every: int = 1):
    """Record HIP events around every `every`-th time step (cntr_profile_begin_every)."""
    _abi.check(_abi.lib().cntr_profile_begin_every(int(every)))


def profile_end() -> dict:
    p = _abi.Profile()
    _abi.check(_abi.lib().cntr_profile_end(C.byref(p)))
    return {f: getattr(p, f) for f, _ in _abi.Profile._fields_}


@dataclasses.dataclass
class Solve2BStats:
    mats_iter: int
    boot_iter: int
    mats_err: float
    boot_err: float


def solve_2b(G: Contour, Sigma: Contour, Gscratch: Contour, eps0: torch.Tensor, U: torch.Tensor,
             eps_mf: torch.Tensor, nbar=0.5, mats_maxit=200, mats_tol=1e-14, mats_mix=0.5,
             boot_maxit=100, boot_tol=1e-14, ncorr=6, nt_stop=None, stream=None) -> Solve2BStats:
    g = G.g
    nt_stop = g.nt if nt_stop is None else nt_stop
    st = (C.c_double * 4)()
    gc = grid_c(g)
    _abi.check(_abi.lib().cntr_solve_2b(C.byref(gc), C.byref(G.gf()), C.byref(Sigma.gf()),
                                        C.byref(Gscratch.gf()), eps0.data_ptr(), U.data_ptr(),
                                        eps_mf.data_ptr(), nbar, mats_maxit, mats_tol, mats_mix,
                                        boot_maxit,
                                        boot_tol, ncorr, nt_stop, st, _stream(stream)))
    return Solve2BStats(int(st[0]), int(st[1]), st[2], st[3])


def solve_2b_batch(G: list, Sigma: list, Gscratch: list, eps0: list, U: list, eps_mf: list, nbar=0.5,
                   mats_maxit=200, mats_tol=1e-14, mats_mix=0.5, boot_maxit=100, boot_tol=1e-14, ncorr=6,
                   stream=None) -> Solve2BStats:
    """Self-consistent 2B + Hartree for problems sharing d, k and ntau
    (cntr_solve_2b_batch): one launch per kernel and step for the batch."""
    st = (C.c_double * 4)()
    _abi.check(_abi.lib().cntr_solve_2b_batch(len(G), _grids(G), _gfs(G), _gfs(Sigma), _gfs(Gscratch), _ptrs(eps0),
                                              _ptrs(U), _ptrs(eps_mf), nbar, mats_maxit, mats_tol, mats_mix,
                                              boot_maxit, boot_tol, ncorr, st, _stream(stream)))
    return Solve2BStats(int(st[0]), int(st[1]), st[2], st[3])


def solve_uneven(problems: list, nbar=0.5, mats_maxit=200, mats_tol=1e-14, mats_mix=0.5, boot_maxit=100,
                 boot_tol=1e-14, ncorr=6, stream=None) -> Solve2BStats:
    """An uneven set of second-Born problems (dicts with G, Sigma, Gscratch,
    eps0, U, eps_mf; any d and nt) in one call (cntr_solve_2b_uneven): the
    groups of equal orbital count advance side by side on streams of their
    own."""
    st = (C.c_double * 4)()
    G = [p["G"] for p in problems]
    _abi.check(_abi.lib().cntr_solve_2b_uneven(len(G), _grids(G), _gfs(G), _gfs([p["Sigma"] for p in problems]),
                                               _gfs([p["Gscratch"] for p in problems]),
                                               _ptrs([p["eps0"] for p in problems]), _ptrs([p["U"] for p in problems]),
                                               _ptrs([p["eps_mf"] for p in problems]), nbar, mats_maxit, mats_tol,
                                               mats_mix, boot_maxit, boot_tol, ncorr, st, _stream(stream)))
    return Solve2BStats(int(st[0]), int(st[1]), st[2], st[3])


def plan_waves(footprints: list, cap_bytes: float) -> list:
    """Waves of problems whose device footprints fit under cap_bytes each
    (first fit in order of decreasing footprint): lists of problem indices."""
    order = sorted(range(len(footprints)), key=lambda i: -footprints[i])
    waves, used = [], []
    for i in order:
        if footprints[i] > cap_bytes:
            raise ValueError(f"problem {i} needs {footprints[i]:.3g} B, above the wave cap {cap_bytes:.3g} B")
        for w in range(len(waves)):
            if used[w] + footprints[i] <= cap_bytes:
                waves[w].append(i)
                used[w] += footprints[i]
                break
        else:
            waves.append([i])
            used.append(footprints[i])
    return [sorted(w) for w in waves]

"""GPU adjoint sweep (cntr_adjoint_sweep, the reverse mode of the Dyson
solution for a given self-energy) against central differences of the CPU
oracle. For a random linear objective J = Re <C, G> over every stored block
of slices 0..nt, the directional derivative of J along random directions of
eps, Sigma and M, taken by Richardson-extrapolated central differences of
the oracle's forward solve, must equal Re <grad, direction> from the GPU
gradients. Bar: error <= 1e-7 relative to max(|derivative|, 1e-2 x the summed
magnitude of its contributions). The difference steps (4e-3 and 2e-3 over
the direction's largest entry) keep the oracle's round-off (about 1e-13 of J,
divided by the step) and the O(t^4) truncation of the extrapolation below
about 1e-9 of the derivative."""
import sys

import numpy as np
import pytest
import torch

from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_oracle_dyson import hm

pytestmark = pytest.mark.gpu
TOL = 1e-7
DEV = "cuda"
KEYS3 = ("ret", "les", "tv")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def forward(O, g, S, eps, M):
    """Oracle solution of slices 0..nt for the given Sigma, eps and M."""
    G = hm(O, g)
    G.mat[...] = M
    assert O.dyson_start(G, S, eps) == 0
    for n in range(g.k + 1, g.nt + 1):
        assert O.dyson_timestep(n, G, S, eps, "B") == 0
    return G


def objective(G, C):
    return sum(float(np.vdot(C[f], getattr(G, f)).real) for f in KEYS3)


def fd(O, g, S, eps, M, C, dS, de, dM):
    """Richardson-extrapolated central difference of J along (dS, de, dM)."""
    out = []
    big = max(np.abs(de).max(), np.abs(dM).max(), max(np.abs(dS[f]).max() for f in KEYS3))
    for t in (4e-3 / big, 2e-3 / big):
        Jpm = []
        for sgn in (1.0, -1.0):
            Sp = hm(O, g)
            Sp.mat[...] = S.mat
            for f in KEYS3:
                getattr(Sp, f)[...] = getattr(S, f) + sgn * t * dS[f]
            Jpm.append(objective(forward(O, g, Sp, eps + sgn * t * de, M + sgn * t * dM), C))
        out.append((Jpm[0] - Jpm[1]) / (2 * t))
    return (4 * out[1] - out[0]) / 3


def cplx_normal(r, shape):
    return r.normal(size=shape) + 1j * r.normal(size=shape)


def setup(O, d, nt, ntau, seed):
    g = W.GridSpec(nt=nt, ntau=ntau, d=d, beta=2.0, h=0.05, k=5, mu=0.1)
    r = W.rng(400, seed, d)
    c = W.random_contour(r, g, 0.3)
    S = hm(O, g, c)
    eps = np.array([W.random_hermitian(r, d, 1.0) for _ in range(nt + 2)])
    M = 0.7 * c["mat"][::-1].copy()
    G = forward(O, g, S, eps, M)
    C = {f: cplx_normal(r, getattr(G, f).shape) for f in KEYS3}
    return g, r, S, eps, M, G, C


def gpu_gradients(g, G, S, eps, C, with_sigma=True):
    Gd = K.Contour(g, data={f: getattr(G, f) for f in K.KEYS})
    Sd = K.Contour(g, data={f: getattr(S, f) for f in K.KEYS})
    seed = {f: C[f] for f in KEYS3}
    seed["mat"] = np.zeros_like(G.mat)
    Gb = K.Contour(g, data=seed)
    Sb = K.Contour(g) if with_sigma else None
    e = torch.as_tensor(eps).to(DEV)
    eb = torch.zeros_like(e)
    K.adjoint_sweep([Gd], [Sd], [e], [Gb], [eb], None if Sb is None else [Sb])
    K.sync()
    grads = {"eps": eb.cpu().numpy(), "mat": Gb.mat.cpu().numpy()}
    if Sb is not None:
        grads.update({f: getattr(Sb, f).cpu().numpy() for f in KEYS3})
    return grads


@pytest.mark.parametrize("d,nt,ntau", [(1, 16, 13), (2, 18, 14), (3, 13, 12), (4, 9, 12), (2, 24, 20), (8, 12, 12)])
def test_adjoint_matches_oracle_differences(O, d, nt, ntau):
    say(f"adjoint d={d} nt={nt} ntau={ntau}")
    g, r, S, eps, M, G, C = setup(O, d, nt, ntau, 1)
    grads = gpu_gradients(g, G, S, eps, C)
    zS = {f: np.zeros_like(getattr(S, f)) for f in KEYS3}
    cases = {
        "eps": (zS, cplx_normal(r, eps.shape), np.zeros_like(M)),
        "M": (zS, np.zeros_like(eps), cplx_normal(r, M.shape)),
    }
    for f in KEYS3:
        dS = dict(zS)
        dS[f] = cplx_normal(r, getattr(S, f).shape)
        cases["Sigma." + f] = (dS, np.zeros_like(eps), np.zeros_like(M))
    # single coordinates: the last time step's level and an early one
    for n in (1, g.k, g.k + 1, nt):
        de = np.zeros_like(eps)
        de[n + 1][0, d - 1] = 1.0 + 0.5j
        cases[f"eps[{n}]"] = (zS, de, np.zeros_like(M))
    for name, (dS, de, dM) in cases.items():
        de = de.copy()
        de[0] = 0.0  # eps_{-1} enters only M, which is held fixed here
        ref = fd(O, g, S, eps, M, C, dS, de, dM)
        got = float(np.vdot(grads["eps"], de).real + np.vdot(grads["mat"], dM).real +
                    sum(np.vdot(grads[f], dS[f]).real for f in KEYS3))
        # scale: summed magnitude of the contributions (guards cancellation)
        scale = float(np.abs(grads["eps"].conj() * de).sum() + np.abs(grads["mat"].conj() * dM).sum() +
                      sum(np.abs(grads[f].conj() * dS[f]).sum() for f in KEYS3))
        err = abs(got - ref) / max(abs(ref), 1e-2 * scale, 1e-300)
        say(f"  {name}: adjoint {got:.12e} differences {ref:.12e} rel {err:.2e}")
        assert err < TOL, (name, got, ref, err)


def test_adjoint_without_sigma_output_and_batch(O):
    """Sigmabar = NULL gives the same eps and M gradients; a batch of two
    problems with different nt gives each problem its single-instance result."""
    say("adjoint batch")
    g1, _, S1, e1, M1, G1, C1 = setup(O, 2, 17, 12, 2)
    g2, _, S2, e2, M2, G2, C2 = setup(O, 2, 13, 12, 3)
    ref1 = gpu_gradients(g1, G1, S1, e1, C1)
    ref2 = gpu_gradients(g2, G2, S2, e2, C2)
    alone = gpu_gradients(g1, G1, S1, e1, C1, with_sigma=False)
    for key in ("eps", "mat"):
        assert np.abs(alone[key] - ref1[key]).max() <= 1e-13 * np.abs(ref1[key]).max()
    items = []
    for g, G, S, e, C in ((g1, G1, S1, e1, C1), (g2, G2, S2, e2, C2)):
        seed = {f: C[f] for f in KEYS3}
        seed["mat"] = np.zeros_like(G.mat)
        items.append(dict(G=K.Contour(g, data={f: getattr(G, f) for f in K.KEYS}),
                          S=K.Contour(g, data={f: getattr(S, f) for f in K.KEYS}),
                          e=torch.as_tensor(e).to(DEV), Gb=K.Contour(g, data=seed), Sb=K.Contour(g)))
    for it in items:
        it["eb"] = torch.zeros_like(it["e"])
    K.adjoint_sweep([it["G"] for it in items], [it["S"] for it in items], [it["e"] for it in items],
                    [it["Gb"] for it in items], [it["eb"] for it in items], [it["Sb"] for it in items])
    K.sync()
    for it, ref in zip(items, (ref1, ref2)):
        assert np.abs(it["eb"].cpu().numpy() - ref["eps"]).max() <= 1e-12 * np.abs(ref["eps"]).max()
        assert np.abs(it["Gb"].mat.cpu().numpy() - ref["mat"]).max() <= 1e-12 * np.abs(ref["mat"]).max()
        for f in KEYS3:
            x = getattr(it["Sb"], f).cpu().numpy()
            assert np.abs(x - ref[f]).max() <= 1e-12 * np.abs(ref[f]).max()


# ------------------------------------------------------------ second-Born chain
def forward_2b(O, g, e0, U):
    """Oracle self-consistent 2B + Hartree solution (tight loops)."""
    G, S = hm(O, g), hm(O, g)
    rc, emf, _ = O.solve_2b(G, S, e0, U, ncorr=12, mats_tol=1e-15, boot_tol=1e-15, boot_maxit=200)
    assert rc == 0
    return G, S, emf


def setup_2b(O, d, nt, ntau, seed):
    g = W.GridSpec(nt=nt, ntau=ntau, d=d, beta=2.0, h=0.05, k=5)
    r = W.rng(401, seed, d)
    H0 = W.random_hermitian(r, d, 1.0)
    e0 = np.array([H0 + (0.3 * np.sin(0.7 * n) * W.random_hermitian(r, d, 1.0) if n > 0 else 0)
                   for n in range(nt + 2)])
    U = 0.8 + 0.2 * r.uniform(size=nt + 2)
    C = {f: 0.3 * cplx_normal(r, s) for f, s in (("ret", (g.ntri, d, d)), ("les", (g.ntri, d, d)),
                                                   ("tv", ((nt + 1) * (ntau + 1), d, d)))}
    return g, r, e0, U, C


def gpu_gradients_2b(g, e0, U, C, niter=10, tol=1e-13):
    """GPU forward (cntr_solve_2b) then the second-Born adjoint sweep."""
    G, S, Gs = K.Contour(g), K.Contour(g), K.Contour(g)
    e0d = torch.as_tensor(e0).to(DEV)
    Ud = torch.as_tensor(U).to(DEV)
    emf = torch.zeros_like(e0d)
    K.solve_2b(G, S, Gs, e0d, Ud, emf, mats_tol=1e-15, boot_tol=1e-15, boot_maxit=200, ncorr=12)
    seed = {f: C[f] for f in KEYS3}
    seed["mat"] = np.zeros((g.ntau + 1, g.d, g.d), np.complex128)
    Gb, Sb = K.Contour(g, data=seed), K.Contour(g)
    eb = torch.zeros_like(e0d)
    ub = torch.zeros_like(Ud)
    conv = K.adjoint_sweep([G], [S], [emf], [Gb], [eb], [Sb], U=[Ud], U_bar=[ub], niter=niter, tol=tol)
    K.sync()
    return eb.cpu().numpy(), ub.cpu().numpy(), conv


@pytest.mark.parametrize("d,nt,ntau", [(2, 14, 12), (1, 17, 13), (3, 12, 12), (4, 11, 12), (8, 9, 12)])
def test_adjoint_2b_matches_oracle_differences(O, d, nt, ntau):
    """Gradients of J = Re <C, G> of the self-consistent 2B + Hartree solution
    with respect to eps0_n and U_n, n = -1..nt (n = -1 enters through the
    Matsubara solve; eps0 directions hermitian, as the solution assumes)."""
    say(f"adjoint 2B d={d} nt={nt} ntau={ntau}")
    g, r, e0, U, C = setup_2b(O, d, nt, ntau, 1)
    ge, ub, conv = gpu_gradients_2b(g, e0, U, C)
    say(f"  fixed points: largest relative change {conv:.2e}")
    assert conv < 1e-13
    cases = {}
    de = cplx_normal(r, e0.shape)
    de[0] = 0.0
    cases["eps0"] = (de, np.zeros_like(U))
    dU = r.normal(size=U.shape)
    dU[0] = 0.0
    cases["U"] = (np.zeros_like(e0), dU)
    x = np.zeros_like(U)
    x[0] = 1.0
    cases["U[-1]"] = (np.zeros_like(e0), x)
    y = np.zeros_like(e0)
    y[0] = W.random_hermitian(r, d, 1.0)
    cases["eps0[-1]"] = (y, np.zeros_like(U))
    y = np.array([W.random_hermitian(r, d, 1.0) for _ in range(nt + 2)])
    cases["all"] = (y, r.normal(size=U.shape))
    for n in (g.k, nt):
        x = np.zeros_like(U)
        x[n + 1] = 1.0
        cases[f"U[{n}]"] = (np.zeros_like(e0), x)
        y = np.zeros_like(e0)
        y[n + 1][0, d - 1] = 1.0 - 0.5j
        y[n + 1][d - 1, 0] = 1.0 + 0.5j
        cases[f"eps0[{n}]"] = (y, np.zeros_like(U))
    for name, (de, dU) in cases.items():
        big = max(np.abs(de).max(), np.abs(dU).max())
        out = []
        for t in (4e-3 / big, 2e-3 / big):
            Jp = objective(forward_2b(O, g, e0 + t * de, U + t * dU)[0], C)
            Jm = objective(forward_2b(O, g, e0 - t * de, U - t * dU)[0], C)
            out.append((Jp - Jm) / (2 * t))
        ref = (4 * out[1] - out[0]) / 3
        got = float(np.vdot(ge, de).real + np.dot(ub, dU))
        scale = float(np.abs(ge.conj() * de).sum() + np.abs(ub * dU).sum())
        err = abs(got - ref) / max(abs(ref), 1e-2 * scale, 1e-300)
        say(f"  {name}: adjoint {got:.12e} differences {ref:.12e} rel {err:.2e}")
        assert err < TOL, (name, got, ref, err)


def test_adjoint_2b_reports_unconverged_fixed_points(O):
    """One fixed-point iteration per slice leaves a change far above 1e-13:
    with that tolerance the sweep returns CNTR_ENOCONV; without it, the
    change is still reported."""
    from paper_1911_01211_amd import _abi
    say("adjoint 2B tolerance")
    g, r, e0, U, C = setup_2b(O, 2, 12, 12, 2)
    with pytest.raises(_abi.CntrError) as ex:
        gpu_gradients_2b(g, e0, U, C, niter=1, tol=1e-13)
    assert ex.value.code == -8
    _, _, conv = gpu_gradients_2b(g, e0, U, C, niter=1, tol=0.0)
    assert conv > 1e-13

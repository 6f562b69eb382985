"""GPU parity of the momentum-convolution self-energies (cntr_polarization_k,
cntr_sigma_gw_k; Eqs. Pol and Sigmak) against the oracle (oracle/kspace.py):
every component of the slice, every momentum, max-norm error <= 1e-10
relative to the slice's largest value. Inputs: per momentum a quenched free
function (a band
eps_k = -2 cos(2 pi k / Nk) plus a seeded hermitian part for d > 1; bosonic
dW from the same recipe with mu below the levels); d = 1, 2, 3; Nk up to
260 (more momenta than threads of a workgroup); slices -1 (Matsubara), 0, a
middle one and the last."""
import numpy as np
import pytest

from oracle import free_green as FG
from oracle import kspace as KS
from oracle import oracle as O
from paper_1911_01211_amd import _abi
from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import require_gpu, say
from tests.vie2_inputs import herm

pytestmark = pytest.mark.gpu


def band(nk, d, k, nt, ntau, sig, seed, h=0.1, beta=2.0, korder=3):
    """Free functions of eps_k(0^-) = b_k + H0, eps_k(t >= 0) = b_k' + H1 (quench)."""
    r = W.rng(1914, seed)
    H0, H1 = herm(r, d, 0.5), herm(r, d, 0.5)
    out = []
    mus = []
    eps_all = []
    for kk in range(nk):
        bk = -2.0 * np.cos(2 * np.pi * kk / nk)
        eps = np.zeros((nt + 2, d, d), np.complex128)
        eps[0] = bk * np.eye(d) + H0
        eps[1:] = -2.0 * np.cos(2 * np.pi * kk / nk - 0.4) * np.eye(d) + H1
        eps_all.append(eps)
        mus.append(min(np.linalg.eigvalsh(eps[0]).min(), np.linalg.eigvalsh(eps[1]).min()))
    mu = 0.0 if sig < 0 else min(mus) - 0.5
    for kk in range(nk):
        out.append(FG.green_from_H(O.Grid(nt, ntau, d, sig, korder, beta, h, mu), eps_all[kk]))
    return out


def spec(g):
    return W.GridSpec(nt=g.nt, ntau=g.ntau, d=g.d, sig=g.sig, k=g.k, beta=g.beta, h=g.h, mu=g.mu)


def dev(X):
    return K.Contour(spec(X.g), "cuda", data={f: getattr(X, f) for f in K.KEYS})


def comp_slices(g, n):
    if n == -1:
        return {"mat": slice(0, g.ntau + 1)}
    o = n * (n + 1) // 2
    return {"ret": slice(o, o + n + 1), "les": slice(o, o + n + 1),
            "tv": slice(n * (g.ntau + 1), (n + 1) * (g.ntau + 1))}


@pytest.mark.parametrize("d,nk,nt,ntau,kord", [(1, 8, 10, 12, 3), (2, 5, 7, 10, 2), (3, 3, 6, 8, 2),
                                               (1, 260, 1, 4, 1)])
def test_kspace_bubbles_parity(O, d, nk, nt, ntau, kord):
    require_gpu()
    say(f"kspace d={d} nk={nk} nt={nt} ntau={ntau}")
    G = band(nk, d, kord, nt, ntau, -1, seed=11, korder=kord)
    Wb = band(nk, d, kord, nt, ntau, 1, seed=12, korder=kord)
    g = G[0].g
    Gd = [dev(x) for x in G]
    Wd = [dev(x) for x in Wb]
    slices = [-1, 0, nt] if nt < 4 else [-1, 0, nt // 2, nt]
    for n in slices:
        Pi = [O.HM(g) for _ in range(nk)]
        Sg = [O.HM(g) for _ in range(nk)]
        KS.polarization(n, G, Pi, 0.7)
        KS.sigma_gw(n, G, Wb, Sg, -1.3)
        Pid = [K.Contour(spec(g), "cuda") for _ in range(nk)]
        Sgd = [K.Contour(spec(g), "cuda") for _ in range(nk)]
        K.polarization_k(n, Gd, Pid, 0.7)
        K.sigma_gw_k(n, Gd, Wd, Sgd, -1.3)
        K.sync()
        for name, ref, got in (("Pi", Pi, Pid), ("Sigma", Sg, Sgd)):
            # (a component can vanish identically, e.g. Pi^R at t = t' off the
            # orbital diagonal: the norm is the slice's largest value)
            rs = {c: np.stack([getattr(x, c)[sl] for x in ref]) for c, sl in comp_slices(g, n).items()}
            scale = max(np.abs(r).max() for r in rs.values())
            for comp, sl in comp_slices(g, n).items():
                o = np.stack([getattr(x, comp)[sl].cpu().numpy() for x in got])
                e = float(np.abs(o - rs[comp]).max() / scale)
                assert e <= 1e-10, (name, n, comp, e)
        say(f"  slices {slices} ok")


def test_kspace_equal_time_lesser_as_stored(O):
    """A computed G^<(t,t) is anti-hermitian only up to the solver's error:
    the bubbles take the stored equal-time lesser value as it is (the oracle
    reads it so). Inputs whose G^<(t_n,t_n) carry a hermitian part of 1e-2."""
    require_gpu()
    d, nk, nt, ntau = 2, 3, 6, 8
    G = band(nk, d, 2, nt, ntau, -1, seed=14, korder=2)
    Wb = band(nk, d, 2, nt, ntau, 1, seed=15, korder=2)
    r = W.rng(1915, 0)
    for X in G + Wb:
        for n in range(nt + 1):
            X.les[n * (n + 1) // 2 + n] += 1e-2 * herm(r, d)
    g = G[0].g
    Gd, Wd = [dev(x) for x in G], [dev(x) for x in Wb]
    for n in (0, 3, nt):
        Pi, Sg = [O.HM(g) for _ in range(nk)], [O.HM(g) for _ in range(nk)]
        KS.polarization(n, G, Pi)
        KS.sigma_gw(n, G, Wb, Sg)
        Pid, Sgd = [K.Contour(spec(g), "cuda") for _ in range(nk)], [K.Contour(spec(g), "cuda") for _ in range(nk)]
        K.polarization_k(n, Gd, Pid)
        K.sigma_gw_k(n, Gd, Wd, Sgd)
        K.sync()
        for name, ref, got in (("Pi", Pi, Pid), ("Sigma", Sg, Sgd)):
            for comp, sl in comp_slices(g, n).items():
                rr = np.stack([getattr(x, comp)[sl] for x in ref])
                o = np.stack([getattr(x, comp)[sl].cpu().numpy() for x in got])
                assert np.abs(o - rr).max() <= 1e-12 * max(1.0, np.abs(rr).max()), (name, n, comp)


def test_kspace_errors(O):
    require_gpu()
    G = band(2, 1, 2, 4, 6, -1, seed=13, korder=2)
    Gd = [dev(x) for x in G]
    with pytest.raises(_abi.CntrError) as e:
        K.polarization_k(5, Gd, [K.Contour(spec(G[0].g), "cuda") for _ in range(2)])
    assert e.value.code == -3
    L = _abi.lib()
    rc = L.cntr_sigma_gw_k(1, 2, K._grids(Gd), K._gfs(Gd), None, K._gfs(Gd), 1.0, K._stream())
    assert rc == -2


def test_gw_propagation_matches_oracle(O):
    """The whole self-consistent GW loop (Matsubara, start-up, predictor-
    corrector steps) on four momenta with a field pulse: every component of
    every G_k and Sigma_k against the oracle's solve_gw."""
    require_gpu()
    import torch
    from tests.test_oracle_kspace import gw_band
    say("gw loop nk=4 nt=16")
    g, eps = gw_band(16, 0.1, ntau=20)
    G = [O.HM(g) for _ in range(4)]
    _, _, S = KS.solve_gw(G, eps, 1.0, mats_iters=6, boot_iters=4, ncorr=3)
    Gd = [K.Contour(spec(g), "cuda") for _ in range(4)]
    ed = [torch.as_tensor(e).to("cuda") for e in eps]
    _, _, Sd = K.solve_gw_k(Gd, ed, 1.0, mats_iters=6, boot_iters=4, ncorr=3)
    K.sync()
    for name, ref, got in (("G", G, Gd), ("Sigma", S, Sd)):
        for comp in K.KEYS:
            r = np.stack([getattr(x, comp) for x in ref])
            o = np.stack([getattr(x, comp).cpu().numpy() for x in got])
            e = float(np.abs(o - r).max() / np.abs(r).max())
            say(f"  {name} {comp}: {e:.2e}")
            assert e <= 1e-10, (name, comp, e)


def test_kspace_bench_shape_sampled(O):
    """The momentum sums at the bench's shape (256 momenta, d = 1, ntau = 500,
    slice 400, and the Matsubara slice) on seeded random contour functions:
    every component of Pi_k and Sigma_k for three sampled momenta against the
    oracle's sums over q written out here (Eqs. Pol, Sigmak), <= 1e-10
    relative to the slice's largest value."""
    require_gpu()
    nk, n = 256, 400
    g = O.Grid(n, 500, 1, -1, 5, 10.0, 0.02, 0.0)
    gb = O.Grid(n, 500, 1, 1, 5, 10.0, 0.02, 0.0)
    say(f"kspace bench shape nk={nk} n={n}")
    r = W.rng(1920, 0)

    def rnd(gg):
        X = O.HM(gg)
        data = W.random_contour(r, spec(gg), 0.5)
        for f in K.KEYS:
            getattr(X, f)[...] = data[f]
        return X

    G = [rnd(g) for _ in range(nk)]
    Wq = [rnd(gb) for _ in range(nk)]
    Gd, Wd = [dev(x) for x in G], [dev(x) for x in Wq]
    Pid = [K.Contour(spec(g), "cuda") for _ in range(nk)]
    Sgd = [K.Contour(spec(g), "cuda") for _ in range(nk)]
    KB = K.KBatch(Gd, Pid, Wd, Sgd)
    for tstp in (-1, n):
        KB.polarization(tstp, 1.0)
        KB.sigma(tstp, 1.0)
    K.sync()
    for kk in (0, 97, 255):
        for tstp in (-1, n):
            pi = None
            sg = None
            for q in range(nk):
                b1 = KS.bubble1(tstp, G[(kk + q) % nk], G[q])
                b2 = KS.bubble2(tstp, G[(kk - q) % nk], Wq[q])
                pi = b1 if pi is None else {c: pi[c] + b1[c] for c in pi}
                sg = b2 if sg is None else {c: sg[c] + b2[c] for c in sg}
            for name, ref, got, sc in (("Pi", pi, Pid[kk], -1.0 / nk), ("Sigma", sg, Sgd[kk], 1.0 / nk)):
                sl = comp_slices(g, tstp)
                scale = max(np.abs(sc * ref[c]).max() for c in sl)
                for comp, s_ in sl.items():
                    e = float(np.abs(getattr(got, comp)[s_].cpu().numpy() - sc * ref[comp]).max() / scale)
                    assert e <= 1e-10, (name, kk, tstp, comp, e)
    say("  sampled momenta 0, 97, 255 ok")

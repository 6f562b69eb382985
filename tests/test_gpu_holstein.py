"""GPU parity of the Holstein DMFT pieces (cntr_phonon_free, cntr_scale_slice,
cntr_holstein_mf; Sec. "DMFT for the Holstein model") and of the whole
Bethe-lattice uMig loop (contour.solve_holstein) against the oracle
(oracle/holstein.py), max-norm error relative to the largest value <= 1e-10.
The GPU's D0 comes from closed forms, the oracle's from the contour
transposition of its free single-pole function. Inputs: seeded random
contour functions (d = 1, 2) and real series for the scaling and the
displacement; the loop runs the pinned drive of the oracle tests (g(t), J(t)
modulated, mu = -1.3, beta = 2)."""
import numpy as np
import pytest
import torch

from oracle import holstein as H
from paper_1911_01211_amd import _abi
from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import require_gpu, say
from tests.test_oracle_holstein import drive

pytestmark = pytest.mark.gpu


def spec(g):
    return W.GridSpec(nt=g.nt, ntau=g.ntau, d=g.d, sig=g.sig, k=g.k, beta=g.beta, h=g.h, mu=g.mu)


def rel(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def check(X, ref, tol=1e-10, what=""):
    for f in K.KEYS:
        e = rel(getattr(X, f).cpu().numpy(), getattr(ref, f))
        assert e <= tol, (what, f, e)


def test_phonon_free_parity(O):
    require_gpu()
    for nt, ntau, beta, h, w0 in ((20, 30, 3.0, 0.1, 0.7), (13, 17, 40.0, 0.05, 2.5)):
        g = O.Grid(nt, ntau, 1, -1, 4, beta, h, 0.0)
        ref = H.phonon_d0(g, w0)
        D = K.Contour(spec(ref.g), "cuda")
        K.phonon_free([D], [w0])
        K.sync()
        check(D, ref, 1e-12, f"D0 w0={w0} beta={beta}")


@pytest.mark.parametrize("d", [1, 2])
def test_scale_slice_parity(O, d):
    require_gpu()
    g = O.Grid(9, 11, d, -1, 3, 2.0, 0.1, 0.0)
    r = W.rng(1917, d)
    A = O.HM(g)
    Cr = O.HM(g)
    for X in (A, Cr):
        data = W.random_contour(r, spec(g), 1.0)
        for f in K.KEYS:
            getattr(X, f)[...] = data[f]
    f = r.normal(size=g.nt + 2)
    Ad = K.Contour(spec(g), "cuda", data={k: getattr(A, k) for k in K.KEYS})
    Cd = K.Contour(spec(g), "cuda", data={k: getattr(Cr, k) for k in K.KEYS})
    fd = torch.as_tensor(f).to("cuda")
    for n, beta in ((-1, 0.0), (0, 0.7), (4, 0.0), (9, 1.0), (-1, 1.0)):
        H.scale(n, Cr, A, f, beta)
        K.scale_slice(n, [Cd], [Ad], [fd], beta)
    K.sync()
    check(Cd, Cr, 1e-14, f"scale d={d}")


def test_holstein_mf_parity(O):
    require_gpu()
    g = O.Grid(24, 12, 1, -1, 5, 2.0, 0.1, 0.0)
    r = W.rng(1918, 0)
    G = O.HM(g)
    data = W.random_contour(r, spec(g), 0.5)
    for f in K.KEYS:
        getattr(G, f)[...] = data[f]
    gel = 0.5 + 0.1 * r.normal(size=g.nt + 2)
    w0 = 0.6
    Xr = np.zeros(g.nt + 2)
    Gd = K.Contour(spec(g), "cuda", data={k: getattr(G, k) for k in K.KEYS})
    gd = torch.as_tensor(gel).to("cuda")
    Xd = torch.zeros(g.nt + 2, dtype=torch.float64, device="cuda")
    ed = torch.zeros((g.nt + 2, 1, 1), dtype=torch.complex128, device="cuda")
    for n in range(-1, g.nt + 1):
        H.displacement(n, G, gel, w0, Xr)
        K.holstein_mf(n, [Gd], [gd], [w0], 0.3, [Xd], [ed])
    K.sync()
    assert rel(Xd.cpu().numpy(), Xr) <= 1e-12
    assert rel(ed.cpu().numpy()[:, 0, 0], 0.3 + gel * Xr) <= 1e-12


def test_holstein_dmft_matches_oracle(O):
    require_gpu()
    nt, h = 24, 0.1
    say(f"holstein dmft nt={nt}")
    g = O.Grid(nt, 20, 1, -1, 5, 2.0, h, -1.3)
    J, gel = drive(nt, h)
    G = O.HM(g)
    _, Dr, Sr, Xr, er = H.solve_holstein(G, J, gel, 0.5, mats_iters=20, boot_iters=6, ncorr=4)
    Gd = K.Contour(spec(g), "cuda")
    Jd, gd = torch.as_tensor(J).to("cuda"), torch.as_tensor(gel).to("cuda")
    _, Dd, Sd, Xd, ed = K.solve_holstein(Gd, Jd, gd, 0.5, mats_iters=20, boot_iters=6, ncorr=4)
    K.sync()
    for name, ref, got in (("G", G, Gd), ("Delta", Dr, Dd), ("Sigma", Sr, Sd)):
        for f in K.KEYS:
            e = rel(getattr(got, f).cpu().numpy(), getattr(ref, f))
            say(f"  {name} {f}: {e:.2e}")
            assert e <= 1e-10, (name, f, e)
    assert rel(Xd.cpu().numpy(), Xr) <= 1e-10
    assert rel(ed.cpu().numpy(), er) <= 1e-10


def test_holstein_errors(O):
    require_gpu()
    L = _abi.lib()
    g = W.GridSpec(nt=4, ntau=6, d=2, sig=1, k=2, beta=2.0, h=0.1, mu=0.0)
    D = K.Contour(g, "cuda")
    with pytest.raises(_abi.CntrError) as e:
        K.phonon_free([D], [0.5])
    assert e.value.code == -2
    g1 = W.GridSpec(nt=4, ntau=6, d=1, sig=1, k=2, beta=2.0, h=0.1, mu=0.0)
    D1 = K.Contour(g1, "cuda")
    with pytest.raises(_abi.CntrError) as e:
        K.phonon_free([D1], [0.0])
    assert e.value.code == -1
    f = torch.ones(g1.nt + 2, dtype=torch.float64, device="cuda")
    with pytest.raises(_abi.CntrError) as e:
        K.scale_slice(5, [D1], [D1], [f])
    assert e.value.code == -3
    assert L.cntr_scale_slice(0, 1, K._grids([D1]), K._gfs([D1]), K._gfs([D1]), None, 0.0, K._stream()) == -2
    # the local bubble: slice outside -1..nt, null outputs
    with pytest.raises(_abi.CntrError) as e:
        K.bubble2_local(5, [D1], [D1], [D1])
    assert e.value.code == -3
    assert L.cntr_bubble2_local(0, 1, K._grids([D1]), K._gfs([D1]), K._gfs([D1]), None, 1.0, K._stream()) == -2
    # the displacement: single band only, slices -1..nt, w0 > 0
    X = torch.zeros(g1.nt + 2, dtype=torch.float64, device="cuda")
    ep = torch.zeros((g1.nt + 2, 1, 1), dtype=torch.complex128, device="cuda")
    with pytest.raises(_abi.CntrError) as e:
        K.holstein_mf(0, [D], [f], [0.5], 0.0, [X], [ep])
    assert e.value.code == -2
    with pytest.raises(_abi.CntrError) as e:
        K.holstein_mf(g1.nt + 1, [D1], [f], [0.5], 0.0, [X], [ep])
    assert e.value.code == -3
    with pytest.raises(_abi.CntrError) as e:
        K.holstein_mf(0, [D1], [f], [-1.0], 0.0, [X], [ep])
    assert e.value.code == -1


@pytest.mark.parametrize("d", [1, 2])
def test_bubble2_local_parity(O, d):
    """cntr_bubble2_local: C_i = alpha i A_i B_i per instance (no momentum sum)
    against the oracle's one-momentum Sigma (oracle/kspace.py)."""
    require_gpu()
    from oracle import kspace as KS
    g = O.Grid(8, 12, d, -1, 3, 2.0, 0.1, 0.0)
    r = W.rng(1919, d)
    As, Bs = [], []
    for _ in range(3):
        for L in (As, Bs):
            X = O.HM(g)
            data = W.random_contour(r, spec(g), 1.0)
            for f in K.KEYS:
                getattr(X, f)[...] = data[f]
            L.append(X)
    Cs = [O.HM(g) for _ in range(3)]
    Ad = [K.Contour(spec(g), "cuda", data={k: getattr(x, k) for k in K.KEYS}) for x in As]
    Bd = [K.Contour(spec(g), "cuda", data={k: getattr(x, k) for k in K.KEYS}) for x in Bs]
    Cd = [K.Contour(spec(g), "cuda") for _ in range(3)]
    for n in (-1, 0, 5, 8):
        for i in range(3):
            KS.sigma_gw(n, [As[i]], [Bs[i]], [Cs[i]], -0.8)
        K.bubble2_local(n, Ad, Bd, Cd, -0.8)
    K.sync()
    for i in range(3):
        check(Cd[i], Cs[i], 1e-13, f"bubble2_local d={d} i={i}")


def test_holstein_batch_is_the_single_solve(O):
    """Three impurities (couplings 0.4, 0.5, 0.6 with their half-filling mu)
    advanced together equal three single solves, bit for bit."""
    require_gpu()
    nt, h = 16, 0.1
    gs, Js, gels, Gs = [], [], [], []
    for g0 in (0.4, 0.5, 0.6):
        gg = W.GridSpec(nt=nt, ntau=20, d=1, sig=-1, k=5, beta=2.0, h=h, mu=-2 * g0 * g0 / 0.5)
        J, gel = drive(nt, h)
        gel = gel - 0.5 + g0
        gs.append(gg)
        Js.append(torch.as_tensor(J).to("cuda"))
        gels.append(torch.as_tensor(gel).to("cuda"))
        Gs.append(K.Contour(gg, "cuda"))
    kw = dict(mats_iters=10, boot_iters=4, ncorr=3)
    _, _, _, Xb, _ = K.solve_holstein(Gs, Js, gels, [0.5] * 3, **kw)
    for i in range(3):
        G1 = K.Contour(gs[i], "cuda")
        _, _, _, X1, _ = K.solve_holstein(G1, Js[i], gels[i], 0.5, **kw)
        K.sync()
        for f in K.KEYS:
            assert torch.equal(getattr(Gs[i], f), getattr(G1, f)), (i, f)
        assert torch.equal(Xb[i], X1), i


def test_holstein_dmft_long_matches_oracle(O):
    """The loop to nt = 280 (the d = 1 history sums span two term chunks of
    256): every component of G, Delta and Sigma and the displacement against
    the oracle."""
    require_gpu()
    nt, h = 280, 0.05
    say(f"holstein dmft nt={nt}")
    g = O.Grid(nt, 30, 1, -1, 5, 2.0, h, -1.3)
    J, gel = drive(nt, h)
    G = O.HM(g)
    kw = dict(mats_iters=10, boot_iters=4, ncorr=3)
    _, Dr, Sr, Xr, er = H.solve_holstein(G, J, gel, 0.5, **kw)
    Gd = K.Contour(spec(g), "cuda")
    _, Dd, Sd, Xd, ed = K.solve_holstein(Gd, torch.as_tensor(J).to("cuda"), torch.as_tensor(gel).to("cuda"), 0.5,
                                         **kw)
    K.sync()
    for name, ref, got in (("G", G, Gd), ("Delta", Dr, Dd), ("Sigma", Sr, Sd)):
        for f in K.KEYS:
            e = rel(getattr(got, f).cpu().numpy(), getattr(ref, f))
            assert e <= 1e-10, (name, f, e)
    assert rel(Xd.cpu().numpy(), Xr) <= 1e-10
    assert rel(ed.cpu().numpy(), er) <= 1e-10

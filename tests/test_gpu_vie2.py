"""GPU parity of the Dyson equation in integral form, (1 + F) * G = Q
(cntr_vie2_matsubara, cntr_vie2_step), against the oracle on the same seeded
inputs: every component of every slice, relative max-norm error <= 1e-10.
Inputs: the quenched downfolding kernel (F = -g_A * Sigma, F^R(t,t) = 0) and
the instantaneous kernel (F = -g c, F^R(t,t) = i c), both from
tests/vie2_inputs.py; sizes span several reduce tiles and ragged tails, the
regime k < n <= 2k (every lesser row summed directly), d = 1..8 (the d = 4
one-pass and d = 8 matrix-core history paths), fermions and bosons."""
import numpy as np
import pytest
import torch

from paper_1911_01211_amd import _abi
from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import relerr, require_gpu, say
from tests.vie2_inputs import downfold, instantaneous

pytestmark = pytest.mark.gpu
TOL = 1e-10


def spec(g):
    return W.GridSpec(nt=g.nt, ntau=g.ntau, d=g.d, sig=g.sig, k=g.k, beta=g.beta, h=g.h, mu=g.mu)


def dev(g, X):
    return K.Contour(spec(g), "cuda", data={f: getattr(X, f) for f in K.KEYS})


def inputs(kind, d, k, nt, ntau, sig, seed=3):
    if kind == "down":
        g, F, Fcc, Q, _, _, _ = downfold(k, nt, 0.05, ntau, 2.0, d, 2, seed=seed, sig=sig)
    else:
        g, F, Fcc, Q, _ = instantaneous(k, nt, 0.05, ntau, 2.0, d, seed=seed, sig=sig)
    return g, F, Fcc, Q


def compare(O, g, Gd, G, what):
    out = Gd.numpy()
    for f in K.KEYS:
        e = relerr(out[f], getattr(G, f))
        say(f"  {what} {f}: {e:.2e}")
        assert e <= TOL, (what, f, e)


CASES = [
    ("down", 1, 5, 40, 30, -1),
    ("inst", 1, 1, 6, 5, -1),
    ("inst", 2, 3, 33, 17, 1),
    ("down", 3, 2, 25, 20, -1),
    ("inst", 4, 5, 70, 40, -1),
    ("down", 4, 1, 20, 10, -1),
    ("inst", 4, 4, 9, 12, 1),
    ("inst", 5, 4, 30, 12, -1),
    ("inst", 8, 5, 40, 20, -1),
    ("down", 8, 2, 19, 9, 1),
]


@pytest.mark.parametrize("kind,d,k,nt,ntau,sig", CASES)
def test_vie2_parity(O, kind, d, k, nt, ntau, sig):
    require_gpu()
    say(f"vie2 parity {kind} d={d} k={k} nt={nt} ntau={ntau} sig={sig}")
    g, F, Fcc, Q = inputs(kind, d, k, nt, ntau, sig)
    G = O.HM(g)
    assert O.solve_vie2(G, F, Fcc, Q) == 0
    Gd = K.Contour(spec(g), "cuda")
    Fd, Fccd, Qd = dev(g, F), dev(g, Fcc), dev(g, Q)
    K.solve_vie2([Gd], [Fd], [Fccd], [Qd])
    K.sync()
    compare(O, g, Gd, G, "G")


def test_vie2_long_d4(O):
    """d = 4 up to n = 400: the history kernel's one-pass units of 16 and 32
    slices and many reduce tiles."""
    require_gpu()
    say("vie2 long d=4 nt=400")
    g, F, Fcc, Q = inputs("inst", 4, 5, 400, 60, -1, seed=4)
    G = O.HM(g)
    assert O.solve_vie2(G, F, Fcc, Q) == 0
    Gd = K.Contour(spec(g), "cuda")
    K.solve_vie2([Gd], [dev(g, F)], [dev(g, Fcc)], [dev(g, Q)])
    K.sync()
    compare(O, g, Gd, G, "G")


def test_vie2_batch_uneven_lengths(O):
    """Three problems of one call, nt 12, 25, 31: each step skips the
    problems that have ended; each matches its own oracle solve."""
    require_gpu()
    say("vie2 batch nt=(12,25,31)")
    probs = [inputs("inst", 2, 3, nt, 14, -1, seed=10 + nt) for nt in (12, 25, 31)]
    refs, Gs, Fs, Fccs, Qs = [], [], [], [], []
    for g, F, Fcc, Q in probs:
        G = O.HM(g)
        assert O.solve_vie2(G, F, Fcc, Q) == 0
        refs.append(G)
        Gs.append(K.Contour(spec(g), "cuda"))
        Fs.append(dev(g, F))
        Fccs.append(dev(g, Fcc))
        Qs.append(dev(g, Q))
    K.vie2_matsubara(Gs, Fs, Qs)
    K.vie2_step(3, Gs, Fs, Fccs, Qs)
    for n in range(4, 32):
        K.vie2_step(n, Gs, Fs, Fccs, Qs)
    K.sync()
    for (g, _, _, _), G, Gd in zip(probs, refs, Gs):
        compare(O, g, Gd, G, f"nt={g.nt}")


@pytest.mark.parametrize("nb,d", [(18, 1), (18, 4), (260, 1)])
def test_vie2_large_batch_is_the_single_solve(O, nb, d):
    """nb problems of one call (a reduce workgroup per tile, or from 256 on
    one per problem, which walks its tiles) with nt up to 40: bit for bit the
    one-problem solves, and the oracle for two of them."""
    require_gpu()
    say(f"vie2 batch of {nb}, d={d}")
    probs = [inputs("inst", d, 5, 24 + (i % 3) * 8, 14, -1, seed=40 + i) for i in range(nb)]
    Gs = [K.Contour(spec(g), "cuda") for g, _, _, _ in probs]
    Fs = [dev(g, F) for g, F, _, _ in probs]
    Fccs = [dev(g, Fcc) for g, _, Fcc, _ in probs]
    Qs = [dev(g, Q) for g, _, _, Q in probs]
    K.vie2_matsubara(Gs, Fs, Qs)
    K.vie2_step(5, Gs, Fs, Fccs, Qs)
    for n in range(6, 41):
        K.vie2_step(n, Gs, Fs, Fccs, Qs)
    for i in (0, 7, nb - 1):
        G1 = K.Contour(spec(probs[i][0]), "cuda")
        K.solve_vie2([G1], [Fs[i]], [Fccs[i]], [Qs[i]])
        K.sync()
        for f in K.KEYS:
            assert torch.equal(getattr(Gs[i], f), getattr(G1, f)), (i, f)
    for i in (0, nb - 1):
        g, F, Fcc, Q = probs[i]
        G = O.HM(g)
        assert O.solve_vie2(G, F, Fcc, Q) == 0
        compare(O, g, Gs[i], G, f"batch member {i}")


def test_vie2_errors(O):
    require_gpu()
    g, F, Fcc, Q = inputs("inst", 2, 2, 8, 6, -1)
    Gd, Fd, Fccd, Qd = K.Contour(spec(g), "cuda"), dev(g, F), dev(g, Fcc), dev(g, Q)
    with pytest.raises(_abi.CntrError) as e:
        K.vie2_step(9, [Gd], [Fd], [Fccd], [Qd])
    assert e.value.code == -3
    L = _abi.lib()
    rc = L.cntr_vie2_step(3, 1, K._grids([Gd]), K._gfs([Gd]), K._gfs([Fd]), None, K._gfs([Qd]), K._stream())
    assert rc == -2
    # steps before the start-up are refused when order checks are on
    K.set_checks(order=True)
    try:
        G2 = K.Contour(spec(g), "cuda")
        K.vie2_matsubara([G2], [Fd], [Qd])
        with pytest.raises(_abi.CntrError) as e:
            K.vie2_step(4, [G2], [Fd], [Fccd], [Qd])
        assert e.value.code == -3
        K.vie2_step(2, [G2], [Fd], [Fccd], [Qd])
        K.vie2_step(3, [G2], [Fd], [Fccd], [Qd])
    finally:
        K.set_checks()
    K.sync()
    torch.cuda.synchronize()

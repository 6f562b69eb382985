"""GPU parity of cntr_green_from_H (free Green's function of a driven
Hamiltonian, Eqs. cf4 and G0_free) against the oracle, through the C ABI.
Tolerance: relative max-norm per component <= 1e-12 (both sides propagate
with unitary steps in double precision; the step exponentials differ only
by rounding: Taylor series here, scipy's Pade form in the oracle)."""
import numpy as np
import pytest
import torch

from oracle import free_green as F
from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import relerr, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


def herm(r, d, s=1.0):
    a = r.normal(size=(d, d)) + 1j * r.normal(size=(d, d))
    return s * 0.5 * (a + a.conj().T)


def driven(r, g):
    """eps(t) = H0 + cos(1.3 t) H1 + 0.2 t H2 (entry 0: H0)."""
    H0, H1, H2 = herm(r, g.d), herm(r, g.d, 0.6), herm(r, g.d, 0.2)
    eps = np.zeros((g.nt + 2, g.d, g.d), np.complex128)
    eps[0] = H0
    for n in range(g.nt + 1):
        t = n * g.h
        eps[n + 1] = H0 + np.cos(1.3 * t) * H1 + 0.2 * t * H2
    return eps


def ogrid(O, g):
    return O.Grid(g.nt, g.ntau, g.d, g.sig, g.k, g.beta, g.h, g.mu)


def run_gpu(g, eps):
    G = K.Contour(g)
    K.green_from_H([G], [to_dev(eps)])
    K.sync()
    return G.numpy()


@pytest.mark.parametrize("d,sig,nt,k", [(1, -1, 70, 5), (2, -1, 70, 5), (2, 1, 45, 3), (3, -1, 33, 4),
                                        (4, -1, 70, 5), (8, -1, 40, 5), (4, -1, 5, 5), (2, -1, 1, 1)])
def test_free_green_matches_oracle(O, d, sig, nt, k):
    """Every component on grids whose steps span several chunks of 32 with a
    ragged last one (nt = 70, 45, 33, 40), the shortest grids (nt = k), d = 1..8,
    fermions and bosons (mu below the spectrum), k = 1..5."""
    require_gpu()
    say(f"free green d={d} sig={sig} nt={nt} k={k}")
    g = W.GridSpec(nt=nt, ntau=max(2 * k + 2, 24), d=d, sig=sig, k=k, beta=3.0, h=0.05,
                   mu=0.2 if sig < 0 else -6.0)
    r = W.rng(401, d, nt, k)
    eps = driven(r, g)
    got = run_gpu(g, eps)
    ref = F.green_from_H(ogrid(O, g), eps)
    for key in ("mat", "ret", "les", "tv"):
        e = relerr(got[key], getattr(ref, key))
        assert e < TOL, (key, e)


def test_free_green_full_size(O):
    """The bench workload's grid (nt = 1000, ntau = 400, d = 4) with a driven
    Hamiltonian: slices at the start, in the middle and at the end."""
    require_gpu()
    say("free green full size")
    g = W.GridSpec(nt=1000, ntau=400, d=4, sig=-1, k=5, beta=20.0, h=0.02, mu=0.0)
    eps = driven(W.rng(402), g)
    got = run_gpu(g, eps)
    slices = (0, 31, 32, 517, 999, 1000)
    ref = F.green_slices(ogrid(O, g), eps, slices)
    for n in slices:
        o = n * (n + 1) // 2
        rr, ll, tt = ref[n]
        assert relerr(got["ret"][o:o + n + 1], rr) < TOL, ("ret", n)
        assert relerr(got["les"][o:o + n + 1], ll) < TOL, ("les", n)
        assert relerr(got["tv"][n * (g.ntau + 1):(n + 1) * (g.ntau + 1)], tt) < TOL, ("tv", n)


def test_free_green_constant_hamiltonian_and_errors(O):
    """Constant eps: G^R(t_n, t_j) = -i exp(-i eps (t_n - t_j)) to rounding;
    and nt < k is refused before any launch."""
    require_gpu()
    say("free green constant H")
    g = W.GridSpec(nt=90, ntau=20, d=3, sig=-1, k=5, beta=2.0, h=0.04, mu=0.0)
    H = herm(W.rng(403), 3)
    eps = np.repeat(H[None], g.nt + 2, axis=0)
    got = run_gpu(g, eps)
    import scipy.linalg
    for n, j in ((90, 0), (57, 13), (5, 5)):
        ref = -1j * scipy.linalg.expm(-1j * H * (n - j) * g.h)
        assert np.abs(got["ret"][n * (n + 1) // 2 + j] - ref).max() < 1e-12
    bad = W.GridSpec(nt=3, ntau=20, d=2, sig=-1, k=5, beta=2.0, h=0.04, mu=0.0)
    with pytest.raises(RuntimeError):
        K.green_from_H([K.Contour(bad)], [to_dev(np.zeros((bad.nt + 2, 2, 2), np.complex128))])


def test_free_green_batch_of_problems(O):
    """One call for three problems sharing d, k and ntau, with different nt,
    beta, mu and Hamiltonians: each equals its own oracle result."""
    require_gpu()
    say("free green batch")
    grids = [W.GridSpec(nt=nt, ntau=30, d=3, sig=-1, k=4, beta=b, h=0.04, mu=mu)
             for nt, b, mu in ((50, 2.0, 0.1), (17, 5.0, -0.3), (33, 1.0, 0.0))]
    epss = [driven(W.rng(404, i), g) for i, g in enumerate(grids)]
    Gs = [K.Contour(g) for g in grids]
    K.green_from_H(Gs, [to_dev(e) for e in epss])
    K.sync()
    for g, e, G in zip(grids, epss, Gs):
        got = G.numpy()
        ref = F.green_from_H(ogrid(O, g), e)
        for key in ("mat", "ret", "les", "tv"):
            assert relerr(got[key], getattr(ref, key)) < TOL, (g.nt, key)

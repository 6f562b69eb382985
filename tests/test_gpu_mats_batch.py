"""The batched Matsubara solves (cntr_init_matsubara, cntr_vie2_matsubara with
count > 1: the operators of up to 256 problems inverted in one launch
sequence) give the one-problem results bit for bit, across a group boundary
(300 problems), and match the oracle's dense solve (Sec. "Dyson equation:
Matsubara", Eq. Gmat_dyson_integ) to 1e-10. Inputs: seeded hermitian levels
per problem and a seeded Matsubara self-energy of the right symmetry."""
import numpy as np
import pytest
import torch

from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import require_gpu, say

pytestmark = pytest.mark.gpu


def problems(count, d, ntau, seed):
    g = W.GridSpec(nt=4, ntau=ntau, d=d, sig=-1, k=2, beta=3.0, h=0.05, mu=0.0)
    r = W.rng(1916, seed)
    G, S, eps = [], [], []
    for _ in range(count):
        G.append(K.Contour(g, "cuda"))
        data = W.random_contour(r, g, 0.3, decay=0.2)
        S.append(K.Contour(g, "cuda", data=data))
        e = np.zeros((g.nt + 2, d, d), np.complex128)
        H = r.normal(size=(d, d)) + 1j * r.normal(size=(d, d))
        e[:] = 0.5 * (H + H.conj().T)
        eps.append(torch.as_tensor(e).to("cuda"))
    return g, G, S, eps


@pytest.mark.parametrize("d,ntau", [(1, 10), (2, 6)])
def test_batched_matsubara_is_the_single_solve(O, d, ntau):
    require_gpu()
    count = 300
    say(f"batched Matsubara count={count} d={d} ntau={ntau}")
    g, G, S, eps = problems(count, d, ntau, seed=d)
    K.init_matsubara(G, S, eps)
    G1 = [K.Contour(g, "cuda") for _ in range(count)]
    for i in range(count):
        K.init_matsubara([G1[i]], [S[i]], [eps[i]])
    K.sync()
    for i in range(count):
        assert torch.equal(G[i].mat, G1[i].mat), i
    # the oracle's dense solve on a few of them
    for i in (0, 255, 256, count - 1):
        ref = O.HM(O.Grid(g.nt, g.ntau, g.d, g.sig, g.k, g.beta, g.h, g.mu))
        Sh = O.HM(ref.g)
        Sh.mat[...] = S[i].mat.cpu().numpy()
        assert O.dyson_mat(ref, Sh, eps[i][0].cpu().numpy()) == 0
        got = G[i].mat.cpu().numpy()
        assert np.abs(got - ref.mat).max() <= 1e-10 * np.abs(ref.mat).max(), i
    # the integral form's Matsubara solve, F = Sigma, Q = G: batched vs single
    X = [K.Contour(g, "cuda") for _ in range(count)]
    X1 = [K.Contour(g, "cuda") for _ in range(count)]
    K.vie2_matsubara(X, S, G)
    for i in range(count):
        K.vie2_matsubara([X1[i]], [S[i]], [G[i]])
    K.sync()
    for i in range(count):
        assert torch.equal(X[i].mat, X1[i].mat), i

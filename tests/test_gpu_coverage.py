"""GPU parity over the rest of the accepted parameter space: orders k = 1..4
(Matsubara, start-up, time steps, convolution), bosons (start-up and time
steps), orbital counts d = 5, 6, 7, long d = 1 histories (several term
chunks), d = 8 at the adjoint workload's size, the batched k-point driver
over a few hundred slices, and the full-length second-Born chain of the
benchmark against the oracle's stored solution."""
import dataclasses
import os

import numpy as np
import pytest
import torch

from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import TOL, assert_slices, ora, rand_eps, relerr, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "chain_2b_nt1000.npz")


# ---------------------------------------------------------------- Matsubara
@pytest.mark.parametrize("k,sig", [(1, -1), (2, -1), (3, -1), (4, -1), (3, 1)])
def test_matsubara_orders(O, k, sig):
    require_gpu()
    say(f"matsubara k={k} sig={sig}")
    g = W.GridSpec(nt=6, ntau=50, d=2, sig=sig, beta=5.0, h=0.05, k=k, mu=-2.5 if sig > 0 else 0.1)
    r = W.rng(200, k, sig + 2)
    S = W.random_contour(r, g, 0.15)
    eps = rand_eps(r, g)
    Go = ora(O, g, None)
    O.dyson_mat(Go, ora(O, g, S), eps[0])
    Gd = K.Contour(g)
    K.init_matsubara([Gd], [K.Contour(g, data=S)], [to_dev(eps)])
    K.sync()
    assert relerr(Gd.mat.cpu().numpy(), Go.mat) < TOL


# ------------------------------------------------------------------ start-up
STARTUP = [(k, -1, d) for k in (1, 2, 3, 4) for d in (1, 2, 4)] + [(5, 1, d) for d in (1, 2, 4, 8)] + \
          [(5, -1, d) for d in (5, 6, 7)] + [(3, 1, 3)]


@pytest.mark.parametrize("k,sig,d", STARTUP)
def test_startup_orders_bosons_dims(O, k, sig, d):
    require_gpu()
    say(f"startup k={k} sig={sig} d={d}")
    g = W.GridSpec(nt=12, ntau=30, d=d, sig=sig, beta=3.0, h=0.04, k=k, mu=-2.0 if sig > 0 else 0.2)
    r = W.rng(201, k, sig + 2, d)
    S = W.random_contour(r, g, 0.3)
    G0 = W.random_contour(r, g, 0.5)  # Matsubara component taken as a given input
    eps = rand_eps(r, g)
    Go = ora(O, g, G0)
    assert O.dyson_start(Go, ora(O, g, S), eps) == 0
    Gd = K.Contour(g, data=G0)
    K.dyson_step(g.k, [Gd], [K.Contour(g, data=S)], [to_dev(eps)])
    K.sync()
    ref = {key: getattr(Go, key) for key in K.KEYS}
    assert_slices(g, Gd.numpy(), ref, range(0, g.k + 1), what=f"startup k={k} sig={sig} d={d}")


# -------------------------------------------------------------- time steps
STEPS = [(k, -1, d) for k in (1, 2, 3, 4) for d in (1, 2, 4)] + [(5, 1, d) for d in (1, 2, 3, 4, 8)] + \
        [(5, -1, d) for d in (5, 6, 7)] + [(2, 1, 8), (4, -1, 8)]


@pytest.mark.parametrize("k,sig,d", STEPS)
def test_timestep_orders_bosons_dims(O, k, sig, d):
    require_gpu()
    nt = 80 if d <= 4 else 70
    g = W.GridSpec(nt=nt, ntau=41, d=d, sig=sig, beta=4.0, h=0.03, k=k, mu=-2.0 if sig > 0 else -0.3)
    r = W.rng(202, k, sig + 2, d)
    G = W.random_contour(r, g, 0.4, decay=0.5)
    S = W.random_contour(r, g, 0.3, decay=0.5)
    eps = rand_eps(r, g)
    Sd, e = K.Contour(g, data=S), to_dev(eps)
    for n in sorted({k + 1, 2 * k, 2 * k + 1, 2 * k + 2, 33, 64, 65, nt}):
        say(f"timestep k={k} sig={sig} d={d} n={n}")
        Go = ora(O, g, G)
        assert O.dyson_timestep(n, Go, ora(O, g, S), eps, "B") == 0
        Gd = K.Contour(g, data=G)
        K.dyson_step(n, [Gd], [Sd], [e])
        K.sync()
        ref = {key: getattr(Go, key) for key in K.KEYS}
        assert_slices(g, Gd.numpy(), ref, [n], what=f"step k={k} sig={sig} d={d}")


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_convolution_orders(O, k):
    require_gpu()
    say(f"convolution k={k}")
    g = W.GridSpec(nt=24, ntau=30, d=2, beta=2.0, h=0.05, k=k)
    r = W.rng(203, k)
    A, Acc, B, Bcc = (W.random_contour(r, g, 0.5) for _ in range(4))
    f = rand_eps(r, g, 1.0)
    Co, Cd = ora(O, g, None), K.Contour(g)
    args_o = [ora(O, g, x) for x in (A, Acc, B, Bcc)]
    args_d = [[K.Contour(g, data=x)] for x in (A, Acc, B, Bcc)]
    slices = sorted({-1, 0, 1, k, k + 1, 2 * k, 2 * k + 1, 24})
    for n in slices:
        O.convolution_timestep(n, Co, *args_o, f)
        K.convolution(n, [Cd], *args_d, f=[to_dev(f)])
    K.sync()
    assert_slices(g, Cd.numpy(), {key: getattr(Co, key) for key in K.KEYS}, slices, what=f"convolution k={k}")


# ------------------------------------------------------- long histories
def _one_step_cases(O, g, seed, slices, what):
    r = W.rng(*seed)
    G = W.random_contour(r, g, 0.3, decay=0.2)
    S = W.random_contour(r, g, 0.3, decay=0.2)
    eps = rand_eps(r, g)
    Sd, e = K.Contour(g, data=S), to_dev(eps)
    Gd = K.Contour(g, data=G)
    for n in slices:
        say(f"{what} n={n}")
        Go = ora(O, g, G)
        assert O.dyson_timestep(n, Go, ora(O, g, S), eps, "B") == 0
        K.dyson_step(n, [Gd], [Sd], [e])
        K.sync()
        ref = {key: getattr(Go, key) for key in K.KEYS}
        assert_slices(g, Gd.numpy(), ref, [n], what=what)
        Gd = K.Contour(g, data=G)


def test_timestep_d1_long_history(O):
    """d = 1 at the k-point workload's sizes (ntau = 500, nt = 2000): one,
    two and eight term chunks of 256, the last ragged."""
    require_gpu()
    g = W.GridSpec(nt=2000, ntau=500, d=1, beta=10.0, h=0.02, k=5)
    _one_step_cases(O, g, (204,), (257, 512, 1999, 2000), "d=1 long step")


def test_timestep_d8_adjoint_workload_size(O):
    """d = 8 at the eight-site ring's sizes (ntau = 400, nt = 1500)."""
    require_gpu()
    g = W.GridSpec(nt=1500, ntau=400, d=8, beta=10.0, h=0.02, k=5)
    _one_step_cases(O, g, (205,), (1499, 1500), "d=8 long step")


def test_kpoint_batch_several_hundred_slices(O):
    """The batched k-point driver (local Sigma = 0.25 G_loc, the field pulse)
    over 280 slices with ntau = 500: two term chunks of the d = 1 history
    sums, and 34 problems, so that the tau source of the shared Sigma is one
    operator product with a ragged problem tile. Against the oracle's driver
    with the same 34 k-points and iteration counts."""
    require_gpu()
    g = W.GridSpec(nt=280, ntau=500, d=1, beta=10.0, h=0.02, k=5)
    eps = list(W.kpoint_band(g, 34))
    say("k-point batch, 34 x 280 slices: oracle")
    Go, So = [ora(O, g, None) for _ in eps], ora(O, g, None)
    O.solve_local(Go, So, eps, 0.25, mats_iters=8, boot_iters=8, ncorr=5)
    say("k-point batch: gpu")
    Gd, Sd = [K.Contour(g) for _ in eps], K.Contour(g)
    K.solve_local(Gd, Sd, [to_dev(e) for e in eps], 0.25, mats_iters=8, boot_iters=8, ncorr=5)
    K.sync()
    for i in (0, 7, 16, 33):
        got = Gd[i].numpy()
        for key in K.KEYS:
            e = relerr(got[key], getattr(Go[i], key))
            assert e < TOL, (i, key, e)
    got = Sd.numpy()
    for key in K.KEYS:
        assert relerr(got[key], getattr(So, key)) < TOL, ("Sigma", key)


# ------------------------------------------- the benchmark's full solve
def test_full_chain_2b_against_oracle_solution(O):
    """The benchmark workload end to end (4-site chain, second-Born + Hartree,
    U ramp, nt = 1000, ntau = 400, 5 correctors) against the oracle's solution
    stored by tests/golden/make_chain_2b_golden.py: every tau point of G^M,
    whole slices 6, 500 and 1000, and the density n_i(t) at every time (which
    also pins the O(h^k) departure from half filling that the discrete scheme
    and the oracle share)."""
    require_gpu()
    ref = np.load(GOLDEN)
    g = W.GridSpec(nt=1000, ntau=400, d=4, sig=-1, k=5, beta=20.0, h=0.02, mu=0.0)
    e0, U = W.hubbard_ramp(g)
    say("full chain 2B solve")
    G, S, Gs = K.Contour(g), K.Contour(g), K.Contour(g)
    e0d, Ud = to_dev(e0), to_dev(U)
    emf = torch.zeros_like(e0d)
    st = K.solve_2b(G, S, Gs, e0d, Ud, emf, ncorr=5, mats_tol=1e-14, mats_mix=0.5, boot_tol=1e-14)
    K.sync()
    say(f"gpu stats {st}; oracle stats {ref['stats']}")
    assert st.mats_iter == int(ref["stats"][0]) and st.boot_iter == int(ref["stats"][1])
    assert relerr(G.mat.cpu().numpy(), ref["mat"]) < TOL
    got = G.numpy()
    for n in (6, 500, 1000):
        o = n * (n + 1) // 2
        for key, sl in (("ret", slice(o, o + n + 1)), ("les", slice(o, o + n + 1)),
                        ("tv", slice(n * (g.ntau + 1), (n + 1) * (g.ntau + 1)))):
            e = relerr(got[key][sl], ref[f"{key}_{n}"])
            assert e < TOL, (n, key, e)
    les = got["les"]
    dens = np.array([les[n * (n + 1) // 2 + n].diagonal().imag for n in range(g.nt + 1)])
    assert np.abs(dens - ref["dens"]).max() < TOL * np.abs(ref["dens"]).max()
    emf_d = np.array([x.diagonal().real for x in emf.cpu().numpy()])
    assert np.abs(emf_d - ref["emf_diag"]).max() < TOL * max(1.0, np.abs(ref["emf_diag"]).max())
    # the departure from half filling at t_nt is the scheme's own (both sides)
    say(f"max |n_i - 1/2| at t_nt: gpu {np.abs(dens[-1] - 0.5).max():.6e}, "
        f"oracle {np.abs(ref['dens'][-1] - 0.5).max():.6e}")

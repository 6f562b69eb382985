"""Step sequences captured into a HIP graph (cntr_graph_begin / end / launch)
and replayed: every replay, with eager work and synchronizations between the
replays, must reproduce the eager result bit for bit. Covers the plain
two-level solve (start-up and 95 steps), a k-point batch with the local
self-energy (batch descriptors written by kernels, the shared-Sigma tau
source), the allocation-free step, and the calls that must be refused during
capture."""
import numpy as np
import pytest
import torch

from paper_1911_01211_amd import _abi
from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def _equal(a, b, what):
    for key in K.KEYS:
        assert torch.equal(getattr(a, key), getattr(b, key)), (what, key)


def _clear_real_time(G):
    G.ret.zero_()
    G.les.zero_()
    G.tv.zero_()


def test_graph_of_the_plain_solve():
    require_gpu()
    say("graph: two-level solve, nt = 100")
    g = W.GridSpec(nt=100, ntau=100, d=2, beta=5.0, h=0.05, k=5)
    eps, S, _ = W.two_level_embedding(g)
    Sd, e = K.Contour(g, data=S), to_dev(eps)
    side = torch.cuda.Stream()
    G = K.Contour(g)
    K.init_matsubara([G], [Sd], [e])
    torch.cuda.synchronize()
    for n in range(g.k, g.nt + 1):  # eager on the capture stream (sizes its scratch)
        K.dyson_step(n, [G], [Sd], [e], stream=side)
    side.synchronize()
    ref = K.Contour(g, data=G.numpy())
    torch.cuda.synchronize()
    with K.Graph(side) as gr:
        for n in range(g.k, g.nt + 1):
            K.dyson_step(n, [G], [Sd], [e], stream=side)
    torch.cuda.synchronize()
    other = K.Contour(g, data=W.random_contour(W.rng(660), g, 0.3))
    for rep in range(3):
        _clear_real_time(G)
        torch.cuda.synchronize()
        gr.launch(side)
        side.synchronize()
        _equal(G, ref, f"replay {rep}")
        K.dyson_step(20, [other], [Sd], [e])  # eager work between the replays
        K.sync()


def test_graph_of_a_kpoint_batch_and_noalloc_steps():
    require_gpu()
    say("graph: 34 k-points with the local Sigma, and allocation-free steps")
    g = W.GridSpec(nt=30, ntau=60, d=1, beta=10.0, h=0.02, k=5)
    eps = [to_dev(x) for x in W.kpoint_band(g, 34)]
    G = [K.Contour(g) for _ in eps]
    S = K.Contour(g)
    K.solve_local(G, S, eps, 0.25, mats_iters=4, boot_iters=4, ncorr=1, nt_stop=g.k)
    init = [{key: getattr(x, key).clone() for key in K.KEYS} for x in G]
    s_init = {key: getattr(S, key).clone() for key in K.KEYS}

    def restore():
        for x, d in zip(G, init):
            for key in K.KEYS:
                getattr(x, key).copy_(d[key])
        for key in K.KEYS:
            getattr(S, key).copy_(s_init[key])

    def sequence(B, stream):
        for n in range(g.k + 1, g.nt + 1):
            B.extrapolate(n - 1, stream)
            for _ in range(2):
                B.sigma_local(n, 0.25, stream)
                B.step(n, stream)
            B.sigma_local(n, 0.25, stream)
        # allocation-free steps of a three-problem sub-batch on the last slice
        K.dyson_step_noalloc(g.nt, G[:3], [S] * 3, eps[:3], stream=stream)

    B = K.Batch(G, [S] * len(G), eps)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    sequence(B, side)  # eager on the capture stream (sizes its scratch)
    side.synchronize()
    ref = [{key: getattr(x, key).clone() for key in K.KEYS} for x in G]
    restore()
    torch.cuda.synchronize()
    with K.Graph(side) as gr:
        sequence(B, side)
    for rep in range(3):
        restore()
        torch.cuda.synchronize()
        gr.launch(side)
        side.synchronize()
        for i, (x, d) in enumerate(zip(G, ref)):
            for key in K.KEYS:
                assert torch.equal(getattr(x, key), d[key]), (rep, i, key)
        torch.ones(1 << 20, device="cuda").sum().item()  # eager work between the replays
        K.sync()


def test_synchronizing_calls_are_refused_during_capture():
    require_gpu()
    g = W.GridSpec(nt=12, ntau=20, d=2, beta=5.0, h=0.05, k=5)
    eps, S, _ = W.two_level_embedding(g)
    G, Sd, e = K.Contour(g), K.Contour(g, data=S), to_dev(eps)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with pytest.raises(_abi.CntrError) as ex:
        with K.Graph(side):
            K.init_matsubara([G], [Sd], [e], stream=side)
    assert ex.value.code == -1
    with pytest.raises(_abi.CntrError):
        K.Graph(torch.cuda.default_stream()).__enter__()

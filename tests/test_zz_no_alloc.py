"""The allocation-free time step (cntr_dyson_step_noalloc, static device
scratch) against cntr_dyson_step through the C ABI: two calls in a row on
the same GPU, the second with a smaller input, plus a batch and the
start-up; results must be identical (the same kernels), and inputs that need
more scratch than the static array holds are rejected on the host."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1911_01211_amd import _abi
from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import rand_eps, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def _noalloc():
    return _abi.lib().cntr_dyson_step_noalloc


def _call(f, tstp, G, S, eps):
    rc = f(tstp, len(G), K._grids(G), K._gfs(G), K._gfs(S), K._ptrs(eps), K._stream())
    _abi.check(rc)


def _case(seed, d, nt, ntau, count=1):
    grids = [W.GridSpec(nt=nt - (i % 3), ntau=ntau, d=d, beta=3.0, h=0.04, k=5, mu=0.1) for i in range(count)]
    r = W.rng(600, seed)
    data = [(W.random_contour(r, g, 0.4, decay=0.3), W.random_contour(r, g, 0.3, decay=0.3), rand_eps(r, g))
            for g in grids]
    return grids, data


def _compare(f, grids, data, n):
    Ga = [K.Contour(g, data=x[0]) for g, x in zip(grids, data)]
    Gb = [K.Contour(g, data=x[0]) for g, x in zip(grids, data)]
    S = [K.Contour(g, data=x[1]) for g, x in zip(grids, data)]
    e = [to_dev(x[2]) for x in data]
    K.dyson_step(n, Ga, S, e)
    _call(f, n, Gb, S, e)
    K.sync()
    for a, b in zip(Ga, Gb):
        for key in K.KEYS:
            assert torch.equal(getattr(a, key), getattr(b, key)), (n, key)


def test_noalloc_step_matches_allocating_step():
    require_gpu()
    f = _noalloc()
    big = _case(1, 4, 300, 60)
    small = _case(2, 4, 90, 40)
    say("noalloc: step n=300 d=4, then n=70 d=4 (smaller)")
    _compare(f, *big, 300)
    _compare(f, *small, 70)
    say("noalloc: start-up and step, batch of 5 (d = 2)")
    batch = _case(3, 2, 40, 30, count=5)
    _compare(f, *batch, 5)
    _compare(f, *batch, 38)
    say("noalloc: d = 1 batch of 34 sharing one Sigma (tau source as one product)")
    grids = [W.GridSpec(nt=30, ntau=50, d=1, beta=3.0, h=0.04, k=5) for _ in range(34)]
    r = W.rng(601)
    S1 = W.random_contour(r, grids[0], 0.3, decay=0.3)
    G0 = [W.random_contour(r, g, 0.4, decay=0.3) for g in grids]
    Sd = K.Contour(grids[0], data=S1)
    e = [to_dev(rand_eps(r, g)) for g in grids]
    Ga = [K.Contour(g, data=x) for g, x in zip(grids, G0)]
    Gb = [K.Contour(g, data=x) for g, x in zip(grids, G0)]
    K.dyson_step(25, Ga, [Sd] * 34, e)
    _call(f, 25, Gb, [Sd] * 34, e)
    K.sync()
    for a, b in zip(Ga, Gb):
        for key in K.KEYS:
            assert torch.equal(getattr(a, key), getattr(b, key)), key


def test_noalloc_rejects_oversized_input():
    require_gpu()
    f = _noalloc()
    g = W.GridSpec(nt=3000, ntau=300, d=8, beta=3.0, h=0.04, k=5)
    grid = (_abi.Grid * 1)(K.grid_c(g))
    gf = (_abi.GF * 1)(_abi.GF(1, 1, 1, 1))
    eps = (C.c_void_p * 1)(1)
    rc = f(3000, 1, grid, gf, gf, eps, None)
    assert rc == -7, rc
    assert "static array" in _abi.lib().cntr_last_error().decode()

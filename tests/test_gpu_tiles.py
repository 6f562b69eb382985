"""Autotuned term chunks (cntr_set_tiles): every candidate chunk of the
tunable paths gives the oracle's time step, and a table of bands drives a
batched run whose every slice matches the oracle; invalid tables are
refused."""
import numpy as np
import pytest

from paper_1911_01211_amd import autotune as AT
from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import TOL, assert_slices, ora, rand_eps, relerr, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,tj", [(1, 32), (1, 64), (1, 128), (8, 16), (8, 32)])
def test_every_chunk_matches_oracle(O, d, tj):
    require_gpu()
    g = W.GridSpec(nt=300 if d == 1 else 140, ntau=60 if d == 1 else 30, d=d, beta=4.0, h=0.03, k=5, mu=-0.3)
    r = W.rng(210, d, tj)
    G = W.random_contour(r, g, 0.4, decay=0.3)
    S = W.random_contour(r, g, 0.3, decay=0.3)
    eps = rand_eps(r, g)
    Sd, e = K.Contour(g, data=S), to_dev(eps)
    try:
        AT.set_tiles(d, [1 << 30], [tj])
        for n in (11, 12, 70, g.nt):
            say(f"tiles d={d} chunk={tj} n={n}")
            Go = ora(O, g, G)
            assert O.dyson_timestep(n, Go, ora(O, g, S), eps, "B") == 0
            Gd = K.Contour(g, data=G)
            K.dyson_step(n, [Gd], [Sd], [e])
            K.sync()
            assert_slices(g, Gd.numpy(), {key: getattr(Go, key) for key in K.KEYS}, [n], what=f"d={d} tj={tj}")
    finally:
        AT.set_tiles(d, [], [])


def test_banded_table_in_a_kpoint_run(O):
    """Chunk 32 up to slice 20, 64 up to 40, 128 after: the k-point driver
    over 60 slices against the oracle's."""
    require_gpu()
    g = W.GridSpec(nt=60, ntau=40, d=1, beta=10.0, h=0.02, k=5)
    eps = list(W.kpoint_band(g, 12))
    Go, So = [ora(O, g, None) for _ in eps], ora(O, g, None)
    O.solve_local(Go, So, eps, 0.25, mats_iters=6, boot_iters=6, ncorr=3)
    try:
        AT.set_tiles(1, [20, 40, 1 << 30], [32, 64, 128])
        Gd, Sd = [K.Contour(g) for _ in eps], K.Contour(g)
        K.solve_local(Gd, Sd, [to_dev(x) for x in eps], 0.25, mats_iters=6, boot_iters=6, ncorr=3)
        K.sync()
    finally:
        AT.set_tiles(1, [], [])
    for i in (0, 5, 11):
        got = Gd[i].numpy()
        for key in K.KEYS:
            assert relerr(got[key], getattr(Go[i], key)) < TOL, (i, key)


def test_invalid_tables_are_refused():
    require_gpu()
    from paper_1911_01211_amd import _abi
    for d, n_hi, tj in ((4, [100], [32]), (1, [100], [48]), (8, [100], [128]), (1, [100, 50], [64, 64])):
        with pytest.raises(_abi.CntrError):
            AT.set_tiles(d, n_hi, tj)

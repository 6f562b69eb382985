"""Host-side logic without a GPU: the wave plan of an uneven batch and the
seeded uneven-batch generator (stored inputs reproduce it)."""
import os

import numpy as np
import pytest

from paper_1911_01211_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_plan_waves_first_fit():
    pytest.importorskip("torch")
    from paper_1911_01211_amd import contour as K
    foot = [5.0, 3.0, 7.0, 2.0, 2.0, 6.0]
    waves = K.plan_waves(foot, 10.0)
    assert sorted(i for w in waves for i in w) == list(range(len(foot)))
    for w in waves:
        assert sum(foot[i] for i in w) <= 10.0
    # decreasing first fit: 7+3, 6+2+2, 5
    assert sorted(map(tuple, waves)) == sorted([(1, 2), (3, 4, 5), (0,)])
    with pytest.raises(ValueError):
        K.plan_waves([11.0], 10.0)


def test_uneven_batch_file_matches_generator():
    P = W.load_uneven(os.path.join(ROOT, "paper_1911_01211_amd", "data", "uneven_batch_384.npz"))
    assert len(P) == 384
    for p in (0, 1, 5, 100, 383):
        d, nt, U, H = W.uneven_problem(p)
        assert (d, nt) == P[p][:2] and U == P[p][2]
        assert np.array_equal(H, P[p][3])
        assert d in (1, 2, 4, 8) and 400 <= nt <= 3000 and 0.5 <= U <= 2.0
        w = np.linalg.eigvalsh(H)
        assert np.allclose(H, H.conj().T) and w.min() >= -2.0 and w.max() <= 2.0

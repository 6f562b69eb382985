"""Writes uneven_batch_384.npz: the 384 seeded problems of the uneven
second-Born batch (orbital count d in {1, 2, 4, 8}, nt in [400, 3000], U in
[0.5, 2], random hermitian H with spectrum in [-2, 2]; beta = 10, ntau = 300,
h = 0.02 for all), from workloads.uneven_problem. Arrays: d, nt, U [384] and
H [384, 8, 8] (the leading d x d block used). Run from the repository root:
    python paper_1911_01211_amd/data/make_uneven_batch.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_1911_01211_amd import workloads as W  # noqa: E402

COUNT = 384


def main():
    d = np.zeros(COUNT, np.int32)
    nt = np.zeros(COUNT, np.int32)
    U = np.zeros(COUNT)
    H = np.zeros((COUNT, 8, 8), np.complex128)
    for p in range(COUNT):
        dp, ntp, Up, Hp = W.uneven_problem(p)
        d[p], nt[p], U[p] = dp, ntp, Up
        H[p, :dp, :dp] = Hp
    out = os.path.join(HERE, "uneven_batch_384.npz")
    np.savez(out, d=d, nt=nt, U=U, H=H)
    print("wrote", out, "d counts", {k: int((d == k).sum()) for k in (1, 2, 4, 8)})


if __name__ == "__main__":
    main()

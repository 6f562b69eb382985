"""Writes tests/golden/chain_2b_nt1000.npz: the oracle's self-consistent
second-Born + Hartree solution of the 4-site Hubbard chain at full size
(U ramp 2 -> 1 on [0, 5], beta = 20, ntau = 400, nt = 1000, h = 0.02, k = 5,
5 corrector iterations per slice, Matsubara and bootstrap loops to 1e-14;
Sec. "Hubbard chain"), sampled for the full-length GPU parity test:

  mat                  G^M (every tau point)
  ret_n, les_n, tv_n   slice n (row R_{n,.}, column L_{.,n}, row T_{n,.}) for n in SLICES
  dens                 n_i(t_n) = Im L_{n,n}[i,i], every n = 0..nt
  emf_diag             diagonal of the Hartree levels eps_mf, entries n = -1..nt
  stats                Matsubara and bootstrap iterations, last errors

Only the oracle and the seeded workload inputs are used. Run from the
repository root:  python tests/golden/make_chain_2b_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1911_01211_amd import workloads as W  # noqa: E402

SLICES = (6, 500, 1000)
OUT = os.path.join(ROOT, "tests", "golden", "chain_2b_nt1000.npz")


def main():
    g = W.GridSpec(nt=1000, ntau=400, d=4, sig=-1, k=5, beta=20.0, h=0.02, mu=0.0)
    e0, U = W.hubbard_ramp(g)
    og = O.Grid(g.nt, g.ntau, g.d, g.sig, g.k, g.beta, g.h, g.mu)
    G, S = O.HM(og), O.HM(og)
    rc, emf, st = O.solve_2b(G, S, e0, U, ncorr=5, mats_tol=1e-14, mats_mix=0.5, boot_tol=1e-14)
    assert rc == 0, rc
    out = dict(mat=G.mat,
               dens=np.array([G.L(n, n).diagonal().imag for n in range(g.nt + 1)]),
               emf_diag=np.array([emf[n].diagonal().real for n in range(g.nt + 2)]),
               stats=np.array([st["mats_iter"], st["boot_iter"], st["mats_err"], st["boot_err"]]))
    for n in SLICES:
        out[f"ret_{n}"] = G.ret_row(n).copy()
        out[f"les_{n}"] = G.les_col(n).copy()
        out[f"tv_{n}"] = G.tv_row(n).copy()
    np.savez(OUT, **out)
    print("wrote", OUT, st, flush=True)


if __name__ == "__main__":
    main()

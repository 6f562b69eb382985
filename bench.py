"""Benchmark: self-consistent second-Born Kadanoff-Baym propagation on one GPU.

Workload (one bench step = the whole hot path once): 4-site open Hubbard
chain at half filling, spin-symmetric second-Born self-energy + Hartree mean
field, U ramped linearly 2 -> 1 over t in [0, 5], beta = 20, ntau = 400,
nt = 1000, h = 0.02, k = 5, complex128. A step is the Matsubara
self-consistency (with the dense Matsubara solve), the bootstrap of slices
0..k, and the predictor-corrector time steps k+1..nt (ncorr corrector
iterations each), all on the device through the C ABI (cntr_solve_2b).

value = Dyson time steps (slices n > k) completed per second of wall time,
including every corrector iteration. The JSON line also carries the FP64
rate, the roofline fraction of the history-sum kernel (HIP events on its
launch stream around every 8th time step of the timed region, so that the
events add little to the timed work) and the oracle timed on the host cores
as a CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dyson time-steps/s + FP64 TFLOP/s, batched/adjoint vs plain at <=1e-10 rel err"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # FP64 vector (and dense FP64 MFMA) peak of MI355X

# HBM traffic of one history-kernel launch at slice n = 1000, from the
# FETCH_SIZE / WRITE_SIZE counter runs of `bench.py --profile-step 1000`
# (scaled by the counts of a 1 GiB device copy: FETCH x 2.0, WRITE x 1.0).
# Valid only for the kernel sources it was taken on (hash below); reported
# as null once they change.
PROF_EVERY = 8  # time steps per recorded one (HIP events)
TRAFFIC = {"slice": 1000, "bytes": 3.9809e8, "algorithmic_bytes": 3.5891e8,
           "src_sha256_16": "cdd6d266151dfea9",
           "profile": "profiles/k_history_traffic_slice1000_d4.md"}
TRAFFIC_SRCS = ("paper_1911_01211_amd/csrc/step.hip", "paper_1911_01211_amd/csrc/dev_common.h",
                "paper_1911_01211_amd/csrc/cntr_internal.h")


def traffic_entry():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SRCS:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != TRAFFIC["src_sha256_16"]:
        return None, None
    return TRAFFIC["bytes"], {k: TRAFFIC[k] for k in ("slice", "algorithmic_bytes", "profile")}


def workload_grid():
    from paper_1911_01211_amd import workloads as W
    return W.GridSpec(nt=1000, ntau=400, d=4, sig=-1, k=5, beta=20.0, h=0.02, mu=0.0)


def run_gpu(args):
    import torch

    from paper_1911_01211_amd import contour as K
    from paper_1911_01211_amd import workloads as W

    g = workload_grid()
    e0np, Unp = W.hubbard_ramp(g)
    dev = "cuda:0"
    G, S, Gs = K.Contour(g, dev), K.Contour(g, dev), K.Contour(g, dev)
    e0 = torch.as_tensor(e0np).to(dev)
    U = torch.as_tensor(Unp).to(dev)
    emf = torch.zeros_like(e0)

    def one_step():
        G.zero_()
        S.zero_()
        return K.solve_2b(G, S, Gs, e0, U, emf, ncorr=args.ncorr, mats_tol=1e-14, mats_mix=0.5,
                          boot_tol=1e-14)

    stats = None
    for w in range(args.warmup):
        stats = one_step()
        torch.cuda.synchronize()
        print(f"# warmup {w} done: {stats}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    K.profile_begin(PROF_EVERY)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats = one_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = K.profile_end()
    elapsed = t1 - t0
    # physical sanity of the last run: half filling on every site at t_nt
    L = G.les[-1].cpu().numpy()
    dens_dev = float(abs((L.diagonal().imag) - 0.5).max())
    # one slice at n = nt on the converged state: ncorr x (Sigma_2B + step)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.ncorr):
        K.sigma_2b(g.nt, [G], [U], [S], eps0=[e0], eps_mf=[emf], nbar=0.5)
        K.dyson_step(g.nt, [G], [S], [emf])
    ev1.record()
    torch.cuda.synchronize()
    state = dict(G=G, S=S, emf=emf, e0=e0np, U=U, last_slice_ms=ev0.elapsed_time(ev1))
    return g, elapsed, prof, stats, dens_dev, state


def run_adjoint(args):
    """Adjoint workload: 8-site Hubbard ring with a Peierls phase e^{iA(t)} on
    the hopping, second-Born + Hartree, U = 1.5, beta = 10, ntau = 400,
    nt = 1500, h = 0.02, k = 5; A_1..A_1500 seeded samples. J = E_kin(t_nt)
    and its gradient with respect to all 1500 samples A_n and U through
    DysonKineticEnergy (forward: cntr_solve_2b; backward: the second-Born
    adjoint sweep, Matsubara solve included). Checked against central
    differences of the same GPU forward solve (steps 4e-3 and 2e-3 over the
    direction's largest entry, Richardson-combined: smaller steps would
    resolve the forward's own rounding and iteration-stop noise, about 1e-11
    in J) along seeded directions in (A, U)."""
    import numpy as np
    import torch

    from paper_1911_01211_amd import autograd as AG
    from paper_1911_01211_amd import workloads as W

    dev = "cuda:0"
    g = W.GridSpec(nt=args.adj_nt, ntau=400, d=8, sig=-1, k=5, beta=10.0, h=0.02, mu=0.0)
    T, Phi = W.ring_peierls(g, 8)
    A = W.ring_drive(g)
    U0 = 1.5
    m = AG.RingModel(g=g, T=torch.as_tensor(T).to(dev), Phi=torch.as_tensor(Phi).to(dev), ncorr=args.adj_ncorr,
                     niter=args.adj_niter)
    At = torch.tensor(A, dtype=torch.float64, device=dev, requires_grad=True)
    Ut = torch.tensor(U0, dtype=torch.float64, device=dev, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = AG.kinetic_energy(At, Ut.expand(g.nt + 2), m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"# adjoint ring: forward {t1 - t0:.2f}s backward {t2 - t1:.2f}s", file=sys.stderr, flush=True)
    gA, gU = At.grad.cpu().numpy(), float(Ut.grad)
    fd = []
    r = W.rng(191, 5)
    for q in range(args.adj_fd):
        vA, vU = r.normal(size=g.nt), float(r.normal())
        big = max(float(np.abs(vA).max()), abs(vU))
        diffs = []
        for t in (4e-3 / big, 2e-3 / big):  # Richardson over two steps removes the O(t^2) term
            Jpm = []
            for sgn in (1.0, -1.0):
                with torch.no_grad():
                    Ap = torch.tensor(A + sgn * t * vA, dtype=torch.float64, device=dev)
                    Up = torch.full((g.nt + 2,), U0 + sgn * t * vU, dtype=torch.float64, device=dev)
                    Jpm.append(float(AG.kinetic_energy(Ap, Up, m)))
            diffs.append((Jpm[0] - Jpm[1]) / (2 * t))
        ref = (4 * diffs[1] - diffs[0]) / 3
        got = float(np.dot(gA, vA) + gU * vU)
        fd.append({"direction": q, "adjoint": got, "central_difference": diffs, "richardson": ref,
                   "rel_err": abs(got - ref) / max(abs(ref), 1e-300)})
        print(f"# adjoint ring: direction {q} rel err {fd[-1]['rel_err']:.2e} (raw differences {diffs})",
              file=sys.stderr, flush=True)
    nsl = g.nt - g.k
    # FP64 work of the backward's dominant reductions (the Sigma-bar sums of
    # every reverse step: d x d block products, 8 d^3 flops each; counted
    # from the kernels' term ranges) against the whole backward wall time
    sig_flops = (args.adj_niter + 1) * 8.0 * g.d ** 3 * sum(adj_sigma_products(n, g.k, g.ntau)
                                                           for n in range(g.k + 1, g.nt + 1))
    out_roof = {"bound": "fp64", "scope": "Sigma-bar block products / whole backward wall time",
                "achieved": sig_flops / (t2 - t1) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                "frac": sig_flops / (t2 - t1) / 1e12 / 78.6, "flops": sig_flops}
    return {"roofline": out_roof,
            "workload": f"8-site Hubbard ring, Peierls phase e^(iA(t)) on the hopping, second-Born + Hartree, "
                        f"U=1.5, beta=10, ntau=400, nt={g.nt}, h=0.02, k=5; gradient of E_kin(t_nt) w.r.t. the "
                        f"{g.nt} samples A_n and U (torch.autograd.Function over the adjoint sweep)",
            "value": nsl / (t2 - t1), "unit": "adjoint time-steps/s",
            "forward_s": t1 - t0, "backward_s": t2 - t1, "backward_over_forward": (t2 - t1) / (t1 - t0),
            "J": float(J.detach()), "dJ_dU": gU, "max_abs_dJ_dA": float(np.abs(gA).max()),
            "fixed_point_iterations": args.adj_niter, "forward_corrector_iterations": args.adj_ncorr,
            "fixed_point_last_change": m.stats.get("adjoint_last_change"),
            "fd_check": fd}


def run_mats_fourier(state):
    """Fourier-series Matsubara solve (cntr_matsubara_fourier, oversampling 10)
    on the chain's converged Sigma^M and Hartree levels, against one exact
    solve of the same discrete equation (cntr_init_matsubara, dense inverse
    and refinement to 1e-14): time per call and the deviation of the Fourier
    G^M from the exact one."""
    import numpy as np
    import torch

    from paper_1911_01211_amd import contour as K

    G, S, emf = state["G"], state["S"], state["emf"]
    g = G.g
    Gf, Gx = K.Contour(g, "cuda:0"), K.Contour(g, "cuda:0")
    times = {}
    for name, fn in (("fourier", lambda: K.matsubara_fourier([Gf], [S], [emf], 10)),
                     ("exact", lambda: K.init_matsubara([Gx], [S], [emf]))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / 3 * 1e3
    dev = (Gf.mat - Gx.mat).abs()
    return {"workload": "Matsubara equation of the converged 2B chain (d=4, ntau=400, beta=20); "
                        "Fourier-series solve with 8000 frequencies against the exact discrete solve",
            "value": 1e3 / times["fourier"], "unit": "solves/s",
            "ms_per_solve": times, "speedup_vs_exact": times["exact"] / times["fourier"],
            "max_abs_deviation": float(dev.max()), "mean_abs_deviation": float(dev.mean()),
            "max_abs_GM": float(Gx.mat.abs().max())}


def run_vie2(state):
    """Dyson equation in integral form (cntr_vie2_matsubara, cntr_vie2_step) on
    the chain's grid: Q = G_0 (free function of the converged mean-field
    levels), F = -G_0 * Sigma, Fcc = -Sigma * G_0 (Sigma the converged 2B
    self-energy, held fixed; built with cntr_green_from_H and cntr_convolution
    before the timed region). Timed with HIP events on the launch stream: the
    whole solve (Matsubara, start-up, 995 steps) and the steps alone; beside
    it the integro-differential solve of the same equation (fixed Sigma) and
    the largest deviation of the two solutions. `achieved` counts the history
    bytes of the steps (each stored block of G and of F's row once per step)
    over the step phase."""
    import torch

    from paper_1911_01211_amd import contour as K

    G, S, emf = state["G"], state["S"], state["emf"]
    g = G.g
    dev = "cuda:0"
    G0, F, Fcc, Gv, Gd = (K.Contour(g, dev) for _ in range(5))
    K.green_from_H([G0], [emf])

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # the inputs: 2 x (nt + 2) convolution calls (cntr_convolution), timed
    c0, c1 = ev(), ev()
    torch.cuda.synchronize()
    c0.record()
    for n in range(-1, g.nt + 1):
        K.convolution(n, [F], [G0], [G0], [S], [S])
        K.convolution(n, [Fcc], [S], [S], [G0], [G0])
    c1.record()
    torch.cuda.synchronize()
    conv_ms = c0.elapsed_time(c1)
    for X in (F, Fcc):
        for key in K.KEYS:
            getattr(X, key).neg_()
    torch.cuda.synchronize()

    # warm-up, then the timed solves
    K.solve_vie2([Gv], [F], [Fcc], [G0])
    K.sync()
    reps, whole, steps = 2, [], []
    V = K.Vie2Batch([Gv], [F], [Fcc], [G0])
    for _ in range(reps):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record()
        V.matsubara()
        V.step(g.k)
        e1.record()
        for n in range(g.k + 1, g.nt + 1):
            V.step(n)
        e2.record()
        torch.cuda.synchronize()
        whole.append(e0.elapsed_time(e2))
        steps.append(e1.elapsed_time(e2))
    K.sync()
    # the integro-differential form of the same equation
    B = K.Batch([Gd], [S], [emf])
    d0, d1, d2 = ev(), ev(), ev()
    d0.record()
    B.init_matsubara()
    B.step(g.k)
    d1.record()
    for n in range(g.k + 1, g.nt + 1):
        B.step(n)
    d2.record()
    torch.cuda.synchronize()
    K.sync()
    dev_max = max(float((getattr(Gv, key) - getattr(Gd, key)).abs().max()) for key in K.KEYS)
    ref = max(float(getattr(Gd, key).abs().max()) for key in K.KEYS)
    nsteps = g.nt - g.k
    st_ms = min(steps)
    dd = g.d * g.d
    nbytes = 0.0
    for n in range(g.k + 1, g.nt + 1):
        blocks = n * (n + 1) / 2 + n * (g.ntau + 1) + (n * (n + 1) / 2 if n >= 2 * g.k + 1 else 0)
        nbytes += 16.0 * dd * blocks
    gbs = nbytes / (st_ms * 1e-3) / 1e9
    # convolution bytes: per slice n the blocks of the factors' histories that
    # the three components read (B^R and A^R, A^< triangles, A^rceil and
    # B^rceil panels), each once
    cbytes = 0.0
    for n in range(0, g.nt + 1):
        cbytes += 16.0 * dd * (3 * n * (n + 1) / 2 + 2 * (n + 1) * (g.ntau + 1))
    cbytes *= 2
    conv = {"calls": 2 * (g.nt + 2), "ms_per_call": conv_ms / (2 * (g.nt + 2)),
            "roofline": {"bound": "hbm", "achieved": cbytes / (conv_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": cbytes / (conv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes": cbytes}}
    return {"workload": "Dyson equation of the converged 2B chain in integral form (d=4, nt=1000, ntau=400, "
                        "k=5): Q = G_0, F = -G_0*Sigma, Fcc = -Sigma*G_0, Sigma fixed",
            "value": nsteps / (min(whole) * 1e-3), "unit": "time-steps/s",
            "ms_per_solve": min(whole), "ms_steps": st_ms, "us_per_step": st_ms * 1e3 / nsteps,
            "dyson_form": {"ms_per_solve": d0.elapsed_time(d2), "ms_steps": d1.elapsed_time(d2)},
            "max_abs_deviation_from_dyson_form": dev_max, "max_abs_G": ref,
            "convolution": conv,
            "roofline": {"bound": "hbm", "scope": "time steps (k_v2_side beside k_history, then k_v2_reduce)",
                         "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "bytes": nbytes}}


def adj_sigma_products(n, k, ntau):
    """Block products of the Sigma-bar reductions of reverse step n (the term
    ranges of the adjoint kernels: retarded outputs j < n with min(j, nb-1)+1
    retarded, ntau+1 mixing and nb lesser terms; lesser outputs j <= n; mixing
    outputs ntau+1 with nb terms each; nb = n - k; lesser and mixing only for
    n > 2k)."""
    nb = n - k
    tot = 0
    for j in range(n):
        tot += min(j, nb - 1) + 1 + (ntau + 1) + (nb if n > 2 * k else 0)
    if n > 2 * k:
        for j in range(n + 1):
            a = min(k, nb - 1) + 1 if j <= k else 0
            tot += a + max(0, nb - max(j, k + 1))
        tot += (ntau + 1) * nb
    return tot


def run_cfg1(args):
    """Plain Dyson solve of the two-level system with the bath self-energy
    (H = [[-1, 0.5], [0.5, 1]], beta = 5, Sigma = 0.16 g_bath(eps_b = 0.3),
    nt = 100, h = 0.05, ntau = 100, k = 5): a launch-bound run of 95 short
    steps. Timed as whole solves (Matsubara solve, start-up, steps), the
    start-up and steps either launched one by one or replayed from one
    captured HIP graph (cntr_graph_*), on the same stream."""
    import torch

    from paper_1911_01211_amd import contour as K
    from paper_1911_01211_amd import workloads as W

    g = W.GridSpec(nt=100, ntau=100, d=2, beta=5.0, h=0.05, k=5)
    eps, S, _ = W.two_level_embedding(g)
    dev = "cuda:0"
    G, Sd, e = K.Contour(g, dev), K.Contour(g, dev, data=S), torch.as_tensor(eps).to(dev)
    st = torch.cuda.Stream()

    def steps():
        for n in range(g.k, g.nt + 1):
            K.dyson_step(n, [G], [Sd], [e], stream=st)

    def solve(graph=None):
        K.init_matsubara([G], [Sd], [e], stream=st)
        if graph is None:
            steps()
        else:
            graph.launch(st)

    solve()
    st.synchronize()
    with K.Graph(st) as gr:
        steps()
    times = {}
    reps = args.cfg1_reps
    for mode, graph in (("eager", None), ("graph", gr), ("eager", None), ("graph", gr)):
        solve(graph)
        st.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            solve(graph)
        st.synchronize()
        times[mode] = min(times.get(mode, 1e30), (time.perf_counter() - t0) / reps)
    # the step phase alone (start-up + 95 steps), HIP events on the stream
    ph = {}
    for mode in ("eager", "graph"):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            if mode == "eager":
                steps()
            else:
                gr.launch(st)
        e1.record(st)
        st.synchronize()
        ph[mode] = e0.elapsed_time(e1) / reps
    nsl = g.nt - g.k
    return {"workload": "two-level system with a fixed bath self-energy, nt=100, h=0.05, ntau=100, beta=5, k=5, "
                        "d=2 (whole solves: Matsubara, start-up, 95 steps)",
            "value": nsl / times["graph"], "unit": "time-steps/s",
            "eager_time_steps_per_s": nsl / times["eager"],
            "ms_per_solve": {k: v * 1e3 for k, v in times.items()},
            "step_phase_ms": ph, "graph_speedup_step_phase": ph["eager"] / ph["graph"]}


def run_free(args):
    """Free Green's function of a driven Hamiltonian on the chain's grid
    (cntr_green_from_H: nt = 1000, ntau = 400, d = 4): every component of G_0
    from the commutator-free propagator. Timed with HIP events on the launch
    stream; `achieved` counts the bytes of the function written (each block
    once) over the whole call."""
    import numpy as np
    import torch

    from paper_1911_01211_amd import contour as K
    from paper_1911_01211_amd import workloads as W

    g = workload_grid()
    e0, _ = W.hubbard_ramp(g)
    r = W.rng(77)
    H1 = W.random_hermitian(r, g.d, 0.5)
    eps = np.array(e0, np.complex128)
    for n in range(g.nt + 1):
        eps[n + 1] = eps[n + 1] + np.cos(0.7 * n * g.h) * H1
    e = torch.as_tensor(eps).to("cuda:0")
    G = K.Contour(g, "cuda:0")
    for _ in range(3):
        K.green_from_H([G], [e])
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    ev0.record()
    for _ in range(reps):
        K.green_from_H([G], [e])
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    dd = g.d * g.d
    nbytes = 16.0 * dd * ((g.nt + 1) * (g.nt + 2) + (g.nt + 1) * (g.ntau + 1) + (g.ntau + 1))
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": "free G_0 of eps(t) = chain hopping + cos(0.7 t) x random hermitian, "
                        f"nt={g.nt}, ntau={g.ntau}, d={g.d}, k={g.k}",
            "value": (g.nt + 1) / (ms * 1e-3), "unit": "time slices/s", "ms_per_call": ms,
            "roofline": {"bound": "hbm", "scope": "whole call (5 kernels)", "achieved": gbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "bytes": nbytes}}


def run_uneven(args):
    """Uneven batch: the first `uneven_count` of the 384 seeded problems of
    data/uneven_batch_384.npz (d in {1, 2, 4, 8}, nt in [400, 3000], U in
    [0.5, 2], random hermitian H with spectrum [-2, 2]; beta = 10, ntau = 300,
    h = 0.02, k = 5, local second-Born + Hartree), every problem run over its
    first `uneven_nt` slices (a causal prefix: those slices do not depend on
    the later ones). Timed twice on the same problems, whole solves
    (Matsubara loops, bootstrap, time steps): one cntr_solve_2b_uneven call
    (the orbital-count groups side by side, each group one launch per kernel
    and step) against the per-instance loop (cntr_solve_2b per problem).
    Also reported: the wave plan of the full 384-problem batch at its full
    lengths under a 200 GB cap (planning only)."""
    import numpy as np
    import torch

    from paper_1911_01211_amd import contour as K
    from paper_1911_01211_amd import workloads as W

    dev = "cuda:0"
    allp = W.load_uneven(os.path.join(ROOT, "paper_1911_01211_amd", "data", "uneven_batch_384.npz"))
    sel = allp[:args.uneven_count]
    problems = []
    for d, nt_full, U0, H in sel:
        nt = min(nt_full, args.uneven_nt)
        g = W.GridSpec(nt=nt, ntau=300, d=d, sig=-1, k=5, beta=10.0, h=0.02, mu=0.0)
        e0 = torch.as_tensor(np.broadcast_to(H, (nt + 2, d, d)).copy()).to(dev)
        U = torch.full((nt + 2,), U0, dtype=torch.float64, device=dev)
        problems.append(dict(G=K.Contour(g, dev), Sigma=K.Contour(g, dev), Gscratch=K.Contour(g, dev), eps0=e0,
                             U=U, eps_mf=torch.zeros_like(e0)))
    slices = sum(p["G"].g.nt - p["G"].g.k for p in problems)
    opts = dict(ncorr=args.ncorr, mats_tol=1e-14, boot_tol=1e-14)
    times = {}
    for mode in ("batched", "loop"):
        for p in problems:
            p["G"].zero_()
            p["Sigma"].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "batched":
            K.solve_uneven(problems, **opts)
        else:
            for p in problems:
                K.solve_2b(p["G"], p["Sigma"], p["Gscratch"], p["eps0"], p["U"], p["eps_mf"], **opts)
        torch.cuda.synchronize()
        times[mode] = time.perf_counter() - t0
        print(f"# uneven {mode}: {times[mode]:.2f}s", file=sys.stderr, flush=True)
    foot = [3 * 16.0 * d * d * ((nt + 1) * (nt + 2) + (nt + 1) * 301 + 301) for d, nt, _, _ in allp]
    waves = K.plan_waves(foot, 200e9)
    counts = {str(d): sum(1 for p in sel if p[0] == d) for d in (1, 2, 4, 8)}
    return {"workload": f"first {len(sel)} of the 384 seeded uneven second-Born problems (d counts {counts}), "
                        f"slices 0..min(nt, {args.uneven_nt}), ntau=300, beta=10, h=0.02, k=5; whole solves",
            "value": slices / times["batched"], "unit": "instance time-steps/s",
            "per_instance_loop": slices / times["loop"], "speedup_vs_loop": times["loop"] / times["batched"],
            "seconds": times, "corrector_iterations": args.ncorr,
            "full_batch_waves": {"cap_bytes": 200e9, "waves": len(waves), "problems": len(allp),
                                 "bytes_total": sum(foot),
                                 "bytes_per_wave": [sum(foot[i] for i in w) for w in waves]}}


def run_kpoints(args):
    """Batched sample: the single-band lattice with 512 k-points, eps_k(t) =
    -2 cos(k - A(t)) with the pulse A(t), local self-energy Sigma = 0.25 G_loc,
    beta = 10, ntau = 500, nt = 2000, h = 0.02, k = 5 (full grid allocated,
    41 GB). Untimed set-up: one Matsubara pass (free G^M, then Sigma^M) and the
    bootstrap; timed: the predictor-corrector steps k+1..nt_stop for all 512
    instances in one launch per step (ncorr corrector iterations each)."""
    import torch

    from paper_1911_01211_amd import contour as K
    from paper_1911_01211_amd import workloads as W

    g = W.GridSpec(nt=2000, ntau=500, d=1, sig=-1, k=5, beta=10.0, h=0.02, mu=0.0)
    nk = args.nk
    eps = [torch.as_tensor(e).to("cuda:0") for e in W.kpoint_band(g, nk)]
    G = [K.Contour(g, "cuda:0") for _ in range(nk)]
    S = K.Contour(g, "cuda:0")
    lam = 0.25
    B = K.solve_local(G, S, eps, lam, mats_iters=1, boot_iters=8, ncorr=args.ncorr, nt_stop=g.k)
    torch.cuda.synchronize()
    K.profile_begin(PROF_EVERY)
    t0 = time.perf_counter()
    for n in range(g.k + 1, args.kp_steps + 1):
        B.extrapolate(n - 1)
        for _ in range(args.ncorr):
            B.sigma_local(n, lam)
            B.step(n)
        B.sigma_local(n, lam)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = K.profile_end()
    nsteps = (args.kp_steps - g.k) * nk
    gbs = prof["hist_bytes"] / (prof["hist_ms"] * 1e-3) / 1e9 if prof["hist_ms"] > 0 else None

    # the plain per-instance loop at the last timed slice: one step of 16
    # instances, one call each, scaled to all instances, against the batched step
    def timed(f):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    # the whole batched step (every kernel of the corrector sweeps: history
    # sums, reduce, shared tau source, local Sigma, extrapolation) against the
    # HBM roofline at the algorithmic bytes of the history sums (each stored
    # block once per sweep, all instances)
    sweep_bytes = sum(16.0 * (n * (n + 1) + n * (g.ntau + 1)) for n in range(g.k + 1, args.kp_steps + 1)) * nk
    whole_gbs = sweep_bytes * args.ncorr / el / 1e9
    whole = {"bound": "hbm", "scope": "whole corrector sweeps, all kernels", "bytes_per_sweep": sweep_bytes,
             "seconds_per_sweep": el / args.ncorr, "achieved": whole_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": whole_gbs / HBM_PEAK_GBS}
    n_last, nloop = args.kp_steps, min(16, nk)
    t_batch = min(timed(lambda: B.step(n_last)) for _ in range(3))
    t_loop = min(timed(lambda: [K.dyson_step(n_last, [G[i]], [S], [eps[i]]) for i in range(nloop)])
                 for _ in range(2)) * nk / nloop
    return {"workload": f"{nk} k-points, d=1, local Sigma = 0.25 G_loc, pulse A(t), beta=10, ntau=500, "
                        f"nt=2000 grid; steps {g.k + 1}..{args.kp_steps} timed",
            "value": nsteps / el, "unit": "instance time-steps/s", "instances": nk,
            "ms_per_slice": el / (args.kp_steps - g.k) * 1e3, "corrector_iterations": args.ncorr,
            "loop_vs_batched_at_last_slice": {"slice": n_last, "batched_step_ms": t_batch,
                                              "per_instance_loop_ms": t_loop, "speedup": t_loop / t_batch,
                                              "loop_sample": f"{nloop} instances, scaled to {nk}"},
            "roofline": {"bound": "hbm", "kernel": "k_history<1>", "achieved": gbs, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS if gbs else None,
                         "avg_launch_us": prof["hist_ms"] * 1e3 / max(1, prof["hist_launches"])},
            "whole_step": whole,
            "note": ("whole run" if args.kp_steps >= g.nt else "prefix of the run (the per-slice cost grows with n)")}


def bubble_flops(n, nk, d, ntau, mode):
    """Real flops of one momentum-convolution call on slice n (a complex
    product 6, a complex sum 2; per element, momentum k and term q):
    Bubble1 R 16, < 10, rceil 8; Bubble2 R 24, < 8, rceil 8."""
    per = (16 * (n + 1) + 10 * (n + 1) + 8 * (ntau + 1)) if mode == 1 else (24 * (n + 1) + 8 * (n + 1) + 8 * (ntau + 1))
    return float(per) * d * d * nk * nk


def run_gw(args):
    """k-space GW (Eqs. Pol, Sigmak, the screened interaction by the integral
    form) on the batched lattice: nk momenta of eps_k(t) = -2 cos(k - A(t)),
    d = 1, U = 2, beta = 10, ntau = 500, h = 0.02, k = 5; untimed Matsubara
    loop and start-up, then the timed steps k+1..nt, each an extrapolation and
    ncorr x {Pi_k, (1 + F_k) * X_k = F_k, Sigma_k, Dyson step} for all
    momenta (one launch sequence per call). At the last slice every call is
    timed with HIP events on the launch stream; the momentum sums are counted
    in real flops against the FP64 vector peak (plain FMA arithmetic from LDS)."""
    import dataclasses

    import torch

    from paper_1911_01211_amd import contour as K
    from paper_1911_01211_amd import workloads as W

    nk, U, ncorr = args.gw_nk, 2.0, 3
    g = W.GridSpec(nt=args.gw_nt, ntau=500, d=1, sig=-1, k=5, beta=10.0, h=0.02, mu=0.0)
    eps = [torch.as_tensor(e).to("cuda:0") for e in W.kpoint_band(g, nk)]
    gb = dataclasses.replace(g, sig=1)
    G = [K.Contour(g, "cuda:0") for _ in range(nk)]
    F = [K.Contour(gb, "cuda:0") for _ in range(nk)]
    X = [K.Contour(gb, "cuda:0") for _ in range(nk)]
    S = [K.Contour(g, "cuda:0") for _ in range(nk)]
    B = K.Batch(G, S, eps)
    V = K.Vie2Batch(X, F, F, F)
    KB = K.KBatch(G, F, X, S)
    B.init_matsubara()
    for _ in range(10):
        KB.polarization(-1, -U)
        V.matsubara()
        KB.sigma(-1, -U)
        B.init_matsubara()
    for _ in range(6):
        for n in range(g.k + 1):
            KB.polarization(n, -U)
        V.step(g.k)
        for n in range(g.k + 1):
            KB.sigma(n, -U)
        B.step(g.k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(g.k + 1, g.nt + 1):
        B.extrapolate(n - 1)
        for _ in range(ncorr):
            KB.polarization(n, -U)
            V.step(n)
            KB.sigma(n, -U)
            B.step(n)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    def timed(f, reps=5):
        # a GPU-side wait first, so that the calls are queued before the
        # first event and the interval holds the kernels alone
        torch.cuda._sleep(20_000_000)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    n = g.nt
    ms = {"polarization_k": timed(lambda: KB.polarization(n, -U)),
          "vie2_step": timed(lambda: V.step(n)),
          "sigma_gw_k": timed(lambda: KB.sigma(n, -U)),
          "dyson_step": timed(lambda: B.step(n))}
    fl = {"polarization_k": bubble_flops(n, nk, g.d, g.ntau, 1), "sigma_gw_k": bubble_flops(n, nk, g.d, g.ntau, 2)}
    tf = {c: fl[c] / (ms[c] * 1e-3) / 1e12 for c in fl}
    # particle number sum_k n_k(t) = sum_k Im G_k^<(t,t) is conserved by GW
    dens = []
    for m in (0, n // 2, n):
        o = m * (m + 1) // 2 + m
        dens.append(float(sum(x.les[o, 0, 0].imag.item() for x in G)))
    return {"workload": f"k-space GW, {nk} momenta, eps_k = -2 cos(k - A(t)), d=1, U={U}, beta=10, ntau=500, "
                        f"h=0.02, k=5; steps {g.k + 1}..{g.nt} timed, {ncorr} corrector iterations each",
            "value": (g.nt - g.k) * nk / el, "unit": "instance time-steps/s", "seconds": el,
            "ms_per_call_at_last_slice": ms, "slice": n,
            "roofline": {"bound": "alu", "kernel": "k_kbubble<1> (polarization_k)", "achieved": tf["polarization_k"],
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf["polarization_k"] / FP64_PEAK_TFLOPS,
                         "flops": fl["polarization_k"], "sigma_gw_k_tflops": tf["sigma_gw_k"]},
            "check": {"particle_number": dens, "drift": max(abs(x - dens[0]) for x in dens)}}


def run_holstein(args):
    """Holstein DMFT on the Bethe lattice with the uMig impurity solver at the
    parameters of the paper's example: g = 0.5, w0 = 0.5, beta = 10, half
    filling (mu = g X = -2 g^2 / w0), J = 1, the coupling and the hopping
    modulated with a sin^2 envelope (Omega = 1.2, t_end = 15.7, dg = 0.05,
    dJ = 0.1); h = 0.02, nt = 1000, ntau = 400, k = 5, 30 Matsubara and 8
    start-up iterations, 4 corrector iterations per step. One impurity: the
    step is a short sequence of small launches (displacement, three slice
    scalings, the bubble, the Dyson step). Timed: the whole solve, and the
    same solve stopped after the start-up (the difference is the steps).
    Then a batch of impurities (couplings 0.3..0.6) the same way."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1911_01211_amd import contour as K
    from paper_1911_01211_amd import workloads as W

    g0, w0 = 0.5, 0.5
    g = W.GridSpec(nt=1000, ntau=400, d=1, sig=-1, k=5, beta=10.0, h=0.02, mu=-2 * g0 * g0 / w0)
    J, gel = W.holstein_drive(g, g0=g0)
    Jd, gd = torch.as_tensor(J).to("cuda:0"), torch.as_tensor(gel).to("cuda:0")
    kw = dict(mats_iters=30, boot_iters=8, ncorr=4)

    def solve(nt_stop):
        G = K.Contour(g, "cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = K.solve_holstein(G, Jd, gd, w0, nt_stop=nt_stop, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, G, out

    solve(g.k)  # warm-up (library scratch, weights)
    t_set, _, _ = solve(g.k)
    K.profile_begin(PROF_EVERY)
    t_all, G, (_, _, _, X, _) = solve(g.nt)
    prof = K.profile_end()
    t_steps = t_all - t_set
    nsteps = g.nt - g.k
    dens = [2.0 * G.les[m * (m + 1) // 2 + m, 0, 0].imag.item() for m in range(0, g.nt + 1, 100)]
    Xh = X.cpu().numpy()
    gbs = prof["hist_bytes"] / (prof["hist_ms"] * 1e-3) / 1e9 if prof["hist_ms"] > 0 else None

    # a batch of impurities (a sweep of the coupling g0, each at its half
    # filling) advanced together: one launch per call for all of them
    nb = args.holstein_batch
    g0s = np.linspace(0.3, 0.6, nb)
    gsb = [dataclasses.replace(g, mu=-2 * x * x / w0) for x in g0s]
    gelb = [torch.as_tensor(W.holstein_drive(gg, g0=x)[1]).to("cuda:0") for gg, x in zip(gsb, g0s)]

    def solve_batch(nt_stop):
        Gb = [K.Contour(gg, "cuda:0") for gg in gsb]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        K.solve_holstein(Gb, [Jd] * nb, gelb, [w0] * nb, nt_stop=nt_stop, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    tb_set = solve_batch(g.k)
    tb_all = solve_batch(g.nt)
    batch = {"impurities": nb, "g0": [float(g0s[0]), float(g0s[-1])],
             "value": nsteps * nb / (tb_all - tb_set), "unit": "instance time-steps/s",
             "us_per_step": (tb_all - tb_set) / nsteps * 1e6, "seconds": {"whole": tb_all, "setup": tb_set},
             "speedup_vs_single": nsteps * nb / (tb_all - tb_set) / (nsteps / t_steps)}
    return {"workload": "Holstein DMFT (Bethe lattice, uMig), g=0.5, w0=0.5, beta=10, half filling, g(t) and J(t) "
                        "modulated (Omega=1.2, t_end=15.7, dg=0.05, dJ=0.1), h=0.02, nt=1000, ntau=400, k=5",
            "value": nsteps / t_steps, "unit": "time-steps/s", "seconds": {"whole": t_all, "setup": t_set},
            "us_per_step": t_steps / nsteps * 1e6, "corrector_iterations": kw["ncorr"],
            "roofline": {"bound": "hbm", "kernel": "k_history<1>", "achieved": gbs, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS if gbs else None,
                         "avg_launch_us": prof["hist_ms"] * 1e3 / max(1, prof["hist_launches"])},
            "check": {"density_every_100": dens, "X_min_max": [float(Xh[1:].min()), float(Xh[1:].max())],
                      "X_eq": float(Xh[0])},
            "batch": batch}


def stream_bandwidth():
    """Device copy of 1 GiB (1 GiB read + 1 GiB written), best of 5, in GB/s:
    the attainable HBM rate that the roofline is also quoted against."""
    import torch

    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2 * (1 << 30) / (best * 1e-3) / 1e9


def profile_step(args):
    """Counter runs: the time step at slice args.profile_step of a seeded
    history with the workload's shape, 5 launches (each recomputes the same
    slice), then one device copy of 1 GiB (calibration of the HBM byte
    counters: its algorithmic traffic is 1 GiB read + 1 GiB written)."""
    import torch

    from paper_1911_01211_amd import contour as K
    from paper_1911_01211_amd import workloads as W

    g = workload_grid()
    r = W.rng(900)
    G = K.Contour(g, "cuda:0", data=W.random_contour(r, g, 0.3, decay=0.2))
    S = K.Contour(g, "cuda:0", data=W.random_contour(r, g, 0.3, decay=0.2))
    e0, _ = W.hubbard_ramp(g)
    e = torch.as_tensor(e0).to("cuda:0")
    n = args.profile_step
    for _ in range(5):
        K.dyson_step(n, [G], [S], [e])
    torch.cuda.synchronize()
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_step": n, "algorithmic_bytes_history": 16.0 * g.d ** 2 * (
        n * (n + 1) + n * (g.ntau + 1)), "copy_bytes": 2 * src.numel() * 8}), flush=True)


def cpu_baseline(g, ncorr, mats_iter, budget_s):
    """The oracle (OpenMP over the independent loops) on a bounded sample of the
    same workload: one corrector iteration (Sigma_2B + time step) at the
    slices n > k of a history with the workload's shape (seeded random values),
    as many as the time budget allows, one Matsubara solve and one start-up;
    the full run is assembled from these (slices not timed from a quadratic
    fit of the per-slice cost in n)."""
    import numpy as np

    from oracle import oracle as O
    from paper_1911_01211_amd import workloads as W

    og = O.Grid(g.nt, g.ntau, g.d, g.sig, g.k, g.beta, g.h, g.mu)
    r = W.rng(900)
    G, S = O.HM(og), O.HM(og)
    c = W.random_contour(r, g, 0.3, decay=0.2)
    for key in ("mat", "ret", "les", "tv"):
        getattr(G, key)[...] = c[key]
    c = W.random_contour(r, g, 0.3, decay=0.2)
    for key in ("mat", "ret", "les", "tv"):
        getattr(S, key)[...] = c[key]
    e0, U = W.hubbard_ramp(g)
    t_start = time.perf_counter()
    samples = []
    # slices in an interleaved order (every 8th slice, then the ones between),
    # so that the measured ones span the whole range whenever the budget ends
    order = [n for off in (0, 4, 2, 6, 1, 5, 3, 7) for n in range(g.k + 1 + off, g.nt + 1, 8)]
    for n in order:
        t = time.perf_counter()
        O.sigma_2b(n, G, U, S)
        O.dyson_timestep(n, G, S, e0, "B")
        samples.append((n, time.perf_counter() - t))
        if time.perf_counter() - t_start > budget_s:
            break
    ns = np.array([s[0] for s in samples], float)
    ts = np.array([s[1] for s in samples])
    coef = np.polyfit(ns, ts, min(2, len(ns) - 1))
    measured = {int(n): t for n, t in samples}
    steps = np.arange(g.k + 1, g.nt + 1)
    t_steps = ncorr * sum(measured.get(int(n), max(0.0, float(np.polyval(coef, n)))) for n in steps)
    t = time.perf_counter()
    O.dyson_mat(G, S, e0[0])
    t_mat = time.perf_counter() - t
    t = time.perf_counter()
    O.dyson_start(G, S, e0)
    t_start_up = time.perf_counter() - t
    total = t_steps + mats_iter * t_mat + 10 * t_start_up
    # one host thread: the same corrector iteration at eight slices spread
    # over the run, scaled by its ratio to the multi-threaded time there
    cores = O.num_threads()
    picks = [n for n in range(g.k + 1, g.nt + 1, max(1, (g.nt - g.k) // 8)) if n in measured][:8]
    ratio = None
    if picks:
        O.set_threads(1)
        try:
            r1 = []
            for n in picks:
                t = time.perf_counter()
                O.sigma_2b(n, G, U, S)
                O.dyson_timestep(n, G, S, e0, "B")
                r1.append((time.perf_counter() - t) / measured[n])
            ratio = float(np.mean(r1))
        finally:
            O.set_threads(cores)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": (g.nt - g.k) / total,
        "unit": "time-steps/s",
        "cores": cores,
        "cpu_model": model,
        "single_thread_value": (g.nt - g.k) / (total * ratio) if ratio else None,
        "single_thread_sample": f"slices {picks} on one thread, {ratio:.2f} x their {cores}-thread time" if ratio else None,
        "kind": "oracle",
        "sample": (f"oracle (B) time step + Sigma_2B, one corrector iteration at {len(samples)} of the "
                   f"{g.nt - g.k} slices n > k on a seeded history of the workload's shape, one "
                   f"{g.ntau + 1}x{g.d} Matsubara solve and one start-up, timed in "
                   f"{time.perf_counter() - t_start:.1f}s; full run = {ncorr} x sum_n t(n) (measured, "
                   f"else quadratic fit) + {mats_iter} Matsubara solves + 10 start-ups = {total:.1f}s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ncorr", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--nk", type=int, default=512, help="k-points of the batched sample")
    ap.add_argument("--kp-steps", type=int, default=2000, help="last slice of the batched k-point run")
    ap.add_argument("--no-kpoints", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-free", action="store_true")
    ap.add_argument("--no-cfg1", action="store_true")
    ap.add_argument("--no-vie2", action="store_true")
    ap.add_argument("--no-gw", action="store_true")
    ap.add_argument("--no-holstein", action="store_true")
    ap.add_argument("--holstein-batch", type=int, default=64, help="impurities of the batched Holstein sample")
    ap.add_argument("--gw-nk", type=int, default=256, help="momenta of the k-space GW sample")
    ap.add_argument("--gw-nt", type=int, default=400, help="last slice of the k-space GW sample")
    ap.add_argument("--no-tune-cache", action="store_true", help="built-in term chunks instead of tune_cache.json")
    ap.add_argument("--uneven-count", type=int, default=64, help="problems of the uneven batch (of 384)")
    ap.add_argument("--uneven-nt", type=int, default=400, help="slices of each uneven problem (causal prefix)")
    ap.add_argument("--cfg1-reps", type=int, default=50)
    ap.add_argument("--adj-niter", type=int, default=10, help="adjoint fixed-point iterations per slice")
    ap.add_argument("--adj-nt", type=int, default=1500, help="time steps of the adjoint ring workload")
    ap.add_argument("--adj-ncorr", type=int, default=8,
                    help="corrector iterations of the ring's forward solves (the adjoint is that of the converged "
                         "fixed point)")
    ap.add_argument("--adj-fd", type=int, default=2, help="directions of the central-difference check of the adjoint (0: off)")
    ap.add_argument("--profile-step", type=int, default=0,
                    help="only run the time step at this slice (counter runs), then a 1 GiB copy")
    args = ap.parse_args()
    if args.profile_step:
        profile_step(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the per-GPU share of a sharded run is the single-GPU workload).", file=sys.stderr)
        sys.exit(2)
    from paper_1911_01211_amd import autotune
    tiles = autotune.apply_cache() if not args.no_tune_cache else None
    g, elapsed, prof, stats, dens_dev, state = run_gpu(args)
    stream_gbs = stream_bandwidth()
    nsteps = (g.nt - g.k) * args.steps
    value = nsteps / elapsed
    hist_gbs = prof["hist_bytes"] / (prof["hist_ms"] * 1e-3) / 1e9 if prof["hist_ms"] > 0 else None
    # (the recorded steps are every PROF_EVERY-th one: scaled to all of them)
    tflops = prof["hist_flops"] * PROF_EVERY / elapsed / 1e12
    traffic, traffic_at = traffic_entry()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "second-Born Hubbard chain, 4 sites, U ramp 2->1 on [0,5], "
                               "beta=20, ntau=400, nt=1000, h=0.02, k=5",
                   "nt": g.nt, "ntau": g.ntau, "n_orb": g.d, "k": g.k, "h": g.h, "beta": g.beta,
                   "corrector_iterations": args.ncorr, "mats_iterations": stats.mats_iter,
                   "boot_iterations": stats.boot_iter},
        "fp64_tflops": tflops,
        "sweeps_per_s": args.ncorr * args.steps / elapsed,
        "last_slice_ms": state["last_slice_ms"],
        "time_step_share": prof["step_ms"] * PROF_EVERY / (elapsed * 1e3),
        "roofline": {"bound": "hbm", "kernel": "k_history<4>", "achieved": hist_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (hist_gbs / HBM_PEAK_GBS) if hist_gbs else None,
                     "stream_gbs": stream_gbs,
                     "frac_vs_stream": (hist_gbs / stream_gbs) if hist_gbs and stream_gbs else None,
                     "traffic": traffic,
                     "traffic_at": traffic_at,
                     "launches": prof["hist_launches"], "every": PROF_EVERY,
                     "avg_launch_us": prof["hist_ms"] * 1e3 / max(1, prof["hist_launches"])},
        "check": {"max_density_deviation_at_nt": dens_dev},
        "tiles": None if tiles is None else {d: {"n_hi": e["n_hi"], "tj": e["tj"]} for d, e in tiles["entries"].items()},
    }
    out["matsubara_fourier"] = run_mats_fourier(state)
    if not args.no_vie2:
        out["vie2"] = run_vie2(state)
    del state
    if not args.no_adjoint:
        out["adjoint"] = run_adjoint(args)
    if not args.no_cfg1:
        out["plain_two_level"] = run_cfg1(args)
    if not args.no_uneven:
        out["uneven"] = run_uneven(args)
    if not args.no_free:
        out["free_propagator"] = run_free(args)
    if not args.no_kpoints:
        out["batched"] = run_kpoints(args)
    if not args.no_gw:
        out["gw_kspace"] = run_gw(args)
    if not args.no_holstein:
        out["holstein"] = run_holstein(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.ncorr, stats.mats_iter, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

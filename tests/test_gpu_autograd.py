"""The differentiable propagation (DysonKineticEnergy, a torch.autograd.Function
over cntr_solve_2b, cntr_adjoint_sweep and the Peierls substitution) against
central differences of the CPU oracle on a small driven ring: gradients of
the final-time kinetic energy with respect to every drive sample A_n and to
U, to 1e-6 relative, and the exact zero of dJ/dA at A = 0 (the ring's
inversion symmetry makes J even in A)."""
import numpy as np
import pytest
import torch

from paper_1911_01211_amd import autograd as AG
from paper_1911_01211_amd import contour as K
from paper_1911_01211_amd import workloads as W
from tests.test_gpu_parity import require_gpu, say, to_dev
from tests.test_oracle_dyson import hm

pytestmark = pytest.mark.gpu
TOL = 1e-6
OPTS = dict(ncorr=12, mats_tol=1e-15, boot_tol=1e-15)


def oracle_J(O, g, T, Phi, A, U):
    eps = W.peierls_levels(T, Phi, A)
    G, S = hm(O, g), hm(O, g)
    rc, emf, _ = O.solve_2b(G, S, eps, U, boot_maxit=200, **OPTS)
    assert rc == 0
    N = g.nt
    return float((-2j * np.trace(eps[N + 1] @ G.L(N, N))).real)


def model(g, T, Phi):
    return AG.RingModel(g=g, T=to_dev(T), Phi=to_dev(Phi), niter=12, **OPTS)


@pytest.mark.parametrize("nsites,nt", [(4, 20), (6, 16)])
def test_kinetic_energy_gradient_matches_oracle_differences(O, nsites, nt):
    require_gpu()
    say(f"autograd ring nsites={nsites} nt={nt}")
    g = W.GridSpec(nt=nt, ntau=16, d=nsites, beta=2.0, h=0.05, k=5)
    T, Phi = W.ring_peierls(g, nsites)
    A = 4.0 * W.ring_drive(g)  # a drive of order one on this short grid
    U0 = 1.2
    At = torch.tensor(A, dtype=torch.float64, device="cuda", requires_grad=True)
    Ut = torch.tensor(U0, dtype=torch.float64, device="cuda", requires_grad=True)
    m = model(g, T, Phi)
    J = AG.kinetic_energy(At, Ut.expand(nt + 2), m)
    J.backward()
    gA, gU = At.grad.cpu().numpy(), float(Ut.grad.cpu())
    J0 = oracle_J(O, g, T, Phi, A, np.full(nt + 2, U0))
    say(f"  J gpu {float(J):.15e} oracle {J0:.15e}; adjoint last change {m.stats['adjoint_last_change']:.2e}")
    assert abs(float(J) - J0) <= 1e-10 * abs(J0)
    r = W.rng(410, nsites)
    cases = {"A": (r.normal(size=nt), 0.0), "U": (np.zeros(nt), 1.0),
             "A,U": (r.normal(size=nt), r.normal())}
    for n in (1, nt // 2, nt):
        e = np.zeros(nt)
        e[n - 1] = 1.0
        cases[f"A_{n}"] = (e, 0.0)
    for name, (dA, dU) in cases.items():
        big = max(np.abs(dA).max(), abs(dU))
        out = []
        for t in (4e-3 / big, 2e-3 / big):
            Jp = oracle_J(O, g, T, Phi, A + t * dA, np.full(nt + 2, U0 + t * dU))
            Jm = oracle_J(O, g, T, Phi, A - t * dA, np.full(nt + 2, U0 - t * dU))
            out.append((Jp - Jm) / (2 * t))
        ref = (4 * out[1] - out[0]) / 3
        got = float(np.dot(gA, dA) + gU * dU)
        scale = float(np.abs(gA * dA).sum() + abs(gU * dU))
        err = abs(got - ref) / max(abs(ref), 1e-2 * scale, 1e-300)
        say(f"  {name}: adjoint {got:.12e} differences {ref:.12e} rel {err:.2e}")
        assert err < TOL, (name, got, ref, err)


def test_kinetic_energy_gradient_vanishes_without_drive():
    """At A = 0 the ring is inversion symmetric (i -> -i maps A to -A), so J
    is even in A and dJ/dA_n = 0 for every n."""
    require_gpu()
    say("autograd ring at A = 0")
    g = W.GridSpec(nt=18, ntau=16, d=6, beta=2.0, h=0.05, k=5)
    T, Phi = W.ring_peierls(g, 6)
    At = torch.zeros(g.nt, dtype=torch.float64, device="cuda", requires_grad=True)
    Ut = torch.full((g.nt + 2,), 1.1, dtype=torch.float64, device="cuda", requires_grad=True)
    J = AG.kinetic_energy(At, Ut, model(g, T, Phi))
    J.backward()
    gU = Ut.grad.cpu().numpy()
    assert np.abs(gU).max() > 1e-3
    assert np.abs(At.grad.cpu().numpy()).max() <= 1e-12 * np.abs(gU).max()


def test_peierls_substitution_matches_input_definition():
    """cntr_peierls against the input-side definition eps_n = T exp(i A_n Phi)."""
    require_gpu()
    g = W.GridSpec(nt=30, ntau=16, d=8, beta=2.0, h=0.05, k=5)
    T, Phi = W.ring_peierls(g, 8)
    A = W.ring_drive(g)
    m = AG.RingModel(g=g, T=to_dev(T), Phi=to_dev(Phi))
    A_full = to_dev(np.concatenate([[0.0, 0.0], A]))
    eps = AG._peierls(m, A_full)
    K.sync()
    ref = W.peierls_levels(T, Phi, A)
    assert np.abs(eps.cpu().numpy() - ref).max() < 1e-15

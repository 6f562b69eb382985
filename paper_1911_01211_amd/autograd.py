"""Differentiable Kadanoff-Baym propagation: the kinetic energy at the final
time of a self-consistent second-Born run, as a torch.autograd.Function whose
backward pass is the library's discrete adjoint sweep.

Forward:  eps_n = T_n exp(i A_n Phi) (Peierls phase, cntr_peierls), the
          self-consistent 2B + Hartree solve (cntr_solve_2b), and
          J = E_kin(t_N) = -2i Tr[eps_kin(t_N) G^<(t_N, t_N)] (both spins; the
          one-body energy of cntr_observables, eps_kin = eps_N).
Backward: the seed dJ/dG^<(t_N, t_N), the adjoint sweep in its second-Born
          mode (cntr_adjoint_sweep: dJ/deps0_n and dJ/dU_n), the explicit
          dependence of J on eps_N, and the chain rule of the phase
          (cntr_peierls_grad) give dJ/dA_n and dJ/dU_n.

Only marshalling happens here: the solve, the observables, the adjoint and
both halves of the Peierls substitution run in the HIP library.
"""
from __future__ import annotations

import dataclasses

import torch

from . import _abi
from . import contour as K
from .workloads import GridSpec


@dataclasses.dataclass
class RingModel:
    """A lattice with a Peierls-phase drive: bare levels T [nt+2, d, d]
    (complex128, device), phase pattern Phi [d, d] (float64, device), the
    grid, and the solver controls of cntr_solve_2b."""
    g: GridSpec
    T: torch.Tensor
    Phi: torch.Tensor
    nbar: float = 0.5
    ncorr: int = 5
    mats_tol: float = 1e-14
    boot_tol: float = 1e-14
    niter: int = 10  # adjoint fixed-point iterations per slice
    stats: dict = dataclasses.field(default_factory=dict)


def _peierls(m: RingModel, A_full: torch.Tensor) -> torch.Tensor:
    eps = torch.empty_like(m.T)
    g = K.grid_c(m.g)
    _abi.check(_abi.lib().cntr_peierls(1, C_grid(g), K._ptrs([m.T]), K._ptrs([m.Phi]), K._ptrs([A_full]),
                                       K._ptrs([eps]), K._stream()))
    return eps


def C_grid(g):
    return _abi.arr(_abi.Grid, [g])


class DysonKineticEnergy(torch.autograd.Function):
    """J = E_kin(t_N) of the driven, self-consistent second-Born solution.

    apply(A, U, model): A float64 [nt] (the samples A_1..A_nt; A(0^-) = A_0 = 0),
    U float64 [nt+2] (U_n at index n+1, U_{-1} first), both on the device;
    returns a 0-dim float64 tensor. Gradients: dJ/dA [nt] and dJ/dU [nt+2]."""

    @staticmethod
    def forward(ctx, A, U, model: RingModel):
        g = model.g
        dev = A.device
        A = A.detach().contiguous()
        U = U.detach().contiguous()
        zero = torch.zeros(2, dtype=torch.float64, device=dev)
        A_full = torch.cat([zero, A]).contiguous()
        e0 = _peierls(model, A_full)
        G, S, Gs = K.Contour(g, dev), K.Contour(g, dev), K.Contour(g, dev)
        emf = torch.zeros_like(e0)
        st = K.solve_2b(G, S, Gs, e0, U, emf, nbar=model.nbar, ncorr=model.ncorr, mats_tol=model.mats_tol,
                        boot_tol=model.boot_tol)
        model.stats.update(forward=st)
        obs, _ = K.observables(g.nt, [G], [S], [e0], [emf])
        J = 2.0 * obs[0, 1]
        ctx.model = model
        ctx.save_for_backward(A_full, U, e0, emf)
        ctx.state = (G, S)
        return J.detach().clone()

    @staticmethod
    def backward(ctx, gJ):
        model = ctx.model
        g = model.g
        A_full, U, e0, emf = ctx.saved_tensors
        G, S = ctx.state
        N = g.nt
        o = N * (N + 1) // 2 + N
        # J = Re(-2i sum_ab eps_ba L_ab) at t_N: gradients (d/dRe + i d/dIm)
        Gb, Sb = K.Contour(g, G.mat.device), K.Contour(g, G.mat.device)
        Gb.les[o] = gJ * torch.conj(-2j * e0[N + 1].transpose(0, 1))
        eb = torch.zeros_like(e0)
        ub = torch.zeros_like(U)
        conv = K.adjoint_sweep([G], [S], [emf], [Gb], [eb], [Sb], U=[U], U_bar=[ub], nbar=model.nbar,
                               niter=model.niter)
        model.stats.update(adjoint_last_change=conv)
        eb[N + 1] += gJ * torch.conj(-2j * G.les[o].transpose(0, 1))
        Ab = torch.zeros_like(A_full)
        gd = C_grid(K.grid_c(g))
        _abi.check(_abi.lib().cntr_peierls_grad(1, gd, K._ptrs([model.T]), K._ptrs([model.Phi]),
                                                K._ptrs([A_full]), K._ptrs([eb]), K._ptrs([Ab]), K._stream()))
        ctx.state = None
        return Ab[2:], ub, None


def kinetic_energy(A: torch.Tensor, U: torch.Tensor, model: RingModel) -> torch.Tensor:
    return DysonKineticEnergy.apply(A, U, model)

"""E2 as a differentiable function of the TOP-basis Fock matrix and factor.

A torch.autograd.Function over the C ABI: the forward pass binds the problem
in the TOP basis (esmp2_set_problem_top), solves for the first-order
amplitudes and, when a gradient is wanted, evaluates dE2/dF~ and dE2/dB~
with esmp2_gradient.  E2_DL is stationary in the amplitudes and the operator
is symmetric, so the adjoint solution is the solution itself: the backward
pass only scales the stored gradients.  Argument marshalling only; all
arithmetic runs in libesmp2.
"""
from __future__ import annotations

import torch

from ._lib import ESMP2_BASIS_SEMICANONICAL, Handle


class _E2Top(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Ft, Bt, lam, handle, tol, basis, spin):
        n_occ = lam.numel()
        n = Ft.shape[0]
        n_aux = Bt.shape[0]
        Ft_c = Ft.detach().to(torch.float64).contiguous()
        Bt_c = Bt.detach().to(torch.float64).contiguous()
        lam_c = lam.detach().to(device=Ft.device, dtype=torch.float64).contiguous()
        handle.set_problem_top(Ft_c, Bt_c, lam_c, n_occ, n - n_occ, n_aux, spin)
        handle.rotate_top(False)
        handle.build_rhs()
        n_amp, _ = handle.space()
        x = torch.empty(n_amp, dtype=torch.float64, device=Ft.device)
        r = handle.solve(tol=tol, max_iter=1000, basis=basis, x_out=x, allow=())
        dF = torch.empty_like(Ft_c) if ctx.needs_input_grad[0] else None
        dB = torch.empty_like(Bt_c) if ctx.needs_input_grad[1] else None
        if dF is not None or dB is not None:
            handle.gradient(x, dF, dB)
        ctx.save_for_backward(dF, dB)
        return torch.tensor(r["e2"], dtype=torch.float64, device=Ft.device)

    @staticmethod
    def backward(ctx, g):
        dF, dB = ctx.saved_tensors
        return (None if dF is None else g * dF, None if dB is None else g * dB, None, None, None, None, None)


def e2_top(Ft, Bt, lam, handle=None, tol=1e-10, basis=ESMP2_BASIS_SEMICANONICAL, spin=0):
    """E2 of the problem stated in the TOP basis (Ft: N x N, Bt: n_aux x N x N,
    lam: n_occ singular values), differentiable in Ft and Bt with lam and the
    basis held fixed.  The gradients are symmetric: dE2 = sum_pq G[p][q] dF[p][q]
    for symmetric perturbations.  spin: 0 singlet, 1 triplet reference.
    `handle` (bound to Ft's device and torch's
    current stream) is reused when given; its previous problem is replaced."""
    own = handle is None
    if own:
        handle = Handle(Ft.device.index or 0)
    try:
        return _E2Top.apply(Ft, Bt, lam, handle, tol, basis, spin)
    finally:
        if own:
            torch.cuda.current_stream(Ft.device).synchronize()
            handle.close()

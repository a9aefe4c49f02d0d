"""torch.autograd interface of the THIIM adjoint gradient.

``absorption(eps, weight, problem)`` returns the absorption functional
J = sum_p w_p eps''_p |E_p|^2 of the converged THIIM solution for the
permittivity ``eps`` (complex128 tensor on the GPU, eps' + 1j eps'', the
physical eps_r being eps' - i eps''), differentiable with respect to ``eps``.
Forward: thiim_create + thiim_solve + thiim_adjoint_grad (which also returns
J); backward: grad_output times the stored gradient.  The gradient follows
torch's convention for a real function of a complex tensor,
dJ/deps' + 1j dJ/deps''.  All arithmetic runs in the HIP library.
"""
from __future__ import annotations

import dataclasses

import torch

from . import thiim


class _Absorption(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, weight, problem, opts):
        pb = dataclasses.replace(problem, eps=eps.detach().to(torch.complex128).contiguous())
        solver = thiim.Solver(pb, storage="compact", adjoint=True,
                              kernel=opts.get("kernel", "auto"))
        try:
            if opts["iters"] is not None:
                solver.iterate(opts["iters"])
            else:
                rc, it, r = solver.solve(opts["tol"], opts["max_it"], opts["check_every"])
                if rc != thiim.THIIM_OK:
                    raise thiim.ThiimError(rc, f"forward solve stopped at {r:.3e} after {it}")
            rc, J, grad, ait, ar = solver.adjoint_grad(weight, opts["adj_tol"], opts["max_it"],
                                                       opts["check_every"])
            if rc != thiim.THIIM_OK:
                raise thiim.ThiimError(rc, f"adjoint solve stopped at {ar:.3e} after {ait}")
        finally:
            solver.close()
        ctx.save_for_backward(grad)
        return torch.tensor(J, dtype=torch.float64, device=eps.device)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out * grad, None, None, None


def absorption(eps, weight, problem, tol=1e-12, adj_tol=None, max_it=200000,
               check_every=50, kernel="auto", iters=None):
    """J(eps) for the THIIM problem ``problem`` (an ``inputs.Problem`` whose
    own eps is ignored), differentiable in ``eps``.  The forward state is
    solved to ``tol`` (relative residual of the physical fields), or, with
    ``iters``, is the iterate after exactly that many iterations from x0 = 0
    (for finite-difference checks: every evaluation then carries the same
    truncation).  The adjoint is solved to ``adj_tol`` (default ``tol``)."""
    opts = dict(tol=tol, adj_tol=tol if adj_tol is None else adj_tol, max_it=max_it,
                check_every=check_every, kernel=kernel, iters=iters)
    return _Absorption.apply(eps, weight, problem, opts)

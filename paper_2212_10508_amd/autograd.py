"""torch.autograd.Function over the SNAP coefficients beta.

forward(beta, x): total SNAP energy E = sum_i E_i and forces F = -dE/dx of a batch
(through snap_forces).  backward(gE, gF): dE/dbeta and sum_i gF_i . dF_i/dbeta through
snap_beta_grad, so a force-matching loss can be fitted with any torch optimiser.
Positions are inputs only (no gradient with respect to x).
"""
import numpy as np
import torch

from . import snapmd as S


class SnapFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, beta, x, offset, box, J, rcut=4.73, rfac0=0.99363, rmin0=0.0):
        if x.requires_grad:
            raise NotImplementedError("SnapFunction gives gradients with respect to beta only")
        sctx = S.context(x.device.index or 0)
        beta_h = beta.detach().to("cpu", torch.float64).numpy()
        N = int(offset[-1])
        e = torch.zeros(N, dtype=torch.float64, device=x.device)
        f = sctx.snap_forces(x, offset, box, J, beta_h, e_atom=e, rcut=rcut, rfac0=rfac0, rmin0=rmin0)
        fctx.save_for_backward(x)
        fctx.meta = (np.asarray(offset), np.asarray(box), J, beta_h, rcut, rfac0, rmin0, beta.device, beta.dtype)
        return e.sum(), f

    @staticmethod
    def backward(fctx, gE, gF):
        (x,) = fctx.saved_tensors
        offset, box, J, beta_h, rcut, rfac0, rmin0, bdev, bdt = fctx.meta
        sctx = S.context(x.device.index or 0)
        w = gF.contiguous() if gF is not None else torch.zeros_like(x)
        dE, gradF = sctx.snap_beta_grad(x, w, offset, box, J, beta_h, rcut=rcut, rfac0=rfac0, rmin0=rmin0)
        g = gradF
        if gE is not None:
            g = g + gE.to(g.dtype) * dE
        return g.to(bdev, bdt), None, None, None, None, None, None, None


def snap_energy_forces(beta, x, offset, box, J, **kw):
    """Differentiable (in beta) total energy and forces."""
    return SnapFunction.apply(beta, x, offset, box, J, kw.get("rcut", 4.73), kw.get("rfac0", 0.99363),
                              kw.get("rmin0", 0.0))

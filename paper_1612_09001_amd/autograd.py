"""PyTorch autograd wrapper of the predistorter (forward and hand-written
adjoint kernels of libdpd).

``DPDFunction.apply(x, coeffs, plan)`` computes Eq. (1) on x (1-D stream or
rows x n) with the coefficients read from the device tensor ``coeffs`` (K
complex64, the stacking of section 2.2).  Only (x, coeffs) are saved; the
backward kernel recomputes the basis.  Gradients follow PyTorch's convention
for complex tensors (dE/dRe + j dE/dIm), which is the one the C ABI uses.
"""
from __future__ import annotations

import torch

from . import dpd as _dpd


class DPDFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, coeffs, plan):
        x = x.contiguous()
        coeffs = coeffs.contiguous()
        z = plan.apply_coeffs(coeffs, x)
        ctx.save_for_backward(x, coeffs)
        ctx.plan = plan
        return z

    @staticmethod
    def backward(ctx, grad_z):
        x, coeffs = ctx.saved_tensors
        want_dx = ctx.needs_input_grad[0]
        want_dc = ctx.needs_input_grad[1]
        if not (want_dx or want_dc):
            return None, None, None
        gx, gc = ctx.plan.backward(x, grad_z.contiguous(), coeffs=coeffs, want_dx=want_dx,
                                   want_dcoeffs=want_dc)
        return gx, gc, None


def dpd_apply(x, coeffs, plan):
    """Differentiable predistortion: z = DPD_coeffs(x)."""
    return DPDFunction.apply(x, coeffs, plan)


class Predistorter(torch.nn.Module):
    """Learnable predistorter: K complex coefficients as one parameter."""

    def __init__(self, main_orders, conj_orders, L, coeffs):
        super().__init__()
        c = torch.as_tensor(coeffs, dtype=torch.complex64)
        self.plan = _dpd.Plan(main_orders, conj_orders, L, c.cpu().numpy())
        self.coeffs = torch.nn.Parameter(c.clone())

    def forward(self, x):
        return DPDFunction.apply(x, self.coeffs, self.plan)

"""Comparison baselines -- never called by the library path.

``aph_plain`` states Eq. (1) with ordinary PyTorch tensor operations (one
elementwise kernel per basis power and per tap), so ``torch.autograd`` can
differentiate it; ``PlainTrainer`` is the coefficient-learning step built
from it with a PyTorch loss and ``torch.optim.Adam``.  These are the
"autograd of plain ops" reference the hand-written kernels are timed
against, on the same GPU.
"""
from __future__ import annotations

import numpy as np
import torch

from .pa import GAIN, IQ_ORDERS, PA_ORDERS, iq_coeffs, pa_coeffs


def aph_plain(x, coeffs, main_orders, conj_orders, L):
    """Eq. (1) on each row of x (rows, n) with plain tensor ops (complex64)."""
    rows, n = x.shape
    pad = torch.zeros(rows, L - 1, dtype=x.dtype, device=x.device)
    xp = torch.cat([pad, x], dim=1)
    s = xp.real * xp.real + xp.imag * xp.imag
    z = torch.zeros_like(x) + coeffs[-1]
    branches = [(p, False) for p in main_orders] + [(q, True) for q in conj_orders]
    for b, (p, conj) in enumerate(branches):
        basis = xp if p == 1 else s.pow((p - 1) // 2) * xp
        if conj:
            basis = torch.conj(basis)
        for k in range(L):
            z = z + coeffs[b * L + k] * basis[:, L - 1 - k:L - 1 - k + n]
    return z


class PlainTrainer:
    def __init__(self, x, main_orders, conj_orders, L, coeffs0, lr=1e-3):
        self.x = x
        self.orders = (list(main_orders), list(conj_orders), int(L))
        dev = x.device
        self.coeffs = torch.nn.Parameter(
            torch.as_tensor(np.asarray(coeffs0, dtype=np.complex64)).to(dev).clone())
        self.iq_c = torch.as_tensor(iq_coeffs()).to(dev)
        self.pa_c = torch.as_tensor(pa_coeffs()).to(dev)
        self.opt = torch.optim.Adam([self.coeffs], lr=lr)

    def loss_fn(self):
        z = aph_plain(self.x, self.coeffs, *self.orders)
        u = aph_plain(z, self.iq_c, *IQ_ORDERS)
        y = aph_plain(u, self.pa_c, *PA_ORDERS)
        return (torch.abs(y / GAIN - self.x) ** 2).mean()

    def step(self):
        self.opt.zero_grad(set_to_none=True)
        loss = self.loss_fn()
        loss.backward()
        self.opt.step()
        return loss.detach()

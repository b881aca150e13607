"""Learning predistorter coefficients through the fixed synthetic PA.

``FusedTrainer.step()`` runs one full-batch gradient step entirely in libdpd
kernels, on buffers allocated once.  With rows of whole 256-sample chunks it
is one library call, ``dpd_learn_step`` (three launches):

  z, E, dE/dy                the predistorter (its table precombined from the
                             device coefficients by every block), the synthetic transmitter
                             u = IQ(z), y = PA(u) (pa.py) and the loss
                             E = mean |y/G - x|^2 with its gradient in one
                             pass (u and y never stored, z written once)
  dE/dcoeffs                 the adjoint of PA and IQ and the coefficient
                             gradient of the predistorter in one pass (dE/dz
                             never stored)
  finalisation + Adam        loss and gradient summed in FP64, Adam applied
                             to the K complex coefficients in place

With ``device_step=True`` the call is ``dpd_learn_step_dev``: Adam's step
count lives on the device and the call advances it, so ``step()`` can be
captured into a HIP graph and replayed (every replay takes the next step).

Other row lengths run the same passes as separate calls
(dpd_transmit_loss_grad, dpd_transmit_backward through a dE/dz buffer,
dpd_adam_step).  ``one_pass=False`` runs the predistorter as its own launch
before the fused transmitter (dpd_apply_coeffs, dpd_cascade_loss_grad,
dpd_cascade_backward, dpd_backward); ``fused_transmitter=False`` runs the
transmitter and its adjoint as separate launches per stage (IQ, PA, loss; PA
and IQ adjoints) instead.

``AutogradTrainer`` is the same step through ``torch.autograd`` with the
predistorter and both PA stages as ``DPDFunction`` nodes (hand-written
adjoint kernels), a PyTorch loss and ``torch.optim.Adam``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dpd as _dpd
from .autograd import DPDFunction
from .pa import SyntheticPA, iq_coeffs, pa_coeffs


class FusedTrainer:
    def __init__(self, x, main_orders, conj_orders, L, coeffs0, lr=1e-3, betas=(0.9, 0.999),
                 eps=1e-8, fused_transmitter=True, one_pass=True, device_step=False):
        if x.dim() != 2 or not x.is_contiguous():
            raise ValueError("x must be a contiguous (rows, n) complex64 GPU tensor")
        self.x = x
        self.rows, self.n = x.shape
        self.plan = _dpd.Plan(main_orders, conj_orders, L, np.asarray(coeffs0))
        self.K = self.plan.K
        dev = x.device
        self.coeffs = torch.as_tensor(np.asarray(coeffs0, dtype=np.complex64)).to(dev).contiguous()
        self.pa = SyntheticPA()
        self.fused_transmitter = bool(fused_transmitter)
        # predistorter, transmitter and loss in one kernel (dpd_transmit_loss_grad)
        # where the stages are the ones it is built for
        self.one_pass = bool(one_pass) and max(list(main_orders) + list(conj_orders)) <= 9 and L <= 8
        self.z = torch.empty_like(x)
        self.gy = torch.empty_like(x)
        self.gz = torch.empty_like(x)
        if not self.fused_transmitter:
            self.u = torch.empty_like(x)
            self.y = torch.empty_like(x)
            self.gu = torch.empty_like(x)
        self.gc = torch.empty(self.K, dtype=torch.complex64, device=dev)
        self.m = torch.zeros(2 * self.K, dtype=torch.float32, device=dev)
        self.v = torch.zeros(2 * self.K, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.lr, self.betas, self.eps = lr, betas, eps
        self.t = 0
        ws = max(_dpd.dpd_backward_ws_size(p.handle, self.rows, self.n)
                 for p in (self.plan, self.pa.iq, self.pa.pa))
        self.ws_bytes = max(ws, _dpd.dpd_loss_ws_size(self.rows * self.n), _dpd.dpd_learn_step_ws_size(self.plan.handle))
        # the whole step in one library call where its one-pass kernels apply
        # (whole 256-sample chunks; torch's allocations are 16-byte aligned)
        self.one_call = self.one_pass and self.n % 256 == 0
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        # Adam's step count on the device (advanced by each call), for graph capture
        self.step_dev = None
        if device_step:
            if not (self.fused_transmitter and self.one_call):
                raise ValueError("device_step needs the one-call step (one-pass shapes, n a multiple of 256)")
            self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)

    def step(self):
        """One gradient step; returns the loss of the coefficients before it
        (a device tensor, no host synchronization)."""
        st = _dpd.current_stream()
        R, N, ld = self.rows, self.n, self.n
        P = lambda t: t.data_ptr()
        iq, pa = self.pa.iq.handle, self.pa.pa.handle
        if self.step_dev is not None:
            self.t += 1
            _dpd.dpd_learn_step_dev(self.plan.handle, iq, pa, st, P(self.coeffs), P(self.m), P(self.v),
                                    P(self.step_dev), self.lr, self.betas[0], self.betas[1], self.eps, P(self.x),
                                    P(self.z), P(self.gy), R, N, ld, 1.0 / self.pa.gain, P(self.loss), P(self.gc),
                                    P(self.ws), self.ws_bytes)
            return self.loss
        if self.fused_transmitter and self.one_call:
            self.t += 1
            _dpd.dpd_learn_step(self.plan.handle, iq, pa, st, P(self.coeffs), P(self.m), P(self.v), self.t, self.lr,
                                self.betas[0], self.betas[1], self.eps, P(self.x), P(self.z), P(self.gy), R, N, ld,
                                1.0 / self.pa.gain, P(self.loss), P(self.gc), P(self.ws), self.ws_bytes)
            return self.loss
        if self.fused_transmitter and self.one_pass:
            # forward in one pass, backward in another: dE/dz stays on chip where
            # the shapes allow (else dpd_transmit_backward goes through self.gz)
            _dpd.dpd_transmit_loss_grad(self.plan.handle, iq, pa, st, P(self.coeffs), P(self.x), P(self.z), R, N, ld,
                                        1.0 / self.pa.gain, P(self.loss), P(self.gy), P(self.ws), self.ws_bytes)
            gz = 0 if N % 256 == 0 else P(self.gz)
            _dpd.dpd_transmit_backward(self.plan.handle, iq, pa, st, P(self.x), P(self.z), P(self.gy), gz,
                                       P(self.gc), R, N, ld, P(self.ws), self.ws_bytes)
        elif self.fused_transmitter:
            _dpd.dpd_apply_coeffs(self.plan.handle, st, P(self.coeffs), P(self.x), P(self.z), R, N, ld)
            _dpd.dpd_cascade_loss_grad(iq, pa, st, P(self.z), P(self.x), R, N, ld, 1.0 / self.pa.gain,
                                       P(self.loss), P(self.gy), P(self.ws), self.ws_bytes)
            _dpd.dpd_cascade_backward(iq, pa, st, P(self.z), P(self.gy), P(self.gz), R, N, ld)
        else:
            _dpd.dpd_apply_coeffs(self.plan.handle, st, P(self.coeffs), P(self.x), P(self.z), R, N, ld)
            _dpd.dpd_apply_rows(iq, st, P(self.z), P(self.u), R, N, ld)
            _dpd.dpd_apply_rows(pa, st, P(self.u), P(self.y), R, N, ld)
            _dpd.dpd_loss_grad(st, P(self.y), P(self.x), R * N, 1.0 / self.pa.gain, P(self.loss),
                               P(self.gy), P(self.ws), self.ws_bytes)
            _dpd.dpd_backward(pa, st, 0, P(self.u), P(self.gy), P(self.gu), 0, R, N, ld,
                              P(self.ws), self.ws_bytes)
            _dpd.dpd_backward(iq, st, 0, P(self.z), P(self.gu), P(self.gz), 0, R, N, ld,
                              P(self.ws), self.ws_bytes)
        if not (self.fused_transmitter and self.one_pass):
            _dpd.dpd_backward(self.plan.handle, st, P(self.coeffs), P(self.x), P(self.gz), 0, P(self.gc),
                              R, N, ld, P(self.ws), self.ws_bytes)
        self.t += 1
        _dpd.dpd_adam_step(st, P(self.coeffs), P(self.gc), P(self.m), P(self.v), 2 * self.K, self.t,
                           self.lr, self.betas[0], self.betas[1], self.eps)
        return self.loss

    def state_dict(self):
        t = int(self.step_dev.item()) if self.step_dev is not None else self.t
        return {"coeffs": self.coeffs.clone(), "m": self.m.clone(), "v": self.v.clone(), "t": t}

    def load_state_dict(self, d):
        self.coeffs.copy_(d["coeffs"])
        self.m.copy_(d["m"])
        self.v.copy_(d["v"])
        self.t = int(d["t"])
        if self.step_dev is not None:
            self.step_dev.fill_(self.t)


class AutogradTrainer:
    def __init__(self, x, main_orders, conj_orders, L, coeffs0, lr=1e-3):
        self.x = x
        self.plan = _dpd.Plan(main_orders, conj_orders, L, np.asarray(coeffs0))
        self.pa = SyntheticPA()
        dev = x.device
        self.coeffs = torch.nn.Parameter(
            torch.as_tensor(np.asarray(coeffs0, dtype=np.complex64)).to(dev).clone())
        self.iq_c = torch.as_tensor(iq_coeffs()).to(dev)
        self.pa_c = torch.as_tensor(pa_coeffs()).to(dev)
        self.opt = torch.optim.Adam([self.coeffs], lr=lr)

    def loss_fn(self):
        z = DPDFunction.apply(self.x, self.coeffs, self.plan)
        u = DPDFunction.apply(z, self.iq_c, self.pa.iq)
        y = DPDFunction.apply(u, self.pa_c, self.pa.pa)
        return (torch.abs(y / self.pa.gain - self.x) ** 2).mean()

    def step(self):
        self.opt.zero_grad(set_to_none=True)
        loss = self.loss_fn()
        loss.backward()
        self.opt.step()
        return loss.detach()

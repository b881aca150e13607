"""Indirect-learning estimation of the predistorter (section 2.2).

The paper estimates the APH coefficients offline by least squares: a
postdistorter with the predistorter's basis is fitted from the PA output
(divided by the PA gain) to the PA input, and its coefficients are copied into
the predistorter; repeating this moves the predistorter towards the inverse of
the PA.  Every step runs in libdpd kernels: the predistorter and the two
synthetic PA stages (forward apply), the normal equations (matrix-core Gram
kernel, FP64 reduction) and the Cholesky solve, whose result goes into the
plan's table without leaving the device.
"""
from __future__ import annotations

import numpy as np

from . import dpd as _dpd
from . import pa as _pa


def identity_coeffs(n_main: int, n_conj: int, L: int) -> np.ndarray:
    """h_{1,0} = 1 (main branch order 1 first), everything else 0."""
    h = np.zeros((n_main + n_conj) * L + 1, dtype=np.complex64)
    h[0] = 1.0
    return h


class ILA:
    """Iterated least-squares fit of an APH predistorter to the synthetic PA.

    x: contiguous complex64 GPU tensor (rows x n or 1-D) of transmit samples.
    ridge: the diagonal loading of the normal equations, relative to their mean
    diagonal.  Every buffer is allocated once here; an iteration is six
    library calls on the current stream with no host synchronization.
    """

    def __init__(self, x, main_orders, conj_orders, L, ridge=1e-9, pa=None):
        import torch

        if not x.is_contiguous() or x.dim() not in (1, 2):
            raise ValueError("x must be a contiguous 1-D or rows x n tensor")
        self.x = x
        self.plan = _dpd.Plan(main_orders, conj_orders, L,
                              identity_coeffs(len(main_orders), len(conj_orders), L))
        self.pa = pa if pa is not None else _pa.SyntheticPA()
        self.ridge = float(ridge)
        self.rows, self.n = (1, x.numel()) if x.dim() == 1 else tuple(x.shape)
        dev = x.device
        K = self.plan.K
        self.z = torch.empty_like(x)
        self.u = torch.empty_like(x)
        self.y = torch.empty_like(x)
        self.A = torch.empty((K, K), dtype=torch.complex128, device=dev)
        self.b = torch.empty(K, dtype=torch.complex128, device=dev)
        self.ws_bytes = _dpd.dpd_ls_ws_size(self.plan.handle, self.rows, self.n)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=dev)
        self.sws_bytes = _dpd.dpd_ls_solve_ws_size(K)
        self.sws = torch.empty(self.sws_bytes, dtype=torch.uint8, device=dev)
        self.h = torch.zeros(K, dtype=torch.complex64, device=dev)
        self.info = torch.zeros((), dtype=torch.int32, device=dev)

    def transmit(self):
        """Predistorter then PA into the resident buffers: (z, y)."""
        st = _dpd.current_stream()
        R, N = self.rows, self.n
        _dpd.dpd_apply_rows(self.plan.handle, st, self.x.data_ptr(), self.z.data_ptr(), R, N, N)
        _dpd.dpd_apply_rows(self.pa.iq.handle, st, self.z.data_ptr(), self.u.data_ptr(), R, N, N)
        _dpd.dpd_apply_rows(self.pa.pa.handle, st, self.u.data_ptr(), self.y.data_ptr(), R, N, N)
        return self.z, self.y

    def step(self):
        """One iteration: fit the postdistorter (y / G -> z) and copy it into
        the predistorter.  Returns the device info flag of the solve; when it
        is not 0 (the normal equations were not positive definite) the
        predistorter keeps its previous coefficients."""
        z, y = self.transmit()
        st = _dpd.current_stream()
        K = self.plan.K
        _dpd.dpd_ls_normal(self.plan.handle, st, y.data_ptr(), z.data_ptr(), self.rows, self.n, self.n,
                           1.0 / self.pa.gain, self.ws.data_ptr(), self.ws_bytes, self.A.data_ptr(),
                           self.b.data_ptr())
        _dpd.dpd_ls_solve(st, K, self.A.data_ptr(), self.b.data_ptr(), self.ridge, self.sws.data_ptr(),
                          self.sws_bytes, self.h.data_ptr(), self.info.data_ptr())
        # copied into the predistorter only when the solve succeeded (info == 0)
        _dpd.dpd_set_coeffs_device_if(self.plan.handle, self.h.data_ptr(), self.info.data_ptr(), st)
        return self.info

    def nmse_db(self) -> float:
        """Linearization error 10 log10(sum |y/G - x|^2 / sum |x|^2) of the
        current predistorter (a host-side metric)."""
        import torch

        _, y = self.transmit()
        e = (y / self.pa.gain - self.x).abs().pow(2).sum()
        return float(10 * torch.log10(e / self.x.abs().pow(2).sum()).item())

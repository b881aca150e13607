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

    x: complex64 GPU tensor (rows x n or 1-D) of transmit samples.  ridge: the
    diagonal loading of the normal equations, relative to their mean diagonal.
    """

    def __init__(self, x, main_orders, conj_orders, L, ridge=1e-9, pa=None):
        self.x = x
        self.plan = _dpd.Plan(main_orders, conj_orders, L,
                              identity_coeffs(len(main_orders), len(conj_orders), L))
        self.pa = pa if pa is not None else _pa.SyntheticPA()
        self.ridge = float(ridge)
        self.h = None
        self.info = None

    def transmit(self):
        """Predistorter then PA: (z, y)."""
        z = self.plan.apply(self.x)
        _, y = self.pa.forward(z)
        return z, y

    def step(self):
        """One iteration: fit the postdistorter (y / G -> z) and copy it into
        the predistorter.  Returns the device info flag of the solve."""
        z, y = self.transmit()
        A, b = self.plan.ls_normal(y, z, y_scale=1.0 / self.pa.gain)
        self.h, self.info = _dpd.ls_solve(A, b, self.ridge)
        self.plan.set_coeffs(self.h)
        return self.info

    def nmse_db(self) -> float:
        """Linearization error 10 log10(sum |y/G - x|^2 / sum |x|^2) of the
        current predistorter (a host-side metric)."""
        import torch

        _, y = self.transmit()
        e = (y / self.pa.gain - self.x).abs().pow(2).sum()
        return float(10 * torch.log10(e / self.x.abs().pow(2).sum()).item())

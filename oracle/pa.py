"""FP64 statement of the fixed synthetic transmitter -- TEST INFRASTRUCTURE ONLY.

Written independently of the library's copy: I/Q imbalance + LO leakage
u = mu z + nu conj(z) + c_LO (amplitude 1.05, phase 3 degrees, c_LO = 0.01
e^{j pi/4}), then a memory PA y_n = 10 sum_{p in {1,3,5}} sum_{k<3} alpha_p
beta_k |u_{n-k}|^{p-1} u_{n-k} with alpha_p from Eq. (3) (section 4) and
beta = [1, -0.08+0.04j, 0.02-0.01j].  The chain loss is
E = mean |y/10 - x|^2, and ``chain_gradient`` back-propagates it through the
oracle's own forward and adjoint functions.
"""
from __future__ import annotations

import numpy as np


def _iq():
    a, ph = 1.05, np.pi * 3.0 / 180.0
    mu = 0.5 * (1.0 + a * (np.cos(ph) - 1j * np.sin(ph)))
    nu = 0.5 * (1.0 - a * (np.cos(ph) + 1j * np.sin(ph)))
    lo = 0.01 * (np.cos(np.pi / 4) + 1j * np.sin(np.pi / 4))
    return ([1], [1], 1, np.array([mu, nu, lo]))


def _pa():
    alpha = [0.9490 - 0.0197j, 0.4885 + 0.1071j, -1.0156 - 0.0474j]   # Eq. (3)
    beta = [1.0, -0.08 + 0.04j, 0.02 - 0.01j]
    h = np.zeros(3 * 3 + 1, dtype=np.complex128)
    for i in range(3):
        for k in range(3):
            h[i * 3 + k] = 10.0 * alpha[i] * beta[k]
    return ([1, 3, 5], [], 3, h)


def stages(as_complex64=True):
    """(orders, orders, L, coeffs) of both stages; coefficients rounded to
    complex64 when the GPU receives them in that precision."""
    out = []
    for mo, co, L, h in (_iq(), _pa()):
        out.append((mo, co, L, h.astype(np.complex64) if as_complex64 else h))
    return out


def chain_loss_and_gradient(orc, x_rows, dpd_orders, L, coeffs):
    """FP64 loss E and dE/dcoeffs (section 2.2 layout) of the whole chain."""
    (iq_mo, iq_co, iq_L, iq_h), (pa_mo, pa_co, pa_L, pa_h) = stages()
    mo, co = dpd_orders
    total = x_rows.size
    E = 0.0
    g = 0
    for x in x_rows:
        z = orc.forward(x, mo, co, L, coeffs)
        u = orc.forward(z, iq_mo, iq_co, iq_L, iq_h)
        y = orc.forward(u, pa_mo, pa_co, pa_L, pa_h)
        r = y / 10.0 - x.astype(np.complex128)
        E += float(np.sum(np.abs(r) ** 2))
        gy = (2.0 / 10.0 / total) * r
        gu, _ = orc.backward(u, pa_mo, pa_co, pa_L, pa_h, gy, want_dcoef=False)
        gz, _ = orc.backward(z, iq_mo, iq_co, iq_L, iq_h, gu, want_dcoef=False)
        _, gc = orc.backward(x, mo, co, L, coeffs, gz, want_dx=False)
        g = g + gc
    return E / total, g

"""Fixed synthetic transmitter model used to learn predistorter coefficients.

Chain for an input z (the predistorter output):
  1. I/Q modulator imbalance and LO leakage:  u = mu z + nu conj(z) + c_LO,
     mu = (1 + g e^{-j phi}) / 2,  nu = (1 - g e^{+j phi}) / 2,
     g = 1.05 (amplitude), phi = 3 degrees, c_LO = 0.01 e^{j pi/4};
  2. PA with memory:  y_n = G sum_{p in {1,3,5}} sum_{k<3} alpha_p beta_k
     |u_{n-k}|^{p-1} u_{n-k},  G = 10, alpha_p = the 5th-order WARP PA model of
     Eq. (3) (section 4), beta = [1, -0.08+0.04j, 0.02-0.01j].
Both stages are APH maps themselves (stage 1: order 1 in both branches, one
tap, DC term; stage 2: orders {1,3,5} main branch only, three taps), so they
run on the same libdpd forward and adjoint kernels as the predistorter.
"""
from __future__ import annotations

import numpy as np

from . import dpd as _dpd

# Eq. (3), section 4: memoryless 5th-order PA model of the WARP v3 board
ALPHA = {1: 0.9490 - 0.0197j, 3: 0.4885 + 0.1071j, 5: -1.0156 - 0.0474j}
BETA = (1.0, -0.08 + 0.04j, 0.02 - 0.01j)
GAIN = 10.0
IQ_AMPLITUDE = 1.05
IQ_PHASE_DEG = 3.0
LO_LEAKAGE = 0.01 * np.exp(1j * np.pi / 4)

IQ_ORDERS = ([1], [1], 1)
PA_ORDERS = ([1, 3, 5], [], 3)


def iq_coeffs() -> np.ndarray:
    phi = np.deg2rad(IQ_PHASE_DEG)
    mu = (1 + IQ_AMPLITUDE * np.exp(-1j * phi)) / 2
    nu = (1 - IQ_AMPLITUDE * np.exp(1j * phi)) / 2
    return np.array([mu, nu, LO_LEAKAGE], dtype=np.complex64)


def pa_coeffs() -> np.ndarray:
    taps = [GAIN * ALPHA[p] * b for p in (1, 3, 5) for b in BETA]
    return np.array(taps + [0.0], dtype=np.complex64)


class SyntheticPA:
    """The two stages as libdpd plans."""

    def __init__(self):
        self.iq = _dpd.Plan(*IQ_ORDERS, iq_coeffs())
        self.pa = _dpd.Plan(*PA_ORDERS, pa_coeffs())
        self.gain = GAIN

    def forward(self, z):
        u = self.iq.apply(z)
        return u, self.pa.apply(u)

"""FP64 indirect-learning iteration composed from oracle calls -- TEST INFRASTRUCTURE ONLY.

Section 2.2 estimates the predistorter by least squares in an indirect-learning
architecture: a postdistorter with the predistorter's basis is fitted from the
PA output divided by the PA gain (its input) to the PA input (its target), and
its coefficients become the predistorter.  One iteration here:

  1. transmit: z = predistorter(x; h), then the transmitter stages of
     ``oracle/pa.py`` (I/Q imbalance + LO leakage, memory PA): y;
  2. normal equations of the postdistorter: A = Psi^H Psi, b = Psi^H z with Psi
     the Eq. (2) basis of y / gain (``oracle_ls_normal``);
  3. solve (A + delta I) h' = b in FP64 (numpy), delta = ridge * mean(Re diag A);
  4. h <- h'.

The linearization error of a predistorter is
10 log10(sum |y/gain - x|^2 / sum |x|^2) over the whole input.  Everything runs
in complex128; the stages may be replaced (``stages``) to pin the iteration on
transmitters with a known inverse.
"""
from __future__ import annotations

import numpy as np

from . import pa as _pa

GAIN = 10.0


def transmit(orc, x, orders, L, h, stages=None):
    """(z, y): the predistorter output and the transmitter output for rows x."""
    st = _pa.stages() if stages is None else stages
    mo, co = orders
    x = np.atleast_2d(x)
    zs, ys = [], []
    for row in x:
        z = orc.forward(row, mo, co, L, h)
        u = z
        for smo, sco, sL, sh in st:
            u = orc.forward(u, smo, sco, sL, sh)
        zs.append(z)
        ys.append(u)
    return np.stack(zs), np.stack(ys)


def normal_equations(orc, y, z, orders, L, gain=GAIN):
    """A, b of the postdistorter fit, summed over rows (zero history per row)."""
    mo, co = orders
    A = b = 0
    for yr, zr in zip(np.atleast_2d(y), np.atleast_2d(z)):
        Ar, br = orc.ls_normal(yr / gain, mo, co, L, zr)
        A = A + Ar
        b = b + br
    return A, b


def solve(A, b, ridge):
    delta = ridge * float(np.mean(np.real(np.diag(A))))
    return np.linalg.solve(A + delta * np.eye(A.shape[0]), b)


def iteration(orc, x, orders, L, h, ridge=1e-9, gain=GAIN, stages=None):
    """One indirect-learning iteration from coefficients h: the new coefficients."""
    z, y = transmit(orc, x, orders, L, h, stages)
    A, b = normal_equations(orc, y, z, orders, L, gain)
    return solve(A, b, ridge)


def linearization_nmse_db(orc, x, orders, L, h, gain=GAIN, stages=None) -> float:
    _, y = transmit(orc, x, orders, L, h, stages)
    x = np.atleast_2d(np.asarray(x, dtype=np.complex128))
    e = np.sum(np.abs(y / gain - x) ** 2)
    return float(10.0 * np.log10(e / np.sum(np.abs(x) ** 2)))


def run(orc, x, orders, L, h0, iters, ridge=1e-9, gain=GAIN, stages=None):
    """Linearization error before and after each of ``iters`` iterations, and
    the coefficients after each iteration."""
    h = np.asarray(h0, dtype=np.complex128)
    errs = [linearization_nmse_db(orc, x, orders, L, h, gain, stages)]
    hs = []
    for _ in range(iters):
        h = iteration(orc, x, orders, L, h, ridge, gain, stages)
        hs.append(h)
        errs.append(linearization_nmse_db(orc, x, orders, L, h, gain, stages))
    return errs, hs

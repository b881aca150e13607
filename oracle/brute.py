"""Brute-force routes to the predistorter output -- TEST INFRASTRUCTURE ONLY.

``psi_matrix`` builds the basis matrix of Eq. (2) (section 2.2) literally: one
zero-filled (M+L-1) x L Toeplitz element matrix per main-branch order, the
complex conjugate of one per conjugate-branch order, and a column of ones for c,
concatenated side by side.  ``forward_matrix`` then takes the first M rows of
Psi @ h.  This is a different code route from the C oracle (matrix product of a
library-built Toeplitz matrix, powers by ``numpy.abs(x) ** (p-1)``), used to pin
the oracle's tap direction, zero pre-history and coefficient layout.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def basis(x: np.ndarray, p: int) -> np.ndarray:
    """psi_p(x) = |x|^(p-1) x (section 2.1, monomial form)."""
    x = np.asarray(x, dtype=np.complex128)
    return np.abs(x) ** (p - 1) * x


def element_matrix(x: np.ndarray, p: int, L: int) -> np.ndarray:
    """Psi_p of Eq. (2): (M+L-1) x L, column k is psi_p(x) delayed by k samples."""
    v = basis(x, p)
    M = v.size
    col = np.concatenate([v, np.zeros(L - 1, dtype=np.complex128)])
    row = np.zeros(L, dtype=np.complex128)
    row[0] = v[0] if M else 0.0
    return scipy.linalg.toeplitz(col, row)


def psi_matrix(x, main_orders, conj_orders, L: int) -> np.ndarray:
    """Psi = [Psi_1 ... Psi_P  conj(Psi_1) ... conj(Psi_Q)  1], shape (M+L-1) x K."""
    x = np.asarray(x, dtype=np.complex128)
    blocks = [element_matrix(x, p, L) for p in main_orders]
    blocks += [np.conj(element_matrix(x, q, L)) for q in conj_orders]
    blocks.append(np.ones((x.size + L - 1, 1), dtype=np.complex128))
    return np.concatenate(blocks, axis=1)


def forward_matrix(x, main_orders, conj_orders, L: int, coeffs, hist=None) -> np.ndarray:
    """z = first M rows of Psi @ h; with a history, the history is prepended and
    its L-1 outputs are dropped."""
    x = np.asarray(x, dtype=np.complex128)
    h = np.asarray(coeffs, dtype=np.complex128)
    if hist is not None:
        full = np.concatenate([np.asarray(hist, dtype=np.complex128), x])
        z = psi_matrix(full, main_orders, conj_orders, L) @ h
        return z[L - 1:L - 1 + x.size]
    z = psi_matrix(x, main_orders, conj_orders, L) @ h
    return z[:x.size]

"""Accuracy metrics of the GPU path against the FP64 oracle.

NMSE_dB  = 10 log10( sum |zhat - z|^2 / sum |z|^2 )           gate: <= -110 dB
max_rel  = max_n |zhat_n - z_n| / max(|z_n|, rms(z))            gate: <= 2e-5
(the rms floor keeps near-zero samples of an OFDM-like signal from dominating).
"""
import numpy as np

NMSE_DB_MAX = -110.0
MAX_REL_MAX = 2e-5


def nmse_db(zhat, z) -> float:
    zhat = np.asarray(zhat, dtype=np.complex128)
    z = np.asarray(z, dtype=np.complex128)
    num = np.sum(np.abs(zhat - z) ** 2)
    den = np.sum(np.abs(z) ** 2)
    if num == 0:
        return -np.inf
    return float(10.0 * np.log10(num / den))


def max_rel(zhat, z) -> float:
    zhat = np.asarray(zhat, dtype=np.complex128)
    z = np.asarray(z, dtype=np.complex128)
    if z.size == 0:
        return 0.0
    rms = np.sqrt(np.mean(np.abs(z) ** 2))
    den = np.maximum(np.abs(z), rms)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(np.abs(zhat - z) / den))


def assert_parity(zhat, z, what=""):
    nm = nmse_db(zhat, z)
    mr = max_rel(zhat, z)
    assert nm <= NMSE_DB_MAX and mr <= MAX_REL_MAX, "%s: NMSE %.1f dB, max rel %.3g" % (what, nm, mr)
    return nm, mr

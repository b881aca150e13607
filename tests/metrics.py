"""Accuracy metrics of the GPU path against the FP64 oracle.

NMSE_dB  = 10 log10( sum |zhat - z|^2 / sum |z|^2 )           gate: <= -110 dB
max_rel  = max_n |zhat_n - z_n| / max(|z_n|, rms(z))            gate: <= 2e-5
(the rms floor keeps near-zero samples of an OFDM-like signal from dominating).
"""
import numpy as np

NMSE_DB_MAX = -110.0
MAX_REL_MAX = 2e-5
# Coefficient gradients (K entries): each entry within 1e-5 of its FP64 value,
# relative to max(|g_k|, rms(g)) (the floor keeps entries that nearly cancel
# from demanding more than FP32 accumulation gives), and the relative L2 error
# of the whole vector within 1e-5.
DCOEF_ENTRY_MAX = 1e-5
DCOEF_REL_MAX = 1e-5


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


def entry_err(g, ref) -> float:
    """max_k |g_k - ref_k| / max(|ref_k|, rms(ref))."""
    g = np.asarray(g, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    if ref.size == 0:
        return 0.0
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    den = np.maximum(np.abs(ref), rms)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(np.abs(g - ref) / den))


def assert_dcoef(g, ref, what="", entry_max=DCOEF_ENTRY_MAX, rel_max=DCOEF_REL_MAX):
    """Coefficient-gradient parity: every entry and the vector norm."""
    g = np.asarray(g, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    ee = entry_err(g, ref)
    rel = float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300))
    assert ee <= entry_max and rel <= rel_max, "%s: dcoef entry err %.3g, rel L2 %.3g" % (what, ee, rel)
    return ee, rel


# Normal equations of the least-squares fit: errors after the diagonal scaling
# S = diag(A)^(-1/2), where every exact entry of S A S and of S b / |t| is at
# most 1 (Cauchy-Schwarz).
LS_REL_MAX = 2e-5


def ls_errors(A, b, Ar, br, t2):
    """Relative Frobenius errors of S A S and S b, and the largest entry errors
    of S A S and S b / |t| (t2 = sum |t|^2)."""
    A, b, Ar, br = (np.asarray(v, dtype=np.complex128) for v in (A, b, Ar, br))
    dg = np.abs(np.real(np.diag(Ar)))
    d = np.where(dg > 0, 1.0 / np.sqrt(np.where(dg > 0, dg, 1.0)), 1.0)   # all-zero columns (taps past n)
    S = np.outer(d, d)
    ea = np.linalg.norm((A - Ar) * S) / np.linalg.norm(Ar * S)
    eb = np.linalg.norm((b - br) * d) / np.linalg.norm(br * d)
    ma = np.max(np.abs(A - Ar) * S)
    mb = np.max(np.abs(b - br) * d) / np.sqrt(t2)
    return float(ea), float(eb), float(ma), float(mb)

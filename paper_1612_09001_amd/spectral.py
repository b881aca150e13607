"""Spectral regrowth metric (the synthetic analog of the paper's spectrum
measurements, section 5.2): how much power the PA's nonlinearity spreads from
the occupied band into the unoccupied guard band, before and after
predistortion.

The OFDM-like test signals occupy bins +-1..+-600 of a 2048-point symbol
(|f| <= 0.293 cycles/sample), so at this sample rate a full adjacent channel
does not fit below Nyquist; the metric is therefore the mean power spectral
density in the guard band (0.31 <= |f| <= 0.5) relative to the mean density
in the occupied band, in dB (Welch estimate, Hann window, 50 % overlap).  The
generators concatenate symbols without a cyclic prefix or windowing, so a
signal's own splatter sits near -33 dB; ``distortion_regrowth_db`` measures
the guard-band density of the distortion y - x instead, where it cancels.
A host-side measurement (numpy), not part of the GPU path.
"""
from __future__ import annotations

import numpy as np

IN_BAND = 600 / 2048          # occupied band edge of the OFDM-like generators (cycles/sample)
GUARD = (0.31, 0.5)           # guard band used for the regrowth (cycles/sample)


def psd(x, nfft: int = 2048):
    """Welch power spectral density (Hann window, 50 % overlap): (f, P) with f
    in cycles/sample, ascending from -0.5."""
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    if x.size < nfft:
        raise ValueError("need at least nfft samples")
    w = np.hanning(nfft)
    hop = nfft // 2
    segs = (x.size - nfft) // hop + 1
    acc = np.zeros(nfft)
    for i in range(segs):
        acc += np.abs(np.fft.fft(x[i * hop:i * hop + nfft] * w)) ** 2
    p = acc / (segs * np.sum(w ** 2))
    f = np.fft.fftfreq(nfft)
    order = np.argsort(f)
    return f[order], p[order]


def _band_means(x, nfft, in_band, guard):
    f, p = psd(x, nfft)
    a = np.abs(f)
    return np.mean(p[(a > 1.0 / nfft) & (a <= in_band)]), np.mean(p[(a >= guard[0]) & (a <= guard[1])])


def regrowth_db(x, nfft: int = 2048, in_band: float = IN_BAND, guard=GUARD) -> float:
    """Mean PSD in the guard band over mean PSD in the occupied band, dB (of
    one signal; includes the signal's own splatter)."""
    inb, oob = _band_means(x, nfft, in_band, guard)
    return float(10 * np.log10(oob / inb))


def distortion_regrowth_db(y, x, nfft: int = 2048, in_band: float = IN_BAND, guard=GUARD) -> float:
    """Guard-band PSD of the distortion y - x relative to the occupied-band PSD
    of x, dB: the spectral regrowth of a chain that should reproduce x (y =
    PA output / gain), free of x's own splatter, which cancels in y - x."""
    y = np.asarray(y, dtype=np.complex128).reshape(-1)
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    inb, _ = _band_means(x, nfft, in_band, guard)
    _, oob = _band_means(y - x, nfft, in_band, guard)
    return float(10 * np.log10(oob / inb))

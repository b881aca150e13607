"""Spectral regrowth metric (the synthetic analog of the paper's spectrum
measurements, section 5.2 / Fig. 8): how much power the PA's nonlinearity
spreads from the occupied band into unoccupied spectrum, before and after
predistortion, for the single-carrier and the non-contiguous two-carrier
signals.

Bands are sets of |f| intervals in cycles/sample:

* ``SINGLE_CARRIER``: the OFDM-like generator occupies bins +-1..+-600 of a
  2048-point symbol (|f| <= 0.293), so a full adjacent channel does not fit
  below Nyquist; the measured band is the guard band 0.31 <= |f| <= 0.5.
* ``TWO_CARRIER``: two carriers of bins +-1..+-300 (half width 0.146) at
  +-0.3 occupy 0.154 <= |f| <= 0.446; the measured band is the gap between
  the carriers, |f| <= 0.13, where the third-order intermodulation products
  land (2 f1 - f2 = +-0.9, i.e. -+0.1 after aliasing), as in the
  non-contiguous carrier-aggregation measurement of Fig. 8(b).

The metric is the mean power spectral density in the measured band relative
to the mean density in the occupied band, in dB (Welch estimate, Hann window,
50 % overlap).  The generators concatenate symbols without a cyclic prefix or
windowing, so a signal's own splatter sits near -33 dB outside its band;
``distortion_regrowth_db`` measures the out-of-band density of the
distortion y - x instead, where that splatter cancels.  A host-side
measurement (numpy), not part of the GPU path.
"""
from __future__ import annotations

import numpy as np

_HALF1 = 600 / 2048           # occupied half width of the single-carrier generator
_HALF2 = 300 / 2048           # occupied half width of each carrier of the two-carrier generator

SINGLE_CARRIER = {"in_band": ((0.0, _HALF1),), "out_band": ((0.31, 0.5),)}
TWO_CARRIER = {"in_band": ((0.3 - _HALF2, 0.3 + _HALF2),), "out_band": ((0.0, 0.13),)}

# kept for callers of the single-carrier constants
IN_BAND = _HALF1
GUARD = SINGLE_CARRIER["out_band"][0]


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


def _mask(f, bands, nfft):
    a = np.abs(f)
    m = np.zeros(f.size, dtype=bool)
    for lo, hi in bands:
        m |= (a >= lo) & (a <= hi)
    return m & (a > 1.0 / nfft)    # the DC bin is empty in every generator


def _band_means(x, nfft, bands):
    f, p = psd(x, nfft)
    return np.mean(p[_mask(f, bands["in_band"], nfft)]), np.mean(p[_mask(f, bands["out_band"], nfft)])


def regrowth_db(x, nfft: int = 2048, bands=SINGLE_CARRIER) -> float:
    """Mean PSD in the measured band over mean PSD in the occupied band, dB
    (of one signal; includes the signal's own splatter)."""
    inb, oob = _band_means(x, nfft, bands)
    return float(10 * np.log10(oob / inb))


def distortion_regrowth_db(y, x, nfft: int = 2048, bands=SINGLE_CARRIER) -> float:
    """Out-of-band PSD of the distortion y - x relative to the occupied-band
    PSD of x, dB: the spectral regrowth of a chain that should reproduce x
    (y = PA output / gain), free of x's own splatter, which cancels in y - x."""
    y = np.asarray(y, dtype=np.complex128).reshape(-1)
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    inb, _ = _band_means(x, nfft, bands)
    _, oob = _band_means(y - x, nfft, bands)
    return float(10 * np.log10(oob / inb))

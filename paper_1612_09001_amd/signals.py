"""Seeded synthetic inputs for the predistorter: I/Q streams and coefficient sets.

This module only *draws* inputs. It holds none of the predistorter's arithmetic
(no basis functions, no filtering), so the GPU path and the FP64 oracle can both
be fed from it without sharing any of the method's code.

Stand-ins for the paper's workloads (section 5.2 uses one 10 MHz LTE uplink
carrier and two non-contiguous 3 MHz carriers; no waveform files are given):

* ``ofdm_16qam``   - OFDM-like stream: 16-QAM on 1200 of 2048 subcarriers
  (bins +-1..+-600, DC and the band edge empty), one IFFT per 2048-sample
  symbol, no cyclic prefix, concatenated and cut to ``n`` samples, scaled in
  double precision to RMS 0.25, then rounded to complex64.
* ``two_carrier``  - two independent OFDM-like carriers of 600 subcarriers
  each (bins +-1..+-300), shifted to +-0.3 cycles/sample, summed, RMS 0.25.
* ``aph_coeffs``   - a coefficient vector in the stacked layout of section 2.2
  (main-branch filters order-major then tap, conjugate-branch filters, then the
  DC/LO term c); taps drawn CN(0,1) * 10^(-(p-1)/2), c drawn 0.01 * CN(0,1).

Every draw comes from ``numpy.random.SeedSequence(161209001, spawn_key=...)``
so that a (config, stream) pair names one reproducible input.
"""
from __future__ import annotations

import numpy as np

ROOT_SEED = 161209001
NFFT = 2048
RMS = 0.25

# spawn-key namespaces: inputs and coefficients never share a stream of draws
_KEY_SIGNAL = 0
_KEY_COEFF = 1
_KEY_GRAD = 2
_KEY_BATCH = 3


def rng(config_id: int, stream_id: int = 0, kind: int = _KEY_SIGNAL) -> np.random.Generator:
    """Generator for one (config, stream, kind) triple."""
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(int(config_id), int(stream_id), int(kind)))
    return np.random.default_rng(ss)


def _qam16(g: np.random.Generator, shape) -> np.ndarray:
    i = g.integers(0, 4, size=shape)
    q = g.integers(0, 4, size=shape)
    return ((2 * i - 3) + 1j * (2 * q - 3)) / np.sqrt(10.0)


def _ofdm_symbols(g: np.random.Generator, n: int, half_width: int) -> np.ndarray:
    """Complex128 OFDM-like time signal with active bins +-1..+-half_width."""
    nsym = -(-n // NFFT)
    spec = np.zeros((nsym, NFFT), dtype=np.complex128)
    spec[:, 1:half_width + 1] = _qam16(g, (nsym, half_width))
    spec[:, NFFT - half_width:] = _qam16(g, (nsym, half_width))
    t = np.fft.ifft(spec, axis=1).reshape(-1)[:n]
    return t


def _scale_rms(t: np.ndarray, rms: float) -> np.ndarray:
    if t.size == 0:
        return t.astype(np.complex64)
    cur = np.sqrt(np.mean(np.abs(t) ** 2))
    return (t * (rms / cur)).astype(np.complex64)


def ofdm_16qam(n: int, config_id: int = 1, stream_id: int = 0, rms: float = RMS) -> np.ndarray:
    """OFDM-like 16-QAM stream, complex64, 1200 of 2048 subcarriers active."""
    g = rng(config_id, stream_id, _KEY_SIGNAL)
    return _scale_rms(_ofdm_symbols(g, n, 600), rms)


def two_carrier(n: int, config_id: int = 3, stream_id: int = 0, offset: float = 0.3,
                rms: float = RMS) -> np.ndarray:
    """Two non-contiguous OFDM-like carriers at +-offset cycles/sample, complex64."""
    g = rng(config_id, stream_id, _KEY_SIGNAL)
    a = _ofdm_symbols(g, n, 300)
    b = _ofdm_symbols(g, n, 300)
    idx = np.arange(n, dtype=np.float64)
    ph = 2.0 * np.pi * offset * idx
    t = a * np.exp(1j * ph) + b * np.exp(-1j * ph)
    return _scale_rms(t, rms)


def num_coeffs(main_orders, conj_orders, L: int) -> int:
    """K = (|I_P| + |I_Q|) * L + 1 complex coefficients (section 2.2 stacking)."""
    return (len(main_orders) + len(conj_orders)) * L + 1


def aph_coeffs(main_orders, conj_orders, L: int, config_id: int = 1, stream_id: int = 0,
               c_scale: float = 0.01) -> np.ndarray:
    """Random stacked coefficient vector (complex64, length K).

    Layout: for each main order p (in the given order) its L taps, then for each
    conjugate order q its L taps, then c.  Tap (p, k) is CN(0,1) * 10^(-(p-1)/2).
    """
    g = rng(config_id, stream_id, _KEY_COEFF)
    out = []
    for p in list(main_orders) + list(conj_orders):
        scale = 10.0 ** (-(p - 1) / 2.0)
        w = (g.standard_normal(L) + 1j * g.standard_normal(L)) / np.sqrt(2.0)
        out.append(w * scale)
    c = (g.standard_normal() + 1j * g.standard_normal()) / np.sqrt(2.0) * c_scale
    out.append(np.array([c]))
    return np.concatenate(out).astype(np.complex64)


def identity_coeffs(main_orders, conj_orders, L: int) -> np.ndarray:
    """Coefficient vector with h_{1,0} = 1 and every other entry 0 (requires 1 in main_orders)."""
    main_orders = list(main_orders)
    if 1 not in main_orders:
        raise ValueError("identity needs order 1 in the main branch")
    K = num_coeffs(main_orders, conj_orders, L)
    h = np.zeros(K, dtype=np.complex64)
    h[main_orders.index(1) * L + 0] = 1.0
    return h


def cgauss(shape, config_id: int, stream_id: int = 0, scale: float = 1.0) -> np.ndarray:
    """CN(0, scale^2) complex64 draws (used for upstream gradients in tests)."""
    g = rng(config_id, stream_id, _KEY_GRAD)
    z = (g.standard_normal(shape) + 1j * g.standard_normal(shape)) / np.sqrt(2.0) * scale
    return z.astype(np.complex64)


def batch_specs(n_streams: int = 256, lo: int = 1 << 14, hi: int = 1 << 20, config_id: int = 4,
                pmax_choices=(5, 7, 9), L_choices=tuple(range(2, 9))):
    """Per-stream (length, P_max, L) draws for the multi-antenna batch.

    Lengths are uniform integers in [lo, hi] inclusive, P_max uniform over
    ``pmax_choices`` and L uniform over ``L_choices``.  Each stream uses odd
    orders 1..P_max in both branches plus the DC term.
    """
    g = rng(config_id, 0, _KEY_BATCH)
    lens = g.integers(lo, hi + 1, size=n_streams)
    pmax = g.choice(np.asarray(pmax_choices), size=n_streams)
    Ls = g.choice(np.asarray(L_choices), size=n_streams)
    return [(int(a), int(b), int(c)) for a, b, c in zip(lens, pmax, Ls)]


def odd_orders(pmax: int):
    return list(range(1, int(pmax) + 1, 2))

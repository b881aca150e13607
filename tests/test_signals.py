"""Seeded input generators (CPU only)."""
import numpy as np

from paper_1612_09001_amd import signals


def test_ofdm_rms_and_dtype():
    x = signals.ofdm_16qam(3 * 2048, config_id=1)
    assert x.dtype == np.complex64
    rms = np.sqrt(np.mean(np.abs(x.astype(np.complex128)) ** 2))
    assert abs(rms - 0.25) < 1e-6


def test_ofdm_spectrum_and_constellation():
    n = 4 * 2048
    x = signals.ofdm_16qam(n, config_id=1).astype(np.complex128)
    spec = np.fft.fft(x.reshape(-1, 2048), axis=1)
    active = np.zeros(2048, bool)
    active[1:601] = True
    active[2048 - 600:] = True
    inband = np.sum(np.abs(spec[:, active]) ** 2)
    outband = np.sum(np.abs(spec[:, ~active]) ** 2)
    assert outband < 1e-10 * inband
    pts = spec[:, active]
    pts = pts * (3 / np.sqrt(10.0)) / np.max(np.abs(pts.real))   # outer ring at 3/sqrt(10)
    grid = np.array([-3, -1, 1, 3]) / np.sqrt(10.0)
    d_re = np.min(np.abs(pts.real[..., None] - grid), axis=-1)
    d_im = np.min(np.abs(pts.imag[..., None] - grid), axis=-1)
    assert d_re.max() < 1e-3 and d_im.max() < 1e-3


def test_two_carrier_bands():
    n = 8 * 2048
    x = signals.two_carrier(n).astype(np.complex128)
    f = np.fft.fftfreq(n)
    p = np.abs(np.fft.fft(x)) ** 2
    near = (np.abs(f - 0.3) < 0.16) | (np.abs(f + 0.3) < 0.16)
    # symbols are cut without a cyclic prefix, so a full-length FFT leaks a little
    assert np.sum(p[~near]) < 2e-3 * np.sum(p)
    assert np.sum(p[np.abs(f) < 0.1]) < 1e-3 * np.sum(p)
    assert abs(np.sum(p[f > 0]) / np.sum(p) - 0.5) < 0.02


def test_reproducible_and_distinct():
    a = signals.ofdm_16qam(5000, config_id=1, stream_id=3)
    b = signals.ofdm_16qam(5000, config_id=1, stream_id=3)
    c = signals.ofdm_16qam(5000, config_id=1, stream_id=4)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert signals.ofdm_16qam(0).size == 0


def test_coeff_layout_and_scale():
    mo, co, L = [1, 3, 5, 7], [1, 3, 5, 7], 4
    h = signals.aph_coeffs(mo, co, L, config_id=1)
    assert h.dtype == np.complex64
    assert h.size == signals.num_coeffs(mo, co, L) == 33
    hi = signals.identity_coeffs(mo, co, L)
    assert hi[0] == 1 and np.count_nonzero(hi) == 1


def test_batch_specs():
    specs = signals.batch_specs()
    assert len(specs) == 256
    lens = np.array([s[0] for s in specs])
    assert lens.min() >= 1 << 14 and lens.max() <= 1 << 20
    assert set(s[1] for s in specs) <= {5, 7, 9}
    assert set(s[2] for s in specs) <= set(range(2, 9))
    assert specs == signals.batch_specs()


def test_table2_fixture():
    """The Table 2 configuration fixture parses to P = 5, Q = 3, L = 5 (K = 26)."""
    import os

    cfg = {}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_config.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            cfg[k] = [int(t) for t in v]
    assert cfg["main_orders"] == [1, 3, 5] and cfg["conj_orders"] == [1, 3] and cfg["L"] == [5]
    assert signals.num_coeffs(cfg["main_orders"], cfg["conj_orders"], cfg["L"][0]) == 26

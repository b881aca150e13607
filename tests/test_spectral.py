"""Spectral regrowth metric against closed forms (CPU)."""
import numpy as np

from paper_1612_09001_amd import signals, spectral


def _x():
    return signals.ofdm_16qam(1 << 17, config_id=71, rms=0.2).astype(np.complex128)


def test_white_error_matches_closed_form():
    """Error = white noise of variance v: guard-band density v against the
    in-band density P_x / (1200/2048) of the OFDM-like signal."""
    x = _x()
    rng = np.random.default_rng(1)
    w = (rng.normal(size=x.size) + 1j * rng.normal(size=x.size)) * 0.01      # variance 2e-4
    ref = 10 * np.log10(2e-4 / (np.mean(np.abs(x) ** 2) / (1200 / 2048)))
    assert abs(spectral.distortion_regrowth_db(x + w, x) - ref) <= 0.3


def test_cubic_distortion_scales_20_db_per_decade():
    """y = x + a |x|^2 x: the distortion is linear in a, so its power moves
    by 20 log10 of the ratio of the coefficients."""
    x = _x()
    d1 = spectral.distortion_regrowth_db(x + 0.01 * np.abs(x) ** 2 * x, x)
    d2 = spectral.distortion_regrowth_db(x + 0.1 * np.abs(x) ** 2 * x, x)
    assert abs((d2 - d1) - 20.0) <= 0.05


def test_flat_spectrum_has_no_regrowth_contrast():
    rng = np.random.default_rng(2)
    w = rng.normal(size=1 << 17) + 1j * rng.normal(size=1 << 17)
    assert abs(spectral.regrowth_db(w)) <= 0.3


def _x2():
    return signals.two_carrier(1 << 17, config_id=72, rms=0.2).astype(np.complex128)


def test_two_carrier_white_error_closed_form():
    """Two-carrier bands: white error of variance v against the in-band density
    P_x / (2 x 600/2048) of the two carriers."""
    x = _x2()
    rng = np.random.default_rng(3)
    w = (rng.normal(size=x.size) + 1j * rng.normal(size=x.size)) * 0.01      # variance 2e-4
    ref = 10 * np.log10(2e-4 / (np.mean(np.abs(x) ** 2) / (1200 / 2048)))
    got = spectral.distortion_regrowth_db(x + w, x, bands=spectral.TWO_CARRIER)
    assert abs(got - ref) <= 0.3, (got, ref)


def test_two_carrier_intermodulation_lands_in_the_gap():
    """A cubic nonlinearity on two carriers at +-0.3 puts third-order
    intermodulation (2 f1 - f2 = -+0.1 after aliasing) into the gap between the
    carriers: the gap density of |x|^2 x is far above that of a linear error of
    the same power."""
    x = _x2()
    cub = np.abs(x) ** 2 * x
    lin = x * np.sqrt(np.mean(np.abs(cub) ** 2) / np.mean(np.abs(x) ** 2))
    d_cub = spectral.distortion_regrowth_db(x + cub, x, bands=spectral.TWO_CARRIER)
    d_lin = spectral.distortion_regrowth_db(x + lin, x, bands=spectral.TWO_CARRIER)
    assert d_cub > d_lin + 20.0, (d_cub, d_lin)


def test_two_carrier_generator_leaves_the_gap_empty():
    """The two-carrier signal itself has its occupied band where the bands say
    (its own splatter in the gap is far below the carriers)."""
    assert spectral.regrowth_db(_x2(), bands=spectral.TWO_CARRIER) <= -25.0

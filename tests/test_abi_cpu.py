"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before touching a device (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1612_09001_amd import dpd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dpd.LIB_PATH):
        pytest.skip("libdpd.so not built")
    return dpd.lib()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(dpd.EXPORTED) == declared


def test_version_and_status_strings(lib):
    assert "gfx950" in dpd.dpd_version()
    for st in range(5):
        assert dpd.dpd_status_string(st).startswith("DPD_")


def _create(mo, co, L):
    K = (len(mo) + len(co)) * L + 1
    return dpd.dpd_create(mo, co, L, np.zeros(K, np.complex64))


@pytest.mark.parametrize("mo,co,L,status", [
    ([2], [], 3, dpd.DPD_EINVAL),          # even order
    ([3, 1], [], 3, dpd.DPD_EINVAL),       # not ascending
    ([1, 1], [], 3, dpd.DPD_EINVAL),       # duplicate
    ([], [1], 3, dpd.DPD_EINVAL),          # no main branch
    ([1], [], 0, dpd.DPD_EINVAL),          # L = 0
    ([1], [], 17, dpd.DPD_EUNSUPPORTED),   # L > 16
    ([1, 17], [], 2, dpd.DPD_EUNSUPPORTED),  # order > 15
    ([-1], [], 2, dpd.DPD_EINVAL),
])
def test_create_rejects(lib, mo, co, L, status):
    with pytest.raises(dpd.DPDError) as e:
        _create(mo, co, L)
    assert e.value.status == status


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    one = (ctypes.c_int32 * 1)(1)
    assert lib.dpd_create(one, 1, None, 0, 2, None, ctypes.byref(h)) == dpd.DPD_EINVAL
    c = (ctypes.c_float * 6)()
    assert lib.dpd_create(one, 1, None, 0, 2, c, None) == dpd.DPD_EINVAL
    assert lib.dpd_apply(None, None, None, None, 10) == dpd.DPD_EINVAL
    assert lib.dpd_destroy(None) == dpd.DPD_OK
    assert lib.dpd_num_coeffs(None, None) == dpd.DPD_EINVAL
    assert lib.dpd_batch_create(None, 0, None, ctypes.byref(h)) == dpd.DPD_EINVAL
    assert lib.dpd_batch_destroy(None) == dpd.DPD_OK


def test_least_squares_argument_checks(lib):
    sz = ctypes.c_size_t()
    assert lib.dpd_ls_ws_size(None, 1, 10, ctypes.byref(sz)) == dpd.DPD_EINVAL
    assert lib.dpd_ls_normal(None, None, None, None, 1, 10, 10, ctypes.c_float(1.0), None, 0, None,
                             None) == dpd.DPD_EINVAL
    assert lib.dpd_ls_solve_ws_size(0, ctypes.byref(sz)) == dpd.DPD_EINVAL
    assert lib.dpd_ls_solve_ws_size(33, ctypes.byref(sz)) == dpd.DPD_OK
    assert sz.value == 33 * 33 * 16                 # the factor, K x K complex128
    assert lib.dpd_ls_solve_ws_size(1025, ctypes.byref(sz)) == dpd.DPD_EUNSUPPORTED
    assert lib.dpd_ls_solve(None, 0, None, None, ctypes.c_double(0.0), None, 0, None, None) == dpd.DPD_EINVAL
    fake = ctypes.c_void_p(4096)                    # never dereferenced: rejected before any launch
    assert lib.dpd_ls_solve(None, 3, fake, fake, ctypes.c_double(-1.0), fake, 1 << 20, fake,
                            fake) == dpd.DPD_EINVAL  # negative ridge
    assert lib.dpd_ls_solve(None, 3, fake, fake, ctypes.c_double(0.0), fake, 16, fake,
                            fake) == dpd.DPD_EINVAL  # workspace too small
    assert lib.dpd_ls_solve(None, 1025, fake, fake, ctypes.c_double(0.0), fake, 1 << 30, fake,
                            fake) == dpd.DPD_EUNSUPPORTED  # more rows than one wave holds


def test_batch_rejects_overlapping_streams(lib):
    """Outputs may not overlap each other or any input; inputs may be shared.
    Checked on the host before any device call (fake, never dereferenced,
    16-byte aligned addresses)."""
    base = 1 << 24

    def desc(i, o, n):
        return dpd.dpd_stream_desc(base + i, base + o, n, 1, 0, 2, 0, base)

    def create(ds):
        arr = (dpd.dpd_stream_desc * len(ds))(*ds)
        h = ctypes.c_void_p()
        st = lib.dpd_batch_create(arr, len(ds), None, ctypes.byref(h))
        if st == dpd.DPD_OK:
            lib.dpd_batch_destroy(h)
        return st

    many = [desc(0x100000 + 0x1000 * s, 0x800000 + 0x1000 * s, 512) for s in range(1000)]
    assert create([desc(0x10000, 0x20000, 100), desc(0x30000, 0x20000 + 8 * 48, 100)]) == dpd.DPD_EINVAL
    assert create([desc(0x10000, 0x20000, 100), desc(0x20000 + 8 * 99, 0x40000, 100)]) == dpd.DPD_EINVAL
    assert create(many + [desc(0x50000, 0x800000 + 0x1000 * 999 + 8 * 511, 4)]) == dpd.DPD_EINVAL
    # shared inputs and touching (not overlapping) ranges pass the check (then
    # need a device: DPD_OK on a GPU, DPD_EHIP without one)
    assert create([desc(0x10000, 0x20000, 100), desc(0x10000, 0x20000 + 8 * 100, 100)]) != dpd.DPD_EINVAL
    assert create(many) != dpd.DPD_EINVAL


def test_learning_entry_points_reject_on_the_host(lib):
    """The learning-step entry points reject missing plans, absent outputs and
    workspaces before any device call (fake, never dereferenced addresses)."""
    fake = ctypes.c_void_p(1 << 20)
    sz = ctypes.c_size_t()
    assert lib.dpd_learn_step_ws_size(None, ctypes.byref(sz)) == dpd.DPD_EINVAL
    assert lib.dpd_transmit_backward(None, None, None, None, fake, fake, fake, None, fake, 1, 256, 256, fake,
                                     1 << 20) == dpd.DPD_EINVAL
    assert lib.dpd_transmit_loss_grad(None, None, None, None, None, fake, fake, 1, 256, 256, ctypes.c_float(0.1),
                                      None, fake, fake, 1 << 20) == dpd.DPD_EINVAL
    assert lib.dpd_learn_step(None, None, None, None, fake, fake, fake, 1, ctypes.c_float(1e-3),
                              ctypes.c_float(0.9), ctypes.c_float(0.999), ctypes.c_float(1e-8), fake, fake, fake,
                              1, 256, 256, ctypes.c_float(0.1), None, None, fake, 1 << 20) == dpd.DPD_EINVAL
    for step_dev in (None, ctypes.c_void_p((1 << 20) + 2)):   # missing, misaligned
        assert lib.dpd_learn_step_dev(None, None, None, None, fake, fake, fake, step_dev, ctypes.c_float(1e-3),
                                      ctypes.c_float(0.9), ctypes.c_float(0.999), ctypes.c_float(1e-8), fake, fake,
                                      fake, 1, 256, 256, ctypes.c_float(0.1), None, None, fake,
                                      1 << 20) == dpd.DPD_EINVAL
    assert lib.dpd_set_coeffs_async(None, None, None) == dpd.DPD_EINVAL

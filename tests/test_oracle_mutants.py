"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case copies the oracle's C source to a temporary directory, plants one
plausible mistake (a dropped term, a wrong sign or index, a transposed
operand), builds that copy and runs every pin against it.  At least one pin has
to fail, which shows the pins constrain every part of the oracle they cover.
"""
import os

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.lib_path()), "dpd_oracle.c")

MUTANTS = {
    "conj_branch_not_conjugated": (
        "cmac(&fr, &fi, g[0], g[1], pr, -pi);", "cmac(&fr, &fi, g[0], g[1], pr, pi);"),
    "tap_direction_reversed": (
        "sample_at(x, hist, L, n - k, &xr, &xi);\n            psi(mo[b]",
        "sample_at(x, hist, L, n + k - (L - 1), &xr, &xi);\n            psi(mo[b]"),
    "dc_term_dropped": ("*zr = acc_r + c[0];", "*zr = acc_r;"),
    "power_off_by_one": ("i < (p - 1) / 2; ++i) r *= s;", "i <= (p - 1) / 2; ++i) r *= s;"),
    "coefficients_transposed": (
        "const double *h = coeffs + 2 * ((int64_t)b * L + k);\n            cmac(&fr",
        "const double *h = coeffs + 2 * ((int64_t)k * nm + b);\n            cmac(&fr"),
    "history_reversed": ("int64_t h = (int64_t)(L - 1) + m;", "int64_t h = -m - 1;"),
    "prehistory_not_zero": ("*re = 0.0;\n        *im = 0.0;", "*re = x[0];\n        *im = x[1];"),
    "dx_derivative_factor": ("*d_r = (double)(J + 1) * radial(p, s);", "*d_r = (double)(J) * radial(p, s);"),
    "dx_grad_not_conjugated": ("cmac(&sr, &si, Gr, -Gi, Br, Bi);", "cmac(&sr, &si, Gr, Gi, Br, Bi);"),
    "dx_conj_branch_sign": ("cmac(&Ar, &Ai, g[0], g[1], dcr, -dci);", "cmac(&Ar, &Ai, g[0], g[1], dcr, dci);"),
    "dcoef_main_not_conjugated": (
        "G[2 * t + 1], pr, -pi);   /* G conj(psi) */", "G[2 * t + 1], pr, pi);   /* G conj(psi) */"),
    "dcoef_tap_shift": ("sample_at(x, hist, L, t - k, &xr, &xi);", "sample_at(x, hist, L, t - k + 1, &xr, &xi);"),
    "dc_grad_dropped_imag": ("ai += G[2 * t + 1];", "ai += 0.0;"),
    "ls_not_conjugated": ("ii = -row[2 * i + 1];", "ii = row[2 * i + 1];"),
}


def _failures(orc):
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(orc)
        except AssertionError:
            failed.append(pin.__name__)
    return failed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation anchor must be unique: %r" % old
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    lib = oracle.build(str(src), str(tmp_path / "libmutant.so"))
    failed = _failures(oracle.Oracle(lib))
    assert failed, "no pin caught mutant %s" % name

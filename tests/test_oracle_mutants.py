"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case copies the oracle's C source to a temporary directory, plants one
plausible mistake (a dropped term, a wrong sign or index, a transposed
operand), builds that copy and runs every pin against it.  At least one pin has
to fail, which shows the pins constrain every part of the oracle they cover.
"""
import os
import types

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
    "forward_at_wrong_index": (
        "forward_one(x, hist, idx[j], main_orders", "forward_one(x, hist, j, main_orders"),
    "forward_at_drops_history": (
        "forward_one(x, hist, idx[j], main_orders", "forward_one(x, NULL, idx[j], main_orders"),
}

# Planted mistakes in the FP64 transmitter chain (oracle/pa.py), a Python
# module: each copy is executed as a module of its own and handed to the chain
# pins together with the real C oracle.
PA_SRC = os.path.join(os.path.dirname(oracle.lib_path()), "pa.py")
PA_MUTANTS = {
    "chain_gradient_scale": ("gy = (2.0 / 10.0 / total) * r", "gy = (1.0 / 10.0 / total) * r"),
    "chain_stage_order": (
        "u = orc.forward(z, iq_mo, iq_co, iq_L, iq_h)\n        y = orc.forward(u, pa_mo, pa_co, pa_L, pa_h)",
        "u = orc.forward(z, pa_mo, pa_co, pa_L, pa_h)\n        y = orc.forward(u, iq_mo, iq_co, iq_L, iq_h)"),
    "chain_nu_sign": ("nu = 0.5 * (1.0 - a *", "nu = 0.5 * (1.0 + a *"),
    "chain_row_sum_dropped": ("g = g + gc", "g = gc"),
    "chain_iq_adjoint_skipped": (
        "gz, _ = orc.backward(z, iq_mo, iq_co, iq_L, iq_h, gu, want_dcoef=False)", "gz = gu"),
    "chain_memory_taps_reversed": (
        "beta = [1.0, -0.08 + 0.04j, 0.02 - 0.01j]", "beta = [0.02 - 0.01j, -0.08 + 0.04j, 1.0]"),
}


def _failures(orc, pin_list=None, **kw):
    failed = []
    for pin in pin_list or pins.ALL_PINS:
        try:
            pin(orc, **kw)
        except AssertionError:
            failed.append(pin.__name__)
    return failed


def _module_from(text, name):
    mod = types.ModuleType(name)
    exec(compile(text, name + ".py", "exec"), mod.__dict__)
    return mod


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


def test_chain_pins_pass_on_the_real_module(orc):
    text = open(PA_SRC).read()
    assert not _failures(orc, pins.CHAIN_PINS, pa_mod=_module_from(text, "pa_copy"))


@pytest.mark.parametrize("name", sorted(PA_MUTANTS))
def test_pa_mutant_is_caught(orc, name):
    old, new = PA_MUTANTS[name]
    text = open(PA_SRC).read()
    assert text.count(old) == 1, "mutation anchor must be unique: %r" % old
    mod = _module_from(text.replace(old, new), "pa_" + name)
    failed = _failures(orc, pins.CHAIN_PINS, pa_mod=mod)
    assert failed, "no chain pin caught mutant %s" % name


# Planted mistakes in the FP64 indirect-learning iteration (oracle/ila.py).
ILA_SRC = os.path.join(os.path.dirname(oracle.lib_path()), "ila.py")
ILA_MUTANTS = {
    "ila_input_and_target_swapped": (
        "Ar, br = orc.ls_normal(yr / gain, mo, co, L, zr)", "Ar, br = orc.ls_normal(zr, mo, co, L, yr / gain)"),
    "ila_gain_not_removed": (
        "Ar, br = orc.ls_normal(yr / gain, mo, co, L, zr)", "Ar, br = orc.ls_normal(yr, mo, co, L, zr)"),
    "ila_target_is_the_input": (
        "A, b = normal_equations(orc, y, z, orders, L, gain)", "A, b = normal_equations(orc, y, x, orders, L, gain)"),
    "ila_ridge_on_the_trace": (
        "delta = ridge * float(np.mean(np.real(np.diag(A))))", "delta = ridge * float(np.sum(np.real(np.diag(A))))"),
    "ila_error_without_gain": ("e = np.sum(np.abs(y / gain - x) ** 2)", "e = np.sum(np.abs(y - x) ** 2)"),
}


def _ila_copy(text, name):
    """Execute a copy of oracle/ila.py as a module inside the oracle package
    (it imports its sibling pa.py relatively)."""
    mod = types.ModuleType("oracle." + name)
    mod.__package__ = "oracle"
    exec(compile(text, name + ".py", "exec"), mod.__dict__)
    return mod


def test_ila_pins_pass_on_the_real_module(orc):
    assert not _failures(orc, pins.ILA_PINS, ila_mod=_ila_copy(open(ILA_SRC).read(), "ila_copy"))


@pytest.mark.parametrize("name", sorted(ILA_MUTANTS))
def test_ila_mutant_is_caught(orc, name):
    old, new = ILA_MUTANTS[name]
    text = open(ILA_SRC).read()
    assert text.count(old) == 1, "mutation anchor must be unique: %r" % old
    failed = _failures(orc, pins.ILA_PINS, ila_mod=_ila_copy(text.replace(old, new), "ila_" + name))
    assert failed, "no indirect-learning pin caught mutant %s" % name

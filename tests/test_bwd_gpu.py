"""Backward (adjoint) kernels on the GPU against the FP64 oracle gradient,
finite differences on the GPU, and bitwise run-to-run determinism."""
import numpy as np
import pytest

from metrics import assert_dcoef, assert_parity, nmse_db
from paper_1612_09001_amd import signals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def dpd(torch):
    from paper_1612_09001_amd import dpd as d

    d.lib()
    return d


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def _check(torch, dpd, orc, x, G, mo, co, L, h, rows=None, what=""):
    plan = dpd.Plan(mo, co, L, h)
    xd, gd = _dev(torch, x), _dev(torch, G)
    gx, gc = plan.backward(xd, gd)
    torch.cuda.synchronize()
    gx = gx.cpu().numpy()
    gc = gc.cpu().numpy()
    if x.ndim == 1:
        rx, rc = orc.backward(x, mo, co, L, h, G)
    else:
        rx = np.zeros_like(x, dtype=np.complex128)
        rc = 0
        for r in range(x.shape[0]):
            a, b = orc.backward(x[r], mo, co, L, h, G[r])
            rx[r] = a
            rc = rc + b
    assert_parity(gx.reshape(-1), rx.reshape(-1), "dx " + what)
    assert_dcoef(gc, rc, "dcoef " + what)
    return gx, gc


SHAPES = [
    ([1], [], 1), ([1, 3, 5], [1, 3], 5), ([1, 3, 5, 7], [1, 3, 5, 7], 4), ([1, 5], [3], 3),
    ([1, 3, 5, 7], [1, 3, 5, 7], 6), ([1, 3, 5, 7, 9], [1, 3, 5, 7, 9], 8),
    ([1, 3, 5, 7, 9, 11, 13, 15], [1, 3], 8),
    ([1, 3, 5], [1], 11),                      # generic kernels (L > 8)
]
LENGTHS = [1, 2, 7, 255, 256, 257, 1023, 1024, 1025, 5000]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "P%d_Q%d_L%d" % (max(s[0]), max(s[1]) if s[1] else 0, s[2]))
def test_ragged_lengths(torch, dpd, orc, shape):
    mo, co, L = shape
    h = signals.aph_coeffs(mo, co, L, config_id=80, stream_id=L)
    for n in LENGTHS:
        x = signals.ofdm_16qam(n, config_id=80, stream_id=n)
        G = signals.cgauss(n, config_id=80, stream_id=n)
        _check(torch, dpd, orc, x, G, mo, co, L, h, what="%s n=%d" % (shape, n))


def test_rows_and_unaligned(torch, dpd, orc):
    mo, co, L = [1, 3, 5, 7], [1, 3, 5, 7], 6
    h = signals.aph_coeffs(mo, co, L, config_id=81)
    rows, n = 7, 3001
    x = np.stack([signals.ofdm_16qam(n, config_id=81, stream_id=r) for r in range(rows)])
    G = signals.cgauss((rows, n), config_id=81)
    _check(torch, dpd, orc, x, G, mo, co, L, h, what="rows odd ld")
    x2 = np.stack([signals.ofdm_16qam(3000, config_id=81, stream_id=r) for r in range(rows)])
    G2 = signals.cgauss((rows, 3000), config_id=82)
    _check(torch, dpd, orc, x2, G2, mo, co, L, h, what="rows even ld")


def test_partial_requests(torch, dpd, orc):
    """Only dx, only dcoef, and device coefficients that override the plan's."""
    mo, co, L = [1, 3, 5], [1, 3], 5
    h = signals.aph_coeffs(mo, co, L, config_id=83)
    n = 20000
    x = signals.ofdm_16qam(n, config_id=83)
    G = signals.cgauss(n, config_id=83)
    rx, rc = orc.backward(x, mo, co, L, h, G)
    plan = dpd.Plan(mo, co, L, np.zeros_like(h))
    gx, gc = plan.backward(_dev(torch, x), _dev(torch, G), coeffs=_dev(torch, h), want_dcoeffs=False)
    assert gc is None
    assert_parity(gx.cpu().numpy(), rx)
    gx, gc = plan.backward(_dev(torch, x), _dev(torch, G), want_dx=False)
    assert gx is None
    assert_dcoef(gc.cpu().numpy(), rc, "dcoef only")


def test_empty_gives_zero_gradient(torch, dpd):
    mo, co, L = [1, 3], [1], 3
    plan = dpd.Plan(mo, co, L, signals.aph_coeffs(mo, co, L, config_id=84))
    x = torch.zeros(0, dtype=torch.complex64, device="cuda")
    gx, gc = plan.backward(x, x)
    assert gx.numel() == 0 and torch.all(gc == 0)


def test_deterministic(torch, dpd):
    mo = co = [1, 3, 5, 7]
    L = 6
    h = signals.aph_coeffs(mo, co, L, config_id=85)
    plan = dpd.Plan(mo, co, L, h)
    x = _dev(torch, signals.ofdm_16qam(1 << 20, config_id=85))
    G = _dev(torch, signals.cgauss(1 << 20, config_id=85))
    a = [t.cpu().numpy() for t in plan.backward(x, G)]
    b = [t.cpu().numpy() for t in plan.backward(x, G)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_gpu_finite_differences(torch, dpd):
    """Central differences of E = Re sum conj(W) z computed from GPU forward
    calls (FP32) agree with the GPU coefficient gradient.  E is linear in the
    coefficients, so a large step (0.5) has no truncation error and keeps the
    FP32 rounding noise of E small against the difference."""
    mo, co, L = [1, 3, 5], [1, 3], 4
    h = signals.aph_coeffs(mo, co, L, config_id=86).astype(np.complex128)
    n = 50000
    x = signals.ofdm_16qam(n, config_id=86)
    W = signals.cgauss(n, config_id=86)
    xd = _dev(torch, x)
    plan = dpd.Plan(mo, co, L, h.astype(np.complex64))
    _, gc = plan.backward(xd, _dev(torch, W), want_dx=False)
    gc = gc.cpu().numpy()

    def E(hh):
        plan.set_coeffs(hh.astype(np.complex64))
        z = plan.apply(xd).cpu().numpy().astype(np.complex128)
        return float(np.real(np.vdot(W.astype(np.complex128), z)))

    rng = np.random.default_rng(0)
    for idx in list(rng.choice(h.size, 6, replace=False)) + [h.size - 1]:
        step = 0.5
        fd = 0j
        for unit in (1.0, 1j):
            hp, hm = h.copy(), h.copy()
            hp[idx] += unit * step
            hm[idx] -= unit * step
            fd += unit * (E(hp) - E(hm)) / (2 * step)
        assert abs(fd - gc[idx]) <= 1e-2 * max(abs(gc[idx]), 1e-6 * n), (idx, fd, gc[idx])


def test_autograd_function(torch, dpd, orc):
    from paper_1612_09001_amd.autograd import DPDFunction

    mo, co, L = [1, 3, 5, 7], [1, 3, 5, 7], 6
    h = signals.aph_coeffs(mo, co, L, config_id=87)
    plan = dpd.Plan(mo, co, L, h)
    rows, n = 3, 4096
    x = np.stack([signals.ofdm_16qam(n, config_id=87, stream_id=r) for r in range(rows)])
    W = signals.cgauss((rows, n), config_id=87)
    xt = _dev(torch, x).requires_grad_(True)
    ct = _dev(torch, h).requires_grad_(True)
    z = DPDFunction.apply(xt, ct, plan)
    E = (torch.conj(_dev(torch, W)) * z).real.sum()
    E.backward()
    rc = 0
    for r in range(rows):
        rx, b = orc.backward(x[r], mo, co, L, h, W[r])
        rc = rc + b
        assert nmse_db(xt.grad[r].cpu().numpy(), rx) <= -110
    assert_dcoef(ct.grad.cpu().numpy(), rc, "DPDFunction")


def test_config5_shape_full(torch, dpd, orc):
    """64 x 2^18 rows, I = {1,3,5,7} both branches, L = 6 (training shape)."""
    mo = co = [1, 3, 5, 7]
    L = 6
    rows, n = 64, 1 << 18
    x = np.stack([signals.ofdm_16qam(n, config_id=5, stream_id=r) for r in range(rows)])
    G = signals.cgauss((rows, n), config_id=5)
    h = signals.aph_coeffs(mo, co, L, config_id=5)
    _check(torch, dpd, orc, x, G, mo, co, L, h, what="config5")

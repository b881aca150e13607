"""Fused transmitter cascade (a memoryless APH stage A, then an APH stage B,
with the training loss, and its adjoint) through the C ABI, against the FP64
oracle applied stage by stage."""
import numpy as np
import pytest

from metrics import assert_parity
from paper_1612_09001_amd import signals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _stages(kind):
    """(A, B) stage definitions: (main orders, conj orders, L, complex64 coefficients)."""
    import oracle

    if kind == "synthetic_pa":
        return [tuple(s) for s in oracle.pa.stages()]
    # the largest stage B the fused kernels take (orders to 7 in both branches,
    # 4 taps) after a memoryless stage A with a cubic term in both branches
    a = ([1, 3], [1, 3], 1, 0.3 * signals.aph_coeffs([1, 3], [1, 3], 1, config_id=71))
    a[3][0] += 1.0
    b = ([1, 3, 5, 7], [1, 3, 5, 7], 4, signals.aph_coeffs([1, 3, 5, 7], [1, 3, 5, 7], 4, config_id=72))
    return a, b


def _oracle_loss(orc, z, x, A, B, scale):
    total = z.size
    E, gy = 0.0, np.zeros(z.shape, np.complex128)
    for r in range(z.shape[0]):
        u = orc.forward(z[r], *A)
        y = orc.forward(u, *B)
        d = scale * y - x[r].astype(np.complex128)
        E += float(np.sum(np.abs(d) ** 2))
        gy[r] = (2.0 * scale / total) * d
    return E / total, gy


def _oracle_backward(orc, z, gy, A, B):
    gz = np.zeros(z.shape, np.complex128)
    for r in range(z.shape[0]):
        u = orc.forward(z[r], *A)
        gu, _ = orc.backward(u, *B, gy[r], want_dcoef=False)
        gz[r], _ = orc.backward(z[r], *A, gu, want_dcoef=False)
    return gz


def _run(torch, A, B, z, x, scale, ld=None):
    from paper_1612_09001_amd import dpd

    rows, n = z.shape
    ld = n if ld is None else ld
    pa_, pb_ = dpd.Plan(*A), dpd.Plan(*B)
    zd = torch.zeros((rows, ld), dtype=torch.complex64, device="cuda")
    xd = torch.zeros_like(zd)
    zd[:, :n] = torch.from_numpy(z)
    xd[:, :n] = torch.from_numpy(x)
    gy = torch.zeros_like(zd)
    gz = torch.zeros_like(zd)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    wsb = dpd.dpd_loss_ws_size(rows * n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st = dpd.current_stream()
    dpd.dpd_cascade_loss_grad(pa_.handle, pb_.handle, st, zd.data_ptr(), xd.data_ptr(), rows, n, ld, scale,
                              loss.data_ptr(), gy.data_ptr(), ws.data_ptr(), wsb)
    gy_h = gy.cpu().numpy()
    dpd.dpd_cascade_backward(pa_.handle, pb_.handle, st, zd.data_ptr(), gy.data_ptr(), gz.data_ptr(), rows, n, ld)
    gz_h = gz.cpu().numpy()
    # nothing is written past n in a padded row
    if ld > n:
        assert not np.any(gy_h[:, n:]) and not np.any(gz_h[:, n:])
    return float(loss.item()), gy_h[:, :n], gz_h[:, :n]


@pytest.mark.parametrize("kind", ["synthetic_pa", "generic"])
@pytest.mark.parametrize("rows,n,ld", [(1, 20000, None), (3, 5003, 5010), (2, 2, 4), (1, 1, None)])
def test_cascade_matches_oracle(torch, orc, kind, rows, n, ld):
    A, B = _stages(kind)
    z = np.stack([signals.ofdm_16qam(n, config_id=73, stream_id=r) for r in range(rows)])
    x = np.stack([signals.ofdm_16qam(n, config_id=74, stream_id=r) for r in range(rows)])
    scale = 0.1 if kind == "synthetic_pa" else 0.5
    E, gy, gz = _run(torch, A, B, z, x, scale, ld)
    Er, gyr = _oracle_loss(orc, z, x, A, B, scale)
    assert abs(E - Er) <= 1e-5 * Er, (E, Er)
    assert_parity(gy, gyr, "dE/dy")
    # the adjoint from the GPU's dE/dy (complex64) in both paths
    gzr = _oracle_backward(orc, z, gy.astype(np.complex64), A, B)
    assert_parity(gz, gzr, "dE/dz")


def test_cascade_equals_separate_calls(torch):
    """The fused kernels against the stage-by-stage library path (both FP32):
    same loss and gradients to rounding."""
    from paper_1612_09001_amd import dpd
    from paper_1612_09001_amd.pa import SyntheticPA

    rows, n = 4, 1 << 14
    z = torch.from_numpy(np.stack([signals.ofdm_16qam(n, config_id=75, stream_id=r) for r in range(rows)])).cuda()
    x = torch.from_numpy(np.stack([signals.ofdm_16qam(n, config_id=76, stream_id=r) for r in range(rows)])).cuda()
    pa = SyntheticPA()
    st = dpd.current_stream()
    wsb = max(dpd.dpd_loss_ws_size(rows * n), dpd.dpd_backward_ws_size(pa.pa.handle, rows, n))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    u = pa.iq.apply(z)
    y = pa.pa.apply(u)
    loss1 = torch.zeros(1, device="cuda")
    gy1 = torch.empty_like(z)
    dpd.dpd_loss_grad(st, y.data_ptr(), x.data_ptr(), rows * n, 1.0 / pa.gain, loss1.data_ptr(), gy1.data_ptr(),
                      ws.data_ptr(), wsb)
    gu1 = torch.empty_like(z)
    gz1 = torch.empty_like(z)
    dpd.dpd_backward(pa.pa.handle, st, 0, u.data_ptr(), gy1.data_ptr(), gu1.data_ptr(), 0, rows, n, n,
                     ws.data_ptr(), wsb)
    dpd.dpd_backward(pa.iq.handle, st, 0, z.data_ptr(), gu1.data_ptr(), gz1.data_ptr(), 0, rows, n, n,
                     ws.data_ptr(), wsb)
    loss2 = torch.zeros(1, device="cuda")
    gy2 = torch.empty_like(z)
    gz2 = torch.empty_like(z)
    dpd.dpd_cascade_loss_grad(pa.iq.handle, pa.pa.handle, st, z.data_ptr(), x.data_ptr(), rows, n, n,
                              1.0 / pa.gain, loss2.data_ptr(), gy2.data_ptr(), ws.data_ptr(), wsb)
    dpd.dpd_cascade_backward(pa.iq.handle, pa.pa.handle, st, z.data_ptr(), gy2.data_ptr(), gz2.data_ptr(), rows,
                             n, n)
    assert abs(loss1.item() - loss2.item()) <= 1e-6 * loss1.item()
    assert_parity(gy2.cpu().numpy(), gy1.cpu().numpy(), "dE/dy")
    assert_parity(gz2.cpu().numpy(), gz1.cpu().numpy(), "dE/dz")


def test_cascade_rejects_unsupported_stages(torch):
    from paper_1612_09001_amd import dpd

    two_tap = dpd.Plan([1], [], 2, np.array([1, 0, 0], np.complex64))
    big = dpd.Plan([1, 3, 5, 7, 9], [], 2, np.zeros(11, np.complex64))
    ok_a = dpd.Plan([1], [1], 1, np.array([1, 0, 0], np.complex64))
    z = torch.zeros(64, dtype=torch.complex64, device="cuda")
    out = torch.zeros_like(z)
    st = dpd.current_stream()
    with pytest.raises(dpd.DPDError) as e:
        dpd.dpd_cascade_backward(two_tap.handle, ok_a.handle, st, z.data_ptr(), z.data_ptr(), out.data_ptr(), 1,
                                 64, 64)
    assert e.value.status == dpd.DPD_EINVAL
    with pytest.raises(dpd.DPDError) as e:
        dpd.dpd_cascade_backward(ok_a.handle, big.handle, st, z.data_ptr(), z.data_ptr(), out.data_ptr(), 1, 64,
                                 64)
    assert e.value.status == dpd.DPD_EUNSUPPORTED
    with pytest.raises(dpd.DPDError):   # output overlapping an input
        dpd.dpd_cascade_backward(ok_a.handle, ok_a.handle, st, z.data_ptr(), out.data_ptr(), z.data_ptr(), 1, 64,
                                 64)

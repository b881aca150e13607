"""Fused transmitter cascade (a memoryless APH stage A, then an APH stage B,
with the training loss, and its adjoint) through the C ABI, against the FP64
oracle applied stage by stage."""
import numpy as np
import pytest

from metrics import assert_dcoef, assert_parity
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


# Rows of whole 512-sample chunks take the streaming form: one chunk per wave
# (many_rows, one_chunk, three_chunks), and runs of two and three chunks per
# wave over 999-chunk rows, so that runs start inside rows and cross them.
@pytest.mark.parametrize("rows,n,ld,off", [(3, 5000, 5000, 0), (2, 4099, 4104, 0), (1, 1, 1, 0), (2, 777, 781, 1),
                                           (64, 1 << 14, 1 << 14, 0), (1, 512, 512, 0), (1, 1536, 1540, 0),
                                           (3, 512 * 999, 512 * 999, 0), (5, 512 * 999, 512 * 999, 0)],
                         ids=["aligned", "ragged_rows", "one_sample", "unaligned_8B", "many_rows", "one_chunk",
                              "three_chunks", "runs_cross_rows", "runs_of_three"])
@pytest.mark.parametrize("dpd_shape", [([1, 3, 5, 7], [1, 3, 5, 7], 6), ([1, 3, 5], [1, 3], 4),
                                       ([1, 3, 5, 7, 9], [1, 3, 5, 7, 9], 8)], ids=["P7_L6", "P5_L4", "P9_L8"])
def test_transmit_loss_grad_one_pass(torch, orc, rows, n, ld, off, dpd_shape):
    """Predistorter, transmitter and loss in one kernel: z and dE/dy bitwise
    those of dpd_apply_coeffs followed by dpd_cascade_loss_grad, the loss within
    FP32 summation-order rounding of theirs, and all three against the FP64
    oracle applied stage by stage."""
    from paper_1612_09001_amd import dpd

    A, B = _stages("synthetic_pa")
    mo, co, L = dpd_shape
    h = signals.aph_coeffs(mo, co, L, config_id=73)
    h[0] += 1.0
    x = np.stack([signals.ofdm_16qam(n, config_id=74, stream_id=r) for r in range(rows)])
    P = dpd.Plan(mo, co, L, np.zeros_like(h))      # the coefficients come from the device
    pa_, pb_ = dpd.Plan(*A), dpd.Plan(*B)
    base = torch.zeros(rows * ld + off + 2, dtype=torch.complex64, device="cuda")
    xd = base[off:off + rows * ld].view(rows, ld) if rows * ld else base[:0].view(rows, ld)
    xd[:, :n] = torch.from_numpy(x)
    hd = torch.from_numpy(h).cuda()
    outs = []
    for one_pass in (True, False):
        zb = torch.full((rows * ld + off + 2,), complex(5.0, 5.0), dtype=torch.complex64, device="cuda")
        gb = torch.full_like(zb, complex(5.0, 5.0))
        z = zb[off:off + rows * ld]
        g = gb[off:off + rows * ld]
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        wsb = dpd.dpd_loss_ws_size(rows * n)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        st = dpd.current_stream()
        if one_pass:
            dpd.dpd_transmit_loss_grad(P.handle, pa_.handle, pb_.handle, st, hd.data_ptr(), xd.data_ptr(), z.data_ptr(),
                                       rows, n, ld, 0.1, loss.data_ptr(), g.data_ptr(), ws.data_ptr(), wsb)
        else:
            dpd.dpd_apply_coeffs(P.handle, st, hd.data_ptr(), xd.data_ptr(), z.data_ptr(), rows, n, ld)
            dpd.dpd_cascade_loss_grad(pa_.handle, pb_.handle, st, z.data_ptr(), xd.data_ptr(), rows, n, ld, 0.1,
                                      loss.data_ptr(), g.data_ptr(), ws.data_ptr(), wsb)
        torch.cuda.synchronize()
        outs.append((z.view(rows, ld).cpu().numpy(), g.view(rows, ld).cpu().numpy(), float(loss.item())))
    (z1, g1, e1), (z2, g2, e2) = outs
    assert np.array_equal(z1[:, :n], z2[:, :n]) and np.array_equal(g1[:, :n], g2[:, :n])
    assert np.all(z1[:, n:] == np.complex64(complex(5.0, 5.0)))      # nothing written past n
    assert abs(e1 - e2) <= 1e-6 * e2
    zr = np.stack([orc.forward(x[r], mo, co, L, h) for r in range(rows)])
    E, gy = _oracle_loss(orc, zr, x, A, B, 0.1)
    assert_parity(z1[:, :n].reshape(-1), zr.reshape(-1), "z")
    assert_parity(g1[:, :n].reshape(-1), gy.reshape(-1), "dE/dy")
    assert abs(e1 - E) <= 1e-5 * E


def test_transmit_loss_grad_unsupported_stages(torch):
    from paper_1612_09001_amd import dpd

    A, B = _stages("general")
    P = dpd.Plan([1, 3], [1], 2, signals.aph_coeffs([1, 3], [1], 2, config_id=75))
    x = torch.zeros(64, dtype=torch.complex64, device="cuda")
    z, g = torch.zeros_like(x), torch.zeros_like(x)
    ws = torch.empty(dpd.dpd_loss_ws_size(64), dtype=torch.uint8, device="cuda")
    pa_, pb_ = dpd.Plan(*A), dpd.Plan(*B)      # kept alive for the call
    with pytest.raises(dpd.DPDError) as e:
        dpd.dpd_transmit_loss_grad(P.handle, pa_.handle, pb_.handle, dpd.current_stream(), 0,
                                   x.data_ptr(), z.data_ptr(), 1, 64, 64, 0.1, 0, g.data_ptr(), ws.data_ptr(),
                                   ws.numel())
    assert e.value.status == dpd.DPD_EUNSUPPORTED


# Rows of whole 256-sample chunks take the one-pass kernel (one chunk per wave;
# runs of two and three chunks over 999-chunk rows, starting inside rows and
# crossing them); the others the two passes through grad_z.
@pytest.mark.parametrize("rows,n,ld,off", [(3, 5120, 5120, 0), (64, 1 << 14, 1 << 14, 0), (1, 256, 256, 0),
                                           (2, 1280, 1284, 0), (3, 256 * 999, 256 * 999, 0),
                                           (5, 256 * 999, 256 * 999, 0), (2, 4099, 4104, 0), (2, 777, 781, 1),
                                           (1, 1, 1, 0)],
                         ids=["aligned", "many_rows", "one_chunk", "padded_rows", "runs_cross_rows", "runs_of_three",
                              "ragged_rows", "unaligned_8B", "one_sample"])
@pytest.mark.parametrize("dpd_shape", [([1, 3, 5, 7], [1, 3, 5, 7], 6), ([1, 3, 5], [1, 3], 4),
                                       ([1, 3, 5, 7, 9], [1, 3, 5, 7, 9], 8), ([1, 3], [1], 1)],
                         ids=["P7_L6", "P5_L4", "P9_L8", "P3_L1"])
def test_transmit_backward_one_pass(torch, orc, rows, n, ld, off, dpd_shape):
    """Cascade adjoint and coefficient gradient in one kernel: dE/dz (when
    asked for) bitwise that of dpd_cascade_backward, the gradient with and
    without dE/dz written bitwise equal, and every gradient entry against the
    FP64 oracle's coefficient gradient for the same dE/dz."""
    from paper_1612_09001_amd import dpd

    A, B = _stages("synthetic_pa")
    mo, co, L = dpd_shape
    h = signals.aph_coeffs(mo, co, L, config_id=76)
    x = np.stack([signals.ofdm_16qam(n, config_id=77, stream_id=r) for r in range(rows)])
    z = np.stack([signals.ofdm_16qam(n, config_id=78, stream_id=r) for r in range(rows)])
    gy = np.stack([signals.ofdm_16qam(n, config_id=79, stream_id=r) for r in range(rows)]) * 1e-3
    P = dpd.Plan(mo, co, L, h)
    pa_, pb_ = dpd.Plan(*A), dpd.Plan(*B)

    def dev(a):
        b = torch.zeros(rows * ld + off + 2, dtype=torch.complex64, device="cuda")
        v = b[off:off + rows * ld]
        v.view(rows, ld)[:, :n] = torch.from_numpy(a.astype(np.complex64))
        return b, v

    (xb, xd), (zb, zd), (yb, yd) = dev(x), dev(z), dev(gy)
    gzb = torch.full((rows * ld + off + 2,), complex(5.0, 5.0), dtype=torch.complex64, device="cuda")
    gzd = gzb[off:off + rows * ld]
    ref_b = torch.full_like(gzb, complex(5.0, 5.0))
    ref_d = ref_b[off:off + rows * ld]
    wsb = dpd.dpd_backward_ws_size(P.handle, rows, n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st = dpd.current_stream()
    one_pass = n % 256 == 0 and off == 0 and ld % 2 == 0
    gcs = []
    for want_gz in (True, False):
        gc = torch.zeros(P.K, dtype=torch.complex64, device="cuda")
        if not want_gz and not one_pass:
            with pytest.raises(dpd.DPDError) as e:
                dpd.dpd_transmit_backward(P.handle, pa_.handle, pb_.handle, st, xd.data_ptr(), zd.data_ptr(),
                                          yd.data_ptr(), 0, gc.data_ptr(), rows, n, ld, ws.data_ptr(), wsb)
            assert e.value.status == dpd.DPD_EUNSUPPORTED
            continue
        dpd.dpd_transmit_backward(P.handle, pa_.handle, pb_.handle, st, xd.data_ptr(), zd.data_ptr(), yd.data_ptr(),
                                  gzd.data_ptr() if want_gz else 0, gc.data_ptr(), rows, n, ld, ws.data_ptr(), wsb)
        torch.cuda.synchronize()
        gcs.append(gc.cpu().numpy())
    dpd.dpd_cascade_backward(pa_.handle, pb_.handle, st, zd.data_ptr(), yd.data_ptr(), ref_d.data_ptr(), rows, n, ld)
    torch.cuda.synchronize()
    g1 = gzd.view(rows, ld).cpu().numpy()
    g2 = ref_d.view(rows, ld).cpu().numpy()
    assert np.array_equal(g1[:, :n], g2[:, :n]), "dE/dz differs from dpd_cascade_backward"
    assert np.all(g1[:, n:] == np.complex64(complex(5.0, 5.0))) and np.all(
        gzb.cpu().numpy()[:off] == np.complex64(complex(5.0, 5.0)))
    if len(gcs) == 2:
        assert np.array_equal(gcs[0], gcs[1])
    ref = sum(orc.backward(x[r], mo, co, L, h, g2[r, :n].astype(np.complex128), want_dx=False)[1]
              for r in range(rows))
    assert_dcoef(gcs[0], ref, "transmit backward %s" % (dpd_shape,))


def test_transmit_backward_bad_arguments(torch):
    from paper_1612_09001_amd import dpd

    A, B = _stages("synthetic_pa")
    P = dpd.Plan([1, 3], [1], 2, signals.aph_coeffs([1, 3], [1], 2, config_id=80))
    pa_, pb_ = dpd.Plan(*A), dpd.Plan(*B)
    x = torch.zeros(512, dtype=torch.complex64, device="cuda")
    z, gy, gz = torch.zeros_like(x), torch.zeros_like(x), torch.zeros_like(x)
    gc = torch.zeros(P.K, dtype=torch.complex64, device="cuda")
    wsb = dpd.dpd_backward_ws_size(P.handle, 1, 512)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st = dpd.current_stream()
    call = lambda **k: dpd.dpd_transmit_backward(
        P.handle, k.get("a", pa_.handle), pb_.handle, st, x.data_ptr(), z.data_ptr(), k.get("gy", gy.data_ptr()),
        k.get("gz", gz.data_ptr()), k.get("gc", gc.data_ptr()), 1, 512, 512, ws.data_ptr(), k.get("wsb", wsb))
    call()
    for kw in ({"gc": 0}, {"wsb": wsb - 4}, {"gz": z.data_ptr()}, {"gz": gy.data_ptr()}, {"a": pb_.handle}):
        with pytest.raises(dpd.DPDError) as e:
            call(**kw)
        assert e.value.status == dpd.DPD_EINVAL, kw
    torch.cuda.synchronize()


def test_learning_passes_on_empty_input(torch):
    """No samples (rows = 0 or n = 0): the one-pass forward reports a zero
    loss and the one-pass backward a zero gradient, touching no sample."""
    from paper_1612_09001_amd import dpd

    A, B = _stages("synthetic_pa")
    mo = co = [1, 3, 5, 7]
    P = dpd.Plan(mo, co, 6, signals.aph_coeffs(mo, co, 6, config_id=81))
    pa_, pb_ = dpd.Plan(*A), dpd.Plan(*B)
    st = dpd.current_stream()
    wsb = max(dpd.dpd_backward_ws_size(P.handle, 1, 256), dpd.dpd_loss_ws_size(256))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    x = torch.zeros(256, dtype=torch.complex64, device="cuda")
    z, gy = torch.zeros_like(x), torch.zeros_like(x)
    for rows, n in ((0, 256), (4, 0)):
        loss = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
        gc = torch.full((P.K,), complex(7.0, 7.0), dtype=torch.complex64, device="cuda")
        dpd.dpd_transmit_loss_grad(P.handle, pa_.handle, pb_.handle, st, 0, x.data_ptr(), z.data_ptr(), rows, n,
                                   max(n, 1), 0.1, loss.data_ptr(), gy.data_ptr(), ws.data_ptr(), wsb)
        dpd.dpd_transmit_backward(P.handle, pa_.handle, pb_.handle, st, x.data_ptr(), z.data_ptr(), gy.data_ptr(),
                                  0, gc.data_ptr(), rows, n, max(n, 1), ws.data_ptr(), wsb)
        torch.cuda.synchronize()
        assert float(loss.item()) == 0.0 and not np.any(gc.cpu().numpy()), (rows, n)

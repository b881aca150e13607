"""dpd_backward_noalloc: the backward pass with the library's fixed device
scratch instead of a caller workspace, against dpd_backward (bitwise) and the
FP64 oracle, on consecutive calls (the second smaller, so stale partial sums
of the first stay in the scratch) and replayed from a captured graph."""
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


@pytest.fixture(scope="module")
def dpd(torch):
    from paper_1612_09001_amd import dpd as d

    d.lib()
    return d


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def _both(torch, dpd, plan, xd, gd, rows, n, coeffs=None):
    """(gx, gc) from dpd_backward with a workspace and from dpd_backward_noalloc."""
    st = dpd.current_stream()
    K = plan.K
    cp = 0 if coeffs is None else coeffs.data_ptr()
    out = []
    for noalloc in (False, True):
        gx = torch.full_like(xd, complex(9.0, -9.0))
        gc = torch.full((K,), complex(9.0, -9.0), dtype=torch.complex64, device="cuda")
        if noalloc:
            dpd.dpd_backward_noalloc(plan.handle, st, cp, xd.data_ptr(), gd.data_ptr(), gx.data_ptr(),
                                     gc.data_ptr(), rows, n, n)
        else:
            wsb = dpd.dpd_backward_ws_size(plan.handle, rows, n)
            ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
            dpd.dpd_backward(plan.handle, st, cp, xd.data_ptr(), gd.data_ptr(), gx.data_ptr(), gc.data_ptr(),
                             rows, n, n, ws.data_ptr(), wsb)
        torch.cuda.synchronize()
        out.append((gx.cpu().numpy(), gc.cpu().numpy()))
    return out


@pytest.mark.parametrize("shape", [([1, 3, 5, 7], [1, 3, 5, 7], 4), ([1, 3, 5, 7], [1, 3, 5, 7], 6),
                                   ([1, 3, 5], [1], 11)], ids=["P7_L4", "P7_L6", "generic_L11"])
def test_noalloc_matches_workspace_form_and_oracle(torch, dpd, orc, shape):
    mo, co, L = shape
    h = signals.aph_coeffs(mo, co, L, config_id=120)
    plan = dpd.Plan(mo, co, L, h)
    for rows, n in [(5, 200003), (2, 3001)]:      # the second call is smaller
        x = np.stack([signals.ofdm_16qam(n, config_id=121, stream_id=r) for r in range(rows)])
        G = signals.cgauss((rows, n), config_id=121, stream_id=n)
        xd, gd = _dev(torch, x), _dev(torch, G)
        (gx_w, gc_w), (gx_n, gc_n) = _both(torch, dpd, plan, xd, gd, rows, n)
        assert np.array_equal(gx_w, gx_n) and np.array_equal(gc_w, gc_n), (shape, rows, n)
        rx = np.zeros_like(x, dtype=np.complex128)
        rc = 0
        for r in range(rows):
            a, b = orc.backward(x[r], mo, co, L, h, G[r])
            rx[r] = a
            rc = rc + b
        assert_parity(gx_n.reshape(-1), rx.reshape(-1), "noalloc dx %s %d x %d" % (shape, rows, n))
        assert_dcoef(gc_n, rc, "noalloc dcoef %s %d x %d" % (shape, rows, n))


def test_noalloc_device_coeffs_and_dx_only(torch, dpd, orc):
    mo, co, L = [1, 3, 5], [1, 3], 5
    h = signals.aph_coeffs(mo, co, L, config_id=122)
    plan = dpd.Plan(mo, co, L, np.zeros_like(h))
    n = 40000
    x = signals.ofdm_16qam(n, config_id=122)
    G = signals.cgauss(n, config_id=122)
    xd, gd, hd = _dev(torch, x), _dev(torch, G), _dev(torch, h)
    (gx_w, gc_w), (gx_n, gc_n) = _both(torch, dpd, plan, xd, gd, 1, n, coeffs=hd)
    assert np.array_equal(gx_w, gx_n) and np.array_equal(gc_w, gc_n)
    rx, rc = orc.backward(x, mo, co, L, h, G)
    assert_parity(gx_n, rx, "noalloc dx, device coefficients")
    assert_dcoef(gc_n, rc, "noalloc dcoef, device coefficients")
    gx = torch.empty_like(xd)
    dpd.dpd_backward_noalloc(plan.handle, dpd.current_stream(), hd.data_ptr(), xd.data_ptr(), gd.data_ptr(),
                             gx.data_ptr(), 0, 1, n, n)
    assert np.array_equal(gx.cpu().numpy(), gx_w)


def test_noalloc_graph_replay(torch, dpd):
    """Captured in a graph and replayed, with eager work between replays: every
    replay equals the eager call bitwise."""
    mo = co = [1, 3, 5, 7]
    L, n = 4, 65536
    plan = dpd.Plan(mo, co, L, signals.aph_coeffs(mo, co, L, config_id=123))
    xd = _dev(torch, signals.ofdm_16qam(n, config_id=123))
    gd = _dev(torch, signals.cgauss(n, config_id=123))
    gx = torch.empty_like(xd)
    gc = torch.empty(plan.K, dtype=torch.complex64, device="cuda")

    def call():
        dpd.dpd_backward_noalloc(plan.handle, dpd.current_stream(), 0, xd.data_ptr(), gd.data_ptr(), gx.data_ptr(),
                                 gc.data_ptr(), 1, n, n)

    call()
    torch.cuda.synchronize()
    ref_x, ref_c = gx.clone(), gc.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        call()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            call()
    torch.cuda.synchronize()
    for r in range(3):
        gx.fill_(complex(r, r))
        gc.fill_(complex(-r, r))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(gx, ref_x) and torch.equal(gc, ref_c), "replay %d" % r


def test_noalloc_rejects_bad_arguments(torch, dpd):
    with pytest.raises(dpd.DPDError):
        dpd.dpd_backward_noalloc(0, 0, 0, 0, 0, 0, 0, 1, 10, 10)

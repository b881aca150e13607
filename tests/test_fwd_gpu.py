"""Forward apply on the GPU (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

from metrics import assert_parity
from paper_1612_09001_amd import signals

pytestmark = pytest.mark.gpu

ALL_TUNES = [(s, lds) for s in (2, 4, 8) for lds in (0, 1)]


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


def _host(t):
    return t.cpu().numpy()


def _run(torch, dpd, x, mo, co, L, h, tune=None):
    plan = dpd.Plan(mo, co, L, h)
    if tune is not None:
        plan.set_tune(samples_per_thread=tune[0], stage_lds=tune[1])
    z = plan.apply(_dev(torch, x))
    torch.cuda.synchronize()
    return _host(z)


@pytest.mark.parametrize("tune", ALL_TUNES)
def test_config1_full(torch, dpd, orc, tune):
    """N = 65536 OFDM-like, I = {1,3,5,7} both branches, L = 4, DC term."""
    mo = co = [1, 3, 5, 7]
    L = 4
    x = signals.ofdm_16qam(65536, config_id=1)
    h = signals.aph_coeffs(mo, co, L, config_id=1)
    z = _run(torch, dpd, x, mo, co, L, h, tune)
    assert_parity(z, orc.forward(x, mo, co, L, h), "config1 %s" % (tune,))


SHAPES = [
    ([1], [], 1), ([1, 3, 5], [1, 3], 5), ([1, 3, 5, 7], [1, 3, 5, 7], 4), ([1, 5], [3], 3),
    ([3, 7], [], 2), ([1, 3, 5, 7, 9], [1, 3, 5, 7, 9], 8), ([1, 3, 5, 7, 9, 11, 13, 15], [1], 6),
    ([1, 3], [1, 3, 5, 7, 9, 11, 13, 15], 7),
    ([1, 3, 5], [1], 12), ([1, 3, 5, 7, 9], [1, 3], 16),   # generic kernel (L > 8)
]
LENGTHS = [1, 2, 3, 7, 8, 9, 511, 512, 513, 1023, 1024, 1025, 2047, 2049, 4097, 9001]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "P%s_Q%s_L%d" % (max(s[0]), max(s[1]) if s[1] else 0, s[2]))
@pytest.mark.parametrize("tune", [(2, 1), (4, 0), (8, 1)])
def test_shapes_and_ragged_lengths(torch, dpd, orc, shape, tune):
    mo, co, L = shape
    h = signals.aph_coeffs(mo, co, L, config_id=90, stream_id=L)
    xs = signals.ofdm_16qam(sum(LENGTHS), config_id=90, stream_id=1)
    off = 0
    plan = dpd.Plan(mo, co, L, h)
    plan.set_tune(samples_per_thread=tune[0], stage_lds=tune[1])
    for n in LENGTHS:
        x = xs[off:off + n]
        off += n
        z = plan.apply(_dev(torch, x))
        torch.cuda.synchronize()
        assert_parity(_host(z), orc.forward(x, mo, co, L, h), "%s n=%d" % (shape, n))


def test_identity_is_exact(torch, dpd):
    mo = co = [1, 3, 5, 7]
    L = 4
    x = signals.ofdm_16qam(100003, config_id=1)
    h = signals.identity_coeffs(mo, co, L)
    for tune in ALL_TUNES:
        z = _run(torch, dpd, x, mo, co, L, h, tune)
        assert np.array_equal(z, x), tune


def test_empty_and_canary(torch, dpd, orc):
    mo = co = [1, 3, 5]
    L = 5
    h = signals.aph_coeffs(mo, co, L, config_id=91)
    plan = dpd.Plan(mo, co, L, h)
    x = _dev(torch, signals.ofdm_16qam(4096, config_id=91))
    out = torch.full((4096 + 64,), complex(7.0, -7.0), dtype=torch.complex64, device="cuda")
    dpd.dpd_apply(plan.handle, dpd.current_stream(), x.data_ptr(), out.data_ptr(), 0)
    torch.cuda.synchronize()
    assert torch.all(out == complex(7.0, -7.0))
    for n in (1, 777, 4095):
        out.fill_(complex(7.0, -7.0))
        dpd.dpd_apply(plan.handle, dpd.current_stream(), x.data_ptr(), out.data_ptr(), n)
        torch.cuda.synchronize()
        o = _host(out)
        assert np.all(o[n:] == np.complex64(complex(7.0, -7.0))), n
        assert_parity(o[:n], orc.forward(_host(x)[:n], mo, co, L, h))


def test_unaligned_and_overlap(torch, dpd, orc):
    """An 8-byte-aligned (not 16) start takes the generic kernel; overlapping
    input and output ranges are rejected."""
    mo = co = [1, 3, 5, 7]
    L = 4
    h = signals.aph_coeffs(mo, co, L, config_id=92)
    plan = dpd.Plan(mo, co, L, h)
    xh = signals.ofdm_16qam(5001, config_id=92)
    buf = _dev(torch, np.concatenate([[0], xh]))
    out = torch.zeros(5002, dtype=torch.complex64, device="cuda")
    dpd.dpd_apply(plan.handle, dpd.current_stream(), buf.data_ptr() + 8, out.data_ptr() + 8, 5001)
    torch.cuda.synchronize()
    assert_parity(_host(out)[1:], orc.forward(xh, mo, co, L, h))
    with pytest.raises(dpd.DPDError) as e:
        dpd.dpd_apply(plan.handle, dpd.current_stream(), buf.data_ptr(), buf.data_ptr() + 8, 100)
    assert e.value.status == dpd.DPD_EINVAL
    with pytest.raises(dpd.DPDError):
        dpd.dpd_apply(plan.handle, dpd.current_stream(), buf.data_ptr() + 4, out.data_ptr(), 100)


@pytest.mark.parametrize("ld_extra", [0, 1, 6])
def test_rows(torch, dpd, orc, ld_extra):
    mo, co, L = [1, 3, 5, 7], [1, 3, 5, 7], 6
    h = signals.aph_coeffs(mo, co, L, config_id=93)
    rows, n = 5, 3001
    ld = n + ld_extra
    xs = np.zeros((rows, ld), np.complex64)
    for r in range(rows):
        xs[r, :n] = signals.ofdm_16qam(n, config_id=93, stream_id=r)
    xt = _dev(torch, xs)
    plan = dpd.Plan(mo, co, L, h)
    out = torch.zeros_like(xt)
    dpd.dpd_apply_rows(plan.handle, dpd.current_stream(), xt.data_ptr(), out.data_ptr(), rows, n, ld)
    torch.cuda.synchronize()
    o = _host(out)
    for r in range(rows):
        assert_parity(o[r, :n], orc.forward(xs[r, :n], mo, co, L, h), "row %d" % r)
        assert np.all(o[r, n:] == 0)


@pytest.mark.parametrize("L", [1, 2, 5, 8, 11])
def test_streaming_history(torch, dpd, orc, L):
    mo, co = [1, 3, 5], [1, 3]
    h = signals.aph_coeffs(mo, co, L, config_id=94)
    x = signals.ofdm_16qam(20000, config_id=94)
    plan = dpd.Plan(mo, co, L, h)
    hist = torch.zeros(max(L - 1, 1), dtype=torch.complex64, device="cuda")[:L - 1]
    cuts = [0, 1, 3, 1000, 1001, 7777, 20000]
    parts = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        parts.append(_host(plan.apply_hist(_dev(torch, x[a:b]), hist)))
    torch.cuda.synchronize()
    z = np.concatenate(parts)
    assert_parity(z, orc.forward(x, mo, co, L, h))
    if L > 1:
        assert np.array_equal(_host(hist), x[-(L - 1):])
    # an explicit non-zero history matches the oracle with that history
    h0 = signals.ofdm_16qam(L - 1 + 10, config_id=94, stream_id=5)[:L - 1]
    ht = _dev(torch, h0) if L > 1 else None
    z2 = _host(plan.apply_hist(_dev(torch, x[:3000]), ht))
    assert_parity(z2, orc.forward(x[:3000], mo, co, L, h, hist=h0 if L > 1 else None))


def test_device_coeffs_match_host(torch, dpd):
    """Precombining on the device gives the same table bits as on the host."""
    mo, co, L = [1, 3, 5, 7], [1, 3], 5
    h = signals.aph_coeffs(mo, co, L, config_id=95)
    x = _dev(torch, signals.ofdm_16qam(50000, config_id=95))
    plan = dpd.Plan(mo, co, L, h)
    z1 = _host(plan.apply(x))
    z2 = _host(plan.apply_coeffs(_dev(torch, h), x))
    plan2 = dpd.Plan(mo, co, L, np.zeros_like(h))
    plan2.set_coeffs(_dev(torch, h))
    z3 = _host(plan2.apply(x))
    assert np.array_equal(z1, z2) and np.array_equal(z1, z3)


def test_device_coeff_calls_leave_plan_coeffs(torch, dpd, orc):
    """dpd_apply_coeffs and dpd_backward with device coefficients use the
    plan's second table: a later dpd_apply still filters with the plan's own
    coefficients."""
    mo, co, L = [1, 3, 5], [1, 3], 4
    h1 = signals.aph_coeffs(mo, co, L, config_id=97)
    h2 = signals.aph_coeffs(mo, co, L, config_id=98)
    x = signals.ofdm_16qam(30001, config_id=97)
    xd = _dev(torch, x)
    plan = dpd.Plan(mo, co, L, h1)
    z2 = _host(plan.apply_coeffs(_dev(torch, h2), xd))
    assert_parity(z2, orc.forward(x, mo, co, L, h2), "apply_coeffs")
    z1 = _host(plan.apply(xd))
    assert_parity(z1, orc.forward(x, mo, co, L, h1), "plan coefficients after apply_coeffs")
    plan.backward(xd, xd, coeffs=_dev(torch, h2))
    z1b = _host(plan.apply(xd))
    assert np.array_equal(z1, z1b), "plan coefficients after backward with device coefficients"


def test_conditional_device_coeffs(torch, dpd, orc):
    """dpd_set_coeffs_device_if copies only when the device flag is 0."""
    mo, co, L = [1, 3], [1], 3
    h1 = signals.aph_coeffs(mo, co, L, config_id=99)
    h2 = signals.aph_coeffs(mo, co, L, config_id=100)
    x = signals.ofdm_16qam(5000, config_id=99)
    xd = _dev(torch, x)
    plan = dpd.Plan(mo, co, L, h1)
    flag = torch.tensor(3, dtype=torch.int32, device="cuda")
    h2d = _dev(torch, h2)
    st = dpd.current_stream()
    dpd.dpd_set_coeffs_device_if(plan.handle, h2d.data_ptr(), flag.data_ptr(), st)
    assert_parity(_host(plan.apply(xd)), orc.forward(x, mo, co, L, h1), "flag set: unchanged")
    flag.zero_()
    dpd.dpd_set_coeffs_device_if(plan.handle, h2d.data_ptr(), flag.data_ptr(), st)
    assert_parity(_host(plan.apply(xd)), orc.forward(x, mo, co, L, h2), "flag clear: replaced")


def test_config2_full_size(torch, dpd, orc):
    """N = 2^24 in the launch shape the benchmark times; every output."""
    mo = co = [1, 3, 5, 7]
    L = 4
    n = 1 << 24
    x = signals.ofdm_16qam(n, config_id=2)
    h = signals.aph_coeffs(mo, co, L, config_id=2)
    plan = dpd.Plan(mo, co, L, h)
    z = _host(plan.apply(_dev(torch, x)))
    assert_parity(z, orc.forward(x, mo, co, L, h), "config2")


def test_config3_full_size(torch, dpd, orc):
    """N = 2^26 two-carrier stream, I = {1..9} both branches, L = 8; every
    output against the FP64 oracle."""
    mo = co = [1, 3, 5, 7, 9]
    L = 8
    n = 1 << 26
    x = signals.two_carrier(n, config_id=3)
    h = signals.aph_coeffs(mo, co, L, config_id=3)
    plan = dpd.Plan(mo, co, L, h)
    xd = _dev(torch, x)
    z = _host(plan.apply(xd))
    del xd
    ref = orc.forward(x, mo, co, L, h)
    assert_parity(z, ref, "config3")


def _table2():
    """The paper's Table 2 configuration, from tests/golden/table2_config.txt."""
    import os

    cfg = {}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_config.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                cfg[k] = [int(t) for t in v]
    return cfg["main_orders"], cfg["conj_orders"], cfg["L"][0]


@pytest.mark.parametrize("tune", [(8, 1), (4, 0)])
def test_table2_configuration(torch, dpd, orc, tune):
    """Section 3.4 / Table 2: P = 5 main, Q = 3 conjugate (I_Q a proper subset
    of I_P), L = 5, DC term -- the configuration of the paper's Table 4."""
    mo, co, L = _table2()
    x = signals.ofdm_16qam(200003, config_id=2)
    h = signals.aph_coeffs(mo, co, L, config_id=2)
    z = _run(torch, dpd, x, mo, co, L, h, tune)
    assert_parity(z, orc.forward(x, mo, co, L, h), "table2 %s" % (tune,))


def test_graph_replay(torch, dpd, orc):
    """dpd_apply and dpd_apply_hist captured in one hipGraph: every replay, with
    eager work and synchronisations between replays, equals the same eager
    calls bitwise, and the history carried across replays matches the oracle."""
    mo = co = [1, 3, 5, 7]
    L, n, reps = 4, 65536, 4
    h = signals.aph_coeffs(mo, co, L, config_id=1)
    xs = [signals.ofdm_16qam(n, config_id=96, stream_id=r) for r in range(reps)]
    plan = dpd.Plan(mo, co, L, h)
    x = torch.empty(n, dtype=torch.complex64, device="cuda")
    z = torch.empty_like(x)
    z2 = torch.empty_like(x)
    hist = torch.zeros(L - 1, dtype=torch.complex64, device="cuda")
    ehist = torch.zeros_like(hist)
    x.copy_(_dev(torch, xs[0]))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.apply(x, out=z)
        plan.apply_hist(x, hist, out=z2)
    hist.zero_()
    torch.cuda.synchronize()
    for r in range(reps):
        x.copy_(_dev(torch, xs[r]))           # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        xe = _dev(torch, xs[r])
        ze = _host(plan.apply(xe))
        ze2 = _host(plan.apply_hist(xe, ehist))
        torch.cuda.synchronize()
        assert np.array_equal(_host(z), ze), "replay %d apply" % r
        assert np.array_equal(_host(z2), ze2), "replay %d apply_hist" % r
        prev = xs[r - 1][-(L - 1):] if r > 0 else np.zeros(L - 1, np.complex64)
        assert_parity(_host(z2), orc.forward(xs[r], mo, co, L, h, hist=prev), "replay %d" % r)


def test_set_coeffs_async_is_stream_ordered(torch, dpd, orc):
    """Host coefficients ordered on the stream: three applies with updates in
    between, no host synchronization, each apply filtering with the
    coefficients set before it (the second update refills the staging buffer
    while the first copy may still be queued behind a long apply)."""
    mo, co, L = [1, 3, 5], [1, 3], 4
    hs = [signals.aph_coeffs(mo, co, L, config_id=c) for c in (131, 132, 133)]
    x = signals.ofdm_16qam(1 << 22, config_id=131)
    xd = _dev(torch, x)
    plan = dpd.Plan(mo, co, L, hs[0])
    outs = [plan.apply(xd)]
    for h in hs[1:]:
        plan.set_coeffs(h, ordered=True)
        outs.append(plan.apply(xd))
    torch.cuda.synchronize()
    for i, (z, h) in enumerate(zip(outs, hs)):
        zr = orc.forward(x[:1 << 16], mo, co, L, h)
        assert_parity(_host(z)[:1 << 16], zr, "apply %d" % i)
    # the async update leaves the same table bits as the device-wide one
    plan2 = dpd.Plan(mo, co, L, hs[0])
    plan2.set_coeffs(hs[2])
    assert np.array_equal(_host(plan2.apply(xd)), _host(outs[2]))

"""More than 2^31 samples in one call (64-bit indexing in every kernel, sums
whose rounding error must not grow with the length): the forward and the
backward of the headline basis on one stream of N = 2^31 + 2^20 + 777
samples, one batch launch over 2^31 + 2^20 + 8 samples in three streams,
the least-squares normal equations over the same long stream, and one
learning step over 8193 rows of 2^18, against the FP64 oracle.  The stream and its output gradient repeat seeded blocks of P = 2^20
samples, so the oracle gets each sampled output from the L-sample window it
depends on, and the whole coefficient gradient from three runs over one
block: the first block (zero history), one later block (the block's own end
as history, weighted by the number of such blocks) and the ragged end.  The
learning rows are all the same seeded row, so the mean loss and its gradient
are those of that row."""
import numpy as np
import pytest

from metrics import LS_REL_MAX, assert_dcoef, assert_parity, ls_errors
from paper_1612_09001_amd import signals

pytestmark = pytest.mark.gpu

P = 1 << 20
N = (1 << 31) + P + 777
MO = CO = [1, 3, 5, 7]
L = 4


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


def _repeat(torch, block):
    """The block repeated to N samples on the device (a contiguous view)."""
    b = torch.from_numpy(np.ascontiguousarray(block, dtype=np.complex64)).cuda()
    return b.repeat(N // P + 1)[:N]


def _sample_indices():
    rng = np.random.default_rng(5)
    edges = [0, 1, 2, 3, P - 2, P - 1, P, P + 1, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, N - 1]
    near = np.concatenate([np.arange(e - 8, e + 8) for e in edges])
    # chunk starts of the 512-sample forward and 256-sample backward walks past 2^31
    chunks = (1 << 31) + np.arange(-4, 5) * 512
    idx = np.concatenate([near, chunks, rng.integers(0, N, 4096)])
    return np.unique(idx[(idx >= 0) & (idx < N)])


def _windows(block, idx, back):
    """Per index i the L samples the oracle needs, as one compact array:
    x_{i-L+1..i} (zero before the stream start) when back is False, else
    x_{i..i+L-1} (zero past the stream end)."""
    off = np.arange(L) - (L - 1) if not back else np.arange(L)
    pos = idx[:, None] + off[None, :]
    w = block[np.mod(pos, P)]
    w[(pos < 0) | (pos >= N)] = 0
    return w.reshape(-1)


def test_forward_past_2_31(torch, dpd, orc):
    x_blk = signals.ofdm_16qam(P, config_id=2).astype(np.complex64)
    h = signals.aph_coeffs(MO, CO, L, config_id=2)
    x = _repeat(torch, x_blk)
    z = dpd.Plan(MO, CO, L, h).apply(x)
    idx = _sample_indices()
    got = z[torch.from_numpy(idx).cuda()].cpu().numpy()
    del z, x
    ref = orc.forward_at(_windows(x_blk, idx, False), MO, CO, L, h, np.arange(idx.size) * L + L - 1)
    assert_parity(got, ref, "forward at N = 2^31 + 2^20 + 777")


def test_backward_past_2_31(torch, dpd, orc):
    x_blk = signals.ofdm_16qam(P, config_id=2).astype(np.complex64)
    g_blk = (signals.ofdm_16qam(P, config_id=12) * 1e-3).astype(np.complex64)
    h = signals.aph_coeffs(MO, CO, L, config_id=2)
    x, g = _repeat(torch, x_blk), _repeat(torch, g_blk)
    gx, gc = dpd.Plan(MO, CO, L, h).backward(x, g)
    idx = _sample_indices()
    got = gx[torch.from_numpy(idx).cuda()].cpu().numpy()
    gc = gc.cpu().numpy()
    del gx, x, g
    # dx_i depends on x_i and G_{i..i+L-1}: the first output of each window
    rx, _ = orc.backward(_windows(x_blk, idx, True), MO, CO, L, h, _windows(g_blk, idx, True), want_dcoef=False)
    assert_parity(got, rx[::L], "dx at N = 2^31 + 2^20 + 777")
    # the coefficient gradient: first block + (full blocks - 1) later blocks + the ragged end
    hist = x_blk[P - (L - 1):]
    _, first = orc.backward(x_blk, MO, CO, L, h, g_blk, want_dx=False)
    _, later = orc.backward(x_blk, MO, CO, L, h, g_blk, hist=hist, want_dx=False)
    R = N % P
    _, end = orc.backward(x_blk[:R], MO, CO, L, h, g_blk[:R], hist=hist, want_dx=False)
    ref = first + (N // P - 1) * later + end
    assert_dcoef(gc, ref, "dcoef at N = 2^31 + 2^20 + 777")


def test_learning_step_past_2_31(torch, orc):
    """One dpd_learn_step over 8193 identical rows of 2^18 samples (2^31 + 2^18
    in all): the loss and every coefficient-gradient entry against the FP64
    chain over the one row, at coefficients away from the optimum."""
    import oracle.pa as opa
    from paper_1612_09001_amd.train import FusedTrainer

    orders, Lt, n, rows = [1, 3, 5, 7], 6, 1 << 18, (1 << 13) + 1
    row = signals.ofdm_16qam(n, config_id=9, stream_id=0)
    xd = torch.from_numpy(row).cuda().reshape(1, n).repeat(rows, 1)
    h = signals.aph_coeffs(orders, orders, Lt, config_id=52)
    h[0] += 1.0
    tr = FusedTrainer(xd, orders, orders, Lt, h, lr=0.0)
    assert tr.one_call
    loss = float(tr.step().item())
    gc = tr.gc.cpu().numpy()
    del tr, xd
    E, g = opa.chain_loss_and_gradient(orc, row[None, :], (orders, orders), Lt, h)
    assert abs(loss - E) <= 1e-5 * E, (loss, E)
    assert_dcoef(gc, g, "chain gradient, 8193 x 2^18", entry_max=1e-4, rel_max=1e-4)


def test_batch_past_2_31(torch, dpd, orc):
    """One persistent batch launch over 2^31 + 2^20 + 8 samples in three
    streams, each repeating its own seeded 2^20-sample block (P_max 9 and L 8,
    P_max 5 and L 3, P_max 7 and L 6): sampled outputs of every stream against
    the oracle."""
    from paper_1612_09001_amd import batch

    specs = [((1 << 30) + 5, 9, 8), ((1 << 29) + 3, 5, 3), ((1 << 29) + (1 << 20), 7, 6)]
    rng = np.random.default_rng(7)
    streams, checks = [], []
    for s, (n, pmax, Ls) in enumerate(specs):
        orders = signals.odd_orders(pmax)
        blk = signals.ofdm_16qam(P, config_id=30 + s).astype(np.complex64)
        h = signals.aph_coeffs(orders, orders, Ls, config_id=30 + s)
        x = torch.from_numpy(blk).cuda().repeat(n // P + 1)[:n]
        z = torch.empty(n, dtype=torch.complex64, device="cuda")
        streams.append({"in": x, "out": z, "n": n, "main_orders": orders, "conj_orders": orders, "L": Ls,
                        "coeffs": torch.from_numpy(h.astype(np.complex64)).cuda()})
        edges = np.concatenate([np.arange(0, 8), np.arange(P - 8, P + 8), np.arange(n - 16, n),
                                rng.integers(0, n, 2048)])
        checks.append((np.unique(edges[(edges >= 0) & (edges < n)]), blk, orders, Ls, h))
    b = batch.Batch(streams)
    b.apply()
    for s, (idx, blk, orders, Ls, h) in enumerate(checks):
        got = streams[s]["out"][torch.from_numpy(idx).cuda()].cpu().numpy()
        pos = idx[:, None] + (np.arange(Ls) - (Ls - 1))[None, :]
        w = blk[np.mod(pos, P)]
        w[pos < 0] = 0
        ref = orc.forward_at(w.reshape(-1), orders, orders, Ls, h, np.arange(idx.size) * Ls + Ls - 1)
        assert_parity(got, ref, "batch stream %d past 2^31 samples in all" % s)
    b.close()


def test_ls_normal_past_2_31(torch, dpd, orc):
    """The normal equations of the headline basis over N = 2^31 + 2^20 + 777
    samples (input and target repeat seeded 2^20-sample blocks): every entry
    of A and b against the FP64 oracle, composed from the first block, one
    later block (its rows with the block's own end as history: the oracle's
    sums over the history followed by the block, less those over the history
    alone, whose target is zero) and the ragged end."""
    y_blk = signals.ofdm_16qam(P, config_id=31, stream_id=7).astype(np.complex64)
    t_blk = (0.5 * signals.ofdm_16qam(P, config_id=32, stream_id=7)).astype(np.complex64)
    plan = dpd.Plan(MO, CO, L, signals.aph_coeffs(MO, CO, L, config_id=3))
    y, t = _repeat(torch, y_blk), _repeat(torch, t_blk)
    A, b = plan.ls_normal(y, t)
    A, b = A.cpu().numpy(), b.cpu().numpy()
    del y, t
    hist = y_blk[P - (L - 1):]
    zh = np.zeros(L - 1, np.complex64)
    R = N % P

    def with_hist(yy, tt):
        a1, b1 = orc.ls_normal(np.concatenate([hist, yy]), MO, CO, L, np.concatenate([zh, tt]))
        a0, b0 = orc.ls_normal(hist, MO, CO, L, zh)
        return a1 - a0, b1 - b0

    a_first, b_first = orc.ls_normal(y_blk, MO, CO, L, t_blk)
    a_later, b_later = with_hist(y_blk, t_blk)
    a_end, b_end = with_hist(y_blk[:R], t_blk[:R])
    m = N // P
    Ar = a_first + (m - 1) * a_later + a_end
    br = b_first + (m - 1) * b_later + b_end
    t2 = m * float(np.sum(np.abs(t_blk.astype(np.complex128)) ** 2)) + float(
        np.sum(np.abs(t_blk[:R].astype(np.complex128)) ** 2))
    ea, eb, ma, mb = ls_errors(A, b, Ar, br, t2)
    assert max(ea, eb, ma, mb) <= LS_REL_MAX, "A frob %.3g, b frob %.3g, A entry %.3g, b entry %.3g" % (
        ea, eb, ma, mb)

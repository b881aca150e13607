"""Least-squares estimation (section 2.2, Eq. 2) on the GPU: the matrix-core
normal equations against the FP64 oracle's, the FP64 Cholesky solve against
numpy's solve of the same matrices, end-to-end recovery of known coefficients,
and the indirect-learning loop on the synthetic PA."""
import numpy as np
import pytest

from metrics import LS_REL_MAX, ls_errors
from paper_1612_09001_amd import signals

pytestmark = pytest.mark.gpu

# Tolerance of the normal equations, after the diagonal scaling
# S = diag(A)^(-1/2) that gives every entry of S A S, and of S b / |t|, a bound
# of 1 (Cauchy-Schwarz): the relative Frobenius error and the largest error of
# one entry in those units.  Features are FP32 (order 2j+1 by j repeated
# multiplications: relative error <= ~(2j+2) 2^-24 <= 1.2e-6 for order 9); on
# the matrix cores each is a bf16 high part plus the bf16 rounding of the
# remainder, whose four cross products leave ~2^-17 of each product, random in
# sign; each FP32 accumulator adds at most 256 eight-sample steps of a slab
# (512 when the basis needs 8 or more column tiles, K >= 57, and the slabs are
# 8192 samples) and the four wave partials of a slab are added in FP32 before
# the FP64 slab sum (relative error ~1e-6 for random rounding; measured
# 2e-7..9e-7 on A and ~3e-6 on b).  2e-5 leaves a margin of 6 or more.


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


def _assert_ls(A, b, Ar, br, t2, what=""):
    ea, eb, ma, mb = ls_errors(A, b, Ar, br, t2)
    assert max(ea, eb, ma, mb) <= LS_REL_MAX, "%s: A frob %.3g, b frob %.3g, A entry %.3g, b entry %.3g" % (
        what, ea, eb, ma, mb)


def _t2(t):
    return float(np.sum(np.abs(np.asarray(t, dtype=np.complex128)) ** 2))


def _target(n, mo, co, L, seed):
    """A target sequence: the input through other APH coefficients plus a
    second independent signal (so b is not in the span of A exactly)."""
    y = signals.ofdm_16qam(n, config_id=31, stream_id=seed)
    w = signals.ofdm_16qam(n, config_id=32, stream_id=seed)
    return y, (0.5 * w).astype(np.complex64)


CASES = [  # (main orders, conj orders, L, n)
    ([1, 3, 5, 7], [1, 3, 5, 7], 4, 20000),     # headline basis, ragged slab and tile
    ([1, 3, 5], [1, 3], 3, 4096),               # exactly one slab
    ([1, 3, 5, 7, 9], [1, 3, 5, 7, 9], 8, 9000),  # K = 81 (2K+2 = 164 -> 11 x 11 tiles)
    ([1], [1], 1, 100),                         # K = 3, mostly padding
    ([1, 3, 5], [], 2, 777),                    # K = 7: 2K+2 = 16, no padding column
    ([1, 3, 5, 7, 9, 11, 13], [], 2, 5000),     # high orders, main branch only
    ([1, 3, 5], [1, 3, 5], 5, 3),               # fewer samples than taps
    ([1, 3, 5, 7], [1, 3, 5, 7], 6, 65536 + 17),  # config-5 basis, 17 slabs
    ([1, 3, 5, 7, 9], [1, 3, 5], 5, 3000),      # K = 41: 6 x 6 tiles
    ([1, 3, 5, 7, 9, 11, 13], [1, 3, 5, 7, 9, 11, 13], 4, 6000),  # K = 57: 8 x 8 tiles, two pair groups
    ([1, 3, 5, 7, 9, 11, 13, 15], [1, 3, 5], 8, 2500),  # K = 89: 12 x 12 tiles, the largest basis
    ([1, 3], [1], 16, 3000),                    # the most taps: 15 rows carried between tiles
    ([1, 5, 9], [3, 7], 3, 2000),               # orders with gaps, levels split between the branches
]


@pytest.mark.parametrize("mo,co,L,n", CASES, ids=["P%d_Q%d_L%d_n%d" % (max(c[0]), max(c[1] or [0]), c[2], c[3])
                                                   for c in CASES])
def test_normal_equations_match_oracle(torch, dpd, orc, mo, co, L, n):
    y, t = _target(n, mo, co, L, seed=L)
    plan = dpd.Plan(mo, co, L, signals.aph_coeffs(mo, co, L, config_id=3))
    A, b = plan.ls_normal(_dev(torch, y), _dev(torch, t))
    Ar, br = orc.ls_normal(y, mo, co, L, t)
    _assert_ls(A.cpu().numpy(), b.cpu().numpy(), Ar, br, _t2(t))
    # Hermitian by construction
    An = A.cpu().numpy()
    assert np.array_equal(An, An.conj().T)


def test_normal_equations_full_size(torch, dpd, orc):
    """The headline basis (K = 33) over the benchmark's 2^24 samples plus a
    ragged tail of 777 (8192-sample slabs, the last one and its last tile
    short), every entry of A and b against the FP64 oracle."""
    mo = co = [1, 3, 5, 7]
    L, n = 4, (1 << 24) + 777
    y, t = _target(n, mo, co, L, seed=24)
    plan = dpd.Plan(mo, co, L, signals.aph_coeffs(mo, co, L, config_id=3))
    A, b = plan.ls_normal(_dev(torch, y), _dev(torch, t))
    Ar, br = orc.ls_normal(y, mo, co, L, t)
    _assert_ls(A.cpu().numpy(), b.cpu().numpy(), Ar, br, _t2(t), "K=33 2^24+777")


def test_normal_equations_two_pair_groups_full_slabs(torch, dpd, orc):
    """K = 57 (8 column tiles: the tile pairs split into two groups of two
    waves, so each FP32 accumulator adds 512 eight-sample steps of a full
    8192-sample slab): 192 rows of 8 x 8192 + 777 samples -- enough slabs
    (192 x 9 = 1728, over six per CU on 256 CUs) that the library picks its
    largest slab -- every entry against the sum of per-row FP64 oracle calls."""
    mo = co = [1, 3, 5, 7, 9, 11, 13]
    L, rows, n = 4, 192, 8 * 8192 + 777
    y = np.stack([signals.ofdm_16qam(n, config_id=43, stream_id=r) for r in range(rows)])
    t = np.stack([signals.ofdm_16qam(n, config_id=44, stream_id=r) for r in range(rows)])
    plan = dpd.Plan(mo, co, L, signals.aph_coeffs(mo, co, L, config_id=3))
    A, b = plan.ls_normal(_dev(torch, y), _dev(torch, t))
    K = plan.K
    Ar, br = np.zeros((K, K), complex), np.zeros(K, complex)
    for r in range(rows):
        a1, b1 = orc.ls_normal(y[r], mo, co, L, t[r])
        Ar += a1
        br += b1
    _assert_ls(A.cpu().numpy(), b.cpu().numpy(), Ar, br, _t2(t), "K=57 8192-sample slabs")


def test_rows_scale_and_stride(torch, dpd, orc):
    mo, co, L, rows, n, ld = [1, 3, 5], [1, 3], 4, 3, 5000, 5008
    scale = 0.1
    yb = np.zeros((rows, ld), np.complex64)
    tb = np.zeros((rows, ld), np.complex64)
    for r in range(rows):
        yb[r, :n] = signals.ofdm_16qam(n, config_id=41, stream_id=r) * 10
        tb[r, :n] = signals.ofdm_16qam(n, config_id=42, stream_id=r)
    plan = dpd.Plan(mo, co, L, signals.aph_coeffs(mo, co, L, config_id=3))
    yd, td = _dev(torch, yb), _dev(torch, tb)
    A, b = plan.ls_normal(yd[:, :n], td[:, :n], y_scale=scale)
    K = A.shape[0]
    Ar, br = np.zeros((K, K), complex), np.zeros(K, complex)
    for r in range(rows):
        a1, b1 = orc.ls_normal(scale * yb[r, :n].astype(np.complex128), mo, co, L, tb[r, :n])
        Ar += a1
        br += b1
    _assert_ls(A.cpu().numpy(), b.cpu().numpy(), Ar, br, _t2(tb[:, :n]), "rows, scale, stride")


def test_empty_and_limits(torch, dpd):
    plan = dpd.Plan([1, 3], [1], 2, signals.aph_coeffs([1, 3], [1], 2))
    e = torch.empty(0, dtype=torch.complex64, device="cuda")
    A, b = plan.ls_normal(e, e)
    assert not A.abs().any() and not b.abs().any()
    big = dpd.Plan([1, 3, 5, 7, 9, 11], [1, 3, 5, 7, 9, 11], 8, signals.aph_coeffs([1, 3, 5, 7, 9, 11],
                                                                                   [1, 3, 5, 7, 9, 11], 8))
    with pytest.raises(dpd.DPDError):   # K = 97 > 95
        big.ls_normal(_dev(torch, np.ones(10)), _dev(torch, np.ones(10)))


def test_deterministic(torch, dpd):
    mo, co, L, n = [1, 3, 5, 7], [1, 3, 5, 7], 4, 50000
    y, t = _target(n, mo, co, L, seed=9)
    plan = dpd.Plan(mo, co, L, signals.aph_coeffs(mo, co, L))
    A1, b1 = plan.ls_normal(_dev(torch, y), _dev(torch, t))
    A2, b2 = plan.ls_normal(_dev(torch, y), _dev(torch, t))
    assert torch.equal(A1, A2) and torch.equal(b1, b2)


@pytest.mark.parametrize("mo,co,L", [([1, 3, 5, 7], [1, 3, 5, 7], 4),          # K = 33: factor in LDS
                                     ([1, 3, 5, 7, 9], [1, 3, 5, 7, 9], 8)])   # K = 81: factor in the workspace
def test_solve_matches_numpy(torch, dpd, orc, mo, co, L):
    n = 20000
    y, t = _target(n, mo, co, L, seed=2)
    Ar, br = orc.ls_normal(y, mo, co, L, t)
    Ad = torch.from_numpy(Ar).cuda()
    bd = torch.from_numpy(br).cuda()
    for ridge in (0.0, 1e-6):
        h, info = dpd.ls_solve(Ad, bd, ridge)
        assert int(info.item()) == 0
        K = Ar.shape[0]
        ref = np.linalg.solve(Ar + ridge * np.mean(np.real(np.diag(Ar))) * np.eye(K), br)
        # FP64 Cholesky vs LU agree to ~cond * 1e-16; h is rounded to complex64
        rel = np.linalg.norm(h.cpu().numpy() - ref) / np.linalg.norm(ref)
        assert rel <= 1e-6, (ridge, rel)


@pytest.mark.parametrize("K", [1, 2, 33, 56, 57, 63, 64, 65, 130, 300])
def test_solve_random_sizes(torch, dpd, K):
    """Every solve kernel against numpy on a random Hermitian positive definite
    matrix: four waves up to K = 56, then one wave with the factor in LDS up to
    K = 64 and 2, 4 and 8 rows per lane beyond."""
    rng = np.random.default_rng(K)
    X = rng.standard_normal((2 * K + 8, K)) + 1j * rng.standard_normal((2 * K + 8, K))
    A = X.conj().T @ X
    A = (A + A.conj().T) / 2
    b = rng.standard_normal(K) + 1j * rng.standard_normal(K)
    h, info = dpd.ls_solve(torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda(), 1e-3)
    assert int(info.item()) == 0
    ref = np.linalg.solve(A + 1e-3 * np.mean(np.real(np.diag(A))) * np.eye(K), b)
    rel = np.linalg.norm(h.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert rel <= 1e-6, rel


def test_solve_reports_indefinite(torch, dpd):
    K = 5
    A = -torch.eye(K, dtype=torch.complex128, device="cuda")
    b = torch.ones(K, dtype=torch.complex128, device="cuda")
    h, info = dpd.ls_solve(A, b)
    assert int(info.item()) == 1
    assert torch.isnan(h.real).all()
    A2 = torch.eye(K, dtype=torch.complex128, device="cuda")
    A2[2, 2] = 0
    _, info2 = dpd.ls_solve(A2, b)
    assert int(info2.item()) == 3
    # the same through the one-wave kernel (K above the four-wave limit)
    K = 60
    A3 = torch.eye(K, dtype=torch.complex128, device="cuda")
    A3[41, 41] = -1
    h3, info3 = dpd.ls_solve(A3, torch.ones(K, dtype=torch.complex128, device="cuda"))
    assert int(info3.item()) == 42
    assert torch.isnan(h3.real).all()


def test_recovers_generating_coefficients(torch, dpd, orc):
    """t = D_h(y) exactly (FP64 oracle): GPU normal equations + GPU solve give
    coefficients whose model reproduces t to far below the FP32 noise floor of
    the fit (the solution itself carries cond(A) x the normal-equation error)."""
    mo, co, L, n = [1, 3, 5], [1, 3], 3, 40000
    y = signals.ofdm_16qam(n, config_id=51)
    h = signals.aph_coeffs(mo, co, L, config_id=51)
    t = orc.forward(y, mo, co, L, h).astype(np.complex64)
    plan = dpd.Plan(mo, co, L, h)
    A, b = plan.ls_normal(_dev(torch, y), _dev(torch, t))
    hh, info = dpd.ls_solve(A, b)
    assert int(info.item()) == 0
    fit = orc.forward(y, mo, co, L, hh.cpu().numpy())
    nmse = 10 * np.log10(np.sum(np.abs(fit - t) ** 2) / np.sum(np.abs(t) ** 2))
    assert nmse <= -80.0, nmse


def test_indirect_learning_linearizes_the_synthetic_pa(torch, dpd):
    """Drive level RMS 0.2: the polynomial PA of Eq. (3) turns non-physical
    above |u| ~ 0.9, and at RMS 0.25 the predistorted peaks pass it (the FP64
    oracle loop oscillates there too); at RMS 0.2 the FP64 loop reaches
    -52 dB after one iteration and stays."""
    from paper_1612_09001_amd import ila

    from paper_1612_09001_amd import spectral

    x = _dev(torch, signals.ofdm_16qam(1 << 18, config_id=5, rms=0.2))
    est = ila.ILA(x, [1, 3, 5, 7], [1, 3, 5, 7], 4)
    xh = x.cpu().numpy()

    def regrowth():
        _, y = est.transmit()
        return spectral.distortion_regrowth_db(y.cpu().numpy() / est.pa.gain, xh)

    e0, r0 = est.nmse_db(), regrowth()
    errs = []
    for _ in range(3):
        assert int(est.step().item()) == 0
        errs.append(est.nmse_db())
    r1 = regrowth()
    assert e0 > -25.0 and errs[0] <= -45.0 and errs[-1] <= -45.0, (e0, errs)
    # section 5.2 reports > 10 dB suppression of the spectral spurs
    assert r1 <= r0 - 10.0, (r0, r1)


def _oracle_chain(orc, x, orders, L, h):
    """PA output / gain of the FP64 transmitter chain for predistorter h."""
    import oracle.ila as oila

    _, y = oila.transmit(orc, x, orders, L, h)
    return y[0] / oila.GAIN


def test_indirect_learning_follows_the_fp64_loop(torch, dpd, orc):
    """The GPU loop's linearization error before and after each of three
    iterations within 0.5 dB of the same iteration composed from FP64 oracle
    calls (oracle forward, oracle normal equations, numpy solve)."""
    import oracle.ila as oila
    from paper_1612_09001_amd import ila

    orders, L = ([1, 3, 5, 7], [1, 3, 5, 7]), 4
    xh = signals.ofdm_16qam(1 << 16, config_id=5, stream_id=7, rms=0.2)
    est = ila.ILA(_dev(torch, xh), *orders, L)
    gpu = [est.nmse_db()]
    for _ in range(3):
        assert int(est.step().item()) == 0
        gpu.append(est.nmse_db())
    ref, _ = oila.run(orc, xh, orders, L, signals.identity_coeffs(*orders, L), 3, ridge=est.ridge)
    assert np.all(np.abs(np.array(gpu) - np.array(ref)) <= 0.5), (gpu, ref)


def test_indirect_learning_keeps_coefficients_when_the_solve_fails(torch, dpd):
    """A transmitter that outputs zeros makes the normal equations singular
    (without diagonal loading the solve reports info != 0): the predistorter
    keeps its coefficients."""
    from paper_1612_09001_amd import ila, pa

    orders, L = ([1, 3, 5], [1, 3]), 3
    x = _dev(torch, signals.ofdm_16qam(1 << 14, config_id=5, stream_id=8, rms=0.2))
    est = ila.ILA(x, *orders, L)
    assert int(est.step().item()) == 0
    e1 = est.nmse_db()
    est.pa.pa.set_coeffs(np.zeros_like(pa.pa_coeffs()))
    est.ridge = 0.0                 # A = diag(0, ..., 0, n): the first pivot is 0
    assert int(est.step().item()) != 0
    est.ridge = 1e-9
    est.pa.pa.set_coeffs(pa.pa_coeffs())
    e2 = est.nmse_db()
    assert np.isfinite(e2) and e2 == e1, (e1, e2)


def test_two_carrier_suppression(torch, dpd, orc):
    """Non-contiguous two-carrier signal (the Fig. 8(b) case of section 5.2):
    indirect learning suppresses the intermodulation in the gap between the
    carriers by more than 10 dB; the GPU chain's figures before and after are
    within 0.5 dB of the FP64 chain's for the same coefficients."""
    from paper_1612_09001_amd import ila, spectral

    orders, L = ([1, 3, 5, 7], [1, 3, 5, 7]), 4
    xh = signals.two_carrier(1 << 18, config_id=3, stream_id=5, rms=0.2)
    est = ila.ILA(_dev(torch, xh), *orders, L)
    band = spectral.TWO_CARRIER

    def both(h):
        _, y = est.transmit()
        g = spectral.distortion_regrowth_db(y.cpu().numpy() / est.pa.gain, xh, bands=band)
        o = spectral.distortion_regrowth_db(_oracle_chain(orc, xh, orders, L, h), xh, bands=band)
        return g, o

    g0, o0 = both(signals.identity_coeffs(*orders, L))
    for _ in range(3):
        assert int(est.step().item()) == 0      # every solve succeeds: the plan holds est.h
    g1, o1 = both(est.h.cpu().numpy())
    assert abs(g0 - o0) <= 0.5 and abs(g1 - o1) <= 0.5, (g0, o0, g1, o1)
    assert g1 <= g0 - 10.0, (g0, g1)


def test_graph_replay(torch, dpd):
    """dpd_ls_normal and dpd_ls_solve allocate nothing and launch only kernels
    (no memset), so they replay from a captured graph; every replay, with eager
    work in between, equals the eager result bitwise."""
    mo, co, L, n = [1, 3, 5, 7], [1, 3, 5, 7], 4, 30000
    y, t = _target(n, mo, co, L, seed=11)
    plan = dpd.Plan(mo, co, L, signals.aph_coeffs(mo, co, L))
    yd, td = _dev(torch, y), _dev(torch, t)
    K = plan.K
    A = torch.empty((K, K), dtype=torch.complex128, device="cuda")
    b = torch.empty(K, dtype=torch.complex128, device="cuda")
    h = torch.empty(K, dtype=torch.complex64, device="cuda")
    info = torch.empty((), dtype=torch.int32, device="cuda")
    wsb = dpd.dpd_ls_ws_size(plan.handle, 1, n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    swsb = dpd.dpd_ls_solve_ws_size(K)
    sws = torch.empty(swsb, dtype=torch.uint8, device="cuda")

    def run():
        st = dpd.current_stream()
        dpd.dpd_ls_normal(plan.handle, st, yd.data_ptr(), td.data_ptr(), 1, n, n, 1.0, ws.data_ptr(), wsb,
                          A.data_ptr(), b.data_ptr())
        dpd.dpd_ls_solve(st, K, A.data_ptr(), b.data_ptr(), 1e-9, sws.data_ptr(), swsb, h.data_ptr(),
                         info.data_ptr())

    run()
    torch.cuda.synchronize()
    ref_a, ref_h = A.clone(), h.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        run()                      # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            run()
    torch.cuda.synchronize()
    for r in range(4):
        A.fill_(complex(r, -r))     # eager work between replays
        h.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(A, ref_a) and torch.equal(h, ref_h), "replay %d" % r
        assert int(info.item()) == 0

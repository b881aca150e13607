"""Batched persistent multi-stream apply against the oracle and against the
per-stream launches; hipGraph replay; self-resetting work counter."""
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


@pytest.fixture(scope="module")
def mods(torch):
    from paper_1612_09001_amd import batch, dpd

    dpd.lib()
    return dpd, batch


SMALL_SPECS = [  # (n, P_max, L) -- ragged lengths, every class shape, fallbacks
    (0, 5, 3), (1, 5, 2), (7, 7, 8), (8191, 9, 8), (8192, 5, 1), (8193, 7, 4), (20000, 3, 6),
    (12345, 1, 5), (70001, 9, 2), (3, 11, 3), (5000, 5, 11), (65536, 7, 4), (1023, 9, 5),
    (16384, 9, 8), (16900, 7, 7), (24577, 3, 3), (511, 9, 8), (512, 7, 7), (513, 5, 3), (129, 3, 2),
    (256, 9, 1), (127, 7, 6),
]


def _check_streams(wl, z, orc, count=None):
    rng = np.random.default_rng(1)
    for s, (n, pmax, L) in enumerate(wl.specs):
        if n == 0:
            continue
        orders = signals.odd_orders(pmax)
        x = wl.stream_input(s)
        got = z[wl.offsets[s]:wl.offsets[s] + n]
        h = wl.coeffs_host[s]
        if count is None or n <= count:
            ref = orc.forward(x, orders, orders, L, h)
            assert_parity(got, ref, "stream %d" % s)
        else:
            # chunk (512-sample) edges: every 16th, and all in the first 32768 samples
            edges = (np.arange(1, n // 8192 + 1) * 8192)[:, None] + np.arange(-9, 9)[None, :]
            chunks = (np.arange(1, min(n, 32768) // 512 + 1) * 512)[:, None] + np.arange(-2, 2)[None, :]
            idx = np.unique(np.concatenate([np.arange(0, 20), np.arange(n - 20, n), edges.reshape(-1),
                                            chunks.reshape(-1)]))
            idx = idx[(idx >= 0) & (idx < n)]
            idx = np.unique(np.concatenate([idx, rng.integers(0, n, count)]))
            assert_parity(got[idx], orc.forward_at(x, orders, orders, L, h, idx), "stream %d" % s)


@pytest.mark.parametrize("S", [2, 4, 8])
def test_small_batch_matches_oracle_and_each(torch, mods, orc, S):
    dpd, batch = mods
    wl = batch.BatchWorkload(SMALL_SPECS, config_id=70)
    b = batch.Batch(wl.streams(), tune={"samples_per_thread": S, "grid_mult": 4})
    wl.z.fill_(complex(7.0, -7.0))
    b.apply()
    z1 = wl.z.cpu().numpy()
    _check_streams(wl, z1, orc)
    wl.z.fill_(complex(7.0, -7.0))
    b.apply_each()
    z2 = wl.z.cpu().numpy()
    assert np.array_equal(z1, z2), "persistent batch differs from per-stream launches"
    # padding slots between streams are never written
    for s, (n, _, _) in enumerate(wl.specs):
        if n % 2:
            assert z1[wl.offsets[s] + n] == np.complex64(complex(7.0, -7.0))
    b.close()


def test_many_short_streams(torch, mods, orc):
    """3000 streams of seeded random length 0..3000 (mostly ragged chunks), P_max
    1..11 and L 1..10 (classes outside the persistent kernel's included): every
    output against the oracle and bitwise against the per-stream launches, at
    the default launch shape (whole slots of blocks: the heavy/light split)."""
    dpd, batch = mods
    rng = np.random.default_rng(2024)
    specs = [(int(rng.integers(0, 3001)), int(rng.choice([1, 3, 5, 7, 9, 11])), int(rng.integers(1, 11)))
             for _ in range(3000)]
    wl = batch.BatchWorkload(specs, config_id=72)
    b = batch.Batch(wl.streams())
    wl.z.fill_(complex(7.0, -7.0))
    b.apply()
    z1 = wl.z.cpu().numpy()
    _check_streams(wl, z1, orc)
    wl.z.fill_(complex(7.0, -7.0))
    b.apply_each()
    assert np.array_equal(z1, wl.z.cpu().numpy()), "persistent batch differs from per-stream launches"
    b.close()


def _written(wl, z):
    """Concatenation of the stream regions (the padding between is never written)."""
    return np.concatenate([z[o:o + n] for o, (n, _, _) in zip(wl.offsets, wl.specs)])


def test_repeat_and_graph_replay(torch, mods):
    dpd, batch = mods
    wl = batch.BatchWorkload(SMALL_SPECS, config_id=71)
    b = batch.Batch(wl.streams())
    b.apply()
    ref = _written(wl, wl.z.cpu().numpy())
    for _ in range(3):
        wl.z.fill_(0)
        b.apply()
        assert np.array_equal(_written(wl, wl.z.cpu().numpy()), ref)
    g = torch.cuda.CUDAGraph()
    wl.z.fill_(0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        b.apply()
    for r in range(4):
        wl.z.fill_(complex(r, -r))          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_written(wl, wl.z.cpu().numpy()), ref), "replay %d" % r
    b.apply()
    assert np.array_equal(_written(wl, wl.z.cpu().numpy()), ref)


def test_invalid_descriptors(torch, mods):
    dpd, batch = mods
    x = torch.zeros(100, dtype=torch.complex64, device="cuda")
    c = torch.zeros(20, dtype=torch.complex64, device="cuda")
    bad = [
        dict(main_orders=[1, 17], conj_orders=[], L=2),   # order > 15 (mask bit 8)
        dict(main_orders=[], conj_orders=[1], L=2),       # no main branch
        dict(main_orders=[1], conj_orders=[], L=0),
        dict(main_orders=[1], conj_orders=[], L=17),
    ]
    for kw in bad:
        with pytest.raises(dpd.DPDError):
            batch.Batch([dict(kw, **{"in": x[:50], "out": x[50:], "n": 50, "coeffs": c})])
    with pytest.raises(dpd.DPDError):   # stream 1 writes over stream 0's input
        batch.Batch([dict(main_orders=[1], conj_orders=[], L=2, **{"in": x[:50], "out": x[50:], "n": 50, "coeffs": c}),
                     dict(main_orders=[1], conj_orders=[], L=2, **{"in": x[60:70], "out": x[:10], "n": 10, "coeffs": c})])


@pytest.fixture(scope="module")
def config4(torch, mods, orc):
    """The 256-stream workload and its FP64 oracle outputs (computed once)."""
    dpd, batch = mods
    wl = batch.BatchWorkload(signals.batch_specs(), config_id=4)
    refs = []
    for s, (n, pmax, L) in enumerate(wl.specs):
        orders = signals.odd_orders(pmax)
        refs.append(orc.forward(wl.stream_input(s), orders, orders, L, wl.coeffs_host[s]))
    return wl, refs


# the library's default launch shape and the benchmark's autotuned ones
# (whole slots of blocks per CU: the heavy/light split with two, three and
# more slots)
@pytest.mark.parametrize("tune", [None, {"samples_per_thread": 8, "grid_mult": 16},
                                  {"samples_per_thread": 8, "grid_mult": 4},
                                  {"samples_per_thread": 8, "grid_mult": 2},
                                  {"samples_per_thread": 4, "grid_mult": 8}],
                         ids=["default", "S8_g16", "S8_g4", "S8_g2", "S4_g8"])
def test_config4_every_stream_full(torch, mods, config4, tune):
    """256 streams, lengths U[2^14, 2^20], P_max in {5,7,9}, L in {2..8}: every
    output of every stream against the FP64 oracle."""
    dpd, batch = mods
    wl, refs = config4
    b = batch.Batch(wl.streams(), tune=tune)
    S = (tune or {}).get("samples_per_thread", 8)
    ntiles, nblocks = b.info()
    assert ntiles == sum((n + 64 * S - 1) // (64 * S) for n, _, _ in wl.specs)
    wl.z.fill_(complex(7.0, -7.0))
    b.apply()
    z = wl.z.cpu().numpy()
    for s, (n, _, _) in enumerate(wl.specs):
        assert_parity(z[wl.offsets[s]:wl.offsets[s] + n], refs[s], "stream %d %s" % (s, tune))
    b.close()

"""Host ingestion: the chunked pinned-host pipeline (copies overlapped with
filtering on two streams, history carried across chunks) against the FP64
oracle over the whole stream."""
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


@pytest.mark.parametrize("chunk,nbuf", [(1 << 20, 2), (77777, 3)])
def test_pipeline_matches_oracle_and_carries_history(torch, orc, chunk, nbuf):
    from paper_1612_09001_amd import dpd, ingest

    mo = co = [1, 3, 5, 7]
    L, n = 4, 3000001
    x = signals.ofdm_16qam(n, config_id=81)
    h = signals.aph_coeffs(mo, co, L, config_id=81)
    plan = dpd.Plan(mo, co, L, h)
    pipe = ingest.HostPipeline(plan, chunk=chunk, nbuf=nbuf)
    xh = torch.from_numpy(x).pin_memory()
    zh = torch.empty(n, dtype=torch.complex64).pin_memory()
    pipe.run(xh, zh)
    z1 = zh.numpy().copy()
    assert_parity(z1, orc.forward(x, mo, co, L, h), "pipeline")
    # the same as one device call over the whole stream
    zd = plan.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(z1, zd)
    # without a reset the next run continues the stream: the second half of x ++ x
    pipe.run(xh, zh)
    xx = np.concatenate([x[-(L - 1):], x])
    assert_parity(zh.numpy(), orc.forward(xx, mo, co, L, h)[L - 1:], "continued")
    pipe.reset()
    pipe.run(xh, zh)
    assert np.array_equal(zh.numpy(), z1)


def test_rejects_pageable_buffers(torch):
    from paper_1612_09001_amd import dpd, ingest

    plan = dpd.Plan([1], [], 2, np.array([1, 0, 0], np.complex64))
    pipe = ingest.HostPipeline(plan, chunk=1024)
    with pytest.raises(ValueError):
        pipe.run(torch.zeros(10, dtype=torch.complex64), torch.zeros(10, dtype=torch.complex64))


def test_zero_copy_matches_oracle_and_device_call(torch, orc):
    from paper_1612_09001_amd import dpd, ingest

    mo, co = [1, 3, 5, 7], [1, 3]
    L, n = 5, 1000003
    x = signals.ofdm_16qam(n, config_id=82)
    h = signals.aph_coeffs(mo, co, L, config_id=82)
    plan = dpd.Plan(mo, co, L, h)
    xh = torch.from_numpy(x).pin_memory()
    zh = torch.zeros(n, dtype=torch.complex64).pin_memory()
    ingest.ZeroCopy(plan).run(xh, zh)
    z1 = zh.numpy().copy()
    assert_parity(z1, orc.forward(x, mo, co, L, h), "zero-copy")
    zd = plan.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(z1, zd)


def test_zero_copy_rejects_pageable(torch):
    from paper_1612_09001_amd import dpd, ingest

    plan = dpd.Plan([1], [], 2, np.array([1, 0, 0], np.complex64))
    with pytest.raises(ValueError):
        ingest.ZeroCopy(plan).run(torch.zeros(10, dtype=torch.complex64), torch.zeros(10, dtype=torch.complex64))

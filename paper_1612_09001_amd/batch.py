"""Batched multi-stream apply (many antennas, uneven lengths, own coefficients).

``Batch`` wraps ``dpd_batch_create`` / ``dpd_batch_apply``: one coefficient
precombine launch, one persistent launch over the full chunks of all streams
and one small launch for their ragged ends; graph-capturable (no allocation,
no host synchronization, no device state carried between calls).
``BatchWorkload`` builds the multi-antenna workload in two device arenas
(inputs, outputs) with 16-byte aligned stream offsets plus one coefficient
arena, from the seeded generators in ``signals``.
"""
from __future__ import annotations

import numpy as np

from . import dpd as _dpd
from . import signals


def orders_mask(orders) -> int:
    m = 0
    for p in orders:
        m |= 1 << ((int(p) - 1) // 2)
    return m


class Batch:
    """Streams: list of dicts with keys in, out (complex64 GPU tensors or raw
    device pointers with n), main_orders, conj_orders, L, coeffs (K complex64
    GPU tensor)."""

    def __init__(self, streams, tune=None):
        self._keep = []
        descs = []
        for s in streams:
            xin, xout, c = s["in"], s["out"], s["coeffs"]
            n = int(s.get("n", xin.numel() if hasattr(xin, "numel") else 0))
            ptr = lambda t: t if isinstance(t, int) else t.data_ptr()
            self._keep.extend([xin, xout, c])
            descs.append(_dpd.dpd_stream_desc(
                ptr(xin), ptr(xout), n, orders_mask(s["main_orders"]),
                orders_mask(s["conj_orders"]), int(s["L"]), 0, ptr(c)))
        t = None
        if tune is not None:
            t = _dpd.dpd_tune(tune.get("samples_per_thread", 8), 1, 256, tune.get("grid_mult", 16))
        self.handle = _dpd.dpd_batch_create(descs, t)
        self.n_streams = len(descs)

    def apply(self):
        _dpd.dpd_batch_apply(self.handle, _dpd.current_stream())

    def apply_each(self):
        _dpd.dpd_batch_apply_each(self.handle, _dpd.current_stream())

    def info(self):
        return _dpd.dpd_batch_info(self.handle)

    def close(self):
        if self.handle:
            _dpd.dpd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchWorkload:
    """Streams drawn by ``signals.batch_specs`` (lengths, P_max, L), laid out in
    one input and one output arena (offsets rounded up to 2 samples = 16 B)."""

    def __init__(self, specs, config_id=4, device="cuda"):
        import torch

        self.specs = specs
        offs, off = [], 0
        for n, _, _ in specs:
            offs.append(off)
            off += (n + 1) & ~1
        self.offsets = offs
        self.total = off
        host = np.zeros(max(off, 2), dtype=np.complex64)
        self.coeffs_host = []
        coff, cofs = 0, []
        for s, (n, pmax, L) in enumerate(specs):
            host[offs[s]:offs[s] + n] = signals.ofdm_16qam(n, config_id=config_id, stream_id=s)
            orders = signals.odd_orders(pmax)
            h = signals.aph_coeffs(orders, orders, L, config_id=config_id, stream_id=s)
            self.coeffs_host.append(h)
            cofs.append(coff)
            coff += (h.size + 1) & ~1
        chost = np.zeros(max(coff, 2), dtype=np.complex64)
        for s, h in enumerate(self.coeffs_host):
            chost[cofs[s]:cofs[s] + h.size] = h
        self.x_host = host
        self.x = torch.from_numpy(host).to(device)
        self.z = torch.zeros_like(self.x)
        self.c = torch.from_numpy(chost).to(device)
        self.coeff_offsets = cofs

    def streams(self, out=None):
        out = self.z if out is None else out
        res = []
        for s, (n, pmax, L) in enumerate(self.specs):
            orders = signals.odd_orders(pmax)
            k = self.coeffs_host[s].size
            res.append({"in": self.x[self.offsets[s]:self.offsets[s] + n] if n else self.x[:0],
                        "out": out[self.offsets[s]:self.offsets[s] + n] if n else out[:0],
                        "n": n, "main_orders": orders, "conj_orders": orders, "L": L,
                        "coeffs": self.c[self.coeff_offsets[s]:self.coeff_offsets[s] + k]})
        return res

    def stream_input(self, s):
        n = self.specs[s][0]
        return self.x_host[self.offsets[s]:self.offsets[s] + n]

    def samples(self) -> int:
        return int(sum(n for n, _, _ in self.specs))

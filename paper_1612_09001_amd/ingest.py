"""Host ingestion: predistort a stream held in pinned host memory.

The paper's mobile GPUs read the samples in place from zero-copy host memory
(section 3.3.1); on a discrete GPU the samples cross the host link either way.
``HostPipeline`` cuts the stream into chunks and, on nbuf streams of default
priority (one device buffer pair each), overlaps the host-to-device copy of
one chunk and the device-to-host copy of another with the filtering of a
third.  Three buffers let a chunk's input copy start without waiting for the
output copy two chunks back (measured on 2^25 samples: 2^21-sample chunks,
31.8 GB/s each way with three buffers against 28.5 with two; the copies alone
reach 33.9).  Each chunk is filtered by
``dpd_apply_hist`` with the L-1 samples before it carried on the device, so
the chunked result equals one call over the whole stream; the filtering of
consecutive chunks is chained by events, the copies are not.  PyTorch supplies
the pinned buffers, device buffers, streams and copies; the filtering is
libdpd's.

``ZeroCopy`` is the paper's zero-copy form on this machine: the kernel reads
and writes the pinned host buffers in place through their device mapping, so
every sample crosses the host link inside the kernel and nothing is staged in
HBM.  On MI355X it measured about 1.5 times the rate of the copy pipeline
(41.7 against 28.5 GB/s each way with two buffers, 2^25 samples).
"""
from __future__ import annotations

import ctypes

from . import dpd as _dpd


def _hip_runtime():
    """The HIP runtime this process already uses (the one torch and libdpd are
    bound to), opened by its loaded path so no second copy is loaded."""
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64.so" in line:
                return ctypes.CDLL(line.split()[-1])
    raise RuntimeError("the HIP runtime is not loaded (initialise torch.cuda first)")


def device_pointer(host_tensor) -> int:
    """Device address of a pinned host tensor's memory (hipHostGetDevicePointer);
    raises if the memory is not mapped into the device's address space."""
    if host_tensor.is_cuda or not host_tensor.is_pinned():
        raise ValueError("expected a pinned host tensor")
    rt = _hip_runtime()
    rt.hipHostGetDevicePointer.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_uint]
    rt.hipHostGetDevicePointer.restype = ctypes.c_int
    dev = ctypes.c_void_p()
    err = rt.hipHostGetDevicePointer(ctypes.byref(dev), ctypes.c_void_p(host_tensor.data_ptr()), 0)
    if err != 0 or not dev.value:
        raise RuntimeError("hipHostGetDevicePointer failed (hip error %d)" % err)
    return dev.value


class ZeroCopy:
    """Predistort pinned host memory in place: one ``dpd_apply`` whose input
    and output are the device mappings of the host buffers (the analog of the
    paper's zero-copy buffers, section 3.3.1)."""

    def __init__(self, plan):
        self.plan = plan

    def run(self, x_host, z_host):
        """z_host[:] = predistorter(x_host) (zero pre-history); both pinned
        complex64 host tensors of one length.  Returns when z_host is written."""
        import torch

        if (x_host.dtype != torch.complex64 or z_host.dtype != torch.complex64
                or x_host.numel() != z_host.numel() or not x_host.is_contiguous() or not z_host.is_contiguous()):
            raise TypeError("x_host and z_host must be contiguous complex64 tensors of one length")
        xd, zd = device_pointer(x_host), device_pointer(z_host)
        s = torch.cuda.current_stream()
        s.synchronize()     # earlier work on the buffers is done
        _dpd.dpd_apply(self.plan.handle, s.cuda_stream, xd, zd, x_host.numel())
        s.synchronize()
        return z_host


class HostPipeline:
    def __init__(self, plan, chunk: int = 1 << 21, nbuf: int = 3):
        import torch

        if chunk < 1 or nbuf < 1:
            raise ValueError("chunk and nbuf must be positive")
        self.torch = torch
        self.plan = plan
        self.chunk = int(chunk)
        self.nbuf = int(nbuf)
        self.streams = [torch.cuda.Stream() for _ in range(self.nbuf)]
        self.din = [torch.empty(self.chunk, dtype=torch.complex64, device="cuda") for _ in range(self.nbuf)]
        self.dout = [torch.empty(self.chunk, dtype=torch.complex64, device="cuda") for _ in range(self.nbuf)]
        self.hist = torch.zeros(max(plan.L - 1, 1), dtype=torch.complex64, device="cuda")

    def reset(self):
        """Forget the carried history (the next run starts from zeros)."""
        self.hist.zero_()
        self.torch.cuda.synchronize()

    def run(self, x_host, z_host):
        """z_host[:] = predistorter(x_host); both pinned complex64 host tensors
        of the same length.  Returns after the last copy has landed."""
        torch = self.torch
        if (x_host.dtype != torch.complex64 or z_host.dtype != torch.complex64 or x_host.is_cuda
                or z_host.is_cuda or x_host.numel() != z_host.numel()):
            raise TypeError("x_host and z_host must be host complex64 tensors of one length")
        if not (x_host.is_pinned() and z_host.is_pinned()):
            raise ValueError("host buffers must be pinned (torch pin_memory=True)")
        x = x_host.reshape(-1)
        z = z_host.reshape(-1)
        n = x.numel()
        hp = self.hist.data_ptr() if self.plan.L > 1 else 0
        torch.cuda.current_stream().synchronize()   # the history and buffers are ready
        prev = None
        for i, t0 in enumerate(range(0, n, self.chunk)):
            b = i % self.nbuf
            s = self.streams[b]
            m = min(self.chunk, n - t0)
            with torch.cuda.stream(s):
                self.din[b][:m].copy_(x[t0:t0 + m], non_blocking=True)
                if prev is not None:
                    s.wait_event(prev)
                _dpd.dpd_apply_hist(self.plan.handle, s.cuda_stream, self.din[b].data_ptr(),
                                    self.dout[b].data_ptr(), m, hp)
                prev = torch.cuda.Event()
                prev.record(s)
                z[t0:t0 + m].copy_(self.dout[b][:m], non_blocking=True)
        for s in self.streams:
            s.synchronize()
        return z_host

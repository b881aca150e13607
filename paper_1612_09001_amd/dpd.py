"""Python binding of libdpd (the C ABI of include/dpd.h).

Argument marshalling only: every step of the predistorter runs in the HIP
kernels of libdpd.so.  PyTorch provides device memory (complex64 CUDA/HIP
tensors) and the current stream.  The module refuses to work without the
built library -- there is no fallback.

The ``dpd_*`` functions mirror the C entry points one to one; ``Plan`` and
``Batch`` wrap them for tensors.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdpd.so")

DPD_OK, DPD_EINVAL, DPD_EUNSUPPORTED, DPD_ENOMEM, DPD_EHIP = range(5)


class DPDError(RuntimeError):
    def __init__(self, status: int, where: str, hip: int = 0):
        self.status = status
        self.hip = hip
        msg = "%s failed: %s" % (where, _status_string(status))
        if status == DPD_EHIP:
            msg += " (hipError %d)" % hip
        super().__init__(msg)


class dpd_tune(ctypes.Structure):
    _fields_ = [("samples_per_thread", ctypes.c_int32), ("stage_lds", ctypes.c_int32),
                ("block", ctypes.c_int32), ("grid_mult", ctypes.c_int32)]


class dpd_stream_desc(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("main_mask", ctypes.c_uint32), ("conj_mask", ctypes.c_uint32),
                ("L", ctypes.c_int32), ("pad_", ctypes.c_int32), ("coeffs_dev", ctypes.c_void_p)]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)

_SIGS = {
    "dpd_create": [_i32p, _i32, _i32p, _i32, _i32, _f32p, ctypes.POINTER(_vp)],
    "dpd_destroy": [_vp],
    "dpd_num_coeffs": [_vp, _i32p],
    "dpd_set_coeffs": [_vp, _f32p],
    "dpd_set_coeffs_async": [_vp, _f32p, _vp],
    "dpd_set_coeffs_device": [_vp, _vp, _vp],
    "dpd_set_coeffs_device_if": [_vp, _vp, _vp, _vp],
    "dpd_set_tune": [_vp, ctypes.POINTER(dpd_tune)],
    "dpd_get_tune": [_vp, ctypes.POINTER(dpd_tune)],
    "dpd_apply": [_vp, _vp, _vp, _vp, _i64],
    "dpd_apply_rows": [_vp, _vp, _vp, _vp, _i64, _i64, _i64],
    "dpd_apply_coeffs": [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64],
    "dpd_apply_hist": [_vp, _vp, _vp, _vp, _i64, _vp],
    "dpd_backward_ws_size": [_vp, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
    "dpd_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64, _vp, ctypes.c_size_t],
    "dpd_backward_noalloc": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64],
    "dpd_batch_create": [ctypes.POINTER(dpd_stream_desc), _i32, ctypes.POINTER(dpd_tune),
                         ctypes.POINTER(_vp)],
    "dpd_batch_apply": [_vp, _vp],
    "dpd_batch_apply_each": [_vp, _vp],
    "dpd_batch_info": [_vp, ctypes.POINTER(_i64), _i32p],
    "dpd_batch_destroy": [_vp],
    "dpd_loss_ws_size": [_i64, ctypes.POINTER(ctypes.c_size_t)],
    "dpd_loss_grad": [_vp, _vp, _vp, _i64, ctypes.c_float, _vp, _vp, _vp, ctypes.c_size_t],
    "dpd_cascade_loss_grad": [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64, ctypes.c_float, _vp, _vp, _vp,
                              ctypes.c_size_t],
    "dpd_cascade_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64],
    "dpd_transmit_loss_grad": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64, ctypes.c_float, _vp, _vp, _vp,
                               ctypes.c_size_t],
    "dpd_transmit_backward": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64, _vp, ctypes.c_size_t],
    "dpd_learn_step_ws_size": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "dpd_learn_step": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                       ctypes.c_float, _vp, _vp, _vp, _i64, _i64, _i64, ctypes.c_float, _vp, _vp, _vp,
                       ctypes.c_size_t],
    "dpd_learn_step_dev": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, _vp, _vp, _vp, _i64, _i64, _i64, ctypes.c_float, _vp, _vp, _vp,
                           ctypes.c_size_t],
    "dpd_adam_step": [_vp, _vp, _vp, _vp, _vp, _i64, _i32, ctypes.c_float, ctypes.c_float,
                      ctypes.c_float, ctypes.c_float],
    "dpd_ls_ws_size": [_vp, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
    "dpd_ls_normal": [_vp, _vp, _vp, _vp, _i64, _i64, _i64, ctypes.c_float, _vp, ctypes.c_size_t, _vp, _vp],
    "dpd_ls_solve_ws_size": [_i32, ctypes.POINTER(ctypes.c_size_t)],
    "dpd_ls_solve": [_vp, _i32, _vp, _vp, ctypes.c_double, _vp, ctypes.c_size_t, _vp, _vp],
    "dpd_copy": [_vp, _vp, _vp, _i64],
}

# Symbols the header declares (checked by the CPU test-suite).
EXPORTED = sorted(list(_SIGS) + ["dpd_status_string", "dpd_last_hip_error", "dpd_version"])


def lib():
    """Load libdpd.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdpd.so is not built (%s); run `python -m "
                               "paper_1612_09001_amd.build` first" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.dpd_status_string.argtypes = [ctypes.c_int]
        L.dpd_status_string.restype = ctypes.c_char_p
        L.dpd_last_hip_error.restype = ctypes.c_int
        L.dpd_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _status_string(st: int) -> str:
    return lib().dpd_status_string(int(st)).decode()


def _check(st: int, where: str):
    if st != DPD_OK:
        raise DPDError(st, where, lib().dpd_last_hip_error() if st == DPD_EHIP else 0)


def dpd_version() -> str:
    return lib().dpd_version().decode()


def dpd_status_string(st: int) -> str:
    return _status_string(st)


def dpd_last_hip_error() -> int:
    return int(lib().dpd_last_hip_error())


def _orders_arr(orders):
    arr = (ctypes.c_int32 * max(1, len(orders)))(*[int(o) for o in orders])
    return arr, len(orders)


def _coeff_floats(coeffs) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.complex64))
    return c.view(np.float32)


# ---------------------------------------------------------------- C ABI ---

def dpd_create(main_orders, conj_orders, L: int, coeffs_host) -> int:
    mo, nm = _orders_arr(main_orders)
    co, nc = _orders_arr(conj_orders)
    f = _coeff_floats(coeffs_host)
    K = (len(main_orders) + len(conj_orders)) * int(L) + 1
    if f.size != 2 * K:
        raise ValueError("expected %d complex coefficients, got %d" % (K, f.size // 2))
    h = _vp()
    _check(lib().dpd_create(mo, nm, co if nc else None, nc, int(L), f.ctypes.data_as(_f32p),
                            ctypes.byref(h)), "dpd_create")
    return h.value


def dpd_destroy(plan: int):
    _check(lib().dpd_destroy(plan), "dpd_destroy")


def dpd_num_coeffs(plan: int) -> int:
    k = ctypes.c_int32()
    _check(lib().dpd_num_coeffs(plan, ctypes.byref(k)), "dpd_num_coeffs")
    return k.value


def dpd_set_coeffs(plan: int, coeffs_host):
    f = _coeff_floats(coeffs_host)
    if f.size != 2 * dpd_num_coeffs(plan):
        raise ValueError("coefficient count does not match the plan")
    _check(lib().dpd_set_coeffs(plan, f.ctypes.data_as(_f32p)), "dpd_set_coeffs")


def dpd_set_coeffs_async(plan: int, coeffs_host, stream: int):
    f = _coeff_floats(coeffs_host)
    if f.size != 2 * dpd_num_coeffs(plan):
        raise ValueError("coefficient count does not match the plan")
    _check(lib().dpd_set_coeffs_async(plan, f.ctypes.data_as(_f32p), stream), "dpd_set_coeffs_async")


def dpd_set_coeffs_device(plan: int, coeffs_dev_ptr: int, stream: int):
    _check(lib().dpd_set_coeffs_device(plan, coeffs_dev_ptr, stream), "dpd_set_coeffs_device")


def dpd_set_coeffs_device_if(plan: int, coeffs_dev_ptr: int, flag_dev_ptr: int, stream: int):
    _check(lib().dpd_set_coeffs_device_if(plan, coeffs_dev_ptr, flag_dev_ptr, stream), "dpd_set_coeffs_device_if")


def dpd_set_tune(plan: int, samples_per_thread=4, stage_lds=1, block=256, grid_mult=8):
    t = dpd_tune(samples_per_thread, stage_lds, block, grid_mult)
    _check(lib().dpd_set_tune(plan, ctypes.byref(t)), "dpd_set_tune")


def dpd_get_tune(plan: int) -> dict:
    t = dpd_tune()
    _check(lib().dpd_get_tune(plan, ctypes.byref(t)), "dpd_get_tune")
    return {f: getattr(t, f) for f, _ in dpd_tune._fields_}


def dpd_apply(plan: int, stream: int, in_ptr: int, out_ptr: int, n: int):
    _check(lib().dpd_apply(plan, stream, in_ptr, out_ptr, int(n)), "dpd_apply")


def dpd_apply_rows(plan, stream, in_ptr, out_ptr, rows, n, ld):
    _check(lib().dpd_apply_rows(plan, stream, in_ptr, out_ptr, int(rows), int(n), int(ld)),
           "dpd_apply_rows")


def dpd_apply_coeffs(plan, stream, coeffs_ptr, in_ptr, out_ptr, rows, n, ld):
    _check(lib().dpd_apply_coeffs(plan, stream, coeffs_ptr, in_ptr, out_ptr, int(rows), int(n),
                                  int(ld)), "dpd_apply_coeffs")


def dpd_apply_hist(plan, stream, in_ptr, out_ptr, n, hist_ptr):
    _check(lib().dpd_apply_hist(plan, stream, in_ptr, out_ptr, int(n), hist_ptr), "dpd_apply_hist")


def dpd_backward_ws_size(plan, rows, n) -> int:
    b = ctypes.c_size_t()
    _check(lib().dpd_backward_ws_size(plan, int(rows), int(n), ctypes.byref(b)),
           "dpd_backward_ws_size")
    return b.value


def dpd_backward(plan, stream, coeffs_ptr, x_ptr, gz_ptr, gx_ptr, gc_ptr, rows, n, ld, ws_ptr,
                 ws_bytes):
    _check(lib().dpd_backward(plan, stream, coeffs_ptr, x_ptr, gz_ptr, gx_ptr, gc_ptr, int(rows),
                              int(n), int(ld), ws_ptr, int(ws_bytes)), "dpd_backward")


def dpd_backward_noalloc(plan, stream, coeffs_ptr, x_ptr, gz_ptr, gx_ptr, gc_ptr, rows, n, ld):
    _check(lib().dpd_backward_noalloc(plan, stream, coeffs_ptr, x_ptr, gz_ptr, gx_ptr, gc_ptr, int(rows), int(n),
                                      int(ld)), "dpd_backward_noalloc")


def dpd_batch_create(descs, tune: dpd_tune | None = None) -> int:
    arr = (dpd_stream_desc * len(descs))(*descs)
    h = _vp()
    _check(lib().dpd_batch_create(arr, len(descs), ctypes.byref(tune) if tune else None,
                                  ctypes.byref(h)), "dpd_batch_create")
    return h.value


def dpd_batch_apply(batch, stream):
    _check(lib().dpd_batch_apply(batch, stream), "dpd_batch_apply")


def dpd_batch_apply_each(batch, stream):
    _check(lib().dpd_batch_apply_each(batch, stream), "dpd_batch_apply_each")


def dpd_batch_info(batch):
    nt = ctypes.c_int64()
    nb = ctypes.c_int32()
    _check(lib().dpd_batch_info(batch, ctypes.byref(nt), ctypes.byref(nb)), "dpd_batch_info")
    return nt.value, nb.value


def dpd_batch_destroy(batch):
    _check(lib().dpd_batch_destroy(batch), "dpd_batch_destroy")


def dpd_loss_ws_size(n) -> int:
    b = ctypes.c_size_t()
    _check(lib().dpd_loss_ws_size(int(n), ctypes.byref(b)), "dpd_loss_ws_size")
    return b.value


def dpd_loss_grad(stream, y_ptr, x_ptr, n, scale, loss_ptr, gy_ptr, ws_ptr, ws_bytes):
    _check(lib().dpd_loss_grad(stream, y_ptr, x_ptr, int(n), float(scale), loss_ptr, gy_ptr, ws_ptr,
                               int(ws_bytes)), "dpd_loss_grad")


def dpd_cascade_loss_grad(plan_a, plan_b, stream, z_ptr, x_ptr, rows, n, ld, scale, loss_ptr, gy_ptr, ws_ptr,
                          ws_bytes):
    _check(lib().dpd_cascade_loss_grad(plan_a, plan_b, stream, z_ptr, x_ptr, int(rows), int(n), int(ld),
                                       float(scale), loss_ptr, gy_ptr, ws_ptr, int(ws_bytes)),
           "dpd_cascade_loss_grad")


def dpd_cascade_backward(plan_a, plan_b, stream, z_ptr, gy_ptr, gz_ptr, rows, n, ld):
    _check(lib().dpd_cascade_backward(plan_a, plan_b, stream, z_ptr, gy_ptr, gz_ptr, int(rows), int(n), int(ld)),
           "dpd_cascade_backward")


def dpd_transmit_loss_grad(plan_p, plan_a, plan_b, stream, coeffs_ptr, x_ptr, z_ptr, rows, n, ld, scale, loss_ptr,
                           gy_ptr, ws_ptr, ws_bytes):
    _check(lib().dpd_transmit_loss_grad(plan_p, plan_a, plan_b, stream, coeffs_ptr, x_ptr, z_ptr, int(rows), int(n),
                                        int(ld), float(scale), loss_ptr, gy_ptr, ws_ptr, int(ws_bytes)),
           "dpd_transmit_loss_grad")


def dpd_transmit_backward(plan_p, plan_a, plan_b, stream, x_ptr, z_ptr, gy_ptr, gz_ptr, gc_ptr, rows, n, ld,
                          ws_ptr, ws_bytes):
    _check(lib().dpd_transmit_backward(plan_p, plan_a, plan_b, stream, x_ptr, z_ptr, gy_ptr, gz_ptr, gc_ptr,
                                       int(rows), int(n), int(ld), ws_ptr, int(ws_bytes)),
           "dpd_transmit_backward")


def dpd_learn_step_ws_size(plan_p) -> int:
    b = ctypes.c_size_t()
    _check(lib().dpd_learn_step_ws_size(plan_p, ctypes.byref(b)), "dpd_learn_step_ws_size")
    return b.value


def dpd_learn_step(plan_p, plan_a, plan_b, stream, coeffs_ptr, m_ptr, v_ptr, step, lr, beta1, beta2, eps, x_ptr,
                   z_ptr, gy_ptr, rows, n, ld, scale, loss_ptr, gc_ptr, ws_ptr, ws_bytes):
    _check(lib().dpd_learn_step(plan_p, plan_a, plan_b, stream, coeffs_ptr, m_ptr, v_ptr, int(step), float(lr),
                                float(beta1), float(beta2), float(eps), x_ptr, z_ptr, gy_ptr, int(rows), int(n),
                                int(ld), float(scale), loss_ptr, gc_ptr, ws_ptr, int(ws_bytes)), "dpd_learn_step")


def dpd_learn_step_dev(plan_p, plan_a, plan_b, stream, coeffs_ptr, m_ptr, v_ptr, step_ptr, lr, beta1, beta2, eps,
                       x_ptr, z_ptr, gy_ptr, rows, n, ld, scale, loss_ptr, gc_ptr, ws_ptr, ws_bytes):
    _check(lib().dpd_learn_step_dev(plan_p, plan_a, plan_b, stream, coeffs_ptr, m_ptr, v_ptr, step_ptr, float(lr),
                                    float(beta1), float(beta2), float(eps), x_ptr, z_ptr, gy_ptr, int(rows), int(n),
                                    int(ld), float(scale), loss_ptr, gc_ptr, ws_ptr, int(ws_bytes)),
           "dpd_learn_step_dev")


def dpd_adam_step(stream, p_ptr, g_ptr, m_ptr, v_ptr, count, step, lr, beta1=0.9, beta2=0.999,
                  eps=1e-8):
    _check(lib().dpd_adam_step(stream, p_ptr, g_ptr, m_ptr, v_ptr, int(count), int(step), float(lr),
                               float(beta1), float(beta2), float(eps)), "dpd_adam_step")


def dpd_ls_ws_size(plan, rows, n) -> int:
    b = ctypes.c_size_t()
    _check(lib().dpd_ls_ws_size(plan, int(rows), int(n), ctypes.byref(b)), "dpd_ls_ws_size")
    return b.value


def dpd_ls_normal(plan, stream, y_ptr, t_ptr, rows, n, ld, y_scale, ws_ptr, ws_bytes, a_ptr, b_ptr):
    _check(lib().dpd_ls_normal(plan, stream, y_ptr, t_ptr, int(rows), int(n), int(ld), float(y_scale), ws_ptr,
                               int(ws_bytes), a_ptr, b_ptr), "dpd_ls_normal")


def dpd_copy(stream, in_ptr, out_ptr, n):
    _check(lib().dpd_copy(stream, in_ptr, out_ptr, int(n)), "dpd_copy")


def dpd_ls_solve_ws_size(K) -> int:
    b = ctypes.c_size_t()
    _check(lib().dpd_ls_solve_ws_size(int(K), ctypes.byref(b)), "dpd_ls_solve_ws_size")
    return b.value


def dpd_ls_solve(stream, K, a_ptr, b_ptr, ridge, ws_ptr, ws_bytes, h_ptr, info_ptr):
    _check(lib().dpd_ls_solve(stream, int(K), a_ptr, b_ptr, float(ridge), ws_ptr, int(ws_bytes), h_ptr,
                              info_ptr), "dpd_ls_solve")


def ls_solve(A, b, ridge=0.0):
    """Cholesky solve of (A + ridge * mean(diag A) I) h = b on the device.
    A: (K, K) complex128 GPU tensor (Hermitian), b: (K,) complex128.  Returns
    (h complex64 (K,), info int32 GPU scalar: 0 = ok, j+1 = not positive
    definite at column j)."""
    torch = _torch()
    if (not isinstance(A, torch.Tensor) or not A.is_cuda or A.dtype != torch.complex128 or A.dim() != 2
            or A.shape[0] != A.shape[1]):
        raise TypeError("A must be a square complex128 GPU tensor")
    K = A.shape[0]
    if not isinstance(b, torch.Tensor) or not b.is_cuda or b.dtype != torch.complex128 or b.numel() != K:
        raise TypeError("b must be a complex128 GPU tensor of K values")
    A = A.contiguous()
    b = b.contiguous()
    h = torch.empty(K, dtype=torch.complex64, device=A.device)
    info = torch.empty((), dtype=torch.int32, device=A.device)
    wsb = dpd_ls_solve_ws_size(K)
    ws = torch.empty(wsb, dtype=torch.uint8, device=A.device)
    dpd_ls_solve(current_stream(), K, A.data_ptr(), b.data_ptr(), ridge, ws.data_ptr(), wsb, h.data_ptr(),
                 info.data_ptr())
    return h, info


# ------------------------------------------------------- tensor wrappers ---

def _torch():
    import torch
    return torch


def current_stream() -> int:
    torch = _torch()
    return int(torch.cuda.current_stream().cuda_stream)


def _dev_c64(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.complex64:
        raise TypeError("%s must be a complex64 GPU tensor" % name)
    return t


class Plan:
    """One predistorter: order sets, L and coefficients (section 2.2 layout)."""

    def __init__(self, main_orders, conj_orders, L, coeffs):
        self.main_orders = [int(p) for p in main_orders]
        self.conj_orders = [int(q) for q in conj_orders]
        self.L = int(L)
        self.K = (len(self.main_orders) + len(self.conj_orders)) * self.L + 1
        self.handle = dpd_create(self.main_orders, self.conj_orders, self.L, coeffs)

    def close(self):
        if self.handle:
            dpd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_coeffs(self, coeffs, ordered=False):
        """Device coefficients: stream-ordered on torch's current stream.  Host
        coefficients: the device-wide update, or with ordered=True the update
        ordered on the current stream (dpd_set_coeffs_async)."""
        torch = _torch()
        if isinstance(coeffs, torch.Tensor) and coeffs.is_cuda:
            c = _dev_c64(coeffs, "coeffs").contiguous()
            if c.numel() != self.K:
                raise ValueError("expected %d coefficients" % self.K)
            dpd_set_coeffs_device(self.handle, c.data_ptr(), current_stream())
        elif ordered:
            dpd_set_coeffs_async(self.handle, coeffs, current_stream())
        else:
            dpd_set_coeffs(self.handle, coeffs)

    def set_tune(self, **kw):
        dpd_set_tune(self.handle, **kw)

    def get_tune(self):
        return dpd_get_tune(self.handle)

    def apply(self, x, out=None):
        """Eq. (1) on a 1-D stream or on each row of a 2-D (rows, n) tensor."""
        torch = _torch()
        x = _dev_c64(x, "x")
        if x.dim() == 1:
            x = x.contiguous()
            out = torch.empty_like(x) if out is None else out
            dpd_apply(self.handle, current_stream(), x.data_ptr(), out.data_ptr(), x.numel())
            return out
        if x.dim() != 2 or x.stride(1) != 1:
            raise ValueError("x must be 1-D or a row-major 2-D tensor")
        out = torch.empty_like(x) if out is None else out
        if out.stride() != x.stride():
            raise ValueError("out must have the strides of x")
        dpd_apply_rows(self.handle, current_stream(), x.data_ptr(), out.data_ptr(), x.shape[0],
                       x.shape[1], x.stride(0))
        return out

    def apply_coeffs(self, coeffs, x, out=None):
        torch = _torch()
        x = _dev_c64(x, "x")
        c = _dev_c64(coeffs, "coeffs").contiguous()
        if c.numel() != self.K:
            raise ValueError("expected %d coefficients" % self.K)
        x2 = x.reshape(1, -1) if x.dim() == 1 else x
        if x2.stride(1) != 1:
            raise ValueError("rows must be contiguous")
        out = torch.empty_like(x) if out is None else out
        o2 = out.reshape(1, -1) if out.dim() == 1 else out
        dpd_apply_coeffs(self.handle, current_stream(), c.data_ptr(), x2.data_ptr(), o2.data_ptr(),
                         x2.shape[0], x2.shape[1], x2.stride(0))
        return out

    def apply_hist(self, x, hist, out=None):
        torch = _torch()
        x = _dev_c64(x, "x").contiguous()
        out = torch.empty_like(x) if out is None else out
        hp = 0
        if self.L > 1:
            hist = _dev_c64(hist, "hist")
            if hist.numel() != self.L - 1 or not hist.is_contiguous():
                raise ValueError("hist must be a contiguous tensor of L-1 samples")
            hp = hist.data_ptr()
        dpd_apply_hist(self.handle, current_stream(), x.data_ptr(), out.data_ptr(), x.numel(), hp)
        return out

    def backward(self, x, grad_z, coeffs=None, want_dx=True, want_dcoeffs=True):
        """Gradients (dE/dRe + j dE/dIm) of a real loss E with respect to the
        inputs and the coefficients, given grad_z = dE/dz."""
        torch = _torch()
        x = _dev_c64(x, "x")
        gz = _dev_c64(grad_z, "grad_z")
        x2 = x.reshape(1, -1) if x.dim() == 1 else x
        g2 = gz.reshape(1, -1) if gz.dim() == 1 else gz
        if x2.shape != g2.shape or x2.stride() != g2.stride() or x2.stride(1) != 1:
            raise ValueError("x and grad_z must have the same row-major layout")
        rows, n, ld = x2.shape[0], x2.shape[1], x2.stride(0)
        gx = torch.empty_like(x) if want_dx else None
        gc = torch.empty(self.K, dtype=torch.complex64, device=x.device) if want_dcoeffs else None
        ws_bytes = dpd_backward_ws_size(self.handle, rows, n)
        ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=x.device)
        cp = 0
        if coeffs is not None:
            c = _dev_c64(coeffs, "coeffs").contiguous()
            cp = c.data_ptr()
        dpd_backward(self.handle, current_stream(), cp, x2.data_ptr(), g2.data_ptr(),
                     gx.data_ptr() if gx is not None else 0, gc.data_ptr() if gc is not None else 0,
                     rows, n, ld, ws.data_ptr(), ws_bytes)
        return gx, gc

    def ls_normal(self, y, t, y_scale=1.0):
        """Normal equations (Psi^H Psi, Psi^H t) of the least-squares fit of
        this plan's basis on input y_scale * y to target t (section 2.2,
        Eq. 2): (K, K) and (K,) complex128 GPU tensors.  y, t: complex64,
        1-D or rows x n."""
        torch = _torch()
        y = _dev_c64(y, "y")
        t = _dev_c64(t, "t")
        y2 = y.reshape(1, -1) if y.dim() == 1 else y
        t2 = t.reshape(1, -1) if t.dim() == 1 else t
        if y2.shape != t2.shape or y2.stride() != t2.stride() or y2.stride(1) != 1:
            raise ValueError("y and t must have the same row-major layout")
        rows, n, ld = y2.shape[0], y2.shape[1], y2.stride(0)
        A = torch.empty((self.K, self.K), dtype=torch.complex128, device=y.device)
        b = torch.empty(self.K, dtype=torch.complex128, device=y.device)
        wsb = dpd_ls_ws_size(self.handle, rows, n)
        ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=y.device)
        dpd_ls_normal(self.handle, current_stream(), y2.data_ptr(), t2.data_ptr(), rows, n, ld, y_scale,
                      ws.data_ptr(), wsb, A.data_ptr(), b.data_ptr())
        return A, b

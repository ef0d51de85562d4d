"""Python binding of libdbp (MI355X digital backpropagation), argument marshalling only.

Every step of the split-step path runs in the HIP kernels of lib/libdbp.so;
this module converts Python/torch arguments into the C ABI of include/dbp.h
(pointers, sizes and the current HIP stream).  PyTorch provides device memory
and streams.  There is no fallback: if the library is not built, or a call
fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32, c_void_p
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libdbp.so")

SSFM, ESSFM = 0, 1
LINEAR_FFT, LINEAR_FIR = 0, 1
FP32, FP32_FP64PHASE, BF16X3 = 0, 1, 2
FLAG_FORWARD, FLAG_WHOLE, FLAG_GRAD_SPARSE, FLAG_TUNE, FLAG_PERSISTENT = 0x1, 0x2, 0x4, 0x8, 0x10
MAX_TAPS = 129
NOALLOC_SCRATCH_BYTES = 32 << 20    # DBP_NOALLOC_SCRATCH_BYTES
MAX_FIR = 129

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported configuration",
          3: "workspace missing or too small", 4: "out of memory", 5: "HIP runtime error"}


class DbpError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [
        ("n_pol", c_int32), ("batch", c_int32), ("n_samples", c_int64), ("fs_thz", c_double),
        ("n_spans", c_int32), ("steps_per_span", c_int32), ("span_km", c_double),
        ("beta2_ps2_km", c_double), ("gamma_w_km", c_double), ("alpha_db_km", c_double),
        ("method", c_int32), ("n_taps", c_int32), ("taps", POINTER(c_float)), ("taps_per_step", c_int32),
        ("linear", c_int32), ("n_fir", c_int32), ("fir", POINTER(c_float)), ("fir_per_step", c_int32),
        ("fir_band_thz", c_double), ("block", c_int32), ("overlap", c_int32), ("steps_per_pass", c_int32),
        ("precision", c_int32), ("flags", c_uint32), ("spans_per_step", c_int32),
    ]


_lib = None


def lib():
    """The loaded libdbp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python paper_1507_00921_amd/_build.py)")
        L = ctypes.CDLL(LIB_PATH)
        L.dbp_desc_init.argtypes = [POINTER(Desc)]
        L.dbp_desc_init.restype = None
        L.dbp_plan.argtypes = [POINTER(Desc), POINTER(c_void_p)]
        L.dbp_plan.restype = c_int32
        L.dbp_destroy.argtypes = [c_void_p]
        L.dbp_destroy.restype = None
        L.dbp_plan_geometry.argtypes = [c_void_p] + [POINTER(c_int32)] * 5
        L.dbp_plan_geometry.restype = c_int32
        L.dbp_plan_kernel.argtypes = [c_void_p]
        L.dbp_plan_kernel.restype = ctypes.c_char_p
        L.dbp_choose_geometry.argtypes = [POINTER(Desc)] + [POINTER(c_int32)] * 3
        L.dbp_choose_geometry.restype = c_int32
        L.dbp_schedule.argtypes = [POINTER(Desc), POINTER(c_double), POINTER(c_double), c_int32]
        L.dbp_schedule.restype = c_int32
        L.dbp_workspace_size.argtypes = [c_void_p, c_int32]
        L.dbp_workspace_size.restype = c_size_t
        L.dbp_backprop.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_size_t, c_void_p]
        L.dbp_backprop.restype = c_int32
        L.dbp_backprop_noalloc.argtypes = [c_void_p] * 6
        L.dbp_backprop_noalloc.restype = c_int32
        L.dbp_backprop_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.dbp_backprop_grad.restype = c_int32
        L.dbp_backprop_save.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                        c_void_p]
        L.dbp_backprop_save.restype = c_int32
        L.dbp_backprop_grad_saved.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                              c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.dbp_backprop_grad_saved.restype = c_int32
        L.dbp_plan_batch.argtypes = [POINTER(Desc), c_int32, POINTER(c_void_p)]
        L.dbp_plan_batch.restype = c_int32
        L.dbp_batch_offsets.argtypes = [c_void_p, POINTER(c_int64), c_int32]
        L.dbp_batch_offsets.restype = c_int32
        L.dbp_backprop_batch.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.dbp_backprop_batch.restype = c_int32
        L.dbp_batch_geometry.argtypes = [c_void_p, c_int32] + [POINTER(c_int32)] * 3
        L.dbp_batch_geometry.restype = c_int32
        L.dbp_batch_status.argtypes = [c_void_p, POINTER(c_int32)]
        L.dbp_batch_status.restype = c_int32
        L.dbp_fir_taps.argtypes = [POINTER(Desc), c_int32, POINTER(c_float)]
        L.dbp_fir_taps.restype = c_int32
        L.dbp_rx_create.argtypes = [POINTER(Desc), c_int64, POINTER(c_void_p)]
        L.dbp_rx_create.restype = c_int32
        L.dbp_rx_info.argtypes = [c_void_p, POINTER(c_int64)] + [POINTER(c_int32)] * 4
        L.dbp_rx_info.restype = c_int32
        L.dbp_rx_push.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        L.dbp_rx_push.restype = c_int32
        L.dbp_rx_reset.argtypes = [c_void_p, c_void_p]
        L.dbp_rx_reset.restype = c_int32
        L.dbp_rx_destroy.argtypes = [c_void_p]
        L.dbp_rx_destroy.restype = None
        L.dbp_dsp_create.argtypes = [POINTER(DspDesc), c_int64, POINTER(c_void_p)]
        L.dbp_dsp_create.restype = c_int32
        L.dbp_dsp_info.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int64)]
        L.dbp_dsp_info.restype = c_int32
        L.dbp_dsp_resample.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        L.dbp_dsp_resample.restype = c_int32
        L.dbp_dsp_train.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
        L.dbp_dsp_train.restype = c_int32
        L.dbp_dsp_status.argtypes = [c_void_p, POINTER(c_int32)]
        L.dbp_dsp_status.restype = c_int32
        L.dbp_dsp_equalize.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.dbp_dsp_equalize.restype = c_int32
        L.dbp_dsp_cpr.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, POINTER(c_int64), c_void_p]
        L.dbp_dsp_cpr.restype = c_int32
        L.dbp_dsp_destroy.argtypes = [c_void_p]
        L.dbp_dsp_destroy.restype = None
        L.dbp_mse_create.argtypes = [c_int64, c_int32, c_int32, POINTER(c_double), c_double, POINTER(c_void_p)]
        L.dbp_mse_create.restype = c_int32
        L.dbp_mse_forward.argtypes = [c_void_p] * 5
        L.dbp_mse_forward.restype = c_int32
        L.dbp_mse_backward.argtypes = [c_void_p] * 4
        L.dbp_mse_backward.restype = c_int32
        L.dbp_mse_destroy.argtypes = [c_void_p]
        L.dbp_mse_destroy.restype = None
        L.dbp_status_string.argtypes = [c_int32]
        L.dbp_status_string.restype = ctypes.c_char_p
        L.dbp_version.argtypes = []
        L.dbp_version.restype = c_int32
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != 0:
        raise DbpError(status, what)


def make_desc(n_samples: int, n_spans: int, steps_per_span: int = 1, *, n_pol: int = 2,
              batch: int = 1, fs_thz: float = 0.056, span_km: float = 80.0,
              beta2_ps2_km: float = -21.682619, gamma_w_km: float = 1.3, alpha_db_km: float = 0.2,
              taps=None, taps_per_step: bool = False, fir=None, fir_per_step: bool = False,
              n_fir: int = 0, fir_band_thz: float = 0.0, linear: int = LINEAR_FFT, block: int = 0,
              overlap: int = 0,
              steps_per_pass: int = 0, precision: int = FP32_FP64PHASE, forward: bool = False,
              whole: bool = False, spans_per_step: int = 1, grad_sparse: bool = False, tune: bool = False,
              persistent: bool = False):
    """Build a Desc.  taps (ESSFM) and fir are host arrays kept alive on the returned object.
    tune: the planner times candidate geometries on the plan's size and keeps the fastest.
    persistent: all passes in one resident launch (calls on the plan must not overlap)."""
    d = Desc()
    lib().dbp_desc_init(ctypes.byref(d))
    d.n_pol, d.batch, d.n_samples, d.fs_thz = n_pol, batch, n_samples, fs_thz
    d.n_spans, d.steps_per_span, d.span_km = n_spans, steps_per_span, span_km
    d.beta2_ps2_km, d.gamma_w_km, d.alpha_db_km = beta2_ps2_km, gamma_w_km, alpha_db_km
    keep = []
    if taps is not None:
        t = np.ascontiguousarray(np.asarray(taps, dtype=np.float32))
        keep.append(t)
        d.method = ESSFM
        d.n_taps = t.shape[-1]
        d.taps = t.ctypes.data_as(POINTER(c_float))
        d.taps_per_step = 1 if taps_per_step else 0
    else:
        d.method = SSFM
        d.n_taps = 1
    d.linear = linear
    if linear == LINEAR_FIR:
        if fir is not None:
            f = np.ascontiguousarray(np.asarray(fir, dtype=np.complex64))
            keep.append(f)
            d.n_fir = f.shape[-1]
            d.fir = f.ctypes.data_as(POINTER(c_float))
            d.fir_per_step = 1 if fir_per_step else 0
        else:
            d.n_fir = n_fir
        d.fir_band_thz = fir_band_thz
    d.block, d.overlap, d.steps_per_pass = block, overlap, steps_per_pass
    d.precision = precision
    d.flags = ((FLAG_FORWARD if forward else 0) | (FLAG_WHOLE if whole else 0) |
               (FLAG_GRAD_SPARSE if grad_sparse else 0) | (FLAG_TUNE if tune else 0) |
               (FLAG_PERSISTENT if persistent else 0))
    d.spans_per_step = spans_per_step
    d._keep = keep
    return d


def schedule(desc: Desc):
    """Host-only FP64 step schedule (b, phi) the planner builds for desc."""
    m = desc.spans_per_step
    ns = desc.n_spans // m if m > 1 else desc.n_spans * desc.steps_per_span
    b = (c_double * ns)()
    p = (c_double * ns)()
    _check(lib().dbp_schedule(ctypes.byref(desc), b, p, ns), "dbp_schedule")
    return np.array(b[:]), np.array(p[:])


def choose_geometry(desc: Desc):
    """Host-only (block, overlap, steps_per_pass) the planner would choose."""
    nb, o, k = c_int32(), c_int32(), c_int32()
    _check(lib().dbp_choose_geometry(ctypes.byref(desc), ctypes.byref(nb), ctypes.byref(o),
                                     ctypes.byref(k)), "dbp_choose_geometry")
    return nb.value, o.value, k.value


def fir_taps(desc: Desc, step: int = 0):
    """Host-only: the FIR taps the planner designs for `step` (complex128 array)."""
    out = (c_float * (2 * desc.n_fir))()
    _check(lib().dbp_fir_taps(ctypes.byref(desc), step, out), "dbp_fir_taps")
    a = np.array(out[:], dtype=np.float64)
    return a[0::2] + 1j * a[1::2]


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """A dbp_plan: immutable geometry, schedule and device tables."""

    def __init__(self, desc: Desc):
        self.desc = desc
        h = c_void_p()
        _check(lib().dbp_plan(ctypes.byref(desc), ctypes.byref(h)), "dbp_plan")
        self._h = h
        nb, o, k, ns, npass = (c_int32() for _ in range(5))
        _check(lib().dbp_plan_geometry(h, ctypes.byref(nb), ctypes.byref(o), ctypes.byref(k),
                                       ctypes.byref(ns), ctypes.byref(npass)), "dbp_plan_geometry")
        self.block, self.overlap, self.steps_per_pass = nb.value, o.value, k.value
        self.n_steps, self.n_passes = ns.value, npass.value
        self.kernel = lib().dbp_plan_kernel(h).decode()
        self.shape = (desc.batch, desc.n_pol, desc.n_samples)

    def close(self):
        if getattr(self, "_h", None):
            lib().dbp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def workspace_size(self, grad: bool = False) -> int:
        return int(lib().dbp_workspace_size(self._h, 1 if grad else 0))

    def _check_field(self, t, name):
        import torch
        if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous complex64 CUDA tensor")
        if t.numel() != self.shape[0] * self.shape[1] * self.shape[2]:
            raise ValueError(f"{name} has {t.numel()} elements, plan expects {self.shape}")

    def workspace(self, grad: bool = False):
        import torch
        n = self.workspace_size(grad)
        return torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")

    def backprop(self, x, out=None, taps=None, fir=None, workspace=None, stream=None):
        """Run the plan on x (complex64 [batch][n_pol][L] on the GPU); returns out."""
        import torch
        self._check_field(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check_field(out, "output")
        if workspace is None:
            workspace = self.workspace()
        self._check_params(taps, fir)
        st = lib().dbp_backprop(self._h, _ptr(x), _ptr(out), _ptr(taps), _ptr(fir), _ptr(workspace),
                                workspace.numel(), _stream_ptr(stream))
        _check(st, "dbp_backprop")
        return out

    def persistent_status(self) -> int:
        """Error flags of the last persistent run (DBP_FLAG_PERSISTENT plans; synchronous)."""
        v = c_int32()
        _check(lib().dbp_batch_status(self._h, ctypes.byref(v)), "dbp_batch_status")
        return v.value

    def backprop_noalloc(self, x, out, taps=None, fir=None, stream=None):
        """Run the plan on x into the caller's out with the library's fixed device scratch as
        workspace (dbp_backprop_noalloc: no device allocation in the call).  Calls that
        overlap in time on one device share that scratch and must be serialized."""
        self._check_field(x, "input")
        self._check_field(out, "output")
        self._check_params(taps, fir)
        st = lib().dbp_backprop_noalloc(self._h, _ptr(x), _ptr(out), _ptr(taps), _ptr(fir),
                                        _stream_ptr(stream))
        _check(st, "dbp_backprop_noalloc")
        return out

    def _check_params(self, taps, fir):
        import torch
        ns = self.n_steps
        if taps is not None and (taps.dtype != torch.float32 or not taps.is_cuda or not taps.is_contiguous()
                                 or taps.numel() != ns * self.desc.n_taps):
            raise ValueError(f"taps must be a contiguous float32 CUDA tensor [{ns}][{self.desc.n_taps}]")
        if fir is not None and (fir.dtype != torch.complex64 or not fir.is_cuda or not fir.is_contiguous()
                                or fir.numel() != ns * self.desc.n_fir):
            raise ValueError(f"fir must be a contiguous complex64 CUDA tensor [{ns}][{self.desc.n_fir}]")

    def backprop_grad(self, x, grad_out, taps=None, fir=None, want_input=True, workspace=None,
                      stream=None):
        """Reverse-mode gradient through backprop(x, taps, fir) for upstream grad_out.

        Returns (grad_x or None, grad_taps [N_s][n_taps] float32 or None (SSFM),
        grad_fir [N_s][n_fir] complex64 or None (FFT-step plans)).  Complex gradients are
        dL/dRe + j dL/dIm.
        """
        import torch
        self._check_field(x, "input")
        self._check_field(grad_out, "grad_out")
        self._check_params(taps, fir)
        ns = self.n_steps
        gx = torch.empty_like(x) if want_input else None
        gt = (torch.empty(ns, self.desc.n_taps, dtype=torch.float32, device=x.device)
              if self.desc.method == ESSFM else None)
        gf = (torch.empty(ns, self.desc.n_fir, dtype=torch.complex64, device=x.device)
              if self.desc.linear == LINEAR_FIR else None)
        if workspace is None:
            workspace = self.workspace(grad=True)
        st = lib().dbp_backprop_grad(self._h, _ptr(x), _ptr(taps), _ptr(fir), _ptr(grad_out), _ptr(gx),
                                     _ptr(gt), _ptr(gf), _ptr(workspace), workspace.numel(),
                                     _stream_ptr(stream))
        _check(st, "dbp_backprop_grad")
        return gx, gt, gf

    def backprop_save(self, x, taps=None, fir=None, out=None, workspace=None, stream=None):
        """Forward pass that keeps what the reverse pass needs: returns (out, workspace);
        pass both, unchanged, to backprop_grad_saved (dbp_backprop_save)."""
        import torch
        self._check_field(x, "input")
        self._check_params(taps, fir)
        if out is None:
            out = torch.empty_like(x)
        self._check_field(out, "output")
        if workspace is None:
            workspace = self.workspace(grad=True)
        st = lib().dbp_backprop_save(self._h, _ptr(x), _ptr(out), _ptr(taps), _ptr(fir), _ptr(workspace),
                                     workspace.numel(), _stream_ptr(stream))
        _check(st, "dbp_backprop_save")
        return out, workspace

    def backprop_grad_saved(self, x, out, workspace, grad_out, taps=None, fir=None, want_input=True,
                            stream=None):
        """Reverse pass after backprop_save(x, taps, fir) -> (out, workspace), without running
        the forward steps again (dbp_backprop_grad_saved); returns as backprop_grad."""
        import torch
        self._check_field(x, "input")
        self._check_field(out, "output")
        self._check_field(grad_out, "grad_out")
        self._check_params(taps, fir)
        ns = self.n_steps
        gx = torch.empty_like(x) if want_input else None
        gt = (torch.empty(ns, self.desc.n_taps, dtype=torch.float32, device=x.device)
              if self.desc.method == ESSFM else None)
        gf = (torch.empty(ns, self.desc.n_fir, dtype=torch.complex64, device=x.device)
              if self.desc.linear == LINEAR_FIR else None)
        st = lib().dbp_backprop_grad_saved(self._h, _ptr(x), _ptr(out), _ptr(taps), _ptr(fir), _ptr(grad_out),
                                           _ptr(gx), _ptr(gt), _ptr(gf), _ptr(workspace), workspace.numel(),
                                           _stream_ptr(stream))
        _check(st, "dbp_backprop_grad_saved")
        return gx, gt, gf


class BatchPlan:
    """A dbp_plan_batch: many signals (one Desc each, batch = 1) in one packed buffer."""

    def __init__(self, descs):
        self.descs = list(descs)
        arr = (Desc * len(self.descs))(*self.descs)
        h = c_void_p()
        _check(lib().dbp_plan_batch(arr, len(self.descs), ctypes.byref(h)), "dbp_plan_batch")
        self._h = h
        n = len(self.descs)
        offs = (c_int64 * (n + 1))()
        _check(lib().dbp_batch_offsets(h, offs, n + 1), "dbp_batch_offsets")
        self.offsets = np.array(offs[:], dtype=np.int64)
        self.n_pol = self.descs[0].n_pol

    def close(self):
        if getattr(self, "_h", None):
            lib().dbp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def geometry(self, i):
        nb, o, k = c_int32(), c_int32(), c_int32()
        _check(lib().dbp_batch_geometry(self._h, i, ctypes.byref(nb), ctypes.byref(o), ctypes.byref(k)),
               "dbp_batch_geometry")
        return nb.value, o.value, k.value

    def workspace_size(self) -> int:
        return int(lib().dbp_workspace_size(self._h, 0))

    def workspace(self):
        import torch
        return torch.empty(max(self.workspace_size(), 1), dtype=torch.uint8, device="cuda")

    def pack(self, fields):
        """Host list of [n_pol][L_i] complex arrays -> packed complex64 CUDA tensor."""
        import torch
        flat = np.concatenate([np.asarray(f, dtype=np.complex64).reshape(-1) for f in fields])
        assert flat.size == self.offsets[-1]
        return torch.from_numpy(flat).cuda()

    def unpack(self, packed):
        """Packed tensor -> list of [n_pol][L_i] complex64 host arrays."""
        a = packed.cpu().numpy()
        return [a[self.offsets[i]:self.offsets[i + 1]].reshape(self.n_pol, -1)
                for i in range(len(self.descs))]

    def backprop(self, packed, out=None, workspace=None, stream=None):
        import torch
        if packed.dtype != torch.complex64 or not packed.is_cuda or packed.numel() != self.offsets[-1]:
            raise ValueError("packed input must be a complex64 CUDA tensor of the batch's total size")
        if out is None:
            out = torch.empty_like(packed)
        if workspace is None:
            workspace = self.workspace()
        st = lib().dbp_backprop_batch(self._h, _ptr(packed), _ptr(out), _ptr(workspace), workspace.numel(),
                                      _stream_ptr(stream))
        _check(st, "dbp_backprop_batch")
        return out

    def status(self) -> int:
        v = c_int32()
        _check(lib().dbp_batch_status(self._h, ctypes.byref(v)), "dbp_batch_status")
        return v.value


class Receiver:
    """A dbp_rx: the receiver mode (an unbounded stream pushed in chunks, fixed latency)."""

    def __init__(self, desc: Desc, chunk: int):
        self.desc = desc
        h = c_void_p()
        _check(lib().dbp_rx_create(ctypes.byref(desc), chunk, ctypes.byref(h)), "dbp_rx_create")
        self._h = h
        lat = c_int64()
        nb, o, k, npass = (c_int32() for _ in range(4))
        _check(lib().dbp_rx_info(h, ctypes.byref(lat), ctypes.byref(nb), ctypes.byref(o), ctypes.byref(k),
                                 ctypes.byref(npass)), "dbp_rx_info")
        self.latency = lat.value
        self.block, self.overlap, self.steps_per_pass, self.n_passes = nb.value, o.value, k.value, npass.value
        self.chunk = chunk
        self.n_pol = desc.n_pol

    def close(self):
        if getattr(self, "_h", None):
            lib().dbp_rx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, x, out=None, stream=None):
        """Push complex64 [n_pol][chunk] (CUDA); returns the output samples
        [i C - latency, (i + 1) C - latency) of push i."""
        import torch
        if x.dtype != torch.complex64 or not x.is_cuda or not x.is_contiguous() or \
                x.numel() != self.n_pol * self.chunk:
            raise ValueError(f"chunk must be a contiguous complex64 CUDA tensor of {self.n_pol} x {self.chunk}")
        if out is None:
            out = torch.empty_like(x)
        _check(lib().dbp_rx_push(self._h, _ptr(x), _ptr(out), _stream_ptr(stream)), "dbp_rx_push")
        return out

    def reset(self, stream=None):
        _check(lib().dbp_rx_reset(self._h, _stream_ptr(stream)), "dbp_rx_reset")


def receiver(chunk: int, n_spans: int, steps_per_span: int = 1, **kw) -> Receiver:
    return Receiver(make_desc(chunk, n_spans, steps_per_span, **kw), chunk)


def plan_batch(descs) -> BatchPlan:
    return BatchPlan(descs)


class DspDesc(ctypes.Structure):
    _fields_ = [("up", c_int32), ("down", c_int32), ("resample_taps", c_int32), ("kaiser_beta", c_double),
                ("eq_taps", c_int32), ("cpr_half_window", c_int32)]


class ReceiverDsp:
    """A dbp_dsp: resampling to two samples per symbol, least-squares butterfly equalizer,
    carrier-phase recovery and decisions after backpropagation (Sec. IV).  Fields are
    complex64 CUDA tensors [2][n]."""

    def __init__(self, n_in: int, up: int = 28, down: int = 25, resample_taps: int = 48, kaiser_beta: float = 8.0,
                 eq_taps: int = 15, cpr_half_window: int = 16):
        self.desc = DspDesc(up, down, resample_taps, kaiser_beta, eq_taps, cpr_half_window)
        h = c_void_p()
        _check(lib().dbp_dsp_create(ctypes.byref(self.desc), n_in, ctypes.byref(h)), "dbp_dsp_create")
        self._h = h
        no, ns = c_int64(), c_int64()
        _check(lib().dbp_dsp_info(h, ctypes.byref(no), ctypes.byref(ns)), "dbp_dsp_info")
        self.n_in, self.n_out, self.n_sym = n_in, no.value, ns.value

    def close(self):
        if getattr(self, "_h", None):
            lib().dbp_dsp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _field(t, n, what):
        import torch
        if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous() or t.numel() != 2 * n:
            raise ValueError(f"{what} must be a contiguous complex64 CUDA tensor [2][{n}]")

    def resample(self, x, out=None, stream=None):
        import torch
        self._field(x, self.n_in, "x")
        if out is None:
            out = torch.empty(2, self.n_out, dtype=torch.complex64, device=x.device)
        _check(lib().dbp_dsp_resample(self._h, _ptr(x), _ptr(out), _stream_ptr(stream)), "dbp_dsp_resample")
        return out

    def train(self, x2, sym, n_train: int, stream=None):
        """Least-squares butterfly taps [2][2][N] (complex64, device) from the first n_train symbols."""
        import torch
        self._field(x2, self.n_out, "x2")
        self._field(sym, self.n_sym, "sym")
        taps = torch.empty(2, 2, self.desc.eq_taps, dtype=torch.complex64, device=x2.device)
        _check(lib().dbp_dsp_train(self._h, _ptr(x2), _ptr(sym), n_train, _ptr(taps), _stream_ptr(stream)),
               "dbp_dsp_train")
        return taps

    def status(self) -> int:
        """Flags of the last completed training (bit 0: singular system; synchronous)."""
        v = c_int32()
        _check(lib().dbp_dsp_status(self._h, ctypes.byref(v)), "dbp_dsp_status")
        return v.value

    def equalize(self, x2, taps, out=None, stream=None):
        import torch
        self._field(x2, self.n_out, "x2")
        if taps.dtype != torch.complex64 or not taps.is_cuda or taps.numel() != 4 * self.desc.eq_taps:
            raise ValueError("taps must be a complex64 CUDA tensor [2][2][eq_taps]")
        if out is None:
            out = torch.empty(2, self.n_sym, dtype=torch.complex64, device=x2.device)
        _check(lib().dbp_dsp_equalize(self._h, _ptr(x2), _ptr(taps.contiguous()), _ptr(out), _stream_ptr(stream)),
               "dbp_dsp_equalize")
        return out

    def cpr(self, y, sym=None, n_ref: int = 0, out=None, stream=None):
        """(z, bit errors or None): phase-recovered symbols (the quarter turn resolved on the
        first n_ref transmitted symbols) and, with sym, the number of wrong decision bits."""
        import torch
        self._field(y, self.n_sym, "y")
        if sym is not None:
            self._field(sym, self.n_sym, "sym")
        if out is None:
            out = torch.empty_like(y)
        n = c_int64(-1)
        _check(lib().dbp_dsp_cpr(self._h, _ptr(y), _ptr(sym), n_ref, _ptr(out),
                                 ctypes.byref(n) if sym is not None else None, _stream_ptr(stream)), "dbp_dsp_cpr")
        return out, (n.value if sym is not None else None)


def receiver_dsp(n_in: int, **kw) -> ReceiverDsp:
    return ReceiverDsp(n_in, **kw)


class SymbolMse:
    """A dbp_mse: the loss head of the differentiation workload, mean |MF(z)[::2] / amp - s|^2
    over every symbol, with its reverse mode (Sec. IV footnote).  mf: the real receive filter on
    the length-n DFT grid (numpy); fields complex64 CUDA tensors [batch][n_pol][n], symbols
    [batch][n_pol][n / 2]."""

    def __init__(self, n_samples: int, n_pol: int, batch: int, mf, amplitude: float):
        mf = np.ascontiguousarray(mf, dtype=np.float64)
        if mf.shape != (n_samples,):
            raise ValueError(f"mf must have {n_samples} values")
        h = c_void_p()
        _check(lib().dbp_mse_create(n_samples, n_pol, batch, mf.ctypes.data_as(POINTER(c_double)), amplitude,
                                    ctypes.byref(h)), "dbp_mse_create")
        self._h = h
        self.n, self.n_pol, self.batch = n_samples, n_pol, batch
        self.generation = 0          # forward calls so far (the reverse mode uses the last one's residual)

    def close(self):
        if getattr(self, "_h", None):
            lib().dbp_mse_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, t, n, what, dtype=None):
        import torch
        want = (self.batch, self.n_pol, n)
        if t.dtype != (dtype or torch.complex64) or not t.is_cuda or not t.is_contiguous() or t.numel() != np.prod(want):
            raise ValueError(f"{what} must be a contiguous complex64 CUDA tensor {list(want)}")

    def forward(self, z, symbols, loss=None, stream=None):
        """Loss (float32 CUDA tensor [1]); keeps the residual for backward()."""
        import torch
        self._check(z, self.n, "z")
        self._check(symbols, self.n // 2, "symbols")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=z.device)
        _check(lib().dbp_mse_forward(self._h, _ptr(z), _ptr(symbols), _ptr(loss), _stream_ptr(stream)),
               "dbp_mse_forward")
        self.generation += 1
        return loss

    def backward(self, grad_loss=None, grad_z=None, stream=None):
        """dloss/dz (times the device scalar grad_loss) for the last forward()."""
        import torch
        if grad_z is None:
            grad_z = torch.empty(self.batch, self.n_pol, self.n, dtype=torch.complex64, device="cuda")
        self._check(grad_z, self.n, "grad_z")
        if grad_loss is not None and (grad_loss.dtype != torch.float32 or not grad_loss.is_cuda
                                      or grad_loss.numel() != 1):
            raise ValueError("grad_loss must be a float32 CUDA tensor of one value")
        g = grad_loss.contiguous() if grad_loss is not None else None
        _check(lib().dbp_mse_backward(self._h, _ptr(g), _ptr(grad_z), _stream_ptr(stream)), "dbp_mse_backward")
        return grad_z


def _mse_function():
    import torch

    class MseFunction(torch.autograd.Function):
        """loss = head.forward(z, symbols) with the library's reverse mode of the loss head."""

        @staticmethod
        def forward(ctx, z, symbols, head):
            loss = head.forward(z.contiguous(), symbols)
            ctx.head = head
            ctx.generation = head.generation
            return loss.reshape(())

        @staticmethod
        def backward(ctx, g):
            if ctx.head.generation != ctx.generation:
                raise RuntimeError("SymbolMse: another forward ran after this loss; its residual is gone")
            return ctx.head.backward(g.reshape(1).to(torch.float32)), None, None

    return MseFunction


_MseFunction = None


def mse_function():
    """The torch.autograd.Function wrapping SymbolMse.forward / backward."""
    global _MseFunction
    if _MseFunction is None:
        _MseFunction = _mse_function()
    return _MseFunction


def _autograd_function():
    import torch

    class DBPFunction(torch.autograd.Function):
        """out = plan.backprop(x, taps, fir) with a hand-written adjoint (FIR or FFT linear step).

        x: complex64 [batch][n_pol][L]; taps: float32 [N_s][n_taps] (ESSFM) or None;
        fir: complex64 [N_s][n_fir].  Gradients follow PyTorch's convention for
        complex tensors (dL/dRe + j dL/dIm), which is the library's.
        """

        @staticmethod
        def forward(ctx, x, taps, fir, plan):
            x = x.contiguous()
            ctx.plan = plan
            if plan.workspace_size(grad=True) > 0:
                # keep the forward's step states for the reverse pass (no forward step reruns)
                out, ctx.ws = plan.backprop_save(x, taps=taps, fir=fir)
                ctx.save_for_backward(x, taps, fir, out)
            else:
                out = plan.backprop(x, taps=taps, fir=fir)
                ctx.ws = None
                ctx.save_for_backward(x, taps, fir, None)
            return out

        @staticmethod
        def backward(ctx, g):
            x, taps, fir, out = ctx.saved_tensors
            if ctx.ws is not None:
                gx, gt, gf = ctx.plan.backprop_grad_saved(x, out, ctx.ws, g.contiguous(), taps=taps, fir=fir,
                                                          want_input=ctx.needs_input_grad[0])
            else:
                gx, gt, gf = ctx.plan.backprop_grad(x, g.contiguous(), taps=taps, fir=fir,
                                                    want_input=ctx.needs_input_grad[0])
            return (gx, gt if ctx.needs_input_grad[1] else None,
                    gf if ctx.needs_input_grad[2] and gf is not None else None, None)

    return DBPFunction


_DBPFunction = None


def dbp_function():
    """The torch.autograd.Function wrapping backprop / backprop_grad."""
    global _DBPFunction
    if _DBPFunction is None:
        _DBPFunction = _autograd_function()
    return _DBPFunction


def plan(n_samples: int, n_spans: int, steps_per_span: int = 1, **kw) -> Plan:
    return Plan(make_desc(n_samples, n_spans, steps_per_span, **kw))


def version() -> int:
    return int(lib().dbp_version())

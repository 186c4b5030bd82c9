"""Python binding of the MI355X volume-potential library (libvgconv.so).

Thin ctypes marshalling over the C ABI declared in include/vg.h: every step of
the computation (kernel precompute, FFT passes, multiplies) runs in the HIP
library.  PyTorch provides device memory and streams only.  There is no
fallback: importing this package fails if the library has not been built
(`python paper_1604_03155_amd/build.py`).

Method: Vico, Greengard, Ferrando, "Fast convolution with free-space Green's
functions" -- the truncated-kernel FFT convolution phi = g * f on the uniform
grid x_a = (a - N/2 + 1)/N of [-1/2, 1/2]^d (Section 4), with the kernel's
truncated Fourier transform from Tables 1 and 2.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "LIBRARY_PATH", "VGError", "Plan", "apply_batched", "batched_workspace_size", "check_workspace",
    "LAPLACE", "HELMHOLTZ", "FP32", "FP64", "status_string", "profiler_enable", "profiler_collect", "hbm_copy",
]

LIBRARY_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvgconv.so")

LAPLACE, HELMHOLTZ, BIHARMONIC, LAPLACE_HELMHOLTZ, CONVECTION = 0, 1, 2, 3, 4
FP32, FP64 = 0, 1
_TUNE = {"off": 0, "quick": 1, "full": 2}
_KERNELS = {"laplace": LAPLACE, "helmholtz": HELMHOLTZ, "biharmonic": BIHARMONIC, "laplace_helmholtz": LAPLACE_HELMHOLTZ,
            "convection": CONVECTION}

if not os.path.exists(LIBRARY_PATH):
    raise ImportError(f"{LIBRARY_PATH} is missing: build it with `python paper_1604_03155_amd/build.py`")

# torch is loaded first so that the library binds to the HIP runtime torch
# already carries: loading the library first would bring in a second HIP
# runtime (the system one), and the two then disagree about the devices.
import torch as _torch_mod  # noqa: E402,F401

_lib = ctypes.CDLL(LIBRARY_PATH)


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("L", ctypes.c_double), ("P", ctypes.c_int),
                ("tune", ctypes.c_int), ("keep_operator", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("h", ctypes.c_double * 3)]


class _Info(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("N", ctypes.c_int), ("kernel", ctypes.c_int), ("precision", ctypes.c_int),
                ("k", ctypes.c_double), ("L", ctypes.c_double), ("P", ctypes.c_int),
                ("precompute_ms", ctypes.c_double), ("table_bytes", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t), ("gradient_workspace_bytes", ctypes.c_size_t),
                ("tune", ctypes.c_int), ("tune_ms", ctypes.c_double), ("tune_candidates", ctypes.c_int),
                ("pad_bytes", ctypes.c_int), ("xcd_map", ctypes.c_int), ("four_step_L1", ctypes.c_int),
                ("generic_passes", ctypes.c_int), ("tune_cached", ctypes.c_int)]


class _LsResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("matvecs", ctypes.c_int), ("residual", ctypes.c_double),
                ("converged", ctypes.c_int)]


class _PassTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("bytes_per_launch", ctypes.c_double)]


_vp = ctypes.c_void_p
_sig = {
    "vg_plan_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(_vp)]),
    "vg_plan_create_ex": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.POINTER(_Opts), ctypes.POINTER(_vp)]),
    "vg_plan_destroy": (None, [_vp]),
    "vg_plan_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(_Info)]),
    "vg_workspace_size": (ctypes.c_size_t, [_vp]),
    "vg_gradient_workspace_size": (ctypes.c_size_t, [_vp]),
    "vg_apply": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vg_apply_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "vg_gradient": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "vg_batched_workspace_size": (ctypes.c_size_t, [ctypes.c_int, ctypes.POINTER(_vp)]),
    "vg_apply_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                        ctypes.POINTER(_vp), _vp, _vp]),
    "vg_plan_kernel_hat": (ctypes.c_int, [_vp, _vp]),
    "vg_plan_operator_entries": (ctypes.c_int, [_vp, _vp]),
    "vg_profiler_enable": (ctypes.c_int, [ctypes.c_int]),
    "vg_profiler_collect": (ctypes.c_int, [ctypes.POINTER(_PassTime), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "vg_hbm_copy": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp]),
    "vg_ls_workspace_size": (ctypes.c_size_t, [_vp]),
    "vg_real_workspace_size": (ctypes.c_size_t, [_vp]),
    "vg_apply_real": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vg_ls_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _vp, _vp,
                                   ctypes.POINTER(_LsResult)]),
    "vg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "vg_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sig)


def status_string(code: int) -> str:
    return _lib.vg_status_string(code).decode()


class VGError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.vg_last_error().decode()
        super().__init__(f"{where}: {status_string(code)}: {msg}")


def _check(code: int, where: str):
    if code != 0:
        raise VGError(code, where)


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def check_workspace(ws, need, device_index=None):
    """Validate a caller workspace: a contiguous, 256-byte aligned tensor of at
    least `need` bytes on the CUDA device `device_index` (None: any).  Returns
    its device pointer as a ctypes void pointer, or None for ws None (the
    library's own buffer)."""
    if ws is None:
        return None
    torch = _torch()
    if not isinstance(ws, torch.Tensor):
        raise TypeError("workspace must be a torch tensor")
    nbytes = ws.numel() * ws.element_size()
    if nbytes < need:
        raise ValueError(f"workspace holds {nbytes} bytes; this call needs {need}")
    if not ws.is_contiguous():
        raise ValueError("workspace must be contiguous")
    if not ws.is_cuda:
        raise ValueError("workspace must be a CUDA tensor")
    if device_index is not None and ws.device.index != device_index:
        raise ValueError(f"workspace is on cuda:{ws.device.index}, the arrays on cuda:{device_index}")
    if ws.data_ptr() % 256:
        raise ValueError("workspace must be 256-byte aligned")
    return _vp(ws.data_ptr())


class Plan:
    """A precomputed truncated-kernel convolution operator for one grid.

    d: 2 or 3; N: even points per side (h = 1/N); kernel: 'laplace',
    'helmholtz' (wavenumber k > 0), 'biharmonic' or 'laplace_helmholtz'
    (Delta (Delta + k^2), kernel g_k - g_0, k > 0) or 'convection' (Delta -
    2i h.grad for the vector h, |h| > 0; k is ignored and set to |h|) (Tables
    1-2); precision: 'fp32' (complex64 data, tables
    built in FP64 and rounded once) or 'fp64'.  L and P default to the paper's
    truncation radius (1.8 in 3D, 1.5 in 2D) and 4-fold oversampling."""

    def __init__(self, d, N, kernel="laplace", k=0.0, precision="fp32", L=None, P=None, tune="off",
                 keep_operator=False, stream=None, h=None):
        torch = _torch()
        self.d, self.N, self.kernel, self.k = int(d), int(N), kernel, float(k)
        self.precision = precision
        self._h = None
        hv = [0.0, 0.0, 0.0]
        if h is not None:
            hl = [float(x) for x in h]
            if len(hl) != self.d:
                raise ValueError(f"h must have {self.d} components")
            hv[:self.d] = hl
        opts = _Opts(FP64 if precision == "fp64" else FP32, float(L or 0.0), int(P or 0), _TUNE[tune],
                     1 if keep_operator else 0,
                     stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream,
                     (ctypes.c_double * 3)(*hv))
        h = _vp()
        _check(_lib.vg_plan_create_ex(self.d, self.N, _KERNELS[kernel], self.k, ctypes.byref(opts), ctypes.byref(h)),
               "vg_plan_create_ex")
        self._h = h
        info = _Info()
        _check(_lib.vg_plan_get_info(h, ctypes.byref(info)), "vg_plan_get_info")
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}
        self.dtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.k = self.info["k"]

    # -- housekeeping ------------------------------------------------------
    def close(self):
        if self._h:
            _lib.vg_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def shape(self):
        return (self.N,) * self.d

    def workspace_size(self, gradient=False):
        return int((_lib.vg_gradient_workspace_size if gradient else _lib.vg_workspace_size)(self._h))

    def new_workspace(self, gradient=False, device="cuda"):
        torch = _torch()
        return torch.empty(max(self.workspace_size(gradient), 1), dtype=torch.uint8, device=device)

    def _check_array(self, a, name, shape=None):
        torch = _torch()
        shape = shape or self.shape
        if not isinstance(a, torch.Tensor) or not a.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if a.dtype != self.dtype or tuple(a.shape) != tuple(shape) or not a.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {tuple(shape)}")

    # -- operations ---------------------------------------------------------
    def apply(self, f, out=None, workspace=None, stream=None):
        """phi = T * f (Section 4's discrete convolution)."""
        torch = _torch()
        self._check_array(f, "f")
        if out is None:
            out = torch.empty_like(f)
        self._check_array(out, "out")
        ws = check_workspace(workspace, self.workspace_size(), f.device.index)
        _check(_lib.vg_apply(self._h, _vp(f.data_ptr()), _vp(out.data_ptr()), ws, _stream_ptr(stream)), "vg_apply")
        return out

    def apply_noalloc(self, f, out, stream=None):
        """phi = T * f like apply(), with no device allocation: the workspace is
        the library's fixed per-GPU array (plans up to VG_NOALLOC_WORKSPACE_BYTES
        of workspace); calls that overlap on one GPU race."""
        self._check_array(f, "f")
        self._check_array(out, "out")
        _check(_lib.vg_apply_noalloc(self._h, _vp(f.data_ptr()), _vp(out.data_ptr()), _stream_ptr(stream)),
               "vg_apply_noalloc")
        return out

    def gradient(self, f, with_phi=True, phi=None, grad=None, workspace=None, stream=None):
        """Returns (phi or None, grad) with grad of shape (d,) + (N,)*d."""
        torch = _torch()
        self._check_array(f, "f")
        if grad is None:
            grad = torch.empty((self.d,) + self.shape, dtype=self.dtype, device=f.device)
        self._check_array(grad, "grad", (self.d,) + self.shape)
        if with_phi and phi is None:
            phi = torch.empty_like(f)
        if phi is not None:
            self._check_array(phi, "phi")
        ws = check_workspace(workspace, self.workspace_size(gradient=True), f.device.index)
        _check(_lib.vg_gradient(self._h, _vp(f.data_ptr()), _vp(phi.data_ptr()) if phi is not None else None,
                                _vp(grad.data_ptr()), ws, _stream_ptr(stream)), "vg_gradient")
        return phi, grad

    def apply_real(self, f, out=None, workspace=None, stream=None):
        """phi = T * f for a real density f and a real kernel (Laplace,
        biharmonic): float32 / float64 arrays of shape (N,)*d."""
        torch = _torch()
        rdt = torch.float64 if self.precision == "fp64" else torch.float32
        for a, name in ((f, "f"), (out, "out")):
            if a is None:
                continue
            if not isinstance(a, torch.Tensor) or not a.is_cuda:
                raise TypeError(f"{name} must be a CUDA tensor")
            if a.dtype != rdt or tuple(a.shape) != self.shape or not a.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {rdt} tensor of shape {self.shape}")
        if out is None:
            out = torch.empty_like(f)
        ws = check_workspace(workspace, self.real_workspace_size(), f.device.index)
        _check(_lib.vg_apply_real(self._h, _vp(f.data_ptr()), _vp(out.data_ptr()), ws, _stream_ptr(stream)),
               "vg_apply_real")
        return out

    def real_workspace_size(self):
        return int(_lib.vg_real_workspace_size(self._h))

    def ls_solve(self, q, phi_in, tol=1e-12, max_iter=500, sigma=None, workspace=None, stream=None):
        """Density sigma of the scattered field of the Lippmann-Schwinger
        equation -sigma + k^2 q (g_k * sigma) = -k^2 q phi_in (Section 5.3),
        by Bi-CGStab on the device.  Returns (sigma, info dict)."""
        torch = _torch()
        self._check_array(q, "q")
        self._check_array(phi_in, "phi_in")
        if sigma is None:
            sigma = torch.empty_like(phi_in)
        self._check_array(sigma, "sigma")
        res = _LsResult()
        ws = check_workspace(workspace, self.ls_workspace_size(), q.device.index)
        _check(_lib.vg_ls_solve(self._h, _vp(q.data_ptr()), _vp(phi_in.data_ptr()), _vp(sigma.data_ptr()),
                                float(tol), int(max_iter), ws, _stream_ptr(stream), ctypes.byref(res)), "vg_ls_solve")
        return sigma, {f: getattr(res, f) for f, _ in _LsResult._fields_}

    def ls_workspace_size(self):
        return int(_lib.vg_ls_workspace_size(self._h))

    def kernel_hat(self):
        """Khat on the octant [0, N]^d as complex128 numpy (Section 4); the
        convection kernel: on the whole box [0, 2N)^d."""
        import numpy as np
        n = 2 * self.N if self.kernel == "convection" else self.N + 1
        out = np.empty((n,) * self.d, dtype=np.complex128)
        _check(_lib.vg_plan_kernel_hat(self._h, _vp(out.ctypes.data)), "vg_plan_kernel_hat")
        return out

    def operator_entries(self):
        """T(n) on the octant [0, N)^d as complex128 numpy (needs keep_operator);
        the convection kernel: on all offsets |n_j| <= N - 1, index n + N - 1."""
        import numpy as np
        n = 2 * self.N - 1 if self.kernel == "convection" else self.N
        out = np.empty((n,) * self.d, dtype=np.complex128)
        _check(_lib.vg_plan_operator_entries(self._h, _vp(out.ctypes.data)), "vg_plan_operator_entries")
        return out


def profiler_enable(enable=True, dominant_only=False):
    """Record device time per pass of every apply / gradient call; with
    dominant_only, only of each call's pass with the most algorithmic bytes
    (two events per call instead of one per pass)."""
    _check(_lib.vg_profiler_enable((2 if dominant_only else 1) if enable else 0), "vg_profiler_enable")


def profiler_collect():
    """Wait for recorded passes; return [{name, launches, total_ms, bytes_per_launch}] and clear."""
    buf = (_PassTime * 64)()
    n = ctypes.c_int(0)
    _check(_lib.vg_profiler_collect(buf, 64, ctypes.byref(n)), "vg_profiler_collect")
    return [dict(name=buf[i].name.decode(), launches=buf[i].launches, total_ms=buf[i].total_ms,
                 bytes_per_launch=buf[i].bytes_per_launch) for i in range(n.value)]


def hbm_copy(dst, src, stream=None):
    """Streaming copy between two CUDA tensors of equal byte size."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    _check(_lib.vg_hbm_copy(_vp(dst.data_ptr()), _vp(src.data_ptr()), nbytes, _stream_ptr(stream)), "vg_hbm_copy")


def _handles(plans):
    arr = (_vp * len(plans))()
    for i, p in enumerate(plans):
        arr[i] = p.handle
    return arr


def batched_workspace_size(plans):
    return int(_lib.vg_batched_workspace_size(len(plans), _handles(plans)))


def apply_batched(plans, fs, outs=None, workspace=None, stream=None):
    """phi_i = T_i * f_i for a batch of plans of mixed size and kernel."""
    torch = _torch()
    if len(plans) != len(fs):
        raise ValueError("plans and densities differ in length")
    for p, f in zip(plans, fs):
        p._check_array(f, "f")
    if outs is None:
        outs = [torch.empty_like(f) for f in fs]
    for p, o in zip(plans, outs):
        p._check_array(o, "out")
    n = len(plans)
    fa = (_vp * n)(*[f.data_ptr() for f in fs])
    oa = (_vp * n)(*[o.data_ptr() for o in outs])
    ws = check_workspace(workspace, batched_workspace_size(plans), fs[0].device.index if fs else None)
    _check(_lib.vg_apply_batched(n, _handles(plans), fa, oa, ws, _stream_ptr(stream)), "vg_apply_batched")
    return outs

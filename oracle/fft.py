"""The oracle's own FP64 DFTs (test infrastructure only; see the package docstring).

fftn / ifftn: multi-dimensional transforms through the recursive mixed-radix
Cooley-Tukey FFT of fft.c (every axis in turn), with numpy's conventions:
forward X[k] = sum_j x[j] e^{-2 pi i j.k / n}, inverse carrying 1/prod(n).

dft_naive: the O(n^2) definition along one axis, the pin of the FFT.

fft.c is compiled with gcc into _fft.so next to it on first use (and by the
package build); a stale or missing library is rebuilt.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import tempfile
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fft.c")
_LIB = os.path.join(_HERE, "_fft.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile fft.c into _fft.so (gcc, OpenMP); returns the library path."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    fd, tmp = tempfile.mkstemp(prefix="_fft.", suffix=".so.tmp", dir=_HERE)
    os.close(fd)
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", _SRC, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        os.unlink(tmp)
        raise RuntimeError(f"oracle FFT build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            for name in ("oracle_fft_axis", "oracle_fft_nd"):
                getattr(lib, name).restype = ctypes.c_int
            lib.oracle_fft_axis.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                            ctypes.c_int, ctypes.c_int, ctypes.c_int]
            lib.oracle_fft_nd.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                          ctypes.c_int, ctypes.c_int]
            _lib = lib
    return _lib


def threads(workers=None):
    """OpenMP threads a transform uses: `workers`, else OMP_NUM_THREADS, else all cores."""
    if workers:
        return int(workers)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, os.cpu_count() or 1)


def _transform(a, sign, axes, workers):
    x = np.array(a, dtype=np.complex128, order="C", copy=True)
    if x.ndim == 0 or x.size == 0:
        return x
    shape = (ctypes.c_longlong * x.ndim)(*x.shape)
    lib = _load()
    axes = range(x.ndim) if axes is None else [ax % x.ndim for ax in axes]
    for ax in axes:
        if lib.oracle_fft_axis(x.ctypes.data, x.ndim, shape, ax, sign, threads(workers)) != 0:
            raise MemoryError("oracle FFT failed")
    return x


def fftn(a, axes=None, workers=None):
    """Forward DFT over `axes` (default: all), unnormalised."""
    return _transform(a, -1, axes, workers)


def ifftn(a, axes=None, workers=None):
    """Inverse DFT over `axes` (default: all), divided by the product of their lengths."""
    x = _transform(a, +1, axes, workers)
    axes = range(x.ndim) if axes is None else axes
    n = math.prod(x.shape[ax] for ax in axes)
    x /= n
    return x


def dft_naive(a, axis=-1, sign=-1, block=256):
    """X[k] = sum_j x[j] exp(sign 2 pi i (j k mod n) / n) along `axis`, by the
    definition (O(n^2) per pencil; the exponent is reduced in integers, the
    angle formed in FP64).  Unnormalised for either sign."""
    x = np.moveaxis(np.asarray(a, dtype=np.complex128), axis, -1)
    n = x.shape[-1]
    j = np.arange(n, dtype=np.int64)
    roots = np.exp(sign * 2j * np.pi * np.arange(n) / n)  # e^{sign 2 pi i t / n}, t < n
    out = np.empty_like(x)
    for k0 in range(0, n, block):
        k = np.arange(k0, min(n, k0 + block), dtype=np.int64)
        W = roots[(k[:, None] * j[None, :]) % n]
        out[..., k0:k0 + len(k)] = x @ W.T
    return np.moveaxis(out, -1, axis)
